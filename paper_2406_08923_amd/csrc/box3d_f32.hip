// box3d_f32.hip -- instantiations of the dense 3-D box kernel for float storage.
#include "box3d.hpp"

namespace stn {
int launch_box3d(const float *in, float *out, const Geo &g, const BoxCoefAny &cf, int ty, int ny,
                 int pf, int lz, int flags, hipStream_t s)
{
    return launch_box3d_impl<float>(in, out, g, cf, ty, ny, pf, lz, flags, s);
}
} // namespace stn
