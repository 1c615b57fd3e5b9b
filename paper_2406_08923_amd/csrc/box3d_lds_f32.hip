// box3d_lds_f32.hip -- instantiations of the LDS dense-box kernel for float storage.
#include "box3d_lds.hpp"

namespace stn {
int launch_box3d_lds(const float *in, float *out, const Geo &g, int R, const void *cf, int e, int ty,
                     int lz, int flags, hipStream_t s)
{
    return launch_box3d_lds_impl<float>(in, out, g, R, cf, e, ty, lz, flags, s);
}
} // namespace stn
