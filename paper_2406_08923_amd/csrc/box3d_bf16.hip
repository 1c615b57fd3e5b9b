// box3d_bf16.hip -- instantiations of the dense 3-D box kernel for bf16 storage.
#include "box3d.hpp"

namespace stn {
int launch_box3d(const bf16 *in, bf16 *out, const Geo &g, const BoxCoefAny &cf, int ty, int ny,
                 int pf, int lz, int flags, hipStream_t s)
{
    return launch_box3d_impl<bf16>(in, out, g, cf, ty, ny, pf, lz, flags, s);
}
} // namespace stn
