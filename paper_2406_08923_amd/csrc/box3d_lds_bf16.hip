// box3d_lds_bf16.hip -- instantiations of the LDS dense-box kernel for bf16 storage.
#include "box3d_lds.hpp"

namespace stn {
int launch_box3d_lds(const bf16 *in, bf16 *out, const Geo &g, int R, const void *cf, int e, int ty,
                     int lz, int flags, hipStream_t s)
{
    return launch_box3d_lds_impl<bf16>(in, out, g, R, cf, e, ty, lz, flags, s);
}
} // namespace stn
