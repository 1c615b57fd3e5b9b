// box3d_lds_f64.hip -- instantiations of the LDS dense-box kernel for double storage.
#include "box3d_lds.hpp"

namespace stn {
int launch_box3d_lds(const double *in, double *out, const Geo &g, int R, const void *cf, int e, int ty,
                     int lz, int flags, hipStream_t s)
{
    return launch_box3d_lds_impl<double>(in, out, g, R, cf, e, ty, lz, flags, s);
}
} // namespace stn
