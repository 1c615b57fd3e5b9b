// box3d_f64.hip -- instantiations of the dense 3-D box kernel for double storage.
#include "box3d.hpp"

namespace stn {
int launch_box3d(const double *in, double *out, const Geo &g, const BoxCoefAny &cf, int ty, int ny,
                 int pf, int lz, int flags, hipStream_t s)
{
    return launch_box3d_impl<double>(in, out, g, cf, ty, ny, pf, lz, flags, s);
}
} // namespace stn
