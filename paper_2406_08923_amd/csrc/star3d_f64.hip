// star3d_f64.hip -- instantiations of the 3-D star kernel for double storage.
#include "star3d.hpp"

namespace stn {
int launch_star3d(const double *in, double *out, const Geo &g, const StarCoefAny &cf, int R, int xw,
                  int ty, int ny, int pf, int lz, int flags, hipStream_t s)
{
    return launch_star3d_impl<double>(in, out, g, cf, R, xw, ty, ny, pf, lz, flags, s);
}
int launch_star3d_t2(const double *in, double *out, const Geo &g, const StarCoefAny &cf, int R, int xw,
                     int ty, int ny, int lz, int flags, hipStream_t s)
{
    return launch_star3d_t2_impl<double>(in, out, g, cf, R, xw, ty, ny, lz, flags, s);
}
} // namespace stn
