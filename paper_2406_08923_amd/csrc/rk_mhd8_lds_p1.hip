// rk_mhd8_lds_p1.hip -- LDS-brick substep instances for the proxy, diagonal mixed derivatives.
#include "rk_mhd8_lds.hpp"

namespace stn {
template int launch_lds_model<MHD_PROXY, MIX_DIAG>(int, const RkArgs &, int, int, int, int, hipStream_t);
} // namespace stn
