// rk_mhd8_lds_f0.hip -- LDS-brick substep instances for the full model, tensor-product mixed derivatives.
#include "rk_mhd8_lds.hpp"

namespace stn {
template int launch_lds_model<MHD_FULL, MIX_TENSOR>(int, const RkArgs &, int, int, int, int, hipStream_t);
} // namespace stn
