// rk_mhd8_lds.hip -- dispatch of the LDS-brick 8-field substep (the kernel
// is in rk_mhd8_lds.hpp; each model and mixed form is instantiated in its own
// unit, rk_mhd8_lds_*.hip, so they compile in parallel).
#include "mhd_phi.hpp"
#include "rk_point.hpp"

namespace stn {

template <int MODEL, int MIXED>
int launch_lds_model(int policy, const RkArgs &a, int bx, int by, int bz, int occ, hipStream_t s);

int launch_rk_mhd8_lds(int model, int mixed, int policy, const RkArgs &a, int bx, int by,
                       int bz, int occ, hipStream_t s)
{
    if (uint64_t(padded_elems(a.g)) * 8 >= (uint64_t(1) << 32))
        return fail(STENCIL_EUNSUPPORTED, "rk_mhd8: arrays of 4 GiB or more are not supported");
#define RK_MODEL_MIXED(M_, X_)                                                               \
    if (model == M_ && mixed == X_) return launch_lds_model<M_, X_>(policy, a, bx, by, bz, occ, s);
    RK_MODEL_MIXED(MHD_PROXY, MIX_TENSOR)
    RK_MODEL_MIXED(MHD_PROXY, MIX_DIAG)
    RK_MODEL_MIXED(MHD_FULL, MIX_TENSOR)
    RK_MODEL_MIXED(MHD_FULL, MIX_DIAG)
#undef RK_MODEL_MIXED
    return fail(STENCIL_EINVAL, "rk_mhd8 (LDS): unknown model %d / mixed form %d", model, mixed);
}

} // namespace stn
