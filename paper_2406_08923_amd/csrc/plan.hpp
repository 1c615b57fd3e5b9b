// plan.hpp -- the opaque plan object behind stencil_plan_t (internal).
#pragma once

#include "linear_kernels.hpp"
#include "rk_kernels.hpp"

#include <vector>

namespace stn {

enum PlanKind { PLAN_LINEAR = 1, PLAN_RK = 2 };

struct LinearPlan {
    int dtype = 0, bc = 0;
    Geo g{};
    std::vector<double> dense; // (2r+1)^ndim coefficients, x fastest
    int ntaps = 0, reff = 0;   // pruned taps and their radius
    bool is_star = false;
    int op = STENCIL_OP_XCORR; // window filters: STENCIL_OP_MAX / MIN / MEDIAN
    bool is_box = false;       // 3-D window covering the full (2r+1)^3 box
    bool is_dense3 = false;    // 3-D cross-correlation with all (2R+1)^3 taps of its
                               // radius-R box nonzero, R = reff = 1..4
    bool is_dense2 = false;    // the same for a 2-D cross-correlation ((2R+1)^2 taps)
    StarCoefAny star{};
    BoxCoefAny box{};
    void *d_offs = nullptr;  // int32 tap offsets in the padded array
    void *d_taps = nullptr;  // tap coefficients, arithmetic type
    void *d_dense = nullptr; // 1-D dense coefficients, arithmetic type
    // chosen variant and its launch parameters
    int variant = STENCIL_VARIANT_GENERIC;
    int ty = 8, ny = 2, lz = 32, sflags = 0, pf = 2, xw = 1; // STAR3D
    int tstar = 1;          // STAR3D iterations per launch (1 or 2)
    int pairs = 0;          // two-iteration STAR3D with pair-layout LDS planes
    int dpp = 0;            // one-iteration STAR3D / box filter with x taps
                            // exchanged across lanes (no LDS)
    int s1[5] = {0};        // one-iteration STAR3D shape used beside tstar = 2:
                            // {ty, ny, lz, flags, xw}
    int gbx = 64, gby = 4;                   // GENERIC
    int e1d = 4, t1d = 1, rb1d = 0;          // LINE1D: outputs per lane, fused
                                             // iterations, adjacent (register-blocked)
};

struct RkPlan {
    int model = 0, policy = 0, nf = 0;
    int mixed = 0; // STENCIL_MIXED_*
    Geo g{};
    FdWeights fd{};
    double inv_ds[3] = {1, 1, 1};
    double nu = 0, adv[3] = {0, 0, 0}; // ADVDIFF
    MhdParams mhd{};                     // MHD8 / MHD_FULL
    int variant = STENCIL_RK_VARIANT_CACHED;
    int bx = 64, by = 4, bz = 1; // CACHED: lanes; LDS: brick
    int occ = 0;                 // LDS bricks: occupancy target (waves per SIMD)
    size_t store_size = 8, reg_size = 8; // bytes per element of f and of w
    int resident = 0; // run whole runs in one launch in LDS (small 2-D FP64 advection)
};

// validation helpers shared by the C-ABI translation units
int check_dims(int ndim, const int *dims, int r, int bc);
int check_buffers(const void *a, const void *b, size_t bytes, size_t align);
int check_device(int plan_device);

} // namespace stn

struct stencil_plan_s {
    int kind = 0;
    int device = 0;
    int sticky = 0; // device error latched by an earlier call
    stn::LinearPlan lin;
    stn::RkPlan rk;
};

namespace stn {
inline void plan_release_device(stencil_plan_s *p)
{
    void *bufs[] = {p->lin.d_offs, p->lin.d_taps, p->lin.d_dense};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
    p->lin.d_offs = p->lin.d_taps = p->lin.d_dense = nullptr;
}
} // namespace stn
