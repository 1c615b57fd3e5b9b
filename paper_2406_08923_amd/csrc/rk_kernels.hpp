// rk_kernels.hpp -- fused derivative bank + nonlinear right-hand side +
// low-storage RK3 substep kernels (internal).
#pragma once

#include "common.hpp"

namespace stn {

constexpr int MAX_NF = 8;

// Sixth-order (radius 3) central-difference weights, unit spacing, offsets
// +1..+3 (the -m weights follow by symmetry): first derivative w1[m-1] is the
// weight of f(+m) (that of f(-m) is -w1[m-1]); second derivative w2[0] is the
// centre and w2[m] the weight of f(+-m).
struct FdWeights {
    double w1[3];
    double w2[4];
};

// Precision policies of the fused substep.
enum RkPolicy {
    POL_F64 = 0,           // FP64 storage, FP64 register, FP64 arithmetic
    POL_F32_MASTER64 = 1,  // FP32 storage, FP32 registers, FP64 master at the last substep
    POL_BF16_MASTER64 = 2, // BF16 storage, FP32 registers, FP64 master at the last substep
    POL_F32_ONLY = 3,      // FP32 storage, FP32 register, no master (ablation)
    POL_BF16_ONLY = 4,     // BF16 storage, FP32 register, no master (ablation)
};

// Constants of the MHD right-hand sides (the proxy reads nu, eta, cs2; the
// full model all of them, with cs2 = cs0^2, the sound speed squared at s = 0,
// lnrho = lnrho0).
struct MhdParams {
    double nu, eta, cs2;
    double zeta, mu0, gamma, cp, lnrho0, K, heat, cool;
};

// Kernel arguments of one substep. Pointers are padded fields (radius 3).
struct RkArgs {
    const void *fin[MAX_NF]; // stencil input, storage type
    void *fout[MAX_NF];      // substep output, storage type
    const void *wrd[MAX_NF]; // register read (alpha * w); unused at stage 0
    void *wwr[MAX_NF];       // register written
    const void *w1[MAX_NF];  // master policies, stage 2: first-stage register
    double *master[MAX_NF];  // master policies, stage 2: FP64 state (read + written)
    Geo g;
    double alpha, beta, dt;
    double beta_all[3];
    double inv_ds[3];
    double nu;               // ADVDIFF diffusivity
    double adv[3];           // ADVDIFF velocity
    MhdParams mhd;           // MHD models
    FdWeights fd;
    int stage;
    int fuse;                // write periodic images
    int phases;              // always all-ones: uniform branches that split the
                             // fused kernel into basic blocks (see k_rk_mhd8)
};

// model: 0 = the 8-field proxy, 2 = the full non-ideal MHD equations;
// mixed: 0 = tensor-product mixed derivatives, 1 = diagonal (12 taps)
int launch_rk_mhd8(int model, int mixed, int policy, const RkArgs &a, int bx, int by,
                   hipStream_t s);

// LDS-brick variant of the MHD8 substep (rk_mhd8_lds.hpp): bricks of
// bx x by x bz output points with an occupancy target (waves per SIMD the
// compiler is held to; 0 = its own choice), one of RK_BRICK_SHAPES
#define RK_BRICK_SHAPES(X)                                                                   \
    X(16, 8, 4, 0) X(16, 8, 4, 4) X(16, 8, 8, 0) X(32, 4, 4, 0) X(32, 4, 4, 4) X(8, 8, 8, 0)  \
    X(8, 8, 8, 4)
int launch_rk_mhd8_lds(int model, int mixed, int policy, const RkArgs &a, int bx, int by,
                       int bz, int occ, hipStream_t s);
int launch_rk_advdiff(int policy, const RkArgs &a, int bx, int by, hipStream_t s);
// Small 2-D FP64 advection-diffusion grids whose state fits in LDS: every
// step of a run in one launch of one workgroup (k_rk_advdiff2_resident).
// LDS: two states with a 3-cell halo (at most RES_MAX_CELLS cells each) and
// the register (at most RES_MAX_POINTS), FP64: 8 B x (2 x 7000 + 5200) = 150 KiB
constexpr int RES_MAX_POINTS = 5200, RES_MAX_CELLS = 7000;
inline bool resident_fits(int ndim, int nx, int ny)
{
    return ndim == 2 && nx >= 6 && ny >= 6 && int64_t(nx) * ny <= RES_MAX_POINTS &&
           int64_t(nx + 6) * (ny + 6) <= RES_MAX_CELLS;
}
struct ResidentArgs {
    const double *fin;  // padded input state
    double *out_last;   // receives the last substep's state (with its images)
    double *out_prev;   // receives the state of the substep before it
    double *w;          // the register, as the last substep that wrote it left it
    Geo g;
    FdWeights fd;
    double inv_ds[2], adv[2], nu, dt;
    double alpha[3], beta[3];
    int nsteps;
};
int launch_rk_advdiff2_resident(const ResidentArgs &a, hipStream_t s);
// 3-D advection-diffusion substep as a z march (64 x 16 tiles, lz planes)
int launch_rk_advdiff3_zm(int policy, const RkArgs &a, int lz, hipStream_t s);
// z planes per tile of the z march (solo and batched)
constexpr int ZM_LZ = 32;
// The z march pays off once a 3-D grid fills the GPU with its 64 x 16 x ZM_LZ
// tiles; smaller grids keep the per-point kernel (more, smaller workgroups).
// The solo plan and the batched job table apply the same rule, so a job's
// arithmetic does not depend on how it is run.
constexpr long long ZM_MIN_POINTS = 1ll << 20;
inline bool advdiff_uses_zmarch(const Geo &g)
{
    return g.ndim == 3 && (long long)g.nx * g.ny * g.nz >= ZM_MIN_POINTS;
}
// z planes per z-march tile for a grid: deep tiles (ZM_LZ) on large grids,
// shallower ones (down to 8) where that is needed for about 1024 tiles, so a
// mid-size job still spreads over every CU. The depth changes no result.
inline int advdiff_zmarch_lz(const Geo &g)
{
    const long long txy = (long long)((g.nx + 63) / 64) * ((g.ny + 15) / 16);
    const long long lz = (long long)g.nz * txy / 1024;
    return (int)(lz < 8 ? 8 : lz > ZM_LZ ? ZM_LZ : lz);
}

} // namespace stn
