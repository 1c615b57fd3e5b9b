// rk_kernels.hip -- fused substep phi(gamma(psi(f))) for gfx950: the sixth-order
// derivative bank gamma = AB (Eq. 8), the nonlinear right-hand side phi
// (Eq. 9) and the low-storage RK3 update, in one pass over the grid.
//
// One lane per output point; every tap is read through the hardware caches
// (the hardware-cached strategy of Sec. 4.4, which the paper found fastest for
// the fused MHD kernel on all of its devices) as a buffer load whose tap offset
// is a wave-uniform scalar, so taps cost no per-lane address arithmetic. First and second derivatives
// along an axis share their seven loads; mixed derivatives use the
// antisymmetry of the first-derivative weights to fold the 36 taps into 9
// weighted four-point differences. The periodic images of each output are
// written by the kernel itself, so no halo pass follows.
#include "advdiff_zm.hpp"
#include "mhd_phi.hpp"
#include "rk_point.hpp"

namespace stn {

namespace {

// PointIO of field k of a substep
__device__ __forceinline__ PointIO point_io(const RkArgs &a, int k)
{
    PointIO io;
    io.fout = a.fout[k];
    io.wrd = a.wrd[k];
    io.wwr = a.wwr[k];
    io.w1 = a.w1[k];
    io.master = a.master[k];
    io.alpha = a.alpha;
    io.beta = a.beta;
    io.dt = a.dt;
    for (int i = 0; i < 3; ++i) io.beta_all[i] = a.beta_all[i];
    io.stage = a.stage;
    io.fuse = a.fuse;
    return io;
}

} // namespace

// Derivative bank of one 3-vector field v (three consecutive fields): values,
// the first derivatives d1[ax][b] = d_ax v_b, the Laplacians lap[b] and
// grad(div v)_a = sum_b d_a d_b v_b (pure second derivative for b == a, mixed
// otherwise). Scheduling fences between the groups of loads keep the
// compiler from hoisting all of them, which would exhaust the registers.
// MIXED selects the mixed derivatives: the folded tensor product (36 taps)
// or the diagonals (12 taps).
template <typename S, typename C, int MIXED>
__device__ __forceinline__ C dmix_form(const Buf &b, uint32_t vo, uint32_t c, uint32_t sa,
                                       uint32_t sb, const FdWeights &w)
{
    if constexpr (MIXED == MIX_DIAG)
        return dmix_diag<S, C>(b, vo, c, sa, sb, w);
    else
        return dmix<S, C>(b, vo, c, sa, sb, w);
}

template <typename S, typename C, int MIXED>
__device__ __forceinline__ void vector_bank(const Buf *fb, uint32_t vo, uint32_t c,
                                            const uint32_t *st, const FdWeights &w,
                                            const C *ids, C *val, C (*d1)[3], C *lap, C *gdiv)
{
    C diag[3];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        lap[b] = 0;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            C c0, a1, a2;
            d12<S, C>(fb[b], vo, c, st[ax], w, a1, a2, c0);
            val[b] = c0;
            d1[ax][b] = a1 * ids[ax];
            const C t = a2 * (ids[ax] * ids[ax]);
            lap[b] += t;
            if (ax == b) diag[b] = t;
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    const C sxy = ids[0] * ids[1], sxz = ids[0] * ids[2], syz = ids[1] * ids[2];
    gdiv[0] = diag[0];
    gdiv[1] = diag[1];
    gdiv[2] = diag[2];
    C m;
    m = dmix_form<S, C, MIXED>(fb[1], vo, c, st[0], st[1], w); // d_x d_y v_y
    gdiv[0] = fma(sxy, m, gdiv[0]);
    __builtin_amdgcn_sched_barrier(0);
    m = dmix_form<S, C, MIXED>(fb[2], vo, c, st[0], st[2], w); // d_x d_z v_z
    gdiv[0] = fma(sxz, m, gdiv[0]);
    __builtin_amdgcn_sched_barrier(0);
    m = dmix_form<S, C, MIXED>(fb[0], vo, c, st[0], st[1], w); // d_x d_y v_x
    gdiv[1] = fma(sxy, m, gdiv[1]);
    __builtin_amdgcn_sched_barrier(0);
    m = dmix_form<S, C, MIXED>(fb[2], vo, c, st[1], st[2], w); // d_y d_z v_z
    gdiv[1] = fma(syz, m, gdiv[1]);
    __builtin_amdgcn_sched_barrier(0);
    m = dmix_form<S, C, MIXED>(fb[0], vo, c, st[0], st[2], w); // d_x d_z v_x
    gdiv[2] = fma(sxz, m, gdiv[2]);
    __builtin_amdgcn_sched_barrier(0);
    m = dmix_form<S, C, MIXED>(fb[1], vo, c, st[1], st[2], w); // d_y d_z v_y
    gdiv[2] = fma(syz, m, gdiv[2]);
    __builtin_amdgcn_sched_barrier(0);
}

// Gradient, Laplacian and value of one scalar field.
template <typename S, typename C>
__device__ __forceinline__ void scalar_bank(const Buf &fb, uint32_t vo, uint32_t c,
                                            const uint32_t *st, const FdWeights &w,
                                            const C *ids, C &val, C *grad, C &lap)
{
    lap = 0;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        C a1, a2;
        d12<S, C>(fb, vo, c, st[ax], w, a1, a2, val);
        grad[ax] = a1 * ids[ax];
        lap += a2 * (ids[ax] * ids[ax]);
    }
    __builtin_amdgcn_sched_barrier(0);
}

// Field order (Table A1): lnrho, u_x, u_y, u_z, s, A_x, A_y, A_z. The bank is
// evaluated field group by field group (A, then u, then the scalars) and each
// group is reduced at once to the quantities phi needs, so few values stay
// live at a time. MODEL selects phi (mhd_phi.hpp).
template <typename S, typename W, typename C, bool MASTER, int MODEL, int MIXED>
__global__ void __launch_bounds__(256) k_rk_mhd8(RkArgs a)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    const Geo &g = a.g;
    if (x >= g.nx || y >= g.ny)
        return;
    const int64_t p = g.at(x, y, z);
    constexpr uint32_t es = sizeof(S);
    const uint32_t st[3] = {es, uint32_t(g.sy) * es, uint32_t(g.sz) * es};
    const uint32_t c = 3 * (st[0] + st[1] + st[2]); // centre, from the lowest corner
    const uint32_t vo = uint32_t(p) * es - c;
    const uint64_t bytes = uint64_t(padded_elems(g)) * es;
    Buf fb[8];
#pragma unroll
    for (int k = 0; k < 8; ++k)
        fb[k] = make_buf(a.fin[k], bytes);
    const C ids[3] = {C(a.inv_ds[0]), C(a.inv_ds[1]), C(a.inv_ds[2])};

    // Each group below sits behind its own wave-uniform branch on a kernel
    // argument that is always all-ones: the branches split the kernel into
    // basic blocks, so no scheduler hoists the loads of a later group above an
    // earlier one (which would keep hundreds of values live at once).
    MhdBank<C> k{};
    // gamma, magnetic potential: B = curl A, J = grad(div A) - lap A
    if (a.phases & 1) {
        C dA[3][3], gdivA[3];
        vector_bank<S, C, MIXED>(fb + 5, vo, c, st, a.fd, ids, k.A, dA, k.lapA, gdivA);
        k.B[0] = dA[1][2] - dA[2][1];
        k.B[1] = dA[2][0] - dA[0][2];
        k.B[2] = dA[0][1] - dA[1][0];
#pragma unroll
        for (int i = 0; i < 3; ++i)
            k.J[i] = gdivA[i] - k.lapA[i];
    }
    // gamma, velocity
    if (a.phases & 2)
        vector_bank<S, C, MIXED>(fb + 1, vo, c, st, a.fd, ids, k.u, k.du, k.lapu, k.gdivu);
    // gamma, log density and entropy
    if (a.phases & 4)
        scalar_bank<S, C>(fb[0], vo, c, st, a.fd, ids, k.l, k.gl, k.lapl);
    if (a.phases & 8)
        scalar_bank<S, C>(fb[4], vo, c, st, a.fd, ids, k.s, k.gs, k.laps);

    // phi: the 8-field right-hand side
    C R[8];
    mhd_phi<MODEL, C>(k, a.mhd, R);
    const C val[8] = {k.l, k.u[0], k.u[1], k.u[2], k.s, k.A[0], k.A[1], k.A[2]};
#pragma unroll
    for (int q = 0; q < 8; ++q)
        rk_update<S, W, C, MASTER>(point_io(a, q), g, p, x, y, z, R[q], val[q]);
}

// Scalar advection-diffusion R = -c.grad f + nu lap f, NDIM = 2 or 3.
template <typename S, typename W, typename C, bool MASTER, int NDIM>
__global__ void __launch_bounds__(256) k_rk_advdiff(RkArgs a)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    const Geo &g = a.g;
    if (x >= g.nx || y >= g.ny)
        return;
    advdiff_point<S, W, C, MASTER, NDIM>(a.fin[0], point_io(a, 0), g, a.fd, a.inv_ds, a.adv, a.nu,
                                         x, y, z);
}

// 3-D advection-diffusion as a z march over 64 x 16 tiles and lz planes: the
// right-hand side is a radius-3 star, computed like the linear star, with the
// RK update as the epilogue (advdiff_zm.hpp; the batched job kernel uses the
// same routine).
template <typename S, typename W, typename C, bool MASTER>
__global__ void __launch_bounds__(ZM_NT) k_rk_advdiff3_zm(RkArgs a, int lz)
{
    __shared__ ZmLds<C> lds;
    const StarCoef<C, 3> cf = advdiff_star<C>(a.fd, a.inv_ds, a.adv, a.nu);
    const int x0 = blockIdx.x * ZM_TX, y0 = blockIdx.y * ZM_ROWS, z0 = blockIdx.z * lz;
    advdiff3_zmarch<S, W, C, MASTER>(a.fin[0], point_io(a, 0), a.g, cf, x0, y0, z0,
                                     min(z0 + lz, a.g.nz), lds);
}

namespace {
template <typename K> int launch_grid(K kern, const RkArgs &a, int bx, int by, hipStream_t s,
                                      const char *what)
{
    dim3 block(bx, by);
    dim3 grid((a.g.nx + bx - 1) / bx, (a.g.ny + by - 1) / by, a.g.nz);
    hipLaunchKernelGGL(kern, grid, block, 0, s, a);
    return check_launch(what);
}
} // namespace

namespace {
template <int MODEL, int MIXED>
int launch_mhd_model(int policy, const RkArgs &a, int bx, int by, hipStream_t s)
{
    switch (policy) {
    case POL_F64: return launch_grid(k_rk_mhd8<double, double, double, false, MODEL, MIXED>, a, bx, by, s, "rk_mhd8");
    case POL_F32_MASTER64: return launch_grid(k_rk_mhd8<float, float, float, true, MODEL, MIXED>, a, bx, by, s, "rk_mhd8");
    case POL_BF16_MASTER64: return launch_grid(k_rk_mhd8<bf16, float, float, true, MODEL, MIXED>, a, bx, by, s, "rk_mhd8");
    case POL_F32_ONLY: return launch_grid(k_rk_mhd8<float, float, float, false, MODEL, MIXED>, a, bx, by, s, "rk_mhd8");
    case POL_BF16_ONLY: return launch_grid(k_rk_mhd8<bf16, float, float, false, MODEL, MIXED>, a, bx, by, s, "rk_mhd8");
    }
    return fail(STENCIL_EINVAL, "unknown precision policy %d", policy);
}
} // namespace

int launch_rk_mhd8(int model, int mixed, int policy, const RkArgs &a, int bx, int by,
                   hipStream_t s)
{
#define RK_MODEL_MIXED(M_, X_)                                                               \
    if (model == M_ && mixed == X_) return launch_mhd_model<M_, X_>(policy, a, bx, by, s);
    RK_MODEL_MIXED(MHD_PROXY, MIX_TENSOR)
    RK_MODEL_MIXED(MHD_PROXY, MIX_DIAG)
    RK_MODEL_MIXED(MHD_FULL, MIX_TENSOR)
    RK_MODEL_MIXED(MHD_FULL, MIX_DIAG)
#undef RK_MODEL_MIXED
    return fail(STENCIL_EINVAL, "rk_mhd8: unknown model %d / mixed form %d", model, mixed);
}

namespace {
template <typename S, typename W, typename C, bool M>
int launch_zm(const RkArgs &a, int lz, hipStream_t s)
{
    const dim3 grid((a.g.nx + ZM_TX - 1) / ZM_TX, (a.g.ny + ZM_ROWS - 1) / ZM_ROWS,
                    (a.g.nz + lz - 1) / lz);
    hipLaunchKernelGGL((k_rk_advdiff3_zm<S, W, C, M>), grid, dim3(ZM_TX, ZM_TY), 0, s, a, lz);
    return check_launch("rk_advdiff3_zm");
}
} // namespace

int launch_rk_advdiff3_zm(int policy, const RkArgs &a, int lz, hipStream_t s)
{
    if (a.g.ndim != 3 || lz < 1)
        return fail(STENCIL_EINVAL, "advdiff z march: needs a 3-D plan and lz >= 1");
    if (uint64_t(padded_elems(a.g)) * 8 >= (uint64_t(1) << 32))
        return fail(STENCIL_EUNSUPPORTED, "advdiff: arrays of 4 GiB or more are not supported");
    switch (policy) {
    case POL_F64: return launch_zm<double, double, double, false>(a, lz, s);
    case POL_F32_MASTER64: return launch_zm<float, float, float, true>(a, lz, s);
    case POL_BF16_MASTER64: return launch_zm<bf16, float, float, true>(a, lz, s);
    case POL_F32_ONLY: return launch_zm<float, float, float, false>(a, lz, s);
    case POL_BF16_ONLY: return launch_zm<bf16, float, float, false>(a, lz, s);
    }
    return fail(STENCIL_EINVAL, "unknown precision policy %d", policy);
}

// Every step of a run of a small 2-D FP64 advection-diffusion grid, in LDS:
// one 1024-lane workgroup holds both states with a 3-cell periodic halo (each
// point also writes its images into the halo, so taps are fixed offsets and
// a substep needs one barrier), runs 3 nsteps substeps and writes the two
// last states (with their periodic images) and the register back. The point
// arithmetic is the per-substep kernel's (d12_vals, advdiff_axis,
// rk_register, the same update), so the states are bitwise those of
// 3 nsteps substep launches; HBM is touched once per run.
constexpr int RES_THREADS = 1024, RES_PER = (RES_MAX_POINTS + RES_THREADS - 1) / RES_THREADS;

__global__ void __launch_bounds__(RES_THREADS) k_rk_advdiff2_resident(ResidentArgs a)
{
    __shared__ double lf[2][RES_MAX_CELLS];
    __shared__ double lw[RES_MAX_POINTS];
    const Geo &g = a.g;
    const int nx = g.nx, ny = g.ny, n = nx * ny, lw_ = nx + 6;
    // the lane's points: LDS cell and the cell offsets of their x / y images
    int cell[RES_PER], dxi[RES_PER], dyi[RES_PER];
#pragma unroll
    for (int k = 0; k < RES_PER; ++k) {
        const int p = threadIdx.x + k * RES_THREADS;
        const int x = p < n ? p % nx : 0, y = p < n ? p / nx : 0;
        cell[k] = (y + 3) * lw_ + x + 3;
        dxi[k] = x < 3 ? nx : x >= nx - 3 ? -nx : 0;
        dyi[k] = (y < 3 ? ny : y >= ny - 3 ? -ny : 0) * lw_;
    }
    auto put = [&](double *f, int k, double v) {
        const int c = cell[k];
        f[c] = v;
        if (dxi[k]) f[c + dxi[k]] = v;
        if (dyi[k]) f[c + dyi[k]] = v;
        if (dxi[k] && dyi[k]) f[c + dxi[k] + dyi[k]] = v;
    };
#pragma unroll
    for (int k = 0; k < RES_PER; ++k) {
        const int p = threadIdx.x + k * RES_THREADS;
        if (p < n) {
            put(lf[0], k, a.fin[g.at(p % nx, p / nx, 0)]);
            lw[p] = 0.0;
        }
    }
    __syncthreads();
    int cur = 0;
    for (int step = 0; step < a.nsteps; ++step) {
        for (int stage = 0; stage < 3; ++stage) {
            const double *f = lf[cur];
            double *fo = lf[cur ^ 1];
#pragma unroll
            for (int k = 0; k < RES_PER; ++k) {
                const int p = threadIdx.x + k * RES_THREADS;
                if (p >= n)
                    break;
                const double *q = f + cell[k];
                const double c0 = q[0];
                double a1, a2, R = 0;
                d12_vals(c0, q[-1], q[1], q[-2], q[2], q[-3], q[3], a.fd, a1, a2);
                R = advdiff_axis(R, a1, a2, a.adv[0], a.inv_ds[0], a.nu);
                d12_vals(c0, q[-lw_], q[lw_], q[-2 * lw_], q[2 * lw_], q[-3 * lw_], q[3 * lw_],
                         a.fd, a1, a2);
                R = advdiff_axis(R, a1, a2, a.adv[1], a.inv_ds[1], a.nu);
                const double wn = rk_register<double, double>(a.dt, a.alpha[stage], stage, R, lw[p]);
                if (stage < 2)
                    lw[p] = wn;
                put(fo, k, fma(a.beta[stage], wn, c0));
            }
            __syncthreads();
            cur ^= 1;
        }
    }
#pragma unroll
    for (int k = 0; k < RES_PER; ++k) {
        const int p = threadIdx.x + k * RES_THREADS;
        if (p < n) {
            const int x = p % nx, y = p / nx;
            store_periodic(a.out_last, g, x, y, 0, lf[cur][cell[k]], true);
            store_periodic(a.out_prev, g, x, y, 0, lf[cur ^ 1][cell[k]], true);
            a.w[g.at(x, y, 0)] = lw[p];
        }
    }
}

int launch_rk_advdiff2_resident(const ResidentArgs &a, hipStream_t s)
{
    if (!resident_fits(a.g.ndim, a.g.nx, a.g.ny) || a.nsteps < 1)
        return fail(STENCIL_EINVAL, "resident run: a 2-D grid of at most %d points", RES_MAX_POINTS);
    hipLaunchKernelGGL(k_rk_advdiff2_resident, dim3(1), dim3(RES_THREADS), 0, s, a);
    return check_launch("rk_advdiff2_resident");
}

int launch_rk_advdiff(int policy, const RkArgs &a, int bx, int by, hipStream_t s)
{
    const bool d3 = a.g.ndim == 3;
#define ADV(S_, W_, C_, M_)                                                                  \
    return d3 ? launch_grid(k_rk_advdiff<S_, W_, C_, M_, 3>, a, bx, by, s, "rk_advdiff")     \
              : launch_grid(k_rk_advdiff<S_, W_, C_, M_, 2>, a, bx, by, s, "rk_advdiff")
    switch (policy) {
    case POL_F64: ADV(double, double, double, false);
    case POL_F32_MASTER64: ADV(float, float, float, true);
    case POL_BF16_MASTER64: ADV(bf16, float, float, true);
    case POL_F32_ONLY: ADV(float, float, float, false);
    case POL_BF16_ONLY: ADV(bf16, float, float, false);
    }
#undef ADV
    return fail(STENCIL_EINVAL, "unknown precision policy %d", policy);
}

} // namespace stn
