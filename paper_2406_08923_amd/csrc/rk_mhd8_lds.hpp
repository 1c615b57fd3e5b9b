// rk_mhd8_lds.hpp -- the fused 8-field substep phi(gamma(psi(f))) with the
// derivative bank read from LDS: a workgroup owns a BX x BY x BZ brick of
// output points (one per lane) and streams the eight fields, one at a time,
// through a double-buffered LDS tile of the brick plus its radius-3 halo
// (Sec. 4.1's shared-memory strategy applied to the Eq. 8 bank). The next
// field's tile is in flight (straight into the other LDS buffer, or through
// registers for BF16 storage) while the current one is differentiated, so a
// field costs one barrier. Every derivative tap is an LDS read; HBM/L2 see
// each field once per brick (times the halo overhead).
#pragma once

#include <type_traits>

#include "mhd_phi.hpp"
#include "rk_point.hpp"

namespace stn {

namespace {

// LDS tile of one field: (BX+6) x (BY+6) x (BZ+6), x fastest.
template <int BX, int BY, int BZ> struct Brick {
    static constexpr int TX = BX + 6, TY = BY + 6, TZ = BZ + 6;
    static constexpr int TN = TX * TY * TZ;
    static constexpr int NT = BX * BY * BZ;
    static constexpr int PER = (TN + NT - 1) / NT; // tile cells loaded per lane
    static constexpr int SY = TX, SZ = TX * TY;    // LDS strides
};

// d1 and d2 (unit spacing) along one axis from LDS, stride st (elements);
// the same expression as the cached kernel's d12
template <typename C>
__device__ __forceinline__ void d12_lds(const C *t, int c, int st, const FdWeights &w, C &d1,
                                        C &d2, C &c0)
{
    c0 = t[c];
    const C m1 = t[c - st], q1 = t[c + st];
    const C m2 = t[c - 2 * st], q2 = t[c + 2 * st];
    const C m3 = t[c - 3 * st], q3 = t[c + 3 * st];
    d1 = C(w.w1[0]) * (q1 - m1) + C(w.w1[1]) * (q2 - m2) + C(w.w1[2]) * (q3 - m3);
    d2 = C(w.w2[0]) * c0 + C(w.w2[1]) * (q1 + m1) + C(w.w2[2]) * (q2 + m2) +
         C(w.w2[3]) * (q3 + m3);
}

// d_a d_b (unit spacing) from LDS along the two diagonals of the a-b plane:
// second-derivative weights along (+a, +b) minus along (+a, -b) give
// 4 d_a d_b; the centre cancels, 12 reads.
template <typename C>
__device__ __forceinline__ C dmix_diag_lds(const C *t, int c, int sa, int sb, const FdWeights &w)
{
    C acc = 0;
#pragma unroll
    for (int m = 1; m <= 3; ++m) {
        const int ma = m * sa, mb = m * sb;
        const C along = t[c + ma + mb] + t[c - ma - mb];
        const C across = t[c + ma - mb] + t[c - ma + mb];
        acc = fma(C(0.25 * w.w2[m]), along - across, acc);
    }
    return acc;
}

// Materialise v here: an empty volatile asm that reads and writes v keeps the
// compiler from sinking the arithmetic that produced it past later barriers
// (it would otherwise move the whole bank into the block that stores the
// results, keeping every raw LDS value live across the barriers).
__device__ __forceinline__ void pin(double &v) { asm volatile("" : "+v"(v)); }
__device__ __forceinline__ void pin(float &v) { asm volatile("" : "+v"(v)); }

// Quantities phi needs from a 3-vector field v: value, first derivatives
// d1[ax][b] = d_ax v_b, Laplacian, and the mixed part of grad(div v)
// (gdivm[a] = sum_{b != a} d_a d_b v_b); pure second derivatives d_aa v_a are
// kept in diag and added at the end.
template <typename C> struct VecAcc {
    C val[3], d1[3][3], lap[3], diag[3], gdivm[3];
};

// One component b of a vector field from the tile: its d1/d2 along every
// axis and its two mixed derivatives, scattered into the grad(div v) sums.
// Tensor form (MIX_TENSOR): the mixed derivatives d_a d_b v_b (a != b) are
// taken separably: g = d_b v_b (unit spacing) is evaluated once per cell of
// the brick widened by 3 along both other axes and staged in LDS (gb), then
// d_a g is read from there (mixed_from_stage): about 15 LDS accesses per
// point for the pair instead of 72. The caller reads the staged values after
// the next barrier it passes anyway (the next field's), with the staging
// buffers alternating between components, so the staging costs no barrier of
// its own. Diagonal form (MIX_DIAG): 12 tile reads per mixed derivative,
// taken here, no staging (gb unused).
template <typename C, int BX, int BY, int BZ, int MIXED>
__device__ __forceinline__ void vec_component(const C *t, C *gb, int tid, int lx, int ly, int lz,
                                              int b, const FdWeights &w, const C *ids,
                                              VecAcc<C> &v)
{
    using B = Brick<BX, BY, BZ>;
    const int st[3] = {1, B::SY, B::SZ};
    const int c = (lx + 3) + B::SY * (ly + 3) + B::SZ * (lz + 3);
    v.lap[b] = 0;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        C c0, a1, a2;
        d12_lds<C>(t, c, st[ax], w, a1, a2, c0);
        v.val[b] = c0;
        v.d1[ax][b] = a1 * ids[ax];
        const C q = a2 * (ids[ax] * ids[ax]);
        v.lap[b] += q;
        if (ax == b) v.diag[b] = q;
    }
    pin(v.val[b]);
    pin(v.lap[b]);
    pin(v.diag[b]);
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) pin(v.d1[ax][b]);

    if constexpr (MIXED == MIX_DIAG) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            if (a == b) continue;
            const C m = dmix_diag_lds<C>(t, c, st[a], st[b], w);
            v.gdivm[a] = fma(ids[a] * ids[b], m, v.gdivm[a]);
            pin(v.gdivm[a]);
        }
        return;
    }
    // region: the brick widened by 3 on both sides of every axis except b
    const int RX = b == 0 ? BX : BX + 6, RY = b == 1 ? BY : BY + 6, RZ = b == 2 ? BZ : BZ + 6;
    const int ox = b == 0 ? 3 : 0, oy = b == 1 ? 3 : 0, oz = b == 2 ? 3 : 0; // tile offset
    const int RN = RX * RY * RZ;
    const int sb = st[b];
    for (int e = tid; e < RN; e += B::NT) {
        const int ex = e % RX, ey = (e / RX) % RY, ez = e / (RX * RY);
        const int ce = (ex + ox) + B::SY * (ey + oy) + B::SZ * (ez + oz);
        gb[e] = C(w.w1[0]) * (t[ce + sb] - t[ce - sb]) + C(w.w1[1]) * (t[ce + 2 * sb] - t[ce - 2 * sb]) +
                C(w.w1[2]) * (t[ce + 3 * sb] - t[ce - 3 * sb]);
    }
}

// Tensor form: the two mixed derivatives d_a d_b v_b (a != b) of component b
// from its staged d_b v_b (a barrier separates the staging from this).
template <typename C, int BX, int BY, int BZ>
__device__ __forceinline__ void mixed_from_stage(const C *gb, int lx, int ly, int lz, int b,
                                                 const FdWeights &w, const C *ids, VecAcc<C> &v)
{
    const int RX = b == 0 ? BX : BX + 6, RY = b == 1 ? BY : BY + 6;
    const int ox = b == 0 ? 3 : 0, oy = b == 1 ? 3 : 0, oz = b == 2 ? 3 : 0; // tile offset
    // this lane's point in the region, and the region strides
    const int cg = (lx + 3 - ox) + RX * ((ly + 3 - oy) + RY * (lz + 3 - oz));
    const int rs[3] = {1, RX, RX * RY};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (a == b) continue;
        const int sa = rs[a];
        const C m = C(w.w1[0]) * (gb[cg + sa] - gb[cg - sa]) +
                    C(w.w1[1]) * (gb[cg + 2 * sa] - gb[cg - 2 * sa]) +
                    C(w.w1[2]) * (gb[cg + 3 * sa] - gb[cg - 3 * sa]);
        v.gdivm[a] = fma(ids[a] * ids[b], m, v.gdivm[a]);
        pin(v.gdivm[a]);
    }
}

template <typename C, int SY, int SZ>
__device__ __forceinline__ void scalar_field(const C *t, int c, const FdWeights &w, const C *ids,
                                             C &val, C *grad, C &lap)
{
    const int st[3] = {1, SY, SZ};
    lap = 0;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        C a1, a2;
        d12_lds<C>(t, c, st[ax], w, a1, a2, val);
        grad[ax] = a1 * ids[ax];
        lap += a2 * (ids[ax] * ids[ax]);
        pin(grad[ax]);
    }
    pin(val);
    pin(lap);
}

} // namespace

// Field order (Table A1): lnrho, u_x, u_y, u_z, s, A_x, A_y, A_z; streamed as
// A_x, A_y, A_z, u_x, u_y, u_z, lnrho, s. MODEL selects phi (mhd_phi.hpp),
// MIXED the form of the mixed derivatives.
// OCC: the occupancy the compiler is asked for, in waves per SIMD (0 = its
// own choice; 4 with a 512-lane brick holds the kernel to 128 VGPRs so two
// workgroups share a CU). The arithmetic does not depend on it.
template <typename S, typename W, typename C, bool MASTER, int MODEL, int MIXED, int BX, int BY,
          int BZ, int OCC>
__global__ void __launch_bounds__(BX *BY *BZ, (OCC > 0 ? OCC : 1))
    k_rk_mhd8_lds(RkArgs a, int gx, int gy, int gz)
{
    using B = Brick<BX, BY, BZ>;
    // Where the stored type is the arithmetic type (FP64, FP32 storage), a
    // field's tile goes from HBM straight into LDS (buffer loads to LDS: each
    // wave fills chunks of 64 x EPL consecutive tile cells, lane l the EPL
    // cells at 64 EPL j + EPL l; a tile row has an even number of cells, so
    // an FP64 pair never straddles rows), with no registers in between and no
    // LDS stores. BF16 storage is widened on the way, through registers.
    constexpr bool DMA = std::is_same<S, C>::value;
    constexpr int EPL = DMA && sizeof(C) == 8 ? 2 : 1; // cells per lane and load
    constexpr int CH = 64 * EPL;                        // cells per wave and load
    constexpr int NCH = (B::TN + CH - 1) / CH;          // chunks per tile
    constexpr int NW = B::NT / 64;                      // waves
    constexpr int Q = (NCH + NW - 1) / NW;              // loads per lane and field
    constexpr int TNP = DMA ? NCH * CH : B::TN;         // tile padded to whole chunks
    static_assert(B::TX % 2 == 0 && B::NT % 64 == 0, "tile rows of even length, whole waves");
    static_assert(!DMA || EPL * sizeof(C) == 16 || EPL * sizeof(C) == 4, "load size");
    // two arrays, so the compiler's wait counting tells a load into one
    // buffer from reads of the other
    __shared__ C tile0[TNP];
    __shared__ C tile1[TNP];
    // tensor form: staging of d_b v_b on the brick widened along the other two
    // axes (the largest of the three regions); the diagonal form needs none
    constexpr int G0 = BX * (BY + 6) * (BZ + 6), G1 = (BX + 6) * BY * (BZ + 6),
                  G2 = (BX + 6) * (BY + 6) * BZ;
    constexpr int GT = G0 > G1 ? (G0 > G2 ? G0 : G2) : (G1 > G2 ? G1 : G2);
    constexpr int GN = MIXED == MIX_TENSOR ? GT : 1;
    __shared__ C gbuf0[GN];
    __shared__ C gbuf1[GN];
    constexpr uint32_t es = sizeof(S);
    const Geo &g = a.g;

    int lin = blockIdx.x;
    const int total = gx * gy * gz;
    {   // XCD-aware order: XCD k gets a contiguous run of bricks (x fastest)
        const int per = total / 8, rem = total % 8;
        const int xcd = lin % 8, slot = lin / 8;
        lin = xcd < rem ? xcd * (per + 1) + slot : rem * (per + 1) + (xcd - rem) * per + slot;
    }
    const int bxi = lin % gx, byi = (lin / gx) % gy, bzi = lin / (gx * gy);
    const int x0 = bxi * BX, y0 = byi * BY, z0 = bzi * BZ;
    const int tid = threadIdx.x;
    const int lx = tid % BX, ly = (tid / BX) % BY, lz = tid / (BX * BY);
    const int x = x0 + lx, y = y0 + ly, z = z0 + lz;
    const bool live = x < g.nx && y < g.ny && z < g.nz;

    // byte offsets (into the padded array) of tile cells; cells past the
    // padded extent of a ragged brick are clamped onto it (they feed only
    // points outside the grid; so does the second cell of a clamped pair)
    auto cell_off = [&](int e) {
        const int ex = e % B::TX, ey = (e / B::TX) % B::TY, ez = e / (B::TX * B::TY);
        const int px = min(x0 - 3 + ex, g.nx + 2), py = min(y0 - 3 + ey, g.ny + 2),
                  pz = min(z0 - 3 + ez, g.nz + 2);
        return uint32_t(g.at(px, py, pz)) * es;
    };
    const uint64_t bytes = uint64_t(padded_elems(g)) * es;
    constexpr int NOFF = DMA ? Q : B::PER;
    uint32_t off[NOFF];
    const int wv = __builtin_amdgcn_readfirstlane(tid / 64);
#pragma unroll
    for (int q = 0; q < NOFF; ++q) {
        const int e = DMA ? EPL * ((wv + NW * q) * 64 + tid % 64) : tid + q * B::NT;
        off[q] = e < B::TN ? cell_off(e) : 0u;
    }
    C reg[DMA ? 1 : B::PER];
    // FETCH(k, dst): start loading field k's tile (into dst, or into
    // registers); LAND(dst): write the registers to dst (register path)
#define FETCH(k, dst)                                                                        \
    do {                                                                                     \
        const Buf fb = make_buf(a.fin[k], bytes);                                            \
        if constexpr (DMA) {                                                                 \
            _Pragma("unroll") for (int q = 0; q < Q; ++q) {                                  \
                const int j = wv + NW * q;                                                   \
                if (NW * (q + 1) <= NCH || j < NCH) { /* every wave has chunk q, or this one */ \
                    if constexpr (EPL * sizeof(C) == 16)                                     \
                        buf_to_lds16(fb, (dst) + j * CH, off[q]);                            \
                    else                                                                     \
                        buf_to_lds4(fb, (dst) + j * CH, off[q]);                             \
                }                                                                            \
            }                                                                                \
        } else {                                                                             \
            _Pragma("unroll") for (int q = 0; q < B::PER; ++q) reg[q] =                      \
                BufLd<S>::ld(fb, off[q], 0);                                                 \
        }                                                                                    \
    } while (0)
#define LAND(dst)                                                                            \
    do {                                                                                     \
        if constexpr (!DMA) {                                                                \
            _Pragma("unroll") for (int q = 0; q < B::PER; ++q) if (tid + q * B::NT < B::TN)  \
                (dst)[tid + q * B::NT] = reg[q];                                             \
        }                                                                                    \
    } while (0)

    const C ids[3] = {C(a.inv_ds[0]), C(a.inv_ds[1]), C(a.inv_ds[2])};
    const int c = (lx + 3) + B::SY * (ly + 3) + B::SZ * (lz + 3);
    VecAcc<C> A{}, U{};
    C vl = 0, vs = 0, gl[3] = {}, gs[3] = {}, lapl = 0, laps = 0;

    // the streaming order A_x, A_y, A_z, u_x, u_y, u_z, lnrho, s; the loads
    // of the next field are issued before the current one is differentiated,
    // into the buffer whose last reads the preceding barrier closed. Tensor
    // form: component k stages into gbuf(k mod 2) and its mixed derivatives
    // are read after the next barrier (MIXED_PREV), before component k + 1
    // stages into the other buffer.
    constexpr bool T = MIXED == MIX_TENSOR;
#define MIXED_PREV(gb, b, V)                                                                 \
    do {                                                                                     \
        if constexpr (T)                                                                     \
            mixed_from_stage<C, BX, BY, BZ>(gb, lx, ly, lz, b, a.fd, ids, V);                \
    } while (0)
    FETCH(5, tile0);
    LAND(tile0);
    __syncthreads();
    FETCH(6, tile1);
    vec_component<C, BX, BY, BZ, MIXED>(tile0, gbuf0, tid, lx, ly, lz, 0, a.fd, ids, A);
    LAND(tile1);
    __syncthreads();
    MIXED_PREV(gbuf0, 0, A);
    FETCH(7, tile0);
    vec_component<C, BX, BY, BZ, MIXED>(tile1, gbuf1, tid, lx, ly, lz, 1, a.fd, ids, A);
    LAND(tile0);
    __syncthreads();
    MIXED_PREV(gbuf1, 1, A);
    FETCH(1, tile1);
    vec_component<C, BX, BY, BZ, MIXED>(tile0, gbuf0, tid, lx, ly, lz, 2, a.fd, ids, A);
    LAND(tile1);
    __syncthreads();
    MIXED_PREV(gbuf0, 2, A);
    // magnetic field B = curl A, current j = grad(div A) - lap A: reduce the
    // A bank at once so its 21 values need not stay live
    C Bf[3] = {A.d1[1][2] - A.d1[2][1], A.d1[2][0] - A.d1[0][2], A.d1[0][1] - A.d1[1][0]};
    C J[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        J[i] = (A.diag[i] + A.gdivm[i]) - A.lap[i];
        pin(Bf[i]);
        pin(J[i]);
    }
    FETCH(2, tile0);
    vec_component<C, BX, BY, BZ, MIXED>(tile1, gbuf1, tid, lx, ly, lz, 0, a.fd, ids, U);
    LAND(tile0);
    __syncthreads();
    MIXED_PREV(gbuf1, 0, U);
    FETCH(3, tile1);
    vec_component<C, BX, BY, BZ, MIXED>(tile0, gbuf0, tid, lx, ly, lz, 1, a.fd, ids, U);
    LAND(tile1);
    __syncthreads();
    MIXED_PREV(gbuf0, 1, U);
    FETCH(0, tile0);
    vec_component<C, BX, BY, BZ, MIXED>(tile1, gbuf1, tid, lx, ly, lz, 2, a.fd, ids, U);
    LAND(tile0);
    __syncthreads();
    MIXED_PREV(gbuf1, 2, U);
    FETCH(4, tile1);
    scalar_field<C, B::SY, B::SZ>(tile0, c, a.fd, ids, vl, gl, lapl);
    LAND(tile1);
    __syncthreads();
    // The register (and, at the master policies' last stage, the first-stage
    // register and the FP64 state) of the eight fields is read in batches of
    // NB: a point reads and writes only its own cells, so the reads need not
    // wait for the stores of earlier fields (one memory latency per batch
    // instead of one per field). A batch of all eight is issued by the lanes
    // inside the grid before the last field's derivatives, whose LDS work
    // hides its latency; the FP64 full model has no registers to spare for
    // that and reads two batches of four after phi.
    const int64_t p = g.at(x, y, z);
    const bool last = MASTER && a.stage == 2;
    constexpr int NB = (MODEL == MHD_FULL && sizeof(C) == 8) ? 4 : 8;
    W wold[NB], w1v[NB];
    double mst[NB];
    auto read_regs = [&](int k0) {
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const int k = k0 + j;
            wold[j] = a.stage > 0 ? static_cast<const W *>(a.wrd[k])[p] : W(0);
            w1v[j] = last ? static_cast<const W *>(a.w1[k])[p] : W(0);
            mst[j] = last ? a.master[k][p] : 0.0;
        }
    };
    if constexpr (NB == 8)
        if (live)
            read_regs(0);
    scalar_field<C, B::SY, B::SZ>(tile1, c, a.fd, ids, vs, gs, laps);
#undef MIXED_PREV
#undef FETCH
#undef LAND
    if (!live)
        return;

    MhdBank<C> bank;
    bank.l = vl;
    bank.s = vs;
    bank.lapl = lapl;
    bank.laps = laps;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        bank.gl[i] = gl[i];
        bank.gs[i] = gs[i];
        bank.u[i] = U.val[i];
        bank.lapu[i] = U.lap[i];
        bank.gdivu[i] = U.diag[i] + U.gdivm[i];
        bank.A[i] = A.val[i];
        bank.B[i] = Bf[i];
        bank.J[i] = J[i];
        bank.lapA[i] = A.lap[i];
#pragma unroll
        for (int j = 0; j < 3; ++j)
            bank.du[i][j] = U.d1[i][j];
    }


    // phi: the 8-field right-hand side
    C R[8];
    mhd_phi<MODEL, C>(bank, a.mhd, R);
    const C val[8] = {vl, bank.u[0], bank.u[1], bank.u[2], vs, bank.A[0], bank.A[1], bank.A[2]};
    auto io_of = [&](int k) {
        PointIO io;
        io.fout = a.fout[k];
        io.wrd = a.wrd[k];
        io.wwr = a.wwr[k];
        io.w1 = a.w1[k];
        io.master = a.master[k];
        io.alpha = a.alpha;
        io.beta = a.beta;
        io.dt = a.dt;
        for (int q = 0; q < 3; ++q) io.beta_all[q] = a.beta_all[q];
        io.stage = a.stage;
        io.fuse = a.fuse;
        return io;
    };
    // the point's periodic images, found once for the eight stores (this
    // also freed the FP64 full model's spilled registers); with FP32 storage
    // it measured slower, so that policy finds them per store
    if (sizeof(S) != 4 && images_simple(g)) {
        const PointImages im = point_images(g, x, y, z);
#pragma unroll
        for (int k0 = 0; k0 < 8; k0 += NB) {
            if constexpr (NB < 8)
                read_regs(k0);
#pragma unroll
            for (int j = 0; j < NB; ++j)
                rk_update_pre<S, W, C, MASTER, true>(io_of(k0 + j), g, p, x, y, z, R[k0 + j],
                                                     val[k0 + j], wold[j], w1v[j], mst[j], &im);
        }
    } else {
#pragma unroll
        for (int k0 = 0; k0 < 8; k0 += NB) {
            if constexpr (NB < 8)
                read_regs(k0);
#pragma unroll
            for (int j = 0; j < NB; ++j)
                rk_update_pre<S, W, C, MASTER>(io_of(k0 + j), g, p, x, y, z, R[k0 + j], val[k0 + j],
                                               wold[j], w1v[j], mst[j]);
        }
    }
}

namespace {

template <typename S, typename W, typename C, bool M, int MODEL, int MIXED, int BX, int BY,
          int BZ, int OCC>
int launch_brick(const RkArgs &a, hipStream_t s)
{
    const int gx = (a.g.nx + BX - 1) / BX, gy = (a.g.ny + BY - 1) / BY,
              gz = (a.g.nz + BZ - 1) / BZ;
    const int64_t total = (int64_t)gx * gy * gz;
    if (total > 0x7fffffff)
        return fail(STENCIL_EUNSUPPORTED, "rk_mhd8 (LDS): grid too large");
    hipLaunchKernelGGL((k_rk_mhd8_lds<S, W, C, M, MODEL, MIXED, BX, BY, BZ, OCC>), dim3((unsigned)total),
                       dim3(BX * BY * BZ), 0, s, a, gx, gy, gz);
    return check_launch("rk_mhd8_lds");
}

template <typename S, typename W, typename C, bool M, int MODEL, int MIXED>
int launch_brick_shape(const RkArgs &a, int bx, int by, int bz, int occ, hipStream_t s)
{
#define RK_BRICK(BX_, BY_, BZ_, OCC_)                                                        \
    if (bx == BX_ && by == BY_ && bz == BZ_ && occ == OCC_)                                  \
        return launch_brick<S, W, C, M, MODEL, MIXED, BX_, BY_, BZ_, OCC_>(a, s);
    RK_BRICK_SHAPES(RK_BRICK)
#undef RK_BRICK
    return fail(STENCIL_EUNSUPPORTED, "rk_mhd8 (LDS): brick %dx%dx%d with occupancy %d not built",
                bx, by, bz, occ);
}

} // namespace

template <int MODEL, int MIXED>
int launch_lds_model(int policy, const RkArgs &a, int bx, int by, int bz, int occ, hipStream_t s)
{
    switch (policy) {
    case POL_F64: return launch_brick_shape<double, double, double, false, MODEL, MIXED>(a, bx, by, bz, occ, s);
    case POL_F32_MASTER64: return launch_brick_shape<float, float, float, true, MODEL, MIXED>(a, bx, by, bz, occ, s);
    case POL_BF16_MASTER64: return launch_brick_shape<bf16, float, float, true, MODEL, MIXED>(a, bx, by, bz, occ, s);
    case POL_F32_ONLY: return launch_brick_shape<float, float, float, false, MODEL, MIXED>(a, bx, by, bz, occ, s);
    case POL_BF16_ONLY: return launch_brick_shape<bf16, float, float, false, MODEL, MIXED>(a, bx, by, bz, occ, s);
    }
    return fail(STENCIL_EINVAL, "unknown precision policy %d", policy);
}

} // namespace stn
