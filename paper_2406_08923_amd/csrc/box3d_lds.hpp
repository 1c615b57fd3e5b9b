// box3d_lds.hpp -- dense 3-D box cross-correlation of radius R = 1 .. 8 (Eq. 3
// with every tap of the (2R+1)^3 box nonzero: 27 .. 4913 multiply-adds per
// point; from radius 2 on the taps, not HBM, bound the pass), and dense 2-D
// boxes of radius 1 .. 8. The inputs are served from LDS (the shared-memory
// strategy of Sec. 4.1).
//
// A workgroup owns a 64 x (TY*E) block of output columns over lz z planes and
// marches z one input plane at a time: the halo'd input plane, (64 + 2R) x
// (TY*E + 2R) cells, is staged in LDS, and the next plane's loads are in
// flight in registers while the current one is used. Lane (lx, ly) of wave w
// owns the E adjacent outputs x0 + E*lx .. x0 + E*lx + E - 1 of row
// y0 + E*w + ly and keeps per output a register ring of 2R + 1 partial sums:
// input plane p feeds output planes p - R .. p + R (with z tap p - z_out), so
// per row offset dy a lane reads E + 2R inputs from LDS once and uses them for
// (2R+1) x (2R+1) x E multiply-adds (E = 4 or 8; 4 from radius 5 on, where
// the ring holds 11 .. 17 sums). After plane p the output plane p - R is
// complete and stored, and the ring moves by one. The coefficients are read
// one z tap (2R + 1 values) at a time, the next tap's while the current one's
// multiply-adds run: in FP64 through the scalar cache into scalar registers
// (the multiply-adds take them as their scalar operand, and LDS serves only
// the inputs), in FP32 from an LDS copy as wave-uniform vector loads (the
// scalar loads measured slower there: they share a wait counter with the LDS
// reads, and the shorter FP32 multiply-adds hide less of the wait). LDS rows
// are padded by two cells after every E cells, so the vector reads of the
// lanes of a row fall on distinct banks.
//
// A 2-D box (radius 1 .. 8) runs the same march with a ring of one partial
// sum per output (RZ = 0): a workgroup walks lz row blocks of its 64-column
// strip, staging block b + 1 while block b is summed. It writes each block's
// outputs through LDS as whole rows, and so does the 27-point 3-D box, where
// HBM bounds the pass too.
//
// Per output the taps are summed by input plane (z offset -R .. R), then by y
// offset, then by x offset, a fixed order the FP64 tolerance covers. The
// kernel stores the interior only: with (2R+1)^3 multiply-adds per point a
// separate periodic halo pass costs far less than the image stores' registers
// would inside the march.
#pragma once

#include "linear_kernels.hpp"

namespace stn {

template <typename C> struct LdsPair;
template <> struct LdsPair<double> {
    typedef double T __attribute__((ext_vector_type(2)));
};
template <> struct LdsPair<float> {
    typedef float T __attribute__((ext_vector_type(2)));
};

// Lane grid and LDS layout. E outputs per lane along x, so a wave is
// 64 / E lanes wide (64 columns) and E rows tall. RZ: z radius of the box
// (R in 3-D; 0 for a 2-D box, which is one plane with a ring of one sum).
template <int R, int E, int TY, int RZ = R> struct BoxLdsShape {
    static constexpr int K = 2 * R + 1, KZ = 2 * RZ + 1;
    static constexpr int NT = 64 * TY;
    static constexpr int LX = 64 / E;
    static constexpr int TX = 64, TYR = TY * E;              // outputs per plane
    static constexpr int LW = TX + 2 * R, LH = TYR + 2 * R;  // staged cells
    static constexpr int PW = (LW + E - 1) / E * (E + 2);    // padded row (cells)
    static constexpr int PLANE = PW * LH;
    static constexpr int NLD = (LW * LH + NT - 1) / NT;      // staged cells per lane
    static constexpr bool LAST_FULL = LW * LH % NT == 0;
    static __host__ __device__ constexpr int phys(int col) { return col + 2 * (col / E); }
    static_assert(PLANE >= TX * TYR, "a 2-D block's outputs pass through the plane buffer");
};

template <typename S, int R, int E, int TY, bool BIG, int RZ>
__global__ void __launch_bounds__(64 * TY)
    k_box3d_lds(const S *__restrict__ in, S *__restrict__ out, Geo g,
                const typename Store<S>::C *__restrict__ cg, int lz, int gx, int gy, int gz,
                int flags)
{
    using C = typename Store<S>::C;
    using P2 = typename LdsPair<C>::T;
    using SH = BoxLdsShape<R, E, TY, RZ>;
    constexpr int K = SH::K, KZ = SH::KZ, NT = SH::NT, NV = E + 2 * R;
    constexpr uint32_t es = sizeof(S);
    constexpr bool SCOEF = sizeof(C) == 8; // coefficients in scalar registers
    // outputs stored as whole rows through LDS: where HBM, not the taps,
    // bounds the pass (2-D boxes, the 27-point 3-D box)
    constexpr bool ROWSTORE = RZ == 0 || R == 1;
    __shared__ __attribute__((aligned(16))) C plane[SH::PLANE];
    // LDS copy of the taps (FP32): rows of one z tap padded to four cells, so
    // that one ds_read_b128 brings four taps
    constexpr int KQ = (K + 3) / 4 * 4, CQ = KZ * KQ;
    typedef C Q4 __attribute__((ext_vector_type(4)));
    __shared__ __attribute__((aligned(16))) C cl[SCOEF ? 4 : K * CQ];

    int lin = blockIdx.x;
    const int total = gx * gy * gz;
    if (flags & STAR_FLAG_XCD) lin = xcd_remap(lin, total);
    const int bxi = lin % gx, byi = (lin / gx) % gy, bzi = lin / (gx * gy);
    const int tid = threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6;
    const int lx = lane % SH::LX, ly = lane / SH::LX;
    const int x0 = bxi * SH::TX;
    // 3-D: planes z0 .. z1 - 1 of the row block y0; 2-D (RZ = 0): the
    // "planes" are the lz row blocks z0 .. z1 - 1 of the column, each TYR
    // rows, marched the same way so that one block's loads overlap the
    // previous block's multiply-adds
    const int nzb = RZ == 0 ? (g.ny + SH::TYR - 1) / SH::TYR : g.nz;
    const int y0 = RZ == 0 ? 0 : byi * SH::TYR;
    const int z0 = bzi * lz, z1 = min(z0 + lz, nzb);

    // coefficients of y offset dy: cl[dy * CQ + dz * KQ + dx] = c[dz][dy][dx]
    // (the dense box in z, y, x order); the pad cells of each row are zero
    if constexpr (!SCOEF)
        for (int i = tid; i < K * CQ; i += NT) {
            const int dx = i % KQ, dz = (i / KQ) % KZ, dy = i / CQ;
            cl[i] = dx < K ? cg[(dz * K + dy) * K + dx] : C(0);
        }

    // the cells this lane stages: byte offset within an input plane and LDS
    // index (coordinates clamped into the padded array; clamped cells only
    // feed outputs past the grid, which are not stored)
    // (3-D: goff is the whole offset within a plane; 2-D: the column part,
    // and srow the staged row, whose offset follows the row block)
    uint32_t goff[SH::NLD];
    int ldst[SH::NLD], srow[SH::NLD];
#pragma unroll
    for (int q = 0; q < SH::NLD; ++q) {
        const int t = min(tid + NT * q, SH::LW * SH::LH - 1);
        const int row = t / SH::LW, col = t % SH::LW;
        const int xs = min(x0 - R + col, g.nx + R - 1), ys = min(y0 - R + row, g.ny + R - 1);
        goff[q] = RZ == 0 ? uint32_t(xs + g.ox) : uint32_t(xs + g.ox + g.sy * (ys + g.ry)) * es;
        srow[q] = row;
        ldst[q] = row * SH::PW + SH::phys(col);
    }
    const bool last_ok = SH::LAST_FULL || tid + NT * (SH::NLD - 1) < SH::LW * SH::LH;
    const PlaneSrc<S, BIG> src(in, g.sz, uint64_t(padded_elems(g)));
    C stage[SH::NLD];
    auto fetch = [&](int zin) {
        if constexpr (RZ == 0) {
            const PlaneRef pb = src.plane(0);
            const int yb = zin * SH::TYR - R; // first staged row of block zin
#pragma unroll
            for (int q = 0; q < SH::NLD; ++q) {
                const int ys = min(yb + srow[q], g.ny + R - 1);
                stage[q] = plane_ld<S>(pb, uint32_t(goff[q] + g.sy * (ys + g.ry)) * es);
            }
        } else {
            const PlaneRef pb = src.plane(zin + g.rz);
#pragma unroll
            for (int q = 0; q < SH::NLD; ++q)
                stage[q] = plane_ld<S>(pb, goff[q]);
        }
    };

    C acc[KZ][E];
#pragma unroll
    for (int k = 0; k < KZ; ++k)
#pragma unroll
        for (int e = 0; e < E; ++e) acc[k][e] = C(0);

    const int zs = z0 - RZ, ze = z1 + RZ; // input planes zs .. ze - 1
    const int row0 = wv * E + ly;       // LDS row of the lane's inputs at y offset -R
    const int colp = lx * (E + 2);      // padded LDS column of its first input
    const int xo = x0 + lx * E;
    fetch(zs);
    for (int p = zs; p < ze; ++p) {
        __syncthreads(); // every wave is done with plane p - 1
#pragma unroll
        for (int q = 0; q < SH::NLD; ++q)
            if (q < SH::NLD - 1 || last_ok)
                plane[ldst[q]] = stage[q];
        __syncthreads();
        if (p + 1 < ze)
            fetch(p + 1);
#pragma unroll 1
        for (int dy = 0; dy < K; ++dy) {
            const C *rp = plane + (row0 + dy) * SH::PW + colp;
            C v[NV];
            static_for<NV / 2>([&](auto jj) {
                constexpr int j = 2 * jj;
                const P2 t = *reinterpret_cast<const P2 *>(rp + SH::phys(j));
                v[j] = t.x;
                v[j + 1] = t.y;
            });
            // slot k holds output plane p - R + k, whose z tap here is 2R - k;
            // the coefficients of one z tap are loaded while the previous
            // tap's multiply-adds run (a scheduling barrier per tap keeps
            // the compiler from loading all (2R+1)^2 at once)
            const C *cb = cl + dy * CQ;     // LDS copy: c[dz][dy][dx] at dz KQ + dx
            const C *cq = cg + dy * K;      // device: c[dz][dy][dx] at dz K^2 + dx
            auto ldc = [&](int dz, C (&c)[KQ]) {
                if constexpr (SCOEF) {
                    static_for<K>([&](auto dx) { c[dx] = cq[dz * K * K + dx]; });
                } else {
                    static_for<KQ / 4>([&](auto ii) {
                        const Q4 t = *reinterpret_cast<const Q4 *>(cb + dz * KQ + 4 * ii);
                        c[4 * ii] = t.x;
                        c[4 * ii + 1] = t.y;
                        c[4 * ii + 2] = t.z;
                        c[4 * ii + 3] = t.w;
                    });
                }
            };
            C cc[2][KQ];
            ldc(2 * RZ, cc[0]);
            static_for<KZ>([&](auto kk) {
                constexpr int k = kk;
                if constexpr (k + 1 < KZ)
                    ldc(2 * RZ - k - 1, cc[(k + 1) & 1]);
                static_for<K>([&](auto dx) {
                    static_for<E>([&](auto e) {
                        acc[k][e] = fma(cc[k & 1][dx], v[e + dx], acc[k][e]);
                    });
                });
                __builtin_amdgcn_sched_barrier(0);
            });
        }
        const int zo = p - RZ; // complete
        if constexpr (ROWSTORE) {
            // the completed outputs go out through LDS, so that each store
            // instruction of a wave writes 64 consecutive cells of a row (a
            // lane's E adjacent outputs would otherwise be E stores at a
            // stride of E cells). The plane is free once every wave has
            // summed it; the next landing waits at the loop head's barrier.
            // (zo >= z0 is uniform over the workgroup.)
            if (zo >= z0) {
                __syncthreads();
#pragma unroll
                for (int e = 0; e < E; ++e)
                    plane[row0 * SH::TX + lx * E + e] = acc[0][e];
                __syncthreads();
                const int yb = RZ == 0 ? zo * SH::TYR : y0;
#pragma unroll
                for (int i = tid; i < SH::TX * SH::TYR; i += NT) {
                    const int x = x0 + i % SH::TX, y = yb + i / SH::TX;
                    if (x < g.nx && y < g.ny)
                        Store<S>::st(out + g.at(x, y, RZ == 0 ? 0 : zo), plane[i]);
                }
            }
        } else {
            const int y = y0 + row0;
            if (zo >= z0 && y < g.ny) {
                S *o = out + g.at(xo, y, zo);
#pragma unroll
                for (int e = 0; e < E; ++e)
                    if (xo + e < g.nx)
                        Store<S>::st(o + e, acc[0][e]);
            }
        }
#pragma unroll
        for (int k = 0; k + 1 < KZ; ++k)
#pragma unroll
            for (int e = 0; e < E; ++e) acc[k][e] = acc[k + 1][e];
#pragma unroll
        for (int e = 0; e < E; ++e) acc[KZ - 1][e] = C(0);
    }
}

// Outputs per lane along x (E) and waves per workgroup (TY) that are built
// (8 waves only for the HBM-bound forms: 2-D boxes and the 27-point box).
#define BOX3D_LDS_SHAPES(X) X(4, 4) X(8, 4) X(4, 8) X(8, 8)

template <typename S, int R, int E, int TY, int RZ>
int launch_box3d_lds_t(const S *in, S *out, const Geo &g, const typename Store<S>::C *cf, int lz,
                       int flags, hipStream_t s)
{
    using SH = BoxLdsShape<R, E, TY, RZ>;
    const int nby = (g.ny + SH::TYR - 1) / SH::TYR;
    // 2-D: a workgroup marches lz row blocks of its 64-column strip
    const int gx = (g.nx + SH::TX - 1) / SH::TX, gy = RZ == 0 ? 1 : nby,
              gz = RZ == 0 ? (nby + lz - 1) / lz : (g.nz + lz - 1) / lz;
    const int64_t total = (int64_t)gx * gy * gz;
    if (total > 0x7fffffff)
        return fail(STENCIL_EUNSUPPORTED, "box3d (LDS): grid too large");
    const bool big = uint64_t(padded_elems(g)) * sizeof(S) >= (uint64_t(1) << 32);
    if (big)
        hipLaunchKernelGGL((k_box3d_lds<S, R, E, TY, true, RZ>), dim3((unsigned)total), dim3(SH::NT),
                           0, s, in, out, g, cf, lz, gx, gy, gz, flags);
    else
        hipLaunchKernelGGL((k_box3d_lds<S, R, E, TY, false, RZ>), dim3((unsigned)total), dim3(SH::NT),
                           0, s, in, out, g, cf, lz, gx, gy, gz, flags);
    return check_launch("xcorr_box3d_lds");
}

template <typename S, int R, int RZ>
int launch_box3d_lds_r(const S *in, S *out, const Geo &g, const typename Store<S>::C *cf, int e,
                       int ty, int lz, int flags, hipStream_t s)
{
// (3-D rings of 11 .. 17 sums at radius 5 .. 8 leave registers for 4 outputs
// per lane only)
#define BOX3D_LDS_CASE(E_, TY_)                                                              \
    if constexpr ((RZ < 5 || E_ == 4) && (TY_ == 4 || RZ == 0 || R == 1))                    \
        if (e == E_ && ty == TY_)                                                            \
            return launch_box3d_lds_t<S, R, E_, TY_, RZ>(in, out, g, cf, lz, flags, s);
    BOX3D_LDS_SHAPES(BOX3D_LDS_CASE)
#undef BOX3D_LDS_CASE
    return fail(STENCIL_EUNSUPPORTED, "box3d (LDS): %d outputs per lane with %d waves not built",
                e, ty);
}

template <typename S>
int launch_box3d_lds_impl(const S *in, S *out, const Geo &g, int R, const void *cf, int e, int ty,
                          int lz, int flags, hipStream_t s)
{
    using C = typename Store<S>::C;
    const C *c = static_cast<const C *>(cf);
    if ((g.ndim != 3 && g.ndim != 2) || R > g.r || cf == nullptr)
        return fail(STENCIL_EINVAL, "box (LDS): needs a 2-D or 3-D box within the padding and "
                                    "its coefficients on the device");
    if (lz < 1)
        return fail(STENCIL_EINVAL, "box (LDS): z planes per workgroup must be >= 1");
    if (g.ndim == 2) {
        if (uint64_t(padded_elems(g)) * sizeof(S) >= (uint64_t(1) << 32))
            return fail(STENCIL_EUNSUPPORTED, "box (LDS): 2-D arrays of 4 GiB or more");
        switch (R) {
        case 1: return launch_box3d_lds_r<S, 1, 0>(in, out, g, c, e, ty, lz, flags, s);
        case 2: return launch_box3d_lds_r<S, 2, 0>(in, out, g, c, e, ty, lz, flags, s);
        case 3: return launch_box3d_lds_r<S, 3, 0>(in, out, g, c, e, ty, lz, flags, s);
        case 4: return launch_box3d_lds_r<S, 4, 0>(in, out, g, c, e, ty, lz, flags, s);
        case 5: return launch_box3d_lds_r<S, 5, 0>(in, out, g, c, e, ty, lz, flags, s);
        case 6: return launch_box3d_lds_r<S, 6, 0>(in, out, g, c, e, ty, lz, flags, s);
        case 7: return launch_box3d_lds_r<S, 7, 0>(in, out, g, c, e, ty, lz, flags, s);
        case 8: return launch_box3d_lds_r<S, 8, 0>(in, out, g, c, e, ty, lz, flags, s);
        default:
            return fail(STENCIL_EUNSUPPORTED, "box (LDS): 2-D radius %d not built (1..8)", R);
        }
    }
    switch (R) {
    case 1: return launch_box3d_lds_r<S, 1, 1>(in, out, g, c, e, ty, lz, flags, s);
    case 2: return launch_box3d_lds_r<S, 2, 2>(in, out, g, c, e, ty, lz, flags, s);
    case 3: return launch_box3d_lds_r<S, 3, 3>(in, out, g, c, e, ty, lz, flags, s);
    case 4: return launch_box3d_lds_r<S, 4, 4>(in, out, g, c, e, ty, lz, flags, s);
    case 5: return launch_box3d_lds_r<S, 5, 5>(in, out, g, c, e, ty, lz, flags, s);
    case 6: return launch_box3d_lds_r<S, 6, 6>(in, out, g, c, e, ty, lz, flags, s);
    case 7: return launch_box3d_lds_r<S, 7, 7>(in, out, g, c, e, ty, lz, flags, s);
    case 8: return launch_box3d_lds_r<S, 8, 8>(in, out, g, c, e, ty, lz, flags, s);
    default:
        return fail(STENCIL_EUNSUPPORTED, "box (LDS): 3-D radius %d not built (1..8)", R);
    }
}

} // namespace stn
