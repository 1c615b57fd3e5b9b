// star3d_t2p.hpp -- the two-iteration 3-D star z march (star3d_t2.hpp) with
// its LDS planes in pair layout. Included by star3d.hpp after star3d_t2.hpp.
//
// Each lane owns two adjacent rows. The f0 and f1 planes are stored with y
// fastest (one column of H cells per x), and a lane's two rows sit at an even
// cell index, so the two values a lane needs at any x (its own rows, or two
// consecutive rows of a y tap) are one aligned 2-wide LDS read: 16 bytes in
// FP64, which the LDS serves at about twice the byte rate of 8-byte reads. An
// x tap then costs one read for both rows, a y tap half a read per row. H is
// 2 mod 32 cells, so consecutive lanes (consecutive columns) hit disjoint
// banks. The arithmetic is that of the row-layout kernel, tap for tap, so the
// result is bitwise that of two chained one-iteration launches.
#pragma once

namespace stn {

template <typename C> struct Pair2;
template <> struct Pair2<double> {
    typedef double T __attribute__((ext_vector_type(2)));
};
template <> struct Pair2<float> {
    typedef float T __attribute__((ext_vector_type(2)));
};

template <int R, int TY, int XW> struct PairShape {
    static constexpr int NY = 2;
    static constexpr int TXW = 64 * XW;   // lanes along x
    static constexpr int ROWS = TY * NY;  // lane-grid rows
    static constexpr int LW = TXW + 2 * R; // f0 columns: lane grid plus x halo
    // lane-grid row y sits at cell y + E: E even and >= R, so own pairs start
    // even and the aligned pairs around them cover the y taps
    static constexpr int E = 2 * ((R + 1) / 2);
    static constexpr int HMIN = ROWS + 2 * E; // cells touched by any pair read
    static constexpr int H = HMIN + ((2 - HMIN % 32) + 32) % 32;
    static constexpr int NT = TXW * TY;
    static constexpr int NXH = 2 * R * ROWS; // x-halo cells per f0 plane
    static constexpr int NYH = 2 * R * TXW;  // y-halo cells per f0 plane
    static constexpr int HX_PER = (NXH + NT - 1) / NT;
    static constexpr int HY_PER = (NYH + NT - 1) / NT;
    static_assert(H % 32 == 2 && H >= HMIN, "column height");
};

// One segment (planes z0..z1-1 of tile column (bxi, byi)) of the register-ring
// march of star3d_t2_segment with pair-layout LDS planes.
template <typename S, int R, int TY, int XW, bool IMG, bool BIG>
__device__ __forceinline__ void star3d_t2p_segment(
    const S *__restrict__ in, S *__restrict__ out, const Geo g,
    const StarCoef<typename Store<S>::C, R> cf, int bxi, int byi, int z0, int z1, int flags,
    typename Store<S>::C (&lda)[2][PairShape<R, TY, XW>::LW][PairShape<R, TY, XW>::H],
    typename Store<S>::C (&ldb)[2][PairShape<R, TY, XW>::TXW][PairShape<R, TY, XW>::H])
{
    using C = typename Store<S>::C;
    using P = typename Pair2<C>::T;
    using SH = PairShape<R, TY, XW>;
    constexpr int NY = 2, E = SH::E, H = SH::H;
    // PF planes of loads in flight ahead of the step that consumes them. The
    // march waits on memory latency more than on any unit (about two steps'
    // worth of loads in flight per CU at 3.6 TB/s), so the FP64 launches
    // without images take three (0.366 against 0.396 ms per iteration at
    // 512^3); with image stores or 4-byte storage the longer unrolled round
    // spills, so those keep two (one at r = 1 and r = 4, where the rings of
    // nine-point columns leave no registers for more; three at r = 2).
    constexpr int PF = R == 1 || R == 4 ? 1 : R == 3 ? (IMG || sizeof(S) != 8 ? 2 : 3) : 3;
    constexpr int NR = 2 * R + 1 + PF, NH = PF + 1;
    constexpr int U = lcm_int(NR, NH); // steps per unrolled round: whole turns of both rings
    constexpr int NP = (R + 1) / 2; // y-tap pairs on each side of the own pair
    constexpr uint32_t es = sizeof(S);
    const PlaneSrc<S, BIG> src(in, g.sz, uint64_t(padded_elems(g)));
    constexpr int OX = SH::TXW - 2 * R, OY = SH::ROWS - 2 * R;

    const int tx = threadIdx.x, ty = threadIdx.y;
    const int tid = tx + SH::TXW * ty;
    const int r0 = ty * NY; // the lane's first lane-grid row
    const int fx0 = bxi * OX - R, fy0 = byi * OY - R;
    constexpr bool fuse = IMG; // write the output's periodic images

    auto col = [&](int xx, int yy) {
        return uint32_t(wrap_mod(xx, g.nx) + g.ox + g.sy * (wrap_mod(yy, g.ny) + g.ry)) * es;
    };
    auto pair = [](const C *p) { return *reinterpret_cast<const P *>(p); };

    uint32_t col_off[NY];
#pragma unroll
    for (int j = 0; j < NY; ++j) col_off[j] = col(fx0 + tx, fy0 + r0 + j);

    // halo cells of f0 (as in the row layout, star: no corners); a lane
    // without one writes its own first cell, before its pair lands there
    const int own = (tx + R) * H + r0 + E;
    uint32_t hx_off[SH::HX_PER], hy_off[SH::HY_PER];
    int hx_dst[SH::HX_PER], hy_dst[SH::HY_PER];
#pragma unroll
    for (int k = 0; k < SH::HX_PER; ++k) {
        const int cidx = tid + k * SH::NT;
        if (cidx < SH::NXH) {
            const int row = cidx / (2 * R), e = cidx % (2 * R);
            const int lc = e < R ? e : SH::TXW + e; // LDS column
            hx_off[k] = col(fx0 - R + lc, fy0 + row);
            hx_dst[k] = lc * H + row + E;
        } else {
            hx_off[k] = 0;
            hx_dst[k] = own;
        }
    }
#pragma unroll
    for (int k = 0; k < SH::HY_PER; ++k) {
        const int cidx = tid + k * SH::NT;
        if (cidx < SH::NYH) {
            const int e = cidx / SH::TXW, cc = cidx % SH::TXW;
            const int yr = e < R ? e - R : SH::ROWS + e - R; // lane-grid row
            hy_off[k] = col(fx0 + cc, fy0 + yr);
            hy_dst[k] = (cc + R) * H + yr + E;
        } else {
            hy_off[k] = 0;
            hy_dst[k] = own;
        }
    }

    // Register rings: f0 / f1 plane p in slot (p - zs + R) mod NR, the f0
    // halo of plane p in slot (p - zs) mod NH; the march is unrolled by U
    // steps so every slot index is a compile-time constant.
    const int zs = z0 - R, ze = z1 + R; // steps zA; stage B is live from zA = z0 + R + 1 on
    C ring[NY][NR], r1[NY][NR];
    C hxr[NH][SH::HX_PER], hyr[NH][SH::HY_PER];
#pragma unroll
    for (int j = 0; j < NY; ++j)
#pragma unroll
        for (int k = 0; k < NR; ++k) r1[j][k] = 0;
#pragma unroll
    for (int k = 0; k < 2 * R + PF; ++k)
#pragma unroll
        for (int j = 0; j < NY; ++j)
            ring[j][k] = plane_ld<S>(src.plane(wrap_mod(zs - R + k, g.nz) + g.rz), col_off[j]);
#pragma unroll
    for (int q = 0; q < PF; ++q) {
#pragma unroll
        for (int k = 0; k < SH::HX_PER; ++k) hxr[q][k] = plane_ld<S>(src.plane(wrap_mod(zs + q, g.nz) + g.rz), hx_off[k]);
#pragma unroll
        for (int k = 0; k < SH::HY_PER; ++k) hyr[q][k] = plane_ld<S>(src.plane(wrap_mod(zs + q, g.nz) + g.rz), hy_off[k]);
    }
    const bool xin = tx >= R && tx < SH::TXW - R;                 // stage B lanes
    const bool yin = r0 + 1 >= R && r0 < SH::ROWS - R;            // a stage-B row
    for (int zb = zs; zb <= ze; zb += U) {
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int zA = zb + q;
            if (zA > ze)
                break;
            const int b = (zA - zs) & 1;
            C *la = &lda[b][0][0];
#define F0(k_) ((q + R + (k_) + 2 * NR) % NR)
#define F1(k_) ((q - 1 + (k_) + 2 * NR) % NR)
#pragma unroll
            for (int k = 0; k < SH::HX_PER; ++k) la[hx_dst[k]] = hxr[q % NH][k];
#pragma unroll
            for (int k = 0; k < SH::HY_PER; ++k) la[hy_dst[k]] = hyr[q % NH][k];
            {
                P v0, v1;
                v0.x = ring[0][F0(0)];
                v0.y = ring[1][F0(0)];
                v1.x = r1[0][F1(0)];
                v1.y = r1[1][F1(0)];
                *reinterpret_cast<P *>(&lda[b][tx + R][r0 + E]) = v0;
                *reinterpret_cast<P *>(&ldb[b][tx][r0 + E]) = v1;
            }
            __syncthreads();

            {
                // plane zA + R + PF into the slot of plane zA - R - 1, halo of
                // plane zA + PF likewise; zA >= -R and a periodic axis holds
                // at least R planes, so zA + PF + nz >= 0 (unsigned remainder)
                const uint32_t nzu = uint32_t(g.nz), zu = uint32_t(zA + PF + g.nz);
                const PlaneRef bw = src.plane(int((zu + R) % nzu) + g.rz);
                const PlaneRef bh = src.plane(int(zu % nzu) + g.rz);
#pragma unroll
                for (int j = 0; j < NY; ++j) ring[j][F0(R + PF)] = plane_ld<S>(bw, col_off[j]);
#pragma unroll
                for (int k = 0; k < SH::HX_PER; ++k) hxr[(q + PF) % NH][k] = plane_ld<S>(bh, hx_off[k]);
#pragma unroll
                for (int k = 0; k < SH::HY_PER; ++k) hyr[(q + PF) % NH][k] = plane_ld<S>(bh, hy_off[k]);
            }

            // stage B: f2 at plane zB from the f1 ring and f1's plane in LDS
            const int zB = zA - 1 - R;
            if (zB >= z0 && xin && yin) {
                P xm[R], xp[R], ym[NP], yp[NP];
#pragma unroll
                for (int m = 1; m <= R; ++m) {
                    xm[m - 1] = pair(&ldb[b][tx - m][r0 + E]);
                    xp[m - 1] = pair(&ldb[b][tx + m][r0 + E]);
                }
#pragma unroll
                for (int t = 1; t <= NP; ++t) {
                    ym[t - 1] = pair(&ldb[b][tx][r0 + E - 2 * t]);
                    yp[t - 1] = pair(&ldb[b][tx][r0 + E + 2 * t]);
                }
#pragma unroll
                for (int j = 0; j < NY; ++j) {
                    const int row = r0 + j;
                    const int xo = fx0 + tx, yo = fy0 + row;
                    if (row >= R && row < SH::ROWS - R && xo < g.nx && yo < g.ny) {
                        C acc = cf.c0 * r1[j][F1(0)];
#pragma unroll
                        for (int m = 1; m <= R; ++m) {
                            acc = fma(cf.zm[m - 1], r1[j][F1(-m)], acc);
                            acc = fma(cf.zp[m - 1], r1[j][F1(m)], acc);
                        }
#pragma unroll
                        for (int m = 1; m <= R; ++m) {
                            acc = fma(cf.xm[m - 1], j ? xm[m - 1].y : xm[m - 1].x, acc);
                            acc = fma(cf.xp[m - 1], j ? xp[m - 1].y : xp[m - 1].x, acc);
                        }
#pragma unroll
                        for (int m = 1; m <= R; ++m) {
                            // rows j - m and j + m relative to r0: own pair in
                            // registers, others in the pair holding them
                            const int dm = j - m, dp = j + m;
                            const C vm = dm >= 0 ? r1[dm >= 0 ? dm : 0][F1(0)]
                                                 : ((-dm + 1) / 2 <= NP
                                                        ? (((dm % 2) != 0) ? ym[(-dm + 1) / 2 - 1].y
                                                                           : ym[(-dm + 1) / 2 - 1].x)
                                                        : C(0));
                            const C vp = dp < NY ? r1[dp < NY ? dp : 0][F1(0)]
                                                 : (dp / 2 <= NP ? ((dp % 2) ? yp[dp / 2 - 1].y
                                                                             : yp[dp / 2 - 1].x)
                                                                 : C(0));
                            acc = fma(cf.ym[m - 1], vm, acc);
                            acc = fma(cf.yp[m - 1], vp, acc);
                        }
                        store_periodic(out, g, xo, yo, zB, acc, fuse);
                    }
                }
            }

            // stage A: f1 at plane zA on the whole lane grid
            {
                P xm[R], xp[R], ym[NP], yp[NP];
#pragma unroll
                for (int m = 1; m <= R; ++m) {
                    xm[m - 1] = pair(&lda[b][tx + R - m][r0 + E]);
                    xp[m - 1] = pair(&lda[b][tx + R + m][r0 + E]);
                }
#pragma unroll
                for (int t = 1; t <= NP; ++t) {
                    ym[t - 1] = pair(&lda[b][tx + R][r0 + E - 2 * t]);
                    yp[t - 1] = pair(&lda[b][tx + R][r0 + E + 2 * t]);
                }
#pragma unroll
                for (int j = 0; j < NY; ++j) {
                    C acc = cf.c0 * ring[j][F0(0)];
#pragma unroll
                    for (int m = 1; m <= R; ++m) {
                        acc = fma(cf.zm[m - 1], ring[j][F0(-m)], acc);
                        acc = fma(cf.zp[m - 1], ring[j][F0(m)], acc);
                    }
#pragma unroll
                    for (int m = 1; m <= R; ++m) {
                        acc = fma(cf.xm[m - 1], j ? xm[m - 1].y : xm[m - 1].x, acc);
                        acc = fma(cf.xp[m - 1], j ? xp[m - 1].y : xp[m - 1].x, acc);
                    }
#pragma unroll
                    for (int m = 1; m <= R; ++m) {
                        const int dm = j - m, dp = j + m;
                        const C vm = dm >= 0 ? ring[dm >= 0 ? dm : 0][F0(0)]
                                             : ((-dm + 1) / 2 <= NP
                                                    ? (((dm % 2) != 0) ? ym[(-dm + 1) / 2 - 1].y
                                                                       : ym[(-dm + 1) / 2 - 1].x)
                                                    : C(0));
                        const C vp = dp < NY ? ring[dp < NY ? dp : 0][F0(0)]
                                             : (dp / 2 <= NP ? ((dp % 2) ? yp[dp / 2 - 1].y
                                                                         : yp[dp / 2 - 1].x)
                                                             : C(0));
                        acc = fma(cf.ym[m - 1], vm, acc);
                        acc = fma(cf.yp[m - 1], vp, acc);
                    }
                    r1[j][F0(0)] = RoundS<S>::f(acc); // f1 plane zA: same slot rule as f0
                }
            }
#undef F0
#undef F1
        }
    }
}

// Workgroup = (tile column, z chunk of lz planes), gx * gy * gz of them;
// IMG as in k_star3d_t2.
template <typename S, int R, int TY, int XW, bool IMG, bool BIG>
__global__ void __launch_bounds__(64 * XW * TY, (t2_min_waves<S, XW, TY, IMG>()))
    k_star3d_t2p(const S *__restrict__ in, S *__restrict__ out, Geo g,
                 StarCoef<typename Store<S>::C, R> cf, int lz, int gx, int gy, int gz, int flags)
{
    using C = typename Store<S>::C;
    using SH = PairShape<R, TY, XW>;
    __shared__ __attribute__((aligned(16))) C lda[2][SH::LW][SH::H];   // f0 plane zA, x/y halo
    __shared__ __attribute__((aligned(16))) C ldb[2][SH::TXW][SH::H];  // f1 plane zB

    int lin = blockIdx.x;
    const int total = gx * gy * gz;
    if (flags & STAR_FLAG_XCD) lin = xcd_remap(lin, total);
    const bool yfirst = (flags & STAR_FLAG_YFIRST) != 0;
    const int byi = yfirst ? lin % gy : (lin / gx) % gy;
    const int bxi = yfirst ? (lin / gy) % gx : lin % gx;
    const int z0 = (lin / (gx * gy)) * lz;
    star3d_t2p_segment<S, R, TY, XW, IMG, BIG>(in, out, g, cf, bxi, byi, z0, min(z0 + lz, g.nz), flags, lda,
                                     ldb);
}

} // namespace stn
