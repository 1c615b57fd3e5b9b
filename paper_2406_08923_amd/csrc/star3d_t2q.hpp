// star3d_t2q.hpp -- the two-iteration 3-D star z march with its LDS planes in
// quad layout, for 4-byte arithmetic (FP32 and BF16 storage). Included by
// star3d.hpp after star3d_t2p.hpp.
//
// The FP32 counterpart of the pair layout: each lane owns four adjacent rows,
// the f0 and f1 planes are stored y fastest (one column of H cells per x) and
// a lane's four rows sit at a cell index divisible by four, so its values at
// any x, or the four rows above or below its own, are one aligned 16-byte LDS
// read. An x tap costs one read for four rows; the y taps of radius up to 4
// need the quad below and the quad above the own one. H is 4 mod 32 cells, so
// the 16-byte reads of consecutive lanes (consecutive columns) hit disjoint
// banks. The taps are summed in the order of the row-layout kernel, so the
// result is bitwise that of two chained one-iteration launches.
#pragma once

namespace stn {

template <int R, int TY> struct QuadShape {
    static constexpr int NY = 4;
    static constexpr int TXW = 64;          // lanes along x (one wave per row of lanes)
    static constexpr int ROWS = TY * NY;    // lane-grid rows
    static constexpr int LW = TXW + 2 * R;  // f0 columns: lane grid plus x halo
    static constexpr int E = 4;             // lane-grid row y sits at cell y + E (r <= 4)
    static constexpr int HMIN = ROWS + 2 * E;
    static constexpr int H = HMIN + ((4 - HMIN % 32) + 32) % 32;
    static constexpr int NT = TXW * TY;
    static constexpr int NXH = 2 * R * ROWS; // x-halo cells per f0 plane
    static constexpr int NYH = 2 * R * TXW;  // y-halo cells per f0 plane
    static constexpr int HX_PER = (NXH + NT - 1) / NT;
    static constexpr int HY_PER = (NYH + NT - 1) / NT;
    static_assert(R <= E && H % 32 == 4 && H >= HMIN, "column height");
};

// One segment (planes z0..z1-1 of tile column (bxi, byi)) of the register-ring
// march with quad-layout LDS planes; the structure of star3d_t2p_segment with
// four rows per lane.
template <typename S, int R, int TY, bool IMG, bool BIG>
__device__ __forceinline__ void star3d_t2q_segment(
    const S *__restrict__ in, S *__restrict__ out, const Geo g, const StarCoef<float, R> cf,
    int bxi, int byi, int z0, int z1,
    float (&lda)[2][QuadShape<R, TY>::LW][QuadShape<R, TY>::H],
    float (&ldb)[2][QuadShape<R, TY>::TXW][QuadShape<R, TY>::H])
{
    using C = float;
    static_assert(sizeof(typename Store<S>::C) == 4, "quad layout: 4-byte arithmetic");
    typedef float Q __attribute__((ext_vector_type(4)));
    using SH = QuadShape<R, TY>;
    constexpr int NY = 4, E = SH::E, H = SH::H;
    constexpr int PF = R == 1 ? 1 : R == 3 ? 2 : 3; // PF + 1 divides 2R
    constexpr int NR = 2 * R + 1 + PF, NH = PF + 1;
    static_assert(NR % NH == 0, "the unrolled march must cover whole halo rings");
    constexpr uint32_t es = sizeof(S);
    const PlaneSrc<S, BIG> src(in, g.sz, uint64_t(padded_elems(g)));
    constexpr int OX = SH::TXW - 2 * R, OY = SH::ROWS - 2 * R;

    const int tx = threadIdx.x, ty = threadIdx.y;
    const int tid = tx + SH::TXW * ty;
    const int r0 = ty * NY; // the lane's first lane-grid row
    const int fx0 = bxi * OX - R, fy0 = byi * OY - R;
    constexpr bool fuse = IMG;

    auto col = [&](int xx, int yy) {
        return uint32_t(wrap_mod(xx, g.nx) + g.ox + g.sy * (wrap_mod(yy, g.ny) + g.ry)) * es;
    };
    auto quad = [](const C *p) { return *reinterpret_cast<const Q *>(p); };

    uint32_t col_off[NY];
#pragma unroll
    for (int j = 0; j < NY; ++j) col_off[j] = col(fx0 + tx, fy0 + r0 + j);

    // halo cells of f0 (no corners); a lane without one writes its own first
    // cell, before its quad lands there
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
    // halo of plane p in slot (p - zs) mod NH; the march is unrolled by NR
    // steps so every slot index is a compile-time constant.
    const int zs = z0 - R, ze = z1 + R;
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
    const bool xin = tx >= R && tx < SH::TXW - R;       // stage B lanes
    const bool yin = r0 + NY - 1 >= R && r0 < SH::ROWS - R; // a stage-B row
    // the steps of a round are expanded by static_for: the body is too large
    // for the loop unroller, and a rolled round would index the rings at run
    // time (registers spilled to scratch)
    int zb = zs;
    auto step = [&](auto qc) {
        constexpr int q = decltype(qc)::value;
        const int zA = zb + q;
        if (zA > ze)
            return;
        const int b = (zA - zs) & 1;
        C *la = &lda[b][0][0];
#define F0(k_) ((q + R + (k_) + 2 * NR) % NR)
#define F1(k_) ((q - 1 + (k_) + 2 * NR) % NR)
#pragma unroll
        for (int k = 0; k < SH::HX_PER; ++k) la[hx_dst[k]] = hxr[q % NH][k];
#pragma unroll
        for (int k = 0; k < SH::HY_PER; ++k) la[hy_dst[k]] = hyr[q % NH][k];
        {
            Q v0, v1;
#pragma unroll
            for (int j = 0; j < NY; ++j) {
                v0[j] = ring[j][F0(0)];
                v1[j] = r1[j][F1(0)];
            }
            *reinterpret_cast<Q *>(&lda[b][tx + R][r0 + E]) = v0;
            *reinterpret_cast<Q *>(&ldb[b][tx][r0 + E]) = v1;
        }
        __syncthreads();

        {
            // plane zA + R + PF into the slot of plane zA - R - 1, halo of
            // plane zA + PF likewise (unsigned remainder: zA + PF + nz >= 0)
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

        // row j - m (m >= 1) of the own quad, else of the quad below;
        // row j + m of the own quad, else of the quad above
        auto ytap = [](const C (&own4)[NY], const Q &lo, const Q &hi, int j, int m, bool up) {
            const int d = up ? j + m : j - m;
            return up ? (d < NY ? own4[d < NY ? d : 0] : hi[d < NY ? 0 : d - NY])
                      : (d >= 0 ? own4[d >= 0 ? d : 0] : lo[d >= 0 ? 0 : d + NY]);
        };

        // stage B: f2 at plane zB from the f1 ring and f1's plane in LDS
        const int zB = zA - 1 - R;
        if (zB >= z0 && xin && yin) {
            Q xm[R], xp[R];
#pragma unroll
            for (int m = 1; m <= R; ++m) {
                xm[m - 1] = quad(&ldb[b][tx - m][r0 + E]);
                xp[m - 1] = quad(&ldb[b][tx + m][r0 + E]);
            }
            const Q ylo = quad(&ldb[b][tx][r0 + E - 4]), yhi = quad(&ldb[b][tx][r0 + E + 4]);
            C own4[NY];
#pragma unroll
            for (int j = 0; j < NY; ++j) own4[j] = r1[j][F1(0)];
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
                        acc = fma(cf.xm[m - 1], xm[m - 1][j], acc);
                        acc = fma(cf.xp[m - 1], xp[m - 1][j], acc);
                    }
#pragma unroll
                    for (int m = 1; m <= R; ++m) {
                        acc = fma(cf.ym[m - 1], ytap(own4, ylo, yhi, j, m, false), acc);
                        acc = fma(cf.yp[m - 1], ytap(own4, ylo, yhi, j, m, true), acc);
                    }
                    store_periodic(out, g, xo, yo, zB, acc, fuse);
                }
            }
        }

        // stage A: f1 at plane zA on the whole lane grid
        {
            Q xm[R], xp[R];
#pragma unroll
            for (int m = 1; m <= R; ++m) {
                xm[m - 1] = quad(&lda[b][tx + R - m][r0 + E]);
                xp[m - 1] = quad(&lda[b][tx + R + m][r0 + E]);
            }
            const Q ylo = quad(&lda[b][tx + R][r0 + E - 4]),
                    yhi = quad(&lda[b][tx + R][r0 + E + 4]);
            C own4[NY];
#pragma unroll
            for (int j = 0; j < NY; ++j) own4[j] = ring[j][F0(0)];
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
                    acc = fma(cf.xm[m - 1], xm[m - 1][j], acc);
                    acc = fma(cf.xp[m - 1], xp[m - 1][j], acc);
                }
#pragma unroll
                for (int m = 1; m <= R; ++m) {
                    acc = fma(cf.ym[m - 1], ytap(own4, ylo, yhi, j, m, false), acc);
                    acc = fma(cf.yp[m - 1], ytap(own4, ylo, yhi, j, m, true), acc);
                }
                r1[j][F0(0)] = RoundS<S>::f(acc); // f1 plane zA: same slot rule as f0
            }
        }
#undef F0
#undef F1
    };
    for (; zb <= ze; zb += NR)
        static_for<NR>(step);
}

// Workgroup = (tile column, z chunk of lz planes); 64 x TY lanes.
template <typename S, int R, int TY, bool IMG, bool BIG>
__global__ void __launch_bounds__(64 * TY)
    k_star3d_t2q(const S *__restrict__ in, S *__restrict__ out, Geo g, StarCoef<float, R> cf,
                 int lz, int gx, int gy, int gz, int flags)
{
    using SH = QuadShape<R, TY>;
    __shared__ __attribute__((aligned(16))) float lda[2][SH::LW][SH::H];  // f0 plane zA, x/y halo
    __shared__ __attribute__((aligned(16))) float ldb[2][SH::TXW][SH::H]; // f1 plane zB

    int lin = blockIdx.x;
    const int total = gx * gy * gz;
    if (flags & STAR_FLAG_XCD) lin = xcd_remap(lin, total);
    const bool yfirst = (flags & STAR_FLAG_YFIRST) != 0;
    const int byi = yfirst ? lin % gy : (lin / gx) % gy;
    const int bxi = yfirst ? (lin / gy) % gx : lin % gx;
    const int z0 = (lin / (gx * gy)) * lz;
    star3d_t2q_segment<S, R, TY, IMG, BIG>(in, out, g, cf, bxi, byi, z0, min(z0 + lz, g.nz), lda,
                                           ldb);
}

} // namespace stn
