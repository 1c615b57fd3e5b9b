// star3d_t2.hpp -- two chained iterations of the 3-D star cross-correlation in
// one pass over HBM (temporal blocking of the z march), periodic boundaries.
// Included by star3d.hpp.
#pragma once

namespace stn {

// Shapes (XW, TY, NY) built for the two-iteration kernel: the lane grid is
// 64*XW x TY*NY; each tile produces (64*XW - 2R) x (TY*NY - 2R) outputs.
#define STAR_T2_SHAPES(X) X(1, 8, 2) X(1, 16, 1) X(1, 16, 2) X(1, 12, 2) X(2, 8, 2) X(1, 8, 4)

// storage rounding of an intermediate iterate: what a one-iteration launch
// would have stored and the next launch read back
template <typename S> struct RoundS {
    static __device__ __forceinline__ typename Store<S>::C f(typename Store<S>::C v) { return v; }
};
template <> struct RoundS<bf16> {
    static __device__ __forceinline__ float f(float v) { return bf16_to_f32(f32_to_bf16(v)); }
};

__device__ __forceinline__ int wrap_mod(int v, int n)
{
    int m = v % n;
    return m < 0 ? m + n : m;
}

// One segment: planes z0..z1-1 of output column (bxi, byi) of the tile grid.
// Lane (tx, ty) owns column xf = fx0 + tx and rows yf = fy0 + ty*NY + j of the
// lane grid, which is the tile's output region widened by R on every side.
// The workgroup marches a z step zA at a time:
//   * the f0 window (planes zA-R..zA+R of the lane's columns) and f0's plane zA
//     with its x/y halo in LDS give f1 at plane zA on the whole lane grid
//     (stage A), rounded to the storage type and pushed into the lane's f1
//     window;
//   * the f1 window (planes zB-R..zB+R, zB = zA-1-R) and f1's plane zB in LDS
//     give f2 at plane zB on the inner lanes (stage B), stored with its
//     periodic images.
// Stage B runs one plane behind stage A so that a single barrier per step
// covers both LDS planes (each double-buffered). Every f0 read uses wrapped
// interior coordinates, so the input halo is never read and any grid size
// works. Both stages evaluate every point with the taps in the order of the
// one-iteration kernel, so the result is bitwise that of two chained launches.
template <typename S, int R, int NY, int TY, int XW, bool IMG, bool BIG>
__device__ __forceinline__ void star3d_t2_segment(
    const S *__restrict__ in, S *__restrict__ out, const Geo g,
    const StarCoef<typename Store<S>::C, R> cf, int bxi, int byi, int z0, int z1, int flags,
    typename Store<S>::C (&lda)[2][StarShape<R, NY, TY, XW>::LH][StarShape<R, NY, TY, XW>::LW],
    typename Store<S>::C (&ldb)[2][StarShape<R, NY, TY, XW>::ROWS][StarShape<R, NY, TY, XW>::TXW])
{
    using C = typename Store<S>::C;
    using SH = StarShape<R, NY, TY, XW>;
    // Register-ring march (below) for workgroups of up to 768 lanes, r <= 3
    // and up to two rows per lane, where the rings fit the register budget;
    // otherwise the
    // shifting-window march. Planes in flight, ring march: PF + 1 must divide
    // 2R so that the halo ring (PF + 1 slots) divides the f0 ring (2R + 1 + PF
    // slots): 1 for r = 1, 3 for r = 2, 2 for r = 3; shifting-window march: 2.
    constexpr bool RING = 64 * XW * TY <= 768 && R <= 3 && NY <= 2;
    constexpr int PF = !RING ? 2 : R == 1 ? 1 : R == 3 ? 2 : 3;
    constexpr uint32_t es = sizeof(S);
    const PlaneSrc<S, BIG> src(in, g.sz, uint64_t(padded_elems(g)));
    constexpr int OX = SH::TXW - 2 * R, OY = SH::ROWS - 2 * R;

    const int tx = threadIdx.x, ty = threadIdx.y;
    const int tid = tx + SH::TXW * ty;
    const int fx0 = bxi * OX - R, fy0 = byi * OY - R;
    constexpr bool fuse = IMG; // write the output's periodic images

    auto col = [&](int xx, int yy) {
        return uint32_t(wrap_mod(xx, g.nx) + g.ox + g.sy * (wrap_mod(yy, g.ny) + g.ry)) * es;
    };

    uint32_t col_off[NY];
#pragma unroll
    for (int j = 0; j < NY; ++j) col_off[j] = col(fx0 + tx, fy0 + ty * NY + j);

    uint32_t hx_off[SH::HX_PER], hy_off[SH::HY_PER];
    int hx_slot[SH::HX_PER], hy_slot[SH::HY_PER];
#pragma unroll
    for (int k = 0; k < SH::HX_PER; ++k) {
        const int cidx = tid + k * SH::NT;
        if (cidx < SH::NXH) {
            const int row = cidx / (2 * R), e = cidx % (2 * R);
            const int lc = e < R ? e : SH::TXW + e; // LDS column
            hx_off[k] = col(fx0 - R + lc, fy0 + row);
            hx_slot[k] = (row + R) * SH::LW + lc;
        } else {
            hx_off[k] = 0;
            hx_slot[k] = -1;
        }
    }
#pragma unroll
    for (int k = 0; k < SH::HY_PER; ++k) {
        const int cidx = tid + k * SH::NT;
        if (cidx < SH::NYH) {
            const int e = cidx / SH::TXW, cc = cidx % SH::TXW;
            const int lr = e < R ? e : SH::ROWS + e; // LDS row
            hy_off[k] = col(fx0 + cc, fy0 - R + lr);
            hy_slot[k] = lr * SH::LW + cc + R;
        } else {
            hy_off[k] = 0;
            hy_slot[k] = -1;
        }
    }

    if constexpr (RING) {
        // Register rings. f0 plane p and f1 plane p live in slot
        // (p - zs + R) mod NR of ring / r1 (NR = 2R + 1 + PF: the 2R + 1 window
        // planes plus PF planes in flight), the x/y halo of f0 plane p in slot
        // (p - zs) mod (PF + 1) of hxr / hyr. The z march is unrolled by NR steps,
        // a multiple of PF + 1, so every slot index below is a compile-time
        // constant: a load lands in the register its plane is read from, the
        // window advances by renaming, and no register is copied across the loop
        // back-edge (a copy there would wait for a load issued just before).
        constexpr int NR = 2 * R + 1 + PF, NH = PF + 1;
        static_assert(NR % NH == 0, "the unrolled march must cover whole halo rings");
        const int zs = z0 - R, ze = z1 + R; // steps zA; stage B is live from zA = z0 + R + 1 on
        C ring[NY][NR], r1[NY][NR];
        C hxr[NH][SH::HX_PER], hyr[NH][SH::HY_PER];
    #pragma unroll
        for (int j = 0; j < NY; ++j)
    #pragma unroll
            for (int k = 0; k < NR; ++k) r1[j][k] = 0;
        // planes zs - R .. zs + R - 1 (slots 0 .. 2R - 1) and the first PF planes
        // ahead, zs + R .. zs + R + PF - 1 (slots 2R .. 2R + PF - 1)
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

        // Halo cells are written unconditionally: a lane without one writes
        // into its own first interior cell, before the interior value is
        // stored there (one lane's LDS writes complete in program order), so
        // no lane mask is kept live across the march.
        const int own = (ty * NY + R) * SH::LW + tx + R;
        int hx_dst[SH::HX_PER], hy_dst[SH::HY_PER];
    #pragma unroll
        for (int k = 0; k < SH::HX_PER; ++k) hx_dst[k] = hx_slot[k] >= 0 ? hx_slot[k] : own;
    #pragma unroll
        for (int k = 0; k < SH::HY_PER; ++k) hy_dst[k] = hy_slot[k] >= 0 ? hy_slot[k] : own;
        for (int zb = zs; zb <= ze; zb += NR) {
    #pragma unroll
            for (int q = 0; q < NR; ++q) {
                const int zA = zb + q;
                if (zA > ze)
                    break;
                const int b = (zA - zs) & 1;
                C *la = &lda[b][0][0];
                // slots at this step: f0 plane zA + k in (q + R + k) % NR, f1 plane
                // zB + k (zB = zA - 1 - R) in (q - 1 + k) % NR
    #define F0(k_) ((q + R + (k_) + 2 * NR) % NR)
    #define F1(k_) ((q - 1 + (k_) + 2 * NR) % NR)
    #pragma unroll
                for (int k = 0; k < SH::HX_PER; ++k) la[hx_dst[k]] = hxr[q % NH][k];
    #pragma unroll
                for (int k = 0; k < SH::HY_PER; ++k) la[hy_dst[k]] = hyr[q % NH][k];
    #pragma unroll
                for (int j = 0; j < NY; ++j) {
                    lda[b][ty * NY + j + R][tx + R] = ring[j][F0(0)];
                    ldb[b][ty * NY + j][tx] = r1[j][F1(0)];
                }
                __syncthreads();

                {
                    // plane zA + R + PF into the slot of plane zA - R - 1 (free
                    // since the previous step); halo of plane zA + PF likewise
                    // zA >= -R and a periodic axis holds at least R planes,
                    // so zA + PF + nz >= 0: an unsigned remainder wraps it, at
                    // half the scalar work of a signed one
                    const uint32_t nzu = uint32_t(g.nz), zu = uint32_t(zA + PF + g.nz);
                    const PlaneRef bw = src.plane(int((zu + R) % nzu) + g.rz);
                    const PlaneRef bh = src.plane(int(zu % nzu) + g.rz);
    #pragma unroll
                    for (int j = 0; j < NY; ++j)
                        ring[j][F0(R + PF)] = plane_ld<S>(bw, col_off[j]);
    #pragma unroll
                    for (int k = 0; k < SH::HX_PER; ++k)
                        hxr[(q + PF) % NH][k] = plane_ld<S>(bh, hx_off[k]);
    #pragma unroll
                    for (int k = 0; k < SH::HY_PER; ++k)
                        hyr[(q + PF) % NH][k] = plane_ld<S>(bh, hy_off[k]);
                }

                // stage B: f2 at plane zB from the f1 ring and f1's plane in LDS
                const int zB = zA - 1 - R;
                if (zB >= z0) {
    #pragma unroll
                    for (int j = 0; j < NY; ++j) {
                        const int row = ty * NY + j;
                        const int xo = fx0 + tx, yo = fy0 + row;
                        if (tx >= R && tx < SH::TXW - R && row >= R && row < SH::ROWS - R &&
                            xo < g.nx && yo < g.ny) {
                            C acc = cf.c0 * r1[j][F1(0)];
    #pragma unroll
                            for (int m = 1; m <= R; ++m) {
                                acc = fma(cf.zm[m - 1], r1[j][F1(-m)], acc);
                                acc = fma(cf.zp[m - 1], r1[j][F1(m)], acc);
                            }
    #pragma unroll
                            for (int m = 1; m <= R; ++m) {
                                acc = fma(cf.xm[m - 1], ldb[b][row][tx - m], acc);
                                acc = fma(cf.xp[m - 1], ldb[b][row][tx + m], acc);
                            }
    #pragma unroll
                            for (int m = 1; m <= R; ++m) {
                                C vm = (j - m >= 0) ? r1[(j - m >= 0) ? j - m : 0][F1(0)]
                                                    : ldb[b][row - m][tx];
                                C vp = (j + m < NY) ? r1[(j + m < NY) ? j + m : 0][F1(0)]
                                                    : ldb[b][row + m][tx];
                                acc = fma(cf.ym[m - 1], vm, acc);
                                acc = fma(cf.yp[m - 1], vp, acc);
                            }
                            store_periodic(out, g, xo, yo, zB, acc, fuse);
                        }
                    }
                }

                // stage A: f1 at plane zA on the whole lane grid
    #pragma unroll
                for (int j = 0; j < NY; ++j) {
                    const int row = ty * NY + j + R;
                    C acc = cf.c0 * ring[j][F0(0)];
    #pragma unroll
                    for (int m = 1; m <= R; ++m) {
                        acc = fma(cf.zm[m - 1], ring[j][F0(-m)], acc);
                        acc = fma(cf.zp[m - 1], ring[j][F0(m)], acc);
                    }
    #pragma unroll
                    for (int m = 1; m <= R; ++m) {
                        acc = fma(cf.xm[m - 1], lda[b][row][tx + R - m], acc);
                        acc = fma(cf.xp[m - 1], lda[b][row][tx + R + m], acc);
                    }
    #pragma unroll
                    for (int m = 1; m <= R; ++m) {
                        C vm = (j - m >= 0) ? ring[(j - m >= 0) ? j - m : 0][F0(0)]
                                            : lda[b][row - m][tx + R];
                        C vp = (j + m < NY) ? ring[(j + m < NY) ? j + m : 0][F0(0)]
                                            : lda[b][row + m][tx + R];
                        acc = fma(cf.ym[m - 1], vm, acc);
                        acc = fma(cf.yp[m - 1], vp, acc);
                    }
                    r1[j][F0(0)] = RoundS<S>::f(acc); // f1 plane zA: same slot rule as f0
                }
    #undef F0
    #undef F1
            }
        }
    } else {
        // shifting-window march (1024-lane workgroups, capped at 128 VGPRs,
        // and r = 4): the window shifts by register moves each step
        // steps zA = zs .. ze; stage B is live from zA = z0 + R + 1 on
        const int zs = z0 - R, ze = z1 + R;
        C win[NY][2 * R + 1], w1[NY][2 * R + 1];
    #pragma unroll
        for (int j = 0; j < NY; ++j)
    #pragma unroll
            for (int k = 0; k <= 2 * R; ++k) w1[j][k] = 0;
    #pragma unroll
        for (int k = 0; k < 2 * R; ++k)
    #pragma unroll
            for (int j = 0; j < NY; ++j)
                win[j][k + 1] = plane_ld<S>(src.plane(wrap_mod(zs - R + k, g.nz) + g.rz), col_off[j]);

        C pre_w[PF][NY], pre_hx[PF][SH::HX_PER], pre_hy[PF][SH::HY_PER];
    #pragma unroll
        for (int q = 0; q < PF; ++q) {
    #pragma unroll
            for (int j = 0; j < NY; ++j) pre_w[q][j] = plane_ld<S>(src.plane(wrap_mod(zs + q + R, g.nz) + g.rz), col_off[j]);
    #pragma unroll
            for (int k = 0; k < SH::HX_PER; ++k) pre_hx[q][k] = plane_ld<S>(src.plane(wrap_mod(zs + q, g.nz) + g.rz), hx_off[k]);
    #pragma unroll
            for (int k = 0; k < SH::HY_PER; ++k) pre_hy[q][k] = plane_ld<S>(src.plane(wrap_mod(zs + q, g.nz) + g.rz), hy_off[k]);
        }

        // halo cells written unconditionally, as in the ring march
        const int own = (ty * NY + R) * SH::LW + tx + R;
        int hx_dst[SH::HX_PER], hy_dst[SH::HY_PER];
    #pragma unroll
        for (int k = 0; k < SH::HX_PER; ++k) hx_dst[k] = hx_slot[k] >= 0 ? hx_slot[k] : own;
    #pragma unroll
        for (int k = 0; k < SH::HY_PER; ++k) hy_dst[k] = hy_slot[k] >= 0 ? hy_slot[k] : own;

        for (int zb = zs; zb <= ze; zb += PF) {
    #pragma unroll
            for (int q = 0; q < PF; ++q) {
                const int zA = zb + q;
                if (zA > ze)
                    break;
                const int b = (zA - zs) & 1;
                C *la = &lda[b][0][0];
    #pragma unroll
                for (int k = 0; k < SH::HX_PER; ++k) la[hx_dst[k]] = pre_hx[q][k];
    #pragma unroll
                for (int k = 0; k < SH::HY_PER; ++k) la[hy_dst[k]] = pre_hy[q][k];
    #pragma unroll
                for (int j = 0; j < NY; ++j) {
    #pragma unroll
                    for (int k = 0; k < 2 * R; ++k) win[j][k] = win[j][k + 1];
                    win[j][2 * R] = pre_w[q][j];
                    lda[b][ty * NY + j + R][tx + R] = win[j][R];
                    ldb[b][ty * NY + j][tx] = w1[j][R];
                }
                __syncthreads();

                {
                    // zA + PF + nz >= 0: unsigned remainder, as in the ring march
                    const uint32_t nzu = uint32_t(g.nz), zu = uint32_t(zA + PF + g.nz);
                    const PlaneRef bw = src.plane(int((zu + R) % nzu) + g.rz);
                    const PlaneRef bh = src.plane(int(zu % nzu) + g.rz);
    #pragma unroll
                    for (int j = 0; j < NY; ++j)
                        pre_w[q][j] = plane_ld<S>(bw, col_off[j]);
    #pragma unroll
                    for (int k = 0; k < SH::HX_PER; ++k)
                        pre_hx[q][k] = plane_ld<S>(bh, hx_off[k]);
    #pragma unroll
                    for (int k = 0; k < SH::HY_PER; ++k)
                        pre_hy[q][k] = plane_ld<S>(bh, hy_off[k]);
                }

                // stage B: f2 at plane zB from the f1 window and f1's plane in LDS
                const int zB = zA - 1 - R;
                if (zB >= z0) {
    #pragma unroll
                    for (int j = 0; j < NY; ++j) {
                        const int row = ty * NY + j;
                        const int xo = fx0 + tx, yo = fy0 + row;
                        if (tx >= R && tx < SH::TXW - R && row >= R && row < SH::ROWS - R &&
                            xo < g.nx && yo < g.ny) {
                            C acc = cf.c0 * w1[j][R];
    #pragma unroll
                            for (int m = 1; m <= R; ++m) {
                                acc = fma(cf.zm[m - 1], w1[j][R - m], acc);
                                acc = fma(cf.zp[m - 1], w1[j][R + m], acc);
                            }
    #pragma unroll
                            for (int m = 1; m <= R; ++m) {
                                acc = fma(cf.xm[m - 1], ldb[b][row][tx - m], acc);
                                acc = fma(cf.xp[m - 1], ldb[b][row][tx + m], acc);
                            }
    #pragma unroll
                            for (int m = 1; m <= R; ++m) {
                                C vm = (j - m >= 0) ? w1[(j - m >= 0) ? j - m : 0][R] : ldb[b][row - m][tx];
                                C vp = (j + m < NY) ? w1[(j + m < NY) ? j + m : 0][R] : ldb[b][row + m][tx];
                                acc = fma(cf.ym[m - 1], vm, acc);
                                acc = fma(cf.yp[m - 1], vp, acc);
                            }
                            store_periodic(out, g, xo, yo, zB, acc, fuse);
                        }
                    }
                }

                // stage A: f1 at plane zA on the whole lane grid
    #pragma unroll
                for (int j = 0; j < NY; ++j) {
                    const int row = ty * NY + j + R;
                    C acc = cf.c0 * win[j][R];
    #pragma unroll
                    for (int m = 1; m <= R; ++m) {
                        acc = fma(cf.zm[m - 1], win[j][R - m], acc);
                        acc = fma(cf.zp[m - 1], win[j][R + m], acc);
                    }
    #pragma unroll
                    for (int m = 1; m <= R; ++m) {
                        acc = fma(cf.xm[m - 1], lda[b][row][tx + R - m], acc);
                        acc = fma(cf.xp[m - 1], lda[b][row][tx + R + m], acc);
                    }
    #pragma unroll
                    for (int m = 1; m <= R; ++m) {
                        C vm = (j - m >= 0) ? win[(j - m >= 0) ? j - m : 0][R] : lda[b][row - m][tx + R];
                        C vp = (j + m < NY) ? win[(j + m < NY) ? j + m : 0][R] : lda[b][row + m][tx + R];
                        acc = fma(cf.ym[m - 1], vm, acc);
                        acc = fma(cf.yp[m - 1], vp, acc);
                    }
    #pragma unroll
                    for (int k = 0; k < 2 * R; ++k) w1[j][k] = w1[j][k + 1];
                    w1[j][2 * R] = RoundS<S>::f(acc);
                }
            }
        }
    }
}

// Occupancy target: BF16 512-lane workgroups are held to 128 VGPRs (4 waves
// per SIMD, two workgroups per CU, so one's barrier waits overlap the other's
// work), which they reach without spills; other instances take the
// compiler's choice.
// Two 512-lane workgroups per CU (4 waves per SIMD, at most 128 VGPRs) for
// BF16, and for FP32 without the image store (with it, the cap spills).
template <typename S, int XW, int TY, bool IMG> constexpr int t2_min_waves()
{
    return (64 * XW * TY == 512 && (sizeof(S) == 2 || (sizeof(S) == 4 && !IMG))) ? 4 : 1;
}

// Workgroup = (tile column, z chunk of lz planes), gx * gy * gz of them.
// IMG: the output's periodic images are written (a compile-time choice, so a
// launch without them carries none of their scalar and exec-mask work).
template <typename S, int R, int NY, int TY, int XW, bool IMG, bool BIG>
__global__ void __launch_bounds__(64 * XW * TY, (t2_min_waves<S, XW, TY, IMG>()))
    k_star3d_t2(const S *__restrict__ in, S *__restrict__ out, Geo g,
                StarCoef<typename Store<S>::C, R> cf, int lz, int gx, int gy, int gz, int flags)
{
    using C = typename Store<S>::C;
    using SH = StarShape<R, NY, TY, XW>;
    __shared__ C lda[2][SH::LH][SH::LW];      // f0 plane zA with its halo
    __shared__ C ldb[2][SH::ROWS][SH::TXW];   // f1 plane zB on the lane grid

    int lin = blockIdx.x;
    const int total = gx * gy * gz;
    if (flags & STAR_FLAG_XCD) lin = xcd_remap(lin, total);
    const bool yfirst = (flags & STAR_FLAG_YFIRST) != 0;
    const int byi = yfirst ? lin % gy : (lin / gx) % gy;
    const int bxi = yfirst ? (lin / gy) % gx : lin % gx;
    const int z0 = (lin / (gx * gy)) * lz;
    star3d_t2_segment<S, R, NY, TY, XW, IMG, BIG>(in, out, g, cf, bxi, byi, z0, min(z0 + lz, g.nz),
                                             flags, lda, ldb);
}

} // namespace stn
