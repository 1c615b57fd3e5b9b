// advdiff_zm.hpp -- the 3-D scalar advection-diffusion substep as a z march:
// the right-hand side R = -c.grad f + nu lap f of the sixth-order radius-3
// operators is a 19-point star (Sec. 3.2 with an advection term), so a tile
// of it is computed like the linear star (x-y plane in LDS, z taps from a
// per-lane register window, two planes prefetched) with the low-storage RK3
// update of the point as the epilogue. Shared by the solo substep kernel and
// the batched job kernel, so a job's arithmetic is the same in both.
#pragma once

#include "linear_kernels.hpp"
#include "rk_point.hpp"

namespace stn {

// Tile of the z march: 64 lanes along x, ZM_TY along y with ZM_NY rows each.
constexpr int ZM_TX = 64, ZM_TY = 8, ZM_NY = 2, ZM_R = 3, ZM_PF = 2;
constexpr int ZM_ROWS = ZM_TY * ZM_NY;
constexpr int ZM_LW = ZM_TX + 2 * ZM_R, ZM_LH = ZM_ROWS + 2 * ZM_R;
constexpr int ZM_NT = ZM_TX * ZM_TY;
constexpr int ZM_NXH = 2 * ZM_R * ZM_ROWS, ZM_NYH = 2 * ZM_R * ZM_TX;
constexpr int ZM_HX = (ZM_NXH + ZM_NT - 1) / ZM_NT, ZM_HY = (ZM_NYH + ZM_NT - 1) / ZM_NT;

template <typename C> using ZmLds = C[2][ZM_LH][ZM_LW];

// Star coefficients of R for one job: along axis a the tap at +m is
// -c_a/ds_a w1_m + nu/ds_a^2 w2_m, at -m it is +c_a/ds_a w1_m + nu/ds_a^2 w2_m,
// and the centre sums nu/ds_a^2 w2_0 (w1, w2: unit-spacing sixth-order first
// and second derivative weights).
template <typename C>
__device__ __forceinline__ StarCoef<C, 3> advdiff_star(const FdWeights &fd, const double *inv_ds,
                                                      const double *adv, double nu)
{
    StarCoef<C, 3> cf;
    double c0 = 0, p[3][3], q[3][3];
    for (int a = 0; a < 3; ++a) {
        const double id = inv_ds[a], a1 = adv[a] * id, a2 = nu * id * id;
        c0 += a2 * fd.w2[0];
        for (int m = 1; m <= 3; ++m) {
            p[a][m - 1] = -a1 * fd.w1[m - 1] + a2 * fd.w2[m];
            q[a][m - 1] = a1 * fd.w1[m - 1] + a2 * fd.w2[m];
        }
    }
    cf.c0 = C(c0);
    for (int m = 0; m < 3; ++m) {
        cf.xp[m] = C(p[0][m]);
        cf.xm[m] = C(q[0][m]);
        cf.yp[m] = C(p[1][m]);
        cf.ym[m] = C(q[1][m]);
        cf.zp[m] = C(p[2][m]);
        cf.zm[m] = C(q[2][m]);
    }
    return cf;
}

// One tile: output columns x0.. x0+63, rows y0.. y0+15, planes z0..z1-1 of a
// 3-D job (padding 3, periodic images in the input's halo). Every lane of the
// workgroup (ZM_TX x ZM_TY) must call it; it ends with a barrier, so the LDS
// may be reused at once.
//
// Register rings: plane p of the input's z window lives in slot
// (p - z0 + R) mod NR (NR = 2R + 1 + PF: the window plus PF planes in
// flight); the x/y halo of plane p, and the old register values the RK update
// of plane p reads, in slot (p - z0) mod NH (NH = PF + 1). The march is
// unrolled by NR steps (a multiple of NH), so every slot index is a
// compile-time constant: loads land in the registers they are read from and
// no register is copied across the loop back-edge (such a copy would wait for
// a load issued just before). The register values of plane z + PF are loaded
// at step z with the rest of that plane, so the update does not wait for them.
template <typename S, typename W, typename C, bool MASTER>
__device__ __forceinline__ void advdiff3_zmarch(const void *fin_v, const PointIO &io, const Geo &g,
                                                const StarCoef<C, 3> &cf, int x0, int y0, int z0,
                                                int z1, ZmLds<C> &lds)
{
    constexpr int R = ZM_R, NY = ZM_NY, PF = ZM_PF;
    constexpr int NR = 2 * R + 1 + PF, NH = PF + 1;
    static_assert(NR % NH == 0, "the unrolled march must cover whole halo rings");
    constexpr uint32_t es = sizeof(S);
    const S *fin = static_cast<const S *>(fin_v);
    const uint64_t n_el = uint64_t(padded_elems(g));
    const Buf src = make_buf(fin, n_el * es);
    const int tx = threadIdx.x, ty = threadIdx.y, tid = tx + ZM_TX * ty;

    auto cl = [](int v, int n) { return min(max(v, -R), n + R - 1); };
    auto cole = [&](int xx, int yy) { return uint32_t(xx + g.ox + g.sy * (yy + g.ry)); };
    auto col = [&](int xx, int yy) { return cole(xx, yy) * es; };
    auto plane_e = [&](int zz) { return uint32_t(zz + g.rz) * uint32_t(g.sz); };
    auto plane = [&](int zz) { return plane_e(zz) * es; };

    const int x = x0 + tx;
    uint32_t col_off[NY], col_el[NY];
#pragma unroll
    for (int j = 0; j < NY; ++j) {
        col_el[j] = cole(cl(x, g.nx), cl(y0 + ty * NY + j, g.ny));
        col_off[j] = col_el[j] * es;
    }
    uint32_t hx_off[ZM_HX], hy_off[ZM_HY];
    int hx_slot[ZM_HX], hy_slot[ZM_HY];
#pragma unroll
    for (int k = 0; k < ZM_HX; ++k) {
        const int cidx = tid + k * ZM_NT;
        if (cidx < ZM_NXH) {
            const int row = cidx / (2 * R), e = cidx % (2 * R);
            const int lc = e < R ? e : ZM_TX + e;
            hx_off[k] = col(cl(x0 - R + lc, g.nx), cl(y0 + row, g.ny));
            hx_slot[k] = (row + R) * ZM_LW + lc;
        } else {
            hx_off[k] = col(0, 0);
            hx_slot[k] = -1;
        }
    }
#pragma unroll
    for (int k = 0; k < ZM_HY; ++k) {
        const int cidx = tid + k * ZM_NT;
        if (cidx < ZM_NYH) {
            const int e = cidx / ZM_TX, cc = cidx % ZM_TX;
            const int lr = e < R ? e : ZM_ROWS + e;
            hy_off[k] = col(cl(x0 + cc, g.nx), cl(y0 - R + lr, g.ny));
            hy_slot[k] = lr * ZM_LW + cc + R;
        } else {
            hy_off[k] = col(0, 0);
            hy_slot[k] = -1;
        }
    }

    // Halo cells are written unconditionally: a lane without one writes into
    // its own first interior cell, before the interior value is stored there
    // (one lane's LDS writes complete in program order), so no lane mask is
    // kept live across the march.
    const int own = (ty * NY + R) * ZM_LW + tx + R;
    int hx_dst[ZM_HX], hy_dst[ZM_HY];
#pragma unroll
    for (int k = 0; k < ZM_HX; ++k) hx_dst[k] = hx_slot[k] >= 0 ? hx_slot[k] : own;
#pragma unroll
    for (int k = 0; k < ZM_HY; ++k) hy_dst[k] = hy_slot[k] >= 0 ? hy_slot[k] : own;

    // which old values the update reads (uniform over the launch)
    const bool rd_w = io.stage > 0, rd_m = MASTER && io.stage == 2;
    const Buf wsrc = make_buf(rd_w ? io.wrd : fin_v, n_el * sizeof(W));
    const Buf w1src = make_buf(rd_m ? io.w1 : fin_v, n_el * sizeof(W));
    const Buf msrc = make_buf(rd_m ? (const void *)io.master : fin_v, n_el * sizeof(double));

    C ring[NY][NR];
    C hxr[NH][ZM_HX], hyr[NH][ZM_HY];
    W wr[NH][NY], w1r[NH][NY];
    double mr[NH][NY];
    // the old register values of plane zz (zero where the substep reads none)
    auto load_old = [&](int zz, W (&wv)[NY], W (&w1v)[NY], double (&mv)[NY]) {
#pragma unroll
        for (int j = 0; j < NY; ++j) {
            wv[j] = W(0);
            w1v[j] = W(0);
            mv[j] = 0.0;
        }
        if (rd_w) {
#pragma unroll
            for (int j = 0; j < NY; ++j)
                wv[j] = W(BufLd<W>::ld(wsrc, col_el[j] * uint32_t(sizeof(W)),
                                       plane_e(zz) * uint32_t(sizeof(W))));
        }
        if (rd_m) {
#pragma unroll
            for (int j = 0; j < NY; ++j) {
                w1v[j] = W(BufLd<W>::ld(w1src, col_el[j] * uint32_t(sizeof(W)),
                                        plane_e(zz) * uint32_t(sizeof(W))));
                mv[j] = BufLd<double>::ld(msrc, col_el[j] * 8u, plane_e(zz) * 8u);
            }
        }
    };
    // planes z0 - R .. z0 + R - 1 (slots 0 .. 2R - 1), then the first PF
    // planes ahead (clamped to the chunk: a clamped load is never used)
#pragma unroll
    for (int k = 0; k < 2 * R; ++k)
#pragma unroll
        for (int j = 0; j < NY; ++j)
            ring[j][k] = BufLd<S>::ld(src, col_off[j], plane(z0 - R + k));
#pragma unroll
    for (int q = 0; q < PF; ++q) {
        const int zq = min(z0 + q, z1 - 1);
#pragma unroll
        for (int j = 0; j < NY; ++j) ring[j][2 * R + q] = BufLd<S>::ld(src, col_off[j], plane(zq + R));
#pragma unroll
        for (int k = 0; k < ZM_HX; ++k) hxr[q][k] = BufLd<S>::ld(src, hx_off[k], plane(zq));
#pragma unroll
        for (int k = 0; k < ZM_HY; ++k) hyr[q][k] = BufLd<S>::ld(src, hy_off[k], plane(zq));
        load_old(zq, wr[q], w1r[q], mr[q]);
    }

    for (int zb = z0; zb < z1; zb += NR) {
#pragma unroll
        for (int q = 0; q < NR; ++q) {
            const int z = zb + q;
            if (z >= z1)
                break;
#define RS(k_) ((q + R + (k_) + 2 * NR) % NR)
            const int b = (z - z0) & 1;
            C *lb = &lds[b][0][0];
#pragma unroll
            for (int k = 0; k < ZM_HX; ++k) lb[hx_dst[k]] = hxr[q % NH][k];
#pragma unroll
            for (int k = 0; k < ZM_HY; ++k) lb[hy_dst[k]] = hyr[q % NH][k];
#pragma unroll
            for (int j = 0; j < NY; ++j) lds[b][ty * NY + j + R][tx + R] = ring[j][RS(0)];
            __syncthreads();
            {
                // plane z + PF (clamped) into the slots freed by plane z - R - 1
                const int zn = min(z + PF, z1 - 1);
#pragma unroll
                for (int j = 0; j < NY; ++j)
                    ring[j][RS(R + PF)] = BufLd<S>::ld(src, col_off[j], plane(zn + R));
#pragma unroll
                for (int k = 0; k < ZM_HX; ++k)
                    hxr[(q + PF) % NH][k] = BufLd<S>::ld(src, hx_off[k], plane(zn));
#pragma unroll
                for (int k = 0; k < ZM_HY; ++k)
                    hyr[(q + PF) % NH][k] = BufLd<S>::ld(src, hy_off[k], plane(zn));
                load_old(zn, wr[(q + PF) % NH], w1r[(q + PF) % NH], mr[(q + PF) % NH]);
            }
#pragma unroll
            for (int j = 0; j < NY; ++j) {
                const int row = ty * NY + j + R;
                C acc = cf.c0 * ring[j][RS(0)];
#pragma unroll
                for (int m = 1; m <= R; ++m) {
                    acc = fma(cf.zm[m - 1], ring[j][RS(-m)], acc);
                    acc = fma(cf.zp[m - 1], ring[j][RS(m)], acc);
                }
#pragma unroll
                for (int m = 1; m <= R; ++m) {
                    acc = fma(cf.xm[m - 1], lds[b][row][tx + R - m], acc);
                    acc = fma(cf.xp[m - 1], lds[b][row][tx + R + m], acc);
                }
#pragma unroll
                for (int m = 1; m <= R; ++m) {
                    C vm = (j - m >= 0) ? ring[(j - m >= 0) ? j - m : 0][RS(0)]
                                        : lds[b][row - m][tx + R];
                    C vp = (j + m < NY) ? ring[(j + m < NY) ? j + m : 0][RS(0)]
                                        : lds[b][row + m][tx + R];
                    acc = fma(cf.ym[m - 1], vm, acc);
                    acc = fma(cf.yp[m - 1], vp, acc);
                }
                const int y = y0 + ty * NY + j;
                if (x < g.nx && y < g.ny)
                    rk_update_pre<S, W, C, MASTER>(io, g, g.at(x, y, z), x, y, z, acc,
                                                   ring[j][RS(0)], wr[q % NH][j], w1r[q % NH][j],
                                                   mr[q % NH][j]);
            }
#undef RS
        }
    }
    __syncthreads();
}

} // namespace stn
