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
template <typename S, typename W, typename C, bool MASTER>
__device__ __forceinline__ void advdiff3_zmarch(const void *fin_v, const PointIO &io, const Geo &g,
                                                const StarCoef<C, 3> &cf, int x0, int y0, int z0,
                                                int z1, ZmLds<C> &lds)
{
    constexpr int R = ZM_R, NY = ZM_NY, PF = ZM_PF;
    constexpr uint32_t es = sizeof(S);
    const S *fin = static_cast<const S *>(fin_v);
    const Buf src = make_buf(fin, uint64_t(padded_elems(g)) * es);
    const int tx = threadIdx.x, ty = threadIdx.y, tid = tx + ZM_TX * ty;

    auto cl = [](int v, int n) { return min(max(v, -R), n + R - 1); };
    auto col = [&](int xx, int yy) { return uint32_t(xx + g.ox + g.sy * (yy + g.ry)) * es; };
    auto plane = [&](int zz) { return uint32_t(zz + g.rz) * uint32_t(g.sz) * es; };

    const int x = x0 + tx;
    uint32_t col_off[NY];
#pragma unroll
    for (int j = 0; j < NY; ++j) col_off[j] = col(cl(x, g.nx), cl(y0 + ty * NY + j, g.ny));
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

    C win[NY][2 * R + 1];
#pragma unroll
    for (int k = 0; k < 2 * R; ++k)
#pragma unroll
        for (int j = 0; j < NY; ++j)
            win[j][k + 1] = BufLd<S>::ld(src, col_off[j], plane(z0 - R + k));
    C pre_w[PF][NY], pre_hx[PF][ZM_HX], pre_hy[PF][ZM_HY];
#pragma unroll
    for (int q = 0; q < PF; ++q) {
        const int zq = min(z0 + q, z1 - 1);
#pragma unroll
        for (int j = 0; j < NY; ++j) pre_w[q][j] = BufLd<S>::ld(src, col_off[j], plane(zq + R));
#pragma unroll
        for (int k = 0; k < ZM_HX; ++k) pre_hx[q][k] = BufLd<S>::ld(src, hx_off[k], plane(zq));
#pragma unroll
        for (int k = 0; k < ZM_HY; ++k) pre_hy[q][k] = BufLd<S>::ld(src, hy_off[k], plane(zq));
    }

    for (int zb = z0; zb < z1; zb += PF) {
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            const int z = zb + q;
            if (z >= z1)
                break;
            const int b = (z - z0) & 1;
            C *lb = &lds[b][0][0];
#pragma unroll
            for (int j = 0; j < NY; ++j) {
#pragma unroll
                for (int k = 0; k < 2 * R; ++k) win[j][k] = win[j][k + 1];
                win[j][2 * R] = pre_w[q][j];
                lds[b][ty * NY + j + R][tx + R] = win[j][R];
            }
#pragma unroll
            for (int k = 0; k < ZM_HX; ++k)
                if (hx_slot[k] >= 0) lb[hx_slot[k]] = pre_hx[q][k];
#pragma unroll
            for (int k = 0; k < ZM_HY; ++k)
                if (hy_slot[k] >= 0) lb[hy_slot[k]] = pre_hy[q][k];
            __syncthreads();
            {
                const int zn = min(z + PF, z1 - 1);
#pragma unroll
                for (int j = 0; j < NY; ++j)
                    pre_w[q][j] = BufLd<S>::ld(src, col_off[j], plane(zn + R));
#pragma unroll
                for (int k = 0; k < ZM_HX; ++k)
                    pre_hx[q][k] = BufLd<S>::ld(src, hx_off[k], plane(zn));
#pragma unroll
                for (int k = 0; k < ZM_HY; ++k)
                    pre_hy[q][k] = BufLd<S>::ld(src, hy_off[k], plane(zn));
            }
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
                    acc = fma(cf.xm[m - 1], lds[b][row][tx + R - m], acc);
                    acc = fma(cf.xp[m - 1], lds[b][row][tx + R + m], acc);
                }
#pragma unroll
                for (int m = 1; m <= R; ++m) {
                    C vm = (j - m >= 0) ? win[(j - m >= 0) ? j - m : 0][R] : lds[b][row - m][tx + R];
                    C vp = (j + m < NY) ? win[(j + m < NY) ? j + m : 0][R] : lds[b][row + m][tx + R];
                    acc = fma(cf.ym[m - 1], vm, acc);
                    acc = fma(cf.yp[m - 1], vp, acc);
                }
                const int y = y0 + ty * NY + j;
                if (x < g.nx && y < g.ny)
                    rk_update<S, W, C, MASTER>(io, g, g.at(x, y, z), x, y, z, acc, win[j][R]);
            }
        }
    }
    __syncthreads();
}

} // namespace stn
