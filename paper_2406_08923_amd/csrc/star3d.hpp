// star3d.hpp -- the 3-D axis-aligned (star) cross-correlation kernel for
// gfx950: x-y plane tile staged in LDS, z taps from a per-lane register window
// marching along z, a register ring prefetching PF planes ahead. Included by
// the per-dtype instantiation units star3d_*.hip.
#pragma once

#include "linear_kernels.hpp"

namespace stn {

// Supported shapes (XW, TY, NY): tile width 64*XW lanes along x, TY lanes
// along y, NY rows per lane. Tiles are 64*XW x TY*NY points.
#define STAR_SHAPES(X)                                                                       \
    X(1, 8, 2) X(1, 4, 4) X(1, 8, 4) X(1, 16, 2) X(2, 4, 2) X(2, 4, 4) X(2, 8, 2)             \
    X(4, 2, 2) X(4, 2, 4) X(4, 4, 2) X(8, 1, 4) X(8, 2, 2)
// Supported prefetch depths (planes in flight ahead of the one computed).
#define STAR_PREFETCH(X) X(2)

template <int R, int NY, int TY, int XW> struct StarShape {
    static constexpr int TXW = 64 * XW;      // lanes along x
    static constexpr int ROWS = TY * NY;     // output rows per tile
    static constexpr int LW = TXW + 2 * R;   // LDS row width
    static constexpr int LH = ROWS + 2 * R;  // LDS rows
    static constexpr int NXH = 2 * R * ROWS; // x-halo cells per plane
    static constexpr int NYH = 2 * R * TXW;  // y-halo cells per plane
    static constexpr int NT = TXW * TY;      // lanes per workgroup
    static constexpr int HX_PER = (NXH + NT - 1) / NT;
    static constexpr int HY_PER = (NYH + NT - 1) / NT;
};

// Workgroup = 64*XW x TY lanes; lane (tx, ty) owns column x = x0 + tx and the NY
// consecutive rows y0 + ty*NY + j, and marches along z over a chunk of lz
// output planes. Per lane and row the 2R+1 column values around the current
// plane live in registers (the z taps). The current plane with its x and y
// halo (a star needs no corners) is staged in LDS, double-buffered, so one
// barrier per plane suffices; x taps and the y taps outside the lane's own
// rows come from LDS, y taps inside them from registers. Loads of plane z+PF
// (its leading window value and halo cells) are issued right after the
// barrier of plane z, so PF planes of HBM latency overlap the arithmetic.
// All loads are buffer loads: the lane supplies its in-plane byte offset, the
// plane offset is a wave-uniform scalar.
template <typename S, int R, int NY, int TY, int XW, int PF>
__global__ void __launch_bounds__(64 * XW * TY)
    k_star3d(const S *__restrict__ in, S *__restrict__ out, Geo g,
             StarCoef<typename Store<S>::C, R> cf, int lz, int gx, int gy, int gz, int flags)
{
    using C = typename Store<S>::C;
    using SH = StarShape<R, NY, TY, XW>;
    constexpr uint32_t es = sizeof(S);
    __shared__ C lds[2][SH::LH][SH::LW];

    int lin = blockIdx.x;
    const int total = gx * gy * gz;
    if (flags & STAR_FLAG_XCD) lin = xcd_remap(lin, total);
    const bool yfirst = (flags & STAR_FLAG_YFIRST) != 0;
    const int byi = yfirst ? lin % gy : (lin / gx) % gy;
    const int bxi = yfirst ? (lin / gy) % gx : lin % gx;
    const int bzi = lin / (gx * gy);

    const int tx = threadIdx.x, ty = threadIdx.y;
    const int tid = tx + SH::TXW * ty;
    const int x0 = bxi * SH::TXW, y0 = byi * SH::ROWS;
    const int z0 = bzi * lz;
    const int z1 = min(z0 + lz, g.nz);
    const bool fuse = (flags & STAR_FLAG_NOFUSE) == 0;
    // clamp reads into the padded array: any coordinate in [-R, n+R) is valid
    auto cl = [](int v, int n) { return min(max(v, -R), n + R - 1); };
    // byte offset of interior column (x, y) within a plane; each plane is
    // read through its own buffer resource (plane_buf)
    auto col = [&](int xx, int yy) {
        return uint32_t(xx + g.ox + g.sy * (yy + g.ry)) * es;
    };

    const int x = x0 + tx;
    const int xl = cl(x, g.nx);
    uint32_t col_off[NY];
#pragma unroll
    for (int j = 0; j < NY; ++j) col_off[j] = col(xl, cl(y0 + ty * NY + j, g.ny));

    // halo cells of this lane (fixed per plane)
    uint32_t hx_off[SH::HX_PER], hy_off[SH::HY_PER];
    int hx_slot[SH::HX_PER], hy_slot[SH::HY_PER];
#pragma unroll
    for (int k = 0; k < SH::HX_PER; ++k) {
        const int cidx = tid + k * SH::NT;
        if (cidx < SH::NXH) {
            const int row = cidx / (2 * R), e = cidx % (2 * R);
            const int lc = e < R ? e : SH::TXW + e; // LDS column
            hx_off[k] = col(cl(x0 - R + lc, g.nx), cl(y0 + row, g.ny));
            hx_slot[k] = (row + R) * SH::LW + lc;
        } else {
            hx_off[k] = col(0, 0);
            hx_slot[k] = -1;
        }
    }
#pragma unroll
    for (int k = 0; k < SH::HY_PER; ++k) {
        const int cidx = tid + k * SH::NT;
        if (cidx < SH::NYH) {
            const int e = cidx / SH::TXW, cc = cidx % SH::TXW;
            const int lr = e < R ? e : SH::ROWS + e; // LDS row
            hy_off[k] = col(cl(x0 + cc, g.nx), cl(y0 - R + lr, g.ny));
            hy_slot[k] = lr * SH::LW + cc + R;
        } else {
            hy_off[k] = col(0, 0);
            hy_slot[k] = -1;
        }
    }

    // Halo cells are written unconditionally: a lane without one writes into
    // its own first interior cell, before the interior value is stored there
    // (one lane's LDS writes complete in program order), so no lane mask is
    // kept live across the march.
    const int own = (ty * NY + R) * SH::LW + tx + R;
    int hx_dst[SH::HX_PER], hy_dst[SH::HY_PER];
#pragma unroll
    for (int k = 0; k < SH::HX_PER; ++k) hx_dst[k] = hx_slot[k] >= 0 ? hx_slot[k] : own;
#pragma unroll
    for (int k = 0; k < SH::HY_PER; ++k) hy_dst[k] = hy_slot[k] >= 0 ? hy_slot[k] : own;

    // Register-ring march where the halo ring (PF + 1 slots) divides the z
    // ring (2R + 1 + PF slots), i.e. PF + 1 divides 2R (r = 3 with PF = 2):
    // plane p lives in slot (p - z0 + R) mod NR of ring, its halo in slot
    // (p - z0) mod NH; the march is unrolled by NR steps so every slot index
    // is a compile-time constant, loads land in the registers they are read
    // from and nothing is copied across the loop back-edge (such a copy
    // would wait for a load issued just before). Other radii keep the
    // shifting window below.
    constexpr int NR = 2 * R + 1 + PF, NH = PF + 1;
    if constexpr (NR % NH == 0) {
        C ring[NY][NR];
        C hxr[NH][SH::HX_PER], hyr[NH][SH::HY_PER];
#pragma unroll
        for (int k = 0; k < 2 * R; ++k)
#pragma unroll
            for (int j = 0; j < NY; ++j)
                ring[j][k] = BufLd<S>::ld(plane_buf(in, g.sz, z0 - R + k + g.rz), col_off[j], 0);
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            const int zq = min(z0 + q, z1 - 1); // in range: any valid plane will do
#pragma unroll
            for (int j = 0; j < NY; ++j)
                ring[j][2 * R + q] = BufLd<S>::ld(plane_buf(in, g.sz, zq + R + g.rz), col_off[j], 0);
#pragma unroll
            for (int k = 0; k < SH::HX_PER; ++k) hxr[q][k] = BufLd<S>::ld(plane_buf(in, g.sz, zq + g.rz), hx_off[k], 0);
#pragma unroll
            for (int k = 0; k < SH::HY_PER; ++k) hyr[q][k] = BufLd<S>::ld(plane_buf(in, g.sz, zq + g.rz), hy_off[k], 0);
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
                for (int k = 0; k < SH::HX_PER; ++k) lb[hx_dst[k]] = hxr[q % NH][k];
#pragma unroll
                for (int k = 0; k < SH::HY_PER; ++k) lb[hy_dst[k]] = hyr[q % NH][k];
#pragma unroll
                for (int j = 0; j < NY; ++j) lds[b][ty * NY + j + R][tx + R] = ring[j][RS(0)];
                __syncthreads();
                {
                    // plane z + PF (clamped) into the slots of plane z - R - 1
                    const int zn = min(z + PF, z1 - 1);
#pragma unroll
                    for (int j = 0; j < NY; ++j)
                        ring[j][RS(R + PF)] = BufLd<S>::ld(plane_buf(in, g.sz, zn + R + g.rz), col_off[j], 0);
#pragma unroll
                    for (int k = 0; k < SH::HX_PER; ++k)
                        hxr[(q + PF) % NH][k] = BufLd<S>::ld(plane_buf(in, g.sz, zn + g.rz), hx_off[k], 0);
#pragma unroll
                    for (int k = 0; k < SH::HY_PER; ++k)
                        hyr[(q + PF) % NH][k] = BufLd<S>::ld(plane_buf(in, g.sz, zn + g.rz), hy_off[k], 0);
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
                        store_periodic(out, g, x, y, z, acc, fuse);
                }
#undef RS
            }
        }
    } else {
        // z window: win[j][k] holds plane z - R + k of row j
        C win[NY][2 * R + 1];
    #pragma unroll
        for (int k = 0; k < 2 * R; ++k)
    #pragma unroll
            for (int j = 0; j < NY; ++j)
                win[j][k + 1] = BufLd<S>::ld(plane_buf(in, g.sz, z0 - R + k + g.rz), col_off[j], 0);

        // prefetch ring: slot q holds plane z0 + q (+R for the window value)
        C pre_w[PF][NY], pre_hx[PF][SH::HX_PER], pre_hy[PF][SH::HY_PER];
    #pragma unroll
        for (int q = 0; q < PF; ++q) {
            const int zq = min(z0 + q, z1 - 1); // in range: any valid plane will do
    #pragma unroll
            for (int j = 0; j < NY; ++j) pre_w[q][j] = BufLd<S>::ld(plane_buf(in, g.sz, zq + R + g.rz), col_off[j], 0);
    #pragma unroll
            for (int k = 0; k < SH::HX_PER; ++k) pre_hx[q][k] = BufLd<S>::ld(plane_buf(in, g.sz, zq + g.rz), hx_off[k], 0);
    #pragma unroll
            for (int k = 0; k < SH::HY_PER; ++k) pre_hy[q][k] = BufLd<S>::ld(plane_buf(in, g.sz, zq + g.rz), hy_off[k], 0);
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
                }
    #pragma unroll
                for (int k = 0; k < SH::HX_PER; ++k) lb[hx_dst[k]] = pre_hx[q][k];
    #pragma unroll
                for (int k = 0; k < SH::HY_PER; ++k) lb[hy_dst[k]] = pre_hy[q][k];
    #pragma unroll
                for (int j = 0; j < NY; ++j) lds[b][ty * NY + j + R][tx + R] = win[j][R];
                __syncthreads();

                // refill slot q with plane z + PF (clamped: past the chunk end the
                // values are never used, the load only has to stay in range)
                {
                    const int zn = min(z + PF, z1 - 1);
    #pragma unroll
                    for (int j = 0; j < NY; ++j)
                        pre_w[q][j] = BufLd<S>::ld(plane_buf(in, g.sz, zn + R + g.rz), col_off[j], 0);
    #pragma unroll
                    for (int k = 0; k < SH::HX_PER; ++k)
                        pre_hx[q][k] = BufLd<S>::ld(plane_buf(in, g.sz, zn + g.rz), hx_off[k], 0);
    #pragma unroll
                    for (int k = 0; k < SH::HY_PER; ++k)
                        pre_hy[q][k] = BufLd<S>::ld(plane_buf(in, g.sz, zn + g.rz), hy_off[k], 0);
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
                        store_periodic(out, g, x, y, z, acc, fuse);
                }
            }
        }
    }
}

template <typename S, int R, int NY, int TY, int XW, int PF>
int launch_star3d_t(const S *in, S *out, const Geo &g,
                    const StarCoef<typename Store<S>::C, R> &cf, int lz, int flags, hipStream_t s)
{
    using SH = StarShape<R, NY, TY, XW>;
    int gx = (g.nx + SH::TXW - 1) / SH::TXW, gy = (g.ny + SH::ROWS - 1) / SH::ROWS;
    int gz = (g.nz + lz - 1) / lz;
    int64_t total = (int64_t)gx * gy * gz;
    if (total > 0x7fffffff)
        return fail(STENCIL_EUNSUPPORTED, "star3d: grid too large");
    hipLaunchKernelGGL((k_star3d<S, R, NY, TY, XW, PF>), dim3((unsigned)total),
                       dim3(SH::TXW, TY), 0, s, in, out, g, cf, lz, gx, gy, gz, flags);
    return check_launch("xcorr_star3d");
}

template <typename S, int R, int NY, int TY, int XW>
int launch_star3d_pf(const S *in, S *out, const Geo &g,
                     const StarCoef<typename Store<S>::C, R> &cf, int pf, int lz, int flags,
                     hipStream_t s)
{
#define STAR_CASE_PF(PF_)                                                                    \
    if (pf == PF_)                                                                           \
        return launch_star3d_t<S, R, NY, TY, XW, PF_>(in, out, g, cf, lz, flags, s);
    STAR_PREFETCH(STAR_CASE_PF)
#undef STAR_CASE_PF
    return fail(STENCIL_EUNSUPPORTED, "star3d: unsupported prefetch depth %d", pf);
}

template <typename S, int R>
int launch_star3d_r(const S *in, S *out, const Geo &g, const StarCoef<typename Store<S>::C, R> &cf,
                    int xw, int ty, int ny, int pf, int lz, int flags, hipStream_t s)
{
#define STAR_CASE(XW_, TY_, NY_)                                                             \
    if (xw == XW_ && ty == TY_ && ny == NY_)                                                 \
        return launch_star3d_pf<S, R, NY_, TY_, XW_>(in, out, g, cf, pf, lz, flags, s);
    STAR_SHAPES(STAR_CASE)
#undef STAR_CASE
    return fail(STENCIL_EUNSUPPORTED, "star3d: unsupported tile (xw=%d, ty=%d, ny=%d)", xw, ty,
                ny);
}


// Hardware-cached variant (the HWC strategy of Sec. 4.1/4.4) of the z march:
// no LDS and no barriers. Lane (tx, ty) owns column x and NY consecutive rows
// and marches along z with the 2R+1 column values in registers (z taps); the
// x and y taps of the current plane are buffer loads that hit in L1/L2 because
// neighbouring lanes and waves load the same lines in the same plane. Per
// lane the base offset is the corner (x - R, y - R) of its neighbourhood, so
// x taps differ by an immediate and y taps by a wave-uniform scalar.
template <typename S, int R, int NY, int TY>
__global__ void __launch_bounds__(64 * TY)
    k_star3d_hwc(const S *__restrict__ in, S *__restrict__ out, Geo g,
                 StarCoef<typename Store<S>::C, R> cf, int lz, int gx, int gy, int gz, int flags)
{
    using C = typename Store<S>::C;
    constexpr uint32_t es = sizeof(S);
    constexpr int ROWS = TY * NY;
    int lin = blockIdx.x;
    const int total = gx * gy * gz;
    if (flags & STAR_FLAG_XCD) lin = xcd_remap(lin, total);
    const bool yfirst = (flags & STAR_FLAG_YFIRST) != 0;
    const int byi = yfirst ? lin % gy : (lin / gx) % gy;
    const int bxi = yfirst ? (lin / gy) % gx : lin % gx;
    const int bzi = lin / (gx * gy);
    const int x = bxi * 64 + threadIdx.x;
    const int y0 = byi * ROWS + threadIdx.y * NY;
    const int z0 = bzi * lz;
    const int z1 = min(z0 + lz, g.nz);
    const bool fuse = (flags & STAR_FLAG_NOFUSE) == 0;
    const Buf src = make_buf(in, uint64_t(padded_elems(g)) * es);
    const uint32_t row = uint32_t(g.sy) * es;
    auto cl = [](int v, int n) { return min(max(v, -R), n + R - 1); };
    auto plane = [&](int zz) { return uint32_t(zz + g.rz) * uint32_t(g.sz) * es; };
    // lowest corner of the lane's neighbourhood (x - R, y0 - R), clamped in x
    const int xc = min(max(x, 0), g.nx - 1);
    const uint32_t base = uint32_t(xc - R + g.ox + g.sy * (y0 - R + g.ry)) * es;
    // window values: column x, rows y0 + j (clamped rows read valid memory)
    uint32_t col_off[NY];
#pragma unroll
    for (int j = 0; j < NY; ++j)
        col_off[j] = uint32_t(xc + g.ox + g.sy * (cl(y0 + j, g.ny) + g.ry)) * es;
    C win[NY][2 * R + 1];
#pragma unroll
    for (int k = 0; k < 2 * R; ++k)
#pragma unroll
        for (int j = 0; j < NY; ++j)
            win[j][k + 1] = BufLd<S>::ld(src, col_off[j], plane(z0 - R + k));
    C pre[NY];
#pragma unroll
    for (int j = 0; j < NY; ++j)
        pre[j] = BufLd<S>::ld(src, col_off[j], plane(min(z0, z1 - 1) + R));
    // the y range of the neighbourhood may leave the padded array only for
    // clamped rows past the grid; their outputs are not stored, and loads
    // beyond the buffer return zero
    for (int z = z0; z < z1; ++z) {
#pragma unroll
        for (int j = 0; j < NY; ++j) {
#pragma unroll
            for (int k = 0; k < 2 * R; ++k) win[j][k] = win[j][k + 1];
            win[j][2 * R] = pre[j];
        }
        const int zn = min(z + 1, z1 - 1);
#pragma unroll
        for (int j = 0; j < NY; ++j)
            pre[j] = BufLd<S>::ld(src, col_off[j], plane(zn + R));
        const uint32_t pz = plane(z);
        // y taps outside the lane's own rows: rows y0 - R .. y0 - 1 and
        // y0 + NY .. y0 + NY + R - 1 of column x
        C yl[R], yh[R];
#pragma unroll
        for (int m = 0; m < R; ++m) {
            yl[m] = BufLd<S>::ld(src, base + R * es, pz + m * row);
            yh[m] = BufLd<S>::ld(src, base + R * es, pz + (R + NY + m) * row);
        }
#pragma unroll
        for (int j = 0; j < NY; ++j) {
            C acc = cf.c0 * win[j][R];
#pragma unroll
            for (int m = 1; m <= R; ++m) {
                acc = fma(cf.zm[m - 1], win[j][R - m], acc);
                acc = fma(cf.zp[m - 1], win[j][R + m], acc);
            }
            const uint32_t prow = pz + (R + j) * row;
#pragma unroll
            for (int m = 1; m <= R; ++m) {
                acc = fma(cf.xm[m - 1], BufLd<S>::ld(src, base + (R - m) * es, prow), acc);
                acc = fma(cf.xp[m - 1], BufLd<S>::ld(src, base + (R + m) * es, prow), acc);
            }
#pragma unroll
            for (int m = 1; m <= R; ++m) {
                const int jm = j - m, jp = j + m;
                const C vm = jm >= 0 ? win[jm >= 0 ? jm : 0][R] : yl[R + jm];
                const C vp = jp < NY ? win[jp < NY ? jp : 0][R] : yh[jp - NY];
                acc = fma(cf.ym[m - 1], vm, acc);
                acc = fma(cf.yp[m - 1], vp, acc);
            }
            const int y = y0 + j;
            if (x < g.nx && y < g.ny)
                store_periodic(out, g, x, y, z, acc, fuse);
        }
    }
}

template <typename S, int R, int NY, int TY>
int launch_star3d_hwc_t(const S *in, S *out, const Geo &g,
                        const StarCoef<typename Store<S>::C, R> &cf, int lz, int flags,
                        hipStream_t s)
{
    constexpr int ROWS = TY * NY;
    int gx = (g.nx + 63) / 64, gy = (g.ny + ROWS - 1) / ROWS, gz = (g.nz + lz - 1) / lz;
    int64_t total = (int64_t)gx * gy * gz;
    if (total > 0x7fffffff)
        return fail(STENCIL_EUNSUPPORTED, "star3d: grid too large");
    hipLaunchKernelGGL((k_star3d_hwc<S, R, NY, TY>), dim3((unsigned)total), dim3(64, TY), 0, s,
                       in, out, g, cf, lz, gx, gy, gz, flags);
    return check_launch("xcorr_star3d_hwc");
}

// Shapes (TY, NY) of the hardware-cached variant.
#define STAR_HWC_SHAPES(X) X(4, 1) X(4, 2) X(4, 4) X(2, 4) X(8, 2)

template <typename S, int R>
int launch_star3d_hwc_r(const S *in, S *out, const Geo &g,
                        const StarCoef<typename Store<S>::C, R> &cf, int ty, int ny, int lz,
                        int flags, hipStream_t s)
{
#define STAR_HWC_CASE(TY_, NY_)                                                              \
    if (ty == TY_ && ny == NY_)                                                              \
        return launch_star3d_hwc_t<S, R, NY_, TY_>(in, out, g, cf, lz, flags, s);
    STAR_HWC_SHAPES(STAR_HWC_CASE)
#undef STAR_HWC_CASE
    return fail(STENCIL_EUNSUPPORTED, "star3d (cached): unsupported tile (ty=%d, ny=%d)", ty, ny);
}

} // namespace stn

#include "star3d_t2.hpp"
#include "star3d_t2p.hpp"
#include "star3d_t2q.hpp"
#include "star3d_dpp.hpp"

namespace stn {

template <typename S, int R, int NY, int TY, int XW>
int launch_star3d_t2_t(const S *in, S *out, const Geo &g,
                       const StarCoef<typename Store<S>::C, R> &cf, int lz, int flags,
                       hipStream_t s)
{
    using SH = StarShape<R, NY, TY, XW>;
    const int OX = SH::TXW - 2 * R, OY = SH::ROWS - 2 * R;
    int gx = (g.nx + OX - 1) / OX, gy = (g.ny + OY - 1) / OY;
    int gz = (g.nz + lz - 1) / lz;
    int64_t total = (int64_t)gx * gy * gz;
    if (total > 0x7fffffff)
        return fail(STENCIL_EUNSUPPORTED, "star3d (two iterations): grid too large");
    const bool img = (flags & STAR_FLAG_NOFUSE) == 0;
    // arrays of 4 GiB or more: a buffer resource per input plane
    const bool big = uint64_t(padded_elems(g)) * sizeof(S) >= (uint64_t(1) << 32);
#define STAR_T2_LAUNCH(K_, ...)                                                              \
    do {                                                                                     \
        if (img && big)                                                                      \
            hipLaunchKernelGGL((K_<__VA_ARGS__, true, true>), dim3((unsigned)total),          \
                               dim3(SH::TXW, TY), 0, s, in, out, g, cf, lz, gx, gy, gz, flags); \
        else if (img)                                                                        \
            hipLaunchKernelGGL((K_<__VA_ARGS__, true, false>), dim3((unsigned)total),         \
                               dim3(SH::TXW, TY), 0, s, in, out, g, cf, lz, gx, gy, gz, flags); \
        else if (big)                                                                        \
            hipLaunchKernelGGL((K_<__VA_ARGS__, false, true>), dim3((unsigned)total),         \
                               dim3(SH::TXW, TY), 0, s, in, out, g, cf, lz, gx, gy, gz, flags); \
        else                                                                                 \
            hipLaunchKernelGGL((K_<__VA_ARGS__, false, false>), dim3((unsigned)total),        \
                               dim3(SH::TXW, TY), 0, s, in, out, g, cf, lz, gx, gy, gz, flags); \
    } while (0)
    if (flags & STAR_FLAG_PAIRS) {
        if constexpr (NY == 2 && R <= 4 && 64 * XW * TY <= 768) {
            STAR_T2_LAUNCH(k_star3d_t2p, S, R, TY, XW);
            return check_launch("xcorr_star3d_t2 (pair layout)");
        } else if constexpr (NY == 4 && sizeof(typename Store<S>::C) == 4 && XW == 1 &&
                             64 * TY <= 768) {
            STAR_T2_LAUNCH(k_star3d_t2q, S, R, TY);
            return check_launch("xcorr_star3d_t2 (quad layout)");
        } else {
            return fail(STENCIL_EUNSUPPORTED,
                        "star3d (two iterations): the pair layout needs two rows per lane, "
                        "radius <= 4 and at most 768 lanes (FP32/BF16: or four rows per lane "
                        "in a 64-lane-wide tile)");
        }
    }
    // the per-plane resources only for the register-ring instances (the
    // shifting-window ones spill registers, and each spilling instance
    // shipped must be covered by tests: those run arrays below 4 GiB)
    if constexpr (64 * XW * TY <= 768 && R <= 3 && NY <= 2) {
        STAR_T2_LAUNCH(k_star3d_t2, S, R, NY, TY, XW);
    } else {
        if (big)
            return fail(STENCIL_EUNSUPPORTED,
                        "star3d (two iterations): arrays of 4 GiB or more need a tile of at "
                        "most 768 lanes, two rows per lane and radius <= 3");
        if (img)
            hipLaunchKernelGGL((k_star3d_t2<S, R, NY, TY, XW, true, false>), dim3((unsigned)total),
                               dim3(SH::TXW, TY), 0, s, in, out, g, cf, lz, gx, gy, gz, flags);
        else
            hipLaunchKernelGGL((k_star3d_t2<S, R, NY, TY, XW, false, false>), dim3((unsigned)total),
                               dim3(SH::TXW, TY), 0, s, in, out, g, cf, lz, gx, gy, gz, flags);
    }
#undef STAR_T2_LAUNCH
    return check_launch("xcorr_star3d_t2");
}

template <typename S, int R>
int launch_star3d_t2_r(const S *in, S *out, const Geo &g,
                       const StarCoef<typename Store<S>::C, R> &cf, int xw, int ty, int ny,
                       int lz, int flags, hipStream_t s)
{
#define STAR_T2_CASE(XW_, TY_, NY_)                                                          \
    if (xw == XW_ && ty == TY_ && ny == NY_)                                                 \
        return launch_star3d_t2_t<S, R, NY_, TY_, XW_>(in, out, g, cf, lz, flags, s);
    STAR_T2_SHAPES(STAR_T2_CASE)
#undef STAR_T2_CASE
    return fail(STENCIL_EUNSUPPORTED,
                "star3d (two iterations): unsupported tile (xw=%d, ty=%d, ny=%d)", xw, ty, ny);
}


template <typename S>
int launch_star3d_t2_impl(const S *in, S *out, const Geo &g, const StarCoefAny &cfa, int R,
                          int xw, int ty, int ny, int lz, int flags, hipStream_t s)
{
    using C = typename Store<S>::C;
    if (g.ndim != 3 || R < 1)
        return fail(STENCIL_EINVAL, "star3d (two iterations): needs a 3-D star");
    if (lz < 1)
        return fail(STENCIL_EINVAL, "star3d: z planes per workgroup must be >= 1");
    switch (R) {
    case 1: return launch_star3d_t2_r<S, 1>(in, out, g, cfa.get<C, 1>(), xw, ty, ny, lz, flags, s);
    case 2: return launch_star3d_t2_r<S, 2>(in, out, g, cfa.get<C, 2>(), xw, ty, ny, lz, flags, s);
    case 3: return launch_star3d_t2_r<S, 3>(in, out, g, cfa.get<C, 3>(), xw, ty, ny, lz, flags, s);
    case 4: return launch_star3d_t2_r<S, 4>(in, out, g, cfa.get<C, 4>(), xw, ty, ny, lz, flags, s);
    }
    return fail(STENCIL_EUNSUPPORTED, "star3d: radius %d not in 1..4", R);
}

template <typename S>
int launch_star3d_impl(const S *in, S *out, const Geo &g, const StarCoefAny &cfa, int R, int xw,
                       int ty, int ny, int pf, int lz, int flags, hipStream_t s)
{
    using C = typename Store<S>::C;
    if (R > g.r || g.ndim != 3)
        return fail(STENCIL_EINVAL, "star3d: tap radius %d exceeds padding %d", R, g.r);
    if (flags & STAR_FLAG_DPP) {
        switch (R) {
        case 1: return launch_star3d_dpp_r<S, 1>(in, out, g, cfa.get<C, 1>(), ty, ny, pf, lz, flags, s);
        case 2: return launch_star3d_dpp_r<S, 2>(in, out, g, cfa.get<C, 2>(), ty, ny, pf, lz, flags, s);
        case 3: return launch_star3d_dpp_r<S, 3>(in, out, g, cfa.get<C, 3>(), ty, ny, pf, lz, flags, s);
        case 4: return launch_star3d_dpp_r<S, 4>(in, out, g, cfa.get<C, 4>(), ty, ny, pf, lz, flags, s);
        }
        return fail(STENCIL_EUNSUPPORTED, "star3d: radius %d not in 1..4", R);
    }
    if (flags & STAR_FLAG_HWC) {
        if (uint64_t(padded_elems(g)) * sizeof(S) >= (uint64_t(1) << 32))
            return fail(STENCIL_EUNSUPPORTED,
                        "star3d (hardware-cached): arrays of 4 GiB or more are not supported");
        switch (R) {
        case 1: return launch_star3d_hwc_r<S, 1>(in, out, g, cfa.get<C, 1>(), ty, ny, lz, flags, s);
        case 2: return launch_star3d_hwc_r<S, 2>(in, out, g, cfa.get<C, 2>(), ty, ny, lz, flags, s);
        case 3: return launch_star3d_hwc_r<S, 3>(in, out, g, cfa.get<C, 3>(), ty, ny, lz, flags, s);
        case 4: return launch_star3d_hwc_r<S, 4>(in, out, g, cfa.get<C, 4>(), ty, ny, lz, flags, s);
        }
        return fail(STENCIL_EUNSUPPORTED, "star3d: radius %d not in 1..4", R);
    }
    switch (R) {
    case 1: return launch_star3d_r<S, 1>(in, out, g, cfa.get<C, 1>(), xw, ty, ny, pf, lz, flags, s);
    case 2: return launch_star3d_r<S, 2>(in, out, g, cfa.get<C, 2>(), xw, ty, ny, pf, lz, flags, s);
    case 3: return launch_star3d_r<S, 3>(in, out, g, cfa.get<C, 3>(), xw, ty, ny, pf, lz, flags, s);
    case 4: return launch_star3d_r<S, 4>(in, out, g, cfa.get<C, 4>(), xw, ty, ny, pf, lz, flags, s);
    }
    return fail(STENCIL_EUNSUPPORTED, "star3d: radius %d not in 1..4", R);
}

} // namespace stn
