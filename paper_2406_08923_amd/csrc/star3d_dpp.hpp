// star3d_dpp.hpp -- the one-iteration 3-D star z march with its x taps
// exchanged across lanes: no LDS and no barriers. Included by star3d.hpp.
//
// A wave is one row of 64 consecutive columns. Lane tx holds column
// x = x0 - R + tx and NY consecutive rows; the 2R lanes at the wave's two
// edges are halo lanes (their values feed their neighbours' x taps, their own
// outputs are not stored), so a wave yields 64 - 2R output columns. Per lane
// and row the z taps come from a register ring of the column, the x taps from
// R one-lane shifts of the centre value in each direction (DPP moves), and the
// y taps from the lane's own rows or, for the R rows above and below them,
// from loads of the current plane (rows other waves hold, so they hit L1/L2).
// The taps are summed in the order of the other star kernels (centre, z, x,
// y), so results are bitwise theirs.
#pragma once

namespace stn {

// Shapes (TY, NY): TY waves per workgroup stacked along y, NY rows per lane.
#define STAR_DPP_SHAPES(X) X(4, 2) X(4, 4) X(8, 2) X(8, 4)

// PF: planes loaded ahead of the window (1 or 3).
template <typename S, int R, int NY, int TY, int PF, bool BIG>
__global__ void __launch_bounds__(64 * TY)
    k_star3d_dpp(const S *__restrict__ in, S *__restrict__ out, Geo g,
                 StarCoef<typename Store<S>::C, R> cf, int lz, int gx, int gy, int gz, int flags)
{
    using C = typename Store<S>::C;
    constexpr uint32_t es = sizeof(S);
    constexpr int OXW = 64 - 2 * R, ROWS = TY * NY;
    // ring of column values: plane p in slot (p - z0 + R) mod NR, PF planes
    // loaded ahead of the window; NR is even (PF odd), so the two-slot ring
    // of the y-halo rows (loaded one plane ahead: they were fetched from HBM
    // by the neighbouring waves already) also has compile-time slots in the
    // march unrolled by NR
    constexpr int NR = 2 * R + 1 + PF;
    static_assert(PF % 2 == 1, "prefetch depth must be odd");

    int lin = blockIdx.x;
    const int total = gx * gy * gz;
    if (flags & STAR_FLAG_XCD) lin = xcd_remap(lin, total);
    const bool yfirst = (flags & STAR_FLAG_YFIRST) != 0;
    const int byi = yfirst ? lin % gy : (lin / gx) % gy;
    const int bxi = yfirst ? (lin / gy) % gx : lin % gx;
    const int bzi = lin / (gx * gy);
    const int tx = threadIdx.x;
    const int x = bxi * OXW - R + tx;
    const int y0 = byi * ROWS + threadIdx.y * NY;
    const int z0 = bzi * lz;
    const int z1 = min(z0 + lz, g.nz);
    const bool fuse = (flags & STAR_FLAG_NOFUSE) == 0;
    const bool xout = tx >= R && tx < 64 - R && x < g.nx;

    // coordinates clamped into the padded array ([-R, n + R) is valid)
    auto cl = [](int v, int n) { return min(max(v, -R), n + R - 1); };
    const int xc = cl(x, g.nx);
    auto col = [&](int yy) { return uint32_t(xc + g.ox + g.sy * (cl(yy, g.ny) + g.ry)) * es; };
    uint32_t own[NY], hal[2 * R];
#pragma unroll
    for (int j = 0; j < NY; ++j) own[j] = col(y0 + j);
#pragma unroll
    for (int m = 0; m < R; ++m) {
        hal[m] = col(y0 - R + m);      // rows y0 - R .. y0 - 1
        hal[R + m] = col(y0 + NY + m); // rows y0 + NY .. y0 + NY + R - 1
    }
    const PlaneSrc<S, BIG> src(in, g.sz, uint64_t(padded_elems(g)));
    // padded plane index of interior plane zz, clamped into the array
    auto pl = [&](int zz) { return src.plane(min(zz, g.nz + R - 1) + g.rz); };

    C ring[NY][NR];
    C yh[2][2 * R];
#pragma unroll
    for (int k = 0; k < 2 * R + PF; ++k) {
        const PlaneRef b = pl(z0 - R + k);
#pragma unroll
        for (int j = 0; j < NY; ++j) ring[j][k] = plane_ld<S>(b, own[j]);
    }
    {
        const PlaneRef b = pl(z0);
#pragma unroll
        for (int m = 0; m < 2 * R; ++m) yh[0][m] = plane_ld<S>(b, hal[m]);
    }
#pragma unroll
    for (int j = 0; j < NY; ++j)
#pragma unroll
        for (int k = 2 * R + PF; k < NR; ++k) ring[j][k] = C(0);
#pragma unroll
    for (int m = 0; m < 2 * R; ++m) yh[1][m] = C(0);

    for (int zb = z0; zb < z1; zb += NR) {
#pragma unroll
        for (int q = 0; q < NR; ++q) {
            const int z = zb + q;
            if (z >= z1)
                break;
#define SL(k_) ((q + R + (k_) + NR) % NR) // slot of plane z + k_
            {
                // plane z + R + PF into the slot of plane z - R - 1; the
                // y-halo rows of plane z + 1 into the other halo slot
                const PlaneRef bw = pl(z + R + PF);
#pragma unroll
                for (int j = 0; j < NY; ++j) ring[j][SL(R + PF)] = plane_ld<S>(bw, own[j]);
                const PlaneRef bh = pl(z + 1);
#pragma unroll
                for (int m = 0; m < 2 * R; ++m) yh[(q + 1) & 1][m] = plane_ld<S>(bh, hal[m]);
            }
#pragma unroll
            for (int j = 0; j < NY; ++j) {
                const C c = ring[j][SL(0)];
                C acc = cf.c0 * c;
#pragma unroll
                for (int m = 1; m <= R; ++m) {
                    acc = fma(cf.zm[m - 1], ring[j][SL(-m)], acc);
                    acc = fma(cf.zp[m - 1], ring[j][SL(m)], acc);
                }
                C lo = c, hi = c;
#pragma unroll
                for (int m = 1; m <= R; ++m) {
                    lo = lane_up(lo);   // column x - m
                    hi = lane_down(hi); // column x + m
                    acc = fma(cf.xm[m - 1], lo, acc);
                    acc = fma(cf.xp[m - 1], hi, acc);
                }
#pragma unroll
                for (int m = 1; m <= R; ++m) {
                    const int jm = j - m, jp = j + m;
                    const C vm = jm >= 0 ? ring[jm >= 0 ? jm : 0][SL(0)] : yh[q & 1][R + jm];
                    const C vp = jp < NY ? ring[jp < NY ? jp : 0][SL(0)]
                                         : yh[q & 1][R + (jp < NY ? 0 : jp - NY)];
                    acc = fma(cf.ym[m - 1], vm, acc);
                    acc = fma(cf.yp[m - 1], vp, acc);
                }
                const int y = y0 + j;
                if (xout && y < g.ny)
                    store_periodic(out, g, x, y, z, acc, fuse);
            }
#undef SL
        }
    }
}

template <typename S, int R, int NY, int TY, int PF>
int launch_star3d_dpp_t(const S *in, S *out, const Geo &g,
                        const StarCoef<typename Store<S>::C, R> &cf, int lz, int flags,
                        hipStream_t s)
{
    constexpr int OXW = 64 - 2 * R, ROWS = TY * NY;
    const int gx = (g.nx + OXW - 1) / OXW, gy = (g.ny + ROWS - 1) / ROWS,
              gz = (g.nz + lz - 1) / lz;
    const int64_t total = (int64_t)gx * gy * gz;
    if (total > 0x7fffffff)
        return fail(STENCIL_EUNSUPPORTED, "star3d (lane exchange): grid too large");
    const bool big = uint64_t(padded_elems(g)) * sizeof(S) >= (uint64_t(1) << 32);
    if (big)
        hipLaunchKernelGGL((k_star3d_dpp<S, R, NY, TY, PF, true>), dim3((unsigned)total),
                           dim3(64, TY), 0, s, in, out, g, cf, lz, gx, gy, gz, flags);
    else
        hipLaunchKernelGGL((k_star3d_dpp<S, R, NY, TY, PF, false>), dim3((unsigned)total),
                           dim3(64, TY), 0, s, in, out, g, cf, lz, gx, gy, gz, flags);
    return check_launch("xcorr_star3d_dpp");
}

template <typename S, int R>
int launch_star3d_dpp_r(const S *in, S *out, const Geo &g,
                        const StarCoef<typename Store<S>::C, R> &cf, int ty, int ny, int pf,
                        int lz, int flags, hipStream_t s)
{
    if (pf == 0 || pf == 2) // the tile word's default depth: one plane ahead here
        pf = 1;
#define STAR_DPP_CASE(TY_, NY_)                                                              \
    if (ty == TY_ && ny == NY_ && pf == 1)                                                   \
        return launch_star3d_dpp_t<S, R, NY_, TY_, 1>(in, out, g, cf, lz, flags, s);          \
    if (ty == TY_ && ny == NY_ && pf == 3)                                                   \
        return launch_star3d_dpp_t<S, R, NY_, TY_, 3>(in, out, g, cf, lz, flags, s);
    STAR_DPP_SHAPES(STAR_DPP_CASE)
#undef STAR_DPP_CASE
    return fail(STENCIL_EUNSUPPORTED,
                "star3d (lane exchange): unsupported tile (ty=%d, ny=%d, prefetch %d)", ty, ny, pf);
}

} // namespace stn
