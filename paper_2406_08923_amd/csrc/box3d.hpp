// box3d.hpp -- dense 3-D box cross-correlation (Eq. 3 with every tap of the
// (2R+1)^3 box nonzero) as a z march with no LDS: the regime where the taps,
// not HBM, set the cost ((2R+1)^3 multiply-adds per point). Built for R = 1
// (27 taps, whose coefficients stay in scalar registers); at R = 2 .. 4 the
// 125 .. 729 coefficients, with the fully unrolled tap loops this ring of
// partial sums needs, do not fit the register files, so those boxes run the
// LDS march of box3d_lds.hpp instead, which is also the default at R = 1
// (this march is chosen by tiles of 1 or 2 rows per lane).
//
// A wave is one row of 64 consecutive columns: lane tx holds column
// x0 - R + tx (the 2R edge lanes only feed their neighbours, so a wave yields
// 64 - 2R columns) and NY consecutive rows. The march reads each input plane
// once: per plane a lane loads its column over its rows and R rows on either
// side, forms the 2R + 1 x-shifted copies of those values with one-lane DPP
// moves, and adds every tap's product into the partial sums of the 2R + 1
// output planes the input plane contributes to (a register ring of partial
// sums per row). The output plane z - R is then complete and stored. The
// loads of the next planes are in flight meanwhile. Per output the taps are
// summed input plane by input plane (z offset -R .. R), and within a plane by
// x offset (0, -1, +1, ..., -R, +R), then y offset, a fixed order the FP64
// tolerance covers.
#pragma once

#include "linear_kernels.hpp"

namespace stn {

// Shapes (TY, NY): TY waves per workgroup stacked along y, NY rows per lane.
#define BOX3D_SHAPES(X) X(4, 1) X(4, 2) X(8, 1) X(8, 2)

template <typename S, int R, int NY, int TY, int PF, bool BIG>
__global__ void __launch_bounds__(64 * TY)
    k_box3d_dpp(const S *__restrict__ in, S *__restrict__ out, Geo g,
                BoxCoef<typename Store<S>::C, R> cf, int lz, int gx, int gy, int gz, int flags)
{
    using C = typename Store<S>::C;
    constexpr uint32_t es = sizeof(S);
    constexpr int W = 2 * R + 1, NL = NY + 2 * R, OXW = 64 - 2 * R, ROWS = TY * NY;
    constexpr int NP = PF + 1;             // prefetch buffers
    constexpr int U = lcm_int(W, NP);      // steps per unrolled round
    auto coef = [&](int dz, int dy, int dx) { return cf.c[((dz + R) * W + (dy + R)) * W + dx + R]; };

    int lin = blockIdx.x;
    const int total = gx * gy * gz;
    if (flags & STAR_FLAG_XCD) lin = xcd_remap(lin, total);
    const int bxi = lin % gx, byi = (lin / gx) % gy, bzi = lin / (gx * gy);
    const int tx = threadIdx.x;
    const int x = bxi * OXW - R + tx;
    const int y0 = byi * ROWS + threadIdx.y * NY;
    const int z0 = bzi * lz, z1 = min(z0 + lz, g.nz);
    const bool fuse = (flags & STAR_FLAG_NOFUSE) == 0;
    const bool xout = tx >= R && tx < 64 - R && x < g.nx;

    // padded coordinates clamped into the array ([-R, n + R) is valid; the
    // taps read the input halo)
    auto cl = [](int v, int n) { return min(max(v, -R), n + R - 1); };
    const int xc = cl(x, g.nx);
    uint32_t off[NL];
#pragma unroll
    for (int i = 0; i < NL; ++i)
        off[i] = uint32_t(xc + g.ox + g.sy * (cl(y0 - R + i, g.ny) + g.ry)) * es;
    const PlaneSrc<S, BIG> src(in, g.sz, uint64_t(padded_elems(g)));
    auto pl = [&](int zz) { return src.plane(zz + g.rz); };

    // partial sums: output plane zo in slot (zo - zs) mod W
    C acc[NY][W];
#pragma unroll
    for (int j = 0; j < NY; ++j)
#pragma unroll
        for (int k = 0; k < W; ++k) acc[j][k] = C(0);
    C pre[NP][NL];
    const int zs = z0 - R, ze = z1 + R; // input planes zs .. ze - 1
#pragma unroll
    for (int b = 0; b < NP; ++b) {
        const PlaneRef pb = pl(min(zs + b, ze - 1));
#pragma unroll
        for (int i = 0; i < NL; ++i) pre[b][i] = b < PF ? plane_ld<S>(pb, off[i]) : C(0);
    }

    for (int zb = zs; zb < ze; zb += U) {
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int p = zb + q; // input plane
            if (p >= ze)
                break;
            if (p + PF < ze) {
                const PlaneRef pb = pl(p + PF);
#pragma unroll
                for (int i = 0; i < NL; ++i) pre[(q + PF) % NP][i] = plane_ld<S>(pb, off[i]);
            }
            // output plane p + R (slot (q + R) mod W) starts here; the slot
            // held output plane p - R - 1, stored at the previous step
#pragma unroll
            for (int j = 0; j < NY; ++j) acc[j][(q + R) % W] = C(0);
            C v[NL], lo[NL], hi[NL];
#pragma unroll
            for (int i = 0; i < NL; ++i) lo[i] = hi[i] = v[i] = pre[q % NP][i];
            // input plane p feeds output plane p - dz with tap dz
            auto add = [&](int dx, const C (&s)[NL]) {
#pragma unroll
                for (int dz = -R; dz <= R; ++dz)
#pragma unroll
                    for (int j = 0; j < NY; ++j)
#pragma unroll
                        for (int dy = -R; dy <= R; ++dy) {
                            C &a = acc[j][(q - dz + 2 * W) % W];
                            a = fma(coef(dz, dy, dx), s[j + R + dy], a);
                        }
            };
            add(0, v);
#pragma unroll
            for (int m = 1; m <= R; ++m) {
#pragma unroll
                for (int i = 0; i < NL; ++i) {
                    lo[i] = lane_up(lo[i]);   // column x - m
                    hi[i] = lane_down(hi[i]); // column x + m
                }
                add(-m, lo);
                add(m, hi);
            }
            // output plane p - R is complete
            const int zo = p - R;
            if (zo >= z0) {
#pragma unroll
                for (int j = 0; j < NY; ++j) {
                    const int y = y0 + j;
                    if (xout && y < g.ny)
                        store_periodic(out, g, x, y, zo, acc[j][(q - R + 2 * W) % W], fuse);
                }
            }
        }
    }
}

template <typename S, int R, int NY, int TY, int PF>
int launch_box3d_t(const S *in, S *out, const Geo &g, const BoxCoef<typename Store<S>::C, R> &cf,
                   int lz, int flags, hipStream_t s)
{
    constexpr int OXW = 64 - 2 * R, ROWS = TY * NY;
    const int gx = (g.nx + OXW - 1) / OXW, gy = (g.ny + ROWS - 1) / ROWS,
              gz = (g.nz + lz - 1) / lz;
    const int64_t total = (int64_t)gx * gy * gz;
    if (total > 0x7fffffff)
        return fail(STENCIL_EUNSUPPORTED, "box3d: grid too large");
    const bool big = uint64_t(padded_elems(g)) * sizeof(S) >= (uint64_t(1) << 32);
    if (big)
        hipLaunchKernelGGL((k_box3d_dpp<S, R, NY, TY, PF, true>), dim3((unsigned)total),
                           dim3(64, TY), 0, s, in, out, g, cf, lz, gx, gy, gz, flags);
    else
        hipLaunchKernelGGL((k_box3d_dpp<S, R, NY, TY, PF, false>), dim3((unsigned)total),
                           dim3(64, TY), 0, s, in, out, g, cf, lz, gx, gy, gz, flags);
    return check_launch("xcorr_box3d");
}

template <typename S, int R>
int launch_box3d_r(const S *in, S *out, const Geo &g, const BoxCoef<typename Store<S>::C, R> &cf,
                   int ty, int ny, int pf, int lz, int flags, hipStream_t s)
{
    if (pf == 0 || pf == 2) // the tile word's default depth: one plane ahead here
        pf = 1;
#define BOX3D_CASE(TY_, NY_)                                                                 \
    if (ty == TY_ && ny == NY_ && pf == 1)                                                   \
        return launch_box3d_t<S, R, NY_, TY_, 1>(in, out, g, cf, lz, flags, s);               \
    if (ty == TY_ && ny == NY_ && pf == 3)                                                   \
        return launch_box3d_t<S, R, NY_, TY_, 3>(in, out, g, cf, lz, flags, s);
    BOX3D_SHAPES(BOX3D_CASE)
#undef BOX3D_CASE
    return fail(STENCIL_EUNSUPPORTED, "box3d: unsupported tile (ty=%d, ny=%d, prefetch %d)", ty,
                ny, pf);
}

template <typename S>
int launch_box3d_impl(const S *in, S *out, const Geo &g, const BoxCoefAny &cfa, int ty, int ny,
                      int pf, int lz, int flags, hipStream_t s)
{
    using C = typename Store<S>::C;
    if (g.ndim != 3 || cfa.R < 1 || cfa.R > g.r)
        return fail(STENCIL_EINVAL, "box3d: needs a 3-D box of radius 1..padding");
    if (lz < 1)
        return fail(STENCIL_EINVAL, "box3d: z planes per workgroup must be >= 1");
    if (cfa.R == 1)
        return launch_box3d_r<S, 1>(in, out, g, cfa.get<C, 1>(), ty, ny, pf, lz, flags, s);
    return fail(STENCIL_EUNSUPPORTED, "box3d: radius %d boxes are not built (radius 1 only)", cfa.R);
}

} // namespace stn
