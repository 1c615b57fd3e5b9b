// linear_kernels.hpp -- launchers of the linear-path kernels (internal).
#pragma once

#include "common.hpp"

namespace stn {

// Axis-aligned (star) coefficients of radius R: centre, and per axis the taps
// at -m (xm[m-1]) and +m (xp[m-1]), m = 1..R. Passed by value as kernel
// arguments, so they sit in scalar registers.
template <typename C, int R> struct StarCoef {
    C c0;
    C xm[R], xp[R], ym[R], yp[R], zm[R], zp[R];
};

constexpr int STAR_MAX_R = 4;

struct StarCoefAny {
    double c0;
    double xm[STAR_MAX_R], xp[STAR_MAX_R], ym[STAR_MAX_R], yp[STAR_MAX_R];
    double zm[STAR_MAX_R], zp[STAR_MAX_R];

    template <typename C, int R> StarCoef<C, R> get() const
    {
        StarCoef<C, R> o;
        o.c0 = static_cast<C>(c0);
        for (int m = 0; m < R; ++m) {
            o.xm[m] = static_cast<C>(xm[m]);
            o.xp[m] = static_cast<C>(xp[m]);
            o.ym[m] = static_cast<C>(ym[m]);
            o.yp[m] = static_cast<C>(yp[m]);
            o.zm[m] = static_cast<C>(zm[m]);
            o.zp[m] = static_cast<C>(zp[m]);
        }
        return o;
    }
};

// Dense box coefficients of radius R: c[((dz + R) W + dy + R) W + dx + R],
// W = 2R + 1. Passed by value as a kernel argument.
template <typename C, int R> struct BoxCoef {
    C c[(2 * R + 1) * (2 * R + 1) * (2 * R + 1)];
};

constexpr int BOX_MAX_R = 1; // dense boxes with a dedicated kernel: radius 1

struct BoxCoefAny {
    int R;
    double c[(2 * BOX_MAX_R + 1) * (2 * BOX_MAX_R + 1) * (2 * BOX_MAX_R + 1)];

    template <typename C, int RR> BoxCoef<C, RR> get() const
    {
        BoxCoef<C, RR> o;
        for (int k = 0; k < (2 * RR + 1) * (2 * RR + 1) * (2 * RR + 1); ++k)
            o.c[k] = static_cast<C>(c[k]);
        return o;
    }
};

// star kernel flags (the tile[3] word of stencil_desc)
constexpr int STAR_FLAG_XCD = 1;    // XCD-aware workgroup order
constexpr int STAR_FLAG_NOFUSE = 2; // do not write periodic images
constexpr int STAR_FLAG_YFIRST = 4; // tile numbers run fastest along y
constexpr int STAR_FLAG_HWC = 8;    // hardware-cached z march (no LDS)
constexpr int STAR_FLAG_PAIRS = 16; // two-iteration march with pair-layout LDS planes
constexpr int STAR_FLAG_DPP = 32;   // one-iteration march, x taps across lanes (no LDS)
constexpr int STAR_PF_SHIFT = 4;    // bits 4..7: prefetch depth (0 = default)
constexpr int STAR_XW_SHIFT = 8;    // bits 8..11: tile width in waves (0 = 1)
constexpr int STAR_T_SHIFT = 12;    // bits 12..15: iterations per launch (0/1 = 1, or 2)
constexpr int STAR_PAIRS_BIT = 1 << 16; // bit 16: pair-layout LDS planes (two iterations)
constexpr int STAR_DPP_BIT = 1 << 17;   // bit 17: x taps across lanes (one iteration; filters too)


template <typename S> int launch_halo(S *a, const Geo &g, hipStream_t s);

template <typename S>
int launch_generic(const S *in, S *out, const Geo &g, const int *offs,
                   const typename Store<S>::C *cs, int ntaps, bool fuse, int bx, int by,
                   hipStream_t s);

// 3-D star kernel (star3d.hpp), one overload per storage type (star3d_*.hip).
// R: tap radius (<= padding); xw, ty, ny: tile shape (64*xw x ty*ny points);
// pf: prefetch depth; lz: z planes per workgroup; flags: STAR_FLAG_*.
#define STAR_DECL(S)                                                                         \
    int launch_star3d(const S *in, S *out, const Geo &g, const StarCoefAny &cf, int R, int xw, \
                      int ty, int ny, int pf, int lz, int flags, hipStream_t s);              \
    int launch_star3d_t2(const S *in, S *out, const Geo &g, const StarCoefAny &cf, int R,      \
                         int xw, int ty, int ny, int lz, int flags, hipStream_t s);
STAR_DECL(double)
STAR_DECL(float)
STAR_DECL(bf16)
#undef STAR_DECL

// Dense 3-D box (box3d.hpp), one overload per storage type (box3d_*.hip):
// ty waves per workgroup, ny rows per lane, pf planes in flight (1 or 3; 0
// and 2 mean 1), lz z planes per workgroup, flags: STAR_FLAG_XCD / NOFUSE.
#define BOX_DECL(S)                                                                          \
    int launch_box3d(const S *in, S *out, const Geo &g, const BoxCoefAny &cf, int ty, int ny, \
                     int pf, int lz, int flags, hipStream_t s);
BOX_DECL(double)
BOX_DECL(float)
BOX_DECL(bf16)
#undef BOX_DECL

// Dense 3-D box of radius R = 1 .. 8, or 2-D box (box3d_lds.hpp), one overload
// per storage type (box3d_lds_*.hip): cf = the (2R+1)^ndim coefficients on the
// device in the arithmetic type, z, y, x order; e outputs per lane along x (4
// or 8; 4 for 3-D boxes of radius 5 .. 8),
// ty waves per workgroup (4), lz z planes per workgroup, flags:
// STAR_FLAG_XCD. Writes the output interior only.
#define BOXL_DECL(S)                                                                         \
    int launch_box3d_lds(const S *in, S *out, const Geo &g, int R, const void *cf, int e,      \
                         int ty, int lz, int flags, hipStream_t s);
BOXL_DECL(double)
BOXL_DECL(float)
BOXL_DECL(bf16)
#undef BOXL_DECL
constexpr int BOX_LDS_MAX_R = 8;

template <typename S>
int launch_line1d(const S *in, S *out, const Geo &g, const typename Store<S>::C *cs, bool fuse,
                  int e, hipStream_t s);

// T chained iterations of a 1-D stencil in one launch (periodic only; reads
// the interior with wrap, writes the output interior and its images).
template <typename S>
int launch_line1d_t(const S *in, S *out, const Geo &g, const typename Store<S>::C *cs, bool fuse,
                    int e, int T, hipStream_t s);

// Register-blocked 1-D line: e in {4, 8, 16} adjacent outputs per lane, for
// large radii (2r + 1 >= e - 1); bitwise equal to launch_line1d.
template <typename S>
int launch_line1d_rb(const S *in, S *out, const Geo &g, const typename Store<S>::C *cs,
                     bool fuse, int e, hipStream_t s);

int launch_copy(const void *src, void *dst, size_t nbytes, hipStream_t s);

} // namespace stn
