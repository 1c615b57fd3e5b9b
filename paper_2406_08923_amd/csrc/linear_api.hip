// linear_api.hip -- C ABI of the linear path: plans, variant choice and
// autotuning, chained application with periodic halos, finite-difference
// weights, copy.
#include "linear_kernels.hpp"
#include "filter_kernels.hpp"
#include "plan.hpp"
#include "tune_cache.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

namespace stn {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------

static thread_local char g_err[1024] = "";

int fail(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

int check_launch(const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return fail(STENCIL_EDEVICE, "%s launch failed: %s", what, hipGetErrorString(e));
    return STENCIL_OK;
}

// ---------------------------------------------------------------------------
// validation helpers
// ---------------------------------------------------------------------------

// Largest radius a plan accepts: 1-D lines reach the large-radius regime of
// the paper's radius study (Sec. 5, Fig. 8); multi-dimensional dense boxes
// stop at 8 ((2r+1)^3 = 4913 taps).
int max_radius(int ndim) { return ndim == 1 ? 1024 : 8; }

int check_dims(int ndim, const int *dims, int r, int bc)
{
    if (ndim < 1 || ndim > 3)
        return fail(STENCIL_EINVAL, "ndim must be 1, 2 or 3 (got %d)", ndim);
    if (!dims)
        return fail(STENCIL_EINVAL, "dims is NULL");
    int64_t cells = 1;
    for (int a = 0; a < ndim; ++a) {
        if (dims[a] < 1)
            return fail(STENCIL_EINVAL, "dims[%d] = %d must be >= 1", a, dims[a]);
        if (bc == STENCIL_BC_PERIODIC && dims[a] < r)
            return fail(STENCIL_EINVAL, "periodic padding needs dims[%d] = %d >= radius %d", a,
                        dims[a], r);
        cells *= (int64_t)dims[a] + 2 * r;
    }
    if (cells > (int64_t(1) << 40))
        return fail(STENCIL_EINVAL, "padded array too large");
    return STENCIL_OK;
}

int check_buffers(const void *a, const void *b, size_t bytes, size_t align)
{
    if (!a || !b)
        return fail(STENCIL_EINVAL, "NULL device buffer");
    auto ua = reinterpret_cast<uintptr_t>(a), ub = reinterpret_cast<uintptr_t>(b);
    if (ua % align || ub % align)
        return fail(STENCIL_EINVAL, "device buffer not aligned to %zu bytes", align);
    if (ua < ub + bytes && ub < ua + bytes)
        return fail(STENCIL_EINVAL, "input and output buffers overlap");
    return STENCIL_OK;
}

int check_device(int plan_device)
{
    int dev = -1;
    STN_HIP(hipGetDevice(&dev));
    if (dev != plan_device)
        return fail(STENCIL_EINVAL, "plan was created on device %d but device %d is current",
                    plan_device, dev);
    return STENCIL_OK;
}

} // namespace stn

using namespace stn;

// ---------------------------------------------------------------------------
// plan internals
// ---------------------------------------------------------------------------

namespace {

struct TuneChoice {
    int variant, p0, p1, p2, p3;
};

// Dense 2-D boxes (the LDS march over row blocks, 8 waves per workgroup):
// outputs per lane. The
// march addresses the array with 32-bit offsets, so it takes arrays below
// 4 GiB; larger ones stay on the gather kernel.
constexpr int BOX2D_DEFAULT_E = 4;

// the dense box runs the LDS march (box3d_lds.hpp): every 2-D box and 3-D box
// of radius 2..4; at radius 1 when the tile asks for 4 or 8 outputs per lane
// (1 or 2 rows per lane select the lane-exchange march)
bool box_lds(const LinearPlan &L)
{
    return L.reff >= 2 || L.g.ndim == 2 || L.ny >= 4;
}

bool box2d_fits(const stencil_plan_s *p)
{
    return uint64_t(padded_elems(p->lin.g)) * dtype_size(p->lin.dtype) < (uint64_t(1) << 32);
}


template <typename S> int run_linear_once(stencil_plan_s *p, const S *in, S *out, hipStream_t s)
{
    using C = typename Store<S>::C;
    const bool periodic = p->lin.bc == STENCIL_BC_PERIODIC;
    int rc;
    if (p->lin.op != STENCIL_OP_XCORR) {
        if (p->lin.variant == STENCIL_VARIANT_STAR3D)
            return launch_filter_box3d<S>(in, out, p->lin.g, p->lin.reff, p->lin.op, periodic,
                                          p->lin.ty, p->lin.ny, p->lin.pf, p->lin.lz,
                                          p->lin.dpp != 0,
                                          p->lin.sflags & STAR_FLAG_XCD, s);
        return launch_filter_gather<S>(in, out, p->lin.g, static_cast<const int *>(p->lin.d_offs),
                                       p->lin.ntaps, p->lin.op, periodic, p->lin.gbx, p->lin.gby,
                                       s);
    }
    switch (p->lin.variant) {
    case STENCIL_VARIANT_STAR3D: {
        int fl = p->lin.sflags | (periodic ? 0 : STAR_FLAG_NOFUSE);
        rc = launch_star3d(in, out, p->lin.g, p->lin.star, p->lin.reff, p->lin.xw, p->lin.ty,
                           p->lin.ny, p->lin.pf, p->lin.lz,
                           (fl & 15) | (p->lin.dpp ? STAR_FLAG_DPP : 0), s);
        if (rc == STENCIL_OK && periodic && (p->lin.sflags & STAR_FLAG_NOFUSE))
            rc = launch_halo<S>(out, p->lin.g, s);
        return rc;
    }
    case STENCIL_VARIANT_BOX3D:
        if (box_lds(p->lin)) {
            // 3-D radius 2..4, 2-D boxes, and the 27-point box with 4 or 8
            // outputs per lane: the LDS march writes the interior; the halo
            // refresh follows on periodic plans
            rc = launch_box3d_lds(in, out, p->lin.g, p->lin.reff, p->lin.d_taps, p->lin.ny,
                                  p->lin.ty, p->lin.lz, p->lin.sflags & STAR_FLAG_XCD, s);
            if (rc == STENCIL_OK && periodic)
                rc = launch_halo<S>(out, p->lin.g, s);
            return rc;
        }
        return launch_box3d(in, out, p->lin.g, p->lin.box, p->lin.ty, p->lin.ny, p->lin.pf,
                            p->lin.lz, (p->lin.sflags & STAR_FLAG_XCD) | (periodic ? 0 : STAR_FLAG_NOFUSE),
                            s);
    case STENCIL_VARIANT_LINE1D:
        if (p->lin.rb1d)
            return launch_line1d_rb<S>(in, out, p->lin.g, static_cast<const C *>(p->lin.d_dense),
                                       periodic, p->lin.e1d, s);
        return launch_line1d<S>(in, out, p->lin.g, static_cast<const C *>(p->lin.d_dense),
                                periodic, p->lin.e1d, s);
    default:
        return launch_generic<S>(in, out, p->lin.g, static_cast<const int *>(p->lin.d_offs),
                                 static_cast<const C *>(p->lin.d_taps), p->lin.ntaps, periodic,
                                 p->lin.gbx, p->lin.gby, s);
    }
}

template <typename S>
int apply_t(stencil_plan_s *p, void *da, void *db, int iters, hipStream_t s, bool halo_valid)
{
    S *a = static_cast<S *>(da), *b = static_cast<S *>(db);
    int rc = STENCIL_OK;
    if (p->lin.bc == STENCIL_BC_PERIODIC && p->lin.variant == STENCIL_VARIANT_LINE1D &&
        p->lin.t1d > 1 && p->lin.op == STENCIL_OP_XCORR) {
        // temporally blocked: nl launches of up to T iterations each, with nl
        // of the same parity as iters so the result lands where the
        // one-iteration-per-launch contract puts it
        using C = typename Store<S>::C;
        const int T = p->lin.t1d;
        int nl = (iters + T - 1) / T;
        if ((nl & 1) != (iters & 1))
            ++nl;
        int done = 0;
        for (int k = 0; k < nl && rc == STENCIL_OK; ++k) {
            const int left = nl - k;
            const int tk = (iters - done + left - 1) / left;
            rc = launch_line1d_t<S>(a, b, p->lin.g, static_cast<const C *>(p->lin.d_dense), true,
                                    p->lin.e1d, tk, s);
            done += tk;
            std::swap(a, b);
        }
        return rc;
    }
    if (p->lin.bc == STENCIL_BC_PERIODIC && p->lin.variant == STENCIL_VARIANT_STAR3D &&
        p->lin.tstar == 2 && p->lin.op == STENCIL_OP_XCORR) {
        // nl launches of two or one iterations, nl of the parity of iters;
        // the two-iteration launches come first. They read the input with
        // periodic wrap, never its halo, so only the last of them writes
        // its output's periodic images (which the one-iteration launches
        // after it and the caller read).
        int nl = (iters + 1) / 2;
        if ((nl & 1) != (iters & 1))
            ++nl;
        const int n2 = iters - nl, n1 = nl - n2;
        const int fl = (p->lin.sflags & (STAR_FLAG_XCD | STAR_FLAG_YFIRST)) |
                       (p->lin.pairs ? STAR_FLAG_PAIRS : 0);
        if (n2 == 0 && !halo_valid)
            rc = launch_halo<S>(a, p->lin.g, s);
        for (int k = 0; k < n2 && rc == STENCIL_OK; ++k) {
            rc = launch_star3d_t2(a, b, p->lin.g, p->lin.star, p->lin.reff, p->lin.xw, p->lin.ty,
                                  p->lin.ny, p->lin.lz, fl | (k + 1 < n2 ? STAR_FLAG_NOFUSE : 0),
                                  s);
            std::swap(a, b);
        }
        const int *q = p->lin.s1;
        for (int k = 0; k < n1 && rc == STENCIL_OK; ++k) {
            rc = launch_star3d(a, b, p->lin.g, p->lin.star, p->lin.reff, q[4], q[0], q[1], 2,
                               q[2], q[3] & 15, s);
            std::swap(a, b);
        }
        return rc;
    }
    if (p->lin.bc == STENCIL_BC_PERIODIC && !halo_valid)
        rc = launch_halo<S>(a, p->lin.g, s);
    for (int k = 0; k < iters && rc == STENCIL_OK; ++k) {
        rc = run_linear_once<S>(p, a, b, s);
        std::swap(a, b);
    }
    return rc;
}

int apply_any(stencil_plan_s *p, void *a, void *b, int iters, hipStream_t s,
              bool halo_valid = false)
{
    switch (p->lin.dtype) {
    case STENCIL_F64: return apply_t<double>(p, a, b, iters, s, halo_valid);
    case STENCIL_F32: return apply_t<float>(p, a, b, iters, s, halo_valid);
    default: return apply_t<bf16>(p, a, b, iters, s, halo_valid);
    }
}

std::string tune_key(const stencil_plan_s *p)
{
    char buf[256];
    snprintf(buf, sizeof(buf), "lin|dt%d|nd%d|%dx%dx%d|r%d|ox%d|sy%lld|reff%d|star%d|bc%d|nt%d|op%d|box%d",
             p->lin.dtype, p->lin.g.ndim, p->lin.g.nx, p->lin.g.ny, p->lin.g.nz, p->lin.g.r,
             p->lin.g.ox, (long long)p->lin.g.sy, p->lin.reff, p->lin.is_star ? 1 : 0, p->lin.bc,
             p->lin.ntaps, p->lin.op, p->lin.is_box ? 1 : 0);
    return buf;
}

void set_choice(stencil_plan_s *p, const TuneChoice &c)
{
    p->lin.variant = c.variant;
    if (c.variant == STENCIL_VARIANT_STAR3D) {
        p->lin.ty = c.p0;
        p->lin.ny = c.p1;
        p->lin.lz = c.p2;
        p->lin.sflags = c.p3 & 15;
        const int pf = (c.p3 >> STAR_PF_SHIFT) & 15;
        const int xw = (c.p3 >> STAR_XW_SHIFT) & 15;
        const int t = (c.p3 >> STAR_T_SHIFT) & 15;
        p->lin.pf = pf ? pf : 2;
        p->lin.xw = xw ? xw : 1;
        p->lin.tstar = t == 2 ? 2 : 1;
        p->lin.pairs = (c.p3 & STAR_PAIRS_BIT) != 0 && t == 2;
        p->lin.dpp = (c.p3 & STAR_DPP_BIT) != 0 && t != 2;
    } else if (c.variant == STENCIL_VARIANT_BOX3D) {
        p->lin.ty = c.p0;
        p->lin.ny = c.p1;
        p->lin.lz = c.p2;
        p->lin.sflags = c.p3 & STAR_FLAG_XCD;
        const int pf = (c.p3 >> STAR_PF_SHIFT) & 15;
        p->lin.pf = pf ? pf : 1;
    } else if (c.variant == STENCIL_VARIANT_LINE1D) {
        p->lin.e1d = c.p0;
        p->lin.t1d = c.p1 > 1 ? c.p1 : 1;
        p->lin.rb1d = c.p2 ? 1 : 0;
    } else {
        p->lin.gbx = c.p0;
        p->lin.gby = c.p1;
    }
}

std::vector<TuneChoice> candidates(const stencil_plan_s *p)
{
    std::vector<TuneChoice> c;
    const Geo &g = p->lin.g;
    if (p->lin.op != STENCIL_OP_XCORR) {
        if (p->lin.is_box && p->lin.op != STENCIL_OP_MEDIAN) {
            for (int ty : {4, 8})
                for (int lz : {16, 32, 64})
                    c.push_back({STENCIL_VARIANT_STAR3D, ty, 1, lz, 0});
            // lane-exchange march: (waves per workgroup, rows per lane), one
            // or three planes in flight (three with four rows: radius 1 only)
            for (int ty : {4, 8})
                for (int ny : {2, 4})
                    for (int lz : {4, 8, 16, 32})
                        for (int pf : {1, 3})
                            if (pf == 1 || ny == 2 || p->lin.reff == 1)
                                c.push_back({STENCIL_VARIANT_STAR3D, ty, ny, lz,
                                             STAR_FLAG_XCD | STAR_DPP_BIT | (pf << STAR_PF_SHIFT)});
        }
        c.push_back({STENCIL_VARIANT_GENERIC, 64, 4, 0, 0});
        c.push_back({STENCIL_VARIANT_GENERIC, 64, 8, 0, 0});
        c.push_back({STENCIL_VARIANT_GENERIC, 128, 2, 0, 0});
        return c;
    }
    if (p->lin.is_star) {
        // (x waves, y lanes, rows per lane): tiles 64*xw x ty*ny
        const int shapes[][3] = {{1, 8, 2}, {1, 4, 4}, {1, 8, 4}, {1, 16, 2}, {2, 4, 2}, {2, 4, 4},
                                 {2, 8, 2}, {4, 2, 2}, {4, 2, 4}, {4, 4, 2}, {8, 1, 4}, {8, 2, 2}};
        const int lzs[] = {32, 64, 128, g.nz};
        for (auto &sh : shapes) {
            if (64 * sh[0] > 2 * g.nx && sh[0] > 1)
                continue; // tiles much wider than the grid only add idle lanes
            for (int k = 0; k < 4; ++k) {
                const int lz = lzs[k];
                if ((k < 3 && lz >= g.nz && lz != 32) || (k == 3 && g.nz <= 32))
                    continue;
                const int w = (2 << STAR_PF_SHIFT) | (sh[0] << STAR_XW_SHIFT);
                c.push_back({STENCIL_VARIANT_STAR3D, sh[1], sh[2], lz, w | STAR_FLAG_XCD});
                c.push_back({STENCIL_VARIANT_STAR3D, sh[1], sh[2], lz,
                             w | STAR_FLAG_XCD | STAR_FLAG_YFIRST});
            }
        }
        // two iterations per launch (periodic): (x waves, y lanes, rows per lane)
        if (p->lin.bc == STENCIL_BC_PERIODIC) {
            const int t2[][3] = {{1, 8, 2}, {1, 16, 1}, {1, 16, 2}, {1, 12, 2}, {2, 8, 2}, {1, 8, 4}};
            for (auto &sh : t2)
                for (int lz : {32, 64, 128}) {
                    if (lz >= g.nz && lz != 32)
                        continue;
                    const int w = STAR_FLAG_XCD | (sh[0] << STAR_XW_SHIFT) | (2 << STAR_T_SHIFT);
                    c.push_back({STENCIL_VARIANT_STAR3D, sh[1], sh[2], lz, w});
                    if (sh[2] == 2 && p->lin.reff <= 4 && 64 * sh[0] * sh[1] <= 768)
                        c.push_back({STENCIL_VARIANT_STAR3D, sh[1], sh[2], lz, w | STAR_PAIRS_BIT});
                    if (sh[2] == 4 && p->lin.dtype != STENCIL_F64 && sh[0] == 1 &&
                        64 * sh[1] <= 768)
                        c.push_back({STENCIL_VARIANT_STAR3D, sh[1], sh[2], lz, w | STAR_PAIRS_BIT});
                }
        }
        // lane-exchange z march: (waves per workgroup, rows per lane)
        const int dshapes[][2] = {{4, 2}, {4, 4}, {8, 2}, {8, 4}};
        for (auto &sh : dshapes)
            for (int k = 0; k < 3; ++k) {
                const int lz = lzs[k];
                if (lz >= g.nz && lz != 32)
                    continue;
                c.push_back({STENCIL_VARIANT_STAR3D, sh[0], sh[1], lz, STAR_FLAG_XCD | STAR_DPP_BIT});
                c.push_back({STENCIL_VARIANT_STAR3D, sh[0], sh[1], lz,
                             STAR_FLAG_XCD | STAR_FLAG_YFIRST | STAR_DPP_BIT});
            }
        // hardware-cached z march: (lanes along y, rows per lane)
        const int hshapes[][2] = {{4, 1}, {4, 2}, {4, 4}, {2, 4}, {8, 2}};
        for (auto &sh : hshapes)
            for (int k = 0; k < 3; ++k) {
                const int lz = lzs[k];
                if (lz >= g.nz && lz != 32)
                    continue;
                c.push_back({STENCIL_VARIANT_STAR3D, sh[0], sh[1], lz, STAR_FLAG_HWC | STAR_FLAG_XCD});
                c.push_back({STENCIL_VARIANT_STAR3D, sh[0], sh[1], lz, STAR_FLAG_HWC});
            }
    }
    if (g.ndim == 1) {
        for (int e : {1, 2, 4, 8})
            for (int T : {1, 4, 8, 16})
                // fused iterations only where the block's apron (r*T cells a
                // side) stays within the block it serves
                if (T == 1 || (p->lin.bc == STENCIL_BC_PERIODIC && 2 * g.r * T <= 256 * e))
                    c.push_back({STENCIL_VARIANT_LINE1D, e, T, 0, 0});
        // register-blocked lines for the large-radius regime
        for (int e : {4, 8, 16})
            if (2 * g.r + 1 >= e - 1 && g.r >= 8)
                c.push_back({STENCIL_VARIANT_LINE1D, e, 1, 1, 0});
    }
    if (p->lin.is_dense3 && p->lin.reff >= 2)
        for (int e : {4, 8})
            for (int lz : {32, 64, 128})
                if (e == 4 || p->lin.reff <= 4)
                    c.push_back({STENCIL_VARIANT_BOX3D, 4, e, lz, STAR_FLAG_XCD});
    if (p->lin.is_dense2 && box2d_fits(p))
        for (int ty : {4, 8})
            for (int e : {4, 8})
                for (int lz : {1, 4, 16})
                    c.push_back({STENCIL_VARIANT_BOX3D, ty, e, lz, STAR_FLAG_XCD});
    if (p->lin.is_dense3 && p->lin.reff == 1)
        for (int ty : {4, 8})
            for (int e : {4, 8})
                for (int lz : {32, 64, 128})
                    c.push_back({STENCIL_VARIANT_BOX3D, ty, e, lz, STAR_FLAG_XCD});
    if (p->lin.is_dense3 && p->lin.reff == 1)
        for (int ty : {4, 8})
            for (int ny : {1, 2})
                for (int lz : {8, 16, 32})
                    for (int pf : {1, 3})
                        c.push_back({STENCIL_VARIANT_BOX3D, ty, ny, lz,
                                     STAR_FLAG_XCD | (pf << STAR_PF_SHIFT)});
    if (g.ndim == 1) {
        c.push_back({STENCIL_VARIANT_GENERIC, 256, 1, 0, 0});
    } else {
        c.push_back({STENCIL_VARIANT_GENERIC, 64, 4, 0, 0});
        c.push_back({STENCIL_VARIANT_GENERIC, 64, 8, 0, 0});
        c.push_back({STENCIL_VARIANT_GENERIC, 128, 2, 0, 0});
    }
    return c;
}

// Lane-exchange march shape for the dense radius-1 box (waves per workgroup,
// rows per lane, z planes per workgroup, planes in flight): its fastest at
// 512^3 (0.553 / 0.312 ms per launch in FP64 / FP32, against 2.39 / 2.20 ms
// gathering); the LDS march is the default now, this one a search candidate.
constexpr int BOX3D_DEFAULT_TY = 4, BOX3D_DEFAULT_NY = 2, BOX3D_DEFAULT_LZ = 8,
              BOX3D_DEFAULT_PF = 1;


// One-iteration star shape that measured fastest at 512^3: 128 x 8 tiles,
// 64 z planes per workgroup for FP64 and 32 for the narrower types.
TuneChoice default_star1(const stencil_plan_s *p)
{
    return {STENCIL_VARIANT_STAR3D, 4, 2, p->lin.dtype == STENCIL_F64 ? 64 : 32,
            STAR_FLAG_XCD | (2 << STAR_PF_SHIFT) | (2 << STAR_XW_SHIFT)};
}

TuneChoice default_choice(const stencil_plan_s *p)
{
    if (p->lin.op != STENCIL_OP_XCORR) {
        // 3-D box max/min: the lane-exchange march with short z chunks and
        // three planes in flight measured fastest at 512^3 (FP64 and FP32);
        // arrays of 4 GiB or more take the LDS march
        const bool big = uint64_t(padded_elems(p->lin.g)) * dtype_size(p->lin.dtype) >=
                         (uint64_t(1) << 32);
        if (p->lin.is_box && p->lin.op != STENCIL_OP_MEDIAN && !big)
            return {STENCIL_VARIANT_STAR3D, 4, p->lin.reff == 1 ? 4 : 2, 8,
                    STAR_FLAG_XCD | STAR_DPP_BIT | (3 << STAR_PF_SHIFT)};
        if (p->lin.is_box && p->lin.op != STENCIL_OP_MEDIAN)
            return {STENCIL_VARIANT_STAR3D, 4, 1, 32, 0};
        return {STENCIL_VARIANT_GENERIC, p->lin.g.ndim == 1 ? 256 : 64,
                p->lin.g.ndim == 1 ? 1 : 4, 0, 0};
    }
    // periodic stars: two iterations per launch, the lane grids that measured
    // fastest at 512^3 (64 x 24 with pair-layout LDS planes for FP64; 64 x 32
    // with four rows per lane for the narrower types, 64 planes per workgroup
    // from r = 3 on, 32 below)
    if (p->lin.is_star && p->lin.bc == STENCIL_BC_PERIODIC) {
        const bool f64 = p->lin.dtype == STENCIL_F64;
        const int pairs = f64 && p->lin.reff <= 4 ? STAR_PAIRS_BIT : 0;
        const int lz = f64 || p->lin.reff >= 3 ? 64 : 32;
        return {STENCIL_VARIANT_STAR3D, f64 ? 12 : 8, f64 ? 2 : 4, lz,
                STAR_FLAG_XCD | (1 << STAR_XW_SHIFT) | (2 << STAR_T_SHIFT) | pairs};
    }
    if (p->lin.is_star)
        return default_star1(p);
    if (p->lin.is_dense2 && box2d_fits(p))
        // one block of 32 rows per workgroup of 8 waves with 4 outputs per
        // lane: with the outputs stored as whole rows, the fastest at 16384^2
        // at radius 2 and 4 (marching 16 blocks, which the search may still
        // pick, was slower up to radius 2 and 2 % faster at radius 4)
        return {STENCIL_VARIANT_BOX3D, 8, BOX2D_DEFAULT_E, 1, STAR_FLAG_XCD};
    if (p->lin.is_dense3) {
        // dense 3-D boxes run the LDS march: four outputs per lane (eight for
        // FP64 at radius 1 and FP32 at radius 4) and the deepest z chunk, up
        // to 128 planes (64 in FP32 at radius 2 and 3), that still gives 2048
        // waves (two per SIMD): the fastest shapes at 512^3. FP64 at radius
        // 1 takes 8 waves (64 x 64 tiles): 0.468 ms against 0.537 with 4 and
        // 0.577-0.649 on the lane-exchange march.
        const Geo &g = p->lin.g;
        const bool f64 = p->lin.dtype == STENCIL_F64;
        const int R = p->lin.reff;
        const int e = (f64 && R == 1) || (!f64 && R == 4) ? 8 : 4;
        const int ty = f64 && R == 1 ? 8 : 4; // 64 x 64 tiles: 13 % faster at 512^3
        const int64_t cols = (int64_t)((g.nx + 63) / 64) * ((g.ny + ty * e - 1) / (ty * e));
        int lz = f64 || R == 1 || R == 4 ? 128 : 64;
        while (lz > 32 && cols * ((g.nz + lz - 1) / lz) * ty < 2048) // waves
            lz /= 2;
        return {STENCIL_VARIANT_BOX3D, ty, e, lz, STAR_FLAG_XCD};
    }
    if (p->lin.g.ndim == 1)
        return {STENCIL_VARIANT_LINE1D, 4, 0, 0, 0};
    return {STENCIL_VARIANT_GENERIC, 64, 4, 0, 0};
}

// Time every candidate on scratch buffers (best of two timed runs of 3
// launches after one warm-up; launches that fail are dropped, as in the
// paper's heuristic search of Sec. 5.1) and keep the fastest.
int autotune(stencil_plan_s *p)
{
    std::string key = tune_key(p);
    {
        std::vector<int> v;
        if (tune_cache_get(key, v) && v.size() == 5) {
            set_choice(p, {v[0], v[1], v[2], v[3], v[4]});
            return STENCIL_OK;
        }
    }
    const size_t bytes = (size_t)padded_elems(p->lin.g) * dtype_size(p->lin.dtype);
    void *a = nullptr, *b = nullptr;
    if (hipMalloc(&a, bytes) != hipSuccess || hipMalloc(&b, bytes) != hipSuccess) {
        (void)hipGetLastError();
        if (a) (void)hipFree(a);
        return fail(STENCIL_ENOMEM, "autotune: cannot allocate 2 x %zu bytes of scratch", bytes);
    }
    STN_HIP(hipMemset(a, 0, bytes));
    STN_HIP(hipMemset(b, 0, bytes));
    hipEvent_t e0, e1;
    STN_HIP(hipEventCreate(&e0));
    STN_HIP(hipEventCreate(&e1));
    float best = 1e30f;
    TuneChoice best_c = default_choice(p);
    for (const TuneChoice &c : candidates(p)) {
        set_choice(p, c);
        if (apply_any(p, a, b, p->lin.is_star ? 2 : 1, nullptr) != STENCIL_OK) {
            (void)hipGetLastError();
            continue;
        }
        float ms = 1e30f;
        bool ok = true;
        for (int rep = 0; rep < 2 && ok; ++rep) {
            if (hipEventRecord(e0, nullptr) != hipSuccess) { ok = false; break; }
            // 1-D plans are timed on 10 chained iterations so temporal
            // blocking is weighed against per-iteration launches, and
            // 3-D stars on 4, so one- and two-iteration launches do equal work
            const int it = p->lin.g.ndim == 1 ? 10 : p->lin.is_star ? 4 : 3;
            int rc = apply_any(p, a, b, it, nullptr);
            if (hipEventRecord(e1, nullptr) != hipSuccess) { ok = false; break; }
            if (hipEventSynchronize(e1) != hipSuccess || rc != STENCIL_OK) {
                (void)hipGetLastError();
                ok = false;
                break;
            }
            float t = 0;
            (void)hipEventElapsedTime(&t, e0, e1);
            ms = std::min(ms, t);
        }
        if (!ok)
            continue;
        if (ms < best) {
            best = ms;
            best_c = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(a);
    (void)hipFree(b);
    set_choice(p, best_c);
    tune_cache_put(key, {best_c.variant, best_c.p0, best_c.p1, best_c.p2, best_c.p3});
    return STENCIL_OK;
}

} // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

extern "C" {

const char *stencil_last_error(void) { return g_err; }

int stencil_version(void) { return 10000; }

size_t stencil_plan_padded_elems(stencil_plan_t plan)
{
    if (!plan)
        return 0;
    return (size_t)padded_elems(plan->kind == PLAN_LINEAR ? plan->lin.g : plan->rk.g);
}

size_t stencil_padded_elems(int ndim, const int dims[3], int radius)
{
    if (ndim < 1 || ndim > 3 || !dims || radius < 0)
        return 0;
    size_t n = 1;
    for (int a = 0; a < ndim; ++a) {
        if (dims[a] < 1)
            return 0;
        n *= (size_t)dims[a] + 2 * (size_t)radius;
    }
    return n;
}

stencil_status stencil_plan(const stencil_desc *d, stencil_plan_t *out)
{
    if (!d || !out)
        return fail(STENCIL_EINVAL, "NULL descriptor or output");
    *out = nullptr;
    if (d->ndim >= 1 && d->ndim <= 3 && (d->radius < 0 || d->radius > max_radius(d->ndim)))
        return fail(STENCIL_EINVAL, "radius %d not in 0..%d for ndim %d", d->radius,
                    max_radius(d->ndim), d->ndim);
    if (d->dtype < STENCIL_F64 || d->dtype > STENCIL_BF16)
        return fail(STENCIL_EINVAL, "unknown dtype %d", d->dtype);
    if (d->bc != STENCIL_BC_PERIODIC && d->bc != STENCIL_BC_USER_HALO)
        return fail(STENCIL_EINVAL, "unknown boundary mode %d", d->bc);
    if (d->op < STENCIL_OP_XCORR || d->op > STENCIL_OP_MEDIAN)
        return fail(STENCIL_EINVAL, "unknown stencil op %d", d->op);
    if (!d->coeffs)
        return fail(STENCIL_EINVAL, "coeffs is NULL");
    int rc = check_dims(d->ndim, d->dims, d->radius, d->bc);
    if (rc) return rc;
    if (d->variant < STENCIL_VARIANT_AUTO || d->variant > STENCIL_VARIANT_BOX3D)
        return fail(STENCIL_EINVAL, "unknown variant %d", d->variant);
    const int ox = d->x_offset ? d->x_offset : d->radius;
    const int64_t min_pitch = (int64_t)ox + d->dims[0] + d->radius;
    if (d->x_offset < 0 || d->row_pitch < 0)
        return fail(STENCIL_EINVAL, "negative row_pitch or x_offset");
    if (ox < d->radius || ox > (1 << 20))
        return fail(STENCIL_EINVAL, "x_offset %d not in [radius %d, 2^20]", ox, d->radius);
    if (d->row_pitch && d->ndim < 2)
        return fail(STENCIL_EINVAL, "row_pitch needs ndim >= 2");
    if (d->row_pitch && (d->row_pitch < min_pitch || d->row_pitch > (1 << 30)))
        return fail(STENCIL_EINVAL, "row_pitch %d not in [x_offset + dims[0] + radius = %lld, 2^30]",
                    d->row_pitch, (long long)min_pitch);
    {
        int64_t cells = d->row_pitch ? d->row_pitch : min_pitch;
        for (int a = 1; a < d->ndim; ++a) cells *= (int64_t)d->dims[a] + 2 * d->radius;
        if (cells > (int64_t(1) << 40))
            return fail(STENCIL_EINVAL, "padded array too large");
    }
    {
        const size_t K = 2 * (size_t)d->radius + 1;
        size_t nc = K;
        for (int a = 1; a < d->ndim; ++a) nc *= K;
        for (size_t i = 0; i < nc; ++i)
            if (!std::isfinite(d->coeffs[i]))
                return fail(STENCIL_EINVAL, "non-finite coefficient at index %zu", i);
    }

    auto *p = new (std::nothrow) stencil_plan_s();
    if (!p)
        return fail(STENCIL_ENOMEM, "out of host memory");
    p->kind = PLAN_LINEAR;
    if (hipGetDevice(&p->device) != hipSuccess) {
        delete p;
        return fail(STENCIL_EDEVICE, "no HIP device");
    }
    LinearPlan &L = p->lin;
    const int r = d->radius, nd = d->ndim, K = 2 * r + 1;
    L.dtype = d->dtype;
    L.bc = d->bc;
    L.g = make_geo(nd, d->dims, r, d->row_pitch ? d->row_pitch : (int)min_pitch, ox);
    const int Ky = nd > 1 ? K : 1, Kz = nd > 2 ? K : 1;
    L.dense.assign(d->coeffs, d->coeffs + (size_t)K * Ky * Kz);

    // prune zero taps (lexicographic s_z, s_y, s_x); classify the pattern
    std::vector<int> offs;
    std::vector<double> taps;
    int reff = 0;
    bool star = nd == 3;
    for (int sz = -(Kz / 2); sz <= Kz / 2; ++sz)
        for (int sy = -(Ky / 2); sy <= Ky / 2; ++sy)
            for (int sx = -r; sx <= r; ++sx) {
                double c = L.dense[(size_t)(sx + r) + (size_t)K * ((sy + Ky / 2) + (size_t)Ky * (sz + Kz / 2))];
                if (c == 0.0)
                    continue;
                offs.push_back((int)(sx + L.g.sy * sy + L.g.sz * sz));
                taps.push_back(c);
                reff = std::max(reff, std::max(std::abs(sx), std::max(std::abs(sy), std::abs(sz))));
                if ((sx != 0) + (sy != 0) + (sz != 0) > 1)
                    star = false;
            }
    L.reff = reff;
    L.ntaps = (int)taps.size();
    L.op = d->op;
    L.is_star = star && reff >= 1 && reff <= STAR_MAX_R && L.op == STENCIL_OP_XCORR;
    L.is_box = nd == 3 && r >= 1 && r <= 3 && L.ntaps == K * K * K && L.op != STENCIL_OP_XCORR;
    L.is_dense3 = nd == 3 && reff >= 1 && reff <= BOX_LDS_MAX_R &&
                  L.ntaps == (2 * reff + 1) * (2 * reff + 1) * (2 * reff + 1) &&
                  L.op == STENCIL_OP_XCORR;
    L.is_dense2 = nd == 2 && reff >= 1 && reff <= BOX_LDS_MAX_R &&
                  L.ntaps == (2 * reff + 1) * (2 * reff + 1) && L.op == STENCIL_OP_XCORR;
    if (L.is_dense3 && reff == 1) {
        L.box.R = 1;
        for (int sz = -1; sz <= 1; ++sz)
            for (int sy = -1; sy <= 1; ++sy)
                for (int sx = -1; sx <= 1; ++sx)
                    L.box.c[((sz + 1) * 3 + sy + 1) * 3 + sx + 1] =
                        L.dense[(size_t)(sx + r) + (size_t)K * ((sy + r) + (size_t)K * (sz + r))];
    }
    if (L.is_star) {
        std::memset(&L.star, 0, sizeof(L.star));
        for (int sz = -reff; sz <= reff; ++sz)
            for (int sy = -reff; sy <= reff; ++sy)
                for (int sx = -reff; sx <= reff; ++sx) {
                    if ((sx != 0) + (sy != 0) + (sz != 0) > 1)
                        continue;
                    double c = L.dense[(size_t)(sx + r) + (size_t)K * ((sy + r) + (size_t)K * (sz + r))];
                    if (!sx && !sy && !sz) L.star.c0 = c;
                    else if (sx < 0) L.star.xm[-sx - 1] = c;
                    else if (sx > 0) L.star.xp[sx - 1] = c;
                    else if (sy < 0) L.star.ym[-sy - 1] = c;
                    else if (sy > 0) L.star.yp[sy - 1] = c;
                    else if (sz < 0) L.star.zm[-sz - 1] = c;
                    else L.star.zp[sz - 1] = c;
                }
    }

    // device copies of the taps in the arithmetic type
    const bool f64 = L.dtype == STENCIL_F64;
    const size_t csz = f64 ? 8 : 4;
    std::vector<unsigned char> tbuf(std::max<size_t>(1, taps.size()) * csz);
    std::vector<unsigned char> dbuf((size_t)K * csz);
    for (size_t i = 0; i < taps.size(); ++i) {
        if (f64) reinterpret_cast<double *>(tbuf.data())[i] = taps[i];
        else reinterpret_cast<float *>(tbuf.data())[i] = (float)taps[i];
    }
    if (nd == 1)
        for (int i = 0; i < K; ++i) {
            if (f64) reinterpret_cast<double *>(dbuf.data())[i] = L.dense[i];
            else reinterpret_cast<float *>(dbuf.data())[i] = (float)L.dense[i];
        }
    if (offs.empty()) offs.push_back(0);
    if (hipMalloc(&L.d_offs, offs.size() * sizeof(int)) != hipSuccess ||
        hipMalloc(&L.d_taps, tbuf.size()) != hipSuccess ||
        hipMalloc(&L.d_dense, dbuf.size()) != hipSuccess) {
        (void)hipGetLastError();
        stencil_plan_destroy(p);
        return fail(STENCIL_ENOMEM, "cannot allocate plan coefficients on the device");
    }
    if (hipMemcpy(L.d_offs, offs.data(), offs.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(L.d_taps, tbuf.data(), tbuf.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(L.d_dense, dbuf.data(), dbuf.size(), hipMemcpyHostToDevice) != hipSuccess) {
        stencil_plan_destroy(p);
        return fail(STENCIL_EDEVICE, "cannot upload plan coefficients");
    }

    // variant choice
    if (L.op != STENCIL_OP_XCORR) {
        if (L.ntaps < 1 || (L.op == STENCIL_OP_MEDIAN && L.ntaps > STENCIL_MEDIAN_MAX)) {
            stencil_plan_destroy(p);
            return fail(STENCIL_EUNSUPPORTED, "filter window of %d cells (median: 1..%d)", L.ntaps,
                        STENCIL_MEDIAN_MAX);
        }
        if (d->variant == STENCIL_VARIANT_LINE1D ||
            (d->variant == STENCIL_VARIANT_STAR3D && (!L.is_box || L.op == STENCIL_OP_MEDIAN))) {
            stencil_plan_destroy(p);
            return fail(STENCIL_EUNSUPPORTED, "filters run GENERIC, or STAR3D for 3-D box max/min "
                                              "of radius 1..3");
        }
    } else if (d->variant == STENCIL_VARIANT_STAR3D && !L.is_star) {
        stencil_plan_destroy(p);
        return fail(STENCIL_EUNSUPPORTED, "STAR3D needs a 3-D axis-aligned stencil of radius 1..4");
    }
    if (d->variant == STENCIL_VARIANT_BOX3D && !L.is_dense3 && !(L.is_dense2 && box2d_fits(p))) {
        stencil_plan_destroy(p);
        return fail(STENCIL_EUNSUPPORTED, "BOX3D needs a 3-D (2-D, below 4 GiB) "
                                          "cross-correlation with all (2R+1)^3 ((2R+1)^2) taps "
                                          "of a box of radius R = 1..8 nonzero");
    }
    if (d->variant == STENCIL_VARIANT_LINE1D && nd != 1) {
        stencil_plan_destroy(p);
        return fail(STENCIL_EUNSUPPORTED, "LINE1D needs ndim = 1");
    }
    TuneChoice c = default_choice(p);
    if (L.is_star) {
        // the one-iteration shape that runs beside two-iteration launches
        const TuneChoice c1 = default_star1(p);
        L.s1[0] = c1.p0;
        L.s1[1] = c1.p1;
        L.s1[2] = c1.p2;
        L.s1[3] = c1.p3 & 15;
        L.s1[4] = (c1.p3 >> STAR_XW_SHIFT) & 15;
    }
    if (d->variant != STENCIL_VARIANT_AUTO) {
        c.variant = d->variant;
        if (c.variant != default_choice(p).variant) {
            if (c.variant == STENCIL_VARIANT_GENERIC) c = {c.variant, nd == 1 ? 256 : 64, nd == 1 ? 1 : 4, 0, 0};
            else if (c.variant == STENCIL_VARIANT_LINE1D) c = {c.variant, 4, 0, 0, 0};
            else if (c.variant == STENCIL_VARIANT_BOX3D)
                c = {c.variant, BOX3D_DEFAULT_TY, BOX3D_DEFAULT_NY, BOX3D_DEFAULT_LZ,
                     STAR_FLAG_XCD | (BOX3D_DEFAULT_PF << STAR_PF_SHIFT)};
        }
        const int *t = d->tile;
        if (c.variant == STENCIL_VARIANT_STAR3D && (t[0] || t[1] || t[2] || t[3])) {
            if (t[0]) c.p0 = t[0];
            if (t[1]) c.p1 = t[1];
            if (t[2]) c.p2 = t[2];
            c.p3 = t[3] & (0xffff | STAR_PAIRS_BIT | STAR_DPP_BIT); // explicit tiles set the flag word exactly
            const int tb = (c.p3 >> STAR_T_SHIFT) & 15;
            if (tb > 2 || (tb == 2 && d->bc != STENCIL_BC_PERIODIC) ||
                (tb == 2 && (c.p3 & (STAR_FLAG_HWC | STAR_FLAG_NOFUSE)))) {
                stencil_plan_destroy(p);
                return fail(STENCIL_EINVAL, "two iterations per launch need a periodic plan and "
                                            "the LDS variant (and 1 or 2 iterations only)");
            }
            if ((c.p3 & STAR_DPP_BIT) &&
                (tb == 2 || (c.p3 & (STAR_FLAG_HWC | STAR_PAIRS_BIT)) ||
                 (L.op != STENCIL_OP_XCORR && L.reff > 3))) {
                stencil_plan_destroy(p);
                return fail(STENCIL_EINVAL, "the lane-exchange march runs one iteration per "
                                            "launch, without the cached or pair-layout flags");
            }
            const int xwt = ((c.p3 >> STAR_XW_SHIFT) & 15) ? ((c.p3 >> STAR_XW_SHIFT) & 15) : 1;
            const bool pair_ok = c.p1 == 2 && L.reff <= 4 && 64 * xwt * c.p0 <= 768;
            const bool quad_ok = c.p1 == 4 && L.dtype != STENCIL_F64 && xwt == 1 && c.p0 * 64 <= 768;
            if ((c.p3 & STAR_PAIRS_BIT) && (tb != 2 || !(pair_ok || quad_ok))) {
                stencil_plan_destroy(p);
                return fail(STENCIL_EINVAL, "the pair layout needs two iterations per launch, two "
                                            "rows per lane, radius <= 4 and at most 768 lanes "
                                            "(FP32/BF16: or four rows per lane, one wave wide)");
            }
        } else if (c.variant == STENCIL_VARIANT_BOX3D && (t[0] || t[1] || t[2] || t[3])) {
            if (t[0]) c.p0 = t[0];
            if (t[1]) c.p1 = t[1];
            if (t[2]) c.p2 = t[2];
            c.p3 = t[3] & (STAR_FLAG_XCD | (15 << STAR_PF_SHIFT));
            if (c.p2 < 1) {
                stencil_plan_destroy(p);
                return fail(STENCIL_EINVAL, "box3d z chunk must be >= 1");
            }
            const bool ty8 = c.p0 == 8 && (nd == 2 || L.reff == 1); // HBM-bound forms
            if ((L.reff >= 2 || nd == 2 || c.p1 >= 4) &&
                ((c.p0 != 4 && !ty8) || (c.p1 != 4 && c.p1 != 8) ||
                 (nd == 3 && L.reff >= 5 && c.p1 != 4))) {
                stencil_plan_destroy(p);
                return fail(STENCIL_EUNSUPPORTED, "the LDS box march: 4 waves per workgroup (8 "
                                                  "for 2-D boxes and the 27-point box), 4 or 8 "
                                                  "outputs per lane (4 for 3-D radius 5..8)");
            }
        } else if (c.variant == STENCIL_VARIANT_LINE1D) {
            if (t[0]) c.p0 = t[0];
            if (t[1]) c.p1 = t[1];
            c.p2 = t[2] ? 1 : 0;
            if (c.p2 && c.p1 > 1) {
                stencil_plan_destroy(p);
                return fail(STENCIL_EINVAL, "register blocking and fused iterations exclude "
                                            "each other");
            }
            if (c.p1 > 1 && d->bc != STENCIL_BC_PERIODIC) {
                stencil_plan_destroy(p);
                return fail(STENCIL_EINVAL, "temporal blocking needs a periodic plan");
            }
            if (c.p1 < 0 || c.p1 > 64) {
                stencil_plan_destroy(p);
                return fail(STENCIL_EINVAL, "fused iterations must be 1..64");
            }
        } else if (c.variant == STENCIL_VARIANT_GENERIC) {
            if (t[0]) c.p0 = t[0];
            if (t[1]) c.p1 = t[1];
            if (c.p0 < 1 || c.p1 < 1 || c.p0 * c.p1 > 1024 || (c.p0 * c.p1) % 64) {
                stencil_plan_destroy(p);
                return fail(STENCIL_EINVAL, "generic block %dx%d must be a multiple of 64 lanes <= 1024",
                            c.p0, c.p1);
            }
        }
        if (c.variant == STENCIL_VARIANT_STAR3D && c.p2 < 1) {
            stencil_plan_destroy(p);
            return fail(STENCIL_EINVAL, "star z chunk must be >= 1");
        }
        set_choice(p, c);
    } else if (d->flags & STENCIL_FLAG_AUTOTUNE) {
        rc = autotune(p);
        if (rc) {
            stencil_plan_destroy(p);
            return rc;
        }
    } else {
        set_choice(p, c);
    }
    *out = p;
    return STENCIL_OK;
}

stencil_status stencil_plan_destroy(stencil_plan_t p)
{
    if (!p)
        return STENCIL_OK;
    plan_release_device(p);
    delete p;
    return STENCIL_OK;
}

int stencil_plan_variant(stencil_plan_t p)
{
    if (!p || p->kind != PLAN_LINEAR)
        return fail(STENCIL_EINVAL, "not a linear plan");
    return p->lin.variant;
}

stencil_status stencil_plan_tile(stencil_plan_t p, int tile[4])
{
    if (!p || p->kind != PLAN_LINEAR || !tile)
        return fail(STENCIL_EINVAL, "not a linear plan or NULL output");
    const LinearPlan &L = p->lin;
    tile[0] = tile[1] = tile[2] = tile[3] = 0;
    if (L.variant == STENCIL_VARIANT_STAR3D) {
        tile[0] = L.ty;
        tile[1] = L.ny;
        tile[2] = L.lz;
        tile[3] = L.sflags | (L.pf << STAR_PF_SHIFT) | (L.xw << STAR_XW_SHIFT) |
                  (L.tstar == 2 ? 2 << STAR_T_SHIFT : 0) | (L.pairs ? STAR_PAIRS_BIT : 0) |
                  (L.dpp ? STAR_DPP_BIT : 0);
    } else if (L.variant == STENCIL_VARIANT_BOX3D) {
        tile[0] = L.ty;
        tile[1] = L.ny;
        tile[2] = L.lz;
        tile[3] = L.sflags | (box_lds(L) ? 0 : L.pf << STAR_PF_SHIFT);
    } else if (L.variant == STENCIL_VARIANT_LINE1D) {
        tile[0] = L.e1d;
        tile[1] = L.t1d;
        tile[2] = L.rb1d;
    } else {
        tile[0] = L.gbx;
        tile[1] = L.gby;
    }
    return STENCIL_OK;
}

stencil_status stencil_apply(stencil_plan_t p, void *a, void *b, int iters, void *stream)
{
    return stencil_apply_ex(p, a, b, iters, 0u, stream);
}

stencil_status stencil_apply_ex(stencil_plan_t p, void *a, void *b, int iters, unsigned flags,
                                void *stream)
{
    if (flags & ~STENCIL_APPLY_HALO_VALID)
        return fail(STENCIL_EINVAL, "unknown apply flags 0x%x", flags);
    if (!p || p->kind != PLAN_LINEAR)
        return fail(STENCIL_EINVAL, "not a linear plan");
    if (p->sticky)
        return fail(p->sticky, "plan is in an error state from an earlier device failure");
    if (iters < 0)
        return fail(STENCIL_EINVAL, "iters must be >= 0");
    if (p->lin.bc == STENCIL_BC_USER_HALO && iters > 1)
        return fail(STENCIL_EINVAL, "USER_HALO plans apply one iteration at a time");
    const size_t es = dtype_size(p->lin.dtype);
    int rc = check_buffers(a, b, (size_t)padded_elems(p->lin.g) * es, es);
    if (rc) return rc;
    rc = check_device(p->device);
    if (rc) return rc;
    if (iters == 0)
        return STENCIL_OK;
    rc = apply_any(p, a, b, iters, static_cast<hipStream_t>(stream),
                   (flags & STENCIL_APPLY_HALO_VALID) != 0);
    if (rc == STENCIL_EDEVICE)
        p->sticky = rc;
    return rc;
}

stencil_status stencil_halo_periodic(int ndim, const int dims[3], int radius, int dtype,
                                     void *buf, void *stream)
{
    int rc = check_dims(ndim, dims, radius, STENCIL_BC_PERIODIC);
    if (rc) return rc;
    if (radius < 0 || radius > max_radius(ndim))
        return fail(STENCIL_EINVAL, "radius %d not in 0..%d for ndim %d", radius,
                    max_radius(ndim), ndim);
    const size_t es = dtype_size(dtype);
    if (!es)
        return fail(STENCIL_EINVAL, "unknown dtype %d", dtype);
    if (!buf || reinterpret_cast<uintptr_t>(buf) % es)
        return fail(STENCIL_EINVAL, "NULL or misaligned buffer");
    Geo g = make_geo(ndim, dims, radius);
    hipStream_t s = static_cast<hipStream_t>(stream);
    switch (dtype) {
    case STENCIL_F64: return launch_halo<double>(static_cast<double *>(buf), g, s);
    case STENCIL_F32: return launch_halo<float>(static_cast<float *>(buf), g, s);
    default: return launch_halo<bf16>(static_cast<bf16 *>(buf), g, s);
    }
}

stencil_status stencil_plan_halo(stencil_plan_t p, void *buf, void *stream)
{
    if (!p || p->kind != PLAN_LINEAR)
        return fail(STENCIL_EINVAL, "not a linear plan");
    int rc = check_device(p->device);
    if (rc) return rc;
    const size_t es = dtype_size(p->lin.dtype);
    if (!buf || reinterpret_cast<uintptr_t>(buf) % es)
        return fail(STENCIL_EINVAL, "NULL or misaligned buffer");
    hipStream_t s = static_cast<hipStream_t>(stream);
    switch (p->lin.dtype) {
    case STENCIL_F64: return launch_halo<double>(static_cast<double *>(buf), p->lin.g, s);
    case STENCIL_F32: return launch_halo<float>(static_cast<float *>(buf), p->lin.g, s);
    default: return launch_halo<bf16>(static_cast<bf16 *>(buf), p->lin.g, s);
    }
}

stencil_status stencil_copy(const void *src, void *dst, size_t nbytes, void *stream)
{
    if (nbytes % 16)
        return fail(STENCIL_EINVAL, "copy size must be a multiple of 16 bytes");
    int rc = check_buffers(src, dst, nbytes, 16);
    if (rc) return rc;
    if (!nbytes) return STENCIL_OK;
    return launch_copy(src, dst, nbytes, static_cast<hipStream_t>(stream));
}

// Fornberg's recurrence (Math. Comp. 51, 1988) for the weights of the
// derivatives of order 0..m at 0 on the nodes -r..r; we keep order m.
stencil_status stencil_fd_weights(int order, int radius, double *out)
{
    if (!out || radius < 1 || radius > 8 || order < 1 || order > 2 || order > 2 * radius)
        return fail(STENCIL_EINVAL, "need order 1 or 2, radius 1..8, non-NULL out");
    const int n = 2 * radius + 1, m = order;
    std::vector<long double> x(n);
    for (int i = 0; i < n; ++i) x[i] = i - radius;
    // w[j][k]: weight of node j for derivative k
    std::vector<std::vector<long double>> w(n, std::vector<long double>(m + 1, 0.0L));
    long double c1 = 1.0L, c4 = x[0];
    w[0][0] = 1.0L;
    for (int i = 1; i < n; ++i) {
        int mn = std::min(i, m);
        long double c2 = 1.0L, c5 = c4;
        c4 = x[i];
        for (int j = 0; j < i; ++j) {
            long double c3 = x[i] - x[j];
            c2 *= c3;
            if (j == i - 1) {
                for (int k = mn; k >= 1; --k)
                    w[i][k] = c1 * (k * w[i - 1][k - 1] - c5 * w[i - 1][k]) / c2;
                w[i][0] = -c1 * c5 * w[i - 1][0] / c2;
            }
            for (int k = mn; k >= 1; --k)
                w[j][k] = (c4 * w[j][k] - k * w[j][k - 1]) / c3;
            w[j][0] = c4 * w[j][0] / c3;
        }
        c1 = c2;
    }
    // centred nodes: odd orders are exactly antisymmetric, even orders
    // symmetric; average the two halves so rounding cannot break that
    const long double sgn = (m % 2) ? -1.0L : 1.0L;
    for (int i = 0; i < radius; ++i) {
        long double v = 0.5L * (w[n - 1 - i][m] + sgn * w[i][m]);
        out[n - 1 - i] = (double)v;
        out[i] = (double)(sgn * v);
    }
    out[radius] = (m % 2) ? 0.0 : (double)w[radius][m];
    return STENCIL_OK;
}

} // extern "C"
