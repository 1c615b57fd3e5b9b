// filter_kernels.hip -- nonlinear window filters for gfx950: the max filter of
// Sec. 2.3 (and its min twin) and the median filter named in Sec. 1, over the
// window given by the nonzero pattern of a (2r+1)^ndim mask.
//
// Every result is one element of the window, so the kernels compare order-
// preserving integer keys and never round: a value's key orders numbers
// numerically with -0 below +0 (IEEE totalOrder on non-NaN values), and a NaN
// maps to a sentinel that wins every comparison of the op, so a window holding
// a NaN yields NaN. The maximum, minimum and median are therefore unique and
// independent of the order the window is visited in: results are bit-exact.
#include "filter_kernels.hpp"

namespace stn {

namespace {

template <typename C> struct Key;

template <> struct Key<double> {
    using U = uint64_t;
    static constexpr U NAN_MAX = ~U(0), NAN_MIN = U(0);
    static __device__ __forceinline__ U of(double v)
    {
        const U b = __builtin_bit_cast(U, v);
        return (b >> 63) ? ~b : (b | (U(1) << 63));
    }
    static __device__ __forceinline__ double val(U k)
    {
        return __builtin_bit_cast(double, (k >> 63) ? (k & ~(U(1) << 63)) : ~k);
    }
};

template <> struct Key<float> {
    using U = uint32_t;
    static constexpr U NAN_MAX = ~U(0), NAN_MIN = U(0);
    static __device__ __forceinline__ U of(float v)
    {
        const U b = __builtin_bit_cast(U, v);
        return (b >> 31) ? ~b : (b | (U(1) << 31));
    }
    static __device__ __forceinline__ float val(U k)
    {
        return __builtin_bit_cast(float, (k >> 31) ? (k & ~(U(1) << 31)) : ~k);
    }
};

// key of v for a max (NaN on top) or a min (NaN at the bottom) reduction
template <typename C, int OP> __device__ __forceinline__ typename Key<C>::U mkey(C v)
{
    if (v != v)
        return OP == FILTER_OP_MAX ? Key<C>::NAN_MAX : Key<C>::NAN_MIN;
    return Key<C>::of(v);
}

template <typename C, int OP> __device__ __forceinline__ C unkey(typename Key<C>::U k)
{
    if (k == (OP == FILTER_OP_MAX ? Key<C>::NAN_MAX : Key<C>::NAN_MIN))
        return C(__builtin_nan(""));
    return Key<C>::val(k);
}

template <int OP, typename U> __device__ __forceinline__ U pick(U a, U b)
{
    return OP == FILTER_OP_MAX ? (a > b ? a : b) : (a < b ? a : b);
}

} // namespace

// Gather form (the hardware-cached strategy of Sec. 4.1): one lane per output,
// the window's offsets listed in lexicographic (s_z, s_y, s_x) order.
template <typename S, int OP>
__global__ void __launch_bounds__(256)
    k_filter_minmax(const S *__restrict__ in, S *__restrict__ out, Geo g,
                    const int *__restrict__ offs, int ntaps, int fuse)
{
    using C = typename Store<S>::C;
    using U = typename Key<C>::U;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= g.nx || y >= g.ny)
        return;
    const int64_t p = g.at(x, y, z);
    U best = mkey<C, OP>(Store<S>::ld(in + p + offs[0]));
    for (int t = 1; t < ntaps; ++t)
        best = pick<OP>(best, mkey<C, OP>(Store<S>::ld(in + p + offs[t])));
    store_periodic(out, g, x, y, z, unkey<C, OP>(best), fuse != 0);
}

// Median of up to FILTER_MEDIAN_MAX window values: the element whose rank
// (count of smaller keys, ties broken by window position) is (m - 1) / 2.
template <typename S>
__global__ void __launch_bounds__(256)
    k_filter_median(const S *__restrict__ in, S *__restrict__ out, Geo g,
                    const int *__restrict__ offs, int m, int fuse)
{
    using C = typename Store<S>::C;
    using U = typename Key<C>::U;
    constexpr int MM = FILTER_MEDIAN_MAX;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= g.nx || y >= g.ny)
        return;
    const int64_t p = g.at(x, y, z);
    U k[MM];
    bool nan = false;
#pragma unroll
    for (int t = 0; t < MM; ++t) {
        k[t] = 0;
        if (t < m) {
            const C v = Store<S>::ld(in + p + offs[t]);
            nan = nan || (v != v);
            k[t] = Key<C>::of(v);
        }
    }
    const int want = (m - 1) / 2;
    U res = k[0];
    // fully unrolled (compile-time indices keep k in registers); cells past
    // m are excluded by the wave-uniform guards
#pragma unroll
    for (int i = 0; i < MM; ++i) {
        int cnt = 0;
#pragma unroll
        for (int j = 0; j < MM; ++j)
            cnt += (j < m) & ((k[j] < k[i]) | ((k[j] == k[i]) & (j < i)));
        res = (i < m && cnt == want) ? k[i] : res;
    }
    const C v = nan ? C(__builtin_nan("")) : Key<C>::val(res);
    store_periodic(out, g, x, y, z, v, fuse != 0);
}

// Median of an odd number M of window values by forgetful selection: a
// working set of K + 2 values (K = (M - 1) / 2) is kept in registers; each
// round moves the set's minimum and maximum to its two ends with
// compare-exchanges, drops both and takes in the next window value, until
// three remain, whose middle one is the median (the schedule is checked
// against sorting on the CPU, with ties, for every M the kernel is built
// for). About M^2 / 4 compare-exchanges instead of M^2 rank comparisons.
// The compare-exchanges run on the values themselves (one min and one max
// instruction each): distinct numbers order as their keys do, a window with a
// NaN yields NaN anyway, and the one case where the floating-point order is
// coarser than the key order, -0 against +0, is settled afterwards: a zero
// median takes the sign the total order gives it (negative iff more than K
// window values lie below +0, -0 included). So the result is bitwise that of
// the rank count above. All indices are compile-time constants (full
// unrolling), so the values stay in registers.
template <typename C>
__device__ __forceinline__ void cmpx(C &lo, C &hi)
{
    const C a = lo, b = hi;
    lo = fmin(a, b);
    hi = fmax(a, b);
}

template <typename S, int M>
__global__ void __launch_bounds__(256)
    k_filter_median_fs(const S *__restrict__ in, S *__restrict__ out, Geo g,
                       const int *__restrict__ offs, int fuse)
{
    static_assert(M % 2 == 1 && M >= 3, "odd window sizes only");
    using C = typename Store<S>::C;
    constexpr int K = (M - 1) / 2, S0 = K + 2;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= g.nx || y >= g.ny)
        return;
    const int64_t p = g.at(x, y, z);
    C k[M];
    bool nan = false;
#pragma unroll
    for (int t = 0; t < M; ++t) {
        k[t] = Store<S>::ld(in + p + offs[t]);
        nan = nan || (k[t] != k[t]);
    }
    // round r: working set k[r .. S0 - 1]; its minimum goes to k[r] (dropped
    // by advancing r), its maximum to k[S0 - 1], which the next window value
    // then replaces
#pragma unroll
    for (int r = 0; r < M - S0; ++r) {
#pragma unroll
        for (int i = r + 1; i < S0; ++i) cmpx(k[r], k[i]);
#pragma unroll
        for (int i = r + 1; i < S0 - 1; ++i) cmpx(k[i], k[S0 - 1]);
        k[S0 - 1] = k[S0 + r];
    }
    // three values left: k[K - 1], k[K], k[K + 1]; their middle one
    C a = k[K - 1], b = k[K], c = k[K + 1];
    cmpx(a, b);
    C med = fmax(a, fmin(b, c));
    if (!nan && med == C(0)) {
        // the sign of a zero median in the total order (-0 below +0)
        int below = 0;
#pragma unroll
        for (int t = 0; t < M; ++t) {
            const C v = Store<S>::ld(in + p + offs[t]);
            below += (v < C(0)) || (v == C(0) && __builtin_signbit(v));
        }
        med = below > K ? C(-0.0) : C(0.0);
    }
    const C v = nan ? C(__builtin_nan("")) : med;
    store_periodic(out, g, x, y, z, v, fuse != 0);
}

// 3-D box window (all (2R+1)^3 offsets), max or min: a z march. The workgroup
// (64 x TY lanes) stages each plane of its tile plus an R-wide halo (corners
// included) as keys in LDS, reduces the (2R+1)^2 square around each lane's
// column, and keeps the last 2R+1 square reductions in registers; the output
// at plane z is the reduction of the window around z. Planes are double-
// buffered in LDS, so one barrier per plane suffices, and the next plane's
// cells are loaded into registers before the current one is reduced.
template <typename S, int R, int OP, int TY>
__global__ void __launch_bounds__(64 * TY)
    k_filter_box3d(const S *__restrict__ in, S *__restrict__ out, Geo g, int lz, int gx, int gy,
                   int fuse)
{
    using C = typename Store<S>::C;
    using U = typename Key<C>::U;
    constexpr int TX = 64, LW = TX + 2 * R, LH = TY + 2 * R, NT = TX * TY;
    constexpr int CELLS = LW * LH, PER = (CELLS + NT - 1) / NT;
    __shared__ U lds[2][LH][LW];

    const int bxi = blockIdx.x % gx, byi = (blockIdx.x / gx) % gy, bzi = blockIdx.x / (gx * gy);
    const int x0 = bxi * TX, y0 = byi * TY, z0 = bzi * lz;
    const int z1 = min(z0 + lz, g.nz);
    const int tx = threadIdx.x, ty = threadIdx.y, tid = tx + TX * ty;
    const int x = x0 + tx, y = y0 + ty;

    // this lane's cells of a plane tile: padded coordinates clamped into the
    // padded extent (cells past a ragged edge are never used)
    int64_t coff[PER];
    int slot[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int e = tid + q * NT;
        slot[q] = e < CELLS ? e : -1;
        const int ex = e % LW, ey = e / LW;
        const int px = min(x0 - R + ex, g.nx + g.r - 1), py = min(y0 - R + ey, g.ny + g.r - 1);
        coff[q] = e < CELLS ? g.at(px, py, 0) - g.at(0, 0, 0) : 0;
    }
    const int64_t base = g.at(0, 0, 0);
    auto plane_ptr = [&](int zz) { return in + base + (int64_t)zz * g.sz; };

    U win[2 * R + 1];
#pragma unroll
    for (int k = 0; k <= 2 * R; ++k) win[k] = 0;
    U pre[PER];
    const int zs = z0 - R, ze = z1 + R; // planes loaded: zs .. ze-1
#pragma unroll
    for (int q = 0; q < PER; ++q)
        if (slot[q] >= 0) pre[q] = mkey<C, OP>(Store<S>::ld(plane_ptr(zs) + coff[q]));
    for (int zz = zs; zz < ze; ++zz) {
        const int b = (zz - zs) & 1;
        U *lb = &lds[b][0][0];
#pragma unroll
        for (int q = 0; q < PER; ++q)
            if (slot[q] >= 0) lb[slot[q]] = pre[q];
        __syncthreads();
        if (zz + 1 < ze) {
#pragma unroll
            for (int q = 0; q < PER; ++q)
                if (slot[q] >= 0) pre[q] = mkey<C, OP>(Store<S>::ld(plane_ptr(zz + 1) + coff[q]));
        }
        U sq = lds[b][ty][tx];
#pragma unroll
        for (int dy = 0; dy <= 2 * R; ++dy)
#pragma unroll
            for (int dx = 0; dx <= 2 * R; ++dx)
                sq = pick<OP>(sq, lds[b][ty + dy][tx + dx]);
#pragma unroll
        for (int k = 0; k < 2 * R; ++k) win[k] = win[k + 1];
        win[2 * R] = sq;
        const int zo = zz - R;
        if (zo >= z0 && x < g.nx && y < g.ny) {
            U best = win[0];
#pragma unroll
            for (int k = 1; k <= 2 * R; ++k) best = pick<OP>(best, win[k]);
            store_periodic(out, g, x, y, zo, unkey<C, OP>(best), fuse != 0);
        }
    }
}

// The same box window with no LDS and no barriers. A wave is one row of 64
// consecutive columns (lane tx holds column x0 - R + tx; the R lanes at each
// edge only feed their neighbours, so a wave yields 64 - 2R columns) and each
// lane NY consecutive rows. Per plane a lane loads its column over its rows
// and the R rows on either side, reduces every window of 2R + 1 rows in
// registers, then the 2R + 1 columns around it by R one-lane shifts each way
// (DPP moves), and keeps the last 2R + 1 square reductions per row in a
// register ring; the output at plane z reduces the ring around z. The loads
// of the next plane are in flight while the current one is reduced. Max and
// min pick one window element, so the result is bitwise the LDS march's.
template <typename S, int R, int OP, int NY, int TY, int PF>
__global__ void __launch_bounds__(64 * TY)
    k_filter_box3d_dpp(const S *__restrict__ in, S *__restrict__ out, Geo g, int lz, int gx,
                       int gy, int gz, int flags)
{
    using C = typename Store<S>::C;
    using U = typename Key<C>::U;
    constexpr uint32_t es = sizeof(S);
    constexpr int W = 2 * R + 1, NL = NY + 2 * R, OXW = 64 - 2 * R, ROWS = TY * NY;
    // PF planes in flight ahead of the one reduced (NP buffers); the march is
    // unrolled by a common multiple of W and NP, so ring slots (mod W) and
    // prefetch buffers (mod NP) are compile-time indices
    constexpr int NP = PF + 1;
    constexpr int UNR = lcm_int(W, NP);

    int lin = blockIdx.x;
    const int total = gx * gy * gz;
    if (flags & 1) lin = xcd_remap(lin, total);
    const int bxi = lin % gx, byi = (lin / gx) % gy, bzi = lin / (gx * gy);
    const int tx = threadIdx.x;
    const int x = bxi * OXW - R + tx;
    const int y0 = byi * ROWS + threadIdx.y * NY;
    const int z0 = bzi * lz, z1 = min(z0 + lz, g.nz);
    const bool fuse = (flags & 2) != 0;
    const bool xout = tx >= R && tx < 64 - R && x < g.nx;

    // padded coordinates clamped into the array ([-r, n + r) is valid; the
    // window reads the input halo)
    auto cl = [&](int v, int n) { return min(max(v, -R), n + g.r - 1); };
    const int xc = cl(x, g.nx);
    uint32_t off[NL];
#pragma unroll
    for (int i = 0; i < NL; ++i)
        off[i] = uint32_t(xc + g.ox + g.sy * (cl(y0 - R + i, g.ny) + g.ry)) * es;
    const Buf src = make_buf(in, uint64_t(padded_elems(g)) * es);
    auto plane = [&](int zz) { return uint32_t(zz + g.rz) * uint32_t(g.sz) * es; };

    U ring[NY][W];
    C pre[NP][NL];
    const int zs = z0 - R, ze = z1 + R; // planes zs .. ze - 1 are reduced
#pragma unroll
    for (int b = 0; b < NP; ++b)
#pragma unroll
        for (int i = 0; i < NL; ++i)
            pre[b][i] = b < PF ? BufLd<S>::ld(src, off[i], plane(min(zs + b, ze - 1))) : C(0);
#pragma unroll
    for (int j = 0; j < NY; ++j)
#pragma unroll
        for (int k = 0; k < W; ++k) ring[j][k] = 0;

    for (int zb = zs; zb < ze; zb += UNR) {
#pragma unroll
        for (int q = 0; q < UNR; ++q) {
            const int zz = zb + q;
            if (zz >= ze)
                break;
            if (zz + PF < ze) {
                const uint32_t pn = plane(zz + PF);
#pragma unroll
                for (int i = 0; i < NL; ++i) pre[(q + PF) % NP][i] = BufLd<S>::ld(src, off[i], pn);
            }
            U k[NL];
#pragma unroll
            for (int i = 0; i < NL; ++i) k[i] = mkey<C, OP>(pre[q % NP][i]);
#pragma unroll
            for (int j = 0; j < NY; ++j) {
                U v = k[j];
#pragma unroll
                for (int i = 1; i < W; ++i) v = pick<OP>(v, k[j + i]);
                U sq = v, lo = v, hi = v;
#pragma unroll
                for (int m = 1; m <= R; ++m) {
                    lo = lane_up(lo);
                    hi = lane_down(hi);
                    sq = pick<OP>(sq, pick<OP>(lo, hi));
                }
                ring[j][q % W] = sq;
            }
            const int zo = zz - R;
            if (zo >= z0) {
#pragma unroll
                for (int j = 0; j < NY; ++j) {
                    U best = ring[j][0];
#pragma unroll
                    for (int i = 1; i < W; ++i) best = pick<OP>(best, ring[j][i]);
                    const int y = y0 + j;
                    if (xout && y < g.ny)
                        store_periodic(out, g, x, y, zo, unkey<C, OP>(best), fuse);
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

template <typename S>
int launch_filter_gather(const S *in, S *out, const Geo &g, const int *offs, int ntaps, int op,
                         bool fuse, int bx, int by, hipStream_t s)
{
    dim3 block(bx, by), grid((g.nx + bx - 1) / bx, (g.ny + by - 1) / by, g.nz);
    switch (op) {
    case FILTER_OP_MAX:
        hipLaunchKernelGGL((k_filter_minmax<S, FILTER_OP_MAX>), grid, block, 0, s, in, out, g,
                           offs, ntaps, fuse ? 1 : 0);
        break;
    case FILTER_OP_MIN:
        hipLaunchKernelGGL((k_filter_minmax<S, FILTER_OP_MIN>), grid, block, 0, s, in, out, g,
                           offs, ntaps, fuse ? 1 : 0);
        break;
    case FILTER_OP_MEDIAN:
        if (ntaps > FILTER_MEDIAN_MAX)
            return fail(STENCIL_EUNSUPPORTED, "median of %d > %d values", ntaps, FILTER_MEDIAN_MAX);
        // forgetful selection for the common odd windows (3-D and 2-D 3x3
        // boxes, the radius-1 3-D star), rank counting otherwise
        if (ntaps == 27)
            hipLaunchKernelGGL((k_filter_median_fs<S, 27>), grid, block, 0, s, in, out, g, offs,
                               fuse ? 1 : 0);
        else if (ntaps == 9)
            hipLaunchKernelGGL((k_filter_median_fs<S, 9>), grid, block, 0, s, in, out, g, offs,
                               fuse ? 1 : 0);
        else if (ntaps == 7)
            hipLaunchKernelGGL((k_filter_median_fs<S, 7>), grid, block, 0, s, in, out, g, offs,
                               fuse ? 1 : 0);
        else
            hipLaunchKernelGGL(k_filter_median<S>, grid, block, 0, s, in, out, g, offs, ntaps,
                               fuse ? 1 : 0);
        break;
    default: return fail(STENCIL_EINVAL, "unknown filter op %d", op);
    }
    return check_launch("filter_gather");
}

template <typename S, int R, int OP>
int launch_box3d_t(const S *in, S *out, const Geo &g, int ty, int lz, bool fuse, hipStream_t s)
{
    const int gx = (g.nx + 63) / 64, gy = (g.ny + ty - 1) / ty, gz = (g.nz + lz - 1) / lz;
    const int64_t total = (int64_t)gx * gy * gz;
    if (total > 0x7fffffff)
        return fail(STENCIL_EUNSUPPORTED, "box filter: grid too large");
    switch (ty) {
    case 4:
        hipLaunchKernelGGL((k_filter_box3d<S, R, OP, 4>), dim3((unsigned)total), dim3(64, 4), 0, s,
                           in, out, g, lz, gx, gy, fuse ? 1 : 0);
        break;
    case 8:
        hipLaunchKernelGGL((k_filter_box3d<S, R, OP, 8>), dim3((unsigned)total), dim3(64, 8), 0, s,
                           in, out, g, lz, gx, gy, fuse ? 1 : 0);
        break;
    default: return fail(STENCIL_EUNSUPPORTED, "box filter: lanes along y %d not in {4, 8}", ty);
    }
    return check_launch("filter_box3d");
}

template <typename S, int R, int OP, int NY, int TY, int PF>
int launch_box3d_dpp_t(const S *in, S *out, const Geo &g, int lz, bool fuse, int xcd,
                       hipStream_t s)
{
    constexpr int OXW = 64 - 2 * R, ROWS = TY * NY;
    const int gx = (g.nx + OXW - 1) / OXW, gy = (g.ny + ROWS - 1) / ROWS,
              gz = (g.nz + lz - 1) / lz;
    const int64_t total = (int64_t)gx * gy * gz;
    if (total > 0x7fffffff)
        return fail(STENCIL_EUNSUPPORTED, "box filter: grid too large");
    hipLaunchKernelGGL((k_filter_box3d_dpp<S, R, OP, NY, TY, PF>), dim3((unsigned)total),
                       dim3(64, TY), 0, s, in, out, g, lz, gx, gy, gz,
                       (xcd ? 1 : 0) | (fuse ? 2 : 0));
    return check_launch("filter_box3d (lane exchange)");
}

template <typename S, int R, int OP>
int launch_box3d_dpp_r(const S *in, S *out, const Geo &g, int ty, int ny, int pf, int lz,
                       bool fuse, int xcd, hipStream_t s)
{
    if (pf == 0 || pf == 2) // the tile word's default depth: one plane ahead here
        pf = 1;
#define BOX_DPP_CASE(TY_, NY_)                                                               \
    if (ty == TY_ && ny == NY_ && pf == 1)                                                   \
        return launch_box3d_dpp_t<S, R, OP, NY_, TY_, 1>(in, out, g, lz, fuse, xcd, s);        \
    if constexpr (NY_ == 2 || R == 1) /* deeper prefetch spills with more rows */            \
        if (ty == TY_ && ny == NY_ && pf == 3)                                               \
            return launch_box3d_dpp_t<S, R, OP, NY_, TY_, 3>(in, out, g, lz, fuse, xcd, s);
    BOX_DPP_CASE(4, 2) BOX_DPP_CASE(4, 4) BOX_DPP_CASE(8, 2) BOX_DPP_CASE(8, 4)
#undef BOX_DPP_CASE
    return fail(STENCIL_EUNSUPPORTED,
                "box filter (lane exchange): waves %d, rows %d, prefetch %d not in {4, 8} x "
                "{2, 4} x {1, 3} (prefetch 3 with four rows only at radius 1)", ty, ny, pf);
}

template <typename S, int OP>
int launch_box3d_op(const S *in, S *out, const Geo &g, int R, int ty, int ny, int pf, int lz,
                    bool fuse, bool dpp, int xcd, hipStream_t s)
{
    if (dpp) {
        switch (R) {
        case 1: return launch_box3d_dpp_r<S, 1, OP>(in, out, g, ty, ny, pf, lz, fuse, xcd, s);
        case 2: return launch_box3d_dpp_r<S, 2, OP>(in, out, g, ty, ny, pf, lz, fuse, xcd, s);
        case 3: return launch_box3d_dpp_r<S, 3, OP>(in, out, g, ty, ny, pf, lz, fuse, xcd, s);
        }
        return fail(STENCIL_EUNSUPPORTED, "box filter: radius %d not in 1..3", R);
    }
    switch (R) {
    case 1: return launch_box3d_t<S, 1, OP>(in, out, g, ty, lz, fuse, s);
    case 2: return launch_box3d_t<S, 2, OP>(in, out, g, ty, lz, fuse, s);
    case 3: return launch_box3d_t<S, 3, OP>(in, out, g, ty, lz, fuse, s);
    }
    return fail(STENCIL_EUNSUPPORTED, "box filter: radius %d not in 1..3", R);
}

template <typename S>
int launch_filter_box3d(const S *in, S *out, const Geo &g, int R, int op, bool fuse, int ty,
                        int ny, int pf, int lz, bool dpp, int xcd, hipStream_t s)
{
    if (g.ndim != 3 || R > g.r || lz < 1)
        return fail(STENCIL_EINVAL, "box filter: needs a 3-D plan, radius <= padding, lz >= 1");
    if (dpp && uint64_t(padded_elems(g)) * sizeof(S) >= (uint64_t(1) << 32))
        return fail(STENCIL_EUNSUPPORTED,
                    "box filter (lane exchange): arrays of 4 GiB or more are not supported");
    if (op == FILTER_OP_MAX)
        return launch_box3d_op<S, FILTER_OP_MAX>(in, out, g, R, ty, ny, pf, lz, fuse, dpp, xcd, s);
    if (op == FILTER_OP_MIN)
        return launch_box3d_op<S, FILTER_OP_MIN>(in, out, g, R, ty, ny, pf, lz, fuse, dpp, xcd, s);
    return fail(STENCIL_EUNSUPPORTED, "box filter: op %d is not max or min", op);
}

#define INST(S)                                                                              \
    template int launch_filter_gather<S>(const S *, S *, const Geo &, const int *, int, int,   \
                                         bool, int, int, hipStream_t);                        \
    template int launch_filter_box3d<S>(const S *, S *, const Geo &, int, int, bool, int, int, \
                                        int, int, bool, int, hipStream_t);
INST(double)
INST(float)
INST(bf16)
#undef INST

} // namespace stn
