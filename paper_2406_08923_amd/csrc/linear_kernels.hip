// linear_kernels.hip -- gfx950 kernels of the linear path: periodic halo,
// cross-correlation (generic, 3-D star, 1-D line) and the r = 0 copy.
#include "linear_kernels.hpp"

namespace stn {

// ---------------------------------------------------------------------------
// Periodic halo (Eq. 2 with a periodic boundary function)
// ---------------------------------------------------------------------------
//
// One lane per halo cell. The halo is enumerated as three disjoint groups:
// whole z-slabs (2rz planes of Px*Py cells), then y-slabs of the interior
// planes (2ry rows of Px cells each), then x-slabs of the interior rows (2r
// cells each). Every halo cell copies the interior cell obtained by wrapping
// each of its coordinates independently, so cells do not depend on each other
// and one launch fills edges and corners.

__device__ __forceinline__ int wrap_pad(int q, int r, int n)
{
    // padded coordinate q -> padded coordinate of the congruent interior cell
    int i = q - r;
    i %= n;
    if (i < 0) i += n;
    return i + r;
}

template <typename S>
__global__ void __launch_bounds__(256) k_halo_periodic(S *a, Geo g, int64_t n_z, int64_t n_y,
                                                       int64_t total)
{
    const int64_t Px = g.sy, Py = g.sz / g.sy;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        int qx, qy, qz;
        if (t < n_z) { // z slabs
            int64_t plane = Px * Py;
            int k = static_cast<int>(t / plane);
            int64_t rem = t - k * plane;
            qz = k < g.rz ? k : g.nz + k;
            qy = static_cast<int>(rem / Px);
            qx = static_cast<int>(rem - qy * Px);
        } else if (t < n_z + n_y) { // y slabs
            int64_t u = t - n_z;
            int64_t per_plane = 2 * g.ry * Px;
            int zi = static_cast<int>(u / per_plane);
            int64_t rem = u - zi * per_plane;
            int k = static_cast<int>(rem / Px);
            qx = static_cast<int>(rem - k * Px);
            qy = k < g.ry ? k : g.ny + k;
            qz = zi + g.rz;
        } else { // x slabs
            int64_t u = t - n_z - n_y;
            int w = 2 * g.r;
            int64_t row = u / w;
            int k = static_cast<int>(u - row * w);
            qx = k < g.r ? k : g.nx + k;
            qy = static_cast<int>(row % g.ny) + g.ry;
            qz = static_cast<int>(row / g.ny) + g.rz;
        }
        int sx = wrap_pad(qx, g.r, g.nx);
        int sy = g.ry ? wrap_pad(qy, g.ry, g.ny) : qy;
        int sz = g.rz ? wrap_pad(qz, g.rz, g.nz) : qz;
        a[qx + g.sy * qy + g.sz * qz] = a[sx + g.sy * sy + g.sz * sz];
    }
}

template <typename S> int launch_halo(S *a, const Geo &g, hipStream_t s)
{
    if (g.r == 0)
        return STENCIL_OK;
    const int64_t Px = g.sy, Py = g.sz / g.sy;
    int64_t n_z = g.rz ? 2 * g.rz * Px * Py : 0;
    int64_t n_y = g.ry ? (int64_t)g.nz * 2 * g.ry * Px : 0;
    int64_t n_x = (int64_t)g.nz * g.ny * 2 * g.r;
    int64_t total = n_z + n_y + n_x;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_halo_periodic<S>, dim3((unsigned)blocks), dim3(256), 0, s, a, g, n_z,
                       n_y, total);
    return check_launch("halo_periodic");
}

// ---------------------------------------------------------------------------
// Generic cross-correlation: one lane per output, taps through the caches
// (the hardware-cached strategy of Sec. 4.1). Taps are pruned (nonzero only),
// ordered lexicographically in (s_z, s_y, s_x) and read as wave-uniform
// scalar loads.
// ---------------------------------------------------------------------------

template <typename S>
__global__ void __launch_bounds__(256)
    k_xcorr_generic(const S *__restrict__ in, S *__restrict__ out, Geo g,
                    const int *__restrict__ offs, const typename Store<S>::C *__restrict__ cs,
                    int ntaps, int fuse)
{
    using C = typename Store<S>::C;
    int x = blockIdx.x * blockDim.x + threadIdx.x;
    int y = blockIdx.y * blockDim.y + threadIdx.y;
    int z = blockIdx.z;
    if (x >= g.nx || y >= g.ny)
        return;
    const int64_t p = g.at(x, y, z);
    C acc = 0;
    for (int t = 0; t < ntaps; ++t)
        acc = fma(cs[t], Store<S>::ld(in + p + offs[t]), acc);
    store_periodic(out, g, x, y, z, acc, fuse != 0);
}

template <typename S>
int launch_generic(const S *in, S *out, const Geo &g, const int *offs,
                   const typename Store<S>::C *cs, int ntaps, bool fuse, int bx, int by,
                   hipStream_t s)
{
    dim3 block(bx, by);
    dim3 grid((g.nx + bx - 1) / bx, (g.ny + by - 1) / by, g.nz);
    hipLaunchKernelGGL(k_xcorr_generic<S>, grid, block, 0, s, in, out, g, offs, cs, ntaps,
                       fuse ? 1 : 0);
    return check_launch("xcorr_generic");
}

// ---------------------------------------------------------------------------
// 3-D star: x-y plane tile in LDS + z register window (marching along z)
// ---------------------------------------------------------------------------
//
// Workgroup = 64 x TY lanes; lane (tx, ty) owns column x = x0 + tx and the NY
// consecutive rows y0 + ty*NY + j. The workgroup marches along z over a chunk
// of lz output planes. Per lane and row, the 2R+1 values of the column around
// the current plane live in registers (the z taps). The current plane with
// its x and y halo (no corners: a star needs none) is staged in LDS, double
// buffered so one barrier per plane suffices; x taps and the y taps outside
// the lane's own rows come from LDS, y taps inside them from registers.
// The next plane's leading value and halo cells are fetched before the
// current plane is computed, so their latency hides behind the arithmetic.

template <int R, int NY, int TY> struct StarShape {
    static constexpr int TXW = 64;          // lanes along x
    static constexpr int ROWS = TY * NY;    // output rows per tile
    static constexpr int LW = TXW + 2 * R;  // LDS row width
    static constexpr int LH = ROWS + 2 * R; // LDS rows
    static constexpr int NXH = 2 * R * ROWS; // x-halo cells per plane
    static constexpr int NYH = 2 * R * TXW;  // y-halo cells per plane
    static constexpr int NT = TXW * TY;      // lanes per workgroup
    static constexpr int HX_PER = (NXH + NT - 1) / NT;
    static constexpr int HY_PER = (NYH + NT - 1) / NT;
};

// Remap the hardware workgroup order so that consecutive tiles land on the
// same XCD. Dispatch sends workgroup i to XCD i % 8; this bijection gives
// XCD k the contiguous tile range [start_k, start_k + count_k), where the
// first total % 8 XCDs take one tile more than the others.
__device__ __forceinline__ int xcd_remap(int lin, int total)
{
    const int nxcd = 8;
    const int per = total / nxcd, rem = total % nxcd;
    const int xcd = lin % nxcd, slot = lin / nxcd;
    return xcd < rem ? xcd * (per + 1) + slot : rem * (per + 1) + (xcd - rem) * per + slot;
}

template <typename S, int R, int NY, int TY>
__global__ void __launch_bounds__(64 * TY)
    k_star3d(const S *__restrict__ in, S *__restrict__ out, Geo g, StarCoef<typename Store<S>::C, R> cf,
             int lz, int gx, int gy, int gz, int flags)
{
    using C = typename Store<S>::C;
    using SH = StarShape<R, NY, TY>;
    __shared__ C lds[2][SH::LH][SH::LW];

    int lin = blockIdx.x;
    const int total = gx * gy * gz;
    if (flags & STAR_FLAG_XCD) lin = xcd_remap(lin, total);
    const int bxi = lin % gx;
    const int byi = (lin / gx) % gy;
    const int bzi = lin / (gx * gy);

    const int tx = threadIdx.x, ty = threadIdx.y;
    const int tid = tx + 64 * ty;
    const int x0 = bxi * 64, y0 = byi * SH::ROWS;
    const int z0 = bzi * lz;
    const int z1 = min(z0 + lz, g.nz);
    const bool fuse = (flags & STAR_FLAG_NOFUSE) == 0;

    // clamp reads into the padded array: any coordinate in [-R, n+R) is valid
    auto cl = [](int v, int n) { return min(max(v, -R), n + R - 1); };
    const int x = x0 + tx;
    const int xl = cl(x, g.nx);
    int yl[NY];
#pragma unroll
    for (int j = 0; j < NY; ++j) yl[j] = cl(y0 + ty * NY + j, g.ny);

    // halo cell assignments (fixed per lane)
    int64_t hx_off[SH::HX_PER], hy_off[SH::HY_PER];
    int hx_slot[SH::HX_PER], hy_slot[SH::HY_PER];
#pragma unroll
    for (int k = 0; k < SH::HX_PER; ++k) {
        int c = tid + k * SH::NT;
        if (c < SH::NXH) {
            int row = c / (2 * R), e = c % (2 * R);
            int lc = e < R ? e : SH::TXW + e; // LDS column
            int gxx = cl(x0 - R + lc, g.nx);
            int gyy = cl(y0 + row, g.ny);
            hx_off[k] = g.at(gxx, gyy, 0);
            hx_slot[k] = (row + R) * SH::LW + lc;
        } else {
            hx_off[k] = g.at(0, 0, 0);
            hx_slot[k] = -1;
        }
    }
#pragma unroll
    for (int k = 0; k < SH::HY_PER; ++k) {
        int c = tid + k * SH::NT;
        if (c < SH::NYH) {
            int e = c / SH::TXW, col = c % SH::TXW;
            int lr = e < R ? e : SH::ROWS + e; // LDS row
            int gxx = cl(x0 + col, g.nx);
            int gyy = cl(y0 - R + lr, g.ny);
            hy_off[k] = g.at(gxx, gyy, 0);
            hy_slot[k] = lr * SH::LW + col + R;
        } else {
            hy_off[k] = g.at(0, 0, 0);
            hy_slot[k] = -1;
        }
    }

    // z window: win[j][k] holds plane z - R + k of row j
    C win[NY][2 * R + 1];
    int64_t col_off[NY];
#pragma unroll
    for (int j = 0; j < NY; ++j) col_off[j] = g.at(xl, yl[j], 0);
#pragma unroll
    for (int k = 0; k < 2 * R; ++k)
#pragma unroll
        for (int j = 0; j < NY; ++j)
            win[j][k + 1] = Store<S>::ld(in + col_off[j] + g.sz * (z0 - R + k));

    C hx_v[SH::HX_PER], hy_v[SH::HY_PER], nxt[NY];
#pragma unroll
    for (int k = 0; k < SH::HX_PER; ++k) hx_v[k] = Store<S>::ld(in + hx_off[k] + g.sz * z0);
#pragma unroll
    for (int k = 0; k < SH::HY_PER; ++k) hy_v[k] = Store<S>::ld(in + hy_off[k] + g.sz * z0);
#pragma unroll
    for (int j = 0; j < NY; ++j) nxt[j] = Store<S>::ld(in + col_off[j] + g.sz * (z0 + R));

    for (int z = z0; z < z1; ++z) {
        const int b = (z - z0) & 1;
#pragma unroll
        for (int j = 0; j < NY; ++j) {
#pragma unroll
            for (int k = 0; k < 2 * R; ++k) win[j][k] = win[j][k + 1];
            win[j][2 * R] = nxt[j];
            lds[b][ty * NY + j + R][tx + R] = win[j][R];
        }
        C *lb = &lds[b][0][0];
#pragma unroll
        for (int k = 0; k < SH::HX_PER; ++k)
            if (hx_slot[k] >= 0) lb[hx_slot[k]] = hx_v[k];
#pragma unroll
        for (int k = 0; k < SH::HY_PER; ++k)
            if (hy_slot[k] >= 0) lb[hy_slot[k]] = hy_v[k];
        __syncthreads();

        if (z + 1 < z1) { // prefetch the next plane
            const int64_t zn = g.sz * (z + 1);
#pragma unroll
            for (int k = 0; k < SH::HX_PER; ++k) hx_v[k] = Store<S>::ld(in + hx_off[k] + zn);
#pragma unroll
            for (int k = 0; k < SH::HY_PER; ++k) hy_v[k] = Store<S>::ld(in + hy_off[k] + zn);
#pragma unroll
            for (int j = 0; j < NY; ++j)
                nxt[j] = Store<S>::ld(in + col_off[j] + g.sz * (z + 1 + R));
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

template <typename S, int R, int NY, int TY>
int launch_star3d_t(const S *in, S *out, const Geo &g, const StarCoef<typename Store<S>::C, R> &cf,
                    int lz, int flags, hipStream_t s)
{
    using SH = StarShape<R, NY, TY>;
    int gx = (g.nx + 63) / 64, gy = (g.ny + SH::ROWS - 1) / SH::ROWS, gz = (g.nz + lz - 1) / lz;
    int64_t total = (int64_t)gx * gy * gz;
    if (total > 0x7fffffff)
        return fail(STENCIL_EUNSUPPORTED, "star3d: grid too large");
    hipLaunchKernelGGL((k_star3d<S, R, NY, TY>), dim3((unsigned)total), dim3(64, TY), 0, s, in,
                       out, g, cf, lz, gx, gy, gz, flags);
    return check_launch("xcorr_star3d");
}

// Supported (TY, NY) shapes of the star kernel.
#define STAR_SHAPES(X) X(4, 1) X(4, 2) X(4, 4) X(8, 2) X(2, 4) X(8, 1) X(2, 8)

template <typename S, int R>
int launch_star3d_r(const S *in, S *out, const Geo &g, const StarCoef<typename Store<S>::C, R> &cf,
                    int ty, int ny, int lz, int flags, hipStream_t s)
{
#define STAR_CASE(TY_, NY_)                                                              \
    if (ty == TY_ && ny == NY_)                                                          \
        return launch_star3d_t<S, R, NY_, TY_>(in, out, g, cf, lz, flags, s);
    STAR_SHAPES(STAR_CASE)
#undef STAR_CASE
    return fail(STENCIL_EUNSUPPORTED, "star3d: unsupported tile (ty=%d, ny=%d)", ty, ny);
}

template <typename S>
int launch_star3d(const S *in, S *out, const Geo &g, const StarCoefAny &cfa, int R, int ty,
                  int ny, int lz, int flags, hipStream_t s)
{
    using C = typename Store<S>::C;
    if (R > g.r || g.ndim != 3)
        return fail(STENCIL_EINVAL, "star3d: tap radius %d exceeds padding %d", R, g.r);
    switch (R) {
    case 1: return launch_star3d_r<S, 1>(in, out, g, cfa.get<C, 1>(), ty, ny, lz, flags, s);
    case 2: return launch_star3d_r<S, 2>(in, out, g, cfa.get<C, 2>(), ty, ny, lz, flags, s);
    case 3: return launch_star3d_r<S, 3>(in, out, g, cfa.get<C, 3>(), ty, ny, lz, flags, s);
    case 4: return launch_star3d_r<S, 4>(in, out, g, cfa.get<C, 4>(), ty, ny, lz, flags, s);
    }
    return fail(STENCIL_EUNSUPPORTED, "star3d: radius %d not in 1..4", R);
}

// ---------------------------------------------------------------------------
// 1-D line: block working set staged in LDS (the software-cached strategy of
// Sec. 4.1), E outputs per lane strided by the block width so that LDS reads
// of one tap are consecutive across lanes (no bank conflicts).
// ---------------------------------------------------------------------------

template <typename S, int E>
__global__ void __launch_bounds__(256)
    k_line1d(const S *__restrict__ in, S *__restrict__ out, Geo g,
             const typename Store<S>::C *__restrict__ cs, int fuse)
{
    using C = typename Store<S>::C;
    constexpr int NT = 256, BX = NT * E;
    extern __shared__ unsigned char smem_raw[];
    C *buf = reinterpret_cast<C *>(smem_raw);
    const int r = g.r;
    const int x0 = blockIdx.x * BX;
    const int W = BX + 2 * r;
    // padded index of interior x0 - r is x0
    for (int i = threadIdx.x; i < W; i += NT) {
        int q = min(x0 + i, g.nx + 2 * r - 1);
        buf[i] = Store<S>::ld(in + q);
    }
    __syncthreads();
    const int K = 2 * r + 1;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        int l = threadIdx.x + e * NT;
        int x = x0 + l;
        C acc = 0;
        for (int t = 0; t < K; ++t)
            acc = fma(cs[t], buf[l + t], acc);
        if (x < g.nx)
            store_periodic(out, g, x, 0, 0, acc, fuse != 0);
    }
}

template <typename S>
int launch_line1d(const S *in, S *out, const Geo &g, const typename Store<S>::C *cs, bool fuse,
                  int e, hipStream_t s)
{
    using C = typename Store<S>::C;
    int bx = 256 * e;
    size_t shm = (size_t)(bx + 2 * g.r) * sizeof(C);
    dim3 grid((g.nx + bx - 1) / bx);
    switch (e) {
    case 1: hipLaunchKernelGGL((k_line1d<S, 1>), grid, dim3(256), shm, s, in, out, g, cs, fuse ? 1 : 0); break;
    case 2: hipLaunchKernelGGL((k_line1d<S, 2>), grid, dim3(256), shm, s, in, out, g, cs, fuse ? 1 : 0); break;
    case 4: hipLaunchKernelGGL((k_line1d<S, 4>), grid, dim3(256), shm, s, in, out, g, cs, fuse ? 1 : 0); break;
    case 8: hipLaunchKernelGGL((k_line1d<S, 8>), grid, dim3(256), shm, s, in, out, g, cs, fuse ? 1 : 0); break;
    default: return fail(STENCIL_EUNSUPPORTED, "line1d: outputs per lane %d not in {1,2,4,8}", e);
    }
    return check_launch("xcorr_line1d");
}

// ---------------------------------------------------------------------------
// r = 0 streaming copy (effective-bandwidth measurement, Sec. 5.2)
// ---------------------------------------------------------------------------

// Four 16-byte loads in flight per lane before the stores, non-temporal so the
// stream does not evict useful cache lines.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) k_copy16(const u32x4 *__restrict__ src, u32x4 *__restrict__ dst,
                                                int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n; i += 4 * stride) {
        u32x4 v0 = __builtin_nontemporal_load(src + i);
        u32x4 v1 = __builtin_nontemporal_load(src + i + stride);
        u32x4 v2 = __builtin_nontemporal_load(src + i + 2 * stride);
        u32x4 v3 = __builtin_nontemporal_load(src + i + 3 * stride);
        __builtin_nontemporal_store(v0, dst + i);
        __builtin_nontemporal_store(v1, dst + i + stride);
        __builtin_nontemporal_store(v2, dst + i + 2 * stride);
        __builtin_nontemporal_store(v3, dst + i + 3 * stride);
    }
    for (; i < n; i += stride)
        __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

int launch_copy(const void *src, void *dst, size_t nbytes, hipStream_t s)
{
    int64_t n = (int64_t)(nbytes / 16);
    int64_t blocks = (n + 4 * 256 - 1) / (4 * 256);
    if (blocks > 256 * 32) blocks = 256 * 32;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_copy16, dim3((unsigned)blocks), dim3(256), 0, s,
                       static_cast<const u32x4 *>(src), static_cast<u32x4 *>(dst), n);
    return check_launch("copy");
}

// explicit instantiations used by the plan code
#define INST(S)                                                                              \
    template int launch_halo<S>(S *, const Geo &, hipStream_t);                              \
    template int launch_generic<S>(const S *, S *, const Geo &, const int *,                 \
                                   const typename Store<S>::C *, int, bool, int, int,        \
                                   hipStream_t);                                             \
    template int launch_star3d<S>(const S *, S *, const Geo &, const StarCoefAny &, int, int, \
                                  int, int, int, hipStream_t);                               \
    template int launch_line1d<S>(const S *, S *, const Geo &, const typename Store<S>::C *, \
                                  bool, int, hipStream_t);
INST(double)
INST(float)
INST(bf16)
#undef INST

} // namespace stn
