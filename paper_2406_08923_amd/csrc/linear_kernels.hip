// linear_kernels.hip -- gfx950 kernels of the linear path: periodic halo,
// cross-correlation (generic, 1-D line) and the r = 0 copy. The 3-D star
// kernel lives in star3d.hpp.
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
    // logical padded extents (the cells that hold data; a longer row pitch
    // only adds unused columns)
    const int64_t Px = g.nx + 2 * g.r, Py = g.ny + 2 * g.ry;
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
        a[g.at(qx - g.r, qy - g.ry, qz - g.rz)] = a[g.at(sx - g.r, sy - g.ry, sz - g.rz)];
    }
}

template <typename S> int launch_halo(S *a, const Geo &g, hipStream_t s)
{
    if (g.r == 0)
        return STENCIL_OK;
    const int64_t Px = g.nx + 2 * g.r, Py = g.ny + 2 * g.ry;
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
    // buf[i] holds interior x0 - r + i (clamped to the padded row)
    for (int i = threadIdx.x; i < W; i += NT) {
        int xi = min(x0 - r + i, g.nx + r - 1);
        buf[i] = Store<S>::ld(in + g.at(xi, 0, 0));
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
// 1-D line, register-blocked for large radii: lane l owns the E adjacent
// outputs x0 + l*E + e and walks the inputs once, each value feeding all E
// accumulators (with the matching tap from a sliding window of coefficients),
// so LDS is read once per input instead of once per tap. The LDS row is
// padded by one cell every E cells, so the lanes' stride-E reads hit distinct
// banks. Every output is the same fma chain over taps 0..K-1 as in k_line1d,
// so results are bitwise equal. Needs K = 2r + 1 >= E - 1.
// ---------------------------------------------------------------------------

template <typename S, int E>
__global__ void __launch_bounds__(256)
    k_line1d_rb(const S *__restrict__ in, S *__restrict__ out, Geo g,
                const typename Store<S>::C *__restrict__ cs, int fuse)
{
    using C = typename Store<S>::C;
    constexpr int NT = 256, BX = NT * E;
    extern __shared__ unsigned char smem_raw[];
    C *buf = reinterpret_cast<C *>(smem_raw);
    const int r = g.r, K = 2 * r + 1;
    const int x0 = blockIdx.x * BX;
    const int W = BX + 2 * r;
    for (int i = threadIdx.x; i < W; i += NT) {
        const int xi = min(x0 - r + i, g.nx + r - 1);
        buf[i + i / E] = Store<S>::ld(in + g.at(xi, 0, 0));
    }
    __syncthreads();
    const int base = threadIdx.x * E;
    auto at = [&](int j) { const int i = base + j; return buf[i + i / E]; };
    C acc[E], cw[E];
#pragma unroll
    for (int e = 0; e < E; ++e) acc[e] = cw[e] = 0;
    // head: inputs j = 0..E-2 feed outputs e <= j (taps j - e)
#pragma unroll
    for (int j = 0; j < E - 1; ++j) {
#pragma unroll
        for (int e = E - 1; e > 0; --e) cw[e] = cw[e - 1];
        cw[0] = cs[j];
        const C v = at(j);
#pragma unroll
        for (int e = 0; e <= j; ++e) acc[e] = fma(cw[e], v, acc[e]);
    }
    // body: inputs j = E-1..K-1 feed every output
    for (int j = E - 1; j < K; ++j) {
#pragma unroll
        for (int e = E - 1; e > 0; --e) cw[e] = cw[e - 1];
        cw[0] = cs[j];
        const C v = at(j);
#pragma unroll
        for (int e = 0; e < E; ++e) acc[e] = fma(cw[e], v, acc[e]);
    }
    // tail: inputs j = K..K+E-2 feed outputs e >= j - K + 1
#pragma unroll
    for (int d = 1; d < E; ++d) {
#pragma unroll
        for (int e = E - 1; e > 0; --e) cw[e] = cw[e - 1];
        const C v = at(K - 1 + d);
#pragma unroll
        for (int e = d; e < E; ++e) acc[e] = fma(cw[e], v, acc[e]);
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int x = x0 + base + e;
        if (x < g.nx)
            store_periodic(out, g, x, 0, 0, acc[e], fuse != 0);
    }
}

template <typename S>
int launch_line1d_rb(const S *in, S *out, const Geo &g, const typename Store<S>::C *cs,
                     bool fuse, int e, hipStream_t s)
{
    using C = typename Store<S>::C;
    if (2 * g.r + 1 < e - 1)
        return fail(STENCIL_EUNSUPPORTED, "line1d: register blocking of %d needs radius >= %d", e,
                    (e - 2) / 2);
    const int bx = 256 * e;
    const size_t w = (size_t)bx + 2 * g.r;
    const size_t shm = (w + w / e + 1) * sizeof(C);
    if (shm > 160 * 1024)
        return fail(STENCIL_EUNSUPPORTED, "line1d: radius %d too large for LDS", g.r);
    dim3 grid((g.nx + bx - 1) / bx);
    switch (e) {
    case 4: hipLaunchKernelGGL((k_line1d_rb<S, 4>), grid, dim3(256), shm, s, in, out, g, cs, fuse ? 1 : 0); break;
    case 8: hipLaunchKernelGGL((k_line1d_rb<S, 8>), grid, dim3(256), shm, s, in, out, g, cs, fuse ? 1 : 0); break;
    case 16: hipLaunchKernelGGL((k_line1d_rb<S, 16>), grid, dim3(256), shm, s, in, out, g, cs, fuse ? 1 : 0); break;
    default: return fail(STENCIL_EUNSUPPORTED, "line1d: register blocking %d not in {4,8,16}", e);
    }
    return check_launch("xcorr_line1d_rb");
}

// ---------------------------------------------------------------------------
// 1-D line, temporally blocked: T chained iterations in one launch. A block
// owning outputs [x0, x0 + BX) loads [x0 - rT, x0 + BX + rT) from the interior
// with periodic wrap (the input halo is not read), iterates T times in LDS
// (iteration i is valid on a region shrunk by r(i+1) on each side) and writes
// its outputs and their periodic images. Each point of each iteration uses
// the same taps in the same order as a single-iteration launch.
// ---------------------------------------------------------------------------

template <typename S, int E>
__global__ void __launch_bounds__(256)
    k_line1d_t(const S *__restrict__ in, S *__restrict__ out, Geo g,
               const typename Store<S>::C *__restrict__ cs, int T, int fuse)
{
    using C = typename Store<S>::C;
    constexpr int NT = 256, BX = NT * E;
    extern __shared__ unsigned char smem_raw[];
    const int r = g.r, n = g.nx;
    const int W = BX + 2 * r * T;
    C *cur = reinterpret_cast<C *>(smem_raw);
    C *nxt = cur + W;
    const int x0 = blockIdx.x * BX;
    for (int i = threadIdx.x; i < W; i += NT) {
        int xi = (x0 - r * T + i) % n;
        if (xi < 0) xi += n;
        cur[i] = Store<S>::ld(in + g.at(xi, 0, 0));
    }
    __syncthreads();
    const int K = 2 * r + 1;
    for (int it = 0; it < T; ++it) {
        const int lo = r * (it + 1), hi = W - r * (it + 1);
        for (int l = lo + threadIdx.x; l < hi; l += NT) {
            C acc = 0;
            for (int t = 0; t < K; ++t)
                acc = fma(cs[t], cur[l - r + t], acc);
            nxt[l] = acc;
        }
        __syncthreads();
        C *tmp = cur;
        cur = nxt;
        nxt = tmp;
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int k = threadIdx.x + e * NT;
        const int x = x0 + k;
        if (x < n)
            store_periodic(out, g, x, 0, 0, cur[r * T + k], fuse != 0);
    }
}

template <typename S>
int launch_line1d_t(const S *in, S *out, const Geo &g, const typename Store<S>::C *cs, bool fuse,
                    int e, int T, hipStream_t s)
{
    using C = typename Store<S>::C;
    const int bx = 256 * e;
    const size_t shm = 2 * (size_t)(bx + 2 * g.r * T) * sizeof(C);
    if (shm > 160 * 1024)
        return fail(STENCIL_EUNSUPPORTED, "line1d: %d fused iterations need too much LDS", T);
    dim3 grid((g.nx + bx - 1) / bx);
    switch (e) {
    case 1: hipLaunchKernelGGL((k_line1d_t<S, 1>), grid, dim3(256), shm, s, in, out, g, cs, T, fuse ? 1 : 0); break;
    case 2: hipLaunchKernelGGL((k_line1d_t<S, 2>), grid, dim3(256), shm, s, in, out, g, cs, T, fuse ? 1 : 0); break;
    case 4: hipLaunchKernelGGL((k_line1d_t<S, 4>), grid, dim3(256), shm, s, in, out, g, cs, T, fuse ? 1 : 0); break;
    case 8: hipLaunchKernelGGL((k_line1d_t<S, 8>), grid, dim3(256), shm, s, in, out, g, cs, T, fuse ? 1 : 0); break;
    default: return fail(STENCIL_EUNSUPPORTED, "line1d: outputs per lane %d not in {1,2,4,8}", e);
    }
    return check_launch("xcorr_line1d_t");
}

// ---------------------------------------------------------------------------
// r = 0 streaming copy (effective-bandwidth measurement, Sec. 5.2)
// ---------------------------------------------------------------------------

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) k_copy16(const u32x4 *__restrict__ src, u32x4 *__restrict__ dst,
                                                int64_t n)
{
    // one 16-byte vector per lane over a grid covering the whole array (the
    // shape that measured fastest on gfx950); the loop only runs again when
    // the array exceeds the grid limit
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride)
        dst[i] = src[i];
}

int launch_copy(const void *src, void *dst, size_t nbytes, hipStream_t s)
{
    int64_t n = (int64_t)(nbytes / 16);
    int64_t blocks = (n + 255) / 256;
    if (blocks > (int64_t(1) << 30)) blocks = int64_t(1) << 30;
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
    template int launch_line1d<S>(const S *, S *, const Geo &, const typename Store<S>::C *, \
                                  bool, int, hipStream_t);                                   \
    template int launch_line1d_t<S>(const S *, S *, const Geo &,                             \
                                    const typename Store<S>::C *, bool, int, int, hipStream_t); \
    template int launch_line1d_rb<S>(const S *, S *, const Geo &,                            \
                                     const typename Store<S>::C *, bool, int, hipStream_t);
INST(double)
INST(float)
INST(bf16)
#undef INST

} // namespace stn
