// common.hpp -- internals shared by the translation units of libstencil.so.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstddef>
#include <cstdint>
#include <type_traits>

#include "../../include/stencil.h"

namespace stn {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------

// Record a printf-style message as this thread's last error; returns code.
int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));

#define STN_HIP(expr)                                                                   \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            return ::stn::fail(STENCIL_EDEVICE, "%s failed: %s", #expr,                 \
                               hipGetErrorString(e_));                                  \
    } while (0)

// Status of the launches just enqueued (hipGetLastError).
int check_launch(const char *what);

// ---------------------------------------------------------------------------
// storage types
// ---------------------------------------------------------------------------

struct bf16 {
    uint16_t bits;
};

// Storage type S with its arithmetic type C, a widening load and a rounding
// store. BF16 is widened exactly (the 16 stored bits are the high half of the
// FP32 pattern) and narrowed with round-to-nearest-even.
template <typename S> struct Store;

template <> struct Store<double> {
    using C = double;
    static __device__ __forceinline__ double ld(const double *p) { return *p; }
    static __device__ __forceinline__ void st(double *p, double v) { *p = v; }
};

template <> struct Store<float> {
    using C = float;
    static __device__ __forceinline__ float ld(const float *p) { return *p; }
    static __device__ __forceinline__ void st(float *p, float v) { *p = v; }
};

__device__ __forceinline__ float bf16_to_f32(uint16_t b)
{
    return __uint_as_float(static_cast<uint32_t>(b) << 16);
}

__device__ __forceinline__ uint16_t f32_to_bf16(float v)
{
    uint32_t u = __float_as_uint(v);
    if ((u & 0x7fffffffu) > 0x7f800000u) // NaN: keep sign, force a quiet NaN
        return static_cast<uint16_t>(((u >> 16) & 0x8000u) | 0x7fc0u);
    // round to nearest, ties to even: add 0x7fff plus the lsb of the kept half
    u += 0x7fffu + ((u >> 16) & 1u);
    return static_cast<uint16_t>(u >> 16);
}

template <> struct Store<bf16> {
    using C = float;
    static __device__ __forceinline__ float ld(const bf16 *p) { return bf16_to_f32(p->bits); }
    static __device__ __forceinline__ void st(bf16 *p, float v) { p->bits = f32_to_bf16(v); }
};

// ---------------------------------------------------------------------------
// buffer loads
// ---------------------------------------------------------------------------
//
// A raw buffer load takes a per-lane 32-bit byte offset (VGPR) plus a
// wave-uniform byte offset (SGPR): a stencil tap whose offset is the same for
// every lane then costs one load instruction and no address arithmetic.
// Offsets are unsigned, so callers index from the lowest address a lane can
// touch. Loads past num_records bytes return zero (no fault). Usable for
// arrays below 4 GiB.

constexpr int BUF_DWORD3 = 0x00020000; // raw 32-bit data format, gfx9 family

struct Buf {
    __amdgpu_buffer_rsrc_t r;
};

__device__ __forceinline__ Buf make_buf(const void *base, uint64_t bytes)
{
    const uint32_t n = bytes > 0xffffffffull ? 0xffffffffu : static_cast<uint32_t>(bytes);
    return Buf{__builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0,
                                                 static_cast<int>(n), BUF_DWORD3)};
}

// Buffer loads straight into LDS: lane l's SZ bytes (16 or 4) from the
// buffer at byte offset voff land at lds + SZ * l, where lds is the same for
// the whole wave. The size is a literal in each helper: the builtin accepts
// no other form, and the host pass silently drops a kernel that passes one.
__device__ __forceinline__ void buf_to_lds16(const Buf &b, void *lds, uint32_t voff)
{
    __builtin_amdgcn_raw_ptr_buffer_load_lds(b.r, (__attribute__((address_space(3))) void *)lds, 16,
                                             voff, 0, 0, 0);
}
__device__ __forceinline__ void buf_to_lds4(const Buf &b, void *lds, uint32_t voff)
{
    __builtin_amdgcn_raw_ptr_buffer_load_lds(b.r, (__attribute__((address_space(3))) void *)lds, 4,
                                             voff, 0, 0, 0);
}

// Buffer resource of one padded plane zp (0 .. nz + 2 rz - 1) of an array:
// lane offsets within a plane stay far below 4 GiB, so kernels that address
// the input plane by plane work for arrays of any size.
template <typename S>
__device__ __forceinline__ Buf plane_buf(const S *base, int64_t sz, int zp)
{
    const uint64_t pb = uint64_t(sz) * sizeof(S);
    return make_buf(reinterpret_cast<const char *>(base) + uint64_t(zp) * pb, pb);
}

// The input of a z march, addressed plane by plane. BIG = false: one buffer
// resource for the whole array, the plane's byte offset as the scalar operand
// (arrays below 4 GiB); BIG = true: a resource per plane (plane_buf), for
// arrays of any size at a few more scalar instructions per plane.
struct PlaneRef {
    Buf b;
    uint32_t soff;
};

template <typename S, bool BIG> struct PlaneSrc {
    const S *base;
    int64_t sz;
    Buf whole;
    __device__ __forceinline__ PlaneSrc(const S *in, int64_t sz_, uint64_t elems)
        : base(in), sz(sz_), whole(make_buf(in, elems * sizeof(S)))
    {
    }
    __device__ __forceinline__ PlaneRef plane(int zp) const
    {
        if constexpr (BIG)
            return {plane_buf(base, sz, zp), 0u};
        else
            return {whole, uint32_t(zp) * uint32_t(sz) * uint32_t(sizeof(S))};
    }
};

template <typename S> struct BufLd;

template <> struct BufLd<double> {
    static __device__ __forceinline__ double ld(const Buf &b, uint32_t voff, uint32_t soff)
    {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(b.r, voff, soff, 0));
    }
};

template <> struct BufLd<float> {
    static __device__ __forceinline__ float ld(const Buf &b, uint32_t voff, uint32_t soff)
    {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(b.r, voff, soff, 0));
    }
};

template <> struct BufLd<bf16> {
    static __device__ __forceinline__ float ld(const Buf &b, uint32_t voff, uint32_t soff)
    {
        return bf16_to_f32(__builtin_amdgcn_raw_buffer_load_b16(b.r, voff, soff, 0));
    }
};

// Load at lane byte offset voff within a plane.
template <typename S>
__device__ __forceinline__ typename Store<S>::C plane_ld(const PlaneRef &p, uint32_t voff)
{
    return BufLd<S>::ld(p.b, voff, p.soff);
}

// f(std::integral_constant<int, I>{}) for I = 0 .. N - 1, expanded at compile
// time whatever the loop unroller's size limits (register arrays indexed by
// I stay in registers).
template <int N, int I = 0, typename F> __device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<N, I + 1>(f);
    }
}

// least common multiple, for the lengths of unrolled rounds over several
// register rings
constexpr int lcm_int(int a, int b)
{
    int x = a, y = b;
    while (y) {
        const int t = x % y;
        x = y;
        y = t;
    }
    return a / x * b;
}

// ---------------------------------------------------------------------------
// workgroup order
// ---------------------------------------------------------------------------

// Workgroup order. Dispatch sends workgroup i to XCD i % 8. With the XCD flag
// the bijection below gives XCD k a contiguous range of tile numbers (the first
// total % 8 XCDs one more than the others), so tiles that run on one XCD at the
// same time are neighbours and share halo lines in that XCD's L2. Tile numbers
// run fastest along x (x-neighbours share the cache lines that hold their x
// halo), or along y with STAR_FLAG_YFIRST (y-neighbours share halo rows), then
// along the other axis, then over z chunks.
__device__ __forceinline__ int xcd_remap(int lin, int total)
{
    const int nxcd = 8;
    const int per = total / nxcd, rem = total % nxcd;
    const int xcd = lin % nxcd, slot = lin / nxcd;
    return xcd < rem ? xcd * (per + 1) + slot : rem * (per + 1) + (xcd - rem) * per + slot;
}

// ---------------------------------------------------------------------------
// cross-lane moves
// ---------------------------------------------------------------------------
//
// One-lane shifts across the whole 64-lane wave through the data-parallel
// primitive (DPP) source modifier: lane_up gives lane i the value of lane
// i - 1 (wave_shr:1), lane_down the value of lane i + 1 (wave_shl:1). The lane
// with no source (0, resp. 63) keeps its own value. DPP moves 32 bits, so a
// 64-bit value takes two. Every lane of the wave must execute the shift (the
// kernels call them outside divergent code).
constexpr int DPP_WAVE_SHL1 = 0x130, DPP_WAVE_SHR1 = 0x138;

template <int CTRL> __device__ __forceinline__ uint32_t dpp32(uint32_t v)
{
    return uint32_t(__builtin_amdgcn_update_dpp(int(v), int(v), CTRL, 0xf, 0xf, false));
}

template <int CTRL> __device__ __forceinline__ uint64_t dpp64(uint64_t v)
{
    const uint32_t lo = dpp32<CTRL>(uint32_t(v)), hi = dpp32<CTRL>(uint32_t(v >> 32));
    return uint64_t(lo) | (uint64_t(hi) << 32);
}

template <int CTRL> __device__ __forceinline__ float dpp_val(float v)
{
    return __builtin_bit_cast(float, dpp32<CTRL>(__builtin_bit_cast(uint32_t, v)));
}
template <int CTRL> __device__ __forceinline__ double dpp_val(double v)
{
    return __builtin_bit_cast(double, dpp64<CTRL>(__builtin_bit_cast(uint64_t, v)));
}
template <int CTRL> __device__ __forceinline__ uint32_t dpp_val(uint32_t v) { return dpp32<CTRL>(v); }
template <int CTRL> __device__ __forceinline__ uint64_t dpp_val(uint64_t v) { return dpp64<CTRL>(v); }

template <typename T> __device__ __forceinline__ T lane_up(T v) { return dpp_val<DPP_WAVE_SHR1>(v); }
template <typename T> __device__ __forceinline__ T lane_down(T v) { return dpp_val<DPP_WAVE_SHL1>(v); }

inline size_t dtype_size(int dtype)
{
    return dtype == STENCIL_F64 ? 8 : dtype == STENCIL_F32 ? 4 : dtype == STENCIL_BF16 ? 2 : 0;
}

// ---------------------------------------------------------------------------
// padded geometry
// ---------------------------------------------------------------------------

// Interior extents n, radius r, padded strides. Unused axes have n = 1 and no
// padding. Interior point (x, y, z) lives at padded cell (x+ox, y+ry, z+rz):
// by default ox = r and rows hold nx + 2r cells; a layout may instead start
// the interior at column ox >= r and use a longer row pitch sy, e.g. to put
// the interior of every row on a cache-line boundary.
struct Geo {
    int ndim;
    int nx, ny, nz;
    int r, ry, rz;
    int ox;         // column of interior x = 0
    int64_t sy, sz; // element strides of y and z in the padded array

    __host__ __device__ int64_t at(int x, int y, int z) const
    {
        return static_cast<int64_t>(x + ox) + sy * (y + ry) + sz * (z + rz);
    }
};

// pitch 0 / ox < 0 select the default layout (rows of nx + 2r, ox = r)
inline Geo make_geo(int ndim, const int *dims, int r, int pitch = 0, int ox = -1)
{
    Geo g;
    g.ndim = ndim;
    g.nx = dims[0];
    g.ny = ndim > 1 ? dims[1] : 1;
    g.nz = ndim > 2 ? dims[2] : 1;
    g.r = r;
    g.ry = ndim > 1 ? r : 0;
    g.rz = ndim > 2 ? r : 0;
    g.ox = ox < 0 ? r : ox;
    g.sy = pitch > 0 ? pitch : g.nx + 2 * r;
    g.sz = g.sy * (g.ny + 2 * g.ry);
    return g;
}

__host__ __device__ inline int64_t padded_elems(const Geo &g)
{
    return g.sz * (g.nz + 2 * g.rz);
}

// Store v at interior point (x, y, z) and, when fuse is set, at every periodic
// image of the point that falls inside the halo, so the output's halo is valid
// without a separate pass (Eq. 2 with a periodic beta). Images along an axis:
// x + n when x < r, x - n when x >= n - r (both when n < 2r).
template <typename S>
__device__ __forceinline__ void store_periodic(S *out, const Geo &g, int x, int y, int z,
                                               typename Store<S>::C v, bool fuse)
{
    Store<S>::st(out + g.at(x, y, z), v);
    if (!fuse)
        return;
    const int r = g.r;
    bool nx_ = x < r || x >= g.nx - r;
    bool ny_ = g.ry && (y < r || y >= g.ny - r);
    bool nz_ = g.rz && (z < r || z >= g.nz - r);
    if (!(nx_ || ny_ || nz_))
        return;
    int xs[3], ys[3], zs[3];
    int cx = 0, cy = 0, cz = 0;
    xs[cx++] = x;
    if (x < r) xs[cx++] = x + g.nx;
    if (x >= g.nx - r) xs[cx++] = x - g.nx;
    ys[cy++] = y;
    if (g.ry) {
        if (y < r) ys[cy++] = y + g.ny;
        if (y >= g.ny - r) ys[cy++] = y - g.ny;
    }
    zs[cz++] = z;
    if (g.rz) {
        if (z < r) zs[cz++] = z + g.nz;
        if (z >= g.nz - r) zs[cz++] = z - g.nz;
    }
    for (int iz = 0; iz < cz; ++iz)
        for (int iy = 0; iy < cy; ++iy)
            for (int ix = 0; ix < cx; ++ix)
                if (ix | iy | iz)
                    Store<S>::st(out + g.at(xs[ix], ys[iy], zs[iz]), v);
}

// Periodic images of one interior point on a grid whose axes all hold at
// least 2r points (then a point has at most one image per axis): the element
// offsets of its x, y and z images, 0 where it has none. A kernel that stores
// several fields at the point computes them once. Offsets fit 32 bits for
// arrays below 4 GiB.
struct PointImages {
    int32_t dx, dy, dz;
};

__host__ __device__ inline bool images_simple(const Geo &g)
{
    return g.nx >= 2 * g.r && (!g.ry || g.ny >= 2 * g.r) && (!g.rz || g.nz >= 2 * g.r);
}

__device__ __forceinline__ PointImages point_images(const Geo &g, int x, int y, int z)
{
    const int r = g.r;
    PointImages m;
    m.dx = x < r ? g.nx : x >= g.nx - r ? -g.nx : 0;
    m.dy = !g.ry ? 0 : (y < r ? g.ny : y >= g.ny - r ? -g.ny : 0) * int32_t(g.sy);
    m.dz = !g.rz ? 0 : (z < r ? g.nz : z >= g.nz - r ? -g.nz : 0) * int32_t(g.sz);
    return m;
}

// store_periodic for a point whose images point_images gave
template <typename S>
__device__ __forceinline__ void store_images(S *out, int64_t p, const PointImages &m,
                                             typename Store<S>::C v, bool fuse)
{
    S *const q = out + p;
    Store<S>::st(q, v);
    if (!fuse || !(m.dx | m.dy | m.dz))
        return;
    if (m.dx) Store<S>::st(q + m.dx, v);
    if (m.dy) Store<S>::st(q + m.dy, v);
    if (m.dx && m.dy) Store<S>::st(q + m.dx + m.dy, v);
    if (m.dz) {
        Store<S>::st(q + m.dz, v);
        if (m.dx) Store<S>::st(q + m.dz + m.dx, v);
        if (m.dy) Store<S>::st(q + m.dz + m.dy, v);
        if (m.dx && m.dy) Store<S>::st(q + m.dz + m.dx + m.dy, v);
    }
}

} // namespace stn
