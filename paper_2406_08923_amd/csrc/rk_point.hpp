// rk_point.hpp -- per-point pieces of the fused substep shared by the solo
// kernels (rk_kernels.hip) and the batched job kernel (batch_kernels.hip):
// buffer-load derivative taps, the 2N register update and the scalar
// advection-diffusion point. Sharing them keeps the arithmetic of a point
// identical whether its job runs alone or in a batch.
#pragma once

#include "rk_kernels.hpp"

namespace stn {

// Taps are buffer loads: vo is the lane's byte offset of the lowest corner of
// its radius-3 neighbourhood, so every tap offset (bytes, wave-uniform) is
// non-negative: c is the centre's offset, st the axis stride in bytes.

// d1 (unit spacing) and d2 (unit spacing) along one axis from the centre c0
// and the taps m_k / q_k at -k / +k.
template <typename C>
__device__ __forceinline__ void d12_vals(C c0, C m1, C q1, C m2, C q2, C m3, C q3,
                                         const FdWeights &w, C &d1, C &d2)
{
    d1 = C(w.w1[0]) * (q1 - m1) + C(w.w1[1]) * (q2 - m2) + C(w.w1[2]) * (q3 - m3);
    d2 = C(w.w2[0]) * c0 + C(w.w2[1]) * (q1 + m1) + C(w.w2[2]) * (q2 + m2) +
         C(w.w2[3]) * (q3 + m3);
}

// d1 and d2 along one axis, taps read from the buffer.
template <typename S, typename C>
__device__ __forceinline__ void d12(const Buf &b, uint32_t vo, uint32_t c, uint32_t st,
                                    const FdWeights &w, C &d1, C &d2, C &c0)
{
    c0 = BufLd<S>::ld(b, vo, c);
    C m1 = BufLd<S>::ld(b, vo, c - st), q1 = BufLd<S>::ld(b, vo, c + st);
    C m2 = BufLd<S>::ld(b, vo, c - 2 * st), q2 = BufLd<S>::ld(b, vo, c + 2 * st);
    C m3 = BufLd<S>::ld(b, vo, c - 3 * st), q3 = BufLd<S>::ld(b, vo, c + 3 * st);
    d12_vals(c0, m1, q1, m2, q2, m3, q3, w, d1, d2);
}

// One axis of the advection-diffusion right-hand side added to R:
// R - c_a/ds_a d1 + nu/ds_a^2 d2.
template <typename C>
__device__ __forceinline__ C advdiff_axis(C R, C a1, C a2, double adv, double inv_ds, double nu)
{
    const C id = C(inv_ds);
    R = fma(-C(adv) * id, a1, R);
    return fma(C(nu) * id * id, a2, R);
}

// The new register of the 2N scheme: w = alpha w + dt R (w not read at the
// first stage).
template <typename C, typename W>
__device__ __forceinline__ C rk_register(double dt, double alpha, int stage, C R, W wold)
{
    C wn = C(dt) * R;
    if (stage > 0)
        wn = fma(C(alpha), C(wold), wn);
    return wn;
}

// d_a d_b (unit spacing), byte strides sa, sb: tensor product of the
// first-derivative weights folded by antisymmetry into 9 four-point terms.
template <typename S, typename C>
__device__ __forceinline__ C dmix(const Buf &b, uint32_t vo, uint32_t c, uint32_t sa,
                                  uint32_t sb, const FdWeights &w)
{
    C acc = 0;
#pragma unroll
    for (int i = 1; i <= 3; ++i)
#pragma unroll
        for (int j = 1; j <= 3; ++j) {
            const uint32_t ia = i * sa, jb = j * sb;
            C q = (BufLd<S>::ld(b, vo, c + ia + jb) - BufLd<S>::ld(b, vo, c - ia + jb)) -
                  (BufLd<S>::ld(b, vo, c + ia - jb) - BufLd<S>::ld(b, vo, c - ia - jb));
            acc = fma(C(w.w1[i - 1] * w.w1[j - 1]), q, acc);
        }
    return acc;
}

// d_a d_b (unit spacing) from the two diagonals of the a-b plane: the
// second-derivative weights taken along (+a, +b) and along (+a, -b); the
// difference of the two is 4 d_a d_b, the centre cancels, 12 loads.
template <typename S, typename C>
__device__ __forceinline__ C dmix_diag(const Buf &b, uint32_t vo, uint32_t c, uint32_t sa,
                                       uint32_t sb, const FdWeights &w)
{
    C acc = 0;
#pragma unroll
    for (int m = 1; m <= 3; ++m) {
        const uint32_t ma = m * sa, mb = m * sb;
        const C along = BufLd<S>::ld(b, vo, c + ma + mb) + BufLd<S>::ld(b, vo, c - ma - mb);
        const C across = BufLd<S>::ld(b, vo, c + ma - mb) + BufLd<S>::ld(b, vo, c - ma + mb);
        acc = fma(C(0.25 * w.w2[m]), along - across, acc);
    }
    return acc;
}

// Forms of the mixed derivatives in the MHD banks (STENCIL_MIXED_*).
constexpr int MIX_TENSOR = 0, MIX_DIAG = 1;

// Register update of the 2N scheme and the new state, per policy.
//   non-master: w = alpha w + dt R (w not read at stage 0, not written at
//               the last stage where it is dead), f_out = f_in + beta w
//   master, stages 0-1: as above in FP32 on the low-precision state
//   master, stage 2: w3 = alpha w2 + dt R; f = f64 + b0 w1 + b1 w2 + b2 w3 in
//               FP64, written to the master and rounded into f_out
struct PointIO {
    void *fout;
    const void *wrd;
    void *wwr;
    const void *w1;
    double *master;
    double alpha, beta, dt;
    double beta_all[3];
    int stage;
    int fuse;
};

// The update with its reads already done: wold = the register (read when
// stage > 0), w1v and mst = the first-stage register and the FP64 state
// (read at the master policies' last stage); unused otherwise.
// IMG: the point's periodic images come precomputed in *im (point_images on
// a grid with images_simple), else store_periodic finds them.
template <typename S, typename W, typename C, bool MASTER, bool IMG = false>
__device__ __forceinline__ void rk_update_pre(const PointIO &io, const Geo &g, int64_t p, int x,
                                              int y, int z, C R, C fc, W wold, W w1v, double mst,
                                              const PointImages *im = nullptr)
{
    const C wn = rk_register<C, W>(io.dt, io.alpha, io.stage, R, wold);
    auto store = [&](C v) {
        if constexpr (IMG)
            store_images(static_cast<S *>(io.fout), p, *im, v, io.fuse != 0);
        else
            store_periodic(static_cast<S *>(io.fout), g, x, y, z, v, io.fuse != 0);
    };
    if (MASTER && io.stage == 2) {
        double f = mst;
        f = fma(io.beta_all[0], double(w1v), f);
        f = fma(io.beta_all[1], double(wold), f);
        f = fma(io.beta_all[2], double(wn), f);
        io.master[p] = f;
        store(C(f));
        return;
    }
    if (io.stage < 2)
        static_cast<W *>(io.wwr)[p] = W(wn);
    store(fma(C(io.beta), wn, fc));
}

template <typename S, typename W, typename C, bool MASTER, bool IMG = false>
__device__ __forceinline__ void rk_update(const PointIO &io, const Geo &g, int64_t p, int x,
                                          int y, int z, C R, C fc,
                                          const PointImages *im = nullptr)
{
    const W wold = io.stage > 0 ? static_cast<const W *>(io.wrd)[p] : W(0);
    const bool last = MASTER && io.stage == 2;
    const W w1v = last ? static_cast<const W *>(io.w1)[p] : W(0);
    const double mst = last ? io.master[p] : 0.0;
    rk_update_pre<S, W, C, MASTER, IMG>(io, g, p, x, y, z, R, fc, wold, w1v, mst, im);
}

// Scalar advection-diffusion R = -c.grad f + nu lap f at interior point
// (x, y, z), NDIM = 2 or 3, followed by the register update.
template <typename S, typename W, typename C, bool MASTER, int NDIM>
__device__ __forceinline__ void advdiff_point(const void *fin, const PointIO &io, const Geo &g,
                                              const FdWeights &fd, const double *inv_ds,
                                              const double *adv, double nu, int x, int y, int z)
{
    const int64_t p = g.at(x, y, z);
    constexpr uint32_t es = sizeof(S);
    const uint32_t st[3] = {es, uint32_t(g.sy) * es, uint32_t(g.sz) * es};
    const uint32_t c = 3 * (st[0] + st[1] + (NDIM == 3 ? st[2] : 0u));
    const uint32_t vo = uint32_t(p) * es - c;
    const Buf fb = make_buf(fin, uint64_t(padded_elems(g)) * es);
    C R = 0, c0 = 0;
#pragma unroll
    for (int ax = 0; ax < NDIM; ++ax) {
        C a1, a2;
        d12<S, C>(fb, vo, c, st[ax], fd, a1, a2, c0);
        R = advdiff_axis(R, a1, a2, adv[ax], inv_ds[ax], nu);
    }
    rk_update<S, W, C, MASTER>(io, g, p, x, y, z, R, c0);
}

} // namespace stn
