// rk_api.hip -- C ABI of the fused nonlinear substep (derivative bank + phi +
// low-storage RK3) and of the FP64 diagnostics.
#include "advdiff_zm.hpp"
#include "batch.hpp"
#include "plan.hpp"
#include "reduce_kernels.hpp"
#include "tune_cache.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <new>
#include <utility>
#include <string>
#include <vector>

using namespace stn;

namespace {

// Williamson's 2N-storage third-order Runge-Kutta coefficients.
const double RK_ALPHA[3] = {0.0, -5.0 / 9.0, -153.0 / 128.0};
const double RK_BETA[3] = {1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0};

} // namespace

namespace stn {
RkCoeffs rk3_coeffs()
{
    RkCoeffs c;
    for (int i = 0; i < 3; ++i) {
        c.alpha[i] = RK_ALPHA[i];
        c.beta[i] = RK_BETA[i];
    }
    return c;
}
} // namespace stn

namespace {

bool master_policy(int pol) { return pol == POL_F32_MASTER64 || pol == POL_BF16_MASTER64; }

int store_dtype(int pol)
{
    switch (pol) {
    case POL_F64: return STENCIL_F64;
    case POL_F32_MASTER64:
    case POL_F32_ONLY: return STENCIL_F32;
    default: return STENCIL_BF16;
    }
}

int launch_substep(const stencil_plan_s *p, const stencil_fields *f, int sub, double dt,
                   hipStream_t s)
{
    const RkPlan &P = p->rk;
    RkArgs a{};
    const bool master = master_policy(P.policy);
    for (int k = 0; k < P.nf; ++k) {
        a.fin[k] = f->f_in[k];
        a.fout[k] = f->f_out[k];
        if (master) {
            a.wrd[k] = sub == 1 ? f->w[k] : f->w2[k];
            a.wwr[k] = sub == 0 ? f->w[k] : f->w2[k];
            a.w1[k] = f->w[k];
            a.master[k] = f->f64[k];
        } else {
            a.wrd[k] = f->w[k];
            a.wwr[k] = f->w[k];
        }
    }
    a.g = P.g;
    a.alpha = RK_ALPHA[sub];
    a.beta = RK_BETA[sub];
    for (int i = 0; i < 3; ++i) {
        a.beta_all[i] = RK_BETA[i];
        a.inv_ds[i] = P.inv_ds[i];
        a.adv[i] = P.adv[i];
    }
    a.dt = dt;
    a.nu = P.nu;
    a.mhd = P.mhd;
    a.fd = P.fd;
    a.stage = sub;
    a.fuse = 1;
    a.phases = -1;
    if (P.model == STENCIL_MODEL_ADVDIFF)
        return P.variant == STENCIL_RK_VARIANT_LDS ? launch_rk_advdiff3_zm(P.policy, a, P.bz, s)
                                                   : launch_rk_advdiff(P.policy, a, P.bx, P.by, s);
    if (P.variant == STENCIL_RK_VARIANT_LDS)
        return launch_rk_mhd8_lds(P.model, P.mixed, P.policy, a, P.bx, P.by, P.bz, P.occ, s);
    return launch_rk_mhd8(P.model, P.mixed, P.policy, a, P.bx, P.by, s);
}

int check_fields(const stencil_plan_s *p, const stencil_fields *f, int sub)
{
    if (!f)
        return fail(STENCIL_EINVAL, "fields is NULL");
    const RkPlan &P = p->rk;
    const size_t n = (size_t)padded_elems(P.g);
    const bool master = master_policy(P.policy);
    for (int k = 0; k < P.nf; ++k) {
        int rc = check_buffers(f->f_in[k], f->f_out[k], n * P.store_size, P.store_size);
        if (rc) return rc;
        if (!f->w[k] || reinterpret_cast<uintptr_t>(f->w[k]) % P.reg_size)
            return fail(STENCIL_EINVAL, "w[%d] is NULL or misaligned", k);
        if (master && (sub < 0 || sub >= 1)) {
            if (!f->w2[k] || reinterpret_cast<uintptr_t>(f->w2[k]) % P.reg_size)
                return fail(STENCIL_EINVAL, "w2[%d] is NULL or misaligned", k);
        }
        if (master && (sub < 0 || sub == 2)) {
            if (!f->f64[k] || reinterpret_cast<uintptr_t>(f->f64[k]) % 8)
                return fail(STENCIL_EINVAL, "f64[%d] is NULL or misaligned", k);
        }
    }
    return STENCIL_OK;
}

template <typename S> int halo_fields(const stencil_plan_s *p, void *const *bufs, hipStream_t s)
{
    for (int k = 0; k < p->rk.nf; ++k) {
        int rc = launch_halo<S>(static_cast<S *>(bufs[k]), p->rk.g, s);
        if (rc) return rc;
    }
    return STENCIL_OK;
}

bool brick_built(int bx, int by, int bz, int occ)
{
    bool ok = false;
#define RK_BRICK_OK(X_, Y_, Z_, O_) ok = ok || (bx == X_ && by == Y_ && bz == Z_ && occ == O_);
    RK_BRICK_SHAPES(RK_BRICK_OK)
#undef RK_BRICK_OK
    return ok;
}

// A schedule of an RK plan: variant, block (bx, by, bz), occupancy target.
struct RkSched {
    int variant, bx, by, bz, occ;
};

std::string rk_tune_key(const RkPlan &P)
{
    char buf[256];
    snprintf(buf, sizeof(buf), "rk|m%d|x%d|p%d|nd%d|%dx%dx%d|ox%d|sy%lld", P.model, P.mixed,
             P.policy, P.g.ndim, P.g.nx, P.g.ny, P.g.nz, P.g.ox, (long long)P.g.sy);
    return buf;
}

// Candidate schedules; fixed_* restrict the search to what the descriptor
// pinned.
std::vector<RkSched> rk_candidates(const RkPlan &P, int fixed_variant, bool fixed_block,
                                   bool fixed_occ)
{
    std::vector<RkSched> c;
    const bool mhd = P.model != STENCIL_MODEL_ADVDIFF;
    auto want = [&](int v) { return fixed_variant == STENCIL_RK_VARIANT_AUTO || fixed_variant == v; };
    if (want(STENCIL_RK_VARIANT_LDS)) {
        if (mhd) {
#define RK_BRICK_CAND(X_, Y_, Z_, O_)                                                        \
    if ((!fixed_block || (P.bx == X_ && P.by == Y_ && P.bz == Z_)) && (!fixed_occ || P.occ == O_)) \
        c.push_back({STENCIL_RK_VARIANT_LDS, X_, Y_, Z_, O_});
            RK_BRICK_SHAPES(RK_BRICK_CAND)
#undef RK_BRICK_CAND
        } else if (P.g.ndim == 3) {
            for (int lz : {8, 16, 32, 64})
                if (!fixed_block || P.bz == lz)
                    c.push_back({STENCIL_RK_VARIANT_LDS, ZM_TX, ZM_ROWS, lz, 0});
        }
    }
    if (want(STENCIL_RK_VARIANT_CACHED) && !fixed_occ) {
        const int tiles[][2] = {{64, 4}, {64, 2}, {128, 2}, {256, 1}, {64, 1}};
        for (auto &t : tiles)
            if (!fixed_block || (P.bx == t[0] && P.by == t[1]))
                c.push_back({STENCIL_RK_VARIANT_CACHED, t[0], t[1], 1, 0});
    }
    return c;
}

void set_sched(RkPlan &P, const RkSched &c)
{
    P.variant = c.variant;
    P.bx = c.bx;
    P.by = c.by;
    P.bz = c.bz;
    P.occ = c.occ;
}

// Time one RK3 step of every candidate on scratch buffers (one warm-up step,
// best of two timed steps; candidates whose launch fails are dropped) and keep
// the fastest. The field values do not matter for the timing: the buffers are
// zero (a valid state of every model).
int rk_autotune(stencil_plan_s *p, int fixed_variant, bool fixed_block, bool fixed_occ)
{
    RkPlan &P = p->rk;
    const std::string key = rk_tune_key(P) + "|v" + std::to_string(fixed_variant) +
                            (fixed_block ? "|b" + std::to_string(P.bx) + "x" + std::to_string(P.by) +
                                               "x" + std::to_string(P.bz)
                                         : std::string()) +
                            (fixed_occ ? "|o" + std::to_string(P.occ) : std::string());
    {
        std::vector<int> v;
        if (tune_cache_get(key, v) && v.size() == 5) {
            set_sched(P, {v[0], v[1], v[2], v[3], v[4]});
            return STENCIL_OK;
        }
    }
    const std::vector<RkSched> cands = rk_candidates(P, fixed_variant, fixed_block, fixed_occ);
    if (cands.empty())
        return STENCIL_OK;
    const size_t n = (size_t)padded_elems(P.g);
    auto up = [](size_t b) { return (b + 255) / 256 * 256; }; // keep every buffer aligned
    const size_t fb = up(n * P.store_size), wb = up(n * P.reg_size), mb = up(n * 8);
    const bool master = master_policy(P.policy);
    const size_t per = 2 * fb + wb + (master ? wb + mb : 0);
    char *base = nullptr;
    if (hipMalloc(reinterpret_cast<void **>(&base), per * P.nf) != hipSuccess) {
        (void)hipGetLastError();
        return fail(STENCIL_ENOMEM, "rk autotune: cannot allocate %zu bytes of scratch",
                    per * P.nf);
    }
    if (hipMemset(base, 0, per * P.nf) != hipSuccess) {
        (void)hipFree(base);
        return fail(STENCIL_EDEVICE, "rk autotune: cannot clear the scratch buffers");
    }
    stencil_fields f{};
    for (int k = 0; k < P.nf; ++k) {
        char *q = base + per * k;
        f.f_in[k] = q;
        f.f_out[k] = q + fb;
        f.w[k] = q + 2 * fb;
        if (master) {
            f.w2[k] = q + 2 * fb + wb;
            f.f64[k] = reinterpret_cast<double *>(q + 2 * fb + 2 * wb);
        }
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        (void)hipFree(base);
        return fail(STENCIL_EDEVICE, "rk autotune: cannot create timing events");
    }
    const double dt = 1e-3;
    auto one_step = [&]() {
        stencil_fields cur = f;
        int rc = STENCIL_OK;
        for (int sub = 0; sub < 3 && rc == STENCIL_OK; ++sub) {
            rc = launch_substep(p, &cur, sub, dt, nullptr);
            for (int k = 0; k < P.nf; ++k)
                std::swap(cur.f_in[k], cur.f_out[k]);
        }
        return rc;
    };
    float best = 1e30f;
    RkSched best_c = {P.variant, P.bx, P.by, P.bz, P.occ};
    for (const RkSched &c : cands) {
        set_sched(P, c);
        if (one_step() != STENCIL_OK || hipDeviceSynchronize() != hipSuccess) {
            (void)hipGetLastError();
            continue;
        }
        float ms = 1e30f;
        bool ok = true;
        for (int rep = 0; rep < 2 && ok; ++rep) {
            ok = hipEventRecord(e0, nullptr) == hipSuccess && one_step() == STENCIL_OK &&
                 hipEventRecord(e1, nullptr) == hipSuccess &&
                 hipEventSynchronize(e1) == hipSuccess;
            float t = 0;
            if (ok && hipEventElapsedTime(&t, e0, e1) == hipSuccess)
                ms = std::min(ms, t);
        }
        if (!ok) {
            (void)hipGetLastError();
            continue;
        }
        if (ms < best) {
            best = ms;
            best_c = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(base);
    set_sched(P, best_c);
    tune_cache_put(key, {best_c.variant, best_c.bx, best_c.by, best_c.bz, best_c.occ});
    return STENCIL_OK;
}

} // namespace

extern "C" {

stencil_status stencil_plan_rk(const stencil_rk_desc *d, stencil_plan_t *out)
{
    if (!d || !out)
        return fail(STENCIL_EINVAL, "NULL descriptor or output");
    *out = nullptr;
    if (d->model != STENCIL_MODEL_MHD8 && d->model != STENCIL_MODEL_ADVDIFF &&
        d->model != STENCIL_MODEL_MHD_FULL)
        return fail(STENCIL_EINVAL, "unknown model %d", d->model);
    const bool mhd = d->model != STENCIL_MODEL_ADVDIFF;
    if (mhd && d->ndim != 3)
        return fail(STENCIL_EINVAL, "the MHD models are three-dimensional");
    if (d->mixed != STENCIL_MIXED_TENSOR && d->mixed != STENCIL_MIXED_DIAGONAL)
        return fail(STENCIL_EINVAL, "unknown mixed-derivative form %d", d->mixed);
    if (!mhd && d->mixed != STENCIL_MIXED_TENSOR)
        return fail(STENCIL_EINVAL, "ADVDIFF has no mixed derivatives (mixed must be 0)");
    if (d->model == STENCIL_MODEL_ADVDIFF && d->ndim != 2 && d->ndim != 3)
        return fail(STENCIL_EINVAL, "ADVDIFF needs ndim 2 or 3");
    if (d->precision < STENCIL_PREC_F64 || d->precision > STENCIL_PREC_BF16_ONLY)
        return fail(STENCIL_EINVAL, "unknown precision policy %d", d->precision);
    int rc = check_dims(d->ndim, d->dims, 3, STENCIL_BC_PERIODIC);
    if (rc) return rc;
    for (int a = 0; a < d->ndim; ++a)
        if (!(d->ds[a] > 0.0) || !std::isfinite(d->ds[a]))
            return fail(STENCIL_EINVAL, "ds[%d] must be positive and finite", a);
    const double prm[] = {d->nu, d->eta, d->cs2, d->adv[0], d->adv[1], d->adv[2]};
    for (double v : prm)
        if (!std::isfinite(v))
            return fail(STENCIL_EINVAL, "non-finite model parameter");
    if (d->model == STENCIL_MODEL_MHD_FULL) {
        const double full[] = {d->zeta, d->mu0, d->gamma, d->cp, d->lnrho0, d->K, d->heat,
                               d->cool};
        for (double v : full)
            if (!std::isfinite(v))
                return fail(STENCIL_EINVAL, "non-finite model parameter");
        if (!(d->mu0 > 0.0) || !(d->cp > 0.0) || !(d->gamma > 1.0) || !(d->cs2 > 0.0))
            return fail(STENCIL_EINVAL,
                        "MHD_FULL needs mu0 > 0, cp > 0, gamma > 1 and cs2 (cs0^2) > 0");
    }
    const int ox = d->x_offset ? d->x_offset : 3;
    const int64_t min_pitch = (int64_t)ox + d->dims[0] + 3;
    if (d->x_offset < 0 || d->row_pitch < 0 || ox < 3 || ox > (1 << 20))
        return fail(STENCIL_EINVAL, "x_offset %d must be in [3, 2^20]", ox);
    if (d->row_pitch && (d->row_pitch < min_pitch || d->row_pitch > (1 << 30)))
        return fail(STENCIL_EINVAL, "row_pitch %d not in [x_offset + dims[0] + 3 = %lld, 2^30]",
                    d->row_pitch, (long long)min_pitch);
    if (d->variant < STENCIL_RK_VARIANT_AUTO || d->variant > STENCIL_RK_VARIANT_LDS)
        return fail(STENCIL_EINVAL, "unknown derivative-bank variant %d", d->variant);
    if (d->flags & ~STENCIL_RK_FLAG_AUTOTUNE)
        return fail(STENCIL_EINVAL, "unknown RK plan flags 0x%x", d->flags);
    if (d->occupancy < 0 || d->occupancy > 8)
        return fail(STENCIL_EINVAL, "occupancy %d not in 0..8", d->occupancy);
    if (d->occupancy && (!mhd || d->variant == STENCIL_RK_VARIANT_CACHED))
        return fail(STENCIL_EINVAL, "an occupancy target applies to the MHD LDS bricks only");
    if (d->variant == STENCIL_RK_VARIANT_LDS && d->model == STENCIL_MODEL_ADVDIFF &&
        d->ndim != 3)
        return fail(STENCIL_EUNSUPPORTED, "the staged advection kernel is 3-D");
    // AUTO: LDS bricks for the MHD models, the z march for 3-D advection grids of at
    // least ZM_MIN_POINTS points (the rule the batched job kernel applies),
    // the cached per-point kernel otherwise
    long long npts = 1;
    for (int a = 0; a < d->ndim && a < 3; ++a) npts *= d->dims[a];
    const int variant = d->variant != STENCIL_RK_VARIANT_AUTO ? d->variant
                        : (mhd || (d->ndim == 3 && npts >= ZM_MIN_POINTS))
                            ? STENCIL_RK_VARIANT_LDS
                            : STENCIL_RK_VARIANT_CACHED;
    int bx, by, bz;
    if (variant == STENCIL_RK_VARIANT_LDS && d->model == STENCIL_MODEL_ADVDIFF) {
        // z march: fixed 64 x 16 tiles; block[2] = z planes per tile
        if (d->block[0] || d->block[1])
            return fail(STENCIL_EINVAL, "the advection z march takes only block[2] (z planes)");
        bx = ZM_TX;
        by = ZM_ROWS;
        bz = d->block[2];
        if (bz < 0 || bz > 4096)
            return fail(STENCIL_EINVAL, "z planes per tile must be 1..4096 (0 = by grid size)");
    } else if (variant == STENCIL_RK_VARIANT_LDS) {
        // bricks that measured fastest at 256^3: 16x8x8 (FP64 state, 1024
        // lanes), 32x4x4 (FP32/BF16 storage, 512 lanes)
        const bool f64 = d->precision == STENCIL_PREC_F64;
        bx = d->block[0] ? d->block[0] : f64 ? 16 : 32;
        by = d->block[1] ? d->block[1] : f64 ? 8 : 4;
        bz = d->block[2] ? d->block[2] : f64 ? 8 : 4;
        if (!brick_built(bx, by, bz, d->occupancy))
            return fail(STENCIL_EINVAL, "brick %dx%dx%d with occupancy %d is not built", bx, by,
                        bz, d->occupancy);
    } else {
        bx = d->block[0] ? d->block[0] : 64;
        by = d->block[1] ? d->block[1] : 4;
        bz = 1;
        if (bx < 1 || by < 1 || bx * by > 256 || (bx * by) % 64)
            return fail(STENCIL_EINVAL, "block %dx%d must be a multiple of 64 lanes <= 256",
                        bx, by);
        if (d->block[2] != 0 && d->block[2] != 1)
            return fail(STENCIL_EINVAL, "block[2] must be 0 or 1 (one z plane per workgroup)");
    }

    {
        // the fused-substep kernels address each buffer with 32-bit offsets
        // (raw buffer loads): FP64 buffers must stay below 4 GiB
        int64_t cells = d->row_pitch ? d->row_pitch : min_pitch;
        for (int a = 1; a < d->ndim; ++a) cells *= (int64_t)d->dims[a] + 6;
        if (cells * 8 >= (int64_t(1) << 32))
            return fail(STENCIL_EUNSUPPORTED,
                        "RK plans need padded buffers below 4 GiB in FP64 (%lld cells)",
                        (long long)cells);
    }
    auto *p = new (std::nothrow) stencil_plan_s();
    if (!p)
        return fail(STENCIL_ENOMEM, "out of host memory");
    p->kind = PLAN_RK;
    if (hipGetDevice(&p->device) != hipSuccess) {
        delete p;
        return fail(STENCIL_EDEVICE, "no HIP device");
    }
    RkPlan &P = p->rk;
    P.model = d->model;
    P.policy = d->precision;
    P.nf = mhd ? 8 : 1;
    P.mixed = d->mixed;
    P.g = make_geo(d->ndim, d->dims, 3, d->row_pitch ? d->row_pitch : (int)min_pitch, ox);
    double w1[7], w2[7];
    stencil_fd_weights(1, 3, w1);
    stencil_fd_weights(2, 3, w2);
    for (int m = 1; m <= 3; ++m) {
        P.fd.w1[m - 1] = w1[3 + m];
        P.fd.w2[m] = w2[3 + m];
    }
    P.fd.w2[0] = w2[3];
    for (int a = 0; a < 3; ++a) {
        P.inv_ds[a] = a < d->ndim ? 1.0 / d->ds[a] : 0.0;
        P.adv[a] = a < d->ndim ? d->adv[a] : 0.0;
    }
    P.nu = d->nu;
    P.mhd.nu = d->nu;
    P.mhd.eta = d->eta;
    P.mhd.cs2 = d->cs2;
    if (d->model == STENCIL_MODEL_MHD_FULL) {
        P.mhd.zeta = d->zeta;
        P.mhd.mu0 = d->mu0;
        P.mhd.gamma = d->gamma;
        P.mhd.cp = d->cp;
        P.mhd.lnrho0 = d->lnrho0;
        P.mhd.K = d->K;
        P.mhd.heat = d->heat;
        P.mhd.cool = d->cool;
    }
    P.variant = variant;
    P.bx = bx;
    P.by = by;
    P.bz = bz;
    P.occ = variant == STENCIL_RK_VARIANT_LDS && mhd ? d->occupancy : 0;
    if (P.model == STENCIL_MODEL_ADVDIFF && variant == STENCIL_RK_VARIANT_LDS && !P.bz)
        P.bz = advdiff_zmarch_lz(P.g);
    P.store_size = dtype_size(store_dtype(P.policy));
    P.reg_size = P.policy == POL_F64 ? 8 : 4;
    // AUTO, 2-D FP64 advection grid small enough for LDS: stencil_rk_run keeps
    // the state in LDS for the whole run (one launch)
    P.resident = d->variant == STENCIL_RK_VARIANT_AUTO && d->model == STENCIL_MODEL_ADVDIFF &&
                 P.policy == POL_F64 && resident_fits(d->ndim, d->dims[0], d->dims[1]);
    if ((d->flags & STENCIL_RK_FLAG_AUTOTUNE) && !P.resident) {
        const bool fixed_block = d->block[0] || d->block[1] || d->block[2];
        const int rc2 = rk_autotune(p, d->variant, fixed_block, d->occupancy != 0);
        if (rc2) {
            delete p;
            return rc2;
        }
    }
    *out = p;
    return STENCIL_OK;
}

stencil_status stencil_plan_rk_schedule(stencil_plan_t p, int out[5])
{
    if (!p || p->kind != PLAN_RK)
        return fail(STENCIL_EINVAL, "not an RK plan");
    if (!out)
        return fail(STENCIL_EINVAL, "NULL output");
    const RkPlan &P = p->rk;
    out[0] = P.variant;
    out[1] = P.bx;
    out[2] = P.by;
    out[3] = P.bz;
    out[4] = P.occ;
    return STENCIL_OK;
}

int stencil_plan_nfields(stencil_plan_t p)
{
    if (!p || p->kind != PLAN_RK)
        return fail(STENCIL_EINVAL, "not an RK plan");
    return p->rk.nf;
}

stencil_status stencil_step(stencil_plan_t p, const stencil_fields *f, int sub, double dt,
                            void *stream)
{
    if (!p || p->kind != PLAN_RK)
        return fail(STENCIL_EINVAL, "not an RK plan");
    if (p->sticky)
        return fail(p->sticky, "plan is in an error state from an earlier device failure");
    if (sub < 0 || sub > 2)
        return fail(STENCIL_EINVAL, "substep %d not in 0..2", sub);
    if (!std::isfinite(dt))
        return fail(STENCIL_EINVAL, "dt is not finite");
    int rc = check_fields(p, f, sub);
    if (rc) return rc;
    rc = check_device(p->device);
    if (rc) return rc;
    rc = launch_substep(p, f, sub, dt, static_cast<hipStream_t>(stream));
    if (rc == STENCIL_EDEVICE)
        p->sticky = rc;
    return rc;
}

stencil_status stencil_rk_run(stencil_plan_t p, const stencil_fields *f, int nsteps, double dt,
                              void *stream)
{
    if (!p || p->kind != PLAN_RK)
        return fail(STENCIL_EINVAL, "not an RK plan");
    if (p->sticky)
        return fail(p->sticky, "plan is in an error state from an earlier device failure");
    if (nsteps < 0 || !std::isfinite(dt))
        return fail(STENCIL_EINVAL, "nsteps must be >= 0 and dt finite");
    int rc = check_fields(p, f, -1);
    if (rc) return rc;
    rc = check_device(p->device);
    if (rc) return rc;
    if (nsteps == 0)
        return STENCIL_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (p->rk.resident) {
        // the whole run in LDS; the states land where 3 nsteps substeps with
        // ping-pong buffers would leave them (the last in f_out when 3 nsteps
        // is odd), the register as the last substep that wrote it left it
        const RkPlan &P = p->rk;
        ResidentArgs ra{};
        const bool odd = (nsteps & 1) != 0;
        ra.fin = static_cast<const double *>(f->f_in[0]);
        ra.out_last = static_cast<double *>(odd ? f->f_out[0] : f->f_in[0]);
        ra.out_prev = static_cast<double *>(odd ? f->f_in[0] : f->f_out[0]);
        ra.w = static_cast<double *>(f->w[0]);
        ra.g = P.g;
        ra.fd = P.fd;
        for (int a = 0; a < 2; ++a) {
            ra.inv_ds[a] = P.inv_ds[a];
            ra.adv[a] = P.adv[a];
        }
        ra.nu = P.nu;
        ra.dt = dt;
        for (int i = 0; i < 3; ++i) {
            ra.alpha[i] = RK_ALPHA[i];
            ra.beta[i] = RK_BETA[i];
        }
        ra.nsteps = nsteps;
        rc = launch_rk_advdiff2_resident(ra, s);
        if (rc == STENCIL_EDEVICE)
            p->sticky = rc;
        return rc;
    }
    switch (store_dtype(p->rk.policy)) {
    case STENCIL_F64: rc = halo_fields<double>(p, f->f_in, s); break;
    case STENCIL_F32: rc = halo_fields<float>(p, f->f_in, s); break;
    default: rc = halo_fields<bf16>(p, f->f_in, s); break;
    }
    stencil_fields cur = *f;
    for (int step = 0; step < nsteps && rc == STENCIL_OK; ++step)
        for (int sub = 0; sub < 3 && rc == STENCIL_OK; ++sub) {
            rc = launch_substep(p, &cur, sub, dt, s);
            for (int k = 0; k < p->rk.nf; ++k) {
                void *t = cur.f_in[k];
                cur.f_in[k] = cur.f_out[k];
                cur.f_out[k] = t;
            }
        }
    if (rc == STENCIL_EDEVICE)
        p->sticky = rc;
    return rc;
}

stencil_status stencil_reduce(stencil_plan_t p, const void *const *fields, int nfields,
                              int dtype, double *host_out, void *stream)
{
    if (!p || (p->kind != PLAN_RK && p->kind != PLAN_LINEAR))
        return fail(STENCIL_EINVAL, "not a plan");
    if (!fields || !host_out || nfields < 1 || nfields > 64)
        return fail(STENCIL_EINVAL, "need 1..64 fields and a host output");
    const size_t es = dtype_size(dtype);
    if (!es)
        return fail(STENCIL_EINVAL, "unknown dtype %d", dtype);
    for (int k = 0; k < nfields; ++k)
        if (!fields[k] || reinterpret_cast<uintptr_t>(fields[k]) % es)
            return fail(STENCIL_EINVAL, "field %d is NULL or misaligned", k);
    int rc = check_device(p->device);
    if (rc) return rc;
    const Geo &g = p->kind == PLAN_RK ? p->rk.g : p->lin.g;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int nb = reduce_nblocks(g);
    const int chunk = nfields < 8 ? nfields : 8;
    double *d_partial = nullptr, *d_out = nullptr;
    STN_HIP(hipMallocAsync(reinterpret_cast<void **>(&d_partial),
                           sizeof(double) * 3 * (size_t)nb * chunk, s));
    if (hipMallocAsync(reinterpret_cast<void **>(&d_out), sizeof(double) * 3 * nfields, s) !=
        hipSuccess) {
        (void)hipFreeAsync(d_partial, s);
        return fail(STENCIL_ENOMEM, "reduce: cannot allocate scratch");
    }
    for (int k0 = 0; k0 < nfields && rc == STENCIL_OK; k0 += 8) {
        FieldPtrs fp{};
        int m = nfields - k0 < 8 ? nfields - k0 : 8;
        for (int i = 0; i < m; ++i)
            fp.p[i] = fields[k0 + i];
        rc = launch_reduce(fp, m, dtype, g, d_partial, d_out + 3 * k0, s);
    }
    if (rc == STENCIL_OK &&
        hipMemcpyAsync(host_out, d_out, sizeof(double) * 3 * nfields, hipMemcpyDeviceToHost,
                       s) != hipSuccess)
        rc = fail(STENCIL_EDEVICE, "reduce: copy to host failed");
    (void)hipFreeAsync(d_partial, s);
    (void)hipFreeAsync(d_out, s);
    if (hipStreamSynchronize(s) != hipSuccess && rc == STENCIL_OK)
        rc = fail(STENCIL_EDEVICE, "reduce: stream synchronisation failed");
    return rc;
}

stencil_status stencil_energy(stencil_plan_t p, const void *const *fields, int dtype,
                              double *host_out, void *stream)
{
    if (!p || p->kind != PLAN_RK || p->rk.nf != 8)
        return fail(STENCIL_EINVAL, "energy needs an MHD plan (MHD8 or MHD_FULL)");
    if (!fields || !host_out)
        return fail(STENCIL_EINVAL, "NULL fields or host output");
    const size_t es = dtype_size(dtype);
    if (!es)
        return fail(STENCIL_EINVAL, "unknown dtype %d", dtype);
    for (int k = 0; k < 8; ++k)
        if (!fields[k] || reinterpret_cast<uintptr_t>(fields[k]) % es)
            return fail(STENCIL_EINVAL, "field %d is NULL or misaligned", k);
    int rc = check_device(p->device);
    if (rc) return rc;
    const RkPlan &P = p->rk;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int nb = reduce_nblocks(P.g);
    double *d_partial = nullptr, *d_out = nullptr;
    STN_HIP(hipMallocAsync(reinterpret_cast<void **>(&d_partial), sizeof(double) * 3 * (size_t)nb,
                           s));
    if (hipMallocAsync(reinterpret_cast<void **>(&d_out), sizeof(double) * 3, s) != hipSuccess) {
        (void)hipFreeAsync(d_partial, s);
        return fail(STENCIL_ENOMEM, "energy: cannot allocate scratch");
    }
    FieldPtrs fp{};
    for (int k = 0; k < 8; ++k)
        fp.p[k] = fields[k];
    EnergyCoef ec{};
    for (int a = 0; a < 3; ++a) {
        ec.w1[a] = P.fd.w1[a];
        ec.ids[a] = P.inv_ds[a];
    }
    double sums[3] = {0, 0, 0};
    rc = launch_energy(fp, dtype, P.g, ec, d_partial, d_out, s);
    if (rc == STENCIL_OK &&
        hipMemcpyAsync(sums, d_out, sizeof(sums), hipMemcpyDeviceToHost, s) != hipSuccess)
        rc = fail(STENCIL_EDEVICE, "energy: copy to host failed");
    (void)hipFreeAsync(d_partial, s);
    (void)hipFreeAsync(d_out, s);
    if (hipStreamSynchronize(s) != hipSuccess && rc == STENCIL_OK)
        rc = fail(STENCIL_EDEVICE, "energy: stream synchronisation failed");
    if (rc == STENCIL_OK) {
        host_out[0] = 0.5 * sums[0];
        host_out[1] = 0.5 * sums[1];
    }
    return rc;
}

} // extern "C"
