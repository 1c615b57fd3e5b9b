// batch_kernels.hip -- batched scalar advection-diffusion substep over a
// device job table: one persistent launch per substep advances every resident
// job (2-D or 3-D, FP64 or FP32 storage with FP64 master). The per-point
// arithmetic is advdiff_point, the same code as the solo kernel, so a job's
// result does not depend on what else is in the batch.
#include "advdiff_zm.hpp"
#include "batch.hpp"
#include "linear_kernels.hpp"

namespace stn {

__global__ void __launch_bounds__(BT_X * BT_Y) k_batch_advdiff(const void *__restrict__ table,
                                                               int sub, RkCoeffs rk)
{
    const BatchTableHeader *hdr = static_cast<const BatchTableHeader *>(table);
    const BatchJob *jobs = reinterpret_cast<const BatchJob *>(hdr + 1);
    const int njobs = hdr->n2d, total = hdr->total_tiles; // the per-point jobs
    const int stage = sub % 3, step = sub / 3;
    for (int item = blockIdx.x; item < total; item += gridDim.x) {
        // job owning the item: last job whose first item is <= item
        int lo = 0, hi = njobs - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (jobs[mid].tile_begin <= item) lo = mid;
            else hi = mid - 1;
        }
        const BatchJob &J = jobs[lo];
        if (step >= J.steps)
            continue;
        const int t = item - J.tile_begin;
        const int bx = t % J.tiles_x, rest = t / J.tiles_x;
        const int by = rest % J.tiles_y, z = rest / J.tiles_y;
        const int lid = threadIdx.x + BT_X * threadIdx.y;
        const int x = bx * J.tile_w + lid % J.tile_w, y = by * J.tile_h + lid / J.tile_w;
        if (x >= J.g.nx || y >= J.g.ny)
            continue;
        const int pin = (J.parity + sub) & 1;
        PointIO io;
        io.fout = J.f[pin ^ 1];
        const bool master = J.policy == POL_F32_MASTER64 || J.policy == POL_BF16_MASTER64;
        io.wrd = master ? (stage == 1 ? J.w : J.w2) : J.w;
        io.wwr = master ? (stage == 0 ? J.w : J.w2) : J.w;
        io.w1 = J.w;
        io.master = J.f64;
        io.alpha = rk.alpha[stage];
        io.beta = rk.beta[stage];
        io.dt = J.dt;
        for (int i = 0; i < 3; ++i) io.beta_all[i] = rk.beta[i];
        io.stage = stage;
        io.fuse = 1;
        const void *fin = J.f[pin];
        const bool d3 = J.g.ndim == 3;
        switch (J.policy) {
        case POL_F64:
            if (d3) advdiff_point<double, double, double, false, 3>(fin, io, J.g, J.fd, J.inv_ds, J.adv, J.nu, x, y, z);
            else advdiff_point<double, double, double, false, 2>(fin, io, J.g, J.fd, J.inv_ds, J.adv, J.nu, x, y, z);
            break;
        case POL_F32_MASTER64:
            if (d3) advdiff_point<float, float, float, true, 3>(fin, io, J.g, J.fd, J.inv_ds, J.adv, J.nu, x, y, z);
            else advdiff_point<float, float, float, true, 2>(fin, io, J.g, J.fd, J.inv_ds, J.adv, J.nu, x, y, z);
            break;
        case POL_F32_ONLY:
            if (d3) advdiff_point<float, float, float, false, 3>(fin, io, J.g, J.fd, J.inv_ds, J.adv, J.nu, x, y, z);
            else advdiff_point<float, float, float, false, 2>(fin, io, J.g, J.fd, J.inv_ds, J.adv, J.nu, x, y, z);
            break;
        default:
            break; // other policies are rejected at submission
        }
    }
}

// The z-march jobs (3-D, at least ZM_MIN_POINTS points): items are z-march
// tiles (advdiff_zm.hpp), the same routine and arithmetic as the solo substep
// of such a job.
__global__ void __launch_bounds__(ZM_NT) k_batch_advdiff3(const void *__restrict__ table, int sub,
                                                          RkCoeffs rk)
{
    __shared__ ZmLds<double> lds;
    const BatchTableHeader *hdr = static_cast<const BatchTableHeader *>(table);
    const BatchJob *jobs = reinterpret_cast<const BatchJob *>(hdr + 1);
    const int first = hdr->n2d, last = hdr->njobs - 1, total = hdr->total3;
    const int stage = sub % 3, step = sub / 3;
    for (int item = blockIdx.x; item < total; item += gridDim.x) {
        int lo = first, hi = last;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (jobs[mid].tile_begin <= item) lo = mid;
            else hi = mid - 1;
        }
        const BatchJob &J = jobs[lo];
        if (step >= J.steps)
            continue; // the whole workgroup skips: no barrier is left unmatched
        const int t = item - J.tile_begin;
        const int bx = t % J.tiles_x, rest = t / J.tiles_x;
        const int by = rest % J.tiles_y, bz = rest / J.tiles_y;
        const int x0 = bx * ZM_TX, y0 = by * ZM_ROWS, z0 = bz * J.lz;
        const int z1 = min(z0 + J.lz, J.g.nz);
        const int pin = (J.parity + sub) & 1;
        PointIO io;
        io.fout = J.f[pin ^ 1];
        const bool master = J.policy == POL_F32_MASTER64 || J.policy == POL_BF16_MASTER64;
        io.wrd = master ? (stage == 1 ? J.w : J.w2) : J.w;
        io.wwr = master ? (stage == 0 ? J.w : J.w2) : J.w;
        io.w1 = J.w;
        io.master = J.f64;
        io.alpha = rk.alpha[stage];
        io.beta = rk.beta[stage];
        io.dt = J.dt;
        for (int i = 0; i < 3; ++i) io.beta_all[i] = rk.beta[i];
        io.stage = stage;
        io.fuse = 1;
        const void *fin = J.f[pin];
        switch (J.policy) {
        case POL_F64:
            advdiff3_zmarch<double, double, double, false>(
                fin, io, J.g, advdiff_star<double>(J.fd, J.inv_ds, J.adv, J.nu), x0, y0, z0, z1,
                lds);
            break;
        case POL_F32_MASTER64:
            advdiff3_zmarch<float, float, float, true>(
                fin, io, J.g, advdiff_star<float>(J.fd, J.inv_ds, J.adv, J.nu), x0, y0, z0, z1,
                *reinterpret_cast<ZmLds<float> *>(&lds));
            break;
        case POL_F32_ONLY:
            advdiff3_zmarch<float, float, float, false>(
                fin, io, J.g, advdiff_star<float>(J.fd, J.inv_ds, J.adv, J.nu), x0, y0, z0, z1,
                *reinterpret_cast<ZmLds<float> *>(&lds));
            break;
        default:
            break; // other policies are rejected at submission
        }
    }
}

int launch_batch_substep(const void *d_table, int sub, const RkCoeffs &rk, int blocks,
                         hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_advdiff, dim3(blocks), dim3(BT_X, BT_Y), 0, s, d_table, sub, rk);
    int rc = check_launch("batch_advdiff");
    if (rc)
        return rc;
    hipLaunchKernelGGL(k_batch_advdiff3, dim3(blocks), dim3(ZM_TX, ZM_TY), 0, s, d_table, sub,
                       rk);
    return check_launch("batch_advdiff3");
}

template <typename S>
__global__ void __launch_bounds__(256) k_job_upload(const double *__restrict__ src, S *dst,
                                                    double *master, Geo g)
{
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int x = int(i % g.nx);
        const int64_t r = i / g.nx;
        const int y = int(r % g.ny), z = int(r / g.ny);
        const int64_t p = g.at(x, y, z);
        const double v = src[i];
        Store<S>::st(dst + p, typename Store<S>::C(v));
        if (master) master[p] = v;
    }
}

template <typename S>
__global__ void __launch_bounds__(256) k_job_download(const S *src, const double *master,
                                                      double *__restrict__ dst, Geo g)
{
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int x = int(i % g.nx);
        const int64_t r = i / g.nx;
        const int y = int(r % g.ny), z = int(r / g.ny);
        const int64_t p = g.at(x, y, z);
        dst[i] = master ? master[p] : double(Store<S>::ld(src + p));
    }
}

static unsigned grid_for(int64_t n)
{
    int64_t b = (n + 255) / 256;
    return (unsigned)(b < 1 ? 1 : b > 65536 ? 65536 : b);
}

int launch_job_upload(const double *src, const BatchJob &j, int which, hipStream_t s)
{
    const int64_t n = (int64_t)j.g.nx * j.g.ny * j.g.nz;
    const bool master = j.policy == POL_F32_MASTER64;
    int rc;
    if (j.policy == POL_F64) {
        hipLaunchKernelGGL(k_job_upload<double>, dim3(grid_for(n)), dim3(256), 0, s, src,
                           static_cast<double *>(j.f[which]), (double *)nullptr, j.g);
        rc = check_launch("job_upload");
        if (!rc) rc = launch_halo<double>(static_cast<double *>(j.f[which]), j.g, s);
    } else {
        hipLaunchKernelGGL(k_job_upload<float>, dim3(grid_for(n)), dim3(256), 0, s, src,
                           static_cast<float *>(j.f[which]), master ? j.f64 : nullptr, j.g);
        rc = check_launch("job_upload");
        if (!rc) rc = launch_halo<float>(static_cast<float *>(j.f[which]), j.g, s);
    }
    return rc;
}

int launch_job_download(const BatchJob &j, int which, double *dst, hipStream_t s)
{
    const int64_t n = (int64_t)j.g.nx * j.g.ny * j.g.nz;
    if (j.policy == POL_F64)
        hipLaunchKernelGGL(k_job_download<double>, dim3(grid_for(n)), dim3(256), 0, s,
                           static_cast<const double *>(j.f[which]), (const double *)nullptr, dst, j.g);
    else
        hipLaunchKernelGGL(k_job_download<float>, dim3(grid_for(n)), dim3(256), 0, s,
                           static_cast<const float *>(j.f[which]),
                           j.policy == POL_F32_MASTER64 ? j.f64 : nullptr, dst, j.g);
    return check_launch("job_download");
}

} // namespace stn
