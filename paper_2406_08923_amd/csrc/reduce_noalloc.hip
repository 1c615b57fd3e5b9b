// reduce_noalloc.hip -- stencil_reduce_noalloc: the FP64 diagnostics of
// stencil_reduce without any device allocation, for callers that cannot
// allocate (code under graph capture, tight serving loops). The pass-1
// partials and the per-field results live in a file-scope device array,
// `scratch`, of fixed size; each GPU holds its own copy until the process
// ends. Host code never passes the array's name to a kernel (on the host it
// is only a stand-in symbol): the device address is looked up once per device
// with hipGetSymbolAddress and kept here.
#include "plan.hpp"
#include "reduce_kernels.hpp"

#include <mutex>

namespace {

// up to 8 fields per pass-1 launch, at most 2048 workgroups each (the fixed
// partition of reduce_nblocks), and the results of up to 64 fields
constexpr int NOALLOC_MAX_FIELDS = 64;
constexpr size_t PARTIAL_DOUBLES = 3 * 8 * 2048;
constexpr size_t SCRATCH_DOUBLES = PARTIAL_DOUBLES + 3 * NOALLOC_MAX_FIELDS;

__device__ __align__(256) double scratch[SCRATCH_DOUBLES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
double *g_ptr[MAX_DEVICES] = {};

// Device address of `scratch` on the current device (looked up on the first
// call on that device, with that device current).
int scratch_on_device(int dev, double **out)
{
    if (dev < 0 || dev >= MAX_DEVICES)
        return stn::fail(STENCIL_EUNSUPPORTED, "reduce_noalloc: device %d beyond %d", dev,
                         MAX_DEVICES);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return stn::fail(STENCIL_EDEVICE, "reduce_noalloc: hipGetSymbolAddress failed: %s",
                             hipGetErrorString(e));
        g_ptr[dev] = static_cast<double *>(p);
    }
    *out = g_ptr[dev];
    return STENCIL_OK;
}

} // namespace

using namespace stn;

extern "C" stencil_status stencil_reduce_noalloc(stencil_plan_t p, const void *const *fields,
                                                 int nfields, int dtype, double *host_out,
                                                 void *stream)
{
    if (!p || (p->kind != PLAN_RK && p->kind != PLAN_LINEAR))
        return fail(STENCIL_EINVAL, "not a plan");
    if (!fields || !host_out || nfields < 1)
        return fail(STENCIL_EINVAL, "need at least one field and a host output");
    if (nfields > NOALLOC_MAX_FIELDS)
        return fail(STENCIL_EINVAL, "reduce_noalloc: %d fields exceed the scratch limit of %d",
                    nfields, NOALLOC_MAX_FIELDS);
    const size_t es = dtype_size(dtype);
    if (!es)
        return fail(STENCIL_EINVAL, "unknown dtype %d", dtype);
    for (int k = 0; k < nfields; ++k)
        if (!fields[k] || reinterpret_cast<uintptr_t>(fields[k]) % es)
            return fail(STENCIL_EINVAL, "field %d is NULL or misaligned", k);
    int rc = check_device(p->device);
    if (rc) return rc;
    const Geo &g = p->kind == PLAN_RK ? p->rk.g : p->lin.g;
    if ((size_t)reduce_nblocks(g) * 3 * 8 > PARTIAL_DOUBLES)
        return fail(STENCIL_EUNSUPPORTED, "reduce_noalloc: partition exceeds the scratch");
    double *base = nullptr;
    rc = scratch_on_device(p->device, &base);
    if (rc) return rc;
    double *d_partial = base, *d_out = base + PARTIAL_DOUBLES;
    hipStream_t s = static_cast<hipStream_t>(stream);
    // every partial and result slot read is written first by the same call
    // (pass 1 writes one triple per workgroup and field, pass 2 one per
    // field), so nothing needs clearing
    for (int k0 = 0; k0 < nfields && rc == STENCIL_OK; k0 += 8) {
        FieldPtrs fp{};
        const int m = nfields - k0 < 8 ? nfields - k0 : 8;
        for (int i = 0; i < m; ++i)
            fp.p[i] = fields[k0 + i];
        rc = launch_reduce(fp, m, dtype, g, d_partial, d_out + 3 * k0, s);
    }
    if (rc == STENCIL_OK &&
        hipMemcpyAsync(host_out, d_out, sizeof(double) * 3 * nfields, hipMemcpyDeviceToHost,
                       s) != hipSuccess)
        rc = fail(STENCIL_EDEVICE, "reduce_noalloc: copy to host failed");
    if (hipStreamSynchronize(s) != hipSuccess && rc == STENCIL_OK)
        rc = fail(STENCIL_EDEVICE, "reduce_noalloc: stream synchronisation failed");
    return rc;
}
