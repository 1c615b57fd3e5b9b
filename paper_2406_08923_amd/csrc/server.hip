// server.hip -- continuous-batching server for stencil-integration jobs.
//
// One host thread per server owns two HIP streams (default priority: one for
// compute, one for copies) and loops:
//   1. admit queued jobs, first fit in arrival order, while their resident
//      state fits the free HBM budget and a slot is free;
//   2. enqueue one tick on the compute stream: upload the job table, then
//      tick_steps x 3 substeps of the persistent batched kernels (replayed
//      from a captured hipGraph whose launches do not depend on the job set);
//   3. while the tick runs, on the copy stream: download and free the jobs
//      that finished in the previous tick, allocate and upload the jobs just
//      admitted (they join the next tick);
//   4. wait for both streams; retire finished and cancelled jobs.
// Host-device transfers thus overlap the batched compute. Jobs arriving while
// a tick runs wait at most one tick for admission plus one for their upload;
// a finished job's result lands one tick later. A device error fails the
// running jobs and latches the server.
#include "advdiff_zm.hpp"
#include "batch.hpp"
#include "tune_cache.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

using namespace stn;

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr int STARVE_TICKS = 16;

struct SJob {
    uint64_t ticket = 0;
    stencil_job d{};
    int state = STENCIL_JOB_QUEUED;
    int error = 0;
    double t_submit = -1, t_admit = -1, t_first = -1, t_done = -1;
    long long steps_done = 0;
    bool cancel = false;
    size_t bytes = 0;
    BatchJob bj{};
    int steps_tick = 0;
    int idle_ticks = 0; // consecutive ticks the job was resident but left out
};

size_t job_bytes(const stencil_job &j)
{
    size_t pad = 1;
    for (int a = 0; a < j.ndim; ++a) pad *= (size_t)j.dims[a] + 6;
    // f (two buffers), registers, master
    if (j.precision == STENCIL_PREC_F64) return pad * (8 + 8 + 8);
    if (j.precision == STENCIL_PREC_F32_MASTER64) return pad * (4 + 4 + 4 + 4 + 8);
    return pad * (4 + 4 + 4);
}

int check_job(const stencil_job *j)
{
    if (!j)
        return fail(STENCIL_EINVAL, "job is NULL");
    if (j->ndim != 2 && j->ndim != 3)
        return fail(STENCIL_EINVAL, "job ndim must be 2 or 3");
    for (int a = 0; a < j->ndim; ++a)
        if (j->dims[a] < 3 || j->dims[a] > 65536)
            return fail(STENCIL_EINVAL, "job dims[%d] = %d out of range", a, j->dims[a]);
    if (j->steps < 1)
        return fail(STENCIL_EINVAL, "job steps must be >= 1");
    if (j->precision != STENCIL_PREC_F64 && j->precision != STENCIL_PREC_F32_MASTER64 &&
        j->precision != STENCIL_PREC_F32_ONLY)
        return fail(STENCIL_EINVAL, "job precision must be F64, F32_MASTER64 or F32_ONLY");
    if (!std::isfinite(j->nu) || !std::isfinite(j->dt) || !std::isfinite(j->adv[0]) ||
        !std::isfinite(j->adv[1]) || !std::isfinite(j->adv[2]))
        return fail(STENCIL_EINVAL, "job parameters must be finite");
    if (!j->init || !j->result)
        return fail(STENCIL_EINVAL, "job init and result must be host pointers");
    size_t pad = 1;
    for (int a = 0; a < j->ndim; ++a) pad *= (size_t)j->dims[a] + 6;
    if (pad * 8 >= (size_t(1) << 32))
        return fail(STENCIL_EINVAL, "job grid too large (padded state must stay below 4 GiB)");
    return STENCIL_OK;
}

} // namespace

struct stencil_server_s {
    stencil_server_desc d{};
    int device = 0;
    hipStream_t stream = nullptr;  // compute
    hipStream_t cstream = nullptr; // copies, allocation and frees
    std::thread worker;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    bool stop = false;
    int sticky = 0;
    std::deque<std::shared_ptr<SJob>> queue;
    std::vector<std::shared_ptr<SJob>> active; // worker thread only
    std::unordered_map<uint64_t, std::shared_ptr<SJob>> jobs;
    uint64_t next_ticket = 1;
    size_t used = 0;
    std::chrono::steady_clock::time_point t0;
    void *d_table = nullptr, *h_table = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    RkCoeffs rk{};
    stencil_server_stats st{};
    FdWeights fd{};
    long long min_points = 0;
    // batch schedule per job class (ndim, dims, policy): z-march jobs {lz, 0},
    // per-point jobs {tile_w, tile_h}; filled by the search (desc.tune)
    std::unordered_map<std::string, std::pair<int, int>> sched;

    double clock() const
    {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }

    // --- worker side -------------------------------------------------------

    // stream-ordered free on the copy stream (no device-wide synchronisation;
    // callers only free jobs that no enqueued tick uses)
    void free_job(SJob &j)
    {
        void *bufs[] = {j.bj.f[0], j.bj.f[1], j.bj.w, j.bj.w2, j.bj.f64};
        for (void *b : bufs)
            if (b) (void)hipFreeAsync(b, cstream);
        j.bj.f[0] = j.bj.f[1] = j.bj.w = j.bj.w2 = nullptr;
        j.bj.f64 = nullptr;
    }

    void finish(const std::shared_ptr<SJob> &j, int state, int err)
    {
        std::lock_guard<std::mutex> lk(mu);
        j->state = state;
        j->error = err;
        j->t_done = clock();
        used -= j->bytes;
        if (state == STENCIL_JOB_DONE) {
            st.completed++;
            size_t pts = 1;
            for (int a = 0; a < j->d.ndim; ++a) pts *= (size_t)j->d.dims[a];
            st.point_steps += (long long)pts * j->d.steps;
        } else if (state == STENCIL_JOB_FAILED) {
            st.failed++;
        } else {
            st.cancelled++;
        }
        cv_done.notify_all();
    }

    static int job_policy(const stencil_job &d)
    {
        return d.precision == STENCIL_PREC_F64 ? POL_F64
               : d.precision == STENCIL_PREC_F32_MASTER64 ? POL_F32_MASTER64
                                                          : POL_F32_ONLY;
    }

    static std::string class_key(const stencil_job &d)
    {
        return "batch|nd" + std::to_string(d.ndim) + "|" + std::to_string(d.dims[0]) + "x" +
               std::to_string(d.dims[1]) + "x" + std::to_string(d.ndim == 3 ? d.dims[2] : 1) +
               "|p" + std::to_string(job_policy(d));
    }

    // the default schedule of a job (no search): z march depth from the grid
    // size, 64 x 4 per-point tiles
    static std::pair<int, int> default_sched(const BatchJob &b)
    {
        if (advdiff_uses_zmarch(b.g))
            return {advdiff_zmarch_lz(b.g), 0};
        return {BT_X, BT_Y};
    }

    // Search of a job class's batch schedule (Sec. 5.1: candidates timed,
    // failed launches dropped): the job's substeps are run through the
    // batched kernels as a one-job table on scratch buffers of its size, for
    // every candidate (z-march jobs: 8, 16, 32, 64 planes per tile; per-point
    // jobs: 64 x 4, 128 x 2, 256 x 1, 32 x 8 point tiles); one warm-up step,
    // best of two timed steps. Runs between ticks (the device is idle), on the
    // compute stream. Every candidate computes the same arithmetic per point.
    void tune_class(const SJob &j)
    {
        const std::string key = class_key(j.d);
        if (sched.count(key))
            return;
        std::vector<int> v;
        if (tune_cache_get(key, v) && v.size() == 2) {
            sched[key] = {v[0], v[1]};
            return;
        }
        BatchJob b{};
        fill_job(j.d, b);
        const bool zm = advdiff_uses_zmarch(b.g);
        std::vector<std::pair<int, int>> cands;
        if (zm) {
            for (int lz : {8, 16, 32, 64})
                if (lz <= b.g.nz || lz == 8)
                    cands.push_back({lz, 0});
        } else {
            cands = {{64, 4}, {128, 2}, {256, 1}, {32, 8}};
        }
        const size_t pad = (size_t)padded_elems(b.g);
        const size_t es = b.policy == POL_F64 ? 8 : 4;
        const bool master = b.policy == POL_F32_MASTER64;
        char *base = nullptr;
        void *tab = nullptr;
        auto up = [](size_t n) { return (n + 255) / 256 * 256; };
        const size_t fb = up(pad * es), mb = up(pad * 8);
        const size_t total = 3 * fb + (master ? fb + mb : 0);
        hipEvent_t e0 = nullptr, e1 = nullptr;
        std::pair<int, int> best = default_sched(b);
        float best_ms = 1e30f;
        bool ok = hipMalloc(reinterpret_cast<void **>(&base), total) == hipSuccess &&
                  hipMalloc(&tab, batch_table_bytes(1)) == hipSuccess &&
                  hipMemset(base, 0, total) == hipSuccess &&
                  hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess;
        if (ok) {
            b.f[0] = base;
            b.f[1] = base + fb;
            b.w = base + 2 * fb;
            if (master) {
                b.w2 = base + 3 * fb;
                b.f64 = reinterpret_cast<double *>(base + 4 * fb);
            }
            b.steps = 1;
            b.parity = 0;
            b.tile_begin = 0;
            for (const auto &c : cands) {
                BatchTableHeader h{};
                BatchJob r = b;
                if (zm) {
                    r.tiles_x = (b.g.nx + ZM_TX - 1) / ZM_TX;
                    r.tiles_y = (b.g.ny + ZM_ROWS - 1) / ZM_ROWS;
                    r.lz = c.first;
                    h.njobs = 1;
                    h.n2d = 0;
                    h.total3 = r.tiles_x * r.tiles_y * ((b.g.nz + r.lz - 1) / r.lz);
                } else {
                    r.tile_w = c.first;
                    r.tile_h = c.second;
                    r.tiles_x = (b.g.nx + r.tile_w - 1) / r.tile_w;
                    r.tiles_y = (b.g.ny + r.tile_h - 1) / r.tile_h;
                    h.njobs = 1;
                    h.n2d = 1;
                    h.total_tiles = r.tiles_x * r.tiles_y * b.g.nz;
                }
                std::vector<char> host(batch_table_bytes(1));
                std::memcpy(host.data(), &h, sizeof(h));
                std::memcpy(host.data() + sizeof(h), &r, sizeof(r));
                if (hipMemcpy(tab, host.data(), host.size(), hipMemcpyHostToDevice) != hipSuccess)
                    break;
                auto one_step = [&]() {
                    int rc = STENCIL_OK;
                    for (int sub = 0; sub < 3 && !rc; ++sub)
                        rc = launch_batch_substep(tab, sub, rk, d.blocks, stream);
                    return rc;
                };
                if (one_step() || hipStreamSynchronize(stream) != hipSuccess) {
                    (void)hipGetLastError();
                    continue;
                }
                float ms = 1e30f;
                bool good = true;
                for (int rep = 0; rep < 2 && good; ++rep) {
                    good = hipEventRecord(e0, stream) == hipSuccess && one_step() == STENCIL_OK &&
                           hipEventRecord(e1, stream) == hipSuccess &&
                           hipEventSynchronize(e1) == hipSuccess;
                    float t = 0;
                    if (good && hipEventElapsedTime(&t, e0, e1) == hipSuccess)
                        ms = std::min(ms, t);
                }
                if (!good) {
                    (void)hipGetLastError();
                    continue;
                }
                if (ms < best_ms) {
                    best_ms = ms;
                    best = c;
                }
            }
        }
        (void)hipGetLastError();
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (tab) (void)hipFree(tab);
        if (base) (void)hipFree(base);
        sched[key] = best;
        tune_cache_put(key, {best.first, best.second});
        std::lock_guard<std::mutex> lk(mu);
        st.tuned_classes++;
    }

    // geometry and constants of a job's batch record (buffers not set)
    void fill_job(const stencil_job &d, BatchJob &b) const
    {
        b.g = make_geo(d.ndim, d.dims, 3);
        b.fd = fd;
        double dsmin = 1e300;
        for (int a = 0; a < 3; ++a) {
            const double ds = a < d.ndim ? 2.0 * kPi / d.dims[a] : 1.0;
            b.inv_ds[a] = a < d.ndim ? 1.0 / ds : 0.0;
            b.adv[a] = a < d.ndim ? d.adv[a] : 0.0;
            if (a < d.ndim) dsmin = std::min(dsmin, ds);
        }
        double cmax = 1.0;
        for (int a = 0; a < d.ndim; ++a) cmax = std::max(cmax, std::fabs(d.adv[a]));
        b.nu = d.nu;
        b.dt = d.dt > 0 ? d.dt : 0.1 * dsmin / cmax;
        b.policy = job_policy(d);
        b.parity = 0;
        b.tile_w = BT_X;
        b.tile_h = BT_Y;
    }

    // allocate and upload one admitted job; returns a status
    int start_job(SJob &j)
    {
        const stencil_job &d = j.d;
        BatchJob &b = j.bj;
        fill_job(d, b);
        // stream-ordered allocation and upload on the copy stream; the caller
        // waits for the copy stream before the job joins a tick
        const size_t pad = (size_t)padded_elems(b.g);
        const size_t es = b.policy == POL_F64 ? 8 : 4;
        auto alloc = [&](void **p, size_t bytes) {
            return hipMallocAsync(p, bytes, cstream) == hipSuccess;
        };
        bool ok = alloc(&b.f[0], pad * es) && alloc(&b.f[1], pad * es) && alloc(&b.w, pad * es);
        if (ok && b.policy == POL_F32_MASTER64)
            ok = alloc(&b.w2, pad * 4) && alloc(reinterpret_cast<void **>(&b.f64), pad * 8);
        if (!ok) {
            (void)hipGetLastError();
            free_job(j);
            return STENCIL_ENOMEM;
        }
        const size_t n = pad ? (size_t)b.g.nx * b.g.ny * b.g.nz : 0;
        double *stage = nullptr;
        if (!alloc(reinterpret_cast<void **>(&stage), n * 8)) {
            (void)hipGetLastError();
            free_job(j);
            return STENCIL_ENOMEM;
        }
        int rc = STENCIL_OK;
        if (hipMemcpyAsync(stage, d.init, n * 8, hipMemcpyHostToDevice, cstream) != hipSuccess)
            rc = STENCIL_EDEVICE;
        if (!rc)
            rc = launch_job_upload(stage, b, 0, cstream);
        (void)hipFreeAsync(stage, cstream);
        if (rc)
            free_job(j);
        return rc;
    }

    int download_job(SJob &j)
    {
        const BatchJob &b = j.bj;
        const size_t n = (size_t)b.g.nx * b.g.ny * b.g.nz;
        double *stage = nullptr;
        if (hipMallocAsync(reinterpret_cast<void **>(&stage), n * 8, cstream) != hipSuccess) {
            (void)hipGetLastError();
            return STENCIL_ENOMEM;
        }
        int rc = launch_job_download(b, b.parity, stage, cstream);
        if (!rc && hipMemcpyAsync(j.d.result, stage, n * 8, hipMemcpyDeviceToHost, cstream) !=
                       hipSuccess)
            rc = STENCIL_EDEVICE;
        (void)hipFreeAsync(stage, cstream);
        return rc;
    }

    int capture_graph()
    {
        const int nsub = 3 * d.tick_steps;
        if (hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return STENCIL_EDEVICE;
        int rc = STENCIL_OK;
        for (int s = 0; s < nsub && !rc; ++s)
            rc = launch_batch_substep(d_table, s, rk, d.blocks, stream);
        hipGraph_t g = nullptr;
        if (hipStreamEndCapture(stream, &g) != hipSuccess || rc) {
            if (g) (void)hipGraphDestroy(g);
            (void)hipGetLastError();
            return STENCIL_EDEVICE;
        }
        if (hipGraphInstantiate(&gexec, g, nullptr, nullptr, 0) != hipSuccess) {
            (void)hipGraphDestroy(g);
            (void)hipGetLastError();
            return STENCIL_EDEVICE;
        }
        graph = g;
        return STENCIL_OK;
    }

    // one tick; returns a status, *launches the number of kernel launches it
    // enqueued. The tick takes resident jobs until it holds at least
    // min_points points per substep (enough to fill the GPU); the others wait
    // resident for a later tick. STENCIL_SERVE_OLDEST (the default) takes them
    // in submission order (no job is passed by a later one, which bounds the
    // tail as a first-come queue does), then adds shorter jobs, least
    // remaining work first, while the tick's points grow by at most a quarter,
    // so small jobs still pass a large one. STENCIL_SERVE_SHORTEST takes them
    // in order of remaining point-steps, so short jobs finish within a few
    // ticks while long ones keep the device busy (the lowest median latency
    // under overload, at the cost of the tail); a job left out for
    // STARVE_TICKS ticks in a row is taken regardless, so none waits without
    // bound.
    int tick(long long *launches)
    {
        auto *hdr = static_cast<BatchTableHeader *>(h_table);
        auto *rec = reinterpret_cast<BatchJob *>(hdr + 1);
        std::vector<std::shared_ptr<SJob>> order(active);
        auto pts = [](const SJob &j) { return (double)(j.bj.g.nx) * j.bj.g.ny * j.bj.g.nz; };
        auto remaining = [&](const SJob &j) { return pts(j) * (double)(j.d.steps - j.steps_done); };
        auto by_remaining = [&](const std::shared_ptr<SJob> &a, const std::shared_ptr<SJob> &b) {
            return remaining(*a) < remaining(*b);
        };
        if (d.policy == STENCIL_SERVE_OLDEST)
            std::stable_sort(order.begin(), order.end(),
                             [](const std::shared_ptr<SJob> &a, const std::shared_ptr<SJob> &b) {
                                 return a->ticket < b->ticket;
                             });
        else
            std::stable_sort(order.begin(), order.end(), by_remaining);
        for (auto &j : active)
            j->steps_tick = 0;
        int maxsteps = 0, nsel = 0;
        double points = 0;
        std::vector<SJob *> sel;
        auto take = [&](SJob &j) {
            j.steps_tick = (int)std::min<long long>(d.tick_steps, j.d.steps - j.steps_done);
            maxsteps = std::max(maxsteps, j.steps_tick);
            points += pts(j);
            sel.push_back(&j);
            ++nsel;
        };
        if (d.policy == STENCIL_SERVE_OLDEST) {
            std::vector<std::shared_ptr<SJob>> rest;
            for (auto &jp : order) {
                if (nsel == 0 || points < (double)min_points)
                    take(*jp);
                else
                    rest.push_back(jp);
            }
            std::stable_sort(rest.begin(), rest.end(), by_remaining);
            const double cap = 1.25 * points;
            for (auto &jp : rest)
                if (points + pts(*jp) <= cap)
                    take(*jp);
        } else {
            for (auto &jp : order) {
                SJob &j = *jp;
                if (nsel > 0 && points >= (double)min_points && j.idle_ticks < STARVE_TICKS)
                    continue;
                take(j);
            }
        }
        // table: the 2-D jobs (per-point tiles), then the 3-D jobs (z-march
        // tiles), each kind numbering its own work items
        int tiles = 0, tiles3 = 0, njobs = 0, n2d = 0;
        for (int pass = 0; pass < 2; ++pass) {
            if (pass == 1)
                n2d = njobs;
            for (SJob *jp : sel) {
                const bool d3 = advdiff_uses_zmarch(jp->bj.g);
                if (d3 != (pass == 1))
                    continue;
                BatchJob b = jp->bj;
                b.steps = jp->steps_tick;
                std::pair<int, int> sc = default_sched(b);
                if (d.tune) {
                    auto it = sched.find(class_key(jp->d));
                    if (it != sched.end())
                        sc = it->second;
                }
                if (!d3) {
                    b.tile_w = sc.first;
                    b.tile_h = sc.second;
                    b.tiles_x = (b.g.nx + b.tile_w - 1) / b.tile_w;
                    b.tiles_y = (b.g.ny + b.tile_h - 1) / b.tile_h;
                    b.tile_begin = tiles;
                    tiles += b.tiles_x * b.tiles_y * b.g.nz;
                } else {
                    b.tiles_x = (b.g.nx + ZM_TX - 1) / ZM_TX;
                    b.tiles_y = (b.g.ny + ZM_ROWS - 1) / ZM_ROWS;
                    b.lz = sc.first;
                    b.tile_begin = tiles3;
                    tiles3 += b.tiles_x * b.tiles_y * ((b.g.nz + b.lz - 1) / b.lz);
                }
                rec[njobs++] = b;
            }
        }
        hdr->n2d = n2d;
        hdr->njobs = njobs;
        hdr->total_tiles = tiles;
        hdr->total3 = tiles3;
        if (hipMemcpyAsync(d_table, h_table, batch_table_bytes(njobs),
                           hipMemcpyHostToDevice, stream) != hipSuccess)
            return STENCIL_EDEVICE;
        int rc = STENCIL_OK;
        if (gexec && maxsteps == d.tick_steps) {
            if (hipGraphLaunch(gexec, stream) != hipSuccess)
                rc = STENCIL_EDEVICE;
            *launches = 3 * d.tick_steps;
        } else {
            for (int s = 0; s < 3 * maxsteps && !rc; ++s)
                rc = launch_batch_substep(d_table, s, rk, d.blocks, stream);
            *launches = 3 * maxsteps;
        }
        return rc; // enqueued; the caller waits for the stream
    }

    void fail_all(int err)
    {
        for (auto &j : active) {
            free_job(*j);
            finish(j, STENCIL_JOB_FAILED, err);
        }
        active.clear();
        std::lock_guard<std::mutex> lk(mu);
        sticky = err;
        for (auto &j : queue) {
            j->state = STENCIL_JOB_FAILED;
            j->error = err;
            j->t_done = clock();
            st.failed++;
        }
        queue.clear();
        cv_done.notify_all();
    }

    void run()
    {
        (void)hipSetDevice(device);
        if (d.use_graph && capture_graph() != STENCIL_OK) {
            fail_all(STENCIL_EDEVICE);
            return;
        }
        // jobs whose steps finished in the previous tick: their results are
        // copied out (and their memory freed) while the next tick runs
        std::vector<std::shared_ptr<SJob>> to_download;
        auto fail_lists = [&](int err, std::vector<std::shared_ptr<SJob>> &extra) {
            for (auto *lst : {&to_download, &extra})
                for (auto &j : *lst) {
                    free_job(*j);
                    finish(j, STENCIL_JOB_FAILED, err);
                }
            to_download.clear();
            extra.clear();
            fail_all(err);
        };
        for (;;) {
            std::vector<std::shared_ptr<SJob>> admit;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_work.wait(lk, [&] {
                    return stop || !queue.empty() || !active.empty() || !to_download.empty();
                });
                if (stop)
                    break;
                int slots = d.max_slots - (int)active.size() - (int)to_download.size();
                for (auto it = queue.begin(); it != queue.end();) {
                    auto &j = *it;
                    if (j->cancel) {
                        j->state = STENCIL_JOB_CANCELLED;
                        j->t_done = clock();
                        st.cancelled++;
                        cv_done.notify_all();
                        it = queue.erase(it);
                    } else if (j->bytes > d.hbm_budget) {
                        j->state = STENCIL_JOB_FAILED;
                        j->error = STENCIL_ENOMEM;
                        j->t_done = clock();
                        st.failed++;
                        cv_done.notify_all();
                        it = queue.erase(it);
                    } else if (slots > 0 && used + j->bytes <= d.hbm_budget) {
                        used += j->bytes;
                        slots--;
                        admit.push_back(j);
                        it = queue.erase(it);
                    } else {
                        ++it;
                    }
                }
            }

            // 0. schedule search for job classes seen for the first time (the
            //    device is idle here: the previous tick and copies finished)
            if (d.tune)
                for (auto &j : admit)
                    tune_class(*j);

            // 1. the tick of the resident jobs, enqueued on the compute stream
            const double tb = clock();
            long long nl = 0;
            const bool ticked = !active.empty();
            int rc = ticked ? tick(&nl) : STENCIL_OK;
            if (rc) {
                fail_lists(rc, admit);
                return;
            }
            // 2. meanwhile, on the copy stream: results of the jobs finished in
            //    the previous tick, then the initial states of the admitted ones
            std::vector<int> drc(to_download.size());
            for (size_t k = 0; k < to_download.size(); ++k) {
                drc[k] = download_job(*to_download[k]);
                free_job(*to_download[k]);
            }
            std::vector<std::shared_ptr<SJob>> started;
            for (auto &j : admit) {
                const int urc = start_job(*j);
                if (urc == STENCIL_EDEVICE) {
                    finish(j, STENCIL_JOB_FAILED, urc);
                    fail_lists(urc, started);
                    return;
                }
                if (urc)
                    finish(j, STENCIL_JOB_FAILED, urc);
                else
                    started.push_back(j);
            }
            // 3. wait for both streams
            const bool ok_compute = hipStreamSynchronize(stream) == hipSuccess;
            const bool ok_copy = hipStreamSynchronize(cstream) == hipSuccess;
            const double te = clock();
            if (!ok_compute || !ok_copy) {
                fail_lists(STENCIL_EDEVICE, started);
                return;
            }
            for (size_t k = 0; k < to_download.size(); ++k)
                finish(to_download[k], drc[k] ? STENCIL_JOB_FAILED : STENCIL_JOB_DONE, drc[k]);
            to_download.clear();

            // 4. bookkeeping of the tick
            if (ticked) {
                std::vector<std::shared_ptr<SJob>> keep;
                for (auto &j : active) {
                    j->steps_done += j->steps_tick;
                    j->idle_ticks = j->steps_tick ? 0 : j->idle_ticks + 1;
                    j->bj.parity ^= (3 * j->steps_tick) & 1;
                    if (j->t_first < 0 && j->steps_tick > 0) j->t_first = te;
                    bool cancel;
                    {
                        std::lock_guard<std::mutex> lk(mu);
                        cancel = j->cancel;
                    }
                    if (j->steps_done >= j->d.steps) {
                        to_download.push_back(j);
                    } else if (cancel) {
                        free_job(*j);
                        finish(j, STENCIL_JOB_CANCELLED, 0);
                    } else {
                        keep.push_back(j);
                    }
                }
                active.swap(keep);
            }
            std::lock_guard<std::mutex> lk(mu);
            for (auto &j : started) {
                j->state = STENCIL_JOB_RUNNING;
                j->t_admit = te;
                st.admitted++;
                active.push_back(j);
            }
            if (ticked) {
                st.ticks++;
                st.launches += nl;
                st.busy_s += te - tb;
            }
        }
        // stopping: deliver the results already computed, cancel the rest
        std::vector<int> drc(to_download.size());
        for (size_t k = 0; k < to_download.size(); ++k) {
            drc[k] = download_job(*to_download[k]);
            free_job(*to_download[k]);
        }
        const bool ok = hipStreamSynchronize(cstream) == hipSuccess;
        for (size_t k = 0; k < to_download.size(); ++k)
            finish(to_download[k], (!ok || drc[k]) ? STENCIL_JOB_FAILED : STENCIL_JOB_DONE,
                   !ok ? STENCIL_EDEVICE : drc[k]);
        for (auto &j : active) {
            free_job(*j);
            finish(j, STENCIL_JOB_CANCELLED, 0);
        }
        active.clear();
        (void)hipStreamSynchronize(cstream);
    }
};

extern "C" {

stencil_status stencil_server_create(const stencil_server_desc *desc, stencil_server_t *out)
{
    if (!desc || !out)
        return fail(STENCIL_EINVAL, "NULL descriptor or output");
    *out = nullptr;
    if (desc->max_slots < 1 || desc->max_slots > 4096)
        return fail(STENCIL_EINVAL, "max_slots must be 1..4096");
    if (desc->tick_steps < 1 || desc->tick_steps > 10000)
        return fail(STENCIL_EINVAL, "tick_steps must be 1..10000");
    if (desc->blocks < 0 || desc->queue_cap < 0)
        return fail(STENCIL_EINVAL, "blocks and queue_cap must be >= 0");
    if (desc->policy != STENCIL_SERVE_SHORTEST && desc->policy != STENCIL_SERVE_OLDEST)
        return fail(STENCIL_EINVAL, "policy must be STENCIL_SERVE_SHORTEST or STENCIL_SERVE_OLDEST");
    auto *s = new (std::nothrow) stencil_server_s();
    if (!s)
        return fail(STENCIL_ENOMEM, "out of host memory");
    s->d = *desc;
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return fail(STENCIL_EDEVICE, "no HIP device");
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, s->device) != hipSuccess) {
        delete s;
        return fail(STENCIL_EDEVICE, "cannot query the device");
    }
    if (!s->d.blocks)
        s->d.blocks = 8 * prop.multiProcessorCount;
    if (!s->d.hbm_budget) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
            delete s;
            return fail(STENCIL_EDEVICE, "cannot query free device memory");
        }
        s->d.hbm_budget = fr / 5 * 4;
    }
    if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) {
        delete s;
        return fail(STENCIL_EDEVICE, "cannot create a stream");
    }
    if (hipStreamCreateWithFlags(&s->cstream, hipStreamNonBlocking) != hipSuccess) {
        (void)hipStreamDestroy(s->stream);
        delete s;
        return fail(STENCIL_EDEVICE, "cannot create a stream");
    }
    const size_t tb = batch_table_bytes(s->d.max_slots);
    if (hipMalloc(&s->d_table, tb) != hipSuccess || hipHostMalloc(&s->h_table, tb) != hipSuccess) {
        (void)hipGetLastError();
        if (s->d_table) (void)hipFree(s->d_table);
        (void)hipStreamDestroy(s->stream);
        (void)hipStreamDestroy(s->cstream);
        delete s;
        return fail(STENCIL_ENOMEM, "cannot allocate the job table");
    }
    std::memset(s->h_table, 0, tb);
    s->rk = rk3_coeffs();
    double w1[7], w2[7];
    stencil_fd_weights(1, 3, w1);
    stencil_fd_weights(2, 3, w2);
    for (int m = 1; m <= 3; ++m) {
        s->fd.w1[m - 1] = w1[3 + m];
        s->fd.w2[m] = w2[3 + m];
    }
    s->fd.w2[0] = w2[3];
    s->st.bytes_budget = s->d.hbm_budget;
    s->min_points = s->d.min_points > 0 ? s->d.min_points : (long long)4 << 20;
    s->t0 = std::chrono::steady_clock::now();
    try {
        s->worker = std::thread([s] { s->run(); });
    } catch (...) {
        (void)hipFree(s->d_table);
        (void)hipHostFree(s->h_table);
        (void)hipStreamDestroy(s->stream);
        (void)hipStreamDestroy(s->cstream);
        delete s;
        return fail(STENCIL_ENOMEM, "cannot start the server thread");
    }
    *out = s;
    return STENCIL_OK;
}

stencil_status stencil_server_destroy(stencil_server_t s)
{
    if (!s)
        return STENCIL_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        for (auto &j : s->queue) {
            j->state = STENCIL_JOB_CANCELLED;
            j->t_done = s->clock();
        }
        s->queue.clear();
    }
    s->cv_work.notify_all();
    if (s->worker.joinable())
        s->worker.join();
    if (s->gexec) (void)hipGraphExecDestroy(s->gexec);
    if (s->graph) (void)hipGraphDestroy(s->graph);
    (void)hipFree(s->d_table);
    (void)hipHostFree(s->h_table);
    (void)hipStreamDestroy(s->stream);
    (void)hipStreamDestroy(s->cstream);
    s->cv_done.notify_all();
    delete s;
    return STENCIL_OK;
}

stencil_status stencil_submit(stencil_server_t s, const stencil_job *job, uint64_t *ticket)
{
    if (!s || !ticket)
        return fail(STENCIL_EINVAL, "NULL server or ticket");
    int rc = check_job(job);
    if (rc) return rc;
    auto j = std::make_shared<SJob>();
    j->d = *job;
    j->bytes = job_bytes(*job);
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->sticky)
        return fail(s->sticky, "server stopped after a device failure");
    if (s->d.queue_cap && (int)s->queue.size() >= s->d.queue_cap)
        return fail(STENCIL_EAGAIN, "server queue is full");
    j->ticket = s->next_ticket++;
    j->t_submit = s->clock();
    s->queue.push_back(j);
    s->jobs[j->ticket] = j;
    *ticket = j->ticket;
    s->cv_work.notify_one();
    return STENCIL_OK;
}

static void fill_status(const SJob &j, stencil_job_status *st)
{
    st->state = j.state;
    st->error = j.error;
    st->t_submit = j.t_submit;
    st->t_admit = j.t_admit;
    st->t_first_tick = j.t_first;
    st->t_done = j.t_done;
    st->steps_done = j.steps_done;
}

stencil_status stencil_poll(stencil_server_t s, uint64_t ticket, stencil_job_status *st)
{
    if (!s || !st)
        return fail(STENCIL_EINVAL, "NULL server or status");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->jobs.find(ticket);
    if (it == s->jobs.end())
        return fail(STENCIL_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    fill_status(*it->second, st);
    return STENCIL_OK;
}

stencil_status stencil_wait(stencil_server_t s, uint64_t ticket, stencil_job_status *st,
                            int timeout_ms)
{
    if (!s || !st)
        return fail(STENCIL_EINVAL, "NULL server or status");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->jobs.find(ticket);
    if (it == s->jobs.end())
        return fail(STENCIL_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    auto j = it->second;
    auto done = [&] { return j->state >= STENCIL_JOB_DONE; };
    if (timeout_ms < 0)
        s->cv_done.wait(lk, done);
    else if (!s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), done)) {
        fill_status(*j, st);
        return fail(STENCIL_ETIMEOUT, "job %llu not finished", (unsigned long long)ticket);
    }
    fill_status(*j, st);
    return STENCIL_OK;
}

stencil_status stencil_cancel(stencil_server_t s, uint64_t ticket)
{
    if (!s)
        return fail(STENCIL_EINVAL, "NULL server");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->jobs.find(ticket);
    if (it == s->jobs.end())
        return fail(STENCIL_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    it->second->cancel = true;
    s->cv_work.notify_one();
    return STENCIL_OK;
}

stencil_status stencil_server_stats_get(stencil_server_t s, stencil_server_stats *st)
{
    if (!s || !st)
        return fail(STENCIL_EINVAL, "NULL server or stats");
    std::lock_guard<std::mutex> lk(s->mu);
    *st = s->st;
    st->bytes_in_use = s->used;
    st->queued = (int)s->queue.size();
    int resident = 0;
    for (auto &kv : s->jobs)
        if (kv.second->state == STENCIL_JOB_RUNNING) resident++;
    st->resident = resident;
    return STENCIL_OK;
}

double stencil_server_clock(stencil_server_t s) { return s ? s->clock() : -1.0; }

} // extern "C"
