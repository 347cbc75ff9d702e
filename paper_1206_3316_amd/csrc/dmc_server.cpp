// dmc_server.cpp -- continuous batching of simulation requests on one device.
//
// Requests wait in a FIFO until a slot and enough device memory (a first-fit
// arena carved out of one allocation made at creation) are free.  Each epoch is
// ONE persistent launch over slices of the admitted requests' particle ranges,
// so a request that arrives while others run joins at a later epoch and its
// particles share the device with theirs.  An epoch runs the estimated flights
// that equal shares would give its requests, handed out to the requests with
// the fewest flights left first; a request that starts nothing and has no
// particle suspended sits the epoch out.
// With class epochs, an epoch takes only the requests of one class (the classes
// take turns), so it runs that class's specialised kernel.
// Particles are independent and their random numbers are keyed by (seed, pid),
// so a request's realisation does not depend on how it was sliced or with
// which other requests it ran.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <vector>

#include "dmc_host_internal.h"
#include "dmc_sched.h"

using namespace dmc;

namespace {

// Epoch classes: the kernel specialisation a request runs in when an epoch
// holds only its class (wall-driven slabs, transient half spaces, gradient
// films and pore cells, others).  Without class epochs every request is in
// group 0.
constexpr int kClasses = 4;

int class_of(const JobHost &h)
{
    switch (kernel_spec(&h.dev, 1)) {
    case GEOM_SLAB: return 0;
    case GEOM_HALF: return 1;
    case GEOM_GRAD: return 2;
    default: return 3;
    }
}

struct Request {
    uint64_t ticket = 0;
    int cls = 3;              // epoch class
    JobHost jh;
    size_t bytes = 0, arena_off = 0;
    uint64_t cursor = 0;      // next pid not yet emitted
    uint64_t suspended = 0;   // particles suspended at the end of the last epoch
    double flights_per_particle = 1.0;
    unsigned long long stats[kStats] = {};
    double kernel_ms = 0.0;
    std::vector<double> host_tally;  // filled when complete
};

}  // namespace

struct dmc_server {
    const dmc_material *M = nullptr;
    dmc_server_opts opts{};
    std::mutex mu;
    void *arena_mem = nullptr;
    std::unique_ptr<sched::Arena> arena;
    void *scratch = nullptr;
    LaunchBuffers sb;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    std::deque<std::unique_ptr<Request>> pending;
    std::vector<std::unique_ptr<Request>> active;
    std::map<uint64_t, std::unique_ptr<Request>> done;
    uint64_t next_ticket = 1;
    std::vector<JobDev> epoch_table;  // upload sources of the running epoch
    std::vector<double> epoch_times;
    // Suspended particles wait per epoch group (one group per class with class
    // epochs, else a single group) until their group's next epoch, which resumes them from the
    // group's buffer and suspends into the spare one; the two then swap.
    Suspended *rest[kClasses] = {nullptr, nullptr, nullptr, nullptr};
    Suspended *spare = nullptr;
    uint32_t susp_cap = 0;
    uint32_t n_rest[kClasses] = {0, 0, 0, 0};
    // each group's last epoch: its members and how many particles each left
    // suspended; a member with none may have finished and been collected since,
    // so its pointer is never followed
    std::vector<Request *> prev_members[kClasses];
    std::vector<uint64_t> prev_suspended[kClasses];
    int next_class = 0;              // round-robin start of the class choice
    int32_t *d_resume_job = nullptr;
    std::vector<int32_t> h_resume_job;
    dmc_stats totals{};              // all epochs so far
    ~dmc_server()
    {
        if (ev0) (void)hipEventDestroy(ev0);
        if (ev1) (void)hipEventDestroy(ev1);
        if (arena_mem) (void)hipFree(arena_mem);
        if (scratch) (void)hipFree(scratch);
        for (Suspended *p : rest)
            if (p) (void)hipFree(p);
        if (spare) (void)hipFree(spare);
        if (d_resume_job) (void)hipFree(d_resume_job);
    }
};

namespace {

size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

double flights_estimate(const dmc_material &M, const JobHost &h)
{
    const JobDev &d = h.dev;
    if (d.src == SRC_WALLS) return 2.0 * h.geom.length * M.G_tau / M.G_v + 1.0;  // mean scatters + absorption
    if (d.src == SRC_GAUSSIAN) return h.times.back() * M.G_tau / M.C_tot + 1.0;
    return d.kmax >= 0 ? 1.5 * d.kmax + 1.0 : 1000.0;
}

}  // namespace

extern "C" dmc_status dmc_server_create(const dmc_material *material, const dmc_server_opts *opts, dmc_server **out)
{
    if (!out) return fail(DMC_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!material || !opts) return fail(DMC_E_INVALID, "material / opts is NULL");
    if (opts->max_active < 1 || opts->max_active > kLdsStatJobs) return fail(DMC_E_INVALID, "max_active must be 1..64");
    if (opts->memory_budget < 4096) return fail(DMC_E_INVALID, "memory budget too small");
    dmc_status st = run_opts_check(opts->run);
    if (st != DMC_OK) return st;
    if (opts->run.workspace || opts->run.nscat_out)
        return fail(DMC_E_INVALID, "the server manages its own device memory");
    std::unique_ptr<dmc_server> S(new (std::nothrow) dmc_server());
    if (!S) return fail(DMC_E_NOMEM, "host allocation failed");
    S->M = material;
    S->opts = *opts;
    if (hipMalloc(&S->arena_mem, opts->memory_budget) != hipSuccess) {
        (void)hipGetLastError();
        S->arena_mem = nullptr;
        return fail(DMC_E_NOMEM, "cannot allocate the server's memory budget");
    }
    S->arena.reset(new (std::nothrow) sched::Arena(opts->memory_budget));
    if (!S->arena) return fail(DMC_E_NOMEM, "host allocation failed");
    const size_t nj = (size_t)opts->max_active;
    const size_t jb = a256(nj * sizeof(JobDev)), tb = a256(nj * kMaxTimes * sizeof(double)),
                 stb = a256(nj * kStats * 8), qb = a256(16);
    if (hipMalloc(&S->scratch, jb + tb + stb + qb) != hipSuccess) {
        (void)hipGetLastError();
        S->scratch = nullptr;
        return fail(DMC_E_NOMEM, "cannot allocate server scratch");
    }
    char *p = (char *)S->scratch;
    S->sb.jobs = (JobDev *)p;
    S->sb.times = (double *)(p + jb);
    S->sb.stats = (unsigned long long *)(p + jb + tb);
    S->sb.queue = (unsigned long long *)(p + jb + tb + stb);
    S->sb.tally = (double *)S->arena_mem;
    // every lane of an epoch launch may suspend one particle
    int cus = 256, dev = 0;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    // each lane of an epoch may suspend its particle and each wave up to one
    // chunk (<= 64) of unstarted indices: twice the resident lanes
    S->susp_cap = (uint32_t)cus * 4096u;
    if (hipMalloc(&S->spare, (size_t)S->susp_cap * sizeof(Suspended)) != hipSuccess) {
        (void)hipGetLastError();
        S->spare = nullptr;
        return fail(DMC_E_NOMEM, "cannot allocate the suspended-particle buffers");
    }
    if (hipMalloc(&S->d_resume_job, (size_t)nj * sizeof(int32_t)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(DMC_E_NOMEM, "cannot allocate server scratch");
    }
    DMC_HIP_OR_FAIL(hipEventCreate(&S->ev0));
    DMC_HIP_OR_FAIL(hipEventCreate(&S->ev1));
    *out = S.release();
    return DMC_OK;
}

extern "C" dmc_status dmc_server_submit(dmc_server *S, const dmc_job *job, uint64_t *ticket)
{
    if (!S || !job || !ticket) return fail(DMC_E_INVALID, "NULL argument");
    *ticket = 0;
    if (job->material != S->M) return fail(DMC_E_INVALID, "request uses another material");
    std::unique_ptr<Request> r(new (std::nothrow) Request());
    if (!r) return fail(DMC_E_NOMEM, "host allocation failed");
    dmc_status st = prepare_job(*job, r->jh);
    if (st != DMC_OK) return st;
    r->jh.job.times = nullptr;  // the copy in jh.times is what is used
    r->bytes = a256((size_t)std::max<int64_t>(r->jh.size, 1) * sizeof(double));
    if (r->bytes > S->opts.memory_budget) return fail(DMC_E_INVALID, "request can never fit the memory budget");
    r->flights_per_particle = flights_estimate(*S->M, r->jh);
    r->cls = S->opts.class_epochs ? class_of(r->jh) : 0;  // without class epochs: a single group
    std::lock_guard<std::mutex> g(S->mu);
    r->ticket = S->next_ticket++;
    *ticket = r->ticket;
    S->pending.push_back(std::move(r));
    return DMC_OK;
}

extern "C" dmc_status dmc_server_step(dmc_server *S, int32_t *n_done)
{
    if (!S) return fail(DMC_E_INVALID, "server is NULL");
    if (n_done) *n_done = 0;
    hipStream_t s = (hipStream_t)S->opts.run.stream;
    std::vector<JobDev> devs;
    std::vector<double> &times = S->epoch_times;
    times.clear();
    std::vector<Request *> members;
    LaunchBuffers lb = S->sb;
    int cls = 0;
    if (!S->spare) {  // the buffer the coming epoch suspends into
        if (hipMalloc(&S->spare, (size_t)S->susp_cap * sizeof(Suspended)) != hipSuccess) {
            (void)hipGetLastError();
            S->spare = nullptr;
            return fail(DMC_E_NOMEM, "cannot allocate a suspended-particle buffer");
        }
    }
    {
        std::lock_guard<std::mutex> g(S->mu);
        // admit in arrival order while a slot and memory are free
        {
            const int room = std::max(0, S->opts.max_active - (int)S->active.size());
            const int look = std::min<int>(room, (int)S->pending.size());
            std::vector<size_t> want(look), off(look);
            for (int i = 0; i < look; ++i) want[i] = S->pending[i]->bytes;
            const int n_in = sched::admit(*S->arena, want.data(), look, (int)S->active.size(), S->opts.max_active,
                                          off.data());
            for (int i = 0; i < n_in; ++i) {
                S->pending.front()->arena_off = off[i];
                S->active.push_back(std::move(S->pending.front()));
                S->pending.pop_front();
            }
            for (int i = 0; i < n_in; ++i) {
                const Request *r = S->active[S->active.size() - (size_t)n_in + (size_t)i].get();
                DMC_HIP_OR_FAIL(launch_fill((double *)((char *)S->arena_mem + r->arena_off), r->bytes / 8, nullptr, 0, s));
            }
        }
        if (S->active.empty()) return DMC_OK;
        // the epoch's group: the next class, in turn, with admitted requests
        // (always group 0 without class epochs)
        bool has[kClasses] = {false, false, false, false};
        for (auto &rp : S->active) has[rp->cls] = true;
        cls = sched::next_group(has, kClasses, S->next_class);
        if (cls < 0) return fail(DMC_E_DEVICE, "internal: no epoch group");
        S->next_class = (cls + 1) % kClasses;
        const double epoch_flights = S->opts.epoch_flights ? (double)S->opts.epoch_flights : 2.0e10;
        std::vector<double> fpp;
        std::vector<uint64_t> left, given;
        for (auto &rp : S->active) {
            if (rp->cls != cls) continue;
            fpp.push_back(rp->flights_per_particle);
            left.push_back(rp->jh.dev.n - rp->cursor);
        }
        given.resize(left.size());
        sched::slices(epoch_flights, left.size(), fpp.data(), left.data(), given.data());
        uint64_t base = 0;
        size_t k = 0;
        for (auto &rp : S->active) {
            Request *r = rp.get();
            if (r->cls != cls) continue;
            const uint64_t n = given[k++];
            // a request that starts no particle this epoch and has none suspended
            // stays out of it, so that the epoch's kernel is chosen by the
            // requests that run (one class: its specialised kernel)
            if (n == 0 && r->suspended == 0) continue;
            JobDev d = r->jh.dev;
            const int64_t shift = (int64_t)(r->arena_off / sizeof(double));
            if (d.off_bins >= 0) d.off_bins += shift;
            if (d.off_kappa >= 0) d.off_kappa += shift;
            if (d.off_hj >= 0) d.off_hj += shift;
            if (d.off_snap >= 0) d.off_snap += shift;
            if (d.off_snap_abs >= 0) d.off_snap_abs += shift;
            if (d.off_dispx >= 0) d.off_dispx += shift;
            if (d.off_region >= 0) d.off_region += shift;
            if (d.off_field >= 0) d.off_field += shift;
            d.base = base;
            d.n = n;
            d.pid0 = r->jh.dev.pid0 + r->cursor;
            d.stat_slot = (int32_t)devs.size();
            d.times_off = (int32_t)times.size();
            times.insert(times.end(), r->jh.times.begin(), r->jh.times.end());
            base += n;
            devs.push_back(d);
            members.push_back(r);
        }
        // the member with the fewest flights left starts particles if any has some
        // left, and a member with none left has particles suspended (else it was
        // complete and collected from the active set)
        if (members.empty()) return fail(DMC_E_DEVICE, "internal: an epoch without work");
        // particles suspended last epoch resume first; their slots map to this
        // epoch's job table (jobs are queued in member order, so index = member)
        S->h_resume_job.assign((size_t)S->opts.max_active, 0);
        const std::vector<Request *> &pm = S->prev_members[cls];
        std::vector<const void *> prev_keys(pm.begin(), pm.end()), keys(members.begin(), members.end());
        if (!sched::resume_map(prev_keys.data(), S->prev_suspended[cls].data(), pm.size(), keys.data(), keys.size(),
                               S->h_resume_job.data(), S->h_resume_job.size()))
            return fail(DMC_E_DEVICE, "internal: a request with suspended particles left the epoch");
    }
    DMC_HIP_OR_FAIL(hipMemcpyAsync(S->d_resume_job, S->h_resume_job.data(), S->h_resume_job.size() * sizeof(int32_t),
                                   hipMemcpyHostToDevice, s));
    // while requests still have unstarted particles, epochs stay short so new
    // arrivals join quickly; once only continuations remain, they run longer
    bool fresh = false;
    for (size_t i = 0; i < members.size(); ++i) fresh = fresh || devs[i].n > 0;
    const uint32_t drain = S->opts.drain_flights ? S->opts.drain_flights : 2048u;
    lb.drain_iters = fresh ? drain : 16u * drain;
    lb.n_resume = S->n_rest[cls];
    lb.resume_in = S->rest[cls];  // NULL only while the group has never suspended (n_resume = 0)
    lb.resume_job = S->d_resume_job;
    lb.suspend_out = S->spare;
    lb.suspend_cap = S->susp_cap;
    dmc_status st = enqueue_launch(S->M, devs, times, S->epoch_table, lb, 0, false, S->opts.run, s, S->ev0, S->ev1);
    if (st != DMC_OK) return st;
    DMC_HIP_OR_FAIL(hipEventSynchronize(S->ev1));
    float ms = 0.0f;
    DMC_HIP_OR_FAIL(hipEventElapsedTime(&ms, S->ev0, S->ev1));
    std::vector<unsigned long long> stats(members.size() * kStats);
    DMC_HIP_OR_FAIL(hipMemcpy(stats.data(), S->sb.stats, stats.size() * 8, hipMemcpyDeviceToHost));
    int32_t finished = 0;
    std::lock_guard<std::mutex> g(S->mu);
    uint64_t n_susp = 0;
    for (size_t i = 0; i < members.size(); ++i) {
        Request *r = members[i];
        for (int k = 0; k < kStats; ++k)
            if (k != 5) r->stats[k] += stats[i * kStats + k];  // slot 5 counts this epoch's suspensions
        r->suspended = stats[i * kStats + 5];
        n_susp += r->suspended;
        r->kernel_ms += ms;
        r->cursor += devs[i].n;
    }
    S->n_rest[cls] = (uint32_t)n_susp;
    for (size_t i = 0; i < members.size(); ++i) {
        S->totals.particles += stats[i * kStats + 0];
        S->totals.scatters += stats[i * kStats + 1];
        S->totals.boundary += stats[i * kStats + 2];
        S->totals.iterations += stats[i * kStats + 3];
        S->totals.capped += stats[i * kStats + 4];
        S->totals.flights += stats[i * kStats + 6];
    }
    S->totals.kernel_ms += ms;
    std::swap(S->rest[cls], S->spare);  // the group's particles now wait in what was the spare
    S->prev_members[cls] = members;
    S->prev_suspended[cls].resize(members.size());
    for (size_t i = 0; i < members.size(); ++i) S->prev_suspended[cls][i] = members[i]->suspended;
    for (size_t i = 0; i < S->active.size();) {
        Request *r = S->active[i].get();
        if (r->cursor >= r->jh.dev.n && r->suspended == 0) {
            r->host_tally.assign((size_t)std::max<int64_t>(r->jh.size, 1), 0.0);
            DMC_HIP_OR_FAIL(hipMemcpy(r->host_tally.data(), (char *)S->arena_mem + r->arena_off,
                                      (size_t)r->jh.size * sizeof(double), hipMemcpyDeviceToHost));
            complete_tally(r->jh.dev, r->host_tally.data());
            S->arena->release(r->arena_off);
            S->done[r->ticket] = std::move(S->active[i]);
            S->active.erase(S->active.begin() + (long)i);
            ++finished;
        } else {
            ++i;
        }
    }
    if (n_done) *n_done = finished;
    return DMC_OK;
}

extern "C" dmc_status dmc_server_poll(dmc_server *S, uint64_t ticket, int32_t *done)
{
    if (!S || !done) return fail(DMC_E_INVALID, "NULL argument");
    std::lock_guard<std::mutex> g(S->mu);
    *done = S->done.count(ticket) ? 1 : 0;
    if (*done) return DMC_OK;
    for (auto &r : S->active)
        if (r->ticket == ticket) return DMC_OK;
    for (auto &r : S->pending)
        if (r->ticket == ticket) return DMC_OK;
    return fail(DMC_E_INVALID, "unknown ticket");
}

extern "C" dmc_status dmc_server_wait(dmc_server *S, uint64_t ticket, int32_t *n_epochs)
{
    if (n_epochs) *n_epochs = 0;
    for (;;) {
        int32_t done = 0;
        dmc_status st = dmc_server_poll(S, ticket, &done);
        if (st != DMC_OK || done) return st;
        // the request is queued or running: every epoch admits what fits (a
        // request is only accepted if it fits alone) and starts particles of
        // at least the admitted request with the fewest flights left, so with
        // no new submissions every request ahead of this one, and it, complete
        if ((st = dmc_server_step(S, nullptr)) != DMC_OK) return st;
        if (n_epochs) ++*n_epochs;
    }
}

extern "C" dmc_status dmc_server_collect(dmc_server *S, uint64_t ticket, dmc_result **out)
{
    if (!S || !out) return fail(DMC_E_INVALID, "NULL argument");
    *out = nullptr;
    std::unique_ptr<Request> r;
    {
        std::lock_guard<std::mutex> g(S->mu);
        auto it = S->done.find(ticket);
        if (it == S->done.end()) return fail(DMC_E_INVALID, "request not complete (or unknown ticket)");
        r = std::move(it->second);
        S->done.erase(it);
    }
    std::unique_ptr<dmc_result> R(new (std::nothrow) dmc_result());
    if (!R) return fail(DMC_E_NOMEM, "host allocation failed");
    R->mat = S->M;
    R->jobs.push_back(r->jh);
    R->tally_doubles = (size_t)r->jh.size;
    R->h_tally = std::move(r->host_tally);
    R->h_stats.assign(r->stats, r->stats + kStats);
    R->kernel_ms = r->kernel_ms;
    R->synced = true;
    *out = R.release();
    return DMC_OK;
}

extern "C" dmc_status dmc_server_load(const dmc_server *cs, int32_t *queued, int32_t *running)
{
    dmc_server *S = const_cast<dmc_server *>(cs);
    if (!S) return fail(DMC_E_INVALID, "server is NULL");
    std::lock_guard<std::mutex> g(S->mu);
    if (queued) *queued = (int32_t)S->pending.size();
    if (running) *running = (int32_t)S->active.size();
    return DMC_OK;
}

extern "C" dmc_status dmc_server_totals(const dmc_server *cs, dmc_stats *out)
{
    dmc_server *S = const_cast<dmc_server *>(cs);
    if (!S || !out) return fail(DMC_E_INVALID, "server / out is NULL");
    std::lock_guard<std::mutex> g(S->mu);
    *out = S->totals;
    return DMC_OK;
}

extern "C" dmc_status dmc_server_destroy(dmc_server *S)
{
    if (S && S->opts.run.stream) (void)hipStreamSynchronize((hipStream_t)S->opts.run.stream);
    else if (S) (void)hipDeviceSynchronize();
    delete S;
    return DMC_OK;
}
