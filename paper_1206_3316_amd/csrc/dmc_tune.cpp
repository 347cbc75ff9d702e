// dmc_tune.cpp -- autotuner of the persistent form's launch parameters.
//
// A batch's throughput depends on the block size (waves per CU against LDS
// per workgroup), the queue chunk (queue atomics against lanes left idle at the
// end of a chunk), the refill threshold (divergence against refill cost) and
// whether tallies are privatised in LDS.  None of them changes an estimate, so
// they are picked by timing: trial launches of a sample of the batch, searched
// one parameter at a time, cached per batch signature.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "dmc_host_internal.h"

using namespace dmc;

namespace {

struct Choice {
    int32_t block = 0, chunk = 0, refill_min = 0, lds_tally = 1;
};

std::mutex g_cache_mu;
std::map<std::string, Choice> g_cache;

// Signature of a batch: what decides the trajectory mix and the tally layout.
std::string signature(const std::vector<JobHost> &jh, const dmc_run_opts &o)
{
    std::string s;
    char buf[256];
    std::snprintf(buf, sizeof(buf), "%p|%d|%d|", (const void *)jh[0].job.material, o.precision, (int)jh.size());
    s += buf;
    for (const auto &h : jh) {
        const auto &g = h.geom;
        const auto &t = h.job.tally;
        std::snprintf(buf, sizeof(buf), "%d:%.6g:%.6g:%d%d:%.3g%.3g:%d:%d:%d:%d:%d:%d%d%d:%d;", g.kind, g.length,
                      g.radius, g.wall[0].type, g.wall[1].type, g.wall[0].specularity, g.wall[1].specularity,
                      h.job.source.kind, t.n_bins, t.n_batches, t.kmax, t.n_hj, t.grid[0], t.grid[1], t.grid[2],
                      (int)std::lround(std::log2((double)h.job.n_particles)));
        s += buf;
    }
    return s;
}

struct Trial {
    std::vector<dmc_job> jobs;  // the sample
    dmc_run_opts base{};
    uint32_t cap = 0;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    uint64_t flights = 0;

    // Times one launch of the sample with the given parameters (kernel time in ms).
    dmc_status run(const Choice &c, double &ms)
    {
        dmc_run_opts o = base;
        o.block = c.block;
        o.chunk = c.chunk;
        o.refill_min = c.refill_min;
        o.lds_tally = c.lds_tally;
        o.grid_blocks = 0;
        o.workspace = ws;
        o.workspace_bytes = ws_bytes;
        o.nscat_out = nullptr;
        std::vector<JobHost> jh;
        dmc_status st = gather_jobs(jobs.data(), (int32_t)jobs.size(), jh);
        if (st != DMC_OK) return st;
        dmc_result *r = nullptr;
        if ((st = launch(jh, o, &r, cap)) != DMC_OK) return st;
        st = sync_result(r);
        ms = r->kernel_ms;
        flights = 0;
        for (size_t j = 0; j < r->jobs.size(); ++j) flights += r->h_stats[j * kStats + 3];
        delete r;
        return st;
    }
};

}  // namespace

extern "C" dmc_status dmc_autotune(const dmc_job *jobs, int32_t n_jobs, const dmc_run_opts *base, dmc_tune_opts *tune,
                                   dmc_run_opts *best)
{
    if (!best) return fail(DMC_E_INVALID, "best is NULL");
    dmc_run_opts o;
    if (base)
        o = *base;
    else
        dmc_run_opts_default(&o);
    dmc_status st = run_opts_check(o);
    if (st != DMC_OK) return st;
    dmc_tune_opts dflt{};
    dflt.use_cache = 1;
    dmc_tune_opts &t = tune ? *tune : dflt;
    t.n_trials = 0;
    t.from_cache = 0;
    *best = o;
    best->grid_blocks = 0;
    std::vector<JobHost> jh;
    if ((st = gather_jobs(jobs, n_jobs, jh)) != DMC_OK) return st;
    if (o.form != DMC_FORM_PERSISTENT) return DMC_OK;

    const std::string key = signature(jh, o);
    if (t.use_cache) {
        std::lock_guard<std::mutex> g(g_cache_mu);
        auto it = g_cache.find(key);
        if (it != g_cache.end()) {
            best->block = it->second.block;
            best->chunk = it->second.chunk;
            best->refill_min = it->second.refill_min;
            best->lds_tally = it->second.lds_tally;
            t.from_cache = 1;
            return DMC_OK;
        }
    }

    // sample: the first particles of every job, a common fraction of each, so
    // that a trial runs about sample_flights flights
    const uint32_t cap = t.trial_cap ? t.trial_cap : 4096u;
    const double target = t.sample_flights ? (double)t.sample_flights : 5e10;
    const dmc_material &M = *jobs[0].material;
    double total = 0.0;
    for (const auto &h : jh) total += (double)h.job.n_particles * std::min(flights_per_particle(M, h), (double)cap);
    const double frac = std::min(1.0, target / std::max(total, 1.0));
    auto sample = [&](double f) {
        std::vector<dmc_job> s;
        for (const auto &h : jh) {
            dmc_job j = h.job;
            const uint64_t n = j.n_particles;
            uint64_t m = (uint64_t)std::ceil((double)n * f);
            m = std::max<uint64_t>(m, std::min<uint64_t>(n, 512));
            j.n_particles = std::min(m, n);
            s.push_back(j);
        }
        return s;
    };
    Trial tr, pilot;
    tr.base = pilot.base = o;
    tr.cap = pilot.cap = cap;
    tr.jobs = sample(frac);
    pilot.jobs = sample(frac / 16.0);
    {
        std::vector<JobHost> sj;
        if ((st = gather_jobs(tr.jobs.data(), (int32_t)tr.jobs.size(), sj)) != DMC_OK) return st;
        tr.ws_bytes = pilot.ws_bytes = workspace_bytes(sj);
    }
    if (hipMalloc(&tr.ws, tr.ws_bytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(DMC_E_NOMEM, "autotune: sample workspace allocation failed");
    }
    pilot.ws = tr.ws;

    auto record = [&](const Choice &c, double ms, const Trial &x, int is_pilot) {
        if (t.trials && t.n_trials < t.max_trials) {
            dmc_tune_trial &r = t.trials[t.n_trials];
            r.block = c.block;
            r.chunk = c.chunk;
            r.refill_min = c.refill_min;
            r.lds_tally = c.lds_tally;
            r.pilot = is_pilot;
            r.ms = ms;
            r.flights_per_s = ms > 0.0 ? (double)x.flights / (ms * 1e-3) : 0.0;
        }
        ++t.n_trials;
    };

    Choice cur;  // the planner's defaults (block 0: sized from the LDS the batch needs)
    cur.block = 0;
    cur.chunk = 1024;
    cur.refill_min = 16;
    cur.lds_tally = o.lds_tally;
    double cur_ms = 0.0;
    // the first launch loads the code object and sets LDS attributes: not timed
    if ((st = tr.run(cur, cur_ms)) == DMC_OK) st = tr.run(cur, cur_ms);
    if (st == DMC_OK) record(cur, cur_ms, tr, 0);

    struct Axis {
        int32_t Choice::*field;
        std::vector<int32_t> values;
    };
    const std::vector<Axis> axes = {
        {&Choice::lds_tally, {1, 0}},
        {&Choice::block, {256, 512, 1024}},
        {&Choice::chunk, {256, 1024, 4096}},
        {&Choice::refill_min, {1, 4, 16, 32}},
    };
    for (const auto &ax : axes) {
        if (st != DMC_OK) break;
        for (int32_t v : ax.values) {
            if (cur.*(ax.field) == v) continue;
            Choice c = cur;
            c.*(ax.field) = v;
            double ms = 0.0;
            if (c.lds_tally == 0 && cur.lds_tally != 0) {
                // unprivatised tallies can serialise on contended FP64 atomics
                // (a few conductivity sums shared by every particle) and run
                // orders of magnitude slower: screen them on 1/16 of the sample
                st = pilot.run(c, ms);
                if (st == DMC_E_DEVICE) break;
                if (st == DMC_OK) record(c, ms, pilot, 1);
                if (st != DMC_OK || ms > cur_ms) {
                    st = DMC_OK;
                    continue;
                }
            }
            st = tr.run(c, ms);
            if (st == DMC_E_DEVICE) break;
            if (st != DMC_OK) {  // a candidate the planner rejects is skipped
                st = DMC_OK;
                continue;
            }
            record(c, ms, tr, 0);
            if (ms < 0.98 * cur_ms) {
                cur = c;
                cur_ms = ms;
            }
        }
    }
    (void)hipFree(tr.ws);
    if (st != DMC_OK) return st;
    best->block = cur.block;
    best->chunk = cur.chunk;
    best->refill_min = cur.refill_min;
    best->lds_tally = cur.lds_tally;
    {
        std::lock_guard<std::mutex> g(g_cache_mu);
        g_cache[key] = cur;
    }
    return DMC_OK;
}
