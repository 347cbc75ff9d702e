// dmc_tune.cpp -- planning helpers: the autotuner of the persistent form's
// launch parameters, and truncation planning for periodic problems.
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

    Choice cur;  // start: block 0 (sized from the LDS the batch needs), chunk 1024, refill at 4 free lanes
    cur.block = 0;
    cur.chunk = 1024;
    cur.refill_min = 4;
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

// ------------------------------------------------------ truncation planning ----

namespace {

// One pilot: H_j and its standard error (j < kp), kappa and its standard error.
dmc_status run_pilot(const dmc_job &job, const dmc_run_opts &o, uint64_t n_pilot, int32_t kp, std::vector<double> &hj,
                     std::vector<double> &hse, double &kap, double &kse)
{
    dmc_job pj = job;  // the next n_pilot particle ids of the same realisation
    pj.first_particle = job.first_particle + job.n_particles;
    pj.n_particles = n_pilot;
    pj.tally.kmax = kp;
    pj.tally.n_hj = kp;
    pj.tally.first_event = 0;
    std::vector<JobHost> jh;
    dmc_status st = gather_jobs(&pj, 1, jh);
    if (st != DMC_OK) return st;
    dmc_result *r = nullptr;
    if ((st = launch(jh, o, &r)) != DMC_OK) return st;
    hj.assign(kp, 0.0);
    hse.assign(kp, 0.0);
    st = dmc_tally_read(r, 0, DMC_Q_HJ, 0, hj.data(), hse.data(), (size_t)kp);
    if (st == DMC_OK) st = dmc_tally_read(r, 0, DMC_Q_KAPPA, 0, &kap, &kse, 1);
    dmc_result_destroy(r);
    return st;
}

}  // namespace

extern "C" dmc_status dmc_plan_truncation(const dmc_job *job, const dmc_run_opts *opts, const dmc_trunc_opts *t,
                                          dmc_trunc_plan *out)
{
    if (!job || !out) return fail(DMC_E_INVALID, "job / out is NULL");
    *out = dmc_trunc_plan{};
    if (job->source.kind != DMC_SRC_GRADIENT) return fail(DMC_E_INVALID, "truncation planning needs a gradient source");
    dmc_run_opts o;
    if (opts)
        o = *opts;
    else
        dmc_run_opts_default(&o);
    o.workspace = nullptr;
    o.workspace_bytes = 0;
    o.nscat_out = nullptr;
    dmc_status st = run_opts_check(o);
    if (st != DMC_OK) return st;
    const uint64_t N = job->n_particles;
    const bool fixed = t && t->n_pilot;
    uint64_t n_pilot = fixed ? t->n_pilot : std::min<uint64_t>(N, 1000000);
    const int32_t kp = (t && t->k_pilot) ? t->k_pilot : 200;
    const double frac = (t && t->bias_fraction > 0.0) ? t->bias_fraction : 0.2;
    if (n_pilot < 2 || kp < 3 || kp > kMaxHj) return fail(DMC_E_INVALID, "n_pilot >= 2 and 3 <= k_pilot <= 1024");
    if (N < 1 || job->first_particle + N + (fixed ? n_pilot : std::max<uint64_t>(n_pilot, 10000000)) <
                     job->first_particle)
        return fail(DMC_E_INVALID, "particle ids overflow");

    // The run of significant events j = 1, 2, ..., n: |<H_j>| above 4 pilot
    // standard errors; the first insignificant event ends it, so chance
    // excursions further out do not count.  A pilot that resolves fewer than 3
    // is grown tenfold (to at most min(N, 1e7) particles) unless its size was given.
    std::vector<double> hj, hse;
    double kap = 0.0, kse = 0.0;
    int n = 0;
    for (;;) {
        if ((st = run_pilot(*job, o, n_pilot, kp, hj, hse, kap, kse)) != DMC_OK) return st;
        n = 0;
        while (n + 1 < kp && std::fabs(hj[n + 1]) > 4.0 * hse[n + 1]) ++n;
        const uint64_t cap = std::min<uint64_t>(N, 10000000);
        if (fixed || n >= 3 || n_pilot >= cap) break;
        n_pilot = std::min<uint64_t>(cap, n_pilot * 10);
    }
    out->n_fit = n;
    out->n_pilot = n_pilot;

    // standard errors of the job itself scale as 1/sqrt(N)
    const double scale = std::sqrt((double)n_pilot / (double)N);
    out->kappa_pilot = kap;
    out->kappa_se = kse * scale;
    out->k_uncertain = kp;
    for (int j = 1; j < kp; ++j)
        if (std::fabs(hj[j]) <= hse[j] * scale) {
            out->k_uncertain = j;
            break;
        }
    if (n == 0) {
        // nothing after the first event is distinguishable from zero at the
        // pilot's size (exactly zero in expectation for films): the pilot's
        // signed sum beyond the first event is the estimate of what is cut
        out->kmax = 1;
        out->fit_ok = 1;
        double tail = 0.0;
        for (int j = 1; j < kp; ++j) tail += hj[j];
        out->bias_bound = std::fabs(tail);
        return DMC_OK;
    }
    // Exponential tail |<H_j>| ~ A r^j after the first free path (j = 0 is not
    // part of the decay): n >= 3, a log-linear fit weighted by (|<H_j>| / se_j)^2,
    // the inverse variance of ln|<H_j>|; n = 2, the ratio of the two events;
    // n = 1, the upper bound 4 se_2 / |<H_1>| on the first step into the noise.
    double rr = 0.0, A = 0.0;
    if (n >= 3) {
        double sw = 0, sx = 0, sy = 0, sxx = 0, sxy = 0;
        for (int j = 1; j <= n; ++j) {
            const double h = std::fabs(hj[j]);
            const double w = (hse[j] > 0.0) ? (h / hse[j]) * (h / hse[j]) : 1.0;
            const double y = std::log(h);
            sw += w;
            sx += w * j;
            sy += w * y;
            sxx += w * (double)j * j;
            sxy += w * j * y;
        }
        const double den = sw * sxx - sx * sx;
        if (den > 0.0) {
            const double slope = (sw * sxy - sx * sy) / den;
            rr = std::exp(slope);
            A = std::exp((sy - slope * sx) / sw);
        } else {
            rr = 1.0;
        }
    } else {
        rr = (n == 2) ? std::fabs(hj[2]) / std::fabs(hj[1]) : 4.0 * hse[2] / std::fabs(hj[1]);
        A = std::fabs(hj[n]) / std::pow(rr, n);
    }
    if (!(rr < 1.0) || !(rr > 0.0)) {
        // no decay resolved: the paper's empirical criterion, and the pilot's own
        // signed sum beyond it as the estimate of what is cut
        out->kmax = std::min(kp, std::max(n + 1, out->k_uncertain));
        out->fit_ok = 0;
        double tail = 0.0;
        for (int j = out->kmax; j < kp; ++j) tail += hj[j];
        out->bias_bound = std::fabs(tail);
        return DMC_OK;
    }
    const double target = frac * out->kappa_se;
    // smallest K > n with A r^K / (1 - r) <= target
    double K = std::ceil(std::log(target * (1.0 - rr) / A) / std::log(rr));
    if (!(K >= n + 1)) K = n + 1;
    out->kmax = (int32_t)std::min<double>(K, (double)kp);
    out->fit_ok = 1;
    out->decay = rr;
    out->amplitude = A;
    out->bias_bound = A * std::pow(rr, out->kmax) / (1.0 - rr);
    return DMC_OK;
}
