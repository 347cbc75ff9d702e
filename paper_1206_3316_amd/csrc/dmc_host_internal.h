// Host-side internals shared by dmc_host.cpp and dmc_server.cpp.
#pragma once

#include <hip/hip_runtime.h>

#include <functional>
#include <string>
#include <vector>

#include "../../include/dmc.h"
#include "dmc_internal.h"

namespace dmc {

dmc_status fail(dmc_status code, const std::string &msg);

#define DMC_HIP_OR_FAIL(expr)                                                                                   \
    do {                                                                                                        \
        hipError_t e_ = (expr);                                                                                 \
        if (e_ != hipSuccess) return ::dmc::fail(DMC_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

struct AliasTable {
    int bits = 0;
    std::vector<uint64_t> mass;    // integer masses, sum 2^32
    std::vector<uint32_t> thresh;  // canonical thresholds (a full column holds 2^(32-bits))
    std::vector<uint32_t> alias;
    std::vector<uint32_t> packed;  // device form (pack_alias)
};

bool build_alias(const std::vector<double> &w, AliasTable &t, std::string &why);

// A job of a launch: the caller's description plus its normalisation and its
// device descriptor (offsets relative to the launch's tally base).
struct JobHost {
    dmc_job job{};
    std::vector<double> times;
    dmc_geometry_desc geom{};
    double power = 0.0;       // steady: source power per unit area (slab, film) or length (cell); transient: energy
    double avg_volume = 1.0;  // mu(R) of the conductivity average
    int64_t size = 0;         // doubles of its tally block
    int64_t hidden = 0;       // trailing doubles of the block that a caller does not read
    JobDev dev{};
};

// Normalisation and tally size of a job, as prepare_job_core computes them.
struct JobMeta {
    double power = 0.0;
    double avg_volume = 1.0;
    int64_t size = 0;
    int64_t hidden = 0;
};

dmc_status prepare_job(const dmc_job &jb, JobHost &h);
// Validates a job and fills its device descriptor (offsets relative to the job's
// block) and normalisation, without allocating.
dmc_status prepare_job_core(const dmc_job &jb, JobDev &d, JobMeta &meta);
// Host-side completion of a job's tally block after the copy from the device
// (offsets of d relative to block): fills the sections the device skips.
void complete_tally(const JobDev &d, double *block);
dmc_status run_opts_check(const dmc_run_opts &o);

// Device regions a launch uses besides the material tables.
struct LaunchBuffers {
    JobDev *jobs = nullptr;           // n_jobs descriptors
    double *times = nullptr;          // concatenated snapshot times
    double *tally = nullptr;          // tally base (job offsets are relative to it)
    unsigned long long *stats = nullptr;  // n_jobs * kStats counters
    unsigned long long *queue = nullptr;  // 2 words
    // time-bounded launches (server epochs)
    uint32_t drain_iters = 0;
    uint32_t n_resume = 0;
    const Suspended *resume_in = nullptr;
    const int32_t *resume_job = nullptr;
    Suspended *suspend_out = nullptr;
    uint32_t suspend_cap = 0;
    // autotuner trials stop trajectories early so that a sample measures the
    // bulk rate rather than its longest particle; 0 = the safety cap
    uint32_t iter_cap = 0;
};

// Launch geometry of a batch: kernel specialisation, arguments (LDS plan,
// chunk, refill threshold), workgroup size and count.
struct LaunchPlan {
    KArgs a{};
    const struct ::dmc_material *material = nullptr;
    int spec = 0, block = 0, grid = 0;
    size_t lds_bytes = 0;
};

// The kernel specialisation for a launch of these jobs of material M.
int launch_spec(const struct ::dmc_material *M, const JobDev *devs, int n_jobs);
// Chooses the kernel and plans LDS privatisation and occupancy for devs (whose
// LDS offsets it sets); host work only, no allocation.
dmc_status plan_launch(const struct ::dmc_material *M, JobDev *devs, int n_jobs, const LaunchBuffers &b,
                       const dmc_run_opts &o, LaunchPlan &plan);
// Enqueues the trajectory launch(es) of a plan on stream s.
dmc_status submit_launch(const LaunchPlan &plan, const JobDev *devs, int n_jobs, const dmc_run_opts &o, hipStream_t s);
// Launch order of jobs: descending expected flights per particle, or the flights
// of a gradient job's longest likely trajectory where that is larger (ties:
// caller's order).  length: slab / film / cell size per job; t_final: last
// snapshot time (transient jobs).  rank[r] = job index; key: scratch of n_jobs.
// No allocation.
void queue_order(const struct ::dmc_material &M, const JobDev *devs, const double *length, const double *t_final,
                 int n_jobs, int *rank, double *key);
// Queue bases in rank order, and tally / time / per-particle-output offsets in
// job order (size: doubles of each job's tally block, n_times: its snapshot
// times).  No allocation.
void assign_offsets(JobDev *devs, const int64_t *size, const int32_t *n_times, const int *rank, int n_jobs);

// Plans LDS privatisation and occupancy, uploads the descriptors, clears the
// counters (and the tallies if zero_tally), records ev0, enqueues the
// trajectory launch(es) and records ev1, all on `stream`.  `devs` receives the
// LDS offsets chosen.
// `table` receives the host copy of the uploaded descriptor table; it and
// `times` must stay alive until the launch has completed (asynchronous copies).
dmc_status enqueue_launch(const struct ::dmc_material *M, std::vector<JobDev> &devs, const std::vector<double> &times,
                          std::vector<JobDev> &table, const LaunchBuffers &b, size_t tally_doubles, bool zero_tally,
                          const dmc_run_opts &o, hipStream_t stream, hipEvent_t ev0, hipEvent_t ev1);

// Validates a batch and prepares its jobs (queue order, tally offsets).
dmc_status gather_jobs(const dmc_job *jobs, int32_t n_jobs, std::vector<JobHost> &jh);
// Expected flights per particle of a prepared job (queue order, tuner sample sizes).
double flights_per_particle(const struct ::dmc_material &M, const JobHost &h);
// Device bytes a batch needs (descriptors, times, tallies, counters, queue).
size_t workspace_bytes(const std::vector<JobHost> &jh);
// Enqueues a batch (consumes jh) and returns its result handle.
dmc_status launch(std::vector<JobHost> &jh, const dmc_run_opts &o, ::dmc_result **out, uint32_t iter_cap = 0);
// Waits for a result and copies its tallies and counters to the host.
dmc_status sync_result(::dmc_result *R);

}  // namespace dmc

struct dmc_material {
    int32_t K = 0;
    double T_eq = 0.0;
    std::vector<double> v, tau, C;
    std::vector<double> lam_desc, cv_cum;  // free paths, descending, and the running sum of C v
    double C_tot = 0.0, G_tau = 0.0, G_v = 0.0;
    double scatter_g = 0.0;  // mean cosine of the scattering angle (Henyey-Greenstein); 0: isotropic
    dmc::AliasTable gain, init, flux;
    uint32_t *d_gain = nullptr, *d_init = nullptr, *d_flux = nullptr;
    float4 *d_st32 = nullptr;
    double2 *d_st64 = nullptr;
    int device = 0;
    ~dmc_material();
};

struct dmc_geometry {
    dmc_geometry_desc d;
};

struct dmc_result {
    const dmc_material *mat = nullptr;
    std::vector<dmc::JobHost> jobs;
    void *dev_mem = nullptr;          // device allocation owned by this result (hipFree on destroy)
    std::function<void()> on_destroy; // releases memory owned elsewhere (server arena)
    double *d_tally = nullptr;
    unsigned long long *d_stats = nullptr;
    size_t tally_doubles = 0;
    hipStream_t stream = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    bool synced = false;
    std::vector<double> h_tally;
    std::vector<unsigned long long> h_stats;
    std::vector<dmc::JobDev> h_table;  // upload sources, alive until the launch completes
    std::vector<double> h_times;
    double kernel_ms = 0.0;
    ~dmc_result();
};
