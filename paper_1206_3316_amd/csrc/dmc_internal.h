// Internal layout shared by the library's host code and its HIP kernels.
// Nothing here is part of the public C ABI (include/dmc.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dmc {

constexpr uint32_t kIterCap = 1u << 24;  // safety cap on flights per particle
constexpr int kPosAttempts = 64;         // rejection attempts for positions in a pore cell
constexpr int kMaxJobs = 4096;
constexpr int kMaxBins = 4096;
constexpr int kMaxTimes = 1024;
constexpr int kMaxHj = 1024;
constexpr int kLdsJobsBytes = 48 * 1024;  // job table staged in LDS by the persistent kernels, at most
constexpr int kLdsTimes = 2048;           // sample times staged with it, at most
constexpr int kLdsStatJobs = 64;         // per-job counters privatised in LDS up to this many jobs
constexpr int kStats = 7;                // particles, scatters, boundary, iterations, capped, suspended,
                                         // flights (Philox STEP blocks drawn)

enum Geom : int32_t { GEOM_SLAB = 0, GEOM_FILM = 1, GEOM_PORE = 2, GEOM_HALF = 3, GEOM_GRAD = 8, GEOM_ANY = 9 };
// GEOM_GRAD and GEOM_ANY only select kernel specialisations (see kernel_spec).
enum Wall : int32_t { WALL_ISOTHERMAL = 0, WALL_ADIABATIC = 1, WALL_PERIODIC = 2 };
enum Src : int32_t { SRC_WALLS = 0, SRC_GAUSSIAN = 1, SRC_GRADIENT = 2 };
// FORM_EPOCH: the persistent form in time-bounded launches (serving epochs),
// whose particles may be suspended and resumed in a later launch.
enum Form : int32_t { FORM_PLAIN = 0, FORM_PERSISTENT = 1, FORM_EPOCH = 2 };
enum Tag : uint32_t { TAG_STEP = 0, TAG_EMIT_A = 1, TAG_EMIT_B = 2 };
constexpr int32_t kNoSurface = -1;

// One simulation inside a launch.  Particle pid of the job has queue index base + pid.
struct alignas(16) JobDev {
    uint64_t base, n;       // queue range [base, base + n) of this launch
    uint64_t pid0;          // pid of the range's first particle (a slice of a longer job)
    uint32_t key0, key1;
    int32_t geom, src;
    double length, radius;
    int32_t wall_type[2];
    uint64_t spec_thr[2];   // specular iff the word is below this (p = 1 gives 2^32)
    int32_t n_src;          // wall sources (1 or 2)
    int32_t src_wall[2];
    uint32_t src_packed[2]; // alias table of the two wall-source powers (1 index bit)
    double wall_sign[2];    // sign of particles emitted by each wall
    double sign0;           // gaussian: sign(dT); gradient: -sign(dT/dz)
    double sigma;           // gaussian: radius / sqrt(2)
    // tallies: offsets are in doubles from the launch's tally base / the LDS tally base
    int32_t n_bins, n_batches;
    double bins_per_len, bin_width;
    int64_t off_bins, off_kappa, off_hj, off_snap, off_snap_abs;
    int32_t lds_bins, lds_kappa, lds_hj;  // -1: accumulate in global memory
    int32_t kmax, n_hj;
    int32_t n_times, times_off;
    int32_t grid[3], pad0;
    double grid_lo[3], grid_ext[3];  // lower bound and extent hi - lo
    float grid_lof[3], grid_scf[3];  // FP32 lower bound and cells per metre (production form)
    int64_t ncell;
    int32_t stat_slot;      // index of this job's counters (the caller's job index)
    int32_t snap_abs_on;    // 0: every particle has the same sign, the host derives sum|s| = |sum s|
    uint64_t out_off;       // per-particle outputs of pid are at out_off + pid - pid0 (caller's job order)
    int64_t off_dispx;      // bins: per-batch net transmissions (s per particle), expanded by the host
    int32_t lds_dispx;      // -1: in global memory
    int32_t disp_tel;       // 1: the displacement is telescoped (persistent slab kernel)
    int32_t first_event;    // 1: a diffuse wall reflection (or the first scattering event) ends the particle
    int32_t lds_region;     // -1: in global memory
    int64_t off_region;     // windowed region tally [n_times][4]: sum v_T, v_T^2, v_Q, v_Q^2 (-1: none)
    double region_c[2], region_r, region_z[2];
    int64_t off_field;      // steady pore-cell field [batch][TIME, DISPZ][nz][nx] (-1: none)
    int32_t lds_field;      // -1: accumulated in global memory
    int32_t pad_field;
};

// A particle suspended at the end of a time-bounded launch (serving epochs):
// everything needed to continue its trajectory bit for bit in a later launch.
struct alignas(16) Suspended {
    double x, y, z, ox, oy, oz;
    double t, Lz, h;
    uint64_t pid;
    uint32_t k, nscat, nbound, m;
    int32_t last, tcur, slot, sign;
    double rt, rq;          // region tally sums of the current window
    int32_t rwin;
    uint32_t nseg;          // segments so far
    double rem;             // free-flight time left after a periodic face (< 0: none)
};
static_assert(sizeof(Suspended) == 144, "Suspended layout");

struct KArgs {
    const JobDev *jobs;
    int32_t n_jobs;
    int32_t K;
    uint64_t qbegin;                // plain form: first queue index of this launch
    uint64_t total;                 // one past the last queue index of this launch
    unsigned long long *queue;      // next queue index (persistent form)
    int32_t gain_bits, flux_bits, init_bits;
    int32_t any_region;             // 1: some job of the launch has a windowed region tally
    int32_t times_lds;              // doubles of times staged in LDS (with the job table), else 0
    int32_t jobs_lds;               // 1: the job table and the times are staged in LDS (persistent launches where both fit)
    const uint32_t *gain_packed, *flux_packed, *init_packed;
    const float4 *st32;             // per state: v, tau, 1/tau, 0
    const double2 *st64;            // per state: v, tau
    double *tally;
    const double *times;
    uint32_t *nscat_out;            // optional, indexed by JobDev::out_off + pid
    unsigned long long *stats;      // [n_jobs][kStats]
    int32_t chunk, refill_min;
    int32_t lds_tally_doubles;      // LDS tally size; 0 = none
    int32_t lds_stats;              // 1: per-job counters in LDS
    int32_t kpad;                   // 2^gain_bits
    int32_t bins_lds_all;           // 1: every job's bins are privatised in LDS
    // time-bounded launches (persistent form): queue indices [0, n_resume) resume
    // suspended particles; a wave that finds the queue empty runs at most
    // drain_iters more flights, then suspends its live particles
    uint32_t drain_iters;           // 0: run every particle to completion
    uint32_t n_resume;
    const Suspended *resume_in;
    const int32_t *resume_job;      // device-table job of each resumed particle's slot
    Suspended *suspend_out;
    uint32_t suspend_cap;
    uint32_t iter_cap;              // segments after which a particle is stopped and counted as capped
    // scattering direction (step IVb): g = 0 isotropic; else Henyey-Greenstein of mean
    // cosine g, mu = (hg[3] - f^2) / hg[2] with f = hg[0] / (hg[1] + hg[2] u):
    // hg = {1 - g^2, 1 - g, 2 g, 1 + g^2} (FP64 and FP32 copies, and 1 / (2 g))
    double scatter_g;
    double hg[4];
    float hgf[4], hgf_inv2g;
    uint32_t prio_flights;          // persistent: waves holding a particle past this many flights (4x,
                                    // 16x) get SIMD issue priority 1 (2, 3); 0: off; at most 2^27
};

// Packed alias entry: column idx of a table with b index bits keeps idx iff
// the low (32 - b) bits of the word are below the entry's low bits, else it
// takes the entry's high b bits as the state.  Full columns are stored as
// threshold U - 1 with alias = self, which draws identically to threshold U.
inline uint32_t pack_alias(uint32_t thresh, uint32_t alias, uint32_t idx, int bits)
{
    const uint64_t U = 1ull << (32 - bits);
    uint32_t t = thresh, a = alias;
    if ((uint64_t)thresh >= U) { t = (uint32_t)(U - 1); a = idx; }
    return (uint32_t)(((uint64_t)a << (32 - bits)) | t);
}

// Launch entry points (dmc_kernels.hip).
// spec: GEOM_SLAB (every job a steady wall-driven slab), GEOM_HALF (every job a
// transient half-space Gaussian with snapshots only), GEOM_GRAD (every job a
// film or pore cell under the gradient source, without bins or snapshots) or
// GEOM_ANY.
hipError_t launch_trajectories(const KArgs &a, int precision, int form, int spec, int block, int grid,
                               size_t lds_bytes, hipStream_t stream);
hipError_t launch_fill(double *p, size_t n_doubles, unsigned long long *q, size_t n_u64, hipStream_t stream);
hipError_t launch_debug_philox(uint64_t seed, const uint64_t *pid, const uint32_t *k, const uint32_t *tag,
                               uint32_t *out, size_t n, hipStream_t stream);
hipError_t launch_debug_alias(const uint32_t *packed, int bits, const uint32_t *words, uint32_t *states, size_t n,
                              hipStream_t stream);
hipError_t launch_debug_math(const double *x, double *lg, double *sn, double *cs, size_t n, hipStream_t stream);
// Instruction-cost probes (dmc_debug_op_cost): which operation a probe launch chains.
enum OpCost : int32_t {
    COST_FMA = 0,
    COST_PHILOX_UNIFORM_KEY = 1,
    COST_PHILOX_LANE_KEY = 2,
    COST_LOG = 3,
    COST_SIN = 4,
    COST_COS = 5,
    COST_SQRT = 6,
    COST_RCP = 7,
    COST_F64_ADD = 8,
    COST_N = 9
};
hipError_t launch_op_cost(int op, uint32_t iters, int blocks, uint32_t *out, hipStream_t stream);
int max_lds_bytes();
int occupancy_blocks(int precision, int form, int spec, bool bounded, bool jl, int block, size_t lds_bytes);
// The specialised kernel a set of jobs can use.
int kernel_spec(const JobDev *jobs, int n_jobs);

}  // namespace dmc
