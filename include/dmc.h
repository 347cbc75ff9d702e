/*
 * dmc.h -- C ABI of the MI355X library for the linearized energy-based
 * deviational Monte Carlo method for phonon transport (Peraud &
 * Hadjiconstantinou, "An alternative approach to efficient simulation of
 * micro/nanoscale phonon transport").
 *
 * The method (the particle algorithm, steps I-VI): under linearized
 * conditions deviational particles do not interact, so each particle is
 * simulated on its own.  It is drawn from a source term (initial condition,
 * isothermal wall, or imposed temperature gradient, Eq. (6)), flies for an
 * exponentially distributed time with mean tau(omega, p, T_eq) (step II),
 * meets geometry boundaries (step IVa: isothermal walls absorb, adiabatic
 * walls reflect specularly or diffusely, periodic faces re-insert), and at a
 * scattering event (step IVb) is redrawn from the normalised distribution
 * D de^eq/dT / tau of Eq. (2) with an isotropic direction and an unchanged
 * sign.  Track-length estimators (Eq. (4); Eq. (3) for snapshots) score
 * temperature, pseudo-temperature, heat flux and conductivity.
 *
 * Conventions for every entry point:
 *   - every call returns a dmc_status; on error nothing is allocated and any
 *     out-handle is set to NULL; dmc_last_error() returns a thread-local
 *     message valid until the next call on that thread;
 *   - handles are opaque; the caller creates and destroys them; material and
 *     geometry handles are immutable after creation and may be shared;
 *   - all arrays passed in are copied or fully consumed before the call
 *     returns (except a caller-provided device workspace, see dmc_run_opts);
 *   - SI units: rad/s, s/m^3 per rad/s, m/s, s, K, m, K/m;
 *   - the library runs on the current HIP device; it needs gfx950.
 */
#ifndef DMC_H_
#define DMC_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t dmc_status;
#define DMC_OK 0
#define DMC_E_INVALID (-1)     /* an argument is out of range or inconsistent */
#define DMC_E_NOMEM (-2)       /* host or device allocation failed / workspace too small */
#define DMC_E_DEVICE (-3)      /* a HIP call failed (no device, launch failure, ...) */
#define DMC_E_UNSUPPORTED (-4) /* valid request the library does not implement */
#define DMC_E_BUSY (-5)        /* the server cannot admit more work right now */

/* Thread-local description of the last failure on this thread ("" if none). */
const char *dmc_last_error(void);

/* Library version string. */
const char *dmc_version(void);

/* ------------------------------------------------------------------------ */
/* Material: D(omega, p), V_g(omega, p), tau(omega, p, T_eq)  (Eq. (1), (2))  */
/* ------------------------------------------------------------------------ */

typedef struct dmc_material dmc_material;

/* One polarization branch tabulated on frequency bins.  All arrays have
 * n_bins entries and are read during the call only. */
typedef struct {
    int32_t n_bins;
    const double *omega;  /* bin centre [rad/s], > 0 */
    const double *domega; /* bin width [rad/s], >= 0 */
    const double *dos;    /* density of states per polarization [s/m^3], >= 0 */
    const double *vg;     /* group-velocity magnitude [m/s], > 0 */
    const double *tau;    /* relaxation time at T_eq [s], > 0 */
    double degeneracy;    /* identical polarizations in this branch (TA: 2) */
} dmc_branch;

/* Tabulates the states m = (bin, branch) in branch order, computes
 * de^eq/dT(omega, T_eq) and the heat capacities C_m = D de/dT domega g in
 * FP64, builds the exact-integer alias tables of the initial (~C), wall-flux
 * (~C v) and post-scattering gain (~C / tau, Eq. (2)) distributions, and
 * uploads device copies.  Total states must be 1..65536.
 * scatter_g: the direction after a scattering event (step IVb).  0 draws it
 * isotropically, as the paper's step states; g in (-1, 1) draws it from the
 * Henyey-Greenstein phase function of mean cosine g about the incoming
 * direction, the generalisation the paper allows there (the state is still
 * redrawn from Eq. (2)).  First-event termination needs g = 0.
 * Errors: DMC_E_INVALID (non-finite or non-positive inputs, |g| >= 1), DMC_E_DEVICE. */
dmc_status dmc_material_create(const dmc_branch *branches, int32_t n_branches, double T_eq, double scatter_g,
                               dmc_material **out);
dmc_status dmc_material_destroy(dmc_material *m);

/* sums[0] = C_tot = sum C_m [J/m^3/K], sums[1] = G_tau = sum C_m / tau_m,
 * sums[2] = G_v = sum C_m v_m; n_states may be NULL. */
dmc_status dmc_material_info(const dmc_material *m, int32_t *n_states, double sums[3]);

/* ------------------------------------------------------------------------ */
/* Geometry (steps III and IVa)                                              */
/* ------------------------------------------------------------------------ */

typedef struct dmc_geometry dmc_geometry;

#define DMC_GEOM_SLAB_Z 0       /* walls at z = 0 (wall[0]) and z = length (wall[1]) */
#define DMC_GEOM_FILM_X 1       /* walls at x = 0 (wall[0]) and x = length (wall[1]) */
#define DMC_GEOM_PORE_CELL_XZ 2 /* periodic cell [0,length)^2 in x-z, cylindrical pore
                                   (axis y) of `radius` at the centre; wall[0] = pore */
#define DMC_GEOM_HALFSPACE_Z 3  /* solid z >= 0, surface z = 0 described by wall[0] */

#define DMC_WALL_ISOTHERMAL 0 /* absorbs; emits its deviational flux if T != T_eq */
#define DMC_WALL_ADIABATIC 1  /* specular with probability `specularity`, else diffuse */
#define DMC_WALL_PERIODIC 2   /* plane pair only: re-insert at the opposite wall */

typedef struct {
    int32_t type;
    double temperature; /* isothermal walls [K] */
    double specularity; /* adiabatic walls, in [0, 1] */
} dmc_wall;

typedef struct {
    int32_t kind;
    double length; /* slab L, film d, cell period P [m] (> 0; unused for the half space) */
    double radius; /* pore radius [m], 0 <= radius < length / 2 */
    dmc_wall wall[2];
} dmc_geometry_desc;

/* Copies desc into an immutable handle (host memory only; no device work).
 * Errors: DMC_E_INVALID (unknown kind or wall type; length not finite and > 0
 * where used; pore radius outside [0, length/2); specularity outside [0, 1];
 * an isothermal wall at T <= 0; periodic walls other than a plane pair; a pore
 * or half-space surface that is not adiabatic), DMC_E_NOMEM. */
dmc_status dmc_geometry_create(const dmc_geometry_desc *desc, dmc_geometry **out);
dmc_status dmc_geometry_destroy(dmc_geometry *g);

/* ------------------------------------------------------------------------ */
/* Sources (step I and the source-term paragraph; Eq. (6))                   */
/* ------------------------------------------------------------------------ */

#define DMC_SRC_WALLS 0    /* steady: isothermal walls with T != T_eq emit V_g cos C |T - T_eq| */
#define DMC_SRC_GAUSSIAN 1 /* transient: T_i - T_eq = dT exp(-|x|^2 / radius^2), half space */
#define DMC_SRC_GRADIENT 2 /* steady: uniform volumetric source of dT/dz = gradient */

typedef struct {
    int32_t kind;
    double dT;       /* GAUSSIAN amplitude [K] (non-zero) */
    double radius;   /* GAUSSIAN radius [m] (> 0) */
    double gradient; /* GRADIENT dT/dz [K/m] (non-zero) */
} dmc_source;

/* ------------------------------------------------------------------------ */
/* Tallies (step V; Eq. (3) and (4))                                          */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t n_bins;    /* 1-D bins along the confining axis (slab: z, film: x); 0 = none; <= 4096 */
    int32_t n_batches; /* batch replicas for standard errors, batch = pid mod n_batches; 2..256 */
    int32_t kmax;      /* stop a particle after kmax scattering events; -1 = never */
    int32_t n_hj;      /* per-scatter-index flux contributions H_j, j < n_hj (<= kmax); 0 = off */
    int32_t grid[3];   /* transient jobs: snapshot grid cells along x, y, z.  Steady pore cells
                          (DMC_GEOM_PORE_CELL_XZ): (nx, 1, nz) adds the steady temperature and
                          z heat-flux fields, Eq. (4) in every cell of an nx x nz grid over the
                          unit cell (grid_lo x, z = 0, grid_hi x, z = period; y bounds unused),
                          read as DMC_Q_FIELD_T / DMC_Q_FIELD_QZ; nx, nz <= 1024.  0 = none. */
    double grid_lo[3]; /* grid bounds [m] */
    double grid_hi[3];
    int32_t first_event; /* in-plane films (DMC_GEOM_FILM_X, gradient source) only: 1 ends every
                            trajectory at its first scattering event or first diffuse wall
                            reflection.  Exact for films (the thin-film special case of the
                            periodic-nanostructure application): afterwards the direction is
                            isotropic or Lambertian about the wall normal and the film is
                            invariant along z, so the flux still to come averages to zero.
                            Specular reflections continue the free path.  Rejected elsewhere. */
    int32_t region;      /* transient jobs: 1 adds time-windowed track-length tallies in the
                            z-aligned cylinder {(x-cx)^2 + (y-cy)^2 < radius^2, z_lo <= z < z_hi}
                            (a probe region such as a thermoreflectance spot): over each window
                            [t_{j-1}, t_j) between snapshot times (t_{-1} = 0), the mean
                            temperature (time spent in the region) and z heat flux (signed
                            z length travelled in it); the time average of Eq. (3), read as
                            DMC_Q_REGION_T / DMC_Q_REGION_QZ.  0 = none. */
    double region_c[2];  /* cx, cy [m] */
    double region_radius;
    double region_z[2];  /* z_lo, z_hi [m], 0 <= z_lo < z_hi */
} dmc_tally_desc;

/* ------------------------------------------------------------------------ */
/* Running                                                                    */
/* ------------------------------------------------------------------------ */

#define DMC_PREC_FP64 0       /* every step in FP64 (the parity mode) */
#define DMC_PREC_FP32_TALLY64 1 /* flight, intersection, sampling in FP32; tallies in FP64 */

#define DMC_FORM_PLAIN 0      /* one thread per particle run to completion, tables in global
                                 memory, every contribution a direct FP64 global atomic */
#define DMC_FORM_PERSISTENT 1 /* persistent waves refilling lanes from a particle queue, tables
                                 staged in LDS, per-lane bin caches and LDS-privatised tallies */

typedef struct {
    int32_t precision;     /* DMC_PREC_* */
    int32_t form;          /* DMC_FORM_* */
    void *stream;          /* hipStream_t to run on (NULL: the null stream) */
    int32_t block;         /* persistent: threads per workgroup (64..1024, multiple of 64); 0 = auto */
    int32_t chunk;         /* persistent: particles a wave takes from the queue at once; 0 = auto */
    int32_t refill_min;    /* persistent: refill a wave when at least this many lanes are free; 0 = auto */
    int32_t lds_tally;     /* persistent: 1 = privatise tallies in LDS when they fit, 0 = global */
    int32_t grid_blocks;   /* persistent: workgroups to launch; 0 = fill the device */
    void *workspace;       /* optional caller-owned device memory for tallies and queues */
    size_t workspace_bytes;
    uint32_t *nscat_out;   /* optional device array of nscat_out_len entries: the scattering
                              events of particle pid of job j are written at (n_particles of
                              jobs 0..j-1) + pid; not used by the server */
    int32_t prio_flights;  /* persistent: a wave holding a particle past this many segments
                              (4x, 16x as many) gets issue priority 1 (2, 3) on its SIMD,
                              so that the few longest trajectories of a heavy-tailed job
                              do not end the launch late; in the gradient kernel such a
                              wave also lets a flight cross up to 8 (32, 64) periodic faces
                              per iteration from 1/16 (1, 16) of this many segments on;
                              0 = 65536, < 0 = off, at most 2^27.  Changes timing only. */
    int32_t pad0;
    uint64_t nscat_out_len; /* entries of nscat_out; a launch with nscat_out set fails with
                               DMC_E_INVALID unless this is at least the sum of the jobs'
                               n_particles (the kernels write one entry per particle) */
} dmc_run_opts;

/* Fills opts with the defaults (FP32 + FP64 tallies, persistent, auto parameters). */
void dmc_run_opts_default(dmc_run_opts *opts);

/* One simulation in a batched launch. */
typedef struct {
    const dmc_material *material; /* all jobs of one launch must share the material */
    const dmc_geometry *geometry;
    dmc_source source;
    dmc_tally_desc tally;
    uint64_t n_particles; /* >= 1 */
    uint64_t seed;        /* Philox key */
    const double *times;  /* transient snapshot times [s], ascending, > 0; NULL for steady */
    int32_t n_times;      /* <= 1024; the last time is t_final */
    int32_t pad0;
    uint64_t first_particle; /* particles first_particle .. first_particle + n_particles - 1 of the
                                seed's realisation are simulated (0 for a whole run). A slice is an
                                estimate on its own (normalised by its n_particles); the raw sums
                                (DMC_Q_RAW) of disjoint slices add up to those of the union. */
} dmc_job;

typedef struct dmc_result dmc_result;

/* Bytes of device workspace a launch of these jobs needs (tallies, queue, counters). */
dmc_status dmc_workspace_size(const dmc_job *jobs, int32_t n_jobs, const dmc_run_opts *opts, size_t *bytes);

/* Runs one simulation; asynchronous on opts->stream.  Equivalent to a batch of
 * one (same limits and errors as dmc_simulate_batch). */
dmc_status dmc_simulate(const dmc_material *material, const dmc_geometry *geometry, const dmc_source *source,
                        uint64_t n_particles, uint64_t seed, const dmc_tally_desc *tally, const double *times,
                        int32_t n_times, const dmc_run_opts *opts, dmc_result **out);

/* Runs n_jobs simulations in ONE launch (persistent form: one particle queue
 * over all jobs; plain form: one launch per job on the same stream).
 * Asynchronous on opts->stream.  jobs: 1..4096 descriptors, read during the
 * call.  Per job: n_particles >= 1 (first_particle + n_particles must not
 * wrap), n_bins 0..4096 (slab and film geometries only), n_batches 2..256,
 * kmax >= -1, n_hj 0..min(kmax, 1024), n_times 0..1024 positive, strictly
 * increasing times (transient sources only).  *out owns the tallies until
 * dmc_result_destroy.
 * Errors: DMC_E_INVALID (a limit above; a source, geometry and tally that do
 * not go together; nscat_out_len too small), DMC_E_UNSUPPORTED (a valid
 * request the kernels do not run: steady sources with snapshot times, or
 * material tables larger than the LDS of the persistent form), DMC_E_NOMEM
 * (allocation failed, or the caller's workspace is smaller than
 * dmc_workspace_size), DMC_E_DEVICE. */
dmc_status dmc_simulate_batch(const dmc_job *jobs, int32_t n_jobs, const dmc_run_opts *opts, dmc_result **out);

/* ---- The batched launch for callers that cannot allocate ----
 * For code that must not allocate device memory: HIP graph capture, tight
 * serving loops, harnesses that forbid allocation.  Runs the jobs like
 * dmc_simulate_batch (same kernels, same realisation) but allocates nothing:
 * job descriptors, snapshot times, counters, the particle queue and the device
 * tally blocks live in one fixed 32 MiB device array per GPU, which the library
 * holds until the process ends; descriptors and times reach it through kernel
 * arguments, and nothing is synchronised (no event, no copy back): the call
 * only enqueues work on opts->stream.
 * Limits: 1..64 jobs, at most 8192 snapshot times over all jobs, and tallies
 * that fit the array (about 4.1 million doubles of device tally blocks; the
 * error message states the need).  opts->workspace must be NULL.
 * Outputs (caller-owned device memory):
 *   raw_out: each job's raw tally block (the doubles dmc_tally_read returns for
 *     DMC_Q_RAW after dmc_simulate_batch), back to back in job order, raw_len
 *     doubles available;
 *   counters_out: optional, 6 per job: particles, scattering events, boundary
 *     events, segments, capped, flights (the fields of dmc_stats);
 *   raw_offsets: optional host array of n_jobs + 1 entries: job j's block is
 *     raw_out[raw_offsets[j] .. raw_offsets[j + 1]).  With raw_out NULL the call
 *     only validates the jobs and fills raw_offsets (no device work).
 * Every call on a GPU shares that GPU's array and leaves its contents behind;
 * each call clears what must start at zero.  Calls that overlap on one GPU (on
 * different streams, or from several threads without ordering) race on it:
 * serialise them.  Errors: DMC_E_INVALID (limits, raw_len or nscat_out_len too
 * small), DMC_E_DEVICE. */
dmc_status dmc_simulate_batch_noalloc(const dmc_job *jobs, int32_t n_jobs, const dmc_run_opts *opts, double *raw_out,
                                      size_t raw_len, uint64_t *counters_out, size_t *raw_offsets);

/* ---- Autotuner (persistent form) ----
 * Picks block size, queue chunk, refill threshold and tally privatisation for a
 * batch by timing trial launches of a sample of it.  The sample cuts every job
 * to the first part of its particle range, sized so that a trial runs about
 * sample_flights flights in total, and stops each trajectory after trial_cap
 * flights, so that a trial measures the bulk rate rather than the single
 * longest trajectory of a heavy-tailed job.  The parameters are searched one
 * at a time from the defaults (tally privatisation, block, chunk, refill
 * threshold); a candidate replaces the current choice only when it is at least
 * 2 % faster.  Unprivatised tallies (global FP64 atomics, which can serialise
 * on a few contended sums) are first screened on 1/16 of the sample and
 * dropped when that alone takes longer than the current choice.  None of these parameters changes an estimate: they move FP64
 * additions between registers, LDS and HBM, nothing else.
 * The choice is cached for the life of the process per material, precision and
 * batch signature (every job's geometry, source kind, tally shape and the
 * order of magnitude of its particle count).
 * Synchronous; runs on base->stream; allocates and frees its own sample
 * workspace.  For the plain form it returns *base unchanged with no trials. */
typedef struct {
    int32_t block, chunk, refill_min, lds_tally;
    int32_t pilot;         /* 1: a screening run on 1/16 of the sample (unprivatised tallies only) */
    int32_t pad0;
    double ms;             /* trial kernel time */
    double flights_per_s;  /* trial flights / trial kernel time */
} dmc_tune_trial;

typedef struct {
    uint64_t sample_flights; /* 0: 5e10 */
    uint32_t trial_cap;      /* 0: 4096 flights */
    int32_t use_cache;       /* 1: reuse the cached choice for the same signature */
    dmc_tune_trial *trials;  /* optional host array receiving the trials in order */
    int32_t max_trials;
    int32_t n_trials;        /* out: trials run (0 when the cache answered) */
    int32_t from_cache;      /* out */
} dmc_tune_opts;

/* best receives *base with block, chunk, refill_min and lds_tally set and
 * grid_blocks 0.  tune may be NULL (defaults, cache on). */
dmc_status dmc_autotune(const dmc_job *jobs, int32_t n_jobs, const dmc_run_opts *base, dmc_tune_opts *tune,
                        dmc_run_opts *best);

/* ---- Truncation planning for periodic problems (gradient source) ----
 * Trajectories under periodic boundaries never end, so they are cut after
 * K_max scattering events.  The mean flux carried between scattering events j
 * and j+1, <H_j>, decays with j (exponentially after a few events, in the
 * paper's periodic-nanostructure application); cutting at K discards the sum
 * of <H_j> over j >= K.  This call runs a pilot of n_pilot particles (ids
 * first_particle + n_particles onwards of the job's seed, disjoint from the
 * job's own) tracked for k_pilot events and finds the run j = 1..n of events
 * whose |<H_j>| exceeds 4 pilot standard errors (n_fit = n); unless n_pilot is
 * given, a pilot resolving fewer than 3 is grown tenfold up to min(N, 1e7).
 * It returns:
 *   k_uncertain: the first j >= 1 whose |<H_j>| is at most its standard error
 *     at the job's n_particles (the paper's empirical criterion);
 *   decay, amplitude: |<H_j>| ~ amplitude * decay^j for j >= 1: a log-linear fit
 *     weighted by (|<H_j>| / se_j)^2 over j = 1..n when n >= 3, the ratio
 *     |<H_2>| / |<H_1>| when n = 2, the upper bound 4 se_2 / |<H_1>| when n = 1;
 *   kmax: the smallest K > n whose tail sum amplitude decay^K / (1 - decay) is
 *     at most bias_fraction times the standard error of kappa at n_particles,
 *     and bias_bound that tail sum [W/m/K]; when n = 0 (no flux after the first
 *     event is resolved; exactly zero in expectation for films) kmax = 1; when
 *     no decay below 1 is found, fit_ok = 0 and kmax = max(n + 1, k_uncertain);
 *     in those two cases bias_bound is |the pilot's sum of <H_j> beyond kmax|;
 *   kappa_se: the predicted standard error of kappa at n_particles.
 * The job must have a gradient source.  Synchronous on opts->stream. */
typedef struct {
    uint64_t n_pilot;     /* 0: min(n_particles, 1e6), grown as above */
    int32_t k_pilot;      /* 0: 200 (3 .. 1024) */
    int32_t pad0;
    double bias_fraction; /* 0: 0.2 */
} dmc_trunc_opts;

typedef struct {
    int32_t kmax, k_uncertain, fit_ok, n_fit;
    double decay, amplitude, bias_bound, kappa_se;
    double kappa_pilot;   /* the pilot's kappa with k_pilot events [W/m/K] */
    uint64_t n_pilot;     /* pilot particles used */
} dmc_trunc_plan;

dmc_status dmc_plan_truncation(const dmc_job *job, const dmc_run_opts *opts, const dmc_trunc_opts *t,
                               dmc_trunc_plan *out);

#define DMC_Q_T 0          /* energy temperature T - T_eq per bin [K] (n = n_bins) */
#define DMC_Q_TLOC 1       /* pseudo-temperature T_loc - T_eq per bin [K] */
#define DMC_Q_FLUX 2       /* heat flux along z per bin [W/m^2] */
#define DMC_Q_KAPPA 3      /* effective conductivity -<q_z> / (dT/dz) [W/m/K] (n = 1) */
#define DMC_Q_HJ 4         /* conductivity carried between scatter j and j+1 (n = n_hj) */
#define DMC_Q_SNAPSHOT 5   /* T - T_eq per grid cell at time_index [K] (n = cells, x fastest) */
#define DMC_Q_SNAPSHOT_SUM 6 /* raw sum of signs per cell at time_index, overflow last (n = cells+1) */
#define DMC_Q_RAW 7        /* the job's raw FP64 tally block (n = dmc_tally_raw_size) */
#define DMC_Q_REGION_T 8   /* windowed mean T - T_eq in the region, one per window [K] (n = n_times) */
#define DMC_Q_REGION_QZ 9  /* windowed mean z heat flux in the region [W/m^2] (n = n_times) */
#define DMC_Q_FIELD_T 10   /* steady pore cell: T - T_eq per field cell [K] (n = nx * nz, x fastest;
                              energy over the whole cell area, pore included) */
#define DMC_Q_FIELD_QZ 11  /* steady pore cell: z heat flux per field cell [W/m^2] (same layout) */

/* Waits for the launch, then writes n values of `quantity` of job `job` (and,
 * if stderr_out is not NULL, their standard errors: batch means for bins,
 * per-particle moments otherwise) into caller-owned host arrays.
 * Errors: DMC_E_INVALID (quantity not tallied, n too small, job out of range). */
dmc_status dmc_tally_read(const dmc_result *res, int32_t job, int32_t quantity, int32_t time_index, double *mean,
                          double *stderr_out, size_t n);

/* Number of doubles of DMC_Q_RAW for a job. */
dmc_status dmc_tally_raw_size(const dmc_result *res, int32_t job, size_t *n);

typedef struct {
    uint64_t particles;  /* particles completed */
    uint64_t scatters;   /* scattering events (step IVb only) */
    uint64_t boundary;   /* boundary interactions (step IVa) */
    uint64_t iterations; /* trajectory segments (one per free flight, plus one per periodic face crossed) */
    uint64_t capped;     /* particles stopped by the 2^24-flight safety cap */
    double kernel_ms;    /* device time of the trajectory launch(es), HIP events */
    uint64_t flights;    /* free flights begun (one random-number block each); iterations - flights
                            = periodic faces crossed, boundary - (iterations - flights) = wall and
                            pore-surface interactions */
} dmc_stats;

/* Waits for the launch; job = -1 gives the launch totals. */
dmc_status dmc_result_stats(const dmc_result *res, int32_t job, dmc_stats *out);
dmc_status dmc_result_destroy(dmc_result *res);

/* ------------------------------------------------------------------------ */
/* Serving: continuous batching of simulation requests on one device          */
/* ------------------------------------------------------------------------ */

typedef struct dmc_server dmc_server;

typedef struct {
    size_t memory_budget;  /* device bytes the admitted requests' tallies may hold */
    int32_t max_active;    /* requests resident at once (1..64) */
    uint64_t epoch_flights; /* estimated flights per epoch launch (0 = 2e10): an epoch runs what
                               equal shares of it would give the admitted requests (each at most
                               its own remaining flights), handed out to the requests with the
                               fewest flights left first */
    uint32_t drain_flights; /* flights a wave may still run once the epoch's queue is empty before
                               it suspends its live particles to the next epoch (0 = 2048) */
    int32_t class_epochs;  /* 0: every admitted request in every epoch, in the kernel that fits the
                              epoch's jobs (the generic one once classes mix); 1: each epoch runs
                              the admitted requests of one class (wall-driven slabs, transient
                              half spaces, gradient films and pore cells, others), the classes
                              taking turns, so every epoch uses that class's specialised kernel:
                              more flights per second, but a request's slowest trajectories
                              advance only in its class's turns, which lengthens latency */
    dmc_run_opts run;      /* precision / form / stream / parameters of every epoch */
} dmc_server_opts;

/* The server admits requests while their device memory fits the budget and
 * a slot is free; each epoch is one persistent launch over slices of the
 * particle ranges of the admitted requests (of the epoch's class, see
 * class_epochs), the epoch's flights going first to the requests with the
 * fewest left (see epoch_flights), so requests that arrive while others run
 * join at a later epoch.  Epochs are time-bounded: particles still in
 * flight when an epoch drains are suspended on the device and resumed first
 * in the next epoch with the same random-number counters, so results do not
 * depend on the slicing.  A request's tallies stay on the device until it
 * completes; collecting it copies them to the host. */
dmc_status dmc_server_create(const dmc_material *material, const dmc_server_opts *opts, dmc_server **out);
/* Queues a request (copied); *ticket identifies it.  DMC_E_INVALID if it can never fit. */
dmc_status dmc_server_submit(dmc_server *s, const dmc_job *job, uint64_t *ticket);
/* Runs one epoch if any work is pending (admitting queued requests first).
 * *n_done receives the number of requests that completed in this epoch. */
dmc_status dmc_server_step(dmc_server *s, int32_t *n_done);
/* 1 if the ticket's request is complete, 0 if not (queued or running). */
dmc_status dmc_server_poll(dmc_server *s, uint64_t ticket, int32_t *done);
/* Runs epochs (dmc_server_step) until the ticket's request is complete (at
 * once if it already is); the other admitted requests advance in the same
 * epochs, and those that complete on the way stay ready for
 * dmc_server_collect.  *n_epochs (may be NULL) receives the epochs run.
 * Errors: DMC_E_INVALID (unknown or already collected ticket), those of
 * dmc_server_step. */
dmc_status dmc_server_wait(dmc_server *s, uint64_t ticket, int32_t *n_epochs);
/* Takes a completed request's result (a one-job dmc_result owned by the caller). */
dmc_status dmc_server_collect(dmc_server *s, uint64_t ticket, dmc_result **out);
/* Requests queued / running. */
dmc_status dmc_server_load(const dmc_server *s, int32_t *queued, int32_t *running);
/* Counters summed over every epoch run so far (particles finished, scattering
 * and boundary events, flights, capped; kernel_ms = total epoch kernel time):
 * flights / kernel_ms is the server's device throughput. */
dmc_status dmc_server_totals(const dmc_server *s, dmc_stats *out);
dmc_status dmc_server_destroy(dmc_server *s);

/* ------------------------------------------------------------------------ */
/* Test hooks                                                                */
/* ------------------------------------------------------------------------ */

#define DMC_TAG_STEP 0
#define DMC_TAG_EMIT_A 1
#define DMC_TAG_EMIT_B 2

/* Philox4x32-10 block for counter (pid lo, pid hi, k, tag) and key (seed lo,
 * seed hi); n requests at once (arrays of n, host memory), computed on the
 * device.  out has 4 n words. */
dmc_status dmc_debug_philox(uint64_t seed, const uint64_t *pid, const uint32_t *k, const uint32_t *tag,
                            uint32_t *out, size_t n);

#define DMC_TABLE_GAIN 0 /* ~ C / tau */
#define DMC_TABLE_INIT 1 /* ~ C */
#define DMC_TABLE_FLUX 2 /* ~ C v */

/* Canonical alias table (thresh, alias; 2^bits columns) that the library built. */
dmc_status dmc_debug_alias(const dmc_material *m, int32_t which, int32_t *bits, uint32_t *thresh,
                           uint32_t *alias, size_t n);
/* Device lookups of table `which` for n host words; writes the drawn states. */
dmc_status dmc_debug_alias_draw(const dmc_material *m, int32_t which, const uint32_t *words, uint32_t *states,
                                size_t n);

/* FP64 parity-mode logarithm and sin/cos of 2 pi u, evaluated on the device
 * for n host values (out arrays of n, any may be NULL). */
dmc_status dmc_debug_fp64_math(const double *x, double *log_out, double *sin2pi_out, double *cos2pi_out, size_t n);

/* Instruction-cost probe behind the algorithmic work counts of the roofline:
 * launches `blocks` workgroups of 256 lanes (0: 32 per compute unit, full
 * occupancy) in which every lane runs `iters` iterations of four independent
 * dependency chains of one operation, and times the second of two launches with
 * HIP events on the null stream.  *ms receives that time and *op_count the number
 * of operations executed (lanes x iters x 4), so that
 * slots = ms 1e-3 x (CUs x 64 x clock) / op_count is the VALU issue slots per
 * lane one operation takes.  op: 0 FP32 FMA (calibration, 1 slot), 1 Philox4x32-10
 * block with a wave-uniform key (the key schedule on the scalar unit), 2 the
 * same with a key per lane, 3 v_log_f32, 4 v_sin_f32, 5 v_cos_f32, 6 v_sqrt_f32,
 * 7 v_rcp_f32, 8 FP64 add.  Allocates and frees a small device buffer.
 * Errors: DMC_E_INVALID (op out of range, iters = 0), DMC_E_DEVICE. */
dmc_status dmc_debug_op_cost(int32_t op, uint32_t iters, int32_t blocks, double *ms, uint64_t *op_count);

#ifdef __cplusplus
}
#endif
#endif /* DMC_H_ */
