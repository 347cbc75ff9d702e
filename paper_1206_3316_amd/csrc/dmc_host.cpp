// dmc_host.cpp -- host side of the MI355X deviational Monte Carlo library:
// material tabulation and alias tables, geometry/source/tally validation,
// launch planning (LDS privatisation, occupancy), result finalisation, the
// serving loop and the C ABI of include/dmc.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <deque>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "dmc_host_internal.h"

using namespace dmc;

namespace dmc {

namespace {
thread_local std::string g_err;
}

dmc_status fail(dmc_status code, const std::string &msg)
{
    g_err = msg;
    return code;
}

}  // namespace dmc

#define HIP_OR_FAIL DMC_HIP_OR_FAIL

namespace {

constexpr double kHbar = 1.054571817e-34;  // J s (CODATA 2018)
constexpr double kBoltz = 1.380649e-23;    // J/K (CODATA 2018)
constexpr double kPi = 3.14159265358979323846;

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }
bool finite_nonneg(double x) { return std::isfinite(x) && x >= 0.0; }

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

// ------------------------------------------------------------ alias tables ----

namespace dmc {

// Exact-integer Walker/Vose construction.  Masses: floor((w_j / W) 2^32) with W
// summed in index order, the shortfall to 2^32 handed out one unit each to the
// largest fractional parts (lower index first on ties).  Columns of capacity
// U = 2^(32-b); under-full and over-full columns wait in two FIFO queues in
// index order; the front under-full column takes its threshold and the front
// over-full column as alias, which gives up (U - threshold) and rejoins the
// back of whichever queue it now belongs to; left-over columns are full.
bool build_alias(const std::vector<double> &w, AliasTable &t, std::string &why)
{
    const size_t K = w.size();
    if (K == 0 || K > 65536) {
        why = "alias table needs 1..65536 weights";
        return false;
    }
    int b = 1;
    while ((size_t(1) << b) < K) ++b;
    const size_t n = size_t(1) << b;
    double W = 0.0;
    for (size_t j = 0; j < K; ++j) {
        if (!finite_nonneg(w[j])) {
            why = "alias weight is negative or not finite";
            return false;
        }
        W += w[j];
    }
    if (!(W > 0.0) || !std::isfinite(W)) {
        why = "alias weights sum to zero";
        return false;
    }
    std::vector<uint64_t> q(n, 0);
    std::vector<double> frac(n, 0.0);
    uint64_t assigned = 0;
    for (size_t j = 0; j < K; ++j) {
        const double sc = (w[j] / W) * 4294967296.0;
        const double fl = std::floor(sc);
        q[j] = (uint64_t)fl;
        frac[j] = sc - fl;
        assigned += q[j];
    }
    const uint64_t total = uint64_t(1) << 32;
    if (assigned > total || total - assigned > n) {
        why = "alias rounding failed";
        return false;
    }
    std::vector<uint32_t> order(n);
    for (size_t j = 0; j < n; ++j) order[j] = (uint32_t)j;
    std::stable_sort(order.begin(), order.end(), [&](uint32_t x, uint32_t y) { return frac[x] > frac[y]; });
    for (uint64_t r = 0; r < total - assigned; ++r) q[order[r]] += 1;

    t.bits = b;
    t.mass = q;
    t.thresh.assign(n, 0);
    t.alias.assign(n, 0);
    const uint64_t U = uint64_t(1) << (32 - b);
    std::deque<uint32_t> under, over;
    for (size_t j = 0; j < n; ++j) (q[j] < U ? under : over).push_back((uint32_t)j);
    while (!under.empty() && !over.empty()) {
        const uint32_t l = under.front();
        under.pop_front();
        const uint32_t g = over.front();
        over.pop_front();
        t.thresh[l] = (uint32_t)q[l];
        t.alias[l] = g;
        q[g] -= (U - q[l]);
        (q[g] < U ? under : over).push_back(g);
    }
    for (uint32_t g : over) {
        t.thresh[g] = (uint32_t)U;
        t.alias[g] = g;
    }
    for (uint32_t l : under) {
        t.thresh[l] = (uint32_t)U;
        t.alias[l] = l;
    }
    t.packed.resize(n);
    for (size_t j = 0; j < n; ++j) t.packed[j] = pack_alias(t.thresh[j], t.alias[j], (uint32_t)j, b);
    return true;
}

}  // namespace dmc

// ------------------------------------------------------------------ handles ----

dmc_material::~dmc_material()
{
    for (void *p : {(void *)d_gain, (void *)d_init, (void *)d_flux, (void *)d_st32, (void *)d_st64})
        if (p) (void)hipFree(p);
}

dmc_result::~dmc_result()
{
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    if (dev_mem) (void)hipFree(dev_mem);
    if (on_destroy) on_destroy();
}

namespace dmc {

// --------------------------------------------------------- job validation ----

// Two-entry alias table of the wall-source powers, packed for the device, with
// the rule of build_alias (largest-remainder integer masses summing to 2^32, then
// Vose's pairing): the under-full column keeps its mass and aliases the other,
// which is left full.  Written without containers so that every launch path can
// use it.
static void alias_two(double w0, double w1, uint32_t packed[2])
{
    const double W = w0 + w1;
    const double s0 = (w0 / W) * 4294967296.0, s1 = (w1 / W) * 4294967296.0;
    uint64_t q[2] = {(uint64_t)std::floor(s0), (uint64_t)std::floor(s1)};
    const double f[2] = {s0 - std::floor(s0), s1 - std::floor(s1)};
    uint64_t rem = (uint64_t(1) << 32) - q[0] - q[1];
    const int first = (f[1] > f[0]) ? 1 : 0;  // ties: the lower index first
    for (int r = 0; rem > 0; ++r, --rem) q[r == 0 ? first : 1 - first] += 1;
    const uint64_t U = uint64_t(1) << 31;
    uint32_t thresh[2] = {(uint32_t)U, (uint32_t)U}, alias[2] = {0u, 1u};
    if (q[0] < U) {
        thresh[0] = (uint32_t)q[0];
        alias[0] = 1;
    } else if (q[1] < U) {
        thresh[1] = (uint32_t)q[1];
        alias[1] = 0;
    }
    for (uint32_t j = 0; j < 2; ++j) packed[j] = pack_alias(thresh[j], alias[j], j, 1);
}

dmc_status prepare_job(const dmc_job &jb, JobHost &h)
{
    JobMeta meta;
    dmc_status st = prepare_job_core(jb, h.dev, meta);
    if (st != DMC_OK) return st;
    h.job = jb;
    h.geom = jb.geometry->d;
    h.times.assign(jb.times, jb.times + jb.n_times);
    h.power = meta.power;
    h.avg_volume = meta.avg_volume;
    h.size = meta.size;
    h.hidden = meta.hidden;
    return DMC_OK;
}

dmc_status prepare_job_core(const dmc_job &jb, JobDev &d, JobMeta &h)
{
    if (!jb.material || !jb.geometry) return fail(DMC_E_INVALID, "job without material or geometry");
    const dmc_material &M = *jb.material;
    const dmc_geometry_desc &g = jb.geometry->d;
    const dmc_source &s = jb.source;
    const dmc_tally_desc &t = jb.tally;
    if (jb.n_particles < 1) return fail(DMC_E_INVALID, "n_particles must be >= 1");
    if (jb.first_particle + jb.n_particles < jb.first_particle)
        return fail(DMC_E_INVALID, "first_particle + n_particles overflows");
    if (t.n_bins < 0 || t.n_bins > kMaxBins) return fail(DMC_E_INVALID, "n_bins out of range");
    if (t.n_batches < 2 || t.n_batches > 256) return fail(DMC_E_INVALID, "n_batches must be 2..256");
    if (t.kmax < -1) return fail(DMC_E_INVALID, "kmax must be >= -1");
    if (t.n_hj < 0 || t.n_hj > kMaxHj || (t.n_hj > 0 && (t.kmax < 0 || t.n_hj > t.kmax)))
        return fail(DMC_E_INVALID, "n_hj must be in 0..kmax");
    if (t.first_event != 0 && (t.first_event != 1 || g.kind != DMC_GEOM_FILM_X || s.kind != DMC_SRC_GRADIENT))
        return fail(DMC_E_INVALID, "first_event applies to in-plane films under the gradient source");
    if (t.first_event && M.scatter_g != 0.0)
        return fail(DMC_E_INVALID, "first_event needs isotropic scattering (scatter_g = 0)");
    if (jb.n_times < 0 || jb.n_times > kMaxTimes || (jb.n_times > 0 && !jb.times))
        return fail(DMC_E_INVALID, "bad snapshot times");
    for (int i = 0; i < jb.n_times; ++i)
        if (!finite_pos(jb.times[i]) || (i > 0 && !(jb.times[i] > jb.times[i - 1])))
            return fail(DMC_E_INVALID, "snapshot times must be positive and increasing");
    const bool transient = jb.n_times > 0;
    std::memset(&d, 0, sizeof(d));
    h = JobMeta{};
    d.n = jb.n_particles;
    d.pid0 = jb.first_particle;
    d.key0 = (uint32_t)jb.seed;
    d.key1 = (uint32_t)(jb.seed >> 32);
    d.geom = g.kind;
    d.src = s.kind;
    d.length = g.length;
    d.radius = g.radius;
    for (int i = 0; i < 2; ++i) {
        d.wall_type[i] = g.wall[i].type;
        const double p = g.wall[i].specularity;
        d.spec_thr[i] = std::min<uint64_t>((uint64_t)std::llround(p * 4294967296.0), uint64_t(1) << 32);
    }
    d.n_bins = t.n_bins;
    d.n_batches = t.n_batches;
    d.kmax = t.first_event ? 1 : t.kmax;  // first-event termination: one scattering event at most
    d.first_event = t.first_event;
    d.n_hj = t.n_hj;
    d.n_times = jb.n_times;
    d.lds_bins = d.lds_kappa = d.lds_hj = -1;
    d.off_bins = d.off_kappa = d.off_hj = d.off_snap = d.off_snap_abs = d.off_dispx = d.off_region = -1;
    d.off_field = -1;
    d.lds_field = -1;
    d.lds_dispx = d.lds_region = -1;
    d.disp_tel = 0;
    if ((g.kind == DMC_GEOM_SLAB_Z || g.kind == DMC_GEOM_FILM_X) && t.n_bins > 0) {
        d.bins_per_len = (double)t.n_bins / g.length;
        d.bin_width = g.length / (double)t.n_bins;
    } else if (t.n_bins > 0) {
        return fail(DMC_E_INVALID, "1-D bins need a slab or film geometry");
    }

    if (s.kind == DMC_SRC_WALLS) {
        if (g.kind != DMC_GEOM_SLAB_Z && g.kind != DMC_GEOM_FILM_X)
            return fail(DMC_E_INVALID, "wall sources need a slab or film geometry");
        if (transient) return fail(DMC_E_UNSUPPORTED, "wall sources are steady (no snapshot times)");
        double pw[2];
        int nsrc = 0;
        for (int i = 0; i < 2; ++i) {
            d.wall_sign[i] = (g.wall[i].temperature > M.T_eq) ? 1.0 : -1.0;
            if (g.wall[i].type == DMC_WALL_ISOTHERMAL && g.wall[i].temperature != M.T_eq) {
                pw[nsrc] = std::fabs(g.wall[i].temperature - M.T_eq) * M.G_v / 4.0;
                d.src_wall[nsrc] = i;
                ++nsrc;
            }
        }
        if (nsrc == 0) return fail(DMC_E_INVALID, "no isothermal wall differs from T_eq");
        d.n_src = nsrc;
        h.power = (nsrc == 2) ? pw[0] + pw[1] : pw[0];
        if (nsrc == 2) alias_two(pw[0], pw[1], d.src_packed);
        h.avg_volume = g.length;
    } else if (s.kind == DMC_SRC_GRADIENT) {
        if (!(std::isfinite(s.gradient) && s.gradient != 0.0)) return fail(DMC_E_INVALID, "zero gradient");
        if (transient) return fail(DMC_E_UNSUPPORTED, "gradient sources are steady");
        double vol;
        if (g.kind == DMC_GEOM_FILM_X) {
            vol = g.length;
            h.avg_volume = g.length;
        } else if (g.kind == DMC_GEOM_PORE_CELL_XZ) {
            vol = g.length * g.length - kPi * g.radius * g.radius;
            h.avg_volume = g.length * g.length;
        } else {
            return fail(DMC_E_INVALID, "gradient sources need a film or pore-cell geometry");
        }
        h.power = vol * std::fabs(s.gradient) * M.G_v / 2.0;
        d.sign0 = (s.gradient > 0.0) ? -1.0 : 1.0;
    } else if (s.kind == DMC_SRC_GAUSSIAN) {
        if (g.kind != DMC_GEOM_HALFSPACE_Z || !transient)
            return fail(DMC_E_INVALID, "the gaussian initial condition needs a half space and snapshot times");
        if (!(std::isfinite(s.dT) && s.dT != 0.0) || !finite_pos(s.radius))
            return fail(DMC_E_INVALID, "gaussian needs dT != 0 and radius > 0");
        h.power = M.C_tot * std::fabs(s.dT) * std::pow(kPi, 1.5) * s.radius * s.radius * s.radius / 2.0;
        d.sign0 = (s.dT > 0.0) ? 1.0 : -1.0;
        d.sigma = s.radius / std::sqrt(2.0);
    } else {
        return fail(DMC_E_INVALID, "unknown source kind");
    }
    if (transient) {
        int64_t nc = 1;
        for (int i = 0; i < 3; ++i) {
            if (t.grid[i] < 1 || !(t.grid_hi[i] > t.grid_lo[i]))
                return fail(DMC_E_INVALID, "snapshot grid needs >= 1 cell and hi > lo per axis");
            d.grid[i] = t.grid[i];
            d.grid_lo[i] = t.grid_lo[i];
            d.grid_ext[i] = t.grid_hi[i] - t.grid_lo[i];
            d.grid_lof[i] = (float)t.grid_lo[i];
            d.grid_scf[i] = (float)((double)t.grid[i] / d.grid_ext[i]);
            nc *= t.grid[i];
        }
        if (nc > (int64_t(1) << 31)) return fail(DMC_E_INVALID, "snapshot grid too large");
        d.ncell = nc;
    }
    // tally block layout
    int64_t o = 0;
    if (t.n_bins > 0) {
        d.off_bins = o;
        o += (int64_t)t.n_batches * 3 * t.n_bins;
    }
    if (s.kind == DMC_SRC_GRADIENT) {
        d.off_kappa = o;
        o += 2;
        if (t.n_hj > 0) {
            d.off_hj = o;
            o += 2 * (int64_t)t.n_hj;
        }
    }
    if (transient) {
        d.off_snap = o;
        o += (int64_t)jb.n_times * (d.ncell + 1);
        d.off_snap_abs = o;
        o += (int64_t)jb.n_times * (d.ncell + 1);
        // a Gaussian initial condition gives every particle the sign of dT, so
        // sum |s| = |sum s| per cell: the device skips that second atomic
        d.snap_abs_on = (s.kind == DMC_SRC_GAUSSIAN) ? 0 : 1;
    }
    if (t.region) {
        if (!transient || t.region != 1) return fail(DMC_E_INVALID, "the region tally needs snapshot times");
        if (!finite_pos(t.region_radius) || !finite_nonneg(t.region_z[0]) || !std::isfinite(t.region_z[1]) ||
            !(t.region_z[1] > t.region_z[0]) || !std::isfinite(t.region_c[0]) || !std::isfinite(t.region_c[1]))
            return fail(DMC_E_INVALID, "region: radius > 0, 0 <= z_lo < z_hi, finite centre");
        d.off_region = o;
        o += 4 * (int64_t)jb.n_times;
        d.region_c[0] = t.region_c[0];
        d.region_c[1] = t.region_c[1];
        d.region_r = t.region_radius;
        d.region_z[0] = t.region_z[0];
        d.region_z[1] = t.region_z[1];
    }
    if (!transient && (t.grid[0] != 0 || t.grid[1] != 0 || t.grid[2] != 0)) {
        // steady x-z field over the pore cell (Eq. (4) per cell), batch replicas for the SE
        if (g.kind != DMC_GEOM_PORE_CELL_XZ)
            return fail(DMC_E_INVALID, "a steady field needs a pore-cell geometry (or set grid to 0)");
        if (t.grid[0] < 1 || t.grid[0] > 1024 || t.grid[2] < 1 || t.grid[2] > 1024 || t.grid[1] != 1)
            return fail(DMC_E_INVALID, "steady field grid must be (nx, 1, nz) with 1 <= nx, nz <= 1024");
        if (t.grid_lo[0] != 0.0 || t.grid_lo[2] != 0.0 || t.grid_hi[0] != g.length || t.grid_hi[2] != g.length)
            return fail(DMC_E_INVALID, "a steady field covers the unit cell: grid_lo x, z = 0, grid_hi x, z = period");
        for (int i = 0; i < 3; i += 2) {
            d.grid[i] = t.grid[i];
            d.grid_lo[i] = 0.0;
            d.grid_ext[i] = g.length;
            d.grid_lof[i] = 0.0f;
            d.grid_scf[i] = (float)((double)t.grid[i] / g.length);
        }
        d.grid[1] = 1;
        d.off_field = o;
        o += (int64_t)t.n_batches * 2 * t.grid[0] * t.grid[2];
    }
    if (t.n_bins > 0) {  // last: the visible block stays contiguous
        // hidden: not part of the raw block a caller reads (the host folds it into
        // the displacement bins when the launch used it)
        d.off_dispx = o;
        o += (int64_t)t.n_batches;
        h.hidden = t.n_batches;
    }
    h.size = o;
    return DMC_OK;
}

void complete_tally(const JobDev &d, double *block)
{
    if (d.off_snap_abs >= 0 && !d.snap_abs_on) {
        const int64_t n = (int64_t)d.n_times * (d.ncell + 1);
        for (int64_t i = 0; i < n; ++i) block[d.off_snap_abs + i] = std::fabs(block[d.off_snap + i]);
    }
    if (d.disp_tel && d.off_dispx >= 0 && d.off_bins >= 0) {
        // every net transmission carries one bin width through every bin
        for (int b = 0; b < d.n_batches; ++b) {
            const double x = d.bin_width * block[d.off_dispx + b];
            double *disp = block + d.off_bins + ((int64_t)b * 3 + 2) * d.n_bins;
            for (int k = 0; k < d.n_bins; ++k) disp[k] += x;
            block[d.off_dispx + b] = 0.0;
        }
    }
}

dmc_status run_opts_check(const dmc_run_opts &o)
{
    if (o.precision != DMC_PREC_FP64 && o.precision != DMC_PREC_FP32_TALLY64)
        return fail(DMC_E_INVALID, "unknown precision");
    if (o.form != DMC_FORM_PLAIN && o.form != DMC_FORM_PERSISTENT) return fail(DMC_E_INVALID, "unknown form");
    if (o.block != 0 && (o.block < 64 || o.block > 1024 || o.block % 64 != 0))
        return fail(DMC_E_INVALID, "block must be a multiple of 64 in 64..1024");
    if (o.chunk < 0 || o.refill_min < 0 || o.refill_min > 64 || o.grid_blocks < 0)
        return fail(DMC_E_INVALID, "negative chunk / refill_min / grid_blocks");
    return DMC_OK;
}

namespace {

int device_cus()
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) return 256;
    return cus;
}

}  // namespace

// ----------------------------------------------------------- launch plan ----

int kernel_spec(const JobDev *jobs, int n_jobs)
{
    bool slab = true, half = true, grad = true;
    for (int i = 0; i < n_jobs; ++i) {
        const JobDev &d = jobs[i];
        if (d.geom != GEOM_SLAB || d.src != SRC_WALLS || d.n_times > 0 || d.wall_type[0] == WALL_PERIODIC ||
            d.wall_type[1] == WALL_PERIODIC || d.kmax >= 0 || d.n_bins <= 0)
            slab = false;
        if (d.geom != GEOM_HALF || d.src != SRC_GAUSSIAN || d.n_times == 0 || d.n_bins > 0 || d.off_kappa >= 0 ||
            d.n_hj > 0)
            half = false;
        if ((d.geom != GEOM_FILM && d.geom != GEOM_PORE) || d.src != SRC_GRADIENT || d.n_times > 0 || d.n_bins > 0)
            grad = false;
    }
    return slab ? (int)GEOM_SLAB : half ? (int)GEOM_HALF : grad ? (int)GEOM_GRAD : (int)GEOM_ANY;
}

int launch_spec(const dmc_material *M, const JobDev *devs, int n_jobs)
{
    // the specialised kernels scatter isotropically: another phase function takes
    // the generic kernel
    return M->scatter_g != 0.0 ? (int)GEOM_ANY : kernel_spec(devs, n_jobs);
}

dmc_status plan_launch(const dmc_material *M, JobDev *devs, int n_jobs, const LaunchBuffers &b, const dmc_run_opts &o,
                       LaunchPlan &plan)
{
    int spec = launch_spec(M, devs, n_jobs);
    int32_t n_times_all = 0;
    for (int i = 0; i < n_jobs; ++i) n_times_all = std::max(n_times_all, devs[i].times_off + devs[i].n_times);
    const bool bounded_launch = b.drain_iters > 0 || b.n_resume > 0;
    // LDS of a persistent workgroup: gain table + per-state data, the per-job
    // counters, the sample times and the job table, then privatised tallies while
    // they fit
    const size_t tab = (((size_t)(1 << M->gain.bits) * 4 + 15) & ~size_t(15)) + (size_t)M->K * 16;
    const size_t cap = (size_t)max_lds_bytes();
    const size_t stats_lds = (n_jobs <= kLdsStatJobs) ? (size_t)n_jobs * kStats * 8 : 0;
    // persistent launches read the job table and the sample times from LDS when both
    // fit (beside the material's tables); the specialised kernels exist only in that
    // form, so larger tables take the generic kernel
    const size_t lds_tables = (size_t)n_times_all * 8 + 16 + (size_t)n_jobs * sizeof(JobDev);
    const bool jobs_lds = o.form == DMC_FORM_PERSISTENT &&
                          (size_t)n_jobs * sizeof(JobDev) <= (size_t)kLdsJobsBytes && n_times_all <= kLdsTimes &&
                          tab + stats_lds + lds_tables + 1024 <= cap;
    if (o.form == DMC_FORM_PERSISTENT && !jobs_lds) spec = GEOM_ANY;
    const bool times_lds = jobs_lds;
    KArgs a{};
    {
        const double g = M->scatter_g;
        a.scatter_g = g;
        a.hg[0] = 1.0 - g * g;
        a.hg[1] = 1.0 - g;
        a.hg[2] = 2.0 * g;
        a.hg[3] = 1.0 + g * g;
        for (int i = 0; i < 4; ++i) a.hgf[i] = (float)a.hg[i];
        a.hgf_inv2g = g != 0.0 ? (float)(1.0 / (2.0 * g)) : 0.0f;
    }
    a.jobs = b.jobs;
    a.n_jobs = n_jobs;
    a.K = M->K;
    a.qbegin = 0;
    a.total = 0;
    for (int i = 0; i < n_jobs; ++i) a.total += devs[i].n;
    a.queue = b.queue;
    a.gain_bits = M->gain.bits;
    a.flux_bits = M->flux.bits;
    a.init_bits = M->init.bits;
    a.gain_packed = M->d_gain;
    a.flux_packed = M->d_flux;
    a.init_packed = M->d_init;
    a.st32 = M->d_st32;
    a.st64 = M->d_st64;
    a.tally = b.tally;
    a.times = b.times;
    a.nscat_out = o.nscat_out;
    a.stats = b.stats;
    a.kpad = 1 << M->gain.bits;
    a.lds_stats = stats_lds > 0 ? 1 : 0;
    a.drain_iters = b.drain_iters;
    a.n_resume = b.n_resume;
    a.resume_in = b.resume_in;
    a.resume_job = b.resume_job;
    a.suspend_out = b.suspend_out;
    a.suspend_cap = b.suspend_cap;
    a.iter_cap = b.iter_cap ? std::min(b.iter_cap, kIterCap) : kIterCap;
    a.prio_flights = o.prio_flights == 0 ? 65536u
                     : o.prio_flights < 0            ? 0u
                                                     : (uint32_t)std::min<int32_t>(o.prio_flights, 1 << 27);
    a.total += b.n_resume;
    for (int i = 0; i < n_jobs; ++i)
        if (devs[i].off_region >= 0) a.any_region = 1;
    if ((b.drain_iters || b.n_resume) && o.form != DMC_FORM_PERSISTENT)
        return fail(DMC_E_INVALID, "time-bounded launches need the persistent form");
    if (b.n_resume && !b.drain_iters) return fail(DMC_E_INVALID, "resuming needs a time-bounded launch");
    a.times_lds = times_lds ? n_times_all : 0;
    a.jobs_lds = jobs_lds ? 1 : 0;
    // sample times after the counters, then the job table at a 16-byte boundary
    const size_t tail_bytes = (size_t)a.times_lds * 8 + (jobs_lds ? 16 + (size_t)n_jobs * sizeof(JobDev) : 0);
    for (int i = 0; i < n_jobs; ++i) {
        JobDev &d = devs[i];
        d.lds_bins = d.lds_kappa = d.lds_hj = d.lds_dispx = d.lds_region = d.lds_field = -1;
        d.disp_tel = (o.form == DMC_FORM_PERSISTENT && spec == GEOM_SLAB && !(b.drain_iters || b.n_resume)) ? 1 : 0;
    }
    int block = 256, grid = 1;
    size_t lds_bytes = 0;
    if (o.form == DMC_FORM_PERSISTENT) {
        if (tab + stats_lds + tail_bytes + 1024 > cap)
            return fail(DMC_E_UNSUPPORTED, "persistent form: material tables do not fit in LDS");
        const size_t budget = (cap - tab - stats_lds - tail_bytes - 16) / 8;  // doubles
        int32_t lo = 0;
        if (o.lds_tally) {
            for (int i = 0; i < n_jobs; ++i) {
                JobDev &d = devs[i];
                if (d.off_bins >= 0) {
                    const int32_t n = d.n_batches * 3 * d.n_bins;
                    if ((size_t)(lo + n) <= budget) {
                        d.lds_bins = lo;
                        lo += n;
                    }
                    if ((size_t)(lo + d.n_batches) <= budget) {
                        d.lds_dispx = lo;
                        lo += d.n_batches;
                    }
                }
                if (d.off_kappa >= 0 && (size_t)(lo + 2) <= budget) {
                    d.lds_kappa = lo;
                    lo += 2;
                }
                if (d.off_hj >= 0 && (size_t)(lo + 2 * d.n_hj) <= budget) {
                    d.lds_hj = lo;
                    lo += 2 * d.n_hj;
                }
                if (d.off_region >= 0 && (size_t)(lo + 4 * d.n_times) <= budget) {
                    d.lds_region = lo;
                    lo += 4 * d.n_times;
                }
            }
            // fields last: they are large, and the small sections of every job come first
            for (int i = 0; i < n_jobs; ++i) {
                JobDev &d = devs[i];
                if (d.off_field < 0) continue;
                const int64_t n = (int64_t)d.n_batches * 2 * d.grid[0] * d.grid[2];
                if ((size_t)(lo + n) <= budget) {
                    d.lds_field = lo;
                    lo += (int32_t)n;
                }
            }
        }
        a.lds_tally_doubles = lo;
        a.bins_lds_all = 1;
        for (int i = 0; i < n_jobs; ++i)
            if (devs[i].off_bins >= 0 && devs[i].lds_bins < 0) a.bins_lds_all = 0;
        lds_bytes = ((tab + 15) & ~size_t(15)) + (size_t)lo * 8 + stats_lds + tail_bytes;
        a.chunk = o.chunk > 0 ? o.chunk : 1024;
        a.refill_min = o.refill_min > 0 ? o.refill_min : 16;
        block = o.block > 0 ? o.block : (lds_bytes > 64 * 1024 ? 1024 : 512);
        const int per_cu = occupancy_blocks(o.precision, o.form, spec, bounded_launch, jobs_lds, block, lds_bytes);
        grid = o.grid_blocks > 0 ? o.grid_blocks : device_cus() * per_cu;
        if (b.drain_iters) {
            // every lane may suspend one particle and every wave the unstarted rest of
            // its chunk: chunks are capped at one index per lane
            a.chunk = std::min(a.chunk, 64);
            const uint32_t per_block = (uint32_t)block + (uint32_t)(block / 64) * (uint32_t)a.chunk;
            const int max_grid = (int)(b.suspend_cap / per_block);
            if (max_grid < 1) return fail(DMC_E_INVALID, "suspend buffer smaller than one workgroup");
            grid = std::min(grid, max_grid);
        }
    } else {
        a.lds_tally_doubles = 0;
        a.chunk = 0;
        a.refill_min = 64;
        lds_bytes = stats_lds;
    }
    plan.a = a;
    plan.material = M;
    plan.spec = spec;
    plan.block = block;
    plan.grid = grid;
    plan.lds_bytes = lds_bytes;
    return DMC_OK;
}

dmc_status submit_launch(const LaunchPlan &plan, const JobDev *devs, int n_jobs, const dmc_run_opts &o, hipStream_t s)
{
    if (o.form == DMC_FORM_PERSISTENT) {
        DMC_HIP_OR_FAIL(launch_trajectories(plan.a, o.precision, o.form, plan.spec, plan.block, plan.grid,
                                            plan.lds_bytes, s));
    } else {
        // one launch per simulation, in order, on the same stream
        for (int i = 0; i < n_jobs; ++i) {
            KArgs aj = plan.a;
            aj.qbegin = devs[i].base;
            aj.total = devs[i].base + devs[i].n;
            const uint64_t blocks = (devs[i].n + 255) / 256;
            if (blocks > 0x7fffffffull) return fail(DMC_E_INVALID, "too many particles for one plain launch");
            DMC_HIP_OR_FAIL(launch_trajectories(aj, o.precision, o.form, launch_spec(plan.material, &devs[i], 1), 256,
                                                (int)blocks, plan.lds_bytes, s));
        }
    }
    return DMC_OK;
}

dmc_status enqueue_launch(const dmc_material *M, std::vector<JobDev> &devs, const std::vector<double> &times,
                          std::vector<JobDev> &table, const LaunchBuffers &b, size_t tally_doubles, bool zero_tally,
                          const dmc_run_opts &o, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1)
{
    const int n_jobs = (int)devs.size();
    LaunchPlan plan;
    dmc_status st = plan_launch(M, devs.data(), n_jobs, b, o, plan);
    if (st != DMC_OK) return st;
    // the device table is ordered by queue position (the kernels search it by base)
    table = devs;
    std::stable_sort(table.begin(), table.end(), [](const JobDev &x, const JobDev &y) { return x.base < y.base; });
    DMC_HIP_OR_FAIL(hipMemcpyAsync(b.jobs, table.data(), table.size() * sizeof(JobDev), hipMemcpyHostToDevice, s));
    if (!times.empty())
        DMC_HIP_OR_FAIL(hipMemcpyAsync(b.times, times.data(), times.size() * sizeof(double), hipMemcpyHostToDevice, s));
    DMC_HIP_OR_FAIL(launch_fill(zero_tally ? b.tally : nullptr, zero_tally ? tally_doubles : 0, b.stats,
                                (size_t)n_jobs * kStats, s));
    DMC_HIP_OR_FAIL(launch_fill(nullptr, 0, b.queue, 2, s));
    DMC_HIP_OR_FAIL(hipEventRecord(ev0, s));
    st = submit_launch(plan, devs.data(), n_jobs, o, s);
    if (st != DMC_OK) return st;
    DMC_HIP_OR_FAIL(hipEventRecord(ev1, s));
    return DMC_OK;
}

}  // namespace dmc

extern "C" void dmc_run_opts_default(dmc_run_opts *o)
{
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->precision = DMC_PREC_FP32_TALLY64;
    o->form = DMC_FORM_PERSISTENT;
    o->lds_tally = 1;
}

namespace dmc {

struct Layout {
    size_t jobs_off, times_off, tally_off, stats_off, queue_off, total;
    size_t tally_doubles, n_times;
};

Layout layout_of(const std::vector<JobHost> &jh)
{
    Layout L{};
    size_t o = 0;
    L.jobs_off = o;
    o = align256(o + jh.size() * sizeof(JobDev));
    L.n_times = 0;
    for (auto &h : jh) L.n_times += h.times.size();
    L.times_off = o;
    o = align256(o + std::max<size_t>(L.n_times, 1) * sizeof(double));
    L.tally_doubles = 0;
    for (auto &h : jh) L.tally_doubles += (size_t)h.size;
    L.tally_off = o;
    o = align256(o + std::max<size_t>(L.tally_doubles, 1) * sizeof(double));
    L.stats_off = o;
    o = align256(o + jh.size() * kStats * sizeof(unsigned long long));
    L.queue_off = o;
    o = align256(o + 2 * sizeof(unsigned long long));
    L.total = o;
    return L;
}

// Expected flights per particle, used to queue the longest trajectories first:
// trajectory lengths are heavy-tailed, and the longest single particle bounds
// a launch's duration unless it starts early.
static double expected_flights(const dmc_material &M, const JobDev &d, double length, double t_final)
{
    if (d.src == SRC_WALLS) return 2.0 * length * M.G_tau / M.G_v + 1.0;
    if (d.src == SRC_GAUSSIAN) return t_final * M.G_tau / M.C_tot + 1.0;
    return d.kmax >= 0 ? 1.5 * d.kmax + 1.0 : 1000.0;
}

double flights_per_particle(const dmc_material &M, const JobHost &h)
{
    return expected_flights(M, h.dev, h.geom.length, h.times.empty() ? 0.0 : h.times.back());
}

// Flights of the longest trajectory a gradient job is likely to hold, when one
// free path sets it: the source emits states with weight C v, and a free path
// of mean length Lambda crosses a film or pore cell of size l about Lambda / l
// times, each crossing or wall hit being one flight.  Among N particles the
// longest free path is drawn from about the states whose emission weight above
// it is 1/N (the material keeps its free paths sorted with the running sum of
// C v).  Jobs with such a tail go first, so that it runs beside the bulk of the
// launch rather than after it.
static double longest_flights(const dmc_material &M, const JobDev &d, double cell)
{
    if (d.src != SRC_GRADIENT || !(cell > 0.0) || d.n == 0) return 0.0;
    const double target = M.G_v / (double)d.n;
    const auto it = std::lower_bound(M.cv_cum.begin(), M.cv_cum.end(), target);
    if (it == M.cv_cum.end()) return 0.0;
    return M.lam_desc[(size_t)(it - M.cv_cum.begin())] / cell;
}

void queue_order(const dmc_material &M, const JobDev *devs, const double *length, const double *t_final, int n_jobs,
                 int *rank, double *key)
{
    for (int i = 0; i < n_jobs; ++i) {
        key[i] = std::max(expected_flights(M, devs[i], length[i], t_final[i]), longest_flights(M, devs[i], length[i]));
        rank[i] = i;
    }
    // stable insertion sort, descending key (a batch holds at most a few thousand jobs)
    for (int i = 1; i < n_jobs; ++i) {
        const int v = rank[i];
        int p = i - 1;
        while (p >= 0 && key[rank[p]] < key[v]) {
            rank[p + 1] = rank[p];
            --p;
        }
        rank[p + 1] = v;
    }
}

void assign_offsets(JobDev *devs, const int64_t *size, const int32_t *n_times, const int *rank, int n_jobs)
{
    uint64_t base = 0;
    for (int r = 0; r < n_jobs; ++r) {
        JobDev &d = devs[rank[r]];
        d.base = base;
        base += d.n;
    }
    int64_t toff = 0, tim = 0;
    uint64_t out = 0;
    for (int i = 0; i < n_jobs; ++i) {
        JobDev &d = devs[i];
        d.stat_slot = i;
        d.out_off = out;
        out += d.n;
        if (d.off_bins >= 0) d.off_bins += toff;
        if (d.off_kappa >= 0) d.off_kappa += toff;
        if (d.off_hj >= 0) d.off_hj += toff;
        if (d.off_snap >= 0) d.off_snap += toff;
        if (d.off_snap_abs >= 0) d.off_snap_abs += toff;
        if (d.off_dispx >= 0) d.off_dispx += toff;
        if (d.off_region >= 0) d.off_region += toff;
        if (d.off_field >= 0) d.off_field += toff;
        toff += size[i];
        d.times_off = (int32_t)tim;
        tim += n_times[i];
    }
}

dmc_status gather_jobs(const dmc_job *jobs, int32_t n_jobs, std::vector<JobHost> &jh)
{
    if (!jobs || n_jobs < 1 || n_jobs > kMaxJobs) return fail(DMC_E_INVALID, "n_jobs must be 1..4096");
    jh.resize(n_jobs);
    const dmc_material *M = jobs[0].material;
    uint64_t total = 0;
    for (int i = 0; i < n_jobs; ++i) {
        if (jobs[i].material != M) return fail(DMC_E_INVALID, "all jobs of a launch must share one material");
        dmc_status st = prepare_job(jobs[i], jh[i]);
        if (st != DMC_OK) return st;
        if (total + jh[i].dev.n < total) return fail(DMC_E_INVALID, "particle count overflow");
        total += jh[i].dev.n;
    }
    std::vector<JobDev> devs(n_jobs);
    std::vector<double> len(n_jobs), tf(n_jobs), key(n_jobs);
    std::vector<int64_t> size(n_jobs);
    std::vector<int32_t> nt(n_jobs);
    std::vector<int> rank(n_jobs);
    for (int i = 0; i < n_jobs; ++i) {
        devs[i] = jh[i].dev;
        len[i] = jh[i].geom.length;
        tf[i] = jh[i].times.empty() ? 0.0 : jh[i].times.back();
        size[i] = jh[i].size;
        nt[i] = (int32_t)jh[i].times.size();
    }
    queue_order(*M, devs.data(), len.data(), tf.data(), n_jobs, rank.data(), key.data());
    assign_offsets(devs.data(), size.data(), nt.data(), rank.data(), n_jobs);
    for (int i = 0; i < n_jobs; ++i) jh[i].dev = devs[i];
    return DMC_OK;
}

dmc_status launch(std::vector<JobHost> &jh, const dmc_run_opts &o, dmc_result **out, uint32_t iter_cap)
{
    *out = nullptr;
    const dmc_material *M = jh[0].job.material;
    int dev = 0;
    HIP_OR_FAIL(hipGetDevice(&dev));
    if (dev != M->device) return fail(DMC_E_INVALID, "material was created on another device");
    std::unique_ptr<dmc_result> R(new (std::nothrow) dmc_result());
    if (!R) return fail(DMC_E_NOMEM, "host allocation failed");
    R->mat = M;
    R->stream = (hipStream_t)o.stream;
    const Layout L = layout_of(jh);
    char *base = nullptr;
    if (o.workspace) {
        if (o.workspace_bytes < L.total)
            return fail(DMC_E_NOMEM, "workspace too small: need " + std::to_string(L.total) + " bytes");
        if (((uintptr_t)o.workspace) % 256 != 0) return fail(DMC_E_INVALID, "workspace must be 256-byte aligned");
        base = (char *)o.workspace;
    } else {
        if (hipMalloc(&R->dev_mem, L.total) != hipSuccess) {
            (void)hipGetLastError();
            R->dev_mem = nullptr;
            return fail(DMC_E_NOMEM, "hipMalloc of " + std::to_string(L.total) + " bytes failed");
        }
        base = (char *)R->dev_mem;
    }
    LaunchBuffers b;
    b.jobs = (JobDev *)(base + L.jobs_off);
    b.times = (double *)(base + L.times_off);
    b.tally = (double *)(base + L.tally_off);
    b.stats = (unsigned long long *)(base + L.stats_off);
    b.queue = (unsigned long long *)(base + L.queue_off);
    b.iter_cap = iter_cap;
    R->d_tally = b.tally;
    R->d_stats = b.stats;
    R->tally_doubles = L.tally_doubles;
    std::vector<JobDev> devs(jh.size());
    std::vector<double> &times = R->h_times;
    for (size_t i = 0; i < jh.size(); ++i) {
        devs[i] = jh[i].dev;
        times.insert(times.end(), jh[i].times.begin(), jh[i].times.end());
    }
    HIP_OR_FAIL(hipEventCreate(&R->ev0));
    HIP_OR_FAIL(hipEventCreate(&R->ev1));
    dmc_status st =
        enqueue_launch(M, devs, times, R->h_table, b, L.tally_doubles, true, o, R->stream, R->ev0, R->ev1);
    if (st != DMC_OK) {
        (void)hipStreamSynchronize(R->stream);
        return st;
    }
    for (size_t i = 0; i < jh.size(); ++i) jh[i].dev = devs[i];
    R->jobs = std::move(jh);
    *out = R.release();
    return DMC_OK;
}

size_t workspace_bytes(const std::vector<JobHost> &jh) { return layout_of(jh).total; }

dmc_status sync_result(dmc_result *R)
{
    if (R->synced) return DMC_OK;
    HIP_OR_FAIL(hipEventSynchronize(R->ev1));
    float ms = 0.0f;
    HIP_OR_FAIL(hipEventElapsedTime(&ms, R->ev0, R->ev1));
    R->kernel_ms = ms;
    R->h_tally.assign(std::max<size_t>(R->tally_doubles, 1), 0.0);
    HIP_OR_FAIL(hipMemcpy(R->h_tally.data(), R->d_tally, R->tally_doubles * sizeof(double), hipMemcpyDeviceToHost));
    for (const auto &h : R->jobs) complete_tally(h.dev, R->h_tally.data());
    R->h_stats.assign(R->jobs.size() * kStats, 0ull);
    HIP_OR_FAIL(hipMemcpy(R->h_stats.data(), R->d_stats, R->h_stats.size() * sizeof(unsigned long long),
                          hipMemcpyDeviceToHost));
    R->synced = true;
    return DMC_OK;
}

}  // namespace dmc

extern "C" dmc_status dmc_workspace_size(const dmc_job *jobs, int32_t n_jobs, const dmc_run_opts *opts, size_t *bytes)
{
    if (!bytes) return fail(DMC_E_INVALID, "bytes is NULL");
    *bytes = 0;
    std::vector<JobHost> jh;
    dmc_status st = gather_jobs(jobs, n_jobs, jh);
    if (st != DMC_OK) return st;
    *bytes = workspace_bytes(jh);
    (void)opts;
    return DMC_OK;
}

// ------------------------------------------------------------------- C ABI ----

extern "C" const char *dmc_last_error(void) { return dmc::g_err.c_str(); }
extern "C" const char *dmc_version(void) { return "dmc 0.1 gfx950"; }

extern "C" dmc_status dmc_material_create(const dmc_branch *br, int32_t nbr, double T_eq, double scatter_g,
                                         dmc_material **out)
{
    if (!out) return fail(DMC_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!br || nbr < 1) return fail(DMC_E_INVALID, "need at least one branch");
    if (!finite_pos(T_eq)) return fail(DMC_E_INVALID, "T_eq must be positive");
    if (!(scatter_g > -1.0 && scatter_g < 1.0)) return fail(DMC_E_INVALID, "scatter_g must lie in (-1, 1)");
    std::unique_ptr<dmc_material> M(new (std::nothrow) dmc_material());
    if (!M) return fail(DMC_E_NOMEM, "host allocation failed");
    M->T_eq = T_eq;
    M->scatter_g = scatter_g;
    std::vector<double> wg, wi, wf;
    for (int b = 0; b < nbr; ++b) {
        const dmc_branch &B = br[b];
        if (B.n_bins < 1 || !B.omega || !B.domega || !B.dos || !B.vg || !B.tau)
            return fail(DMC_E_INVALID, "branch " + std::to_string(b) + " is empty or has NULL arrays");
        if (!finite_nonneg(B.degeneracy)) return fail(DMC_E_INVALID, "bad degeneracy");
        for (int i = 0; i < B.n_bins; ++i) {
            if (!finite_pos(B.omega[i]) || !finite_nonneg(B.domega[i]) || !finite_nonneg(B.dos[i]) ||
                !finite_pos(B.vg[i]) || !finite_pos(B.tau[i]))
                return fail(DMC_E_INVALID, "branch " + std::to_string(b) + " bin " + std::to_string(i) +
                                               " has a non-physical value");
            // de^eq/dT of hbar w / (exp(hbar w / k_B T) - 1), then C = D de/dT dw g
            const double x = (kHbar * B.omega[i]) / (kBoltz * T_eq);
            const double ex = std::exp(x);
            const double em1 = std::expm1(x);
            const double dedT = kBoltz * x * x * ex / (em1 * em1);
            const double C = ((B.dos[i] * dedT) * B.domega[i]) * B.degeneracy;
            M->v.push_back(B.vg[i]);
            M->tau.push_back(B.tau[i]);
            M->C.push_back(C);
            M->C_tot += C;
            M->G_tau += C / B.tau[i];
            M->G_v += C * B.vg[i];
            wg.push_back(C / B.tau[i]);
            wi.push_back(C);
            wf.push_back(C * B.vg[i]);
        }
    }
    M->K = (int32_t)M->v.size();
    if (M->K > 65536) return fail(DMC_E_INVALID, "more than 65536 states");
    {
        // free paths in descending order with the running sum of the wall-flux weight C v
        // (the longest trajectory a batch job is likely to hold, see longest_flights)
        std::vector<std::pair<double, double>> lw(M->K);
        for (int m = 0; m < M->K; ++m) lw[m] = {M->v[m] * M->tau[m], M->C[m] * M->v[m]};
        std::sort(lw.begin(), lw.end(), [](const auto &x, const auto &y) { return x.first > y.first; });
        double cum = 0.0;
        for (const auto &e : lw) {
            cum += e.second;
            M->lam_desc.push_back(e.first);
            M->cv_cum.push_back(cum);
        }
    }
    std::string why;
    if (!build_alias(wg, M->gain, why) || !build_alias(wi, M->init, why) || !build_alias(wf, M->flux, why))
        return fail(DMC_E_INVALID, "material: " + why);
    HIP_OR_FAIL(hipGetDevice(&M->device));
    std::vector<float4> s32(M->K);
    std::vector<double2> s64(M->K);
    for (int m = 0; m < M->K; ++m) {
        // v, tau, 1/tau and -tau ln 2 (the flight time is -tau ln2 log2 u)
        s32[m] = make_float4((float)M->v[m], (float)M->tau[m], (float)(1.0 / M->tau[m]),
                             (float)(-M->tau[m] * 0.69314718055994530942));
        s64[m] = make_double2(M->v[m], M->tau[m]);
    }
    auto up = [&](void **dst, const void *src, size_t bytes) -> dmc_status {
        if (hipMalloc(dst, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return fail(DMC_E_NOMEM, "hipMalloc failed");
        }
        HIP_OR_FAIL(hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice));
        return DMC_OK;
    };
    dmc_status st;
    if ((st = up((void **)&M->d_gain, M->gain.packed.data(), M->gain.packed.size() * 4)) != DMC_OK) return st;
    if ((st = up((void **)&M->d_init, M->init.packed.data(), M->init.packed.size() * 4)) != DMC_OK) return st;
    if ((st = up((void **)&M->d_flux, M->flux.packed.data(), M->flux.packed.size() * 4)) != DMC_OK) return st;
    if ((st = up((void **)&M->d_st32, s32.data(), s32.size() * sizeof(float4))) != DMC_OK) return st;
    if ((st = up((void **)&M->d_st64, s64.data(), s64.size() * sizeof(double2))) != DMC_OK) return st;
    *out = M.release();
    return DMC_OK;
}

extern "C" dmc_status dmc_material_destroy(dmc_material *m)
{
    delete m;
    return DMC_OK;
}

extern "C" dmc_status dmc_material_info(const dmc_material *m, int32_t *n_states, double sums[3])
{
    if (!m) return fail(DMC_E_INVALID, "material is NULL");
    if (n_states) *n_states = m->K;
    if (sums) {
        sums[0] = m->C_tot;
        sums[1] = m->G_tau;
        sums[2] = m->G_v;
    }
    return DMC_OK;
}

extern "C" dmc_status dmc_geometry_create(const dmc_geometry_desc *d, dmc_geometry **out)
{
    if (!out) return fail(DMC_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!d) return fail(DMC_E_INVALID, "desc is NULL");
    if (d->kind < DMC_GEOM_SLAB_Z || d->kind > DMC_GEOM_HALFSPACE_Z) return fail(DMC_E_INVALID, "unknown geometry");
    if (d->kind != DMC_GEOM_HALFSPACE_Z && !finite_pos(d->length)) return fail(DMC_E_INVALID, "length must be > 0");
    if (d->kind == DMC_GEOM_PORE_CELL_XZ && !(finite_nonneg(d->radius) && d->radius < 0.5 * d->length))
        return fail(DMC_E_INVALID, "pore radius must be in [0, length/2)");
    const int nw = (d->kind == DMC_GEOM_SLAB_Z || d->kind == DMC_GEOM_FILM_X) ? 2 : 1;
    for (int i = 0; i < nw; ++i) {
        const dmc_wall &w = d->wall[i];
        if (w.type < DMC_WALL_ISOTHERMAL || w.type > DMC_WALL_PERIODIC) return fail(DMC_E_INVALID, "unknown wall type");
        if (w.type == DMC_WALL_ADIABATIC && !(w.specularity >= 0.0 && w.specularity <= 1.0))
            return fail(DMC_E_INVALID, "specularity must be in [0, 1]");
        if (w.type == DMC_WALL_ISOTHERMAL && !finite_pos(w.temperature))
            return fail(DMC_E_INVALID, "isothermal wall temperature must be > 0");
        if (w.type == DMC_WALL_PERIODIC && nw != 2) return fail(DMC_E_INVALID, "periodic walls need a plane pair");
        if (w.type != DMC_WALL_ADIABATIC && nw == 1) return fail(DMC_E_INVALID, "pore / half-space surface must be adiabatic");
    }
    if (nw == 2 && ((d->wall[0].type == DMC_WALL_PERIODIC) != (d->wall[1].type == DMC_WALL_PERIODIC)))
        return fail(DMC_E_INVALID, "periodic walls come in pairs");
    dmc_geometry *g = new (std::nothrow) dmc_geometry();
    if (!g) return fail(DMC_E_NOMEM, "host allocation failed");
    g->d = *d;
    if (nw == 1) g->d.wall[1] = g->d.wall[0];
    *out = g;
    return DMC_OK;
}

extern "C" dmc_status dmc_geometry_destroy(dmc_geometry *g)
{
    delete g;
    return DMC_OK;
}

extern "C" dmc_status dmc_simulate_batch(const dmc_job *jobs, int32_t n_jobs, const dmc_run_opts *opts,
                                         dmc_result **out)
{
    if (!out) return fail(DMC_E_INVALID, "out is NULL");
    *out = nullptr;
    dmc_run_opts o;
    if (opts)
        o = *opts;
    else
        dmc_run_opts_default(&o);
    dmc_status st = run_opts_check(o);
    if (st != DMC_OK) return st;
    std::vector<JobHost> jh;
    if ((st = gather_jobs(jobs, n_jobs, jh)) != DMC_OK) return st;
    if (o.nscat_out) {
        uint64_t total = 0;
        for (const auto &h : jh) total += h.dev.n;
        if (o.nscat_out_len < total)
            return fail(DMC_E_INVALID, "nscat_out holds " + std::to_string(o.nscat_out_len) + " entries, the launch has " +
                                           std::to_string(total) + " particles");
    }
    return launch(jh, o, out);
}

extern "C" dmc_status dmc_simulate(const dmc_material *material, const dmc_geometry *geometry,
                                   const dmc_source *source, uint64_t n_particles, uint64_t seed,
                                   const dmc_tally_desc *tally, const double *times, int32_t n_times,
                                   const dmc_run_opts *opts, dmc_result **out)
{
    if (!source || !tally) {
        if (out) *out = nullptr;
        return fail(DMC_E_INVALID, "source / tally is NULL");
    }
    dmc_job j{};
    j.material = material;
    j.geometry = geometry;
    j.source = *source;
    j.tally = *tally;
    j.n_particles = n_particles;
    j.seed = seed;
    j.times = times;
    j.n_times = n_times;
    return dmc_simulate_batch(&j, 1, opts, out);
}

extern "C" dmc_status dmc_tally_raw_size(const dmc_result *res, int32_t job, size_t *n)
{
    if (!res || !n || job < 0 || job >= (int32_t)res->jobs.size()) return fail(DMC_E_INVALID, "bad result / job");
    *n = (size_t)(res->jobs[job].size - res->jobs[job].hidden);
    return DMC_OK;
}

extern "C" dmc_status dmc_tally_read(const dmc_result *cres, int32_t job, int32_t q, int32_t time_index, double *mean,
                                     double *se, size_t n)
{
    dmc_result *R = const_cast<dmc_result *>(cres);
    if (!R || !mean || job < 0 || job >= (int32_t)R->jobs.size()) return fail(DMC_E_INVALID, "bad result / job");
    dmc_status st = sync_result(R);
    if (st != DMC_OK) return st;
    const JobHost &h = R->jobs[job];
    const JobDev &d = h.dev;
    const dmc_material &M = *R->mat;
    const double N = (double)d.n;
    // all offsets are relative to the launch's tally buffer
    const double *T = R->h_tally.data();
    if (q == DMC_Q_T || q == DMC_Q_TLOC || q == DMC_Q_FLUX) {
        if (d.off_bins < 0) return fail(DMC_E_INVALID, "no bins tallied");
        if (n < (size_t)d.n_bins) return fail(DMC_E_INVALID, "output too small");
        const int qi = q == DMC_Q_T ? 0 : (q == DMC_Q_TLOC ? 1 : 2);
        const double dz = h.geom.length / d.n_bins;
        const double norm = (qi == 0 ? 1.0 / M.C_tot : (qi == 1 ? 1.0 / M.G_tau : 1.0)) * h.power / dz;
        const int B = d.n_batches;
        for (int k = 0; k < d.n_bins; ++k) {
            double tot = 0.0;
            std::vector<double> per;
            for (int b = 0; b < B; ++b) {
                const double v = T[d.off_bins + ((int64_t)b * 3 + qi) * d.n_bins + k];
                tot += v;
                const double nb = (d.n > (uint64_t)b) ? (double)((d.n - b + B - 1) / B) : 0.0;
                if (nb > 0) per.push_back(v * norm / nb);
            }
            mean[k] = tot * norm / N;
            if (se) {
                const size_t m = per.size();
                if (m < 2) {
                    se[k] = NAN;
                } else {
                    double mu = 0.0;
                    for (double x : per) mu += x;
                    mu /= (double)m;
                    double var = 0.0;
                    for (double x : per) var += (x - mu) * (x - mu);
                    var /= (double)(m - 1);
                    se[k] = std::sqrt(var / (double)m);
                }
            }
        }
        return DMC_OK;
    }
    if (q == DMC_Q_KAPPA || q == DMC_Q_HJ) {
        if (d.off_kappa < 0) return fail(DMC_E_INVALID, "conductivity needs a gradient source");
        const double f = h.power / (h.avg_volume * h.job.source.gradient);
        auto one = [&](double s1, double s2, double *m_out, double *se_out) {
            const double m = s1 / N;
            const double var = std::max(s2 / N - m * m, 0.0);
            *m_out = -f * m;
            if (se_out) *se_out = std::fabs(f) * std::sqrt(var / std::max(N - 1.0, 1.0));
        };
        if (q == DMC_Q_KAPPA) {
            if (n < 1) return fail(DMC_E_INVALID, "output too small");
            one(T[d.off_kappa], T[d.off_kappa + 1], mean, se);
            return DMC_OK;
        }
        if (d.off_hj < 0) return fail(DMC_E_INVALID, "H_j not tallied");
        if (n < (size_t)d.n_hj) return fail(DMC_E_INVALID, "output too small");
        for (int j = 0; j < d.n_hj; ++j) one(T[d.off_hj + j], T[d.off_hj + d.n_hj + j], mean + j, se ? se + j : nullptr);
        return DMC_OK;
    }
    if (q == DMC_Q_SNAPSHOT || q == DMC_Q_SNAPSHOT_SUM) {
        if (d.off_snap < 0) return fail(DMC_E_INVALID, "no snapshots tallied");
        if (time_index < 0 || time_index >= d.n_times) return fail(DMC_E_INVALID, "time_index out of range");
        const int64_t nc = d.ncell;
        const double *S = T + d.off_snap + (int64_t)time_index * (nc + 1);
        const double *A = T + d.off_snap_abs + (int64_t)time_index * (nc + 1);
        if (q == DMC_Q_SNAPSHOT_SUM) {
            if (n < (size_t)(nc + 1)) return fail(DMC_E_INVALID, "output too small");
            for (int64_t c = 0; c <= nc; ++c) {
                mean[c] = S[c];
                if (se) se[c] = A[c];
            }
            return DMC_OK;
        }
        if (n < (size_t)nc) return fail(DMC_E_INVALID, "output too small");
        double vcell = 1.0;
        for (int i = 0; i < 3; ++i) vcell *= d.grid_ext[i] / d.grid[i];
        const double e_eff = h.power / N;
        const double sc = e_eff / (vcell * M.C_tot);
        for (int64_t c = 0; c < nc; ++c) {
            mean[c] = sc * S[c];
            if (se) {
                const double m = S[c] / N;
                const double var = std::max(A[c] / N - m * m, 0.0);
                se[c] = sc * std::sqrt(N * var);
            }
        }
        return DMC_OK;
    }
    if (q == DMC_Q_REGION_T || q == DMC_Q_REGION_QZ) {
        // time average over window [t_{j-1}, t_j): E_eff sum_i s_i (time in R) / (T_w mu(R) C_tot),
        // z heat flux E_eff sum_i s_i (z length in R) / (T_w mu(R)); per-particle moments for the SE
        if (d.off_region < 0) return fail(DMC_E_INVALID, "no region tallied");
        if (n < (size_t)d.n_times) return fail(DMC_E_INVALID, "output too small");
        const double mu = M_PI * d.region_r * d.region_r * (d.region_z[1] - d.region_z[0]);
        const double e_eff = h.power / N;
        const int col = (q == DMC_Q_REGION_T) ? 0 : 2;
        const double den = (q == DMC_Q_REGION_T) ? mu * M.C_tot : mu;
        double w0 = 0.0;
        for (int j = 0; j < d.n_times; ++j) {
            const double tw = h.times[j] - w0;
            w0 = h.times[j];
            const double s1 = T[d.off_region + 4 * j + col], s2 = T[d.off_region + 4 * j + col + 1];
            mean[j] = e_eff * s1 / (tw * den);
            if (se) {
                const double m = s1 / N;
                const double var = std::max(s2 / N - m * m, 0.0) * N / std::max(N - 1.0, 1.0);
                se[j] = e_eff * std::sqrt(N * var) / (tw * den);
            }
        }
        return DMC_OK;
    }
    if (q == DMC_Q_FIELD_T || q == DMC_Q_FIELD_QZ) {
        // E_dot sum(s t_c) / (A_c C_tot) and E_dot sum(s v Omega_z t_c) / A_c per unit length
        // along y, A_c the whole cell area; batch means for the SE
        if (d.off_field < 0) return fail(DMC_E_INVALID, "no field tallied");
        const int nx = d.grid[0], nz = d.grid[2];
        const int64_t nc = (int64_t)nx * nz;
        if (n < (size_t)nc) return fail(DMC_E_INVALID, "output too small");
        const int qi = (q == DMC_Q_FIELD_T) ? 0 : 1;
        const double area = (d.grid_ext[0] / nx) * (d.grid_ext[2] / nz);
        const double norm = h.power / (qi == 0 ? area * M.C_tot : area);
        const int B = d.n_batches;
        for (int64_t c = 0; c < nc; ++c) {
            double tot = 0.0;
            std::vector<double> per;
            for (int b = 0; b < B; ++b) {
                const double v = T[d.off_field + ((int64_t)b * 2 + qi) * nc + c];
                tot += v;
                const double nb = (d.n > (uint64_t)b) ? (double)((d.n - b + B - 1) / B) : 0.0;
                if (nb > 0) per.push_back(v * norm / nb);
            }
            mean[c] = tot * norm / N;
            if (se) {
                const size_t m = per.size();
                if (m < 2) {
                    se[c] = NAN;
                } else {
                    double mu = 0.0;
                    for (double x : per) mu += x;
                    mu /= (double)m;
                    double var = 0.0;
                    for (double x : per) var += (x - mu) * (x - mu);
                    var /= (double)(m - 1);
                    se[c] = std::sqrt(var / (double)m);
                }
            }
        }
        return DMC_OK;
    }
    if (q == DMC_Q_RAW) {
        const size_t visible = (size_t)(h.size - h.hidden);
        if (n < visible) return fail(DMC_E_INVALID, "output too small");
        const int64_t first = (d.off_bins >= 0)    ? d.off_bins
                              : (d.off_kappa >= 0) ? d.off_kappa
                              : (d.off_snap >= 0)  ? d.off_snap
                                                   : -1;
        if (first >= 0) std::memcpy(mean, T + first, visible * sizeof(double));
        return DMC_OK;
    }
    return fail(DMC_E_INVALID, "unknown quantity");
}

extern "C" dmc_status dmc_result_stats(const dmc_result *cres, int32_t job, dmc_stats *out)
{
    dmc_result *R = const_cast<dmc_result *>(cres);
    if (!R || !out || job < -1 || job >= (int32_t)R->jobs.size()) return fail(DMC_E_INVALID, "bad result / job");
    dmc_status st = sync_result(R);
    if (st != DMC_OK) return st;
    std::memset(out, 0, sizeof(*out));
    const int j0 = job < 0 ? 0 : job, j1 = job < 0 ? (int)R->jobs.size() : job + 1;
    for (int j = j0; j < j1; ++j) {
        const unsigned long long *s = R->h_stats.data() + (size_t)j * kStats;
        out->particles += s[0];
        out->scatters += s[1];
        out->boundary += s[2];
        out->iterations += s[3];
        out->capped += s[4];
        out->flights += s[6];
    }
    out->kernel_ms = R->kernel_ms;
    return DMC_OK;
}

extern "C" dmc_status dmc_result_destroy(dmc_result *res)
{
    if (res && !res->synced && res->ev1) (void)hipEventSynchronize(res->ev1);
    delete res;
    return DMC_OK;
}

// ---------------------------------------------------------------- test hooks ----

extern "C" dmc_status dmc_debug_philox(uint64_t seed, const uint64_t *pid, const uint32_t *k, const uint32_t *tag,
                                       uint32_t *out, size_t n)
{
    if (!pid || !k || !tag || !out) return fail(DMC_E_INVALID, "NULL argument");
    if (n == 0) return DMC_OK;
    uint64_t *dp = nullptr;
    uint32_t *dk = nullptr, *dt = nullptr, *dout = nullptr;
    auto cleanup = [&]() {
        (void)hipFree(dp);
        (void)hipFree(dk);
        (void)hipFree(dt);
        (void)hipFree(dout);
    };
    if (hipMalloc(&dp, n * 8) != hipSuccess || hipMalloc(&dk, n * 4) != hipSuccess || hipMalloc(&dt, n * 4) != hipSuccess ||
        hipMalloc(&dout, n * 16) != hipSuccess) {
        cleanup();
        return fail(DMC_E_NOMEM, "hipMalloc failed");
    }
    hipError_t e = hipMemcpy(dp, pid, n * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dk, k, n * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dt, tag, n * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_debug_philox(seed, dp, dk, dt, dout, n, nullptr);
    if (e == hipSuccess) e = hipMemcpy(out, dout, n * 16, hipMemcpyDeviceToHost);
    cleanup();
    if (e != hipSuccess) return fail(DMC_E_DEVICE, hipGetErrorString(e));
    return DMC_OK;
}

namespace {
const AliasTable *table_of(const dmc_material *m, int32_t which, const uint32_t **dev)
{
    if (which == DMC_TABLE_GAIN) {
        *dev = m->d_gain;
        return &m->gain;
    }
    if (which == DMC_TABLE_INIT) {
        *dev = m->d_init;
        return &m->init;
    }
    if (which == DMC_TABLE_FLUX) {
        *dev = m->d_flux;
        return &m->flux;
    }
    return nullptr;
}
}  // namespace

extern "C" dmc_status dmc_debug_alias(const dmc_material *m, int32_t which, int32_t *bits, uint32_t *thresh,
                                      uint32_t *alias, size_t n)
{
    if (!m) return fail(DMC_E_INVALID, "material is NULL");
    const uint32_t *dev;
    const AliasTable *t = table_of(m, which, &dev);
    if (!t) return fail(DMC_E_INVALID, "unknown table");
    if (bits) *bits = t->bits;
    const size_t cols = t->thresh.size();
    if ((thresh || alias) && n < cols) return fail(DMC_E_INVALID, "output too small");
    if (thresh) std::memcpy(thresh, t->thresh.data(), cols * 4);
    if (alias) std::memcpy(alias, t->alias.data(), cols * 4);
    return DMC_OK;
}

extern "C" dmc_status dmc_debug_alias_draw(const dmc_material *m, int32_t which, const uint32_t *words,
                                           uint32_t *states, size_t n)
{
    if (!m || !words || !states) return fail(DMC_E_INVALID, "NULL argument");
    const uint32_t *dev;
    const AliasTable *t = table_of(m, which, &dev);
    if (!t) return fail(DMC_E_INVALID, "unknown table");
    if (n == 0) return DMC_OK;
    uint32_t *dw = nullptr, *ds = nullptr;
    if (hipMalloc(&dw, n * 4) != hipSuccess || hipMalloc(&ds, n * 4) != hipSuccess) {
        (void)hipFree(dw);
        (void)hipFree(ds);
        return fail(DMC_E_NOMEM, "hipMalloc failed");
    }
    hipError_t e = hipMemcpy(dw, words, n * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_debug_alias(dev, t->bits, dw, ds, n, nullptr);
    if (e == hipSuccess) e = hipMemcpy(states, ds, n * 4, hipMemcpyDeviceToHost);
    (void)hipFree(dw);
    (void)hipFree(ds);
    if (e != hipSuccess) return fail(DMC_E_DEVICE, hipGetErrorString(e));
    return DMC_OK;
}

extern "C" dmc_status dmc_debug_op_cost(int32_t op, uint32_t iters, int32_t blocks, double *ms, uint64_t *op_count)
{
    if (!ms || !op_count) return fail(DMC_E_INVALID, "NULL argument");
    if (op < 0 || op >= COST_N) return fail(DMC_E_INVALID, "unknown operation");
    if (iters == 0 || blocks < 0 || blocks > (1 << 20)) return fail(DMC_E_INVALID, "iters must be > 0, blocks 0..2^20");
    if (blocks == 0) blocks = device_cus() * 32;
    uint32_t *d = nullptr;
    if (hipMalloc(&d, (size_t)blocks * 256 * sizeof(uint32_t)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(DMC_E_NOMEM, "hipMalloc failed");
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    // a first launch loads the code object; the second is timed
    if (e == hipSuccess) e = launch_op_cost(op, iters, blocks, d, nullptr);
    if (e == hipSuccess) e = hipEventRecord(e0, nullptr);
    if (e == hipSuccess) e = launch_op_cost(op, iters, blocks, d, nullptr);
    if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float t = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(d);
    if (e != hipSuccess) return fail(DMC_E_DEVICE, hipGetErrorString(e));
    *ms = t;
    *op_count = (uint64_t)blocks * 256 * (uint64_t)iters * 4;
    return DMC_OK;
}

extern "C" dmc_status dmc_debug_fp64_math(const double *x, double *log_out, double *sin_out, double *cos_out, size_t n)
{
    if (!x) return fail(DMC_E_INVALID, "x is NULL");
    if (n == 0) return DMC_OK;
    double *d = nullptr;
    if (hipMalloc(&d, 4 * n * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(DMC_E_NOMEM, "hipMalloc failed");
    }
    hipError_t e = hipMemcpy(d, x, n * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_debug_math(d, d + n, d + 2 * n, d + 3 * n, n, nullptr);
    if (e == hipSuccess && log_out) e = hipMemcpy(log_out, d + n, n * sizeof(double), hipMemcpyDeviceToHost);
    if (e == hipSuccess && sin_out) e = hipMemcpy(sin_out, d + 2 * n, n * sizeof(double), hipMemcpyDeviceToHost);
    if (e == hipSuccess && cos_out) e = hipMemcpy(cos_out, d + 3 * n, n * sizeof(double), hipMemcpyDeviceToHost);
    (void)hipFree(d);
    if (e != hipSuccess) return fail(DMC_E_DEVICE, hipGetErrorString(e));
    return DMC_OK;
}
