// dmc_noalloc.hip -- the batched launch for callers that cannot allocate.
//
// dmc_simulate_batch_noalloc runs the same kernels as dmc_simulate_batch, but
// every device buffer it needs besides the caller's inputs and outputs (job
// descriptors, snapshot times, per-job counters, the particle queue and the
// device tally blocks) lives in one file-scope device array, `scratch`, of a
// fixed size.  The host side uses only fixed-size arrays on the stack, uploads
// descriptors and times through kernel arguments, clears what must start at
// zero with a fill kernel and writes the finished raw tallies and counters to
// the caller's device buffers with a completion kernel.  Nothing is allocated,
// no event is created and nothing synchronises: the call only enqueues work on
// the stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>

#include "dmc_host_internal.h"

namespace dmc {
namespace {

constexpr size_t kScratchBytes = size_t(32) << 20;  // 32 MiB per device
constexpr int kNoAllocJobs = 64;
constexpr int kNoAllocTimes = 8192;  // snapshot times over all jobs
constexpr int kMaxDevices = 64;

constexpr size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// scratch layout: descriptor table, times, counters, queue head, tally blocks
constexpr size_t kTableOff = 0;
constexpr size_t kTimesOff = align256(kTableOff + kNoAllocJobs * sizeof(JobDev));
constexpr size_t kStatsOff = align256(kTimesOff + kNoAllocTimes * sizeof(double));
constexpr size_t kQueueOff = align256(kStatsOff + kNoAllocJobs * kStats * sizeof(unsigned long long));
constexpr size_t kTallyOff = align256(kQueueOff + 2 * sizeof(unsigned long long));
constexpr size_t kTallyDoubles = (kScratchBytes - kTallyOff) / sizeof(double);

}  // namespace
}  // namespace dmc

// The device memory of every dmc_simulate_batch_noalloc call on a device.  In
// host code this name is only a handle for hipGetSymbolAddress: kernels receive
// the address that call returns for the current device.
static __device__ __align__(256) unsigned char scratch[dmc::kScratchBytes];

namespace dmc {
namespace {

std::mutex g_mu;
unsigned char *g_scratch[kMaxDevices] = {};

// Device address of `scratch` on the current device, resolved once per device.
dmc_status scratch_address(unsigned char **out)
{
    int dev = 0;
    DMC_HIP_OR_FAIL(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(DMC_E_UNSUPPORTED, "device index beyond 63");
    std::lock_guard<std::mutex> g(g_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(DMC_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch[dev] = (unsigned char *)p;
    }
    *out = g_scratch[dev];
    return DMC_OK;
}

// Host-to-device copies through kernel arguments (no staging buffer).
constexpr int kUploadWords = 384;
struct Upload {
    uint64_t dst;  // byte offset in the destination
    uint32_t n;    // 8-byte words
    uint32_t pad;
    uint64_t w[kUploadWords];
};

__global__ void upload_kernel(Upload u, unsigned char *base)
{
    uint64_t *d = reinterpret_cast<uint64_t *>(base + u.dst);
    for (uint32_t i = threadIdx.x; i < u.n; i += blockDim.x) d[i] = u.w[i];
}

hipError_t upload(unsigned char *base, size_t dst, const void *src, size_t bytes, hipStream_t s)
{
    const unsigned char *p = (const unsigned char *)src;
    Upload u;
    for (size_t done = 0; done < bytes;) {
        const size_t chunk = std::min(bytes - done, sizeof(u.w));
        std::memset(u.w, 0, sizeof(u.w));
        std::memcpy(u.w, p + done, chunk);
        u.dst = dst + done;
        u.n = (uint32_t)((chunk + 7) / 8);
        u.pad = 0;
        void *params[] = {&u, &base};
        const hipError_t e = hipLaunchKernel((const void *)upload_kernel, dim3(1), dim3(128), params, 0, s);
        if (e != hipSuccess) return e;
        done += chunk;
    }
    return hipSuccess;
}

// Completion: the raw block a caller reads from each job's device block, with
// the telescoped net transmissions expanded into the displacement bins and the
// sums of |s| of snapshot cells whose particles share one sign; and the
// per-job counters.
struct Complete {
    uint32_t vis[kNoAllocJobs];      // doubles of job j's raw block
    uint32_t out_off[kNoAllocJobs];  // its offset in the output
    uint32_t blk[kNoAllocJobs];      // its device block's offset in the tally region
    uint16_t tab[kNoAllocJobs];      // its descriptor's position in the (queue-ordered) table
    int32_t n_jobs;
};

__global__ void complete_kernel(Complete c, const unsigned char *base, double *out, uint64_t *counters)
{
    const int j = blockIdx.y;
    const JobDev &d = reinterpret_cast<const JobDev *>(base + kTableOff)[c.tab[j]];
    const double *tally = reinterpret_cast<const double *>(base + kTallyOff);
    const unsigned long long *stats = reinterpret_cast<const unsigned long long *>(base + kStatsOff);
    const int64_t nbins_all = (d.off_bins >= 0) ? (int64_t)d.n_batches * 3 * d.n_bins : 0;
    const int64_t nsnap = (d.off_snap_abs >= 0) ? (int64_t)d.n_times * (d.ncell + 1) : 0;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < c.vis[j]; i += gridDim.x * blockDim.x) {
        const int64_t g = (int64_t)c.blk[j] + i;
        double v = tally[g];
        if (d.disp_tel && d.off_dispx >= 0) {
            const int64_t rel = g - d.off_bins;
            if (rel >= 0 && rel < nbins_all) {
                const int64_t row = rel / d.n_bins;
                if (row % 3 == 2) v += d.bin_width * tally[d.off_dispx + row / 3];
            }
        }
        if (nsnap > 0 && !d.snap_abs_on) {
            const int64_t rel = g - d.off_snap_abs;
            if (rel >= 0 && rel < nsnap) v = fabs(tally[d.off_snap + rel]);
        }
        out[c.out_off[j] + i] = v;
    }
    if (counters && blockIdx.x == 0 && threadIdx.x < 6) {
        // particles, scattering events, boundary events, segments, capped, flights
        const int src[6] = {0, 1, 2, 3, 4, 6};
        counters[(size_t)j * 6 + threadIdx.x] = stats[(size_t)j * kStats + src[threadIdx.x]];
    }
}

}  // namespace
}  // namespace dmc

using namespace dmc;

extern "C" dmc_status dmc_simulate_batch_noalloc(const dmc_job *jobs, int32_t n_jobs, const dmc_run_opts *opts,
                                                 double *raw_out, size_t raw_len, uint64_t *counters_out,
                                                 size_t *raw_offsets)
{
    if (!jobs || n_jobs < 1 || n_jobs > kNoAllocJobs)
        return fail(DMC_E_INVALID, "n_jobs must be 1..64 for the no-allocation launch");
    dmc_run_opts o;
    if (opts)
        o = *opts;
    else
        dmc_run_opts_default(&o);
    dmc_status st = run_opts_check(o);
    if (st != DMC_OK) return st;
    if (o.workspace) return fail(DMC_E_INVALID, "the no-allocation launch uses its own scratch: workspace must be NULL");
    const dmc_material *M = jobs[0].material;
    JobDev devs[kNoAllocJobs], table[kNoAllocJobs];
    JobMeta meta[kNoAllocJobs];
    double len[kNoAllocJobs], tf[kNoAllocJobs], key[kNoAllocJobs];
    int64_t size[kNoAllocJobs];
    int32_t nt[kNoAllocJobs];
    int rank[kNoAllocJobs];
    uint64_t particles = 0;
    int64_t tally = 0, vis = 0, times = 0;
    for (int i = 0; i < n_jobs; ++i) {
        if (jobs[i].material != M) return fail(DMC_E_INVALID, "all jobs of a launch must share one material");
        if ((st = prepare_job_core(jobs[i], devs[i], meta[i])) != DMC_OK) return st;
        if (particles + devs[i].n < particles) return fail(DMC_E_INVALID, "particle count overflow");
        particles += devs[i].n;
        len[i] = jobs[i].geometry->d.length;
        tf[i] = jobs[i].n_times > 0 ? jobs[i].times[jobs[i].n_times - 1] : 0.0;
        size[i] = meta[i].size;
        nt[i] = jobs[i].n_times;
        tally += meta[i].size;
        vis += meta[i].size - meta[i].hidden;
        times += jobs[i].n_times;
    }
    if (times > kNoAllocTimes)
        return fail(DMC_E_INVALID, "the no-allocation launch holds at most 8192 snapshot times over all jobs");
    if (tally > (int64_t)kTallyDoubles)
        return fail(DMC_E_INVALID, "the jobs' tallies need " + std::to_string(tally * 8) +
                                       " bytes; the no-allocation launch holds at most " +
                                       std::to_string(kTallyDoubles * 8));
    if (raw_offsets) {
        size_t o2 = 0;
        for (int i = 0; i < n_jobs; ++i) {
            raw_offsets[i] = o2;
            o2 += (size_t)(meta[i].size - meta[i].hidden);
        }
        raw_offsets[n_jobs] = o2;
    }
    if (!raw_out) return DMC_OK;  // sizes only
    if (raw_len < (size_t)vis)
        return fail(DMC_E_INVALID, "raw_out holds " + std::to_string(raw_len) + " doubles, the jobs need " +
                                       std::to_string(vis));
    if (o.nscat_out && o.nscat_out_len < particles)
        return fail(DMC_E_INVALID, "nscat_out holds " + std::to_string(o.nscat_out_len) + " entries, the launch has " +
                                       std::to_string(particles) + " particles");
    int dev = 0;
    DMC_HIP_OR_FAIL(hipGetDevice(&dev));
    if (dev != M->device) return fail(DMC_E_INVALID, "material was created on another device");
    unsigned char *base = nullptr;
    if ((st = scratch_address(&base)) != DMC_OK) return st;

    queue_order(*M, devs, len, tf, n_jobs, rank, key);
    assign_offsets(devs, size, nt, rank, n_jobs);
    LaunchBuffers b;
    b.jobs = (JobDev *)(base + kTableOff);
    b.times = (double *)(base + kTimesOff);
    b.tally = (double *)(base + kTallyOff);
    b.stats = (unsigned long long *)(base + kStatsOff);
    b.queue = (unsigned long long *)(base + kQueueOff);
    LaunchPlan plan;
    if ((st = plan_launch(M, devs, n_jobs, b, o, plan)) != DMC_OK) return st;
    // the device table is ordered by queue position (the kernels search it by base)
    Complete c{};
    c.n_jobs = n_jobs;
    for (int r = 0; r < n_jobs; ++r) {
        table[r] = devs[rank[r]];
        c.tab[rank[r]] = (uint16_t)r;
    }
    hipStream_t s = (hipStream_t)o.stream;
    DMC_HIP_OR_FAIL(upload(base, kTableOff, table, (size_t)n_jobs * sizeof(JobDev), s));
    for (int i = 0; i < n_jobs; ++i)
        if (jobs[i].n_times > 0)
            DMC_HIP_OR_FAIL(upload(base, kTimesOff + (size_t)devs[i].times_off * sizeof(double), jobs[i].times,
                                   (size_t)jobs[i].n_times * sizeof(double), s));
    // every call shares this device's scratch: tallies, counters and queue start at zero
    DMC_HIP_OR_FAIL(launch_fill(b.tally, (size_t)tally, b.stats, (size_t)n_jobs * kStats, s));
    DMC_HIP_OR_FAIL(launch_fill(nullptr, 0, b.queue, 2, s));
    if ((st = submit_launch(plan, devs, n_jobs, o, s)) != DMC_OK) return st;
    int64_t blk = 0, off = 0, most = 1;
    for (int i = 0; i < n_jobs; ++i) {
        c.blk[i] = (uint32_t)blk;
        c.out_off[i] = (uint32_t)off;
        c.vis[i] = (uint32_t)(meta[i].size - meta[i].hidden);
        blk += meta[i].size;
        off += c.vis[i];
        most = std::max<int64_t>(most, c.vis[i]);
    }
    const unsigned gx = (unsigned)std::min<int64_t>((most + 255) / 256, 1024);
    void *params[] = {&c, &base, &raw_out, &counters_out};
    DMC_HIP_OR_FAIL(hipLaunchKernel((const void *)complete_kernel, dim3(gx, (unsigned)n_jobs), dim3(256), params, 0, s));
    return DMC_OK;
}
