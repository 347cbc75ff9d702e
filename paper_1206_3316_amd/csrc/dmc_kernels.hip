// dmc_kernels.hip -- trajectory kernels for gfx950 (CDNA4).
//
// One wavefront lane carries one deviational particle through steps I-VI of
// the particle algorithm (draw from the source term, exponential free flight
// with mean tau, boundary search, boundary interaction or scattering from the
// normalised gain distribution of Eq. (2), segment scoring with the
// track-length estimator of Eq. (4) or the snapshot estimator of Eq. (3)).
// Particles never interact, so lanes never communicate except to take work
// from the particle queue and to combine tallies.
//
// Compile-time policies of the single kernel template:
//   R      float  : flight, intersection and sampling in FP32 (tallies FP64)
//          double : every step in FP64 (parity mode; arithmetic in the same
//                   order as the FP64 reference so that realisations agree)
//   FORM   PLAIN      one thread per particle run to completion; tables read
//                     from global memory; every contribution a direct FP64
//                     global atomic
//          PERSISTENT waves take chunks of particle indices from a queue and
//                     refill free lanes; gain table and state data staged in
//                     LDS; per-lane bin caches flushed to LDS-privatised
//                     tallies that are added to HBM once per workgroup
//          EPOCH      the persistent form in time-bounded launches (serving
//                     epochs): particles are resumed and suspended, and every
//                     tally is complete within each launch (no telescoping, no
//                     deferred snapshot scoring)
//   G      GEOM_SLAB  cross-plane slab, wall sources, steady (dead components
//                     eliminated)
//          GEOM_HALF  half space, Gaussian initial condition, snapshots only
//          GEOM_GRAD  in-plane films and pore cells under the gradient source of
//                     Eq. (6), conductivity and H_j tallies only
//          GEOM_ANY   every geometry and source, chosen per lane
//
// Random numbers: Philox4x32-10 (Salmon et al., SC'11) with key = seed and
// counter = (pid lo, pid hi, k, tag); one block per flight k (tag STEP), one
// or more blocks at emission (tags EMIT_A, EMIT_B).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "dmc_internal.h"

namespace dmc {
namespace {

// ---------------------------------------------------------------- Philox ----

__device__ __forceinline__ uint4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        // three-way XORs as one gfx950 three-input bit operation each (lookup
        // table 0x96 = a ^ b ^ c); the compiler does not merge the pairs itself
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
    }
    return make_uint4(c0, c1, c2, c3);
}

// The same block with the key schedule given: rk[2 r], rk[2 r + 1] are the key
// words of round r (kernels that keep every lane's schedule in vector registers:
// a three-input xor with a vector operand issues faster than with a scalar one).
__device__ __forceinline__ uint4 philox_rk(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, const uint32_t *rk)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, rk[2 * r], 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, rk[2 * r + 1], 0x96);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
    }
    return make_uint4(c0, c1, c2, c3);
}

__device__ __forceinline__ uint32_t alias_draw(const uint32_t *tab, int bits, uint32_t w)
{
    const uint32_t idx = w >> (32 - bits);
    const uint32_t mask = (1u << (32 - bits)) - 1u;
    const uint32_t e = tab[idx];
    return ((w & mask) < (e & mask)) ? idx : (e >> (32 - bits));
}

// ------------------------------------------------------ precision traits ----

template <typename R>
struct Pr;

// FP64 logarithm and sin/cos of 2 pi u built only from IEEE-exact basic
// operations (no contraction), following fixed steps that the FP64 reference
// also follows, so the parity mode reproduces its trajectories bit for bit
// (paths among convex pores are chaotic and would amplify one-ulp library
// differences).
//   log x:  x = m 2^e, m in [sqrt(1/2), sqrt(2)); log m = 2 atanh(s),
//           s = (m-1)/(m+1), odd series in s to s^23; + e ln2 (two-part ln 2).
//   sincos 2 pi u: v = 4u, k = floor(v + 1/2), t = (v - k) pi/2 in [-pi/4, pi/4],
//           Taylor series to t^17 (sin) and t^18 (cos), quadrant k mod 4.
__device__ __forceinline__ double det_log(double x)
{
    int e;
    double m = frexp(x, &e);
    if (m < 0x1.6a09e667f3bcdp-1) {
        m = m * 2.0;
        e = e - 1;
    }
    const double s = (m - 1.0) / (m + 1.0);
    const double z = s * s;
    double p = 1.0 / 23.0;
    p = p * z + 1.0 / 21.0;
    p = p * z + 1.0 / 19.0;
    p = p * z + 1.0 / 17.0;
    p = p * z + 1.0 / 15.0;
    p = p * z + 1.0 / 13.0;
    p = p * z + 1.0 / 11.0;
    p = p * z + 1.0 / 9.0;
    p = p * z + 1.0 / 7.0;
    p = p * z + 1.0 / 5.0;
    p = p * z + 1.0 / 3.0;
    p = p * z + 1.0;
    const double lm = (2.0 * s) * p;
    const double de = (double)e;
    return de * 0x1.62e42ff000000p-1 + (de * -0x1.718432a1b0e26p-35 + lm);
}

__device__ __forceinline__ void det_sincos2pi(double u, double &sn, double &cs)
{
    const double v = 4.0 * u;
    const double k = floor(v + 0.5);
    const double t = (v - k) * 0x1.921fb54442d18p+0;
    const double t2 = t * t;
    double ps = -1.0 / 355687428096000.0;
    ps = ps * t2 + 1.0 / 1307674368000.0;
    ps = ps * t2 - 1.0 / 6227020800.0;
    ps = ps * t2 + 1.0 / 39916800.0;
    ps = ps * t2 - 1.0 / 362880.0;
    ps = ps * t2 + 1.0 / 5040.0;
    ps = ps * t2 - 1.0 / 120.0;
    ps = ps * t2 + 1.0 / 6.0;
    const double st = t - t * (t2 * ps);
    double pc = 1.0 / 6402373705728000.0;
    pc = pc * t2 - 1.0 / 20922789888000.0;
    pc = pc * t2 + 1.0 / 87178291200.0;
    pc = pc * t2 - 1.0 / 479001600.0;
    pc = pc * t2 + 1.0 / 3628800.0;
    pc = pc * t2 - 1.0 / 40320.0;
    pc = pc * t2 + 1.0 / 720.0;
    pc = pc * t2 - 1.0 / 24.0;
    pc = pc * t2 + 1.0 / 2.0;
    const double ct = 1.0 - t2 * pc;
    const int q = ((int)k) & 3;
    sn = (q == 0) ? st : (q == 1) ? ct : (q == 2) ? -st : -ct;
    cs = (q == 0) ? ct : (q == 1) ? -st : (q == 2) ? -ct : st;
}

template <>
struct Pr<double> {
    static constexpr double inf() { return __builtin_huge_val(); }
    __device__ static double u(uint32_t w) { return ((double)w + 0.5) * (1.0 / 4294967296.0); }
    __device__ static double flight(double tau, uint32_t w) { return -tau * det_log(u(w)); }
    __device__ static double sq(double x) { return sqrt(x); }
    __device__ static void cs(uint32_t w, double &c, double &s) { det_sincos2pi(u(w), s, c); }
    __device__ static double div(double a, double b) { return a / b; }
    __device__ static double ptime(double t, double tau, double) { return t / tau; }
    __device__ static double lg(double x) { return det_log(x); }
    __device__ static double mu(uint32_t w) { return 2.0 * u(w) - 1.0; }
    // FP64 keeps the reference's arithmetic unchanged
    __device__ static double nonneg(double t) { return t; }
    // Henyey-Greenstein polar cosine, the reference's operations in its order
    __device__ static double hg_mu(const KArgs &a, uint32_t w)
    {
        const double f = a.hg[0] / (a.hg[1] + a.hg[2] * u(w));
        const double m = (a.hg[3] - f * f) / a.hg[2];
        return m > 1.0 ? 1.0 : (m < -1.0 ? -1.0 : m);
    }
};

template <>
struct Pr<float> {
    static constexpr float inf() { return __builtin_huge_valf(); }
    // ((w >> 9) + 1/2) 2^-23, strictly inside (0, 1), never denormal.  One funnel
    // shift puts the top 23 bits of w under the exponent of 1.0 (a = 1 + (w >> 9)
    // 2^-23, in [1, 2)); subtracting 1 - 2^-24 is exact (the difference has 24
    // significant bits).
    __device__ static float one_plus(uint32_t w) { return __uint_as_float(__builtin_amdgcn_alignbit(0x7Fu, w, 9u)); }
    __device__ static float u(uint32_t w) { return one_plus(w) - 0x1.fffffep-1f; }
    // -tau ln u with the hardware log2 (u >= 2^-24, so no range fix-ups are needed)
    __device__ static float flight(float ntl, uint32_t w) { return ntl * __builtin_amdgcn_logf(u(w)); }
    __device__ static float sq(float x) { return __builtin_amdgcn_sqrtf(x); }
    // v_sin / v_cos take revolutions: sin(2 pi u) = sin_rev(u)
    __device__ static void cs(uint32_t w, float &c, float &s)
    {
        const float r = u(w);
        c = __builtin_amdgcn_cosf(r);
        s = __builtin_amdgcn_sinf(r);
    }
    __device__ static float div(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
    __device__ static float ptime(float t, float, float itau) { return t * itau; }
    __device__ static float lg(float x) { return __builtin_amdgcn_logf(x) * 0.693147182f; }
    // 2u - 1 = (2a - 3) + 2^-23 with a = 1 + (w >> 9) 2^-23: both steps exact
    __device__ static float mu(uint32_t w) { return fmaf(one_plus(w), 2.0f, -3.0f) + 0x1p-23f; }
    // a position rounded just past a wall must not yield a negative flight time
    __device__ static float nonneg(float t) { return fmaxf(t, 0.0f); }
    // Henyey-Greenstein polar cosine through reciprocals
    __device__ static float hg_mu(const KArgs &a, uint32_t w)
    {
        const float f = a.hgf[0] * __builtin_amdgcn_rcpf(fmaf(a.hgf[2], u(w), a.hgf[1]));
        return fminf(fmaxf((a.hgf[3] - f * f) * a.hgf_inv2g, -1.0f), 1.0f);
    }
};

// ------------------------------------------------------------ lane state ----

template <typename R>
struct Lane {
    R x, y, z, ox, oy, oz;  // position and unit direction
    R v, tau, itau;         // group speed, relaxation time, 1/tau of the current state
    R ntl;                  // FP32: -tau ln 2 of the current state
    uint32_t m;             // state index
    R s;                    // sign
    int32_t last;           // surface the particle rests on (excluded from the next search)
    uint32_t k, nscat, nbound;
    uint32_t nseg;          // segments so far (kernels with periodic faces; elsewhere every segment is a flight)
    R rem;                  // free-flight time left after a periodic face (< 0: none)
    uint64_t pid;
    int32_t job, batch, slot;
    // cached job parameters
    int32_t geom, src, n_bins, n_hj, kmax, n_times;
    R len, bpl, bw;
    R rad2;  // pore radius squared (pore cells); kept in a register so the boundary
             // search of every flight does not wait on a load of the job descriptor
    uint32_t key0, key1;
    uint32_t rk[20];        // key schedule of the STEP blocks (kernels with lane_round_keys)
    // tally addresses of this particle: bins of its batch (LDS index or, if
    // bl < 0, HBM offset) and the H_j block
    int32_t bl, hl;
    int64_t bg, hg;
    // accumulators
    double t, Lz, h;
    int32_t cbin, dbin;     // bins of the two per-lane tally cache entries (-1: empty)
    int32_t kbin;           // bin that holds the current position
    double c0, c1, c2;      // entry A: the bin the particle is in
    double d0, d1, d2;      // entry B: the bin it came from
    int32_t tcur;           // index of the next snapshot time
    int32_t toff;           // the job's first sample time in KArgs::times (half-space kernel)
    double tnext, tend;     // next snapshot time and final time (+inf when steady)
    int32_t pend;           // deferred snapshot crossing: time index (-1: none) and position
    R px, py, pz;
    // windowed region tally: top of the region (-inf without one), the window
    // whose sums the particle is accumulating (-1: none), those sums and the
    // window's bounds
    R rzhi;
    int32_t rwin;
    double rt, rq;
    double rwbeg, rwend;
    int32_t fld;            // the job tallies the steady x-z field (gradient and generic kernels)
};

struct Shared {
    uint32_t *gain;              // packed gain table: LDS (persistent) or global (plain)
    const void *st;              // per-state data: LDS (persistent) or global (plain)
    double *ltally;              // LDS tallies (slots used only where a job's lds offset >= 0)
    unsigned long long *lstats;  // LDS per-job counters (used only if KArgs::lds_stats)
    double *ltimes;              // LDS copy of the launch's sample times (persistent launches whose tables fit)
    JobDev *ljobs;               // LDS copy of the job table (the same launches)
    const double *times;         // the sample times read: the LDS copy in those launches, else KArgs::times
};

template <typename R>
__device__ __forceinline__ void load_state(Lane<R> &p, const KArgs &a, const Shared &sh, uint32_t m);

template <>
__device__ __forceinline__ void load_state<float>(Lane<float> &p, const KArgs &a, const Shared &sh, uint32_t m)
{
    p.m = m;
    const float4 q = reinterpret_cast<const float4 *>(sh.st)[m];
    p.v = q.x;
    p.tau = q.y;
    p.itau = q.z;
    p.ntl = q.w;
}

template <>
__device__ __forceinline__ void load_state<double>(Lane<double> &p, const KArgs &a, const Shared &sh, uint32_t m)
{
    p.m = m;
    const double2 q = reinterpret_cast<const double2 *>(sh.st)[m];
    p.v = q.x;
    p.tau = q.y;
    p.itau = 0.0;
}

// ------------------------------------------------------- tally helpers ----

__device__ __forceinline__ void gadd(double *p, double v) { atomicAdd(p, v); }
__device__ __forceinline__ void gaddu(unsigned long long *p, unsigned long long v) { atomicAdd(p, v); }

// Adds to a tally slot that lives in LDS when lds_off >= 0, else in HBM.
__device__ __forceinline__ void tadd(const KArgs &a, const Shared &sh, int32_t lds_off, int64_t g_off, int32_t idx,
                                     double v)
{
    if (lds_off >= 0)
        atomicAdd(sh.ltally + (lds_off + idx), v);
    else
        gadd(a.tally + (g_off + idx), v);
}

// Bin of coordinate c among nb bins of width 1/bpl, clamped to the slab.
template <typename R>
__device__ __forceinline__ int bin_of(R c, R bpl, int nb)
{
    // truncation instead of floor: a product in (-1, 0) gives 0, which is the
    // clamped bin either way
    const int k = (int)(c * bpl);
    return min(max(k, 0), nb - 1);
}

template <typename R>
__device__ __forceinline__ void set_kbin(Lane<R> &p)
{
    if (p.n_bins > 0) p.kbin = bin_of((p.geom != GEOM_FILM) ? p.z : p.x, p.bpl, p.n_bins);
}

template <typename R, int FORM, int G>
__device__ __forceinline__ void bin_enter(Lane<R> &p, const KArgs &a, const Shared &sh, int32_t k);

// ------------------------------------------------------------ emission ----

// Lambertian direction about the inward normal sgn * e_axis (axis 0 or 2):
// mu = sqrt(u); tangent frame (x, y) for a z normal and (y, z) for an x normal.
template <typename R>
__device__ __forceinline__ void lambertian_plane(Lane<R> &p, int axis, R sgn, uint32_t w2, uint32_t w3)
{
    const R mu = Pr<R>::sq(Pr<R>::u(w2));
    R c, s;
    Pr<R>::cs(w3, c, s);
    const R st = Pr<R>::sq((R)1 - mu * mu);
    if (axis == 2) {
        p.ox = st * c;
        p.oy = st * s;
        p.oz = mu * sgn;
    } else {
        p.ox = mu * sgn;
        p.oy = st * c;
        p.oz = st * s;
    }
}

template <typename R>
__device__ __forceinline__ void isotropic(Lane<R> &p, uint32_t w2, uint32_t w3)
{
    const R mu = Pr<R>::mu(w2);
    R c, s;
    Pr<R>::cs(w3, c, s);
    const R st = Pr<R>::sq((R)1 - mu * mu);
    p.ox = st * c;
    p.oy = st * s;
    p.oz = mu;
}

// Direction after a scattering event with a Henyey-Greenstein phase function
// (the generalisation of step IVb): polar cosine mu about the incoming direction
// n, uniform azimuth in the frame t1 = (n_x n_z, n_y n_z, -s) / s,
// t2 = (-n_y, n_x, 0) / s, s = sqrt(n_x^2 + n_y^2) (x, y when n is along z);
// the FP64 form follows the reference's operations.
template <typename R>
__device__ __forceinline__ void scatter_hg(Lane<R> &p, const KArgs &a, uint32_t w2, uint32_t w3)
{
    const R mu = Pr<R>::hg_mu(a, w2);
    R c, s;
    Pr<R>::cs(w3, c, s);
    const R st = Pr<R>::sq((R)1 - mu * mu);
    const R nx = p.ox, ny = p.oy, nz = p.oz;
    const R s2 = nx * nx + ny * ny;
    R t1x = (R)1, t1y = (R)0, t1z = (R)0, t2x = (R)0, t2y = (R)1, t2z = (R)0;
    if (s2 > (R)1e-12) {
        const R sn = Pr<R>::sq(s2);
        t1x = Pr<R>::div(nx * nz, sn);
        t1y = Pr<R>::div(ny * nz, sn);
        t1z = -sn;
        t2x = Pr<R>::div(-ny, sn);
        t2y = Pr<R>::div(nx, sn);
    }
    p.ox = mu * nx + st * (c * t1x + s * t2x);
    p.oy = mu * ny + st * (c * t1y + s * t2y);
    p.oz = mu * nz + st * (c * t1z + s * t2z);
}

// Kernels that keep each lane's Philox key schedule in vector registers (20
// words, computed when a particle is bound to the lane) instead of deriving it
// per flight on the scalar unit from a wave-uniform key: the FP32 slab,
// half-space and gradient kernels, which have the registers to spare.
template <typename R, int G>
__device__ constexpr bool lane_round_keys()
{
    return sizeof(R) == 4 && (G == GEOM_SLAB || G == GEOM_HALF || G == GEOM_GRAD);
}

// Per-particle copies of its job's parameters.
template <typename R, int G>
__device__ __forceinline__ void bind_job(Lane<R> &p, const JobDev &J, uint64_t pid, int job)
{
    p.pid = pid;
    p.job = job;
    p.slot = J.stat_slot;
    p.batch = (int32_t)(pid % (uint64_t)J.n_batches);
    p.geom = (G == GEOM_ANY || G == GEOM_GRAD) ? J.geom : G;
    p.src = J.src;
    p.n_bins = (G == GEOM_HALF || G == GEOM_GRAD) ? 0 : J.n_bins;
    p.n_hj = J.n_hj;
    p.kmax = (G == GEOM_SLAB) ? -1 : J.kmax;
    p.n_times = (G == GEOM_SLAB || G == GEOM_GRAD) ? 0 : J.n_times;
    p.len = (R)J.length;
    p.rad2 = (R)J.radius * (R)J.radius;
    p.bpl = (R)J.bins_per_len;
    p.bw = (R)J.bin_width;
    p.key0 = J.key0;
    p.key1 = J.key1;
    if constexpr (lane_round_keys<R, G>()) {
#pragma unroll
        for (int r = 0; r < 10; ++r) {
            p.rk[2 * r] = J.key0 + (uint32_t)r * 0x9E3779B9u;
            p.rk[2 * r + 1] = J.key1 + (uint32_t)r * 0xBB67AE85u;
        }
    }
    p.rzhi = (J.off_region >= 0 && (G == GEOM_HALF || G == GEOM_ANY)) ? (R)J.region_z[1] : -Pr<R>::inf();
    p.rwin = -1;
    p.rt = p.rq = 0.0;
    p.pend = -1;
    if constexpr (G == GEOM_HALF) p.toff = J.times_off;
    p.fld = (G == GEOM_GRAD || G == GEOM_ANY) ? (J.off_field >= 0 ? 1 : 0) : 0;
    {
        const int32_t boff = p.batch * 3 * p.n_bins;
        p.bl = (J.lds_bins >= 0) ? J.lds_bins + boff : -1;
        p.bg = J.off_bins + boff;
        p.hl = J.lds_hj;
        p.hg = J.off_hj;
    }
    p.cbin = p.dbin = -1;
    p.c0 = p.c1 = p.c2 = 0.0;
    p.d0 = p.d1 = p.d2 = 0.0;
}

// Keeps the next snapshot time and the final time in registers.
template <typename R, int FORM, int G>
__device__ __forceinline__ void set_times(Lane<R> &p, const KArgs &a, const Shared &sh, const JobDev &J)
{
    const double *times = sh.times + J.times_off;
    p.tnext = (p.tcur < p.n_times) ? times[p.tcur] : __builtin_huge_val();
    p.tend = (p.n_times > 0) ? times[p.n_times - 1] : __builtin_huge_val();
}

template <typename R, int FORM, int G>
__device__ void emit(Lane<R> &p, const KArgs &a, const Shared &sh, const JobDev &J, uint64_t qidx, int job)
{
    const uint64_t pid = J.pid0 + (qidx - J.base - (uint64_t)a.n_resume);
    bind_job<R, G>(p, J, pid, job);
    p.x = p.y = p.z = (R)0;
    p.last = kNoSurface;
    p.k = 0;
    p.nseg = 0;
    p.rem = (R)-1;
    p.nscat = 0;
    p.nbound = 0;
    p.t = 0.0;
    p.Lz = 0.0;
    p.h = 0.0;
    p.tcur = 0;
    set_times<R, FORM, G>(p, a, sh, J);

    const uint32_t plo = (uint32_t)pid, phi = (uint32_t)(pid >> 32);
    // the emission blocks, with the lane's key schedule where the kernel keeps one
    auto emit_block = [&](uint32_t c2, uint32_t tag) {
        if constexpr (lane_round_keys<R, G>()) return philox_rk(plo, phi, c2, tag, p.rk);
        return philox(plo, phi, c2, tag, p.key0, p.key1);
    };
    const uint4 A = emit_block(0u, TAG_EMIT_A);
    uint32_t m;
    const int src = (G == GEOM_SLAB)   ? (int)SRC_WALLS
                    : (G == GEOM_HALF) ? (int)SRC_GAUSSIAN
                    : (G == GEOM_GRAD) ? (int)SRC_GRADIENT
                                       : p.src;
    if (src == SRC_WALLS) {
        const uint32_t j = (J.n_src > 1) ? alias_draw(J.src_packed, 1, A.x) : 0u;
        const int wall = J.src_wall[j];
        m = alias_draw(a.flux_packed, a.flux_bits, A.y);
        const int axis = (p.geom == GEOM_FILM) ? 0 : 2;
        lambertian_plane(p, axis, wall == 0 ? (R)1 : (R)-1, A.z, A.w);
        const R c = (wall == 0) ? (R)0 : p.len;
        if (axis == 2)
            p.z = c;
        else
            p.x = c;
        p.last = wall;
        p.s = (R)J.wall_sign[wall];
        if (J.disp_tel && wall == 1 && axis == 2) tadd(a, sh, J.lds_dispx, J.off_dispx, p.batch, -(double)p.s);
    } else if (src == SRC_GAUSSIAN) {
        const uint4 B = emit_block(0u, TAG_EMIT_B);
        m = alias_draw(a.init_packed, a.init_bits, A.y);
        isotropic(p, A.z, A.w);
        const R sigma = (R)J.sigma;
        const R rho = Pr<R>::sq((R)-2 * Pr<R>::lg(Pr<R>::u(B.x)));
        R c, s;
        Pr<R>::cs(B.y, c, s);
        p.x = sigma * rho * c;
        p.y = sigma * rho * s;
        const R rz = Pr<R>::sq((R)-2 * Pr<R>::lg(Pr<R>::u(B.z)));
        R c2, s2;
        Pr<R>::cs(B.w, c2, s2);
        p.z = fabs(sigma * rz * c2);
        p.s = (R)J.sign0;
    } else {  // gradient source, Eq. (6)
        const uint4 B = emit_block(0u, TAG_EMIT_B);
        m = alias_draw(a.flux_packed, a.flux_bits, A.y);
        const R sz = (B.w >> 31) ? (R)-1 : (R)1;
        lambertian_plane(p, 2, sz, A.z, A.w);
        p.s = sz * (R)J.sign0;
        if (p.geom == GEOM_FILM) {
            p.x = p.len * Pr<R>::u(B.x);
        } else {
            const R c = (R)0.5 * p.len;
            const R r2 = p.rad2;
            bool ok = false;
            for (uint32_t att = 0; att < (uint32_t)kPosAttempts && !ok; ++att) {
                const uint4 Bb = (att == 0) ? B : emit_block(att, TAG_EMIT_B);
                const R x = p.len * Pr<R>::u(Bb.x), z = p.len * Pr<R>::u(Bb.y);
                if ((x - c) * (x - c) + (z - c) * (z - c) > r2) {
                    p.x = x;
                    p.z = z;
                    ok = true;
                }
            }
            if (!ok) {
                p.x = (R)0;
                p.z = (R)0;
            }
        }
    }
    load_state(p, a, sh, m);
    set_kbin(p);
    p.cbin = (p.n_bins > 0) ? p.kbin : -1;  // cache entry A: the bin the particle is in
}

// ------------------------------------------------------------- scoring ----

// Adds v to slot idx of the particle's bins: LDS when every job of the launch
// has its bins privatised there (a launch-wide, wave-uniform test), else per
// job (LDS or HBM).
template <typename R, int FORM>
__device__ __forceinline__ void bins_add(const Lane<R> &p, const KArgs &a, const Shared &sh, int32_t idx, double v)
{
    if (FORM != FORM_PLAIN && a.bins_lds_all)
        atomicAdd(sh.ltally + (p.bl + idx), v);
    else
        tadd(a, sh, p.bl, p.bg, idx, v);
}

// Kernels whose geometries have periodic faces (pore cells, films with periodic
// walls); elsewhere every segment is a whole free flight.
template <int G>
__device__ constexpr bool has_periodic()
{
    return G == GEOM_GRAD || G == GEOM_ANY;
}

// Segments a particle has run (what the flight cap and the age-graded priority count).
template <typename R, int G>
__device__ __forceinline__ uint32_t segments(const Lane<R> &p)
{
    return has_periodic<G>() ? p.nseg : p.k;
}

// Deferred snapshot scoring: FP32 persistent half-space kernel.
template <typename R, int FORM, int G>
__device__ constexpr bool defer_snapshots()
{
    return sizeof(R) == 4 && FORM == FORM_PERSISTENT && G == GEOM_HALF;
}

// Telescoped displacement (persistent slab kernel): the signed length a particle
// adds to bin k over its whole path is s (F_k(z_end) - F_k(z_start)) with
// F_k(z) = clamp(z - k w, 0, w), because the per-segment overlaps telescope along
// a continuous path.  Slab particles start and end on a wall, where F_k is 0 (z =
// 0) or w (z = L) for every bin, so a per-batch count of net transmissions
// replaces the per-flight displacement sum; the host expands it into the bins.
// Not in time-bounded launches: a suspended particle may finish in another
// launch, and the per-flight sums must then be complete in every launch.
template <int FORM, int G>
__device__ constexpr bool telescoped()
{
    return FORM == FORM_PERSISTENT && G == GEOM_SLAB;
}

// Per-lane bin cache (persistent form): entry A holds the sums of the bin the
// particle is in; in the slab kernel entry B holds those of the bin it came
// from, so a particle that walks back and forth across one bin edge adds to
// registers only.  An entry is added to the tallies when a bin displaces it or
// the particle ends.
template <typename R, int FORM, int G>
__device__ __forceinline__ void flush_entry(Lane<R> &p, const KArgs &a, const Shared &sh, int32_t bin, double &s0,
                                            double &s1, double &s2)
{
    if (bin < 0) return;
    const double sg = (double)p.s;  // the entries hold unsigned sums
    bins_add<R, FORM>(p, a, sh, bin, sg * s0);
    bins_add<R, FORM>(p, a, sh, bin + p.n_bins, sg * s1);
    if (!telescoped<FORM, G>()) bins_add<R, FORM>(p, a, sh, bin + 2 * p.n_bins, sg * s2);
    s0 = s1 = s2 = 0.0;
}

template <typename R, int FORM, int G>
__device__ __forceinline__ void bin_flush(Lane<R> &p, const KArgs &a, const Shared &sh)
{
    if (FORM == FORM_PLAIN) return;  // the plain form adds every contribution directly
    flush_entry<R, FORM, G>(p, a, sh, p.cbin, p.c0, p.c1, p.c2);
    if (G == GEOM_SLAB) flush_entry<R, FORM, G>(p, a, sh, p.dbin, p.d0, p.d1, p.d2);
    p.cbin = p.dbin = -1;
}

// Makes entry A the one of bin k (the particle's new bin).
template <typename R, int FORM, int G>
__device__ __forceinline__ void bin_enter(Lane<R> &p, const KArgs &a, const Shared &sh, int32_t k)
{
    if (k == p.cbin) return;
    if (G != GEOM_SLAB) {
        // one entry outside the slab kernel (registers are scarcer in the
        // general kernels, and bins matter most in thick slabs)
        flush_entry<R, FORM, G>(p, a, sh, p.cbin, p.c0, p.c1, p.c2);
        p.cbin = k;
        return;
    }
    int32_t tb = p.cbin;
    p.cbin = p.dbin;
    p.dbin = tb;
    double t0 = p.c0, t1 = p.c1, t2 = p.c2;
    p.c0 = p.d0;
    p.c1 = p.d1;
    p.c2 = p.d2;
    p.d0 = t0;
    p.d1 = t1;
    p.d2 = t2;
    if (p.cbin != k) {
        flush_entry<R, FORM, G>(p, a, sh, p.cbin, p.c0, p.c1, p.c2);
        p.cbin = k;
    }
}

// Time t spent in bin k: TIME += s t, PTIME += s t / tau, DISP += s v Omega_z t.
// cached: k is the bin of entry A (persistent form); otherwise a direct add.
template <typename R, int FORM, int G>
__device__ __forceinline__ void bin_add(Lane<R> &p, const KArgs &a, const Shared &sh, int k, R t, R vz, bool cached)
{
    constexpr bool T = telescoped<FORM, G>();
    if (FORM != FORM_PLAIN && cached) {
        // unsigned sums: the particle's sign multiplies them when they are added
        p.c0 += (double)t;
        p.c1 += (double)Pr<R>::ptime(t, p.tau, p.itau);
        if (!T) p.c2 += (double)(vz * t);
        return;
    }
    const double d0 = (double)(p.s * t);
    const double d1 = (double)(p.s * Pr<R>::ptime(t, p.tau, p.itau));
    const double d2 = T ? 0.0 : (double)(p.s * vz * t);
    {
        bins_add<R, FORM>(p, a, sh, k, d0);
        bins_add<R, FORM>(p, a, sh, k + p.n_bins, d1);
        if (!T) bins_add<R, FORM>(p, a, sh, k + 2 * p.n_bins, d2);
    }
}

// Track-length scoring of one segment into the 1-D bins (slab: z, film: x).
// Persistent form: the whole segment is added to the cache entry of the
// current bin (every lane does the same work); a segment that leaves the bin
// then moves the part beyond the bin's edge to the bins it reaches.  The plain
// form adds each bin's part directly.
template <typename R, int FORM, int G>
__device__ void score_bins(Lane<R> &p, const KArgs &a, const Shared &sh, const JobDev &J, R seg)
{
    const bool zax = (p.geom != GEOM_FILM);
    const R ca = zax ? p.z : p.x;
    const R wa = p.v * (zax ? p.oz : p.ox);
    const R vz = p.v * p.oz;
    const int nb = p.n_bins;
    const int ka = p.kbin;  // bin_of(ca): the end bin of the previous segment
    if constexpr (FORM != FORM_PLAIN) {
        bin_add<R, FORM, G>(p, a, sh, ka, seg, vz, true);
        // the position update of the step computes exactly cb, so kb is the next
        // segment's start bin (a boundary interaction recomputes it); a flight
        // parallel to the bins stays in bin ka
        const R cb = ca + wa * seg;
        const int kb = bin_of(cb, p.bpl, nb);
        p.kbin = kb;
        if (ka == kb) return;
        // time past the edge the particle crossed last: (cb - edge) / wa, one
        // expression for both directions (the same value as |cb - edge| / |wa|)
        const R inv = Pr<R>::div((R)1, wa);
        const R bw = p.bw;
        const bool up = wa > (R)0;
        const R t1 = fmax((cb - (R)(up ? kb : kb + 1) * bw) * inv, (R)0);
        const int nin = (up ? kb - ka : ka - kb) - 1;  // bins crossed from edge to edge
        if (nin > 0) {
            const R tin = bw * fabs(inv);
            const int step = up ? 1 : -1;
            for (int k = ka + step; k != kb; k += step) bin_add<R, FORM, G>(p, a, sh, k, tin, vz, false);
            bin_add<R, FORM, G>(p, a, sh, ka, -((R)nin * tin), vz, true);
        }
        constexpr bool T = telescoped<FORM, G>();
        const double e0 = (double)t1;  // unsigned, like the cache entries
        const double e1 = (double)Pr<R>::ptime(t1, p.tau, p.itau);
        const double e2 = T ? 0.0 : (double)(vz * t1);
        p.c0 -= e0;
        p.c1 -= e1;
        if (!T) p.c2 -= e2;
        bin_enter<R, FORM, G>(p, a, sh, kb);
        p.c0 += e0;
        p.c1 += e1;
        if (!T) p.c2 += e2;
    } else {
        if (wa == (R)0) {
            bin_add<R, FORM, G>(p, a, sh, ka, seg, vz, false);
            return;
        }
        const R cb = ca + wa * seg;
        const int kb = bin_of(cb, p.bpl, nb);
        p.kbin = kb;
        if (ka == kb) {
            bin_add<R, FORM, G>(p, a, sh, ka, seg, vz, false);
            return;
        }
        const R inv = Pr<R>::div((R)1, fabs(wa));
        const R bw = p.bw;
        const bool up = wa > (R)0;
        const R t0 = up ? fmax(((R)(ka + 1) * bw - ca) * inv, (R)0) : fmax((ca - (R)ka * bw) * inv, (R)0);
        const R t1 = up ? fmax((cb - (R)kb * bw) * inv, (R)0) : fmax(((R)(kb + 1) * bw - cb) * inv, (R)0);
        bin_add<R, FORM, G>(p, a, sh, ka, t0, vz, false);
        const R tin = bw * inv;
        const int step = up ? 1 : -1;
        for (int k = ka + step; k != kb; k += step) bin_add<R, FORM, G>(p, a, sh, k, tin, vz, false);
        bin_add<R, FORM, G>(p, a, sh, kb, t1, vz, false);
    }
}

// Adds s to snapshot tally time_index at the cell that holds position (x, y, z).
template <typename R>
__device__ __forceinline__ void snapshot_add(const Lane<R> &p, const KArgs &a, const JobDev &J, int32_t ti, R x, R y,
                                             R z, double dt)
{
    int32_t idx[3];  // each below grid[d], an int32
    bool inside = true;
    if constexpr (sizeof(R) == 4) {
        // production: the cell in FP32 with a precomputed scale (no divisions),
        // the three axes without branches (the grid is read once)
        const float pos[3] = {x, y, z};
        const float lo[3] = {J.grid_lof[0], J.grid_lof[1], J.grid_lof[2]};
        const float sc[3] = {J.grid_scf[0], J.grid_scf[1], J.grid_scf[2]};
        const float gn[3] = {(float)J.grid[0], (float)J.grid[1], (float)J.grid[2]};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const float fl = floorf((pos[d] - lo[d]) * sc[d]);
            inside = inside && fl >= 0.0f && fl < gn[d];
            idx[d] = (int32_t)fminf(fmaxf(fl, 0.0f), gn[d]);  // clamped: a defined conversion
        }
    } else {
        // parity: the FP64 reference's operations
        const double pos[3] = {(double)p.x + (double)(p.v * p.ox) * dt, (double)p.y + (double)(p.v * p.oy) * dt,
                               (double)p.z + (double)(p.v * p.oz) * dt};
        for (int d = 0; d < 3; ++d) {
            const double f = (pos[d] - J.grid_lo[d]) / J.grid_ext[d] * (double)J.grid[d];
            const double fl = floor(f);
            if (!(fl >= 0.0 && fl < (double)J.grid[d])) {
                inside = false;
                break;
            }
            idx[d] = (int32_t)fl;
        }
    }
    const int64_t cell =
        inside ? ((int64_t)idx[2] * J.grid[1] + idx[1]) * (int64_t)J.grid[0] + idx[0] : J.ncell;
    const int64_t o = (int64_t)ti * (J.ncell + 1) + cell;
    gadd(a.tally + J.off_snap + o, (double)p.s);
    if (J.snap_abs_on) gadd(a.tally + J.off_snap_abs + o, 1.0);
}

// Scores the particle's recorded snapshot crossing, if any.
template <typename R>
__device__ __forceinline__ void snapshot_commit(Lane<R> &p, const KArgs &a, const JobDev &J)
{
    if (p.pend < 0) return;
    snapshot_add(p, a, J, p.pend, p.px, p.py, p.pz, 0.0);
    p.pend = -1;
}

// Snapshot estimator (Eq. (3)) at every sample time in [t, t + seg): the
// particle's position there, by linear interpolation along the segment,
// selects the grid cell (or the overflow slot) that receives s.  With DEFER
// (production half-space kernel) a crossing is recorded in registers and scored
// later together with other lanes' (snapshot_commit), so that the divergent
// cell and atomic work runs once for many lanes.
template <typename R, int FORM, int G>
__device__ void score_snapshots(Lane<R> &p, const KArgs &a, const Shared &sh, const JobDev &J, double seg)
{
    constexpr bool DEFER = defer_snapshots<R, FORM, G>();
    const double ta = p.t, tb = p.t + seg;
    // the production kernel keeps the job's offset in the lane (one load fewer in turn)
    const double *times = sh.times + (DEFER ? p.toff : J.times_off);
    while (p.tnext < tb) {
        const double tj = p.tnext;
        if (tj >= ta) {
            const double dt = tj - ta;
            if constexpr (DEFER) {
                snapshot_commit(p, a, J);  // a second crossing before the last was scored
                const R dtf = (R)dt;
                p.pend = p.tcur;
                p.px = p.x + (p.v * p.ox) * dtf;
                p.py = p.y + (p.v * p.oy) * dtf;
                p.pz = p.z + (p.v * p.oz) * dtf;
            } else if constexpr (sizeof(R) == 4) {
                const R dtf = (R)dt;
                snapshot_add(p, a, J, p.tcur, p.x + (p.v * p.ox) * dtf, p.y + (p.v * p.oy) * dtf,
                             p.z + (p.v * p.oz) * dtf, dt);
            } else {
                snapshot_add(p, a, J, p.tcur, p.x, p.y, p.z, dt);
            }
        }
        ++p.tcur;
        p.tnext = (p.tcur < p.n_times) ? times[p.tcur] : __builtin_huge_val();
    }
}

// Edge i of the steady field along an axis of n cells over [0, P): P i / n,
// evaluated as the FP64 reference does (FP32 kernels: i times the FP32 width).
template <typename R>
__device__ __forceinline__ R field_edge(int i, int n, double P, R width)
{
    if constexpr (sizeof(R) == 8) return P * (double)i / (double)n;
    return (R)i * width;
}

// Cell of coordinate c along an axis (the cell whose [edge i, edge i+1) holds c,
// clamped), from a first guess corrected against the edges themselves.
template <typename R>
__device__ __forceinline__ int field_cell(R c, int n, double P, R width)
{
    int i = (int)(c * (R)n / (R)P);
    i = min(max(i, 0), n - 1);
    if (i > 0 && c < field_edge<R>(i, n, P, width)) --i;
    if (i < n - 1 && c >= field_edge<R>(i + 1, n, P, width)) ++i;
    return i;
}

// Steady x-z field of the pore cell: Eq. (4) in every cell of the grid.  The
// segment from (x, z) along (wx, wz) = v (Omega_x, Omega_z), u in [0, seg], is
// walked cell by cell: the current cell is left at the earlier of its x and z
// exit times (edge - c) / w, and it holds the segment from its entry time to
// that exit (or seg).  These are the interval ends the FP64 reference computes
// cell by cell, so both give every cell the same time.  TIME_c += s t_c and
// DISPZ_c += s wz t_c go to the particle's batch of the field, privatised in LDS when it fits, else global FP64 atomics.
template <typename R>
__device__ void score_field(const Lane<R> &p, const KArgs &a, const Shared &sh, const JobDev &J, R seg)
{
    const int nx = J.grid[0], nz = J.grid[2];
    const double P = J.grid_ext[0];
    const R cwx = (R)(P / nx), cwz = (R)(P / nz);
    const R wx = p.v * p.ox, wz = p.v * p.oz;
    int ix = field_cell<R>(p.x, nx, P, cwx), iz = field_cell<R>(p.z, nz, P, cwz);
    const int32_t nc = nx * nz;
    const int32_t b0 = p.batch * 2 * nc;
    const double sg = (double)p.s;
    R t0 = (R)0;
    for (int it = 0; it < nx + nz + 2; ++it) {  // a segment inside the cell visits at most nx + nz cells
        R tx = Pr<R>::inf(), tz = Pr<R>::inf();
        if (wx > (R)0)
            tx = Pr<R>::div(field_edge<R>(ix + 1, nx, P, cwx) - p.x, wx);
        else if (wx < (R)0)
            tx = Pr<R>::div(field_edge<R>(ix, nx, P, cwx) - p.x, wx);
        if (wz > (R)0)
            tz = Pr<R>::div(field_edge<R>(iz + 1, nz, P, cwz) - p.z, wz);
        else if (wz < (R)0)
            tz = Pr<R>::div(field_edge<R>(iz, nz, P, cwz) - p.z, wz);
        R t1 = tx < tz ? tx : tz;
        if (seg < t1) t1 = seg;
        if (t1 > t0) {
            const int32_t c = iz * nx + ix;
            const double dt = (double)(t1 - t0);
            tadd(a, sh, J.lds_field, J.off_field, b0 + c, sg * dt);
            tadd(a, sh, J.lds_field, J.off_field, b0 + nc + c, sg * (double)wz * dt);
        }
        if (!(t1 < seg)) break;
        if (tx <= tz)
            ix += (wx > (R)0) ? 1 : -1;
        else
            iz += (wz > (R)0) ? 1 : -1;
        if (ix < 0 || ix >= nx || iz < 0 || iz >= nz) break;
        if (t1 > t0) t0 = t1;
    }
}

// Adds the particle's sums of its current region window to the tallies.
template <typename R>
__device__ __forceinline__ void region_flush(Lane<R> &p, const KArgs &a, const Shared &sh, const JobDev &J)
{
    if (p.rwin < 0) return;
    const int32_t o = 4 * p.rwin;
    tadd(a, sh, J.lds_region, J.off_region, o, p.rt);
    tadd(a, sh, J.lds_region, J.off_region, o + 1, p.rt * p.rt);
    tadd(a, sh, J.lds_region, J.off_region, o + 2, p.rq);
    tadd(a, sh, J.lds_region, J.off_region, o + 3, p.rq * p.rq);
    p.rt = p.rq = 0.0;
    p.rwin = -1;
}

// Time average of Eq. (3) over windows [t_{j-1}, t_j) in a z-aligned cylinder:
// the part [lo, hi] of the segment x + v Omega u, u in [0, seg], inside the
// region adds s (hi - lo) and s v Omega_z (hi - lo) to the particle's sums of the
// window(s) it falls in.  Same operations, in the same order, as the FP64
// reference, so the parity mode agrees.
template <typename R, int FORM, int G>
__device__ void score_region(Lane<R> &p, const KArgs &a, const Shared &sh, const JobDev &J, R seg)
{
    // the region's bounds, read together (one wait for all of them)
    const R zlo = (R)J.region_z[0], zhi = (R)J.region_z[1];
    const R cx = (R)J.region_c[0], cy = (R)J.region_c[1], rr = (R)J.region_r;
    R lo = (R)0, hi = seg;
    const R wz = p.v * p.oz;
    if (wz == (R)0) {
        if (!(p.z >= zlo && p.z < zhi)) return;
    } else {
        R ta = Pr<R>::div(zlo - p.z, wz), tb = Pr<R>::div(zhi - p.z, wz);
        if (ta > tb) {
            const R s = ta;
            ta = tb;
            tb = s;
        }
        if (ta > lo) lo = ta;
        if (tb < hi) hi = tb;
    }
    const R wx = p.v * p.ox, wy = p.v * p.oy;
    const R dx = p.x - cx, dy = p.y - cy;
    const R A = wx * wx + wy * wy, B = dx * wx + dy * wy, Cc = dx * dx + dy * dy - rr * rr;
    bool within = false;
    if constexpr (sizeof(R) == 4) {
        // production: a segment whose two ends are inside the cylinder lies in
        // it (the disc is convex), the usual case for a wide probe
        const R ex = dx + wx * seg, ey = dy + wy * seg;
        within = (Cc < (R)0) && (ex * ex + ey * ey < rr * rr);
    }
    if (!within) {
        if (A == (R)0) {
            if (!(Cc < (R)0)) return;
        } else {
            const R disc = B * B - A * Cc;
            if (!(disc > (R)0)) return;
            const R sq = Pr<R>::sq(disc);
            const R ta = Pr<R>::div(-B - sq, A), tb = Pr<R>::div(-B + sq, A);
            if (ta > lo) lo = ta;
            if (tb < hi) hi = tb;
        }
    }
    if (!(hi > lo)) return;
    const double t0 = p.t + (double)lo, t1 = p.t + (double)hi;
    if (p.rwin >= 0 && t1 <= p.rwend && t0 >= p.rwbeg) {  // inside the window being summed
        p.rt += (double)p.s * (t1 - t0);
        p.rq += (double)p.s * (double)p.v * (double)p.oz * (t1 - t0);
        return;
    }
    const double *times = sh.times + J.times_off;
    int j = (p.rwin > 0) ? p.rwin : 0;
    double w0 = (j == 0) ? 0.0 : times[j - 1];
    for (; j < p.n_times; ++j) {
        const double w1 = times[j];
        const double l = (t0 > w0) ? t0 : w0, h = (t1 < w1) ? t1 : w1;
        if (h > l) {
            if (j != p.rwin) {
                region_flush(p, a, sh, J);
                p.rwin = j;
                p.rwbeg = w0;
                p.rwend = w1;
            }
            p.rt += (double)p.s * (h - l);
            p.rq += (double)p.s * (double)p.v * (double)p.oz * (h - l);
        }
        if (w1 >= t1) break;
        w0 = w1;
    }
}

// ------------------------------------------------------ boundary search ----

// Earliest surface hit time along x + v Omega t, excluding p.last.
template <typename R>
__device__ __forceinline__ R search(const Lane<R> &p, const JobDev &J, int geom, int32_t &surf)
{
    R best = Pr<R>::inf();
    surf = kNoSurface;
    if (geom == GEOM_SLAB || geom == GEOM_FILM) {
        // one candidate plane, chosen by the sign of the axial speed; one division
        const R c = (geom == GEOM_SLAB) ? p.z : p.x;
        const R w = p.v * ((geom == GEOM_SLAB) ? p.oz : p.ox);
        const bool up = w > (R)0;
        const int32_t cand = up ? 1 : 0;
        const bool ok = (up || w < (R)0) && p.last != cand;
        const R dist = up ? (p.len - c) : ((R)0 - c);
        best = ok ? Pr<R>::div(dist, w) : best;
        surf = ok ? cand : kNoSurface;
    } else if (geom == GEOM_HALF) {
        const R w = p.v * p.oz;
        const bool ok = w < (R)0 && p.last != 0;
        best = ok ? Pr<R>::div((R)0 - p.z, w) : best;
        surf = ok ? 0 : kNoSurface;
    } else {  // pore cell: faces 0: x=0, 1: x=P, 2: z=0, 3: z=P, 4: pore surface
        // every candidate is evaluated and kept by selects, without branches (the
        // lanes of a wave differ in the signs of their speeds and in what they hit)
#pragma unroll
        for (int f = 0; f < 2; ++f) {
            // one face per axis, chosen by the sign of the speed along it
            const R c = (f == 0) ? p.x : p.z;
            const R w = p.v * ((f == 0) ? p.ox : p.oz);
            const bool up = w > (R)0;
            const int32_t id = up ? 2 * f + 1 : 2 * f;
            const bool ok = (up || w < (R)0) && p.last != id;
            const R t = Pr<R>::div(up ? p.len - c : (R)0 - c, w);
            const bool take = ok && t < best;
            best = take ? t : best;
            surf = take ? id : surf;
        }
        // the pore: the entry root of |x - c|^2 = r^2 along the flight in x-z (a
        // particle found inside, moving inward, meets it at once)
        const R r2 = p.rad2;
        const R c = (R)0.5 * p.len;
        const R dx = p.x - c, dz = p.z - c;
        const R aq = p.ox * p.ox + p.oz * p.oz;
        const R bq = dx * p.ox + dz * p.oz;
        const R cq = dx * dx + dz * dz - r2;
        const R disc = bq * bq - aq * cq;
        const bool inside = cq <= (R)0;
        const bool ok = r2 > (R)0 && p.last != 4 && aq > (R)0 && bq < (R)0 && (inside || disc > (R)0);
        const R dist = inside ? (R)0 : Pr<R>::div(-bq - Pr<R>::sq(disc > (R)0 ? disc : (R)0), aq);
        const R t = Pr<R>::div(dist, p.v);
        const bool take = ok && t < best;
        best = take ? t : best;
        surf = take ? (int32_t)4 : surf;
    }
    return Pr<R>::nonneg(best);
}

enum { HIT_REFLECTED = 0, HIT_ABSORBED = 1, HIT_PERIODIC = 2 };

// Step IVa.  Returns HIT_ABSORBED if the particle ends, HIT_PERIODIC if it was
// moved to the opposite periodic face, HIT_REFLECTED otherwise.
template <typename R>
__device__ int interact(Lane<R> &p, const JobDev &J, int32_t surf, const uint4 &w)
{
    if (p.geom == GEOM_PORE) {
        if (surf < 4) {
            const bool xf = surf < 2;
            const R v = (surf % 2 == 1) ? (R)0 : p.len;
            if (xf)
                p.x = v;
            else
                p.z = v;
            p.last = (surf % 2 == 1) ? surf - 1 : surf + 1;
            return HIT_PERIODIC;
        }
        const R c = (R)0.5 * p.len;
        const R nx = p.x - c, nz = p.z - c;
        const R nn = Pr<R>::sq(nx * nx + nz * nz);
        const R n0 = Pr<R>::div(nx, nn), n2 = Pr<R>::div(nz, nn);
        if ((uint64_t)w.y < J.spec_thr[0]) {
            const R dn = p.ox * n0 + p.oz * n2;
            p.ox = p.ox - (R)2 * dn * n0;
            p.oz = p.oz - (R)2 * dn * n2;
        } else {
            const R mu = Pr<R>::sq(Pr<R>::u(w.z));
            R c3, s3;
            Pr<R>::cs(w.w, c3, s3);
            const R st = Pr<R>::sq((R)1 - mu * mu);
            p.ox = mu * n0 + st * (s3 * -n2);
            p.oy = st * c3;
            p.oz = mu * n2 + st * (s3 * n0);
        }
        p.last = 4;
        return HIT_REFLECTED;
    }
    const int wall = (p.geom == GEOM_HALF) ? 0 : surf;
    const int ax = (p.geom == GEOM_FILM) ? 0 : 2;
    const int32_t type = J.wall_type[wall];
    if (type == WALL_ISOTHERMAL) return HIT_ABSORBED;
    if (type == WALL_PERIODIC) {
        const R v = (wall == 1) ? (R)0 : p.len;
        if (ax == 2)
            p.z = v;
        else
            p.x = v;
        p.last = (wall == 1) ? 0 : 1;
        return HIT_PERIODIC;
    }
    if ((uint64_t)w.y < J.spec_thr[wall]) {
        if (ax == 2)
            p.oz = -p.oz;
        else
            p.ox = -p.ox;
    } else {
        if (J.first_event) return HIT_ABSORBED;  // a diffuse reflection ends the first free path
        lambertian_plane(p, ax, wall == 0 ? (R)1 : (R)-1, w.z, w.w);
    }
    p.last = wall;
    return HIT_REFLECTED;
}

// ------------------------------------------------------- suspend / resume ----

template <typename R, int FORM, int G>
__device__ void suspend(Lane<R> &p, const KArgs &a, const Shared &sh)
{
    if (p.n_bins > 0) bin_flush<R, FORM, G>(p, a, sh);
    const uint32_t slot = atomicAdd(reinterpret_cast<unsigned int *>(a.queue + 1), 1u);
    Suspended &S = a.suspend_out[slot];  // the host sizes the buffer for every lane of the grid
    S.x = (double)p.x;
    S.y = (double)p.y;
    S.z = (double)p.z;
    S.ox = (double)p.ox;
    S.oy = (double)p.oy;
    S.oz = (double)p.oz;
    S.t = p.t;
    S.Lz = p.Lz;
    S.h = p.h;
    S.pid = p.pid;
    S.k = p.k;
    // kernels without periodic faces: every segment is a flight and none is pending
    S.nseg = has_periodic<G>() ? p.nseg : p.k;
    S.rem = has_periodic<G>() ? (double)p.rem : -1.0;
    S.nscat = p.nscat;
    S.nbound = p.nbound;
    S.m = p.m;
    S.last = p.last;
    S.tcur = p.tcur;
    S.slot = p.slot;
    S.sign = p.s > (R)0 ? 1 : -1;
    S.rt = p.rt;
    S.rq = p.rq;
    S.rwin = p.rwin;
    if (a.lds_stats)
        atomicAdd(sh.lstats + p.slot * kStats + 5, 1ull);
    else
        gaddu(a.stats + (int64_t)p.slot * kStats + 5, 1ull);
}

template <typename R, int G>
__device__ void resume(Lane<R> &p, const KArgs &a, const Shared &sh, uint32_t i)
{
    const Suspended &S = a.resume_in[i];
    const int job = a.resume_job[S.slot];
    const JobDev &J = a.jobs[job];
    bind_job<R, G>(p, J, S.pid, job);
    p.x = (R)S.x;
    p.y = (R)S.y;
    p.z = (R)S.z;
    p.ox = (R)S.ox;
    p.oy = (R)S.oy;
    p.oz = (R)S.oz;
    p.t = S.t;
    p.Lz = S.Lz;
    p.h = S.h;
    p.k = S.k;
    if (has_periodic<G>()) {
        p.nseg = S.nseg;
        p.rem = (R)S.rem;
    }
    p.nscat = S.nscat;
    p.nbound = S.nbound;
    p.last = S.last;
    p.tcur = S.tcur;
    set_times<R, FORM_EPOCH, G>(p, a, sh, J);
    p.s = (R)S.sign;
    p.rt = S.rt;
    p.rq = S.rq;
    p.rwin = S.rwin;
    if (p.rwin >= 0) {
        p.rwbeg = (p.rwin == 0) ? 0.0 : sh.times[J.times_off + p.rwin - 1];
        p.rwend = sh.times[J.times_off + p.rwin];
    }
    load_state(p, a, sh, S.m);
    set_kbin(p);
    p.cbin = (p.n_bins > 0) ? p.kbin : -1;
}

// ---------------------------------------------------------------- finish ----

template <typename R, int FORM, int G>
__device__ void finish(Lane<R> &p, const KArgs &a, const Shared &sh, const JobDev &J, bool capped)
{
    if (p.n_bins > 0) bin_flush<R, FORM, G>(p, a, sh);
    if (G == GEOM_HALF || G == GEOM_ANY) region_flush(p, a, sh, J);
    if (defer_snapshots<R, FORM, G>()) snapshot_commit(p, a, J);
    if (telescoped<FORM, G>() && p.n_bins > 0) {
        // end term of the telescoped displacement: F_k(z_end) for every bin
        const R z = p.z;
        if (z >= p.len) {
            tadd(a, sh, J.lds_dispx, J.off_dispx, p.batch, (double)p.s);
        } else if (z > (R)0) {  // ended inside the slab (flight cap or truncation)
            const int kz = bin_of(z, p.bpl, p.n_bins);
            for (int kk = 0; kk < kz; ++kk) bins_add<R, FORM>(p, a, sh, kk + 2 * p.n_bins, (double)(p.s * p.bw));
            bins_add<R, FORM>(p, a, sh, kz + 2 * p.n_bins, (double)(p.s * (z - (R)kz * p.bw)));
        }
    }
    if (J.off_kappa >= 0) {
        tadd(a, sh, J.lds_kappa, J.off_kappa, 0, p.Lz);
        tadd(a, sh, J.lds_kappa, J.off_kappa, 1, p.Lz * p.Lz);
    }
    if (p.n_hj > 0 && p.nscat < (uint32_t)p.n_hj) {
        tadd(a, sh, p.hl, p.hg, (int32_t)p.nscat, p.h);
        tadd(a, sh, p.hl, p.hg, p.n_hj + (int32_t)p.nscat, p.h * p.h);
    }
    if (a.nscat_out) a.nscat_out[J.out_off + (p.pid - J.pid0)] = p.nscat;
    const unsigned long long vals[kStats] = {1ull, p.nscat, p.nbound, segments<R, G>(p), capped ? 1ull : 0ull,
                                             0ull, p.k};
    if (a.lds_stats) {
#pragma unroll
        for (int i = 0; i < kStats; ++i)
            if (vals[i]) atomicAdd(sh.lstats + p.slot * kStats + i, vals[i]);
    } else {
#pragma unroll
        for (int i = 0; i < kStats; ++i)
            if (vals[i]) gaddu(a.stats + (int64_t)p.slot * kStats + i, vals[i]);
    }
}

// ------------------------------------------------------------------ step ----

// Key of a wave's particles when they all carry the same one (the usual case:
// a wave's particles come from one job): the Philox key schedule of the STEP
// block then runs once on the scalar unit instead of once per lane.
struct WaveKey {
    uint32_t k0, k1;
    bool uniform;
};

// Over the live lanes; particles change only where lanes are refilled, so the
// persistent loop refreshes it there.
template <typename R>
__device__ __forceinline__ WaveKey wave_key(const Lane<R> &p, bool alive)
{
    WaveKey w{0u, 0u, false};
    const uint64_t live = __ballot(alive);
    if (live == 0ull) return w;
    const int src = __ffsll((unsigned long long)live) - 1;
    w.k0 = __builtin_amdgcn_readlane(p.key0, src);
    w.k1 = __builtin_amdgcn_readlane(p.key1, src);
    w.uniform = __ballot(alive && (p.key0 != w.k0 || p.key1 != w.k1)) == 0ull;
    return w;
}

// Over the active lanes (plain form).
template <typename R>
__device__ __forceinline__ WaveKey wave_key_active(const Lane<R> &p)
{
    WaveKey w;
    w.k0 = __builtin_amdgcn_readfirstlane(p.key0);
    w.k1 = __builtin_amdgcn_readfirstlane(p.key1);
    w.uniform = __ballot(p.key0 != w.k0 || p.key1 != w.k1) == 0ull;
    return w;
}

// The STEP block of flight k.
template <typename R, int G>
__device__ __forceinline__ uint4 philox_step(const Lane<R> &p, const WaveKey &wk, uint32_t k)
{
    const uint32_t c0 = (uint32_t)p.pid, c1 = (uint32_t)(p.pid >> 32);
    if constexpr (lane_round_keys<R, G>()) return philox_rk(c0, c1, k, TAG_STEP, p.rk);
    if (wk.uniform) return philox(c0, c1, k, TAG_STEP, wk.k0, wk.k1);
    return philox(c0, c1, k, TAG_STEP, p.key0, p.key1);
}


// One iteration of steps II-VI.  Returns 0 if the particle goes on, 1 if it
// ended, 2 if it hit the flight cap.  A free flight that reaches a periodic face
// continues from the opposite face with the time it has left and the words of
// the block drawn when it began.  In the gradient kernel one call runs up to
// `hops` segments of the particle: periodic continuations under any budget above
// one (waves holding a long-running particle), new free flights as well under
// the full budget of 64 (waves down to a few live lanes, where no other lane
// waits on the loop), so a long trajectory does not pay a whole iteration of its
// wave per segment; elsewhere one segment.
template <typename R, int FORM, int G>
__device__ __forceinline__ int step(Lane<R> &p, const KArgs &a, const Shared &sh, const JobDev &J, const WaveKey &wk,
                                    uint32_t hops)
{
    constexpr bool PER = has_periodic<G>();
    const int geom = (G == GEOM_ANY || G == GEOM_GRAD) ? p.geom : G;
    const bool gradient = (G == GEOM_GRAD) || ((G == GEOM_ANY) && (p.src == SRC_GRADIENT));
    uint4 w;
    R dt;
    bool carried = false;  // a periodic continuation in this call: the block of its flight is at hand
    for (uint32_t hop = 1;; ++hop) {
        if (carried) {
            dt = p.rem;
        } else {
            const bool cont = PER && p.rem >= (R)0;
            w = philox_step<R, G>(p, wk, cont ? p.k - 1u : p.k);
            if (cont) {
                dt = p.rem;
            } else {
                ++p.k;
                dt = Pr<R>::flight(sizeof(R) == 4 ? p.ntl : p.tau, w.x);  // step II
            }
        }
        if (PER) {
            p.rem = (R)-1;
            ++p.nseg;
        }
        int32_t surf;
        const R tb = search(p, J, geom, surf);                           // step III
        const bool boundary = (tb <= dt);
        const R seg = boundary ? tb : dt;
        // step V: sample the segment
        if (G == GEOM_SLAB || p.n_bins > 0) score_bins<R, FORM, G>(p, a, sh, J, seg);  // the slab kernel always has bins
        if constexpr (G == GEOM_GRAD || G == GEOM_ANY) {
            if (p.fld) score_field(p, a, sh, J, seg);
        }
        if (gradient) {
            const double dz = (double)(p.s * p.v * p.oz * seg);
            p.Lz += dz;
            if (p.nscat < (uint32_t)p.n_hj) p.h += dz;
        }
        if (G == GEOM_ANY || G == GEOM_HALF) {
            const double tb_abs = p.t + (double)seg;
            if (p.tnext < tb_abs) score_snapshots<R, FORM, G>(p, a, sh, J, (double)seg);
            // windowed region tally (a launch-wide flag skips the test when no job
            // has one); most segments lie wholly above the region
            if (a.any_region && fmin(p.z, p.z + p.v * p.oz * seg) < p.rzhi) score_region<R, FORM, G>(p, a, sh, J, seg);
            if (tb_abs > p.tend) return 1;  // step VI
        }
        // move
        p.x += p.v * p.ox * seg;
        p.y += p.v * p.oy * seg;
        p.z += p.v * p.oz * seg;
        p.t += (double)seg;
        if (boundary) {                                                   // step IVa
            if (geom == GEOM_SLAB || geom == GEOM_HALF)
                p.z = (surf == 1) ? p.len : (R)0;
            else if (geom == GEOM_FILM)
                p.x = (surf == 1) ? p.len : (R)0;
            else if (surf < 4) {
                const R v = (surf % 2 == 1) ? p.len : (R)0;
                if (surf < 2)
                    p.x = v;
                else
                    p.z = v;
            }
            ++p.nbound;
            const int hit = interact(p, J, surf, w);
            if (hit == HIT_ABSORBED) return 1;
            if (G == GEOM_SLAB || p.n_bins > 0) {
                set_kbin(p);  // a periodic face moves the particle to the other end
                if (FORM != FORM_PLAIN) bin_enter<R, FORM, G>(p, a, sh, p.kbin);
            }
            if (PER && hit == HIT_PERIODIC) p.rem = dt - seg;
        } else {                                                          // step IVb
            const uint32_t m = alias_draw(sh.gain, a.gain_bits, w.y);
            load_state(p, a, sh, m);
            // the specialised kernels scatter isotropically (the slab kernel tracks the
            // z direction cosine alone); launches with another phase function take the
            // generic kernel
            if (G != GEOM_ANY || a.scatter_g == 0.0)
                isotropic(p, w.z, w.w);
            else
                scatter_hg(p, a, w.z, w.w);
            p.last = kNoSurface;
            if (gradient && p.nscat < (uint32_t)p.n_hj) {
                tadd(a, sh, p.hl, p.hg, (int32_t)p.nscat, p.h);
                tadd(a, sh, p.hl, p.hg, p.n_hj + (int32_t)p.nscat, p.h * p.h);
                p.h = 0.0;
            }
            ++p.nscat;
            if (p.kmax >= 0 && p.nscat >= (uint32_t)p.kmax) return 1;
        }
        if (segments<R, G>(p) >= a.iter_cap) return 2;
        // the generic kernel continues in the next iteration (registers are
        // scarcer there)
        // periodic continuations within the budget; new free flights too at the
        // full budget (a wave down to a few live lanes), where no other lane waits
        carried = p.rem >= (R)0;
        if (!(G == GEOM_GRAD && hop < hops && (carried || hops >= 64u))) return 0;
    }
}

__device__ __forceinline__ int find_job(const JobDev *jt, int n_jobs, uint64_t q, int hint)
{
    int j = hint;
    while (j + 1 < n_jobs && q >= jt[j + 1].base) ++j;
    return j;
}

// ------------------------------------------------------------ LDS setup ----

// LDS layout (persistent form): packed gain table (2^bits u32, padded to 16
// bytes), per-state data (16 bytes each), privatised tallies (doubles), per-job
// counters.  The plain form keeps the tables in global memory and only the
// counters in LDS.  Pointers into LDS are always derived from the shared
// array so the compiler emits LDS instructions for them.
// JL: the launch's job table and sample times are staged in LDS (the host sizes
// LDS for them whenever both fit) and read from there.
template <typename R, int FORM, bool JL>
__device__ Shared setup_shared(const KArgs &a, unsigned char *smem)
{
    Shared sh;
    size_t off = 0;
    if (FORM == FORM_PERSISTENT) {
        uint32_t *g = reinterpret_cast<uint32_t *>(smem);
        for (int i = threadIdx.x; i < a.kpad; i += blockDim.x) g[i] = a.gain_packed[i];
        off = ((size_t)a.kpad * 4 + 15) & ~(size_t)15;
        if (sizeof(R) == 4) {
            float4 *st = reinterpret_cast<float4 *>(smem + off);
            for (int i = threadIdx.x; i < a.K; i += blockDim.x) st[i] = a.st32[i];
            sh.st = st;
        } else {
            double2 *st = reinterpret_cast<double2 *>(smem + off);
            for (int i = threadIdx.x; i < a.K; i += blockDim.x) st[i] = a.st64[i];
            sh.st = st;
        }
        off += (size_t)a.K * 16;
        sh.gain = g;
        off = (off + 15) & ~(size_t)15;
        sh.ltally = reinterpret_cast<double *>(smem + off);
        for (int i = threadIdx.x; i < a.lds_tally_doubles; i += blockDim.x) sh.ltally[i] = 0.0;
        off += (size_t)a.lds_tally_doubles * 8;
    } else {
        sh.gain = const_cast<uint32_t *>(a.gain_packed);
        sh.st = (sizeof(R) == 4) ? (const void *)a.st32 : (const void *)a.st64;
        sh.ltally = reinterpret_cast<double *>(smem);
    }
    sh.lstats = reinterpret_cast<unsigned long long *>(smem + off);
    if (a.lds_stats)
        for (int i = threadIdx.x; i < a.n_jobs * kStats; i += blockDim.x) sh.lstats[i] = 0ull;
    // the sample times after the counters, then the job table at a 16-byte boundary
    const size_t toff = off + (a.lds_stats ? (size_t)a.n_jobs * kStats * 8 : 0);
    sh.ltimes = reinterpret_cast<double *>(smem + toff);
    for (int i = threadIdx.x; i < a.times_lds; i += blockDim.x) sh.ltimes[i] = a.times[i];
    const size_t joff = (toff + (size_t)a.times_lds * 8 + 15) & ~(size_t)15;
    sh.ljobs = reinterpret_cast<JobDev *>(smem + joff);
    sh.times = JL ? sh.ltimes : a.times;
    if (a.jobs_lds) {
        const uint4 *src = reinterpret_cast<const uint4 *>(a.jobs);
        uint4 *dst = reinterpret_cast<uint4 *>(sh.ljobs);
        const int words = a.n_jobs * (int)(sizeof(JobDev) / 16);
        for (int i = threadIdx.x; i < words; i += blockDim.x) dst[i] = src[i];
    }
    __syncthreads();
    return sh;
}

// Adds the workgroup's LDS tallies and counters to HBM.
__device__ void flush_shared(const KArgs &a, const Shared &sh)
{
    __syncthreads();
    if (a.lds_tally_doubles > 0) {
        for (int j = 0; j < a.n_jobs; ++j) {
            const JobDev &J = a.jobs[j];
            if (J.lds_bins >= 0) {
                const int n = J.n_batches * 3 * J.n_bins;
                for (int i = threadIdx.x; i < n; i += blockDim.x) {
                    const double v = sh.ltally[J.lds_bins + i];
                    if (v != 0.0) gadd(a.tally + J.off_bins + i, v);
                }
            }
            if (J.lds_dispx >= 0) {
                for (int i = threadIdx.x; i < J.n_batches; i += blockDim.x) {
                    const double v = sh.ltally[J.lds_dispx + i];
                    if (v != 0.0) gadd(a.tally + J.off_dispx + i, v);
                }
            }
            if (J.lds_region >= 0) {
                for (int i = threadIdx.x; i < 4 * J.n_times; i += blockDim.x) {
                    const double v = sh.ltally[J.lds_region + i];
                    if (v != 0.0) gadd(a.tally + J.off_region + i, v);
                }
            }
            if (J.lds_kappa >= 0 && threadIdx.x < 2) {
                const double v = sh.ltally[J.lds_kappa + threadIdx.x];
                if (v != 0.0) gadd(a.tally + J.off_kappa + threadIdx.x, v);
            }
            if (J.lds_hj >= 0) {
                for (int i = threadIdx.x; i < 2 * J.n_hj; i += blockDim.x) {
                    const double v = sh.ltally[J.lds_hj + i];
                    if (v != 0.0) gadd(a.tally + J.off_hj + i, v);
                }
            }
            if (J.lds_field >= 0) {
                const int n = J.n_batches * 2 * J.grid[0] * J.grid[2];
                for (int i = threadIdx.x; i < n; i += blockDim.x) {
                    const double v = sh.ltally[J.lds_field + i];
                    if (v != 0.0) gadd(a.tally + J.off_field + i, v);
                }
            }
        }
    }
    if (a.lds_stats) {
        for (int i = threadIdx.x; i < a.n_jobs * kStats; i += blockDim.x) {
            const unsigned long long v = sh.lstats[i];
            if (v) gaddu(a.stats + i, v);
        }
    }
}

// --------------------------------------------------------------- kernels ----

template <typename R, int G>
__global__ void __launch_bounds__(256) plain_kernel(KArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const Shared sh = setup_shared<R, FORM_PLAIN, false>(a, smem);
    const uint64_t q = a.qbegin + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < a.total) {
        const int job = find_job(a.jobs, a.n_jobs, q, 0);
        const JobDev &J = a.jobs[job];
        Lane<R> p;
        emit<R, FORM_PLAIN, G>(p, a, sh, J, q, job);
        int r;
        do {
            r = step<R, FORM_PLAIN, G>(p, a, sh, J, wave_key_active(p), 1u);
        } while (r == 0);
        finish<R, FORM_PLAIN, G>(p, a, sh, J, r == 2);
    }
    flush_shared(a, sh);
}

__device__ __forceinline__ uint64_t readlane64(uint64_t v, int src)
{
    // src is wave-uniform, so the value lands in scalar registers: the queue
    // state derived from it stays scalar and the loop's control stays uniform
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)v, src);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(v >> 32), src);
    return ((uint64_t)hi << 32) | lo;
}

// BOUNDED: time-bounded launch (serving epochs): resumes suspended particles
// and suspends the live ones a fixed number of flights after the queue runs dry.
// JL: the job table is read from its LDS copy (the host stages it whenever it
// fits, and runs the specialised kernels only then).
template <typename R, int G, bool BOUNDED, bool JL>
__global__ void __launch_bounds__(1024) persistent_kernel(KArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const Shared sh = setup_shared<R, FORM_PERSISTENT, JL>(a, smem);
    constexpr int PF = BOUNDED ? FORM_EPOCH : FORM_PERSISTENT;
    const JobDev *const jt = JL ? sh.ljobs : a.jobs;
    const int lane = (int)(threadIdx.x & 63);
    Lane<R> p;
    bool alive = false;
    // a particle that ended keeps its registers until the lane is refilled, so
    // that its closing tally work runs together with other lanes' (0: none, 1:
    // ended, 2: stopped at the flight cap). Not in time-bounded launches: there
    // the longer live ranges push the generic kernel past 128 VGPRs into spills.
    constexpr bool DEFER_FINISH = !BOUNDED;
    int ended = 0;
    int job = 0;
    // wave-uniform slice of the queue: next index and how many are left (a chunk
    // fits 32 bits, so the tests below are scalar compares)
    uint64_t pool_cur = 0;
    uint32_t pool_left = 0;
    bool qdry = false;  // the global queue has handed out every index (wave-uniform)
    uint32_t drain = 0, poll = 0, iter = 0;
    uint32_t old_hops = 1;  // segment budget of a wave holding a long-running particle
    bool hold = false;      // the wave holds a very long trajectory: its free lanes are not refilled
    WaveKey wk{0u, 0u, false};
    const uint64_t wave_lanes = __ballot(true);
    for (;;) {
        // refill free lanes from this wave's chunk, taking a new chunk from the
        // queue (one atomic per wave) when it is used up; need stays the mask of
        // the free lanes through the refill
        uint64_t need = __ballot(!alive);
        const int n_free = __popcll(need);
        const bool have_work = pool_left > 0u || !qdry;
        constexpr bool HOLD = G == GEOM_GRAD && !BOUNDED;  // not in time-bounded launches (registers)
        if (HOLD && n_free == 64) hold = false;
        if (n_free > 0 && have_work && !(HOLD && hold) && (n_free >= a.refill_min || n_free == 64)) {
            if (ended) {
                finish<R, PF, G>(p, a, sh, jt[p.job], ended == 2);
                ended = 0;
            }
            while (need) {
                if (pool_left == 0u) {
                    if (qdry) break;
                    const int leader = __ffsll((unsigned long long)need) - 1;
                    uint64_t b = 0;
                    if (lane == leader) b = atomicAdd(a.queue, (unsigned long long)a.chunk);
                    b = readlane64(b, leader);
                    if (b >= a.total) {
                        qdry = true;
                        break;
                    }
                    pool_cur = b;
                    pool_left = (b + (uint64_t)a.chunk < a.total) ? (uint32_t)a.chunk : (uint32_t)(a.total - b);
                }
                const uint32_t avail = pool_left;
                const int cnt = __popcll(need);
                const int take = ((uint64_t)cnt < avail) ? cnt : (int)avail;
                const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(need >> 32),
                                                                 __builtin_amdgcn_mbcnt_lo((uint32_t)need, 0u));
                const bool mine = ((need >> lane) & 1ull) && (int)below < take;
                if (mine) {
                    const uint64_t q = pool_cur + below;
                    if (BOUNDED && q < (uint64_t)a.n_resume) {
                        resume<R, G>(p, a, sh, (uint32_t)q);
                    } else {
                        const uint64_t qn = BOUNDED ? q - (uint64_t)a.n_resume : q;
                        job = find_job(jt, a.n_jobs, qn, job);
                        emit<R, PF, G>(p, a, sh, jt[job], q, job);
                    }
                    alive = true;
                }
                pool_cur += (uint64_t)take;
                pool_left -= (uint32_t)take;
                need &= ~__ballot(mine);
            }
            wk = wave_key(p, alive);
        }
        if (BOUNDED && !qdry && ((++poll) & 63u) == 0u) {
            // waves whose lanes are all busy also learn when the queue ran dry
            const unsigned long long head = __hip_atomic_load(a.queue, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (head >= a.total) qdry = true;
        }
        if (need == wave_lanes && !(pool_left > 0u || !qdry)) break;  // no lane is live
        if (BOUNDED && qdry) {
            // time-bounded launch: the queue is dry; a fixed number of flights later
            // this wave hands its live particles, and any indices of its chunk not yet
            // started, to the next launch
            if (++drain > a.drain_iters) {
                if (ended) {
                    finish<R, PF, G>(p, a, sh, jt[p.job], ended == 2);
                    ended = 0;
                }
                if (alive) suspend<R, PF, G>(p, a, sh);
                alive = false;
                while (pool_left > 0u) {
                    const uint32_t avail = pool_left;
                    const bool mine = (uint64_t)lane < avail;
                    if (mine) {
                        const uint64_t q = pool_cur + (uint64_t)lane;
                        if (q < (uint64_t)a.n_resume) {
                            resume<R, G>(p, a, sh, (uint32_t)q);
                        } else {
                            job = find_job(jt, a.n_jobs, q - (uint64_t)a.n_resume, job);
                            emit<R, PF, G>(p, a, sh, jt[job], q, job);
                        }
                        suspend<R, PF, G>(p, a, sh);
                    }
                    const uint32_t n = (avail < 64u) ? avail : 64u;
                    pool_cur += n;
                    pool_left -= n;
                }
                break;
            }
        }
        if (a.prio_flights && ((++iter) & 63u) == 0u) {
            // trajectory lengths are heavy-tailed and a launch ends with its longest
            // particle, whose flights are otherwise paced by a fair share of its
            // SIMD: waves get issue priority by the age of their oldest particle
            // (past prio_flights, 4x and 16x that), so the longest-running
            // trajectories advance first; their other lanes keep refilling as usual
            const uint32_t t1 = a.prio_flights;
            const uint32_t age = segments<R, G>(p);
            if (__ballot(alive && age >= 16u * t1))
                __builtin_amdgcn_s_setprio(3);
            else if (__ballot(alive && age >= 4u * t1))
                __builtin_amdgcn_s_setprio(2);
            else if (__ballot(alive && age >= t1))
                __builtin_amdgcn_s_setprio(1);
            else
                __builtin_amdgcn_s_setprio(0);
            if constexpr (G == GEOM_GRAD) {
                // a wave holding a long-running particle also runs several
                // segments of each particle per iteration (8 from t1 / 16
                // segments on, 32 from t1, 64 from 16 t1), so the longest
                // trajectories do not pace the launch
                old_hops = __ballot(alive && age >= 16u * t1) ? 64u
                         : __ballot(alive && age >= t1) ? 32u
                         : __ballot(alive && age >= t1 / 16u) ? 8u : 1u;
                // from t1 segments on, the wave stops refilling: its other lanes end
                // their particles, and the long one runs alone at the full budget
                // below, no longer paced by their divergent paths (one wave of the
                // thousands in a launch gives up its other lanes for it)
                hold = old_hops >= 32u;
            }
        }
        // a wave down to a few live lanes (the tail of a launch) runs up to 64
        // segments of each particle per iteration; a wave holding a
        // long-running particle, the budget graded by its age
        const uint32_t hops = (G == GEOM_GRAD && __popcll(wave_lanes & ~need) <= 4) ? 64u : old_hops;
        if (alive) {
            const JobDev &J = jt[p.job];
            const int r = step<R, PF, G>(p, a, sh, J, wk, hops);
            if (r != 0) {
                if (DEFER_FINISH)
                    ended = r;
                else
                    finish<R, PF, G>(p, a, sh, J, r == 2);
                alive = false;
            }
        }
        if (defer_snapshots<R, PF, G>()) {
            // score the recorded crossings together once a quarter of the wave has one;
            // when those lanes share one job its fields are read through the scalar unit
            const bool mine = alive && p.pend >= 0;
            const uint64_t cm = __ballot(mine);
            if (__popcll(cm) >= 16) {
                const int jw = __builtin_amdgcn_readlane(p.job, __ffsll((unsigned long long)cm) - 1);
                if (__ballot(mine && p.job != jw) == 0ull) {
                    if (mine) snapshot_commit(p, a, jt[jw]);
                } else if (mine) {
                    snapshot_commit(p, a, jt[p.job]);
                }
            }
        }
    }
    if (ended) finish<R, PF, G>(p, a, sh, jt[p.job], ended == 2);
    flush_shared(a, sh);
}

__global__ void fill_kernel(double *p, size_t n, unsigned long long *q, size_t nq)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0.0;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nq; i += stride) q[i] = 0ull;
}

__global__ void debug_philox_kernel(uint64_t seed, const uint64_t *pid, const uint32_t *k, const uint32_t *tag,
                                    uint32_t *out, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint4 r = philox((uint32_t)pid[i], (uint32_t)(pid[i] >> 32), k[i], tag[i], (uint32_t)seed,
                           (uint32_t)(seed >> 32));
    out[4 * i + 0] = r.x;
    out[4 * i + 1] = r.y;
    out[4 * i + 2] = r.z;
    out[4 * i + 3] = r.w;
}

__global__ void debug_alias_kernel(const uint32_t *packed, int bits, const uint32_t *words, uint32_t *states, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    states[i] = alias_draw(packed, bits, words[i]);
}

__global__ void debug_math_kernel(const double *x, double *lg, double *sn, double *cs, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s, c;
    det_sincos2pi(x[i], s, c);
    lg[i] = (x[i] > 0.0) ? det_log(x[i]) : 0.0;
    sn[i] = s;
    cs[i] = c;
}

// ----------------------------------------------------- instruction costs ----

// Throughput probes behind the algorithmic work counts: every lane runs `iters`
// iterations of four independent chains of one operation (the operation's
// result feeds its next input, so nothing can be hoisted or folded).  Launched
// at full occupancy, the kernel time gives the VALU issue slots per lane one
// operation takes: slots = time x (CUs x 64 lanes x clock) / (lanes x iters x 4).
// The Philox chains feed a block's four output words back as the next counter,
// with the key either wave-uniform (the kernels' usual case: the key schedule
// runs on the scalar unit) or different in every lane.
template <int OP>
__global__ void __launch_bounds__(256) op_cost_kernel(uint32_t iters, uint32_t key0, uint32_t key1, uint32_t *out)
{
    const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t acc = 0;
    if constexpr (OP == COST_PHILOX_UNIFORM_KEY || OP == COST_PHILOX_LANE_KEY) {
        const uint32_t k0 = (OP == COST_PHILOX_LANE_KEY) ? key0 ^ gid : key0;
        const uint32_t k1 = (OP == COST_PHILOX_LANE_KEY) ? key1 + gid : key1;
        uint4 c[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) c[j] = make_uint4(gid, (uint32_t)j, 0u, 0u);
        for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
            for (int j = 0; j < 4; ++j) c[j] = philox(c[j].x, c[j].y, c[j].z, c[j].w, k0, k1);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) acc ^= c[j].x ^ c[j].y ^ c[j].z ^ c[j].w;
    } else if constexpr (OP == COST_F64_ADD) {
        double d[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) d[j] = (double)(gid + j);
        const double inc = __uint_as_float(key0 | 0x3f800000u);
        for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
            for (int j = 0; j < 4; ++j) d[j] = d[j] + inc;
        }
        acc = (uint32_t)(d[0] + d[1] + d[2] + d[3]);
    } else {
        float x[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) x[j] = 1.0f + (float)(gid & 255u) * 0x1p-9f + (float)j * 0.125f;
        const float a = __uint_as_float(key0 | 0x3f000000u), b = __uint_as_float(key1 | 0x3c000000u);
        for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if constexpr (OP == COST_FMA) x[j] = fmaf(x[j], a, b);
                else if constexpr (OP == COST_LOG) x[j] = __builtin_amdgcn_logf(fabsf(x[j]));
                else if constexpr (OP == COST_SIN) x[j] = __builtin_amdgcn_sinf(x[j]);
                else if constexpr (OP == COST_COS) x[j] = __builtin_amdgcn_cosf(x[j]);
                else if constexpr (OP == COST_SQRT) x[j] = __builtin_amdgcn_sqrtf(fabsf(x[j]));
                else if constexpr (OP == COST_RCP) x[j] = __builtin_amdgcn_rcpf(x[j]);
            }
        }
        acc = __float_as_uint(x[0]) ^ __float_as_uint(x[1]) ^ __float_as_uint(x[2]) ^ __float_as_uint(x[3]);
    }
    out[gid] = acc;
}

template <int OP>
const void *op_cost_ptr()
{
    return (const void *)op_cost_kernel<OP>;
}

}  // namespace

hipError_t launch_op_cost(int op, uint32_t iters, int blocks, uint32_t *out, hipStream_t stream)
{
    const void *f = nullptr;
    switch (op) {
    case COST_FMA: f = op_cost_ptr<COST_FMA>(); break;
    case COST_PHILOX_UNIFORM_KEY: f = op_cost_ptr<COST_PHILOX_UNIFORM_KEY>(); break;
    case COST_PHILOX_LANE_KEY: f = op_cost_ptr<COST_PHILOX_LANE_KEY>(); break;
    case COST_LOG: f = op_cost_ptr<COST_LOG>(); break;
    case COST_SIN: f = op_cost_ptr<COST_SIN>(); break;
    case COST_COS: f = op_cost_ptr<COST_COS>(); break;
    case COST_SQRT: f = op_cost_ptr<COST_SQRT>(); break;
    case COST_RCP: f = op_cost_ptr<COST_RCP>(); break;
    case COST_F64_ADD: f = op_cost_ptr<COST_F64_ADD>(); break;
    default: return hipErrorInvalidValue;
    }
    uint32_t k0 = 0x12345u, k1 = 0x6789u;
    uint32_t it = iters;
    void *params[] = {&it, &k0, &k1, &out};
    return hipLaunchKernel(f, dim3((unsigned)blocks), dim3(256), params, 0, stream);
}

hipError_t launch_debug_math(const double *x, double *lg, double *sn, double *cs, size_t n, hipStream_t stream)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(debug_math_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, x, lg, sn, cs, n);
    return hipGetLastError();
}

// ------------------------------------------------------------- launchers ----

namespace {

// The specialised kernels exist only with the job table in LDS (the host runs the
// generic kernel when it does not fit); the generic kernel in both forms.
template <typename R, int G>
const void *kernel_ptr(int form, bool bounded, bool jl)
{
    if (form == FORM_PLAIN) return (const void *)plain_kernel<R, G>;
    if constexpr (G == GEOM_ANY) {
        if (!jl)
            return bounded ? (const void *)persistent_kernel<R, G, true, false>
                           : (const void *)persistent_kernel<R, G, false, false>;
    } else {
        if (!jl) return nullptr;
    }
    return bounded ? (const void *)persistent_kernel<R, G, true, true> : (const void *)persistent_kernel<R, G, false, true>;
}

template <typename R>
const void *pick_geom(int spec, int form, bool bounded, bool jl)
{
    if (spec == GEOM_SLAB) return kernel_ptr<R, GEOM_SLAB>(form, bounded, jl);
    if (spec == GEOM_HALF) return kernel_ptr<R, GEOM_HALF>(form, bounded, jl);
    if (spec == GEOM_GRAD) return kernel_ptr<R, GEOM_GRAD>(form, bounded, jl);
    return kernel_ptr<R, GEOM_ANY>(form, bounded, jl);
}

const void *pick_kernel(int precision, int form, int spec, bool bounded, bool jl)
{
    return precision == 0 ? pick_geom<double>(spec, form, bounded, jl) : pick_geom<float>(spec, form, bounded, jl);
}

}  // namespace

hipError_t launch_trajectories(const KArgs &a, int precision, int form, int spec, int block, int grid,
                               size_t lds_bytes, hipStream_t stream)
{
    const void *f = pick_kernel(precision, form, spec, a.drain_iters > 0 || a.n_resume > 0, a.jobs_lds != 0);
    if (!f) return hipErrorInvalidValue;
    if (lds_bytes > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
        if (e != hipSuccess) return e;
    }
    KArgs arg = a;
    void *params[] = {&arg};
    return hipLaunchKernel(f, dim3(grid), dim3(block), params, lds_bytes, stream);
}

hipError_t launch_fill(double *p, size_t n_doubles, unsigned long long *q, size_t n_u64, hipStream_t stream)
{
    const size_t n = n_doubles > n_u64 ? n_doubles : n_u64;
    size_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks == 0) blocks = 1;
    hipLaunchKernelGGL(fill_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, p, n_doubles, q, n_u64);
    return hipGetLastError();
}

hipError_t launch_debug_philox(uint64_t seed, const uint64_t *pid, const uint32_t *k, const uint32_t *tag,
                               uint32_t *out, size_t n, hipStream_t stream)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(debug_philox_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, seed, pid, k, tag,
                       out, n);
    return hipGetLastError();
}

hipError_t launch_debug_alias(const uint32_t *packed, int bits, const uint32_t *words, uint32_t *states, size_t n,
                              hipStream_t stream)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(debug_alias_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, packed, bits, words,
                       states, n);
    return hipGetLastError();
}

int max_lds_bytes() { return 160 * 1024; }

int occupancy_blocks(int precision, int form, int spec, bool bounded, bool jl, int block, size_t lds_bytes)
{
    const void *f = pick_kernel(precision, form, spec, bounded, jl);
    if (!f) return 1;
    if (lds_bytes > 64 * 1024) {
        if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes) != hipSuccess) {
            (void)hipGetLastError();
            return 1;
        }
    }
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, block, lds_bytes) != hipSuccess) {
        (void)hipGetLastError();
        return 1;
    }
    return n > 0 ? n : 1;
}

}  // namespace dmc
