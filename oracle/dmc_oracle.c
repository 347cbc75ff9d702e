/*
 * dmc_oracle.c -- plain FP64 CPU oracle of the linearized energy-based
 * deviational Monte Carlo method for the phonon Boltzmann equation in the
 * relaxation-time approximation (Peraud & Hadjiconstantinou, "An alternative
 * approach to efficient simulation of micro/nanoscale phonon transport").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference that the GPU library is checked against.  Only the tests, the
 * smoke check and the benchmark's CPU-baseline leg may load it.  It shares no
 * code with the GPU library: the Philox generator, the alias-table builder,
 * the heat-capacity tabulation, the samplers, the ray/surface intersection and
 * the scoring below are written here independently.
 *
 * What each part follows:
 *   - philox4x32_10: the Philox-4x32 counter-based generator with 10 rounds of
 *     Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as easy as 1, 2, 3"
 *     (SC'11), section 3: multiply-hi/lo S-box with two multipliers, a Weyl key
 *     schedule, and the word permutation of the 4x32 variant.
 *   - oracle_tabulate: de^eq/dT of the Bose-Einstein energy (defined after
 *     Eq. (1)) and the per-state heat capacity D de^eq/dT domega g.
 *   - oracle_alias: Walker/Vose alias table on exact integer masses (the
 *     normalised gain distribution of Eq. (2) and the source distributions of
 *     the source-term paragraph are sampled with it).
 *   - oracle_run: steps I-VI of the particle algorithm, the steady
 *     track-length estimator (Eq. (4), algebraic-length form for the heat
 *     flux) and the transient estimator (Eq. (3)), the imposed-gradient source
 *     (Eq. (6)) with periodic reinsertion, and truncation after a fixed number
 *     of scattering events (the H_j discussion of the periodic-nanostructure
 *     application).
 *
 * Every floating-point quantity is FP64.  Loops are deliberately unblocked
 * and unfused: per-bin scoring loops over every bin.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_HBAR 1.054571817e-34 /* J s (CODATA 2018) */
#define OR_KB 1.380649e-23      /* J/K (CODATA 2018) */

/* ------------------------------------------------------------------------ */
/* Philox4x32-10                                                             */
/* ------------------------------------------------------------------------ */

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    /* multipliers and Weyl increments of the Philox4x32 family (SC'11, sec. 3.3) */
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += W0; k1 += W1; }
        uint64_t p0 = (uint64_t)M0 * (uint64_t)x0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Counter layout: (pid low word, pid high word, k, tag); key = seed words. */
enum { OR_TAG_STEP = 0, OR_TAG_EMIT_A = 1, OR_TAG_EMIT_B = 2 };

static void rng_block(uint64_t seed, uint64_t pid, uint32_t k, uint32_t tag, uint32_t w[4])
{
    uint32_t ctr[4] = {(uint32_t)pid, (uint32_t)(pid >> 32), k, tag};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    oracle_philox4x32_10(ctr, key, w);
}

/* R in ]0,1[ (step II): (w + 1/2) 2^-32, exact in FP64. */
static double unif(uint32_t w) { return ((double)w + 0.5) * (1.0 / 4294967296.0); }

/* ------------------------------------------------------------------------ */
/* Elementary functions from IEEE basic operations                          */
/* ------------------------------------------------------------------------ */
/* The reference fixes its logarithm and its sine/cosine of 2 pi u to these
 * algorithms (only +, -, *, /, floor and frexp, no contraction), so that any
 * implementation following the same steps reproduces every trajectory bit for
 * bit.  Trajectories among convex pores are chaotic: a one-ulp difference in a
 * library logarithm or cosine grows until the path changes.  Accuracy is about
 * one ulp (pinned against the C library in the tests). */

static const double OR_LN2_HI = 0x1.62e42ff000000p-1; /* ln 2 to 32 bits: e * hi is exact */
static const double OR_LN2_LO = -0x1.718432a1b0e26p-35; /* ln 2 - hi */
static const double OR_SQRT_HALF = 0x1.6a09e667f3bcdp-1;
static const double OR_PIO2 = 0x1.921fb54442d18p+0;  /* pi / 2 rounded to double */

/* log x for normal x > 0: x = m 2^e with m in [sqrt(1/2), sqrt(2)),
 * log m = 2 atanh(s) = 2 s sum_k s^(2k) / (2k + 1), s = (m - 1)/(m + 1),
 * |s| <= 0.1716, series to s^23 (next term below 1e-18 relative). */
double oracle_log(double x)
{
    int e;
    double m = frexp(x, &e); /* m in [0.5, 1) */
    if (m < OR_SQRT_HALF) { m = m * 2.0; e = e - 1; }
    double s = (m - 1.0) / (m + 1.0);
    double z = s * s;
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
    double lm = (2.0 * s) * p;
    double de = (double)e;
    return de * OR_LN2_HI + (de * OR_LN2_LO + lm);
}

/* sin and cos of 2 pi u for u in [0, 1): v = 4u quarter turns (exact), nearest
 * quarter k, r = v - k in [-1/2, 1/2] (exact), t = r pi/2 in [-pi/4, pi/4],
 * Taylor series of sin t to t^17 and cos t to t^18, then the quadrant k. */
void oracle_sincos2pi(double u, double *sn, double *cs)
{
    double v = 4.0 * u;
    double k = floor(v + 0.5);
    double r = v - k;
    double t = r * OR_PIO2;
    double t2 = t * t;
    double ps = -1.0 / 355687428096000.0;            /* -1/17! */
    ps = ps * t2 + 1.0 / 1307674368000.0;            /* 1/15! */
    ps = ps * t2 - 1.0 / 6227020800.0;               /* 1/13! */
    ps = ps * t2 + 1.0 / 39916800.0;                 /* 1/11! */
    ps = ps * t2 - 1.0 / 362880.0;                   /* 1/9! */
    ps = ps * t2 + 1.0 / 5040.0;                     /* 1/7! */
    ps = ps * t2 - 1.0 / 120.0;                      /* 1/5! */
    ps = ps * t2 + 1.0 / 6.0;                        /* 1/3! */
    double st = t - t * (t2 * ps);
    double pc = 1.0 / 6402373705728000.0;            /* 1/18! */
    pc = pc * t2 - 1.0 / 20922789888000.0;           /* 1/16! */
    pc = pc * t2 + 1.0 / 87178291200.0;              /* 1/14! */
    pc = pc * t2 - 1.0 / 479001600.0;                /* 1/12! */
    pc = pc * t2 + 1.0 / 3628800.0;                  /* 1/10! */
    pc = pc * t2 - 1.0 / 40320.0;                    /* 1/8! */
    pc = pc * t2 + 1.0 / 720.0;                      /* 1/6! */
    pc = pc * t2 - 1.0 / 24.0;                       /* 1/4! */
    pc = pc * t2 + 1.0 / 2.0;                        /* 1/2! */
    double ct = 1.0 - t2 * pc;
    int q = ((int)k) & 3;
    if (q == 0) { *sn = st; *cs = ct; }
    else if (q == 1) { *sn = ct; *cs = -st; }
    else if (q == 2) { *sn = -st; *cs = -ct; }
    else { *sn = -ct; *cs = st; }
}

/* ------------------------------------------------------------------------ */
/* Material tabulation                                                      */
/* ------------------------------------------------------------------------ */

/* de^eq/dT of e^eq = hbar omega / (exp(hbar omega / k_B T) - 1) per state and
 * the heat capacity C_m = D de/dT domega g.  sums = {sum C, sum C/tau, sum C v}
 * accumulated in index order.  Returns 0, or -1 on a non-physical input. */
int oracle_tabulate(int32_t K, const double *omega, const double *domega, const double *dos,
                    const double *vg, const double *tau, const double *deg, double T_eq,
                    double *dedT_out, double *C_out, double sums[3])
{
    if (K <= 0 || !(T_eq > 0.0)) return -1;
    sums[0] = sums[1] = sums[2] = 0.0;
    for (int32_t m = 0; m < K; ++m) {
        if (!(omega[m] > 0.0) || !(domega[m] >= 0.0) || !(dos[m] >= 0.0) || !(vg[m] > 0.0) ||
            !(tau[m] > 0.0) || !(deg[m] >= 0.0))
            return -1;
        double x = (OR_HBAR * omega[m]) / (OR_KB * T_eq);
        double ex = exp(x);
        double em1 = expm1(x);
        double dedT = OR_KB * x * x * ex / (em1 * em1);
        double C = ((dos[m] * dedT) * domega[m]) * deg[m];
        dedT_out[m] = dedT;
        C_out[m] = C;
        sums[0] += C;
        sums[1] += C / tau[m];
        sums[2] += C * vg[m];
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Alias tables on exact integer masses                                     */
/* ------------------------------------------------------------------------ */

/* Number of index bits b of the padded table: K_pad = 2^b >= max(K, 2). */
int32_t oracle_alias_bits(int32_t K)
{
    int32_t b = 1;
    while ((1 << b) < K) ++b;
    return b;
}

/* Integer masses q_j (sum exactly 2^32) for weights w_j (j < K, zero for the
 * padding up to 2^b): floor of (w_j / W) 2^32 with W the index-order sum, and
 * the remaining units given one each to the largest fractional parts (ties to
 * the lower index).  Then Vose's construction: columns of capacity U = 2^(32-b);
 * small (q < U) and large (q >= U) columns are FIFO queues in index order; each
 * step pairs the front small column l with the front large column g, sets
 * thresh[l] = q_l, alias[l] = g, removes (U - q_l) from g and re-queues g at the
 * back of the queue it now belongs to.  Columns left over are full:
 * thresh = U, alias = self.  Lookup with one word w: idx = w >> (32 - b), keep
 * idx iff (w & (U - 1)) < thresh[idx], else alias[idx].  Returns b, or -1. */
int32_t oracle_alias(int32_t K, const double *w, uint64_t *q_out, uint32_t *thresh, uint32_t *alias)
{
    if (K <= 0 || K > 65536) return -1;
    int32_t b = oracle_alias_bits(K);
    int32_t n = 1 << b;
    double W = 0.0;
    for (int32_t j = 0; j < K; ++j) {
        if (!(w[j] >= 0.0) || !isfinite(w[j])) return -1;
        W += w[j];
    }
    if (!(W > 0.0) || !isfinite(W)) return -1;
    uint64_t *q = (uint64_t *)calloc((size_t)n, sizeof(uint64_t));
    double *frac = (double *)calloc((size_t)n, sizeof(double));
    int32_t *order = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    int32_t *small = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    int32_t *large = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    uint64_t total = 0;
    for (int32_t j = 0; j < n; ++j) {
        double s = (j < K) ? (w[j] / W) * 4294967296.0 : 0.0;
        double f = floor(s);
        q[j] = (uint64_t)f;
        frac[j] = s - f;
        total += q[j];
        order[j] = j;
    }
    /* largest remainders first; stable insertion sort keeps the lower index first on ties */
    for (int32_t i = 1; i < n; ++i) {
        int32_t v = order[i];
        int32_t p = i - 1;
        while (p >= 0 && frac[order[p]] < frac[v]) { order[p + 1] = order[p]; --p; }
        order[p + 1] = v;
    }
    uint64_t rem = (1ull << 32) - total;
    for (uint64_t i = 0; i < rem; ++i) q[order[i]] += 1;

    const uint64_t U = 1ull << (32 - b);
    /* FIFO ring queues: each holds at most n columns at a time */
    int32_t sh = 0, sc = 0, lh = 0, lc = 0; /* head index and count */
    for (int32_t j = 0; j < n; ++j) {
        if (q_out) q_out[j] = q[j];
        if (q[j] < U) small[(sh + sc++) % n] = j;
        else large[(lh + lc++) % n] = j;
    }
    while (sc > 0 && lc > 0) {
        int32_t l = small[sh]; sh = (sh + 1) % n; --sc;
        int32_t g = large[lh]; lh = (lh + 1) % n; --lc;
        thresh[l] = (uint32_t)q[l];
        alias[l] = (uint32_t)g;
        q[g] -= (U - q[l]);
        if (q[g] < U) small[(sh + sc++) % n] = g;
        else large[(lh + lc++) % n] = g;
    }
    while (lc > 0) { int32_t g = large[lh]; lh = (lh + 1) % n; --lc; thresh[g] = (uint32_t)U; alias[g] = (uint32_t)g; }
    while (sc > 0) { int32_t l = small[sh]; sh = (sh + 1) % n; --sc; thresh[l] = (uint32_t)U; alias[l] = (uint32_t)l; }
    free(q); free(frac); free(order); free(small); free(large);
    return b;
}

static uint32_t alias_draw(uint32_t w, int32_t b, const uint32_t *thresh, const uint32_t *alias)
{
    uint32_t idx = w >> (32 - b);
    uint32_t low = w & ((1u << (32 - b)) - 1u);
    return (low < thresh[idx]) ? idx : alias[idx];
}

/* ------------------------------------------------------------------------ */
/* Problem description                                                      */
/* ------------------------------------------------------------------------ */

enum { OR_GEOM_SLAB_Z = 0, OR_GEOM_FILM_X = 1, OR_GEOM_PORE_XZ = 2, OR_GEOM_HALFSPACE_Z = 3 };
enum { OR_WALL_ISOTHERMAL = 0, OR_WALL_ADIABATIC = 1, OR_WALL_PERIODIC = 2 };
enum { OR_SRC_WALLS = 0, OR_SRC_GAUSSIAN = 1, OR_SRC_GRADIENT = 2 };
#define OR_NO_SURFACE (-1)
#define OR_ITER_CAP (1u << 24)
#define OR_POS_ATTEMPTS 64

typedef struct {
    /* material */
    int32_t K;
    const double *v;   /* group speed per state */
    const double *tau; /* relaxation time per state */
    int32_t gain_bits; const uint32_t *gain_thresh, *gain_alias; /* C/tau   */
    int32_t init_bits; const uint32_t *init_thresh, *init_alias; /* C       */
    int32_t flux_bits; const uint32_t *flux_thresh, *flux_alias; /* C v     */
    /* sources: n_src terms chosen by an alias over their powers */
    int32_t n_src; int32_t src_bits; const uint32_t *src_thresh, *src_alias;
    const int32_t *src_wall; /* walls source: source j -> wall index */
    /* geometry */
    int32_t geom; double length, radius;
    int32_t wall_type[2]; double wall_T[2]; uint64_t wall_spec[2]; /* specular iff w < wall_spec */
    /* source */
    int32_t src_kind; double T_eq, dT, r0, G;
    /* tallies */
    int32_t n_bins, n_batches, kmax, n_hj, n_times;
    const double *times;
    int32_t grid[3]; double grid_lo[3], grid_hi[3];
    uint64_t seed;
    /* in-plane film: end a trajectory at its first scattering event or first
     * diffuse wall reflection (the flux carried afterwards averages to zero) */
    int32_t first_event;
    /* time-windowed track-length tally in a z-aligned cylinder (transient jobs):
     * region_kind 1 = {(x-cx)^2 + (y-cy)^2 < R^2, zlo <= z < zhi}; windows
     * [0, t_0), [t_0, t_1), ... [t_{n-2}, t_{n-1}) from the snapshot times */
    int32_t region_kind;
    double region_c[2], region_r, region_z[2];
    /* steady pore cell: field of field_n[0] x field_n[1] cells over
     * [field_lo, field_hi) in (x, z) (0 cells: none); Eq. (4) in every cell */
    int32_t field_n[2];
    double field_lo[2], field_hi[2];
    /* mean cosine g of the angle between the directions before and after a
     * scattering event (Henyey-Greenstein phase function); 0: isotropic */
    double scatter_g;
} oracle_problem;

typedef struct {
    uint64_t particles, scatters, boundary, iterations, absorbed, capped, periodic;
} oracle_counters;

/* offsets of the tally sections inside the flat FP64 output buffer */
typedef struct { size_t bins, kappa, hj, snap, snap_abs, region, field, total; int64_t ncell; } tally_layout;

static tally_layout layout_of(const oracle_problem *P)
{
    tally_layout t;
    size_t o = 0;
    t.bins = o; o += (size_t)P->n_batches * 3 * (size_t)P->n_bins;
    t.kappa = o; o += 2;
    t.hj = o; o += 2 * (size_t)P->n_hj;
    t.ncell = (int64_t)P->grid[0] * P->grid[1] * P->grid[2];
    t.snap = o; o += (size_t)P->n_times * (size_t)(t.ncell + 1);
    t.snap_abs = o; o += (size_t)P->n_times * (size_t)(t.ncell + 1);
    /* per window: sum of each particle's s * (time in region), its square, the
     * same for s * (z displacement in region) */
    t.region = o; o += (P->region_kind && P->n_times > 0) ? (size_t)4 * (size_t)P->n_times : 0;
    /* per batch: TIME (s t_c) and DISPZ (s v Omega_z t_c) of every field cell, x fastest */
    t.field = o; o += (size_t)P->n_batches * 2 * (size_t)P->field_n[0] * (size_t)P->field_n[1];
    t.total = o;
    return t;
}

size_t oracle_tally_size(const oracle_problem *P) { return layout_of(P).total; }

/* ------------------------------------------------------------------------ */
/* Particle state and its pieces                                            */
/* ------------------------------------------------------------------------ */

typedef struct {
    double x[3];   /* position */
    double o[3];   /* unit direction Omega */
    uint32_t m;    /* state (omega bin, polarization) */
    double s;      /* sign +1 / -1 */
    int32_t last;  /* surface the particle rests on, excluded from the next search */
} particle;

/* Direction with polar cosine mu about the unit normal n and azimuth
 * phi = 2 pi u, in the tangent frame (t1, t2):
 * Omega = mu n + sqrt(1-mu^2)(cos phi t1 + sin phi t2). */
static void dir_about(double mu, double u, const double n[3], const double t1[3], const double t2[3], double o[3])
{
    double st = sqrt(1.0 - mu * mu);
    double c, s;
    oracle_sincos2pi(u, &s, &c);
    for (int i = 0; i < 3; ++i) o[i] = mu * n[i] + st * (c * t1[i] + s * t2[i]);
}

static const double EX[3] = {1, 0, 0}, EY[3] = {0, 1, 0}, EZ[3] = {0, 0, 1};

/* Isotropic direction (step IVb): mu = 2u - 1 along z, azimuth about z from x. */
static void isotropic(uint32_t w2, uint32_t w3, double o[3])
{
    double mu = 2.0 * unif(w2) - 1.0;
    dir_about(mu, unif(w3), EZ, EX, EY, o);
}

/* Direction after a scattering event (step IVb).  g = 0: isotropic, the step as
 * the paper states it.  g != 0: the generalisation the paper allows there; the
 * cosine mu of the angle to the incoming direction n follows the Henyey-Greenstein
 * phase function p(mu) = (1 - g^2) / (2 (1 + g^2 - 2 g mu)^(3/2)) of mean g,
 * drawn by inverting its cumulative distribution,
 *   mu = (1 + g^2 - f^2) / (2 g),  f = (1 - g^2) / (1 - g + 2 g u),
 * and the azimuth is uniform in the frame t1 = (n_x n_z, n_y n_z, -s) / s,
 * t2 = (-n_y, n_x, 0) / s, s = sqrt(n_x^2 + n_y^2) (x, y for n along z). */
static void scatter_direction(double g, uint32_t w2, uint32_t w3, double o[3])
{
    if (g == 0.0) {
        isotropic(w2, w3, o);
        return;
    }
    double u = unif(w2);
    double f = (1.0 - g * g) / (1.0 - g + 2.0 * g * u);
    double mu = (1.0 + g * g - f * f) / (2.0 * g);
    if (mu > 1.0) mu = 1.0;
    if (mu < -1.0) mu = -1.0;
    double n[3] = {o[0], o[1], o[2]};
    double s2 = n[0] * n[0] + n[1] * n[1];
    if (s2 > 1e-12) {
        double s = sqrt(s2);
        double t1[3] = {n[0] * n[2] / s, n[1] * n[2] / s, -s};
        double t2[3] = {-n[1] / s, n[0] / s, 0.0};
        dir_about(mu, unif(w3), n, t1, t2, o);
    } else {
        dir_about(mu, unif(w3), n, EX, EY, o);
    }
}

/* Lambertian (cosine-weighted) direction about an inward normal: mu = sqrt(u).
 * Tangent frames: normal +-z -> (x, y); normal +-x -> (y, z). */
static void lambertian_plane(int axis, double sgn, uint32_t w2, uint32_t w3, double o[3])
{
    double mu = sqrt(unif(w2));
    double n[3] = {0, 0, 0};
    n[axis] = sgn;
    if (axis == 2) dir_about(mu, unif(w3), n, EX, EY, o);
    else dir_about(mu, unif(w3), n, EY, EZ, o);
}

/* Step I: draw sign, position, state and direction from the source term. */
static void emit(const oracle_problem *P, uint64_t pid, particle *p)
{
    uint32_t a[4], b[4];
    rng_block(P->seed, pid, 0, OR_TAG_EMIT_A, a);
    memset(p, 0, sizeof(*p));
    p->last = OR_NO_SURFACE;
    if (P->src_kind == OR_SRC_WALLS) {
        uint32_t j = (P->n_src > 1) ? alias_draw(a[0], P->src_bits, P->src_thresh, P->src_alias) : 0;
        int32_t wall = P->src_wall[j];
        p->m = alias_draw(a[1], P->flux_bits, P->flux_thresh, P->flux_alias);
        int axis = (P->geom == OR_GEOM_FILM_X) ? 0 : 2;
        double sgn = (wall == 0) ? 1.0 : -1.0; /* inward normal */
        lambertian_plane(axis, sgn, a[2], a[3], p->o);
        p->x[axis] = (wall == 0) ? 0.0 : P->length;
        p->last = wall;
        p->s = (P->wall_T[wall] > P->T_eq) ? 1.0 : -1.0;
    } else if (P->src_kind == OR_SRC_GAUSSIAN) {
        /* initial condition C |T_i - T_eq| delta(t): state ~ C, isotropic, position
         * ~ exp(-|x|^2/r0^2) restricted to z >= 0 (Box-Muller, sigma = r0/sqrt 2). */
        rng_block(P->seed, pid, 0, OR_TAG_EMIT_B, b);
        p->m = alias_draw(a[1], P->init_bits, P->init_thresh, P->init_alias);
        isotropic(a[2], a[3], p->o);
        double sigma = P->r0 / sqrt(2.0);
        double rho = sqrt(-2.0 * oracle_log(unif(b[0])));
        double c1, s1, c2, s2;
        oracle_sincos2pi(unif(b[1]), &s1, &c1);
        p->x[0] = sigma * rho * c1;
        p->x[1] = sigma * rho * s1;
        double rz = sqrt(-2.0 * oracle_log(unif(b[2])));
        oracle_sincos2pi(unif(b[3]), &s2, &c2);
        p->x[2] = fabs(sigma * rz * c2);
        p->s = (P->dT > 0.0) ? 1.0 : -1.0;
    } else { /* OR_SRC_GRADIENT, Eq. (6): state ~ C v, |cos theta| weighted, uniform in the solid */
        rng_block(P->seed, pid, 0, OR_TAG_EMIT_B, b);
        p->m = alias_draw(a[1], P->flux_bits, P->flux_thresh, P->flux_alias);
        double sz = (b[3] >> 31) ? -1.0 : 1.0;
        lambertian_plane(2, sz, a[2], a[3], p->o);
        p->s = (-p->o[2] * P->G > 0.0) ? 1.0 : -1.0;
        if (P->geom == OR_GEOM_FILM_X) {
            p->x[0] = P->length * unif(b[0]);
        } else { /* pore cell: rejection in the unit cell */
            double c = 0.5 * P->length, r2 = P->radius * P->radius;
            int ok = 0;
            for (uint32_t att = 0; att < OR_POS_ATTEMPTS && !ok; ++att) {
                uint32_t bb[4];
                rng_block(P->seed, pid, att, OR_TAG_EMIT_B, bb);
                double x = P->length * unif(bb[0]), z = P->length * unif(bb[1]);
                if ((x - c) * (x - c) + (z - c) * (z - c) > r2) { p->x[0] = x; p->x[2] = z; ok = 1; }
            }
            if (!ok) { p->x[0] = 0.0; p->x[2] = 0.0; }
        }
    }
}

/* Step III: earliest surface hit time along x + v Omega t, excluding the
 * surface the particle rests on.  Returns INFINITY if none. */
static double boundary_search(const oracle_problem *P, const particle *p, double v, int32_t *surf)
{
    double best = INFINITY;
    *surf = OR_NO_SURFACE;
    if (P->geom == OR_GEOM_SLAB_Z || P->geom == OR_GEOM_FILM_X) {
        int ax = (P->geom == OR_GEOM_SLAB_Z) ? 2 : 0;
        double w = v * p->o[ax];
        if (w > 0.0 && p->last != 1) { best = (P->length - p->x[ax]) / w; *surf = 1; }
        else if (w < 0.0 && p->last != 0) { best = (0.0 - p->x[ax]) / w; *surf = 0; }
    } else if (P->geom == OR_GEOM_HALFSPACE_Z) {
        double w = v * p->o[2];
        if (w < 0.0 && p->last != 0) { best = (0.0 - p->x[2]) / w; *surf = 0; }
    } else { /* pore cell: faces 0: x=0, 1: x=P, 2: z=0, 3: z=P, 4: pore */
        const int axes[2] = {0, 2};
        for (int f = 0; f < 2; ++f) {
            int ax = axes[f];
            double w = v * p->o[ax];
            double t = INFINITY; int32_t id = OR_NO_SURFACE;
            if (w > 0.0 && p->last != 2 * f + 1) { t = (P->length - p->x[ax]) / w; id = 2 * f + 1; }
            else if (w < 0.0 && p->last != 2 * f) { t = (0.0 - p->x[ax]) / w; id = 2 * f; }
            if (t < best) { best = t; *surf = id; }
        }
        if (P->radius > 0.0 && p->last != 4) {
            double c = 0.5 * P->length;
            double dx = p->x[0] - c, dz = p->x[2] - c;
            double a = p->o[0] * p->o[0] + p->o[2] * p->o[2];
            double bq = dx * p->o[0] + dz * p->o[2];
            double cq = dx * dx + dz * dz - P->radius * P->radius;
            if (a > 0.0 && bq < 0.0) {
                double dist = INFINITY;
                if (cq <= 0.0) dist = 0.0;
                else {
                    double disc = bq * bq - a * cq;
                    if (disc > 0.0) dist = (-bq - sqrt(disc)) / a;
                }
                double t = dist / v;
                if (t < best) { best = t; *surf = 4; }
            }
        }
    }
    return best;
}

/* Step IVa: interaction with the surface just reached. Returns 1 if absorbed. */
static int wall_interaction(const oracle_problem *P, particle *p, int32_t surf, const uint32_t w[4],
                            oracle_counters *cnt)
{
    if (P->geom == OR_GEOM_PORE_XZ) {
        if (surf < 4) { /* periodic reinsertion through the opposite face */
            int ax = (surf < 2) ? 0 : 2;
            if (surf % 2 == 1) { p->x[ax] = 0.0; p->last = surf - 1; }
            else { p->x[ax] = P->length; p->last = surf + 1; }
            cnt->periodic++;
            return 0;
        }
        /* pore surface: normal pointing from the pore axis into the solid */
        double c = 0.5 * P->length;
        double nx = p->x[0] - c, nz = p->x[2] - c;
        double nn = sqrt(nx * nx + nz * nz);
        double n[3] = {nx / nn, 0.0, nz / nn};
        if ((uint64_t)w[1] < P->wall_spec[0]) {
            double dn = p->o[0] * n[0] + p->o[2] * n[2];
            for (int i = 0; i < 3; ++i) p->o[i] -= 2.0 * dn * n[i];
        } else {
            double t2[3] = {-n[2], 0.0, n[0]};
            double mu = sqrt(unif(w[2]));
            dir_about(mu, unif(w[3]), n, EY, t2, p->o);
        }
        p->last = 4;
        return 0;
    }
    int wall = (P->geom == OR_GEOM_HALFSPACE_Z) ? 0 : surf;
    int ax = (P->geom == OR_GEOM_FILM_X) ? 0 : 2;
    int32_t type = P->wall_type[wall];
    if (type == OR_WALL_ISOTHERMAL) { cnt->absorbed++; return 1; }
    if (type == OR_WALL_PERIODIC) {
        /* a plane pair that is periodic: reinsert at the opposite wall */
        if (wall == 1) { p->x[ax] = 0.0; p->last = 0; } else { p->x[ax] = P->length; p->last = 1; }
        cnt->periodic++;
        return 0;
    }
    /* adiabatic: specular with probability p, else diffuse (Lambertian about the inward normal) */
    if ((uint64_t)w[1] < P->wall_spec[wall]) {
        p->o[ax] = -p->o[ax];
    } else {
        if (P->first_event) return 1; /* a diffuse reflection ends the first free path */
        lambertian_plane(ax, (wall == 0) ? 1.0 : -1.0, w[2], w[3], p->o);
    }
    p->last = wall;
    return 0;
}

/* Time spent in each 1-D bin along `ax` by a segment; adds the three tallies
 * TIME (s t_k), PTIME (s t_k / tau), DISP (s v Omega_z t_k) of batch `bt`. */
static void score_bins(const oracle_problem *P, double *bins, int bt, const particle *p, double v, double tau_m,
                       double seg)
{
    int ax = (P->geom == OR_GEOM_FILM_X) ? 0 : 2;
    int nb = P->n_bins;
    double L = P->length;
    double ca = p->x[ax];
    double wa = v * p->o[ax];
    double cb = ca + wa * seg;
    double lo = (ca < cb) ? ca : cb, hi = (ca < cb) ? cb : ca;
    double *T = bins + ((size_t)bt * 3 + 0) * nb;
    double *PT = bins + ((size_t)bt * 3 + 1) * nb;
    double *D = bins + ((size_t)bt * 3 + 2) * nb;
    double vz = v * p->o[2];
    if (wa == 0.0) {
        int k = (int)floor(ca * nb / L);
        if (k < 0) k = 0;
        if (k > nb - 1) k = nb - 1;
        T[k] += p->s * seg;
        PT[k] += p->s * seg / tau_m;
        D[k] += p->s * vz * seg;
        return;
    }
    for (int k = 0; k < nb; ++k) {
        double blo = L * k / nb, bhi = L * (k + 1) / nb;
        double a = (lo > blo) ? lo : blo;
        double b = (hi < bhi) ? hi : bhi;
        if (b > a) {
            double tk = (b - a) / fabs(wa);
            T[k] += p->s * tk;
            PT[k] += p->s * tk / tau_m;
            D[k] += p->s * vz * tk;
        }
    }
}

/* The part [a, b] of u in [0, seg] where c + w u lies in [e0, e1); 0 if none. */
static int axis_interval(double c, double w, double e0, double e1, double seg, double *a, double *b)
{
    if (w == 0.0) {
        if (!(c >= e0 && c < e1)) return 0;
        *a = 0.0;
        *b = seg;
        return 1;
    }
    double ta = (e0 - c) / w, tb = (e1 - c) / w;
    if (ta > tb) { double t = ta; ta = tb; tb = t; }
    *a = (ta > 0.0) ? ta : 0.0;
    *b = (tb < seg) ? tb : seg;
    return *b > *a;
}

/* Steady field: Eq. (4) applied to every cell of an x-z grid.  The segment
 * x + v Omega u, u in [0, seg], spends in cell c the time of the overlap of its
 * x and z intervals there: TIME_c += s t_c, DISPZ_c += s v Omega_z t_c (batch bt).
 * Every cell is visited (slow and plain). */
static void score_field(const oracle_problem *P, double *fld, int bt, const particle *p, double v, double seg)
{
    int nx = P->field_n[0], nz = P->field_n[1];
    double wx = v * p->o[0], wz = v * p->o[2];
    double *T = fld + ((size_t)bt * 2 + 0) * (size_t)nx * nz;
    double *D = fld + ((size_t)bt * 2 + 1) * (size_t)nx * nz;
    for (int iz = 0; iz < nz; ++iz) {
        double z0 = P->field_lo[1] + (P->field_hi[1] - P->field_lo[1]) * iz / nz;
        double z1 = P->field_lo[1] + (P->field_hi[1] - P->field_lo[1]) * (iz + 1) / nz;
        double za, zb;
        if (!axis_interval(p->x[2], wz, z0, z1, seg, &za, &zb)) continue;
        for (int ix = 0; ix < nx; ++ix) {
            double x0 = P->field_lo[0] + (P->field_hi[0] - P->field_lo[0]) * ix / nx;
            double x1 = P->field_lo[0] + (P->field_hi[0] - P->field_lo[0]) * (ix + 1) / nx;
            double xa, xb;
            if (!axis_interval(p->x[0], wx, x0, x1, seg, &xa, &xb)) continue;
            double a = (xa > za) ? xa : za, b = (xb < zb) ? xb : zb;
            if (b > a) {
                T[(size_t)iz * nx + ix] += p->s * (b - a);
                D[(size_t)iz * nx + ix] += p->s * wz * (b - a);
            }
        }
    }
}

/* Transient estimator (Eq. (3)) at the snapshot times inside [ta, ta + seg):
 * the particle's position there, by linear interpolation along the segment,
 * selects the grid cell (or the overflow slot) that receives s. */
static void score_snapshots(const oracle_problem *P, double *snap, double *snap_abs, int64_t ncell,
                            const particle *p, double v, double ta, double seg)
{
    double tb = ta + seg;
    for (int32_t j = 0; j < P->n_times; ++j) {
        double tj = P->times[j];
        if (!(tj >= ta && tj < tb)) continue;
        double dt = tj - ta;
        int64_t idx[3];
        int inside = 1;
        for (int d = 0; d < 3; ++d) {
            double xd = p->x[d] + v * p->o[d] * dt;
            double f = (xd - P->grid_lo[d]) / (P->grid_hi[d] - P->grid_lo[d]) * P->grid[d];
            double fl = floor(f);
            if (!(fl >= 0.0 && fl < (double)P->grid[d])) { inside = 0; break; }
            idx[d] = (int64_t)fl;
        }
        int64_t cell = inside ? (idx[2] * P->grid[1] + idx[1]) * P->grid[0] + idx[0] : ncell;
        snap[(size_t)j * (size_t)(ncell + 1) + (size_t)cell] += p->s;
        snap_abs[(size_t)j * (size_t)(ncell + 1) + (size_t)cell] += 1.0;
    }
}

/* Time-averaged estimator (the sampling of the steady-state paragraph applied
 * over a finite window): the part [u0, u1] of the segment x + v Omega u,
 * u in [0, seg], that lies in the region; returns 0 if there is none. */
static int region_interval(const oracle_problem *P, const particle *p, double v, double seg, double *u0, double *u1)
{
    double lo = 0.0, hi = seg;
    /* the slab zlo <= z < zhi */
    double wz = v * p->o[2];
    if (wz == 0.0) {
        if (!(p->x[2] >= P->region_z[0] && p->x[2] < P->region_z[1])) return 0;
    } else {
        double ta = (P->region_z[0] - p->x[2]) / wz, tb = (P->region_z[1] - p->x[2]) / wz;
        if (ta > tb) { double s = ta; ta = tb; tb = s; }
        if (ta > lo) lo = ta;
        if (tb < hi) hi = tb;
    }
    /* the cylinder (x - cx)^2 + (y - cy)^2 < R^2 */
    double wx = v * p->o[0], wy = v * p->o[1];
    double dx = p->x[0] - P->region_c[0], dy = p->x[1] - P->region_c[1];
    double a = wx * wx + wy * wy, b = dx * wx + dy * wy, cc = dx * dx + dy * dy - P->region_r * P->region_r;
    if (a == 0.0) {
        if (!(cc < 0.0)) return 0;
    } else {
        double disc = b * b - a * cc;
        if (!(disc > 0.0)) return 0;
        double sq = sqrt(disc);
        double ta = (-b - sq) / a, tb = (-b + sq) / a;
        if (ta > lo) lo = ta;
        if (tb < hi) hi = tb;
    }
    if (!(hi > lo)) return 0;
    *u0 = lo;
    *u1 = hi;
    return 1;
}

/* Adds s * (time in region) and s * (z displacement in region) of a segment
 * starting at time ta to the particle's per-window sums rt, rq. */
static void score_region(const oracle_problem *P, double *rt, double *rq, const particle *p, double v, double ta,
                         double seg)
{
    double u0, u1;
    if (!region_interval(P, p, v, seg, &u0, &u1)) return;
    double a = ta + u0, b = ta + u1, w0 = 0.0;
    for (int32_t j = 0; j < P->n_times; ++j) {
        double w1 = P->times[j];
        double lo = (a > w0) ? a : w0, hi = (b < w1) ? b : w1;
        if (hi > lo) {
            rt[j] += p->s * (hi - lo);
            rq[j] += p->s * v * p->o[2] * (hi - lo);
        }
        w0 = w1;
    }
}

/* ------------------------------------------------------------------------ */
/* Steps I-VI for particles pid0 .. pid1-1                                  */
/* ------------------------------------------------------------------------ */

/* Adds this range's contributions to `tally` (size oracle_tally_size) and the
 * event counters to `cnt`; optionally writes each particle's number of
 * scattering events to nscat_out[pid - pid0] and counts the post-scattering
 * states in scatter_hist[m].  Returns 0 or -1. */
int oracle_run(const oracle_problem *P, uint64_t pid0, uint64_t pid1, double *tally, oracle_counters *cnt,
               uint32_t *nscat_out, uint64_t *scatter_hist)
{
    tally_layout lay = layout_of(P);
    int transient = P->n_times > 0;
    double t_final = transient ? P->times[P->n_times - 1] : INFINITY;
    double *h = (P->n_hj > 0) ? (double *)calloc((size_t)P->n_hj, sizeof(double)) : NULL;
    int region = P->region_kind && transient;
    double *rt = region ? (double *)calloc((size_t)P->n_times, sizeof(double)) : NULL;
    double *rq = region ? (double *)calloc((size_t)P->n_times, sizeof(double)) : NULL;
    for (uint64_t pid = pid0; pid < pid1; ++pid) {
        particle p;
        emit(P, pid, &p);                                             /* step I */
        int bt = (int)(pid % (uint64_t)P->n_batches);
        double t = 0.0, Lz = 0.0;
        uint32_t k = 0, nscat = 0;
        if (h) memset(h, 0, (size_t)P->n_hj * sizeof(double));
        if (region) {
            memset(rt, 0, (size_t)P->n_times * sizeof(double));
            memset(rq, 0, (size_t)P->n_times * sizeof(double));
        }
        cnt->particles++;
        /* A free flight that reaches a periodic face continues from the opposite
         * face with the time it has left (rem >= 0), using the words of the block
         * drawn when it began; any other event ends it and the next flight draws
         * a new block.  One loop iteration is one segment. */
        uint32_t w[4];
        double rem = -1.0;
        uint32_t nseg = 0;
        for (;;) {
            double v = P->v[p.m], tau_m = P->tau[p.m];
            double dt;
            if (rem < 0.0) {
                rng_block(P->seed, pid, k, OR_TAG_STEP, w);
                ++k;
                dt = -tau_m * oracle_log(unif(w[0]));                    /* step II */
            } else {
                dt = rem;
            }
            rem = -1.0;
            ++nseg;
            cnt->iterations++;
            int32_t surf;
            double tb = boundary_search(P, &p, v, &surf);             /* step III */
            int boundary = (tb <= dt);
            double seg = boundary ? tb : dt;
            /* step V: sample the segment */
            if (P->n_bins > 0) score_bins(P, tally + lay.bins, bt, &p, v, tau_m, seg);
            if (P->field_n[0] > 0) score_field(P, tally + lay.field, bt, &p, v, seg);
            double dz = p.s * v * p.o[2] * seg;
            Lz += dz;
            if (h && nscat < (uint32_t)P->n_hj) h[nscat] += dz;
            if (transient) score_snapshots(P, tally + lay.snap, tally + lay.snap_abs, lay.ncell, &p, v, t, seg);
            if (region) score_region(P, rt, rq, &p, v, t, seg);
            double t_new = t + seg;
            if (transient && t_new > t_final) break;                 /* step VI */
            /* move */
            for (int i = 0; i < 3; ++i) p.x[i] += v * p.o[i] * seg;
            if (boundary) {                                           /* step IVa */
                /* place the particle exactly on the plane it reached */
                if (P->geom == OR_GEOM_SLAB_Z || P->geom == OR_GEOM_HALFSPACE_Z) p.x[2] = (surf == 1) ? P->length : 0.0;
                else if (P->geom == OR_GEOM_FILM_X) p.x[0] = (surf == 1) ? P->length : 0.0;
                else if (surf < 4) { int ax = (surf < 2) ? 0 : 2; p.x[ax] = (surf % 2 == 1) ? P->length : 0.0; }
                cnt->boundary++;
                int periodic = (P->geom == OR_GEOM_PORE_XZ) ? (surf < 4)
                             : (P->wall_type[(P->geom == OR_GEOM_HALFSPACE_Z) ? 0 : surf] == OR_WALL_PERIODIC);
                if (wall_interaction(P, &p, surf, w, cnt)) { t = t_new; break; }
                if (periodic) rem = dt - seg;
            } else {                                                  /* step IVb */
                p.m = alias_draw(w[1], P->gain_bits, P->gain_thresh, P->gain_alias);
                if (scatter_hist) scatter_hist[p.m] += 1;
                scatter_direction(P->scatter_g, w[2], w[3], p.o);
                p.last = OR_NO_SURFACE;
                ++nscat;
                cnt->scatters++;
                if (P->kmax >= 0 && nscat >= (uint32_t)P->kmax) { t = t_new; break; }
                if (P->first_event) { t = t_new; break; }              /* the first free path ends here */
            }
            t = t_new;
            if (nseg >= OR_ITER_CAP) { cnt->capped++; break; }
        }
        tally[lay.kappa + 0] += Lz;
        tally[lay.kappa + 1] += Lz * Lz;
        for (int32_t j = 0; j < P->n_hj; ++j) {
            tally[lay.hj + j] += h[j];
            tally[lay.hj + P->n_hj + j] += h[j] * h[j];
        }
        for (int32_t j = 0; region && j < P->n_times; ++j) {
            double *r = tally + lay.region + 4 * (size_t)j;
            r[0] += rt[j];
            r[1] += rt[j] * rt[j];
            r[2] += rq[j];
            r[3] += rq[j] * rq[j];
        }
        if (nscat_out) nscat_out[pid - pid0] = nscat;
    }
    free(h);
    free(rt);
    free(rq);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Geometry hooks for the tests                                              */
/* ------------------------------------------------------------------------ */

/* Step III for one given state: the surface hit time along x + v Omega t and
 * the surface index (pore cell: 0 x=0, 1 x=P, 2 z=0, 3 z=P, 4 pore). */
double oracle_boundary_search(const oracle_problem *P, const double x[3], const double o[3], double v,
                              int32_t last, int32_t *surf)
{
    particle p;
    memset(&p, 0, sizeof(p));
    for (int i = 0; i < 3; ++i) { p.x[i] = x[i]; p.o[i] = o[i]; }
    p.last = last;
    return boundary_search(P, &p, v, surf);
}

/* Step I for one particle id: position, direction, state and sign. */
void oracle_emit(const oracle_problem *P, uint64_t pid, double x[3], double o[3], uint32_t *m, double *s)
{
    particle p;
    emit(P, pid, &p);
    for (int i = 0; i < 3; ++i) { x[i] = p.x[i]; o[i] = p.o[i]; }
    *m = p.m;
    *s = p.s;
}

/* Ballistic walk in a pore cell (no scattering): each particle of [pid0, pid1)
 * is emitted, then moved from surface to surface with the same search, wrap
 * and pore interaction as oracle_run (pore words from the STEP blocks, one
 * block per interaction), until it has completed n_chords chords between
 * consecutive pore hits.  Sums the chord lengths (unwrapped, 3-D) and their
 * projections on the x-z plane; a walk whose ray meets no surface (parallel to
 * the pore axis) ends early.  Returns the number of chords. */
uint64_t oracle_pore_chords(const oracle_problem *P, uint64_t pid0, uint64_t pid1, uint32_t n_chords,
                            double *sum_len, double *sum_len_xz)
{
    uint64_t done = 0;
    double s3 = 0.0, s2 = 0.0;
    oracle_counters cnt;
    memset(&cnt, 0, sizeof(cnt));
    if (P->geom != OR_GEOM_PORE_XZ) return 0;
    for (uint64_t pid = pid0; pid < pid1; ++pid) {
        particle p;
        emit(P, pid, &p);
        uint32_t k = 0, chords = 0;
        int started = 0;
        double len = 0.0;
        while (chords < n_chords && k < OR_ITER_CAP) {
            int32_t surf;
            double t = boundary_search(P, &p, 1.0, &surf);
            if (!isfinite(t)) break;
            for (int i = 0; i < 3; ++i) p.x[i] += p.o[i] * t;
            len += t;
            uint32_t w[4];
            rng_block(P->seed, pid, k, OR_TAG_STEP, w);
            ++k;
            if (surf < 4) {
                int ax = (surf < 2) ? 0 : 2;
                p.x[ax] = (surf % 2 == 1) ? P->length : 0.0;
            } else {
                if (started) {
                    double sxz = sqrt(p.o[0] * p.o[0] + p.o[2] * p.o[2]);
                    s3 += len;
                    s2 += len * sxz;
                    ++chords;
                    ++done;
                }
                started = 1;
                len = 0.0;
            }
            wall_interaction(P, &p, surf, w, &cnt);
        }
    }
    *sum_len = s3;
    *sum_len_xz = s2;
    return done;
}

/* Step IVb's direction for one incoming direction and two words, exported for the tests. */
void oracle_scatter_direction(double g, uint32_t w2, uint32_t w3, const double o_in[3], double o_out[3])
{
    for (int i = 0; i < 3; ++i) o_out[i] = o_in[i];
    scatter_direction(g, w2, w3, o_out);
}

/* Raw Philox words for one (seed, pid, k, tag), exported for the tests. */
void oracle_rng_block(uint64_t seed, uint64_t pid, uint32_t k, uint32_t tag, uint32_t out[4])
{
    rng_block(seed, pid, k, tag, out);
}
