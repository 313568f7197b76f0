/*
 * rt3d_oracle.c -- plain FP64 CPU oracle of the Monte Carlo solar photon
 * tracer of Veerman, van Stratum and van Heerwaarden (GRL 2022), sec. 2.3.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this library.  It shares no code,
 * header or constant table with the HIP path; the two meet only through the
 * documented inputs (FP32 fields) and the documented random-number contract
 * (Philox4x32-10 counter layout, written out below from its definition).
 *
 * The algorithm, step by step, in the paper's order (sec. 2.3):
 *   1. emission at the top of the domain, along the sun beam or (with the
 *      diffuse fraction) isotropically downward;
 *   2. optical depth of the next tentative collision, tau = -ln(xi);
 *   3. null-collision tracking on the one-level acceleration grid (each
 *      coarse cell holds the largest fine-cell extinction); tau is spent
 *      cell by cell until the tentative collision, the surface or the top;
 *   4. at a tentative collision the local properties come from the fine
 *      grid; the weight is multiplied by the probability of not being
 *      absorbed, 1 - k_abs/K, and the removed weight is stored as heating;
 *   5. the event is a scattering with probability k_sca/(K - k_abs), else a
 *      null collision; a scatterer is a cloud droplet with probability
 *      k_ext,cloud/k_ext (Henyey-Greenstein, no delta scaling) or gas
 *      (Rayleigh);
 *   6. Russian roulette: below weight 0.5 the photon survives with
 *      probability w and is then reset to weight one;
 *   7. the surface is Lambertian: irradiance is tallied, the albedo scales
 *      the weight, the photon leaves with a cosine-weighted direction;
 *   8. a photon leaving the top is tallied as TOD upward flux.
 * Weights are integers in units of 2^-31 (exact energy ledger); every
 * real-valued quantity is FP64.
 *
 * Readings where the paper is silent (each listed in the design notes):
 * absorption weighting at every tentative collision, scatter vs null with
 * the conditional probability; isotropic radiance (cosine-weighted
 * directions) for the diffuse entry and for the Lambertian surface;
 * periodic x/y, open top; roulette after every collision and surface hit.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_ABI 2
#define W_ONE 2147483648.0 /* 2^31: weight one */
#define W_ONE_U 2147483648ull

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

int oracle_abi(void) { return ORACLE_ABI; }

/* ------------------------------------------------------------------------
 * Philox (Salmon, Moraes, Dror, Shaw: "Parallel random numbers: as easy as
 * 1, 2, 3", SC'11).  A Philox-4xW round multiplies counter words 0 and 2 by
 * two round multipliers, and the new counter is
 *   (hi(M1*c2) ^ c1 ^ k0,  lo(M1*c2),  hi(M0*c0) ^ c3 ^ k1,  lo(M0*c0));
 * between rounds the key is bumped by the two Weyl constants.  Ten rounds.
 * ------------------------------------------------------------------------ */
void oracle_philox4x32_10(const uint32_t* ctr_in, const uint32_t* key_in, uint32_t* out)
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t WA = 0x9E3779B9u, WB = 0xBB67AE85u;
    uint32_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += WA;
            k1 += WB;
        }
        uint64_t p0 = (uint64_t)M0 * (uint64_t)c[0];
        uint64_t p1 = (uint64_t)M1 * (uint64_t)c[2];
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
    }
    out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; out[3] = c[3];
}

void oracle_philox4x64_10(const uint64_t* ctr_in, const uint64_t* key_in, uint64_t* out)
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t WA = 0x9E3779B97F4A7C15ull, WB = 0xBB67AE8584CAA73Bull;
    uint64_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
    uint64_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += WA;
            k1 += WB;
        }
        unsigned __int128 p0 = (unsigned __int128)M0 * c[0];
        unsigned __int128 p1 = (unsigned __int128)M1 * c[2];
        uint64_t n0 = (uint64_t)(p1 >> 64) ^ c[1] ^ k0;
        uint64_t n1 = (uint64_t)p1;
        uint64_t n2 = (uint64_t)(p0 >> 64) ^ c[3] ^ k1;
        uint64_t n3 = (uint64_t)p0;
        c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
    }
    out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; out[3] = c[3];
}

/* Batch helpers for the test suite (n counters, 4 words each). */
void oracle_philox4x32_10_n(const uint32_t* ctr, uint64_t seed, uint32_t* out, uint64_t n)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (uint64_t i = 0; i < n; ++i) oracle_philox4x32_10(ctr + 4 * i, key, out + 4 * i);
}

/* A 32-bit word as a uniform variate in (0,1): (u + 1/2) 2^-32. */
static double unit_open(uint32_t u) { return ((double)u + 0.5) * (1.0 / 4294967296.0); }

/* ------------------------------------------------------------------------
 * Scrambled Sobol entry points (sec. 2.3, initialisation paragraph: rays
 * start at the top of the domain following a scrambled Sobol sequence).
 * Reading: photons keep the systematic column sampling, under which photon
 * id enters column (id + o) mod ncol as that column's p-th photon with
 * p = id div ncol (counting from 0); it takes the p-th point of the
 * two-dimensional Sobol sequence as its position inside the column, after a
 * nested uniform (Owen) scramble that is drawn independently per column and
 * per run.
 * ------------------------------------------------------------------------ */

/* Dimension 1: the radical inverse of i in base 2, i.e. i's 32 bits in
 * reverse order read as a binary fraction (times 2^32). */
uint32_t oracle_sobol_dim1(uint32_t i)
{
    uint32_t r = 0;
    for (int b = 0; b < 32; ++b)
        if (i & (1u << b)) r |= 1u << (31 - b);
    return r;
}

/* Dimension 2: Sobol's construction with the primitive polynomial x + 1:
 * direction numbers m_1 = 1, m_j = 2 m_{j-1} xor m_{j-1}, i.e.
 * v_j = m_j 2^(32-j) = v_{j-1} xor (v_{j-1} >> 1) with v_1 = 2^31; the point
 * is the xor of v_j over the set bits j (j = 1 for the lowest) of i. */
uint32_t oracle_sobol_dim2(uint32_t i)
{
    uint32_t v = 0x80000000u, r = 0;
    for (int j = 0; j < 32; ++j) {
        if (i & (1u << j)) r ^= v;
        v ^= v >> 1;
    }
    return r;
}

/* The finaliser of MurmurHash3 (Appleby): a bijective 32-bit mix. */
static uint32_t fmix32(uint32_t h)
{
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

/* Nested uniform scramble (Owen 1995) of the 32-digit binary fraction v:
 * digit d (d = 0 the most significant) is flipped by a random bit attached
 * to the node of the binary tree reached by v's first d digits; the node is
 * numbered (first d digits) | 2^d and its bit is the top bit of
 * fmix32(node xor seed). */
uint32_t oracle_owen_scramble(uint32_t v, uint32_t seed)
{
    uint32_t out = 0;
    for (int d = 0; d < 32; ++d) {
        uint32_t prefix = d ? v >> (32 - d) : 0u;
        uint32_t node = prefix | (1u << d);
        uint32_t flip = fmix32(node ^ seed) >> 31;
        uint32_t digit = (v >> (31 - d)) & 1u;
        out |= (digit ^ flip) << (31 - d);
    }
    return out;
}

/* Array forms for the tests: out[k] = dim1/dim2(i[k]) or owen(v[k], seed). */
void oracle_sobol_points_n(const uint32_t* i, uint32_t n, uint32_t* out1, uint32_t* out2)
{
    for (uint32_t k = 0; k < n; ++k) {
        out1[k] = oracle_sobol_dim1(i[k]);
        out2[k] = oracle_sobol_dim2(i[k]);
    }
}

void oracle_owen_scramble_n(const uint32_t* v, uint32_t n, uint32_t seed, uint32_t* out)
{
    for (uint32_t k = 0; k < n; ++k) out[k] = oracle_owen_scramble(v[k], seed);
}

/* Scramble seeds of column `col` under run key `key`: Philox counter
 * (col_lo, col_hi, 0xfffffffd, 0), words 0 (x) and 1 (y). */
static void column_scramble(const uint32_t key[2], uint64_t col, uint32_t s[2])
{
    uint32_t c[4] = {(uint32_t)col, (uint32_t)(col >> 32), 0xfffffffdu, 0u}, r[4];
    oracle_philox4x32_10(c, key, r);
    s[0] = r[0];
    s[1] = r[1];
}

/* Scrambled entry coordinates (32-bit fractions of the column width) of
 * passes first .. first+n-1 of column `col` in a run with Philox key
 * `seed`: out[2k] = x, out[2k+1] = y. */
void oracle_sobol_entry(uint64_t first, uint32_t n, uint64_t col, uint64_t seed, uint32_t* out)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)}, s[2];
    column_scramble(key, col, s);
    for (uint32_t k = 0; k < n; ++k) {
        uint32_t p = (uint32_t)(first + k);
        out[2 * k] = oracle_owen_scramble(oracle_sobol_dim1(p), s[0]);
        out[2 * k + 1] = oracle_owen_scramble(oracle_sobol_dim2(p), s[1]);
    }
}

/* ------------------------------------------------------------------------
 * Phase-function samplers (sec. 2.3, phase-function paragraph)
 * ------------------------------------------------------------------------ */

/* Henyey-Greenstein (1941): invert the cumulative distribution of
 * p(mu) = (1 - g^2) / (2 (1 + g^2 - 2 g mu)^{3/2}) on [-1, 1]. */
double oracle_hg_cos(double g, double xi)
{
    if (fabs(g) < 1e-6) return 2.0 * xi - 1.0;
    double s = (1.0 - g * g) / (1.0 - g + 2.0 * g * xi);
    double mu = (1.0 + g * g - s * s) / (2.0 * g);
    if (mu > 1.0) mu = 1.0;
    if (mu < -1.0) mu = -1.0;
    return mu;
}

/* Rayleigh: p(mu) = 3/8 (1 + mu^2) on [-1, 1]; the cumulative distribution
 * (mu^3 + 3 mu + 4)/8 = xi is a depressed cubic, solved with Cardano's
 * formula: mu = u - 1/u, u = cbrt(q + sqrt(q^2 + 1)), q = 4 xi - 2. */
double oracle_rayleigh_cos(double xi)
{
    double q = 4.0 * xi - 2.0;
    double u = cbrt(q + sqrt(q * q + 1.0));
    double mu = u - 1.0 / u;
    if (mu > 1.0) mu = 1.0;
    if (mu < -1.0) mu = -1.0;
    return mu;
}

/* New direction at angle acos(mu) from d and azimuth phi around it, using
 * an orthonormal frame (e1, e2, d). */
void oracle_turn(const double* d, double mu, double phi, double* out)
{
    double a[3];
    if (fabs(d[0]) < 0.5) { a[0] = 1.0; a[1] = 0.0; a[2] = 0.0; }
    else { a[0] = 0.0; a[1] = 1.0; a[2] = 0.0; }
    /* e1 = normalise(a x d), e2 = d x e1 */
    double e1[3] = {a[1] * d[2] - a[2] * d[1], a[2] * d[0] - a[0] * d[2], a[0] * d[1] - a[1] * d[0]};
    double n1 = sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
    e1[0] /= n1; e1[1] /= n1; e1[2] /= n1;
    double e2[3] = {d[1] * e1[2] - d[2] * e1[1], d[2] * e1[0] - d[0] * e1[2], d[0] * e1[1] - d[1] * e1[0]};
    double st = sqrt(fmax(0.0, 1.0 - mu * mu));
    double cp = cos(phi), sp = sin(phi);
    double r[3];
    for (int k = 0; k < 3; ++k) r[k] = mu * d[k] + st * (cp * e1[k] + sp * e2[k]);
    double nr = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    out[0] = r[0] / nr; out[1] = r[1] / nr; out[2] = r[2] / nr;
}

/* Vectorised sampler entry points for the tests. */
void oracle_hg_cos_n(double g, const double* xi, double* mu, uint64_t n)
{
    for (uint64_t i = 0; i < n; ++i) mu[i] = oracle_hg_cos(g, xi[i]);
}

void oracle_rayleigh_cos_n(const double* xi, double* mu, uint64_t n)
{
    for (uint64_t i = 0; i < n; ++i) mu[i] = oracle_rayleigh_cos(xi[i]);
}

/* ------------------------------------------------------------------------
 * Acceleration grid (sec. 2.3): K[b] = max k_ext over the fine cells of b.
 * ------------------------------------------------------------------------ */
int oracle_majorant(int32_t nx, int32_t ny, int32_t nz, int32_t bx, int32_t by, int32_t bz,
                    const float* k_ext, float* K)
{
    if (nx <= 0 || ny <= 0 || nz <= 0 || bx <= 0 || by <= 0 || bz <= 0) return 1;
    if (nx % bx || ny % by || nz % bz) return 1;
    int32_t mx = nx / bx, my = ny / by, mz = nz / bz;
    for (int32_t c = 0; c < mx * my * mz; ++c) K[c] = 0.0f;
    for (int32_t k = 0; k < nz; ++k)
        for (int32_t j = 0; j < ny; ++j)
            for (int32_t i = 0; i < nx; ++i) {
                float v = k_ext[((int64_t)k * ny + j) * nx + i];
                float* dst = &K[((int64_t)(k / bz) * my + j / by) * mx + i / bx];
                if (v > *dst) *dst = v;
            }
    return 0;
}

/* ------------------------------------------------------------------------
 * Tracing
 * ------------------------------------------------------------------------ */
typedef struct {
    int32_t nx, ny, nz, bx, by, bz;
    double dx, dy, dz;
    const float* k_ext;
    const float* k_ext_cloud;
    const float* ssa;
    const float* g;
    const float* albedo;
    double sza_deg, azimuth_deg;
    uint64_t photons, seed, photon_offset;
    double diffuse_fraction, rr_threshold;
    uint32_t max_iters;
    int32_t nthreads;
    int32_t sobol_entry; /* 1: scrambled Sobol positions inside the column */
} oracle_problem;

typedef struct {
    uint64_t* abs_dir;
    uint64_t* abs_dif;
    uint64_t* sfc_dir;
    uint64_t* sfc_dif;
    uint64_t* sfc_abs;
    uint64_t* toa_up;
    uint64_t* ledger; /* [8]: incoming toa atm_dir atm_dif sfc rr_gain rr_loss lost */
    uint64_t* stats;  /* [12]: photons collisions null gas cloud surface escape
                         rr_kill rr_survive crossings absorbed capped */
} oracle_tallies;

enum { L_IN, L_TOA, L_ATM_DIR, L_ATM_DIF, L_SFC, L_RR_GAIN, L_RR_LOSS, L_LOST, L_N };
enum { S_PHOT, S_COLL, S_NULL, S_GAS, S_CLOUD, S_SFC, S_ESC, S_RR_KILL, S_RR_SURV,
       S_CROSS, S_ABSORBED, S_CAPPED, S_N };

typedef struct {
    const oracle_problem* p;
    const oracle_tallies* t;
    const float* K; /* majorants */
    int32_t mx, my, mz;
    double Lx, Ly, H;
    double sun[3];
    uint32_t key[2];
    uint64_t ncol, col_offset;
    uint64_t rr_below; /* roulette when w < rr_below */
    uint64_t first, last; /* photon range of this worker (local indices) */
    uint64_t ledger[L_N];
    uint64_t stats[S_N];
} worker;

static void add(uint64_t* a, uint64_t v)
{
    if (v) __atomic_fetch_add(a, v, __ATOMIC_RELAXED);
}

static void draw(const worker* w, uint64_t id, uint32_t c2, uint32_t c3, uint32_t r[4])
{
    uint32_t ctr[4] = {(uint32_t)id, (uint32_t)(id >> 32), c2, c3};
    oracle_philox4x32_10(ctr, w->key, r);
}

/* Round-half-even of x >= 0 to an integer. */
static uint64_t round_even(double x) { return (uint64_t)nearbyint(x); }

static int32_t clampi(int32_t v, int32_t lo, int32_t hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* Roulette (sec. 2.3): for w below the threshold draw rho in [0,1); the
 * photon ends if rho*2^31 >= w (probability 1 - w), else w becomes one.
 * Returns 0 when the photon ends. */
static int roulette(worker* W, uint64_t id, uint32_t step, uint64_t* w)
{
    if (*w >= W->rr_below) return 1;
    uint32_t r[4];
    draw(W, id, step, 1u, r);
    uint64_t rho = (uint64_t)(r[0] >> 1); /* floor(xi * 2^31) */
    if (rho < *w) {
        W->ledger[L_RR_GAIN] += W_ONE_U - *w;
        W->stats[S_RR_SURV]++;
        *w = W_ONE_U;
        return 1;
    }
    W->ledger[L_RR_LOSS] += *w;
    W->stats[S_RR_KILL]++;
    return 0;
}

static void trace_one(worker* W, uint64_t id)
{
    const oracle_problem* P = W->p;
    const oracle_tallies* T = W->t;
    const int32_t nx = P->nx, ny = P->ny;
    const int32_t bx = P->bx, by = P->by, bz = P->bz;
    const double dx = P->dx, dy = P->dy, dz = P->dz;
    uint32_t r[4];

    W->stats[S_PHOT]++;
    W->ledger[L_IN] += W_ONE_U;

    /* 1. emission at the top of the domain in column (id + o) mod ncol */
    uint64_t col = (id + W->col_offset) % W->ncol;
    int32_t ic = (int32_t)(col % (uint64_t)nx), jc = (int32_t)(col / (uint64_t)nx);
    draw(W, id, 0xffffffffu, 0u, r);
    double p[3] = {(ic + unit_open(r[0])) * dx, (jc + unit_open(r[1])) * dy, W->H};
    if (P->sobol_entry) {
        uint32_t xy[2];
        oracle_sobol_entry(id / W->ncol, 1u, col, P->seed, xy);
        p[0] = (ic + unit_open(xy[0])) * dx;
        p[1] = (jc + unit_open(xy[1])) * dy;
    }
    double d[3];
    int direct;
    if (unit_open(r[2]) < P->diffuse_fraction) {
        uint32_t q[4];
        draw(W, id, 0xffffffffu, 1u, q);
        double mu = sqrt(unit_open(q[0])), phi = 2.0 * M_PI * unit_open(q[1]);
        double st = sqrt(fmax(0.0, 1.0 - mu * mu));
        d[0] = st * cos(phi); d[1] = st * sin(phi); d[2] = -mu;
        direct = 0;
    } else {
        d[0] = W->sun[0]; d[1] = W->sun[1]; d[2] = W->sun[2];
        direct = 1;
    }
    uint64_t w = W_ONE_U;
    /* acceleration-grid cell holding the photon */
    int32_t b[3] = {ic / bx, jc / by, W->mz - 1};
    uint32_t iters = 0;

    for (uint32_t step = 0;; ++step) {
        /* 2. optical depth to the next tentative collision */
        draw(W, id, step, 0u, r);
        double tau = -log(unit_open(r[0]));

        /* 3. spend tau across acceleration-grid cells */
        int outcome; /* 0 collision, 1 surface, 2 escape, 3 capped */
        for (;;) {
            if (iters >= P->max_iters) { outcome = 3; break; }
            ++iters;
            double K = (double)W->K[((int64_t)b[2] * W->my + b[1]) * W->mx + b[0]];
            double lo[3] = {(double)(b[0] * bx) * dx, (double)(b[1] * by) * dy, (double)(b[2] * bz) * dz};
            double hi[3] = {(double)((b[0] + 1) * bx) * dx, (double)((b[1] + 1) * by) * dy,
                            (double)((b[2] + 1) * bz) * dz};
            double s_exit = INFINITY;
            int axis = -1;
            for (int a = 0; a < 3; ++a) {
                double t;
                if (d[a] > 0.0) t = (hi[a] - p[a]) / d[a];
                else if (d[a] < 0.0) t = (lo[a] - p[a]) / d[a];
                else continue;
                if (t < 0.0) t = 0.0;
                if (t < s_exit) { s_exit = t; axis = a; }
            }
            if (K * s_exit >= tau) {
                double s = tau / K;
                for (int a = 0; a < 3; ++a) p[a] += s * d[a];
                outcome = 0;
                break;
            }
            tau -= K * s_exit;
            for (int a = 0; a < 3; ++a) p[a] += s_exit * d[a];
            int up = d[axis] > 0.0;
            if (axis == 2) {
                if (!up && b[2] == 0) { p[2] = 0.0; outcome = 1; break; }
                if (up && b[2] == W->mz - 1) { p[2] = W->H; outcome = 2; break; }
                /* enter the next layer of cells on its near face */
                b[2] += up ? 1 : -1;
                p[2] = up ? (double)(b[2] * bz) * dz : (double)((b[2] + 1) * bz) * dz;
            } else {
                /* periodic in x and y: leaving the last cell re-enters the first */
                int32_t m = axis == 0 ? W->mx : W->my;
                int32_t n = b[axis] + (up ? 1 : -1);
                if (n == m) n = 0;
                if (n < 0) n = m - 1;
                b[axis] = n;
                double cell = axis == 0 ? bx * dx : by * dy;
                p[axis] = up ? (double)n * cell : (double)(n + 1) * cell;
            }
            W->stats[S_CROSS]++;
        }

        if (outcome == 3) {
            W->ledger[L_LOST] += w;
            W->stats[S_CAPPED]++;
            return;
        }

        /* fine cell / column under the photon, kept inside the current
         * acceleration-grid cell so that k_ext <= K holds there */
        int32_t i = clampi((int32_t)floor(p[0] / dx), b[0] * bx, b[0] * bx + bx - 1);
        int32_t j = clampi((int32_t)floor(p[1] / dy), b[1] * by, b[1] * by + by - 1);

        if (outcome == 2) { /* 8. leaves through the top */
            add(&T->toa_up[(int64_t)j * nx + i], w);
            W->ledger[L_TOA] += w;
            W->stats[S_ESC]++;
            return;
        }

        if (outcome == 1) { /* 7. Lambertian surface */
            W->stats[S_SFC]++;
            int64_t c2 = (int64_t)j * nx + i;
            add(direct ? &T->sfc_dir[c2] : &T->sfc_dif[c2], w);
            uint64_t w_new = round_even((double)P->albedo[c2] * (double)w);
            if (w_new > w) w_new = w;
            add(&T->sfc_abs[c2], w - w_new);
            W->ledger[L_SFC] += w - w_new;
            w = w_new;
            if (w == 0) { W->stats[S_ABSORBED]++; return; }
            double mu = sqrt(unit_open(r[2])), phi = 2.0 * M_PI * unit_open(r[3]);
            double st = sqrt(fmax(0.0, 1.0 - mu * mu));
            d[0] = st * cos(phi); d[1] = st * sin(phi); d[2] = mu;
            direct = 0;
            if (!roulette(W, id, step, &w)) return;
            continue;
        }

        /* 4. tentative collision: local properties from the fine grid */
        int32_t k = clampi((int32_t)floor(p[2] / dz), b[2] * bz, b[2] * bz + bz - 1);
        int64_t c3 = ((int64_t)k * ny + j) * nx + i;
        double K = (double)W->K[((int64_t)b[2] * W->my + b[1]) * W->mx + b[0]];
        double ke = P->k_ext[c3], om = P->ssa[c3];
        double ka = ke * (1.0 - om);
        W->stats[S_COLL]++;
        if (ka > 0.0) {
            uint64_t dep = round_even((double)w * (ka / K));
            if (dep > w) dep = w;
            if (direct) { add(&T->abs_dir[c3], dep); W->ledger[L_ATM_DIR] += dep; }
            else { add(&T->abs_dif[c3], dep); W->ledger[L_ATM_DIF] += dep; }
            w -= dep;
            if (w == 0) { W->stats[S_ABSORBED]++; return; }
        }
        /* 5. scattering or null collision */
        double ks = ke * om;
        double ps = (K - ka > 0.0) ? ks / (K - ka) : 0.0;
        double xi = unit_open(r[1]);
        if (xi < ps) {
            double kc = P->k_ext_cloud[c3];
            double mu;
            if (ke > 0.0 && xi < ps * (kc / ke)) {
                mu = oracle_hg_cos((double)P->g[c3], unit_open(r[2]));
                W->stats[S_CLOUD]++;
            } else {
                mu = oracle_rayleigh_cos(unit_open(r[2]));
                W->stats[S_GAS]++;
            }
            double nd[3];
            oracle_turn(d, mu, 2.0 * M_PI * unit_open(r[3]), nd);
            d[0] = nd[0]; d[1] = nd[1]; d[2] = nd[2];
            direct = 0;
        } else {
            W->stats[S_NULL]++;
        }
        /* 6. roulette */
        if (!roulette(W, id, step, &w)) return;
    }
}

static void* run_worker(void* arg)
{
    worker* W = (worker*)arg;
    for (uint64_t i = W->first; i < W->last; ++i) trace_one(W, W->p->photon_offset + i);
    return NULL;
}

/* Returns 0 on success, 1 on bad arguments, 2 on allocation failure.  The
 * tallies are overwritten. */
int oracle_trace(const oracle_problem* P, const oracle_tallies* T)
{
    if (!P || !T) return 1;
    if (P->nx <= 0 || P->ny <= 0 || P->nz <= 0 || P->bx <= 0 || P->by <= 0 || P->bz <= 0) return 1;
    if (P->nx % P->bx || P->ny % P->by || P->nz % P->bz) return 1;
    if (!(P->dx > 0) || !(P->dy > 0) || !(P->dz > 0)) return 1;
    if (!(P->sza_deg >= 0.0 && P->sza_deg < 90.0) || P->photons == 0) return 1;
    const int64_t ncell = (int64_t)P->nx * P->ny * P->nz, ncol = (int64_t)P->nx * P->ny;
    memset(T->abs_dir, 0, sizeof(uint64_t) * ncell);
    memset(T->abs_dif, 0, sizeof(uint64_t) * ncell);
    memset(T->sfc_dir, 0, sizeof(uint64_t) * ncol);
    memset(T->sfc_dif, 0, sizeof(uint64_t) * ncol);
    memset(T->sfc_abs, 0, sizeof(uint64_t) * ncol);
    memset(T->toa_up, 0, sizeof(uint64_t) * ncol);
    memset(T->ledger, 0, sizeof(uint64_t) * L_N);
    memset(T->stats, 0, sizeof(uint64_t) * S_N);

    int32_t mx = P->nx / P->bx, my = P->ny / P->by, mz = P->nz / P->bz;
    float* K = (float*)malloc(sizeof(float) * (size_t)mx * my * mz);
    if (!K) return 2;
    oracle_majorant(P->nx, P->ny, P->nz, P->bx, P->by, P->bz, P->k_ext, K);

    int nt = P->nthreads > 0 ? P->nthreads : 1;
    if ((uint64_t)nt > P->photons) nt = (int)P->photons;
    worker* ws = (worker*)calloc((size_t)nt, sizeof(worker));
    pthread_t* th = (pthread_t*)calloc((size_t)nt, sizeof(pthread_t));
    if (!ws || !th) { free(K); free(ws); free(th); return 2; }

    double th0 = P->sza_deg * M_PI / 180.0, ph0 = P->azimuth_deg * M_PI / 180.0;
    uint32_t key[2] = {(uint32_t)P->seed, (uint32_t)(P->seed >> 32)};
    uint32_t r[4];
    uint32_t c0[4] = {0u, 0u, 0xfffffffeu, 0u};
    oracle_philox4x32_10(c0, key, r);
    uint64_t col_offset = ((uint64_t)r[0] * (uint64_t)ncol) >> 32;
    uint64_t rr_below = (uint64_t)round_even(P->rr_threshold * W_ONE);

    for (int t = 0; t < nt; ++t) {
        worker* W = &ws[t];
        W->p = P; W->t = T; W->K = K;
        W->mx = mx; W->my = my; W->mz = mz;
        W->Lx = P->nx * P->dx; W->Ly = P->ny * P->dy; W->H = P->nz * P->dz;
        W->sun[0] = -sin(th0) * sin(ph0);
        W->sun[1] = -sin(th0) * cos(ph0);
        W->sun[2] = -cos(th0);
        W->key[0] = key[0]; W->key[1] = key[1];
        W->ncol = (uint64_t)ncol; W->col_offset = col_offset;
        W->rr_below = rr_below;
        W->first = P->photons * (uint64_t)t / (uint64_t)nt;
        W->last = P->photons * (uint64_t)(t + 1) / (uint64_t)nt;
    }
    if (nt == 1) run_worker(&ws[0]);
    else {
        for (int t = 0; t < nt; ++t) pthread_create(&th[t], NULL, run_worker, &ws[t]);
        for (int t = 0; t < nt; ++t) pthread_join(th[t], NULL);
    }
    for (int t = 0; t < nt; ++t) {
        for (int l = 0; l < L_N; ++l) T->ledger[l] += ws[t].ledger[l];
        for (int s = 0; s < S_N; ++s) T->stats[s] += ws[t].stats[s];
    }
    free(K); free(ws); free(th);
    return 0;
}

/* Deterministic direct-beam transmittance onto one surface column: the
 * mean, over an n x n lattice of cell-centred points of surface column
 * (ic, jc), of exp(-integral of k_ext along the line from that point back
 * towards the sun up to the top of the domain), periodic in x and y.  The
 * integral is summed exactly fine cell by fine cell.  With a horizontally
 * uniform incoming flux this is the expected direct surface irradiance of
 * the column as a fraction of the TOD flux (Beer-Lambert law). */
double oracle_direct_transmittance(int32_t nx, int32_t ny, int32_t nz, double dx, double dy, double dz,
                                   const float* k_ext, double sza_deg, double azimuth_deg,
                                   int32_t ic, int32_t jc, int32_t n)
{
    double th0 = sza_deg * M_PI / 180.0, ph0 = azimuth_deg * M_PI / 180.0;
    /* towards the sun */
    double u[3] = {sin(th0) * sin(ph0), sin(th0) * cos(ph0), cos(th0)};
    double acc = 0.0;
    for (int32_t a = 0; a < n; ++a)
        for (int32_t bb = 0; bb < n; ++bb) {
            int32_t i = ic, j = jc, k = 0;
            double px = (ic + (a + 0.5) / n) * dx, py = (jc + (bb + 0.5) / n) * dy, pz = 0.0;
            double optical = 0.0;
            for (;;) {
                double tx = u[0] > 0 ? ((i + 1) * dx - px) / u[0] : (u[0] < 0 ? (i * dx - px) / u[0] : INFINITY);
                double ty = u[1] > 0 ? ((j + 1) * dy - py) / u[1] : (u[1] < 0 ? (j * dy - py) / u[1] : INFINITY);
                double tz = ((k + 1) * dz - pz) / u[2];
                if (tx < 0) tx = 0;
                if (ty < 0) ty = 0;
                if (tz < 0) tz = 0;
                double t = tz;
                int axis = 2;
                if (tx < t) { t = tx; axis = 0; }
                if (ty < t) { t = ty; axis = 1; }
                optical += t * (double)k_ext[((int64_t)k * ny + j) * nx + i];
                px += t * u[0]; py += t * u[1]; pz += t * u[2];
                if (axis == 2) {
                    if (k == nz - 1) break;
                    ++k; pz = k * dz;
                } else if (axis == 0) {
                    if (u[0] > 0) { ++i; if (i == nx) i = 0; px = i * dx; }
                    else { --i; if (i < 0) i = nx - 1; px = (i + 1) * dx; }
                } else {
                    if (u[1] > 0) { ++j; if (j == ny) j = 0; py = j * dy; }
                    else { --j; if (j < 0) j = ny - 1; py = (j + 1) * dy; }
                }
            }
            acc += exp(-optical);
        }
    return acc / ((double)n * n);
}
