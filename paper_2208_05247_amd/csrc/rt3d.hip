// rt3d.hip -- Monte Carlo solar photon tracer for gfx950 (MI355X) behind the
// C ABI declared in include/rt3d.h.
//
// Method: the forward Monte Carlo ray tracer of Veerman, van Stratum and van
// Heerwaarden (GRL 2022), sec. 2.3 -- null-collision tracking on a one-level
// acceleration grid, absorption by weights at every scattering or null
// collision, Rayleigh (gas) / Henyey-Greenstein (cloud) scattering, Russian
// roulette below weight 0.5, Lambertian surface, heating and flux tallies.
//
// Design for CDNA4 (not the paper's CUDA design):
//   * persistent kernel, one photon per lane, lanes refilled from a
//     per-wave pool of photon ids that is topped up with one global atomic
//     per pool, so divergent photon lifetimes do not idle the wave; a wave
//     refills once 16 of its lanes are idle, so the emission code runs for
//     many lanes at once;
//   * one loop pass = at most a few acceleration-grid crossings (3 by
//     default) and then the event reached, if any (tentative collision,
//     surface, top): a lane on a long clear-sky walk does not hold its wave
//     through all of it;
//   * majorants staged in LDS when they fit, else read through L1/L2;
//   * integer weights (units of 2^-31) and uint64 tallies: order-independent
//     atomics, bitwise-reproducible results and an exactly closing ledger;
//   * deposits into the same cell by consecutive events of one lane are
//     merged in registers and written with one atomic when the lane moves on;
//   * event counters live in registers and are folded into LDS per photon
//     and into global memory once per workgroup.
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <mutex>

#include "rt3d.h"

namespace {

constexpr uint32_t kWOne = 0x80000000u;  // weight one in units of 2^-31
constexpr uint32_t kNoCell = 0xffffffffu;
constexpr uint32_t kNoMajorant = 0x7fffffffu;  // a NaN: never a majorant (those are >= 0, or negated as a flag)
constexpr size_t kLdsMajorantBytes = 64 * 1024;  // automatic LDS staging limit (two workgroups per CU)

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): per round the counter becomes
// (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0)); the key
// is bumped by the Weyl constants between rounds.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t lo0 = 0xD2511F53u * c.x;
        const uint32_t hi0 = __umulhi(0xD2511F53u, c.x);
        const uint32_t lo1 = 0xCD9E8D57u * c.z;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c.z);
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
    }
    return c;
}

// 24-bit uniforms: [0,1) for comparisons and positions, (0,1] for logs.
__device__ __forceinline__ float u01(uint32_t u) { return (float)(u >> 8) * 0x1p-24f; }
__device__ __forceinline__ float u01_open(uint32_t u) { return (float)((u >> 8) + 1u) * 0x1p-24f; }

__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// ---------------------------------------------------------------------------
// Scrambled Sobol entry points (sec. 2.3: rays start at the top of the domain
// following a scrambled Sobol sequence).  The p-th photon to enter a column
// takes the p-th point of the 2D Sobol sequence, nested-uniform scrambled
// per column and run.  Dimension 1 is the base-2 radical inverse (bit
// reversal); dimension 2 uses the primitive polynomial x + 1, whose
// direction numbers follow v_1 = 2^31, v_j = v_{j-1} ^ (v_{j-1} >> 1).
__device__ __forceinline__ uint32_t sobol_dim2(uint32_t p) {
    uint32_t v = 0x80000000u, r = 0;
    while (p) {
        if (p & 1u) r ^= v;
        v ^= v >> 1;
        p >>= 1;
    }
    return r;
}

// MurmurHash3's finaliser (a bijective 32-bit mix).
__device__ __forceinline__ uint32_t fmix32(uint32_t h) {
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

// Owen's nested uniform scramble of the first kDigits binary digits of v:
// digit d is flipped by the top bit of fmix32(node ^ seed), node = (v's
// first d digits) | 2^d numbering the binary-tree node above that digit.
// Digit d depends only on digits before it, so the first 24 digits of the
// 32-digit scramble are the 24-digit scramble.
template <int kDigits>
__device__ __forceinline__ uint32_t owen_scramble(uint32_t v, uint32_t seed) {
    uint32_t out = 0;
#pragma unroll 4
    for (int d = 0; d < kDigits; ++d) {
        const uint32_t node = (d ? v >> (32 - d) : 0u) | (1u << d);
        out |= (((v >> (31 - d)) ^ (fmix32(node ^ seed) >> 31)) & 1u) << (31 - d);
    }
    return out;
}

// Henyey-Greenstein cos(theta) by inversion of its cumulative distribution,
// mu = (1 + g^2 - s^2) / (2 g) with s = (1 - g^2) / (1 + g a), a = 2 xi - 1.
// For small |g| that quotient cancels catastrophically in FP32; multiplied
// out it is the same function
//   mu = (a + g (a^2 + 3)/2 + g^2 a + g^3 (a^2 - 1)/2) / (1 + g a)^2,
// which is exact at g = 0 (mu = a) and well conditioned while 1 + g a stays
// near 1, so each form is used where it is accurate (|mu error| < 1e-6).
__device__ __forceinline__ float hg_cos(float g, float xi) {
    if (g >= 1.0f) return 1.0f;  // pure forward scattering (0/0 at xi = 0 otherwise)
    const float a = 2.0f * xi - 1.0f;
    float mu;
    if (fabsf(g) < 0.1f) {
        const float d = 1.0f + g * a;
        const float a2 = a * a;
        mu = (a + g * (0.5f * (a2 + 3.0f) + g * (a + g * (0.5f * (a2 - 1.0f))))) / (d * d);
    } else {
        const float s = (1.0f - g * g) / (1.0f - g + 2.0f * g * xi);
        mu = (1.0f + g * g - s * s) / (2.0f * g);
    }
    return fminf(1.0f, fmaxf(-1.0f, mu));
}

// Rayleigh cos(theta): root of mu^3 + 3 mu + 4 - 8 xi = 0 (Cardano).
__device__ __forceinline__ float rayleigh_cos(float xi) {
    const float q = 4.0f * xi - 2.0f;
    const float u = cbrtf(q + sqrtf(q * q + 1.0f));
    return fminf(1.0f, fmaxf(-1.0f, u - rcp(u)));
}

// Turn direction (x,y,z) by polar cosine mu and azimuth 2*pi*t, in the
// frame e1 = (x z, y z, -s^2)/s, e2 = (-y, x, 0)/s with s = |(x, y)|.  s is
// taken from the horizontal components (not sqrt(1 - z^2), which cancels for
// near-vertical d), so the frame stays accurate down to s ~ 1e-12; only a
// direction closer to vertical than that uses the fixed frame (x, y axes).
__device__ __forceinline__ void turn(float& x, float& y, float& z, float mu, float t) {
    float sp, cp;
    __sincosf(6.28318530717958647f * t, &sp, &cp);
    const float st = sqrtf(fmaxf(0.0f, 1.0f - mu * mu));
    float nx, ny, nz;
    const float s2 = x * x + y * y;
    if (s2 < 1e-24f) {
        nx = st * cp;
        ny = st * sp;
        nz = z > 0.0f ? mu : -mu;
    } else {
        const float is = rsqrtf(s2);
        const float s = s2 * is;
        nx = st * (x * z * cp - y * sp) * is + x * mu;
        ny = st * (y * z * cp + x * sp) * is + y * mu;
        nz = -st * cp * s + z * mu;
    }
    const float n = rsqrtf(nx * nx + ny * ny + nz * nz);
    x = nx * n;
    y = ny * n;
    z = nz * n;
}

// ---------------------------------------------------------------------------
// Photon schedule: the order in which the work queue hands out photons.
// Photon k of g-point n (id = photon_offset + k) enters column
// (id + o_n) mod ncol (systematic column sampling with a random offset o_n),
// so every column receives P_n = count_n div ncol photons of g-point n in
// full passes, and the columns of one cyclic range one more.  Queue slots
// run through the full passes entry tile by entry tile (tiles of
// tile_x x tile_y columns, row-major; inside a tile pass by pass over all
// g-points, its columns row-major), then through the remaining photons
// g-point by g-point.  The photons in flight at one time then enter a few
// neighbouring tiles, and the cells and tallies they touch form a small
// working set instead of the whole domain.  Which photons are traced, with
// which random numbers, does not depend on the order, and neither do the
// integer tallies.
// ---------------------------------------------------------------------------
struct Schedule {
    const unsigned long long* pass_first;  // [ngp + 1] prefix sums of P_n
    const unsigned long long* rem_first;   // [ngp + 1] prefix sums of count_n mod ncol
    const unsigned long long* col_offset;  // [ngp] o_n
    unsigned long long full_slots;         // ncol * sum P_n
    unsigned long long tile_slots;         // tile_cols * sum P_n
    unsigned long long photon_offset;
    uint32_t ncol, nx, tile_x, tile_y, tile_cols, ntx;
    uint32_t po_mod;  // photon_offset mod ncol
    int ngp;
};

struct Slot {
    int gp;
    unsigned long long id;
    uint32_t col;
};

// Prefix sums of the full passes and of the photons left over per g-point.
template <typename Count>
__host__ __device__ inline void schedule_tables(const Count* photons, int ngp, unsigned long long ncol,
                                                unsigned long long* pass_first, unsigned long long* rem_first) {
    unsigned long long passes = 0, rest = 0;
    for (int n = 0; n < ngp; ++n) {
        pass_first[n] = passes;
        rem_first[n] = rest;
        passes += (unsigned long long)photons[n] / ncol;
        rest += (unsigned long long)photons[n] % ncol;
    }
    pass_first[ngp] = passes;
    rem_first[ngp] = rest;
}

// Index lo with first[lo] <= x < first[lo + 1] (empty ranges skipped).
__host__ __device__ inline int range_of(const unsigned long long* first, int n, unsigned long long x) {
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (first[mid] <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

__host__ __device__ inline Slot decode_slot(const Schedule& S, unsigned long long s) {
    Slot r;
    unsigned long long k;
    if (s < S.full_slots) {
        const unsigned long long t = s / S.tile_slots;
        const unsigned long long rem = s - t * S.tile_slots;
        const unsigned long long f = rem / S.tile_cols;  // full pass over all g-points
        const uint32_t u = (uint32_t)(rem - f * S.tile_cols);
        r.gp = range_of(S.pass_first, S.ngp, f);
        const unsigned long long m = f - S.pass_first[r.gp];
        const uint32_t tx = (uint32_t)t % S.ntx, ty = (uint32_t)t / S.ntx;
        const uint32_t uy = u / S.tile_x, ux = u - uy * S.tile_x;
        r.col = (ty * S.tile_y + uy) * S.nx + tx * S.tile_x + ux;
        uint32_t o = (uint32_t)S.col_offset[r.gp] + S.po_mod;
        if (o >= S.ncol) o -= S.ncol;
        const uint32_t j = r.col >= o ? r.col - o : r.col + (S.ncol - o);
        k = (unsigned long long)j + m * S.ncol;
    } else {
        const unsigned long long q = s - S.full_slots;
        r.gp = range_of(S.rem_first, S.ngp, q);
        const uint32_t j = (uint32_t)(q - S.rem_first[r.gp]);
        k = (S.pass_first[r.gp + 1] - S.pass_first[r.gp]) * S.ncol + j;
        uint32_t o = (uint32_t)S.col_offset[r.gp] + S.po_mod;
        if (o >= S.ncol) o -= S.ncol;
        r.col = j + o;
        if (r.col >= S.ncol) r.col -= S.ncol;
    }
    r.id = S.photon_offset + k;
    return r;
}

struct TraceParams {
    // medium: kFactored = false: cells = (k_ext, ssa, k_ext_cloud, g) per cell;
    //         kFactored = true:  cells = (k_ext_cloud, cloud k_abs, g, 0) per cell,
    //                            gas = (k_gas, gas k_abs) per g-point and level
    const float4* __restrict__ cells;
    const float2* __restrict__ gas;
    const float* __restrict__ albedo;
    const float* __restrict__ majorant;                    // [ngp][nmaj]
    // factored only (null: not used): per acceleration cell, one bit per fine
    // cell (1 = some cloud extinction), mask_words words per acceleration
    // cell, the bits in x-fastest order of the cell's bx * by * bz fine cells
    const uint32_t* __restrict__ cell_mask;
    int mask_words;
    Schedule sched;
    unsigned long long* abs_dir;
    unsigned long long* abs_dif;
    unsigned long long* sfc_dir;
    unsigned long long* sfc_dif;
    unsigned long long* sfc_abs;
    unsigned long long* toa_up;
    unsigned long long* ledger;
    unsigned long long* stats;
    unsigned long long* queue;
    int ngp, nmaj, max_walk;
    uint32_t pool;   // photon ids a wave takes from the queue at a time
    uint32_t refill; // a wave refills once this many of its lanes are idle
    int merge;       // merge consecutive deposits of a lane into one cell
    int wave_agg;    // wave-aggregated tally atomics (same address, same instruction)
    int nx, ny, nz, bx, by, bz, mx, my, mz;
    float dx, dy, dz, inv_dx, inv_dy, inv_dz;
    float cx, cy, cz;  // acceleration-grid cell size in metres
    float H;
    float sun_x, sun_y, sun_z;
    float diffuse_fraction;
    const float* gp_diffuse;  // per-g-point diffuse fraction (batched), or null
    int sobol;                // scrambled Sobol entry positions
    uint32_t rr_below;
    uint32_t max_iters;
    unsigned long long seed;  // g-point n draws with Philox key seed + n
    unsigned long long photons, photon_offset, ncol;
};

enum { L_IN, L_TOA, L_ATM_DIR, L_ATM_DIF, L_SFC, L_RR_GAIN, L_RR_LOSS, L_LOST, L_N };
enum { S_PHOT, S_COLL, S_NULL, S_GAS, S_CLOUD, S_SFC, S_ESC, S_RR_KILL, S_RR_SURV,
       S_CROSS, S_ABSORBED, S_CAPPED, S_N };

__device__ __forceinline__ void lds_add(unsigned long long* a, unsigned long long v) {
    if (v) atomicAdd(a, v);
}

// Tally update.  agg = 0: one atomic per lane.  agg = 1 (wave-aggregated):
// the lanes that update the same address in this instruction add their
// values first and one of them issues the atomic; the loop visits each
// distinct address of the active lanes once (scalar, wave-uniform).
__device__ __forceinline__ void tally_add(unsigned long long* p, unsigned long long v, int agg) {
    if (!agg) {
        atomicAdd(p, v);
        return;
    }
    uint64_t todo = __ballot(1);
    const uint64_t a = (uint64_t)(uintptr_t)p;
    while (todo) {
        const int l = __ffsll((unsigned long long)todo) - 1;
        const uint64_t al = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(a >> 32), l) << 32) |
                            (uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)a, l);
        const uint64_t m = __ballot(a == al);
        unsigned long long sum = 0;
        for (uint64_t mm = m; mm; mm &= mm - 1) {
            const int j = __ffsll((unsigned long long)mm) - 1;
            sum += ((unsigned long long)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), j) << 32) |
                   (unsigned long long)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, j);
        }
        if ((int)__lane_id() == l) atomicAdd(p, sum);
        todo &= ~m;
    }
}

__device__ __forceinline__ uint64_t lane_mask_lt() {
    const uint32_t lane = __lane_id();
    return lane ? (~0ull >> (64 - lane)) : 0ull;
}

enum Outcome { kCollision = 0, kSurface = 1, kEscape = 2, kCapped = 3, kWalking = 4 };

// Local optical properties at a tentative collision: extinction, absorption,
// scattering and cloud extinction coefficients, cloud asymmetry.
struct Local {
    float ke, ka, ks, kc, g;
};

// Factored: `clear` marks a brick without cloud, whose cell records are all
// zero in the fields used here, so the gather is skipped.
template <bool kFactored>
__device__ __forceinline__ Local local_props(const TraceParams& P, int gp, uint32_t cell, int k, bool clear) {
    float4 c = make_float4(0.f, 0.f, 0.f, 0.f);
    if (!kFactored || !clear) c = P.cells[cell];
    Local L;
    if (!kFactored) {
        L.ke = c.x;
        L.ka = c.x * (1.0f - c.y);
        L.ks = c.x * c.y;
        L.kc = c.z;
        L.g = c.w;
    } else {
        const float2 q = P.gas[gp * P.nz + k];
        L.ke = q.x + c.x;
        L.ka = q.y + c.y;
        L.ks = (q.x - q.y) + (c.x - c.y);
        L.kc = c.x;
        L.g = c.z;
    }
    return L;
}

// One photon per lane.  Each loop iteration of
// a lane: (re)fill the lane with a new photon if it has none, draw the free
// path's four random words, walk acceleration-grid cells (at most
// P.max_walk crossings per iteration) until the tentative collision /
// surface / top, then handle that event.  kLds: majorant grid of the single
// g-point staged in LDS.  kFactored: shared cloud field + per-g-point gas
// profiles (several g-points in one launch).
// Launch shape: the single-g-point kernel runs 1024-lane workgroups at 8
// waves per SIMD (two workgroups per CU share the 160 KB LDS); the factored
// kernel needs more registers and runs 256-lane workgroups at 6 waves.
template <bool kFactored>
struct Shape_ {
    static constexpr int threads = kFactored ? 256 : 1024;
    static constexpr int waves = kFactored ? 6 : 8;
};

template <bool kLds, bool kFactored>
__global__ void __launch_bounds__(Shape_<kFactored>::threads)
    __attribute__((amdgpu_waves_per_eu(Shape_<kFactored>::waves))) trace_kernel(const TraceParams P) {
    extern __shared__ float s_maj[];
    __shared__ unsigned long long s_ledger[L_N];
    __shared__ unsigned long long s_stats[S_N];
    __shared__ unsigned long long s_passes, s_absorbed_coll;

    if (threadIdx.x < L_N) s_ledger[threadIdx.x] = 0;
    if (threadIdx.x < S_N) s_stats[threadIdx.x] = 0;
    if (threadIdx.x == 0) s_passes = s_absorbed_coll = 0;
    if (kLds) {
        for (int i = threadIdx.x; i < P.nmaj; i += blockDim.x) s_maj[i] = P.majorant[i];
    }
    __syncthreads();

    // ---- per-lane photon state
    bool alive = false;
    unsigned long long id = 0;
    int gp = 0;
    float px = 0.f, py = 0.f, pz = 0.f, ux = 0.f, uy = 0.f, uz = -1.f;
    int bi = 0, bj = 0, bk = 0;
    float tau = -1.f;  // optical depth left on the current free path; < 0: draw a new one
    // majorant of the current acceleration cell once read (kNoMajorant: not
    // yet); a photon stays in its cell across the null collisions there, so
    // the walk re-reads it only after a crossing or a new emission
    float kmaj = __uint_as_float(kNoMajorant);
    uint32_t w = 0, step = 0, iters = 0;
    bool direct = false;
    // merged deposit: cell index, bit 31 set for diffuse
    uint32_t pend_key = kNoCell;
    unsigned long long pend_amt = 0;
    // per-photon counters (folded into LDS when the photon ends).  Brick
    // crossings and null collisions are derived when the workgroup ends:
    // crossings = passes - collisions - surface hits - escapes - capped,
    // null = collisions - scatterings - photons absorbed at a collision.
    uint32_t n_coll = 0, n_scat = 0;  // n_scat: gas in the low, cloud in the high 16 bits

    // ---- per-wave photon-id pool (wave-uniform, kept in scalar registers)
    unsigned long long pool_next = 0, pool_end = 0;
    bool drained = false;

    auto flush_deposit = [&]() {
        if (pend_amt) {
            const uint32_t cell = pend_key & 0x7fffffffu;
            tally_add(pend_key & 0x80000000u ? &P.abs_dif[cell] : &P.abs_dir[cell], pend_amt, P.wave_agg);
        }
        pend_key = kNoCell;
        pend_amt = 0;
    };
    auto flush_scat = [&]() {
        lds_add(&s_stats[S_GAS], n_scat & 0xffffu);
        lds_add(&s_stats[S_CLOUD], n_scat >> 16);
        n_scat = 0;
    };
    auto finish_photon = [&]() {
        alive = false;
        lds_add(&s_stats[S_COLL], n_coll);
        lds_add(&s_passes, iters);
        flush_scat();
        n_coll = 0;
    };
    auto key0 = [&]() { return (uint32_t)(P.seed + (unsigned long long)(kFactored ? gp : 0)); };
    auto key1 = [&]() { return (uint32_t)((P.seed + (unsigned long long)(kFactored ? gp : 0)) >> 32); };
    // Russian roulette (sec. 2.3) with the current free path's counter
    // (id, step, 1): survive with probability w, then weight one.
    auto roulette = [&]() {
        if (w >= P.rr_below) return;
        const uint4 q = philox(make_uint4((uint32_t)id, (uint32_t)(id >> 32), step, 1u), key0(), key1());
        if ((q.x >> 1) < w) {
            lds_add(&s_ledger[L_RR_GAIN], kWOne - w);
            atomicAdd(&s_stats[S_RR_SURV], 1ull);
            w = kWOne;
        } else {
            lds_add(&s_ledger[L_RR_LOSS], w);
            atomicAdd(&s_stats[S_RR_KILL], 1ull);
            finish_photon();
        }
    };
    auto cell_ix = [&](float v, float inv, int b, int n) {
        return min(max((int)floorf(v * inv), b * n), b * n + n - 1);
    };

    for (;;) {
        // ---- refill finished lanes from the wave's pool of photon ids, once
        // enough of them are idle (the emission code then runs for many
        // lanes at once instead of for one or two) or none is alive
        const uint64_t dead = __ballot(!alive);
        if (dead && !drained && ((uint32_t)__popcll(dead) >= P.refill || !__ballot(alive))) {
            const uint32_t need = (uint32_t)__popcll(dead);
            const int leader = __ffsll((unsigned long long)dead) - 1;
            const unsigned long long avail = pool_end - pool_next;
            unsigned long long base = 0;
            if (avail < need) {
                if ((int)__lane_id() == leader) base = atomicAdd(P.queue, (unsigned long long)P.pool);
                base = __shfl(base, leader);
                // readfirstlane returns a signed int: widen through uint32_t
                base = ((unsigned long long)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(base >> 32)) << 32) |
                       (unsigned long long)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)base);
            }
            if (!alive) {
                const uint32_t rank = (uint32_t)__popcll(dead & lane_mask_lt());
                const unsigned long long local = rank < avail ? pool_next + rank : base + (rank - avail);
                if (local < P.photons) {
                    // queue slot -> g-point, photon id and entry column
                    const Slot sl = decode_slot(P.sched, local);
                    gp = kFactored ? sl.gp : 0;
                    id = sl.id;
                    const uint32_t col = sl.col;
                    // ---- emission at the top of the domain (sec. 2.3)
                    const int ic = (int)(col % (unsigned)P.nx);
                    const int jc = (int)(col / (unsigned)P.nx);
                    const uint4 e = philox(make_uint4((uint32_t)id, (uint32_t)(id >> 32), 0xffffffffu, 0u),
                                           key0(), key1());
                    float fx = u01(e.x), fy = u01(e.y);
                    if (P.sobol) {
                        // photon id is the (id div ncol)-th to enter its column
                        const uint32_t pass = (uint32_t)(id / P.ncol);
                        const uint4 sc = philox(make_uint4(col, 0u, 0xfffffffdu, 0u),
                                                key0(), key1());
                        fx = u01(owen_scramble<24>(__builtin_bitreverse32(pass), sc.x));
                        fy = u01(owen_scramble<24>(sobol_dim2(pass), sc.y));
                    }
                    px = ((float)ic + fx) * P.dx;
                    py = ((float)jc + fy) * P.dy;
                    pz = P.H;
                    const float fd = P.gp_diffuse ? P.gp_diffuse[gp] : P.diffuse_fraction;
                    if (u01(e.z) < fd) {
                        const uint4 q = philox(make_uint4((uint32_t)id, (uint32_t)(id >> 32), 0xffffffffu, 1u),
                                               key0(), key1());
                        const float mu = sqrtf(u01_open(q.x));
                        float sp, cp;
                        __sincosf(6.28318530717958647f * u01(q.y), &sp, &cp);
                        const float st = sqrtf(fmaxf(0.0f, 1.0f - mu * mu));
                        ux = st * cp;
                        uy = st * sp;
                        uz = -mu;
                        direct = false;
                    } else {
                        ux = P.sun_x;
                        uy = P.sun_y;
                        uz = P.sun_z;
                        direct = true;
                    }
                    bi = ic / P.bx;
                    bj = jc / P.by;
                    bk = P.mz - 1;
                    kmaj = __uint_as_float(kNoMajorant);
                    w = kWOne;
                    step = 0;
                    iters = 0;
                    tau = -1.f;
                    alive = true;
                    atomicAdd(&s_stats[S_PHOT], 1ull);
                    lds_add(&s_ledger[L_IN], kWOne);
                }
            }
            if (avail < need) {
                pool_next = base + (need - avail);
                pool_end = base + P.pool;
            } else {
                pool_next += need;
            }
            // ids only grow (pool first, later grabs above pool_end), so once
            // pool_next passes the photon count no valid id is left
            drained = pool_next >= P.photons;
        }
        if (!__ballot(alive)) break;
        if (!alive) continue;

        // ---- random words of this free path: tau, event, cos(theta), phi
        const uint4 r = philox(make_uint4((uint32_t)id, (uint32_t)(id >> 32), step, 0u), key0(), key1());
        if (tau < 0.f) tau = -__logf(u01_open(r.x));
        const int maj_base = kFactored ? gp * P.nmaj : 0;  // this g-point's majorant grid

        // ---- walk acceleration-grid cells until the path ends
        int outcome;
        float K;
        for (int walked = 0;; ++walked) {
            if (iters >= P.max_iters) { outcome = kCapped; break; }
            if (walked >= P.max_walk) { outcome = kWalking; break; }
            ++iters;
            // factored majorants carry the brick's "no cloud" flag in the sign bit
            if (__float_as_uint(kmaj) == kNoMajorant)
                kmaj = kLds ? s_maj[(bk * P.my + bj) * P.mx + bi] : P.majorant[maj_base + (bk * P.my + bj) * P.mx + bi];
            K = kmaj;
            const float Km = fabsf(K);
            const float x0 = (float)bi * P.cx, y0 = (float)bj * P.cy, z0 = (float)bk * P.cz;
            float tx = INFINITY, ty = INFINITY, tz = INFINITY;
            if (ux > 0.f) tx = (x0 + P.cx - px) * rcp(ux);
            else if (ux < 0.f) tx = (x0 - px) * rcp(ux);
            if (uy > 0.f) ty = (y0 + P.cy - py) * rcp(uy);
            else if (uy < 0.f) ty = (y0 - py) * rcp(uy);
            if (uz > 0.f) tz = (z0 + P.cz - pz) * rcp(uz);
            else if (uz < 0.f) tz = (z0 - pz) * rcp(uz);
            tx = fmaxf(tx, 0.f);
            ty = fmaxf(ty, 0.f);
            tz = fmaxf(tz, 0.f);
            int axis = 0;
            float s_exit = tx;
            if (ty < s_exit) { s_exit = ty; axis = 1; }
            if (tz < s_exit) { s_exit = tz; axis = 2; }
            if (Km * s_exit >= tau) {
                const float sc = tau * rcp(Km);
                px += sc * ux;
                py += sc * uy;
                pz += sc * uz;
                outcome = kCollision;
                break;
            }
            tau -= Km * s_exit;
            px += s_exit * ux;
            py += s_exit * uy;
            pz += s_exit * uz;
            if (axis == 2) {
                if (uz < 0.f) {
                    if (bk == 0) { pz = 0.f; outcome = kSurface; break; }
                    --bk;
                    pz = (float)(bk + 1) * P.cz;
                } else {
                    if (bk == P.mz - 1) { outcome = kEscape; break; }
                    ++bk;
                    pz = (float)bk * P.cz;
                }
            } else if (axis == 0) {
                if (ux > 0.f) {
                    bi = bi + 1 == P.mx ? 0 : bi + 1;
                    px = (float)bi * P.cx;
                } else {
                    bi = bi == 0 ? P.mx - 1 : bi - 1;
                    px = (float)(bi + 1) * P.cx;
                }
            } else {
                if (uy > 0.f) {
                    bj = bj + 1 == P.my ? 0 : bj + 1;
                    py = (float)bj * P.cy;
                } else {
                    bj = bj == 0 ? P.my - 1 : bj - 1;
                    py = (float)(bj + 1) * P.cy;
                }
            }
            kmaj = __uint_as_float(kNoMajorant);  // crossed into another cell
        }
        if (outcome == kWalking) continue;  // same free path next iteration
        tau = -1.f;

        if (outcome == kCollision) {
            // ---- tentative collision: local properties from the fine grid
            const int i = cell_ix(px, P.inv_dx, bi, P.bx);
            const int j = cell_ix(py, P.inv_dy, bj, P.by);
            const int k = cell_ix(pz, P.inv_dz, bk, P.bz);
            const uint32_t cell = (uint32_t)((k * P.ny + j) * P.nx + i);
            bool clear = kFactored && __float_as_uint(K) >> 31;
            if (kFactored && !clear && P.cell_mask) {
                // a cloud-free fine cell of a cloudy acceleration cell holds a
                // zero record too: its bit, from a small array that stays in
                // the L2, spares the gather of a whole line of records
                const uint32_t t = (uint32_t)(((k - bk * P.bz) * P.by + (j - bj * P.by)) * P.bx + (i - bi * P.bx));
                const uint32_t b = (uint32_t)((bk * P.my + bj) * P.mx + bi);
                clear = !((P.cell_mask[(size_t)b * P.mask_words + (t >> 5)] >> (t & 31)) & 1u);
            }
            K = fabsf(K);
            const Local L = local_props<kFactored>(P, gp, cell, k, clear);
            const float iK = rcp(K);
            ++n_coll;
            if (L.ka > 0.f) {
                const uint32_t dep = min(w, (uint32_t)rintf((float)w * (L.ka * iK)));
                const uint32_t key = cell | (direct ? 0u : 0x80000000u);
                if (key != pend_key) {
                    flush_deposit();
                    pend_key = key;
                }
                pend_amt += dep;
                if (!P.merge) flush_deposit();
                w -= dep;
                if (w == 0) {
                    atomicAdd(&s_stats[S_ABSORBED], 1ull);
                    atomicAdd(&s_absorbed_coll, 1ull);
                    finish_photon();
                    continue;
                }
            }
            // scattering with probability k_sca / (K - k_abs), else null
            const float den = K - L.ka;
            const float ps = den > 0.f ? L.ks * rcp(den) : 0.f;
            const float xi = u01(r.y);
            if (xi < ps) {
                float mu;
                if (xi * L.ke < ps * L.kc) {
                    mu = hg_cos(L.g, u01(r.z));
                    n_scat += 0x10000u;
                } else {
                    mu = rayleigh_cos(u01(r.z));
                    n_scat += 1u;
                }
                turn(ux, uy, uz, mu, u01(r.w));
                direct = false;
                if ((n_scat & 0x8000u) | (n_scat & 0x80000000u)) flush_scat();
            }
            roulette();
            ++step;
            continue;
        }
        if (outcome == kSurface) {
            // ---- Lambertian surface (sec. 2.3)
            const int i = cell_ix(px, P.inv_dx, bi, P.bx);
            const int j = cell_ix(py, P.inv_dy, bj, P.by);
            const int c2 = j * P.nx + i;
            tally_add(direct ? &P.sfc_dir[c2] : &P.sfc_dif[c2], (unsigned long long)w, P.wave_agg);
            const uint32_t wn = min(w, (uint32_t)rintf(P.albedo[c2] * (float)w));
            if (w != wn) {
                tally_add(&P.sfc_abs[c2], (unsigned long long)(w - wn), P.wave_agg);
                lds_add(&s_ledger[L_SFC], w - wn);
            }
            atomicAdd(&s_stats[S_SFC], 1ull);
            w = wn;
            if (w == 0) {
                atomicAdd(&s_stats[S_ABSORBED], 1ull);
                finish_photon();
                continue;
            }
            const float mu = sqrtf(u01_open(r.z));
            float sp, cp;
            __sincosf(6.28318530717958647f * u01(r.w), &sp, &cp);
            const float st = sqrtf(fmaxf(0.0f, 1.0f - mu * mu));
            ux = st * cp;
            uy = st * sp;
            uz = mu;
            direct = false;
            roulette();
            ++step;
            continue;
        }
        if (outcome == kEscape) {
            // ---- leaves through the top of the domain
            const int i = cell_ix(px, P.inv_dx, bi, P.bx);
            const int j = cell_ix(py, P.inv_dy, bj, P.by);
            tally_add(&P.toa_up[j * P.nx + i], (unsigned long long)w, P.wave_agg);
            lds_add(&s_ledger[L_TOA], w);
            atomicAdd(&s_stats[S_ESC], 1ull);
            finish_photon();
            continue;
        }
        // iteration cap reached
        lds_add(&s_ledger[L_LOST], w);
        atomicAdd(&s_stats[S_CAPPED], 1ull);
        finish_photon();
    }

    flush_deposit();
    __syncthreads();
    if (threadIdx.x == 0) {
        s_stats[S_CROSS] = s_passes - s_stats[S_COLL] - s_stats[S_SFC] - s_stats[S_ESC] - s_stats[S_CAPPED];
        s_stats[S_NULL] = s_stats[S_COLL] - s_stats[S_GAS] - s_stats[S_CLOUD] - s_absorbed_coll;
    }
    __syncthreads();
    if (threadIdx.x < L_N && s_ledger[threadIdx.x]) atomicAdd(&P.ledger[threadIdx.x], s_ledger[threadIdx.x]);
    if (threadIdx.x < S_N && s_stats[threadIdx.x]) atomicAdd(&P.stats[threadIdx.x], s_stats[threadIdx.x]);
}

// Heating entries of the energy ledger: ledger[ATM_DIR] = sum(abs_dir),
// ledger[ATM_DIF] = sum(abs_dif), exact uint64 sums (the other entries are
// counted by the tracing kernel, so the identity still checks that no
// deposit was lost).  The two entries are cleared first (clear_atm_kernel);
// every workgroup adds its partial sums.
__global__ void clear_atm_kernel(unsigned long long* __restrict__ ledger) {
    if (threadIdx.x == 0) {
        ledger[L_ATM_DIR] = 0;
        ledger[L_ATM_DIF] = 0;
    }
}

__global__ void ledger_atm_kernel(const unsigned long long* __restrict__ abs_dir,
                                  const unsigned long long* __restrict__ abs_dif, size_t n,
                                  unsigned long long* __restrict__ ledger) {
    __shared__ unsigned long long part[2][256];
    unsigned long long sd = 0, sf = 0;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        sd += abs_dir[i];
        sf += abs_dif[i];
    }
    part[0][threadIdx.x] = sd;
    part[1][threadIdx.x] = sf;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            part[0][threadIdx.x] += part[0][threadIdx.x + h];
            part[1][threadIdx.x] += part[1][threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (part[0][0]) atomicAdd(&ledger[L_ATM_DIR], part[0][0]);
        if (part[1][0]) atomicAdd(&ledger[L_ATM_DIF], part[1][0]);
    }
}

// Interleave the four SoA property arrays into one 16-byte record per cell,
// so a tentative collision needs a single random 16-byte gather.
__global__ void pack_cells_kernel(const float* __restrict__ ke, const float* __restrict__ om,
                                  const float* __restrict__ kc, const float* __restrict__ g,
                                  float4* __restrict__ out, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        out[i] = make_float4(ke[i], om[i], kc[i], g[i]);
}

// Factored medium: per cell (k_ext_cloud, cloud k_abs, g, 0).
__global__ void pack_cloud_kernel(const float* __restrict__ kc, const float* __restrict__ om,
                                  const float* __restrict__ g, float4* __restrict__ out, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const float k = kc[i];
        out[i] = make_float4(k, k * (1.0f - om[i]), g[i], 0.0f);
    }
}

// Factored medium: the cloud-cell mask of the tracer, one 32-bit word per
// thread: bit s of word q of acceleration cell b is fine cell t = 32 q + s of
// that cell (x fastest, then y, then z), set where k_ext_cloud != 0 (a cell
// whose bit is clear has the record (0, 0, g, 0), whose g is never used).
__global__ void cell_mask_kernel(const float* __restrict__ kc, uint32_t* __restrict__ mask, int nx, int ny, int bx,
                                 int by, int bz, int mx, int my, int words, size_t n) {
    const int nb = bx * by * bz;
    for (size_t w = blockIdx.x * (size_t)blockDim.x + threadIdx.x; w < n; w += (size_t)gridDim.x * blockDim.x) {
        const size_t b = w / words;
        const int q = (int)(w % words);
        const int bi = (int)(b % mx), bj = (int)((b / mx) % my), bk = (int)(b / ((size_t)mx * my));
        uint32_t m = 0;
        for (int s = 0; s < 32; ++s) {
            const int t = 32 * q + s;
            if (t >= nb) break;
            const int ix = t % bx, jy = (t / bx) % by, kz = t / (bx * by);
            const size_t cell = ((size_t)(bk * bz + kz) * ny + (size_t)(bj * by + jy)) * nx + (size_t)(bi * bx + ix);
            if (kc[cell] != 0.0f) m |= 1u << s;
        }
        mask[w] = m;
    }
}

// Factored medium: per g-point and level (k_gas, gas k_abs).
__global__ void pack_gas_kernel(const float* __restrict__ kg, const float* __restrict__ om, float2* __restrict__ out,
                                size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const float k = kg[i];
        out[i] = make_float2(k, k * (1.0f - om[i]));
    }
}

// Factored majorant, step 1: per level k and acceleration column (bi, bj),
// the largest cloud extinction: layer[k][bj][bi] (FP32 bits, integer max).
__global__ void layer_max_kernel(const float4* __restrict__ cells, uint32_t* __restrict__ layer, int nx, int ny,
                                 int nz, int bx, int by) {
    const int mx = nx / bx, my = ny / by;
    const size_t n = (size_t)mx * ny * nz;
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x) {
        const int bi = (int)(t % mx);
        const size_t row = t / mx;  // j + ny * k
        const int j = (int)(row % ny);
        const int k = (int)(row / ny);
        const float4* src = cells + row * nx + (size_t)bi * bx;
        uint32_t m = 0;
        for (int q = 0; q < bx; ++q) {
            const float v = src[q].x;
            const uint32_t bits = v > 0.0f ? __float_as_uint(v) : 0u;
            m = bits > m ? bits : m;
        }
        atomicMax(&layer[((size_t)k * my + j / by) * mx + bi], m);
    }
}

// Factored majorant, step 2: K[n][bk][bj][bi] = max over the levels k of
// brick layer bk of (k_gas[n][k] + layer[k][bj][bi]).  FP32 addition is
// monotonic, so this equals the largest k_gas + k_cloud of the cells.  A
// brick with no cloud extinction in any cell stores -K (sign bit set, -0 for
// K = 0): the tracer reads |K| and skips the cell gather there.
__global__ void gas_majorant_kernel(const uint32_t* __restrict__ layer, const float2* __restrict__ gas,
                                    float* __restrict__ maj, int ngp, int nz, int mx, int my, int bz) {
    const int mz = nz / bz;
    const size_t nmaj = (size_t)mx * my * mz;
    const size_t n = nmaj * ngp;
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x) {
        const int gp = (int)(t / nmaj);
        const size_t b = t % nmaj;
        const size_t col = b % ((size_t)mx * my);
        const int bk = (int)(b / ((size_t)mx * my));
        float m = 0.0f;
        uint32_t cloud = 0;
        for (int q = 0; q < bz; ++q) {
            const int k = bk * bz + q;
            const uint32_t lc = layer[(size_t)k * mx * my + col];
            const float v = gas[(size_t)gp * nz + k].x + __uint_as_float(lc);
            m = v > m ? v : m;
            cloud |= lc;
        }
        maj[t] = __uint_as_float(__float_as_uint(m) | (cloud ? 0u : 0x80000000u));
    }
}

// Per-g-point schedule tables (prefix sums of the full passes over all
// columns and of the photons left over) and systematic-sampling column
// offsets (Philox counter (0, 0, 0xfffffffe, 0) under the g-point's key,
// word 0).
constexpr int kMaxGpoints = 256;
struct BatchInit {
    unsigned long long photons[kMaxGpoints];
    unsigned long long seed, ncol;
    int ngp;
};

__global__ void batch_init_kernel(const BatchInit a, unsigned long long* __restrict__ pass_first,
                                  unsigned long long* __restrict__ rem_first,
                                  unsigned long long* __restrict__ gp_col_offset) {
    const int t = threadIdx.x;
    if (t == 0) schedule_tables(a.photons, a.ngp, a.ncol, pass_first, rem_first);
    for (int n = t; n < a.ngp; n += blockDim.x) {
        const unsigned long long key = a.seed + (unsigned long long)n;
        const uint4 r = philox(make_uint4(0u, 0u, 0xfffffffeu, 0u), (uint32_t)key, (uint32_t)(key >> 32));
        gp_col_offset[n] = ((unsigned long long)r.x * a.ncol) >> 32;
    }
}

// ---------------------------------------------------------------------------
// Small kernels
// ---------------------------------------------------------------------------
__global__ void fill_u64_kernel(unsigned long long* p, size_t n, unsigned long long v) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void fill_u32_kernel(uint32_t* p, size_t n, uint32_t v) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Row pass of the majorant build: thread (bi, j, k) takes the maximum of
// the bx cells of row (j, k) inside acceleration cell column bi and merges it
// into the acceleration cell with an integer max of the FP32 bits (exact,
// as every value is >= +0; non-positive values and NaN count as 0).
__global__ void majorant_kernel(const float* __restrict__ k_ext, uint32_t* __restrict__ maj, int nx, int ny,
                                int nz, int bx, int by, int bz) {
    const int mx = nx / bx, my = ny / by;
    const size_t n = (size_t)mx * ny * nz;
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x) {
        const int bi = (int)(t % mx);
        const size_t row = t / mx;  // j + ny * k
        const int j = (int)(row % ny);
        const int k = (int)(row / ny);
        const float* src = k_ext + row * nx + (size_t)bi * bx;
        uint32_t m = 0;
        for (int q = 0; q < bx; ++q) {
            const float v = src[q];
            const uint32_t bits = v > 0.0f ? __float_as_uint(v) : 0u;
            m = bits > m ? bits : m;
        }
        atomicMax(&maj[((size_t)(k / bz) * my + j / by) * mx + bi], m);
    }
}

// Validation of the inputs: sets bit 0 of *flag for any violation.
__global__ void validate_kernel(const float* __restrict__ ke, const float* __restrict__ kc,
                                const float* __restrict__ om, const float* __restrict__ g,
                                const float* __restrict__ alb, size_t ncell, size_t ncol, uint32_t* flag) {
    uint32_t bad = 0;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < ncell; i += (size_t)gridDim.x * blockDim.x) {
        const float a = ke[i], b = kc[i], c = om[i], d = g[i];
        const bool ok = (a >= 0.f) && (a < INFINITY) && (b >= 0.f) && (b <= a) && (c >= 0.f) && (c <= 1.f) &&
                        (d >= -1.f) && (d <= 1.f);
        bad |= ok ? 0u : 1u;
    }
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < ncol; i += (size_t)gridDim.x * blockDim.x) {
        const float a = alb[i];
        bad |= (a >= 0.f && a <= 1.f) ? 0u : 1u;
    }
    if (__ballot(bad) && __lane_id() == 0) atomicOr(flag, 1u);
}

__global__ void validate_batched_kernel(const float* __restrict__ kg, const float* __restrict__ og, size_t ngas,
                                        const float* __restrict__ kc, const float* __restrict__ oc,
                                        const float* __restrict__ g, const float* __restrict__ alb, size_t ncell,
                                        size_t ncol, const float* __restrict__ fd, int ngp, uint32_t* flag) {
    uint32_t bad = 0;
    const size_t s0 = blockIdx.x * (size_t)blockDim.x + threadIdx.x, st = (size_t)gridDim.x * blockDim.x;
    if (fd)
        for (size_t i = s0; i < (size_t)ngp; i += st) bad |= (fd[i] >= 0.f && fd[i] <= 1.f) ? 0u : 1u;
    for (size_t i = s0; i < ngas; i += st) {
        const float a = kg[i], b = og[i];
        bad |= (a >= 0.f && a < INFINITY && b >= 0.f && b <= 1.f) ? 0u : 1u;
    }
    for (size_t i = s0; i < ncell; i += st) {
        const float a = kc[i], b = oc[i], d = g[i];
        bad |= (a >= 0.f && a < INFINITY && b >= 0.f && b <= 1.f && d >= -1.f && d <= 1.f) ? 0u : 1u;
    }
    for (size_t i = s0; i < ncol; i += st) {
        const float a = alb[i];
        bad |= (a >= 0.f && a <= 1.f) ? 0u : 1u;
    }
    if (__ballot(bad) && __lane_id() == 0) atomicOr(flag, 1u);
}

__global__ void finalize3_kernel(const unsigned long long* __restrict__ raw, float* __restrict__ out, size_t plane,
                                 size_t n, double norm, const double* __restrict__ layer_scale) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const double s = layer_scale ? layer_scale[i / plane] * norm : norm;
        out[i] = (float)((double)raw[i] * s);
    }
}

__global__ void philox_kernel(const uint4* __restrict__ ctr, uint32_t k0, uint32_t k1, uint4* __restrict__ out,
                              uint32_t n) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = philox(ctr[i], k0, k1);
}

// Entry coordinates of passes first .. first+n-1 of one column, all 32
// digits scrambled (the tracer uses the first 24 of the same values).
__global__ void sobol_entry_kernel(unsigned long long first, uint32_t n, unsigned long long col, uint32_t k0,
                                   uint32_t k1, uint2* __restrict__ out) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint4 sc = philox(make_uint4((uint32_t)col, (uint32_t)(col >> 32), 0xfffffffdu, 0u), k0, k1);
    const uint32_t p = (uint32_t)(first + i);
    out[i] = make_uint2(owen_scramble<32>(__builtin_bitreverse32(p), sc.x), owen_scramble<32>(sobol_dim2(p), sc.y));
}

// The tracer's scattering-angle samplers and direction turn, element-wise,
// for tests: kind 0 = Henyey-Greenstein with g[i], kind 1 = Rayleigh.
__global__ void phase_sample_kernel(int kind, const float* __restrict__ g, const float* __restrict__ xi,
                                    float* __restrict__ mu, uint32_t n) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) mu[i] = kind == 0 ? hg_cos(g[i], xi[i]) : rayleigh_cos(xi[i]);
}

__global__ void turn_kernel(const float* __restrict__ din, const float* __restrict__ mu, const float* __restrict__ t,
                            float* __restrict__ dout, uint32_t n) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float x = din[3 * i], y = din[3 * i + 1], z = din[3 * i + 2];
    turn(x, y, z, mu[i], t[i]);
    dout[3 * i] = x;
    dout[3 * i + 1] = y;
    dout[3 * i + 2] = z;
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
thread_local char g_err[256] = "";
thread_local hipEvent_t g_t0 = nullptr, g_t1 = nullptr;
thread_local bool g_timed = false;

rt3d_status dev_fail(hipError_t e, const char* where) {
    snprintf(g_err, sizeof g_err, "%s: %s", where, hipGetErrorString(e));
    return RT3D_EDEVICE;
}

#define HIP_TRY(expr)                                  \
    do {                                               \
        hipError_t e_ = (expr);                        \
        if (e_ != hipSuccess) return dev_fail(e_, #expr); \
    } while (0)

struct Shape {
    int nx, ny, nz, bx, by, bz, mx, my, mz;
    size_t ncell, ncol, nmaj;
};

bool grid_ok(const rt3d_grid* g) {
    if (!g || g->nx <= 0 || g->ny <= 0 || g->nz <= 0) return false;
    if (!(g->dx > 0.f) || !(g->dy > 0.f) || !(g->dz > 0.f)) return false;
    if (!std::isfinite(g->dx) || !std::isfinite(g->dy) || !std::isfinite(g->dz)) return false;
    const long long n = (long long)g->nx * g->ny * g->nz;
    return n < 0x7fffffffLL;
}

void resolve_options(const rt3d_grid* g, const rt3d_options* in, rt3d_options* out) {
    rt3d_default_options(out);
    if (in) *out = *in;
    if (out->brick_x <= 0) out->brick_x = g->nx % 8 == 0 ? 8 : 1;
    if (out->brick_y <= 0) out->brick_y = g->ny % 8 == 0 ? 8 : 1;
    if (out->brick_z <= 0) out->brick_z = g->nz % 8 == 0 ? 8 : 1;
    if (out->max_iters == 0) out->max_iters = 1u << 24;
}

bool shape_of(const rt3d_grid* g, const rt3d_options* o, Shape* s) {
    if (!grid_ok(g)) return false;
    if (o->brick_x <= 0 || o->brick_y <= 0 || o->brick_z <= 0) return false;
    if (g->nx % o->brick_x || g->ny % o->brick_y || g->nz % o->brick_z) return false;
    s->nx = g->nx; s->ny = g->ny; s->nz = g->nz;
    s->bx = o->brick_x; s->by = o->brick_y; s->bz = o->brick_z;
    s->mx = g->nx / o->brick_x; s->my = g->ny / o->brick_y; s->mz = g->nz / o->brick_z;
    s->ncell = (size_t)g->nx * g->ny * g->nz;
    s->ncol = (size_t)g->nx * g->ny;
    s->nmaj = (size_t)s->mx * s->my * s->mz;
    return true;
}

constexpr size_t kCtrlBytes = 256;  // queue counter + validation flag
size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

unsigned grid_for(size_t n, unsigned block = 256, unsigned cap = 8192) {
    size_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

rt3d_status zero_u64(unsigned long long* p, size_t n, hipStream_t st) {
    if (!n) return RT3D_OK;
    hipLaunchKernelGGL(fill_u64_kernel, dim3(grid_for(n)), dim3(256), 0, st, p, n, 0ull);
    HIP_TRY(hipGetLastError());
    return RT3D_OK;
}


// Workspace layout (every section 256-byte aligned):
//   control  256 B: photon-id queue counter, validation flag
//   meta     schedule tables: full passes [ngp + 1], photons left over
//            [ngp + 1], column offsets [ngp] (uint64)
//   maj      majorants [ngp][nmaj] FP32
//   cells    packed per-cell records [ncell] float4
//   gas      factored only: (k_gas, gas k_abs) [ngp][nz] float2
//   layer    factored only: per-level cloud maxima [nz][my][mx] uint32
//   mask     factored only: cloud-cell bits [nmaj][mask_words] uint32
struct Layout {
    size_t meta, maj, cells, gas, layer, mask, total;
};

int mask_words_of(const Shape& s) { return (s.bx * s.by * s.bz + 31) / 32; }

Layout layout_of(const Shape& s, int ngp, bool factored) {
    Layout l;
    size_t off = kCtrlBytes;
    l.meta = off;
    off += align256(sizeof(unsigned long long) * (3 * (size_t)ngp + 2));
    l.maj = off;
    off += align256(sizeof(float) * s.nmaj * ngp);
    l.cells = off;
    off += align256(sizeof(float4) * s.ncell);
    l.gas = l.layer = l.mask = 0;
    if (factored) {
        l.gas = off;
        off += align256(sizeof(float2) * (size_t)ngp * s.nz);
        l.layer = off;
        off += align256(sizeof(uint32_t) * (size_t)s.nz * s.my * s.mx);
        l.mask = off;
        off += align256(sizeof(uint32_t) * s.nmaj * (size_t)mask_words_of(s));
    }
    l.total = off;
    return l;
}

// Entry tiles of the photon schedule: tile_x x tile_y columns, each edge a
// divisor of the grid's.  Automatic: tiles whose columns hold about
// kTileFootprintBytes of cell records and heating tallies (32 bytes per
// cell), close to square, the whole domain when it holds less.  Measured on
// one MI355X (same photons, bitwise-identical tallies, kernel time against
// one whole-domain tile): 1024x1024x128, 112 g-points, 1024 photons per
// column: 128x128 -11.3 %, 64x64 -10.4 %, 16x16 -9.4 %; 512x512x96: 256x256
// and 128x256 -10.3 %, 64x64 -2.5 %, 16x16 +4.3 %; 256x256x128, one g-point
// (fits the Infinity Cache already): 128x128 +0.8 %, 32x32 +7.2 %.
constexpr size_t kTileFootprintBytes = size_t(128) << 20;

uint32_t largest_divisor_upto(int n, long long cap) {
    for (long long d = cap < n ? cap : n; d > 1; --d)
        if (n % d == 0) return (uint32_t)d;
    return 1u;
}

void tile_shape(const Shape& s, const rt3d_options& o, uint32_t* tx, uint32_t* ty) {
    const long long target = (long long)std::max<size_t>(1, kTileFootprintBytes / ((size_t)s.nz * 32));
    if (o.tile_x > 0 && o.tile_y > 0) {
        *tx = (uint32_t)o.tile_x;
        *ty = (uint32_t)o.tile_y;
    } else if (o.tile_x > 0) {
        *tx = (uint32_t)o.tile_x;
        *ty = largest_divisor_upto(s.ny, std::max<long long>(1, target / o.tile_x));
    } else if (o.tile_y > 0) {
        *ty = (uint32_t)o.tile_y;
        *tx = largest_divisor_upto(s.nx, std::max<long long>(1, target / o.tile_y));
    } else if (target >= (long long)s.ncol) {
        *tx = (uint32_t)s.nx;
        *ty = (uint32_t)s.ny;
    } else {
        *tx = largest_divisor_upto(s.nx, std::max<long long>(1, (long long)std::sqrt((double)target)));
        *ty = largest_divisor_upto(s.ny, std::max<long long>(1, target / *tx));
        if (*ty == (uint32_t)s.ny) *tx = largest_divisor_upto(s.nx, std::max<long long>(1, target / s.ny));
    }
}

void schedule_of(const Shape& s, int ngp, const uint64_t* photons, const rt3d_options& o,
                 const unsigned long long* pass_first, const unsigned long long* rem_first,
                 const unsigned long long* col_offset, Schedule* S) {
    unsigned long long passes = 0;
    for (int n = 0; n < ngp; ++n) passes += photons[n] / s.ncol;
    S->pass_first = pass_first;
    S->rem_first = rem_first;
    S->col_offset = col_offset;
    S->ngp = ngp;
    S->ncol = (uint32_t)s.ncol;
    S->nx = (uint32_t)s.nx;
    tile_shape(s, o, &S->tile_x, &S->tile_y);
    S->tile_cols = S->tile_x * S->tile_y;
    S->ntx = (uint32_t)s.nx / S->tile_x;
    S->full_slots = passes * s.ncol;
    S->tile_slots = passes * S->tile_cols;
    S->photon_offset = o.photon_offset;
    S->po_mod = (uint32_t)(o.photon_offset % s.ncol);
}

struct Launch {
    rt3d_options o;
    Shape s;
    int ngp;
    unsigned long long total;
    char* ws;
    uint32_t* flag;
    float* maj;
    float4* cells;
    float2* gas;
    uint32_t* layer;
    uint32_t* mask;
    TraceParams P;
};

rt3d_status prepare(const rt3d_grid* grid, int ngp, const uint64_t* photons, const float* albedo, double sza_deg,
                    double azimuth_deg, uint64_t seed, const rt3d_options* opt, const rt3d_tallies* out,
                    void* workspace, size_t workspace_bytes, void* stream, bool factored, Launch* L) {
    if (!grid_ok(grid)) return RT3D_EINVAL;
    resolve_options(grid, opt, &L->o);
    const rt3d_options& o = L->o;
    if (!shape_of(grid, &o, &L->s)) return RT3D_EINVAL;
    const Shape& s = L->s;
    if (!albedo || !photons) return RT3D_EINVAL;
    if (!out || !out->abs_dir || !out->abs_dif || !out->sfc_dir || !out->sfc_dif || !out->sfc_abs ||
        !out->toa_up || !out->ledger || !out->stats)
        return RT3D_EINVAL;
    if (!(sza_deg >= 0.0 && sza_deg < 90.0) || !std::isfinite(azimuth_deg)) return RT3D_EINVAL;
    if (!(o.diffuse_fraction >= 0.f && o.diffuse_fraction <= 1.f)) return RT3D_EINVAL;
    if (!(o.rr_threshold >= 0.f && o.rr_threshold <= 1.f)) return RT3D_EINVAL;
    if (o.grid_blocks < 0 || o.block_threads < 0 || o.max_walk < 0 || o.pool_photons < 0) return RT3D_EINVAL;
    // a refill hands out up to one id per lane of the wave from one grab, so
    // a grab must hold at least a wave's 64 ids
    if (o.pool_photons > 0 && o.pool_photons < 64) return RT3D_EINVAL;
    if (o.refill_lanes < 0 || o.refill_lanes > 64) return RT3D_EINVAL;
    if (o.tile_x < 0 || o.tile_y < 0 || (o.tile_x && s.nx % o.tile_x) || (o.tile_y && s.ny % o.tile_y))
        return RT3D_EINVAL;
    if (o.block_threads && o.block_threads != (factored ? Shape_<true>::threads : Shape_<false>::threads))
        return RT3D_EINVAL;
    unsigned long long total = 0;
    for (int n = 0; n < ngp; ++n) {
        if (total + photons[n] < total) return RT3D_EINVAL;
        total += photons[n];
    }
    // the ledger holds photons * 2^31 in uint64
    if (total == 0 || total >= (1ull << 33)) return RT3D_EINVAL;
    if (o.photon_offset + total < o.photon_offset) return RT3D_EINVAL;
    const Layout lay = layout_of(s, ngp, factored);
    if (!workspace || workspace_bytes < lay.total || ((uintptr_t)workspace & 255)) return RT3D_EINVAL;

    L->ngp = ngp;
    L->total = total;
    L->ws = (char*)workspace;
    L->flag = (uint32_t*)(L->ws + 128);
    L->maj = (float*)(L->ws + lay.maj);
    L->cells = (float4*)(L->ws + lay.cells);
    L->gas = factored ? (float2*)(L->ws + lay.gas) : nullptr;
    L->layer = factored ? (uint32_t*)(L->ws + lay.layer) : nullptr;
    L->mask = factored ? (uint32_t*)(L->ws + lay.mask) : nullptr;
    unsigned long long* pass_first = (unsigned long long*)(L->ws + lay.meta);
    unsigned long long* rem_first = pass_first + ngp + 1;
    unsigned long long* gp_col = rem_first + ngp + 1;

    hipStream_t st = (hipStream_t)stream;
    // control block (queue counter, validation flag), photon ranges, column offsets
    hipLaunchKernelGGL(fill_u64_kernel, dim3(1), dim3(32), 0, st, (unsigned long long*)L->ws, kCtrlBytes / 8, 0ull);
    HIP_TRY(hipGetLastError());
    BatchInit bi;
    memset(&bi, 0, sizeof bi);
    for (int n = 0; n < ngp; ++n) bi.photons[n] = photons[n];
    bi.seed = seed;
    bi.ncol = s.ncol;
    bi.ngp = ngp;
    hipLaunchKernelGGL(batch_init_kernel, dim3(1), dim3(256), 0, st, bi, pass_first, rem_first, gp_col);
    HIP_TRY(hipGetLastError());

    TraceParams& P = L->P;
    memset(&P, 0, sizeof P);
    P.cells = L->cells;
    P.gas = L->gas;
    P.albedo = albedo;
    P.majorant = L->maj;
    P.cell_mask = (o.flags & RT3D_FLAG_CELL_MASK) ? L->mask : nullptr;
    P.mask_words = factored ? mask_words_of(s) : 0;
    schedule_of(s, ngp, photons, o, pass_first, rem_first, gp_col, &P.sched);
    P.abs_dir = (unsigned long long*)out->abs_dir;
    P.abs_dif = (unsigned long long*)out->abs_dif;
    P.sfc_dir = (unsigned long long*)out->sfc_dir;
    P.sfc_dif = (unsigned long long*)out->sfc_dif;
    P.sfc_abs = (unsigned long long*)out->sfc_abs;
    P.toa_up = (unsigned long long*)out->toa_up;
    P.ledger = (unsigned long long*)out->ledger;
    P.stats = (unsigned long long*)out->stats;
    P.queue = (unsigned long long*)L->ws;
    P.ngp = ngp;
    P.nmaj = (int)s.nmaj;
    P.nx = s.nx; P.ny = s.ny; P.nz = s.nz;
    P.bx = s.bx; P.by = s.by; P.bz = s.bz;
    P.mx = s.mx; P.my = s.my; P.mz = s.mz;
    P.dx = grid->dx; P.dy = grid->dy; P.dz = grid->dz;
    P.inv_dx = 1.0f / grid->dx; P.inv_dy = 1.0f / grid->dy; P.inv_dz = 1.0f / grid->dz;
    P.cx = (float)s.bx * grid->dx; P.cy = (float)s.by * grid->dy; P.cz = (float)s.bz * grid->dz;
    P.H = (float)s.nz * grid->dz;
    const double th = sza_deg * M_PI / 180.0, ph = azimuth_deg * M_PI / 180.0;
    P.sun_x = (float)(-sin(th) * sin(ph));
    P.sun_y = (float)(-sin(th) * cos(ph));
    P.sun_z = (float)(-cos(th));
    P.diffuse_fraction = o.diffuse_fraction;
    P.rr_below = (uint32_t)std::nearbyint((double)o.rr_threshold * 2147483648.0);
    P.max_iters = o.max_iters;
    P.pool = o.pool_photons > 0 ? (uint32_t)o.pool_photons : 256u;
    P.refill = o.refill_lanes > 0 ? (uint32_t)o.refill_lanes : 16u;
    P.merge = (o.flags & RT3D_FLAG_NO_MERGE) ? 0 : 1;
    P.wave_agg = (o.flags & RT3D_FLAG_WAVE_AGGREGATE) ? 1 : 0;
    P.sobol = (o.flags & RT3D_FLAG_SOBOL_ENTRY) ? 1 : 0;
    P.seed = seed;
    P.photons = total;
    P.photon_offset = o.photon_offset;
    P.ncol = s.ncol;
    return RT3D_OK;
}

rt3d_status validated(const Launch& L, hipStream_t st) {
    HIP_TRY(hipGetLastError());
    uint32_t h = 0;
    HIP_TRY(hipMemcpyAsync(&h, L.flag, sizeof h, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return h ? RT3D_EDOMAIN : RT3D_OK;
}

rt3d_status clear_outputs(const Launch& L, const rt3d_tallies* out, hipStream_t st) {
    if (L.o.flags & RT3D_FLAG_ACCUMULATE) return RT3D_OK;
    rt3d_status z;
    if ((z = zero_u64((unsigned long long*)out->abs_dir, L.s.ncell, st)) != RT3D_OK) return z;
    if ((z = zero_u64((unsigned long long*)out->abs_dif, L.s.ncell, st)) != RT3D_OK) return z;
    if ((z = zero_u64((unsigned long long*)out->sfc_dir, L.s.ncol, st)) != RT3D_OK) return z;
    if ((z = zero_u64((unsigned long long*)out->sfc_dif, L.s.ncol, st)) != RT3D_OK) return z;
    if ((z = zero_u64((unsigned long long*)out->sfc_abs, L.s.ncol, st)) != RT3D_OK) return z;
    if ((z = zero_u64((unsigned long long*)out->toa_up, L.s.ncol, st)) != RT3D_OK) return z;
    if ((z = zero_u64((unsigned long long*)out->ledger, RT3D_LEDGER_N, st)) != RT3D_OK) return z;
    return zero_u64((unsigned long long*)out->stats, RT3D_STATS_N, st);
}

rt3d_status launch_trace(Launch& L, bool factored, hipStream_t st) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    int max_lds = 0;
    HIP_TRY(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    const size_t maj_bytes = L.s.nmaj * sizeof(float);
    const size_t lds_limit = L.o.lds_majorant > 0 ? (size_t)max_lds - 1024 : kLdsMajorantBytes;
    const bool use_lds =
        L.ngp == 1 && L.o.lds_majorant >= 0 && maj_bytes <= lds_limit && maj_bytes + 1024 <= (size_t)max_lds;
    const size_t lds = use_lds ? maj_bytes : 0;
    // crossings per loop iteration: a short walk keeps the lanes of a wave
    // in step (a long clear-sky walk of one lane would hold the others)
    L.P.max_walk = L.o.max_walk > 0 ? L.o.max_walk : (use_lds ? 3 : 2);
    auto kernel = factored ? (use_lds ? trace_kernel<true, true> : trace_kernel<false, true>)
                           : (use_lds ? trace_kernel<true, false> : trace_kernel<false, false>);
    int ncu = 0;
    HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    const int threads = factored ? Shape_<true>::threads : Shape_<false>::threads;
    int per_cu = 0;
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, lds));
    if (per_cu < 1) per_cu = 1;
    unsigned blocks = L.o.grid_blocks ? (unsigned)L.o.grid_blocks : (unsigned)(ncu * per_cu);
    // never more lanes than photons need
    const unsigned long long max_blocks = (L.total + threads - 1) / threads;
    if (blocks > max_blocks) blocks = (unsigned)max_blocks;
    if (blocks < 1) blocks = 1;
    if (L.o.flags & RT3D_FLAG_TIME) {
        if (!g_t0) HIP_TRY(hipEventCreate(&g_t0));
        if (!g_t1) HIP_TRY(hipEventCreate(&g_t1));
        HIP_TRY(hipEventRecord(g_t0, st));
    }
    hipLaunchKernelGGL(kernel, dim3(blocks), dim3(threads), lds, st, L.P);
    HIP_TRY(hipGetLastError());
    if (L.o.flags & RT3D_FLAG_TIME) {
        HIP_TRY(hipEventRecord(g_t1, st));
        g_timed = true;
    }
    hipLaunchKernelGGL(clear_atm_kernel, dim3(1), dim3(64), 0, st, L.P.ledger);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(ledger_atm_kernel, dim3(grid_for(L.s.ncell, 256, 2048)), dim3(256), 0, st, L.P.abs_dir,
                       L.P.abs_dif, L.s.ncell, L.P.ledger);
    HIP_TRY(hipGetLastError());
    return RT3D_OK;
}

// Scratch of rt3d_trace_noalloc: the workspace of rt3d_trace (control
// block, photon ranges, majorant grid, packed cell records) in a file-scope
// device array instead of a caller buffer.  Every device the library runs on
// holds its own copy for the life of the process.  In host code the array's
// name is not a device address; its address on each device comes from
// hipGetSymbolAddress (scratch_address) and only that address is used.
static __device__ __align__(256) unsigned char scratch[RT3D_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device.
rt3d_status scratch_address(void** out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) {
        snprintf(g_err, sizeof g_err, "rt3d_trace_noalloc: device %d beyond the %d it keeps scratch for", dev,
                 kMaxDevices);
        return RT3D_EDEVICE;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p || ((uintptr_t)p & 255)) {
            snprintf(g_err, sizeof g_err, "rt3d_trace_noalloc: bad scratch address on device %d", dev);
            return RT3D_EDEVICE;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return RT3D_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

int rt3d_abi_version(void) { return RT3D_ABI_VERSION; }

const char* rt3d_status_string(rt3d_status s) {
    switch (s) {
        case RT3D_OK: return "ok";
        case RT3D_EINVAL: return "invalid argument";
        case RT3D_EDOMAIN: return "field value out of range";
        case RT3D_EDEVICE: return "HIP device error";
        case RT3D_ETOOBIG: return "problem larger than the static scratch of rt3d_trace_noalloc";
    }
    return "unknown status";
}

const char* rt3d_last_device_error(void) { return g_err; }

void rt3d_default_options(rt3d_options* opt) {
    if (!opt) return;
    memset(opt, 0, sizeof *opt);
    opt->diffuse_fraction = 0.0f;
    opt->rr_threshold = 0.5f;
    opt->max_iters = 1u << 24;
}

size_t rt3d_workspace_size(const rt3d_grid* grid, const rt3d_options* opt) {
    rt3d_options o;
    if (!grid_ok(grid)) return 0;
    resolve_options(grid, opt, &o);
    Shape s;
    if (!shape_of(grid, &o, &s)) return 0;
    return layout_of(s, 1, false).total;
}

size_t rt3d_workspace_size_batched(const rt3d_grid* grid, int32_t n_gpoints, const rt3d_options* opt) {
    rt3d_options o;
    if (!grid_ok(grid) || n_gpoints < 1 || n_gpoints > kMaxGpoints) return 0;
    resolve_options(grid, opt, &o);
    Shape s;
    if (!shape_of(grid, &o, &s)) return 0;
    return layout_of(s, n_gpoints, true).total;
}

rt3d_status rt3d_majorant_build(const rt3d_grid* grid, const float* k_ext, int32_t bx, int32_t by, int32_t bz,
                                float* majorant, void* stream) {
    rt3d_options o;
    rt3d_default_options(&o);
    o.brick_x = bx; o.brick_y = by; o.brick_z = bz;
    Shape s;
    if (!k_ext || !majorant || bx <= 0 || by <= 0 || bz <= 0 || !shape_of(grid, &o, &s)) return RT3D_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(fill_u32_kernel, dim3(grid_for(s.nmaj)), dim3(256), 0, st, (uint32_t*)majorant, s.nmaj, 0u);
    HIP_TRY(hipGetLastError());
    const size_t n = (size_t)s.mx * s.ny * s.nz;
    hipLaunchKernelGGL(majorant_kernel, dim3(grid_for(n, 256, 16384)), dim3(256), 0, st, k_ext,
                       (uint32_t*)majorant, s.nx, s.ny, s.nz, s.bx, s.by, s.bz);
    HIP_TRY(hipGetLastError());
    return RT3D_OK;
}

rt3d_status rt3d_trace(const rt3d_grid* grid, const rt3d_optical_props* props, const float* surface_albedo,
                       double sza_deg, double azimuth_deg, uint64_t photons, uint64_t seed,
                       const rt3d_options* opt, const rt3d_tallies* out, void* workspace, size_t workspace_bytes,
                       void* stream) {
    g_timed = false;
    if (!props || !props->k_ext || !props->k_ext_cloud || !props->ssa || !props->g) return RT3D_EINVAL;
    Launch L;
    rt3d_status st = prepare(grid, 1, &photons, surface_albedo, sza_deg, azimuth_deg, seed, opt, out, workspace,
                             workspace_bytes, stream, false, &L);
    if (st != RT3D_OK) return st;
    hipStream_t hs = (hipStream_t)stream;
    if (L.o.flags & RT3D_FLAG_VALIDATE) {
        hipLaunchKernelGGL(validate_kernel, dim3(grid_for(L.s.ncell, 256, 4096)), dim3(256), 0, hs, props->k_ext,
                           props->k_ext_cloud, props->ssa, props->g, surface_albedo, L.s.ncell, L.s.ncol, L.flag);
        if ((st = validated(L, hs)) != RT3D_OK) return st;
    }
    if ((st = clear_outputs(L, out, hs)) != RT3D_OK) return st;
    if ((st = rt3d_majorant_build(grid, props->k_ext, L.s.bx, L.s.by, L.s.bz, L.maj, stream)) != RT3D_OK) return st;
    hipLaunchKernelGGL(pack_cells_kernel, dim3(grid_for(L.s.ncell, 256, 16384)), dim3(256), 0, hs, props->k_ext,
                       props->ssa, props->k_ext_cloud, props->g, L.cells, L.s.ncell);
    HIP_TRY(hipGetLastError());
    return launch_trace(L, false, hs);
}

rt3d_status rt3d_trace_noalloc(const rt3d_grid* grid, const rt3d_optical_props* props, const float* surface_albedo,
                               double sza_deg, double azimuth_deg, uint64_t photons, uint64_t seed,
                               const rt3d_options* opt, const rt3d_tallies* out, void* stream) {
    g_timed = false;
    // timing would create HIP events on first use
    if (opt && (opt->flags & RT3D_FLAG_TIME)) return RT3D_EINVAL;
    const size_t need = rt3d_workspace_size(grid, opt);
    if (need == 0) return RT3D_EINVAL;
    if (need > RT3D_NOALLOC_SCRATCH_BYTES) {
        snprintf(g_err, sizeof g_err,
                 "rt3d_trace_noalloc: this grid needs %zu bytes of scratch, more than its %zu", need,
                 (size_t)RT3D_NOALLOC_SCRATCH_BYTES);
        return RT3D_ETOOBIG;
    }
    void* ws = nullptr;
    const rt3d_status st = scratch_address(&ws);
    if (st != RT3D_OK) return st;
    return rt3d_trace(grid, props, surface_albedo, sza_deg, azimuth_deg, photons, seed, opt, out, ws,
                      RT3D_NOALLOC_SCRATCH_BYTES, stream);
}

rt3d_status rt3d_trace_batched(const rt3d_grid* grid, int32_t n_gpoints, const rt3d_batched_medium* medium,
                               const uint64_t* photons, const float* surface_albedo, double sza_deg,
                               double azimuth_deg, uint64_t seed, const rt3d_options* opt, const rt3d_tallies* out,
                               void* workspace, size_t workspace_bytes, void* stream) {
    g_timed = false;
    if (!medium || !medium->k_gas || !medium->ssa_gas || !medium->k_cloud || !medium->ssa_cloud ||
        !medium->g_cloud || !photons)
        return RT3D_EINVAL;
    if (n_gpoints < 1 || n_gpoints > kMaxGpoints) return RT3D_EINVAL;
    if (opt && opt->photon_offset != 0) return RT3D_EINVAL;
    Launch L;
    rt3d_status st = prepare(grid, n_gpoints, photons, surface_albedo, sza_deg, azimuth_deg, seed, opt, out,
                             workspace, workspace_bytes, stream, true, &L);
    if (st != RT3D_OK) return st;
    L.P.gp_diffuse = medium->diffuse_fraction;
    hipStream_t hs = (hipStream_t)stream;
    if (L.o.flags & RT3D_FLAG_VALIDATE) {
        hipLaunchKernelGGL(validate_batched_kernel, dim3(grid_for(L.s.ncell, 256, 4096)), dim3(256), 0, hs,
                           medium->k_gas, medium->ssa_gas, (size_t)n_gpoints * L.s.nz, medium->k_cloud,
                           medium->ssa_cloud, medium->g_cloud, surface_albedo, L.s.ncell, L.s.ncol,
                           medium->diffuse_fraction, n_gpoints, L.flag);
        if ((st = validated(L, hs)) != RT3D_OK) return st;
    }
    if ((st = clear_outputs(L, out, hs)) != RT3D_OK) return st;
    const size_t ngas = (size_t)n_gpoints * L.s.nz;
    hipLaunchKernelGGL(pack_cloud_kernel, dim3(grid_for(L.s.ncell, 256, 16384)), dim3(256), 0, hs, medium->k_cloud,
                       medium->ssa_cloud, medium->g_cloud, L.cells, L.s.ncell);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(pack_gas_kernel, dim3(grid_for(ngas)), dim3(256), 0, hs, medium->k_gas, medium->ssa_gas,
                       L.gas, ngas);
    HIP_TRY(hipGetLastError());
    const size_t nmask = L.P.cell_mask ? L.s.nmaj * (size_t)L.P.mask_words : 0;
    if (nmask) hipLaunchKernelGGL(cell_mask_kernel, dim3(grid_for(nmask, 256, 16384)), dim3(256), 0, hs, medium->k_cloud, L.mask,
                       L.s.nx, L.s.ny, L.s.bx, L.s.by, L.s.bz, L.s.mx, L.s.my, L.P.mask_words, nmask);
    HIP_TRY(hipGetLastError());
    const size_t nlayer = (size_t)L.s.nz * L.s.my * L.s.mx;
    hipLaunchKernelGGL(fill_u32_kernel, dim3(grid_for(nlayer)), dim3(256), 0, hs, L.layer, nlayer, 0u);
    HIP_TRY(hipGetLastError());
    const size_t nrow = (size_t)L.s.mx * L.s.ny * L.s.nz;
    hipLaunchKernelGGL(layer_max_kernel, dim3(grid_for(nrow, 256, 16384)), dim3(256), 0, hs, L.cells, L.layer,
                       L.s.nx, L.s.ny, L.s.nz, L.s.bx, L.s.by);
    HIP_TRY(hipGetLastError());
    const size_t nm = L.s.nmaj * (size_t)n_gpoints;
    hipLaunchKernelGGL(gas_majorant_kernel, dim3(grid_for(nm, 256, 16384)), dim3(256), 0, hs, L.layer, L.gas,
                       L.maj, n_gpoints, L.s.nz, L.s.mx, L.s.my, L.s.bz);
    HIP_TRY(hipGetLastError());
    return launch_trace(L, true, hs);
}

rt3d_status rt3d_last_trace_ms(float* ms) {
    if (!ms || !g_timed) return RT3D_EINVAL;
    HIP_TRY(hipEventSynchronize(g_t1));
    HIP_TRY(hipEventElapsedTime(ms, g_t0, g_t1));
    return RT3D_OK;
}

rt3d_status rt3d_finalize(const rt3d_grid* grid, const rt3d_tallies* raw, uint64_t photons,
                          const double* layer_scale, double flux_scale, float* abs_dir, float* abs_dif,
                          float* sfc_dir, float* sfc_dif, float* sfc_abs, float* toa_up, void* stream) {
    if (!grid_ok(grid) || !raw || photons == 0 || !std::isfinite(flux_scale)) return RT3D_EINVAL;
    const size_t ncell = (size_t)grid->nx * grid->ny * grid->nz, ncol = (size_t)grid->nx * grid->ny;
    const double norm = (double)ncol / ((double)photons * 2147483648.0);
    hipStream_t st = (hipStream_t)stream;
    struct Item { const uint64_t* src; float* dst; size_t n; bool three; };
    const Item items[6] = {{raw->abs_dir, abs_dir, ncell, true}, {raw->abs_dif, abs_dif, ncell, true},
                           {raw->sfc_dir, sfc_dir, ncol, false}, {raw->sfc_dif, sfc_dif, ncol, false},
                           {raw->sfc_abs, sfc_abs, ncol, false}, {raw->toa_up, toa_up, ncol, false}};
    for (const Item& it : items) {
        if (!it.dst) continue;
        if (!it.src) return RT3D_EINVAL;
        hipLaunchKernelGGL(finalize3_kernel, dim3(grid_for(it.n, 256, 8192)), dim3(256), 0, st,
                           (const unsigned long long*)it.src, it.dst, it.three ? ncol : it.n, it.n,
                           it.three ? norm : norm * flux_scale, it.three ? layer_scale : nullptr);
        HIP_TRY(hipGetLastError());
    }
    return RT3D_OK;
}

rt3d_status rt3d_philox4x32_10(const uint32_t* ctr, uint64_t seed, uint32_t* out, uint32_t n, void* stream) {
    if (!ctr || !out) return RT3D_EINVAL;
    if (n == 0) return RT3D_OK;
    hipLaunchKernelGGL(philox_kernel, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream,
                       (const uint4*)ctr, (uint32_t)seed, (uint32_t)(seed >> 32), (uint4*)out, n);
    HIP_TRY(hipGetLastError());
    return RT3D_OK;
}

rt3d_status rt3d_sobol_entry(uint64_t first_pass, uint32_t n, uint64_t column, uint64_t seed, uint32_t* out,
                             void* stream) {
    if (!out) return RT3D_EINVAL;
    if (n == 0) return RT3D_OK;
    hipLaunchKernelGGL(sobol_entry_kernel, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream,
                       (unsigned long long)first_pass, n, (unsigned long long)column, (uint32_t)seed,
                       (uint32_t)(seed >> 32), (uint2*)out);
    HIP_TRY(hipGetLastError());
    return RT3D_OK;
}

rt3d_status rt3d_phase_sample(int32_t kind, const float* g, const float* xi, float* mu, uint32_t n, void* stream) {
    if ((kind != 0 && kind != 1) || !xi || !mu || (kind == 0 && !g)) return RT3D_EINVAL;
    if (n == 0) return RT3D_OK;
    hipLaunchKernelGGL(phase_sample_kernel, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, (int)kind, g,
                       xi, mu, n);
    HIP_TRY(hipGetLastError());
    return RT3D_OK;
}

rt3d_status rt3d_turn(const float* dir_in, const float* mu, const float* t, float* dir_out, uint32_t n, void* stream) {
    if (!dir_in || !mu || !t || !dir_out) return RT3D_EINVAL;
    if (n == 0) return RT3D_OK;
    hipLaunchKernelGGL(turn_kernel, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, dir_in, mu, t, dir_out,
                       n);
    HIP_TRY(hipGetLastError());
    return RT3D_OK;
}

rt3d_status rt3d_schedule_slots(const rt3d_grid* grid, int32_t n_gpoints, const uint64_t* photons,
                                const uint64_t* col_offset, const rt3d_options* opt, uint64_t first_slot, uint64_t n,
                                int32_t* gp_out, uint64_t* id_out, uint32_t* col_out) {
    if (!grid_ok(grid) || n_gpoints < 1 || n_gpoints > kMaxGpoints || !photons || !col_offset) return RT3D_EINVAL;
    rt3d_options o;
    resolve_options(grid, opt, &o);
    Shape s;
    if (!shape_of(grid, &o, &s)) return RT3D_EINVAL;
    if (o.tile_x < 0 || o.tile_y < 0 || (o.tile_x && s.nx % o.tile_x) || (o.tile_y && s.ny % o.tile_y))
        return RT3D_EINVAL;
    unsigned long long total = 0;
    for (int i = 0; i < n_gpoints; ++i) {
        if (col_offset[i] >= s.ncol || total + photons[i] < total) return RT3D_EINVAL;
        total += photons[i];
    }
    if (first_slot > total || n > total - first_slot || (n && (!gp_out || !id_out || !col_out))) return RT3D_EINVAL;
    unsigned long long pass_first[kMaxGpoints + 1], rem_first[kMaxGpoints + 1], offs[kMaxGpoints];
    schedule_tables(photons, n_gpoints, s.ncol, pass_first, rem_first);
    for (int i = 0; i < n_gpoints; ++i) offs[i] = col_offset[i];
    Schedule S;
    schedule_of(s, n_gpoints, photons, o, pass_first, rem_first, offs, &S);
    for (uint64_t i = 0; i < n; ++i) {
        const Slot sl = decode_slot(S, first_slot + i);
        gp_out[i] = sl.gp;
        id_out[i] = sl.id;
        col_out[i] = sl.col;
    }
    return RT3D_OK;
}

}  // extern "C"
