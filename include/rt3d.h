/*
 * rt3d.h -- C ABI of the MI355X Monte Carlo solar photon tracer.
 *
 * The library traces solar photon packets through a 3D grid of gas and cloud
 * optical properties and returns per-cell absorption (heating) and
 * direct/diffuse surface irradiance tallies.  The method is the forward
 * Monte Carlo ray tracer of Veerman, van Stratum and van Heerwaarden,
 * "Shallow cumulus convection over land in cloud-resolving simulations with
 * a coupled ray tracer" (GRL 2022), section 2.3 "The ray tracer":
 *   - inputs: 3D fields of total extinction k_ext, cloud extinction
 *     k_ext,cloud, single-scattering albedo omega0 and asymmetry g (sec. 2.3,
 *     the paragraph on required inputs);
 *   - photons enter at the top of the domain (TOD) along the solar beam or,
 *     with probability equal to the diffuse fraction, isotropically
 *     downwards, at positions from independent uniforms or a scrambled
 *     Sobol sequence; the TOD flux and diffuse fraction come from a
 *     clear-sky two-stream column (sec. 2.3, initialisation paragraph;
 *     RT3D_FLAG_SOBOL_ENTRY, rt3d_two_stream);
 *   - null-collision tracking on a one-level coarse acceleration grid whose
 *     cells hold the maximum fine-cell extinction (sec. 2.3, acceleration
 *     grid paragraph);
 *   - Rayleigh scattering by gas, Henyey-Greenstein scattering (no delta
 *     scaling) by cloud droplets, cloud chosen with probability
 *     k_ext,cloud / k_ext (sec. 2.3, phase-function paragraph);
 *   - absorption by weights at every scattering or null-collision event,
 *     the removed weight stored as heating; Russian roulette below weight
 *     0.5; Lambertian surface whose albedo scales the weight (sec. 2.3,
 *     weights paragraph);
 *   - surface and TOD fluxes are the summed weights of photons reaching the
 *     surface or leaving the top; "direct" means never scattered (sec. 2.3
 *     and sec. 3.3.1, definition of direct radiation).
 *
 * Every entry point is `extern "C"`, takes plain pointers and sizes, and
 * reports errors only through `rt3d_status`.  Unless stated otherwise a
 * pointer argument is a DEVICE pointer owned by the caller; the library
 * never allocates or frees device memory (its one static device array, the
 * scratch of rt3d_trace_noalloc, is part of the loaded code).  `stream` is a hipStream_t passed
 * as `void*` (NULL = the null stream).  All work is enqueued asynchronously
 * on `stream`; results are valid once that stream has completed.  Host-side
 * argument checks run before anything is enqueued, so a call that returns an
 * error has launched nothing (except RT3D_EDOMAIN, see RT3D_FLAG_VALIDATE).
 *
 * ---------------------------------------------------------------------------
 * Conventions
 * ---------------------------------------------------------------------------
 * Grid: nx x ny x nz cells of size dx x dy x dz metres.  x points east, y
 * north, z up; the domain is [0, nx*dx) x [0, ny*dy) x [0, nz*dz] with
 * periodic x and y boundaries, an open top at z = H = nz*dz (a photon moving
 * up through it escapes for good) and the surface at z = 0.
 * 3D arrays are [nz][ny][nx] with x fastest (cell (i,j,k) at
 * (k*ny + j)*nx + i); 2D arrays are [ny][nx].
 *
 * Sun: zenith angle sza in [0, 90) degrees; azimuth measured clockwise from
 * north (+y), the direction the sun is seen in.  Photons travel along
 *   d0 = (-sin(sza) sin(az), -sin(sza) cos(az), -cos(sza)).
 *
 * Weights: a photon packet carries an integer weight in units of 2^-31 of
 * the initial weight (W1 = 2^31 = weight one).  Every tally and every entry
 * of the energy ledger is a uint64 sum of such integers, so tallies are
 * exact, independent of the order of atomic updates, bitwise reproducible,
 * and the energy budget closes exactly (see RT3D_LEDGER_*).
 *
 * Random numbers: Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC'11),
 * key = (seed & 0xffffffff, seed >> 32).  For photon index id (counted from
 * 0 over the whole run, so `photon_offset` + local index) with
 * id_lo/id_hi its 32-bit halves, counters are:
 *   run offset      (0, 0, 0xfffffffe, 0)        word 0 -> column offset o
 *   emission        (id_lo, id_hi, 0xffffffff, 0) words 0,1 -> x, y inside
 *                                                 the column, word 2 ->
 *                                                 diffuse/direct choice
 *   diffuse entry   (id_lo, id_hi, 0xffffffff, 1) words 0,1 -> mu^2, phi
 *   free path s     (id_lo, id_hi, s, 0)          word 0 -> optical depth,
 *                                                 word 1 -> event choice,
 *                                                 word 2 -> cos(theta) or
 *                                                 surface mu^2, word 3 -> phi
 *   roulette at s   (id_lo, id_hi, s, 1)          word 0 -> rho
 *   Sobol scramble  (c_lo, c_hi, 0xfffffffd, 0)   words 0,1 -> scramble
 *                                                 seeds of column c (x, y)
 * s counts the free paths of one photon from 0.  Photon id enters column
 * c = (id + o) mod (nx*ny), cell (c mod nx, c div nx) (systematic sampling:
 * every column receives floor or ceil of photons/(nx*ny) photons), as the
 * column's (id div (nx*ny))-th photon.
 */
#ifndef RT3D_H
#define RT3D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RT3D_ABI_VERSION 3

typedef enum {
    RT3D_OK = 0,
    RT3D_EINVAL = 1,  /* bad argument: null pointer, non-positive size, brick
                         not dividing the grid, sza outside [0,90), photons 0
                         or >= 2^33, workspace too small, too many cells */
    RT3D_EDOMAIN = 2, /* RT3D_FLAG_VALIDATE found a field value out of range */
    RT3D_EDEVICE = 3, /* a HIP runtime call failed; see rt3d_last_device_error */
    RT3D_ETOOBIG = 4  /* rt3d_trace_noalloc: the grid needs more scratch than
                         RT3D_NOALLOC_SCRATCH_BYTES (text in
                         rt3d_last_device_error); nothing launched */
} rt3d_status;

/* Uniform grid; every size positive, nx*ny*nz < 2^31. */
typedef struct {
    int32_t nx, ny, nz;
    float dx, dy, dz; /* metres */
} rt3d_grid;

/* Optical properties (sec. 2.3, required inputs), device pointers to FP32
 * [nz][ny][nx] arrays:
 *   k_ext        total extinction coefficient, m^-1, >= 0
 *   k_ext_cloud  cloud-droplet extinction, m^-1, 0 <= k_ext_cloud <= k_ext
 *   ssa          total single-scattering albedo omega0 in [0,1]
 *   g            Henyey-Greenstein asymmetry of the cloud droplets in [-1,1]
 *                (gas always scatters with the Rayleigh phase function)    */
typedef struct {
    const float* k_ext;
    const float* k_ext_cloud;
    const float* ssa;
    const float* g;
} rt3d_optical_props;

/* Raw tallies, caller-owned device buffers of uint64 in units of 2^-31 of a
 * photon's initial weight (see rt3d_finalize for physical units):
 *   abs_dir [nz][ny][nx]  weight absorbed in the cell while never scattered
 *   abs_dif [nz][ny][nx]  weight absorbed in the cell after scattering
 *   sfc_dir [ny][nx]      weight reaching the surface unscattered (direct)
 *   sfc_dif [ny][nx]      weight reaching the surface after scattering
 *   sfc_abs [ny][nx]      weight absorbed by the surface
 *   toa_up  [ny][nx]      weight leaving through the top of the domain
 *   ledger  [RT3D_LEDGER_N] energy ledger (below)
 *   stats   [RT3D_STATS_N]  event counters (below)                        */
typedef struct {
    uint64_t* abs_dir;
    uint64_t* abs_dif;
    uint64_t* sfc_dir;
    uint64_t* sfc_dif;
    uint64_t* sfc_abs;
    uint64_t* toa_up;
    uint64_t* ledger;
    uint64_t* stats;
} rt3d_tallies;

/* Energy ledger.  For every run the identity
 *   INCOMING + RR_GAIN == TOA + ATM_DIR + ATM_DIF + SFC + RR_LOSS + LOST
 * holds exactly in integers; ATM_DIR == sum(abs_dir), ATM_DIF ==
 * sum(abs_dif), SFC == sum(sfc_abs), TOA == sum(toa_up).                  */
enum {
    RT3D_LEDGER_INCOMING = 0, /* photons * 2^31 */
    RT3D_LEDGER_TOA = 1,
    RT3D_LEDGER_ATM_DIR = 2,
    RT3D_LEDGER_ATM_DIF = 3,
    RT3D_LEDGER_SFC = 4,
    RT3D_LEDGER_RR_GAIN = 5,  /* weight added by roulette survivors */
    RT3D_LEDGER_RR_LOSS = 6,  /* weight of photons ended by roulette */
    RT3D_LEDGER_LOST = 7,     /* weight of photons stopped by max_iters */
    RT3D_LEDGER_N = 8
};

/* Event counters.  A "photon event" (the throughput unit) is one tentative
 * collision or one surface interaction: STAT_EVENTS = COLLISIONS + SURFACE. */
enum {
    RT3D_STAT_PHOTONS = 0,
    RT3D_STAT_COLLISIONS = 1,   /* tentative (null + real) collisions */
    RT3D_STAT_NULL = 2,
    RT3D_STAT_SCAT_GAS = 3,
    RT3D_STAT_SCAT_CLOUD = 4,
    RT3D_STAT_SURFACE = 5,
    RT3D_STAT_ESCAPE = 6,
    RT3D_STAT_RR_KILL = 7,
    RT3D_STAT_RR_SURVIVE = 8,
    RT3D_STAT_CROSSINGS = 9,    /* acceleration-grid cell crossings */
    RT3D_STAT_ABSORBED = 10,    /* photons whose weight reached exactly 0 */
    RT3D_STAT_CAPPED = 11,      /* photons stopped by max_iters */
    RT3D_STATS_N = 12
};

/* Flags for rt3d_options.flags */
#define RT3D_FLAG_ACCUMULATE 0x1u /* add to the tallies instead of zeroing */
#define RT3D_FLAG_VALIDATE 0x2u   /* check the fields on the device first
                                     (synchronises the stream) */
#define RT3D_FLAG_TIME 0x4u       /* time the tracing kernel with HIP events;
                                     read with rt3d_last_trace_ms */
#define RT3D_FLAG_NO_MERGE 0x8u   /* one tally atomic per deposit instead of
                                     merging a lane's consecutive deposits
                                     into the same cell (same results) */
#define RT3D_FLAG_SOBOL_ENTRY 0x10u /* entry positions inside each column from
                                     a scrambled 2D Sobol sequence (sec. 2.3,
                                     initialisation paragraph) instead of
                                     independent uniforms; see
                                     rt3d_sobol_entry for the definition */
#define RT3D_FLAG_WAVE_AGGREGATE 0x20u /* wave-aggregated tally atomics: lanes of
                                     a wavefront that update the same tally
                                     element in the same instruction add
                                     their values first and one atomic is
                                     issued per distinct element (same
                                     results; speed only) */
#define RT3D_FLAG_CELL_MASK 0x40u /* rt3d_trace_batched: at a tentative
                                     collision in an acceleration cell with
                                     cloud, first read the fine cell's bit in
                                     a cloud-cell mask (built in the
                                     workspace) and skip the record gather
                                     for a cloud-free cell, instead of
                                     gathering at every one (same results;
                                     speed only) */

typedef struct {
    /* acceleration-grid cell ("brick") in fine cells; must divide nx, ny, nz */
    int32_t brick_x, brick_y, brick_z;
    float diffuse_fraction;  /* probability of an isotropic diffuse entry */
    float rr_threshold;      /* roulette below this weight (paper: 0.5); 0 = off */
    uint32_t flags;
    uint32_t max_iters;      /* per-photon cap on collisions + surface hits +
                                brick crossings; the rest of its weight goes to
                                RT3D_LEDGER_LOST.  0 = default (1<<24) */
    uint64_t photon_offset;  /* first photon id of this call (chunked runs) */
    int32_t grid_blocks;     /* persistent workgroups, 0 = automatic */
    int32_t block_threads;   /* threads per workgroup, 0 = automatic */
    int32_t lds_majorant;    /* stage the majorant grid in LDS: 0 = automatic,
                                1 = when it fits, -1 = never */
    int32_t max_walk;        /* acceleration-grid crossings a lane makes per
                                loop iteration before the wave re-converges;
                                0 = automatic (3 with LDS majorants, else 2) */
    int32_t pool_photons;    /* photon ids a wave takes from the work queue
                                at a time, 0 = 256, else >= 64 (one grab
                                must cover every lane of a wave);
                                1..63 and negative values: RT3D_EINVAL */
    int32_t refill_lanes;    /* a wave starts new photons once at least this
                                many of its 64 lanes are idle (or none is
                                alive), 1..64; 0 = 16 */
    int32_t tile_x, tile_y;  /* entry tile of the photon schedule in columns
                                (see rt3d_schedule_slots): the work queue
                                hands out the photons of all full passes
                                tile by tile, so the photons in flight at one
                                time enter a few neighbouring tiles; each must
                                divide nx (ny).  0 = automatic: tiles whose
                                columns hold about 128 MiB of cell records and
                                heating tallies (nz * 32 bytes per column),
                                close to square (edges: divisors of nx, ny),
                                or the whole domain when it holds less.  Order
                                only: results do not depend on it. */
} rt3d_options;

/* Several g-points in one launch (sec. 2.2: 112 shortwave quadrature points;
 * sec. 2.3: each traced independently).  Factored medium: the gas of each
 * g-point is horizontally uniform, the cloud field is shared by all
 * g-points.  For g-point n and cell (i,j,k) the optical properties are
 *   k_ext = k_gas[n][k] + k_cloud[k][j][i],  k_ext,cloud = k_cloud[k][j][i],
 *   omega0 k_ext = ssa_gas[n][k] k_gas[n][k] + ssa_cloud[k][j][i] k_cloud,
 *   g = g_cloud[k][j][i] (gas scatters with the Rayleigh phase function).
 * Device FP32 pointers; k_gas, ssa_gas are [n_gpoints][nz]; the cloud
 * fields are [nz][ny][nx].                                                 */
typedef struct {
    const float* k_gas;
    const float* ssa_gas;
    const float* k_cloud;
    const float* ssa_cloud;
    const float* g_cloud;
    /* diffuse fraction of the TOD flux of each g-point, device FP32
     * [n_gpoints] in [0,1] (e.g. from rt3d_two_stream); NULL = every g-point
     * uses opt->diffuse_fraction */
    const float* diffuse_fraction;
} rt3d_batched_medium;

#define RT3D_MAX_GPOINTS 256

/* ---------------------------------------------------------------------- */

/* ABI version (RT3D_ABI_VERSION). */
int rt3d_abi_version(void);

/* Static description of a status code; never NULL. */
const char* rt3d_status_string(rt3d_status s);

/* Text of the last HIP error seen by the calling thread ("" if none). */
const char* rt3d_last_device_error(void);

/* Fill *opt with defaults: brick 8x8x8 clamped to the grid by the trace call
 * when 0, diffuse_fraction 0, rr_threshold 0.5, no flags, max_iters 1<<24,
 * photon_offset 0, automatic launch shape.  Host pointer. */
void rt3d_default_options(rt3d_options* opt);

/* Bytes of device workspace rt3d_trace needs for this grid and options
 * (majorant grid, work-queue counter and flags).  Returns 0 on bad input. */
size_t rt3d_workspace_size(const rt3d_grid* grid, const rt3d_options* opt);

/* Acceleration grid (sec. 2.3, acceleration grid paragraph): majorant[b] =
 * max of k_ext over the fine cells of brick b, exactly (FP32 max).
 * majorant: device FP32 [nz/bz][ny/by][nx/bx].  k_ext must be >= 0. */
rt3d_status rt3d_majorant_build(const rt3d_grid* grid, const float* k_ext,
                                int32_t bx, int32_t by, int32_t bz,
                                float* majorant, void* stream);

/* Trace `photons` photon packets (sec. 2.3) entering the top of the domain
 * (1 <= photons < 2^33 per call, so that photons * 2^31 fits the uint64
 * ledger; larger runs are several calls with ACCUMULATE)
 * with the sun at (sza_deg, azimuth_deg) and write raw tallies to `out`
 * (zeroed first unless RT3D_FLAG_ACCUMULATE).  surface_albedo: device FP32
 * [ny][nx] in [0,1].  seed: Philox key.  opt: host pointer or NULL for
 * defaults.  workspace: device buffer of at least rt3d_workspace_size bytes,
 * 256-byte aligned; its contents need not be initialised.  Same inputs and
 * seed give bitwise-identical tallies; calls over disjoint photon_offset
 * ranges with ACCUMULATE sum to exactly the single-call result. */
rt3d_status rt3d_trace(const rt3d_grid* grid, const rt3d_optical_props* props,
                       const float* surface_albedo, double sza_deg,
                       double azimuth_deg, uint64_t photons, uint64_t seed,
                       const rt3d_options* opt, const rt3d_tallies* out,
                       void* workspace, size_t workspace_bytes, void* stream);

/* Bytes of static device scratch behind rt3d_trace_noalloc (32 MiB: the
 * rt3d_trace workspace of grids up to about 2 million cells). */
#define RT3D_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)

/* rt3d_trace for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same arguments, results and errors as rt3d_trace, but the workspace is a
 * static device array of RT3D_NOALLOC_SCRATCH_BYTES held by the library on
 * every device it runs on until the process ends; the caller passes only
 * inputs and outputs.  The call allocates nothing (no hipMalloc, no events):
 * RT3D_FLAG_TIME is rejected with RT3D_EINVAL, a grid whose
 * rt3d_workspace_size exceeds the scratch with RT3D_ETOOBIG.  The device is
 * the current one; its scratch address is looked up on the first call there
 * (RT3D_EDEVICE if that fails).  All calls on one device share its scratch
 * and every call re-initialises what it reads, so sequential calls are
 * independent; calls that overlap on one device (two streams, two threads)
 * race and give undefined tallies. */
rt3d_status rt3d_trace_noalloc(const rt3d_grid* grid, const rt3d_optical_props* props,
                               const float* surface_albedo, double sza_deg,
                               double azimuth_deg, uint64_t photons, uint64_t seed,
                               const rt3d_options* opt, const rt3d_tallies* out, void* stream);

/* Bytes of device workspace rt3d_trace_batched needs (per-g-point majorant
 * grids, packed cloud records, gas tables).  Returns 0 on bad input. */
size_t rt3d_workspace_size_batched(const rt3d_grid* grid, int32_t n_gpoints, const rt3d_options* opt);

/* Trace n_gpoints g-points (1 <= n_gpoints <= RT3D_MAX_GPOINTS) of the
 * factored medium in ONE persistent launch and write broadband raw tallies
 * (the sum over g-points) to `out`.  photons: HOST array [n_gpoints] of photon
 * counts (zeros allowed, 0 < total < 2^33); g-point n is traced exactly as
 * rt3d_trace would trace its fields with photons[n] photons and Philox key
 * seed + n, so with photon counts proportional to the g-points' shares of
 * the TOD flux every photon carries the same energy and the broadband tally
 * normalised by the total photon count is the flux-weighted sum.  Each
 * g-point has its own majorant grid (max over its fine cells of k_gas +
 * k_cloud).  opt->photon_offset must be 0.  Other arguments and errors as
 * rt3d_trace; RT3D_FLAG_VALIDATE checks every input range. */
rt3d_status rt3d_trace_batched(const rt3d_grid* grid, int32_t n_gpoints, const rt3d_batched_medium* medium,
                               const uint64_t* photons, const float* surface_albedo, double sza_deg,
                               double azimuth_deg, uint64_t seed, const rt3d_options* opt,
                               const rt3d_tallies* out, void* workspace, size_t workspace_bytes, void* stream);

/* Milliseconds spent in the tracing kernel of the last rt3d_trace or
 * rt3d_trace_batched call made with RT3D_FLAG_TIME on this thread (waits for
 * it to finish).  Host *ms. */
rt3d_status rt3d_last_trace_ms(float* ms);

/* Normalise raw tallies (sec. 2.3: fluxes are mean weights; heating is the
 * absorbed weight) for a run of `photons` photons: every tally is divided by
 * (photons / (nx*ny)) * 2^31, giving fractions of the downward flux at the
 * top of the domain per column area.  3D outputs are then multiplied by
 * layer_scale[k] (FP64 device [nz], NULL = 1), 2D outputs by flux_scale; e.g.
 * layer_scale = F_TOD*86400/(rho_k*c_p*dz) turns absorption into heating
 * rates in K/day and flux_scale = F_TOD turns fluxes into W/m^2.  Any output
 * pointer may be NULL to skip it.  Outputs: FP32 device arrays shaped like
 * the matching raw tallies.  raw: the tallies written by rt3d_trace. */
rt3d_status rt3d_finalize(const rt3d_grid* grid, const rt3d_tallies* raw,
                          uint64_t photons, const double* layer_scale,
                          double flux_scale, float* abs_dir, float* abs_dif,
                          float* sfc_dir, float* sfc_dif, float* sfc_abs,
                          float* toa_up, void* stream);

/* Philox4x32-10 as used by the tracer, for bit-level tests: for each of n
 * counters ctr[4*i .. 4*i+3] (device uint32) write the four output words to
 * out[4*i .. 4*i+3] (device uint32), key = (seed lo, seed hi). */
rt3d_status rt3d_philox4x32_10(const uint32_t* ctr, uint64_t seed,
                               uint32_t* out, uint32_t n, void* stream);

/* Entry points of RT3D_FLAG_SOBOL_ENTRY (sec. 2.3, initialisation
 * paragraph: rays start at the top of the domain following a scrambled
 * Sobol sequence), for bit-level tests.  The p-th photon to enter column
 * `column` (p counted from 0, see the counter layout above) of a run with
 * Philox key `seed` starts at fractions (x, y) of the column's width, where
 * x, y are the 2D Sobol point p (dimension 1: bits of p reversed; dimension
 * 2: primitive polynomial x + 1, direction numbers v_1 = 2^31,
 * v_j = v_{j-1} xor (v_{j-1} >> 1), xor over the set bits of p), each under
 * Owen's nested uniform scramble: binary digit d (0 = most significant) is
 * flipped by the top bit of fmix32(node xor s), node = (first d digits) |
 * 2^d, fmix32 = MurmurHash3's finaliser, s = the column's scramble seed for
 * that coordinate.  For passes first_pass .. first_pass+n-1 writes the
 * 32-digit scrambled x, y to out[2*i], out[2*i+1] (device uint32); the tracer
 * uses their first 24 digits.  p is taken mod 2^32. */
rt3d_status rt3d_sobol_entry(uint64_t first_pass, uint32_t n, uint64_t column,
                             uint64_t seed, uint32_t* out, void* stream);

/* The photon schedule of a trace call, evaluated on the HOST (no device
 * work), for tests and inspection.  The work queue of rt3d_trace /
 * rt3d_trace_batched hands out slots 0 .. total-1 (total = sum of photons[]);
 * slot s is traced as photon id of g-point gp, entering column col (both
 * independent of the schedule: photon k of g-point n has id =
 * photon_offset + k and enters column (id + o_n) mod (nx*ny)).  With
 * P_n = photons[n] div (nx*ny), slots first cover the P_n full passes of
 * every g-point tile by tile (tiles of opt->tile_x x opt->tile_y columns,
 * row-major; inside a tile pass by pass, g-point by g-point, the tile's
 * columns row-major), then the photons left over, g-point by g-point in
 * order of k.  col_offset: o_n per g-point (host uint64 [n_gpoints]; the
 * tracer draws them from Philox, the hook takes any values in [0, nx*ny)).
 * For slots first_slot .. first_slot+n-1 writes gp_out[i], id_out[i],
 * col_out[i] (host arrays [n]).  RT3D_EINVAL for a bad grid or options, a
 * tile not dividing the grid, offsets out of range or slots beyond total. */
rt3d_status rt3d_schedule_slots(const rt3d_grid* grid, int32_t n_gpoints, const uint64_t* photons,
                                const uint64_t* col_offset, const rt3d_options* opt,
                                uint64_t first_slot, uint64_t n, int32_t* gp_out,
                                uint64_t* id_out, uint32_t* col_out);

/* The tracer's scattering samplers, element-wise, for tests (sec. 2.3,
 * phase-function paragraph).  kind 0: Henyey-Greenstein cosine of the
 * scattering angle by inversion of its distribution,
 *   mu = (1 + g^2 - s^2) / (2 g),  s = (1 - g^2) / (1 + g (2 xi - 1)),
 * evaluated for |g| < 0.1 in the multiplied-out form
 *   mu = (a + g (a^2+3)/2 + g^2 a + g^3 (a^2-1)/2) / (1 + g a)^2, a = 2 xi - 1
 * (the same function without its cancellation; mu = 2 xi - 1 at g = 0),
 * clamped to [-1, 1]; mu = 1 for g = 1.  kind 1: Rayleigh (phase function proportional to
 * 1 + mu^2), mu = u - 1/u with u = cbrt(q + sqrt(q^2 + 1)), q = 4 xi - 2
 * (g unused, may be NULL).  For i < n: mu[i] = sampler(g[i], xi[i]) with
 * xi in [0, 1).  DEVICE FP32 arrays [n]. */
rt3d_status rt3d_phase_sample(int32_t kind, const float* g, const float* xi, float* mu, uint32_t n, void* stream);

/* The tracer's change of direction at a scattering, element-wise, for
 * tests: unit direction dir_in[3i..3i+2] turned to polar cosine mu[i] about
 * itself and azimuth 2 pi t[i] (t in [0, 1)) into dir_out[3i..3i+2],
 * renormalised.  The azimuth's zero is fixed by the kernel's own frame; for
 * uniform t the result is uniform in azimuth.  DEVICE FP32 arrays. */
rt3d_status rt3d_turn(const float* dir_in, const float* mu, const float* t, float* dir_out, uint32_t n, void* stream);

/* Clear-sky two-stream column for the flux entering the top of the domain
 * (sec. 2.3, initialisation paragraph: the total incoming flux and its
 * diffuse fraction at the domain top come from a two-stream solution of a
 * clear-sky profile from the surface to the top of the atmosphere, so that
 * tracing can be confined to the domain).  Readings: practical improved
 * flux method coefficients (Zdunkowski, Welch and Korb 1980; Meador and
 * Weaver 1980, Table 1) gamma1 = (8 - w(5 + 3g))/4, gamma2 = 3w(1 - g)/4,
 * gamma3 = (2 - 3 mu0 g)/4, gamma4 = 1 - gamma3; homogeneous layers combined
 * by the adding method; Lambertian surface with one albedo; near the
 * resonance k mu0 = 1 (|1 - k^2 mu0^2| < 1e-3) the direct-beam terms of a
 * layer are the mean of their values at mu0 (1 -+ 1e-3).
 * n_cols independent columns (e.g. the g-points of a spectral set) of nlay
 * layers, layer 0 at the top of the atmosphere; all arrays DEVICE FP64:
 *   tau, ssa, g      [n_cols][nlay] optical depth, single-scattering albedo,
 *                    asymmetry parameter (0 for Rayleigh gas);
 *   albedo           [n_cols] surface albedo in [0,1];
 *   flux_toa         [n_cols] flux normal to the beam at the top of the
 *                    atmosphere, or NULL for 1;
 *   flux_dir, flux_dn_dif, flux_up
 *                    [n_cols][nlay+1] outputs at the levels (0 = top of the
 *                    atmosphere): direct horizontal flux, diffuse downward
 *                    and upward flux (also used as scratch; all required);
 *   tod_flux         [n_cols] or NULL: direct + diffuse downward flux at
 *                    level tod_level (the top of the ray tracer's domain);
 *   tod_diffuse_fraction [n_cols] FP32 or NULL: its diffuse share (0 where
 *                    the flux is 0), the input of rt3d_batched_medium.
 * mu0 = cos(solar zenith angle) in (0, 1] (host); 0 <= tod_level <= nlay.
 * RT3D_EINVAL on bad arguments (nothing launched).  One lane per column;
 * asynchronous on `stream`. */
rt3d_status rt3d_two_stream(int32_t n_cols, int32_t nlay, const double* tau,
                            const double* ssa, const double* g,
                            const double* albedo, double mu0,
                            const double* flux_toa, double* flux_dir,
                            double* flux_dn_dif, double* flux_up,
                            int32_t tod_level, double* tod_flux,
                            float* tod_diffuse_fraction, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* RT3D_H */
