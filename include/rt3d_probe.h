/*
 * rt3d_probe.h -- C ABI of librt3d_probe.so, a measurement of what the
 * memory system delivers for the tracer's access pattern.  It is not a step
 * of the method and not part of the tracer library (librt3d.so); the
 * benchmark loads it to set the tracer's collision rate against a measured
 * ceiling, and to calibrate hardware traffic counters on random accesses.
 *
 * The pattern: in the tracer (sec. 2.3 of Veerman, van Stratum and van
 * Heerwaarden, GRL 2022: tentative collisions looked up in the fine grid,
 * absorbed weight stored per cell) a photon's next tentative collision
 * depends on the values its last one read, so each photon has one random
 * 16-byte cell-record gather in flight at a time, and most collisions add
 * a deposit to a random heating-tally cell with a 64-bit atomic.
 *
 * Status codes are those of rt3d.h (0 ok, 1 bad argument, 3 device error).
 */
#ifndef RT3D_PROBE_H
#define RT3D_PROBE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RT3D_PROBE_MAX_CHAINS 4

/* Flags of rt3d_probe_gathers */
#define RT3D_PROBE_LINE_PAIR 0x1u /* after each gather, a second 16-byte
                                     gather from the other 64-byte half of
                                     the same 128-byte line (record index
                                     xor 4), issued without waiting for the
                                     first: separates 64-byte from 128-byte
                                     fetch granularity in the counters */

/* A persistent grid of 1024-lane workgroups (8 waves per SIMD).  Every lane
 * runs `chains` (1..RT3D_PROBE_MAX_CHAINS) independent chains of `events`
 * dependent random gathers each, the chains interleaved so that the lane
 * has `chains` gathers in flight at a time.  Chain c of lane l starts from
 * h = mix64(seed ^ mix64(l * chains + c + 1)) (mix64 = the splitmix64
 * finaliser); its gather e reads record r = (lo32(h) * n_records) >> 32 of
 * `records` (DEVICE, 16-byte records) and then sets
 * h = mix64(h ^ (bits(x) << 32 | bits(y)) ^ e) from the record's first two
 * FP32 words x, y, so each index depends on the value the previous gather
 * returned.  If (e mod 16) < atomics_per_16 the lane then adds 1 to
 * tally[(hi32(h) * n_tally) >> 32] (DEVICE uint64) with a 64-bit atomic.
 * For every gather, in chain order, the lane adds x + w (FP32) of the
 * record to a running sum; with RT3D_PROBE_LINE_PAIR it also adds y of
 * record r xor 4.  sink (DEVICE FP32, n_sink >= rt3d_probe_lanes(grid_blocks))
 * receives each lane's sum, so no gather is dead.
 * grid_blocks: workgroups, 0 = two per compute unit.
 * RT3D_EINVAL (nothing launched) on null pointers, zero sizes,
 * n_records or n_tally >= 2^32, atomics_per_16 > 16, chains outside
 * 1..RT3D_PROBE_MAX_CHAINS, unknown flags, records not 16-byte aligned
 * (128-byte aligned and n_records a multiple of 8 with LINE_PAIR), a short
 * sink.  Asynchronous on `stream` (hipStream_t as void*); time it with
 * events on that stream. */
int rt3d_probe_gathers(const void* records, uint64_t n_records, uint64_t* tally, uint64_t n_tally,
                       uint32_t events, uint32_t chains, uint32_t atomics_per_16, uint32_t flags,
                       uint32_t grid_blocks, uint64_t seed, float* sink, uint64_t n_sink, void* stream);

/* Lanes rt3d_probe_gathers launches for grid_blocks (0 = two workgroups per
 * compute unit of the current device); 0 if the device cannot be queried. */
uint64_t rt3d_probe_lanes(uint32_t grid_blocks);

#ifdef __cplusplus
}
#endif

#endif /* RT3D_PROBE_H */
