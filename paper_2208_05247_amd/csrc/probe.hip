// probe.hip -- measured ceiling of the tracer's memory access pattern
// (dependent random 16-byte gathers plus random 64-bit atomic adds over the
// same footprint), so that the tracer's collision rate can be set against
// what the memory system delivers for that pattern rather than only against
// nominal HBM bandwidth.  Not a step of the method; built into its own
// library, librt3d_probe.so, with the C ABI of include/rt3d_probe.h.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "rt3d_probe.h"

namespace {

constexpr int kThreads = 1024;
constexpr int kOk = 0, kInval = 1, kDevice = 3;

// splitmix64 finaliser (Steele, Lea and Flood 2014)
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// uniform index in [0, n) from 32 random bits (n < 2^32)
__device__ __forceinline__ uint32_t bounded(uint32_t r, uint32_t n) {
    return (uint32_t)(((uint64_t)r * n) >> 32);
}

// kChains independent dependent-gather chains per lane; all kChains
// gathers of one step are issued before any of their values is used.
template <int kChains, bool kPair>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(8)))
    probe_kernel(const float4* __restrict__ rec, uint32_t nrec, unsigned long long* __restrict__ tally,
                 uint32_t ntally, uint32_t events, uint32_t atomics_per_16, uint64_t seed,
                 float* __restrict__ sink) {
    const uint64_t lane = blockIdx.x * (uint64_t)kThreads + threadIdx.x;
    uint64_t h[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) h[c] = mix64(seed ^ mix64(lane * kChains + c + 1));
    float acc = 0.0f;
    for (uint32_t e = 0; e < events; ++e) {
        float4 v[kChains];
        float p[kChains];
#pragma unroll
        for (int c = 0; c < kChains; ++c) {
            const uint32_t r = bounded((uint32_t)h[c], nrec);
            v[c] = rec[r];
            if (kPair) p[c] = rec[r ^ 4u].y;
        }
#pragma unroll
        for (int c = 0; c < kChains; ++c) {
            acc += v[c].x + v[c].w;
            if (kPair) acc += p[c];
            // the next index depends on the value just loaded
            h[c] = mix64(h[c] ^ ((uint64_t)__float_as_uint(v[c].x) << 32 | __float_as_uint(v[c].y)) ^ e);
            if ((e & 15u) < atomics_per_16) atomicAdd(&tally[bounded((uint32_t)(h[c] >> 32), ntally)], 1ull);
        }
    }
    sink[lane] = acc;
}

uint32_t default_blocks() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) return 0;
    return 2u * (uint32_t)cus;
}

template <bool kPair>
void launch(uint32_t chains, dim3 g, hipStream_t st, const float4* rec, uint32_t nrec, unsigned long long* tally,
            uint32_t ntally, uint32_t events, uint32_t a16, uint64_t seed, float* sink) {
    switch (chains) {
        case 1: hipLaunchKernelGGL((probe_kernel<1, kPair>), g, dim3(kThreads), 0, st, rec, nrec, tally, ntally,
                                   events, a16, seed, sink); break;
        case 2: hipLaunchKernelGGL((probe_kernel<2, kPair>), g, dim3(kThreads), 0, st, rec, nrec, tally, ntally,
                                   events, a16, seed, sink); break;
        case 3: hipLaunchKernelGGL((probe_kernel<3, kPair>), g, dim3(kThreads), 0, st, rec, nrec, tally, ntally,
                                   events, a16, seed, sink); break;
        default: hipLaunchKernelGGL((probe_kernel<4, kPair>), g, dim3(kThreads), 0, st, rec, nrec, tally, ntally,
                                    events, a16, seed, sink); break;
    }
}

}  // namespace

extern "C" {

uint64_t rt3d_probe_lanes(uint32_t grid_blocks) {
    const uint32_t b = grid_blocks ? grid_blocks : default_blocks();
    return (uint64_t)b * kThreads;
}

int rt3d_probe_gathers(const void* records, uint64_t n_records, uint64_t* tally, uint64_t n_tally, uint32_t events,
                       uint32_t chains, uint32_t atomics_per_16, uint32_t flags, uint32_t grid_blocks, uint64_t seed,
                       float* sink, uint64_t n_sink, void* stream) {
    if (!records || !tally || !sink || n_records == 0 || n_tally == 0) return kInval;
    if (n_records >= (1ull << 32) || n_tally >= (1ull << 32) || atomics_per_16 > 16) return kInval;
    if (chains < 1 || chains > RT3D_PROBE_MAX_CHAINS || (flags & ~RT3D_PROBE_LINE_PAIR)) return kInval;
    const bool pair = flags & RT3D_PROBE_LINE_PAIR;
    if ((uintptr_t)records & (pair ? 127 : 15)) return kInval;
    if (pair && (n_records & 7)) return kInval;
    const uint32_t blocks = grid_blocks ? grid_blocks : default_blocks();
    if (blocks == 0) return kDevice;
    if (n_sink < (uint64_t)blocks * kThreads) return kInval;
    const hipStream_t st = (hipStream_t)stream;
    if (pair)
        launch<true>(chains, dim3(blocks), st, (const float4*)records, (uint32_t)n_records,
                     (unsigned long long*)tally, (uint32_t)n_tally, events, atomics_per_16, seed, sink);
    else
        launch<false>(chains, dim3(blocks), st, (const float4*)records, (uint32_t)n_records,
                      (unsigned long long*)tally, (uint32_t)n_tally, events, atomics_per_16, seed, sink);
    return hipGetLastError() == hipSuccess ? kOk : kDevice;
}

}  // extern "C"
