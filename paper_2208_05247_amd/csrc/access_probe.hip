// access_probe.hip -- measured ceiling of the tracer's memory access
// pattern (dependent random 16-byte gathers plus random 64-bit atomic adds
// over the same footprint), so that the tracer's collision rate can be set
// against what the memory system delivers for that pattern rather than
// only against nominal HBM bandwidth.  Not a step of the method.
// C ABI declared in include/rt3d.h (rt3d_access_probe).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "rt3d.h"

namespace {

constexpr int kThreads = 1024;

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

__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(8)))
    access_probe_kernel(const float4* __restrict__ rec, uint32_t nrec, unsigned long long* __restrict__ tally,
                        uint32_t ntally, uint32_t events, uint32_t atomics_per_16, uint64_t seed,
                        float* __restrict__ sink) {
    const uint64_t lane = blockIdx.x * (uint64_t)kThreads + threadIdx.x;
    uint64_t h = mix64(seed ^ mix64(lane + 1));
    float acc = 0.0f;
    for (uint32_t e = 0; e < events; ++e) {
        const float4 c = rec[bounded((uint32_t)h, nrec)];
        acc += c.x + c.w;
        // the next index depends on the value just loaded
        h = mix64(h ^ ((uint64_t)__float_as_uint(c.x) << 32 | __float_as_uint(c.y)) ^ e);
        if ((e & 15u) < atomics_per_16) atomicAdd(&tally[bounded((uint32_t)(h >> 32), ntally)], 1ull);
    }
    sink[lane] = acc;
}

uint32_t default_blocks() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) return 0;
    return 2u * (uint32_t)cus;
}

}  // namespace

extern "C" {

uint64_t rt3d_access_probe_lanes(uint32_t grid_blocks) {
    const uint32_t b = grid_blocks ? grid_blocks : default_blocks();
    return (uint64_t)b * kThreads;
}

rt3d_status rt3d_access_probe(const void* records, uint64_t n_records, uint64_t* tally, uint64_t n_tally,
                              uint32_t events, uint32_t atomics_per_16, uint32_t grid_blocks, uint64_t seed,
                              float* sink, uint64_t n_sink, void* stream) {
    if (!records || !tally || !sink || n_records == 0 || n_tally == 0) return RT3D_EINVAL;
    if (n_records >= (1ull << 32) || n_tally >= (1ull << 32) || atomics_per_16 > 16) return RT3D_EINVAL;
    if ((uintptr_t)records & 15) return RT3D_EINVAL;
    const uint32_t blocks = grid_blocks ? grid_blocks : default_blocks();
    if (blocks == 0) return RT3D_EDEVICE;
    if (n_sink < (uint64_t)blocks * kThreads) return RT3D_EINVAL;
    hipLaunchKernelGGL(access_probe_kernel, dim3(blocks), dim3(kThreads), 0, (hipStream_t)stream,
                       (const float4*)records, (uint32_t)n_records, (unsigned long long*)tally, (uint32_t)n_tally,
                       events, atomics_per_16, seed, sink);
    return hipGetLastError() == hipSuccess ? RT3D_OK : RT3D_EDEVICE;
}

}  // extern "C"
