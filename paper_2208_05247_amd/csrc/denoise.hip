// denoise.hip -- BF16 MFMA kernels of the learned heating-rate denoiser:
// a 3D convolutional encoder-decoder trained on low/high-photon tally pairs
// produced by the tracer.  Declared in include/rt3d_denoise.h.
//
// Conventions: activations are BF16 channels-last [D][H][W][C] (C a multiple
// of 16, or 4 for the first layer's input); weights BF16 [Cout][KS^3][Cin]
// with FP32 master copies; all products accumulate in FP32 on the matrix
// cores.
//
// Convolution = implicit GEMM on v_mfma_f32_32x32x16_bf16: GEMM rows are 32
// consecutive voxels along x, columns 32 output channels, and the reduction
// runs over the KS^3 taps and 16-channel chunks.  A lane feeds the A operand
// with 8 channels of one voxel (zero outside the domain) and the B operand
// with 8 input channels of one output channel's weights.  The accumulator of
// lane l, element r holds row 8*(r/4) + 4*(l/32) + r%4, column l%32.
// 3x3x3 layers run from an input halo staged in LDS (conv3_tiled_kernel,
// conv3_c32_kernel, conv3_c4_kernel); the 1x1x1 head uses conv_fwd_kernel,
// one wave per 32 x 32 output tile with its operands read directly, or in
// inference runs inside conv3_c32_kernel after the last 3x3x3 layer.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include "rt3d.h"
#include "rt3d_denoise.h"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

thread_local char d_err[256] = "";

rt3d_status dfail(hipError_t e, const char* where) {
    snprintf(d_err, sizeof d_err, "%s: %s", where, hipGetErrorString(e));
    return RT3D_EDEVICE;
}

#define DN_TRY(expr)                                   \
    do {                                               \
        hipError_t e_ = (expr);                        \
        if (e_ != hipSuccess) return dfail(e_, #expr); \
    } while (0)

// 16 zero bytes in global memory (read in place of voxels outside the domain)
__device__ __align__(16) const uint32_t dn_zero16[4] = {0u, 0u, 0u, 0u};

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// FP32 -> BF16, round to nearest even (inputs are finite).
__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ bf16x8 as_bf16x8(uint4 v) { return __builtin_bit_cast(bf16x8, v); }

unsigned blocks_for(size_t n, unsigned threads = 256, unsigned cap = 65535) {
    size_t g = (n + threads - 1) / threads;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

// ---------------------------------------------------------------------------
// Convolution forward (also the data gradient, with flipped weights)
// ---------------------------------------------------------------------------
struct ConvArgs {
    const uint16_t* x1;
    const uint16_t* x2;
    int c1, c2;            // input channels from x1 and x2 (multiples of 16)
    const uint16_t* w;     // [cout][taps][c1 + c2]
    const float* bias;     // [cout] or null
    uint16_t* y1;          // channels [0, o1)
    uint16_t* y2;          // channels [o1, cout)
    int o1;
    float* yf;             // optional FP32 copy [vox][yf_cols] of channels < yf_cols
    int D, H, W, cout, relu;
    int up1;               // x1 at half resolution, read nearest-upsampled
    int yf_cols;
    // optional 1x1x1 head fused after a 32-output 3x3x3 convolution:
    // hy[vox][hcols] = FP32 channels [0, hcols) of conv1(bf16(y), hw) + hb
    const uint16_t* hw;    // [32][32] (head output, input channel)
    const float* hb;       // [32] or null
    float* hy;
    int hcols;
};

template <int KS>
__global__ void __launch_bounds__(256) conv_fwd_kernel(const ConvArgs a) {
    const int lane = threadIdx.x & 63;
    const long wave = (long)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int ntco = a.cout / 32;
    const int tiles_x = (a.W + 31) / 32;
    const long ntiles = (long)a.D * a.H * tiles_x * ntco;
    if (wave >= ntiles) return;
    const int cot = (int)(wave % ntco);
    long rest = wave / ntco;
    const int tx = (int)(rest % tiles_x);
    rest /= tiles_x;
    const int yy = (int)(rest % a.H);
    const int zz = (int)(rest / a.H);
    const int m = lane & 31, half = lane >> 5;
    const int xv = tx * 32 + m;
    const int co = cot * 32 + m;
    const int cin = a.c1 + a.c2;
    constexpr int taps = KS * KS * KS;
    f32x16 acc;
    for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
    for (int t = 0; t < taps; ++t) {
        const int dz = t / (KS * KS) - KS / 2, dy = (t / KS) % KS - KS / 2, dx = t % KS - KS / 2;
        const int z = zz + dz, y = yy + dy, x = xv + dx;
        const bool inb = z >= 0 && z < a.D && y >= 0 && y < a.H && x >= 0 && x < a.W;
        const long vox = ((long)z * a.H + y) * a.W + x;
        const uint16_t* wrow = a.w + ((long)co * taps + t) * cin + 8 * half;
        for (int c0 = 0; c0 < cin; c0 += 16) {
            uint4 av = make_uint4(0u, 0u, 0u, 0u);
            if (inb) {
                const uint16_t* src = c0 < a.c1 ? a.x1 + vox * a.c1 + c0 : a.x2 + vox * a.c2 + (c0 - a.c1);
                av = *(const uint4*)(src + 8 * half);
            }
            const uint4 bv = *(const uint4*)(wrow + c0);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(av), as_bf16x8(bv), acc, 0, 0, 0);
        }
    }
    const int n = cot * 32 + m;
    const float b = a.bias ? a.bias[n] : 0.0f;
    for (int r = 0; r < 16; ++r) {
        const int mm = 8 * (r >> 2) + 4 * half + (r & 3);
        const int x = tx * 32 + mm;
        if (x >= a.W) continue;
        float v = acc[r] + b;
        if (a.relu) v = fmaxf(v, 0.0f);
        const long vox = ((long)zz * a.H + yy) * a.W + x;
        if (a.yf && n < a.yf_cols) a.yf[vox * a.yf_cols + n] = v;
        if (n < a.o1) {
            if (a.y1) a.y1[vox * a.o1 + n] = f2bf(v);
        } else if (a.y2) {
            a.y2[vox * (a.cout - a.o1) + (n - a.o1)] = f2bf(v);
        }
    }
}

// Tiled 3x3x3 convolution.  A workgroup (4 waves) owns an output tile of
// kZ z-slices x kTY y-rows x kTX x-voxels and a slab of up to 64 output
// channels.  For each 16-channel input chunk the
// ((kZ+2) x (kTY+2) x (kTX+2))-voxel input halo is loaded straight into LDS
// once (zero outside the domain), so a staged plane serves kZ output planes;
// every wave then runs the 27 taps over its 2 rows x 2 cout tiles in each output
// plane: A fragments are contiguous 1 KiB rows of the staged halo, B
// fragments (weights) come from global memory, where the small weight
// tensor stays cache resident, one tap ahead of their use, and each is used
// by 2 kZ MFMAs.
constexpr int kTY = 8, kTX = 32, kZ = 2;
constexpr int kHaloY = kTY + 2, kHaloX = kTX + 2;
constexpr int kHaloVox = (kZ + 2) * kHaloY * kHaloX;

// Stages the input halo of one 16-channel chunk, planes z0-1 .. z0+NZ and
// rows y0-1 .. y0+HY-2 of columns x0-1 .. x0+kTX, into LDS as two 16-byte
// halves per voxel (slot 2 v + part), with NT threads.  The loads go
// straight to LDS (global_load_lds_dwordx4: lane l of a wave writes its 16
// bytes at the wave's LDS base + 16 l, checked on the device), so no
// registers hold the data and all of a chunk's loads are in flight at once.
// Slots are filled in batches of 64, one wave instruction each; the tile
// holds a whole number of batches (tile_slots), and slots outside the domain
// or past the halo read the 16-byte zero block.  The caller waits for the
// loads (vmcnt) before the barrier that publishes the tile.
constexpr int tile_slots(int halo_vox) { return (halo_vox * 2 + 63) / 64 * 64; }

template <int NZ, int HY, int NT>
__device__ __forceinline__ void stage_halo16_lds(uint4* tile, const ConvArgs& a, int c0, int x0, int y0, int z0) {
    constexpr int kSlots = NZ * HY * kHaloX * 2, kBatches = (kSlots + 63) / 64, kWaves = NT / 64;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const bool from1 = c0 < a.c1;
    const uint16_t* base = from1 ? a.x1 + c0 : a.x2 + (c0 - a.c1);
    const long cs = from1 ? a.c1 : a.c2;
    const bool half_res = from1 && a.up1;
    for (int bt = wave; bt < kBatches; bt += kWaves) {
        const int i = bt * 64 + lane;
        const int vx = i >> 1, part = i & 1;
        const int hx = vx % kHaloX, hy = (vx / kHaloX) % HY, hz = vx / (kHaloX * HY);
        const int x = x0 + hx - 1, y = y0 + hy - 1, z = z0 + hz - 1;
        const bool in = i < kSlots && x >= 0 && x < a.W && y >= 0 && y < a.H && z >= 0 && z < a.D;
        const long vox = half_res ? ((long)(z >> 1) * (a.H >> 1) + (y >> 1)) * (a.W >> 1) + (x >> 1)
                                  : ((long)z * a.H + y) * a.W + x;
        const uint16_t* src = in ? base + vox * cs + 8 * part : reinterpret_cast<const uint16_t*>(dn_zero16);
        __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)src,
                                         (__attribute__((address_space(3))) void*)(tile + bt * 64), 16, 0, 0);
    }
}

__device__ __forceinline__ void wait_loads() { __asm__ volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) conv3_tiled_kernel(const ConvArgs a) {
    __shared__ uint4 tile[tile_slots(kHaloVox)];  // 16 channels = two 16-byte halves per voxel
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int m = lane & 31, half = lane >> 5;
    const int nslab = (a.cout + 63) / 64;
    const int tiles_x = (a.W + kTX - 1) / kTX, tiles_y = (a.H + kTY - 1) / kTY;
    long b = blockIdx.x;
    const int slab = (int)(b % nslab);
    b /= nslab;
    const int txi = (int)(b % tiles_x);
    b /= tiles_x;
    const int tyi = (int)(b % tiles_y);
    const int z0 = (int)(b / tiles_y) * kZ;
    const int x0 = txi * kTX, y0 = tyi * kTY;
    const int co0 = slab * 64;
    const int nct = min(2, (a.cout - co0) / 32);
    const int cin = a.c1 + a.c2;
    const int row0 = 2 * wave;  // rows row0, row0 + 1 of the tile
    f32x16 acc[kZ][2][2];
#pragma unroll
    for (int oz = 0; oz < kZ; ++oz)
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
            for (int ct = 0; ct < 2; ++ct)
#pragma unroll
                for (int e = 0; e < 16; ++e) acc[oz][r][ct][e] = 0.0f;

    // weight fragments of (chunk c, tap t) for this lane's output channels;
    // the next tap's are loaded before the current tap's MFMAs run, so their
    // latency hides behind them (branch-free: past the last chunk or channel
    // tile the address is clamped in bounds and the fragment is never used)
    auto load_b = [&](int c, int t, uint4* out) {
        const int cc = min(c, cin - 16);
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) {
            const int co = min(co0 + 32 * ct + m, a.cout - 1);
            out[ct] = *(const uint4*)(a.w + ((long)co * 27 + t) * cin + cc + 8 * half);
        }
    };
    uint4 bv[2];
    load_b(0, 0, bv);
    for (int c0 = 0; c0 < cin; c0 += 16) {
        __syncthreads();  // the previous chunk's halo is no longer read
        stage_halo16_lds<kZ + 2, kHaloY, 256>(tile, a, c0, x0, y0, z0);
        wait_loads();
        __syncthreads();
#pragma unroll
        for (int t = 0; t < 27; ++t) {
            const int dz = t / 9, dy = (t / 3) % 3, dx = t % 3;
            uint4 bn[2];
            if (t < 26) load_b(c0, t + 1, bn);
            else load_b(c0 + 16, 0, bn);
            __builtin_amdgcn_sched_barrier(0);  // keep the prefetch ahead of the MFMAs
#pragma unroll
            for (int oz = 0; oz < kZ; ++oz)
#pragma unroll
                for (int r = 0; r < 2; ++r) {
                    // output plane oz reads staged plane oz + dz
                    const uint4 av = tile[(((oz + dz) * kHaloY + row0 + r + dy) * kHaloX + m + dx) * 2 + half];
#pragma unroll
                    for (int ct = 0; ct < 2; ++ct)
                        if (ct < nct)
                            acc[oz][r][ct] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                                as_bf16x8(av), as_bf16x8(bv[ct]), acc[oz][r][ct], 0, 0, 0);
                }
            bv[0] = bn[0];
            bv[1] = bn[1];
        }
    }
    if (!a.yf && a.y1 && a.o1 == a.cout && nct == 2) {
        // BF16 output through LDS, as in conv3_c4_kernel: each wave writes
        // one output row of its slab (32 voxels x 64 channels, 4 KiB) to its
        // own slice of the halo tile and stores it as 16-byte pieces (8
        // channels of one voxel), 4 per lane, instead of 2-byte stores
        static_assert(4 * 32 * 64 * 2 <= tile_slots(kHaloVox) * 16, "row scratch exceeds the halo tile");
        __syncthreads();  // every wave is done reading the halo
        uint16_t* row = reinterpret_cast<uint16_t*>(tile) + wave * (32 * 64);
        float bias[2];
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) bias[ct] = a.bias ? a.bias[co0 + 32 * ct + m] : 0.0f;
#pragma unroll
        for (int oz = 0; oz < kZ; ++oz) {
            const int zz = z0 + oz;
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                const int y = y0 + row0 + r;
#pragma unroll
                for (int ct = 0; ct < 2; ++ct)
#pragma unroll
                    for (int e = 0; e < 16; ++e) {
                        float v = acc[oz][r][ct][e] + bias[ct];
                        if (a.relu) v = fmaxf(v, 0.0f);
                        row[(8 * (e >> 2) + 4 * half + (e & 3)) * 64 + 32 * ct + m] = f2bf(v);
                    }
                // LDS instructions of one wave complete in order; the barrier
                // keeps the compiler from moving the reads across the writes
                __builtin_amdgcn_wave_barrier();
#pragma unroll
                for (int it = 0; it < 4; ++it) {
                    const int q = it * 64 + lane;  // voxel q / 8, channels co0 + 8 (q % 8) ..
                    const int x = x0 + (q >> 3);
                    const uint4 v = *reinterpret_cast<const uint4*>(row + (q >> 3) * 64 + 8 * (q & 7));
                    if (zz < a.D && y < a.H && x < a.W)
                        *reinterpret_cast<uint4*>(a.y1 + (((long)zz * a.H + y) * a.W + x) * a.cout + co0 + 8 * (q & 7)) = v;
                }
                __builtin_amdgcn_wave_barrier();  // the next row's writes follow these reads
            }
        }
        return;
    }
#pragma unroll
    for (int oz = 0; oz < kZ; ++oz) {
        const int zz = z0 + oz;
        if (zz >= a.D) continue;
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int y = y0 + row0 + r;
            if (y >= a.H) continue;
#pragma unroll
            for (int ct = 0; ct < 2; ++ct) {
                if (ct >= nct) continue;
                const int n = co0 + 32 * ct + m;
                const float bias = a.bias ? a.bias[n] : 0.0f;
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    const int x = x0 + 8 * (e >> 2) + 4 * half + (e & 3);
                    if (x >= a.W) continue;
                    float v = acc[oz][r][ct][e] + bias;
                    if (a.relu) v = fmaxf(v, 0.0f);
                    const long vox = ((long)zz * a.H + y) * a.W + x;
                    if (a.yf && n < a.yf_cols) a.yf[vox * a.yf_cols + n] = v;
                    if (n < a.o1) {
                        if (a.y1) a.y1[vox * a.o1 + n] = f2bf(v);
                    } else if (a.y2) {
                        a.y2[vox * (a.cout - a.o1) + (n - a.o1)] = f2bf(v);
                    }
                }
            }
        }
    }
}

// 3x3x3 convolution with exactly 32 output channels (one MFMA column tile,
// so an input fragment cannot be shared between output-channel tiles).
// Instead each wave owns 4 output rows in each of the workgroup's 2 output
// z-slices and, per z-slice of the kernel, keeps its 9 weight fragments of
// the current 16-channel chunk in registers: it walks the 6 staged input
// rows its outputs need in both input planes that kernel slice reaches,
// 3 x-shifts each, and feeds every fragment it reads from LDS to all (up
// to 3) of its output rows that use it.  Workgroup tile: 2 z x 16 rows x
// 32 voxels, so a staged input plane serves two output planes (4 planes
// staged per 2 outputs instead of 3 per 1).  With a head (ConvArgs::hw) the
// 1x1x1 convolution follows in the epilogue and only its output is stored.
constexpr int kTY32 = 16;
constexpr int kHaloY32 = kTY32 + 2;
constexpr int kZ32 = 2;
constexpr int kHaloVox32 = (kZ32 + 2) * kHaloY32 * kHaloX;
// the fused head reuses the halo tile: 4 waves x kZ32 x 4 rows x 32 x 32 BF16
// activations, then per wave one output row of 32 voxels x 2 FP32
static_assert(4 * kZ32 * 4 * 32 * 32 * 2 <= kHaloVox32 * 2 * 16, "head scratch exceeds the halo tile");
constexpr int kHeadOutOffset = 4 * kZ32 * 4 * 32 * 32 * 2;  // bytes
static_assert(kHeadOutOffset + 4 * 32 * 2 * 4 <= kHaloVox32 * 2 * 16, "head output scratch exceeds the halo tile");

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) conv3_c32_kernel(const ConvArgs a) {
    __shared__ uint4 tile[tile_slots(kHaloVox32)];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int m = lane & 31, half = lane >> 5;
    const int tiles_x = (a.W + kTX - 1) / kTX, tiles_y = (a.H + kTY32 - 1) / kTY32;
    long b = blockIdx.x;
    const int txi = (int)(b % tiles_x);
    b /= tiles_x;
    const int tyi = (int)(b % tiles_y);
    const int z0 = (int)(b / tiles_y) * kZ32;
    const int x0 = txi * kTX, y0 = tyi * kTY32;
    const int cin = a.c1 + a.c2;
    const int row0 = 4 * wave;
    f32x16 acc[kZ32][4];
#pragma unroll
    for (int oz = 0; oz < kZ32; ++oz)
#pragma unroll
        for (int o = 0; o < 4; ++o)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[oz][o][e] = 0.0f;

    for (int c0 = 0; c0 < cin; c0 += 16) {
        __syncthreads();
        stage_halo16_lds<kZ32 + 2, kHaloY32, 256>(tile, a, c0, x0, y0, z0);
        wait_loads();
        __syncthreads();
        for (int dz = 0; dz < 3; ++dz) {
            // the 9 weight fragments of this z-slice of the kernel
            uint4 bv[9];
#pragma unroll
            for (int t = 0; t < 9; ++t)
                bv[t] = *(const uint4*)(a.w + ((long)m * 27 + dz * 9 + t) * cin + c0 + 8 * half);
            // the 12 staged rows (2 output planes x 6 input rows) this wave
            // reads for this kernel slice, each as 3 x-shifted fragments; the
            // fragments of the next row are read before this row's MFMAs
            // run, so the LDS latency hides behind them
            auto row_frags = [&](int step, uint4* av) {
                const int oz = step / 6, r = step % 6;  // output plane oz reads staged plane oz + dz
#pragma unroll
                for (int dx = 0; dx < 3; ++dx)
                    av[dx] = tile[(((oz + dz) * kHaloY32 + row0 + r) * kHaloX + m + dx) * 2 + half];
            };
            uint4 cur[3], nxt[3];
            row_frags(0, cur);
#pragma unroll
            for (int step = 0; step < kZ32 * 6; ++step) {
                const int oz = step / 6, r = step % 6;
                if (step + 1 < kZ32 * 6) row_frags(step + 1, nxt);
                // keeps the scheduler from hoisting the reads of later rows
                // ahead of these MFMAs (it would spill at 2 waves/SIMD)
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int dx = 0; dx < 3; ++dx)
#pragma unroll
                    for (int o = 0; o < 4; ++o) {
                        const int dy = r - o;  // output row o reads halo row o + dy
                        if (dy >= 0 && dy <= 2)
                            acc[oz][o] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                                as_bf16x8(cur[dx]), as_bf16x8(bv[dy * 3 + dx]), acc[oz][o], 0, 0, 0);
                    }
#pragma unroll
                for (int dx = 0; dx < 3; ++dx) cur[dx] = nxt[dx];
            }
        }
    }
    const int n = m;
    const float bias = a.bias ? a.bias[n] : 0.0f;
    if (a.hw) {
        // Fused head.  Each wave writes its BF16 activations, 32 voxels x 32
        // channels per output row, to its own part of the (no longer needed)
        // halo tile, so that a lane can read the 8 consecutive channels of
        // one voxel that the A operand takes; the head then runs the same
        // two MFMAs per row as the 1x1x1 convolution kernel, in the same
        // order, so its output is bitwise that of the unfused pair.
        uint16_t* ht = reinterpret_cast<uint16_t*>(tile) + wave * (kZ32 * 4 * 32 * 32);
        __syncthreads();  // every wave is done reading the halo
#pragma unroll
        for (int oz = 0; oz < kZ32; ++oz)
#pragma unroll
            for (int o = 0; o < 4; ++o)
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    float v = acc[oz][o][e] + bias;
                    if (a.relu) v = fmaxf(v, 0.0f);
                    ht[((oz * 4 + o) * 32 + 8 * (e >> 2) + 4 * half + (e & 3)) * 32 + n] = f2bf(v);
                }
        __syncthreads();
        uint4 hwv[2];
#pragma unroll
        for (int c = 0; c < 2; ++c) hwv[c] = *(const uint4*)(a.hw + m * 32 + 16 * c + 8 * half);
        const float hbias = a.hb ? a.hb[n] : 0.0f;
#pragma unroll
        for (int oz = 0; oz < kZ32; ++oz) {
            const int zz = z0 + oz;
            if (zz >= a.D) continue;
#pragma unroll
            for (int o = 0; o < 4; ++o) {
                const int y = y0 + row0 + o;
                if (y >= a.H) continue;
                f32x16 h;
#pragma unroll
                for (int e = 0; e < 16; ++e) h[e] = 0.0f;
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    const uint4 av = *(const uint4*)(ht + ((oz * 4 + o) * 32 + m) * 32 + 16 * c + 8 * half);
                    h = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(av), as_bf16x8(hwv[c]), h, 0, 0, 0);
                }
                if (a.hcols == 2) {
                    // the two used outputs of the row go through LDS (behind
                    // the activations' part of the tile), so that the row is
                    // stored as one 8-byte piece per voxel by 32 lanes instead
                    // of 16 stores of 4 bytes by 4 lanes each
                    float* hrow = reinterpret_cast<float*>(tile) + kHeadOutOffset / 4 + wave * 64;
                    if (n < 2) {
#pragma unroll
                        for (int e = 0; e < 16; ++e) hrow[(8 * (e >> 2) + 4 * half + (e & 3)) * 2 + n] = h[e] + hbias;
                    }
                    // LDS instructions of one wave complete in order; the
                    // barrier keeps the compiler from moving the read across
                    // the writes
                    __builtin_amdgcn_wave_barrier();
                    if (lane < 32) {
                        const float2 v = *reinterpret_cast<const float2*>(hrow + 2 * lane);
                        if (x0 + lane < a.W)
                            *reinterpret_cast<float2*>(a.hy + (((long)zz * a.H + y) * a.W + x0 + lane) * 2) = v;
                    }
                    __builtin_amdgcn_wave_barrier();  // the next row's writes follow this read
                    continue;
                }
                if (n >= a.hcols) continue;
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    const int x = x0 + 8 * (e >> 2) + 4 * half + (e & 3);
                    if (x >= a.W) continue;
                    a.hy[(((long)zz * a.H + y) * a.W + x) * a.hcols + n] = h[e] + hbias;
                }
            }
        }
        return;
    }
#pragma unroll
    for (int oz = 0; oz < kZ32; ++oz) {
        const int zz = z0 + oz;
        if (zz >= a.D) continue;
#pragma unroll
        for (int o = 0; o < 4; ++o) {
            const int y = y0 + row0 + o;
            if (y >= a.H) continue;
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int x = x0 + 8 * (e >> 2) + 4 * half + (e & 3);
                if (x >= a.W) continue;
                float v = acc[oz][o][e] + bias;
                if (a.relu) v = fmaxf(v, 0.0f);
                const long vox = ((long)zz * a.H + y) * a.W + x;
                if (a.yf && n < a.yf_cols) a.yf[vox * a.yf_cols + n] = v;
                if (n < a.o1) {
                    if (a.y1) a.y1[vox * a.o1 + n] = f2bf(v);
                } else if (a.y2) {
                    a.y2[vox * (a.cout - a.o1) + (n - a.o1)] = f2bf(v);
                }
            }
        }
    }
}

// First layer: 3x3x3 convolution of 4 input channels to 32 outputs, input
// [vox][4] (8 bytes per voxel), weights [32][27][4].  One MFMA K-chunk of 16
// holds the three x-taps of one (z, y) tap pair: A = channels 0-3 of voxels
// x-1, x, x+1 and four zeros, B = the matching 12 weights and four zeros, so
// a row takes 9 MFMAs instead of 27 of 16 mostly-zero channels.  Tile and
// reuse as in conv3_c32_kernel (16 rows x 32 voxels, 4 rows per wave, every
// staged input row fed to all output rows that use it).
constexpr int kHaloVoxC4 = 3 * kHaloY32 * kHaloX;

__global__ void __launch_bounds__(256) conv3_c4_kernel(const ConvArgs a) {
    __shared__ uint2 tile[kHaloVoxC4];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int m = lane & 31, half = lane >> 5;
    const int tiles_x = (a.W + kTX - 1) / kTX, tiles_y = (a.H + kTY32 - 1) / kTY32;
    long b = blockIdx.x;
    const int txi = (int)(b % tiles_x);
    b /= tiles_x;
    const int tyi = (int)(b % tiles_y);
    const int zz = (int)(b / tiles_y);
    const int x0 = txi * kTX, y0 = tyi * kTY32;
    const int row0 = 4 * wave;
    {
        // straight-line staging in batches of four loads per thread in
        // flight
        constexpr int kPer = (kHaloVoxC4 + 255) / 256, SB = 4;
#pragma unroll 1
        for (int j0 = 0; j0 < kPer; j0 += SB) {
            uint2 vv[SB];
#pragma unroll
            for (int j = 0; j < SB; ++j) {
                const int v = threadIdx.x + 256 * (j0 + j);
                const int hx = v % kHaloX, hy = (v / kHaloX) % kHaloY32, hz = v / (kHaloX * kHaloY32);
                const int x = x0 + hx - 1, y = y0 + hy - 1, z = zz + hz - 1;
                const bool in = x >= 0 && x < a.W && y >= 0 && y < a.H && z >= 0 && z < a.D;
                const int xc = min(max(x, 0), a.W - 1), yc = min(max(y, 0), a.H - 1), zc = min(max(z, 0), a.D - 1);
                // a voxel outside the domain reads zeros from dn_zero16: the
                // address is selected, so the load cannot sink into a branch
                // (which would wait for it before the next one is issued)
                vv[j] = *(in ? (const uint2*)(a.x1 + (((long)zc * a.H + yc) * a.W + xc) * 4)
                             : reinterpret_cast<const uint2*>(dn_zero16));
            }
#pragma unroll
            for (int j = 0; j < SB; ++j) {
                const int v = threadIdx.x + 256 * (j0 + j);
                if (j0 + j < kPer && v < kHaloVoxC4) tile[v] = vv[j];
            }
        }
    }
    // B fragments of the 9 (z, y) tap pairs: lane half 0 holds taps dx = 0, 1,
    // half 1 tap dx = 2 and zeros
    uint4 bv[9];
    const uint16_t* wrow = a.w + (long)m * 27 * 4;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        const uint2 lo = *(const uint2*)(wrow + (q * 3 + 2 * half) * 4);
        const uint2 hi = half ? make_uint2(0u, 0u) : *(const uint2*)(wrow + (q * 3 + 1) * 4);
        bv[q] = make_uint4(lo.x, lo.y, hi.x, hi.y);
    }
    __syncthreads();
    f32x16 acc[4];
#pragma unroll
    for (int o = 0; o < 4; ++o)
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[o][e] = 0.0f;
#pragma unroll
    for (int dz = 0; dz < 3; ++dz)
#pragma unroll
        for (int r = 0; r < 6; ++r) {
            const int i = (dz * kHaloY32 + row0 + r) * kHaloX + m;  // voxel x-1 of output column m
            const uint2 lo = tile[i + 2 * half];
            const uint2 hi = half ? make_uint2(0u, 0u) : tile[i + 1];
            const uint4 av = make_uint4(lo.x, lo.y, hi.x, hi.y);
#pragma unroll
            for (int o = 0; o < 4; ++o) {
                const int dy = r - o;
                if (dy >= 0 && dy <= 2)
                    acc[o] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(av), as_bf16x8(bv[dz * 3 + dy]), acc[o],
                                                                     0, 0, 0);
            }
        }
    const int n = m;
    const float bias = a.bias ? a.bias[n] : 0.0f;
    if (!a.yf && a.y1 && a.o1 == 32) {
        // BF16 output through LDS: a lane holds one channel of 16 voxels, so
        // direct stores would be 2 bytes each; each wave instead writes one
        // output row (32 voxels x 32 channels, 2 KiB) to its own slice of the
        // halo tile (every wave is done reading it) and stores it back as
        // 16-byte pieces (8 channels of one voxel), 2 per lane
        static_assert(4 * 32 * 32 * 2 <= kHaloVoxC4 * 8, "row scratch exceeds the halo tile");
        __syncthreads();
        uint16_t* row = reinterpret_cast<uint16_t*>(tile) + wave * (32 * 32);
#pragma unroll
        for (int o = 0; o < 4; ++o) {
            const int y = y0 + row0 + o;
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                float v = acc[o][e] + bias;
                if (a.relu) v = fmaxf(v, 0.0f);
                row[(8 * (e >> 2) + 4 * half + (e & 3)) * 32 + n] = f2bf(v);
            }
            // LDS instructions of one wave complete in order: the reads below
            // see this row; the barrier only keeps the compiler from moving
            // them across the writes
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int it = 0; it < 2; ++it) {
                const int q = it * 64 + lane;  // 16-byte piece: voxel q / 4, channels 8 (q % 4) ..
                const int x = x0 + (q >> 2);
                const uint4 v = *reinterpret_cast<const uint4*>(row + (q >> 2) * 32 + 8 * (q & 3));
                if (y < a.H && x < a.W)
                    *reinterpret_cast<uint4*>(a.y1 + (((long)zz * a.H + y) * a.W + x) * 32 + 8 * (q & 3)) = v;
            }
            __builtin_amdgcn_wave_barrier();  // the next row's writes follow these reads
        }
        return;
    }
#pragma unroll
    for (int o = 0; o < 4; ++o) {
        const int y = y0 + row0 + o;
        if (y >= a.H) continue;
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int x = x0 + 8 * (e >> 2) + 4 * half + (e & 3);
            if (x >= a.W) continue;
            float v = acc[o][e] + bias;
            if (a.relu) v = fmaxf(v, 0.0f);
            const long vox = ((long)zz * a.H + y) * a.W + x;
            if (a.yf && n < a.yf_cols) a.yf[vox * a.yf_cols + n] = v;
            if (a.y1) a.y1[vox * a.o1 + n] = f2bf(v);
        }
    }
}

// The first layer and the 2x2x2 average pooling of its output in one launch
// (inference).  A workgroup computes both output planes of one pooled plane
// from four staged input planes (the MFMAs of each output in
// conv3_c4_kernel's order), stores them as conv3_c4_kernel does, and pools
// each wave's pairs of output rows from LDS as they pass, adding in
// pool2_kernel's order (z, then y, then x, in FP32) with the sums of the
// first plane kept in registers: the full-resolution and the pooled output
// are bitwise those of the two separate launches, and the full-resolution
// output is not read back.  D, H, W even.
constexpr int kHaloVoxC4P = 4 * kHaloY32 * kHaloX;

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
conv3_c4_pool_kernel(const ConvArgs a, uint16_t* __restrict__ yp) {
    __shared__ uint2 tile[kHaloVoxC4P];
    __shared__ uint4 rows[4 * 2 * 32 * 32 * 2 / 16];  // per wave two output rows, 32 voxels x 32 BF16 channels
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int m = lane & 31, half = lane >> 5;
    const int tiles_x = (a.W + kTX - 1) / kTX, tiles_y = (a.H + kTY32 - 1) / kTY32;
    long b = blockIdx.x;
    const int txi = (int)(b % tiles_x);
    b /= tiles_x;
    const int tyi = (int)(b % tiles_y);
    const int zp = (int)(b / tiles_y);  // pooled plane: output planes 2 zp, 2 zp + 1
    const int z0 = 2 * zp;
    const int x0 = txi * kTX, y0 = tyi * kTY32;
    const int row0 = 4 * wave;
    {
        constexpr int kPer = (kHaloVoxC4P + 255) / 256, SB = 4;
#pragma unroll 1
        for (int j0 = 0; j0 < kPer; j0 += SB) {
            uint2 vv[SB];
#pragma unroll
            for (int j = 0; j < SB; ++j) {
                const int v = threadIdx.x + 256 * (j0 + j);
                const int hx = v % kHaloX, hy = (v / kHaloX) % kHaloY32, hz = v / (kHaloX * kHaloY32);
                const int x = x0 + hx - 1, y = y0 + hy - 1, z = z0 + hz - 1;
                const bool in = x >= 0 && x < a.W && y >= 0 && y < a.H && z >= 0 && z < a.D;
                const int xc = min(max(x, 0), a.W - 1), yc = min(max(y, 0), a.H - 1), zc = min(max(z, 0), a.D - 1);
                vv[j] = *(in ? (const uint2*)(a.x1 + (((long)zc * a.H + yc) * a.W + xc) * 4)
                             : reinterpret_cast<const uint2*>(dn_zero16));
            }
#pragma unroll
            for (int j = 0; j < SB; ++j) {
                const int v = threadIdx.x + 256 * (j0 + j);
                if (j0 + j < kPer && v < kHaloVoxC4P) tile[v] = vv[j];
            }
        }
    }
    uint4 bv[9];
    const uint16_t* wrow = a.w + (long)m * 27 * 4;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        const uint2 lo = *(const uint2*)(wrow + (q * 3 + 2 * half) * 4);
        const uint2 hi = half ? make_uint2(0u, 0u) : *(const uint2*)(wrow + (q * 3 + 1) * 4);
        bv[q] = make_uint4(lo.x, lo.y, hi.x, hi.y);
    }
    __syncthreads();
    const float bias = a.bias ? a.bias[m] : 0.0f;
    uint16_t* scr = reinterpret_cast<uint16_t*>(rows) + wave * (2 * 32 * 32);
    const int pv = lane >> 2, cg = lane & 3;  // this lane's pooled voxel of a pooled row and 8-channel group
    float s[2][8];
#pragma unroll
    for (int pr = 0; pr < 2; ++pr)
#pragma unroll
        for (int k = 0; k < 8; ++k) s[pr][k] = 0.0f;
#pragma unroll 1
    for (int oz = 0; oz < 2; ++oz) {
        f32x16 acc[4];
#pragma unroll
        for (int o = 0; o < 4; ++o)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[o][e] = 0.0f;
#pragma unroll
        for (int dz = 0; dz < 3; ++dz)
#pragma unroll
            for (int r = 0; r < 6; ++r) {
                const int i = ((oz + dz) * kHaloY32 + row0 + r) * kHaloX + m;  // voxel x-1 of output column m
                const uint2 lo = tile[i + 2 * half];
                const uint2 hi = half ? make_uint2(0u, 0u) : tile[i + 1];
                const uint4 av = make_uint4(lo.x, lo.y, hi.x, hi.y);
#pragma unroll
                for (int o = 0; o < 4; ++o) {
                    const int dy = r - o;
                    if (dy >= 0 && dy <= 2)
                        acc[o] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(av), as_bf16x8(bv[dz * 3 + dy]),
                                                                         acc[o], 0, 0, 0);
                }
            }
        const int zz = z0 + oz;
#pragma unroll
        for (int pr = 0; pr < 2; ++pr) {
#pragma unroll
            for (int oo = 0; oo < 2; ++oo)
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    float v = acc[2 * pr + oo][e] + bias;
                    if (a.relu) v = fmaxf(v, 0.0f);
                    scr[(oo * 32 + 8 * (e >> 2) + 4 * half + (e & 3)) * 32 + m] = f2bf(v);
                }
            // LDS instructions of one wave complete in order; the barrier
            // keeps the compiler from moving the reads across the writes
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int oo = 0; oo < 2; ++oo) {
                const int y = y0 + row0 + 2 * pr + oo;
#pragma unroll
                for (int it = 0; it < 2; ++it) {
                    const int q = it * 64 + lane;  // voxel q / 4, channels 8 (q % 4) ..
                    const int x = x0 + (q >> 2);
                    const uint4 v = *reinterpret_cast<const uint4*>(scr + (oo * 32 + (q >> 2)) * 32 + 8 * (q & 3));
                    if (y < a.H && x < a.W)
                        *reinterpret_cast<uint4*>(a.y1 + (((long)zz * a.H + y) * a.W + x) * 32 + 8 * (q & 3)) = v;
                }
            }
#pragma unroll
            for (int yy = 0; yy < 2; ++yy)
#pragma unroll
                for (int xx = 0; xx < 2; ++xx) {
                    const uint4 u = *reinterpret_cast<const uint4*>(scr + (yy * 32 + 2 * pv + xx) * 32 + 8 * cg);
                    const uint32_t wd[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        s[pr][2 * k] += bf2f((uint16_t)(wd[k] & 0xffffu));
                        s[pr][2 * k + 1] += bf2f((uint16_t)(wd[k] >> 16));
                    }
                }
            __builtin_amdgcn_wave_barrier();  // the next rows' writes follow these reads
        }
    }
    const int hh = a.H / 2, wh = a.W / 2;
#pragma unroll
    for (int pr = 0; pr < 2; ++pr) {
        const int yh = (y0 + row0) / 2 + pr, xh = x0 / 2 + pv;
        if (yh >= hh || xh >= wh) continue;
        uint32_t o[4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            o[k] = (uint32_t)f2bf(0.125f * s[pr][2 * k]) | ((uint32_t)f2bf(0.125f * s[pr][2 * k + 1]) << 16);
        *reinterpret_cast<uint4*>(yp + (((long)zp * hh + yh) * wh + xh) * 32 + 8 * cg) = make_uint4(o[0], o[1], o[2], o[3]);
    }
}

// The same for a network with the fifth (direct-beam) input: the first
// layer reads 5 input channels stored as 8 per voxel (16 bytes, channels
// 5-7 zero), and one MFMA K-chunk of 16 holds the 15 values of the three
// x-taps of a (z, y) tap pair and one zero: lanes of half 0 take channels
// 0-4 of voxel x-1 and 0-2 of voxel x, lanes of half 1 channels 3-4 of voxel
// x, 0-4 of voxel x+1 and the zero (the B operand the matching weights, taken
// from the 16-channel weight rows w[co][t][16]).  Pooling as in
// conv3_c4_pool_kernel; bitwise equal to the unpacked first layer
// (conv3_c32_kernel on 16-channel features) only up to the order of the
// products within a K-chunk, as the packed 4-channel layer is.
constexpr int kHaloVoxC5P = 4 * kHaloY32 * kHaloX;

__device__ __forceinline__ uint32_t hi_lo(uint32_t a, uint32_t b) { return (a >> 16) | (b << 16); }

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
conv3_c5_pool_kernel(const ConvArgs a, uint16_t* __restrict__ yp) {
    __shared__ uint4 tile[kHaloVoxC5P];
    __shared__ uint4 rows[4 * 2 * 32 * 32 * 2 / 16];  // per wave two output rows, 32 voxels x 32 BF16 channels
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int m = lane & 31, half = lane >> 5;
    const int tiles_x = (a.W + kTX - 1) / kTX, tiles_y = (a.H + kTY32 - 1) / kTY32;
    long b = blockIdx.x;
    const int txi = (int)(b % tiles_x);
    b /= tiles_x;
    const int tyi = (int)(b % tiles_y);
    const int zp = (int)(b / tiles_y);  // pooled plane: output planes 2 zp, 2 zp + 1
    const int z0 = 2 * zp;
    const int x0 = txi * kTX, y0 = tyi * kTY32;
    const int row0 = 4 * wave;
    {
        constexpr int kPer = (kHaloVoxC5P + 255) / 256, SB = 4;
#pragma unroll 1
        for (int j0 = 0; j0 < kPer; j0 += SB) {
            uint4 vv[SB];
#pragma unroll
            for (int j = 0; j < SB; ++j) {
                const int v = threadIdx.x + 256 * (j0 + j);
                const int hx = v % kHaloX, hy = (v / kHaloX) % kHaloY32, hz = v / (kHaloX * kHaloY32);
                const int x = x0 + hx - 1, y = y0 + hy - 1, z = z0 + hz - 1;
                const bool in = x >= 0 && x < a.W && y >= 0 && y < a.H && z >= 0 && z < a.D;
                const int xc = min(max(x, 0), a.W - 1), yc = min(max(y, 0), a.H - 1), zc = min(max(z, 0), a.D - 1);
                vv[j] = *(in ? (const uint4*)(a.x1 + (((long)zc * a.H + yc) * a.W + xc) * 8)
                             : reinterpret_cast<const uint4*>(dn_zero16));
            }
#pragma unroll
            for (int j = 0; j < SB; ++j) {
                const int v = threadIdx.x + 256 * (j0 + j);
                if (j0 + j < kPer && v < kHaloVoxC5P) tile[v] = vv[j];
            }
        }
    }
    // B fragments of the 9 (z, y) tap pairs from the 16-channel weight rows:
    // K 0-4 = tap dx 0 channels 0-4, K 5-9 = dx 1, K 10-14 = dx 2, K 15 = 0
    uint4 bv[9];
    const uint16_t* wrow = a.w + (long)m * 27 * 16;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        uint32_t wd[4];
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            uint32_t lohi[2];
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const int k = 8 * half + 2 * p + e;  // K index of this lane's element
                lohi[e] = k < 15 ? (uint32_t)wrow[(q * 3 + k / 5) * 16 + k % 5] : 0u;
            }
            wd[p] = lohi[0] | (lohi[1] << 16);
        }
        bv[q] = make_uint4(wd[0], wd[1], wd[2], wd[3]);
    }
    __syncthreads();
    const float bias = a.bias ? a.bias[m] : 0.0f;
    uint16_t* scr = reinterpret_cast<uint16_t*>(rows) + wave * (2 * 32 * 32);
    const int pv = lane >> 2, cg = lane & 3;
    float s[2][8];
#pragma unroll
    for (int pr = 0; pr < 2; ++pr)
#pragma unroll
        for (int k = 0; k < 8; ++k) s[pr][k] = 0.0f;
#pragma unroll 1
    for (int oz = 0; oz < 2; ++oz) {
        f32x16 acc[4];
#pragma unroll
        for (int o = 0; o < 4; ++o)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[o][e] = 0.0f;
#pragma unroll
        for (int dz = 0; dz < 3; ++dz)
#pragma unroll
            for (int r = 0; r < 6; ++r) {
                const int i = ((oz + dz) * kHaloY32 + row0 + r) * kHaloX + m;  // voxel x-1 of output column m
                // words of a voxel: (c0, c1), (c2, c3), (c4, 0), (0, 0)
                const uint4 u = tile[i + half], v = tile[i + half + 1];
                const uint4 av = half ? make_uint4(hi_lo(u.y, u.z), v.x, v.y, v.z)   // x: c3 c4; x+1: c0-c4, 0
                                      : make_uint4(u.x, u.y, u.z | (v.x << 16), hi_lo(v.x, v.y));  // x-1: c0-c4; x: c0-c2
#pragma unroll
                for (int o = 0; o < 4; ++o) {
                    const int dy = r - o;
                    if (dy >= 0 && dy <= 2)
                        acc[o] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(av), as_bf16x8(bv[dz * 3 + dy]),
                                                                         acc[o], 0, 0, 0);
                }
            }
        const int zz = z0 + oz;
#pragma unroll
        for (int pr = 0; pr < 2; ++pr) {
#pragma unroll
            for (int oo = 0; oo < 2; ++oo)
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    float v = acc[2 * pr + oo][e] + bias;
                    if (a.relu) v = fmaxf(v, 0.0f);
                    scr[(oo * 32 + 8 * (e >> 2) + 4 * half + (e & 3)) * 32 + m] = f2bf(v);
                }
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int oo = 0; oo < 2; ++oo) {
                const int y = y0 + row0 + 2 * pr + oo;
#pragma unroll
                for (int it = 0; it < 2; ++it) {
                    const int q = it * 64 + lane;
                    const int x = x0 + (q >> 2);
                    const uint4 v = *reinterpret_cast<const uint4*>(scr + (oo * 32 + (q >> 2)) * 32 + 8 * (q & 3));
                    if (y < a.H && x < a.W)
                        *reinterpret_cast<uint4*>(a.y1 + (((long)zz * a.H + y) * a.W + x) * 32 + 8 * (q & 3)) = v;
                }
            }
#pragma unroll
            for (int yy = 0; yy < 2; ++yy)
#pragma unroll
                for (int xx = 0; xx < 2; ++xx) {
                    const uint4 u = *reinterpret_cast<const uint4*>(scr + (yy * 32 + 2 * pv + xx) * 32 + 8 * cg);
                    const uint32_t wd[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        s[pr][2 * k] += bf2f((uint16_t)(wd[k] & 0xffffu));
                        s[pr][2 * k + 1] += bf2f((uint16_t)(wd[k] >> 16));
                    }
                }
            __builtin_amdgcn_wave_barrier();
        }
    }
    const int hh = a.H / 2, wh = a.W / 2;
#pragma unroll
    for (int pr = 0; pr < 2; ++pr) {
        const int yh = (y0 + row0) / 2 + pr, xh = x0 / 2 + pv;
        if (yh >= hh || xh >= wh) continue;
        uint32_t o[4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            o[k] = (uint32_t)f2bf(0.125f * s[pr][2 * k]) | ((uint32_t)f2bf(0.125f * s[pr][2 * k + 1]) << 16);
        *reinterpret_cast<uint4*>(yp + (((long)zp * hh + yh) * wh + xh) * 32 + 8 * cg) = make_uint4(o[0], o[1], o[2], o[3]);
    }
}

// wt[ci][taps-1-t][co] = w[co][t][ci]  (data gradient = convolution of the
// output gradient with the flipped, transposed kernel)
__global__ void flip_weights_kernel(const uint16_t* __restrict__ w, uint16_t* __restrict__ wt, int cout, int cin,
                                    int taps) {
    const size_t n = (size_t)cout * cin * taps;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const int ci = (int)(i % cin);
        const int t = (int)((i / cin) % taps);
        const int co = (int)(i / ((size_t)cin * taps));
        wt[((size_t)ci * taps + (taps - 1 - t)) * cout + co] = w[i];
    }
}

// ---------------------------------------------------------------------------
// Weight gradient: dw[co][t][ci] += sum_v dz[v][co] x[v + off(t)][ci]
// GEMM rows = output channels, columns = input channels, reduction over 16
// voxels of one x-row per MFMA.  One wave: (co tile, ci tile, tap, rows).
// ---------------------------------------------------------------------------
struct WgradArgs {
    const uint16_t* dz;
    int cout;
    const uint16_t* x1;
    const uint16_t* x2;
    int c1, c2;
    float* dw;
    float* partial;  // per-row-chunk partial dw [chunks][cout][taps][cin], or null: atomics into dw
    int D, H, W, rows_per_wave;
};

template <int KS>
__global__ void __launch_bounds__(256) conv_wgrad_kernel(const WgradArgs a) {
    const int lane = threadIdx.x & 63;
    const long wave = (long)blockIdx.x * 4 + (threadIdx.x >> 6);
    constexpr int taps = KS * KS * KS;
    const int cin = a.c1 + a.c2;
    const int ntco = a.cout / 32, ntci = (cin + 31) / 32;
    const long nrows = (long)a.D * a.H;
    const long nchunks = (nrows + a.rows_per_wave - 1) / a.rows_per_wave;
    const long ntasks = (long)ntco * ntci * taps * nchunks;
    if (wave >= ntasks) return;
    const int cot = (int)(wave % ntco);
    long rest = wave / ntco;
    const int cit = (int)(rest % ntci);
    rest /= ntci;
    const int t = (int)(rest % taps);
    const long chunk = rest / taps;
    const int dz = t / (KS * KS) - KS / 2, dy = (t / KS) % KS - KS / 2, dx = t % KS - KS / 2;
    const int m = lane & 31, half = lane >> 5;
    const int co = cot * 32 + m;
    const int ci = cit * 32 + m;
    const bool ci_ok = ci < cin;
    const uint16_t* xs = ci < a.c1 ? a.x1 : a.x2;
    const int xc = ci < a.c1 ? a.c1 : a.c2;
    const int xci = ci < a.c1 ? ci : ci - a.c1;
    f32x16 acc;
    for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
    const long r0 = chunk * a.rows_per_wave;
    const long r1 = r0 + a.rows_per_wave < nrows ? r0 + a.rows_per_wave : nrows;
    for (long row = r0; row < r1; ++row) {
        const int zz = (int)(row / a.H), yy = (int)(row % a.H);
        const int z = zz + dz, y = yy + dy;
        const bool row_ok = z >= 0 && z < a.D && y >= 0 && y < a.H;
        const long vrow = row * a.W;                    // first voxel of the output row
        const long srow = ((long)z * a.H + y) * a.W;    // first voxel of the shifted input row
        for (int x0 = 0; x0 < a.W; x0 += 16) {
            bf16x8 av, bv;
            for (int i = 0; i < 8; ++i) {
                const int x = x0 + 8 * half + i;
                const bool xin = x < a.W;
                const uint16_t g = xin ? a.dz[(vrow + x) * a.cout + co] : (uint16_t)0;
                const int xs_ = x + dx;
                const bool sin = row_ok && xin && ci_ok && xs_ >= 0 && xs_ < a.W;
                const uint16_t v = sin ? xs[(srow + xs_) * xc + xci] : (uint16_t)0;
                av[i] = __builtin_bit_cast(__bf16, g);
                bv[i] = __builtin_bit_cast(__bf16, v);
            }
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc, 0, 0, 0);
        }
    }
    const int n = cit * 32 + m;  // input channel (column)
    if (n < cin) {
        for (int r = 0; r < 16; ++r) {
            const int mm = cot * 32 + 8 * (r >> 2) + 4 * half + (r & 3);  // output channel (row)
            if (a.partial)
                a.partial[((chunk * a.cout + mm) * taps + t) * cin + n] = acc[r];
            else
                atomicAdd(&a.dw[((long)mm * taps + t) * cin + n], acc[r]);
        }
    }
}

// db[c] += sum over voxels of dz[v][c]; with `partial`, block b stores its
// sum in partial[b][c] instead (summed in a fixed order afterwards)
__global__ void bias_grad_kernel(const uint16_t* __restrict__ dz, float* __restrict__ db, size_t nvox, int c,
                                 float* __restrict__ partial) {
    __shared__ float part[256];
    const int ch = blockIdx.y;
    float s = 0.0f;
    for (size_t v = blockIdx.x * (size_t)blockDim.x + threadIdx.x; v < nvox; v += (size_t)gridDim.x * blockDim.x)
        s += bf2f(dz[v * c + ch]);
    part[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (partial) partial[(size_t)blockIdx.x * c + ch] = part[0];
        else atomicAdd(&db[ch], part[0]);
    }
}

// out[i] += sum over p = 0 .. nparts-1, in that order, of partial[p][i]
__global__ void sum_partials_kernel(const float* __restrict__ partial, float* __restrict__ out, size_t n,
                                    int nparts) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        float s = 0.0f;
        for (int p = 0; p < nparts; ++p) s += partial[(size_t)p * n + i];
        out[i] += s;
    }
}

// ---------------------------------------------------------------------------
// Elementwise and resampling kernels (BF16 storage, FP32 arithmetic)
// ---------------------------------------------------------------------------
__global__ void relu_bwd_kernel(const uint16_t* __restrict__ dy, const uint16_t* __restrict__ y,
                                uint16_t* __restrict__ dz, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        dz[i] = bf2f(y[i]) > 0.0f ? dy[i] : (uint16_t)0;
}

__global__ void add_kernel(const uint16_t* __restrict__ a, const uint16_t* __restrict__ b, uint16_t* __restrict__ out,
                           size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        out[i] = f2bf(bf2f(a[i]) + bf2f(b[i]));
}

// 2x2x2 average pooling: out [D/2][H/2][W/2][C]
// One thread per output voxel and 8-channel group: eight 16-byte loads, one
// 16-byte store; every channel sums its 8 inputs in the same order.
__global__ void pool2_kernel(const uint16_t* __restrict__ x, uint16_t* __restrict__ y, int D, int H, int W, int C) {
    const int d = D / 2, h = H / 2, w = W / 2, cg = C / 8;
    const size_t n = (size_t)d * h * w * cg;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const int c8 = (int)(i % cg);
        size_t v = i / cg;
        const int xo = (int)(v % w), yo = (int)((v / w) % h), zo = (int)(v / ((size_t)w * h));
        float s[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) s[k] = 0.0f;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int z = 2 * zo + (q >> 2), yy = 2 * yo + ((q >> 1) & 1), xx = 2 * xo + (q & 1);
            const uint4 u = *(const uint4*)(x + (((size_t)z * H + yy) * W + xx) * C + 8 * c8);
            const uint32_t wd[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                s[2 * k] += bf2f((uint16_t)(wd[k] & 0xffffu));
                s[2 * k + 1] += bf2f((uint16_t)(wd[k] >> 16));
            }
        }
        uint32_t o[4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            o[k] = (uint32_t)f2bf(0.125f * s[2 * k]) | ((uint32_t)f2bf(0.125f * s[2 * k + 1]) << 16);
        *(uint4*)(y + v * C + 8 * c8) = make_uint4(o[0], o[1], o[2], o[3]);
    }
}

__global__ void pool2_bwd_kernel(const uint16_t* __restrict__ dy, uint16_t* __restrict__ dx, int D, int H, int W,
                                 int C) {
    const size_t n = (size_t)D * H * W * C;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % C);
        const size_t v = i / C;
        const int x = (int)(v % W), y = (int)((v / W) % H), z = (int)(v / ((size_t)W * H));
        dx[i] = f2bf(0.125f * bf2f(dy[((((size_t)(z / 2)) * (H / 2) + y / 2) * (W / 2) + x / 2) * C + c]));
    }
}

// nearest-neighbour 2x upsampling: out [2D][2H][2W][C]
__global__ void up2_kernel(const uint16_t* __restrict__ x, uint16_t* __restrict__ y, int D, int H, int W, int C) {
    const size_t n = (size_t)8 * D * H * W * C;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % C);
        const size_t v = i / C;
        const int W2 = 2 * W, H2 = 2 * H;
        const int xx = (int)(v % W2), yy = (int)((v / W2) % H2), zz = (int)(v / ((size_t)W2 * H2));
        y[i] = x[((((size_t)(zz / 2)) * H + yy / 2) * W + xx / 2) * C + c];
    }
}

__global__ void up2_bwd_kernel(const uint16_t* __restrict__ dy, uint16_t* __restrict__ dx, int D, int H, int W,
                               int C) {
    const size_t n = (size_t)D * H * W * C;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % C);
        const size_t v = i / C;
        const int x = (int)(v % W), y = (int)((v / W) % H), z = (int)(v / ((size_t)W * H));
        float s = 0.0f;
        for (int q = 0; q < 8; ++q) {
            const int zz = 2 * z + (q >> 2), yy = 2 * y + ((q >> 1) & 1), xx = 2 * x + (q & 1);
            s += bf2f(dy[(((size_t)zz * (2 * H) + yy) * (2 * W) + xx) * C + c]);
        }
        dx[i] = f2bf(s);
    }
}

// Residual output head and loss: pred[v][c] = out[v][c] + base[v][c] for the
// first nout channels of the FP32 network output (cpad channels per voxel);
// loss += sum (pred - target)^2 (FP64 accumulation); dout[v][c] =
// 2 (pred - target) / count as BF16 (0 for padding channels).
__global__ void mse_kernel(const float* __restrict__ out, int cpad, const float* __restrict__ base,
                           const float* __restrict__ target, int nout, size_t nvox, double inv_count,
                           float* __restrict__ pred, uint16_t* __restrict__ dout, double* __restrict__ loss) {
    __shared__ double part[256];
    double s = 0.0;
    const size_t n = nvox * cpad;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % cpad);
        const size_t v = i / cpad;
        float g = 0.0f;
        if (c < nout) {
            const float p = out[i] + base[v * nout + c];
            if (pred) pred[v * nout + c] = p;
            if (target) {
                const float d = p - target[v * nout + c];
                s += (double)d * d;
                g = (float)(2.0 * inv_count) * d;
            }
        }
        if (dout) dout[i] = f2bf(g);
    }
    part[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0 && loss) atomicAdd(loss, part[0]);
}

// Adam on FP32 master parameters, BF16 copy for the forward pass.
__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m1,
                            float* __restrict__ m2, uint16_t* __restrict__ pb, size_t n, float lr, float b1, float b2,
                            float eps, float c1, float c2) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float a = b1 * m1[i] + (1.0f - b1) * gi;
        const float b = b2 * m2[i] + (1.0f - b2) * gi * gi;
        m1[i] = a;
        m2[i] = b;
        const float v = p[i] - lr * (a * c1) / (sqrtf(b * c2) + eps);
        p[i] = v;
        if (pb) pb[i] = f2bf(v);
    }
}

__global__ void to_bf16_kernel(const float* __restrict__ x, uint16_t* __restrict__ y, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        y[i] = f2bf(x[i]);
}

// Input features per voxel: scaled direct and diffuse heating, log optical
// thickness for extinction and for absorption of the cell, zero padding to
// cpad channels (BF16); the scaled heating is also written as the FP32
// residual base [v][2].
__global__ void features_kernel(const float* __restrict__ hdir, const float* __restrict__ hdif,
                                const float* __restrict__ k_ext, const float* __restrict__ k_abs, float dz,
                                float inv_scale, size_t nvox, int cpad, const float* __restrict__ direct,
                                uint16_t* __restrict__ feat, float* __restrict__ base) {
    for (size_t v = blockIdx.x * (size_t)blockDim.x + threadIdx.x; v < nvox; v += (size_t)gridDim.x * blockDim.x) {
        const float a = hdir[v] * inv_scale, b = hdif[v] * inv_scale;
        uint16_t* f = feat + v * cpad;
        f[0] = f2bf(a);
        f[1] = f2bf(b);
        f[2] = f2bf(__logf(1.0f + 20.0f * k_ext[v] * dz));
        f[3] = f2bf(__logf(1.0f + 200.0f * k_abs[v] * dz));
        int q = 4;
        if (direct) f[q++] = f2bf(direct[v] * inv_scale);
        for (; q < cpad; ++q) f[q] = 0;
        if (base) {
            base[2 * v] = a;
            base[2 * v + 1] = b;
        }
    }
}

// Direct-beam feature: a deterministic estimate of the heating by the
// unscattered sun beam in a gray medium (flux-weighted extinction k_e and
// absorption k_a).  T[k][j][i], the beam's transmittance at the centre of
// cell (i, j, k), is carried down level by level: the ray through a centre,
// followed back up towards the sun by one level height, meets the level
// above at a point where that level's T is read bilinearly (periodic in x and
// y); the path between them runs half in each level.  In the top level the
// ray leaves through the domain top after half a level.  The cell absorbs
// T_entry (1 - exp(-k_e dz / mu0)) k_a / k_e of the direct flux, T_entry
// being the transmittance half a level above the centre; times the direct
// fraction of the flux and the level's heating-rate scale.  One launch per
// level, from the top: T of the level above is read from work[(k + 1) & 1],
// this level's written to work[k & 1].
struct DirectArgs {
    int nx, ny, nz;
    float sx, sy;       // horizontal offset of the point one level up, in cells
    float path;         // slant path of one level height (m): dz / mu0
    float fdir;         // direct fraction of the flux at the domain top
};

__global__ void direct_level_kernel(const DirectArgs d, int k, const float* __restrict__ ke,
                                    const float* __restrict__ ka, const double* __restrict__ scale,
                                    float* __restrict__ work, float* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
    if (i >= d.nx) return;
    const size_t plane = (size_t)d.nx * d.ny;
    const size_t c = (size_t)k * plane + (size_t)j * d.nx + i;
    const float kc = ke[c];
    float t;
    if (k == d.nz - 1) {
        t = __expf(-0.5f * kc * d.path);
    } else {
        const float* above = work + ((k + 1) & 1) * plane;
        const float fx = (float)i + d.sx, fy = (float)j + d.sy;
        const float x0 = floorf(fx), y0 = floorf(fy);
        const float wx = fx - x0, wy = fy - y0;
        auto wrap = [](int v, int n) { v %= n; return v < 0 ? v + n : v; };
        const int i0 = wrap((int)x0, d.nx), i1 = wrap((int)x0 + 1, d.nx);
        const int j0 = wrap((int)y0, d.ny), j1 = wrap((int)y0 + 1, d.ny);
        const float tu = (1.0f - wy) * ((1.0f - wx) * above[(size_t)j0 * d.nx + i0] + wx * above[(size_t)j0 * d.nx + i1]) +
                         wy * ((1.0f - wx) * above[(size_t)j1 * d.nx + i0] + wx * above[(size_t)j1 * d.nx + i1]);
        const int im = wrap((int)floorf((float)i + 0.5f + 0.5f * d.sx), d.nx);
        const int jm = wrap((int)floorf((float)j + 0.5f + 0.5f * d.sy), d.ny);
        const float ku = ke[(size_t)(k + 1) * plane + (size_t)jm * d.nx + im];  // the level above, mid-way
        t = tu * __expf(-0.5f * (kc + ku) * d.path);
    }
    work[(k & 1) * plane + (size_t)j * d.nx + i] = t;
    const float tau = kc * d.path;
    const float absorbed = kc > 0.0f ? t * __expf(0.5f * tau) * -expm1f(-tau) * (ka[c] / kc) : 0.0f;
    out[c] = (float)((double)(d.fdir * absorbed) * scale[k]);
}

// Sums of two FP32 fields in FP64, in a fixed order: per-block partial sums
// over a fixed grid of kSumBlocks blocks, then one block over the partials.
constexpr int kSumBlocks = 1024;

__global__ void field_sum_kernel(const float* __restrict__ a, const float* __restrict__ b, size_t n,
                                 double* __restrict__ partial) {
    __shared__ double sa[256], sb[256];
    double xa = 0.0, xb = 0.0;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        xa += (double)a[i];
        xb += (double)b[i];
    }
    sa[threadIdx.x] = xa;
    sb[threadIdx.x] = xb;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            sa[threadIdx.x] += sa[threadIdx.x + h];
            sb[threadIdx.x] += sb[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = sa[0];
        partial[2 * blockIdx.x + 1] = sb[0];
    }
}

// scale = (mean a + mean b) / 2, or 1 if that is not positive
__global__ void field_scale_kernel(const double* __restrict__ partial, size_t n, double* __restrict__ scale) {
    __shared__ double sa[256], sb[256];
    double xa = 0.0, xb = 0.0;
    for (int k = threadIdx.x; k < kSumBlocks; k += 256) {
        xa += partial[2 * k];
        xb += partial[2 * k + 1];
    }
    sa[threadIdx.x] = xa;
    sb[threadIdx.x] = xb;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            sa[threadIdx.x] += sa[threadIdx.x + h];
            sb[threadIdx.x] += sb[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double m = (sa[0] / (double)n + sb[0] / (double)n) / 2.0;
        scale[0] = m > 0.0 ? m : 1.0;
    }
}

// a * b rounded to FP32 on its own: the library is built with FP contraction,
// which would otherwise fuse it with a following addition into one FMA (and
// the backend does so even where the source forbids it)
__device__ __forceinline__ float mul_rounded(float a, float b) {
    float r;
    asm("v_mul_f32 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

// Inference: the residual head and the split back into heating fields in one
// pass, hdir[v] = max(out[v][0] + hdir_in[v] / scale, 0) scale (and hdif
// alike), with the division as features_kernel forms it (times the FP32
// reciprocal, rounded before the addition), so the result is bitwise that of
// features_kernel's base, mse_kernel and unfeature_kernel in turn.
__global__ void residual_unfeature_kernel(const float* __restrict__ out, int cpad, const float* __restrict__ hdir_in,
                                          const float* __restrict__ hdif_in, float inv_scale, float scale, size_t nvox,
                                          float* __restrict__ hdir, float* __restrict__ hdif) {
    for (size_t v = blockIdx.x * (size_t)blockDim.x + threadIdx.x; v < nvox; v += (size_t)gridDim.x * blockDim.x) {
        const float p0 = out[v * cpad] + mul_rounded(hdir_in[v], inv_scale);
        const float p1 = out[v * cpad + 1] + mul_rounded(hdif_in[v], inv_scale);
        hdir[v] = fmaxf(p0, 0.0f) * scale;
        hdif[v] = fmaxf(p1, 0.0f) * scale;
    }
}

// Split a [v][2] prediction back into heating fields, times scale, >= 0.
__global__ void unfeature_kernel(const float* __restrict__ pred, float scale, size_t nvox, float* __restrict__ hdir,
                                 float* __restrict__ hdif) {
    for (size_t v = blockIdx.x * (size_t)blockDim.x + threadIdx.x; v < nvox; v += (size_t)gridDim.x * blockDim.x) {
        hdir[v] = fmaxf(pred[2 * v], 0.0f) * scale;
        hdif[v] = fmaxf(pred[2 * v + 1], 0.0f) * scale;
    }
}

}  // namespace

// ===========================================================================
// C ABI (include/rt3d_denoise.h)
// ===========================================================================
extern "C" {

const char* rt3d_dn_last_error(void) { return d_err; }

rt3d_status rt3d_dn_conv3d_fwd_pool(const rt3d_dn_conv* c, const uint16_t* x1, const uint16_t* w, const float* bias,
                                    int32_t relu, uint16_t* y, uint16_t* ypool, void* stream) {
    if (!c || !x1 || !w || !y || !ypool) return RT3D_EINVAL;
    if ((c->c1 != 4 && c->c1 != 5) || c->c2 != 0 || c->ksize != 3 || c->cout != 32 || c->up1 || c->yf_cols)
        return RT3D_EINVAL;
    if (c->D <= 0 || c->H <= 0 || c->W <= 0 || c->D % 2 || c->H % 2 || c->W % 2) return RT3D_EINVAL;
    ConvArgs a;
    memset(&a, 0, sizeof a);
    a.x1 = x1; a.c1 = c->c1; a.w = w; a.bias = bias; a.y1 = y; a.o1 = 32;
    a.D = c->D; a.H = c->H; a.W = c->W; a.cout = 32; a.relu = relu ? 1 : 0;
    const long tiles = (long)(c->D / 2) * ((c->H + kTY32 - 1) / kTY32) * ((c->W + kTX - 1) / kTX);
    if (tiles > 0x7fffffffL) return RT3D_EINVAL;
    if (c->c1 == 4)
        hipLaunchKernelGGL(conv3_c4_pool_kernel, dim3((unsigned)tiles), dim3(256), 0, (hipStream_t)stream, a, ypool);
    else
        hipLaunchKernelGGL(conv3_c5_pool_kernel, dim3((unsigned)tiles), dim3(256), 0, (hipStream_t)stream, a, ypool);
    DN_TRY(hipGetLastError());
    return RT3D_OK;
}

rt3d_status rt3d_dn_conv3d_fwd(const rt3d_dn_conv* c, const uint16_t* x1, const uint16_t* x2, const uint16_t* w,
                               const float* bias, int32_t relu, uint16_t* y1, uint16_t* y2, int32_t o1, float* yf,
                               void* stream) {
    if (!c || !x1 || !w || (c->c2 > 0 && !x2) || (!y1 && !yf)) return RT3D_EINVAL;
    // 4 input channels: only the first layer's packed form
    const bool four = c->c1 == 4 && c->c2 == 0 && c->ksize == 3 && c->cout == 32 && !c->up1 && o1 == 32;
    if (c->D <= 0 || c->H <= 0 || c->W <= 0 || c->c1 <= 0 || (c->c1 % 16 && !four) || c->c2 < 0 || c->c2 % 16)
        return RT3D_EINVAL;
    if (c->cout <= 0 || c->cout % 32 || (c->ksize != 1 && c->ksize != 3)) return RT3D_EINVAL;
    if (o1 <= 0 || o1 > c->cout || o1 % 32 || (o1 < c->cout && !y2)) return RT3D_EINVAL;
    if (c->up1 && (c->ksize != 3 || c->D % 2 || c->H % 2 || c->W % 2)) return RT3D_EINVAL;
    if (c->yf_cols < 0 || c->yf_cols > c->cout) return RT3D_EINVAL;
    ConvArgs a;
    a.x1 = x1; a.x2 = x2; a.c1 = c->c1; a.c2 = c->c2; a.w = w; a.bias = bias;
    a.y1 = y1; a.y2 = y2; a.o1 = o1; a.yf = yf;
    a.D = c->D; a.H = c->H; a.W = c->W; a.cout = c->cout; a.relu = relu ? 1 : 0;
    a.up1 = c->up1 ? 1 : 0;
    a.yf_cols = c->yf_cols ? c->yf_cols : c->cout;
    a.hw = nullptr; a.hb = nullptr; a.hy = nullptr; a.hcols = 0;
    if (four) {
        const long tiles = (long)c->D * ((c->H + kTY32 - 1) / kTY32) * ((c->W + kTX - 1) / kTX);
        if (tiles > 0x7fffffffL) return RT3D_EINVAL;
        hipLaunchKernelGGL(conv3_c4_kernel, dim3((unsigned)tiles), dim3(256), 0, (hipStream_t)stream, a);
    } else if (c->ksize == 3 && c->cout == 32) {
        const long tiles = (long)((c->D + kZ32 - 1) / kZ32) * ((c->H + kTY32 - 1) / kTY32) * ((c->W + kTX - 1) / kTX);
        if (tiles > 0x7fffffffL) return RT3D_EINVAL;
        hipLaunchKernelGGL(conv3_c32_kernel, dim3((unsigned)tiles), dim3(256), 0, (hipStream_t)stream, a);
    } else if (c->ksize == 3) {
        const long tiles =
            (long)((c->D + kZ - 1) / kZ) * ((c->H + kTY - 1) / kTY) * ((c->W + kTX - 1) / kTX) * ((c->cout + 63) / 64);
        if (tiles > 0x7fffffffL) return RT3D_EINVAL;
        hipLaunchKernelGGL(conv3_tiled_kernel, dim3((unsigned)tiles), dim3(256), 0, (hipStream_t)stream, a);
    } else {
        const long waves = (long)c->D * c->H * ((c->W + 31) / 32) * (c->cout / 32);
        const unsigned blocks = (unsigned)((waves + 3) / 4);
        hipLaunchKernelGGL(conv_fwd_kernel<1>, dim3(blocks), dim3(256), 0, (hipStream_t)stream, a);
    }
    DN_TRY(hipGetLastError());
    return RT3D_OK;
}

rt3d_status rt3d_dn_conv3d_fwd_head(const rt3d_dn_conv* c, const uint16_t* x1, const uint16_t* x2, const uint16_t* w,
                                    const float* bias, int32_t relu, const uint16_t* hw, const float* hb, int32_t hcols,
                                    float* hy, void* stream) {
    if (!c || !x1 || !w || (c->c2 > 0 && !x2) || !hw || !hy) return RT3D_EINVAL;
    if (c->D <= 0 || c->H <= 0 || c->W <= 0 || c->c1 <= 0 || c->c1 % 16 || c->c2 < 0 || c->c2 % 16)
        return RT3D_EINVAL;
    if (c->ksize != 3 || c->cout != 32 || hcols <= 0 || hcols > 32) return RT3D_EINVAL;
    if (c->up1 && (c->D % 2 || c->H % 2 || c->W % 2)) return RT3D_EINVAL;
    ConvArgs a;
    a.x1 = x1; a.x2 = x2; a.c1 = c->c1; a.c2 = c->c2; a.w = w; a.bias = bias;
    a.y1 = nullptr; a.y2 = nullptr; a.o1 = 32; a.yf = nullptr;
    a.D = c->D; a.H = c->H; a.W = c->W; a.cout = 32; a.relu = relu ? 1 : 0;
    a.up1 = c->up1 ? 1 : 0;
    a.yf_cols = 32;
    a.hw = hw; a.hb = hb; a.hy = hy; a.hcols = hcols;
    const long tiles = (long)((c->D + kZ32 - 1) / kZ32) * ((c->H + kTY32 - 1) / kTY32) * ((c->W + kTX - 1) / kTX);
    if (tiles > 0x7fffffffL) return RT3D_EINVAL;
    hipLaunchKernelGGL(conv3_c32_kernel, dim3((unsigned)tiles), dim3(256), 0, (hipStream_t)stream, a);
    DN_TRY(hipGetLastError());
    return RT3D_OK;
}

rt3d_status rt3d_dn_flip_weights(const uint16_t* w, uint16_t* wt, int32_t cout, int32_t cin, int32_t ksize,
                                 void* stream) {
    if (!w || !wt || cout <= 0 || cin <= 0 || (ksize != 1 && ksize != 3)) return RT3D_EINVAL;
    const int taps = ksize * ksize * ksize;
    hipLaunchKernelGGL(flip_weights_kernel, dim3(blocks_for((size_t)cout * cin * taps)), dim3(256), 0,
                       (hipStream_t)stream, w, wt, cout, cin, taps);
    DN_TRY(hipGetLastError());
    return RT3D_OK;
}

}  // extern "C"

namespace {

// Launch plan of the weight gradient: the (output tile, input tile, tap)
// tasks are split over row chunks so that about 4096 waves are in flight.
struct WgradPlan {
    WgradArgs a;
    long chunks, waves;
    int taps;
    size_t nw;            // cout * taps * cin
    unsigned bias_blocks; // blocks per channel of the bias gradient
    size_t ws_bytes;      // workspace of the deterministic variant
};

bool wgrad_plan(const rt3d_dn_conv* c, WgradPlan* p) {
    if (!c || c->up1) return false;
    if (c->D <= 0 || c->H <= 0 || c->W <= 0 || c->c1 <= 0 || c->c1 % 16 || c->c2 < 0 || c->c2 % 16) return false;
    if (c->cout <= 0 || c->cout % 32 || (c->ksize != 1 && c->ksize != 3)) return false;
    WgradArgs& a = p->a;
    a.cout = c->cout; a.c1 = c->c1; a.c2 = c->c2;
    a.D = c->D; a.H = c->H; a.W = c->W;
    a.partial = nullptr;
    p->taps = c->ksize * c->ksize * c->ksize;
    const long base_tasks = (long)(c->cout / 32) * ((c->c1 + c->c2 + 31) / 32) * p->taps;
    const long nrows = (long)c->D * c->H;
    long chunks = 4096 / base_tasks;
    if (chunks < 1) chunks = 1;
    if (chunks > nrows) chunks = nrows;
    a.rows_per_wave = (int)((nrows + chunks - 1) / chunks);
    p->chunks = (nrows + a.rows_per_wave - 1) / a.rows_per_wave;
    p->waves = base_tasks * p->chunks;
    p->nw = (size_t)c->cout * p->taps * (c->c1 + c->c2);
    const size_t nvox = (size_t)c->D * c->H * c->W;
    p->bias_blocks = blocks_for(nvox, 256, 256);
    p->ws_bytes = ((p->chunks * p->nw * sizeof(float) + 255) / 256) * 256 +
                  (size_t)p->bias_blocks * c->cout * sizeof(float);
    return true;
}

rt3d_status wgrad_run(const rt3d_dn_conv* c, const WgradPlan& plan, const uint16_t* x1, const uint16_t* x2,
                      const uint16_t* dz, float* dw, float* db, float* part_w, float* part_b, hipStream_t st) {
    WgradArgs a = plan.a;
    a.dz = dz; a.x1 = x1; a.x2 = x2; a.dw = dw; a.partial = part_w;
    const unsigned blocks = (unsigned)((plan.waves + 3) / 4);
    if (c->ksize == 3)
        hipLaunchKernelGGL(conv_wgrad_kernel<3>, dim3(blocks), dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL(conv_wgrad_kernel<1>, dim3(blocks), dim3(256), 0, st, a);
    DN_TRY(hipGetLastError());
    if (part_w) {
        hipLaunchKernelGGL(sum_partials_kernel, dim3(blocks_for(plan.nw)), dim3(256), 0, st, part_w, dw, plan.nw,
                           (int)plan.chunks);
        DN_TRY(hipGetLastError());
    }
    if (db) {
        const size_t nvox = (size_t)c->D * c->H * c->W;
        hipLaunchKernelGGL(bias_grad_kernel, dim3(plan.bias_blocks, c->cout), dim3(256), 0, st, dz, db, nvox,
                           c->cout, part_b);
        DN_TRY(hipGetLastError());
        if (part_b) {
            hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(256), 0, st, part_b, db, (size_t)c->cout,
                               (int)plan.bias_blocks);
            DN_TRY(hipGetLastError());
        }
    }
    return RT3D_OK;
}

}  // namespace

extern "C" {

rt3d_status rt3d_dn_conv3d_wgrad(const rt3d_dn_conv* c, const uint16_t* x1, const uint16_t* x2, const uint16_t* dz,
                                 float* dw, float* db, void* stream) {
    WgradPlan plan;
    if (!x1 || !dz || !dw || (c && c->c2 > 0 && !x2) || !wgrad_plan(c, &plan)) return RT3D_EINVAL;
    return wgrad_run(c, plan, x1, x2, dz, dw, db, nullptr, nullptr, (hipStream_t)stream);
}

size_t rt3d_dn_wgrad_workspace_size(const rt3d_dn_conv* c) {
    WgradPlan plan;
    return wgrad_plan(c, &plan) ? plan.ws_bytes : 0;
}

rt3d_status rt3d_dn_conv3d_wgrad_ws(const rt3d_dn_conv* c, const uint16_t* x1, const uint16_t* x2,
                                    const uint16_t* dz, float* dw, float* db, void* workspace,
                                    size_t workspace_bytes, void* stream) {
    WgradPlan plan;
    if (!x1 || !dz || !dw || (c && c->c2 > 0 && !x2) || !wgrad_plan(c, &plan)) return RT3D_EINVAL;
    if (!workspace || workspace_bytes < plan.ws_bytes || ((uintptr_t)workspace & 255)) return RT3D_EINVAL;
    float* part_w = (float*)workspace;
    float* part_b = (float*)((char*)workspace + ((plan.chunks * plan.nw * sizeof(float) + 255) / 256) * 256);
    return wgrad_run(c, plan, x1, x2, dz, dw, db, part_w, part_b, (hipStream_t)stream);
}

rt3d_status rt3d_dn_relu_bwd(const uint16_t* dy, const uint16_t* y, uint16_t* dz, uint64_t n, void* stream) {
    if (!dy || !y || !dz) return RT3D_EINVAL;
    hipLaunchKernelGGL(relu_bwd_kernel, dim3(blocks_for(n)), dim3(256), 0, (hipStream_t)stream, dy, y, dz, (size_t)n);
    DN_TRY(hipGetLastError());
    return RT3D_OK;
}

rt3d_status rt3d_dn_add(const uint16_t* a, const uint16_t* b, uint16_t* out, uint64_t n, void* stream) {
    if (!a || !b || !out) return RT3D_EINVAL;
    hipLaunchKernelGGL(add_kernel, dim3(blocks_for(n)), dim3(256), 0, (hipStream_t)stream, a, b, out, (size_t)n);
    DN_TRY(hipGetLastError());
    return RT3D_OK;
}

rt3d_status rt3d_dn_pool2(const uint16_t* x, uint16_t* y, int32_t D, int32_t H, int32_t W, int32_t C, int32_t backward,
                          void* stream) {
    if (!x || !y || D <= 0 || H <= 0 || W <= 0 || C <= 0 || D % 2 || H % 2 || W % 2) return RT3D_EINVAL;
    const size_t n = (size_t)D * H * W * C;
    if (backward) {
        hipLaunchKernelGGL(pool2_bwd_kernel, dim3(blocks_for(n)), dim3(256), 0, (hipStream_t)stream, x, y, D, H, W, C);
    } else {
        // 16-byte accesses: 8-channel groups, aligned tensors
        if (C % 8 || ((uintptr_t)x | (uintptr_t)y) % 16) return RT3D_EINVAL;
        hipLaunchKernelGGL(pool2_kernel, dim3(blocks_for(n / 64)), dim3(256), 0, (hipStream_t)stream, x, y, D, H, W, C);
    }
    DN_TRY(hipGetLastError());
    return RT3D_OK;
}

rt3d_status rt3d_dn_up2(const uint16_t* x, uint16_t* y, int32_t D, int32_t H, int32_t W, int32_t C, int32_t backward,
                        void* stream) {
    if (!x || !y || D <= 0 || H <= 0 || W <= 0 || C <= 0) return RT3D_EINVAL;
    const size_t n = (size_t)D * H * W * C;
    if (backward)
        hipLaunchKernelGGL(up2_bwd_kernel, dim3(blocks_for(n)), dim3(256), 0, (hipStream_t)stream, x, y, D, H, W, C);
    else
        hipLaunchKernelGGL(up2_kernel, dim3(blocks_for(8 * n)), dim3(256), 0, (hipStream_t)stream, x, y, D, H, W, C);
    DN_TRY(hipGetLastError());
    return RT3D_OK;
}

rt3d_status rt3d_dn_mse(const float* out, int32_t cpad, const float* base, const float* target, int32_t nout,
                        uint64_t nvox, float* pred, uint16_t* dout, double* loss, void* stream) {
    if (!out || !base || cpad <= 0 || nout <= 0 || nout > cpad || nvox == 0) return RT3D_EINVAL;
    if ((dout || loss) && !target) return RT3D_EINVAL;
    const double inv = 1.0 / ((double)nvox * nout);
    hipLaunchKernelGGL(mse_kernel, dim3(blocks_for((size_t)nvox * cpad, 256, 4096)), dim3(256), 0,
                       (hipStream_t)stream, out, cpad, base, target, nout, (size_t)nvox, inv, pred, dout, loss);
    DN_TRY(hipGetLastError());
    return RT3D_OK;
}

rt3d_status rt3d_dn_adam(float* p, const float* g, float* m1, float* m2, uint16_t* pb, uint64_t n, float lr, float b1,
                         float b2, float eps, int32_t step, void* stream) {
    if (!p || !g || !m1 || !m2 || step < 1) return RT3D_EINVAL;
    const float c1 = 1.0f / (1.0f - powf(b1, (float)step)), c2 = 1.0f / (1.0f - powf(b2, (float)step));
    hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(n)), dim3(256), 0, (hipStream_t)stream, p, g, m1, m2, pb,
                       (size_t)n, lr, b1, b2, eps, c1, c2);
    DN_TRY(hipGetLastError());
    return RT3D_OK;
}

rt3d_status rt3d_dn_to_bf16(const float* x, uint16_t* y, uint64_t n, void* stream) {
    if (!x || !y) return RT3D_EINVAL;
    hipLaunchKernelGGL(to_bf16_kernel, dim3(blocks_for(n)), dim3(256), 0, (hipStream_t)stream, x, y, (size_t)n);
    DN_TRY(hipGetLastError());
    return RT3D_OK;
}

rt3d_status rt3d_dn_features(const float* hdir, const float* hdif, const float* k_ext, const float* k_abs, float dz,
                             float scale, uint64_t nvox, int32_t cpad, const float* direct, uint16_t* feat, float* base,
                             void* stream) {
    if (!hdir || !hdif || !k_ext || !k_abs || !feat || (cpad != 4 && cpad != 8 && (cpad < 16 || cpad % 16)) ||
        !(scale > 0.0f))
        return RT3D_EINVAL;
    if (direct && cpad < 5) return RT3D_EINVAL;
    hipLaunchKernelGGL(features_kernel, dim3(blocks_for(nvox)), dim3(256), 0, (hipStream_t)stream, hdir, hdif, k_ext,
                       k_abs, dz, 1.0f / scale, (size_t)nvox, cpad, direct, feat, base);
    DN_TRY(hipGetLastError());
    return RT3D_OK;
}

rt3d_status rt3d_dn_unfeature(const float* pred, float scale, uint64_t nvox, float* hdir, float* hdif,
                              void* stream) {
    if (!pred || !hdir || !hdif) return RT3D_EINVAL;
    hipLaunchKernelGGL(unfeature_kernel, dim3(blocks_for(nvox)), dim3(256), 0, (hipStream_t)stream, pred, scale,
                       (size_t)nvox, hdir, hdif);
    DN_TRY(hipGetLastError());
    return RT3D_OK;
}

rt3d_status rt3d_dn_field_scale(const float* hdir, const float* hdif, uint64_t nvox, double* work, void* stream) {
    if (!hdir || !hdif || !work || nvox == 0) return RT3D_EINVAL;
    hipLaunchKernelGGL(field_sum_kernel, dim3(kSumBlocks), dim3(256), 0, (hipStream_t)stream, hdir, hdif,
                       (size_t)nvox, work + 1);
    DN_TRY(hipGetLastError());
    hipLaunchKernelGGL(field_scale_kernel, dim3(1), dim3(256), 0, (hipStream_t)stream, work + 1, (size_t)nvox, work);
    DN_TRY(hipGetLastError());
    return RT3D_OK;
}

rt3d_status rt3d_dn_residual_unfeature(const float* out, int32_t cpad, const float* hdir_in, const float* hdif_in,
                                       float scale, uint64_t nvox, float* hdir, float* hdif, void* stream) {
    if (!out || !hdir_in || !hdif_in || !hdir || !hdif || cpad < 2 || !(scale > 0.0f)) return RT3D_EINVAL;
    hipLaunchKernelGGL(residual_unfeature_kernel, dim3(blocks_for(nvox)), dim3(256), 0, (hipStream_t)stream, out,
                       cpad, hdir_in, hdif_in, 1.0f / scale, scale, (size_t)nvox, hdir, hdif);
    DN_TRY(hipGetLastError());
    return RT3D_OK;
}

rt3d_status rt3d_dn_direct_feature(const rt3d_dn_direct* d, const float* k_ext, const float* k_abs,
                                   const double* layer_scale, float* out, float* work, void* stream) {
    if (!d || !k_ext || !k_abs || !layer_scale || !out || !work) return RT3D_EINVAL;
    if (d->nx <= 0 || d->ny <= 0 || d->nz <= 0 || !(d->dx > 0.f) || !(d->dy > 0.f) || !(d->dz > 0.f)) return RT3D_EINVAL;
    if (!(d->sun_z < 0.f) || !(d->direct_fraction >= 0.f && d->direct_fraction <= 1.f)) return RT3D_EINVAL;
    DirectArgs a;
    const float up = d->dz / -d->sun_z;  // path length of one level height, followed back towards the sun
    a.nx = d->nx; a.ny = d->ny; a.nz = d->nz;
    a.sx = -d->sun_x * up / d->dx;
    a.sy = -d->sun_y * up / d->dy;
    a.path = up;
    a.fdir = d->direct_fraction;
    const dim3 grid((unsigned)((d->nx + 255) / 256), (unsigned)d->ny);
    for (int k = d->nz - 1; k >= 0; --k) {
        hipLaunchKernelGGL(direct_level_kernel, grid, dim3(256), 0, (hipStream_t)stream, a, k, k_ext, k_abs,
                           layer_scale, work, out);
        DN_TRY(hipGetLastError());
    }
    return RT3D_OK;
}

}  // extern "C"
