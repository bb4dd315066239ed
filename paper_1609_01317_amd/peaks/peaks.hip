// Peak-rate probes timed by the benchmark beside the datasheet peaks: the
// FP32 FMA rate that code built like the raycaster (no packed FP32) reaches,
// and the read rate of a buffer that stays in the L2 caches.  Not part of
// the raycaster's library.
#include <hip/hip_runtime.h>

namespace {

constexpr int kChains = 16;

// kChains independent FMA chains per lane, iters steps each: 2 * kChains *
// iters flops per lane.  The sum is stored so nothing is dead code.
__global__ __launch_bounds__(256) void fma_loop(float* __restrict__ out, int iters, float a,
                                                float b) {
    float x[kChains];
#pragma unroll
    for (int i = 0; i < kChains; ++i) x[i] = (float)threadIdx.x * 1e-3f + (float)i;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < kChains; ++i) x[i] = fmaf(x[i], a, b);
    }
    float s = 0.0f;
#pragma unroll
    for (int i = 0; i < kChains; ++i) s += x[i];
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// Each workgroup reads one 4 KiB chunk (256 lanes x float4) per repetition:
// chunk (block + rep * (grid + 1)) mod nchunks, a power of two.  Over the
// repetitions every workgroup walks the whole buffer, so a compute unit's L1
// keeps missing and the reads land in L2 (small buffer) or HBM (large one).
__global__ __launch_bounds__(256) void read_loop(const float4* __restrict__ src, int chunk_mask,
                                                 int reps, float* __restrict__ out) {
    const int step = gridDim.x + 1;
    float ax = 0.0f, ay = 0.0f, az = 0.0f, aw = 0.0f;
#pragma unroll 8
    for (int r = 0; r < reps; ++r) {
        const long long chunk = ((long long)blockIdx.x + (long long)r * step) & chunk_mask;
        float4 v = src[chunk * 256 + threadIdx.x];
        ax += v.x; ay += v.y; az += v.z; aw += v.w;
    }
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = ax + ay + az + aw;
}

}  // namespace

// out: device, blocks * 256 floats.  Returns 0, or the HIP error code.
extern "C" int pk_fma(float* out, int blocks, int iters, void* stream) {
    if (!out || blocks < 1 || iters < 1) return (int)hipErrorInvalidValue;
    hipLaunchKernelGGL(fma_loop, dim3(blocks), dim3(256), 0, (hipStream_t)stream, out, iters,
                       0.999f, 1e-3f);
    return (int)hipGetLastError();
}

// src: device, bytes (a power of two, 4 KiB to 4 TiB); out: device, blocks *
// 256 floats.  Reads blocks * reps * 4 KiB.
extern "C" int pk_read(const void* src, long long bytes, int blocks, int reps, float* out,
                       void* stream) {
    if (!src || !out || bytes < 4096 || (bytes & (bytes - 1)) || bytes / 4096 > (1LL << 30) ||
        blocks < 1 || reps < 1)
        return (int)hipErrorInvalidValue;
    hipLaunchKernelGGL(read_loop, dim3(blocks), dim3(256), 0, (hipStream_t)stream,
                       (const float4*)src, (int)(bytes / 4096 - 1), reps, out);
    return (int)hipGetLastError();
}
