// oz_peak.hip -- microbenchmarks of the rates a roofline report divides by:
// INT8 matrix-core throughput (the instruction the slice GEMM runs on), FP64
// matrix-core throughput (what a native DGEMM / ZGEMM runs on), and HBM copy
// bandwidth (what the split and epilogue passes stream through).
//
// The MFMA kernels (INT8 in the 32 x 32 x 32 shape the slice GEMM uses, also
// with changing full-range operands, and in the 16 x 16 x 64 shape) keep
// kChains independent accumulators per wave and issue the instruction
// round-robin over them, so consecutive instructions never
// depend on each other and one wave keeps its SIMD's matrix pipe fed (the
// 32 x 32 x 32 kernel's 8 chains take 128 accumulator registers, so one wave
// per SIMD is resident and the second block per CU runs after the first).
// The operands come from the lane index (not foldable), and every
// accumulator feeds one value stored per lane, so nothing is dead code.
#include <hip/hip_runtime.h>

#include "../../include/oz.h"
#include "oz_handle.h"
#include "oz_internal.h"

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kChains = 8;
constexpr int kPeakThreads = 256;  // 4 waves per block
constexpr int kBlocksPerCu = 2;    // 8 waves per compute unit

// TOGGLE = false: one operand pair of bytes at most 63, the same for every
// instruction.  TOGGLE = true: two pairs of full-range pseudo-random bytes
// (a splitmix64 hash of lane and register), used by alternate instructions, so
// that consecutive MFMAs see different data as in a GEMM over random digits
// (the matrix cores' power, and with it the clock, depends on the data).
__device__ __forceinline__ int peak_bytes(uint64_t key) {
    key += 0x9E3779B97F4A7C15ull;
    key = (key ^ (key >> 30)) * 0xBF58476D1CE4E5B9ull;
    key = (key ^ (key >> 27)) * 0x94D049BB133111EBull;
    return static_cast<int>((key ^ (key >> 31)) & 0xffffffffull);
}

template <bool TOGGLE>
__global__ __launch_bounds__(kPeakThreads) void peak_i8_kernel(int64_t iters, int* out) {
    const int lane = threadIdx.x & 63;
    v4i a[2], b[2];
    for (int q = 0; q < 2; ++q)
        for (int r = 0; r < 4; ++r) {
            if (TOGGLE) {
                a[q][r] = peak_bytes(static_cast<uint64_t>(((q * 4 + r) * 2) * 64 + lane));
                b[q][r] = peak_bytes(static_cast<uint64_t>(((q * 4 + r) * 2 + 1) * 64 + lane));
            } else {
                a[q][r] = (lane * 0x01030507 + r) & 0x3f3f3f3f;
                b[q][r] = (lane * 0x07050301 + 3 * r) & 0x3f3f3f3f;
            }
        }
    v16i acc[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[c][r] = 0;
    for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) {
            const int q = TOGGLE ? (c & 1) : 0;
            acc[c] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[q], b[q], acc[c], 0, 0, 0);
        }
    }
    int sum = 0;
#pragma unroll
    for (int c = 0; c < kChains; ++c)
#pragma unroll
        for (int r = 0; r < 16; ++r) sum += acc[c][r];
    out[blockIdx.x * kPeakThreads + threadIdx.x] = sum;
}

// the 16 x 16 x 64 INT8 shape: 4 lanes' 16 bytes form a 64-term row, 4 INT32
// results per lane
__global__ __launch_bounds__(kPeakThreads) void peak_i8_16_kernel(int64_t iters, int* out) {
    const int lane = threadIdx.x & 63;
    v4i a, b;
    for (int r = 0; r < 4; ++r) {
        a[r] = (lane * 0x01030507 + r) & 0x3f3f3f3f;
        b[r] = (lane * 0x07050301 + 3 * r) & 0x3f3f3f3f;
    }
    v4i acc[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[c][r] = 0;
    for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) acc[c] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, acc[c], 0, 0, 0);
    }
    int sum = 0;
#pragma unroll
    for (int c = 0; c < kChains; ++c)
#pragma unroll
        for (int r = 0; r < 4; ++r) sum += acc[c][r];
    out[blockIdx.x * kPeakThreads + threadIdx.x] = sum;
}

__global__ __launch_bounds__(kPeakThreads) void peak_f64_kernel(int64_t iters, double* out) {
    const int lane = threadIdx.x & 63;
    const double a = 1.0 + lane * 0x1p-20, b = 1.0 - lane * 0x1p-21;
    v4d acc[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[c][r] = 0.0;
    for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
    }
    double sum = 0.0;
#pragma unroll
    for (int c = 0; c < kChains; ++c)
#pragma unroll
        for (int r = 0; r < 4; ++r) sum += acc[c][r];
    out[blockIdx.x * kPeakThreads + threadIdx.x] = sum;
}

// 16 bytes per lane per step, grid-stride over n16 chunks
__global__ __launch_bounds__(256) void copy_kernel(const uint4* __restrict__ src, uint4* __restrict__ dst, int64_t n16) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n16; i += stride)
        dst[i] = src[i];
}

}  // namespace

extern "C" {

int oz_peak(oz_handle_t h, int kind, int64_t iters, const void* src, void* dst, size_t bytes, double* rate) {
    if (!oz_handle_valid(h)) return OZ_ERR_HANDLE;
    if (kind < 0 || kind > 4 || iters < 1 || !rate) return OZ_ERR_ARG;
    if (kind == 2 && (!src || !dst || bytes == 0 || bytes % 16 != 0)) return OZ_ERR_ARG;
    if (oz_handle_use_device(h)) return OZ_ERR_HIP;
    hipStream_t st = oz_handle_stream(h);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, oz_handle_device(h)) != hipSuccess) return OZ_ERR_HIP;
    const int blocks = prop.multiProcessorCount * kBlocksPerCu;
    void* out = nullptr;
    if (kind != 2 && hipMalloc(&out, sizeof(double) * blocks * kPeakThreads) != hipSuccess) return OZ_ERR_ALLOC;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    auto launch = [&](int64_t n) {
        if (kind == 0)
            hipLaunchKernelGGL(peak_i8_kernel<false>, dim3(blocks), dim3(kPeakThreads), 0, st, n,
                               static_cast<int*>(out));
        else if (kind == 4)
            hipLaunchKernelGGL(peak_i8_kernel<true>, dim3(blocks), dim3(kPeakThreads), 0, st, n,
                               static_cast<int*>(out));
        else if (kind == 3)
            hipLaunchKernelGGL(peak_i8_16_kernel, dim3(blocks), dim3(kPeakThreads), 0, st, n,
                               static_cast<int*>(out));
        else if (kind == 1)
            hipLaunchKernelGGL(peak_f64_kernel, dim3(blocks), dim3(kPeakThreads), 0, st, n, static_cast<double*>(out));
        else
            for (int64_t r = 0; r < n; ++r)
                hipLaunchKernelGGL(copy_kernel, dim3(blocks * 4), dim3(256), 0, st, static_cast<const uint4*>(src),
                                   static_cast<uint4*>(dst), static_cast<int64_t>(bytes / 16));
        return hipGetLastError();
    };
    // one untimed launch (code load, clocks), then the timed one
    if (e == hipSuccess) e = launch(kind == 2 ? 1 : (iters < 64 ? iters : 64));
    if (e == hipSuccess) e = hipEventRecord(e0, st);
    if (e == hipSuccess) e = launch(iters);
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e == hipSuccess) {
        const double waves = static_cast<double>(blocks) * (kPeakThreads / 64);
        double work;
        if (kind == 0 || kind == 4) work = waves * iters * kChains * (32.0 * 32.0 * 32.0 * 2.0);
        else if (kind == 3) work = waves * iters * kChains * (16.0 * 16.0 * 64.0 * 2.0);
        else if (kind == 1) work = waves * iters * kChains * (16.0 * 16.0 * 4.0 * 2.0);
        else work = 2.0 * static_cast<double>(bytes) * iters;
        *rate = ms > 0.f ? work / (ms * 1e-3) : 0.0;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (out) (void)hipFree(out);
    return e == hipSuccess ? OZ_OK : OZ_ERR_HIP;
}

}  // extern "C"
