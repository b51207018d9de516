// Block-level reductions and launch shapes shared by the pattern kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "fft.hpp"

namespace mnf {

constexpr int kMaxBatch = 512;  // positions per mini-batch handled by one launch
constexpr int kMaxModes = 4;    // probe modes of a mixed-state reconstruction
constexpr int kColGroup = 32;   // adjacent columns per column-pass block (32 x 8 B = 256 B of S, 128 B of I per row)

// Launch shapes.  Each pass has two compiled variants (0: the default, 1:
// half as many lines or columns per block); the tuner picks one per size.
//
// Row passes: LINES pattern rows per block, T threads per row.
template <int N, int RV = 0>
struct RowCfg {
    static constexpr int T = PlanInfo<N>::T;
    static constexpr int LINES0 = (256 / T) < N ? (256 / T) : N;
    static constexpr int LINES = RV == 0 ? LINES0 : (LINES0 > 1 ? LINES0 / 2 : 1);
    static constexpr int THREADS = LINES * T;
};

// Column passes: C adjacent columns per block, T threads per column.
template <int N, int CV = 0>
struct ColCfg {
    static constexpr int T = PlanInfo<N>::T;
    static constexpr int C0 = kColGroup < N ? kColGroup : N;
    static constexpr int C = CV == 0 ? C0 : C0 / 2;
    static constexpr int THREADS = C * T;
};

// Loads through a global-address-space view of a device pointer.  A pointer
// read out of a descriptor is generic to the compiler, which then emits flat
// loads; those also count against the LDS counter, so every wait for an LDS
// value would wait for them too.  Only for memory of the device heap.
template <class T>
using gptr = const __attribute__((address_space(1))) T*;
__device__ __forceinline__ float ldg(const float* p, size_t i) { return ((gptr<float>)p)[i]; }
__device__ __forceinline__ double ldg(const double* p, size_t i) { return ((gptr<double>)p)[i]; }
__device__ __forceinline__ float2 ldg(const float2* p, size_t i) {
    typedef float v2 __attribute__((ext_vector_type(2)));
    const v2 v = ((gptr<v2>)p)[i];
    return make_float2(v.x, v.y);
}

// Amplitude sqrt(max(I, 0)) of an intensity: the hardware square root
// (about 1 ulp), the same in every kernel that forms amplitudes, so the
// precomputed and the on-the-fly amplitudes agree bit for bit.
__device__ __forceinline__ float amplitude_of(float I) { return __builtin_amdgcn_sqrtf(fmaxf(I, 0.f)); }

// Stores of results that a later kernel reads.  The L2 of one XCD is not
// coherent with the other seven, so the release at the end of a kernel
// writes back every line its waves left dirty, after the last wave and while
// the next kernel waits.  A device-scope store (a relaxed atomic store at
// agent scope: the scope only, no ordering) is written through the L2 while
// the kernel runs instead.  Each element must be written by one thread.
template <class T>
using gptr_w = __attribute__((address_space(1))) T*;
__device__ __forceinline__ void st_dev(float2* p, size_t i, float2 v) {
    const unsigned long long b = ((unsigned long long)__float_as_uint(v.y) << 32) | __float_as_uint(v.x);
    __hip_atomic_store((gptr_w<unsigned long long>)(p + i), b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev(float* p, size_t i, float v) {
    __hip_atomic_store((gptr_w<float>)(p + i), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The twiddle table staged through registers: load() with a prologue's
// other loads, store() to LDS just before the barrier that precedes the first
// transform, so the table's load needs no wait of its own (a load-to-LDS
// loop waits for every load issued before it).
template <int N, int THREADS>
struct TwRegs {
    static constexpr int K = (N + THREADS - 1) / THREADS;
    float2 v[K];
    __device__ __forceinline__ void load(const float2* tw_g) {
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] = tw_g[min((int)threadIdx.x + k * THREADS, N - 1)];
    }
    __device__ __forceinline__ void store(float2* tw) const {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int i = (int)threadIdx.x + k * THREADS;
            if (i < N) tw[i] = v[k];
        }
    }
};

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Block-wide max / sum in a fixed order (waves combined in index order).
// `red` must hold blockDim.x / 64 elements.  Result valid in every thread.
// `reuse`: `red` was read earlier in the block, so a leading barrier keeps
// those reads ahead of the new writes; a block's first use needs none.
__device__ __forceinline__ float block_max(float v, float* red, bool reuse = true) {
    v = wave_max(v);
    const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    if (reuse) __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    float r = red[0];
    for (int i = 1; i < nw; ++i) r = fmaxf(r, red[i]);
    return r;
}
__device__ __forceinline__ double block_sum(double v, double* red, bool reuse = true) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    if (reuse) __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double r = red[0];
    for (int i = 1; i < nw; ++i) r += red[i];
    return r;
}

}  // namespace mnf
