// Pattern-pass kernels of the reconstruction and gradient paths.
//
// A mini-batch of nb scan positions is processed as three passes over a
// scratch array S[nb][N][N] (complex float, FFT order):
//   rows_fwd : exit wave psi = P * O[window] (Eq. 2, zero-padded to N) and
//              its row transforms
//   cols_*   : column transforms completing Psi = F psi (Eq. 3), then a
//              pointwise step (modulus projection, loss gradient or
//              intensity), then for the first two the inverse column transforms
//   rows_inv : inverse row transforms and the per-pixel result in the window
//              (dpsi = psi' - psi for the update, g_psi for the gradient)
// A pattern is 8 N^2 bytes (512 KiB at N = 256), more than one CU's LDS, so
// each pass keeps only rows or 16-column slabs on chip.
#pragma once

#include "kernels_common.hpp"

namespace mnf {

// -------------------------------------------------------------- rows_fwd
// grid (ceil(Nw / LINES), nb).  Also writes per-block maxima of |O_j|^2
// (maxO2_part[s][blockIdx.x]) and, from slot 0, of |P|^2 (maxP2_part[blockIdx.x]).
template <int N>
__global__ void __launch_bounds__(RowCfg<N>::THREADS)
k_rows_fwd(const float2* __restrict__ O, int Mx, const float2* __restrict__ P, int Nw,
           const int* __restrict__ pos, const int* __restrict__ bj, float2* __restrict__ S,
           float* __restrict__ maxO2_part, float* __restrict__ maxP2_part,
           const float2* __restrict__ tw_g) {
    constexpr int T = RowCfg<N>::T, LINES = RowCfg<N>::LINES, V = PlanInfo<N>::V;
    __shared__ float2 lds[LINES * RowLds<N>::stride];
    __shared__ float2 tw[N];
    __shared__ float red[RowCfg<N>::THREADS / 64 + 1];
    const int s = blockIdx.y;
    const int j = bj[s];
    const int py = pos[2 * j], px = pos[2 * j + 1];
    const int line = threadIdx.x / T, t = threadIdx.x % T;
    const int y = blockIdx.x * LINES + line;
    const bool live = y < Nw;

    float2 x[V];
    float mO = 0.f, mP = 0.f;
    const float2* Orow = O + (size_t)(py + y) * Mx + px;
    const float2* Prow = P + (size_t)y * Nw;
#pragma unroll
    for (int idx = 0; idx < V; ++idx) {
        const int n = in_pos<N, false>(t, idx);
        float2 v = make_float2(0.f, 0.f);
        if (live && n < Nw) {
            const float2 p = Prow[n];
            const float2 o = Orow[n];
            v = cmul(p, o);
            mO = fmaxf(mO, cabs2(o));
            mP = fmaxf(mP, cabs2(p));
        }
        x[idx] = v;
    }
    for (int i = threadIdx.x; i < N; i += blockDim.x) tw[i] = tw_g[i];
    __syncthreads();
    fft_line<N, false>(x, t, lds, RowLds<N>(line), tw);
    if (live) {
        float2* row = S + ((size_t)s * N + y) * N;
#pragma unroll
        for (int idx = 0; idx < V; ++idx) row[out_pos<N, false>(t, idx)] = x[idx];
    }
    if (maxO2_part) {
        mO = block_max(mO, red);
        if (threadIdx.x == 0) maxO2_part[(size_t)s * gridDim.x + blockIdx.x] = mO;
    }
    if (maxP2_part && s == 0) {
        mP = block_max(mP, red);
        if (threadIdx.x == 0) maxP2_part[blockIdx.x] = mP;
    }
}

// Pointwise step applied between the forward and inverse column transforms.
// v is Psi (unitary scaling applied), a_src the fused intensity at that
// frequency (detector-centred source).  Returns the value to inverse-transform
// and accumulates the per-pixel error / loss term.
enum class ColOp { Modulus, PoissonGrad, AmplitudeGrad };

template <ColOp OP>
__device__ __forceinline__ float2 col_pointwise(float2 v, float Iq, float eps, double& acc) {
    const float m2 = cabs2(v);
    if constexpr (OP == ColOp::Modulus) {
        // Fourier-modulus projection against A = sqrt(max(I, 0)); error (|Psi| - A)^2
        const float a = sqrtf(fmaxf(Iq, 0.f));
        const float mag = sqrtf(m2);
        const float d = mag - a;
        acc += (double)d * (double)d;
        return m2 > 1e-30f ? cscale(v, a / mag) : make_float2(a, 0.f);
    } else if constexpr (OP == ColOp::PoissonGrad) {
        // l = |Psi|^2 - I ln(|Psi|^2 + eps); g = 2 (1 - I / (|Psi|^2 + eps)) Psi
        const float I = fmaxf(Iq, 0.f);
        acc += (double)(m2 - I * logf(m2 + eps));
        return cscale(v, 2.f * (1.f - I / (m2 + eps)));
    } else {
        // l = (|Psi| - sqrt I)^2; g = 2 (Psi - sqrt(I) Psi / |Psi|)
        const float a = sqrtf(fmaxf(Iq, 0.f));
        const float mag = sqrtf(m2);
        const float d = mag - a;
        acc += (double)d * (double)d;
        const float f = m2 > 1e-30f ? 2.f * (1.f - a / mag) : 2.f;
        return cscale(v, f);
    }
}

// -------------------------------------------------------- cols_pointwise
// grid (N / C, nb).  Column transforms, pointwise step, inverse column
// transforms; writes back the first Nw rows (the rows_inv pass reads no
// others) and a per-block float64 partial acc_part[j][blockIdx.x].
template <int N, ColOp OP>
__global__ void __launch_bounds__(ColCfg<N>::THREADS)
k_cols_pointwise(float2* __restrict__ S, int Nw, const float* __restrict__ I,
                 const int* __restrict__ bj, double* __restrict__ acc_part, float eps,
                 const float2* __restrict__ tw_g) {
    constexpr int C = ColCfg<N>::C, T = ColCfg<N>::T, V = PlanInfo<N>::V;
    __shared__ float2 lds[C * N];
    __shared__ float2 tw[N];
    __shared__ double red[ColCfg<N>::THREADS / 64 + 1];
    const int s = blockIdx.y;
    const int j = bj[s];
    const int c = threadIdx.x % C, t = threadIdx.x / C;
    const int kx = blockIdx.x * C + c;
    float2* col = S + (size_t)s * N * N + kx;

    float2 x[V];
#pragma unroll
    for (int idx = 0; idx < V; ++idx) {
        const int y = in_pos<N, false>(t, idx);
        x[idx] = y < Nw ? col[(size_t)y * N] : make_float2(0.f, 0.f);
    }
    for (int i = threadIdx.x; i < N; i += blockDim.x) tw[i] = tw_g[i];
    __syncthreads();
    fft_line<N, false>(x, t, lds, ColLds<C>(c), tw);

    const float sc = 1.f / (float)N;
    const float* Ij = I + (size_t)j * N * N;
    const int sx = (kx + N / 2) % N;
    double acc = 0.0;
#pragma unroll
    for (int idx = 0; idx < V; ++idx) {
        const int ky = out_pos<N, false>(t, idx);
        const int sy = (ky + N / 2) % N;
        x[idx] = col_pointwise<OP>(cscale(x[idx], sc), Ij[(size_t)sy * N + sx], eps, acc);
    }
    fft_line<N, true>(x, t, lds, ColLds<C>(c), tw);
#pragma unroll
    for (int idx = 0; idx < V; ++idx) {
        const int y = out_pos<N, true>(t, idx);
        if (y < Nw) col[(size_t)y * N] = x[idx];  // the 1/N of the unitary inverse is applied by rows_inv
    }
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) acc_part[(size_t)j * gridDim.x + blockIdx.x] = acc;
}

// -------------------------------------------------------- cols_intensity
// grid (N / C, nb).  Forward model only: I_out[j] = fftshift |Psi|^2.
template <int N>
__global__ void __launch_bounds__(ColCfg<N>::THREADS)
k_cols_intensity(const float2* __restrict__ S, int Nw, const int* __restrict__ bj,
                 float* __restrict__ I_out, const float2* __restrict__ tw_g) {
    constexpr int C = ColCfg<N>::C, T = ColCfg<N>::T, V = PlanInfo<N>::V;
    __shared__ float2 lds[C * N];
    __shared__ float2 tw[N];
    const int s = blockIdx.y;
    const int j = bj[s];
    const int c = threadIdx.x % C, t = threadIdx.x / C;
    const int kx = blockIdx.x * C + c;
    const float2* col = S + (size_t)s * N * N + kx;
    float2 x[V];
#pragma unroll
    for (int idx = 0; idx < V; ++idx) {
        const int y = in_pos<N, false>(t, idx);
        x[idx] = y < Nw ? col[(size_t)y * N] : make_float2(0.f, 0.f);
    }
    for (int i = threadIdx.x; i < N; i += blockDim.x) tw[i] = tw_g[i];
    __syncthreads();
    fft_line<N, false>(x, t, lds, ColLds<C>(c), tw);
    const float sc2 = 1.f / ((float)N * (float)N);
    float* Ij = I_out + (size_t)j * N * N;
    const int sx = (kx + N / 2) % N;
#pragma unroll
    for (int idx = 0; idx < V; ++idx) {
        const int ky = out_pos<N, false>(t, idx);
        Ij[(size_t)((ky + N / 2) % N) * N + sx] = cabs2(x[idx]) * sc2;
    }
}

// --------------------------------------------------------------- rows_inv
// grid (ceil(Nw / LINES), nb).  Inverse row transforms of the first Nw rows.
// DPSI = true : S[s][y][n] = psi'(y, n) - P(y, n) O_j(y, n) for n < Nw
// DPSI = false: S[s][y][n] = scale * psi'(y, n)              for n < Nw
template <int N, bool DPSI>
__global__ void __launch_bounds__(RowCfg<N>::THREADS)
k_rows_inv(float2* __restrict__ S, const float2* __restrict__ O, int Mx,
           const float2* __restrict__ P, int Nw, const int* __restrict__ pos,
           const int* __restrict__ bj, float scale, const float2* __restrict__ tw_g) {
    constexpr int T = RowCfg<N>::T, LINES = RowCfg<N>::LINES, V = PlanInfo<N>::V;
    __shared__ float2 lds[LINES * RowLds<N>::stride];
    __shared__ float2 tw[N];
    const int s = blockIdx.y;
    const int j = bj[s];
    const int py = pos[2 * j], px = pos[2 * j + 1];
    const int line = threadIdx.x / T, t = threadIdx.x % T;
    const int y = blockIdx.x * LINES + line;
    const bool live = y < Nw;
    float2* row = S + ((size_t)s * N + (live ? y : 0)) * N;

    float2 x[V];
#pragma unroll
    for (int idx = 0; idx < V; ++idx)
        x[idx] = live ? row[in_pos<N, true>(t, idx)] : make_float2(0.f, 0.f);
    for (int i = threadIdx.x; i < N; i += blockDim.x) tw[i] = tw_g[i];
    __syncthreads();
    fft_line<N, true>(x, t, lds, RowLds<N>(line), tw);
    if (!live) return;
    const float sc = 1.f / (float)N;
    const float2* Orow = O + (size_t)(py + y) * Mx + px;
    const float2* Prow = P + (size_t)y * Nw;
#pragma unroll
    for (int idx = 0; idx < V; ++idx) {
        const int n = out_pos<N, true>(t, idx);
        if (n < Nw) {
            const float2 v = cscale(x[idx], sc);
            if constexpr (DPSI) {
                row[n] = csub(v, cmul(Prow[n], Orow[n]));
            } else {
                row[n] = cscale(v, scale);
            }
        }
    }
}

}  // namespace mnf
