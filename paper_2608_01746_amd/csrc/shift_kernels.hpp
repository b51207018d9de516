// Fourier translation of probe-sized fields for real-valued scan positions.
//
// A position r = p + d (p the nearest integer corner, d in [-1/2, 1/2) per
// axis) is modelled by translating the probe by d: the exit wave
// P(m - d) O(p + m) has the far-field intensity of P(m) O(p + m + d) (Eq. 2
// at the real position; a translation only adds a phase ramp to Eq. 3).  The
// translation over the Nw x Nw window is S_d = F^-1 diag(exp(-2 pi i k.d / Nw)) F
// with frequencies k in [-Nw/2, Nw/2), applied as a row pass (x) and a column
// pass (y), each forward transform -> ramp -> inverse transform in registers.
// S_d is unitary with inverse S_-d, which carries the probe-update numerators
// back to the untranslated probe.  Slots with a zero fraction on an axis skip
// that axis's transforms, so whole-pixel positions keep the probe exactly.
//
// Fields are [slot][Nw][Nw] complex float, row-major; frac[slot] = (d_y, d_x).
#pragma once

#include "kernels_common.hpp"
#include "tables.hpp"

namespace mnf {

// exp(-2 pi i k' d / N), k' the signed frequency of FFT-order index k.  The
// angle in turns, -k' d / N, lies in [-1/4, 1/4] (|k'| <= N/2, |d| <= 1/2);
// the hardware sine and cosine take turns directly.
template <int N>
__device__ __forceinline__ float2 shift_ramp(int k, float d) {
    const int ks = k < N / 2 ? k : k - N;
    const float turns = -(float)ks * d * (1.f / (float)N);
    return make_float2(__builtin_amdgcn_cosf(turns), __builtin_amdgcn_sinf(turns));
}

// A line held in registers at the positions in_pos<N, false> (the same as
// out_pos<N, true>) translated by d in place; every thread of the block
// takes part (the transforms synchronise), d may differ between lines.
template <int N, class ADDR>
__device__ __forceinline__ void shift_regs(float2* x, float d, int t, float2* lds, const ADDR& addr,
                                           const float2* tw) {
    constexpr int V = PlanInfo<N>::V;
    fft_line<N, false>(x, t, lds, addr, tw);
    const float inv = 1.f / (float)N;
#pragma unroll
    for (int idx = 0; idx < V; ++idx) x[idx] = cscale(cmul(x[idx], shift_ramp<N>(out_pos<N, false>(t, idx), d)), inv);
    fft_line<N, true>(x, t, lds, addr, tw);
}

// One line of N values (in[i * stride]) loaded into x[] at the positions
// in_pos<N, false>, which are also where a translation (shift_regs) leaves
// them (out_pos<N, true>): a zero fraction needs no transform at all.
template <int N>
__device__ __forceinline__ void line_load(float2* x, const float2* in, size_t stride, int t) {
    constexpr int V = PlanInfo<N>::V;
#pragma unroll
    for (int idx = 0; idx < V; ++idx) x[idx] = in[(size_t)in_pos<N, false>(t, idx) * stride];
}

// grid (N / LINES, nslots).  dst[s][y][:] = row y of src[s] translated along x
// by sign * d_x(s); src_stride 0 reads one shared field (the probe).  dst may
// equal src (each line is read before any of it is written).
template <int N>
__global__ void __launch_bounds__((RowCfg<N, 0>::THREADS))
k_shift_rows(const float2* src, size_t src_stride, float2* dst, const float2* __restrict__ frac, float sign,
             const float2* __restrict__ tw_g) {
    constexpr int T = RowCfg<N, 0>::T, LINES = RowCfg<N, 0>::LINES, V = PlanInfo<N>::V;
    __shared__ float2 lds[LINES * RowLds<N>::stride];
    __shared__ float2 tw[N];
    const int s = blockIdx.y;
    const int line = threadIdx.x / T, t = threadIdx.x % T;
    const int y = blockIdx.x * LINES + line;  // N % LINES == 0
    float2 x[V];
    line_load<N>(x, src + s * src_stride + (size_t)y * N, 1, t);
    TwRegs<N, RowCfg<N, 0>::THREADS> twr;
    twr.load(tw_g);
    const float d = sign * frac[s].y;  // uniform over the block
    twr.store(tw);
    __syncthreads();
    if (d != 0.f) shift_regs<N>(x, d, t, lds, RowLdsWave<N>(line), tw);
    float2* row = dst + ((size_t)s * N + y) * N;
#pragma unroll
    for (int idx = 0; idx < V; ++idx) st_dev(row, out_pos<N, true>(t, idx), x[idx]);
}

// grid (N / C, nslots).  dst[s] column kx = column kx of src[s] translated
// along y by sign * d_y(s); src_stride 0 reads one shared field (the probe).
// dst may equal src (in place; then a zero fraction leaves the column).
template <int N>
__global__ void __launch_bounds__((ColCfg<N, 0>::THREADS))
k_shift_cols(const float2* src, size_t src_stride, float2* dst, const float2* __restrict__ frac, float sign,
             const float2* __restrict__ tw_g) {
    constexpr int C = ColCfg<N, 0>::C, T = ColCfg<N, 0>::T, V = PlanInfo<N>::V;
    __shared__ float2 lds[C * N];
    __shared__ float2 tw[N];
    const int s = blockIdx.y;
    const float d = sign * frac[s].x;
    if (d == 0.f && src == dst) return;  // uniform over the block
    const int c = threadIdx.x % C, t = threadIdx.x / C;
    const float2* in = src + s * src_stride + blockIdx.x * C + c;
    float2* col = dst + (size_t)s * N * N + blockIdx.x * C + c;
    float2 x[V];
    line_load<N>(x, in, N, t);
    TwRegs<N, ColCfg<N, 0>::THREADS> twr;
    twr.load(tw_g);
    twr.store(tw);
    __syncthreads();
    if (d != 0.f) shift_regs<N>(x, d, t, lds, ColLds<C>(c), tw);
#pragma unroll
    for (int idx = 0; idx < V; ++idx) st_dev(col, (size_t)out_pos<N, true>(t, idx) * N, x[idx]);
}

// grid (ceil(N^2 / 256), ngroups).  Probe update at real positions: G[s]
// holds the numerators conj(O_s) dpsi_s translated back by -d_s; per probe
// pixel q the group's slots are summed in slot order and
// P[q] += sum / DP[q] (float64 quotient) where DP > 0.
template <int N>
__global__ void __launch_bounds__(256)
k_probe_sum_update(const float2* __restrict__ G, const GroupDev* __restrict__ groups, float2* __restrict__ P,
                   const double* __restrict__ DP) {
    const GroupDev gd = groups[blockIdx.y];
    const int q = blockIdx.x * 256 + threadIdx.x;
    if (q >= N * N) return;
    const double den = DP[q];
    float2 p = P[q];
    // the slots' numerators, eight loads at a time (slot index clamped),
    // summed in slot order
    float2 acc = make_float2(0.f, 0.f);
    const float2* g = G + (size_t)gd.s0 * N * N + q;
    for (int k0 = 0; k0 < gd.nb; k0 += 8) {
        float2 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = g[(size_t)min(k0 + u, gd.nb - 1) * N * N];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (k0 + u < gd.nb) acc = cadd(acc, v[u]);
    }
    if (!(den > 0.0)) return;
    const float inv = (float)(1.0 / den);  // the float64 denominator, inverted once
    p.x = fmaf(acc.x, inv, p.x);
    p.y = fmaf(acc.y, inv, p.y);
    st_dev(P, q, p);
}

}  // namespace mnf
