// A whole sequential (mini-batch of one) ePIE / rPIE run on small patterns in
// one launch of one workgroup.
//
// With one position per mini-batch every update depends on the previous one,
// so the four passes of a mini-batch (each a kernel of a few microseconds,
// with most of the GPU idle) would run 5000 times back to back for 50
// iterations over 100 positions.  For N <= 64 the pattern (N^2 complex,
// 32 KiB at 64^2) and the probe fit one CU's LDS, so one workgroup runs every
// step of the call: gather of the exit wave psi = P O_j (Eq. 2), the 2D
// transform in LDS (rows, then columns, Eq. 3), the modulus projection, the
// inverse transform (columns, then rows), and the simultaneous object and
// probe updates of ePIE / rPIE, the object window written back to HBM (where
// the next position reads it) and the probe kept in LDS until the end.  Each
// line transform, projection and update is computed exactly as in the
// multi-pass kernels (same radix code, scaling points and update formulas),
// so the object and probe agree with them bit for bit.
#pragma once

#include "kernels_common.hpp"
#include "pattern_kernels.hpp"
#include "tables.hpp"

namespace mnf {

constexpr int kSmallMaxN = 64;

// T threads per line and every line of a pass in one round: N * T threads
// (512 at 64^2, two waves per SIMD), each holding E pattern elements.
template <int N>
struct SmallCfg {
    static constexpr int T = PlanInfo<N>::T, V = PlanInfo<N>::V;
    static constexpr int THREADS = N * T;
    static constexpr int LINES = N;                              // lines transformed per round
    static constexpr int ROUNDS = 1;
    static constexpr int R = N;                                  // rows and columns of the LDS tile
    static constexpr int S = R + R / 16;                         // row stride (one pad element per 16)
    static constexpr int E = (N * N + THREADS - 1) / THREADS;    // elements per thread
    static constexpr int W = (THREADS + 63) / 64;                // waves
};

// pattern element (y, x) of the padded LDS tile
template <int N>
__device__ __forceinline__ int small_at(int y, int x) {
    return y * SmallCfg<N>::S + x + (x >> 4);
}
// A row of the tile as a transform's exchange space.  A row's T threads lie
// in one wavefront (line = threadIdx / T, T divides 64) and its region of
// the tile is touched by them alone between the block barriers around a row
// pass, so the stage exchanges synchronise the wavefront only (as
// RowLdsWave does).
template <int N>
struct SmallRow {
    static_assert(64 % PlanInfo<N>::T == 0, "a row must not span wavefronts");
    int row;
    __device__ __forceinline__ explicit SmallRow(int r) : row(r) {}
    __device__ __forceinline__ int operator()(int p) const { return small_at<N>(row, p); }
    static __device__ __forceinline__ void sync() { RowLdsWave<N>::sync(); }
};
template <int N>
struct SmallCol {
    int col;
    __device__ __forceinline__ explicit SmallCol(int c) : col(c) {}
    __device__ __forceinline__ int operator()(int p) const { return small_at<N>(p, col); }
    static __device__ __forceinline__ void sync() { __syncthreads(); }
};

// One block of SmallCfg<N>::THREADS threads.  scans[0] is the scan (O, P, amplitudes
// A in FFT order or, if A is NULL, the intensities I), slots[it * J + t] the
// t-th position of local iteration it; the probe is updated from local
// iteration upd_from on (n_iter: never).  err (n_iter doubles) receives the
// normalised Fourier error per iteration when not NULL (sumA2: the sum of the
// squared amplitudes); a non-finite error, or one above max(10 x the first,
// 1e-6), is recorded in the scan's status word.
template <int N>
__global__ void __launch_bounds__(SmallCfg<N>::THREADS)
k_small_run(const ScanDev* __restrict__ scans, const SlotDev* __restrict__ slots, int J, int n_iter, int rpie,
            float alpha, float beta, int upd_from, const double* __restrict__ sumA2, double* __restrict__ err,
            const float2* __restrict__ tw_g) {
    using C = SmallCfg<N>;
    constexpr int T = C::T, V = C::V, LINES = C::LINES, E = C::E, NT = C::THREADS, NW = C::W;
    static_assert(N <= kSmallMaxN, "pattern and probe must fit the LDS");
    __shared__ float2 X[C::R * C::S];
    __shared__ float2 Pl[N * N];
    __shared__ float2 tw[N];
    __shared__ float red_f[2 * NW];
    __shared__ double red_d[NW];
    const ScanDev sc = scans[0];
    const int Nw = sc.Nw, Mx = sc.Mx;
    const int tid = threadIdx.x, w = tid >> 6;
    const int line = tid / T, t = tid % T;
    for (int i = tid; i < N; i += NT) tw[i] = tw_g[i];
    for (int e = tid; e < N * N; e += NT) {
        const int y = e / N, x = e % N;
        Pl[e] = y < Nw && x < Nw ? sc.P[(size_t)y * Nw + x] : make_float2(0.f, 0.f);
    }
    __syncthreads();
    const float sc1 = 1.f / (float)N;
    double err0 = 0.0;
    for (int it = 0; it < n_iter; ++it) {
        const bool upd = it >= upd_from;
        double esum = 0.0;
        for (int tp = 0; tp < J; ++tp) {
            const SlotDev sd = slots[(size_t)it * J + tp];
            // amplitudes at this thread's output frequencies of the column
            // rounds, issued first (used after the forward transform)
            float aq[C::ROUNDS][V];
#pragma unroll
            for (int rd = 0; rd < C::ROUNDS; ++rd) {
                const int c = min(rd * LINES + line, N - 1);
#pragma unroll
                for (int idx = 0; idx < V; ++idx) {
                    const int ky = out_pos<N, false>(t, idx);
                    aq[rd][idx] = sc.A ? ldg(sc.A, (size_t)sd.j * N * N + (size_t)ky * N + c)
                                       : ldg(sc.I, (size_t)sd.j * N * N + (size_t)((ky + N / 2) % N) * N + (c + N / 2) % N);
                }
            }
            // gather: the object window (clamped, masked), the exit wave into
            // the tile, maxima of |O_j|^2 and |P|^2
            float2 o[E];
            float mO = 0.f, mP = 0.f;
#pragma unroll
            for (int i = 0; i < E; ++i) {
                const int e = min(tid + i * NT, N * N - 1);
                const int y = e / N, x = e % N;
                o[i] = ldg(sc.O, (size_t)(sd.py + min(y, Nw - 1)) * Mx + sd.px + min(x, Nw - 1));
            }
#pragma unroll
            for (int i = 0; i < E; ++i) {
                const int e = tid + i * NT;
                const int y = e / N, x = e % N;
                const bool in = e < N * N && y < Nw && x < Nw;
                const float2 p = in ? Pl[e] : make_float2(0.f, 0.f);
                if (e < N * N) X[small_at<N>(y, x)] = in ? cmul(p, o[i]) : make_float2(0.f, 0.f);
                mO = fmaxf(mO, in ? cabs2(o[i]) : 0.f);
                mP = fmaxf(mP, in ? cabs2(p) : 0.f);
            }
            if (!sc.A) {  // uniform: amplitudes from the intensities
#pragma unroll
                for (int rd = 0; rd < C::ROUNDS; ++rd)
#pragma unroll
                    for (int idx = 0; idx < V; ++idx) aq[rd][idx] = amplitude_of(aq[rd][idx]);
            }
            mO = wave_max(mO);
            mP = wave_max(mP);
            if ((tid & 63) == 0) {
                red_f[w] = mO;
                red_f[NW + w] = mP;
            }
            __syncthreads();
            mO = red_f[0];
            mP = red_f[NW];
#pragma unroll
            for (int q = 1; q < NW; ++q) {
                mO = fmaxf(mO, red_f[q]);
                mP = fmaxf(mP, red_f[NW + q]);
            }
            // forward row transforms
#pragma unroll
            for (int rd = 0; rd < C::ROUNDS; ++rd) {
                const int row = rd * LINES + line;
                float2 x[V];
#pragma unroll
                for (int idx = 0; idx < V; ++idx) x[idx] = X[small_at<N>(row, in_pos<N, false>(t, idx))];
                SmallRow<N>::sync();  // the row is read before its first exchange overwrites it
                fft_line<N, false>(x, t, X, SmallRow<N>(row), tw);
#pragma unroll
                for (int idx = 0; idx < V; ++idx) X[small_at<N>(row, out_pos<N, false>(t, idx))] = x[idx];
            }
            __syncthreads();
            // column transforms, projection, inverse column transforms
            float accf = 0.f;
            double acc = 0.0;
#pragma unroll
            for (int rd = 0; rd < C::ROUNDS; ++rd) {
                const int c = rd * LINES + line;
                float2 x[V];
#pragma unroll
                for (int idx = 0; idx < V; ++idx) x[idx] = X[small_at<N>(in_pos<N, false>(t, idx), c)];
                fft_line<N, false>(x, t, X, SmallCol<N>(c), tw);
                float af = 0.f;
#pragma unroll
                for (int idx = 0; idx < V; ++idx)
                    x[idx] = col_pointwise<ColOp::Modulus>(cscale(x[idx], sc1), aq[rd][idx], 0.f, af, acc);
                if (c < N) accf += af;
                fft_line<N, true>(x, t, X, SmallCol<N>(c), tw);
#pragma unroll
                for (int idx = 0; idx < V; ++idx) X[small_at<N>(out_pos<N, true>(t, idx), c)] = x[idx];
            }
            esum += (double)accf;
            __syncthreads();
            // inverse row transforms (the unitary 1/N of the inverse applied in the update)
#pragma unroll
            for (int rd = 0; rd < C::ROUNDS; ++rd) {
                const int row = rd * LINES + line;
                float2 x[V];
#pragma unroll
                for (int idx = 0; idx < V; ++idx) x[idx] = X[small_at<N>(row, in_pos<N, true>(t, idx))];
                SmallRow<N>::sync();  // the row is read before its first exchange overwrites it
                fft_line<N, true>(x, t, X, SmallRow<N>(row), tw);
#pragma unroll
                for (int idx = 0; idx < V; ++idx) X[small_at<N>(row, out_pos<N, true>(t, idx))] = x[idx];
            }
            __syncthreads();
            // simultaneous updates from the batch-start O_j and P (float64
            // denominators, as k_object_update and k_rows_inv_update form them)
            const float aO = rpie ? 1.f - alpha : 0.f;
            const double cstO = rpie ? (double)alpha * (double)mP : (double)mP / (double)alpha;
#pragma unroll
            for (int i = 0; i < E; ++i) {
                const int e = tid + i * NT;
                const int y = e / N, x = e % N;
                if (e >= N * N || y >= Nw || x >= Nw) continue;
                const float2 p = Pl[e];
                const float2 d = csub(cscale(X[small_at<N>(y, x)], sc1), cmul(p, o[i]));
                const float2 nO = cconjmul(p, d);
                const double denO = (double)(aO * cabs2(p)) + cstO;
                float2 v = o[i];
                if (denO > 0.0) {
                    const float inv = (float)(1.0 / denO);
                    v.x = fmaf(nO.x, inv, v.x);
                    v.y = fmaf(nO.y, inv, v.y);
                    sc.O[(size_t)(sd.py + y) * Mx + sd.px + x] = v;
                }
                if (upd) {
                    const float o2 = cabs2(o[i]);
                    const double denP = (double)(rpie ? fmaf(1.f - beta, o2, beta * mO) : mO / beta);
                    if (denP > 0.0) {
                        const float2 nP = cconjmul(o[i], d);
                        const float inv = (float)(1.0 / denP);
                        float2 pn = p;
                        pn.x = fmaf(nP.x, inv, pn.x);
                        pn.y = fmaf(nP.y, inv, pn.y);
                        Pl[e] = pn;
                    }
                }
            }
            __syncthreads();  // the tile, the probe and the object window are read again by the next position
        }
        // the iteration's error, in float64 over the block
        double s = wave_sum(esum);
        if ((tid & 63) == 0) red_d[w] = s;
        __syncthreads();
        if (tid == 0 && err) {  // sumA2 exists only when errors are requested
            double tot = red_d[0];
            for (int q = 1; q < NW; ++q) tot += red_d[q];
            const double e = *sumA2 > 0.0 ? tot / *sumA2 : 0.0;
            err[it] = e;
            if (!isfinite(e)) atomicOr(sc.status, kStatusNonFinite);
            else if (it > 0 && e > fmax(10.0 * err0, 1e-6)) atomicOr(sc.status, kStatusDiverged);
            if (it == 0) err0 = e;
        }
        __syncthreads();
    }
    for (int e = tid; e < N * N; e += NT) {
        const int y = e / N, x = e % N;
        if (y < Nw && x < Nw && upd_from < n_iter) sc.P[(size_t)y * Nw + x] = Pl[e];
    }
}

}  // namespace mnf
