// Pattern-pass kernels of the reconstruction, gradient and forward paths.
//
// A launch processes a list of slots (scan positions, possibly of several
// scans of the same detector size N) as three passes over a scratch array
// S[slot][N][N] (complex float, FFT order):
//   rows_fwd : exit wave psi = P * O[window] (Eq. 2, zero-padded to N) and
//              its row transforms
//   cols_*   : column transforms completing Psi = F psi (Eq. 3), a pointwise
//              step (modulus projection, loss gradient or intensity) and, for
//              the first two, the inverse column transforms
//   rows_inv_update : inverse row transforms and the per-pixel results
// A 256^2 pattern is 512 KiB, more than one CU's LDS, so each pass keeps only
// rows or column slabs on chip; Psi never leaves registers between the
// forward and inverse column transforms.
#pragma once

#include "kernels_common.hpp"
#include "shift_kernels.hpp"
#include "tables.hpp"

namespace mnf {

// -------------------------------------------------------------- rows_fwd
// grid (ceil(maxNw / LINES), nslots).  Writes per-block maxima of |O_j|^2,
// maxO2_part[slot][blockIdx.x] (when not NULL).  Pd (when not NULL) is a
// table of probes [k][Nw][Nw] used in place of the scan's probe: slot s reads
// Pd[s % pmod] (one translated probe per slot for real positions, pmod >=
// nslots; probe mode s % M for mixed states, pmod = M).  SUBX (real
// positions, Nw == N): Pd[s] holds the probe translated along y only; each
// row is translated along x by d_x(s) = frac[s].y here, in registers, and the
// fully translated row is stored back to Pd[s] for the inverse row pass.
template <int N, int RV, bool SUBX = false>
__global__ void __launch_bounds__((RowCfg<N, RV>::THREADS))
k_rows_fwd(const ScanDev* __restrict__ scans, const SlotDev* __restrict__ slots,
           float2* __restrict__ S, float* __restrict__ maxO2_part, float2* Pd, int pmod,
           const float2* __restrict__ frac, const float2* __restrict__ tw_g) {
    constexpr int T = RowCfg<N, RV>::T, LINES = RowCfg<N, RV>::LINES, V = PlanInfo<N>::V;
    __shared__ float2 lds[LINES * RowLds<N>::stride];
    __shared__ float2 tw[N];
    __shared__ float red[RowCfg<N, RV>::THREADS / 64 + 1];
    const int s = blockIdx.y;
    const ScanDev sc0 = scans[0];
    const SlotDev sd = slots[s];
    const ScanDev sc = scan_desc(scans, sc0, sd.scan);
    const int Nw = sc.Nw, Mx = sc.Mx;
    const int line = threadIdx.x / T, t = threadIdx.x % T;
    const int y = blockIdx.x * LINES + line;
    const bool live = y < Nw;

    float2 x[V];
    float mO = 0.f;
    const float2* Orow = sc.O + (size_t)(sd.py + (live ? y : 0)) * Mx + sd.px;
    // Every load is issued unconditionally (row and column clamped into the
    // window) and masked afterwards, so a thread's loads are all in flight
    // together instead of one guarded load after another.
    if constexpr (SUBX) {
        float2* Pw = Pd + ((size_t)s * N + (live ? y : 0)) * N;
        const float dx = frac[s].y;  // uniform over the block
        float2 o[V], p[V];
        line_load<N>(p, Pw, 1, t);
#pragma unroll
        for (int idx = 0; idx < V; ++idx) o[idx] = ldg(Orow, in_pos<N, false>(t, idx));  // Nw == N
        TwRegs<N, RowCfg<N, RV>::THREADS> twr;
        twr.load(tw_g);
        twr.store(tw);
        __syncthreads();
        if (dx != 0.f) shift_regs<N>(p, dx, t, lds, RowLdsWave<N>(line), tw);
        if (live && dx != 0.f) {
#pragma unroll
            for (int idx = 0; idx < V; ++idx) st_dev(Pw, in_pos<N, false>(t, idx), p[idx]);
        }
#pragma unroll
        for (int idx = 0; idx < V; ++idx) {
            x[idx] = live ? cmul(p[idx], o[idx]) : make_float2(0.f, 0.f);
            mO = fmaxf(mO, live ? cabs2(o[idx]) : 0.f);
        }
    } else {
        const float2* Prow = (Pd ? Pd + (size_t)(s % pmod) * Nw * Nw : sc.P) + (size_t)(live ? y : 0) * Nw;
        float2 o[V], p[V];
#pragma unroll
        for (int idx = 0; idx < V; ++idx) {
            const int n = min(in_pos<N, false>(t, idx), Nw - 1);
            o[idx] = ldg(Orow, n);
            p[idx] = ldg(Prow, n);
        }
        for (int i = threadIdx.x; i < N; i += blockDim.x) tw[i] = tw_g[i];
        __syncthreads();
#pragma unroll
        for (int idx = 0; idx < V; ++idx) {
            const bool in = live && in_pos<N, false>(t, idx) < Nw;
            x[idx] = in ? cmul(p[idx], o[idx]) : make_float2(0.f, 0.f);
            mO = fmaxf(mO, in ? cabs2(o[idx]) : 0.f);
        }
    }
    fft_line<N, false>(x, t, lds, RowLdsWave<N>(line), tw);
    if (live) {
        float2* row = S + ((size_t)s * N + y) * N;
#pragma unroll
        for (int idx = 0; idx < V; ++idx) st_dev(row, out_pos<N, false>(t, idx), x[idx]);
    }
    if (maxO2_part) {
        mO = block_max(mO, red, false);
        if (threadIdx.x == 0) maxO2_part[(size_t)s * gridDim.x + blockIdx.x] = mO;
    }
}

// Pointwise step applied between the forward and inverse column transforms.
// v is Psi (unitary scaling applied), Iq the fused intensity at that
// frequency.  Returns the value to inverse-transform and accumulates the
// per-pixel error / loss term.
enum class ColOp { Modulus, PoissonGrad, AmplitudeGrad };

template <ColOp OP>
__device__ __forceinline__ float2 col_pointwise(float2 v, float Iq, float eps, float& accf, double& acc) {
    const float m2 = cabs2(v);
    if constexpr (OP == ColOp::Modulus) {
        // Fourier-modulus projection against the amplitude a = Iq (A = sqrt(max(I, 0)),
        // precomputed once per call); error (|Psi| - A)^2.  One hardware reciprocal
        // square root r ~ 1/|Psi| (about 1 ulp) gives both |Psi| = m2 r and the
        // scale A r, in place of a correctly rounded root and quotient per value.
        const float a = Iq;
        const bool nz = m2 > 1e-30f;
        const float r = __builtin_amdgcn_rsqf(nz ? m2 : 1.f);
        const float d = (nz ? m2 * r : 0.f) - a;
        accf += d * d;  // a thread's V terms in float32, then float64 across threads
        return nz ? cscale(v, a * r) : make_float2(a, 0.f);
    } else if constexpr (OP == ColOp::PoissonGrad) {
        // l = |Psi|^2 - I ln(|Psi|^2 + eps); g = 2 (1 - I / (|Psi|^2 + eps)) Psi.
        // One hardware log2 (about 1 ulp) times ln 2 and one hardware
        // reciprocal (about 1 ulp) replace the library logarithm and the
        // correctly rounded quotient, which made this pass bound by their
        // arithmetic at 512^2.  A subnormal q (only with eps below the
        // smallest normal float) is scaled by 2^32 first, as the hardware
        // instructions take normal inputs.
        const float I = fmaxf(Iq, 0.f);
        const float q = m2 + eps;
        const bool sub = q < 1.17549435e-38f;
        const float qs = sub ? q * 4294967296.f : q;
        const float lg = (__builtin_amdgcn_logf(qs) - (sub ? 32.f : 0.f)) * 0.693147180559945309f;
        const float rq = __builtin_amdgcn_rcpf(qs) * (sub ? 4294967296.f : 1.f);
        acc += (double)(m2 - I * lg);
        return cscale(v, 2.f * (1.f - I * rq));
    } else {
        // l = (|Psi| - sqrt I)^2; g = 2 (Psi - sqrt(I) Psi / |Psi|), with one
        // hardware reciprocal square root r ~ 1/|Psi| giving |Psi| = |Psi|^2 r
        // and sqrt(I) / |Psi| = sqrt(I) r
        const float a = amplitude_of(Iq);
        const bool nz = m2 > 1e-30f;
        const float r = __builtin_amdgcn_rsqf(nz ? m2 : 1.f);
        const float d = (nz ? m2 * r : 0.f) - a;
        accf += d * d;
        const float f = nz ? 2.f * (1.f - a * r) : 2.f;
        return cscale(v, f);
    }
}

// -------------------------------------------------------- cols_pointwise
// grid (N / C, nslots).  Column transforms, pointwise step, inverse column
// transforms; writes back the first Nw rows (the inverse row pass reads no
// others) and a float64 partial err_part[j][blockIdx.x] of the scan.
template <int N, int CV, ColOp OP>
__global__ void __launch_bounds__((ColCfg<N, CV>::THREADS))
k_cols_pointwise(const ScanDev* __restrict__ scans, const SlotDev* __restrict__ slots,
                 float2* __restrict__ S, float eps, const float2* __restrict__ tw_g) {
    constexpr int C = ColCfg<N, CV>::C, T = ColCfg<N, CV>::T, V = PlanInfo<N>::V;
    __shared__ float2 lds[C * N];
    __shared__ float2 tw[N];
    __shared__ double red[ColCfg<N, CV>::THREADS / 64 + 1];
    const int s = blockIdx.y;
    const int c = threadIdx.x % C, t = threadIdx.x / C;
    const int kx = blockIdx.x * C + c;
    float2* col = S + (size_t)s * N * N + kx;
    // The column and the twiddles need no descriptor: their loads go out
    // before the descriptors are read (rows at and beyond Nw hold stale
    // values and are zeroed once Nw is known).
    float2 x[V];
#pragma unroll
    for (int idx = 0; idx < V; ++idx) x[idx] = col[(size_t)in_pos<N, false>(t, idx) * N];
    TwRegs<N, ColCfg<N, CV>::THREADS> twr;
    twr.load(tw_g);
    const ScanDev sc0 = scans[0];
    const SlotDev sd = slots[s];
    const ScanDev sc = scan_desc(scans, sc0, sd.scan);
    const int Nw = sc.Nw;

    // the amplitude (projection) or fused intensity (losses) at this thread's
    // output frequencies is loaded with the column, before the transform; the
    // amplitudes are stored in FFT order, the intensities detector-centred
    float Iq[V];
    const bool from_I = OP != ColOp::Modulus || !sc.A;  // no amplitude buffer: square roots below
    if (!from_I) {
        const float* Aj = sc.A + (size_t)sd.j * N * N + kx;
#pragma unroll
        for (int idx = 0; idx < V; ++idx) Iq[idx] = ldg(Aj, (size_t)out_pos<N, false>(t, idx) * N);
    } else {
        const float* Ij = sc.I + (size_t)sd.j * N * N;
        const int sx = (kx + N / 2) % N;
#pragma unroll
        for (int idx = 0; idx < V; ++idx) {
            const int ky = out_pos<N, false>(t, idx);
            Iq[idx] = ldg(Ij, (size_t)((ky + N / 2) % N) * N + sx);
        }
    }
#pragma unroll
    for (int idx = 0; idx < V; ++idx)
        if (in_pos<N, false>(t, idx) >= Nw) x[idx] = make_float2(0.f, 0.f);
    twr.store(tw);
    __syncthreads();
    fft_line<N, false>(x, t, lds, ColLds<C>(c), tw);
    if (from_I) {  // uniform: intensities read directly are checked, square roots taken here
        bool bad = false;
#pragma unroll
        for (int idx = 0; idx < V; ++idx) bad |= !isfinite(Iq[idx]);
        if (__ballot(bad) != 0ull && (threadIdx.x & 63) == 0) atomicOr(sc.status, kStatusNonFinite);
        if constexpr (OP == ColOp::Modulus) {
#pragma unroll
            for (int idx = 0; idx < V; ++idx) Iq[idx] = amplitude_of(Iq[idx]);
        }
    }

    const float sc1 = 1.f / (float)N;
    double acc = 0.0;
    float accf = 0.f;
#pragma unroll
    for (int idx = 0; idx < V; ++idx) x[idx] = col_pointwise<OP>(cscale(x[idx], sc1), Iq[idx], eps, accf, acc);
    acc += (double)accf;
    fft_line<N, true>(x, t, lds, ColLds<C>(c), tw);
#pragma unroll
    for (int idx = 0; idx < V; ++idx) {
        const int y = out_pos<N, true>(t, idx);
        if (y < Nw) st_dev(col, (size_t)y * N, x[idx]);  // the 1/N of the unitary inverse is applied by the row pass
    }
    acc = block_sum(acc, red, false);
    if (threadIdx.x == 0) sc.err_part[(size_t)sd.j * gridDim.x + blockIdx.x] = acc;
}

// -------------------------------------------------------- cols_intensity
// grid (N / C, nslots).  Forward model only: I_out[j] = fftshift |Psi|^2.
template <int N, int CV>
__global__ void __launch_bounds__((ColCfg<N, CV>::THREADS))
k_cols_intensity(const ScanDev* __restrict__ scans, const SlotDev* __restrict__ slots,
                 const float2* __restrict__ S, float* __restrict__ I_out, const float2* __restrict__ tw_g) {
    constexpr int C = ColCfg<N, CV>::C, T = ColCfg<N, CV>::T, V = PlanInfo<N>::V;
    __shared__ float2 lds[C * N];
    __shared__ float2 tw[N];
    const int s = blockIdx.y;
    const ScanDev sc0 = scans[0];
    const SlotDev sd = slots[s];
    const int Nw = scan_desc(scans, sc0, sd.scan).Nw;
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
    float* Ij = I_out + (size_t)sd.j * N * N;
    const int sx = (kx + N / 2) % N;
#pragma unroll
    for (int idx = 0; idx < V; ++idx) {
        const int ky = out_pos<N, false>(t, idx);
        st_dev(Ij, (size_t)((ky + N / 2) % N) * N + sx, cabs2(x[idx]) * sc2);
    }
}

// ------------------------------------------------- mixed-state column passes
// Slots come in runs of M (one per probe mode) for each position; grid
// (N / C, nslots / M), block y owns the M slots of one position.
//
// cols_modulus_modes: the modes' column transforms Psi_m, the shared
// projection Psi'_m = Psi_m A / sqrt(sum_m |Psi_m|^2) (where the sum is 0:
// A in mode 0, 0 in the others), the inverse column transforms; error
// (sqrt(sum_m |Psi_m|^2) - A)^2 into err_part[j][blockIdx.x].  Each mode's
// transformed column is parked in S (every row, by the thread that reads it
// back) while the intensity sum over the modes is formed.
template <int N, int CV>
__global__ void __launch_bounds__((ColCfg<N, CV>::THREADS))
k_cols_modulus_modes(const ScanDev* __restrict__ scans, const SlotDev* __restrict__ slots,
                     float2* __restrict__ S, int M, const float2* __restrict__ tw_g) {
    constexpr int C = ColCfg<N, CV>::C, T = ColCfg<N, CV>::T, V = PlanInfo<N>::V;
    __shared__ float2 lds[C * N];
    __shared__ float2 tw[N];
    __shared__ double red[ColCfg<N, CV>::THREADS / 64 + 1];
    const int s0 = blockIdx.y * M;
    const ScanDev sc0 = scans[0];
    const SlotDev sd = slots[s0];
    const ScanDev sc = scan_desc(scans, sc0, sd.scan);
    const int Nw = sc.Nw;
    const int c = threadIdx.x % C, t = threadIdx.x / C;
    const int kx = blockIdx.x * C + c;
    float a[V], tot[V];
    if (sc.A) {  // amplitudes in FFT order
        const float* Aj = sc.A + (size_t)sd.j * N * N + kx;
#pragma unroll
        for (int idx = 0; idx < V; ++idx) a[idx] = ldg(Aj, (size_t)out_pos<N, false>(t, idx) * N);
    } else {  // from the detector-centred intensities
        const float* Ij = sc.I + (size_t)sd.j * N * N;
        const int sx = (kx + N / 2) % N;
#pragma unroll
        for (int idx = 0; idx < V; ++idx) {
            const int ky = out_pos<N, false>(t, idx);
            a[idx] = amplitude_of(ldg(Ij, (size_t)((ky + N / 2) % N) * N + sx));
        }
    }
#pragma unroll
    for (int idx = 0; idx < V; ++idx) tot[idx] = 0.f;
    for (int i = threadIdx.x; i < N; i += blockDim.x) tw[i] = tw_g[i];
    __syncthreads();
    const float sc1 = 1.f / (float)N;
    for (int m = 0; m < M; ++m) {
        float2* col = S + (size_t)(s0 + m) * N * N + kx;
        float2 x[V];
#pragma unroll
        for (int idx = 0; idx < V; ++idx) x[idx] = col[(size_t)min(in_pos<N, false>(t, idx), Nw - 1) * N];
#pragma unroll
        for (int idx = 0; idx < V; ++idx)
            if (in_pos<N, false>(t, idx) >= Nw) x[idx] = make_float2(0.f, 0.f);
        fft_line<N, false>(x, t, lds, ColLds<C>(c), tw);
#pragma unroll
        for (int idx = 0; idx < V; ++idx) {
            const float2 v = cscale(x[idx], sc1);
            tot[idx] += cabs2(v);
            col[(size_t)out_pos<N, false>(t, idx) * N] = v;
        }
        __syncthreads();  // the next mode's transform reuses the exchange buffer
    }
    float accf = 0.f;
    float f[V];
#pragma unroll
    for (int idx = 0; idx < V; ++idx) {
        const bool nz = tot[idx] > 1e-30f;
        const float r = __builtin_amdgcn_rsqf(nz ? tot[idx] : 1.f);  // ~1 / sqrt(sum_m |Psi_m|^2)
        const float d = (nz ? tot[idx] * r : 0.f) - a[idx];
        accf += d * d;
        f[idx] = nz ? a[idx] * r : -1.f;  // -1: the all-zero case
    }
    for (int m = 0; m < M; ++m) {
        float2* col = S + (size_t)(s0 + m) * N * N + kx;
        float2 x[V];
#pragma unroll
        for (int idx = 0; idx < V; ++idx) {
            const float2 v = col[(size_t)out_pos<N, false>(t, idx) * N];
            x[idx] = f[idx] >= 0.f ? cscale(v, f[idx]) : make_float2(m == 0 ? a[idx] : 0.f, 0.f);
        }
        fft_line<N, true>(x, t, lds, ColLds<C>(c), tw);
#pragma unroll
        for (int idx = 0; idx < V; ++idx) {
            const int y = out_pos<N, true>(t, idx);
            if (y < Nw) st_dev(col, (size_t)y * N, x[idx]);
        }
        __syncthreads();
    }
    const double acc = block_sum((double)accf, red, false);
    if (threadIdx.x == 0) sc.err_part[(size_t)sd.j * gridDim.x + blockIdx.x] = acc;
}

// cols_intensity_modes: forward model only, I_out[j] = fftshift sum_m |Psi_m|^2.
template <int N, int CV>
__global__ void __launch_bounds__((ColCfg<N, CV>::THREADS))
k_cols_intensity_modes(const ScanDev* __restrict__ scans, const SlotDev* __restrict__ slots,
                       const float2* __restrict__ S, int M, float* __restrict__ I_out,
                       const float2* __restrict__ tw_g) {
    constexpr int C = ColCfg<N, CV>::C, T = ColCfg<N, CV>::T, V = PlanInfo<N>::V;
    __shared__ float2 lds[C * N];
    __shared__ float2 tw[N];
    const int s0 = blockIdx.y * M;
    const ScanDev sc0 = scans[0];
    const SlotDev sd = slots[s0];
    const int Nw = scan_desc(scans, sc0, sd.scan).Nw;
    const int c = threadIdx.x % C, t = threadIdx.x / C;
    const int kx = blockIdx.x * C + c;
    for (int i = threadIdx.x; i < N; i += blockDim.x) tw[i] = tw_g[i];
    __syncthreads();
    float tot[V];
#pragma unroll
    for (int idx = 0; idx < V; ++idx) tot[idx] = 0.f;
    for (int m = 0; m < M; ++m) {
        const float2* col = S + (size_t)(s0 + m) * N * N + kx;
        float2 x[V];
#pragma unroll
        for (int idx = 0; idx < V; ++idx) {
            const int y = in_pos<N, false>(t, idx);
            x[idx] = y < Nw ? col[(size_t)y * N] : make_float2(0.f, 0.f);
        }
        fft_line<N, false>(x, t, lds, ColLds<C>(c), tw);
#pragma unroll
        for (int idx = 0; idx < V; ++idx) tot[idx] += cabs2(x[idx]);
        __syncthreads();
    }
    const float sc2 = 1.f / ((float)N * (float)N);
    float* Ij = I_out + (size_t)sd.j * N * N;
    const int sx = (kx + N / 2) % N;
#pragma unroll
    for (int idx = 0; idx < V; ++idx) {
        const int ky = out_pos<N, false>(t, idx);
        st_dev(Ij, (size_t)((ky + N / 2) % N) * N + sx, tot[idx] * sc2);
    }
}

// ------------------------------------------------------- rows_inv_update
// grid (maxNw, ngroups): block (r, g) owns probe row r of group g's scan and
// loops over the group's slots in rounds of ULINES.  For each slot s the
// inverse row transform of S[s][r][:] (with the unitary 1/N) gives
// psi'(r, n), n < Nw, and
//   MODE 0, 1 (reconstruction):
//     dpsi = psi' - P(r, n) O_s(r, n);  S[s][r][n] = conj(P(r, n)) dpsi
//     (the object-update numerator term).  P2[r][n] = |P(r, n)|^2 of the
//     batch-start probe and maxP2_row[r] its row maximum, all the object
//     update still needs of the probe.  MODE 1 also updates the probe row in
//     place from the batch sums (slot order, float64 denominators):
//       P(r, n) += sum_s conj(O_s) dpsi / sum_s d_P,s
//       rPIE: d_P,s = (1 - beta)|O_s|^2 + beta max|O_s|^2;  ePIE: max|O_s|^2 / beta
//   MODE 2 (gradient): g = *upstream * psi' (1 when upstream is NULL);  S[s][r][n] = conj(P(r, n)) g and
//     gP(r, n) += sum_s conj(O_s(r, n)) g  (when the scan has a gP).
//   MODE 3, 4 (real positions): as MODE 0 with each slot's translated probe
//     P_s = Pd[s] in place of P in dpsi and in the object numerator; P2 and
//     maxP2_row still describe the untranslated batch-start probe.  MODE 4
//     (probe updated) writes the probe numerators G[s][r][n] = conj(O_s) dpsi
//     for the inverse translation and the float64 denominator sums
//     DP[r][n] = sum_s d_P,s, and leaves P unchanged.  With gfrac (Nw == N)
//     the numerator rows are translated back along x by -d_x(s) =
//     -gfrac[s].y in registers before they are stored.
//   MODE 5, 6 (mixed states): the group's slots come in runs of nmodes (one
//     per probe mode, mode = slot index % nmodes, modes P[m][Nw][Nw]); as
//     MODE 0, 1 with probe mode m in slot s's dpsi and object numerator.
//     P2 = sum_m |P_m|^2 / nmodes and maxP2_row its row maximum, so the
//     object update's per-slot denominators add up over a position's modes
//     to those of the total probe intensity.  MODE 6 updates every mode's
//     row, P_m += sum_s in mode m conj(O_s) dpsi_s / sum_j d_P,j, with one
//     denominator term per position (its mode-0 slot).
template <int N, int RV = 0>
struct UpdCfg {
    static constexpr int T = PlanInfo<N>::T;
    // lines per block: a whole 32-slot mini-batch in one round where LDS allows
    static constexpr int ULINES0 = N <= 256 ? (512 / T < 32 ? 512 / T : 32) : (N == 384 ? 16 : 8);
    static constexpr int ULINES = RV == 0 ? ULINES0 : (ULINES0 > 1 ? ULINES0 / 2 : 1);
    static constexpr int THREADS = ULINES * T;
};

template <int N, int RV, int MODE>
__global__ void __launch_bounds__((UpdCfg<N, RV>::THREADS))
k_rows_inv_update(const ScanDev* __restrict__ scans, const SlotDev* __restrict__ slots,
                  const GroupDev* __restrict__ groups, float2* __restrict__ S,
                  const float* __restrict__ maxO2_part, int nparts, int rpie, float beta,
                  const double* __restrict__ upstream, int nmodes, const float2* __restrict__ Pd, float2* __restrict__ G,
                  double* __restrict__ DP, const float2* __restrict__ gfrac, const float2* __restrict__ tw_g) {
    constexpr int T = UpdCfg<N, RV>::T, ULINES = UpdCfg<N, RV>::ULINES, V = PlanInfo<N>::V;
    constexpr int THREADS = UpdCfg<N, RV>::THREADS;
    constexpr int COLS = (N + THREADS - 1) / THREADS;  // probe columns owned per thread
    constexpr bool SUB = MODE == 3 || MODE == 4;                  // per-slot translated probes
    constexpr bool MIX = MODE == 5 || MODE == 6;                  // probe modes
    constexpr bool ACC = MODE == 1 || MODE == 2 || MODE == 6;     // probe-row sums over the batch
    constexpr bool DEN = MODE == 1 || MODE == 4 || MODE == 6;
    constexpr int NM = MIX ? kMaxModes : 1;                       // probe rows held
    // The transform's exchange buffer doubles as the per-line numerator
    // buffer once a line's transform is done: line l's numerators go to its
    // own region (c_num[l * CSTR + n]), which only its own wavefront touches
    // until the block barrier before the sums.  Line strides of N + N/16
    // (numerators) and N + T (denominators) put a wavefront's lines on
    // different LDS banks.
    constexpr int CSTR = RowLds<N>::stride, DSTR = N + T;
    __shared__ float2 lds[ULINES * RowLds<N>::stride];
    __shared__ float2 tw[N];
    __shared__ float2 s_prow[NM * N];
    __shared__ float c_den[DEN ? ULINES * DSTR : 1];
    __shared__ float s_max[DEN ? kMaxBatch : 1];
    __shared__ int s_py[kMaxBatch], s_px[kMaxBatch];
    __shared__ float red[THREADS / 64 + 1];
    float2* c_num = lds;
    const ScanDev sc0 = scans[0];
    const GroupDev gd = groups[blockIdx.y];
    const ScanDev sc = scan_desc(scans, sc0, gd.scan);
    const int Nw = sc.Nw, Mx = sc.Mx, nb = gd.nb;
    const int r = blockIdx.x;
    if (r >= Nw) return;  // uniform over the block
    const int line = threadIdx.x / T, t = threadIdx.x % T;
    // Inverse-transform input of a round: row r of slot k0 + line (slot 0 of
    // the group for lines past the end, zeroed after the loads).  The first
    // round's loads go out before the prologue below.
    float2 x[V];
    auto load_rows = [&](int k0) {
        const int k = k0 + line;
        const float2* row = S + ((size_t)(gd.s0 + (k < nb ? k : 0)) * N + r) * N;
#pragma unroll
        for (int idx = 0; idx < V; ++idx) x[idx] = row[in_pos<N, true>(t, idx)];
    };
    load_rows(0);

    // Prologue: the twiddles, probe row(s) and slot table are loaded into
    // registers (indices clamped) and stored to LDS afterwards, so their
    // loads are in flight together rather than one loop's after another's.
    const float2* Prow = sc.P + (size_t)r * Nw;
    TwRegs<N, THREADS> twr;
    twr.load(tw_g);
    constexpr int PK = (NM * N + THREADS - 1) / THREADS;
    const int nrow = MIX ? nmodes * N : N;
    float2 prv[PK];
#pragma unroll
    for (int q = 0; q < PK; ++q) {
        const int i = min((int)threadIdx.x + q * THREADS, nrow - 1);
        prv[q] = ldg(Prow, (size_t)(i / N) * Nw * Nw + min(i % N, Nw - 1));
    }
    // the slot table is held in registers until the per-slot maxima below
    // have been loaded too, so that both wait on one round trip
    constexpr int SK = (kMaxBatch + THREADS - 1) / THREADS;
    int spy[SK], spx[SK];
#pragma unroll
    for (int q = 0; q < SK; ++q) {
        const int k = (int)threadIdx.x + q * THREADS;
        if (k < nb) {
            const SlotDev sd = slots[gd.s0 + k];
            spy[q] = sd.py;
            spx[q] = sd.px;
        }
    }
    if constexpr (DEN) {
        // each slot's maximum of |O_s|^2 from the exit-wave pass's partial
        // maxima (nparts per slot: 16 row blocks, or one per window row):
        // G lanes of one wave per slot, 8 loads each in flight (the index
        // clamped to the slot's last part, which leaves the maximum unchanged)
        int G = 64;
        while (G > 1 && G * nb > THREADS) G >>= 1;
        const int lane = (int)threadIdx.x % G;
        for (int kb = 0; kb < nb; kb += THREADS / G) {
            const int k = kb + (int)threadIdx.x / G;
            const float* part = maxO2_part + (size_t)(gd.s0 + min(k, nb - 1)) * nparts;
            float m = 0.f;
            for (int i0 = lane; i0 < nparts; i0 += 8 * G) {
                float v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) v[u] = part[min(i0 + u * G, nparts - 1)];
#pragma unroll
                for (int u = 0; u < 8; ++u) m = fmaxf(m, v[u]);
            }
            for (int o = G / 2; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
            if (k < nb && lane == 0) s_max[k] = m;
        }
    }
#pragma unroll
    for (int q = 0; q < SK; ++q) {
        const int k = (int)threadIdx.x + q * THREADS;
        if (k < nb) {
            s_py[k] = spy[q];
            s_px[k] = spx[q];
        }
    }
    twr.store(tw);
#pragma unroll
    for (int q = 0; q < PK; ++q) {
        const int i = (int)threadIdx.x + q * THREADS;
        if (i < nrow) s_prow[i] = i % N < Nw ? prv[q] : make_float2(0.f, 0.f);
    }
    float2 num[NM][COLS];
    double den[COLS];
#pragma unroll
    for (int c = 0; c < COLS; ++c) {
#pragma unroll
        for (int q = 0; q < NM; ++q) num[q][c] = make_float2(0.f, 0.f);
        den[c] = 0.0;
    }
    __syncthreads();

    const float scl = (MODE == 2 && upstream ? (float)*upstream : 1.f) / (float)N;
    for (int k0 = 0; k0 < nb; k0 += ULINES) {
        const int k = k0 + line;
        const bool live = k < nb;
        const int kk = live ? k : 0;
        float2* row = S + ((size_t)(gd.s0 + kk) * N + r) * N;
        const float2* Orow = sc.O + (size_t)(s_py[kk] + r) * Mx + s_px[kk];
        // every global load of the round is issued before the transform
        float2 o[V], pv[V];
        const float2* Psrow = SUB ? Pd + ((size_t)(gd.s0 + kk) * Nw + r) * Nw : nullptr;
        if (k0 > 0) load_rows(k0);
#pragma unroll
        for (int idx = 0; idx < V; ++idx) {
            if (!live) x[idx] = make_float2(0.f, 0.f);
            const int n = out_pos<N, true>(t, idx);
            o[idx] = live && n < Nw ? Orow[n] : make_float2(0.f, 0.f);
            if constexpr (SUB) pv[idx] = live && n < Nw ? Psrow[n] : make_float2(0.f, 0.f);
        }
        fft_line<N, true>(x, t, lds, RowLdsWave<N>(line), tw);
        if (live) {
            float mO = 0.f;
            if constexpr (DEN) mO = s_max[k];
#pragma unroll
            for (int idx = 0; idx < V; ++idx) {
                const int n = out_pos<N, true>(t, idx);
                if (n < Nw) {
                    const float2 p = SUB ? pv[idx] : s_prow[(MIX ? k % nmodes : 0) * N + n];
                    const float2 d = MODE == 2 ? cscale(x[idx], scl) : csub(cscale(x[idx], scl), cmul(p, o[idx]));
                    st_dev(row, n, cconjmul(p, d));
                    if constexpr (ACC) c_num[line * CSTR + n] = cconjmul(o[idx], d);
                    if constexpr (MODE == 4) {
                        if (gfrac) x[idx] = cconjmul(o[idx], d);  // translated below, then stored
                        else st_dev(G, ((size_t)(gd.s0 + k) * Nw + r) * Nw + n, cconjmul(o[idx], d));
                    }
                    if constexpr (DEN) {
                        const float o2 = cabs2(o[idx]);
                        c_den[line * DSTR + n] = rpie ? fmaf(1.f - beta, o2, beta * mO) : mO / beta;
                    }
                }
            }
        }
        if constexpr (MODE == 4) {
            if (gfrac) {  // uniform: every line of the round takes part in the transforms
#pragma unroll
                for (int idx = 0; idx < V; ++idx)
                    if (!live) x[idx] = make_float2(0.f, 0.f);
                shift_regs<N>(x, live ? -gfrac[gd.s0 + kk].y : 0.f, t, lds, RowLdsWave<N>(line), tw);
                if (live) {
                    float2* grow = G + ((size_t)(gd.s0 + k) * Nw + r) * Nw;
#pragma unroll
                    for (int idx = 0; idx < V; ++idx) st_dev(grow, out_pos<N, true>(t, idx), x[idx]);
                }
            }
        }
        if constexpr (ACC || DEN) {
            __syncthreads();
            const int nl = min(ULINES, nb - k0);
#pragma unroll
            for (int c = 0; c < COLS; ++c) {
                const int n = threadIdx.x + c * THREADS;
                if (n < Nw) {
                    int l0 = 0;
                    if constexpr (!MIX) {
                        // eight lines' values loaded before their adds, which
                        // keep the line order of the loop below
                        for (; l0 + 8 <= nl; l0 += 8) {
                            float2 cn[8];
                            float cd[8];
#pragma unroll
                            for (int u = 0; u < 8; ++u) {
                                if constexpr (ACC) cn[u] = c_num[(l0 + u) * CSTR + n];
                                if constexpr (DEN) cd[u] = c_den[(l0 + u) * DSTR + n];
                            }
#pragma unroll
                            for (int u = 0; u < 8; ++u) {
                                if constexpr (ACC) num[0][c] = cadd(num[0][c], cn[u]);
                                if constexpr (DEN) den[c] += (double)cd[u];
                            }
                        }
                    }
                    for (int l = l0; l < nl; ++l) {
                        if constexpr (MIX) {
                            const int mm = (k0 + l) % nmodes;
                            if constexpr (ACC) {
#pragma unroll
                                for (int q = 0; q < NM; ++q)
                                    if (q == mm) num[q][c] = cadd(num[q][c], c_num[l * CSTR + n]);
                            }
                            if constexpr (DEN)
                                if (mm == 0) den[c] += (double)c_den[l * DSTR + n];
                        } else {
                            if constexpr (ACC) num[0][c] = cadd(num[0][c], c_num[l * CSTR + n]);
                            if constexpr (DEN) den[c] += (double)c_den[l * DSTR + n];
                        }
                    }
                }
            }
            __syncthreads();
        }
    }
    float pmax = 0.f;
#pragma unroll
    for (int c = 0; c < COLS; ++c) {
        const int n = threadIdx.x + c * THREADS;
        if (n >= Nw) continue;
        if constexpr (MODE == 2) {
            if (sc.gP) {
                float2* g = sc.gP + (size_t)r * Nw + n;
                *g = cadd(*g, num[0][c]);
            }
        } else if constexpr (MIX) {
            float q2 = 0.f;
            for (int q = 0; q < nmodes; ++q) q2 += cabs2(s_prow[q * N + n]);
            const float p2 = q2 / (float)nmodes;
            st_dev(sc.P2, (size_t)r * Nw + n, p2);
            pmax = fmaxf(pmax, p2);
            if (MODE == 6 && den[c] > 0.0) {
                const float inv = (float)(1.0 / den[c]);  // the float64 denominator, inverted once
#pragma unroll
                for (int q = 0; q < NM; ++q) {
                    if (q >= nmodes) break;
                    float2 p = s_prow[q * N + n];
                    p.x = fmaf(num[q][c].x, inv, p.x);
                    p.y = fmaf(num[q][c].y, inv, p.y);
                    st_dev(sc.P, (size_t)q * Nw * Nw + (size_t)r * Nw + n, p);
                }
            }
        } else {
            float2 p = s_prow[n];
            const float p2 = cabs2(p);
            st_dev(sc.P2, (size_t)r * Nw + n, p2);
            pmax = fmaxf(pmax, p2);
            if constexpr (MODE == 4) DP[(size_t)r * Nw + n] = den[c];
            if (MODE == 1 && den[c] > 0.0) {
                const float inv = (float)(1.0 / den[c]);  // the float64 denominator, inverted once
                p.x = fmaf(num[0][c].x, inv, p.x);
                p.y = fmaf(num[0][c].y, inv, p.y);
                st_dev(sc.P, (size_t)r * Nw + n, p);
            }
        }
    }
    if constexpr (MODE != 2) {
        pmax = block_max(pmax, red, false);
        if (threadIdx.x == 0) sc.maxP2_row[r] = pmax;
    }
}

}  // namespace mnf
