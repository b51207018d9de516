// Object update of one mini-batch fused with the exit-wave row transforms of
// the next (the single-scan, integer-position, single-mode reconstruction).
//
// The four passes of a mini-batch b are: exit-wave rows, columns with the
// modulus projection, inverse rows with the probe update, object update.
// The object update of b and the exit-wave rows of b + 1 touch the object
// row by row, so one object-row-stationary pass does both: a block owns
// kObjRowsPerBlock rows of the scan's object box and
//   1. updates them from batch b (every pixel summed over b's windows in slot
//      order, the same sums as k_object_update) and keeps the updated rows
//      in LDS;
//   2. forms every exit-wave row of batch b + 1 that lies in those object
//      rows, psi = P_new(r, :) * O_new(y, px + :) (Eq. 2), from the rows in
//      LDS, transforms it (first half of Eq. 3) and stores it to the other
//      pattern buffer, with the row's maximum of |O|^2 for the probe
//      denominators of batch b + 1.
// The first batch of a call runs step 2 only, the last step 1 only.  Each
// block touches only its own object rows, so the pass needs no ordering
// between blocks; results equal those of k_object_update and k_rows_fwd.
#pragma once

#include "kernels_common.hpp"
#include "tables.hpp"

namespace mnf {

constexpr int kObjRowsPerBlock = 2;   // object rows owned by a block
constexpr int kObjRowThreads = 256;
constexpr int kObjRowMaxWidth = 1024; // widest object box held in LDS (wider boxes take the four-pass path)
constexpr int kObjRowChunk = 8;       // windows whose loads are issued together

// Windows of a slot list that cover any of the object rows [y0, y0 + R):
// wave `wv` builds the list (slot order) with ballots into l_slot / l_py /
// l_px and stores its length in *count; the caller synchronises.
__device__ __forceinline__ void objrow_list(const SlotDev* __restrict__ slots, int nb, int Nw, int y0, int R,
                                            int* l_slot, int* l_py, int* l_px, int* count) {
    const int lane = threadIdx.x & 63;
    int cnt = 0;
    for (int base = 0; base < nb; base += 64) {
        const int k = base + lane;
        bool hit = false;
        int py = 0, px = 0;
        if (k < nb) {
            const SlotDev sd = slots[k];
            py = sd.py;
            px = sd.px;
            hit = py < y0 + R && py + Nw > y0;
        }
        const unsigned long long m = __ballot(hit);
        if (hit) {
            const int q = cnt + __popcll(m & ((1ull << lane) - 1ull));
            l_slot[q] = k;
            l_py[q] = py;
            l_px[q] = px;
        }
        cnt += __popcll(m);
    }
    if (lane == 0) *count = cnt;
}

// grid (ceil(bh / kObjRowsPerBlock)), kObjRowThreads threads; one scan
// (scans[0]).  Batch b: slots_u[0..nb_u), its numerators conj(P) dpsi in
// S_u[slot][Nw rows][N] (left by the inverse row pass); nb_u = 0 skips the
// update.  Batch b + 1: slots_f[0..nb_f), rows written to S_f[slot][r][N]
// (r < Nw) and maxima |O|^2 of each window row to maxO2_part[slot][r];
// nb_f = 0 skips them.
template <int N>
__global__ void __launch_bounds__(kObjRowThreads)
k_obj_rows(const ScanDev* __restrict__ scans, const SlotDev* __restrict__ slots_u, int nb_u,
           const float2* __restrict__ S_u, const SlotDev* __restrict__ slots_f, int nb_f, float2* __restrict__ S_f,
           float* __restrict__ maxO2_part, int rpie, float alpha, const float2* __restrict__ tw_g) {
    constexpr int R = kObjRowsPerBlock, THREADS = kObjRowThreads;
    constexpr int T = PlanInfo<N>::T, V = PlanInfo<N>::V, LINES = THREADS / T;
    static_assert(THREADS % T == 0 && 64 % T == 0, "a transform line lies inside one wave");
    // the exchange buffer of the transforms also holds batch b's window list
    // (only used before the first transform)
    constexpr int XCH = LINES * RowLds<N>::stride;
    static_assert(XCH * 2 >= 3 * kMaxBatch, "window list fits the exchange buffer");
    __shared__ float2 lds[XCH];
    __shared__ float2 tw[N];
    __shared__ float2 orow[R][kObjRowMaxWidth];
    __shared__ int f_slot[kMaxBatch], f_py[kMaxBatch], f_px[kMaxBatch];
    __shared__ int n_u, n_f;
    __shared__ float red[THREADS / 64];
    int* u_slot = (int*)lds;
    int* u_py = u_slot + kMaxBatch;
    int* u_px = u_py + kMaxBatch;

    const ScanDev sc = scans[0];
    const int Nw = sc.Nw, Mx = sc.Mx;
    const int y0 = sc.by0 + blockIdx.x * R;
    const int rows = min(R, sc.by0 + sc.bh - y0);
    const int w = threadIdx.x >> 6;
    // the twiddles and the probe's row maxima are loaded first; wave 0 lists
    // batch b's windows, wave 1 batch b + 1's
    TwRegs<N, THREADS> twr;
    if (nb_f > 0) twr.load(tw_g);
    const int i0 = (int)threadIdx.x, i1 = i0 + THREADS;
    float vmax0 = 0.f, vmax1 = 0.f;
    if (nb_u > 0) {
        vmax0 = ldg(sc.maxP2_row, min(i0, Nw - 1));
        vmax1 = ldg(sc.maxP2_row, min(i1, Nw - 1));
    }
    if (w == 0) {
        if (nb_u > 0) objrow_list(slots_u, nb_u, Nw, y0, rows, u_slot, u_py, u_px, &n_u);
        else if (threadIdx.x == 0) n_u = 0;
    } else if (w == 1) {
        if (nb_f > 0) objrow_list(slots_f, nb_f, Nw, y0, rows, f_slot, f_py, f_px, &n_f);
        else if (threadIdx.x == 64) n_f = 0;
    }
    static_assert(2 * THREADS >= 512, "two row maxima per thread cover the largest probe");
    {
        float m = fmaxf(i0 < Nw ? vmax0 : 0.f, i1 < Nw ? vmax1 : 0.f);
        m = wave_max(m);
        if ((threadIdx.x & 63) == 0) red[w] = m;
    }
    if (nb_f > 0) twr.store(tw);
    __syncthreads();
    const int cu = n_u, cf = n_f;
    if (cu == 0 && cf == 0) return;  // uniform: no window of either batch reaches these rows

    // ---- 1. object update of batch b (output-stationary, slot order)
    float mp = red[0];
#pragma unroll
    for (int q = 1; q < THREADS / 64; ++q) mp = fmaxf(mp, red[q]);
    const float a = rpie ? 1.f - alpha : 0.f;
    const double cst = rpie ? (double)alpha * (double)mp : (double)mp / (double)alpha;
    const int bw = sc.bw;
    for (int xb = 0; xb < bw; xb += THREADS) {
        const int xi = xb + (int)threadIdx.x;  // column in the box
        const int xx = sc.bx0 + min(xi, bw - 1);
        float2 ov[R];
#pragma unroll
        for (int q = 0; q < R; ++q) ov[q] = ldg(sc.O, (size_t)(y0 + min(q, rows - 1)) * Mx + xx);
        float2 num[R];
        double den[R];
#pragma unroll
        for (int q = 0; q < R; ++q) {
            num[q] = make_float2(0.f, 0.f);
            den[q] = 0.0;
        }
        for (int k0 = 0; k0 < cu; k0 += kObjRowChunk) {
            // slots past the window count (uniform) issue no loads; pixels
            // outside a window add zero
            const int nc = min(kObjRowChunk, cu - k0);
            float2 wv[kObjRowChunk][R];
            float p2[kObjRowChunk][R];
            bool in[kObjRowChunk][R];
#pragma unroll
            for (int c = 0; c < kObjRowChunk; ++c) {
                if (c < nc) {
                    const int k = k0 + c;
                    const int ux = xx - u_px[k];
                    const bool inx = ux >= 0 && ux < Nw && xi < bw;
                    const int uxc = min(max(ux, 0), Nw - 1);
                    const float2* Sk = S_u + (size_t)u_slot[k] * N * N + uxc;
#pragma unroll
                    for (int q = 0; q < R; ++q) {
                        const int uy = y0 + q - u_py[k];
                        in[c][q] = inx && q < rows && uy >= 0 && uy < Nw;
                        const int uyc = min(max(uy, 0), Nw - 1);
                        wv[c][q] = Sk[(size_t)uyc * N];
                        p2[c][q] = ldg(sc.P2, (size_t)uyc * Nw + uxc);
                    }
                } else {
#pragma unroll
                    for (int q = 0; q < R; ++q) {
                        in[c][q] = false;
                        wv[c][q] = make_float2(0.f, 0.f);
                        p2[c][q] = 0.f;
                    }
                }
            }
#pragma unroll
            for (int c = 0; c < kObjRowChunk; ++c)
#pragma unroll
                for (int q = 0; q < R; ++q) {
                    const bool u = in[c][q];
                    num[q] = cadd(num[q], u ? wv[c][q] : make_float2(0.f, 0.f));
                    den[q] += u ? (double)(a * p2[c][q]) + cst : 0.0;
                }
        }
#pragma unroll
        for (int q = 0; q < R; ++q) {
            if (q >= rows || xi >= bw) continue;
            float2 v = ov[q];
            if (den[q] > 0.0) {
                const float inv = (float)(1.0 / den[q]);  // the float64 denominator, inverted once
                v.x = fmaf(num[q].x, inv, v.x);
                v.y = fmaf(num[q].y, inv, v.y);
                st_dev(sc.O, (size_t)(y0 + q) * Mx + xx, v);
            }
            orow[q][xi] = v;
        }
    }
    if (cf == 0) return;  // uniform
    __syncthreads();  // the updated rows are in LDS; the window list's space is free

    // ---- 2. exit-wave rows of batch b + 1 from the rows in LDS
    const int line = threadIdx.x / T, t = threadIdx.x % T;
    const int nlines = cf * R;
    for (int l0 = 0; l0 < nlines; l0 += LINES) {
        const int l = l0 + line;
        const int e = min(l, nlines - 1) / R;
        const int yy = y0 + min(l, nlines - 1) % R;
        const int py = f_py[e], px = f_px[e];
        const int r = yy - py;
        const bool live = l < nlines && yy < y0 + rows && r >= 0 && r < Nw;
        const int rc = min(max(r, 0), Nw - 1);
        const float2* Prow = sc.P + (size_t)rc * Nw;
        float2 x[V];
        float mO = 0.f;
        float2 p[V];
#pragma unroll
        for (int idx = 0; idx < V; ++idx) p[idx] = ldg(Prow, min(in_pos<N, false>(t, idx), Nw - 1));
        const float2* orw = orow[min(yy - y0, R - 1)];
        const int ox = px - sc.bx0;
#pragma unroll
        for (int idx = 0; idx < V; ++idx) {
            const int n = in_pos<N, false>(t, idx);
            const bool in = live && n < Nw;
            const float2 o = orw[min(ox + min(n, Nw - 1), kObjRowMaxWidth - 1)];
            x[idx] = in ? cmul(p[idx], o) : make_float2(0.f, 0.f);
            mO = fmaxf(mO, in ? cabs2(o) : 0.f);
        }
        fft_line<N, false>(x, t, lds, RowLdsWave<N>(line), tw);
        if (live) {
            float2* row = S_f + ((size_t)f_slot[e] * N + r) * N;
#pragma unroll
            for (int idx = 0; idx < V; ++idx) st_dev(row, out_pos<N, false>(t, idx), x[idx]);
        }
        // maximum over the line's T lanes (consecutive lanes of one wave)
#pragma unroll
        for (int o = T / 2; o > 0; o >>= 1) mO = fmaxf(mO, __shfl_xor(mO, o, 64));
        if (live && t == 0) st_dev(maxO2_part, (size_t)f_slot[e] * Nw + r, mO);
    }
}

}  // namespace mnf
