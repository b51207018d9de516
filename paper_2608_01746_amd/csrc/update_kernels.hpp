// Object / probe accumulation kernels (mini-batched ePIE / rPIE updates and
// the gradient scatter).  Output-stationary: every output pixel is owned by
// one thread, which sums the contributions of the batch's windows in slot
// order, so results are deterministic and no atomics are used.
#pragma once

#include "kernels_common.hpp"

namespace mnf {

constexpr int kObjTileY = 16, kObjTileX = 64, kObjThreads = 256;

// Ordered list (in slot order) of the batch slots whose window overlaps the
// tile [ty0, ty0 + kObjTileY) x [tx0, tx0 + kObjTileX).  Wave 0 builds it with
// ballots; every thread returns the count.
__device__ __forceinline__ int tile_window_list(const int2* __restrict__ bp, int nb, int Nw, int ty0, int tx0,
                                                int* l_slot, int* l_py, int* l_px) {
    __shared__ int count;
    if (threadIdx.x < 64) {
        int cnt = 0;
        for (int base = 0; base < nb; base += 64) {
            const int s = base + (int)threadIdx.x;
            bool hit = false;
            int py = 0, px = 0;
            if (s < nb) {
                const int2 c = bp[s];
                py = c.x;
                px = c.y;
                hit = py < ty0 + kObjTileY && py + Nw > ty0 && px < tx0 + kObjTileX && px + Nw > tx0;
            }
            const unsigned long long m = __ballot(hit);
            if (hit) {
                const int k = cnt + __popcll(m & ((1ull << threadIdx.x) - 1ull));
                l_slot[k] = s;
                l_py[k] = py;
                l_px[k] = px;
            }
            cnt += __popcll(m);
        }
        if (threadIdx.x == 0) count = cnt;
    }
    __syncthreads();
    return count;
}

// O[x] += sum_s W_s(u_s) / sum_s d_O(u_s),  u_s = x - p_s, over the windows of
// the batch that contain x, where W_s = conj(P) dpsi_s (left in S by
// rows_inv_update) and, from the batch-start probe intensity P2 = |P|^2,
//   rPIE: d_O = (1 - alpha) P2 + alpha max P2;  ePIE: d_O = max P2 / alpha.
// grid (ceil(W / kObjTileX), ceil(H / kObjTileY)) over the box [y0, y0+H) x [x0, x0+W).
// Each thread owns one column and kObjRows rows of the tile; loads are
// issued unconditionally from clamped addresses so that several windows'
// loads are in flight at once.
constexpr int kObjRows = kObjTileY / (kObjThreads / kObjTileX);
constexpr int kObjChunk = 8;

__global__ void __launch_bounds__(kObjThreads)
k_object_update(float2* __restrict__ O, int Mx, int y0, int x0, int H, int W,
                const float2* __restrict__ S, int N, const float* __restrict__ P2, int Nw,
                const int2* __restrict__ bp, int nb,
                const float* __restrict__ maxP2_part, int nparts, int rpie, float alpha) {
    __shared__ int l_slot[kMaxBatch], l_py[kMaxBatch], l_px[kMaxBatch];
    const int ty0 = y0 + blockIdx.y * kObjTileY, tx0 = x0 + blockIdx.x * kObjTileX;
    const int cnt = tile_window_list(bp, nb, Nw, ty0, tx0, l_slot, l_py, l_px);
    if (cnt == 0) return;
    float mp = 0.f;
    for (int i = 0; i < nparts; ++i) mp = fmaxf(mp, maxP2_part[i]);
    const float a = rpie ? 1.f - alpha : 0.f;
    const double cst = rpie ? (double)alpha * (double)mp : (double)mp / (double)alpha;
    const int xx = tx0 + (threadIdx.x % kObjTileX);
    const int yb = ty0 + (threadIdx.x / kObjTileX) * kObjRows;
    float2 num[kObjRows];
    double den[kObjRows];
#pragma unroll
    for (int q = 0; q < kObjRows; ++q) {
        num[q] = make_float2(0.f, 0.f);
        den[q] = 0.0;
    }
    // windows in chunks: every load of a chunk is issued before any is used
    for (int k0 = 0; k0 < cnt; k0 += kObjChunk) {
        float2 w[kObjChunk][kObjRows];
        float p2[kObjChunk][kObjRows];
        bool in[kObjChunk][kObjRows];
#pragma unroll
        for (int c = 0; c < kObjChunk; ++c) {
            const int k = min(k0 + c, cnt - 1);
            const int ux = xx - l_px[k];
            const bool inx = k0 + c < cnt && ux >= 0 && ux < Nw;
            const int uxc = min(max(ux, 0), Nw - 1);
            const float2* Sk = S + (size_t)l_slot[k] * N * N + uxc;
#pragma unroll
            for (int q = 0; q < kObjRows; ++q) {
                const int uy = yb + q - l_py[k];
                in[c][q] = inx && uy >= 0 && uy < Nw;
                const int uyc = min(max(uy, 0), Nw - 1);
                w[c][q] = Sk[(size_t)uyc * N];
                p2[c][q] = P2[(size_t)uyc * Nw + uxc];
            }
        }
#pragma unroll
        for (int c = 0; c < kObjChunk; ++c)
#pragma unroll
            for (int q = 0; q < kObjRows; ++q)
                if (in[c][q]) {
                    num[q] = cadd(num[q], w[c][q]);
                    den[q] += (double)(a * p2[c][q]) + cst;
                }
    }
    if (xx >= x0 + W) return;
#pragma unroll
    for (int q = 0; q < kObjRows; ++q) {
        const int yy = yb + q;
        if (yy < y0 + H && den[q] > 0.0) {
            float2* o = O + (size_t)yy * Mx + xx;
            const double inv = 1.0 / den[q];
            float2 v = *o;
            v.x = (float)((double)v.x + (double)num[q].x * inv);
            v.y = (float)((double)v.y + (double)num[q].y * inv);
            *o = v;
        }
    }
}

// gO[x] += sum_s W_s(u_s) over the box (gradient scatter), W_s = conj(P) g_s
// left in S by rows_inv_update.  Same tiling and load scheme as k_object_update.
__global__ void __launch_bounds__(kObjThreads)
k_grad_object(float2* __restrict__ gO, int Mx, int y0, int x0, int H, int W,
              const float2* __restrict__ S, int N, int Nw, const int2* __restrict__ bp, int nb) {
    __shared__ int l_slot[kMaxBatch], l_py[kMaxBatch], l_px[kMaxBatch];
    const int ty0 = y0 + blockIdx.y * kObjTileY, tx0 = x0 + blockIdx.x * kObjTileX;
    const int cnt = tile_window_list(bp, nb, Nw, ty0, tx0, l_slot, l_py, l_px);
    if (cnt == 0) return;
    const int xx = tx0 + (threadIdx.x % kObjTileX);
    const int yb = ty0 + (threadIdx.x / kObjTileX) * kObjRows;
    float2 acc[kObjRows];
    bool any[kObjRows];
#pragma unroll
    for (int q = 0; q < kObjRows; ++q) {
        acc[q] = make_float2(0.f, 0.f);
        any[q] = false;
    }
    for (int k0 = 0; k0 < cnt; k0 += kObjChunk) {
        float2 w[kObjChunk][kObjRows];
        bool in[kObjChunk][kObjRows];
#pragma unroll
        for (int c = 0; c < kObjChunk; ++c) {
            const int k = min(k0 + c, cnt - 1);
            const int ux = xx - l_px[k];
            const bool inx = k0 + c < cnt && ux >= 0 && ux < Nw;
            const float2* Sk = S + (size_t)l_slot[k] * N * N + min(max(ux, 0), Nw - 1);
#pragma unroll
            for (int q = 0; q < kObjRows; ++q) {
                const int uy = yb + q - l_py[k];
                in[c][q] = inx && uy >= 0 && uy < Nw;
                w[c][q] = Sk[(size_t)min(max(uy, 0), Nw - 1) * N];
            }
        }
#pragma unroll
        for (int c = 0; c < kObjChunk; ++c)
#pragma unroll
            for (int q = 0; q < kObjRows; ++q)
                if (in[c][q]) {
                    acc[q] = cadd(acc[q], w[c][q]);
                    any[q] = true;
                }
    }
    if (xx >= x0 + W) return;
#pragma unroll
    for (int q = 0; q < kObjRows; ++q) {
        const int yy = yb + q;
        if (yy < y0 + H && any[q]) {
            float2* g = gO + (size_t)yy * Mx + xx;
            *g = cadd(*g, acc[q]);
        }
    }
}

__global__ void k_copy_c64(float2* __restrict__ dst, const float2* __restrict__ src, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

__global__ void k_zero_c64(float2* __restrict__ dst, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = make_float2(0.f, 0.f);
}

// out[0] = scale * sum(in[0..n)) in a fixed order (one block of 256 threads);
// if div != NULL the result is divided by *div (0 when *div == 0).
__global__ void __launch_bounds__(256)
k_sum_f64(const double* __restrict__ in, size_t n, const double* __restrict__ div, double scale,
          double* __restrict__ out) {
    __shared__ double red[4];
    double a = 0.0;
    for (size_t i = threadIdx.x; i < n; i += 256) a += in[i];
    a = block_sum(a, red);
    if (threadIdx.x == 0) {
        double r = a * scale;
        if (div) r = *div > 0.0 ? r / *div : 0.0;
        *out = r;
    }
}

// part[j] = sum_q max(I[j][q], 0) (the squared amplitudes), one block per position.
__global__ void __launch_bounds__(256)
k_sum_amplitude2(const float* __restrict__ I, size_t npix, double* __restrict__ part) {
    __shared__ double red[4];
    const float* Ij = I + (size_t)blockIdx.x * npix;
    double a = 0.0;
    for (size_t i = threadIdx.x; i < npix; i += 256) a += (double)fmaxf(Ij[i], 0.f);
    a = block_sum(a, red);
    if (threadIdx.x == 0) part[blockIdx.x] = a;
}

}  // namespace mnf
