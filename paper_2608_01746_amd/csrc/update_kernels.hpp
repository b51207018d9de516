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
__device__ __forceinline__ int tile_window_list(const int* __restrict__ pos, const int* __restrict__ bj,
                                                int nb, int Nw, int ty0, int tx0,
                                                int* l_slot, int* l_py, int* l_px) {
    __shared__ int count;
    if (threadIdx.x < 64) {
        int cnt = 0;
        for (int base = 0; base < nb; base += 64) {
            const int s = base + (int)threadIdx.x;
            bool hit = false;
            int py = 0, px = 0;
            if (s < nb) {
                const int j = bj[s];
                py = pos[2 * j];
                px = pos[2 * j + 1];
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

// O[x] += sum_s conj(P(u_s)) D_s(u_s) / sum_s d_O(u_s),  u_s = x - p_s
//   rPIE: d_O = (1 - alpha)|P|^2 + alpha max|P|^2;  ePIE: d_O = max|P|^2 / alpha
// grid (ceil(W / kObjTileX), ceil(H / kObjTileY)) over the box [y0, y0+H) x [x0, x0+W).
__global__ void __launch_bounds__(kObjThreads)
k_object_update(float2* __restrict__ O, int Mx, int y0, int x0, int H, int W,
                const float2* __restrict__ S, int N, const float2* __restrict__ P, int Nw,
                const int* __restrict__ pos, const int* __restrict__ bj, int nb,
                const float* __restrict__ maxP2_part, int nparts, int rpie, float alpha) {
    __shared__ int l_slot[kMaxBatch], l_py[kMaxBatch], l_px[kMaxBatch];
    const int ty0 = y0 + blockIdx.y * kObjTileY, tx0 = x0 + blockIdx.x * kObjTileX;
    const int cnt = tile_window_list(pos, bj, nb, Nw, ty0, tx0, l_slot, l_py, l_px);
    if (cnt == 0) return;
    float mp = 0.f;
    for (int i = 0; i < nparts; ++i) mp = fmaxf(mp, maxP2_part[i]);
    const double maxP2 = mp;
    const int xx = tx0 + (threadIdx.x % kObjTileX);
    for (int r = threadIdx.x / kObjTileX; r < kObjTileY; r += kObjThreads / kObjTileX) {
        const int yy = ty0 + r;
        if (yy >= y0 + H || xx >= x0 + W) continue;
        float2 num = make_float2(0.f, 0.f);
        double den = 0.0;
        for (int k = 0; k < cnt; ++k) {
            const int uy = yy - l_py[k], ux = xx - l_px[k];
            if (uy < 0 || uy >= Nw || ux < 0 || ux >= Nw) continue;
            const float2 p = P[uy * Nw + ux];
            const float2 d = S[((size_t)l_slot[k] * N + uy) * N + ux];
            num = cadd(num, cconjmul(p, d));
            const double p2 = (double)cabs2(p);
            den += rpie ? (1.0 - (double)alpha) * p2 + (double)alpha * maxP2 : maxP2 / (double)alpha;
        }
        if (den > 0.0) {
            float2* o = O + (size_t)yy * Mx + xx;
            const double inv = 1.0 / den;
            float2 v = *o;
            v.x = (float)((double)v.x + (double)num.x * inv);
            v.y = (float)((double)v.y + (double)num.y * inv);
            *o = v;
        }
    }
}

// Pn(u) = P(u) + sum_s conj(O_s(u)) D_s(u) / sum_s d_P,s(u)   (pre-update O)
//   rPIE: d_P,s = (1 - beta)|O_s|^2 + beta max|O_s|^2;  ePIE: max|O_s|^2 / beta
// grid ceil(Nw^2 / 256), block 256.
__global__ void __launch_bounds__(256)
k_probe_update(const float2* __restrict__ S, int N, const float2* __restrict__ O, int Mx,
               const float2* __restrict__ P, float2* __restrict__ Pn, int Nw,
               const int* __restrict__ pos, const int* __restrict__ bj, int nb,
               const float* __restrict__ maxO2_part, int nparts, int rpie, float beta) {
    __shared__ float s_max[kMaxBatch];
    __shared__ int s_py[kMaxBatch], s_px[kMaxBatch];
    for (int s = threadIdx.x; s < nb; s += blockDim.x) {
        float m = 0.f;
        for (int i = 0; i < nparts; ++i) m = fmaxf(m, maxO2_part[(size_t)s * nparts + i]);
        s_max[s] = m;
        const int j = bj[s];
        s_py[s] = pos[2 * j];
        s_px[s] = pos[2 * j + 1];
    }
    __syncthreads();
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= Nw * Nw) return;
    const int uy = u / Nw, ux = u % Nw;
    float2 num = make_float2(0.f, 0.f);
    double den = 0.0;
    for (int s = 0; s < nb; ++s) {
        const float2 o = O[(size_t)(s_py[s] + uy) * Mx + s_px[s] + ux];
        const float2 d = S[((size_t)s * N + uy) * N + ux];
        num = cadd(num, cconjmul(o, d));
        const double o2 = (double)cabs2(o);
        den += rpie ? (1.0 - (double)beta) * o2 + (double)beta * (double)s_max[s]
                    : (double)s_max[s] / (double)beta;
    }
    float2 p = P[u];
    if (den > 0.0) {
        const double inv = 1.0 / den;
        p.x = (float)((double)p.x + (double)num.x * inv);
        p.y = (float)((double)p.y + (double)num.y * inv);
    }
    Pn[u] = p;
}

// gO[x] += sum_s conj(P(u_s)) G_s(u_s) over the box (gradient scatter).
__global__ void __launch_bounds__(kObjThreads)
k_grad_object(float2* __restrict__ gO, int Mx, int y0, int x0, int H, int W,
              const float2* __restrict__ S, int N, const float2* __restrict__ P, int Nw,
              const int* __restrict__ pos, const int* __restrict__ bj, int nb) {
    __shared__ int l_slot[kMaxBatch], l_py[kMaxBatch], l_px[kMaxBatch];
    const int ty0 = y0 + blockIdx.y * kObjTileY, tx0 = x0 + blockIdx.x * kObjTileX;
    const int cnt = tile_window_list(pos, bj, nb, Nw, ty0, tx0, l_slot, l_py, l_px);
    if (cnt == 0) return;
    const int xx = tx0 + (threadIdx.x % kObjTileX);
    for (int r = threadIdx.x / kObjTileX; r < kObjTileY; r += kObjThreads / kObjTileX) {
        const int yy = ty0 + r;
        if (yy >= y0 + H || xx >= x0 + W) continue;
        float2 acc = make_float2(0.f, 0.f);
        bool any = false;
        for (int k = 0; k < cnt; ++k) {
            const int uy = yy - l_py[k], ux = xx - l_px[k];
            if (uy < 0 || uy >= Nw || ux < 0 || ux >= Nw) continue;
            acc = cadd(acc, cconjmul(P[uy * Nw + ux], S[((size_t)l_slot[k] * N + uy) * N + ux]));
            any = true;
        }
        if (any) {
            float2* g = gO + (size_t)yy * Mx + xx;
            *g = cadd(*g, acc);
        }
    }
}

// gP(u) += sum_s conj(O_s(u)) G_s(u).
__global__ void __launch_bounds__(256)
k_grad_probe(const float2* __restrict__ S, int N, const float2* __restrict__ O, int Mx,
             float2* __restrict__ gP, int Nw, const int* __restrict__ pos,
             const int* __restrict__ bj, int nb) {
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= Nw * Nw) return;
    const int uy = u / Nw, ux = u % Nw;
    float2 acc = make_float2(0.f, 0.f);
    for (int s = 0; s < nb; ++s) {
        const int j = bj[s];
        const float2 o = O[(size_t)(pos[2 * j] + uy) * Mx + pos[2 * j + 1] + ux];
        acc = cadd(acc, cconjmul(o, S[((size_t)s * N + uy) * N + ux]));
    }
    gP[u] = cadd(gP[u], acc);
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
