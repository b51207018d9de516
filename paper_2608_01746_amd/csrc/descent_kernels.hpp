// Full-batch gradient descent on the far-field loss (the adjoint of
// Eqs. 2-3 under the Poisson model of the Introduction): initial step sizes
// from the starting object and probe, and the backtracking step.
//
//   eta_O = 1 / (2 max_x sum_j |P(x - p_j)|^2)   (object grid x)
//   eta_P = 1 / (2 max_u sum_j |O(p_j + u)|^2)   (probe window u)
//
// i.e. the inverse of the largest diagonal curvature of the amplitude loss
// in O (resp. P) with the other held fixed.  Each sum is formed by the
// thread that owns its pixel, over the positions in index order (no
// atomics), and maxima are reduced per block, then over blocks.
#pragma once

#include "kernels_common.hpp"

namespace mnf {

constexpr int kDescentThreads = 256;
constexpr int kDescentPosChunk = 512;  // positions staged in LDS at a time

__device__ __forceinline__ float block_max_f(float v, float* red) {
    v = wave_max(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    float m = red[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = fmaxf(m, red[w]);
    return m;
}

// Illumination max over the box [by0, by0 + bh) x [bx0, bx0 + bw) of the
// object (the union of the windows): thread per pixel, sum over the windows
// that contain it of |P(y - py, x - px)|^2; block maxima to part[blockIdx.x].
// pos int32 [J][2] (y, x) window corners.
__global__ void __launch_bounds__(kDescentThreads)
k_illum_max(const float2* __restrict__ P, int Nw, const int32_t* __restrict__ pos, int J, int by0, int bx0, int bh,
            int bw, float* __restrict__ part) {
    __shared__ int l_py[kDescentPosChunk], l_px[kDescentPosChunk];
    __shared__ float red[kDescentThreads / 64];
    const long long i = (long long)blockIdx.x * kDescentThreads + threadIdx.x;
    const bool live = i < (long long)bh * bw;
    const int y = by0 + (live ? (int)(i / bw) : 0), x = bx0 + (live ? (int)(i % bw) : 0);
    float s = 0.f;
    for (int j0 = 0; j0 < J; j0 += kDescentPosChunk) {
        const int n = min(kDescentPosChunk, J - j0);
        __syncthreads();  // the previous chunk has been read
        for (int k = threadIdx.x; k < n; k += kDescentThreads) {
            l_py[k] = pos[2 * (size_t)(j0 + k)];
            l_px[k] = pos[2 * (size_t)(j0 + k) + 1];
        }
        __syncthreads();
        for (int k = 0; k < n; ++k) {
            const int uy = y - l_py[k], ux = x - l_px[k];
            if (uy >= 0 && uy < Nw && ux >= 0 && ux < Nw) s += cabs2(ldg(P, (size_t)uy * Nw + ux));
        }
    }
    const float m = block_max_f(live ? s : 0.f, red);
    if (threadIdx.x == 0) part[blockIdx.x] = m;
}

// Coverage max over the probe window: thread per probe pixel u, sum over all
// positions of |O(p_j + u)|^2; block maxima to part[blockIdx.x].
__global__ void __launch_bounds__(kDescentThreads)
k_cover_max(const float2* __restrict__ O, int Mx, int Nw, const int32_t* __restrict__ pos, int J,
            float* __restrict__ part) {
    __shared__ int l_py[kDescentPosChunk], l_px[kDescentPosChunk];
    __shared__ float red[kDescentThreads / 64];
    const int i = blockIdx.x * kDescentThreads + threadIdx.x;
    const bool live = i < Nw * Nw;
    const int uy = live ? i / Nw : 0, ux = live ? i % Nw : 0;
    float s = 0.f;
    for (int j0 = 0; j0 < J; j0 += kDescentPosChunk) {
        const int n = min(kDescentPosChunk, J - j0);
        __syncthreads();
        for (int k = threadIdx.x; k < n; k += kDescentThreads) {
            l_py[k] = pos[2 * (size_t)(j0 + k)];
            l_px[k] = pos[2 * (size_t)(j0 + k) + 1];
        }
        __syncthreads();
        for (int k = 0; k < n; ++k) s += cabs2(ldg(O, (size_t)(l_py[k] + uy) * Mx + l_px[k] + ux));
    }
    const float m = block_max_f(live ? s : 0.f, red);
    if (threadIdx.x == 0) part[blockIdx.x] = m;
}

// eta[0] = eta_O, eta[1] = eta_P: the caller's value where it is > 0, else
// 1 / (2 max) over the block maxima (0, i.e. no step, when the maximum is 0).
// One block.
__global__ void __launch_bounds__(kDescentThreads)
k_step_sizes(const float* __restrict__ partO, int nO, const float* __restrict__ partP, int nP, double etaO,
             double etaP, double* __restrict__ eta) {
    __shared__ float red[kDescentThreads / 64];
    float mo = 0.f;
    for (int i = threadIdx.x; i < nO; i += kDescentThreads) mo = fmaxf(mo, partO[i]);
    mo = block_max_f(mo, red);
    __syncthreads();  // red is reused
    float mp = 0.f;
    for (int i = threadIdx.x; i < nP; i += kDescentThreads) mp = fmaxf(mp, partP[i]);
    mp = block_max_f(mp, red);
    if (threadIdx.x == 0) {
        eta[0] = etaO > 0.0 ? etaO : (mo > 0.f ? 1.0 / (2.0 * (double)mo) : 0.0);
        eta[1] = etaP > 0.0 ? etaP : (mp > 0.f ? 1.0 / (2.0 * (double)mp) : 0.0);
    }
}

// Relative increase of a pass's loss over the reference that still counts
// as no increase: a bound on the float32 evaluation error of the loss (the
// Poisson loss carries a large data-only constant, so late improvements are
// small relative to it and rounding noise must not reject a good step).
constexpr double kDescentTol = 1e-6;

// Backtracking state: the loss of the last accepted pass (the reference) and
// the decision of the current pass.
struct DescentState {
    double best;
    int accept;
    int pad_;
};

// After pass `step` (its loss in *loss): accept it (the first pass, or a loss
// <= reference + kDescentTol |reference|; a NaN loss never compares <=) or
// halve both step sizes.  Copies the loss to *loss_dst when set.  One thread.
__global__ void k_descent_decide(const double* __restrict__ loss, int step, DescentState* __restrict__ stt,
                                 double* __restrict__ eta, double* __restrict__ loss_dst) {
    if (threadIdx.x != 0) return;
    const double L = *loss;
    if (loss_dst) *loss_dst = L;
    const bool acc = step == 0 || L <= stt->best + kDescentTol * fabs(stt->best);
    if (acc) {
        stt->best = L;
    } else {
        eta[0] *= 0.5;
        eta[1] *= 0.5;
    }
    stt->accept = acc ? 1 : 0;
}

// The next point along one variable (n values): an accepted pass saves the
// point X and its gradient G as the best (Xb, Gb) and steps X -= eta G; a
// rejected pass restarts from the best, X = Xb - eta Gb (eta = *eta_p, already
// halved, rounded to float once).
__global__ void __launch_bounds__(kDescentThreads)
k_descent_update(float2* __restrict__ X, const float2* __restrict__ G, float2* __restrict__ Xb,
                 float2* __restrict__ Gb, size_t n, const double* __restrict__ eta_p,
                 const DescentState* __restrict__ stt) {
    const size_t i = (size_t)blockIdx.x * kDescentThreads + threadIdx.x;
    if (i >= n) return;
    const float eta = (float)*eta_p;
    float2 x, g;
    if (stt->accept) {
        x = X[i];
        g = ldg(G, i);
        Xb[i] = x;
        Gb[i] = g;
    } else {
        x = Xb[i];
        g = Gb[i];
    }
    x.x = fmaf(-eta, g.x, x.x);
    x.y = fmaf(-eta, g.y, x.y);
    X[i] = x;
}

}  // namespace mnf
