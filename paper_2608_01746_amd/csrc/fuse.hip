// Multi-scale non-linear fusion (Methods 3.4, Eqs. 5-10) of exposure brackets.
//
// Level 0 is never stored.  Its values (I_tilde_k and the weight W_k, Eq. 5
// normalised over the K frames) are pointwise functions of the K raw counts
// of a pixel, cheaper to recompute from the 2-byte counts than to write and
// re-read as 4-byte pyramids:
//   1. k_fuse_level1_tiled (K <= 5; k_fuse_level1 beyond): level 1 of every
//      exposure's image and weight pyramid straight from the raw counts
//      (reduce of the recomputed level 0);
//   2. levels 2..L of every exposure by LDS-tiled reduce (one launch per level);
//   3. from the weighted base of level L down to level 1, one launch per
//      level: the modulated, quantised band-pass coefficients of the level
//      summed over exposures in exposure order, plus the expanded collapse
//      of the level above (R_l = F_l + U(R_{l+1}), R_L = F_L);
//   4. k_fuse_final: per level-0 pixel, the level-0 coefficients of all
//      exposures (recomputed level 0 minus the expanded level 1), quantised
//      per exposure, summed, plus the expanded level-1 collapse.
// The per-exposure reconstructions of Eq. 9 are linear in their
// coefficients, so collapsing the summed pyramid once equals summing the K
// per-exposure collapses (Eq. 10); quantisation is applied per exposure
// before the sum.
//
// Filters (per axis, reflect-101 borders on the grid the filter runs on):
//   reduce : out[i] = sum_{m=-2..2} w[m] x[2i + m],  w = [1 4 6 4 1] / 16
//   expand : out[2i] = (g[i-1] + 6 g[i] + g[i+1]) / 8, out[2i+1] = (g[i] + g[i+1]) / 2
//            with g[-1] = g[1] and g[n] = g[n-1]
// (the expand forms are zero insertion followed by 2 w on the fine grid).
#include <algorithm>
#include <vector>

#include "common.hpp"

using namespace mnf;

namespace {

constexpr int kMaxK = 16;
constexpr int kMaxLevels = 12;

struct FuseConsts {
    float inv_range;          // 1 / (sat - dark)
    float range;              // sat - dark
    float dark;
    float mu, inv_2s2;        // weight centre and 1 / (2 sigma^2)
    float scale[kMaxK];       // I_tilde_k = (I_k - dark) * scale[k]  (radiometric) or I_bar_k
    int radiometric;
};

__device__ __forceinline__ int reflect101(int i, int n) { return i < 0 ? -i : (i >= n ? 2 * (n - 1) - i : i); }

// Tap m of the binomial kernel [1 4 6 4 1] / 16.
__device__ __forceinline__ float binom5(int m) {
    return m == 2 ? 0.375f : ((m & 1) ? 0.25f : 0.0625f);
}

// Level 0 of every exposure at one pixel: I_tilde_k and the weight W_k
// normalised over the K frames of the pixel.  KM >= K is a compile-time bound
// so that the per-exposure values stay in registers.  Split into the loads of
// the K raw counts (exposure index clamped to K - 1 past the end, so every
// load is issued unconditionally and a caller can issue several pixels'
// loads before the first wait) and the pointwise evaluation.
template <int KM>
__device__ __forceinline__ void level0_load(const uint16_t* __restrict__ px, size_t npix, int K, float* cnt) {
#pragma unroll
    for (int kk = 0; kk < KM; ++kk) cnt[kk] = (float)px[(size_t)min(kk, K - 1) * npix];
}

template <int KM>
__device__ __forceinline__ void level0_eval(const float* cnt, int K, const FuseConsts& c, float* gi, float* gw) {
    float wsum = 0.f;
#pragma unroll
    for (int kk = 0; kk < KM; ++kk) {
        gi[kk] = gw[kk] = 0.f;
        if (kk < K) {
            const float I = cnt[kk];
            const float Ib = fminf(fmaxf((I - c.dark) * c.inv_range, 0.f), 1.f);
            const float d = Ib - c.mu;
            const float w = __expf(-d * d * c.inv_2s2);  // hardware exp2 path: a few ulp, far inside the 1e-6 weight bound
            wsum += w;
            gw[kk] = w;
            gi[kk] = c.radiometric ? (I - c.dark) * c.scale[kk] : Ib;
        }
    }
    const float inv = __builtin_amdgcn_rcpf(fmaxf(wsum, 1e-30f));  // ~1 ulp, far inside the 1e-6 weight bound
#pragma unroll
    for (int kk = 0; kk < KM; ++kk) gw[kk] = gw[kk] * inv;
}

// Offset added to the contrast before its exponent: where every exposure is
// flat the common factor cancels in the normalisation and the Eq. 5 weights
// remain.  With exponents up to kMaxContrastExp the factor stays a normal
// float (1e-24 at the cap).
constexpr float kContrastEps = 1e-6f;
constexpr float kMaxContrastExp = 4.f;

// Dark-subtracted count clamped to [0, sat - dark]: I_bar times (sat - dark).
// For integer counts and dark level the Laplacian of these values is an
// exact integer sum, so the contrast is rounded once, when normalised, and
// not cancelled from rounded I_bar values.
__device__ __forceinline__ float clamped_count(const uint16_t* px, const FuseConsts& c) {
    return fminf(fmaxf((float)*px - c.dark, 0.f), c.range);
}

// Optional contrast weights (contrast exponent > 0; the paper's weight is
// Eq. 5 alone): per level-0 pixel of the chunk (total = nj * H * W), the Eq. 5
// weight of every exposure times (C_k + eps)^e, C_k = |4-neighbour Laplacian
// of I_bar_k| (reflect-101 neighbours, clamped into an axis of length one),
// normalised over the K frames into W0 [nj][K][H][W].
template <int KM>
__global__ void __launch_bounds__(256)
k_fuse_contrast_weights(const uint16_t* __restrict__ raw, int K, int H, int W, size_t total, FuseConsts c,
                        float cexp, float* __restrict__ W0) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;  // the chunk keeps totals below 2^31
    if (i >= (int)total) return;
    const size_t npix = (size_t)H * W;
    const int jj = i / (H * W), pq = i - jj * (H * W);
    const int y = pq / W, x = pq - y * W;
    const int ym = min(reflect101(y - 1, H), H - 1), yp = max(reflect101(y + 1, H), 0);
    const int xm = min(reflect101(x - 1, W), W - 1), xp = max(reflect101(x + 1, W), 0);
    float w[KM];
    float wsum = 0.f;
#pragma unroll
    for (int kk = 0; kk < KM; ++kk) {
        w[kk] = 0.f;
        if (kk < K) {
            const uint16_t* im = raw + ((size_t)jj * K + kk) * npix;
            const float v = clamped_count(im + pq, c);
            const float lap = clamped_count(im + (size_t)ym * W + x, c) + clamped_count(im + (size_t)yp * W + x, c) +
                              clamped_count(im + (size_t)y * W + xm, c) + clamped_count(im + (size_t)y * W + xp, c) -
                              4.f * v;
            const float d = v * c.inv_range - c.mu;
            w[kk] = expf(-d * d * c.inv_2s2) * powf(fabsf(lap) * c.inv_range + kContrastEps, cexp);
            wsum += w[kk];
        }
    }
    const float inv = 1.f / fmaxf(wsum, 1e-30f);
#pragma unroll
    for (int kk = 0; kk < KM; ++kk)
        if (kk < K) W0[((size_t)jj * K + kk) * npix + pq] = w[kk] * inv;
}

// Level 1 of the image and weight pyramids of all K exposures, reduced from
// the recomputed level 0: thread per level-1 pixel of the chunk (total =
// nj * (H/2) * (W/2)); GI1 and GW1 are [K][total].  With CW the level-0
// weights are read from W0 (k_fuse_contrast_weights) instead.
template <int KM, bool CW>
__global__ void __launch_bounds__(256)
k_fuse_level1(const uint16_t* __restrict__ raw, int K, int H, int W, size_t total, FuseConsts c,
              const float* __restrict__ W0, float* __restrict__ GI1, float* __restrict__ GW1) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;  // the chunk keeps totals below 2^31
    if (i >= (int)total) return;
    const int h1 = H >> 1, w1 = W >> 1;
    const size_t npix = (size_t)H * W;
    const int jj = i / (h1 * w1);
    const int r = i - jj * (h1 * w1);
    const int oy = r / w1, ox = r - oy * w1;
    const uint16_t* base = raw + (size_t)jj * K * npix;
    float si[KM], sw[KM];
#pragma unroll
    for (int kk = 0; kk < KM; ++kk) si[kk] = sw[kk] = 0.f;
#pragma unroll 1
    for (int a = 0; a < 5; ++a) {
        const int yy = reflect101(2 * oy + a - 2, H);
        // the counts of the row's five taps are loaded before any is used
        float cnt[5][KM];
#pragma unroll
        for (int b = 0; b < 5; ++b)
            level0_load<KM>(base + (size_t)yy * W + reflect101(2 * ox + b - 2, W), npix, K, cnt[b]);
        float ri[KM], rw[KM];
#pragma unroll
        for (int kk = 0; kk < KM; ++kk) ri[kk] = rw[kk] = 0.f;
#pragma unroll
        for (int b = 0; b < 5; ++b) {
            float gi[KM], gw[KM];
            level0_eval<KM>(cnt[b], K, c, gi, gw);
            if (CW) {
                const float* w0 = W0 + (size_t)jj * K * npix + (size_t)yy * W + reflect101(2 * ox + b - 2, W);
#pragma unroll
                for (int kk = 0; kk < KM; ++kk)
                    if (kk < K) gw[kk] = w0[(size_t)kk * npix];
            }
#pragma unroll
            for (int kk = 0; kk < KM; ++kk) {
                ri[kk] += binom5(b) * gi[kk];
                rw[kk] += binom5(b) * gw[kk];
            }
        }
#pragma unroll
        for (int kk = 0; kk < KM; ++kk) {
            si[kk] += binom5(a) * ri[kk];
            sw[kk] += binom5(a) * rw[kk];
        }
    }
#pragma unroll
    for (int kk = 0; kk < KM; ++kk)
        if (kk < K) {
            GI1[(size_t)kk * total + i] = si[kk];
            GW1[(size_t)kk * total + i] = sw[kk];
        }
}

// Level 1 as above with each level-0 value evaluated once: a block owns a
// kL1TY x kL1TX tile of level-1 pixels of one pattern, evaluates level 0 of
// all K exposures over the tile's (2 kL1TY + 3) x (2 kL1TX + 3) footprint into
// LDS (reflected coordinates, clamped into the image beyond the single
// reflection that only pixels past the edge would need), then reduces from
// LDS with the taps in the untiled kernel's order, so the results are the
// same.  grid (tiles_x * tiles_y * nj), 256 threads; K <= KM.
constexpr int kL1TY = 8, kL1TX = 32;
constexpr int kL1RY = 2 * kL1TY + 3, kL1RX = 2 * kL1TX + 3, kL1R = kL1RY * kL1RX;

template <int KM>
__global__ void __launch_bounds__(kL1TY * kL1TX)
k_fuse_level1_tiled(const uint16_t* __restrict__ raw, int K, int H, int W, size_t total, FuseConsts c,
                    float* __restrict__ GI1, float* __restrict__ GW1) {
    constexpr int THREADS = kL1TY * kL1TX, PER = (kL1R + THREADS - 1) / THREADS;
    __shared__ float LI[KM * kL1R], LW[KM * kL1R];
    const int h1 = H >> 1, w1 = W >> 1;
    const int tiles_x = (w1 + kL1TX - 1) / kL1TX, tiles_y = (h1 + kL1TY - 1) / kL1TY;
    const int b = blockIdx.x;
    const int jj = b / (tiles_x * tiles_y);
    const int tb = b - jj * (tiles_x * tiles_y);
    const int oy0 = (tb / tiles_x) * kL1TY, ox0 = (tb % tiles_x) * kL1TX;
    const int y0 = 2 * oy0 - 2, x0 = 2 * ox0 - 2;
    const size_t npix = (size_t)H * W;
    const uint16_t* base = raw + (size_t)jj * K * npix;
    float cnt[PER][KM];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int p = min((int)threadIdx.x + u * THREADS, kL1R - 1);
        const int ry = p / kL1RX, rx = p - ry * kL1RX;
        const int yy = min(max(reflect101(y0 + ry, H), 0), H - 1);
        const int xx = min(max(reflect101(x0 + rx, W), 0), W - 1);
        level0_load<KM>(base + (size_t)yy * W + xx, npix, K, cnt[u]);
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int p = (int)threadIdx.x + u * THREADS;
        if (p < kL1R) {
            float gi[KM], gw[KM];
            level0_eval<KM>(cnt[u], K, c, gi, gw);
#pragma unroll
            for (int kk = 0; kk < KM; ++kk)
                if (kk < K) {
                    LI[kk * kL1R + p] = gi[kk];
                    LW[kk * kL1R + p] = gw[kk];
                }
        }
    }
    __syncthreads();
    // separable reduce: every footprint row filtered along x at the tile's
    // output columns (the same taps and order as the untiled kernel: row sums
    // first, then the column sum).  The row sums are formed in registers and,
    // after a barrier, written over the level-0 tile, so the block's LDS stays
    // that of the tile.
    constexpr int NH = kL1RY * kL1TX, HPER = (NH + THREADS - 1) / THREADS;
    float hi[HPER][KM], hw[HPER][KM];
#pragma unroll
    for (int u = 0; u < HPER; ++u) {
        const int e = min((int)threadIdx.x + u * THREADS, NH - 1);
        const int ry = e / kL1TX, tx = e - ry * kL1TX;
        const int p = ry * kL1RX + 2 * tx;
#pragma unroll
        for (int kk = 0; kk < KM; ++kk) {
            float ri = 0.f, rw = 0.f;
            if (kk < K) {
#pragma unroll
                for (int bb = 0; bb < 5; ++bb) {
                    ri += binom5(bb) * LI[kk * kL1R + p + bb];
                    rw += binom5(bb) * LW[kk * kL1R + p + bb];
                }
            }
            hi[u][kk] = ri;
            hw[u][kk] = rw;
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < HPER; ++u) {
        const int e = (int)threadIdx.x + u * THREADS;
        if (e < NH) {
#pragma unroll
            for (int kk = 0; kk < KM; ++kk)
                if (kk < K) {
                    LI[kk * NH + e] = hi[u][kk];
                    LW[kk * NH + e] = hw[u][kk];
                }
        }
    }
    __syncthreads();
    const int ty = threadIdx.x / kL1TX, tx = threadIdx.x % kL1TX;
    const int oy = oy0 + ty, ox = ox0 + tx;
    if (oy >= h1 || ox >= w1) return;
    float si[KM], sw[KM];
#pragma unroll
    for (int kk = 0; kk < KM; ++kk) si[kk] = sw[kk] = 0.f;
#pragma unroll
    for (int a = 0; a < 5; ++a) {
        const int e = (2 * ty + a) * kL1TX + tx;
#pragma unroll
        for (int kk = 0; kk < KM; ++kk)
            if (kk < K) {
                si[kk] += binom5(a) * LI[kk * NH + e];
                sw[kk] += binom5(a) * LW[kk * NH + e];
            }
    }
    const size_t i = (size_t)jj * h1 * w1 + (size_t)oy * w1 + ox;
#pragma unroll
    for (int kk = 0; kk < KM; ++kk)
        if (kk < K) {
            GI1[(size_t)kk * total + i] = si[kk];
            GW1[(size_t)kk * total + i] = sw[kk];
        }
}

// G_{l+1} = D(G_l * w_G) for the image and the weight pyramids together, for
// every exposure at once: blockIdx.y is the exposure, whose level-l arrays
// start at k * in_stride and level-(l+1) arrays at k * out_stride.  A block
// owns a kL1TY x kL1TX tile of level-(l+1) pixels of one pattern, stages the
// tile's footprint of both level-l arrays in LDS (reflected coordinates,
// clamped into the level beyond the single reflection that only pixels past
// the edge would need) and reduces from LDS with the taps in row-then-column
// order, so each level-l value is read from memory once.
// grid (tiles_x * tiles_y * nj, K), kL1TY * kL1TX threads.
__global__ void __launch_bounds__(kL1TY * kL1TX)
k_fuse_reduce(const float* __restrict__ GI, const float* __restrict__ GW, size_t in_stride, int h, int w,
              float* __restrict__ GI1, float* __restrict__ GW1, size_t out_stride) {
    constexpr int THREADS = kL1TY * kL1TX, PER = (kL1R + THREADS - 1) / THREADS;
    __shared__ float LI[kL1R], LW[kL1R];
    const int h2 = h >> 1, w2 = w >> 1;
    const int tiles_x = (w2 + kL1TX - 1) / kL1TX, tiles_y = (h2 + kL1TY - 1) / kL1TY;
    const int b = blockIdx.x;
    const int jj = b / (tiles_x * tiles_y);
    const int tb = b - jj * (tiles_x * tiles_y);
    const int oy0 = (tb / tiles_x) * kL1TY, ox0 = (tb % tiles_x) * kL1TX;
    const int y0 = 2 * oy0 - 2, x0 = 2 * ox0 - 2;
    const float* gi = GI + blockIdx.y * in_stride + (size_t)jj * h * w;
    const float* gw = GW + blockIdx.y * in_stride + (size_t)jj * h * w;
    float vi[PER], vw[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int p = min((int)threadIdx.x + u * THREADS, kL1R - 1);
        const int ry = p / kL1RX, rx = p - ry * kL1RX;
        const int yy = min(max(reflect101(y0 + ry, h), 0), h - 1);
        const int xx = min(max(reflect101(x0 + rx, w), 0), w - 1);
        vi[u] = gi[(size_t)yy * w + xx];
        vw[u] = gw[(size_t)yy * w + xx];
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int p = (int)threadIdx.x + u * THREADS;
        if (p < kL1R) {
            LI[p] = vi[u];
            LW[p] = vw[u];
        }
    }
    __syncthreads();
    const int ty = threadIdx.x / kL1TX, tx = threadIdx.x % kL1TX;
    const int oy = oy0 + ty, ox = ox0 + tx;
    if (oy >= h2 || ox >= w2) return;
    const float wt[5] = {0.0625f, 0.25f, 0.375f, 0.25f, 0.0625f};
    float si = 0.f, sw = 0.f;
#pragma unroll
    for (int a = 0; a < 5; ++a) {
        float ri = 0.f, rw = 0.f;
#pragma unroll
        for (int bb = 0; bb < 5; ++bb) {
            const int p = (2 * ty + a) * kL1RX + 2 * tx + bb;
            ri += wt[bb] * LI[p];
            rw += wt[bb] * LW[p];
        }
        si += wt[a] * ri;
        sw += wt[a] * rw;
    }
    const size_t o = blockIdx.y * out_stride + (size_t)jj * h2 * w2 + (size_t)oy * w2 + ox;
    GI1[o] = si;
    GW1[o] = sw;
}

// Expand of a coarse image g (hc x wc) evaluated at fine pixel (y, x),
// without branches: always three coarse rows and columns, the third with
// weight 0 at odd positions (adding 0 * g leaves the sum unchanged), so that
// neighbouring lanes of alternating parity run the same instructions.
//   even: taps (c-1, c, c+1) weights (1/8, 3/4, 1/8), c-1 -> 1 at the border
//   odd : taps (c, c+1, -)   weights (1/2, 1/2, 0),   c+1 -> hc-1 at the border
// The taps depend only on the grid and the pixel, so several coarse images
// sampled at one pixel share them; loads and the weighted sum are separate
// so that a caller can issue all the loads first.
struct ExpandTaps {
    int iy[3], ix[3];
    float wy[3], wx[3];
};

__device__ __forceinline__ ExpandTaps expand_taps(int hc, int wc, int y, int x) {
    const int cy = y >> 1, cx = x >> 1;
    const bool ey = (y & 1) == 0, ex = (x & 1) == 0;
    const int up = cy + 1 >= hc ? hc - 1 : cy + 1, rt = cx + 1 >= wc ? wc - 1 : cx + 1;
    ExpandTaps e;
    e.iy[0] = ey ? (cy - 1 < 0 ? 1 : cy - 1) : cy;
    e.iy[1] = ey ? cy : up;
    e.iy[2] = up;
    e.ix[0] = ex ? (cx - 1 < 0 ? 1 : cx - 1) : cx;
    e.ix[1] = ex ? cx : rt;
    e.ix[2] = rt;
    e.wy[0] = ey ? 0.125f : 0.5f;
    e.wy[1] = ey ? 0.75f : 0.5f;
    e.wy[2] = ey ? 0.125f : 0.f;
    e.wx[0] = ex ? 0.125f : 0.5f;
    e.wx[1] = ex ? 0.75f : 0.5f;
    e.wx[2] = ex ? 0.125f : 0.f;
    return e;
}

__device__ __forceinline__ void expand_load(const float* __restrict__ g, int wc, const ExpandTaps& e, float* v) {
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int q = 0; q < 3; ++q) v[3 * r + q] = g[(size_t)e.iy[r] * wc + e.ix[q]];
}

__device__ __forceinline__ float expand_sum(const ExpandTaps& e, const float* v) {
    float s = 0.f;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        float t = 0.f;
        t += e.wx[0] * v[3 * r];
        t += e.wx[1] * v[3 * r + 1];
        t += e.wx[2] * v[3 * r + 2];
        s += e.wy[r] * t;
    }
    return s;
}

__device__ __forceinline__ float expand_at(const float* __restrict__ g, int hc, int wc, int y, int x) {
    const ExpandTaps e = expand_taps(hc, wc, y, x);
    float v[9];
    expand_load(g, wc, e, v);
    return expand_sum(e, v);
}

// Band level l < L: F_l = sum_k Q_k(G_l[W_k] (G_l[I_k] - U(G_{l+1}[I_k])));
// base l = L: F_L = sum_k G_L[W_k] G_L[I_k].  Every exposure in one thread,
// summed in exposure order; exposure k's level-l arrays start at k * stride,
// its level-(l+1) image at k * stride_c.  The loads of four exposures are
// issued before their terms are formed.  With Rc (the collapsed level l + 1,
// [nj][h/2][w/2]) the output is the collapse step R_l = F_l + U(R_{l+1})
// (Eq. 9), so the levels run from the base to level 1 with no separate
// collapse launches.
struct BandSteps {
    float step[kMaxK];  // quantisation step of each exposure at this level (0 = none)
};

__global__ void __launch_bounds__(256)
k_fuse_band(const float* __restrict__ GI, const float* __restrict__ GW, size_t stride,
            const float* __restrict__ GIc, size_t stride_c, int K, int h, int w, size_t total, BandSteps q,
            int base, const float* __restrict__ Rc, float* __restrict__ F) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    constexpr int G = 4;
    float acc = 0.f;
    if (base) {
        for (int k0 = 0; k0 < K; k0 += G) {
            float vi[G], vw[G];
#pragma unroll
            for (int u = 0; u < G; ++u) {
                const size_t o = (size_t)min(k0 + u, K - 1) * stride + i;
                vi[u] = GI[o];
                vw[u] = GW[o];
            }
#pragma unroll
            for (int u = 0; u < G; ++u)
                if (k0 + u < K) {
                    const float v = vw[u] * vi[u];
                    acc = k0 + u == 0 ? v : acc + v;
                }
        }
    } else {
        const size_t jj = i / ((size_t)h * w);
        const int r = (int)(i % ((size_t)h * w));
        const int y = r / w, x = r % w;
        const int hc = h >> 1, wc = w >> 1;
        const ExpandTaps e = expand_taps(hc, wc, y, x);
        for (int k0 = 0; k0 < K; k0 += G) {
            float vi[G], vw[G], ev[G][9];
#pragma unroll
            for (int u = 0; u < G; ++u) {
                const int k = min(k0 + u, K - 1);
                vi[u] = GI[(size_t)k * stride + i];
                vw[u] = GW[(size_t)k * stride + i];
                expand_load(GIc + (size_t)k * stride_c + jj * (size_t)hc * wc, wc, e, ev[u]);
            }
#pragma unroll
            for (int u = 0; u < G; ++u)
                if (k0 + u < K) {
                    const float lap = vi[u] - expand_sum(e, ev[u]);
                    float v = vw[u] * lap;
                    const float st = q.step[k0 + u];
                    if (st > 0.f) v = st * rintf(v / st);
                    acc = k0 + u == 0 ? v : acc + v;
                }
        }
        if (Rc) acc = acc + expand_at(Rc + jj * (size_t)hc * wc, hc, wc, y, x);
    }
    F[i] = acc;
}

// Band level l < L as k_fuse_band, one thread per level-(l+1) pixel, i.e. per
// 2 x 2 quad of level-l pixels (totalc = nj * (h/2) * (w/2)): the quad's
// expand taps share the 3 x 3 neighbourhood of each exposure's level-(l+1)
// image (separable expand as in k_fuse_final_quad); the quad's level-l
// values are two 64-bit loads per array.  K == KM exposures, summed in order.
// With Rc the collapsed level l + 1 is expanded the same way and added
// (R_l = F_l + U(R_{l+1})).
struct BandQuant {
    float step[kMaxK];  // quantisation step of each exposure at this level (0 = none)
    float inv[kMaxK];   // 1 / step
};

template <int KM>
__global__ void __launch_bounds__(256)
k_fuse_band_quad(const float* __restrict__ GI, const float* __restrict__ GW, size_t stride,
                 const float* __restrict__ GIc, size_t stride_c, int h, int w, size_t totalc, BandQuant q,
                 const float* __restrict__ Rc, float* __restrict__ F) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= totalc) return;
    const int hc = h >> 1, wc = w >> 1;
    const size_t jj = i / ((size_t)hc * wc);
    const int r = (int)(i - jj * (size_t)hc * wc);
    const int cy = r / wc, cx = r - cy * wc;
    const int ry[3] = {cy > 0 ? cy - 1 : 1, cy, cy + 1 < hc ? cy + 1 : hc - 1};
    const int rx[3] = {cx > 0 ? cx - 1 : 1, cx, cx + 1 < wc ? cx + 1 : wc - 1};
    const size_t fo = jj * (size_t)h * w + (size_t)(2 * cy) * w + 2 * cx;
    const size_t co = jj * (size_t)hc * wc;
    float g[KM][9];
    float2 vi[KM][2], vw[KM][2];
    float rc[9];
    if (Rc) {
        const float* rp = Rc + co;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) rc[3 * a + b] = rp[(size_t)ry[a] * wc + rx[b]];
    }
#pragma unroll
    for (int k = 0; k < KM; ++k) {
        const float* gc = GIc + (size_t)k * stride_c + co;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) g[k][3 * a + b] = gc[(size_t)ry[a] * wc + rx[b]];
        const float* gi = GI + (size_t)k * stride + fo;
        const float* gw = GW + (size_t)k * stride + fo;
        vi[k][0] = *(const float2*)gi;
        vi[k][1] = *(const float2*)(gi + w);
        vw[k][0] = *(const float2*)gw;
        vw[k][1] = *(const float2*)(gw + w);
    }
    float acc[4];
#pragma unroll
    for (int k = 0; k < KM; ++k) {
        float he[3], ho[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            he[a] = fmaf(0.125f, g[k][3 * a], fmaf(0.75f, g[k][3 * a + 1], 0.125f * g[k][3 * a + 2]));
            ho[a] = fmaf(0.5f, g[k][3 * a + 1], 0.5f * g[k][3 * a + 2]);
        }
        const float up[4] = {fmaf(0.125f, he[0], fmaf(0.75f, he[1], 0.125f * he[2])),
                             fmaf(0.125f, ho[0], fmaf(0.75f, ho[1], 0.125f * ho[2])),
                             fmaf(0.5f, he[1], 0.5f * he[2]), fmaf(0.5f, ho[1], 0.5f * ho[2])};
        const float fi[4] = {vi[k][0].x, vi[k][0].y, vi[k][1].x, vi[k][1].y};
        const float fw[4] = {vw[k][0].x, vw[k][0].y, vw[k][1].x, vw[k][1].y};
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            float v = fw[d] * (fi[d] - up[d]);
            if (q.step[k] > 0.f) v = q.step[k] * rintf(v * q.inv[k]);
            acc[d] = k == 0 ? v : acc[d] + v;
        }
    }
    if (Rc) {
        float he[3], ho[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            he[a] = fmaf(0.125f, rc[3 * a], fmaf(0.75f, rc[3 * a + 1], 0.125f * rc[3 * a + 2]));
            ho[a] = fmaf(0.5f, rc[3 * a + 1], 0.5f * rc[3 * a + 2]);
        }
        acc[0] += fmaf(0.125f, he[0], fmaf(0.75f, he[1], 0.125f * he[2]));
        acc[1] += fmaf(0.125f, ho[0], fmaf(0.75f, ho[1], 0.125f * ho[2]));
        acc[2] += fmaf(0.5f, he[1], 0.5f * he[2]);
        acc[3] += fmaf(0.5f, ho[1], 0.5f * ho[2]);
    }
    *(float2*)(F + fo) = make_float2(acc[0], acc[1]);
    *(float2*)(F + fo + w) = make_float2(acc[2], acc[3]);
}

struct Level0Steps {
    float step[kMaxK];  // level-0 quantisation step of each exposure (0 = none)
};

// Level 0 and the output: per pixel of the chunk (total = nj * H * W), the
// level-0 coefficient of every exposure, G_0[W_k] (G_0[I_k] - U(G_1[I_k])),
// quantised with its own step and summed over k, plus U(R_1) (the fused
// pyramid collapsed to level 1).  With L = 0 the output is the weighted sum
// of the level-0 images.  Optionally writes the normalised weights.  With CW
// the level-0 weights are read from W0 (k_fuse_contrast_weights) instead.
template <int KM, bool CW>
__global__ void __launch_bounds__(256)
k_fuse_final(const uint16_t* __restrict__ raw, int K, int H, int W, size_t total, FuseConsts c, Level0Steps q,
             const float* __restrict__ W0, const float* __restrict__ GI1, const float* __restrict__ R1, int L,
             float* __restrict__ out, float* __restrict__ weights_out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;  // the chunk keeps totals below 2^31
    if (i >= (int)total) return;
    const size_t npix = (size_t)H * W;
    const int jj = i / (H * W), pq = i - jj * (H * W);
    const int y = pq / W, x = pq - y * W;
    float cnt[KM];
    level0_load<KM>(raw + (size_t)jj * K * npix + pq, npix, K, cnt);
    // with K <= 8 the expand taps of every exposure's level 1 and of the
    // collapsed level 1 are loaded together with the counts
    const int h1 = H >> 1, w1 = W >> 1;
    const size_t n1 = (total / npix) * (size_t)h1 * w1;  // level-1 pixels of the chunk
    constexpr bool BATCH = KM <= 8;
    ExpandTaps e{};
    float ev[BATCH ? KM : 1][9], rv[9];
    if (BATCH && L > 0) {
        e = expand_taps(h1, w1, y, x);
#pragma unroll
        for (int kk = 0; kk < (BATCH ? KM : 1); ++kk)
            expand_load(GI1 + (size_t)min(kk, K - 1) * n1 + (size_t)jj * h1 * w1, w1, e, ev[kk]);
        expand_load(R1 + (size_t)jj * h1 * w1, w1, e, rv);
    }
    float gi[KM], gw[KM];
    level0_eval<KM>(cnt, K, c, gi, gw);
    if (CW) {
#pragma unroll
        for (int kk = 0; kk < KM; ++kk)
            if (kk < K) gw[kk] = W0[((size_t)jj * K + kk) * npix + pq];
    }
    if (weights_out) {
#pragma unroll
        for (int kk = 0; kk < KM; ++kk)
            if (kk < K) weights_out[((size_t)jj * K + kk) * npix + pq] = gw[kk];
    }
    float F = 0.f;
    if (L == 0) {
#pragma unroll
        for (int kk = 0; kk < KM; ++kk)
            if (kk < K) {
                const float v = gw[kk] * gi[kk];
                F = kk == 0 ? v : F + v;
            }
        out[i] = F;
        return;
    }
#pragma unroll
    for (int kk = 0; kk < KM; ++kk)
        if (kk < K) {
            const float up = BATCH ? expand_sum(e, ev[BATCH ? kk : 0])
                                   : expand_at(GI1 + (size_t)kk * n1 + (size_t)jj * h1 * w1, h1, w1, y, x);
            const float lap = gi[kk] - up;
            float v = gw[kk] * lap;
            const float st = q.step[kk];
            if (st > 0.f) v = st * rintf(v / st);
            F = kk == 0 ? v : F + v;
        }
    out[i] = F + (BATCH ? expand_sum(e, rv) : expand_at(R1 + (size_t)jj * h1 * w1, h1, w1, y, x));
}

// Level 0 and the output as k_fuse_final (L >= 1), one thread per 2 x 2 quad of
// level-0 pixels, i.e. per level-1 pixel (total1 = nj * (H/2) * (W/2)): the
// expand taps of the quad's four pixels all lie in the 3 x 3 level-1
// neighbourhood rows {c-1, c, c+1} x columns {c-1, c, c+1} of its level-1
// pixel (reflected as in expand_taps), so every exposure's level-1 image and
// R_1 are loaded once per quad, expanded separably (per row the even-column
// value (1 6 1)/8 and the odd-column value (1 1)/2, then the same weights
// down the rows), and the two raw counts of a quad row are one 32-bit load.
// K == KM exposures; quantisation multiplies by the step's reciprocal.
struct Level0Quant {
    float step[kMaxK];  // level-0 quantisation step of each exposure (0 = none)
    float inv[kMaxK];   // 1 / step
};

template <int KM>
__global__ void __launch_bounds__(256)
k_fuse_final_quad(const uint16_t* __restrict__ raw, int H, int W, size_t total1, FuseConsts c, Level0Quant q,
                  const float* __restrict__ GI1, const float* __restrict__ R1, float* __restrict__ out,
                  float* __restrict__ weights_out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;  // the chunk keeps totals below 2^31
    if (i >= (int)total1) return;
    const int h1 = H >> 1, w1 = W >> 1;
    const int jj = i / (h1 * w1), r = i - jj * (h1 * w1);
    const int cy = r / w1, cx = r - cy * w1;
    const size_t npix = (size_t)H * W;
    const size_t n1 = total1;  // level-1 pixels of the chunk (exposure stride of GI1)
    // the quad's raw counts: two adjacent 16-bit counts per row and exposure
    const uint16_t* base = raw + (size_t)jj * KM * npix + (size_t)(2 * cy) * W + 2 * cx;
    uint32_t q0[KM], q1[KM];
#pragma unroll
    for (int k = 0; k < KM; ++k) {
        q0[k] = *(const uint32_t*)(base + (size_t)k * npix);
        q1[k] = *(const uint32_t*)(base + (size_t)k * npix + W);
    }
    // 3 x 3 level-1 neighbourhood (g[-1] = g[1], g[n] = g[n-1])
    const int ry[3] = {cy > 0 ? cy - 1 : 1, cy, cy + 1 < h1 ? cy + 1 : h1 - 1};
    const int rx[3] = {cx > 0 ? cx - 1 : 1, cx, cx + 1 < w1 ? cx + 1 : w1 - 1};
    const size_t off1 = (size_t)jj * h1 * w1;
    float g[KM + 1][9];
#pragma unroll
    for (int k = 0; k <= KM; ++k) {
        const float* src = k < KM ? GI1 + (size_t)k * n1 + off1 : R1 + off1;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) g[k][3 * a + b] = src[(size_t)ry[a] * w1 + rx[b]];
    }
    // separable expand of each coarse image at the quad's four pixels: up[k][2 dy + dx]
    float up[KM + 1][4];
#pragma unroll
    for (int k = 0; k <= KM; ++k) {
        float he[3], ho[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            he[a] = fmaf(0.125f, g[k][3 * a], fmaf(0.75f, g[k][3 * a + 1], 0.125f * g[k][3 * a + 2]));
            ho[a] = fmaf(0.5f, g[k][3 * a + 1], 0.5f * g[k][3 * a + 2]);
        }
        up[k][0] = fmaf(0.125f, he[0], fmaf(0.75f, he[1], 0.125f * he[2]));
        up[k][1] = fmaf(0.125f, ho[0], fmaf(0.75f, ho[1], 0.125f * ho[2]));
        up[k][2] = fmaf(0.5f, he[1], 0.5f * he[2]);
        up[k][3] = fmaf(0.5f, ho[1], 0.5f * ho[2]);
    }
    float res[4];
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        const int dy = d >> 1, dx = d & 1;
        float cnt[KM];
#pragma unroll
        for (int k = 0; k < KM; ++k) cnt[k] = (float)(((dy ? q1[k] : q0[k]) >> (16 * dx)) & 0xffffu);
        float gi[KM], gw[KM];
        level0_eval<KM>(cnt, KM, c, gi, gw);
        if (weights_out) {
            const size_t pq = (size_t)(2 * cy + dy) * W + 2 * cx + dx;
#pragma unroll
            for (int k = 0; k < KM; ++k) weights_out[((size_t)jj * KM + k) * npix + pq] = gw[k];
        }
        float F = 0.f;
#pragma unroll
        for (int k = 0; k < KM; ++k) {
            float v = gw[k] * (gi[k] - up[k][d]);
            if (q.step[k] > 0.f) v = q.step[k] * rintf(v * q.inv[k]);
            F = k == 0 ? v : F + v;
        }
        res[d] = F + up[KM][d];
    }
    float* o = out + (size_t)jj * npix + (size_t)(2 * cy) * W + 2 * cx;
    *(float2*)o = make_float2(res[0], res[1]);
    *(float2*)(o + W) = make_float2(res[2], res[3]);
}

inline dim3 grid1d(size_t n) { return dim3((unsigned)((n + 255) / 256)); }

// Launch helpers dispatching on the exposure count so that the per-exposure
// loops of the level-0 kernels are exactly K long.
template <int KM>
int launch_level1(mnf_ctx* ctx, hipStream_t st, const uint16_t* rawc, int K, int H, int W, size_t n1, int nj,
                  const FuseConsts& c, float* GI1, float* GW1) {
    const size_t tiles = (size_t)((W / 2 + kL1TX - 1) / kL1TX) * ((H / 2 + kL1TY - 1) / kL1TY) * nj;
    MNF_LAUNCH(ctx, MNF_K_FUSE, st, k_fuse_level1_tiled<KM>, dim3((unsigned)tiles), dim3(kL1TY * kL1TX), rawc, K, H,
               W, n1, c, GI1, GW1);
    return MNF_OK;
}

template <int KM>
int launch_band_quad(mnf_ctx* ctx, hipStream_t st, const float* GI, const float* GW, size_t stride, const float* GIc,
                     size_t stride_c, int h, int w, size_t totalc, const BandQuant& q, const float* Rc, float* F) {
    MNF_LAUNCH(ctx, MNF_K_FUSE, st, k_fuse_band_quad<KM>, grid1d(totalc), dim3(256), GI, GW, stride, GIc, stride_c, h,
               w, totalc, q, Rc, F);
    return MNF_OK;
}

template <int KM>
int launch_final_quad(mnf_ctx* ctx, hipStream_t st, const uint16_t* rawc, int H, int W, size_t n1,
                      const FuseConsts& c, const Level0Quant& q, const float* GI1, const float* R1, float* outc,
                      float* wout) {
    MNF_LAUNCH(ctx, MNF_K_FUSE, st, k_fuse_final_quad<KM>, grid1d(n1), dim3(256), rawc, H, W, n1, c, q, GI1, R1, outc,
               wout);
    return MNF_OK;
}

}  // namespace

// Linear baselines: per pixel, the rate sum_k m_k (I_k - dark) / sum_k m_k t_k
// over the frames below saturation (m_k = [I_k < sat]) times t_1 (mode 0),
// the shortest frame's value where every frame is saturated; or the shortest
// frame alone (mode 1).
__global__ void __launch_bounds__(256)
k_fuse_linear(const uint16_t* __restrict__ raw, int K, size_t npix, size_t total, const float* __restrict__ t,
              float sat, float dark, int mode, float* __restrict__ out) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const size_t jj = i / npix, q = i % npix;
    const uint16_t* px = raw + jj * (size_t)K * npix + q;
    const float first = (float)px[0] - dark;
    if (mode == 1) {
        out[i] = first;
        return;
    }
    float num = 0.f, den = 0.f;
    for (int k = 0; k < K; ++k) {
        const float I = (float)px[(size_t)k * npix];
        if (I < sat) {
            num += I - dark;
            den += t[k];
        }
    }
    out[i] = den > 0.f ? num / den * t[0] : first;
}

extern "C" int fuse_exposures(mnf_ctx* ctx, const uint16_t* raw, const float* t, int J, int K, int H, int W,
                              const mnf_fuse_params* p, float* fused, float* weights_out, void* stream) {
    MNF_TRY(begin(ctx));
    if (!raw || !t || !p || !fused) return set_error(ctx, MNF_EINVAL, "null pointer argument");
    if (J <= 0 || K <= 0 || H <= 0 || W <= 0)
        return set_error(ctx, MNF_EINVAL, "sizes must be positive (J=%d K=%d H=%d W=%d)", J, K, H, W);
    if (K > kMaxK) return set_error(ctx, MNF_EUNSUPPORTED, "at most %d exposures (K=%d)", kMaxK, K);
    const int L = p->levels;
    if (L < 0 || L > kMaxLevels) return set_error(ctx, MNF_EUNSUPPORTED, "levels %d outside [0, %d]", L, kMaxLevels);
    if (L > 0 && ((H % (1 << L)) || (W % (1 << L)) || (H >> L) < 2 || (W >> L) < 2))
        return set_error(ctx, MNF_EINVAL, "H=%d and W=%d must be multiples of 2^L with coarsest level >= 2 (L=%d)",
                         H, W, L);
    if (!(p->sat > p->dark)) return set_error(ctx, MNF_EINVAL, "sat must exceed dark");
    if (!(p->sigma > 0.f)) return set_error(ctx, MNF_EINVAL, "sigma must be positive");
    for (int k = 0; k < K; ++k)
        if (!(t[k] > 0.f)) return set_error(ctx, MNF_EINVAL, "exposure time %d must be positive", k);
    for (int l = 0; l < 16; ++l)
        if (!(p->delta[l] >= 0.f)) return set_error(ctx, MNF_EINVAL, "delta[%d] must be >= 0", l);
    if (!(p->contrast_exp >= 0.f && p->contrast_exp <= kMaxContrastExp))
        return set_error(ctx, MNF_EINVAL, "contrast_exp %g outside [0, %g]", (double)p->contrast_exp,
                         (double)kMaxContrastExp);
    const bool cw = p->contrast_exp > 0.f;

    hipStream_t st = (hipStream_t)stream;
    FuseConsts c{};
    c.inv_range = (float)(1.0 / ((double)p->sat - (double)p->dark));
    c.range = (float)((double)p->sat - (double)p->dark);
    c.dark = p->dark;
    c.mu = p->mu;
    c.inv_2s2 = (float)(1.0 / (2.0 * (double)p->sigma * (double)p->sigma));
    for (int k = 0; k < K; ++k) c.scale[k] = (float)((double)t[0] / (double)t[k]);
    c.radiometric = p->radiometric ? 1 : 0;

    // quantisation step of exposure k at level l in I_tilde units
    std::vector<float> step((size_t)(L + 1) * K, 0.f);
    for (int l = 0; l < L; ++l)
        for (int k = 0; k < K; ++k) {
            const double d = p->delta[l];
            step[(size_t)l * K + k] =
                d <= 0.0 ? 0.f
                         : (float)(p->radiometric ? d * (double)t[0] / (double)t[k]
                                                  : d / ((double)p->sat - (double)p->dark));
        }

    const size_t npix_all = (size_t)H * W;
    if (npix_all > (size_t)(INT32_MAX / 2)) return set_error(ctx, MNF_EUNSUPPORTED, "pattern of %d x %d too large", H, W);
    // per-position scratch (floats): levels 1..L of all K image and weight
    // pyramids (level 1 in GI1 / GW1, levels 2..L in SI / SW), fused levels 1..L
    std::vector<size_t> offF(L + 2, 0), offS(L + 2, 0);
    for (int l = 1; l <= L; ++l) offF[l + 1] = offF[l] + (size_t)(H >> l) * (W >> l);
    for (int l = 2; l <= L; ++l) offS[l + 1] = offS[l] + (size_t)(H >> l) * (W >> l);
    const size_t n1pos = L >= 1 ? (size_t)(H >> 1) * (W >> 1) : 0;
    // (plus the level-0 weights of all K exposures with the contrast factor)
    const size_t per_pos =
        2 * (size_t)K * n1pos + 2 * (size_t)K * offS[L + 1] + offF[L + 1] + (cw ? (size_t)K * H * W : 0);
    const size_t budget = (size_t)1 << 30;
    size_t chunk_cap = per_pos == 0 ? (size_t)J : budget / (per_pos * sizeof(float));
    chunk_cap = std::min(chunk_cap, (size_t)(INT32_MAX / 2) / npix_all);  // 32-bit pixel indices in a chunk
    const int chunk = (int)std::max<size_t>(1, std::min<size_t>((size_t)J, chunk_cap));
    float *GI1 = nullptr, *GW1 = nullptr, *SI = nullptr, *SW = nullptr, *F = nullptr;
    if (L >= 1) {
        void *a1, *a2, *a3, *a4, *a5;
        MNF_TRY(scratch(ctx, "fuseGI1", (size_t)chunk * K * n1pos * sizeof(float), &a1));
        MNF_TRY(scratch(ctx, "fuseGW1", (size_t)chunk * K * n1pos * sizeof(float), &a2));
        MNF_TRY(scratch(ctx, "fuseSI", std::max<size_t>(1, (size_t)chunk * K * offS[L + 1]) * sizeof(float), &a3));
        MNF_TRY(scratch(ctx, "fuseSW", std::max<size_t>(1, (size_t)chunk * K * offS[L + 1]) * sizeof(float), &a4));
        MNF_TRY(scratch(ctx, "fuseF", (size_t)chunk * offF[L + 1] * sizeof(float), &a5));
        GI1 = (float*)a1;
        GW1 = (float*)a2;
        SI = (float*)a3;
        SW = (float*)a4;
        F = (float*)a5;
    }
    float* W0 = nullptr;
    if (cw) {
        void* a;
        MNF_TRY(scratch(ctx, "fuseW0", (size_t)chunk * K * H * W * sizeof(float), &a));
        W0 = (float*)a;
    }
    Level0Steps q0{};
    for (int k = 0; k < K; ++k) q0.step[k] = L >= 1 ? step[k] : 0.f;
    const size_t npix = (size_t)H * W;
    const bool small_k = K <= 8;

    for (int j0 = 0; j0 < J; j0 += chunk) {
        const int nj = std::min(chunk, J - j0);
        const uint16_t* rawc = raw + (size_t)j0 * K * npix;
        const size_t n1 = (size_t)nj * n1pos;
        if (cw) {
            const size_t n0 = (size_t)nj * npix;
            if (small_k)
                MNF_LAUNCH(ctx, MNF_K_FUSE, st, k_fuse_contrast_weights<8>, grid1d(n0), dim3(256), rawc, K, H, W, n0,
                           c, p->contrast_exp, W0);
            else
                MNF_LAUNCH(ctx, MNF_K_FUSE, st, k_fuse_contrast_weights<kMaxK>, grid1d(n0), dim3(256), rawc, K, H, W,
                           n0, c, p->contrast_exp, W0);
        }
        if (L >= 1 && !cw && K <= 5) {
            switch (K) {
                case 1: MNF_TRY(launch_level1<1>(ctx, st, rawc, K, H, W, n1, nj, c, GI1, GW1)); break;
                case 2: MNF_TRY(launch_level1<2>(ctx, st, rawc, K, H, W, n1, nj, c, GI1, GW1)); break;
                case 3: MNF_TRY(launch_level1<3>(ctx, st, rawc, K, H, W, n1, nj, c, GI1, GW1)); break;
                case 4: MNF_TRY(launch_level1<4>(ctx, st, rawc, K, H, W, n1, nj, c, GI1, GW1)); break;
                case 5: MNF_TRY(launch_level1<5>(ctx, st, rawc, K, H, W, n1, nj, c, GI1, GW1)); break;
                default: break;
            }
        } else if (L >= 1) {
            // the generic level-1 kernel: more than five exposures, or level-0
            // weights from the contrast pass
            if (small_k && cw)
                MNF_LAUNCH(ctx, MNF_K_FUSE, st, (k_fuse_level1<8, true>), grid1d(n1), dim3(256), rawc, K, H, W, n1, c,
                           (const float*)W0, GI1, GW1);
            else if (small_k)
                MNF_LAUNCH(ctx, MNF_K_FUSE, st, (k_fuse_level1<8, false>), grid1d(n1), dim3(256), rawc, K, H, W, n1, c,
                           (const float*)nullptr, GI1, GW1);
            else if (cw)
                MNF_LAUNCH(ctx, MNF_K_FUSE, st, (k_fuse_level1<kMaxK, true>), grid1d(n1), dim3(256), rawc, K, H, W, n1,
                           c, (const float*)W0, GI1, GW1);
            else
                MNF_LAUNCH(ctx, MNF_K_FUSE, st, (k_fuse_level1<kMaxK, false>), grid1d(n1), dim3(256), rawc, K, H, W, n1,
                           c, (const float*)nullptr, GI1, GW1);
        }
        if (L >= 1) {
            // level-l arrays (l >= 1) of exposure k and of the fused pyramid;
            // exposure k's arrays of level l sit at k * sstride(l) from exposure 0's
            const size_t sS = (size_t)nj * offS[L + 1];
            auto lvlI = [&](int l) { return l == 1 ? GI1 : SI + (size_t)nj * offS[l]; };
            auto lvlW = [&](int l) { return l == 1 ? GW1 : SW + (size_t)nj * offS[l]; };
            auto sstride = [&](int l) { return l == 1 ? n1 : sS; };
            auto lvlF = [&](int l) { return F + (size_t)nj * offF[l]; };
            for (int l = 1; l < L; ++l) {
                const int h = H >> l, w = W >> l;
                const size_t tiles = (size_t)((w / 2 + kL1TX - 1) / kL1TX) * ((h / 2 + kL1TY - 1) / kL1TY) * nj;
                MNF_LAUNCH(ctx, MNF_K_FUSE, st, k_fuse_reduce, dim3((unsigned)tiles, K), dim3(kL1TY * kL1TX), lvlI(l),
                           lvlW(l), sstride(l), h, w, lvlI(l + 1), lvlW(l + 1), sS);
            }
            // bands from the base to level 1, each collapsing onto the level
            // below it: lvlF(l) receives R_l = F_l + U(R_{l+1}) (R_L = F_L)
            for (int l = L; l >= 1; --l) {
                const int h = H >> l, w = W >> l;
                const size_t nn = (size_t)nj * h * w;
                const float* Rc = l < L ? (const float*)lvlF(l + 1) : (const float*)nullptr;
                // the quad form reads each level-l array with 64-bit loads: every
                // exposure's array must start 8-byte aligned (even stride)
                if (l < L && small_k && sstride(l) % 2 == 0) {
                    BandQuant bq{};
                    for (int k = 0; k < K; ++k) {
                        bq.step[k] = step[(size_t)l * K + k];
                        bq.inv[k] = bq.step[k] > 0.f ? (float)(1.0 / (double)bq.step[k]) : 0.f;
                    }
                    const size_t nc = nn / 4;
                    const float *gi = lvlI(l), *gw = lvlW(l), *gc = lvlI(l + 1);
                    const size_t ss = sstride(l);
                    switch (K) {
                        case 1: MNF_TRY(launch_band_quad<1>(ctx, st, gi, gw, ss, gc, sS, h, w, nc, bq, Rc, lvlF(l))); break;
                        case 2: MNF_TRY(launch_band_quad<2>(ctx, st, gi, gw, ss, gc, sS, h, w, nc, bq, Rc, lvlF(l))); break;
                        case 3: MNF_TRY(launch_band_quad<3>(ctx, st, gi, gw, ss, gc, sS, h, w, nc, bq, Rc, lvlF(l))); break;
                        case 4: MNF_TRY(launch_band_quad<4>(ctx, st, gi, gw, ss, gc, sS, h, w, nc, bq, Rc, lvlF(l))); break;
                        case 5: MNF_TRY(launch_band_quad<5>(ctx, st, gi, gw, ss, gc, sS, h, w, nc, bq, Rc, lvlF(l))); break;
                        case 6: MNF_TRY(launch_band_quad<6>(ctx, st, gi, gw, ss, gc, sS, h, w, nc, bq, Rc, lvlF(l))); break;
                        case 7: MNF_TRY(launch_band_quad<7>(ctx, st, gi, gw, ss, gc, sS, h, w, nc, bq, Rc, lvlF(l))); break;
                        default: MNF_TRY(launch_band_quad<8>(ctx, st, gi, gw, ss, gc, sS, h, w, nc, bq, Rc, lvlF(l))); break;
                    }
                    continue;
                }
                BandSteps bs{};
                for (int k = 0; k < K; ++k) bs.step[k] = l < L ? step[(size_t)l * K + k] : 0.f;
                MNF_LAUNCH(ctx, MNF_K_FUSE, st, k_fuse_band, grid1d(nn), dim3(256), lvlI(l), lvlW(l), sstride(l),
                           l < L ? lvlI(l + 1) : (const float*)nullptr, sS, K, h, w, nn, bs, l == L ? 1 : 0, Rc,
                           lvlF(l));
            }
        }
        const size_t n0 = (size_t)nj * npix;
        float* outc = fused + (size_t)j0 * npix;
        float* wout = weights_out ? weights_out + (size_t)j0 * K * npix : (float*)nullptr;
        const float* R1 = L >= 1 ? F : (const float*)nullptr;  // fused level 1 sits first in F
        // the quad kernel reads two counts per 32-bit load and writes two outputs
        // per 64-bit store (W is even when L >= 1)
        const bool quad = L >= 1 && small_k && !cw && (uintptr_t)raw % 4 == 0 && (uintptr_t)fused % 8 == 0;
        if (quad) {
            Level0Quant qq{};
            for (int k = 0; k < K; ++k) {
                qq.step[k] = q0.step[k];
                qq.inv[k] = q0.step[k] > 0.f ? (float)(1.0 / (double)q0.step[k]) : 0.f;
            }
            switch (K) {
                case 1: MNF_TRY(launch_final_quad<1>(ctx, st, rawc, H, W, n1, c, qq, GI1, R1, outc, wout)); break;
                case 2: MNF_TRY(launch_final_quad<2>(ctx, st, rawc, H, W, n1, c, qq, GI1, R1, outc, wout)); break;
                case 3: MNF_TRY(launch_final_quad<3>(ctx, st, rawc, H, W, n1, c, qq, GI1, R1, outc, wout)); break;
                case 4: MNF_TRY(launch_final_quad<4>(ctx, st, rawc, H, W, n1, c, qq, GI1, R1, outc, wout)); break;
                case 5: MNF_TRY(launch_final_quad<5>(ctx, st, rawc, H, W, n1, c, qq, GI1, R1, outc, wout)); break;
                case 6: MNF_TRY(launch_final_quad<6>(ctx, st, rawc, H, W, n1, c, qq, GI1, R1, outc, wout)); break;
                case 7: MNF_TRY(launch_final_quad<7>(ctx, st, rawc, H, W, n1, c, qq, GI1, R1, outc, wout)); break;
                default: MNF_TRY(launch_final_quad<8>(ctx, st, rawc, H, W, n1, c, qq, GI1, R1, outc, wout)); break;
            }
        } else if (small_k && cw)
            MNF_LAUNCH(ctx, MNF_K_FUSE, st, (k_fuse_final<8, true>), grid1d(n0), dim3(256), rawc, K, H, W, n0, c, q0,
                       (const float*)W0, (const float*)GI1, R1, L, outc, wout);
        else if (small_k)
            MNF_LAUNCH(ctx, MNF_K_FUSE, st, (k_fuse_final<8, false>), grid1d(n0), dim3(256), rawc, K, H, W, n0, c, q0,
                       (const float*)nullptr, (const float*)GI1, R1, L, outc, wout);
        else if (cw)
            MNF_LAUNCH(ctx, MNF_K_FUSE, st, (k_fuse_final<kMaxK, true>), grid1d(n0), dim3(256), rawc, K, H, W, n0, c,
                       q0, (const float*)W0, (const float*)GI1, R1, L, outc, wout);
        else
            MNF_LAUNCH(ctx, MNF_K_FUSE, st, (k_fuse_final<kMaxK, false>), grid1d(n0), dim3(256), rawc, K, H, W, n0, c,
                       q0, (const float*)nullptr, (const float*)GI1, R1, L, outc, wout);
    }
    MNF_CHECK_LAUNCH(ctx);
    return MNF_OK;
}

extern "C" int fuse_linear(mnf_ctx* ctx, const uint16_t* raw, const float* t, int J, int K, int H, int W, float sat,
                           float dark, int mode, float* fused, void* stream) {
    MNF_TRY(begin(ctx));
    if (!raw || !t || !fused) return set_error(ctx, MNF_EINVAL, "null pointer argument");
    if (J <= 0 || K <= 0 || H <= 0 || W <= 0)
        return set_error(ctx, MNF_EINVAL, "sizes must be positive (J=%d K=%d H=%d W=%d)", J, K, H, W);
    if (mode != 0 && mode != 1) return set_error(ctx, MNF_EINVAL, "mode must be 0 (linear) or 1 (shortest frame)");
    if (!(sat > dark)) return set_error(ctx, MNF_EINVAL, "sat must exceed dark");
    for (int k = 0; k < K; ++k)
        if (!(t[k] > 0.f)) return set_error(ctx, MNF_EINVAL, "exposure time %d must be positive", k);
    hipStream_t st = (hipStream_t)stream;
    void* dt;
    MNF_TRY(upload(ctx, "linear_t", t, sizeof(float) * K, st, &dt));
    const size_t npix = (size_t)H * W, total = (size_t)J * npix;
    MNF_LAUNCH(ctx, MNF_K_FUSE, st, k_fuse_linear, grid1d(total), dim3(256), raw, K, npix, total, (const float*)dt,
               sat, dark, mode, fused);
    MNF_CHECK_LAUNCH(ctx);
    return MNF_OK;
}
