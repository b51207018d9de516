// Multi-scale non-linear fusion (Methods 3.4, Eqs. 5-10) of exposure brackets.
//
// Positions are processed in chunks sized to a scratch budget.  For each
// exposure k the chunk's Gaussian pyramids of I_tilde_k and W_k are built
// level by level in HBM scratch, and the modulated, quantised band-pass
// coefficients are accumulated over k into one fused pyramid F_l.  The
// per-exposure reconstructions of Eq. 9 are linear in their coefficients,
// so collapsing the summed pyramid once equals summing the K per-exposure
// collapses (Eq. 10); quantisation is applied per exposure before the sum.
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
    float dark;
    float mu, inv_2s2;        // weight centre and 1 / (2 sigma^2)
    float scale[kMaxK];       // I_tilde_k = (I_k - dark) * scale[k]  (radiometric) or I_bar_k
    int radiometric;
};

__device__ __forceinline__ int reflect101(int i, int n) { return i < 0 ? -i : (i >= n ? 2 * (n - 1) - i : i); }

// Level 0 of exposure k for every pixel of the chunk: I_tilde_k and the
// normalised weight W_k (computed from all K frames of the pixel).
__global__ void __launch_bounds__(256)
k_fuse_level0(const uint16_t* __restrict__ raw, int K, int k, size_t npix, size_t total,
              FuseConsts c, float* __restrict__ GI, float* __restrict__ GW,
              float* __restrict__ weights_out) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const size_t jj = i / npix, q = i % npix;
    const uint16_t* px = raw + jj * (size_t)K * npix + q;
    float wsum = 0.f, wk = 0.f, Ik = 0.f, Ibar_k = 0.f;
    for (int kk = 0; kk < K; ++kk) {
        const float I = (float)px[(size_t)kk * npix];
        const float Ib = fminf(fmaxf((I - c.dark) * c.inv_range, 0.f), 1.f);
        const float d = Ib - c.mu;
        const float w = expf(-d * d * c.inv_2s2);
        wsum += w;
        if (kk == k) {
            wk = w;
            Ik = I;
            Ibar_k = Ib;
        }
    }
    const float W = wk / fmaxf(wsum, 1e-30f);
    GI[i] = c.radiometric ? (Ik - c.dark) * c.scale[k] : Ibar_k;
    GW[i] = W;
    if (weights_out) weights_out[(jj * K + k) * npix + q] = W;
}

// G_{l+1} = D(G_l * w_G) for the image and the weight pyramids together.
__global__ void __launch_bounds__(256)
k_fuse_reduce(const float* __restrict__ GI, const float* __restrict__ GW, int h, int w, size_t total,
              float* __restrict__ GI1, float* __restrict__ GW1) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int h2 = h >> 1, w2 = w >> 1;
    const size_t jj = i / ((size_t)h2 * w2);
    const int r = (int)(i % ((size_t)h2 * w2));
    const int oy = r / w2, ox = r % w2;
    const float wt[5] = {0.0625f, 0.25f, 0.375f, 0.25f, 0.0625f};
    const float* gi = GI + jj * (size_t)h * w;
    const float* gw = GW + jj * (size_t)h * w;
    float si = 0.f, sw = 0.f;
#pragma unroll
    for (int a = 0; a < 5; ++a) {
        const int yy = reflect101(2 * oy + a - 2, h);
        float ri = 0.f, rw = 0.f;
#pragma unroll
        for (int b = 0; b < 5; ++b) {
            const int xx = reflect101(2 * ox + b - 2, w);
            ri += wt[b] * gi[(size_t)yy * w + xx];
            rw += wt[b] * gw[(size_t)yy * w + xx];
        }
        si += wt[a] * ri;
        sw += wt[a] * rw;
    }
    GI1[i] = si;
    GW1[i] = sw;
}

// Expand of a coarse image g (hc x wc) evaluated at fine pixel (y, x).
__device__ __forceinline__ float expand_at(const float* __restrict__ g, int hc, int wc, int y, int x) {
    int iy[3], ix[3];
    float wy[3], wx[3];
    int ny, nx;
    const int cy = y >> 1, cx = x >> 1;
    if ((y & 1) == 0) {
        iy[0] = cy - 1 < 0 ? 1 : cy - 1;
        iy[1] = cy;
        iy[2] = cy + 1 >= hc ? hc - 1 : cy + 1;
        wy[0] = 0.125f; wy[1] = 0.75f; wy[2] = 0.125f;
        ny = 3;
    } else {
        iy[0] = cy;
        iy[1] = cy + 1 >= hc ? hc - 1 : cy + 1;
        wy[0] = 0.5f; wy[1] = 0.5f;
        ny = 2;
    }
    if ((x & 1) == 0) {
        ix[0] = cx - 1 < 0 ? 1 : cx - 1;
        ix[1] = cx;
        ix[2] = cx + 1 >= wc ? wc - 1 : cx + 1;
        wx[0] = 0.125f; wx[1] = 0.75f; wx[2] = 0.125f;
        nx = 3;
    } else {
        ix[0] = cx;
        ix[1] = cx + 1 >= wc ? wc - 1 : cx + 1;
        wx[0] = 0.5f; wx[1] = 0.5f;
        nx = 2;
    }
    float s = 0.f;
    for (int a = 0; a < ny; ++a) {
        float r = 0.f;
        for (int b = 0; b < nx; ++b) r += wx[b] * g[(size_t)iy[a] * wc + ix[b]];
        s += wy[a] * r;
    }
    return s;
}

// Band level l < L: F_l (+)= Q(G_l[W] (G_l[I] - U(G_{l+1}[I]))); base l = L:
// F_L (+)= G_L[W] G_L[I].  `first` starts the sum over exposures.
__global__ void __launch_bounds__(256)
k_fuse_band(const float* __restrict__ GI, const float* __restrict__ GW, const float* __restrict__ GIc,
            int h, int w, size_t total, float step, int base, int first, float* __restrict__ F) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    float v;
    if (base) {
        v = GW[i] * GI[i];
    } else {
        const size_t jj = i / ((size_t)h * w);
        const int r = (int)(i % ((size_t)h * w));
        const int y = r / w, x = r % w;
        const int hc = h >> 1, wc = w >> 1;
        const float lap = GI[i] - expand_at(GIc + jj * (size_t)hc * wc, hc, wc, y, x);
        v = GW[i] * lap;
        if (step > 0.f) v = step * rintf(v / step);
    }
    F[i] = first ? v : F[i] + v;
}

// Collapse step: R_l = U(R_{l+1}) + F_l, written to out (F_l in place, or the
// fused output at level 0).
__global__ void __launch_bounds__(256)
k_fuse_collapse(const float* __restrict__ Rc, const float* F, int h, int w, size_t total, float* out) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const size_t jj = i / ((size_t)h * w);
    const int r = (int)(i % ((size_t)h * w));
    const int y = r / w, x = r % w;
    const int hc = h >> 1, wc = w >> 1;
    out[i] = F[i] + expand_at(Rc + jj * (size_t)hc * wc, hc, wc, y, x);
}

__global__ void k_copy_f32(float* __restrict__ dst, const float* __restrict__ src, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

inline dim3 grid1d(size_t n) { return dim3((unsigned)((n + 255) / 256)); }

}  // namespace

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

    hipStream_t st = (hipStream_t)stream;
    FuseConsts c{};
    c.inv_range = (float)(1.0 / ((double)p->sat - (double)p->dark));
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

    // pyramid offsets per position (floats)
    std::vector<size_t> off(L + 2, 0);
    for (int l = 0; l <= L; ++l) off[l + 1] = off[l] + (size_t)(H >> l) * (W >> l);
    const size_t per_pos = off[L + 1];
    const size_t budget = (size_t)1 << 30;  // bytes of scratch for three pyramids
    const int chunk = (int)std::max<size_t>(1, std::min<size_t>((size_t)J, budget / (3 * per_pos * sizeof(float))));
    void *gi_v, *gw_v, *f_v;
    MNF_TRY(scratch(ctx, "fuseGI", (size_t)chunk * per_pos * sizeof(float), &gi_v));
    MNF_TRY(scratch(ctx, "fuseGW", (size_t)chunk * per_pos * sizeof(float), &gw_v));
    MNF_TRY(scratch(ctx, "fuseF", (size_t)chunk * per_pos * sizeof(float), &f_v));
    float* GI = (float*)gi_v;
    float* GWp = (float*)gw_v;
    float* F = (float*)f_v;
    const size_t npix = (size_t)H * W;

    for (int j0 = 0; j0 < J; j0 += chunk) {
        const int nj = std::min(chunk, J - j0);
        // level-l arrays of the chunk are [nj][h_l][w_l] at offset nj * off[l]
        auto lvl = [&](float* base, int l) { return base + (size_t)nj * off[l]; };
        const uint16_t* rawc = raw + (size_t)j0 * K * npix;
        for (int k = 0; k < K; ++k) {
            const size_t n0 = (size_t)nj * npix;
            MNF_LAUNCH(ctx, MNF_K_FUSE, st, k_fuse_level0, grid1d(n0), dim3(256), rawc, K, k, npix, n0, c, GI, GWp, weights_out ? weights_out + (size_t)j0 * K * npix : (float*)nullptr);
            for (int l = 0; l < L; ++l) {
                const int h = H >> l, w = W >> l;
                const size_t n1 = (size_t)nj * (h >> 1) * (w >> 1);
                MNF_LAUNCH(ctx, MNF_K_FUSE, st, k_fuse_reduce, grid1d(n1), dim3(256), lvl(GI, l), lvl(GWp, l), h, w, n1, lvl(GI, l + 1), lvl(GWp, l + 1));
            }
            for (int l = 0; l <= L; ++l) {
                const int h = H >> l, w = W >> l;
                const size_t n = (size_t)nj * h * w;
                const float s = l < L ? step[(size_t)l * K + k] : 0.f;
                MNF_LAUNCH(ctx, MNF_K_FUSE, st, k_fuse_band, grid1d(n), dim3(256), lvl(GI, l), lvl(GWp, l), l < L ? lvl(GI, l + 1) : (const float*)nullptr, h, w, n, s, l == L ? 1 : 0,
                                   k == 0 ? 1 : 0, lvl(F, l));
            }
        }
        float* outc = fused + (size_t)j0 * npix;
        if (L == 0) {
            MNF_LAUNCH(ctx, MNF_K_FUSE, st, k_copy_f32, grid1d((size_t)nj * npix), dim3(256), outc, lvl(F, 0), (size_t)nj * npix);
        }
        for (int l = L - 1; l >= 0; --l) {
            const int h = H >> l, w = W >> l;
            const size_t n = (size_t)nj * h * w;
            MNF_LAUNCH(ctx, MNF_K_FUSE, st, k_fuse_collapse, grid1d(n), dim3(256), lvl(F, l + 1), lvl(F, l), h, w, n, l == 0 ? outc : lvl(F, l));
        }
    }
    MNF_CHECK_LAUNCH(ctx);
    return MNF_OK;
}
