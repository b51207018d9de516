// Supporting kernels of the reconstruction workflow: detector exposures of a
// clean intensity (synthetic data at scale), stitching of predicted object
// patches into a starting object, the object NRMSE, and the resampling that
// turns one far-field pattern into a discrete-spectrum measurement.
#include <cmath>
#include <vector>

#include "common.hpp"
#include "kernels_common.hpp"

using namespace mnf;

namespace {

constexpr int kSyncIters = 200;

// Philox4x32-10 counter-based generator (Salmon, Moraes, Dror & Shaw, SC 2011):
// ten rounds of two 32x32->64 multiplications on a 128-bit counter with a
// 64-bit key bumped by the Weyl constants.
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint2 k) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c = make_uint4(hi1 ^ c.y ^ k.x, lo1, hi0 ^ c.w ^ k.y, lo0);
        k.x += 0x9E3779B9u;
        k.y += 0xBB67AE85u;
    }
    return c;
}

// uniform in (0, 1]
__device__ __forceinline__ float u01(uint32_t v) { return ((float)(v >> 8) + 1.f) * (1.f / 16777216.f); }

// uniform in (0, 1), double, from 32 bits
__device__ __forceinline__ double u01d(uint32_t v) { return ((double)v + 0.5) * (1.0 / 4294967296.0); }

// Exact Poisson variate of mean lam >= 10 by transformed rejection with
// squeeze (W. Hoermann, "The transformed rejection method for generating
// Poisson random variables", Insurance: Mathematics and Economics 12, 1993:
// the method PTRS, its hat and squeeze constants).  Trial t takes the pair
// of uniforms (U, V) = words (2 (t mod 2), 2 (t mod 2) + 1) of the counter
// block t / 2 + 1 of element i (block 0 feeds the read noise); the expected
// number of trials is about 1.1, and after 64 rejections in a row
// (probability below 1e-60) the mean rounded is returned.
__device__ int poisson_ptrs(double lam, size_t i, uint2 key) {
    const double slam = sqrt(lam), loglam = log(lam);
    const double b = 0.931 + 2.53 * slam;
    const double a = -0.059 + 0.02483 * b;
    const double inv_alpha = 1.1239 + 1.1328 / (b - 3.4);
    const double v_r = 0.9277 - 3.6224 / (b - 2.0);
    uint4 r = make_uint4(0u, 0u, 0u, 0u);
    for (int trial = 0; trial < 64; ++trial) {
        if ((trial & 1) == 0)
            r = philox4x32_10(make_uint4((uint32_t)i, (uint32_t)(i >> 32), (uint32_t)(trial / 2 + 1), 0u), key);
        const double U = u01d((trial & 1) ? r.z : r.x) - 0.5;
        const double V = u01d((trial & 1) ? r.w : r.y);
        const double us = 0.5 - fabs(U);
        if (us <= 0.0) continue;
        const double kd = floor((2.0 * a / us + b) * U + lam + 0.43);
        if (us >= 0.07 && V <= v_r) return (int)kd;
        if (kd < 0.0 || (us < 0.013 && V > us)) continue;
        // accept when V lies under the transformed density
        if (log(V) + log(inv_alpha) - log(a / (us * us) + b) <= -lam + kd * loglam - lgamma(kd + 1.0))
            return (int)kd;
    }
    return (int)rint(lam);
}

// counts = clip(rint(Poisson(scale t_k clean) + N(0, sigma^2)), 0, sat).
// Poisson by inversion below lambda = 10, by transformed rejection above
// (exact in both ranges).
__global__ void k_expose(const float* __restrict__ clean, int J, int K, size_t npix, const float* __restrict__ t,
                         float scale, float sat, float sigma, uint2 key, uint16_t* __restrict__ raw) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t total = (size_t)J * K * npix;
    if (i >= total) return;
    const size_t q = i % npix;
    const size_t jk = i / npix;
    const int k = (int)(jk % K);
    const size_t j = jk / K;
    const float lam = fmaxf(clean[j * npix + q], 0.f) * scale * t[k];
    const uint4 r = philox4x32_10(make_uint4((uint32_t)i, (uint32_t)(i >> 32), 0u, 0u), key);
    // r.x drives the Poisson inversion; r.z, r.w give the read noise (Box-Muller).
    const float u1 = u01(r.x), u3 = u01(r.z), u4 = u01(r.w);
    const float z = sqrtf(-2.f * logf(u3)) * sinpif(2.f * u4);
    float c;
    if (lam < 10.f) {
        float p = expf(-lam), F = p;
        int x = 0;
        while (u1 > F && x < 64) {
            ++x;
            p *= lam / (float)x;
            F += p;
        }
        c = (float)x;
    } else if (lam < 1e8f) {
        c = (float)poisson_ptrs((double)lam, i, key);
    } else {
        c = lam;  // far beyond any full scale: the count clips to sat whatever the draw
    }
    c = rintf(c + sigma * z);
    raw[i] = (uint16_t)fminf(fmaxf(c, 0.f), sat);
}

// Block sum of a float in a fixed order (waves combined in index order);
// red must hold blockDim.x / 64 floats.  Result valid in every thread.
__device__ __forceinline__ float block_sum_f(float v, float* red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    float r = red[0];
    for (int i = 1; i < nw; ++i) r += red[i];
    return r;
}

// Phase synchronisation of window predictions z_j = a_j e^{i phi_j}: the
// Hermitian matrix C_jk = sum over the overlap of windows j and k of
// w_j w_k conj(z_j) z_k (w = |P|^2), one block per pair j <= k.
__global__ void __launch_bounds__(256)
k_sync_gram(const float* __restrict__ patches, const float2* __restrict__ P, const int2* __restrict__ pos, int J,
            int Nw, float2* __restrict__ C) {
    __shared__ float red[4];
    const int j = blockIdx.x, k = blockIdx.y;
    if (k < j) return;  // uniform over the block
    const int2 pj = pos[j], pk = pos[k];
    const int y0 = max(pj.x, pk.x), y1 = min(pj.x, pk.x) + Nw;
    const int x0 = max(pj.y, pk.y), x1 = min(pj.y, pk.y) + Nw;
    float re = 0.f, im = 0.f;
    if (y1 > y0 && x1 > x0) {
        const int h = y1 - y0, w = x1 - x0;
        for (int i = threadIdx.x; i < h * w; i += 256) {
            const int yy = y0 + i / w, xx = x0 + i % w;
            const int uj = (yy - pj.x) * Nw + (xx - pj.y), uk = (yy - pk.x) * Nw + (xx - pk.y);
            const float* a = patches + ((size_t)j * Nw * Nw + uj) * 2;
            const float* b = patches + ((size_t)k * Nw * Nw + uk) * 2;
            const float m = cabs2(P[uj]) * cabs2(P[uk]) * a[0] * b[0];
            float sn, cs;
            sincosf(b[1] - a[1], &sn, &cs);
            re += m * cs;
            im += m * sn;
        }
    }
    re = block_sum_f(re, red);
    im = block_sum_f(im, red);
    if (threadIdx.x == 0) {
        C[(size_t)j * J + k] = make_float2(re, im);
        C[(size_t)k * J + j] = make_float2(re, -im);
    }
}

// Leading eigenvector of C by power iteration from the all-ones vector (C is
// positive semidefinite), projected to unit modulus, common phase chosen so
// that sum_j c_j is real and positive.  One block of 64 ceil(J / 64) threads,
// J <= 1024: with J <= 64 the iterations run in one wavefront.  C is staged in
// LDS once when it fits (J^2 <= kSyncLds); each iteration then reads only LDS.
constexpr int kSyncLds = 8192;  // float2 entries of C staged in LDS (J <= 90)

__global__ void __launch_bounds__(1024) k_sync_power(const float2* __restrict__ C, int J, int iters,
                                                     float2* __restrict__ c) {
    __shared__ float2 v[1024];
    __shared__ float2 Cs[kSyncLds];
    __shared__ float red[16];
    const int t = threadIdx.x;
    const bool staged = J * J <= kSyncLds;  // uniform over the block
    if (staged)
        for (int i = t; i < J * J; i += blockDim.x) Cs[i] = C[i];
    if (t < J) v[t] = make_float2(1.f, 0.f);
    __syncthreads();
    for (int it = 0; it < iters; ++it) {
        float2 acc = make_float2(0.f, 0.f);
        if (t < J) {
            // row t of C times v, in k order (indexing the LDS arrays directly
            // keeps their reads LDS reads)
            if (staged) {
                const int r0 = t * J;
                for (int k = 0; k < J; ++k) {
                    const float2 q = cmul(Cs[r0 + k], v[k]);
                    acc.x += q.x;
                    acc.y += q.y;
                }
            } else {
                const float2* row = C + (size_t)t * J;
                for (int k = 0; k < J; ++k) {
                    const float2 q = cmul(row[k], v[k]);
                    acc.x += q.x;
                    acc.y += q.y;
                }
            }
        }
        const float m = block_max(sqrtf(cabs2(acc)), red);
        __syncthreads();
        if (t < J) v[t] = m > 0.f ? make_float2(acc.x / m, acc.y / m) : make_float2(1.f, 0.f);
        __syncthreads();
    }
    float2 u = make_float2(1.f, 0.f);
    if (t < J) {
        const float r = sqrtf(cabs2(v[t]));
        if (r > 0.f) u = make_float2(v[t].x / r, v[t].y / r);
    }
    const float sr = block_sum_f(t < J ? u.x : 0.f, red);
    const float si = block_sum_f(t < J ? u.y : 0.f, red);
    const float sm = sqrtf(sr * sr + si * si);
    if (t < J) c[t] = sm > 0.f ? cmul(u, make_float2(sr / sm, -si / sm)) : u;
}

// The same power iteration for J <= 64 with 16 lanes per row of C: lane l of
// row j forms the partial sum over k = l, l + 16, ... of C_jk v_k, the 16
// partials are combined by butterfly (a fixed order), and the maximum of the
// row norms is taken across the 4 rows of a wavefront and then across
// wavefronts.  C (J^2 <= 4096) is staged in LDS once.  One block of
// 64 ceil(J / 4) threads.
__global__ void __launch_bounds__(1024) k_sync_power16(const float2* __restrict__ C, int J, int iters,
                                                       float2* __restrict__ c) {
    __shared__ float2 Cs[64 * 64];
    __shared__ float2 v[64];
    __shared__ float red[16];
    const int t = threadIdx.x, row = t >> 4, l = t & 15, w = t >> 6, nw = (int)(blockDim.x >> 6);
    for (int i = t; i < J * J; i += blockDim.x) Cs[i] = C[i];
    if (t < J) v[t] = make_float2(1.f, 0.f);
    __syncthreads();
    for (int it = 0; it < iters; ++it) {
        float2 acc = make_float2(0.f, 0.f);
        if (row < J) {
            for (int k = l; k < J; k += 16) {
                const float2 q = cmul(Cs[row * J + k], v[k]);
                acc.x += q.x;
                acc.y += q.y;
            }
        }
#pragma unroll
        for (int o = 8; o > 0; o >>= 1) {
            acc.x += __shfl_xor(acc.x, o, 64);
            acc.y += __shfl_xor(acc.y, o, 64);
        }
        // every lane of a row holds its sum: the wave's maximum over its 4 rows
        float m = row < J ? sqrtf(cabs2(acc)) : 0.f;
        m = fmaxf(m, __shfl_xor(m, 16, 64));
        m = fmaxf(m, __shfl_xor(m, 32, 64));
        if ((t & 63) == 0) red[w] = m;
        __syncthreads();
        m = red[0];
        for (int q = 1; q < nw; ++q) m = fmaxf(m, red[q]);
        if (row < J && l == 0) v[row] = m > 0.f ? make_float2(acc.x / m, acc.y / m) : make_float2(1.f, 0.f);
        __syncthreads();
    }
    float2 u = make_float2(1.f, 0.f);
    if (t < J) {
        const float r = sqrtf(cabs2(v[t]));
        if (r > 0.f) u = make_float2(v[t].x / r, v[t].y / r);
    }
    const float sr = block_sum_f(t < J ? u.x : 0.f, red);
    const float si = block_sum_f(t < J ? u.y : 0.f, red);
    const float sm = sqrtf(sr * sr + si * si);
    if (t < J) c[t] = sm > 0.f ? cmul(u, make_float2(sr / sm, -si / sm)) : u;
}

// O[x] = sum_j |P(u_j)|^2 c_j amp_j(u_j) e^{i phase_j(u_j)} / sum_j |P(u_j)|^2 over the
// windows containing x (u_j = x - p_j; c_j = 1 without phasors); 1 where no window
// (or only zero probe) covers x.
__global__ void __launch_bounds__(256)
k_stitch(const float* __restrict__ patches, const float2* __restrict__ P, const int2* __restrict__ pos,
         const float2* __restrict__ phasors, int J, int Nw, float2* __restrict__ O, int My, int Mx) {
    __shared__ int2 sp[256];
    __shared__ float2 sc[256];
    const int x = blockIdx.x * 16 + (threadIdx.x % 16);
    const int y = blockIdx.y * 16 + (threadIdx.x / 16);
    float2 num = make_float2(0.f, 0.f);
    float den = 0.f;
    for (int j0 = 0; j0 < J; j0 += 256) {
        __syncthreads();
        if (j0 + (int)threadIdx.x < J) {
            sp[threadIdx.x] = pos[j0 + threadIdx.x];
            sc[threadIdx.x] = phasors ? phasors[j0 + threadIdx.x] : make_float2(1.f, 0.f);
        }
        __syncthreads();
        const int nj = min(256, J - j0);
        for (int jj = 0; jj < nj; ++jj) {
            const int uy = y - sp[jj].x, ux = x - sp[jj].y;
            if (uy < 0 || uy >= Nw || ux < 0 || ux >= Nw) continue;
            const float w = cabs2(P[uy * Nw + ux]);
            const float* pa = patches + (((size_t)(j0 + jj) * Nw + uy) * Nw + ux) * 2;
            float s, c;
            sincosf(pa[1], &s, &c);
            const float2 z = cmul(sc[jj], make_float2(pa[0] * c, pa[0] * s));
            num.x += w * z.x;
            num.y += w * z.y;
            den += w;
        }
    }
    if (y < My && x < Mx) O[(size_t)y * Mx + x] = den > 0.f ? make_float2(num.x / den, num.y / den) : make_float2(1.f, 0.f);
}

// Per-block float64 sums over masked pixels: <O, T> (re, im), |O|^2, |T|^2.
__global__ void __launch_bounds__(256)
k_nrmse_part(const float2* __restrict__ O, const float2* __restrict__ T, const uint8_t* __restrict__ mask, size_t n,
             double* __restrict__ part) {
    __shared__ double red[4];
    double s[4] = {0, 0, 0, 0};
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        if (mask && !mask[i]) continue;
        const float2 o = O[i], t = T[i];
        s[0] += (double)o.x * t.x + (double)o.y * t.y;
        s[1] += (double)o.x * t.y - (double)o.y * t.x;
        s[2] += (double)o.x * o.x + (double)o.y * o.y;
        s[3] += (double)t.x * t.x + (double)t.y * t.y;
    }
    for (int c = 0; c < 4; ++c) {
        const double v = block_sum(s[c], red);
        if (threadIdx.x == 0) part[blockIdx.x * 4 + c] = v;
        __syncthreads();
    }
}

// min_gamma ||gamma O - T|| / ||T|| = sqrt(1 - |<O,T>|^2 / (|O|^2 |T|^2)).
__global__ void k_nrmse_final(const double* __restrict__ part, int nb, double* __restrict__ out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s[4] = {0, 0, 0, 0};
    for (int b = 0; b < nb; ++b)
        for (int c = 0; c < 4; ++c) s[c] += part[b * 4 + c];
    const double ip2 = s[0] * s[0] + s[1] * s[1];
    double r = s[3] > 0.0 ? 1.0 - (s[2] > 0.0 ? ip2 / (s[2] * s[3]) : 0.0) : 0.0;
    *out = sqrt(r > 0.0 ? r : 0.0);
}

// Discrete-spectrum measurement: out (+)= w s^2 I(c + (k - c) s) per pixel,
// bilinear between pixels, zero outside the detector (c = Nd / 2).
__global__ void __launch_bounds__(256)
k_resample_add(const float* __restrict__ I, int Nd, size_t total, float s, float w, int accumulate,
               float* __restrict__ out) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const size_t npix = (size_t)Nd * Nd;
    const size_t j = i / npix;
    const int q = (int)(i % npix), ky = q / Nd, kx = q % Nd;
    const int c = Nd / 2;
    const float u = (float)c + (float)(ky - c) * s, v = (float)c + (float)(kx - c) * s;
    const float fy0 = floorf(u), fx0 = floorf(v);
    const int y0 = (int)fy0, x0 = (int)fx0;
    const float fy = u - fy0, fx = v - fx0;
    const float* Ij = I + j * npix;
    float r = 0.f;
#pragma unroll
    for (int dy = 0; dy < 2; ++dy) {
        const int yy = y0 + dy;
        if (yy < 0 || yy >= Nd) continue;
        const float wy = dy ? fy : 1.f - fy;
#pragma unroll
        for (int dx = 0; dx < 2; ++dx) {
            const int xx = x0 + dx;
            if (xx < 0 || xx >= Nd) continue;
            r += wy * (dx ? fx : 1.f - fx) * Ij[(size_t)yy * Nd + xx];
        }
    }
    const float v_out = w * s * s * r;
    out[i] = accumulate ? out[i] + v_out : v_out;
}

}  // namespace

extern "C" {

int detector_expose(mnf_ctx* ctx, const float* clean, int J, int H, int W, const float* t, int K, float scale,
                    float sat, float sigma_read, unsigned long long seed, uint16_t* raw, void* stream) {
    MNF_TRY(begin(ctx));
    if (!clean || !t || !raw || J <= 0 || H <= 0 || W <= 0 || K <= 0 || K > 16)
        return set_error(ctx, MNF_EINVAL, "bad exposure arguments");
    if (!(scale >= 0.f) || !(sat > 0.f) || !(sigma_read >= 0.f) || sat > 65535.f)
        return set_error(ctx, MNF_EINVAL, "scale, sat and sigma_read must be non-negative (sat <= 65535)");
    hipStream_t st = (hipStream_t)stream;
    void* dt;
    MNF_TRY(upload(ctx, "expose_t", t, sizeof(float) * K, st, &dt));
    const size_t npix = (size_t)H * W, total = (size_t)J * K * npix;
    const uint2 key = make_uint2((uint32_t)seed, (uint32_t)(seed >> 32));
    MNF_LAUNCH(ctx, MNF_K_SMALL, st, k_expose, dim3((unsigned)((total + 255) / 256)), dim3(256), clean, J, K, npix,
               (const float*)dt, scale, sat, sigma_read, key, raw);
    MNF_CHECK_LAUNCH(ctx);
    return MNF_OK;
}

int ptycho_stitch(mnf_ctx* ctx, const float* patches, const mnf_c64* P, int Nw, const int32_t* pos, int J,
                  int sync, mnf_c64* O, int My, int Mx, void* stream) {
    MNF_TRY(begin(ctx));
    if (!patches || !P || !pos || !O || J <= 0 || Nw <= 0 || My <= 0 || Mx <= 0)
        return set_error(ctx, MNF_EINVAL, "bad stitching arguments");
    if (sync && J > 1024) return set_error(ctx, MNF_EINVAL, "phase synchronisation takes at most 1024 windows");
    for (int j = 0; j < J; ++j)
        if (pos[2 * j] < 0 || pos[2 * j + 1] < 0 || pos[2 * j] + Nw > My || pos[2 * j + 1] + Nw > Mx)
            return set_error(ctx, MNF_EINVAL, "window %d lies outside the object", j);
    hipStream_t st = (hipStream_t)stream;
    void* dpos;
    MNF_TRY(upload(ctx, "stitch_pos", pos, sizeof(int32_t) * 2 * J, st, &dpos));
    float2* phasors = nullptr;
    if (sync) {
        void* C;
        void* cv;
        MNF_TRY(scratch(ctx, "sync_gram", sizeof(float2) * (size_t)J * J, &C));
        MNF_TRY(scratch(ctx, "sync_phasors", sizeof(float2) * (size_t)J, &cv));
        MNF_LAUNCH(ctx, MNF_K_SMALL, st, k_sync_gram, dim3(J, J), dim3(256), patches, (const float2*)P,
                   (const int2*)dpos, J, Nw, (float2*)C);
        if (J <= 64)
            MNF_LAUNCH(ctx, MNF_K_SMALL, st, k_sync_power16, dim3(1), dim3((unsigned)(64 * ((J + 3) / 4))),
                       (const float2*)C, J, kSyncIters, (float2*)cv);
        else
            MNF_LAUNCH(ctx, MNF_K_SMALL, st, k_sync_power, dim3(1), dim3((unsigned)(64 * ((J + 63) / 64))),
                       (const float2*)C, J, kSyncIters, (float2*)cv);
        phasors = (float2*)cv;
    }
    MNF_LAUNCH(ctx, MNF_K_SMALL, st, k_stitch, dim3((Mx + 15) / 16, (My + 15) / 16), dim3(256), patches,
               (const float2*)P, (const int2*)dpos, (const float2*)phasors, J, Nw, (float2*)O, My, Mx);
    MNF_CHECK_LAUNCH(ctx);
    return MNF_OK;
}

int mnf_nrmse(mnf_ctx* ctx, const mnf_c64* O, const mnf_c64* O_true, const uint8_t* mask, long long n, double* out,
              void* stream) {
    MNF_TRY(begin(ctx));
    if (!O || !O_true || !out || n <= 0) return set_error(ctx, MNF_EINVAL, "bad NRMSE arguments");
    hipStream_t st = (hipStream_t)stream;
    const int nb = 256;
    void* part;
    MNF_TRY(scratch(ctx, "nrmse_part", (size_t)nb * 4 * sizeof(double), &part));
    MNF_LAUNCH(ctx, MNF_K_SMALL, st, k_nrmse_part, dim3(nb), dim3(256), (const float2*)O, (const float2*)O_true, mask,
               (size_t)n, (double*)part);
    MNF_LAUNCH(ctx, MNF_K_SMALL, st, k_nrmse_final, dim3(1), dim3(64), (const double*)part, nb, out);
    MNF_CHECK_LAUNCH(ctx);
    return MNF_OK;
}

int detector_resample(mnf_ctx* ctx, const float* I, int J, int Nd, float scale, float weight, int accumulate,
                      float* out, void* stream) {
    MNF_TRY(begin(ctx));
    if (!I || !out || J <= 0 || Nd <= 0) return set_error(ctx, MNF_EINVAL, "bad resampling arguments");
    if (!(scale > 0.f)) return set_error(ctx, MNF_EINVAL, "scale must be positive");
    if (I == out) return set_error(ctx, MNF_EINVAL, "input and output must not alias");
    hipStream_t st = (hipStream_t)stream;
    const size_t total = (size_t)J * Nd * Nd;
    MNF_LAUNCH(ctx, MNF_K_SMALL, st, k_resample_add, dim3((unsigned)((total + 255) / 256)), dim3(256), I, Nd, total,
               scale, weight, accumulate, out);
    MNF_CHECK_LAUNCH(ctx);
    return MNF_OK;
}

}  // extern "C"
