// BF16 MFMA convolution kernels of the warm-start network (implicit GEMM,
// float32 accumulation, channels-last activations).
//
// Forward and input-gradient convolutions are one GEMM kernel,
//   out[m][n] = sum_k A[m][k] Bt[n][k]  (+ bias, + residual, ReLU),
// where the rows of A are gathered from the input tensor according to the
// layer kind (MODE) and Bt holds bf16 weights in GEMM order [n][k], prepared
// from the float32 parameters by k_prep_weights.  The four kinds are closed
// under taking the input gradient:
//   CONV3 (3x3, stride 1, pad 1) -> CONV3 with flipped taps, transposed;
//   DOWN  (2x2, stride 2)        -> UP  with transposed taps;
//   UP    (2x2 transposed)       -> DOWN with transposed taps;
//   CONV1                        -> CONV1 transposed.
// A ReLU backward is fused into the A gather (A = dAct * (act > 0)).
// The weight gradient is a second GEMM over pixels (split over pixel ranges
// into float32 partials, reduced in a fixed order).
//
// MFMA: v_mfma_f32_32x32x16_bf16.  Lane l supplies A[i = l % 32][k = 8 (l / 32) + 0..7]
// and B[k = 8 (l / 32) + 0..7][j = l % 32]; accumulator register v holds
// C[8 (v / 4) + 4 (l / 32) + (v % 4)][l % 32].
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels_common.hpp"

namespace mnf {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));

enum ConvMode { CONV3 = 0, DOWN = 1, UP = 2, CONV1 = 3 };

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
// float -> bf16, round to nearest even (subnormals included), infinities
// kept, NaNs quiet: the hardware conversion (v_cvt_pk_bf16_f32), which for
// every non-NaN input gives the bits of the integer rounding
// (u + 0x7fff + ((u >> 16) & 1)) >> 16 of the float's bits u.
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }

struct ConvArgs {
    const uint16_t* in;     // [n][Hin][Win][in_cs] bf16, channels [in_co, in_co + Cin)
    int in_cs, in_co;
    const uint16_t* mask;   // ReLU mask source laid out like `in` (MASK), or null
    int mask_cs, mask_co;
    const uint16_t* Bt;     // [taps_b][Nout][Kpad] bf16 (taps_b = 4 for UP, else 1)
    int Kpad;
    const float* bias;      // [Nout] or null
    const uint16_t* resid;  // addend at the output pixels [..][res_cs], channels from res_co, or null
    int res_cs, res_co;
    void* out;              // [n][Hout][Wout][out_cs], channels [out_co, out_co + Nout)
    int out_cs, out_co;
    int n, Hin, Win, Cin, Hout, Wout, Nout;
    int relu;
    int M;                  // rows of the GEMM (output pixels; for UP 4 parity groups of per_pad rows)
    int per_pad;            // UP: input pixels per parity group rounded up to the row tile
};

constexpr int kGemmBM = 128, kGemmBN = 64, kGemmThreads = 256;

// K chunk per global round trip: 64 (four MFMA steps per wave) for long
// reductions, 32 for short ones (the first layer has K = 9); Kpad is K rounded
// up to the chunk, so the chunk follows from Kpad alone (Kpad > 64 <=> 64).
__host__ __device__ constexpr int gemm_bk(int K) { return K <= 64 ? 32 : 64; }

template <int BK>
struct GemmTile {
    static constexpr int LDS = BK + 8;                  // padded LDS row (bf16)
    static constexpr int TPR = BK / 8;                  // threads per row, 8 columns each
    static constexpr int RSTEP = kGemmThreads / TPR;    // rows one pass of the block loads
    static constexpr int ACH = kGemmBM / RSTEP, BCH = kGemmBN / RSTEP;
};

// Input pixel feeding GEMM row m and column k (tap = k / Cin) for the forward
// gather; returns false for zero padding.  For UP the tap is the output
// pixel's parity and every k of a row reads the same input pixel.
template <int MODE>
__device__ __forceinline__ bool gather_pixel(const ConvArgs& a, int m, int tap, size_t* pix) {
    if constexpr (MODE == UP) {
        const int r = m % a.per_pad;
        *pix = (size_t)r;
        return r < a.n * a.Hin * a.Win;
    } else {
        const int x = m % a.Wout;
        const int t1 = m / a.Wout;
        const int y = t1 % a.Hout;
        const int img = t1 / a.Hout;
        int yy, xx;
        if constexpr (MODE == CONV3) {
            yy = y + tap / 3 - 1;
            xx = x + tap % 3 - 1;
        } else if constexpr (MODE == DOWN) {
            yy = 2 * y + tap / 2;
            xx = 2 * x + tap % 2;
        } else {
            yy = y;
            xx = x;
        }
        if (yy < 0 || yy >= a.Hin || xx < 0 || xx >= a.Win) return false;
        *pix = ((size_t)img * a.Hin + yy) * a.Win + xx;
        return true;
    }
}

// Output pixel of GEMM row m (UP rows are grouped by output parity).
template <int MODE>
__device__ __forceinline__ size_t out_pixel(const ConvArgs& a, int m) {
    if constexpr (MODE == UP) {
        const int q = m / a.per_pad, r = m % a.per_pad;
        const int x = r % a.Win, t1 = r / a.Win;
        const int y = t1 % a.Hin, img = t1 / a.Hin;
        return ((size_t)img * a.Hout + 2 * y + q / 2) * a.Wout + 2 * x + q % 2;
    } else {
        return (size_t)m;
    }
}

// Eight consecutive GEMM columns k .. k+7 of row m (bf16 bits), masked.
template <int MODE, bool MASK, bool VEC>
__device__ __forceinline__ uint4 load_a8(const ConvArgs& a, int m, int k) {
    uint4 r = make_uint4(0, 0, 0, 0);
    if (m >= a.M) return r;
    const int K = (MODE == CONV3 ? 9 : (MODE == DOWN ? 4 : 1)) * a.Cin;
    if constexpr (VEC) {
        if (k >= K) return r;
        const int tap = k / a.Cin, ci = k % a.Cin;
        size_t pix;
        if (!gather_pixel<MODE>(a, m, tap, &pix)) return r;
        r = *(const uint4*)(a.in + pix * a.in_cs + a.in_co + ci);
        if constexpr (MASK) {
            const uint4 g = *(const uint4*)(a.mask + pix * a.mask_cs + a.mask_co + ci);
            uint32_t* rv = (uint32_t*)&r;
            const uint32_t* gv = (const uint32_t*)&g;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint32_t lo = (gv[q] & 0xffffu), hi = gv[q] >> 16;
                const bool plo = lo != 0 && !(lo & 0x8000u), phi = hi != 0 && !(hi & 0x8000u);
                rv[q] = (plo ? (rv[q] & 0xffffu) : 0u) | (phi ? (rv[q] & 0xffff0000u) : 0u);
            }
        }
        return r;
    } else {
        uint16_t v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            v[q] = 0;
            const int kk = k + q;
            if (kk < K) {
                const int tap = kk / a.Cin, ci = kk % a.Cin;
                size_t pix;
                if (gather_pixel<MODE>(a, m, tap, &pix)) {
                    uint16_t x = a.in[pix * a.in_cs + a.in_co + ci];
                    if constexpr (MASK) {
                        const uint16_t g = a.mask[pix * a.mask_cs + a.mask_co + ci];
                        if (g == 0 || (g & 0x8000u)) x = 0;
                    }
                    v[q] = x;
                }
            }
        }
        r.x = v[0] | ((uint32_t)v[1] << 16);
        r.y = v[2] | ((uint32_t)v[3] << 16);
        r.z = v[4] | ((uint32_t)v[5] << 16);
        r.w = v[6] | ((uint32_t)v[7] << 16);
        return r;
    }
}

// The output pixel of GEMM row m decomposed once (valid: m < M; for UP the
// input pixel r of the row), so that the K loop's gathers need no division.
struct RowGeom {
    int valid, img, y, x;
};

template <int MODE>
__device__ __forceinline__ RowGeom row_geom(const ConvArgs& a, int m) {
    RowGeom g{m < a.M ? 1 : 0, 0, 0, 0};
    if (!g.valid) return g;
    if constexpr (MODE == UP) {
        g.x = m % a.per_pad;  // the input pixel
        g.valid = g.x < a.n * a.Hin * a.Win;
    } else {
        g.x = m % a.Wout;
        const int t1 = m / a.Wout;
        g.y = t1 % a.Hout;
        g.img = t1 / a.Hout;
    }
    return g;
}

// Eight consecutive GEMM columns of tap `tap`, channels ci .. ci+7 (Cin a
// multiple of 8), of a row with decomposed geometry: load_a8<VEC> without the
// per-load index arithmetic.
template <int MODE, bool MASK>
__device__ __forceinline__ uint4 load_a8_geom(const ConvArgs& a, const RowGeom& g, int tap, int ci, bool kin) {
    uint4 r = make_uint4(0, 0, 0, 0);
    if (!g.valid || !kin) return r;
    size_t pix;
    if constexpr (MODE == UP) {
        pix = (size_t)g.x;
    } else {
        int yy = g.y, xx = g.x;
        if constexpr (MODE == CONV3) {
            yy += tap / 3 - 1;
            xx += tap % 3 - 1;
        } else if constexpr (MODE == DOWN) {
            yy = 2 * g.y + (tap >> 1);
            xx = 2 * g.x + (tap & 1);
        }
        if (yy < 0 || yy >= a.Hin || xx < 0 || xx >= a.Win) return r;
        pix = ((size_t)g.img * a.Hin + yy) * a.Win + xx;
    }
    r = *(const uint4*)(a.in + pix * a.in_cs + a.in_co + ci);
    if constexpr (MASK) {
        const uint4 gm = *(const uint4*)(a.mask + pix * a.mask_cs + a.mask_co + ci);
        uint32_t* rv = (uint32_t*)&r;
        const uint32_t* gv = (const uint32_t*)&gm;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint32_t lo = (gv[q] & 0xffffu), hi = gv[q] >> 16;
            const bool plo = lo != 0 && !(lo & 0x8000u), phi = hi != 0 && !(hi & 0x8000u);
            rv[q] = (plo ? (rv[q] & 0xffffu) : 0u) | (phi ? (rv[q] & 0xffff0000u) : 0u);
        }
    }
    return r;
}

template <int MODE, bool MASK, bool VEC, bool OUT_F32, int BK>
__global__ void __launch_bounds__(kGemmThreads) k_conv_gemm(ConvArgs a) {
    using G = GemmTile<BK>;
    __shared__ __attribute__((aligned(16))) uint16_t sA[kGemmBM * G::LDS];
    __shared__ __attribute__((aligned(16))) uint16_t sB[kGemmBN * G::LDS];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int m0 = blockIdx.x * kGemmBM, n0 = blockIdx.y * kGemmBN;
    const uint16_t* Bt = a.Bt;
    if constexpr (MODE == UP) Bt += (size_t)(m0 / a.per_pad) * a.Nout * a.Kpad;  // the tile's parity selects the tap
    f32x16_t acc0 = {}, acc1 = {};
    // per-thread load slots: A rows tid/TPR + RSTEP q, B rows likewise, eight columns each
    const int ar = tid / G::TPR, ac = (tid % G::TPR) * 8;
    uint4 ra[G::ACH], rb[G::BCH];
    // the thread's A rows, decomposed once (VEC: every column of the thread's
    // eight lies in one tap, the same for all its rows)
    RowGeom geo[G::ACH];
    if constexpr (VEC) {
#pragma unroll
        for (int q = 0; q < G::ACH; ++q) geo[q] = row_geom<MODE>(a, m0 + G::RSTEP * q + ar);
    }
    const int Ktot = (MODE == CONV3 ? 9 : (MODE == DOWN ? 4 : 1)) * a.Cin;
    auto fetch = [&](int k0) {
        if constexpr (VEC) {
            const int k = k0 + ac;
            const int tap = k / a.Cin, ci = k - tap * a.Cin;
#pragma unroll
            for (int q = 0; q < G::ACH; ++q) ra[q] = load_a8_geom<MODE, MASK>(a, geo[q], tap, ci, k < Ktot);
        } else {
#pragma unroll
            for (int q = 0; q < G::ACH; ++q) ra[q] = load_a8<MODE, MASK, VEC>(a, m0 + G::RSTEP * q + ar, k0 + ac);
        }
#pragma unroll
        for (int q = 0; q < G::BCH; ++q) {
            const int n = n0 + G::RSTEP * q + ar;
            rb[q] = n < a.Nout ? *(const uint4*)(Bt + (size_t)n * a.Kpad + k0 + ac) : make_uint4(0, 0, 0, 0);
        }
    };
    fetch(0);
    for (int k0 = 0; k0 < a.Kpad; k0 += BK) {
        __syncthreads();
#pragma unroll
        for (int q = 0; q < G::ACH; ++q) *(uint4*)(sA + (G::RSTEP * q + ar) * G::LDS + ac) = ra[q];
#pragma unroll
        for (int q = 0; q < G::BCH; ++q) *(uint4*)(sB + (G::RSTEP * q + ar) * G::LDS + ac) = rb[q];
        __syncthreads();
        if (k0 + BK < a.Kpad) fetch(k0 + BK);  // next chunk in flight during the MFMAs
#pragma unroll
        for (int s = 0; s < BK / 16; ++s) {
            const int kk = s * 16 + 8 * (lane >> 5);
            const bf16x8_t av = __builtin_bit_cast(bf16x8_t, *(const uint4*)(sA + (32 * w + (lane & 31)) * G::LDS + kk));
            const bf16x8_t b0 = __builtin_bit_cast(bf16x8_t, *(const uint4*)(sB + (lane & 31) * G::LDS + kk));
            const bf16x8_t b1 = __builtin_bit_cast(bf16x8_t, *(const uint4*)(sB + (32 + (lane & 31)) * G::LDS + kk));
            acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, b0, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, b1, acc1, 0, 0, 0);
        }
    }
    // epilogue: the output pixel of each of the thread's 16 rows, once for
    // both column halves
    size_t opv[16];
    bool okv[16];
    if (MODE == UP && a.Win >= 4) {
        // The block's rows lie in one parity group (per_pad is a multiple of
        // the row tile), so the group is uniform; a lane's rows come in four
        // runs of four consecutive input pixels: one division-based
        // decomposition per run, then at most one row carry per step (Win > 3).
        const int q = m0 / a.per_pad, npx = a.n * a.Hin * a.Win;
        const int rl = m0 - q * a.per_pad + 32 * w + 4 * (lane >> 5);
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const int r = rl + 8 * g;
            const int x = r % a.Win, t1 = r / a.Win;
            const int y = t1 % a.Hin, img = t1 / a.Hin;
#pragma unroll
            for (int d = 0; d < 4; ++d) {
                const int v = 4 * g + d;
                int xd = x + d, yd = y, id = img;
                if (xd >= a.Win) {
                    xd -= a.Win;
                    if (++yd == a.Hin) {
                        yd = 0;
                        ++id;
                    }
                }
                okv[v] = m0 + 32 * w + 4 * (lane >> 5) + 8 * g + d < a.M && r + d < npx;
                opv[v] = okv[v] ? ((size_t)id * a.Hout + 2 * yd + q / 2) * a.Wout + 2 * xd + q % 2 : 0;
            }
        }
    } else {
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int m = m0 + 32 * w + 8 * (v / 4) + 4 * (lane >> 5) + (v % 4);
            okv[v] = m < a.M && (MODE != UP || m % a.per_pad < a.n * a.Hin * a.Win);
            opv[v] = okv[v] ? out_pixel<MODE>(a, m) : 0;
        }
    }
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) {
        const int j = n0 + 32 * nb + (lane & 31);
        if (j >= a.Nout) continue;
        const float bj = a.bias ? a.bias[j] : 0.f;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            if (!okv[v]) continue;
            float y = (nb == 0 ? acc0[v] : acc1[v]) + bj;
            const size_t op = opv[v];
            if (a.resid) y += bf2f(a.resid[op * a.res_cs + a.res_co + j]);
            if (a.relu) y = fmaxf(y, 0.f);
            if constexpr (OUT_F32)
                ((float*)a.out)[op * a.out_cs + a.out_co + j] = y;
            else
                ((uint16_t*)a.out)[op * a.out_cs + a.out_co + j] = f2bf(y);
        }
    }
}

// First 3x3 layer (one input channel, bf16 output, no residual): one thread
// per output pixel computes every output channel from the nine input taps,
// loaded once; the bf16 weights (GEMM order Bt[co][tap], row length Kpad) and
// the biases are staged in LDS as float.  Requires Nout <= 256, Nout a
// multiple of 8 and 16-byte aligned output rows.
__global__ void __launch_bounds__(256) k_conv3_c1(ConvArgs a) {
    __shared__ float sw[256 * 9];
    __shared__ float sb[256];
    for (int i = threadIdx.x; i < a.Nout * 9; i += 256) sw[i] = bf2f(a.Bt[(size_t)(i / 9) * a.Kpad + i % 9]);
    for (int i = threadIdx.x; i < a.Nout; i += 256) sb[i] = a.bias ? a.bias[i] : 0.f;
    __syncthreads();
    const int m = blockIdx.x * 256 + threadIdx.x;
    if (m >= a.M) return;
    const int x = m % a.Wout, t1 = m / a.Wout, y = t1 % a.Hout, img = t1 / a.Hout;
    float v[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        const int yy = y + t / 3 - 1, xx = x + t % 3 - 1;
        v[t] = (yy >= 0 && yy < a.Hin && xx >= 0 && xx < a.Win)
                   ? bf2f(a.in[(((size_t)img * a.Hin + yy) * a.Win + xx) * a.in_cs + a.in_co])
                   : 0.f;
    }
    uint16_t* orow = (uint16_t*)a.out + (size_t)m * a.out_cs + a.out_co;
    for (int c0 = 0; c0 < a.Nout; c0 += 8) {
        uint16_t o[8] __attribute__((aligned(16)));
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const float* wq = sw + (c0 + q) * 9;
            float acc = 0.f;
#pragma unroll
            for (int t = 0; t < 9; ++t) acc += v[t] * wq[t];
            float yv = acc + sb[c0 + q];
            if (a.relu) yv = fmaxf(yv, 0.f);
            o[q] = f2bf(yv);
        }
        *(uint4*)(orow + c0) = *(const uint4*)o;
    }
}

// 3x3 convolution (forward, or input gradient with flipped taps) as a direct
// tiled kernel: a block of WV waves computes TH x TW = 32 WV output pixels of
// one image x 32 NB output channels (NB = 1 for layers with at most 32); the
// weights staged per chunk serve all of the block's pixels, so a larger
// block loads them fewer times per pixel.  Per chunk of 32
// input channels it stages the input patch ((TH + 2) x (TW + 2) pixels, zero
// padded, ReLU-masked for MASK) and the 9 x 32 NB x 32 weights in LDS once,
// then every wave runs its 32 pixels x 32 NB channels through 9 taps x 2 K16
// steps x NB MFMA tiles from LDS, so each input pixel is fetched once per
// chunk instead of once per tap.  Same MFMA lane layout and epilogue as
// k_conv_gemm.  Needs Cin % 32 == 0, 16-byte aligned channel offsets,
// W % TW == 0 and H % TH == 0.
constexpr int kTileCh = 32;               // input channels per chunk
constexpr int kTileLds = kTileCh + 8;     // padded LDS row (bf16) per pixel / weight row

template <bool MASK, bool OUT_F32, int TW, int NB = 2, int WV = 4>
__global__ void __launch_bounds__(64 * WV) k_conv3_tiled(ConvArgs a) {
    constexpr int THREADS = 64 * WV, BM = 32 * WV;  // WV waves, 32 output pixels each
    constexpr int TH = BM / TW;
    constexpr int BN = 32 * NB;  // output channels of the block
    constexpr int PW = TW + 2, PH = TH + 2, NPIX = PW * PH;
    constexpr int A_LOADS = NPIX * (kTileCh / 8);        // 16-byte pieces of the patch
    constexpr int B_LOADS = 9 * BN * (kTileCh / 8);      // 16-byte pieces of the weights
    constexpr int A_PER = (A_LOADS + THREADS - 1) / THREADS;
    constexpr int B_PER = (B_LOADS + THREADS - 1) / THREADS;
    __shared__ __attribute__((aligned(16))) uint16_t sA[NPIX * kTileLds];
    __shared__ __attribute__((aligned(16))) uint16_t sB[9 * BN * kTileLds];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int tiles_x = a.Wout / TW, tiles_y = a.Hout / TH;
    const int tile = blockIdx.x;
    const int img = tile / (tiles_x * tiles_y), tr = tile % (tiles_x * tiles_y);
    const int y0 = (tr / tiles_x) * TH, x0 = (tr % tiles_x) * TW;
    const int n0 = blockIdx.y * BN;
    f32x16_t acc0 = {}, acc1 = {};
    uint4 ra[A_PER], rb[B_PER];
    auto fetch = [&](int c0) {
#pragma unroll
        for (int q = 0; q < A_PER; ++q) {
            const int e = tid + q * THREADS;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (e < A_LOADS) {
                const int pix = e / (kTileCh / 8), piece = e % (kTileCh / 8);
                const int yy = y0 - 1 + pix / PW, xx = x0 - 1 + pix % PW;
                if (yy >= 0 && yy < a.Hin && xx >= 0 && xx < a.Win) {
                    const size_t ip = ((size_t)img * a.Hin + yy) * a.Win + xx;
                    v = *(const uint4*)(a.in + ip * a.in_cs + a.in_co + c0 + 8 * piece);
                    if constexpr (MASK) {
                        const uint4 g = *(const uint4*)(a.mask + ip * a.mask_cs + a.mask_co + c0 + 8 * piece);
                        uint32_t* rv = (uint32_t*)&v;
                        const uint32_t* gv = (const uint32_t*)&g;
#pragma unroll
                        for (int k = 0; k < 4; ++k) {
                            const uint32_t lo = (gv[k] & 0xffffu), hi = gv[k] >> 16;
                            const bool plo = lo != 0 && !(lo & 0x8000u), phi = hi != 0 && !(hi & 0x8000u);
                            rv[k] = (plo ? (rv[k] & 0xffffu) : 0u) | (phi ? (rv[k] & 0xffff0000u) : 0u);
                        }
                    }
                }
            }
            ra[q] = v;
        }
#pragma unroll
        for (int q = 0; q < B_PER; ++q) {
            const int e = tid + q * THREADS;
            const int row = e / (kTileCh / 8), piece = e % (kTileCh / 8);  // row = tap * BN + co
            const int t = row / BN, n = n0 + row % BN;
            rb[q] = e < B_LOADS && n < a.Nout
                        ? *(const uint4*)(a.Bt + (size_t)n * a.Kpad + t * a.Cin + c0 + 8 * piece)
                        : make_uint4(0, 0, 0, 0);
        }
    };
    // this wave's 32 output pixels: row py, columns px0 .. px0 + 31 of the tile
    const int py = (32 * w) / TW, px = (32 * w) % TW + (lane & 31);
    fetch(0);
    for (int c0 = 0; c0 < a.Cin; c0 += kTileCh) {
        __syncthreads();
#pragma unroll
        for (int q = 0; q < A_PER; ++q) {
            const int e = tid + q * THREADS;
            if (e < A_LOADS) *(uint4*)(sA + (e / (kTileCh / 8)) * kTileLds + 8 * (e % (kTileCh / 8))) = ra[q];
        }
#pragma unroll
        for (int q = 0; q < B_PER; ++q) {
            const int e = tid + q * THREADS;
            if (e < B_LOADS) *(uint4*)(sB + (e / (kTileCh / 8)) * kTileLds + 8 * (e % (kTileCh / 8))) = rb[q];
        }
        __syncthreads();
        if (c0 + kTileCh < a.Cin) fetch(c0 + kTileCh);  // next chunk in flight during the MFMAs
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int pix = (py + t / 3) * PW + px + t % 3;
#pragma unroll
            for (int s = 0; s < kTileCh / 16; ++s) {
                const int kk = s * 16 + 8 * (lane >> 5);
                const bf16x8_t av = __builtin_bit_cast(bf16x8_t, *(const uint4*)(sA + pix * kTileLds + kk));
                const bf16x8_t b0 =
                    __builtin_bit_cast(bf16x8_t, *(const uint4*)(sB + (t * BN + (lane & 31)) * kTileLds + kk));
                acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, b0, acc0, 0, 0, 0);
                if constexpr (NB == 2) {
                    const bf16x8_t b1 = __builtin_bit_cast(
                        bf16x8_t, *(const uint4*)(sB + (t * BN + 32 + (lane & 31)) * kTileLds + kk));
                    acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, b1, acc1, 0, 0, 0);
                }
            }
        }
    }
    // epilogue: accumulator row i is pixel 32 w + i of the tile.  The wave's
    // 32 pixels lie in one tile row (32 divides TW), so value v of a lane is
    // pixel op0 + 8 (v / 4) + v % 4 of the image: one base address per lane,
    // compile-time pixel offsets scaled by the uniform channel strides.
    const size_t op0 = ((size_t)img * a.Hout + y0 + (32 * w) / TW) * a.Wout + x0 + (32 * w) % TW + 4 * (lane >> 5);
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
        const int j = n0 + 32 * nb + (lane & 31);
        if (j >= a.Nout) continue;
        const float bj = a.bias ? a.bias[j] : 0.f;
        float yv[16];
#pragma unroll
        for (int v = 0; v < 16; ++v) yv[v] = (nb == 0 ? acc0[v] : acc1[v]) + bj;
        if (a.resid) {
            const uint16_t* rp = a.resid + op0 * a.res_cs + a.res_co + j;
            uint16_t rv[16];
#pragma unroll
            for (int v = 0; v < 16; ++v) rv[v] = rp[(size_t)(8 * (v / 4) + v % 4) * a.res_cs];
#pragma unroll
            for (int v = 0; v < 16; ++v) yv[v] += bf2f(rv[v]);
        }
        if (a.relu) {
#pragma unroll
            for (int v = 0; v < 16; ++v) yv[v] = fmaxf(yv[v], 0.f);
        }
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const size_t off = (size_t)(8 * (v / 4) + v % 4) * a.out_cs;
            if constexpr (OUT_F32)
                ((float*)a.out)[(op0 * a.out_cs + a.out_co + j) + off] = yv[v];
            else
                ((uint16_t*)a.out)[(op0 * a.out_cs + a.out_co + j) + off] = f2bf(yv[v]);
        }
    }
}

// ------------------------------------------------------------ weight grad
// dW[tap][ci][co] partials over pixel ranges: grid (ceil(Co/64), ceil(Ci/64), taps * splits).
// Rows of the GEMM are input channels, columns output channels, the reduction
// runs over pixels: output pixels for CONV3/DOWN/CONV1 (input gathered at the
// tap's shift), input pixels for UP (gradient gathered at the tap's parity).
struct WgradArgs {
    const uint16_t* in;    // layer input (bf16), channels [in_co, in_co + Cin) of stride in_cs
    int in_cs, in_co;
    const uint16_t* dout;  // gradient w.r.t. the layer output (bf16), stride dout_cs
    int dout_cs;
    const uint16_t* act;   // layer output for the ReLU mask, or null
    int act_cs, act_co;
    float* part;           // [splits][taps][Ci][Co]
    float* bpart;          // [splits][btaps][Co]: bias-gradient partials (btaps = 4 for UP, else 1)
    int n, Hin, Win, Cin, Hout, Wout, Cout;
    int taps, splits;
    int P;                 // pixels in the reduction
};

constexpr int kWgK = 64;           // pixels per global round trip
constexpr int kWgLds = kWgK + 8;  // padded row (bf16) of the weight-gradient LDS tiles

// Input pixel and output-gradient pixel of reduction index p at this tap;
// false where the input pixel is zero padding.
template <int MODE>
__device__ __forceinline__ bool wgrad_pixels(const WgradArgs& a, int p, int tap, size_t* ipix, size_t* gpix) {
    if constexpr (MODE == UP) {
        const int x = p % a.Win, t1 = p / a.Win, y = t1 % a.Hin, img = t1 / a.Hin;
        *ipix = (size_t)p;
        *gpix = ((size_t)img * a.Hout + 2 * y + tap / 2) * a.Wout + 2 * x + tap % 2;
        return true;
    } else {
        const int x = p % a.Wout, t1 = p / a.Wout, y = t1 % a.Hout, img = t1 / a.Hout;
        int yy = y, xx = x;
        if constexpr (MODE == CONV3) {
            yy = y + tap / 3 - 1;
            xx = x + tap % 3 - 1;
        } else if constexpr (MODE == DOWN) {
            yy = 2 * y + tap / 2;
            xx = 2 * x + tap % 2;
        }
        *ipix = ((size_t)img * a.Hin + yy) * a.Win + xx;
        *gpix = (size_t)p;
        return yy >= 0 && yy < a.Hin && xx >= 0 && xx < a.Win;
    }
}

// Eight input channels (va) and eight masked output-gradient channels (vb) of
// reduction index p (zeros outside the range, the padding and the channels).
template <int MODE, bool VEC>
__device__ __forceinline__ void wgrad_load(const WgradArgs& a, int p, int p_end, int tap, int cia, int cob,
                                           uint16_t* va, uint16_t* vb) {
#pragma unroll
    for (int q = 0; q < 8; ++q) va[q] = vb[q] = 0;
    if (p >= p_end) return;
    size_t ipix, gpix;
    const bool ok = wgrad_pixels<MODE>(a, p, tap, &ipix, &gpix);
    if (VEC && cia + 8 <= a.Cin) {
        if (ok) *(uint4*)va = *(const uint4*)(a.in + ipix * a.in_cs + a.in_co + cia);
    } else {
#pragma unroll
        for (int q = 0; q < 8; ++q)
            if (ok && cia + q < a.Cin) va[q] = a.in[ipix * a.in_cs + a.in_co + cia + q];
    }
    if (VEC && cob + 8 <= a.Cout) {
        *(uint4*)vb = *(const uint4*)(a.dout + gpix * a.dout_cs + cob);
        if (a.act) {
            const uint4 h4 = *(const uint4*)(a.act + gpix * a.act_cs + a.act_co + cob);
            const uint16_t* h = (const uint16_t*)&h4;
#pragma unroll
            for (int q = 0; q < 8; ++q)
                if (h[q] == 0 || (h[q] & 0x8000u)) vb[q] = 0;
        }
    } else {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int co = cob + q;
            if (co < a.Cout) {
                uint16_t g = a.dout[gpix * a.dout_cs + co];
                if (a.act) {
                    const uint16_t h = a.act[gpix * a.act_cs + a.act_co + co];
                    if (h == 0 || (h & 0x8000u)) g = 0;
                }
                vb[q] = g;
            }
        }
    }
}

// VEC: 16-byte loads of 8 channels; needs channel strides and offsets that are
// multiples of 8 (the partial last group of channels falls back to scalar loads).
// Each thread loads two adjacent pixels per round trip, so the transposition
// into the [channel][pixel] LDS tiles writes 32-bit pixel pairs.  The next
// chunk's global loads are issued before the current chunk's MFMAs.
template <int MODE, bool VEC>
__global__ void __launch_bounds__(kGemmThreads) k_conv_wgrad(WgradArgs a) {
    __shared__ __attribute__((aligned(16))) uint16_t sA[64 * kWgLds];  // [ci][pixel]
    __shared__ __attribute__((aligned(16))) uint16_t sB[64 * kWgLds];  // [co][pixel]
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int co0 = blockIdx.x * 64, ci0 = blockIdx.y * 64;
    const int tap = blockIdx.z % a.taps, split = blockIdx.z / a.taps;
    const int per = (a.P + a.splits - 1) / a.splits;
    const int p_begin = split * per, p_end = min(a.P, p_begin + per);
    f32x16_t acc = {};
    const int wr = (w & 1) * 32, wc = (w >> 1) * 32;
    // loader: thread -> (pixels 2 (tid / 8) and 2 (tid / 8) + 1, 8 consecutive channels (tid % 8) * 8)
    const int lp = tid >> 3, lc = (tid & 7) * 8;
    // The bias gradient is the sum of the masked output gradient over the pixels:
    // blocks of the first input-channel tile add up the dout values they load
    // (every tap for UP, whose taps cover disjoint output pixels; tap 0 otherwise).
    const bool do_bias = blockIdx.y == 0 && (MODE == UP || tap == 0);
    float bsum[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    uint16_t va0[8] __attribute__((aligned(16))), vb0[8] __attribute__((aligned(16)));
    uint16_t va1[8] __attribute__((aligned(16))), vb1[8] __attribute__((aligned(16)));
    wgrad_load<MODE, VEC>(a, p_begin + 2 * lp, p_end, tap, ci0 + lc, co0 + lc, va0, vb0);
    wgrad_load<MODE, VEC>(a, p_begin + 2 * lp + 1, p_end, tap, ci0 + lc, co0 + lc, va1, vb1);
    for (int p0 = p_begin; p0 < p_end; p0 += kWgK) {
        if (do_bias) {
#pragma unroll
            for (int q = 0; q < 8; ++q) bsum[q] += bf2f(vb0[q]) + bf2f(vb1[q]);
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            *(uint32_t*)(sA + (lc + q) * kWgLds + 2 * lp) = (uint32_t)va0[q] | ((uint32_t)va1[q] << 16);
            *(uint32_t*)(sB + (lc + q) * kWgLds + 2 * lp) = (uint32_t)vb0[q] | ((uint32_t)vb1[q] << 16);
        }
        __syncthreads();
        if (p0 + kWgK < p_end) {  // uniform over the block
            wgrad_load<MODE, VEC>(a, p0 + kWgK + 2 * lp, p_end, tap, ci0 + lc, co0 + lc, va0, vb0);
            wgrad_load<MODE, VEC>(a, p0 + kWgK + 2 * lp + 1, p_end, tap, ci0 + lc, co0 + lc, va1, vb1);
        }
#pragma unroll
        for (int s = 0; s < kWgK / 16; ++s) {
            const int kk = s * 16 + 8 * (lane >> 5);
            const bf16x8_t av = __builtin_bit_cast(bf16x8_t, *(const uint4*)(sA + (wr + (lane & 31)) * kWgLds + kk));
            const bf16x8_t bv = __builtin_bit_cast(bf16x8_t, *(const uint4*)(sB + (wc + (lane & 31)) * kWgLds + kk));
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc, 0, 0, 0);
        }
    }
    const int j = co0 + wc + (lane & 31);
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int i = ci0 + wr + 8 * (v / 4) + 4 * (lane >> 5) + (v % 4);
        if (i < a.Cin && j < a.Cout)
            a.part[(((size_t)split * a.taps + tap) * a.Cin + i) * a.Cout + j] = acc[v];
    }
    if (do_bias) {
        // sum the 32 pixel-pair rows of each channel in a fixed order
        __shared__ float bred[kGemmThreads * 8];
#pragma unroll
        for (int q = 0; q < 8; ++q) bred[tid * 8 + q] = bsum[q];
        __syncthreads();
        if (tid < 64 && co0 + tid < a.Cout) {
            const int gi = tid >> 3, q = tid & 7;
            float r = 0.f;
            for (int l = 0; l < kGemmThreads / 8; ++l) r += bred[((l << 3) + gi) * 8 + q];
            const int bt = MODE == UP ? tap : 0;
            a.bpart[((size_t)split * (MODE == UP ? 4 : 1) + bt) * a.Cout + co0 + tid] = r;
        }
    }
}

// Weight and bias gradient of a 3x3 convolution, all nine taps per block:
// grid (Cout / (32 NCT), Cin / 32, splits), three waves, wave w owns the taps
// of kernel row dy = w (dx = 0, 1, 2) for a 32-input x 32 NCT-output channel
// tile.  The reduction runs over chunks of 64 output pixels (TR = 64 / TWC
// rows of TWC pixels; chunks [z * per, (z + 1) * per) for grid z).  Per chunk
// the block stages the masked output gradient as [co][pixel] and the TR + 2
// input rows the taps touch as [row][ci][x0 - 8 .. x0 + TWC + 16), once, so
// an input pixel is read once per chunk instead of once per tap.  A lane's
// eight K values of tap (dy, dx) are input columns x + dx - 1 .. + 7: two
// aligned 16-byte LDS reads and one 4-byte read serve all three dx, the
// shifts by one bf16 taken with v_alignbyte.  part [splits][9][Ci][Co]; the
// bias partials bpart [splits][Co] come from the blocks of the first input
// tile.  Needs 16-byte aligned channel groups, Cin % 32 == 0, Cout % (32 NCT)
// == 0, Wout % TWC == 0 and Hout % TR == 0 (stride 1, same size).
constexpr int kWtThreads = 192;

__device__ __forceinline__ uint32_t bf_shift1(uint32_t hi, uint32_t lo) { return __builtin_amdgcn_alignbyte(hi, lo, 2); }

template <int NCT, int TWC>
__global__ void __launch_bounds__(kWtThreads) k_wgrad3_tiled(WgradArgs a, int per) {
    constexpr int TR = 64 / TWC;
    constexpr int XS = TWC + 24;        // sX row (bf16): columns x0 - 8 .. x0 + TWC + 9 used, padded
    constexpr int NCO = 32 * NCT;
    constexpr int GS = 64 + 8;          // sG row (bf16)
    constexpr int NPAIR = TWC / 2 + 2;  // input pixel pairs per row: x0 - 2 .. x0 + TWC + 1
    constexpr int XT = (TR + 2) * NPAIR * 4;
    constexpr int GT = 32 * (NCO / 8);
    constexpr int GPER = (GT + kWtThreads - 1) / kWtThreads;
    __shared__ __attribute__((aligned(16))) uint16_t sX[(TR + 2) * 32 * XS];
    __shared__ __attribute__((aligned(16))) uint16_t sG[NCO * GS];
    __shared__ float bred[GT * 8];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int co0 = blockIdx.x * NCO, ci0 = blockIdx.y * 32;
    const int rows = a.Hout / TR, tiles_x = a.Wout / TWC;
    const int nchunks = a.n * rows * tiles_x;
    const int c_begin = blockIdx.z * per, c_end = min(nchunks, c_begin + per);
    const bool do_bias = blockIdx.y == 0;
    f32x16_t acc[3][NCT];
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int c = 0; c < NCT; ++c) acc[d][c] = f32x16_t{};
    float bsum[GPER][8];
#pragma unroll
    for (int u = 0; u < GPER; ++u)
#pragma unroll
        for (int q = 0; q < 8; ++q) bsum[u][q] = 0.f;
    const uint4 z4 = make_uint4(0, 0, 0, 0);
    constexpr int XPER = (XT + kWtThreads - 1) / kWtThreads;
    // Staging, chosen per variant by measurement: 0 each task loads and writes
    // in turn (one 32-channel output tile, 64-pixel rows); 1 all of a chunk's
    // loads into registers first, then the LDS writes (two tiles, 64-pixel
    // rows); 2 as 1 with the next chunk's loads in flight during the current
    // chunk's MFMAs (two-row chunks).
    constexpr int STYLE = TWC == 32 ? 2 : (NCT == 2 ? 1 : 0);
    uint4 rx[XPER][2], rg[GPER][2], ra[GPER][2];
    auto fetch = [&](int ch) {
        const int img = ch / (rows * tiles_x), rem = ch % (rows * tiles_x);
        const int y0 = (rem / tiles_x) * TR, x0 = (rem % tiles_x) * TWC;
#pragma unroll
        for (int u = 0; u < XPER; ++u) {
            const int t = tid + u * kWtThreads;
            rx[u][0] = rx[u][1] = z4;
            if (t >= XT) continue;
            const int g = t & 3, q = (t >> 2) % NPAIR, r = (t >> 2) / NPAIR;
            const int yy = y0 + r - 1, xx = x0 - 2 + 2 * q;
            if (yy >= 0 && yy < a.Hin) {
                const size_t rowp = ((size_t)img * a.Hin + yy) * a.Win;
                const uint16_t* base = a.in + a.in_co + ci0 + 8 * g;
                if (xx >= 0 && xx < a.Win) rx[u][0] = *(const uint4*)(base + (rowp + xx) * a.in_cs);
                if (xx + 1 >= 0 && xx + 1 < a.Win) rx[u][1] = *(const uint4*)(base + (rowp + xx + 1) * a.in_cs);
            }
        }
#pragma unroll
        for (int u = 0; u < GPER; ++u) {
            const int t = tid + u * kWtThreads;
            rg[u][0] = rg[u][1] = ra[u][0] = ra[u][1] = z4;
            if (t >= GT) continue;
            const int g = t % (NCO / 8), q = t / (NCO / 8);
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const int k = 2 * q + e, ry = k / TWC, xk = k % TWC;
                const size_t gp = ((size_t)img * a.Hout + y0 + ry) * a.Wout + x0 + xk;
                rg[u][e] = *(const uint4*)(a.dout + gp * a.dout_cs + co0 + 8 * g);
                if (a.act) ra[u][e] = *(const uint4*)(a.act + gp * a.act_cs + a.act_co + co0 + 8 * g);
            }
        }
    };
    // staging straight from global memory (no prefetch): each task loads and
    // writes its pieces in turn
    auto stage_direct = [&](int ch) {
        const int img = ch / (rows * tiles_x), rem = ch % (rows * tiles_x);
        const int y0 = (rem / tiles_x) * TR, x0 = (rem % tiles_x) * TWC;
        for (int t = tid; t < XT; t += kWtThreads) {
            const int g = t & 3, q = (t >> 2) % NPAIR, r = (t >> 2) / NPAIR;
            const int yy = y0 + r - 1, xx = x0 - 2 + 2 * q;
            uint4 v0 = z4, v1 = z4;
            if (yy >= 0 && yy < a.Hin) {
                const size_t rowp = ((size_t)img * a.Hin + yy) * a.Win;
                const uint16_t* base = a.in + a.in_co + ci0 + 8 * g;
                if (xx >= 0 && xx < a.Win) v0 = *(const uint4*)(base + (rowp + xx) * a.in_cs);
                if (xx + 1 >= 0 && xx + 1 < a.Win) v1 = *(const uint4*)(base + (rowp + xx + 1) * a.in_cs);
            }
            const uint16_t* e0 = (const uint16_t*)&v0;
            const uint16_t* e1 = (const uint16_t*)&v1;
#pragma unroll
            for (int k = 0; k < 8; ++k)
                *(uint32_t*)(sX + (r * 32 + 8 * g + k) * XS + 6 + 2 * q) = (uint32_t)e0[k] | ((uint32_t)e1[k] << 16);
        }
#pragma unroll
        for (int u = 0; u < GPER; ++u) {
            const int t = tid + u * kWtThreads;
            if (t >= GT) break;
            const int g = t % (NCO / 8), q = t / (NCO / 8);
            uint16_t gv[2][8] __attribute__((aligned(16)));
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const int k = 2 * q + e, ry = k / TWC, xk = k % TWC;
                const size_t gp = ((size_t)img * a.Hout + y0 + ry) * a.Wout + x0 + xk;
                *(uint4*)gv[e] = *(const uint4*)(a.dout + gp * a.dout_cs + co0 + 8 * g);
                if (a.act) {
                    const uint4 h4 = *(const uint4*)(a.act + gp * a.act_cs + a.act_co + co0 + 8 * g);
                    const uint16_t* h = (const uint16_t*)&h4;
#pragma unroll
                    for (int kk = 0; kk < 8; ++kk)
                        if (h[kk] == 0 || (h[kk] & 0x8000u)) gv[e][kk] = 0;
                }
            }
            if (do_bias) {
#pragma unroll
                for (int kk = 0; kk < 8; ++kk) bsum[u][kk] += bf2f(gv[0][kk]) + bf2f(gv[1][kk]);
            }
#pragma unroll
            for (int kk = 0; kk < 8; ++kk)
                *(uint32_t*)(sG + (8 * g + kk) * GS + 2 * q) = (uint32_t)gv[0][kk] | ((uint32_t)gv[1][kk] << 16);
        }
    };
    if constexpr (STYLE == 2) {
        if (c_begin < c_end) fetch(c_begin);
    }
    for (int ch = c_begin; ch < c_end; ++ch) {
        if constexpr (STYLE == 1) fetch(ch);
        __syncthreads();  // the previous chunk's operand reads are done
        if constexpr (STYLE == 0) stage_direct(ch);
#pragma unroll
        for (int u = 0; u < (STYLE ? XPER : 0); ++u) {
            const int t = tid + u * kWtThreads;
            if (t >= XT) continue;
            const int g = t & 3, q = (t >> 2) % NPAIR, r = (t >> 2) / NPAIR;
            const uint16_t* e0 = (const uint16_t*)&rx[u][0];
            const uint16_t* e1 = (const uint16_t*)&rx[u][1];
#pragma unroll
            for (int k = 0; k < 8; ++k)
                *(uint32_t*)(sX + (r * 32 + 8 * g + k) * XS + 6 + 2 * q) = (uint32_t)e0[k] | ((uint32_t)e1[k] << 16);
        }
#pragma unroll
        for (int u = 0; u < (STYLE ? GPER : 0); ++u) {
            const int t = tid + u * kWtThreads;
            if (t >= GT) continue;
            const int g = t % (NCO / 8), q = t / (NCO / 8);
            uint16_t gv[2][8] __attribute__((aligned(16)));
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                *(uint4*)gv[e] = rg[u][e];
                if (a.act) {
                    const uint16_t* h = (const uint16_t*)&ra[u][e];
#pragma unroll
                    for (int kk = 0; kk < 8; ++kk)
                        if (h[kk] == 0 || (h[kk] & 0x8000u)) gv[e][kk] = 0;
                }
            }
            if (do_bias) {
#pragma unroll
                for (int kk = 0; kk < 8; ++kk) bsum[u][kk] += bf2f(gv[0][kk]) + bf2f(gv[1][kk]);
            }
#pragma unroll
            for (int kk = 0; kk < 8; ++kk)
                *(uint32_t*)(sG + (8 * g + kk) * GS + 2 * q) = (uint32_t)gv[0][kk] | ((uint32_t)gv[1][kk] << 16);
        }
        __syncthreads();
        if constexpr (STYLE == 2) {
            if (ch + 1 < c_end) fetch(ch + 1);
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int kb = s * 16 + 8 * (lane >> 5);
            const int ry = kb / TWC, xj = kb % TWC;
            const uint16_t* xr = sX + ((ry + w) * 32 + (lane & 31)) * XS + xj;
            const uint4 E0 = *(const uint4*)xr;
            const uint4 E1 = *(const uint4*)(xr + 8);
            const uint32_t E2 = *(const uint32_t*)(xr + 16);
            const uint4 A0 = make_uint4(bf_shift1(E1.x, E0.w), bf_shift1(E1.y, E1.x), bf_shift1(E1.z, E1.y),
                                        bf_shift1(E1.w, E1.z));
            const uint4 A2 = make_uint4(bf_shift1(E1.y, E1.x), bf_shift1(E1.z, E1.y), bf_shift1(E1.w, E1.z),
                                        bf_shift1(E2, E1.w));
            const bf16x8_t av[3] = {__builtin_bit_cast(bf16x8_t, A0), __builtin_bit_cast(bf16x8_t, E1),
                                    __builtin_bit_cast(bf16x8_t, A2)};
#pragma unroll
            for (int c = 0; c < NCT; ++c) {
                const bf16x8_t bv = __builtin_bit_cast(bf16x8_t, *(const uint4*)(sG + (c * 32 + (lane & 31)) * GS + kb));
#pragma unroll
                for (int d = 0; d < 3; ++d) acc[d][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[d], bv, acc[d][c], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int tap = 3 * w + d;
#pragma unroll
        for (int c = 0; c < NCT; ++c) {
            const int j = co0 + c * 32 + (lane & 31);
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int i = ci0 + 8 * (v / 4) + 4 * (lane >> 5) + (v % 4);
                a.part[(((size_t)blockIdx.z * 9 + tap) * a.Cin + i) * a.Cout + j] = acc[d][c][v];
            }
        }
    }
    if (do_bias) {
        // per output channel, the 32 pixel-pair tasks summed in a fixed order
#pragma unroll
        for (int u = 0; u < GPER; ++u) {
            const int t = tid + u * kWtThreads;
            if (t < GT)
#pragma unroll
                for (int kk = 0; kk < 8; ++kk) bred[t * 8 + kk] = bsum[u][kk];
        }
        __syncthreads();
        if (tid < NCO) {
            const int g = tid / 8, kk = tid % 8;
            float r = 0.f;
            for (int q = 0; q < 32; ++q) r += bred[(q * (NCO / 8) + g) * 8 + kk];
            a.bpart[(size_t)blockIdx.z * a.Cout + co0 + tid] = r;
        }
    }
}

// Weight and bias gradient of the 2x2 stride-2 convolution, all four taps per
// block: grid (Cout / (32 NCT), Cin / 32, splits), four waves, wave w owns tap
// (w / 2, w % 2) for a 32-input x 32 NCT-output channel tile.  The reduction
// runs over chunks of 64 output pixels (TR = 64 / TWC rows of TWC pixels;
// chunks [z * per, (z + 1) * per)).  Every input pixel belongs to one tap, so
// per chunk the block stages each tap's input pixels as [tap][ci][pixel]
// (pixel-contiguous, no halo) and the masked output gradient as [co][pixel]
// once; the gradient and its ReLU mask are read once per chunk instead of
// once per tap.  part [splits][4][Ci][Co], bpart [splits][Co] from the blocks
// of the first input tile.  Needs 16-byte aligned channel groups,
// Cin % 32 == 0, Cout % (32 NCT) == 0, Wout % TWC == 0, Hout % TR == 0.
template <int NCT, int TWC>
__global__ void __launch_bounds__(kGemmThreads) k_wgrad_down_tiled(WgradArgs a, int per) {
    constexpr int TR = 64 / TWC;
    constexpr int XS = 64 + 8, GS = 64 + 8;
    constexpr int NCO = 32 * NCT;
    constexpr int XT = 4 * 32 * 4;        // (tap, pixel pair, channel group) tasks
    constexpr int GT = 32 * (NCO / 8);    // (pixel pair, channel group) tasks
    constexpr int GPER = (GT + kGemmThreads - 1) / kGemmThreads;
    __shared__ __attribute__((aligned(16))) uint16_t sX[4 * 32 * XS];
    __shared__ __attribute__((aligned(16))) uint16_t sG[NCO * GS];
    __shared__ float bred[GT * 8];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int co0 = blockIdx.x * NCO, ci0 = blockIdx.y * 32;
    const int rows = a.Hout / TR, tiles_x = a.Wout / TWC;
    const int nchunks = a.n * rows * tiles_x;
    const int c_begin = blockIdx.z * per, c_end = min(nchunks, c_begin + per);
    const bool do_bias = blockIdx.y == 0;
    f32x16_t acc[NCT];
#pragma unroll
    for (int c = 0; c < NCT; ++c) acc[c] = f32x16_t{};
    float bsum[GPER][8];
#pragma unroll
    for (int u = 0; u < GPER; ++u)
#pragma unroll
        for (int q = 0; q < 8; ++q) bsum[u][q] = 0.f;
    for (int ch = c_begin; ch < c_end; ++ch) {
        const int img = ch / (rows * tiles_x), rem = ch % (rows * tiles_x);
        const int y0 = (rem / tiles_x) * TR, x0 = (rem % tiles_x) * TWC;
        __syncthreads();  // the previous chunk's operand reads are done
        for (int t = tid; t < XT; t += kGemmThreads) {
            const int g = t & 3, q = (t >> 2) & 31, tap = t >> 7;
            const int ry = (2 * q) / TWC, xk = (2 * q) % TWC;
            const int iy = 2 * (y0 + ry) + tap / 2, ix = 2 * (x0 + xk) + tap % 2;
            const uint16_t* base = a.in + (((size_t)img * a.Hin + iy) * a.Win + ix) * a.in_cs + a.in_co + ci0 + 8 * g;
            const uint4 v0 = *(const uint4*)base;
            const uint4 v1 = *(const uint4*)(base + 2 * (size_t)a.in_cs);
            const uint16_t* e0 = (const uint16_t*)&v0;
            const uint16_t* e1 = (const uint16_t*)&v1;
#pragma unroll
            for (int k = 0; k < 8; ++k)
                *(uint32_t*)(sX + (tap * 32 + 8 * g + k) * XS + 2 * q) = (uint32_t)e0[k] | ((uint32_t)e1[k] << 16);
        }
#pragma unroll
        for (int u = 0; u < GPER; ++u) {
            const int t = tid + u * kGemmThreads;
            if (t >= GT) break;
            const int g = t % (NCO / 8), q = t / (NCO / 8);
            uint16_t gv[2][8] __attribute__((aligned(16)));
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const int k = 2 * q + e, ry = k / TWC, xk = k % TWC;
                const size_t gp = ((size_t)img * a.Hout + y0 + ry) * a.Wout + x0 + xk;
                *(uint4*)gv[e] = *(const uint4*)(a.dout + gp * a.dout_cs + co0 + 8 * g);
                if (a.act) {
                    const uint4 h4 = *(const uint4*)(a.act + gp * a.act_cs + a.act_co + co0 + 8 * g);
                    const uint16_t* h = (const uint16_t*)&h4;
#pragma unroll
                    for (int kk = 0; kk < 8; ++kk)
                        if (h[kk] == 0 || (h[kk] & 0x8000u)) gv[e][kk] = 0;
                }
            }
            if (do_bias) {
#pragma unroll
                for (int kk = 0; kk < 8; ++kk) bsum[u][kk] += bf2f(gv[0][kk]) + bf2f(gv[1][kk]);
            }
#pragma unroll
            for (int kk = 0; kk < 8; ++kk)
                *(uint32_t*)(sG + (8 * g + kk) * GS + 2 * q) = (uint32_t)gv[0][kk] | ((uint32_t)gv[1][kk] << 16);
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int kb = s * 16 + 8 * (lane >> 5);
            const bf16x8_t av = __builtin_bit_cast(bf16x8_t, *(const uint4*)(sX + (w * 32 + (lane & 31)) * XS + kb));
#pragma unroll
            for (int c = 0; c < NCT; ++c) {
                const bf16x8_t bv = __builtin_bit_cast(bf16x8_t, *(const uint4*)(sG + (c * 32 + (lane & 31)) * GS + kb));
                acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc[c], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int c = 0; c < NCT; ++c) {
        const int j = co0 + c * 32 + (lane & 31);
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int i = ci0 + 8 * (v / 4) + 4 * (lane >> 5) + (v % 4);
            a.part[(((size_t)blockIdx.z * 4 + w) * a.Cin + i) * a.Cout + j] = acc[c][v];
        }
    }
    if (do_bias) {
#pragma unroll
        for (int u = 0; u < GPER; ++u) {
            const int t = tid + u * kGemmThreads;
            if (t < GT)
#pragma unroll
                for (int kk = 0; kk < 8; ++kk) bred[t * 8 + kk] = bsum[u][kk];
        }
        __syncthreads();
        if (tid < NCO) {
            const int g = tid / 8, kk = tid % 8;
            float r = 0.f;
            for (int q = 0; q < 32; ++q) r += bred[(q * (NCO / 8) + g) * 8 + kk];
            a.bpart[(size_t)blockIdx.z * a.Cout + co0 + tid] = r;
        }
    }
}

// dW = sum over splits (fixed order); grid ceil(taps*Ci*Co / 256).
__global__ void k_wgrad_reduce(const float* __restrict__ part, int splits, size_t count, float* __restrict__ dW) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    float s = 0.f;
    for (int k = 0; k < splits; ++k) s += part[(size_t)k * count + i];
    dW[i] = s;
}

// Weight and bias gradient of a 1x1 convolution to CO output channels (the
// head), unmasked: dW[ci][co] = sum_p x[p][ci] g[p][co], db[co] = sum_p g[p][co].
// Thread t owns input channels 8 (t % G) .. + 7 (G = Cin / 8) and every
// (256 / G)-th pixel of the block's range [z per, (z + 1) per), 16-byte input
// loads; its 8 CO sums (and, for t % G == 0, the CO bias sums) are added
// across the pixel lanes in lane order through LDS.  part [blocks][Cin][CO],
// bpart [blocks][CO].  Needs Cin a multiple of 8 with Cin / 8 dividing 256, and
// 16-byte aligned input channel groups.
template <int CO>
__global__ void __launch_bounds__(256) k_wgrad_head(WgradArgs a, int per) {
    __shared__ float red[256 * 8 * CO];
    __shared__ float bred[256 * CO];
    const int G = a.Cin / 8, lanes = 256 / G;
    const int g = threadIdx.x % G, pl = threadIdx.x / G;
    const int p_begin = blockIdx.x * per, p_end = min(a.P, p_begin + per);
    float acc[8][CO], bs[CO];
#pragma unroll
    for (int c = 0; c < CO; ++c) {
        bs[c] = 0.f;
#pragma unroll
        for (int k = 0; k < 8; ++k) acc[k][c] = 0.f;
    }
#pragma unroll 4
    for (int p = p_begin + pl; p < p_end; p += lanes) {
        const uint4 xv = *(const uint4*)(a.in + (size_t)p * a.in_cs + a.in_co + 8 * g);
        const uint16_t* xs = (const uint16_t*)&xv;
        float gv[CO];
#pragma unroll
        for (int c = 0; c < CO; ++c) gv[c] = bf2f(a.dout[(size_t)p * a.dout_cs + c]);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const float xk = bf2f(xs[k]);
#pragma unroll
            for (int c = 0; c < CO; ++c) acc[k][c] = fmaf(xk, gv[c], acc[k][c]);
        }
#pragma unroll
        for (int c = 0; c < CO; ++c) bs[c] += gv[c];
    }
    // lane pl's sums at red[pl][(8 g + k) CO + c]
#pragma unroll
    for (int k = 0; k < 8; ++k)
#pragma unroll
        for (int c = 0; c < CO; ++c) red[pl * (8 * G * CO) + (8 * g + k) * CO + c] = acc[k][c];
#pragma unroll
    for (int c = 0; c < CO; ++c) bred[threadIdx.x * CO + c] = bs[c];
    __syncthreads();
    for (int o = threadIdx.x; o < a.Cin * CO; o += 256) {
        float r = 0.f;
        for (int l = 0; l < lanes; ++l) r += red[l * (8 * G * CO) + o];
        a.part[(size_t)blockIdx.x * a.Cin * CO + o] = r;
    }
    if (threadIdx.x < CO) {
        float r = 0.f;
        for (int l = 0; l < lanes; ++l) r += bred[(l * G) * CO + threadIdx.x];  // the g == 0 thread of each lane
        a.bpart[(size_t)blockIdx.x * CO + threadIdx.x] = r;
    }
}

// The same sum for many partials: a block owns 64 consecutive outputs; wave w
// adds partials w, w + 4, w + 8, ... of its lane's output in that order (each
// load instruction reads 64 consecutive values of one partial array), and the
// four wave sums are added as (w0 + w1) + (w2 + w3): a fixed order.
// grid ceil(count / 64), block 256.
__global__ void __launch_bounds__(256) k_wgrad_reduce_wide(const float* __restrict__ part, int splits, size_t count,
                                                           float* __restrict__ dW) {
    __shared__ float red[4][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const size_t i = (size_t)blockIdx.x * 64 + lane;
    float s = 0.f;
    if (i < count) {
#pragma unroll 8
        for (int k = w; k < splits; k += 4) s += part[(size_t)k * count + i];
    }
    red[w][lane] = s;
    __syncthreads();
    if (w == 0 && i < count) dW[i] = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
}

// Weight and bias gradient of a 3x3 convolution with one input channel (the
// first layer): thread t owns output channels 8 (t % G) .. + 7 (G = Cout / 8)
// and every (256 / G)-th pixel of the block's range, and accumulates all nine
// taps and the bias; lanes are summed by wave shuffles and then across waves
// in a fixed order.  part [blocks][9][Cout], bpart [blocks][Cout].
// Needs Cout a multiple of 8 dividing 256 / 8, and 16-byte aligned dout rows.
__global__ void __launch_bounds__(256) k_wgrad_c1(WgradArgs a, int per) {
    __shared__ float red[4][10][256];
    const int G = a.Cout / 8;
    const int g = threadIdx.x % G, pl = threadIdx.x / G, lanes = 256 / G;
    const int p0 = blockIdx.x * per, p1 = min(a.P, p0 + per);
    float acc[10][8];
#pragma unroll
    for (int t = 0; t < 10; ++t)
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[t][q] = 0.f;
    for (int p = p0 + pl; p < p1; p += lanes) {
        const uint4 d4 = *(const uint4*)(a.dout + (size_t)p * a.dout_cs + 8 * g);
        uint16_t dv[8] __attribute__((aligned(16)));
        *(uint4*)dv = d4;
        if (a.act) {
            const uint4 h4 = *(const uint4*)(a.act + (size_t)p * a.act_cs + a.act_co + 8 * g);
            const uint16_t* h = (const uint16_t*)&h4;
#pragma unroll
            for (int q = 0; q < 8; ++q)
                if (h[q] == 0 || (h[q] & 0x8000u)) dv[q] = 0;
        }
        float d[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) d[q] = bf2f(dv[q]);
        const int x = p % a.Wout, t1 = p / a.Wout, y = t1 % a.Hout, img = t1 / a.Hout;
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int yy = y + t / 3 - 1, xx = x + t % 3 - 1;
            float v = 0.f;
            if (yy >= 0 && yy < a.Hin && xx >= 0 && xx < a.Win)
                v = bf2f(a.in[(((size_t)img * a.Hin + yy) * a.Win + xx) * a.in_cs + a.in_co]);
#pragma unroll
            for (int q = 0; q < 8; ++q) acc[t][q] += v * d[q];
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[9][q] += d[q];
    }
    // lanes of one wave with the same channel group differ by multiples of G
    // (G a power of two <= 32): butterfly over the higher lane bits
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int t = 0; t < 10; ++t)
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            float v = acc[t][q];
            for (int o = G; o < 64; o <<= 1) v += __shfl_xor(v, o, 64);
            acc[t][q] = v;
        }
    if (lane < G) {
#pragma unroll
        for (int t = 0; t < 10; ++t)
#pragma unroll
            for (int q = 0; q < 8; ++q) red[w][t][lane * 8 + q] = acc[t][q];
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 10 * a.Cout; i += 256) {
        const int t = i / a.Cout, c = i % a.Cout;
        const float r = red[0][t][c] + red[1][t][c] + red[2][t][c] + red[3][t][c];
        if (t < 9)
            a.part[((size_t)blockIdx.x * 9 + t) * a.Cout + c] = r;
        else
            a.bpart[(size_t)blockIdx.x * a.Cout + c] = r;
    }
}



// GEMM-order bf16 weights from float32 W[taps][Ci][Co]:
//   kind 0: Bt[co][tap * Ci + ci] = W[tap][ci][co]            (forward CONV3 / DOWN / CONV1)
//   kind 1: Bt[ci][tap * Co + co] = W[taps - 1 - tap][ci][co] (input gradient of CONV3, flipped)
//   kind 2: Bt[tap][co][ci]       = W[tap][ci][co]            (forward UP)
//   kind 3: Bt[tap][ci][co]       = W[tap][ci][co]            (input gradient of DOWN, as UP)
//   kind 4: Bt[ci][tap * Co + co] = W[tap][ci][co]            (input gradient of UP / CONV1, as DOWN / CONV1)
// Rows are padded with zeros to Kpad.  Every array of a network is packed by
// one launch (a job per array, passed by value): blockIdx.y is the job, the
// blocks along x stride over its elements.
struct PrepJob {
    const float* W;
    uint16_t* Bt;
    unsigned long long total;  // elements of Bt
    int taps, Ci, Co, kind, Kpad, pad_;
};
constexpr int kMaxPrepJobs = 48;
struct PrepJobs {
    PrepJob j[kMaxPrepJobs];
};

__global__ void __launch_bounds__(256) k_prep_weights(const PrepJobs jobs) {
    const PrepJob J = jobs.j[blockIdx.y];
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < J.total; i += (size_t)gridDim.x * blockDim.x) {
        const int k = (int)(i % J.Kpad);
        const size_t row = i / J.Kpad;
        const int taps = J.taps, Ci = J.Ci, Co = J.Co;
        float v = 0.f;
        if (J.kind == 0) {
            const int co = (int)row;
            if (k < taps * Ci) v = J.W[((size_t)(k / Ci) * Ci + k % Ci) * Co + co];
        } else if (J.kind == 1 || J.kind == 4) {
            const int ci = (int)row;
            if (k < taps * Co) {
                const int tap = J.kind == 1 ? taps - 1 - k / Co : k / Co;
                v = J.W[((size_t)tap * Ci + ci) * Co + k % Co];
            }
        } else if (J.kind == 2) {
            const int tap = (int)(row / Co), co = (int)(row % Co);
            if (k < Ci) v = J.W[((size_t)tap * Ci + k) * Co + co];
        } else {
            const int tap = (int)(row / Ci), ci = (int)(row % Ci);
            if (k < Co) v = J.W[((size_t)tap * Ci + ci) * Co + k];
        }
        J.Bt[i] = f2bf(v);
    }
}

}  // namespace mnf
