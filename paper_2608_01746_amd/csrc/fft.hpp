// Device FFT engine: mixed-radix Stockham transforms of length N executed by
// T = N / V threads that each hold V complex values in registers.
//
// A plan is a sequence of radices R_0 .. R_{S-1} (product N, each dividing V).
// Stage s with span L = R_0 ... R_{s-1} runs V / R_s butterflies per thread;
// butterfly b (b = t + i T) reads positions b + m N / R_s (m < R_s), applies
// the twiddles W_{L R_s}^{(b mod L) m}, an R_s-point DFT in registers, and
// writes output q to position (b - b mod L) R_s + (b mod L) + q L.  This is
// the self-sorting (Stockham) ordering: after the last stage the thread holds
// the transform at positions b + q N / R_{S-1}, in natural frequency order.
// Between stages values are exchanged through LDS.
//
// The inverse plan runs the radices in reverse order, so its first stage
// reads exactly the positions the forward transform leaves in registers and
// a forward / pointwise / inverse sequence needs no exchange in between.
// Transforms are unnormalised: forward kernel exp(-2 pi i k n / N), inverse
// exp(+2 pi i k n / N); the callers apply 1/N per 2D unitary transform.
#pragma once

#include <hip/hip_runtime.h>

namespace mnf {

// ---------------------------------------------------------------- complex

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// Products and squared moduli with the fused multiply-adds written out, so
// that every kernel rounds them the same way (left to the compiler, which
// product of a - b or a + b is fused can differ from kernel to kernel).
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(fmaf(a.x, b.x, -(a.y * b.y)), fmaf(a.x, b.y, a.y * b.x));
}
// conj(a) * b
__device__ __forceinline__ float2 cconjmul(float2 a, float2 b) {
    return make_float2(fmaf(a.x, b.x, a.y * b.y), fmaf(a.x, b.y, -(a.y * b.x)));
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float cabs2(float2 a) { return fmaf(a.x, a.x, a.y * a.y); }
// multiply by -i (forward) or +i (inverse)
template <bool INV>
__device__ __forceinline__ float2 cmul_mi(float2 a) {
    return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// ------------------------------------------------- compile-time trigonometry
// Taylor series in double after reduction to [-pi, pi]; used only to build
// the constant twiddles of the in-register DFTs at compile time.

constexpr double kPi = 3.14159265358979323846264338327950288;

constexpr double ct_reduce(double x) {
    while (x > kPi) x -= 2.0 * kPi;
    while (x < -kPi) x += 2.0 * kPi;
    return x;
}
constexpr double ct_sin(double x) {
    x = ct_reduce(x);
    double term = x, sum = x;
    for (int n = 1; n < 30; ++n) {
        term *= -x * x / ((2.0 * n) * (2.0 * n + 1.0));
        sum += term;
    }
    return sum;
}
constexpr double ct_cos(double x) {
    x = ct_reduce(x);
    double term = 1.0, sum = 1.0;
    for (int n = 1; n < 30; ++n) {
        term *= -x * x / ((2.0 * n - 1.0) * (2.0 * n));
        sum += term;
    }
    return sum;
}

template <int R>
struct ConstTwiddles {
    float c[R];
    float s[R];
    constexpr ConstTwiddles() : c(), s() {
        for (int j = 0; j < R; ++j) {
            double a = 2.0 * kPi * (double)j / (double)R;
            double cv = ct_cos(a), sv = ct_sin(a);
            // snap the exactly representable values
            if (cv < 1e-17 && cv > -1e-17) cv = 0.0;
            if (sv < 1e-17 && sv > -1e-17) sv = 0.0;
            c[j] = (float)cv;
            s[j] = (float)sv;
        }
    }
};

constexpr int first_factor(int R) { return (R % 4 == 0 && R != 8) ? 4 : (R % 2 == 0 ? 2 : 3); }

// ------------------------------------------------------- in-register DFTs
// a[0..R-1] in natural order in, natural order out.

template <int R, bool INV>
struct RegDFT {
    static __device__ __forceinline__ void run(float2* a) {
        constexpr int F = first_factor(R);
        constexpr int S = R / F;
        constexpr ConstTwiddles<R> W{};
        float2 y[R];
        // F-point DFTs over n1 for every n2 (n = S n1 + n2), then twiddle W_R^{n2 k1}
#pragma unroll
        for (int n2 = 0; n2 < S; ++n2) {
            float2 b[F];
#pragma unroll
            for (int n1 = 0; n1 < F; ++n1) b[n1] = a[S * n1 + n2];
            RegDFT<F, INV>::run(b);
#pragma unroll
            for (int k1 = 0; k1 < F; ++k1) {
                const int e = (n2 * k1) % R;
                float2 v = b[k1];
                if (e != 0) {
                    const float c = W.c[e];
                    const float s = INV ? W.s[e] : -W.s[e];
                    v = make_float2(fmaf(v.x, c, -(v.y * s)), fmaf(v.x, s, v.y * c));
                }
                y[n2 * F + k1] = v;
            }
        }
        // S-point DFTs over n2 for every k1; output k = k1 + F k2
#pragma unroll
        for (int k1 = 0; k1 < F; ++k1) {
            float2 c[S];
#pragma unroll
            for (int n2 = 0; n2 < S; ++n2) c[n2] = y[n2 * F + k1];
            RegDFT<S, INV>::run(c);
#pragma unroll
            for (int k2 = 0; k2 < S; ++k2) a[k1 + F * k2] = c[k2];
        }
    }
};

template <bool INV>
struct RegDFT<1, INV> {
    static __device__ __forceinline__ void run(float2*) {}
};

template <bool INV>
struct RegDFT<2, INV> {
    static __device__ __forceinline__ void run(float2* a) {
        float2 t = a[0];
        a[0] = cadd(t, a[1]);
        a[1] = csub(t, a[1]);
    }
};

template <bool INV>
struct RegDFT<3, INV> {
    static __device__ __forceinline__ void run(float2* a) {
        // X0 = a0 + a1 + a2; X1,2 = a0 - (a1 + a2)/2 -/+ i (sqrt3/2)(a1 - a2) (forward)
        const float h = 0.86602540378443864676f;
        float2 s = cadd(a[1], a[2]);
        float2 d = csub(a[1], a[2]);
        float2 m = make_float2(fmaf(-0.5f, s.x, a[0].x), fmaf(-0.5f, s.y, a[0].y));
        float2 r = make_float2(__fmul_rn(h, d.y), -__fmul_rn(h, d.x));  // -i h d (products kept out of the sums)
        if (INV) r = make_float2(-r.x, -r.y);
        a[0] = cadd(a[0], s);
        a[1] = cadd(m, r);
        a[2] = csub(m, r);
    }
};

template <bool INV>
struct RegDFT<4, INV> {
    static __device__ __forceinline__ void run(float2* a) {
        float2 s02 = cadd(a[0], a[2]), d02 = csub(a[0], a[2]);
        float2 s13 = cadd(a[1], a[3]), d13 = cmul_mi<INV>(csub(a[1], a[3]));
        a[0] = cadd(s02, s13);
        a[2] = csub(s02, s13);
        a[1] = cadd(d02, d13);
        a[3] = csub(d02, d13);
    }
};

template <bool INV>
struct RegDFT<8, INV> {
    static __device__ __forceinline__ void run(float2* a) {
        // radix-2 split into two 4-point DFTs of the even and odd samples
        const float r = 0.70710678118654752440f;
        float2 e[4] = {a[0], a[2], a[4], a[6]};
        float2 o[4] = {a[1], a[3], a[5], a[7]};
        RegDFT<4, INV>::run(e);
        RegDFT<4, INV>::run(o);
        // twiddles W_8^k, k = 0..3
        // the products are rounded on their own (never fused into the sums below)
        float2 o1 = INV ? make_float2(__fmul_rn(r, o[1].x - o[1].y), __fmul_rn(r, o[1].x + o[1].y))
                        : make_float2(__fmul_rn(r, o[1].x + o[1].y), __fmul_rn(r, o[1].y - o[1].x));
        float2 o2 = cmul_mi<INV>(o[2]);
        float2 o3 = INV ? make_float2(-__fmul_rn(r, o[3].x + o[3].y), __fmul_rn(r, o[3].x - o[3].y))
                        : make_float2(__fmul_rn(r, o[3].y - o[3].x), -__fmul_rn(r, o[3].x + o[3].y));
        a[0] = cadd(e[0], o[0]);
        a[4] = csub(e[0], o[0]);
        a[1] = cadd(e[1], o1);
        a[5] = csub(e[1], o1);
        a[2] = cadd(e[2], o2);
        a[6] = csub(e[2], o2);
        a[3] = cadd(e[3], o3);
        a[7] = csub(e[3], o3);
    }
};

// ------------------------------------------------------------------ plans

template <int N>
struct Plan;
// V values per thread, T = N / V threads per line, S stages, radices R(s)
template <> struct Plan<16>  { static constexpr int V = 4,  S = 2; __host__ __device__ static constexpr int R(int s) { return 4; } };
template <> struct Plan<32>  { static constexpr int V = 8,  S = 2; __host__ __device__ static constexpr int R(int s) { return s == 0 ? 8 : 4; } };
template <> struct Plan<64>  { static constexpr int V = 8,  S = 2; __host__ __device__ static constexpr int R(int s) { return 8; } };
template <> struct Plan<128> { static constexpr int V = 16, S = 2; __host__ __device__ static constexpr int R(int s) { return s == 0 ? 16 : 8; } };
template <> struct Plan<192> { static constexpr int V = 24, S = 2; __host__ __device__ static constexpr int R(int s) { return s == 0 ? 24 : 8; } };
template <> struct Plan<256> { static constexpr int V = 16, S = 2; __host__ __device__ static constexpr int R(int s) { return 16; } };
template <> struct Plan<384> { static constexpr int V = 24, S = 3; __host__ __device__ static constexpr int R(int s) { return s == 0 ? 24 : 4; } };
template <> struct Plan<512> { static constexpr int V = 32, S = 2; __host__ __device__ static constexpr int R(int s) { return s == 0 ? 32 : 16; } };

template <int N>
struct PlanInfo {
    static constexpr int V = Plan<N>::V;
    static constexpr int T = N / V;
    static constexpr int S = Plan<N>::S;
    // radix of stage s in the direction's order (inverse = reversed)
    __host__ __device__ static constexpr int radix(bool inv, int s) { return inv ? Plan<N>::R(S - 1 - s) : Plan<N>::R(s); }
    __host__ __device__ static constexpr int span(bool inv, int s) {
        int L = 1;
        for (int i = 0; i < s; ++i) L *= radix(inv, i);
        return L;
    }
    // radix of the stage whose outputs stay in registers
    static constexpr int last_fwd = Plan<N>::R(S - 1);
    static constexpr int first_fwd = Plan<N>::R(0);
};

// Position of value x[i*R + m] in the first stage of direction INV:
// t + i T + m N / R.  (The same formula gives the output positions of the
// last stage of the opposite direction.)
template <int N, bool INV>
__device__ __forceinline__ int in_pos(int t, int idx) {
    constexpr int R = PlanInfo<N>::radix(INV, 0);
    constexpr int T = PlanInfo<N>::T;
    return t + (idx / R) * T + (idx % R) * (N / R);
}
template <int N, bool INV>
__device__ __forceinline__ int out_pos(int t, int idx) {
    constexpr int R = PlanInfo<N>::radix(INV, PlanInfo<N>::S - 1);
    constexpr int T = PlanInfo<N>::T;
    return t + (idx / R) * T + (idx % R) * (N / R);
}

// twiddle W_N^e (conjugated for the inverse) from the table tw[n] = exp(-2 pi i n / N)
template <bool INV>
__device__ __forceinline__ float2 tw_get(const float2* tw, int e) {
    float2 w = tw[e];
    return INV ? make_float2(w.x, -w.y) : w;
}

template <int N, bool INV, int s>
__device__ __forceinline__ void stage_compute(float2* x, int t, const float2* tw) {
    constexpr int R = PlanInfo<N>::radix(INV, s);
    constexpr int L = PlanInfo<N>::span(INV, s);
    constexpr int V = PlanInfo<N>::V;
    constexpr int T = PlanInfo<N>::T;
#pragma unroll
    for (int i = 0; i < V / R; ++i) {
        if (L > 1) {
            const int b = t + i * T;
            const int k = b % L;
            constexpr int stride = N / (L * R);
#pragma unroll
            for (int m = 1; m < R; ++m) x[i * R + m] = cmul(x[i * R + m], tw_get<INV>(tw, (k * m * stride) % N));
        }
        RegDFT<R, INV>::run(x + i * R);
    }
}

// Exchange the outputs of stage s through LDS into the inputs of stage s+1.
// ADDR maps a position of this thread's line to an LDS element index.
template <int N, bool INV, int s, class ADDR>
__device__ __forceinline__ void stage_exchange(float2* x, int t, float2* lds, const ADDR& addr) {
    constexpr int R = PlanInfo<N>::radix(INV, s);
    constexpr int L = PlanInfo<N>::span(INV, s);
    constexpr int R2 = PlanInfo<N>::radix(INV, s + 1);
    constexpr int V = PlanInfo<N>::V;
    constexpr int T = PlanInfo<N>::T;
#pragma unroll
    for (int i = 0; i < V / R; ++i) {
        const int b = t + i * T;
        const int k = b % L;
        const int base = (b - k) * R + k;
#pragma unroll
        for (int q = 0; q < R; ++q) lds[addr(base + q * L)] = x[i * R + q];
    }
    ADDR::sync();
#pragma unroll
    for (int i = 0; i < V / R2; ++i) {
        const int b = t + i * T;
#pragma unroll
        for (int m = 0; m < R2; ++m) x[i * R2 + m] = lds[addr(b + m * (N / R2))];
    }
    ADDR::sync();
}

template <int N, bool INV, int s, class ADDR>
struct StageRunner {
    static __device__ __forceinline__ void run(float2* x, int t, float2* lds, const ADDR& addr, const float2* tw) {
        stage_compute<N, INV, s>(x, t, tw);
        if constexpr (s + 1 < PlanInfo<N>::S) {
            stage_exchange<N, INV, s>(x, t, lds, addr);
            StageRunner<N, INV, s + 1, ADDR>::run(x, t, lds, addr, tw);
        }
    }
};

// Full 1D transform of one line.  Every thread that ADDR::sync() waits for
// must call it: the whole block, or the whole wavefront for a wave-local
// layout.
template <int N, bool INV, class ADDR>
__device__ __forceinline__ void fft_line(float2* x, int t, float2* lds, const ADDR& addr, const float2* tw) {
    StageRunner<N, INV, 0, ADDR>::run(x, t, lds, addr, tw);
}

// LDS addressing: one line per row of a row-major block (a pad element every
// 16 keeps stride-16 accesses on distinct banks).
template <int N>
struct RowLds {
    int base;
    static constexpr int stride = N + N / 16;
    __device__ __forceinline__ explicit RowLds(int line) : base(line * stride) {}
    __device__ __forceinline__ int operator()(int p) const { return base + p + (p >> 4); }
    static __device__ __forceinline__ void sync() { __syncthreads(); }
};

// The same layout when each line's threads lie in one wavefront (T divides
// 64 and line = threadIdx.x / T): a line's region of LDS is touched by that
// wavefront only, whose LDS operations take effect in issue order, so a
// stage exchange needs no block barrier, only a point the compiler moves no
// LDS access across.  The wavefronts of a block then run their transforms
// independently, one overlapping its loads with another's arithmetic.
template <int N>
struct RowLdsWave : RowLds<N> {
    static_assert(64 % PlanInfo<N>::T == 0, "a line must not span wavefronts");
    __device__ __forceinline__ explicit RowLdsWave(int line) : RowLds<N>(line) {}
    static __device__ __forceinline__ void sync() {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
};

// LDS addressing: C lines stored interleaved (position-major), line fastest.
template <int C>
struct ColLds {
    int line;
    __device__ __forceinline__ explicit ColLds(int l) : line(l) {}
    __device__ __forceinline__ int operator()(int p) const { return p * C + line; }
    static __device__ __forceinline__ void sync() { __syncthreads(); }
};

}  // namespace mnf
