// Host drivers of the pattern paths: forward model, mini-batched ePIE/rPIE
// iterations and the loss gradient.
#include <algorithm>
#include <vector>

#include "common.hpp"
#include "pattern_kernels.hpp"
#include "update_kernels.hpp"

using namespace mnf;

namespace {

constexpr int kSizes[] = {16, 32, 64, 128, 192, 256, 384, 512};

bool size_supported(int N) {
    for (int s : kSizes)
        if (s == N) return true;
    return false;
}

struct Geometry {
    int My, Mx, Nw, Nd, J;
    int by0, bx0, bh, bw;  // union box of all windows
};

int check_geometry(mnf_ctx* ctx, const void* O, int My, int Mx, const void* P, int Nw, int Nd,
                   const int32_t* pos, int J, Geometry* g) {
    if (!O || !P || !pos) return set_error(ctx, MNF_EINVAL, "null pointer argument");
    if (My <= 0 || Mx <= 0 || Nw <= 0 || Nd <= 0 || J <= 0)
        return set_error(ctx, MNF_EINVAL, "sizes must be positive (My=%d Mx=%d Nw=%d Nd=%d J=%d)",
                         My, Mx, Nw, Nd, J);
    if (!size_supported(Nd))
        return set_error(ctx, MNF_EUNSUPPORTED, "detector size %d has no FFT plan", Nd);
    if (Nw > Nd) return set_error(ctx, MNF_EINVAL, "probe window %d larger than detector %d", Nw, Nd);
    int y0 = My, x0 = Mx, y1 = 0, x1 = 0;
    for (int j = 0; j < J; ++j) {
        const int py = pos[2 * j], px = pos[2 * j + 1];
        if (py < 0 || px < 0 || py + Nw > My || px + Nw > Mx)
            return set_error(ctx, MNF_EINVAL, "window %d at (%d, %d) lies outside the %dx%d object", j,
                             py, px, My, Mx);
        y0 = std::min(y0, py);
        x0 = std::min(x0, px);
        y1 = std::max(y1, py + Nw);
        x1 = std::max(x1, px + Nw);
    }
    *g = Geometry{My, Mx, Nw, Nd, J, y0, x0, y1 - y0, x1 - x0};
    return MNF_OK;
}

// ----------------------------------------------------------------- forward

template <int N>
int forward_n(mnf_ctx* ctx, const Geometry& g, const float2* O, const float2* P, const int* d_pos,
              const int* d_idx, float* I_out, hipStream_t st) {
    using RC = RowCfg<N>;
    using CC = ColCfg<N>;
    const float2* tw;
    MNF_TRY(twiddles(ctx, N, &tw));
    const int chunk = std::min(g.J, 64);
    void* S;
    MNF_TRY(scratch(ctx, "S", (size_t)chunk * N * N * sizeof(float2), &S));
    const int gr = (g.Nw + RC::LINES - 1) / RC::LINES;
    for (int j0 = 0; j0 < g.J; j0 += chunk) {
        const int nb = std::min(chunk, g.J - j0);
        MNF_LAUNCH(ctx, MNF_K_ROWS_FWD, st, k_rows_fwd<N>, dim3(gr, nb), dim3(RC::THREADS), O, g.Mx, P, g.Nw,
                   (const int2*)d_pos + j0, (float2*)S, (float*)nullptr, (float*)nullptr, tw);
        MNF_LAUNCH(ctx, MNF_K_FORWARD, st, k_cols_intensity<N>, dim3(N / CC::C, nb), dim3(CC::THREADS), (const float2*)S, g.Nw, d_idx + j0, I_out, tw);
    }
    MNF_CHECK_LAUNCH(ctx);
    return MNF_OK;
}

// --------------------------------------------------------------- iterate

struct IterArgs {
    float2* O;
    float2* P;
    const float* I;
    const int2* d_bpos;   // window corner of every slot of every iteration's order
    const int* d_order;
    size_t order_stride;  // elements between iterations' rows (0: one shared row)
    int n_iter;
    ptycho_params prm;
    double* err_out;
};

template <int N>
int iterate_n(mnf_ctx* ctx, const Geometry& g, const IterArgs& a, hipStream_t st) {
    using RC = RowCfg<N>;
    using CC = ColCfg<N>;
    using UC = UpdCfg<N>;
    const float2* tw;
    MNF_TRY(twiddles(ctx, N, &tw));
    const int B = a.prm.batch;
    const int gr = (g.Nw + RC::LINES - 1) / RC::LINES;
    const int gc = N / CC::C;
    void *S, *mO, *mP, *errp, *P2, *sA2p, *sA2;
    MNF_TRY(scratch(ctx, "S", (size_t)B * N * N * sizeof(float2), &S));
    MNF_TRY(scratch(ctx, "maxO2", (size_t)B * gr * sizeof(float), &mO));
    MNF_TRY(scratch(ctx, "maxP2", (size_t)gr * sizeof(float), &mP));
    MNF_TRY(scratch(ctx, "errpart", (size_t)g.J * gc * sizeof(double), &errp));
    MNF_TRY(scratch(ctx, "P2old", (size_t)g.Nw * g.Nw * sizeof(float), &P2));
    MNF_TRY(scratch(ctx, "sumA2part", (size_t)g.J * sizeof(double), &sA2p));
    MNF_TRY(scratch(ctx, "sumA2", sizeof(double), &sA2));
    const int rpie = a.prm.alg == 1;

    if (a.err_out) {
        MNF_LAUNCH(ctx, MNF_K_SMALL, st, k_sum_amplitude2, dim3(g.J), dim3(256), a.I, (size_t)N * N, (double*)sA2p);
        MNF_LAUNCH(ctx, MNF_K_SMALL, st, k_sum_f64, dim3(1), dim3(256), (const double*)sA2p, (size_t)g.J, (const double*)nullptr, 1.0, (double*)sA2);
    }
    const dim3 obj_grid((g.bw + kObjTileX - 1) / kObjTileX, (g.bh + kObjTileY - 1) / kObjTileY);
    for (int i = 0; i < a.n_iter; ++i) {
        const int it = a.prm.it0 + i;
        const bool upd_probe = a.prm.update_probe && it >= a.prm.probe_start_iter;
        const int* ord = a.d_order + (size_t)i * a.order_stride;
        const int2* bpi = a.d_bpos + (size_t)i * a.order_stride;
        for (int b0 = 0; b0 < g.J; b0 += B) {
            const int nb = std::min(B, g.J - b0);
            const int* bj = ord + b0;
            const int2* bp = bpi + b0;
            MNF_LAUNCH(ctx, MNF_K_ROWS_FWD, st, k_rows_fwd<N>, dim3(gr, nb), dim3(RC::THREADS), a.O, g.Mx, a.P, g.Nw,
                       bp, (float2*)S, (float*)mO, (float*)mP, tw);
            MNF_LAUNCH(ctx, MNF_K_COLS_MODULUS, st, (k_cols_pointwise<N, ColOp::Modulus>), dim3(gc, nb), dim3(CC::THREADS), (float2*)S, g.Nw, a.I, bj, (double*)errp, 0.f, tw);
            if (upd_probe)
                MNF_LAUNCH(ctx, MNF_K_ROWS_INV, st, (k_rows_inv_update<N, 1>), dim3(g.Nw), dim3(UC::THREADS),
                           (float2*)S, (const float2*)a.O, g.Mx, a.P, (float*)P2, (float2*)nullptr, g.Nw,
                           bp, nb, (const float*)mO, gr, rpie, a.prm.beta, 1.f, tw);
            else
                MNF_LAUNCH(ctx, MNF_K_ROWS_INV, st, (k_rows_inv_update<N, 0>), dim3(g.Nw), dim3(UC::THREADS),
                           (float2*)S, (const float2*)a.O, g.Mx, a.P, (float*)P2, (float2*)nullptr, g.Nw,
                           bp, nb, (const float*)mO, gr, rpie, a.prm.beta, 1.f, tw);
            MNF_LAUNCH(ctx, MNF_K_OBJECT_UPDATE, st, k_object_update, obj_grid, dim3(kObjThreads), a.O, g.Mx,
                       g.by0, g.bx0, g.bh, g.bw, (const float2*)S, N, (const float*)P2, g.Nw, bp, nb,
                       (const float*)mP, gr, rpie, a.prm.alpha);
        }
        if (a.err_out)
            MNF_LAUNCH(ctx, MNF_K_SMALL, st, k_sum_f64, dim3(1), dim3(256), (const double*)errp, (size_t)g.J * gc, (const double*)sA2, 1.0, a.err_out + i);
    }
    MNF_CHECK_LAUNCH(ctx);
    return MNF_OK;
}

// ------------------------------------------------------------------ grad

struct GradArgs {
    const float2* O;
    const float2* P;
    const float* I;
    const int* d_pos;
    const int* d_idx;
    int kind;
    float eps;
    int batch;
    double upstream;
    double* loss_out;
    float2* gO;
    float2* gP;
};

template <int N>
int grad_n(mnf_ctx* ctx, const Geometry& g, const GradArgs& a, hipStream_t st) {
    using RC = RowCfg<N>;
    using CC = ColCfg<N>;
    using UC = UpdCfg<N>;
    const float2* tw;
    MNF_TRY(twiddles(ctx, N, &tw));
    const int B = a.batch;
    const int gr = (g.Nw + RC::LINES - 1) / RC::LINES;
    const int gc = N / CC::C;
    void *S, *lossp;
    MNF_TRY(scratch(ctx, "S", (size_t)B * N * N * sizeof(float2), &S));
    MNF_TRY(scratch(ctx, "losspart", (size_t)g.J * gc * sizeof(double), &lossp));
    if (a.gO)
        MNF_LAUNCH(ctx, MNF_K_SMALL, st, k_zero_c64, dim3((unsigned)(((size_t)g.My * g.Mx + 255) / 256)), dim3(256), a.gO, (size_t)g.My * g.Mx);
    if (a.gP)
        MNF_LAUNCH(ctx, MNF_K_SMALL, st, k_zero_c64, dim3((g.Nw * g.Nw + 255) / 256), dim3(256), a.gP, (size_t)g.Nw * g.Nw);
    const dim3 obj_grid((g.bw + kObjTileX - 1) / kObjTileX, (g.bh + kObjTileY - 1) / kObjTileY);
    const bool need_grad = a.gO || a.gP;
    for (int b0 = 0; b0 < g.J; b0 += B) {
        const int nb = std::min(B, g.J - b0);
        const int* bj = a.d_idx + b0;
        const int2* bp = (const int2*)a.d_pos + b0;
        MNF_LAUNCH(ctx, MNF_K_ROWS_FWD, st, k_rows_fwd<N>, dim3(gr, nb), dim3(RC::THREADS), a.O, g.Mx, a.P, g.Nw,
                   bp, (float2*)S, (float*)nullptr, (float*)nullptr, tw);
        if (a.kind == 0)
            MNF_LAUNCH(ctx, MNF_K_GRAD_COLS, st, (k_cols_pointwise<N, ColOp::PoissonGrad>), dim3(gc, nb), dim3(CC::THREADS), (float2*)S, g.Nw, a.I, bj, (double*)lossp, a.eps, tw);
        else
            MNF_LAUNCH(ctx, MNF_K_GRAD_COLS, st, (k_cols_pointwise<N, ColOp::AmplitudeGrad>), dim3(gc, nb), dim3(CC::THREADS), (float2*)S, g.Nw, a.I, bj, (double*)lossp, a.eps, tw);
        if (!need_grad) continue;
        MNF_LAUNCH(ctx, MNF_K_ROWS_INV, st, (k_rows_inv_update<N, 2>), dim3(g.Nw), dim3(UC::THREADS),
                   (float2*)S, a.O, g.Mx, (float2*)a.P, (float*)nullptr, a.gP, g.Nw, bp, nb,
                   (const float*)nullptr, 0, 0, 0.f, (float)a.upstream, tw);
        if (a.gO)
            MNF_LAUNCH(ctx, MNF_K_GRAD_SCATTER, st, k_grad_object, obj_grid, dim3(kObjThreads), a.gO, g.Mx,
                       g.by0, g.bx0, g.bh, g.bw, (const float2*)S, N, g.Nw, bp, nb);
    }
    if (a.loss_out)
        MNF_LAUNCH(ctx, MNF_K_SMALL, st, k_sum_f64, dim3(1), dim3(256), (const double*)lossp, (size_t)g.J * gc, (const double*)nullptr, 1.0, a.loss_out);
    MNF_CHECK_LAUNCH(ctx);
    return MNF_OK;
}

#define MNF_DISPATCH(N, FN, ...)                     \
    switch (N) {                                     \
        case 16: return FN<16>(__VA_ARGS__);         \
        case 32: return FN<32>(__VA_ARGS__);         \
        case 64: return FN<64>(__VA_ARGS__);         \
        case 128: return FN<128>(__VA_ARGS__);       \
        case 192: return FN<192>(__VA_ARGS__);       \
        case 256: return FN<256>(__VA_ARGS__);       \
        case 384: return FN<384>(__VA_ARGS__);       \
        case 512: return FN<512>(__VA_ARGS__);       \
        default: return MNF_EUNSUPPORTED;            \
    }

int forward_any(mnf_ctx* ctx, const Geometry& g, const float2* O, const float2* P, const int* d_pos,
                const int* d_idx, float* I_out, hipStream_t st) {
    MNF_DISPATCH(g.Nd, forward_n, ctx, g, O, P, d_pos, d_idx, I_out, st)
}
int iterate_any(mnf_ctx* ctx, const Geometry& g, const IterArgs& a, hipStream_t st) {
    MNF_DISPATCH(g.Nd, iterate_n, ctx, g, a, st)
}
int grad_any(mnf_ctx* ctx, const Geometry& g, const GradArgs& a, hipStream_t st) {
    MNF_DISPATCH(g.Nd, grad_n, ctx, g, a, st)
}

int upload_identity(mnf_ctx* ctx, int J, hipStream_t st, void** d) {
    std::vector<int32_t> idx(J);
    for (int j = 0; j < J; ++j) idx[j] = j;
    return upload(ctx, "identity", idx.data(), sizeof(int32_t) * J, st, d);
}

}  // namespace

extern "C" {

int mnf_supported_sizes(int32_t* sizes, int cap) {
    const int n = (int)(sizeof(kSizes) / sizeof(kSizes[0]));
    for (int i = 0; i < n && i < cap && sizes; ++i) sizes[i] = kSizes[i];
    return n;
}

int ptycho_forward(mnf_ctx* ctx, const mnf_c64* O, int My, int Mx, const mnf_c64* P, int Nw, int Nd,
                   const int32_t* pos, int J, float* I_out, void* stream) {
    MNF_TRY(begin(ctx));
    if (!I_out) return set_error(ctx, MNF_EINVAL, "null output");
    Geometry g;
    MNF_TRY(check_geometry(ctx, O, My, Mx, P, Nw, Nd, pos, J, &g));
    hipStream_t st = (hipStream_t)stream;
    void *d_pos, *d_idx;
    MNF_TRY(upload(ctx, "pos", pos, sizeof(int32_t) * 2 * J, st, &d_pos));
    MNF_TRY(upload_identity(ctx, J, st, &d_idx));
    return forward_any(ctx, g, (const float2*)O, (const float2*)P, (const int*)d_pos, (const int*)d_idx,
                       I_out, st);
}

int ptycho_iterate(mnf_ctx* ctx, mnf_c64* O, int My, int Mx, mnf_c64* P, int Nw, const float* I, int Nd,
                   const int32_t* pos, int J, const int32_t* order, int n_iter,
                   const ptycho_params* params, double* err_out, void* stream) {
    MNF_TRY(begin(ctx));
    if (!I || !params) return set_error(ctx, MNF_EINVAL, "null pointer argument");
    if (n_iter < 0) return set_error(ctx, MNF_EINVAL, "n_iter must be >= 0");
    Geometry g;
    MNF_TRY(check_geometry(ctx, O, My, Mx, P, Nw, Nd, pos, J, &g));
    const ptycho_params& p = *params;
    if (p.alg != 0 && p.alg != 1) return set_error(ctx, MNF_EINVAL, "alg must be 0 (ePIE) or 1 (rPIE)");
    if (p.batch < 1 || p.batch > kMaxBatch)
        return set_error(ctx, MNF_EINVAL, "batch %d outside [1, %d]", p.batch, kMaxBatch);
    if (!(p.alpha > 0.f) || !(p.beta > 0.f) || p.alpha > 1.f || p.beta > 1.f)
        return set_error(ctx, MNF_EINVAL, "alpha and beta must lie in (0, 1]");
    if (n_iter == 0) return MNF_OK;
    hipStream_t st = (hipStream_t)stream;
    void *d_pos, *d_order;
    size_t stride = 0;
    if (order) {
        std::vector<char> seen(J);
        for (int i = 0; i < n_iter; ++i) {
            std::fill(seen.begin(), seen.end(), 0);
            for (int k = 0; k < J; ++k) {
                const int v = order[(size_t)i * J + k];
                if (v < 0 || v >= J || seen[v])
                    return set_error(ctx, MNF_EINVAL, "order row %d is not a permutation of 0..%d", i, J - 1);
                seen[v] = 1;
            }
        }
        MNF_TRY(upload(ctx, "order", order, sizeof(int32_t) * (size_t)n_iter * J, st, &d_order));
        std::vector<int32_t> bpos((size_t)n_iter * J * 2);
        for (size_t k = 0; k < (size_t)n_iter * J; ++k) {
            bpos[2 * k] = pos[2 * order[k]];
            bpos[2 * k + 1] = pos[2 * order[k] + 1];
        }
        MNF_TRY(upload(ctx, "bpos", bpos.data(), sizeof(int32_t) * bpos.size(), st, &d_pos));
        stride = J;
    } else {
        MNF_TRY(upload_identity(ctx, J, st, &d_order));
        MNF_TRY(upload(ctx, "pos", pos, sizeof(int32_t) * 2 * J, st, &d_pos));
    }
    IterArgs a{(float2*)O, (float2*)P, I, (const int2*)d_pos, (const int*)d_order, stride, n_iter, p, err_out};
    return iterate_any(ctx, g, a, st);
}

int ptycho_grad(mnf_ctx* ctx, const mnf_c64* O, int My, int Mx, const mnf_c64* P, int Nw, const float* I,
                int Nd, const int32_t* pos, int J, int kind, float eps, int batch, double upstream,
                double* loss_out, mnf_c64* gO, mnf_c64* gP, void* stream) {
    MNF_TRY(begin(ctx));
    if (!I) return set_error(ctx, MNF_EINVAL, "null intensity");
    if (kind != 0 && kind != 1) return set_error(ctx, MNF_EINVAL, "kind must be 0 (Poisson) or 1 (amplitude)");
    if (batch < 1 || batch > kMaxBatch)
        return set_error(ctx, MNF_EINVAL, "batch %d outside [1, %d]", batch, kMaxBatch);
    if (!(eps >= 0.f)) return set_error(ctx, MNF_EINVAL, "eps must be >= 0");
    Geometry g;
    MNF_TRY(check_geometry(ctx, O, My, Mx, P, Nw, Nd, pos, J, &g));
    hipStream_t st = (hipStream_t)stream;
    void *d_pos, *d_idx;
    MNF_TRY(upload(ctx, "pos", pos, sizeof(int32_t) * 2 * J, st, &d_pos));
    MNF_TRY(upload_identity(ctx, J, st, &d_idx));
    GradArgs a{(const float2*)O, (const float2*)P, I, (const int*)d_pos, (const int*)d_idx, kind, eps,
               batch, upstream, loss_out, (float2*)gO, (float2*)gP};
    return grad_any(ctx, g, a, st);
}

}  // extern "C"
