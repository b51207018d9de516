// Warm-start network: host driver of the BF16 MFMA convolution kernels
// (forward, backward, Adam) and single-layer entry points.
//
// Network (four levels, widths c0..c3): per level two 3x3 convolutions + ReLU,
// 2x2 stride-2 convolutions + ReLU between levels, a 2x2 transposed
// convolution + ReLU from level 3 to level 2 whose output is concatenated
// (first) with the level-2 encoder output, two 3x3 convolutions + ReLU and a
// 1x1 head to 2 channels at 1/4 of the input size.  Parameters are float32,
// per layer W[taps][c_in][c_out] followed by b[c_out], layers in execution
// order.  Activations and gradients are bf16, channels last; the
// concatenation is a shared 2*c2-channel buffer written in place by its two
// producers.
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "common.hpp"
#include "conv_kernels.hpp"

using namespace mnf;

namespace {

struct LayerDesc {
    const char* name;
    int mode;  // ConvMode
    int ci, co;
    int level_in;  // spatial level of the input (size H >> level)
    int level_out;
};

std::vector<LayerDesc> layers_of(const int* w) {
    return {
        {"e0a", CONV3, 1, w[0], 0, 0},       {"e0b", CONV3, w[0], w[0], 0, 0},
        {"d0", DOWN, w[0], w[1], 0, 1},       {"e1a", CONV3, w[1], w[1], 1, 1},
        {"e1b", CONV3, w[1], w[1], 1, 1},     {"d1", DOWN, w[1], w[2], 1, 2},
        {"e2a", CONV3, w[2], w[2], 2, 2},     {"e2b", CONV3, w[2], w[2], 2, 2},
        {"d2", DOWN, w[2], w[3], 2, 3},       {"e3a", CONV3, w[3], w[3], 3, 3},
        {"e3b", CONV3, w[3], w[3], 3, 3},     {"up", UP, w[3], w[2], 3, 2},
        {"u2a", CONV3, 2 * w[2], w[2], 2, 2}, {"u2b", CONV3, w[2], w[2], 2, 2},
        {"head", CONV1, w[2], 2, 2, 2},
    };
}

int taps_of(int mode) { return mode == CONV3 ? 9 : (mode == CONV1 ? 1 : 4); }

int64_t param_count(const int* w) {
    int64_t n = 0;
    for (const auto& L : layers_of(w)) n += (int64_t)taps_of(L.mode) * L.ci * L.co + L.co;
    return n;
}

int check_shape(mnf_ctx* ctx, const mnf_unet_shape* s) {
    if (!s) return set_error(ctx, MNF_EINVAL, "null shape");
    if (s->H < 16 || s->H % 8)
        return set_error(ctx, MNF_EINVAL, "input size %d must be a multiple of 8 and >= 16", s->H);
    for (int l = 0; l < 4; ++l)
        if (s->widths[l] < 8 || s->widths[l] % 8 || s->widths[l] > 256)
            return set_error(ctx, MNF_EINVAL, "width %d must be a multiple of 8 in [8, 256]", s->widths[l]);
    return MNF_OK;
}

inline unsigned g1(size_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }
int round_up(int x, int m) { return (x + m - 1) / m * m; }
// GEMM reduction length padded to the kernel's K chunk.
int kpad_of(int K) { return round_up(K, gemm_bk(K)); }

// A bf16 channels-last tensor view.
struct View {
    uint16_t* p;
    int cs, co;
};

// One forward / input-gradient GEMM launch.
int launch_conv(mnf_ctx* ctx, int mode, bool mask, bool out_f32, const ConvArgs& a, hipStream_t st) {
    if (a.M <= 0 || a.Nout <= 0) return MNF_OK;
    const bool vec = a.Cin % 8 == 0 && a.in_cs % 8 == 0 && a.in_co % 8 == 0 &&
                     (!mask || (a.mask_cs % 8 == 0 && a.mask_co % 8 == 0));
    if (mode == CONV3 && a.Cin == 1 && !mask && !out_f32 && !a.resid && a.Nout % 8 == 0 && a.Nout <= 256 &&
        a.out_cs % 8 == 0 && a.out_co % 8 == 0) {
        // the one-channel first layer: direct, one thread per output pixel
        hipLaunchKernelGGL(k_conv3_c1, dim3(g1((size_t)a.M)), dim3(256), 0, st, a);
        return MNF_OK;
    }
    if (mode == CONV3 && vec && a.Cin % kTileCh == 0 && a.Hin == a.Hout && a.Win == a.Wout) {
        // direct tiled 3x3: 8-wave blocks of 4 x 64 pixels, or 8 x 32 for
        // narrow images (4-wave blocks of half the height where the height
        // does not divide)
        const int TW = a.Wout % 64 == 0 ? 64 : (a.Wout % 32 == 0 && a.Hout % 4 == 0 ? 32 : 0);
        const bool big = TW > 0 && a.Hout % (256 / TW) == 0;
        const int TH = (big ? 256 : 128) / (TW > 0 ? TW : 1);
        const dim3 bt(big ? 512 : kGemmThreads);
#define MNF_TILED(TWv, NBv)                                                                               \
    do {                                                                                                  \
        if (big) {                                                                                        \
            if (mask) hipLaunchKernelGGL((k_conv3_tiled<true, false, TWv, NBv, 8>), gt, bt, 0, st, a);    \
            else if (out_f32) hipLaunchKernelGGL((k_conv3_tiled<false, true, TWv, NBv, 8>), gt, bt, 0, st, a); \
            else hipLaunchKernelGGL((k_conv3_tiled<false, false, TWv, NBv, 8>), gt, bt, 0, st, a);       \
        } else {                                                                                          \
            if (mask) hipLaunchKernelGGL((k_conv3_tiled<true, false, TWv, NBv, 4>), gt, bt, 0, st, a);    \
            else if (out_f32) hipLaunchKernelGGL((k_conv3_tiled<false, true, TWv, NBv, 4>), gt, bt, 0, st, a); \
            else hipLaunchKernelGGL((k_conv3_tiled<false, false, TWv, NBv, 4>), gt, bt, 0, st, a);       \
        }                                                                                                 \
    } while (0)
        if (TW == 64 && a.Hout % TH == 0 && a.Nout <= 32) {  // one 32-channel output tile
            const dim3 gt((unsigned)(a.n * (a.Hout / TH) * (a.Wout / 64)), 1);
            MNF_TILED(64, 1);
            return MNF_OK;
        }
        if (TW == 64 && a.Hout % TH == 0) {
            const dim3 gt((unsigned)(a.n * (a.Hout / TH) * (a.Wout / 64)), g1((size_t)a.Nout, kGemmBN));
            MNF_TILED(64, 2);
            return MNF_OK;
        }
        if (TW == 32 && a.Hout % TH == 0) {
            const dim3 gt((unsigned)(a.n * (a.Hout / TH) * (a.Wout / 32)), g1((size_t)a.Nout, kGemmBN));
            MNF_TILED(32, 2);
            return MNF_OK;
        }
#undef MNF_TILED
    }
    const dim3 grid(g1((size_t)a.M, kGemmBM), g1((size_t)a.Nout, kGemmBN));
#define MNF_CONV_BK(MD, MK, VC, OF)                                                                    \
    if (a.Kpad > 64) hipLaunchKernelGGL((k_conv_gemm<MD, MK, VC, OF, 64>), grid, dim3(kGemmThreads), 0, st, a); \
    else hipLaunchKernelGGL((k_conv_gemm<MD, MK, VC, OF, 32>), grid, dim3(kGemmThreads), 0, st, a);
#define MNF_CONV_CASE(MD)                                                                              \
    if (mode == MD) {                                                                                  \
        if (mask) {                                                                                    \
            if (vec) { MNF_CONV_BK(MD, true, true, false) } else { MNF_CONV_BK(MD, true, false, false) } \
        } else if (out_f32) {                                                                          \
            if (vec) { MNF_CONV_BK(MD, false, true, true) } else { MNF_CONV_BK(MD, false, false, true) } \
        } else {                                                                                       \
            if (vec) { MNF_CONV_BK(MD, false, true, false) } else { MNF_CONV_BK(MD, false, false, false) } \
        }                                                                                              \
    }
    MNF_CONV_CASE(CONV3)
    MNF_CONV_CASE(DOWN)
    MNF_CONV_CASE(UP)
    MNF_CONV_CASE(CONV1)
#undef MNF_CONV_CASE
#undef MNF_CONV_BK
    return MNF_OK;
}

// Rows of the GEMM: output pixels, or for UP four parity groups of input
// pixels each padded to the row tile (a tile never mixes two taps).
void set_rows(ConvArgs& a, int mode) {
    if (mode == UP) {
        a.per_pad = round_up(a.n * a.Hin * a.Win, kGemmBM);
        a.M = 4 * a.per_pad;
    } else {
        a.per_pad = 0;
        a.M = a.n * a.Hout * a.Wout;
    }
}

// Forward GEMM of one layer: in (dims Hin) -> out (dims Hout).
ConvArgs fwd_args(int mode, View in, int n, int Hin, int Ci, const uint16_t* Bt, const float* bias, void* out,
                  int out_cs, int out_co, int Co, bool relu) {
    ConvArgs a{};
    a.in = in.p;
    a.in_cs = in.cs;
    a.in_co = in.co;
    a.Bt = Bt;
    a.bias = bias;
    a.out = out;
    a.out_cs = out_cs;
    a.out_co = out_co;
    a.n = n;
    a.Hin = a.Win = Hin;
    a.Cin = Ci;
    a.Hout = a.Wout = mode == DOWN ? Hin / 2 : (mode == UP ? Hin * 2 : Hin);
    a.Nout = Co;
    a.relu = relu ? 1 : 0;
    set_rows(a, mode);
    a.Kpad = kpad_of(taps_of(mode) * Ci);
    if (mode == UP) a.Kpad = kpad_of(Ci);
    return a;
}

// Input-gradient GEMM: dY (dims of the layer output) -> dX (dims of the input).
// The dual kind of each layer reads dY as its input.
int dgrad_mode(int mode) { return mode == DOWN ? UP : (mode == UP ? DOWN : mode); }

ConvArgs dgrad_args(int mode, View dY, View act, bool mask, int n, int Hout, int Co, const uint16_t* Bd, View resid,
                    void* dX, int dx_cs, int dx_co, int Ci) {
    const int dm = dgrad_mode(mode);
    ConvArgs a{};
    a.in = dY.p;
    a.in_cs = dY.cs;
    a.in_co = dY.co;
    if (mask) {
        a.mask = act.p;
        a.mask_cs = act.cs;
        a.mask_co = act.co;
    }
    a.Bt = Bd;
    a.resid = resid.p;
    a.res_cs = resid.cs;
    a.res_co = resid.co;
    a.out = dX;
    a.out_cs = dx_cs;
    a.out_co = dx_co;
    a.n = n;
    a.Hin = a.Win = Hout;
    a.Cin = Co;
    a.Hout = a.Wout = dm == DOWN ? Hout / 2 : (dm == UP ? Hout * 2 : Hout);
    a.Nout = Ci;
    set_rows(a, dm);
    a.Kpad = dm == UP ? kpad_of(Co) : kpad_of(taps_of(dm) * Co);
    return a;
}

// bf16 weights for the forward and input-gradient GEMMs of a layer: its
// packing jobs are appended to `jobs` (Bd may be null).
void layer_prep_jobs(const LayerDesc& L, const float* W, uint16_t* Bf, uint16_t* Bd, std::vector<PrepJob>& jobs) {
    const int taps = taps_of(L.mode);
    int kf, kd, Kf, Kd;
    size_t nf, nd;
    switch (L.mode) {
        case CONV3:
            kf = 0; kd = 1;
            Kf = kpad_of(9 * L.ci); Kd = kpad_of(9 * L.co);
            nf = (size_t)L.co * Kf; nd = (size_t)L.ci * Kd;
            break;
        case DOWN:
            kf = 0; kd = 3;
            Kf = kpad_of(4 * L.ci); Kd = kpad_of(L.co);
            nf = (size_t)L.co * Kf; nd = (size_t)4 * L.ci * Kd;
            break;
        case UP:
            kf = 2; kd = 4;
            Kf = kpad_of(L.ci); Kd = kpad_of(4 * L.co);
            nf = (size_t)4 * L.co * Kf; nd = (size_t)L.ci * Kd;
            break;
        default:
            kf = 0; kd = 4;
            Kf = kpad_of(L.ci); Kd = kpad_of(L.co);
            nf = (size_t)L.co * Kf; nd = (size_t)L.ci * Kd;
            break;
    }
    jobs.push_back(PrepJob{W, Bf, (unsigned long long)nf, taps, L.ci, L.co, kf, Kf, 0});
    if (Bd) jobs.push_back(PrepJob{W, Bd, (unsigned long long)nd, taps, L.ci, L.co, kd, Kd, 0});
}

// One launch packing every job (in groups of kMaxPrepJobs).
int launch_prep(mnf_ctx* ctx, const std::vector<PrepJob>& jobs, hipStream_t st) {
    for (size_t j0 = 0; j0 < jobs.size(); j0 += kMaxPrepJobs) {
        const int n = (int)std::min<size_t>(kMaxPrepJobs, jobs.size() - j0);
        PrepJobs pj{};
        size_t most = 1;
        for (int j = 0; j < n; ++j) {
            pj.j[j] = jobs[j0 + j];
            most = std::max<size_t>(most, jobs[j0 + j].total);
        }
        const unsigned gx = (unsigned)std::min<size_t>(256, (most + 255) / 256);
        hipLaunchKernelGGL(k_prep_weights, dim3(gx, n), dim3(256), 0, st, pj);
    }
    MNF_CHECK_LAUNCH(ctx);
    return MNF_OK;
}

int prep_layer_weights(mnf_ctx* ctx, const LayerDesc& L, const float* W, uint16_t* Bf, uint16_t* Bd, hipStream_t st) {
    std::vector<PrepJob> jobs;
    layer_prep_jobs(L, W, Bf, Bd, jobs);
    return launch_prep(ctx, jobs, st);
}

size_t bf_size(const LayerDesc& L) {
    switch (L.mode) {
        case CONV3: return (size_t)L.co * kpad_of(9 * L.ci);
        case DOWN: return (size_t)L.co * kpad_of(4 * L.ci);
        case UP: return (size_t)4 * L.co * kpad_of(L.ci);
        default: return (size_t)L.co * kpad_of(L.ci);
    }
}
size_t bd_size(const LayerDesc& L) {
    switch (L.mode) {
        case CONV3: return (size_t)L.ci * kpad_of(9 * L.co);
        case DOWN: return (size_t)4 * L.ci * kpad_of(L.co);
        case UP: return (size_t)L.ci * kpad_of(4 * L.co);
        default: return (size_t)L.ci * kpad_of(L.co);
    }
}

// Fixed-order sum of `splits` float32 partial arrays of `count` values: one
// thread per value for few partials, four (one per wave) for many.
void reduce_partials(const float* part, int splits, size_t count, float* out, hipStream_t st) {
    if (splits >= 64)
        hipLaunchKernelGGL(k_wgrad_reduce_wide, dim3(g1(count, 64)), dim3(256), 0, st, part, splits, count, out);
    else
        hipLaunchKernelGGL(k_wgrad_reduce, dim3(g1(count)), dim3(256), 0, st, part, splits, count, out);
}

// Weight and bias gradient of a layer into dW (float32, [taps][ci][co]) and db.
int layer_wgrad(mnf_ctx* ctx, const LayerDesc& L, View x, int n, int Hin, View dY, View act, bool mask, float* dW,
                float* db, hipStream_t st) {
    const int taps = taps_of(L.mode);
    const int Hout = L.mode == DOWN ? Hin / 2 : (L.mode == UP ? Hin * 2 : Hin);
    WgradArgs a{};
    a.in = x.p;
    a.in_cs = x.cs;
    a.in_co = x.co;
    a.dout = dY.p + dY.co;
    a.dout_cs = dY.cs;
    a.act = mask ? act.p : nullptr;
    a.act_cs = act.cs;
    a.act_co = act.co;
    a.n = n;
    a.Hin = a.Win = Hin;
    a.Cin = L.ci;
    a.Hout = a.Wout = Hout;
    a.Cout = L.co;
    a.taps = taps;
    a.P = L.mode == UP ? n * Hin * Hin : n * Hout * Hout;
    const bool vec = x.cs % 8 == 0 && x.co % 8 == 0 && dY.cs % 8 == 0 && dY.co % 8 == 0 &&
                     (!mask || (act.cs % 8 == 0 && act.co % 8 == 0));
    const size_t count = (size_t)taps * L.ci * L.co;
    const int Gc = L.co / 8;
    if (L.mode == CONV3 && L.ci == 1 && L.co % 8 == 0 && (Gc & (Gc - 1)) == 0 && Gc <= 32 &&
        dY.cs % 8 == 0 && dY.co % 8 == 0 && (!mask || (act.cs % 8 == 0 && act.co % 8 == 0))) {
        // first layer: one input channel, all taps and the bias per thread
        const int nb = (int)std::min<long long>(1024, ((long long)a.P + 255) / 256);
        const int per = (a.P + nb - 1) / nb;
        void* part;
        void* bpart;
        MNF_TRY(scratch(ctx, "unet_wpart", (size_t)nb * count * sizeof(float), &part));
        MNF_TRY(scratch(ctx, "unet_bpart", (size_t)nb * L.co * sizeof(float), &bpart));
        a.part = (float*)part;
        a.bpart = (float*)bpart;
        hipLaunchKernelGGL(k_wgrad_c1, dim3(nb), dim3(256), 0, st, a, per);
        reduce_partials((const float*)part, nb, count, dW, st);
        reduce_partials((const float*)bpart, nb, (size_t)L.co, db, st);
        return MNF_OK;
    }
    const int target_blocks = 1024;
    // 3x3 layers with 32-channel tiles: all nine taps per block from LDS-staged rows
    const int twc = Hout % 64 == 0 ? 64 : (Hout % 32 == 0 && Hout % 2 == 0 ? 32 : 0);
    if (L.mode == CONV3 && vec && L.ci % 32 == 0 && L.co % 32 == 0 && twc) {
        const int nct = L.co % 64 == 0 ? 2 : 1;
        const int gxy = (L.co / (32 * nct)) * (L.ci / 32);
        const int nchunks = n * Hout * Hout / 64;
        // 64-channel output tiles: two resident blocks per CU on 256 CUs (fewer
        // splits also shrink the partials); 32-channel tiles run lighter blocks
        int splits = std::max(1, std::min((nct == 2 ? 512 : 1024) / gxy, nchunks));
        const int per = (nchunks + splits - 1) / splits;
        splits = (nchunks + per - 1) / per;
        void* part;
        void* bpart;
        MNF_TRY(scratch(ctx, "unet_wpart", (size_t)splits * count * sizeof(float), &part));
        MNF_TRY(scratch(ctx, "unet_bpart", (size_t)splits * L.co * sizeof(float), &bpart));
        a.part = (float*)part;
        a.bpart = (float*)bpart;
        a.splits = splits;
        const dim3 grid((unsigned)(L.co / (32 * nct)), (unsigned)(L.ci / 32), (unsigned)splits);
        if (nct == 2 && twc == 64) hipLaunchKernelGGL((k_wgrad3_tiled<2, 64>), grid, dim3(kWtThreads), 0, st, a, per);
        else if (nct == 2) hipLaunchKernelGGL((k_wgrad3_tiled<2, 32>), grid, dim3(kWtThreads), 0, st, a, per);
        else if (twc == 64) hipLaunchKernelGGL((k_wgrad3_tiled<1, 64>), grid, dim3(kWtThreads), 0, st, a, per);
        else hipLaunchKernelGGL((k_wgrad3_tiled<1, 32>), grid, dim3(kWtThreads), 0, st, a, per);
        reduce_partials((const float*)part, splits, count, dW, st);
        reduce_partials((const float*)bpart, splits, (size_t)L.co, db, st);
        return MNF_OK;
    }
    // 2x2 stride-2 layers with 32-channel tiles: all four taps per block
    const int twd = Hout % 64 == 0 ? 64 : (Hout % 32 == 0 && Hout % 2 == 0 ? 32 : 0);
    if (L.mode == DOWN && vec && L.ci % 32 == 0 && L.co % 32 == 0 && twd) {
        const int nct = L.co % 64 == 0 ? 2 : 1;
        const int gxy = (L.co / (32 * nct)) * (L.ci / 32);
        const int nchunks = n * Hout * Hout / 64;
        int splits = std::max(1, std::min(1024 / gxy, nchunks));
        const int per = (nchunks + splits - 1) / splits;
        splits = (nchunks + per - 1) / per;
        void* part;
        void* bpart;
        MNF_TRY(scratch(ctx, "unet_wpart", (size_t)splits * count * sizeof(float), &part));
        MNF_TRY(scratch(ctx, "unet_bpart", (size_t)splits * L.co * sizeof(float), &bpart));
        a.part = (float*)part;
        a.bpart = (float*)bpart;
        a.splits = splits;
        const dim3 grid((unsigned)(L.co / (32 * nct)), (unsigned)(L.ci / 32), (unsigned)splits);
        if (nct == 2 && twd == 64) hipLaunchKernelGGL((k_wgrad_down_tiled<2, 64>), grid, dim3(kGemmThreads), 0, st, a, per);
        else if (nct == 2) hipLaunchKernelGGL((k_wgrad_down_tiled<2, 32>), grid, dim3(kGemmThreads), 0, st, a, per);
        else if (twd == 64) hipLaunchKernelGGL((k_wgrad_down_tiled<1, 64>), grid, dim3(kGemmThreads), 0, st, a, per);
        else hipLaunchKernelGGL((k_wgrad_down_tiled<1, 32>), grid, dim3(kGemmThreads), 0, st, a, per);
        reduce_partials((const float*)part, splits, count, dW, st);
        reduce_partials((const float*)bpart, splits, (size_t)L.co, db, st);
        return MNF_OK;
    }
    // the 1x1 head to two channels: a streaming reduction over the pixels
    if (L.mode == CONV1 && L.co == 2 && !mask && L.ci % 8 == 0 && 256 % (L.ci / 8) == 0 && x.cs % 8 == 0 &&
        x.co % 8 == 0) {
        const int nb = (int)std::min<long long>(1024, ((long long)a.P + 255) / 256);
        const int per = (a.P + nb - 1) / nb;
        void* part;
        void* bpart;
        MNF_TRY(scratch(ctx, "unet_wpart", (size_t)nb * count * sizeof(float), &part));
        MNF_TRY(scratch(ctx, "unet_bpart", (size_t)nb * L.co * sizeof(float), &bpart));
        a.part = (float*)part;
        a.bpart = (float*)bpart;
        hipLaunchKernelGGL(k_wgrad_head<2>, dim3(nb), dim3(256), 0, st, a, per);
        reduce_partials((const float*)part, nb, count, dW, st);
        reduce_partials((const float*)bpart, nb, (size_t)L.co, db, st);
        return MNF_OK;
    }
    const int tiles = g1((size_t)L.co, 64) * g1((size_t)L.ci, 64) * taps;
    a.splits = std::max(1, std::min(target_blocks / std::max(1, tiles), (a.P + 4095) / 4096));
    const int btaps = L.mode == UP ? 4 : 1;
    void* part;
    void* bpart;
    MNF_TRY(scratch(ctx, "unet_wpart", (size_t)a.splits * count * sizeof(float), &part));
    MNF_TRY(scratch(ctx, "unet_bpart", (size_t)a.splits * btaps * L.co * sizeof(float), &bpart));
    a.part = (float*)part;
    a.bpart = (float*)bpart;
    const dim3 grid(g1((size_t)L.co, 64), g1((size_t)L.ci, 64), taps * a.splits);
#define MNF_WGRAD(M)                                                                              \
    do {                                                                                          \
        if (vec)                                                                                  \
            hipLaunchKernelGGL((k_conv_wgrad<M, true>), grid, dim3(kGemmThreads), 0, st, a);      \
        else                                                                                      \
            hipLaunchKernelGGL((k_conv_wgrad<M, false>), grid, dim3(kGemmThreads), 0, st, a);     \
    } while (0)
    switch (L.mode) {
        case CONV3: MNF_WGRAD(CONV3); break;
        case DOWN: MNF_WGRAD(DOWN); break;
        case UP: MNF_WGRAD(UP); break;
        default: MNF_WGRAD(CONV1); break;
    }
#undef MNF_WGRAD
    reduce_partials((const float*)part, a.splits, count, dW, st);
    // bias: the kernel's per-(split, tap) sums of the masked output gradient
    reduce_partials((const float*)bpart, a.splits * btaps, (size_t)L.co, db, st);
    return MNF_OK;
}

// ---------------------------------------------------------- small kernels

// x = bf16(ln(1 + max(I, 0)) * scale), one channel.
__global__ void k_log_input(const float* __restrict__ I, size_t n, float scale, uint16_t* __restrict__ x) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = f2bf(log1pf(fmaxf(I[i], 0.f)) * scale);
}

// Mean squared error: dOut = 2 (out - target) / count (bf16), per-block float64 partial sums.
__global__ void __launch_bounds__(256)
k_mse(const float* __restrict__ out, const float* __restrict__ target, size_t count, uint16_t* __restrict__ dout,
      double* __restrict__ part) {
    __shared__ double red[4];
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    double e = 0.0;
    if (i < count) {
        const float d = out[i] - target[i];
        e = (double)d * (double)d;
        dout[i] = f2bf(2.f * d / (float)count);
    }
    e = block_sum(e, red);
    if (threadIdx.x == 0) part[blockIdx.x] = e;
}

__global__ void __launch_bounds__(256)
k_sum_scaled(const double* __restrict__ part, size_t n, double scale, double* __restrict__ out) {
    __shared__ double red[4];
    double a = 0.0;
    for (size_t i = threadIdx.x; i < n; i += 256) a += part[i];
    a = block_sum(a, red);
    if (threadIdx.x == 0) *out = a * scale;
}

// Adam (Kingma & Ba 2015) with bias correction; step t >= 1.
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, size_t n, float lr, float b1, float b2, float eps, float c1, float c2) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// --------------------------------------------------------------- network

struct Net {
    std::vector<LayerDesc> L;
    std::vector<size_t> woff;   // parameter offsets (W, then b at woff + taps*ci*co)
    std::vector<View> act;      // output activation of each layer (views into buffers)
    std::vector<View> grad;     // gradient w.r.t. each layer's output
    std::vector<uint16_t*> Bf, Bd;
    View x, cat, dcat;
    float* head_out = nullptr;  // caller's output
    int n, H;
};

int size_at(int H, int level) { return H >> level; }

// Lay out activations, gradients and bf16 weights for batch n.
int build_net(mnf_ctx* ctx, const mnf_unet_shape* s, int n, bool training, Net& net) {
    net.L = layers_of(s->widths);
    net.n = n;
    net.H = s->H;
    size_t off = 0;
    for (const auto& L : net.L) {
        net.woff.push_back(off);
        off += (size_t)taps_of(L.mode) * L.ci * L.co + L.co;
    }
    // activation bytes (bf16)
    const int c2 = s->widths[2];
    auto elems = [&](int level, int c) { return (size_t)n * size_at(s->H, level) * size_at(s->H, level) * c; };
    size_t need = elems(0, 1);
    for (const auto& L : net.L)
        if (std::string(L.name) != "up" && std::string(L.name) != "e2b" && std::string(L.name) != "head")
            need += elems(L.level_out, L.co);
    need += elems(2, 2 * c2);  // concatenation buffer (up | e2b)
    const size_t act_elems = need;
    size_t grad_elems = training ? need + elems(2, 2) : 0;
    size_t wbytes = 0;
    for (const auto& L : net.L) wbytes += bf_size(L) + (training ? bd_size(L) : 0);
    void* buf;
    MNF_TRY(scratch(ctx, training ? "unet_train" : "unet_infer",
                    (act_elems + grad_elems + wbytes) * sizeof(uint16_t) + 1024, &buf));
    uint16_t* p = (uint16_t*)buf;
    net.x = View{p, 1, 0};
    p += elems(0, 1);
    net.cat = View{p, 2 * c2, 0};
    p += elems(2, 2 * c2);
    for (const auto& L : net.L) {
        const std::string nm = L.name;
        if (nm == "up") net.act.push_back(View{net.cat.p, 2 * c2, 0});
        else if (nm == "e2b") net.act.push_back(View{net.cat.p, 2 * c2, c2});
        else if (nm == "head") net.act.push_back(View{nullptr, 2, 0});
        else {
            net.act.push_back(View{p, L.co, 0});
            p += elems(L.level_out, L.co);
        }
    }
    if (training) {
        net.dcat = View{p, 2 * c2, 0};
        p += elems(2, 2 * c2);
        for (const auto& L : net.L) {
            const std::string nm = L.name;
            if (nm == "up") net.grad.push_back(View{net.dcat.p, 2 * c2, 0});
            else {
                net.grad.push_back(View{p, L.co, 0});
                p += elems(L.level_out, L.co);
            }
        }
    }
    for (const auto& L : net.L) {
        net.Bf.push_back(p);
        p += bf_size(L);
        if (training) {
            net.Bd.push_back(p);
            p += bd_size(L);
        } else {
            net.Bd.push_back(nullptr);
        }
    }
    return MNF_OK;
}

int net_forward(mnf_ctx* ctx, Net& net, const float* params, const float* I, float log_scale, float* out,
                hipStream_t st) {
    const size_t nx = (size_t)net.n * net.H * net.H;
    hipLaunchKernelGGL(k_log_input, dim3(g1(nx)), dim3(256), 0, st, I, nx, log_scale, net.x.p);
    std::vector<PrepJob> jobs;
    for (size_t i = 0; i < net.L.size(); ++i) layer_prep_jobs(net.L[i], params + net.woff[i], net.Bf[i], net.Bd[i], jobs);
    MNF_TRY(launch_prep(ctx, jobs, st));
    View in = net.x;
    for (size_t i = 0; i < net.L.size(); ++i) {
        const LayerDesc& L = net.L[i];
        const std::string nm = L.name;
        if (nm == "u2a") in = net.cat;
        const float* W = params + net.woff[i];
        const float* b = W + (size_t)taps_of(L.mode) * L.ci * L.co;
        const int Hin = size_at(net.H, L.level_in);
        const bool head = nm == "head";
        ConvArgs a = fwd_args(L.mode, in, net.n, Hin, L.ci, net.Bf[i], b,
                              head ? (void*)out : (void*)net.act[i].p, head ? 2 : net.act[i].cs,
                              head ? 0 : net.act[i].co, L.co, !head);
        MNF_TRY(launch_conv(ctx, L.mode, false, head, a, st));
        in = net.act[i];
    }
    return MNF_OK;
}

// Backward from dOut (bf16 gradient of the head output) into grads (float32, parameter layout).
int net_backward(mnf_ctx* ctx, Net& net, const float* params, const uint16_t* dout, float* grads, hipStream_t st) {
    const int nl = (int)net.L.size();
    std::vector<View> inputs(nl);
    View prev = net.x;
    for (int i = 0; i < nl; ++i) {
        inputs[i] = std::string(net.L[i].name) == "u2a" ? net.cat : prev;
        prev = net.act[i];
    }
    for (int i = nl - 1; i >= 0; --i) {
        const LayerDesc& L = net.L[i];
        const std::string nm = L.name;
        const bool head = nm == "head";
        const View dY = head ? View{(uint16_t*)dout, 2, 0} : net.grad[i];
        const View act = net.act[i];
        const int Hin = size_at(net.H, L.level_in), Hout = size_at(net.H, L.level_out);
        float* dW = grads + net.woff[i];
        float* db = dW + (size_t)taps_of(L.mode) * L.ci * L.co;
        MNF_TRY(layer_wgrad(ctx, L, inputs[i], net.n, Hin, dY, act, !head, dW, db, st));
        if (i == 0) continue;
        // input gradient into the producer's gradient buffer
        View dst;
        View resid{nullptr, 0, 0};
        if (nm == "u2a") {
            dst = net.dcat;  // up gradient in channels [0, c2), skip gradient in [c2, 2 c2)
        } else {
            dst = net.grad[i - 1];
            if (nm == "d2") resid = View{net.dcat.p, net.dcat.cs, net.act[7].co};  // e2b also feeds the skip
        }
        ConvArgs a = dgrad_args(L.mode, dY, act, !head, net.n, Hout, L.co, net.Bd[i], resid, dst.p, dst.cs, dst.co,
                                L.ci);
        (void)Hin;
        MNF_TRY(launch_conv(ctx, dgrad_mode(L.mode), !head, false, a, st));
    }
    return MNF_OK;
}

}  // namespace

extern "C" {

long long unet_param_count(const mnf_unet_shape* s) { return s ? (long long)param_count(s->widths) : -1; }

int unet_forward(mnf_ctx* ctx, const mnf_unet_shape* s, const float* params, const float* I, float log_scale,
                 int n, float* out, void* stream) {
    MNF_TRY(begin(ctx));
    MNF_TRY(check_shape(ctx, s));
    if (!params || !I || !out || n <= 0) return set_error(ctx, MNF_EINVAL, "null pointer or n <= 0");
    Net net;
    MNF_TRY(build_net(ctx, s, n, false, net));
    MNF_TRY(net_forward(ctx, net, params, I, log_scale, out, (hipStream_t)stream));
    MNF_CHECK_LAUNCH(ctx);
    return MNF_OK;
}

int unet_train_step(mnf_ctx* ctx, const mnf_unet_shape* s, float* params, float* adam_m, float* adam_v, int step,
                    float lr, const float* I, float log_scale, const float* target, int n, double* loss_out,
                    float* grad_out, float* out, void* stream) {
    MNF_TRY(begin(ctx));
    MNF_TRY(check_shape(ctx, s));
    if (!params || !I || !target || n <= 0) return set_error(ctx, MNF_EINVAL, "null pointer or n <= 0");
    const bool update = adam_m && adam_v;
    if (update && step < 1) return set_error(ctx, MNF_EINVAL, "step must be >= 1");
    hipStream_t st = (hipStream_t)stream;
    Net net;
    MNF_TRY(build_net(ctx, s, n, true, net));
    const int Ho = s->H / 4;
    const size_t nout = (size_t)n * Ho * Ho * 2;
    const int64_t np = param_count(s->widths);
    void *obuf, *dbuf, *gbuf, *lpart;
    MNF_TRY(scratch(ctx, "unet_out", nout * sizeof(float), &obuf));
    MNF_TRY(scratch(ctx, "unet_dout", nout * sizeof(uint16_t), &dbuf));
    MNF_TRY(scratch(ctx, "unet_loss", g1(nout) * sizeof(double) + sizeof(double), &lpart));
    float* grads = grad_out;
    if (!grads) {
        MNF_TRY(scratch(ctx, "unet_grads", (size_t)np * sizeof(float), &gbuf));
        grads = (float*)gbuf;
    }
    float* o = out ? out : (float*)obuf;
    MNF_TRY(net_forward(ctx, net, params, I, log_scale, o, st));
    hipLaunchKernelGGL(k_mse, dim3(g1(nout)), dim3(256), 0, st, (const float*)o, target, nout, (uint16_t*)dbuf,
                       (double*)lpart);
    if (loss_out)
        hipLaunchKernelGGL(k_sum_scaled, dim3(1), dim3(256), 0, st, (const double*)lpart, (size_t)g1(nout),
                           1.0 / (double)nout, loss_out);
    MNF_TRY(net_backward(ctx, net, params, (const uint16_t*)dbuf, grads, st));
    if (update) {
        const float b1 = 0.9f, b2 = 0.999f;
        const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
        hipLaunchKernelGGL(k_adam, dim3(g1((size_t)np)), dim3(256), 0, st, params, (const float*)grads, adam_m, adam_v,
                           (size_t)np, lr, b1, b2, 1e-8f, c1, c2);
    }
    MNF_CHECK_LAUNCH(ctx);
    return MNF_OK;
}

int mnf_conv2d(mnf_ctx* ctx, int mode, const uint16_t* x, int n, int H, int Ci, const float* W, const float* b,
               int Co, int relu, float* y, void* stream) {
    MNF_TRY(begin(ctx));
    if (mode < 0 || mode > 3 || !x || !W || !y || n <= 0 || H <= 0 || Ci <= 0 || Co <= 0)
        return set_error(ctx, MNF_EINVAL, "bad convolution arguments");
    if (mode == DOWN && H % 2) return set_error(ctx, MNF_EINVAL, "stride-2 convolution needs an even size");
    hipStream_t st = (hipStream_t)stream;
    LayerDesc L{"t", mode, Ci, Co, 0, 0};
    void* bf;
    MNF_TRY(scratch(ctx, "conv_bf", bf_size(L) * sizeof(uint16_t), &bf));
    MNF_TRY(prep_layer_weights(ctx, L, W, (uint16_t*)bf, nullptr, st));
    ConvArgs a = fwd_args(mode, View{(uint16_t*)x, Ci, 0}, n, H, Ci, (const uint16_t*)bf, b, y, Co, 0, Co, relu != 0);
    MNF_TRY(launch_conv(ctx, mode, false, true, a, st));
    MNF_CHECK_LAUNCH(ctx);
    return MNF_OK;
}

int mnf_conv2d_grad(mnf_ctx* ctx, int mode, const uint16_t* x, int n, int H, int Ci, const float* W, int Co,
                    const uint16_t* dy, const uint16_t* act, uint16_t* dx, float* dW, float* db, void* stream) {
    MNF_TRY(begin(ctx));
    if (mode < 0 || mode > 3 || !x || !W || !dy || n <= 0 || H <= 0 || Ci <= 0 || Co <= 0)
        return set_error(ctx, MNF_EINVAL, "bad convolution arguments");
    hipStream_t st = (hipStream_t)stream;
    LayerDesc L{"t", mode, Ci, Co, 0, 0};
    const int Hout = mode == DOWN ? H / 2 : (mode == UP ? 2 * H : H);
    const View dY{(uint16_t*)dy, Co, 0};
    const View A{(uint16_t*)act, Co, 0};
    if (dW && db) MNF_TRY(layer_wgrad(ctx, L, View{(uint16_t*)x, Ci, 0}, n, H, dY, A, act != nullptr, dW, db, st));
    if (dx) {
        void* bd;
        void* bf;
        MNF_TRY(scratch(ctx, "conv_bd", bd_size(L) * sizeof(uint16_t), &bd));
        MNF_TRY(scratch(ctx, "conv_bf", bf_size(L) * sizeof(uint16_t), &bf));
        MNF_TRY(prep_layer_weights(ctx, L, W, (uint16_t*)bf, (uint16_t*)bd, st));
        ConvArgs a = dgrad_args(mode, dY, A, act != nullptr, n, Hout, Co, (const uint16_t*)bd, View{nullptr, 0, 0}, dx,
                                Ci, 0, Ci);
        MNF_TRY(launch_conv(ctx, dgrad_mode(mode), act != nullptr, false, a, st));
    }
    MNF_CHECK_LAUNCH(ctx);
    return MNF_OK;
}

}  // extern "C"
