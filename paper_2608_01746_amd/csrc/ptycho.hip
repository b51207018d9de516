// Host drivers of the pattern paths: forward model, mini-batched ePIE/rPIE
// iterations (one scan or many) and the loss gradient.
//
// Every path is planned on the host into descriptor tables (scans, slots,
// groups; see tables.hpp) that are uploaded once per call, then issued as a
// sequence of launches, one per pass.  A reconstruction launch covers the
// current mini-batch of every scan of one detector size.
#include <algorithm>
#include <map>
#include <mutex>
#include <vector>

#include <cmath>

#include "common.hpp"
#include "descent_kernels.hpp"
#include "objrow_kernels.hpp"
#include "pattern_kernels.hpp"
#include "small_kernels.hpp"
#include "shift_kernels.hpp"
#include "update_kernels.hpp"

using namespace mnf;

namespace {

constexpr int kSizes[] = {16, 32, 64, 128, 192, 256, 384, 512};

bool size_supported(int N) {
    for (int s : kSizes)
        if (s == N) return true;
    return false;
}

#define MNF_DISPATCH(N, FN, ...)               \
    switch (N) {                               \
        case 16: return FN<16>(__VA_ARGS__);   \
        case 32: return FN<32>(__VA_ARGS__);   \
        case 64: return FN<64>(__VA_ARGS__);   \
        case 128: return FN<128>(__VA_ARGS__); \
        case 192: return FN<192>(__VA_ARGS__); \
        case 256: return FN<256>(__VA_ARGS__); \
        case 384: return FN<384>(__VA_ARGS__); \
        case 512: return FN<512>(__VA_ARGS__); \
        default: return MNF_EUNSUPPORTED;      \
    }

template <int RV>
int row_lines_v(int N) {
    switch (N) {
        case 16: return RowCfg<16, RV>::LINES;
        case 32: return RowCfg<32, RV>::LINES;
        case 64: return RowCfg<64, RV>::LINES;
        case 128: return RowCfg<128, RV>::LINES;
        case 192: return RowCfg<192, RV>::LINES;
        case 256: return RowCfg<256, RV>::LINES;
        case 384: return RowCfg<384, RV>::LINES;
        default: return RowCfg<512, RV>::LINES;
    }
}
int variant_of(mnf_ctx* ctx, int N) {
    auto it = ctx->variant.find(N);
    return it == ctx->variant.end() ? 0 : it->second;
}
int row_lines(mnf_ctx* ctx, int N) { return (variant_of(ctx, N) & 1) ? row_lines_v<1>(N) : row_lines_v<0>(N); }
// variant bit 2: three launches per mini-batch where the object update can be
// fused with the next mini-batch's exit-wave rows (k_obj_rows)
bool three_launch(mnf_ctx* ctx, int N) { return (variant_of(ctx, N) & 4) != 0; }
// variant bit 3: no single-workgroup run for mini-batches of one (k_small_run)
bool small_run_off(mnf_ctx* ctx, int N) { return (variant_of(ctx, N) & 8) != 0; }

int col_groups(mnf_ctx* ctx, int N) {
    const int c0 = kColGroup < N ? kColGroup : N;
    return N / ((variant_of(ctx, N) & 2) ? c0 / 2 : c0);
}

struct ScanIn {
    float2* O;
    int My, Mx;
    float2* P;
    int Nw;
    const float* I;
    int Nd;
    const int32_t* pos;
    int J;
    const int32_t* order;  // [n_iter][J] or NULL
    double* err_out;
    float2* gO;
    float2* gP;
    const float2* frac = nullptr;  // host [J] (d_y, d_x) fractions of real positions, or NULL
    int modes = 1;                 // probe modes (P holds [modes][Nw][Nw]); each position takes `modes` slots
};

struct Box {
    int y0, x0, h, w;
};

int check_scan(mnf_ctx* ctx, const ScanIn& s, int idx, Box* box) {
    if (!s.O || !s.P || !s.pos || !s.I)
        return set_error(ctx, MNF_EINVAL, "scan %d: null pointer argument", idx);
    if (s.My <= 0 || s.Mx <= 0 || s.Nw <= 0 || s.Nd <= 0 || s.J <= 0)
        return set_error(ctx, MNF_EINVAL, "scan %d: sizes must be positive (My=%d Mx=%d Nw=%d Nd=%d J=%d)", idx,
                         s.My, s.Mx, s.Nw, s.Nd, s.J);
    if (!size_supported(s.Nd))
        return set_error(ctx, MNF_EUNSUPPORTED, "scan %d: detector size %d has no FFT plan", idx, s.Nd);
    if (s.Nw > s.Nd)
        return set_error(ctx, MNF_EINVAL, "scan %d: probe window %d larger than detector %d", idx, s.Nw, s.Nd);
    int y0 = s.My, x0 = s.Mx, y1 = 0, x1 = 0;
    for (int j = 0; j < s.J; ++j) {
        const int py = s.pos[2 * j], px = s.pos[2 * j + 1];
        if (py < 0 || px < 0 || py + s.Nw > s.My || px + s.Nw > s.Mx)
            return set_error(ctx, MNF_EINVAL, "scan %d: window %d at (%d, %d) lies outside the %dx%d object", idx, j,
                             py, px, s.My, s.Mx);
        y0 = std::min(y0, py);
        x0 = std::min(x0, px);
        y1 = std::max(y1, py + s.Nw);
        x1 = std::max(x1, px + s.Nw);
    }
    *box = Box{y0, x0, y1 - y0, x1 - x0};
    return MNF_OK;
}

int check_order(mnf_ctx* ctx, const int32_t* order, int n_iter, int J, int idx) {
    if (!order) return MNF_OK;
    std::vector<char> seen(J);
    for (int i = 0; i < n_iter; ++i) {
        std::fill(seen.begin(), seen.end(), 0);
        for (int k = 0; k < J; ++k) {
            const int v = order[(size_t)i * J + k];
            if (v < 0 || v >= J || seen[v])
                return set_error(ctx, MNF_EINVAL, "scan %d: order row %d is not a permutation of 0..%d", idx, i,
                                 J - 1);
            seen[v] = 1;
        }
    }
    return MNF_OK;
}

// One launch of every pass over a list of slots of one detector size.
struct Launch {
    int N;
    size_t slot_off;
    int nslots;
    size_t group_off;
    int ngroups;
    int tiles;
    int maxNw;
};

// Host side of a planned call.
struct CallPlan {
    std::vector<ScanDev> scans;
    std::vector<SlotDev> slots;
    std::vector<GroupDev> groups;
    std::vector<Launch> launches;     // in issue order
    std::vector<int> iter_end;        // launches[iter_end[i-1] .. iter_end[i]) belong to iteration i
    std::vector<float2> fracs;        // per slot (d_y, d_x) of real positions (sub-pixel plans)
    size_t max_S = 0;                 // bytes of pattern scratch
    size_t max_maxO2 = 0;             // floats of max partials
    int max_slots = 0;                // slots of the largest launch
    bool sub = false;                 // real (sub-pixel) positions: one scan, translated probes
    int modes = 1;                    // probe modes (mixed states): one scan, `modes` slots per position
    void* d_scans = nullptr;
    void* d_slots = nullptr;
    void* d_groups = nullptr;
    void* d_fracs = nullptr;
};

// Per-slot translated probes Pd and probe numerators G ([slot][Nw][Nw]) and
// the probe-update denominators DP ([Nw][Nw], float64) of a sub-pixel call.
struct SubBufs {
    float2* Pd;
    float2* G;
    double* DP;
};

void fill_scan_dev(ScanDev& d, const ScanIn& s, const Box& b, unsigned* status) {
    d = ScanDev{};
    d.O = s.O;
    d.P = s.P;
    d.I = s.I;
    d.gO = s.gO;
    d.gP = s.gP;
    d.status = status;
    d.My = s.My;
    d.Mx = s.Mx;
    d.Nw = s.Nw;
    d.J = s.J;
    d.by0 = b.y0;
    d.bx0 = b.x0;
    d.bh = b.h;
    d.bw = b.w;
    d.tiles_x = (b.w + kObjTileX - 1) / kObjTileX;
}

int tiles_of(const ScanDev& d) { return d.tiles_x * ((d.bh + kObjTileY - 1) / kObjTileY); }

// Slot list of iteration i, round b, for the scans of one size class.
void plan_round(mnf_ctx* ctx, CallPlan& pl, const std::vector<ScanIn>& in, const std::vector<int>& cls, int i,
                int b, int B, int N) {
    Launch L{N, pl.slots.size(), 0, pl.groups.size(), 0, 0, 0};
    for (int k : cls) {
        const ScanIn& s = in[k];
        const int t0 = b * B;
        if (t0 >= s.J) continue;
        const int nb = std::min(B, s.J - t0);
        GroupDev g{k, L.nslots, nb * s.modes, L.tiles};
        for (int t = t0; t < t0 + nb; ++t) {
            const int j = s.order ? s.order[(size_t)i * s.J + t] : t;
            for (int m = 0; m < s.modes; ++m) {
                pl.slots.push_back(SlotDev{k, j, s.pos[2 * j], s.pos[2 * j + 1]});
                pl.fracs.push_back(s.frac ? s.frac[j] : make_float2(0.f, 0.f));
            }
        }
        pl.groups.push_back(g);
        L.nslots += nb * s.modes;
        L.ngroups += 1;
        L.tiles += tiles_of(pl.scans[k]);
        L.maxNw = std::max(L.maxNw, s.Nw);
    }
    if (L.nslots == 0) return;
    pl.max_S = std::max(pl.max_S, (size_t)L.nslots * N * N * sizeof(float2));
    pl.max_slots = std::max(pl.max_slots, L.nslots);
    const int gr = (L.maxNw + row_lines(ctx, N) - 1) / row_lines(ctx, N);
    pl.max_maxO2 = std::max(pl.max_maxO2, (size_t)L.nslots * gr);
    pl.launches.push_back(L);
}

int upload_plan(mnf_ctx* ctx, CallPlan& pl, hipStream_t st) {
    MNF_TRY(upload(ctx, "plan_scans", pl.scans.data(), sizeof(ScanDev) * pl.scans.size(), st, &pl.d_scans));
    MNF_TRY(upload(ctx, "plan_slots", pl.slots.data(), sizeof(SlotDev) * pl.slots.size(), st, &pl.d_slots));
    MNF_TRY(upload(ctx, "plan_groups", pl.groups.data(), sizeof(GroupDev) * std::max<size_t>(1, pl.groups.size()),
                   st, &pl.d_groups));
    if (pl.sub)
        MNF_TRY(upload(ctx, "plan_fracs", pl.fracs.data(), sizeof(float2) * pl.fracs.size(), st, &pl.d_fracs));
    return MNF_OK;
}

// ---------------------------------------------------------- launch helpers

template <int N, int RV, bool SUBX = false>
int launch_rows_fwd(mnf_ctx* ctx, const CallPlan& pl, const Launch& L, const ScanDev* scans, float2* S, float* mO,
                    const float2* Pd, int pmod, const float2* tw, hipStream_t st, const float2* frac = nullptr) {
    const int gr = (L.maxNw + RowCfg<N, RV>::LINES - 1) / RowCfg<N, RV>::LINES;
    MNF_LAUNCH(ctx, MNF_K_ROWS_FWD, st, (k_rows_fwd<N, RV, SUBX>), dim3(gr, L.nslots), dim3(RowCfg<N, RV>::THREADS),
               scans, (const SlotDev*)pl.d_slots + L.slot_off, S, mO, (float2*)Pd, pmod, frac, tw);
    return MNF_OK;
}

constexpr int kOwnProbe = 1 << 30;  // pmod for one probe per slot

// Translated probes of a launch's slots: Pd[s] = S_{d_s}[P] (rows, then columns).
template <int NW>
int shift_probe_n(mnf_ctx* ctx, const float2* P, float2* Pd, const float2* fr, int nslots, hipStream_t st) {
    static_assert(NW % RowCfg<NW, 0>::LINES == 0 && NW % ColCfg<NW, 0>::C == 0, "whole blocks");
    const float2* tw;
    MNF_TRY(twiddles(ctx, NW, &tw));
    MNF_LAUNCH(ctx, MNF_K_SHIFT, st, (k_shift_rows<NW>), dim3(NW / RowCfg<NW, 0>::LINES, nslots),
               dim3(RowCfg<NW, 0>::THREADS), P, (size_t)0, Pd, fr, 1.f, tw);
    MNF_LAUNCH(ctx, MNF_K_SHIFT, st, (k_shift_cols<NW>), dim3(NW / ColCfg<NW, 0>::C, nslots),
               dim3(ColCfg<NW, 0>::THREADS), (const float2*)Pd, (size_t)NW * NW, Pd, fr, 1.f, tw);
    return MNF_OK;
}
int shift_probe(mnf_ctx* ctx, int Nw, const float2* P, float2* Pd, const float2* fr, int nslots, hipStream_t st) {
    MNF_DISPATCH(Nw, shift_probe_n, ctx, P, Pd, fr, nslots, st)
}

// The probe translated along y only, Pd[s] = S_{(d_y, 0)}[P] (one column pass
// from the shared probe); the row pass that reads it adds the x translation.
template <int NW>
int shift_probe_y(mnf_ctx* ctx, const float2* P, float2* Pd, const float2* fr, int nslots, hipStream_t st) {
    const float2* tw;
    MNF_TRY(twiddles(ctx, NW, &tw));
    MNF_LAUNCH(ctx, MNF_K_SHIFT, st, (k_shift_cols<NW>), dim3(NW / ColCfg<NW, 0>::C, nslots),
               dim3(ColCfg<NW, 0>::THREADS), P, (size_t)0, Pd, fr, 1.f, tw);
    return MNF_OK;
}

// Probe update of a sub-pixel launch: G[s] translated back by -d_s in place
// (rows, then columns, every slot in parallel), then summed per group and
// applied to P with DP.
template <int NW>
int shift_update_n(mnf_ctx* ctx, float2* G, const float2* fr, const GroupDev* groups, int nslots, int ngroups,
                   float2* P, const double* DP, hipStream_t st) {
    const float2* tw;
    MNF_TRY(twiddles(ctx, NW, &tw));
    MNF_LAUNCH(ctx, MNF_K_SHIFT, st, (k_shift_rows<NW>), dim3(NW / RowCfg<NW, 0>::LINES, nslots),
               dim3(RowCfg<NW, 0>::THREADS), (const float2*)G, (size_t)NW * NW, G, fr, -1.f, tw);
    MNF_LAUNCH(ctx, MNF_K_SHIFT, st, (k_shift_cols<NW>), dim3(NW / ColCfg<NW, 0>::C, nslots),
               dim3(ColCfg<NW, 0>::THREADS), (const float2*)G, (size_t)NW * NW, G, fr, -1.f, tw);
    MNF_LAUNCH(ctx, MNF_K_PROBE_UPDATE, st, (k_probe_sum_update<NW>), dim3((NW * NW + 255) / 256, ngroups),
               dim3(256), (const float2*)G, groups, P, DP);
    return MNF_OK;
}
int shift_update(mnf_ctx* ctx, int Nw, float2* G, const float2* fr, const GroupDev* groups, int nslots, int ngroups,
                 float2* P, const double* DP, hipStream_t st) {
    MNF_DISPATCH(Nw, shift_update_n, ctx, G, fr, groups, nslots, ngroups, P, DP, st)
}

template <int N, int RV, int CV>
int issue_iterate_launch(mnf_ctx* ctx, const CallPlan& pl, const Launch& L, const ptycho_params& p, bool upd,
                         float2* S, float* mO, hipStream_t st) {
    const float2* tw;
    MNF_TRY(twiddles(ctx, N, &tw));
    const ScanDev* scans = (const ScanDev*)pl.d_scans;
    const SlotDev* slots = (const SlotDev*)pl.d_slots + L.slot_off;
    const GroupDev* groups = (const GroupDev*)pl.d_groups + L.group_off;
    const int gr = (L.maxNw + RowCfg<N, RV>::LINES - 1) / RowCfg<N, RV>::LINES;
    const int rpie = p.alg == 1;
    const float2* nP = nullptr;
    float2* nG = nullptr;
    double* nD = nullptr;
    MNF_TRY((launch_rows_fwd<N, RV>(ctx, pl, L, scans, S, mO, nP, 1, tw, st)));
    MNF_LAUNCH(ctx, MNF_K_COLS_MODULUS, st, (k_cols_pointwise<N, CV, ColOp::Modulus>),
               dim3(N / ColCfg<N, CV>::C, L.nslots), dim3(ColCfg<N, CV>::THREADS), scans, slots, S, 0.f, tw);
    if (upd)
        MNF_LAUNCH(ctx, MNF_K_ROWS_INV, st, (k_rows_inv_update<N, RV, 1>), dim3(L.maxNw, L.ngroups),
                   dim3(UpdCfg<N, RV>::THREADS), scans, slots, groups, S, (const float*)mO, gr, rpie, p.beta, (const double*)nullptr, 1,
                   nP, nG, nD, (const float2*)nullptr, tw);
    else
        MNF_LAUNCH(ctx, MNF_K_ROWS_INV, st, (k_rows_inv_update<N, RV, 0>), dim3(L.maxNw, L.ngroups),
                   dim3(UpdCfg<N, RV>::THREADS), scans, slots, groups, S, (const float*)mO, gr, rpie, p.beta, (const double*)nullptr, 1,
                   nP, nG, nD, (const float2*)nullptr, tw);
    MNF_LAUNCH(ctx, MNF_K_OBJECT_UPDATE, st, k_object_update, dim3(L.tiles), dim3(kObjThreads), scans, slots,
               groups, L.ngroups, (const float2*)S, N, rpie, p.alpha);
    return MNF_OK;
}

// The same mini-batch at real positions (one scan): translated probes, the
// three pattern passes with per-slot probes, the object update and, when the
// probe is updated, the inverse translation of its numerators.
template <int N, int RV, int CV>
int issue_subpixel_launch(mnf_ctx* ctx, const CallPlan& pl, const Launch& L, const ptycho_params& p, bool upd,
                          float2* S, float* mO, const SubBufs& sb, hipStream_t st) {
    const float2* tw;
    MNF_TRY(twiddles(ctx, N, &tw));
    const ScanDev* scans = (const ScanDev*)pl.d_scans;
    const SlotDev* slots = (const SlotDev*)pl.d_slots + L.slot_off;
    const GroupDev* groups = (const GroupDev*)pl.d_groups + L.group_off;
    const float2* fr = (const float2*)pl.d_fracs + L.slot_off;
    const int Nw = pl.scans[0].Nw;
    const int gr = (L.maxNw + RowCfg<N, RV>::LINES - 1) / RowCfg<N, RV>::LINES;
    const int rpie = p.alg == 1;
    const float2* Pd = sb.Pd;
    // Nw == N: the x translations run inside the row passes (forward probe
    // rows in the exit-wave pass, probe numerators in the inverse-row pass)
    const bool fused = Nw == N;
    if (fused) {
        MNF_TRY(shift_probe_y<N>(ctx, pl.scans[0].P, sb.Pd, fr, L.nslots, st));
        MNF_TRY((launch_rows_fwd<N, RV, true>(ctx, pl, L, scans, S, mO, Pd, kOwnProbe, tw, st, fr)));
    } else {
        MNF_TRY(shift_probe(ctx, Nw, pl.scans[0].P, sb.Pd, fr, L.nslots, st));
        MNF_TRY((launch_rows_fwd<N, RV>(ctx, pl, L, scans, S, mO, Pd, kOwnProbe, tw, st)));
    }
    MNF_LAUNCH(ctx, MNF_K_COLS_MODULUS, st, (k_cols_pointwise<N, CV, ColOp::Modulus>),
               dim3(N / ColCfg<N, CV>::C, L.nslots), dim3(ColCfg<N, CV>::THREADS), scans, slots, S, 0.f, tw);
    // With the probe updated, each round of the inverse row pass also runs the
    // numerators' translation, so full-height row blocks are used whenever
    // half-height ones would need more rounds (one scan: the group is the
    // launch's slot list).
    const bool full_rows = RV == 1 && L.nslots > UpdCfg<N, 1>::ULINES;
    if (upd && full_rows)
        MNF_LAUNCH(ctx, MNF_K_ROWS_INV, st, (k_rows_inv_update<N, 0, 4>), dim3(L.maxNw, L.ngroups),
                   dim3(UpdCfg<N, 0>::THREADS), scans, slots, groups, S, (const float*)mO, gr, rpie, p.beta, (const double*)nullptr, 1,
                   Pd, sb.G, sb.DP, fused ? fr : (const float2*)nullptr, tw);
    else if (upd)
        MNF_LAUNCH(ctx, MNF_K_ROWS_INV, st, (k_rows_inv_update<N, RV, 4>), dim3(L.maxNw, L.ngroups),
                   dim3(UpdCfg<N, RV>::THREADS), scans, slots, groups, S, (const float*)mO, gr, rpie, p.beta, (const double*)nullptr, 1,
                   Pd, sb.G, sb.DP, fused ? fr : (const float2*)nullptr, tw);
    else
        MNF_LAUNCH(ctx, MNF_K_ROWS_INV, st, (k_rows_inv_update<N, RV, 3>), dim3(L.maxNw, L.ngroups),
                   dim3(UpdCfg<N, RV>::THREADS), scans, slots, groups, S, (const float*)mO, gr, rpie, p.beta, (const double*)nullptr, 1,
                   Pd, (float2*)nullptr, (double*)nullptr, (const float2*)nullptr, tw);
    MNF_LAUNCH(ctx, MNF_K_OBJECT_UPDATE, st, k_object_update, dim3(L.tiles), dim3(kObjThreads), scans, slots,
               groups, L.ngroups, (const float2*)S, N, rpie, p.alpha);
    if (upd) {
        if (fused) {
            MNF_LAUNCH(ctx, MNF_K_SHIFT, st, (k_shift_cols<N>), dim3(N / ColCfg<N, 0>::C, L.nslots),
                       dim3(ColCfg<N, 0>::THREADS), (const float2*)sb.G, (size_t)N * N, sb.G, fr, -1.f, tw);
            MNF_LAUNCH(ctx, MNF_K_PROBE_UPDATE, st, (k_probe_sum_update<N>), dim3((N * N + 255) / 256, L.ngroups),
                       dim3(256), (const float2*)sb.G, groups, pl.scans[0].P, (const double*)sb.DP);
        } else {
            MNF_TRY(shift_update(ctx, Nw, sb.G, fr, groups, L.nslots, L.ngroups, pl.scans[0].P, sb.DP, st));
        }
    }
    return MNF_OK;
}

// The same mini-batch with probe modes (one scan): slots come in runs of M
// per position; the exit-wave pass reads mode s % M, the column pass projects
// the M modes of a position together, the inverse-row pass updates every
// mode, the object update sums the modes' numerators.
template <int N, int RV, int CV>
int issue_modes_launch(mnf_ctx* ctx, const CallPlan& pl, const Launch& L, const ptycho_params& p, bool upd,
                       float2* S, float* mO, hipStream_t st) {
    const float2* tw;
    MNF_TRY(twiddles(ctx, N, &tw));
    const ScanDev* scans = (const ScanDev*)pl.d_scans;
    const SlotDev* slots = (const SlotDev*)pl.d_slots + L.slot_off;
    const GroupDev* groups = (const GroupDev*)pl.d_groups + L.group_off;
    const int M = pl.modes;
    const int gr = (L.maxNw + RowCfg<N, RV>::LINES - 1) / RowCfg<N, RV>::LINES;
    const int rpie = p.alg == 1;
    const float2* nP = nullptr;
    float2* nG = nullptr;
    double* nD = nullptr;
    MNF_TRY((launch_rows_fwd<N, RV>(ctx, pl, L, scans, S, mO, pl.scans[0].P, M, tw, st)));
    MNF_LAUNCH(ctx, MNF_K_COLS_MODULUS, st, (k_cols_modulus_modes<N, CV>), dim3(N / ColCfg<N, CV>::C, L.nslots / M),
               dim3(ColCfg<N, CV>::THREADS), scans, slots, S, M, tw);
    if (upd)
        MNF_LAUNCH(ctx, MNF_K_ROWS_INV, st, (k_rows_inv_update<N, RV, 6>), dim3(L.maxNw, L.ngroups),
                   dim3(UpdCfg<N, RV>::THREADS), scans, slots, groups, S, (const float*)mO, gr, rpie, p.beta, (const double*)nullptr, M,
                   nP, nG, nD, (const float2*)nullptr, tw);
    else
        MNF_LAUNCH(ctx, MNF_K_ROWS_INV, st, (k_rows_inv_update<N, RV, 5>), dim3(L.maxNw, L.ngroups),
                   dim3(UpdCfg<N, RV>::THREADS), scans, slots, groups, S, (const float*)mO, gr, rpie, p.beta, (const double*)nullptr, M,
                   nP, nG, nD, (const float2*)nullptr, tw);
    MNF_LAUNCH(ctx, MNF_K_OBJECT_UPDATE, st, k_object_update, dim3(L.tiles), dim3(kObjThreads), scans, slots,
               groups, L.ngroups, (const float2*)S, N, rpie, p.alpha);
    return MNF_OK;
}

template <int N>
int issue_iterate_n(mnf_ctx* ctx, const CallPlan& pl, const Launch& L, const ptycho_params& p, bool upd, float2* S,
                    float* mO, const SubBufs* sb, hipStream_t st) {
    if (pl.modes > 1) {
        switch (variant_of(ctx, N) & 3) {
            case 1: return issue_modes_launch<N, 1, 0>(ctx, pl, L, p, upd, S, mO, st);
            case 2: return issue_modes_launch<N, 0, 1>(ctx, pl, L, p, upd, S, mO, st);
            case 3: return issue_modes_launch<N, 1, 1>(ctx, pl, L, p, upd, S, mO, st);
            default: return issue_modes_launch<N, 0, 0>(ctx, pl, L, p, upd, S, mO, st);
        }
    }
    if (sb) {
        switch (variant_of(ctx, N) & 3) {
            case 1: return issue_subpixel_launch<N, 1, 0>(ctx, pl, L, p, upd, S, mO, *sb, st);
            case 2: return issue_subpixel_launch<N, 0, 1>(ctx, pl, L, p, upd, S, mO, *sb, st);
            case 3: return issue_subpixel_launch<N, 1, 1>(ctx, pl, L, p, upd, S, mO, *sb, st);
            default: return issue_subpixel_launch<N, 0, 0>(ctx, pl, L, p, upd, S, mO, *sb, st);
        }
    }
    switch (variant_of(ctx, N) & 3) {
        case 1: return issue_iterate_launch<N, 1, 0>(ctx, pl, L, p, upd, S, mO, st);
        case 2: return issue_iterate_launch<N, 0, 1>(ctx, pl, L, p, upd, S, mO, st);
        case 3: return issue_iterate_launch<N, 1, 1>(ctx, pl, L, p, upd, S, mO, st);
        default: return issue_iterate_launch<N, 0, 0>(ctx, pl, L, p, upd, S, mO, st);
    }
}

int issue_iterate_any(mnf_ctx* ctx, const CallPlan& pl, const Launch& L, const ptycho_params& p, bool upd, float2* S,
                      float* mO, const SubBufs* sb, hipStream_t st) {
    MNF_DISPATCH(L.N, issue_iterate_n, ctx, pl, L, p, upd, S, mO, sb, st)
}

// ---- three launches per mini-batch (one scan, integer positions, one mode)
//
// columns + inverse rows of mini-batch L on S (whose rows the previous
// k_obj_rows launch wrote, with one |O|^2 maximum per window row)
template <int N, int RV, int CV>
int issue_cols_inv(mnf_ctx* ctx, const CallPlan& pl, const Launch& L, const ptycho_params& p, bool upd, float2* S,
                   float* mO, hipStream_t st) {
    const float2* tw;
    MNF_TRY(twiddles(ctx, N, &tw));
    const ScanDev* scans = (const ScanDev*)pl.d_scans;
    const SlotDev* slots = (const SlotDev*)pl.d_slots + L.slot_off;
    const GroupDev* groups = (const GroupDev*)pl.d_groups + L.group_off;
    const int nparts = pl.scans[0].Nw;
    const int rpie = p.alg == 1;
    const float2* nP = nullptr;
    float2* nG = nullptr;
    double* nD = nullptr;
    MNF_LAUNCH(ctx, MNF_K_COLS_MODULUS, st, (k_cols_pointwise<N, CV, ColOp::Modulus>),
               dim3(N / ColCfg<N, CV>::C, L.nslots), dim3(ColCfg<N, CV>::THREADS), scans, slots, S, 0.f, tw);
    if (upd)
        MNF_LAUNCH(ctx, MNF_K_ROWS_INV, st, (k_rows_inv_update<N, RV, 1>), dim3(L.maxNw, L.ngroups),
                   dim3(UpdCfg<N, RV>::THREADS), scans, slots, groups, S, (const float*)mO, nparts, rpie, p.beta,
                   (const double*)nullptr, 1, nP, nG, nD, (const float2*)nullptr, tw);
    else
        MNF_LAUNCH(ctx, MNF_K_ROWS_INV, st, (k_rows_inv_update<N, RV, 0>), dim3(L.maxNw, L.ngroups),
                   dim3(UpdCfg<N, RV>::THREADS), scans, slots, groups, S, (const float*)mO, nparts, rpie, p.beta,
                   (const double*)nullptr, 1, nP, nG, nD, (const float2*)nullptr, tw);
    return MNF_OK;
}

template <int N>
int issue_cols_inv_n(mnf_ctx* ctx, const CallPlan& pl, const Launch& L, const ptycho_params& p, bool upd, float2* S,
                     float* mO, hipStream_t st) {
    switch (variant_of(ctx, N) & 3) {
        case 1: return issue_cols_inv<N, 1, 0>(ctx, pl, L, p, upd, S, mO, st);
        case 2: return issue_cols_inv<N, 0, 1>(ctx, pl, L, p, upd, S, mO, st);
        case 3: return issue_cols_inv<N, 1, 1>(ctx, pl, L, p, upd, S, mO, st);
        default: return issue_cols_inv<N, 0, 0>(ctx, pl, L, p, upd, S, mO, st);
    }
}

// object update of mini-batch Lu (from S_u; none for the call's first) and
// exit-wave rows of mini-batch Lf (to S_f; none after the call's last)
template <int N>
int issue_obj_rows_n(mnf_ctx* ctx, const CallPlan& pl, const Launch* Lu, const Launch* Lf, const float2* S_u,
                     float2* S_f, float* mO, const ptycho_params& p, hipStream_t st) {
    const float2* tw;
    MNF_TRY(twiddles(ctx, N, &tw));
    const ScanDev& sc = pl.scans[0];
    const SlotDev* d_slots = (const SlotDev*)pl.d_slots;
    const int kind = Lf ? MNF_K_ROWS_FWD : MNF_K_OBJECT_UPDATE;
    MNF_LAUNCH(ctx, kind, st, k_obj_rows<N>, dim3((unsigned)((sc.bh + kObjRowsPerBlock - 1) / kObjRowsPerBlock)),
               dim3(kObjRowThreads), (const ScanDev*)pl.d_scans, Lu ? d_slots + Lu->slot_off : d_slots,
               Lu ? Lu->nslots : 0, S_u, Lf ? d_slots + Lf->slot_off : d_slots, Lf ? Lf->nslots : 0, S_f, mO,
               p.alg == 1 ? 1 : 0, p.alpha, tw);
    return MNF_OK;
}

int issue_cols_inv_any(mnf_ctx* ctx, const CallPlan& pl, const Launch& L, const ptycho_params& p, bool upd, float2* S,
                       float* mO, hipStream_t st) {
    MNF_DISPATCH(L.N, issue_cols_inv_n, ctx, pl, L, p, upd, S, mO, st)
}

int issue_obj_rows_any(mnf_ctx* ctx, const CallPlan& pl, int N, const Launch* Lu, const Launch* Lf, const float2* S_u,
                       float2* S_f, float* mO, const ptycho_params& p, hipStream_t st) {
    MNF_DISPATCH(N, issue_obj_rows_n, ctx, pl, Lu, Lf, S_u, S_f, mO, p, st)
}

// ----------------------------------------------------------------- iterate

template <int N>
int launch_small_run(mnf_ctx* ctx, const CallPlan& pl, int J, int n_iter, const ptycho_params& p, int upd_from,
                     const double* sumA2, double* err, hipStream_t st) {
    if constexpr (N > kSmallMaxN) {
        return set_error(ctx, MNF_EUNSUPPORTED, "no single-workgroup run at N = %d", N);
    } else {
        const float2* tw;
        MNF_TRY(twiddles(ctx, N, &tw));
        MNF_LAUNCH(ctx, MNF_K_SMALL_RUN, st, k_small_run<N>, dim3(1), dim3(SmallCfg<N>::THREADS), (const ScanDev*)pl.d_scans,
                   (const SlotDev*)pl.d_slots, J, n_iter, p.alg == 1 ? 1 : 0, p.alpha, p.beta, upd_from, sumA2, err, tw);
        return MNF_OK;
    }
}


bool any_err_of(const std::vector<ScanIn>& in) {
    for (const ScanIn& s : in)
        if (s.err_out) return true;
    return false;
}

// At least n streams (default priority, not synchronising with the null
// stream) and n + 1 events on the context, created on first use.
int class_streams(mnf_ctx* ctx, int n) {
    while ((int)ctx->class_streams.size() < n) {
        hipStream_t s;
        MNF_HIP(ctx, hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        ctx->class_streams.push_back(s);
    }
    while ((int)ctx->class_events.size() < n + 1) {
        hipEvent_t e;
        MNF_HIP(ctx, hipEventCreateWithFlags(&e, hipEventDisableTiming));
        ctx->class_events.push_back(e);
    }
    return MNF_OK;
}

// Validation and the host plan of an iterate call: the scan table, the size
// classes and, for n_iter > 0, every launch's slot and group lists.  No
// device work (the scans' device pointers are only copied).
int plan_iterate(mnf_ctx* ctx, const std::vector<ScanIn>& in, int n_iter, const ptycho_params& p, unsigned* status,
                 CallPlan& pl, std::map<int, std::vector<int>>& classes) {
    const int ns = (int)in.size();
    if (ns <= 0) return set_error(ctx, MNF_EINVAL, "no scans");
    if (p.alg != 0 && p.alg != 1) return set_error(ctx, MNF_EINVAL, "alg must be 0 (ePIE) or 1 (rPIE)");
    if (p.batch < 1 || p.batch > kMaxBatch)
        return set_error(ctx, MNF_EINVAL, "batch %d outside [1, %d]", p.batch, kMaxBatch);
    if (!(p.alpha > 0.f) || !(p.beta > 0.f) || p.alpha > 1.f || p.beta > 1.f)
        return set_error(ctx, MNF_EINVAL, "alpha and beta must lie in (0, 1]");
    if (n_iter < 0) return set_error(ctx, MNF_EINVAL, "n_iter must be >= 0");
    pl.scans.resize(ns);
    int max_batches = 0;
    for (int k = 0; k < ns; ++k) {
        Box b;
        MNF_TRY(check_scan(ctx, in[k], k, &b));
        MNF_TRY(check_order(ctx, in[k].order, n_iter, in[k].J, k));
        fill_scan_dev(pl.scans[k], in[k], b, status);
        classes[in[k].Nd].push_back(k);
        max_batches = std::max(max_batches, (in[k].J + p.batch - 1) / p.batch);
    }
    const bool sub = in[0].frac != nullptr;
    if (sub && ns != 1) return set_error(ctx, MNF_EINVAL, "real positions are supported for one scan per call");
    const int modes = in[0].modes;
    if (modes < 1 || modes > kMaxModes)
        return set_error(ctx, MNF_EINVAL, "probe modes %d outside [1, %d]", modes, kMaxModes);
    if (modes > 1 && (ns != 1 || sub))
        return set_error(ctx, MNF_EINVAL, "probe modes are supported for one scan per call at integer positions");
    if ((size_t)p.batch * modes > (size_t)kMaxBatch)
        return set_error(ctx, MNF_EINVAL, "batch x modes = %d exceeds %d", p.batch * modes, kMaxBatch);
    if (sub && !size_supported(in[0].Nw))
        return set_error(ctx, MNF_EUNSUPPORTED, "real positions need a probe window with an FFT plan (Nw=%d)", in[0].Nw);
    pl.sub = sub;
    pl.modes = modes;
    for (int i = 0; i < n_iter; ++i) {
        for (int b = 0; b < max_batches; ++b)
            for (auto& kv : classes) plan_round(ctx, pl, in, kv.second, i, b, p.batch, kv.first);
        pl.iter_end.push_back((int)pl.launches.size());
    }
    return MNF_OK;
}

int run_iterate(mnf_ctx* ctx, const std::vector<ScanIn>& in, int n_iter, const ptycho_params& p, hipStream_t st) {
    const int ns = (int)in.size();
    CallPlan pl;
    std::map<int, std::vector<int>> classes;  // detector size -> scans
    MNF_TRY(plan_iterate(ctx, in, n_iter, p, ctx->d_status, pl, classes));
    if (n_iter == 0) return MNF_OK;
    const bool sub = pl.sub;
    const int modes = pl.modes;

    // per-scan scratch: P2 [Nw^2], maxP2_row [Nw], amplitudes [J][Nd][Nd] (FFT order;
    // a call without allocations takes the square roots in the column pass
    // instead), error partials [J][N/C], |A|^2 partials [J] and sum
    const bool amp = ctx->arena == nullptr;
    size_t f_need = 0, d_need = 0;
    for (int k = 0; k < ns; ++k) {
        f_need += (size_t)in[k].Nw * in[k].Nw + in[k].Nw + (amp ? (size_t)in[k].J * in[k].Nd * in[k].Nd : 0);
        d_need += (size_t)in[k].J * col_groups(ctx, in[k].Nd) + in[k].J + 1;
    }
    void *fbuf, *dbuf;
    MNF_TRY(mnf::scratch(ctx, "scan_f32", f_need * sizeof(float), &fbuf));
    MNF_TRY(mnf::scratch(ctx, "scan_f64", d_need * sizeof(double), &dbuf));
    std::vector<double*> sA2p(ns), sA2(ns);
    {
        float* f = (float*)fbuf;
        double* d = (double*)dbuf;
        for (int k = 0; k < ns; ++k) {
            pl.scans[k].P2 = f;
            f += (size_t)in[k].Nw * in[k].Nw;
            pl.scans[k].maxP2_row = f;
            f += in[k].Nw;
            pl.scans[k].A = amp ? f : nullptr;
            if (amp) f += (size_t)in[k].J * in[k].Nd * in[k].Nd;
            pl.scans[k].err_part = d;
            d += (size_t)in[k].J * col_groups(ctx, in[k].Nd);
            sA2p[k] = d;
            d += in[k].J;
            sA2[k] = d;
            d += 1;
        }
    }
    MNF_TRY(upload_plan(ctx, pl, st));
    // error reduction jobs, one per scan per iteration.  A graph writes the
    // errors to an internal buffer [ns][n_iter], copied to err_out after each
    // replay, so that the caller's output addresses are not part of the graph.
    const bool graph_req = p.graph != 0 && ctx->prof.mask == 0 && ctx->arena == nullptr;
    double* err_buf = nullptr;
    if (graph_req) {
        void* eb;
        MNF_TRY(mnf::scratch(ctx, "err_buf", (size_t)ns * std::max(n_iter, 1) * sizeof(double), &eb));
        err_buf = (double*)eb;
    }
    auto err_dst = [&](int k) { return graph_req ? err_buf + (size_t)k * n_iter : in[k].err_out; };
    std::vector<SumJob> jobs;
    for (int i = 0; i < n_iter; ++i)
        for (int k = 0; k < ns; ++k)
            jobs.push_back(SumJob{pl.scans[k].err_part, (size_t)in[k].J * col_groups(ctx, in[k].Nd), sA2[k],
                                  in[k].err_out ? err_dst(k) + i : nullptr,
                                  in[k].err_out && i > 0 ? err_dst(k) : nullptr, ctx->d_status});
    std::vector<SumJob> a2jobs;
    for (int k = 0; k < ns; ++k) a2jobs.push_back(SumJob{sA2p[k], (size_t)in[k].J, nullptr, sA2[k], nullptr, nullptr});
    void *d_jobs, *d_a2jobs, *S, *mO;
    MNF_TRY(upload(ctx, "plan_jobs", jobs.data(), sizeof(SumJob) * jobs.size(), st, &d_jobs));
    MNF_TRY(upload(ctx, "plan_a2jobs", a2jobs.data(), sizeof(SumJob) * a2jobs.size(), st, &d_a2jobs));
    // With launch-shape bit 2, one scan at integer positions with one probe
    // mode takes three launches per mini-batch (object update fused with the
    // next mini-batch's exit-wave rows, k_obj_rows) when its object box fits
    // the pass's LDS rows; the pattern scratch is then double-buffered (the
    // fused pass reads one mini-batch's numerators and writes the next one's
    // rows) and the |O|^2 maxima are kept per window row.  The results are
    // bit-identical to four launches; which is faster is left to the tuner
    // (at 32 patterns of 256^2 the fused pass, one block's chain of loads,
    // update, transforms and stores, is slower than the two passes it joins).
    const bool fused = ns == 1 && !sub && modes == 1 && pl.scans[0].bw <= kObjRowMaxWidth &&
                       three_launch(ctx, in[0].Nd);
    // Size classes share no data (a scan has one detector size), so with more
    // than one class each class's launches and error sums go on a stream of
    // its own, forked from and joined to the call's stream by events, and the
    // classes' passes overlap on the GPU; each class then takes its own region
    // of the pattern and maxima scratch.  (A call without allocations keeps
    // one stream and shared regions, and so does a context timing its kernel
    // classes, whose per-kernel times would otherwise include the overlap.)
    const int ncls = (int)classes.size();
    const bool multi = ncls > 1 && !fused && ctx->arena == nullptr && ctx->prof.mask == 0;
    std::map<int, size_t> offS, offM;  // class -> byte offset into S, float offset into maxO2
    size_t bytesS = pl.max_S * (fused ? 2 : 1);
    size_t floatsM = std::max(pl.max_maxO2, fused ? (size_t)pl.max_slots * in[0].Nw : (size_t)0);
    if (multi) {
        std::map<int, size_t> needS, needM;
        for (const Launch& L : pl.launches) {
            const int gr = (L.maxNw + row_lines(ctx, L.N) - 1) / row_lines(ctx, L.N);
            needS[L.N] = std::max(needS[L.N], (size_t)L.nslots * L.N * L.N * sizeof(float2));
            needM[L.N] = std::max(needM[L.N], (size_t)L.nslots * gr);
        }
        bytesS = floatsM = 0;
        for (auto& kv : classes) {
            offS[kv.first] = bytesS;
            offM[kv.first] = floatsM;
            bytesS += (needS[kv.first] + 255) & ~(size_t)255;
            floatsM += (needM[kv.first] + 63) & ~(size_t)63;
        }
    }
    const size_t sS = pl.max_S / sizeof(float2);  // complex values of one pattern buffer
    MNF_TRY(mnf::scratch(ctx, "S", bytesS, &S));
    MNF_TRY(mnf::scratch(ctx, "maxO2", std::max<size_t>(floatsM, 1) * sizeof(float), &mO));
    // the error sums of each class's scans, iteration-major within the class
    std::vector<int> cls_job0, cls_nscan;
    void* d_cjobs = nullptr;
    if (multi && any_err_of(in)) {
        std::vector<SumJob> cjobs;
        for (auto& kv : classes) {
            cls_job0.push_back((int)cjobs.size());
            cls_nscan.push_back((int)kv.second.size());
            for (int i = 0; i < n_iter; ++i)
                for (int k : kv.second) cjobs.push_back(jobs[(size_t)i * ns + k]);
        }
        MNF_TRY(upload(ctx, "plan_cjobs", cjobs.data(), sizeof(SumJob) * cjobs.size(), st, &d_cjobs));
    }
    SubBufs sbuf{nullptr, nullptr, nullptr};
    const SubBufs* sb = nullptr;
    if (sub) {
        const size_t nw2 = (size_t)in[0].Nw * in[0].Nw;
        void *pd, *g = nullptr, *dp = nullptr;
        MNF_TRY(mnf::scratch(ctx, "sub_Pd", (size_t)pl.max_slots * nw2 * sizeof(float2), &pd));
        if (p.update_probe) {
            MNF_TRY(mnf::scratch(ctx, "sub_G", (size_t)pl.max_slots * nw2 * sizeof(float2), &g));
            MNF_TRY(mnf::scratch(ctx, "sub_DP", nw2 * sizeof(double), &dp));
        }
        sbuf = SubBufs{(float2*)pd, (float2*)g, (double*)dp};
        sb = &sbuf;
        const float2* tw;
        MNF_TRY(twiddles(ctx, in[0].Nw, &tw));
    }
    // the amplitudes every iteration projects onto, once per call
    for (int k = 0; k < ns && amp; ++k)
        MNF_LAUNCH(ctx, MNF_K_SMALL, st, k_amplitude_prep, dim3((unsigned)in[k].Nd, (unsigned)in[k].J),
                   dim3((unsigned)std::min(in[k].Nd, 256)), in[k].I, in[k].Nd, (float*)pl.scans[k].A,
                   ctx->d_status);
    bool any_err = false;
    for (int k = 0; k < ns; ++k) any_err |= in[k].err_out != nullptr;
    if (any_err) {
        for (int k = 0; k < ns; ++k)
            MNF_LAUNCH(ctx, MNF_K_SMALL, st, k_sum_amplitude2, dim3(in[k].J), dim3(256), in[k].I,
                       (size_t)in[k].Nd * in[k].Nd, sA2p[k]);
        MNF_LAUNCH(ctx, MNF_K_SMALL, st, k_sum_jobs, dim3(ns), dim3(256), (const SumJob*)d_a2jobs, 1.0);
    }
    MNF_CHECK_LAUNCH(ctx);

    // twiddle tables exist before any capture starts (creating one copies from the host)
    for (auto& kv : classes) {
        const float2* tw;
        MNF_TRY(twiddles(ctx, kv.first, &tw));
    }
    // the iterations, optionally as one graph.  Launch timing needs direct
    // launches, so a context with timing enabled does not use graphs.
    hipStream_t run = st;
    const bool graph = graph_req;
    uint64_t key = 0;
    // copies of the graph's errors to the caller's outputs (after a replay)
    auto copy_errs = [&]() -> int {
        for (int k = 0; k < ns; ++k)
            if (in[k].err_out)
                MNF_HIP(ctx, hipMemcpyAsync(in[k].err_out, err_buf + (size_t)k * n_iter, n_iter * sizeof(double),
                                            hipMemcpyDeviceToDevice, st));
        return MNF_OK;
    };
    if (graph) {
        // Everything the launch sequence depends on: plan tables (their device
        // copies are re-uploaded above on every call), scratch addresses,
        // parameters, launch shapes.  The same key replays the cached graph.
        KeyHash kh;
        kh.add_vec(pl.scans);
        kh.add_vec(pl.slots);
        kh.add_vec(pl.groups);
        for (const Launch& L : pl.launches) {  // field by field: the struct has padding
            const long long f[] = {L.N, (long long)L.slot_off, L.nslots, (long long)L.group_off, L.ngroups, L.tiles,
                                   L.maxNw};
            kh.add(f, sizeof f);
        }
        kh.add_vec(pl.iter_end);
        kh.add_vec(pl.fracs);
        kh.add_vec(jobs);
        kh.add(p);
        kh.add(n_iter);
        const void* ptrs[] = {pl.d_scans, pl.d_slots, pl.d_groups, pl.d_fracs, d_jobs, S, mO,
                              sbuf.Pd, sbuf.G, sbuf.DP, d_cjobs};
        kh.add(ptrs, sizeof ptrs);
        for (auto& kv : classes) {
            const float2* tw;
            MNF_TRY(twiddles(ctx, kv.first, &tw));
            const int v = variant_of(ctx, kv.first);
            kh.add(kv.first);
            kh.add(v);
            kh.add(tw);
        }
        kh.add(pl.sub);
        kh.add(pl.modes);
        key = kh.value();
        if (ctx->graph_exec && ctx->graph_key == key) {
            MNF_HIP(ctx, hipGraphLaunch(ctx->graph_exec, st));
            return copy_errs();
        }
        if (!ctx->capture_stream) MNF_HIP(ctx, hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking));
        run = ctx->capture_stream;
        MNF_HIP(ctx, hipStreamBeginCapture(run, hipStreamCaptureModeThreadLocal));
    }
    int rc = MNF_OK;
    // A single scan at integer positions with one mode and mini-batches of one
    // on patterns of at most 64^2 runs in one launch of one workgroup.
    const bool small = ns == 1 && !sub && modes == 1 && p.batch == 1 && in[0].Nd <= kSmallMaxN &&
                       !small_run_off(ctx, in[0].Nd);
    if (small) {
        const int upd_from = !p.update_probe ? n_iter : std::min(n_iter, std::max(0, p.probe_start_iter - p.it0));
        switch (in[0].Nd) {
            case 16: rc = launch_small_run<16>(ctx, pl, in[0].J, n_iter, p, upd_from, sA2[0], in[0].err_out ? err_dst(0) : nullptr, run); break;
            case 32: rc = launch_small_run<32>(ctx, pl, in[0].J, n_iter, p, upd_from, sA2[0], in[0].err_out ? err_dst(0) : nullptr, run); break;
            default: rc = launch_small_run<64>(ctx, pl, in[0].J, n_iter, p, upd_from, sA2[0], in[0].err_out ? err_dst(0) : nullptr, run); break;
        }
    }
    size_t li = small ? pl.launches.size() : 0;
    const size_t nL = pl.launches.size();
    auto Sbuf = [&](size_t b) { return (float2*)S + (fused ? (b % 2) * sS : 0); };
    // the class streams: fork after everything issued so far on the call's stream
    std::map<int, int> cls_of;  // detector size -> class index
    {
        int c = 0;
        for (auto& kv : classes) cls_of[kv.first] = c++;
    }
    if (multi && rc == MNF_OK) {
        rc = class_streams(ctx, ncls);
        if (rc == MNF_OK && hipEventRecord(ctx->class_events[0], run) != hipSuccess) rc = MNF_EHIP;
        for (int c = 0; c < ncls && rc == MNF_OK; ++c)
            if (hipStreamWaitEvent(ctx->class_streams[c], ctx->class_events[0], 0) != hipSuccess) rc = MNF_EHIP;
        if (rc == MNF_EHIP) rc = set_error(ctx, MNF_EHIP, "forking the size-class streams failed");
    }
    auto stream_of = [&](int N) { return multi ? ctx->class_streams[cls_of[N]] : run; };
    for (int i = 0; i < n_iter && rc == MNF_OK; ++i) {
        const int it = p.it0 + i;
        const bool upd = p.update_probe && it >= p.probe_start_iter;
        for (; li < (size_t)pl.iter_end[i] && rc == MNF_OK; ++li) {
            if (!fused) {
                const Launch& L = pl.launches[li];
                float2* SL = multi ? (float2*)((char*)S + offS[L.N]) : (float2*)S;
                float* ML = multi ? (float*)mO + offM[L.N] : (float*)mO;
                rc = issue_iterate_any(ctx, pl, L, p, upd, SL, ML, sb, stream_of(L.N));
                continue;
            }
            const Launch& L = pl.launches[li];
            if (li == 0)
                rc = issue_obj_rows_any(ctx, pl, L.N, nullptr, &L, nullptr, Sbuf(0), (float*)mO, p, run);
            if (rc == MNF_OK) rc = issue_cols_inv_any(ctx, pl, L, p, upd, Sbuf(li), (float*)mO, run);
            if (rc == MNF_OK)
                rc = issue_obj_rows_any(ctx, pl, L.N, &L, li + 1 < nL ? &pl.launches[li + 1] : nullptr, Sbuf(li),
                                        Sbuf(li + 1), (float*)mO, p, run);
        }
        if (rc == MNF_OK && any_err && !small) {
            if (multi) {
                for (int c = 0; c < ncls; ++c)
                    hipLaunchKernelGGL(k_sum_jobs, dim3(cls_nscan[c]), dim3(256), 0, ctx->class_streams[c],
                                       (const SumJob*)d_cjobs + cls_job0[c] + (size_t)i * cls_nscan[c], 1.0);
            } else {
                hipLaunchKernelGGL(k_sum_jobs, dim3(ns), dim3(256), 0, run, (const SumJob*)d_jobs + (size_t)i * ns,
                                   1.0);
            }
        }
    }
    // join the class streams back into the call's stream
    if (multi) {
        for (int c = 0; c < ncls; ++c) {
            hipError_t e = hipEventRecord(ctx->class_events[1 + c], ctx->class_streams[c]);
            if (e == hipSuccess) e = hipStreamWaitEvent(run, ctx->class_events[1 + c], 0);
            if (e != hipSuccess && rc == MNF_OK) rc = set_error(ctx, MNF_EHIP, "joining the size-class streams failed");
        }
    }
    // non-finite objects and probes are reported by mnf_status
    for (int k = 0; k < ns && rc == MNF_OK; ++k) {
        const size_t no = (size_t)in[k].My * in[k].Mx, np = (size_t)in[k].modes * in[k].Nw * in[k].Nw;
        hipLaunchKernelGGL(k_check_finite, dim3((unsigned)std::min<size_t>((no + 255) / 256, 1024)), dim3(256), 0, run,
                           (const float2*)in[k].O, no, ctx->d_status);
        hipLaunchKernelGGL(k_check_finite, dim3((unsigned)std::min<size_t>((np + 255) / 256, 1024)), dim3(256), 0, run,
                           (const float2*)in[k].P, np, ctx->d_status);
    }
    if (graph) {
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(run, &g);
        if (rc != MNF_OK) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) return set_error(ctx, MNF_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
        if (ctx->graph_exec) {
            MNF_HIP(ctx, hipStreamSynchronize(st));
            MNF_HIP(ctx, hipGraphExecDestroy(ctx->graph_exec));
            ctx->graph_exec = nullptr;
            ctx->graph_key = 0;
        }
        e = hipGraphInstantiate(&ctx->graph_exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return set_error(ctx, MNF_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
        ctx->graph_key = key;
        MNF_HIP(ctx, hipGraphLaunch(ctx->graph_exec, st));
        return copy_errs();
    }
    if (rc != MNF_OK) return rc;
    MNF_CHECK_LAUNCH(ctx);
    return MNF_OK;
}

// ----------------------------------------------------------------- forward

template <int N, int RV, int CV>
int forward_v(mnf_ctx* ctx, const CallPlan& pl, float* I_out, const SubBufs* sb, hipStream_t st) {
    const float2* tw;
    MNF_TRY(twiddles(ctx, N, &tw));
    void* S;
    MNF_TRY(mnf::scratch(ctx, "S", pl.max_S, &S));
    for (const Launch& L : pl.launches) {
        const float2* Pd = nullptr;
        int pmod = 1;
        const float2* fr = sb ? (const float2*)pl.d_fracs + L.slot_off : nullptr;
        if (sb && pl.scans[0].Nw == N) {  // x translation inside the exit-wave pass
            MNF_TRY(shift_probe_y<N>(ctx, pl.scans[0].P, sb->Pd, fr, L.nslots, st));
            MNF_TRY((launch_rows_fwd<N, RV, true>(ctx, pl, L, (const ScanDev*)pl.d_scans, (float2*)S, (float*)nullptr,
                                                  sb->Pd, kOwnProbe, tw, st, fr)));
            MNF_LAUNCH(ctx, MNF_K_FORWARD, st, (k_cols_intensity<N, CV>), dim3(N / ColCfg<N, CV>::C, L.nslots),
                       dim3(ColCfg<N, CV>::THREADS), (const ScanDev*)pl.d_scans,
                       (const SlotDev*)pl.d_slots + L.slot_off, (const float2*)S, I_out, tw);
            continue;
        }
        if (sb) {
            MNF_TRY(shift_probe(ctx, pl.scans[0].Nw, pl.scans[0].P, sb->Pd, fr, L.nslots, st));
            Pd = sb->Pd;
            pmod = kOwnProbe;
        } else if (pl.modes > 1) {
            Pd = pl.scans[0].P;
            pmod = pl.modes;
        }
        MNF_TRY((launch_rows_fwd<N, RV>(ctx, pl, L, (const ScanDev*)pl.d_scans, (float2*)S, (float*)nullptr, Pd, pmod,
                                        tw, st)));
        if (pl.modes > 1)
            MNF_LAUNCH(ctx, MNF_K_FORWARD, st, (k_cols_intensity_modes<N, CV>),
                       dim3(N / ColCfg<N, CV>::C, L.nslots / pl.modes), dim3(ColCfg<N, CV>::THREADS),
                       (const ScanDev*)pl.d_scans, (const SlotDev*)pl.d_slots + L.slot_off, (const float2*)S,
                       pl.modes, I_out, tw);
        else
            MNF_LAUNCH(ctx, MNF_K_FORWARD, st, (k_cols_intensity<N, CV>), dim3(N / ColCfg<N, CV>::C, L.nslots),
                       dim3(ColCfg<N, CV>::THREADS), (const ScanDev*)pl.d_scans,
                       (const SlotDev*)pl.d_slots + L.slot_off, (const float2*)S, I_out, tw);
    }
    MNF_CHECK_LAUNCH(ctx);
    return MNF_OK;
}

template <int N>
int forward_n(mnf_ctx* ctx, const CallPlan& pl, float* I_out, const SubBufs* sb, hipStream_t st) {
    switch (variant_of(ctx, N) & 3) {
        case 1: return forward_v<N, 1, 0>(ctx, pl, I_out, sb, st);
        case 2: return forward_v<N, 0, 1>(ctx, pl, I_out, sb, st);
        case 3: return forward_v<N, 1, 1>(ctx, pl, I_out, sb, st);
        default: return forward_v<N, 0, 0>(ctx, pl, I_out, sb, st);
    }
}

// ------------------------------------------------------------------ grad

// Gradient descent on top of the gradient pass: after each pass over all
// positions the pass is accepted or rejected on its loss (k_descent_decide)
// and the object (and the probe with update_probe) moves to the next point
// from the gradients in s.gO / s.gP or the saved best; the pass's loss is
// copied to loss[step].
struct DescentArgs {
    int n_steps;
    int update_probe;
    double* eta;         // device [2]: eta_O, eta_P (halved on rejection)
    double* loss;        // device [n_steps] or NULL
    DescentState* state;
    float2 *Ob, *gOb, *Pb, *gPb;  // the best point and its gradients
};

template <int N, int RV, int CV>
int grad_v(mnf_ctx* ctx, const CallPlan& pl, const ScanIn& s, int kind, float eps, const double* upstream, double* loss_out,
           hipStream_t st, const DescentArgs* dsc) {
    const float2* tw;
    MNF_TRY(twiddles(ctx, N, &tw));
    void *S, *lossp, *d_job;
    MNF_TRY(mnf::scratch(ctx, "S", pl.max_S, &S));
    MNF_TRY(mnf::scratch(ctx, "losspart", (size_t)s.J * col_groups(ctx, N) * sizeof(double), &lossp));
    // the scan's partials live in the loss buffer
    std::vector<ScanDev> sd = pl.scans;
    sd[0].err_part = (double*)lossp;
    void* d_scans;
    MNF_TRY(upload(ctx, "plan_scans", sd.data(), sizeof(ScanDev), st, &d_scans));
    SumJob job{(const double*)lossp, (size_t)s.J * col_groups(ctx, N), nullptr, loss_out, nullptr, ctx->d_status};
    MNF_TRY(upload(ctx, "plan_lossjob", &job, sizeof job, st, &d_job));
    const ScanDev* scans = (const ScanDev*)d_scans;
    const size_t nO = (size_t)s.My * s.Mx, nP = (size_t)s.Nw * s.Nw;
    const int passes = dsc ? dsc->n_steps : 1;
    for (int step = 0; step < passes; ++step) {
    if (s.gO)
        MNF_LAUNCH(ctx, MNF_K_SMALL, st, k_zero_c64, dim3((unsigned)((nO + 255) / 256)), dim3(256), s.gO, nO);
    if (s.gP) MNF_LAUNCH(ctx, MNF_K_SMALL, st, k_zero_c64, dim3((unsigned)((nP + 255) / 256)), dim3(256), s.gP, nP);
    for (const Launch& L : pl.launches) {
        const SlotDev* slots = (const SlotDev*)pl.d_slots + L.slot_off;
        const GroupDev* groups = (const GroupDev*)pl.d_groups + L.group_off;
        MNF_TRY((launch_rows_fwd<N, RV>(ctx, pl, L, scans, (float2*)S, (float*)nullptr, (const float2*)nullptr, 1,
                                        tw, st)));
        if (kind == 0)
            MNF_LAUNCH(ctx, MNF_K_GRAD_COLS, st, (k_cols_pointwise<N, CV, ColOp::PoissonGrad>),
                       dim3(N / ColCfg<N, CV>::C, L.nslots), dim3(ColCfg<N, CV>::THREADS), scans, slots, (float2*)S,
                       eps, tw);
        else
            MNF_LAUNCH(ctx, MNF_K_GRAD_COLS, st, (k_cols_pointwise<N, CV, ColOp::AmplitudeGrad>),
                       dim3(N / ColCfg<N, CV>::C, L.nslots), dim3(ColCfg<N, CV>::THREADS), scans, slots, (float2*)S,
                       eps, tw);
        if (!s.gO && !s.gP) continue;
        MNF_LAUNCH(ctx, MNF_K_ROWS_INV, st, (k_rows_inv_update<N, RV, 2>), dim3(L.maxNw, L.ngroups),
                   dim3(UpdCfg<N, RV>::THREADS), scans, slots, groups, (float2*)S, (const float*)nullptr, 0, 0, 0.f,
                   upstream, 1, (const float2*)nullptr, (float2*)nullptr, (double*)nullptr,
                   (const float2*)nullptr, tw);
        if (s.gO)
            MNF_LAUNCH(ctx, MNF_K_GRAD_SCATTER, st, k_grad_object, dim3(L.tiles), dim3(kObjThreads), scans, slots,
                       groups, L.ngroups, (const float2*)S, N);
    }
    MNF_LAUNCH(ctx, MNF_K_SMALL, st, k_sum_jobs, dim3(1), dim3(256), (const SumJob*)d_job, 1.0);  // loss, status
    if (dsc) {
        // every gradient of this pass was taken at the pass's starting O and P
        double* ldst = dsc->loss ? dsc->loss + step : (double*)nullptr;
        MNF_LAUNCH(ctx, MNF_K_SMALL, st, k_descent_decide, dim3(1), dim3(64), (const double*)loss_out, step,
                   dsc->state, dsc->eta, ldst);
        MNF_LAUNCH(ctx, MNF_K_SMALL, st, k_descent_update,
                   dim3((unsigned)((nO + kDescentThreads - 1) / kDescentThreads)), dim3(kDescentThreads), s.O,
                   (const float2*)s.gO, dsc->Ob, dsc->gOb, nO, (const double*)dsc->eta,
                   (const DescentState*)dsc->state);
        if (dsc->update_probe)
            MNF_LAUNCH(ctx, MNF_K_SMALL, st, k_descent_update,
                       dim3((unsigned)((nP + kDescentThreads - 1) / kDescentThreads)), dim3(kDescentThreads), s.P,
                       (const float2*)s.gP, dsc->Pb, dsc->gPb, nP, (const double*)(dsc->eta + 1),
                       (const DescentState*)dsc->state);
    }
    }
    MNF_CHECK_LAUNCH(ctx);
    return MNF_OK;
}

template <int N>
int grad_n(mnf_ctx* ctx, const CallPlan& pl, const ScanIn& s, int kind, float eps, const double* upstream, double* loss_out,
           hipStream_t st, const DescentArgs* dsc) {
    switch (variant_of(ctx, N) & 3) {
        case 1: return grad_v<N, 1, 0>(ctx, pl, s, kind, eps, upstream, loss_out, st, dsc);
        case 2: return grad_v<N, 0, 1>(ctx, pl, s, kind, eps, upstream, loss_out, st, dsc);
        case 3: return grad_v<N, 1, 1>(ctx, pl, s, kind, eps, upstream, loss_out, st, dsc);
        default: return grad_v<N, 0, 0>(ctx, pl, s, kind, eps, upstream, loss_out, st, dsc);
    }
}

// n_steps descent passes, then the step sizes as they stand to eta_out.
template <int N>
int descend_n(mnf_ctx* ctx, const CallPlan& pl, const ScanIn& s, int kind, float eps, double* lossd, hipStream_t st,
              const DescentArgs& dsc, double* eta_out) {
    MNF_TRY(grad_n<N>(ctx, pl, s, kind, eps, (const double*)nullptr, lossd, st, &dsc));
    if (eta_out) MNF_HIP(ctx, hipMemcpyAsync(eta_out, dsc.eta, 2 * sizeof(double), hipMemcpyDeviceToDevice, st));
    return MNF_OK;
}

// Real positions host float [J][2] -> nearest integer corners (halves round up)
// and the fractions r - corner in [-1/2, 1/2), exact in float.
int split_positions(mnf_ctx* ctx, const float* pos, int J, std::vector<int32_t>& ip, std::vector<float2>& fr) {
    if (!pos) return set_error(ctx, MNF_EINVAL, "null positions");
    if (J <= 0) return set_error(ctx, MNF_EINVAL, "J must be positive (J=%d)", J);
    ip.resize(2 * (size_t)J);
    fr.resize(J);
    for (int j = 0; j < J; ++j) {
        const double y = pos[2 * j], x = pos[2 * j + 1];
        if (!std::isfinite(y) || !std::isfinite(x) || std::fabs(y) > 1e8 || std::fabs(x) > 1e8)
            return set_error(ctx, MNF_EINVAL, "position %d is not a finite coordinate", j);
        const double py = std::floor(y + 0.5), px = std::floor(x + 0.5);
        ip[2 * j] = (int32_t)py;
        ip[2 * j + 1] = (int32_t)px;
        fr[j] = make_float2((float)(y - py), (float)(x - px));
    }
    return MNF_OK;
}

// Single-scan plan with the identity order in chunks of `chunk` positions.
int plan_identity(mnf_ctx* ctx, const ScanIn& s, int chunk, CallPlan& pl, hipStream_t st) {
    Box b;
    MNF_TRY(check_scan(ctx, s, 0, &b));
    pl.scans.resize(1);
    fill_scan_dev(pl.scans[0], s, b, ctx->d_status);
    std::vector<int> cls{0};
    std::vector<ScanIn> in{s};
    const int nr = (s.J + chunk - 1) / chunk;
    for (int r = 0; r < nr; ++r) plan_round(ctx, pl, in, cls, 0, r, chunk, s.Nd);
    pl.sub = s.frac != nullptr;
    pl.modes = s.modes;
    return upload_plan(ctx, pl, st);
}

// Time every launch-shape variant for detector size N on a synthetic scan of
// `nslots` positions iterated `reps` times in mini-batches of `nslots`.
int autotune_impl(mnf_ctx* ctx, int N, int nslots, int reps, double* times_us, hipStream_t st) {
    if (!size_supported(N)) return set_error(ctx, MNF_EUNSUPPORTED, "detector size %d has no FFT plan", N);
    if (nslots < 1 || nslots > kMaxBatch) return set_error(ctx, MNF_EINVAL, "nslots outside [1, %d]", kMaxBatch);
    if (reps < 1) return set_error(ctx, MNF_EINVAL, "reps must be positive");
    // One mini-batch as it occurs in a scan larger than the batch taken in a
    // shuffled order: nslots windows drawn (index stride 7919, coprime with
    // the 625 raster points, so all distinct) from a 25 x 25 raster of step
    // N/8 over an object of side 4N, so the object box the update passes
    // cover is as wide as a real mini-batch's (a compact grid would favour
    // the pass structures whose cost grows with that box).
    constexpr int kGrid = 25;
    const int step = N / 8 > 0 ? N / 8 : 1;
    const int M = N + (kGrid - 1) * step;
    void *O, *P, *I;
    MNF_TRY(mnf::scratch(ctx, "tune_O", (size_t)M * M * sizeof(float2), &O));
    MNF_TRY(mnf::scratch(ctx, "tune_P", (size_t)N * N * sizeof(float2), &P));
    MNF_TRY(mnf::scratch(ctx, "tune_I", (size_t)nslots * N * N * sizeof(float), &I));
    hipLaunchKernelGGL(k_fill_c64, dim3((unsigned)(((size_t)M * M + 255) / 256)), dim3(256), 0, st, (float2*)O,
                       (size_t)M * M, make_float2(1.f, 0.f));
    hipLaunchKernelGGL(k_fill_c64, dim3((unsigned)(((size_t)N * N + 255) / 256)), dim3(256), 0, st, (float2*)P,
                       (size_t)N * N, make_float2(0.5f, 0.5f));
    hipLaunchKernelGGL(k_fill_f32, dim3((unsigned)(((size_t)nslots * N * N + 255) / 256)), dim3(256), 0, st,
                       (float*)I, (size_t)nslots * N * N, 1.f);
    std::vector<int32_t> pos(2 * nslots);
    for (int k = 0; k < nslots; ++k) {
        const int idx = (int)(((long long)k * 7919 + 13) % (kGrid * kGrid));
        pos[2 * k] = (idx / kGrid) * step;
        pos[2 * k + 1] = (idx % kGrid) * step;
    }
    std::vector<ScanIn> in{ScanIn{(float2*)O, M, M, (float2*)P, N, (const float*)I, N, pos.data(), nslots, nullptr,
                                  nullptr, nullptr, nullptr}};
    ptycho_params p{1, 0.1f, 0.1f, nslots, 1, 0, 0, 0};
    hipEvent_t e0, e1;
    MNF_HIP(ctx, hipEventCreate(&e0));
    MNF_HIP(ctx, hipEventCreate(&e1));
    const int saved = variant_of(ctx, N);
    // Three interleaved rounds over the variants (launch shapes x pass
    // structure), the median time of each kept; a variant replaces the default
    // only when it is faster by at least kMargin, so run-to-run noise does not
    // flip the pick.
    constexpr int kVariants = 8, kRounds = 3;
    constexpr double kMargin = 0.03;
    std::vector<double> t((size_t)kVariants * kRounds, 0.0);
    int rc = MNF_OK;
    for (int r = 0; r < kRounds && rc == MNF_OK; ++r)
        for (int v = 0; v < kVariants && rc == MNF_OK; ++v) {
            ctx->variant[N] = v;
            if (r == 0) rc = run_iterate(ctx, in, 1, p, st);  // warm-up (also sizes the scratch)
            if (rc != MNF_OK) break;
            if (hipEventRecord(e0, st) != hipSuccess) { rc = MNF_EHIP; break; }
            rc = run_iterate(ctx, in, reps, p, st);
            if (rc != MNF_OK) break;
            if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) { rc = MNF_EHIP; break; }
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            t[(size_t)v * kRounds + r] = 1e3 * ms / reps;
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != MNF_OK) {
        ctx->variant[N] = saved;
        return rc == MNF_EHIP ? set_error(ctx, MNF_EHIP, "event timing failed during tuning") : rc;
    }
    double med[kVariants];
    for (int v = 0; v < kVariants; ++v) {
        double* x = &t[(size_t)v * kRounds];
        std::sort(x, x + kRounds);
        med[v] = x[kRounds / 2];
        if (times_us) times_us[v] = med[v];
    }
    int best = 0;
    for (int v = 1; v < kVariants; ++v)
        if (med[v] < med[best] && med[v] < (1.0 - kMargin) * med[0]) best = v;
    ctx->variant[N] = best;
    return best;
}

}  // namespace

// ------------------------------------------------------ without allocations
//
// Static scratch of ptycho_iterate_noalloc: a file-scope device array that
// every GPU the library runs on holds until the process ends.  Host code
// never passes its name to a kernel (on the host the name stands for a host
// object): the device address comes from hipGetSymbolAddress, once per
// device at context creation, and only that address is used.
constexpr size_t kNoAllocScratchBytes = (size_t)48 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mutex;
void* g_noalloc_ptr[kMaxDevices] = {};
}  // namespace

int mnf::noalloc_setup(mnf_ctx* ctx) {
    if (ctx->device < 0 || ctx->device >= kMaxDevices)
        return set_error(ctx, MNF_EINVAL, "device %d beyond the %d the static scratch table holds", ctx->device,
                         kMaxDevices);
    std::lock_guard<std::mutex> lock(g_noalloc_mutex);
    if (!g_noalloc_ptr[ctx->device]) {
        void* ptr = nullptr;
        // the context's device is current (mnf_create set it)
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(::scratch));
        if (e != hipSuccess || !ptr)
            return set_error(ctx, MNF_EHIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        g_noalloc_ptr[ctx->device] = ptr;
    }
    ctx->noalloc_ptr = g_noalloc_ptr[ctx->device];
    return MNF_OK;
}

extern "C" {

int ptycho_iterate_noalloc(mnf_ctx* ctx, mnf_c64* O, int My, int Mx, mnf_c64* P, int Nw, const float* I, int Nd,
                           const int32_t* pos, int J, const int32_t* order, int n_iter, const ptycho_params* params,
                           double* err_out, void* stream) {
    MNF_TRY(begin(ctx));
    if (!params) return set_error(ctx, MNF_EINVAL, "null params");
    if (params->graph) return set_error(ctx, MNF_EINVAL, "graph = 1 is not available without allocations");
    if (!ctx->noalloc_ptr) return set_error(ctx, MNF_EHIP, "the static scratch of device %d is not set up", ctx->device);
    // every scratch piece and staged table of this call comes from the static
    // scratch; launch timing (which creates events) is suspended
    MnfArena arena{(char*)ctx->noalloc_ptr, kNoAllocScratchBytes, 0};
    const uint32_t mask = ctx->prof.mask;
    ctx->arena = &arena;
    ctx->prof.mask = 0;
    std::vector<ScanIn> in{ScanIn{(float2*)O, My, Mx, (float2*)P, Nw, I, Nd, pos, J, order, err_out, nullptr,
                                  nullptr}};
    const int rc = run_iterate(ctx, in, n_iter, *params, (hipStream_t)stream);
    ctx->arena = nullptr;
    ctx->prof.mask = mask;
    return rc;
}

int mnf_autotune(mnf_ctx* ctx, int Nd, int nslots, int reps, double* times_us, void* stream) {
    MNF_TRY(begin(ctx));
    return autotune_impl(ctx, Nd, nslots, reps, times_us, (hipStream_t)stream);
}

int mnf_set_variant(mnf_ctx* ctx, int Nd, int variant) {
    MNF_TRY(begin(ctx));
    if (!size_supported(Nd)) return set_error(ctx, MNF_EUNSUPPORTED, "detector size %d has no FFT plan", Nd);
    if (variant < 0 || variant > 15) return set_error(ctx, MNF_EINVAL, "variant must be 0..15");
    ctx->variant[Nd] = variant;
    return MNF_OK;
}

int mnf_get_variant(mnf_ctx* ctx, int Nd) {
    MNF_TRY(begin(ctx));
    return variant_of(ctx, Nd);
}

int mnf_supported_sizes(int32_t* sizes, int cap) {
    const int n = (int)(sizeof(kSizes) / sizeof(kSizes[0]));
    for (int i = 0; i < n && i < cap && sizes; ++i) sizes[i] = kSizes[i];
    return n;
}

int ptycho_forward(mnf_ctx* ctx, const mnf_c64* O, int My, int Mx, const mnf_c64* P, int Nw, int Nd,
                   const int32_t* pos, int J, float* I_out, void* stream) {
    MNF_TRY(begin(ctx));
    if (!I_out) return set_error(ctx, MNF_EINVAL, "null output");
    hipStream_t st = (hipStream_t)stream;
    // I_out stands in for the scan's intensity pointer (validated, not read)
    ScanIn s{(float2*)O, My, Mx, (float2*)P, Nw, I_out, Nd, pos, J, nullptr, nullptr, nullptr, nullptr};
    CallPlan pl;
    MNF_TRY(plan_identity(ctx, s, 64, pl, st));
    MNF_DISPATCH(Nd, forward_n, ctx, pl, I_out, (const SubBufs*)nullptr, st)
}

int ptycho_forward_subpixel(mnf_ctx* ctx, const mnf_c64* O, int My, int Mx, const mnf_c64* P, int Nw, int Nd,
                            const float* pos, int J, float* I_out, void* stream) {
    MNF_TRY(begin(ctx));
    if (!I_out) return set_error(ctx, MNF_EINVAL, "null output");
    hipStream_t st = (hipStream_t)stream;
    std::vector<int32_t> ip;
    std::vector<float2> fr;
    MNF_TRY(split_positions(ctx, pos, J, ip, fr));
    if (!size_supported(Nw))
        return set_error(ctx, MNF_EUNSUPPORTED, "real positions need a probe window with an FFT plan (Nw=%d)", Nw);
    ScanIn s{(float2*)O, My, Mx, (float2*)P, Nw, I_out, Nd, ip.data(), J, nullptr, nullptr, nullptr, nullptr,
             fr.data()};
    CallPlan pl;
    MNF_TRY(plan_identity(ctx, s, 64, pl, st));
    void* pd;
    MNF_TRY(mnf::scratch(ctx, "sub_Pd", (size_t)pl.max_slots * Nw * Nw * sizeof(float2), &pd));
    const SubBufs sb{(float2*)pd, nullptr, nullptr};
    MNF_DISPATCH(Nd, forward_n, ctx, pl, I_out, &sb, st)
}

int ptycho_iterate(mnf_ctx* ctx, mnf_c64* O, int My, int Mx, mnf_c64* P, int Nw, const float* I, int Nd,
                   const int32_t* pos, int J, const int32_t* order, int n_iter, const ptycho_params* params,
                   double* err_out, void* stream) {
    MNF_TRY(begin(ctx));
    if (!params) return set_error(ctx, MNF_EINVAL, "null params");
    std::vector<ScanIn> in{ScanIn{(float2*)O, My, Mx, (float2*)P, Nw, I, Nd, pos, J, order, err_out, nullptr,
                                  nullptr}};
    return run_iterate(ctx, in, n_iter, *params, (hipStream_t)stream);
}

int ptycho_iterate_subpixel(mnf_ctx* ctx, mnf_c64* O, int My, int Mx, mnf_c64* P, int Nw, const float* I, int Nd,
                            const float* pos, int J, const int32_t* order, int n_iter, const ptycho_params* params,
                            double* err_out, void* stream) {
    MNF_TRY(begin(ctx));
    if (!params) return set_error(ctx, MNF_EINVAL, "null params");
    std::vector<int32_t> ip;
    std::vector<float2> fr;
    MNF_TRY(split_positions(ctx, pos, J, ip, fr));
    std::vector<ScanIn> in{ScanIn{(float2*)O, My, Mx, (float2*)P, Nw, I, Nd, ip.data(), J, order, err_out, nullptr,
                                  nullptr, fr.data()}};
    return run_iterate(ctx, in, n_iter, *params, (hipStream_t)stream);
}

int ptycho_forward_modes(mnf_ctx* ctx, const mnf_c64* O, int My, int Mx, const mnf_c64* P, int M, int Nw, int Nd,
                         const int32_t* pos, int J, float* I_out, void* stream) {
    MNF_TRY(begin(ctx));
    if (!I_out) return set_error(ctx, MNF_EINVAL, "null output");
    if (M < 1 || M > kMaxModes) return set_error(ctx, MNF_EINVAL, "probe modes %d outside [1, %d]", M, kMaxModes);
    hipStream_t st = (hipStream_t)stream;
    ScanIn s{(float2*)O, My, Mx, (float2*)P, Nw, I_out, Nd, pos, J, nullptr, nullptr, nullptr, nullptr, nullptr, M};
    CallPlan pl;
    MNF_TRY(plan_identity(ctx, s, 64, pl, st));
    MNF_DISPATCH(Nd, forward_n, ctx, pl, I_out, (const SubBufs*)nullptr, st)
}

int ptycho_iterate_modes(mnf_ctx* ctx, mnf_c64* O, int My, int Mx, mnf_c64* P, int M, int Nw, const float* I,
                         int Nd, const int32_t* pos, int J, const int32_t* order, int n_iter,
                         const ptycho_params* params, double* err_out, void* stream) {
    MNF_TRY(begin(ctx));
    if (!params) return set_error(ctx, MNF_EINVAL, "null params");
    std::vector<ScanIn> in{ScanIn{(float2*)O, My, Mx, (float2*)P, Nw, I, Nd, pos, J, order, err_out, nullptr,
                                  nullptr, nullptr, M}};
    return run_iterate(ctx, in, n_iter, *params, (hipStream_t)stream);
}

int ptycho_iterate_many(mnf_ctx* ctx, const ptycho_scan* scans, int n_scans, int n_iter,
                        const ptycho_params* params, void* stream) {
    MNF_TRY(begin(ctx));
    if (!params || !scans) return set_error(ctx, MNF_EINVAL, "null pointer argument");
    if (n_scans <= 0) return set_error(ctx, MNF_EINVAL, "n_scans must be positive");
    std::vector<ScanIn> in;
    for (int k = 0; k < n_scans; ++k) {
        const ptycho_scan& s = scans[k];
        in.push_back(ScanIn{(float2*)s.O, s.My, s.Mx, (float2*)s.P, s.Nw, s.I, s.Nd, s.pos, s.J, s.order,
                            s.err_out, nullptr, nullptr});
    }
    return run_iterate(ctx, in, n_iter, *params, (hipStream_t)stream);
}

int ptycho_plan_info(mnf_ctx* ctx, const ptycho_scan* scans, int n_scans, int n_iter, const ptycho_params* params,
                     int64_t* info, int n_info) {
    // without a context: a host-only one for messages and the default launch
    // shapes (nothing in it touches a device)
    mnf_ctx host;
    mnf_ctx* c = ctx ? ctx : &host;
    auto done = [&](int rc) {
        if (!ctx) mnf::set_host_error(rc == MNF_OK ? std::string() : host.err);
        return rc;
    };
    if (!params || !scans || (!info && n_info > 0)) return done(set_error(c, MNF_EINVAL, "null pointer argument"));
    if (n_scans <= 0) return done(set_error(c, MNF_EINVAL, "n_scans must be positive"));
    if (n_info < 0) return done(set_error(c, MNF_EINVAL, "n_info must be >= 0"));
    std::vector<ScanIn> in;
    for (int k = 0; k < n_scans; ++k) {
        const ptycho_scan& s = scans[k];
        in.push_back(ScanIn{(float2*)s.O, s.My, s.Mx, (float2*)s.P, s.Nw, s.I, s.Nd, s.pos, s.J, s.order,
                            s.err_out, nullptr, nullptr});
    }
    CallPlan pl;
    std::map<int, std::vector<int>> classes;
    const int rc = plan_iterate(c, in, n_iter, *params, nullptr, pl, classes);
    if (rc != MNF_OK) return done(rc);
    long long tiles = 0;
    for (const Launch& L : pl.launches) tiles += L.tiles;
    const int64_t v[] = {(int64_t)pl.launches.size(), (int64_t)pl.slots.size(), (int64_t)pl.groups.size(), tiles,
                         pl.max_slots, (int64_t)pl.max_S, (int64_t)classes.size()};
    for (int i = 0; i < n_info && i < (int)(sizeof v / sizeof v[0]); ++i) info[i] = v[i];
    for (int i = (int)(sizeof v / sizeof v[0]); i < n_info; ++i) info[i] = 0;
    return done(MNF_OK);
}

int ptycho_grad(mnf_ctx* ctx, const mnf_c64* O, int My, int Mx, const mnf_c64* P, int Nw, const float* I, int Nd,
                const int32_t* pos, int J, int kind, float eps, int batch, const double* upstream, double* loss_out,
                mnf_c64* gO, mnf_c64* gP, void* stream) {
    MNF_TRY(begin(ctx));
    if (kind != 0 && kind != 1) return set_error(ctx, MNF_EINVAL, "kind must be 0 (Poisson) or 1 (amplitude)");
    if (batch < 1 || batch > kMaxBatch) return set_error(ctx, MNF_EINVAL, "batch %d outside [1, %d]", batch, kMaxBatch);
    if (!(eps >= 0.f)) return set_error(ctx, MNF_EINVAL, "eps must be >= 0");
    hipStream_t st = (hipStream_t)stream;
    ScanIn s{(float2*)O, My, Mx, (float2*)P, Nw, I, Nd, pos, J, nullptr, nullptr, (float2*)gO, (float2*)gP};
    CallPlan pl;
    MNF_TRY(plan_identity(ctx, s, batch, pl, st));
    MNF_DISPATCH(Nd, grad_n, ctx, pl, s, kind, eps, upstream, loss_out, st, (const DescentArgs*)nullptr)
}

int ptycho_descend(mnf_ctx* ctx, mnf_c64* O, int My, int Mx, mnf_c64* P, int Nw, const float* I, int Nd,
                   const int32_t* pos, int J, int kind, float eps, int batch, int n_steps, double eta_O, double eta_P,
                   int update_probe, double* loss_out, double* eta_out, void* stream) {
    MNF_TRY(begin(ctx));
    if (kind != 0 && kind != 1) return set_error(ctx, MNF_EINVAL, "kind must be 0 (Poisson) or 1 (amplitude)");
    if (batch < 1 || batch > kMaxBatch) return set_error(ctx, MNF_EINVAL, "batch %d outside [1, %d]", batch, kMaxBatch);
    if (!(eps >= 0.f)) return set_error(ctx, MNF_EINVAL, "eps must be >= 0");
    if (n_steps < 0) return set_error(ctx, MNF_EINVAL, "n_steps must be >= 0 (%d)", n_steps);
    if (!(eta_O >= 0.0) || !(eta_P >= 0.0) || !std::isfinite(eta_O) || !std::isfinite(eta_P))
        return set_error(ctx, MNF_EINVAL, "step sizes must be finite and >= 0 (0: automatic)");
    hipStream_t st = (hipStream_t)stream;
    void *gO, *gP, *lossd, *etad, *partO, *partP, *dpos, *Ob, *gOb, *Pb, *gPb, *stt;
    const size_t bO = sizeof(float2) * (size_t)std::max(My, 1) * std::max(Mx, 1);
    const size_t bP = sizeof(float2) * (size_t)std::max(Nw, 1) * std::max(Nw, 1);
    MNF_TRY(mnf::scratch(ctx, "descent_gO", bO, &gO));
    MNF_TRY(mnf::scratch(ctx, "descent_gP", bP, &gP));
    // a fixed probe needs no probe gradient
    ScanIn s{(float2*)O, My, Mx, (float2*)P, Nw, I, Nd, pos, J, nullptr, nullptr, (float2*)gO,
             update_probe ? (float2*)gP : nullptr};
    CallPlan pl;
    MNF_TRY(plan_identity(ctx, s, batch, pl, st));  // checks the scan (sizes, windows inside O)
    const ScanDev& b = pl.scans[0];
    const size_t box = (size_t)b.bh * b.bw;
    const unsigned nbO = (unsigned)((box + kDescentThreads - 1) / kDescentThreads);
    const unsigned nbP = (unsigned)(((size_t)Nw * Nw + kDescentThreads - 1) / kDescentThreads);
    MNF_TRY(mnf::scratch(ctx, "descent_loss", sizeof(double), &lossd));
    MNF_TRY(mnf::scratch(ctx, "descent_eta", 2 * sizeof(double), &etad));
    MNF_TRY(mnf::scratch(ctx, "descent_partO", sizeof(float) * nbO, &partO));
    MNF_TRY(mnf::scratch(ctx, "descent_partP", sizeof(float) * nbP, &partP));
    MNF_TRY(upload(ctx, "descent_pos", pos, 2 * sizeof(int32_t) * (size_t)J, st, &dpos));
    // step sizes from the starting object and probe, fixed for the call (the
    // maxima only where a step size is not given)
    if (!(eta_O > 0.0))
        MNF_LAUNCH(ctx, MNF_K_SMALL, st, k_illum_max, dim3(nbO), dim3(kDescentThreads), (const float2*)P, Nw,
                   (const int32_t*)dpos, J, b.by0, b.bx0, b.bh, b.bw, (float*)partO);
    if (!(eta_P > 0.0))
        MNF_LAUNCH(ctx, MNF_K_SMALL, st, k_cover_max, dim3(nbP), dim3(kDescentThreads), (const float2*)O, Mx, Nw,
                   (const int32_t*)dpos, J, (float*)partP);
    MNF_LAUNCH(ctx, MNF_K_SMALL, st, k_step_sizes, dim3(1), dim3(kDescentThreads), (const float*)partO,
               eta_O > 0.0 ? 0 : (int)nbO, (const float*)partP, eta_P > 0.0 ? 0 : (int)nbP, eta_O, eta_P,
               (double*)etad);
    if (n_steps == 0) {
        if (eta_out) MNF_HIP(ctx, hipMemcpyAsync(eta_out, etad, 2 * sizeof(double), hipMemcpyDeviceToDevice, st));
        MNF_CHECK_LAUNCH(ctx);
        return MNF_OK;
    }
    MNF_TRY(mnf::scratch(ctx, "descent_Ob", bO, &Ob));
    MNF_TRY(mnf::scratch(ctx, "descent_gOb", bO, &gOb));
    MNF_TRY(mnf::scratch(ctx, "descent_Pb", bP, &Pb));
    MNF_TRY(mnf::scratch(ctx, "descent_gPb", bP, &gPb));
    MNF_TRY(mnf::scratch(ctx, "descent_state", sizeof(DescentState), &stt));
    const DescentArgs dsc{n_steps, update_probe ? 1 : 0, (double*)etad, loss_out, (DescentState*)stt,
                          (float2*)Ob, (float2*)gOb, (float2*)Pb, (float2*)gPb};
    MNF_DISPATCH(Nd, descend_n, ctx, pl, s, kind, eps, (double*)lossd, st, dsc, eta_out)
}

}  // extern "C"
