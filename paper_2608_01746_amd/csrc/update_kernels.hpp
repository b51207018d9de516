// Object accumulation kernels (mini-batched ePIE / rPIE object update and
// the gradient scatter), reductions and small helpers.
//
// Output-stationary: every object pixel is owned by one thread, which sums
// the contributions of its group's windows in slot order, so results are
// deterministic and no atomics are used.  One launch covers every group
// (scan) of the launch: block b belongs to the group whose tile range
// [tile0, tile0 + tiles) contains b.
#pragma once

#include "kernels_common.hpp"
#include "tables.hpp"

namespace mnf {

constexpr int kObjTileY = 16, kObjTileX = 64, kObjThreads = 256;
constexpr int kObjRows = kObjTileY / (kObjThreads / kObjTileX);
constexpr int kObjChunk = 8;

// Group of object-update block `b` (groups ordered by tile0).
__device__ __forceinline__ int find_group(const GroupDev* __restrict__ groups, int ngroups, int b) {
    int lo = 0, hi = ngroups - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (groups[mid].tile0 <= b) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Ordered list (in slot order) of the group's windows overlapping the tile
// [ty0, ty0 + kObjTileY) x [tx0, tx0 + kObjTileX).  Wave 0 builds it with
// ballots; every thread returns the count.  `before_barrier` runs in every
// thread after wave 0's loads are issued and before the barrier that
// publishes the list, so LDS values it writes are published with it.
template <class F>
__device__ __forceinline__ int tile_window_list(const SlotDev* __restrict__ slots, const GroupDev& gd,
                                                int Nw, int ty0, int tx0, int* l_slot, int* l_py,
                                                int* l_px, F&& before_barrier) {
    __shared__ int count;
    if (threadIdx.x < 64) {
        int cnt = 0;
        for (int base = 0; base < gd.nb; base += 64) {
            const int k = base + (int)threadIdx.x;
            bool hit = false;
            int py = 0, px = 0;
            if (k < gd.nb) {
                const SlotDev sd = slots[gd.s0 + k];
                py = sd.py;
                px = sd.px;
                hit = py < ty0 + kObjTileY && py + Nw > ty0 && px < tx0 + kObjTileX && px + Nw > tx0;
            }
            const unsigned long long m = __ballot(hit);
            if (hit) {
                const int q = cnt + __popcll(m & ((1ull << threadIdx.x) - 1ull));
                l_slot[q] = gd.s0 + k;
                l_py[q] = py;
                l_px[q] = px;
            }
            cnt += __popcll(m);
        }
        if (threadIdx.x == 0) count = cnt;
    }
    before_barrier();
    __syncthreads();
    return count;
}

__device__ __forceinline__ int tile_window_list(const SlotDev* __restrict__ slots, const GroupDev& gd,
                                                int Nw, int ty0, int tx0, int* l_slot, int* l_py,
                                                int* l_px) {
    return tile_window_list(slots, gd, Nw, ty0, tx0, l_slot, l_py, l_px, [] {});
}

// O[x] += sum_s W_s(u_s) / sum_s d_O(u_s),  u_s = x - p_s, over the windows
// of the group that contain x, where W_s = conj(P) dpsi_s (left in S by the
// inverse row pass) and, from the batch-start probe intensity P2 = |P|^2,
//   rPIE: d_O = (1 - alpha) P2 + alpha max P2;  ePIE: d_O = max P2 / alpha.
// Each thread owns one column and kObjRows rows of a 16 x 64 tile; the loads
// of a chunk of windows are all issued before any is used.  Slots of a chunk
// past the tile's window count (uniform over the block) issue no loads, and
// pixels outside a window add zero rather than branch.
__global__ void __launch_bounds__(kObjThreads)
k_object_update(const ScanDev* __restrict__ scans, const SlotDev* __restrict__ slots,
                const GroupDev* __restrict__ groups, int ngroups, const float2* __restrict__ S, int N,
                int rpie, float alpha) {
    __shared__ int l_slot[kMaxBatch], l_py[kMaxBatch], l_px[kMaxBatch];
    __shared__ float red[kObjThreads / 64];
    const ScanDev sc0 = scans[0];
    const GroupDev gd = groups[find_group(groups, ngroups, blockIdx.x)];
    const ScanDev sc = scan_desc(scans, sc0, gd.scan);
    const int Nw = sc.Nw;
    const int tile = blockIdx.x - gd.tile0;
    const int ty0 = sc.by0 + (tile / sc.tiles_x) * kObjTileY;
    const int tx0 = sc.bx0 + (tile % sc.tiles_x) * kObjTileX;
    // The probe's row maxima (Nw <= 512: two per thread) are loaded with the
    // slot table and reduced per wave before the window list's barrier,
    // which also publishes the wave maxima.
    static_assert(2 * kObjThreads >= 512, "two row maxima per thread cover the largest probe");
    const int i0 = (int)threadIdx.x, i1 = i0 + kObjThreads;
    const float v0 = ldg(sc.maxP2_row, min(i0, Nw - 1));
    const float v1 = ldg(sc.maxP2_row, min(i1, Nw - 1));
    const int cnt = tile_window_list(slots, gd, Nw, ty0, tx0, l_slot, l_py, l_px, [&] {
        float m = fmaxf(0.f, i0 < Nw ? v0 : 0.f);
        m = wave_max(fmaxf(m, i1 < Nw ? v1 : 0.f));
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    });
    if (cnt == 0) return;
    float mp = red[0];
#pragma unroll
    for (int w = 1; w < kObjThreads / 64; ++w) mp = fmaxf(mp, red[w]);
    const int xx = tx0 + (threadIdx.x % kObjTileX);
    const int yb = ty0 + (threadIdx.x / kObjTileX) * kObjRows;
    const float a = rpie ? 1.f - alpha : 0.f;
    const double cst = rpie ? (double)alpha * (double)mp : (double)mp / (double)alpha;
    const float* P2 = sc.P2;
    float2 num[kObjRows];
    double den[kObjRows];
#pragma unroll
    for (int q = 0; q < kObjRows; ++q) {
        num[q] = make_float2(0.f, 0.f);
        den[q] = 0.0;
    }
    for (int k0 = 0; k0 < cnt; k0 += kObjChunk) {
        const int nc = min(kObjChunk, cnt - k0);  // uniform over the block
        float2 w[kObjChunk][kObjRows];
        float p2[kObjChunk][kObjRows];
        bool in[kObjChunk][kObjRows];
#pragma unroll
        for (int c = 0; c < kObjChunk; ++c) {
            if (c < nc) {
                const int k = k0 + c;
                const int ux = xx - l_px[k];
                const bool inx = ux >= 0 && ux < Nw;
                const int uxc = min(max(ux, 0), Nw - 1);
                const float2* Sk = S + (size_t)l_slot[k] * N * N + uxc;
#pragma unroll
                for (int q = 0; q < kObjRows; ++q) {
                    const int uy = yb + q - l_py[k];
                    in[c][q] = inx && uy >= 0 && uy < Nw;
                    const int uyc = min(max(uy, 0), Nw - 1);
                    w[c][q] = Sk[(size_t)uyc * N];
                    p2[c][q] = ldg(P2, (size_t)uyc * Nw + uxc);
                }
            } else {
#pragma unroll
                for (int q = 0; q < kObjRows; ++q) {
                    in[c][q] = false;
                    w[c][q] = make_float2(0.f, 0.f);
                    p2[c][q] = 0.f;
                }
            }
        }
#pragma unroll
        for (int c = 0; c < kObjChunk; ++c)
#pragma unroll
            for (int q = 0; q < kObjRows; ++q) {
                const bool u = in[c][q];
                num[q] = cadd(num[q], u ? w[c][q] : make_float2(0.f, 0.f));
                den[q] += u ? (double)(a * p2[c][q]) + cst : 0.0;
            }
    }
    if (xx >= sc.bx0 + sc.bw) return;
    // the object values are read together (rows clamped into the box), then
    // the rows inside the box with a positive denominator are written
    float2 ov[kObjRows];
#pragma unroll
    for (int q = 0; q < kObjRows; ++q) ov[q] = ldg(sc.O, (size_t)min(yb + q, sc.by0 + sc.bh - 1) * sc.Mx + xx);
#pragma unroll
    for (int q = 0; q < kObjRows; ++q) {
        const int yy = yb + q;
        if (yy < sc.by0 + sc.bh && den[q] > 0.0) {
            const float inv = (float)(1.0 / den[q]);  // the float64 denominator, inverted once
            float2 v = ov[q];
            v.x = fmaf(num[q].x, inv, v.x);
            v.y = fmaf(num[q].y, inv, v.y);
            sc.O[(size_t)yy * sc.Mx + xx] = v;
        }
    }
}

// gO[x] += sum_s W_s(u_s) (gradient scatter), W_s = conj(P) g_s left in S by
// the inverse row pass.  Same tiling and load scheme as k_object_update.
__global__ void __launch_bounds__(kObjThreads)
k_grad_object(const ScanDev* __restrict__ scans, const SlotDev* __restrict__ slots,
              const GroupDev* __restrict__ groups, int ngroups, const float2* __restrict__ S, int N) {
    __shared__ int l_slot[kMaxBatch], l_py[kMaxBatch], l_px[kMaxBatch];
    const ScanDev sc0 = scans[0];
    const GroupDev gd = groups[find_group(groups, ngroups, blockIdx.x)];
    const ScanDev sc = scan_desc(scans, sc0, gd.scan);
    const int Nw = sc.Nw;
    const int tile = blockIdx.x - gd.tile0;
    const int ty0 = sc.by0 + (tile / sc.tiles_x) * kObjTileY;
    const int tx0 = sc.bx0 + (tile % sc.tiles_x) * kObjTileX;
    const int cnt = tile_window_list(slots, gd, Nw, ty0, tx0, l_slot, l_py, l_px);
    if (cnt == 0 || !sc.gO) return;
    const int xx = tx0 + (threadIdx.x % kObjTileX);
    const int yb = ty0 + (threadIdx.x / kObjTileX) * kObjRows;
    float2 acc[kObjRows];
    bool any[kObjRows];
#pragma unroll
    for (int q = 0; q < kObjRows; ++q) {
        acc[q] = make_float2(0.f, 0.f);
        any[q] = false;
    }
    for (int k0 = 0; k0 < cnt; k0 += kObjChunk) {
        const int nc = min(kObjChunk, cnt - k0);  // uniform over the block
        float2 w[kObjChunk][kObjRows];
        bool in[kObjChunk][kObjRows];
#pragma unroll
        for (int c = 0; c < kObjChunk; ++c) {
            if (c < nc) {
                const int k = k0 + c;
                const int ux = xx - l_px[k];
                const bool inx = ux >= 0 && ux < Nw;
                const float2* Sk = S + (size_t)l_slot[k] * N * N + min(max(ux, 0), Nw - 1);
#pragma unroll
                for (int q = 0; q < kObjRows; ++q) {
                    const int uy = yb + q - l_py[k];
                    in[c][q] = inx && uy >= 0 && uy < Nw;
                    w[c][q] = Sk[(size_t)min(max(uy, 0), Nw - 1) * N];
                }
            } else {
#pragma unroll
                for (int q = 0; q < kObjRows; ++q) {
                    in[c][q] = false;
                    w[c][q] = make_float2(0.f, 0.f);
                }
            }
        }
#pragma unroll
        for (int c = 0; c < kObjChunk; ++c)
#pragma unroll
            for (int q = 0; q < kObjRows; ++q) {
                acc[q] = cadd(acc[q], in[c][q] ? w[c][q] : make_float2(0.f, 0.f));
                any[q] = any[q] || in[c][q];
            }
    }
    if (xx >= sc.bx0 + sc.bw) return;
    float2 gv[kObjRows];
#pragma unroll
    for (int q = 0; q < kObjRows; ++q) gv[q] = ldg(sc.gO, (size_t)min(yb + q, sc.by0 + sc.bh - 1) * sc.Mx + xx);
#pragma unroll
    for (int q = 0; q < kObjRows; ++q) {
        const int yy = yb + q;
        if (yy < sc.by0 + sc.bh && any[q]) st_dev(sc.gO, (size_t)yy * sc.Mx + xx, cadd(gv[q], acc[q]));
    }
}

__global__ void k_fill_c64(float2* __restrict__ dst, size_t n, float2 v) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = v;
}

__global__ void k_fill_f32(float* __restrict__ dst, size_t n, float v) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = v;
}

__global__ void k_zero_c64(float2* __restrict__ dst, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = make_float2(0.f, 0.f);
}

// One block per job: out = scale * sum(in[0..n)) in a fixed order, divided by
// *div when div is given (0 when *div == 0).  With `status`, a non-finite
// result sets kStatusNonFinite, and with `first` a result above
// max(10 * *first, 1e-6) sets kStatusDiverged (the floor keeps runs that
// converge to rounding level from being flagged).
struct SumJob {
    const double* in;
    size_t n;
    const double* div;
    double* out;
    const double* first;
    unsigned* status;
};

__global__ void __launch_bounds__(256)
k_sum_jobs(const SumJob* __restrict__ jobs, double scale) {
    __shared__ double red[4];
    const SumJob jb = jobs[blockIdx.x];
    // a thread's terms in index order, loaded eight at a time (index clamped)
    double a = 0.0;
    for (size_t i0 = threadIdx.x; i0 < jb.n; i0 += 8 * 256) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = ldg(jb.in, min(i0 + (size_t)u * 256, jb.n - 1));
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (i0 + (size_t)u * 256 < jb.n) a += v[u];
    }
    a = block_sum(a, red);
    if (threadIdx.x == 0) {
        double r = a * scale;
        if (jb.div) r = *jb.div > 0.0 ? r / *jb.div : 0.0;
        if (jb.out) *jb.out = r;
        if (jb.status) {
            if (!isfinite(r)) atomicOr(jb.status, kStatusNonFinite);
            else if (jb.first && r > fmax(10.0 * *jb.first, 1e-6)) atomicOr(jb.status, kStatusDiverged);
        }
    }
}

// Sets kStatusNonFinite when any of the n complex values is not finite.
__global__ void __launch_bounds__(256)
k_check_finite(const float2* __restrict__ a, size_t n, unsigned* __restrict__ status) {
    bool bad = false;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        const float2 v = ldg(a, i);
        bad |= !isfinite(v.x) || !isfinite(v.y);
    }
    if (__ballot(bad) != 0ull && (threadIdx.x & 63) == 0) atomicOr(status, kStatusNonFinite);
}

// Amplitudes of the fused intensities in FFT order (the detector-centred
// patterns shifted by N/2 along both axes):
//   A[j][ky][kx] = sqrt(max(I[j][(ky + N/2) mod N][(kx + N/2) mod N], 0)).
// grid (N, J), min(N, 256) threads: block (ky, j) owns row ky of pattern j,
// so the source row is one value per block and no thread divides by N.
// A non-finite intensity sets kStatusNonFinite (its amplitude becomes 0).
__global__ void __launch_bounds__(256)
k_amplitude_prep(const float* __restrict__ I, int N, float* __restrict__ A, unsigned* __restrict__ status) {
    const int ky = blockIdx.x;
    const int sy = ky + N / 2 < N ? ky + N / 2 : ky - N / 2;
    const size_t base = (size_t)blockIdx.y * N * N;
    const float* src = I + base + (size_t)sy * N;
    float* dst = A + base + (size_t)ky * N;
    bool bad = false;
    for (int kx = threadIdx.x; kx < N; kx += blockDim.x) {
        const int sx = kx + N / 2 < N ? kx + N / 2 : kx - N / 2;
        const float v = src[sx];
        bad |= !isfinite(v);
        dst[kx] = amplitude_of(v);
    }
    if (__ballot(bad) != 0ull && (threadIdx.x & 63) == 0) atomicOr(status, kStatusNonFinite);
}

// part[j] = sum_q max(I[j][q], 0) (the squared amplitudes), one block per position.
__global__ void __launch_bounds__(256)
k_sum_amplitude2(const float* __restrict__ I, size_t npix, double* __restrict__ part) {
    __shared__ double red[4];
    const float* Ij = I + (size_t)blockIdx.x * npix;
    double a = 0.0;
    for (size_t i0 = threadIdx.x; i0 < npix; i0 += 8 * 256) {
        float v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = Ij[min(i0 + (size_t)u * 256, npix - 1)];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (i0 + (size_t)u * 256 < npix) a += (double)fmaxf(v[u], 0.f);
    }
    a = block_sum(a, red);
    if (threadIdx.x == 0) part[blockIdx.x] = a;
}

}  // namespace mnf
