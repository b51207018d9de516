// Device descriptor tables shared by the pattern and update kernels.
//
// A launch of a pattern pass processes a list of slots; a slot is one scan
// position of one scan.  Slots of the same scan that form one mini-batch are
// contiguous and described by a group.  One launch can thus cover the
// current mini-batch of many independent scans of the same detector size.
#pragma once

#include <hip/hip_runtime.h>

namespace mnf {

// Status bits of a context, set on the device and read by mnf_status.
constexpr unsigned kStatusNonFinite = 1u;  // a non-finite error, loss, object or probe value
constexpr unsigned kStatusDiverged = 2u;   // an iteration's error above 10x the call's first one

struct ScanDev {
    float2* O;           // [My][Mx]
    float2* P;           // [Nw][Nw]
    float* P2;           // [Nw][Nw] |P|^2 of the batch-start probe (scratch)
    float* maxP2_row;    // [Nw] per-row max of P2 (scratch)
    const float* I;      // [J][N][N] fused intensities, detector-centred
    const float* A;      // [J][N][N] amplitudes sqrt(max(I, 0)) in FFT order (scratch, reconstruction only)
    double* err_part;    // [J][N / kColGroup] error / loss partials (scratch)
    float2* gO;          // gradient outputs (gradient path only)
    float2* gP;
    unsigned* status;    // the context's status word (kStatusNonFinite for non-finite intensities)
    int My, Mx, Nw, J;
    int by0, bx0, bh, bw;  // union box of the scan's windows
    int tiles_x;           // object-update tiles per box row
    int pad_;              // explicit, so the struct has no implicit padding (hashed as bytes)
};

// Scan descriptor `idx` given entry 0 loaded up front, in parallel with the
// slot or group entry that names the scan: a launch over a single scan (the
// common case) then waits for one table load before its data loads instead
// of two dependent ones.
__device__ __forceinline__ ScanDev scan_desc(const ScanDev* __restrict__ scans, const ScanDev& first, int idx) {
    if (idx == 0) return first;
    return scans[idx];
}

struct SlotDev {
    int scan;   // index into the scan table
    int j;      // position index within the scan
    int py, px; // window corner in the scan's object
};

struct GroupDev {
    int scan;   // index into the scan table
    int s0;     // first slot of the group in the launch's slot list
    int nb;     // slots in the group (the mini-batch size, ragged at the end)
    int tile0;  // first object-update block of the group in the launch
};

static_assert(sizeof(ScanDev) == 10 * sizeof(void*) + 10 * sizeof(int), "ScanDev without implicit padding");
static_assert(sizeof(SlotDev) == 4 * sizeof(int) && sizeof(GroupDev) == 4 * sizeof(int), "tables without padding");

}  // namespace mnf
