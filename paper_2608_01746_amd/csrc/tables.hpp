// Device descriptor tables shared by the pattern and update kernels.
//
// A launch of a pattern pass processes a list of slots; a slot is one scan
// position of one scan.  Slots of the same scan that form one mini-batch are
// contiguous and described by a group.  One launch can thus cover the
// current mini-batch of many independent scans of the same detector size.
#pragma once

#include <hip/hip_runtime.h>

namespace mnf {

struct ScanDev {
    float2* O;           // [My][Mx]
    float2* P;           // [Nw][Nw]
    float* P2;           // [Nw][Nw] |P|^2 of the batch-start probe (scratch)
    float* maxP2_row;    // [Nw] per-row max of P2 (scratch)
    const float* I;      // [J][N][N] fused intensities, detector-centred
    double* err_part;    // [J][N / kColGroup] error / loss partials (scratch)
    float2* gO;          // gradient outputs (gradient path only)
    float2* gP;
    int My, Mx, Nw, J;
    int by0, bx0, bh, bw;  // union box of the scan's windows
    int tiles_x;           // object-update tiles per box row
    int pad_[3];
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

}  // namespace mnf
