// Shared host/device helpers of libmnfpty: context, error plumbing, scratch.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <map>
#include <string>
#include <vector>

#include "../../include/mnfpty.h"

// Kernel classes for launch timing (see mnf_profile in the public header).
enum MnfKernelClass {
    MNF_K_ROWS_FWD = 0,   // gather + row transforms
    MNF_K_COLS_MODULUS,   // column transforms + modulus projection + inverse column transforms
    MNF_K_ROWS_INV,       // inverse row transforms + exit-wave difference
    MNF_K_PROBE_UPDATE,
    MNF_K_OBJECT_UPDATE,
    MNF_K_SMALL,          // copies, reductions
    MNF_K_FUSE,           // fusion kernels
    MNF_K_FORWARD,        // forward-model column pass
    MNF_K_GRAD_COLS,      // gradient column pass
    MNF_K_GRAD_SCATTER,   // gradient object/probe scatter
    MNF_K_SHIFT,          // Fourier translation of probes (real positions)
    MNF_K_SMALL_RUN,      // a whole mini-batch-of-one run in one workgroup
    MNF_K_NCLASS
};

struct MnfProfile {
    uint32_t mask = 0;
    int period = 1;                          // time every period-th launch of a class
    long long seen[MNF_K_NCLASS] = {};       // launches of each class since the last reset
    std::vector<hipEvent_t> pool;
    struct Pending { int cls; hipEvent_t a, b; };
    std::vector<Pending> pending;
    long long launches[MNF_K_NCLASS] = {};
    double ms[MNF_K_NCLASS] = {};
};

// Bump allocator over caller-free memory (the library's static scratch):
// while a context has one set, scratch buffers and staged host copies come
// from it instead of device allocations.
struct MnfArena {
    char* base = nullptr;
    size_t cap = 0;
    size_t used = 0;
};

struct mnf_ctx {
    int device = 0;
    MnfProfile prof;
    std::string err;
    // named device scratch buffers, grown on demand and reused across calls
    std::map<std::string, std::pair<void*, size_t>> scratch;
    // unitary FFT twiddles exp(-2 pi i n / N), n < N, one table per N (float2 on device)
    std::map<int, float2*> twiddles;
    // pinned staging for host -> device copies of small host arrays
    void* pinned = nullptr;
    size_t pinned_size = 0;
    hipEvent_t pinned_done = nullptr;
    // launch-shape variant per detector size: bit 0 rows, bit 1 columns (0 = defaults)
    std::map<int, int> variant;
    // stream used to capture graphs; the last instantiated graph and the key
    // of the launch sequence it holds (a call whose sequence hashes to the same
    // key replays it instead of capturing again)
    hipStream_t capture_stream = nullptr;
    // one stream per detector-size class of a many-scan call (forked from and
    // joined to the call's stream by events) and the fork / join events
    std::vector<hipStream_t> class_streams;
    std::vector<hipEvent_t> class_events;  // [0] fork, [1 + c] class c's join
    hipGraphExec_t graph_exec = nullptr;
    uint64_t graph_key = 0;
    // status bits set by kernels (non-finite values, divergence), read and
    // cleared by mnf_status
    unsigned* d_status = nullptr;
    // device address of this device's static scratch (see ptycho_iterate_noalloc)
    void* noalloc_ptr = nullptr;
    // set only for the duration of a call that must not allocate
    MnfArena* arena = nullptr;
};

namespace mnf {

int set_error(mnf_ctx* ctx, int code, const char* fmt, ...);
// the message mnf_last_error(NULL) returns (calls made without a context)
void set_host_error(const std::string& msg);

#define MNF_HIP(ctx, call)                                                          \
    do {                                                                            \
        hipError_t e_ = (call);                                                     \
        if (e_ != hipSuccess)                                                       \
            return ::mnf::set_error((ctx), MNF_EHIP, "%s failed: %s", #call,        \
                                    hipGetErrorString(e_));                         \
    } while (0)

#define MNF_TRY(expr)             \
    do {                          \
        int r_ = (expr);          \
        if (r_ != MNF_OK) return r_; \
    } while (0)

#define MNF_CHECK_LAUNCH(ctx) MNF_HIP(ctx, hipGetLastError())

// Device scratch buffer `name` of at least `bytes`; *out receives its address.
int scratch(mnf_ctx* ctx, const char* name, size_t bytes, void** out);

// Copy `bytes` of host memory into device scratch `name` on `stream`.  The
// host array may be reused as soon as this returns.
int upload(mnf_ctx* ctx, const char* name, const void* host, size_t bytes,
           hipStream_t stream, void** dev_out);

// Device twiddle table for length N (computed in float64, rounded to float).
int twiddles(mnf_ctx* ctx, int N, const float2** out);

// Device address of the static scratch array of the context's device
// (defined beside ptycho_iterate_noalloc); called once per context at creation.
int noalloc_setup(mnf_ctx* ctx);

// Launch timing: a pair of timing events for one launch of class `cls`,
// passed to the launch itself (hipExtLaunchKernel records them at the start
// and the end of that kernel's execution, so the interval excludes the
// queue's dispatch gaps), then queued until read.
int prof_pair(mnf_ctx* ctx, hipEvent_t* e0, hipEvent_t* e1);
void prof_push(mnf_ctx* ctx, int cls, hipEvent_t e0, hipEvent_t e1);

// Whether this launch of class `cls` is one to time (every period-th one,
// the first included).
inline bool prof_take(mnf_ctx* ctx, int cls) {
    if (!(ctx->prof.mask & (1u << cls))) return false;
    return ctx->prof.seen[cls]++ % ctx->prof.period == 0;
}

#define MNF_LAUNCH(ctx, cls, st, kernel, grid, block, ...)                                   \
    do {                                                                                     \
        if (::mnf::prof_take((ctx), (cls))) {                                                \
            hipEvent_t e0_ = nullptr, e1_ = nullptr;                                         \
            MNF_TRY(::mnf::prof_pair((ctx), &e0_, &e1_));                                    \
            hipExtLaunchKernelGGL(kernel, grid, block, 0, st, e0_, e1_, 0, __VA_ARGS__);     \
            ::mnf::prof_push((ctx), (cls), e0_, e1_);                                        \
        } else {                                                                             \
            hipLaunchKernelGGL(kernel, grid, block, 0, st, __VA_ARGS__);                     \
        }                                                                                    \
    } while (0)

// 64-bit hash of byte ranges (FNV-1a over 8-byte words plus a final mix),
// for keys of cached launch sequences.
struct KeyHash {
    uint64_t h = 1469598103934665603ull;
    void add(const void* p, size_t n) {
        const unsigned char* b = (const unsigned char*)p;
        size_t i = 0;
        for (; i + 8 <= n; i += 8) {
            uint64_t w;
            __builtin_memcpy(&w, b + i, 8);
            h = (h ^ w) * 1099511628211ull;
        }
        for (; i < n; ++i) h = (h ^ b[i]) * 1099511628211ull;
    }
    template <class T>
    void add(const T& v) { add(&v, sizeof v); }
    template <class T>
    void add_vec(const std::vector<T>& v) {
        const size_t n = v.size();
        add(n);
        if (n) add(v.data(), n * sizeof(T));
    }
    uint64_t value() const {
        uint64_t x = h;
        x ^= x >> 33;
        x *= 0xff51afd7ed558ccdull;
        x ^= x >> 33;
        return x ? x : 1;
    }
};

inline int begin(mnf_ctx* ctx) {
    if (!ctx) return MNF_EINVAL;
    ctx->err.clear();
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess)
        return set_error(ctx, MNF_EHIP, "hipSetDevice(%d) failed: %s", ctx->device,
                         hipGetErrorString(e));
    return MNF_OK;
}

}  // namespace mnf
