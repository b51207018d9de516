// Context lifetime, error messages, scratch arenas and host staging.
#include <cmath>
#include <cstring>

#include "common.hpp"
#include "tables.hpp"

namespace mnf {

// message of the last failed call made without a context on this thread
// (mnf_create, ptycho_plan_info), read with mnf_last_error(NULL)
static thread_local std::string g_host_error;

void set_host_error(const std::string& msg) { g_host_error = msg; }

int set_error(mnf_ctx* ctx, int code, const char* fmt, ...) {
    if (ctx) {
        char buf[1024];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        ctx->err = buf;
    }
    return code;
}

int scratch(mnf_ctx* ctx, const char* name, size_t bytes, void** out) {
    if (bytes == 0) bytes = 256;
    if (ctx->arena) {
        // 256-byte aligned pieces of the static scratch, in request order
        MnfArena& a = *ctx->arena;
        const size_t off = (a.used + 255) & ~(size_t)255;
        if (off > a.cap || bytes > a.cap - off)
            return set_error(ctx, MNF_EINVAL,
                             "scratch '%s': this call needs more than the %zu bytes of static scratch (%zu used, "
                             "%zu more requested)", name, a.cap, off, bytes);
        *out = a.base + off;
        a.used = off + bytes;
        return MNF_OK;
    }
    auto it = ctx->scratch.find(name);
    if (it != ctx->scratch.end() && it->second.second >= bytes) {
        *out = it->second.first;
        return MNF_OK;
    }
    if (it != ctx->scratch.end()) {
        // the old buffer may still be read by queued work
        MNF_HIP(ctx, hipDeviceSynchronize());
        MNF_HIP(ctx, hipFree(it->second.first));
        ctx->scratch.erase(it);
    }
    size_t cap = bytes + bytes / 4;  // headroom against small regrowths
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, cap);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return set_error(ctx, MNF_ENOMEM, "scratch '%s': hipMalloc(%zu) failed: %s", name, cap,
                         hipGetErrorString(e));
    }
    ctx->scratch[name] = {p, cap};
    *out = p;
    return MNF_OK;
}

int upload(mnf_ctx* ctx, const char* name, const void* host, size_t bytes, hipStream_t stream,
           void** dev_out) {
    MNF_TRY(scratch(ctx, name, bytes, dev_out));
    if (bytes == 0) return MNF_OK;
    if (ctx->arena) {
        // no pinned staging: a copy from pageable memory, which the runtime
        // stages before returning (so the host array may go out of scope)
        MNF_HIP(ctx, hipMemcpyAsync(*dev_out, host, bytes, hipMemcpyHostToDevice, stream));
        return MNF_OK;
    }
    // the previous staged copy must have left the pinned buffer
    if (ctx->pinned_done) MNF_HIP(ctx, hipEventSynchronize(ctx->pinned_done));
    if (ctx->pinned_size < bytes) {
        if (ctx->pinned) MNF_HIP(ctx, hipHostFree(ctx->pinned));
        ctx->pinned = nullptr;
        size_t cap = bytes < (1u << 20) ? (1u << 20) : bytes + bytes / 4;
        MNF_HIP(ctx, hipHostMalloc(&ctx->pinned, cap, hipHostMallocDefault));
        ctx->pinned_size = cap;
    }
    std::memcpy(ctx->pinned, host, bytes);
    MNF_HIP(ctx, hipMemcpyAsync(*dev_out, ctx->pinned, bytes, hipMemcpyHostToDevice, stream));
    if (!ctx->pinned_done) MNF_HIP(ctx, hipEventCreateWithFlags(&ctx->pinned_done, hipEventDisableTiming));
    MNF_HIP(ctx, hipEventRecord(ctx->pinned_done, stream));
    return MNF_OK;
}

int twiddles(mnf_ctx* ctx, int N, const float2** out) {
    auto it = ctx->twiddles.find(N);
    if (it != ctx->twiddles.end()) {
        *out = it->second;
        return MNF_OK;
    }
    std::vector<float2> h(N);
    for (int n = 0; n < N; ++n) {
        // exact for the multiples of pi/4 through sincos of a reduced angle
        double a = -2.0 * M_PI * (double)n / (double)N;
        h[n] = make_float2((float)std::cos(a), (float)std::sin(a));
    }
    float2* d = nullptr;
    MNF_HIP(ctx, hipMalloc(&d, sizeof(float2) * N));
    MNF_HIP(ctx, hipMemcpy(d, h.data(), sizeof(float2) * N, hipMemcpyHostToDevice));
    ctx->twiddles[N] = d;
    *out = d;
    return MNF_OK;
}

static int prof_event(mnf_ctx* ctx, hipEvent_t* e) {
    if (!ctx->prof.pool.empty()) {
        *e = ctx->prof.pool.back();
        ctx->prof.pool.pop_back();
        return MNF_OK;
    }
    MNF_HIP(ctx, hipEventCreate(e));
    return MNF_OK;
}

int prof_pair(mnf_ctx* ctx, hipEvent_t* e0, hipEvent_t* e1) {
    MNF_TRY(prof_event(ctx, e0));
    MNF_TRY(prof_event(ctx, e1));
    return MNF_OK;
}

void prof_push(mnf_ctx* ctx, int cls, hipEvent_t e0, hipEvent_t e1) { ctx->prof.pending.push_back({cls, e0, e1}); }

static int prof_drain(mnf_ctx* ctx) {
    for (auto& p : ctx->prof.pending) {
        MNF_HIP(ctx, hipEventSynchronize(p.b));
        float ms = 0.f;
        MNF_HIP(ctx, hipEventElapsedTime(&ms, p.a, p.b));
        ctx->prof.launches[p.cls] += 1;
        ctx->prof.ms[p.cls] += ms;
        ctx->prof.pool.push_back(p.a);
        ctx->prof.pool.push_back(p.b);
    }
    ctx->prof.pending.clear();
    return MNF_OK;
}

}  // namespace mnf

extern "C" {

static const char* kClassNames[MNF_K_NCLASS] = {
    "rows_fwd", "cols_modulus", "rows_inv", "probe_update", "object_update",
    "small", "fuse", "forward", "grad_cols", "grad_scatter", "shift", "small_run"};

int mnf_profile(mnf_ctx* ctx, uint32_t class_mask) {
    MNF_TRY(mnf::begin(ctx));
    ctx->prof.mask = class_mask;
    ctx->prof.period = 1;
    return MNF_OK;
}

int mnf_profile_sampled(mnf_ctx* ctx, uint32_t class_mask, int period) {
    MNF_TRY(mnf::begin(ctx));
    if (period < 1) return mnf::set_error(ctx, MNF_EINVAL, "sampling period %d (must be >= 1)", period);
    ctx->prof.mask = class_mask;
    ctx->prof.period = period;
    return MNF_OK;
}

int mnf_profile_read(mnf_ctx* ctx, int cls, long long* launches, double* total_ms) {
    MNF_TRY(mnf::begin(ctx));
    if (cls < 0 || cls >= MNF_K_NCLASS) return mnf::set_error(ctx, MNF_EINVAL, "kernel class %d", cls);
    MNF_TRY(mnf::prof_drain(ctx));
    if (launches) *launches = ctx->prof.launches[cls];
    if (total_ms) *total_ms = ctx->prof.ms[cls];
    return MNF_OK;
}

int mnf_profile_reset(mnf_ctx* ctx) {
    MNF_TRY(mnf::begin(ctx));
    MNF_TRY(mnf::prof_drain(ctx));
    for (int i = 0; i < MNF_K_NCLASS; ++i) {
        ctx->prof.launches[i] = 0;
        ctx->prof.ms[i] = 0.0;
        ctx->prof.seen[i] = 0;
    }
    return MNF_OK;
}

const char* mnf_kernel_class_name(int cls) {
    return (cls >= 0 && cls < MNF_K_NCLASS) ? kClassNames[cls] : "";
}

static int create_failed(int code, const std::string& msg) {
    mnf::set_host_error(msg);
    return code;
}

int mnf_create(mnf_ctx** out, int hip_device) {
    if (!out) return create_failed(MNF_EINVAL, "null output pointer");
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || hip_device < 0 || hip_device >= n) {
        (void)hipGetLastError();
        return create_failed(MNF_EINVAL, "no HIP device " + std::to_string(hip_device));
    }
    hipError_t e = hipSetDevice(hip_device);
    if (e != hipSuccess) return create_failed(MNF_EHIP, std::string("hipSetDevice: ") + hipGetErrorString(e));
    mnf_ctx* c = new mnf_ctx();
    c->device = hip_device;
    e = hipMalloc(&c->d_status, 256);
    if (e == hipSuccess) e = hipMemset(c->d_status, 0, 256);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        mnf_destroy(c);
        return create_failed(MNF_ENOMEM, std::string("status word: ") + hipGetErrorString(e));
    }
    // twiddle tables of every supported size up front, so that no later call
    // needs to allocate one; the static scratch's device address
    int32_t sizes[16];
    const int ns = mnf_supported_sizes(sizes, 16);
    for (int i = 0; i < ns; ++i) {
        const float2* tw;
        const int rc = mnf::twiddles(c, sizes[i], &tw);
        if (rc != MNF_OK) {
            const std::string msg = "twiddle table: " + c->err;
            mnf_destroy(c);
            return create_failed(rc, msg);
        }
    }
    const int rc = mnf::noalloc_setup(c);
    if (rc != MNF_OK) {
        const std::string msg = "static scratch: " + c->err;
        mnf_destroy(c);
        return create_failed(rc, msg);
    }
    mnf::set_host_error(std::string());
    *out = c;
    return MNF_OK;
}

int mnf_status(mnf_ctx* ctx, void* stream) {
    MNF_TRY(mnf::begin(ctx));
    MNF_HIP(ctx, hipStreamSynchronize((hipStream_t)stream));
    unsigned h = 0;
    MNF_HIP(ctx, hipMemcpy(&h, ctx->d_status, sizeof h, hipMemcpyDeviceToHost));
    if (h == 0) return MNF_OK;
    MNF_HIP(ctx, hipMemset(ctx->d_status, 0, sizeof h));
    if (h & mnf::kStatusNonFinite)
        return mnf::set_error(ctx, MNF_ENONFINITE, "a non-finite error, loss, object or probe value was produced");
    return mnf::set_error(ctx, MNF_EDIVERGED, "the Fourier error grew above 10x its first value within one call");
}

void mnf_destroy(mnf_ctx* ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    for (auto& kv : ctx->scratch) (void)hipFree(kv.second.first);
    for (auto& kv : ctx->twiddles) (void)hipFree(kv.second);
    for (auto& p : ctx->prof.pending) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    for (auto e : ctx->prof.pool) (void)hipEventDestroy(e);
    if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
    if (ctx->capture_stream) (void)hipStreamDestroy(ctx->capture_stream);
    for (auto s : ctx->class_streams) (void)hipStreamDestroy(s);
    for (auto e : ctx->class_events) (void)hipEventDestroy(e);
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    if (ctx->pinned_done) (void)hipEventDestroy(ctx->pinned_done);
    if (ctx->d_status) (void)hipFree(ctx->d_status);
    delete ctx;
}

const char* mnf_last_error(const mnf_ctx* ctx) { return ctx ? ctx->err.c_str() : mnf::g_host_error.c_str(); }

}  // extern "C"
