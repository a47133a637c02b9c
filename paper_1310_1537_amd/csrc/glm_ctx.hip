// Context, data-set registry, per-stream scratch and error reporting.
#include "runtime.hpp"

#include <chrono>
#include <cstdlib>
#include <cstring>

namespace glmrt {

static thread_local char t_err[512] = "";

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(t_err, sizeof(t_err), fmt, ap);
    va_end(ap);
}

void clear_error() { t_err[0] = 0; }

glm_status validate_desc(const glm_dataset_desc& dd) {
    const glm_dataset_desc* d = &dd;
    const int es = elem_size(d->dtype);
    if (!es) GLM_FAIL(GLM_EDTYPE, "data set: unknown dtype %d", d->dtype);
    if (d->N < 0) GLM_FAIL(GLM_EINVAL, "data set: N = %lld < 0", (long long)d->N);
    if (d->K < 1 || d->K > GLM_K_MAX)
        GLM_FAIL(GLM_EINVAL, "data set: K = %d outside [1, %d]", d->K, GLM_K_MAX);
    if (d->ldx < d->K)
        GLM_FAIL(GLM_EINVAL, "data set: ldx = %lld < K = %d", (long long)d->ldx, d->K);
    if (d->N > 0 && (!d->X || !d->y)) GLM_FAIL(GLM_EINVAL, "data set: X or y is NULL");
    if (d->X && ((uintptr_t)d->X % es))
        GLM_FAIL(GLM_EINVAL, "data set: X not aligned to its %d-byte element", es);
    if (d->family != GLM_LOGISTIC && d->family != GLM_POISSON)
        GLM_FAIL(GLM_EINVAL, "data set: unknown response family %d", d->family);
    if (d->dtype == GLM_FP8_E4M3 && !d->col_scale)
        GLM_FAIL(GLM_EINVAL, "data set: FP8 data needs col_scale");
    if (d->dtype != GLM_FP8_E4M3 && d->col_scale)
        GLM_FAIL(GLM_EINVAL, "data set: col_scale is only for FP8 data");
    return GLM_OK;
}

namespace {
std::mutex g_tune_mu;
std::map<std::string, TuneEntry> g_tune;
bool g_tune_loaded = false;

void tune_load_locked() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char* path = std::getenv("GLM_TUNE_CACHE");
    if (!path) return;
    FILE* f = std::fopen(path, "r");
    if (!f) return;
    char key[512];
    long long a;
    int b;
    double us;
    while (std::fscanf(f, "%511s %lld %d %lf", key, &a, &b, &us) == 4) g_tune[key] = TuneEntry{a, b, us};
    std::fclose(f);
}
}  // namespace

bool tune_cache_get(const std::string& key, TuneEntry* e) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_load_locked();
    auto it = g_tune.find(key);
    if (it == g_tune.end()) return false;
    *e = it->second;
    return true;
}

void tune_cache_put(const std::string& key, const TuneEntry& e) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_load_locked();
    g_tune[key] = e;
    const char* path = std::getenv("GLM_TUNE_CACHE");
    if (!path) return;
    FILE* f = std::fopen(path, "w");
    if (!f) return;
    for (auto& kv : g_tune)
        std::fprintf(f, "%s %lld %d %.3f\n", kv.first.c_str(), (long long)kv.second.a, kv.second.b,
                     kv.second.us);
    std::fclose(f);
}

glm_status use_device(glm_ctx* ctx) {
    GLM_HIP_CHECK(hipSetDevice(ctx->device));
    return GLM_OK;
}

// Tickets must start at zero; a fill kernel keeps the scratch set-up free of
// memset nodes if the caller captures the first call into a graph.
__global__ void fill_u32(unsigned* p, size_t n, unsigned v) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

glm_status get_scratch(glm_ctx* ctx, void* stream, size_t n_partials, size_t n_gpart,
                       size_t n_counters, Scratch** out) {
    Scratch& s = ctx->scratch[stream];
    if (s.base && s.cap_partials >= n_partials && s.cap_gpart >= n_gpart &&
        s.cap_counters >= n_counters) {
        *out = &s;
        return GLM_OK;
    }
    // grow with headroom
    size_t np = std::max(n_partials, s.cap_partials) * 5 / 4 + 1024;
    size_t ng = std::max(n_gpart, s.cap_gpart) * 5 / 4 + 1024;
    size_t nc = std::max(n_counters, s.cap_counters) * 5 / 4 + 64;
    size_t bytes = (np + ng) * sizeof(double) + nc * sizeof(unsigned);
    if (s.base) {
        // earlier launches on any stream may still use the old buffer
        GLM_HIP_CHECK(hipDeviceSynchronize());
        GLM_HIP_CHECK(hipFree(s.base));
        s = Scratch{};
    }
    void* base = nullptr;
    hipError_t e = hipMalloc(&base, bytes);
    if (e != hipSuccess) GLM_FAIL(GLM_ENOMEM, "scratch allocation of %zu bytes failed: %s", bytes,
                                  hipGetErrorString(e));
    s.base = base;
    s.bytes = bytes;
    s.partials = (double*)base;
    s.gpart = s.partials + np;
    s.counters = (unsigned*)(s.gpart + ng);
    s.cap_partials = np;
    s.cap_gpart = ng;
    s.cap_counters = nc;
    hipLaunchKernelGGL(fill_u32, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0,
                       (hipStream_t)stream, s.counters, nc, 0u);
    GLM_HIP_CHECK(hipGetLastError());
    *out = &s;
    return GLM_OK;
}

}  // namespace glmrt

using namespace glmrt;

extern "C" {

const char* glm_last_error(void) { return t_err; }

glm_status glm_create(int device, glm_ctx** out) {
    clear_error();
    if (!out) GLM_FAIL(GLM_EINVAL, "glm_create: out is NULL");
    *out = nullptr;
    int n = 0;
    GLM_HIP_CHECK(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) GLM_FAIL(GLM_EINVAL, "glm_create: device %d of %d", device, n);
    GLM_HIP_CHECK(hipSetDevice(device));
    hipDeviceProp_t prop;
    GLM_HIP_CHECK(hipGetDeviceProperties(&prop, device));
    std::unique_ptr<glm_ctx> c(new glm_ctx);
    c->device = device;
    c->num_cu = prop.multiProcessorCount;
    c->arch = prop.gcnArchName;
    glm_status st = static_scratch_setup(device);
    if (st != GLM_OK) return st;
    GLM_HIP_CHECK(hipStreamCreateWithFlags(&c->own_stream, hipStreamNonBlocking));
    *out = c.release();
    return GLM_OK;
}

glm_status glm_destroy(glm_ctx* ctx) {
    clear_error();
    if (!ctx) return GLM_OK;
    // every release is attempted; the first failure is reported
    hipError_t first = hipSuccess;
    const char* what = nullptr;
    auto note = [&](hipError_t e, const char* call) {
        if (e != hipSuccess && first == hipSuccess) {
            first = e;
            what = call;
        }
    };
    note(hipSetDevice(ctx->device), "hipSetDevice");
    note(hipDeviceSynchronize(), "hipDeviceSynchronize");
    for (auto& kv : ctx->scratch)
        if (kv.second.base) note(hipFree(kv.second.base), "hipFree(scratch)");
    for (auto& kv : ctx->sampler)
        if (kv.second.buf) note(hipFree(kv.second.buf), "hipFree(sampler)");
    for (auto& kv : ctx->hess)
        if (kv.second.buf) note(hipFree(kv.second.buf), "hipFree(hessian)");
    if (ctx->h_stage) note(hipHostFree(ctx->h_stage), "hipHostFree(stage)");
    if (ctx->d_stage) note(hipFree(ctx->d_stage), "hipFree(stage)");
    if (ctx->own_stream) note(hipStreamDestroy(ctx->own_stream), "hipStreamDestroy");
    delete ctx;
    if (first != hipSuccess)
        GLM_FAIL(GLM_EHIP, "glm_destroy: %s: %s", what, hipGetErrorString(first));
    return GLM_OK;
}

glm_status glm_set_option(glm_ctx* ctx, int32_t option, int64_t value) {
    clear_error();
    if (!ctx) GLM_FAIL(GLM_EINVAL, "glm_set_option: NULL context");
    std::lock_guard<std::mutex> lk(ctx->mu);
    switch (option) {
    case GLM_OPT_BLOCKS_PER_CU:
        if (value < 1 || value > 8) GLM_FAIL(GLM_EINVAL, "glm_set_option: blocks per CU %lld outside [1, 8]", (long long)value);
        ctx->blocks_per_cu = (int)value;
        return GLM_OK;
    case GLM_OPT_INTERLEAVE:
    case GLM_OPT_MATRIX_CORES:
        if (value != 0 && value != 1) GLM_FAIL(GLM_EINVAL, "glm_set_option: option %d takes 0 or 1, not %lld", option, (long long)value);
        (option == GLM_OPT_INTERLEAVE ? ctx->interleave : ctx->matrix_cores) = value != 0;
        return GLM_OK;
    }
    GLM_FAIL(GLM_EINVAL, "glm_set_option: unknown option %d", option);
}

glm_status glm_get_option(glm_ctx* ctx, int32_t option, int64_t* value) {
    clear_error();
    if (!ctx || !value) GLM_FAIL(GLM_EINVAL, "glm_get_option: NULL argument");
    std::lock_guard<std::mutex> lk(ctx->mu);
    switch (option) {
    case GLM_OPT_BLOCKS_PER_CU: *value = ctx->blocks_per_cu; return GLM_OK;
    case GLM_OPT_INTERLEAVE: *value = ctx->interleave ? 1 : 0; return GLM_OK;
    case GLM_OPT_MATRIX_CORES: *value = ctx->matrix_cores ? 1 : 0; return GLM_OK;
    }
    GLM_FAIL(GLM_EINVAL, "glm_get_option: unknown option %d", option);
}

glm_status glm_dataset_register(glm_ctx* ctx, const glm_dataset_desc* d, glm_dataset_id* out) {
    clear_error();
    if (!ctx || !d || !out) GLM_FAIL(GLM_EINVAL, "glm_dataset_register: NULL argument");
    glm_status vs = validate_desc(*d);
    if (vs != GLM_OK) return vs;
    std::lock_guard<std::mutex> lk(ctx->mu);
    Dataset ds;
    ds.d = *d;
    glm_status st = make_plan(ctx, *d, &ds.plan);
    if (st != GLM_OK) return st;
    const int64_t id = ctx->next_id++;
    ctx->datasets[id] = ds;
    *out = id;
    return GLM_OK;
}

__global__ void k_empty() {}

glm_status glm_probe_roundtrip(glm_ctx* ctx, int32_t K, int32_t iters, double* us) {
    clear_error();
    if (!ctx || !us || K < 1 || iters < 1) GLM_FAIL(GLM_EINVAL, "glm_probe_roundtrip: bad argument");
    std::lock_guard<std::mutex> lk(ctx->mu);
    glm_status st = use_device(ctx);
    if (st != GLM_OK) return st;
    double* h = nullptr;
    double* d = nullptr;
    GLM_HIP_CHECK(hipHostMalloc((void**)&h, (K + 1) * sizeof(double)));
    if (hipMalloc((void**)&d, (K + 1) * sizeof(double)) != hipSuccess) {
        (void)hipHostFree(h);
        GLM_FAIL(GLM_ENOMEM, "glm_probe_roundtrip: device allocation failed");
    }
    for (int k = 0; k <= K; ++k) h[k] = 0.0;
    hipStream_t s = ctx->own_stream;
    hipError_t e = hipSuccess;
    auto t0 = std::chrono::steady_clock::now();
    for (int i = 0; i < iters && e == hipSuccess; ++i) {
        e = hipMemcpyAsync(d, h, K * sizeof(double), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_empty, dim3(1), dim3(1), 0, s);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipMemcpyAsync(h + K, d + K, sizeof(double), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
    }
    auto t1 = std::chrono::steady_clock::now();
    (void)hipFree(d);
    (void)hipHostFree(h);
    if (e != hipSuccess) GLM_FAIL(GLM_EHIP, "glm_probe_roundtrip: %s", hipGetErrorString(e));
    *us = std::chrono::duration<double, std::micro>(t1 - t0).count() / iters;
    return GLM_OK;
}

// Pure streaming read: every lane reads 16-byte words at a grid stride with
// eight loads in flight and folds them into a register; a lane writes its fold
// only in the (data-dependent, practically never taken) all-ones case, which
// keeps the loads alive without adding traffic.
typedef unsigned int probe_u32x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_read_probe(const probe_u32x4* __restrict__ p, int64_t n,
                                                    unsigned* __restrict__ sink) {
    const int64_t stride = (int64_t)gridDim.x * 256;
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    probe_u32x4 acc = {0u, 0u, 0u, 0u};
    for (; i + 7 * stride < n; i += 8 * stride) {
        probe_u32x4 v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = __builtin_nontemporal_load(p + i + j * stride);
#pragma unroll
        for (int j = 0; j < 8; ++j) acc ^= v[j];
    }
    for (; i < n; i += stride) acc ^= __builtin_nontemporal_load(p + i);
    if ((acc.x & acc.y & acc.z & acc.w) == 0xFFFFFFFFu)
        sink[(int64_t)blockIdx.x * 256 + threadIdx.x] = acc.x ^ acc.y;
}

glm_status glm_probe_read_bandwidth(glm_ctx* ctx, const void* buf, int64_t bytes,
                                    int32_t blocks_per_cu, int32_t iters, double* gbps) {
    clear_error();
    if (!ctx || !buf || !gbps || bytes < 16 || blocks_per_cu < 1 || blocks_per_cu > 16 || iters < 1)
        GLM_FAIL(GLM_EINVAL, "glm_probe_read_bandwidth: bad argument");
    if ((uintptr_t)buf % 16) GLM_FAIL(GLM_EINVAL, "glm_probe_read_bandwidth: buffer not 16-byte aligned");
    std::lock_guard<std::mutex> lk(ctx->mu);
    glm_status st = use_device(ctx);
    if (st != GLM_OK) return st;
    const int blocks = ctx->num_cu * blocks_per_cu;
    const int64_t n = bytes / 16;
    unsigned* sink = nullptr;
    if (hipMalloc((void**)&sink, (size_t)blocks * 256 * sizeof(unsigned)) != hipSuccess)
        GLM_FAIL(GLM_ENOMEM, "glm_probe_read_bandwidth: device allocation failed");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    hipStream_t s = ctx->own_stream;
    // one untimed pass, then iters timed passes
    for (int it = -1; it < iters && e == hipSuccess; ++it) {
        if (it == 0) e = hipEventRecord(e0, s);
        if (e != hipSuccess) break;
        hipLaunchKernelGGL(k_read_probe, dim3(blocks), dim3(256), 0, s,
                           (const probe_u32x4*)buf, n, sink);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(sink);
    if (e != hipSuccess) GLM_FAIL(GLM_EHIP, "glm_probe_read_bandwidth: %s", hipGetErrorString(e));
    *gbps = (double)n * 16.0 * iters / (ms * 1e-3) / 1e9;
    return GLM_OK;
}

glm_status glm_dataset_unregister(glm_ctx* ctx, glm_dataset_id id) {
    clear_error();
    if (!ctx) GLM_FAIL(GLM_EINVAL, "glm_dataset_unregister: ctx is NULL");
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (!ctx->datasets.erase(id)) GLM_FAIL(GLM_ENOTFOUND, "glm_dataset_unregister: unknown id %lld",
                                           (long long)id);
    return GLM_OK;
}

}  // extern "C"
