// Differential update for one-coefficient-at-a-time samplers (Sec. 3.4.4).
//
// A univariate sampler (slice sampling, Gibbs over the coordinates of beta)
// changes one coefficient beta_k at a time.  Keeping u = X beta resident,
// f(beta + delta e_k) needs only column k of X, u and y:
//
//     u' = u + delta X_k,   f = sum_n [ y_n u'_n - b(u'_n) ] + prior,
//
// (b = softplus for the logistic model, exp for the Poisson one),
//
// N (size + 8 + 1) bytes instead of N (K size + 1).  Columns must be
// contiguous for that read to be a stream, so these calls work on a
// column-major copy Xt of X (a "column set"), built on the device by
// glm_transpose.
//
// Kernels:
//   k_transpose    rows -> columns through a 64 x 64 LDS tile
//   k_linpred      u = X beta, FP64 products and sums in k order
//   k_diff_eval    f(beta + delta_j e_k) for up to DMAX step sizes per pass:
//                  each row's u is read once for all of them; per-row terms
//                  in FP64; per-block FP64 partials, the last block to finish
//                  (ticket) adds them in a fixed order and the prior
//   k_diff_commit  u += delta X_k, beta_k += delta (the step's u' bit for bit)
#include <hip/hip_runtime.h>

#include <cmath>

#include "runtime.hpp"

namespace glmrt {
namespace {

constexpr int kDMax = 16;       // step sizes per pass
constexpr int kThreads = 256;

// ---------------------------------------------------------------- elements

template <int DT> struct Elem;
template <> struct Elem<GLM_F64> {
    using T = double;
    static __device__ __forceinline__ double value(T v, float) { return v; }
};
template <> struct Elem<GLM_F32> {
    using T = float;
    static __device__ __forceinline__ double value(T v, float) { return (double)v; }
};
template <> struct Elem<GLM_BF16> {
    using T = unsigned short;
    static __device__ __forceinline__ double value(T v, float) {
        return (double)__uint_as_float((unsigned)v << 16);
    }
};
template <> struct Elem<GLM_FP8_E4M3> {
    using T = unsigned char;
    static __device__ __forceinline__ double value(T v, float s) {
        // native OCP E4M3FN conversion; the code times its column scale is
        // exact in FP64
        const float x = __builtin_amdgcn_cvt_pk_f32_fp8((int)v, false)[0];
        return (double)x * (double)s;
    }
};

// t(v) = y v - b(v) with b the log-partition of the response family:
// softplus (logistic) or exp (Poisson, y a count).
__device__ __forceinline__ double row_term(double v, unsigned yb, int fam) {
    if (fam == GLM_POISSON) return (double)(yb & 0xFFu) * v - exp(v);
    return (double)(yb & 1u) * v - (fmax(v, 0.0) + log1p(exp(-fabs(v))));
}

// ---------------------------------------------------------------- transpose

template <typename T>
__global__ __launch_bounds__(256) void k_transpose(const T* __restrict__ X, int64_t ldx,
                                                   int64_t N, int K, T* __restrict__ Xt,
                                                   int64_t ldt) {
    __shared__ T tile[64][65];
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int64_t r0 = (int64_t)blockIdx.x * 64;
    const int c0 = blockIdx.y * 64;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int64_t r = r0 + ty + 4 * i;
        const int c = c0 + tx;
        if (r < N && c < K) tile[ty + 4 * i][tx] = X[r * ldx + c];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int c = c0 + ty + 4 * i;
        const int64_t r = r0 + tx;
        if (r < N && c < K) Xt[(int64_t)c * ldt + r] = tile[tx][ty + 4 * i];
    }
}

// ---------------------------------------------------------------- u = X beta

template <int DT>
__global__ __launch_bounds__(kThreads) void k_linpred(const void* __restrict__ Xt_, int64_t ldt,
                                                      const float* __restrict__ scale, int64_t N,
                                                      int K, const double* __restrict__ beta,
                                                      double* __restrict__ u) {
    using E = Elem<DT>;
    const typename E::T* Xt = static_cast<const typename E::T*>(Xt_);
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t n = (int64_t)blockIdx.x * kThreads + threadIdx.x; n < N; n += stride) {
        double acc = 0.0;
#pragma unroll 8
        for (int k = 0; k < K; ++k) {
            const float s = DT == GLM_FP8_E4M3 ? scale[k] : 1.0f;
            acc = fma(E::value(Xt[(int64_t)k * ldt + n], s), beta[k], acc);
        }
        u[n] = acc;
    }
}

// ---------------------------------------------------------------- f along e_k

struct DiffParams {
    const void* col;          // column k of Xt (N elements)
    float s;                  // its FP8 scale (1 otherwise)
    const double* u;          // N
    const uint8_t* y;         // N
    int64_t N;
    int K;
    int k;
    const double* beta;       // K
    const double* mean;       // K or nullptr
    double prec;
    const double* deltas;     // nd
    int nd;
    double* out;              // nd
    double* partials;         // gridDim.x x nd
    unsigned* ticket;         // zero between launches
    int family;               // response family
};

template <int DT>
__global__ __launch_bounds__(kThreads) void k_diff_eval(DiffParams p) {
    using E = Elem<DT>;
    const typename E::T* col = static_cast<const typename E::T*>(p.col);
    const int nd = p.nd;
    double d[kDMax];
#pragma unroll
    for (int j = 0; j < kDMax; ++j) d[j] = j < nd ? p.deltas[j] : 0.0;
    double acc[kDMax];
#pragma unroll
    for (int j = 0; j < kDMax; ++j) acc[j] = 0.0;

    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t n = (int64_t)blockIdx.x * kThreads + threadIdx.x; n < p.N; n += stride) {
        const double x = E::value(col[n], p.s);
        const double un = p.u[n];
        const unsigned yb = p.y[n];
#pragma unroll
        for (int j = 0; j < kDMax; ++j) {
            if (j >= nd) break;
            acc[j] += row_term(fma(d[j], x, un), yb, p.family);
        }
    }

    // block partials: waves in order through LDS
    __shared__ double s_w[kThreads / 64][kDMax];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < kDMax; ++j) {
        if (j >= nd) break;
        double v = acc[j];
        for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0) s_w[wave][j] = v;
    }
    __syncthreads();
    if (threadIdx.x < nd) {
        double v = 0.0;
        for (int w = 0; w < kThreads / 64; ++w) v += s_w[w][threadIdx.x];
        p.partials[(int64_t)blockIdx.x * nd + threadIdx.x] = v;
    }

    // last block: partials in block order, plus the prior at beta + delta e_k
    __shared__ unsigned s_last;
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned prev =
            __hip_atomic_fetch_add(p.ticket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_last = prev == gridDim.x - 1 ? 1u : 0u;
        if (s_last) __threadfence();
    }
    __syncthreads();
    if (!s_last) return;

    __shared__ double s_red[kThreads];
    double b = 0.0;   // sum over i != k of (beta_i - m_i)^2
    for (int i = threadIdx.x; i < p.K; i += kThreads) {
        if (i == p.k) continue;
        const double di = p.beta[i] - (p.mean ? p.mean[i] : 0.0);
        b += di * di;
    }
    s_red[threadIdx.x] = b;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s_red[threadIdx.x] += s_red[threadIdx.x + w];
        __syncthreads();
    }
    // 16 fixed interleaved subsets of the blocks per step size, then the
    // subsets in order: a fixed summation order with the loads spread over
    // the block
    __shared__ double s_m[16][kDMax];
    {
        const int j = threadIdx.x & 15, g = threadIdx.x >> 4;
        double v = 0.0;
        if (j < nd) {
#pragma unroll 8
            for (int blk = g; blk < (int)gridDim.x; blk += 16) v += p.partials[(int64_t)blk * nd + j];
        }
        s_m[g][j] = v;
    }
    __syncthreads();
    if (threadIdx.x < nd) {
        const int j = threadIdx.x;
        double f = 0.0;
        for (int g = 0; g < 16; ++g) f += s_m[g][j];
        const double dk = p.beta[p.k] + p.deltas[j] - (p.mean ? p.mean[p.k] : 0.0);
        p.out[j] = f - 0.5 * p.prec * (s_red[0] + dk * dk);
    }
    if (threadIdx.x == 0)
        __hip_atomic_store(p.ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------- commit

template <int DT>
__global__ __launch_bounds__(kThreads) void k_diff_commit(const void* __restrict__ col_, float s,
                                                          int64_t N, const double* __restrict__ delta,
                                                          double* __restrict__ u,
                                                          double* __restrict__ beta, int k) {
    using E = Elem<DT>;
    const typename E::T* col = static_cast<const typename E::T*>(col_);
    const double dl = *delta;
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t n = (int64_t)blockIdx.x * kThreads + threadIdx.x; n < N; n += stride)
        u[n] = fma(dl, E::value(col[n], s), u[n]);
    if (beta && blockIdx.x == 0 && threadIdx.x == 0) beta[k] += dl;
}

// ---------------------------------------------------------------- dispatch

int grid_for(const glm_ctx* ctx, int64_t N, int per_cu) {
    const int64_t need = (N + kThreads - 1) / kThreads;
    return (int)std::max<int64_t>(1, std::min<int64_t>(need, (int64_t)ctx->num_cu * per_cu));
}

glm_status find_colset(glm_ctx* ctx, glm_dataset_id id, const ColSet** out) {
    auto it = ctx->colsets.find(id);
    if (it == ctx->colsets.end())
        GLM_FAIL(GLM_ENOTFOUND, "unknown column set %lld", (long long)id);
    *out = &it->second;
    return GLM_OK;
}

const void* column(const ColSet& c, int k) {
    return static_cast<const unsigned char*>(c.d.Xt) +
           (size_t)k * (size_t)c.d.ldt * (size_t)elem_size(c.d.dtype);
}

}  // namespace
}  // namespace glmrt

using namespace glmrt;

extern "C" {

glm_status glm_transpose(glm_ctx* ctx, const glm_dataset_desc* rows, void* Xt, int64_t ldt,
                         void* stream) {
    clear_error();
    if (!ctx || !rows) GLM_FAIL(GLM_EINVAL, "glm_transpose: NULL argument");
    glm_status st = validate_desc(*rows);
    if (st != GLM_OK) return st;
    if (ldt < rows->N) GLM_FAIL(GLM_EINVAL, "glm_transpose: ldt = %lld < N", (long long)ldt);
    if (rows->N == 0) return GLM_OK;
    const int es = elem_size(rows->dtype);
    if (!Xt || ((uintptr_t)Xt % es)) GLM_FAIL(GLM_EINVAL, "glm_transpose: Xt NULL or misaligned");
    std::lock_guard<std::mutex> lk(ctx->mu);
    st = use_device(ctx);
    if (st != GLM_OK) return st;
    const int64_t gx = (rows->N + 63) / 64;
    if (gx > 0x7FFFFFFFLL) GLM_FAIL(GLM_EINVAL, "glm_transpose: N too large");
    dim3 grid((unsigned)gx, (unsigned)((rows->K + 63) / 64));
    hipStream_t s = (hipStream_t)stream;
    switch (es) {
    case 8:
        hipLaunchKernelGGL(k_transpose<unsigned long long>, grid, dim3(256), 0, s,
                           (const unsigned long long*)rows->X, rows->ldx, rows->N, rows->K,
                           (unsigned long long*)Xt, ldt);
        break;
    case 4:
        hipLaunchKernelGGL(k_transpose<unsigned>, grid, dim3(256), 0, s, (const unsigned*)rows->X,
                           rows->ldx, rows->N, rows->K, (unsigned*)Xt, ldt);
        break;
    case 2:
        hipLaunchKernelGGL(k_transpose<unsigned short>, grid, dim3(256), 0, s,
                           (const unsigned short*)rows->X, rows->ldx, rows->N, rows->K,
                           (unsigned short*)Xt, ldt);
        break;
    default:
        hipLaunchKernelGGL(k_transpose<unsigned char>, grid, dim3(256), 0, s,
                           (const unsigned char*)rows->X, rows->ldx, rows->N, rows->K,
                           (unsigned char*)Xt, ldt);
    }
    GLM_HIP_CHECK(hipGetLastError());
    return GLM_OK;
}

glm_status glm_colset_register(glm_ctx* ctx, const glm_colset_desc* d, glm_dataset_id* out) {
    clear_error();
    if (!ctx || !d || !out) GLM_FAIL(GLM_EINVAL, "glm_colset_register: NULL argument");
    const int es = elem_size(d->dtype);
    if (!es) GLM_FAIL(GLM_EDTYPE, "column set: unknown dtype %d", d->dtype);
    if (d->N < 0) GLM_FAIL(GLM_EINVAL, "column set: N < 0");
    if (d->K < 1 || d->K > GLM_K_MAX) GLM_FAIL(GLM_EINVAL, "column set: K = %d out of range", d->K);
    if (d->ldt < d->N) GLM_FAIL(GLM_EINVAL, "column set: ldt < N");
    if (d->N > 0 && (!d->Xt || !d->y)) GLM_FAIL(GLM_EINVAL, "column set: Xt or y is NULL");
    if (d->Xt && ((uintptr_t)d->Xt % es)) GLM_FAIL(GLM_EINVAL, "column set: Xt misaligned");
    if (d->family != GLM_LOGISTIC && d->family != GLM_POISSON)
        GLM_FAIL(GLM_EINVAL, "column set: unknown response family %d", d->family);
    if ((d->dtype == GLM_FP8_E4M3) != (d->col_scale != nullptr))
        GLM_FAIL(GLM_EINVAL, "column set: col_scale is required for FP8 and only for FP8");
    std::lock_guard<std::mutex> lk(ctx->mu);
    ColSet c;
    c.d = *d;
    if (d->dtype == GLM_FP8_E4M3) {
        // the scales are read on the host once (K floats) so that launches
        // can pass column k's scale by value
        c.scale_host.resize(d->K);
        glm_status st = use_device(ctx);
        if (st != GLM_OK) return st;
        GLM_HIP_CHECK(hipMemcpy(c.scale_host.data(), d->col_scale, d->K * sizeof(float),
                                hipMemcpyDeviceToHost));
    }
    const int64_t id = ctx->next_id++;
    ctx->colsets[id] = std::move(c);
    *out = id;
    return GLM_OK;
}

glm_status glm_colset_unregister(glm_ctx* ctx, glm_dataset_id id) {
    clear_error();
    if (!ctx) GLM_FAIL(GLM_EINVAL, "glm_colset_unregister: ctx is NULL");
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (!ctx->colsets.erase(id))
        GLM_FAIL(GLM_ENOTFOUND, "glm_colset_unregister: unknown id %lld", (long long)id);
    return GLM_OK;
}

glm_status glm_linpred(glm_ctx* ctx, glm_dataset_id id, const double* beta, double* u,
                       void* stream) {
    clear_error();
    if (!ctx || !beta) GLM_FAIL(GLM_EINVAL, "glm_linpred: NULL argument");
    std::lock_guard<std::mutex> lk(ctx->mu);
    const ColSet* c = nullptr;
    glm_status st = find_colset(ctx, id, &c);
    if (st != GLM_OK) return st;
    if (c->d.N == 0) return GLM_OK;
    if (!u) GLM_FAIL(GLM_EINVAL, "glm_linpred: u is NULL");
    st = use_device(ctx);
    if (st != GLM_OK) return st;
    const int grid = grid_for(ctx, c->d.N, 8);
    hipStream_t s = (hipStream_t)stream;
    const auto& d = c->d;
    switch (d.dtype) {
    case GLM_F64: hipLaunchKernelGGL(k_linpred<GLM_F64>, dim3(grid), dim3(kThreads), 0, s, d.Xt, d.ldt, d.col_scale, d.N, d.K, beta, u); break;
    case GLM_F32: hipLaunchKernelGGL(k_linpred<GLM_F32>, dim3(grid), dim3(kThreads), 0, s, d.Xt, d.ldt, d.col_scale, d.N, d.K, beta, u); break;
    case GLM_BF16: hipLaunchKernelGGL(k_linpred<GLM_BF16>, dim3(grid), dim3(kThreads), 0, s, d.Xt, d.ldt, d.col_scale, d.N, d.K, beta, u); break;
    default: hipLaunchKernelGGL(k_linpred<GLM_FP8_E4M3>, dim3(grid), dim3(kThreads), 0, s, d.Xt, d.ldt, d.col_scale, d.N, d.K, beta, u); break;
    }
    GLM_HIP_CHECK(hipGetLastError());
    return GLM_OK;
}

glm_status glm_diff_logpost(glm_ctx* ctx, glm_dataset_id id, const double* u, const double* beta,
                            int32_t k, const double* deltas, int32_t nd, const glm_prior* prior,
                            double* f_out, void* stream) {
    clear_error();
    if (!ctx || !beta || !deltas || !prior || !f_out)
        GLM_FAIL(GLM_EINVAL, "glm_diff_logpost: NULL argument");
    if (nd < 1) GLM_FAIL(GLM_EINVAL, "glm_diff_logpost: nd = %d < 1", nd);
    if (!(prior->prec >= 0.0)) GLM_FAIL(GLM_EINVAL, "glm_diff_logpost: prior precision < 0");
    std::lock_guard<std::mutex> lk(ctx->mu);
    const ColSet* c = nullptr;
    glm_status st = find_colset(ctx, id, &c);
    if (st != GLM_OK) return st;
    const auto& d = c->d;
    if (k < 0 || k >= d.K) GLM_FAIL(GLM_EINVAL, "glm_diff_logpost: k = %d outside [0, K)", k);
    if (d.N > 0 && !u) GLM_FAIL(GLM_EINVAL, "glm_diff_logpost: u is NULL");
    st = use_device(ctx);
    if (st != GLM_OK) return st;
    const int grid = grid_for(ctx, d.N, 4);
    Scratch* sc = nullptr;
    st = get_scratch(ctx, stream, (size_t)grid * kDMax, 0, 1, &sc);
    if (st != GLM_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    for (int j0 = 0; j0 < nd; j0 += kDMax) {
        DiffParams p;
        p.col = column(*c, k);
        p.s = d.dtype == GLM_FP8_E4M3 ? c->scale_host[k] : 1.0f;
        p.u = u;
        p.y = d.y;
        p.N = d.N;
        p.K = d.K;
        p.k = k;
        p.beta = beta;
        p.mean = prior->mean;
        p.prec = prior->prec;
        p.deltas = deltas + j0;
        p.nd = std::min(kDMax, nd - j0);
        p.out = f_out + j0;
        p.partials = sc->partials;
        p.ticket = sc->counters;
        p.family = d.family;
        switch (d.dtype) {
        case GLM_F64: hipLaunchKernelGGL(k_diff_eval<GLM_F64>, dim3(grid), dim3(kThreads), 0, s, p); break;
        case GLM_F32: hipLaunchKernelGGL(k_diff_eval<GLM_F32>, dim3(grid), dim3(kThreads), 0, s, p); break;
        case GLM_BF16: hipLaunchKernelGGL(k_diff_eval<GLM_BF16>, dim3(grid), dim3(kThreads), 0, s, p); break;
        default: hipLaunchKernelGGL(k_diff_eval<GLM_FP8_E4M3>, dim3(grid), dim3(kThreads), 0, s, p); break;
        }
        GLM_HIP_CHECK(hipGetLastError());
    }
    return GLM_OK;
}

glm_status glm_diff_commit(glm_ctx* ctx, glm_dataset_id id, double* u, double* beta, int32_t k,
                           const double* delta, void* stream) {
    clear_error();
    if (!ctx || !delta) GLM_FAIL(GLM_EINVAL, "glm_diff_commit: NULL argument");
    std::lock_guard<std::mutex> lk(ctx->mu);
    const ColSet* c = nullptr;
    glm_status st = find_colset(ctx, id, &c);
    if (st != GLM_OK) return st;
    const auto& d = c->d;
    if (k < 0 || k >= d.K) GLM_FAIL(GLM_EINVAL, "glm_diff_commit: k = %d outside [0, K)", k);
    if (d.N > 0 && !u) GLM_FAIL(GLM_EINVAL, "glm_diff_commit: u is NULL");
    st = use_device(ctx);
    if (st != GLM_OK) return st;
    const int grid = grid_for(ctx, std::max<int64_t>(d.N, 1), 8);
    const float sk = d.dtype == GLM_FP8_E4M3 ? c->scale_host[k] : 1.0f;
    hipStream_t s = (hipStream_t)stream;
    const void* col = column(*c, k);
    switch (d.dtype) {
    case GLM_F64: hipLaunchKernelGGL(k_diff_commit<GLM_F64>, dim3(grid), dim3(kThreads), 0, s, col, sk, d.N, delta, u, beta, k); break;
    case GLM_F32: hipLaunchKernelGGL(k_diff_commit<GLM_F32>, dim3(grid), dim3(kThreads), 0, s, col, sk, d.N, delta, u, beta, k); break;
    case GLM_BF16: hipLaunchKernelGGL(k_diff_commit<GLM_BF16>, dim3(grid), dim3(kThreads), 0, s, col, sk, d.N, delta, u, beta, k); break;
    default: hipLaunchKernelGGL(k_diff_commit<GLM_FP8_E4M3>, dim3(grid), dim3(kThreads), 0, s, col, sk, d.N, delta, u, beta, k); break;
    }
    GLM_HIP_CHECK(hipGetLastError());
    return GLM_OK;
}

}  // extern "C"
