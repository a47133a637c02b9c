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
#include "elem.hpp"
#include "publish.hpp"
#include "tr_math.hpp"

namespace glmrt {
namespace {

constexpr int kDMax = 16;       // step sizes per pass
constexpr int kThreads = 256;

// t(v) = y v - b(v) with b the log-partition of the response family:
// softplus (logistic) or exp (Poisson, y a count).
__device__ __forceinline__ double row_term(double v, unsigned yb, int fam) {
    if (fam == GLM_POISSON) return (double)(yb & 0xFFu) * v - glmk::exp_f64(v);
    return (double)(yb & 1u) * v - (fmax(v, 0.0) + glmk::log1p_unit(glmk::exp_f64(-fabs(v))));
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
    using E = glmk::Elem<DT>;
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
    int vec;                  // rows in aligned groups of four (see k_diff_eval)
};

// Four consecutive entries of a column as doubles, from one aligned vector
// load (16 bytes for FP32, 8 for BF16, 4 for FP8, two 16-byte loads for FP64).
typedef double dv2 __attribute__((ext_vector_type(2)));
typedef float fv4 __attribute__((ext_vector_type(4)));
typedef unsigned uv2 __attribute__((ext_vector_type(2)));

template <int DT>
__device__ __forceinline__ void load4(const void* col, int64_t n0, float s, double (&x)[4]) {
    if constexpr (DT == GLM_F64) {
        const dv2* p = reinterpret_cast<const dv2*>(static_cast<const double*>(col) + n0);
        const dv2 a = __builtin_nontemporal_load(p), b = __builtin_nontemporal_load(p + 1);
        x[0] = a.x; x[1] = a.y; x[2] = b.x; x[3] = b.y;
    } else if constexpr (DT == GLM_F32) {
        const fv4 v = __builtin_nontemporal_load(
            reinterpret_cast<const fv4*>(static_cast<const float*>(col) + n0));
        x[0] = v.x; x[1] = v.y; x[2] = v.z; x[3] = v.w;
    } else if constexpr (DT == GLM_BF16) {
        const uv2 v = __builtin_nontemporal_load(
            reinterpret_cast<const uv2*>(static_cast<const unsigned short*>(col) + n0));
        x[0] = (double)__uint_as_float(v.x << 16);
        x[1] = (double)__uint_as_float(v.x & 0xFFFF0000u);
        x[2] = (double)__uint_as_float(v.y << 16);
        x[3] = (double)__uint_as_float(v.y & 0xFFFF0000u);
    } else {
        const unsigned v = __builtin_nontemporal_load(
            reinterpret_cast<const unsigned*>(static_cast<const unsigned char*>(col) + n0));
        const auto lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)v, false);
        const auto hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)v, true);
        x[0] = (double)lo[0] * (double)s; x[1] = (double)lo[1] * (double)s;
        x[2] = (double)hi[0] * (double)s; x[3] = (double)hi[1] * (double)s;
    }
}

// One block per compute unit (NT lanes): every block publishes a partial and
// takes a ticket, costs that a grid of many small blocks would multiply.
//
// Rows are taken in groups of four (one vector load of the column, two of
// u, one of y), several groups per loop trip with all loads issued first; the
// N mod 4 rows after the last group are taken one at a time.  The vector
// loads need the column 4-element aligned, u 16-byte and y 4-byte aligned
// (checked by the host, which otherwise launches with vec = false).
template <int DT, int DMAX, int NT>
__global__ __launch_bounds__(NT) void k_diff_eval(DiffParams p) {
    static_assert(NT >= 256 && NT % 64 == 0, "the final merge uses 16 x 16 lanes");
    using E = glmk::Elem<DT>;
    const typename E::T* col = static_cast<const typename E::T*>(p.col);
    const int nd = p.nd;
    const int fam = p.family;
    double d[DMAX];
#pragma unroll
    for (int j = 0; j < DMAX; ++j) d[j] = j < nd ? p.deltas[j] : 0.0;
    double acc[DMAX];
#pragma unroll
    for (int j = 0; j < DMAX; ++j) acc[j] = 0.0;

    // (a guarded body rather than an early exit, so that the loop unrolls and
    // d and acc stay in registers)
    auto add_row = [&](double x, double un, unsigned yb) {
#pragma unroll
        for (int j = 0; j < DMAX; ++j)
            if (j < nd) acc[j] += row_term(fma(d[j], x, un), yb, fam);
    };

    const int64_t gtid = (int64_t)blockIdx.x * NT + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * NT;
    int64_t n_scalar = 0;   // first row of the one-at-a-time part
    if (p.vec) {
        const int64_t ng = p.N >> 2;
        const dv2* u2 = reinterpret_cast<const dv2*>(p.u);
        const unsigned* y4 = reinterpret_cast<const unsigned*>(p.y);
        // GT groups per trip, every load of the trip issued before the first
        // row is added (one memory latency per trip; with one step size a
        // trip of four covers this thread's share of 4M rows; wider forms
        // keep two, which fit the registers)
        constexpr int GT = DMAX == 1 && DT != GLM_F64 ? 4 : 2;
        for (int64_t g = gtid; g < ng; g += GT * stride) {
            double x[GT][4];
            dv2 ua[GT][2];
            unsigned yy[GT];
            bool ok[GT];
#pragma unroll
            for (int q = 0; q < GT; ++q) {
                const int64_t gq = g + q * stride;
                ok[q] = gq < ng;
                const int64_t gv = ok[q] ? gq : g;   // a valid address either way
                load4<DT>(p.col, 4 * gv, p.s, x[q]);
                ua[q][0] = u2[2 * gv];
                ua[q][1] = u2[2 * gv + 1];
                yy[q] = y4[gv];
            }
#pragma unroll
            for (int q = 0; q < GT; ++q) {
                if (ok[q]) {
                    add_row(x[q][0], ua[q][0].x, yy[q] & 0xFFu);
                    add_row(x[q][1], ua[q][0].y, (yy[q] >> 8) & 0xFFu);
                    add_row(x[q][2], ua[q][1].x, (yy[q] >> 16) & 0xFFu);
                    add_row(x[q][3], ua[q][1].y, yy[q] >> 24);
                }
            }
        }
        n_scalar = ng << 2;
    }
    for (int64_t n = n_scalar + gtid; n < p.N; n += stride)
        add_row(E::value(col[n], p.s), p.u[n], p.y[n]);

    // block partials: waves in order through LDS
    __shared__ double s_w[NT / 64][DMAX];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < DMAX; ++j) {
        if (j < nd) {
            double v = acc[j];
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
            if (lane == 0) s_w[wave][j] = v;
        }
    }
    __syncthreads();
    if (threadIdx.x < nd) {
        double v = 0.0;
        for (int w = 0; w < NT / 64; ++w) v += s_w[w][threadIdx.x];
        glmk::publish(&p.partials[(int64_t)blockIdx.x * nd + threadIdx.x], v);
    }

    // last block: partials in block order, plus the prior at beta + delta e_k
    // (published partials: stores complete before the barrier and the ticket)
    __shared__ unsigned s_last;
    glmk::publish_wait();
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned prev =
            __hip_atomic_fetch_add(p.ticket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_last = prev == gridDim.x - 1 ? 1u : 0u;
    }
    __syncthreads();
    if (!s_last) return;

    // 16 fixed interleaved subsets of the blocks per step size, then the
    // subsets in order: a fixed summation order with the loads spread over
    // the block.  The prior's sum over i != k of (beta_i - m_i)^2 is taken
    // in the same round trip: thread t adds i = t, t + NT, ..., each wave
    // adds its lanes by butterfly, the waves are added in order.
    __shared__ double s_m[16][DMAX];
    __shared__ double s_wb[NT / 64];
    {
        const int j = threadIdx.x & 15, g = threadIdx.x >> 4;   // NT >= 256: g covers 0..15
        double v = 0.0;
        if (g < 16 && j < nd) {
#pragma unroll 8
            for (int blk = g; blk < (int)gridDim.x; blk += 16)
                v += glmk::fetch_published(&p.partials[(int64_t)blk * nd + j]);
        }
        double b = 0.0;
        for (int i = threadIdx.x; i < p.K; i += NT) {
            const double di = p.beta[i] - (p.mean ? p.mean[i] : 0.0);
            b += i == p.k ? 0.0 : di * di;
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) b += __shfl_xor(b, off, 64);
        if (g < 16 && j < DMAX) s_m[g][j] = v;
        if (lane == 0) s_wb[wave] = b;
    }
    __syncthreads();
    if (threadIdx.x < nd) {
        const int j = threadIdx.x;
        double f = 0.0;
        for (int g = 0; g < 16; ++g) f += s_m[g][j];
        double b = 0.0;
        for (int w = 0; w < NT / 64; ++w) b += s_wb[w];
        const double dk = p.beta[p.k] + p.deltas[j] - (p.mean ? p.mean[p.k] : 0.0);
        p.out[j] = f - 0.5 * p.prec * (b + dk * dk);
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
    using E = glmk::Elem<DT>;
    const typename E::T* col = static_cast<const typename E::T*>(col_);
    const double dl = *delta;
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t n = (int64_t)blockIdx.x * kThreads + threadIdx.x; n < N; n += stride)
        u[n] = fma(dl, E::value(col[n], s), u[n]);
    if (beta && blockIdx.x == 0 && threadIdx.x == 0) beta[k] += dl;
}

// ---------------------------------------------------------------- dispatch

// Block sizes: 16 waves per compute unit where the registers allow it
// (up to 4 step sizes), 8 waves for 16 step sizes.
constexpr int kEvalThreadsSmall = 1024;
constexpr int kEvalThreadsLarge = 512;

// The evaluation's grid: one block per compute unit at most, each block
// covering at least four rows per lane of a 512-lane block.
int eval_grid(const glm_ctx* ctx, int64_t N) {
    return (int)std::max<int64_t>(
        1, std::min<int64_t>(ctx->num_cu, (N + kEvalThreadsLarge * 4 - 1) / (kEvalThreadsLarge * 4)));
}

// The per-row terms alone (glm_probe_diff_map): row n's u and y come from n,
// nothing is loaded; each lane's sum goes to sink so that the work is kept.
__global__ __launch_bounds__(kEvalThreadsSmall) void k_map_probe(double* __restrict__ sink,
                                                                 int64_t N, int fam) {
    const int64_t gtid = (int64_t)blockIdx.x * kEvalThreadsSmall + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * kEvalThreadsSmall;
    double acc = 0.0;
    for (int64_t n = gtid; n < N; n += stride)
        acc += row_term((double)(n & 4095) * 1e-3 - 2.0, (unsigned)n, fam);
    sink[gtid] = acc;
}

template <int DT>
const void* diff_kernel_dt(int nd) {
    if (nd <= 1) return reinterpret_cast<const void*>(&k_diff_eval<DT, 1, kEvalThreadsSmall>);
    if (nd <= 4) return reinterpret_cast<const void*>(&k_diff_eval<DT, 4, kEvalThreadsSmall>);
    return reinterpret_cast<const void*>(&k_diff_eval<DT, kDMax, kEvalThreadsLarge>);
}

const void* diff_kernel(int dtype, int nd) {
    switch (dtype) {
    case GLM_F64: return diff_kernel_dt<GLM_F64>(nd);
    case GLM_F32: return diff_kernel_dt<GLM_F32>(nd);
    case GLM_BF16: return diff_kernel_dt<GLM_BF16>(nd);
    default: return diff_kernel_dt<GLM_FP8_E4M3>(nd);
    }
}

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
    const int grid = eval_grid(ctx, d.N);
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
        const int es = elem_size(d.dtype);
        p.vec = ((uintptr_t)p.col % (4 * es) == 0) && ((uintptr_t)u % 16 == 0) &&
                ((uintptr_t)d.y % 4 == 0) &&
                (d.dtype != GLM_F64 || (uintptr_t)p.col % 16 == 0);
        const void* fn = diff_kernel(d.dtype, p.nd);
        void* args[] = {&p};
        const int nt = p.nd <= 4 ? kEvalThreadsSmall : kEvalThreadsLarge;
        GLM_HIP_CHECK(hipLaunchKernel(fn, dim3(grid), dim3(nt), args, 0, s));
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

glm_status glm_probe_diff_map(glm_ctx* ctx, int64_t n, int32_t family, int32_t iters, double* us) {
    clear_error();
    if (!ctx || !us || n < 0 || iters < 1) GLM_FAIL(GLM_EINVAL, "glm_probe_diff_map: bad argument");
    if (family != GLM_LOGISTIC && family != GLM_POISSON)
        GLM_FAIL(GLM_EINVAL, "glm_probe_diff_map: unknown family %d", family);
    std::lock_guard<std::mutex> lk(ctx->mu);
    glm_status st = use_device(ctx);
    if (st != GLM_OK) return st;
    const int grid = eval_grid(ctx, n);
    double* sink = nullptr;
    if (hipMalloc((void**)&sink, (size_t)grid * kEvalThreadsSmall * sizeof(double)) != hipSuccess)
        GLM_FAIL(GLM_ENOMEM, "glm_probe_diff_map: device allocation failed");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    hipStream_t s = ctx->own_stream;
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_map_probe, dim3(grid), dim3(kEvalThreadsSmall), 0, s, sink, n, family);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    for (int i = 0; i < iters && e == hipSuccess; ++i) {
        hipLaunchKernelGGL(k_map_probe, dim3(grid), dim3(kEvalThreadsSmall), 0, s, sink, n, family);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(sink);
    if (e != hipSuccess) GLM_FAIL(GLM_EHIP, "glm_probe_diff_map: %s", hipGetErrorString(e));
    *us = (double)ms * 1e3 / iters;
    return GLM_OK;
}

}  // extern "C"
