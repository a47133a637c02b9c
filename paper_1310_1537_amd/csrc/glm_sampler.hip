// Samplers run on the device: random-walk Metropolis and Hamiltonian Monte
// Carlo chains, and the batch random-number fill that draws their inputs.
//
// The paper measures that the host round trip of an offloaded log-likelihood
// (copy beta in, launch, copy the result back, wait) costs a fixed ~20 us per
// call on its GPU and argues for porting more of the sampler (Sec. 4.5).  Here
// the whole chain stays on the device: one launch of the fused kernel per
// step evaluates f and g at the proposal beta' = beta + increment_t, and its
// last block compares log U_t with f(beta') - f(beta), keeps either state and
// writes the next proposal.  The host only enqueues; nothing waits between
// steps.  The Metropolis chain's increments and log-uniforms are inputs
// (drawn by the caller, or on the device with glm_rng_fill); the HMC chain
// draws its momenta and accept uniforms itself from counter-based streams,
// so both are reproducible and can be replayed off the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "fg_kernel.hpp"
#include "runtime.hpp"

namespace glmrt {
namespace {

constexpr int kT = 256;

// Chain parameters to their device copy, step counter to zero and the first
// proposal beta + inc[0].
__global__ __launch_bounds__(kT) void k_mh_start(glmk::ChainParams cp, glmk::ChainParams* dst,
                                                 int K) {
    for (int k = threadIdx.x; k < K; k += kT) cp.beta_prop[k] = cp.beta[k] + cp.incs[k];
    if (threadIdx.x == 0) {
        *dst = cp;
        *cp.step = 0;
    }
}

// HMC: chain parameters to their device copy and the first iteration
// started (f and g at the state are already in cp.fg).
__global__ __launch_bounds__(kT) void k_hmc_start(glmk::ChainParams cp, glmk::ChainParams* dst,
                                                  int K) {
    if (threadIdx.x == 0) *dst = cp;
    glmk::hmc_begin<kT>(cp, cp.iter0, K);
}

// Batch fill of n values of one stream, starting at value `offset`: one
// thread per generator block (four uniforms) or per normal pair.
__global__ __launch_bounds__(kT) void k_rng_fill(int kind, uint64_t seed, uint64_t chain,
                                                 uint64_t stream, uint64_t offset, int64_t n,
                                                 double scale, double* out) {
    const uint64_t end = offset + (uint64_t)n;
    const uint64_t stride = (uint64_t)gridDim.x * kT;
    if (kind == GLM_RNG_NORMAL) {
        for (uint64_t q = offset / 2 + (uint64_t)blockIdx.x * kT + threadIdx.x; 2 * q < end;
             q += stride) {
            double z[2];
            glmk::polar_pair(seed, chain, glmk::RNG_NORMAL, stream, q, z[0], z[1]);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const uint64_t i = 2 * q + h;
                if (i >= offset && i < end) out[i - offset] = scale * z[h];
            }
        }
        return;
    }
    for (uint64_t b = offset / 4 + (uint64_t)blockIdx.x * kT + threadIdx.x; 4 * b < end; b += stride) {
        const glmk::Block4 w = glmk::philox4x64_10(b, 0, glmk::RNG_UNIFORM, stream, seed, chain);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint64_t i = 4 * b + j;
            if (i >= offset && i < end) {
                const double u = glmk::u01(w.w[j]);
                out[i - offset] = kind == GLM_RNG_LOG_UNIFORM ? glmk::log_f64(u) : u;
            }
        }
    }
}

}  // namespace
}  // namespace glmrt

using namespace glmrt;

extern "C" {

glm_status glm_mh_run(glm_ctx* ctx, glm_dataset_id id, double* beta, double* fg,
                      const double* incs, const double* logu, int32_t n_steps,
                      const glm_prior* prior, uint8_t* accepted, double* f_trace, void* stream) {
    clear_error();
    if (!ctx || !beta || !fg || !prior || (n_steps > 0 && (!incs || !logu)))
        GLM_FAIL(GLM_EINVAL, "glm_mh_run: NULL argument");
    if (n_steps < 0) GLM_FAIL(GLM_EINVAL, "glm_mh_run: n_steps < 0");
    if (!(prior->prec >= 0.0)) GLM_FAIL(GLM_EINVAL, "glm_mh_run: prior precision < 0");
    std::lock_guard<std::mutex> lk(ctx->mu);
    auto it = ctx->datasets.find(id);
    if (it == ctx->datasets.end())
        GLM_FAIL(GLM_ENOTFOUND, "glm_mh_run: unknown data set %lld", (long long)id);
    glm_status st = use_device(ctx);
    if (st != GLM_OK) return st;
    const Dataset& ds = it->second;
    const int K = ds.d.K;
    hipStream_t s = (hipStream_t)stream;

    // chain state buffers: beta' (K), f and g at beta' (1 + K), step counter,
    // the chain parameters
    constexpr size_t kParamWords = (sizeof(glmk::ChainParams) + 7) / 8;
    SamplerBuf& sb = ctx->sampler[stream];
    const size_t need = 2 * (size_t)K + 2 + kParamWords;
    if (sb.cap < need) {
        if (sb.buf) {
            GLM_HIP_CHECK(hipStreamSynchronize(s));
            GLM_HIP_CHECK(hipFree(sb.buf));
            sb = SamplerBuf{};
        }
        if (hipMalloc((void**)&sb.buf, need * sizeof(double)) != hipSuccess)
            GLM_FAIL(GLM_ENOMEM, "glm_mh_run: device allocation failed");
        sb.cap = need;
    }
    double* beta_prop = sb.buf;
    double* fg_prop = sb.buf + K;
    unsigned* step = reinterpret_cast<unsigned*>(sb.buf + 2 * K + 1);
    glmk::ChainParams* cp_dev = reinterpret_cast<glmk::ChainParams*>(sb.buf + 2 * K + 2);

    size_t np, ng, nc;
    scratch_need(ds.plan, K, 1, &np, &ng, &nc);
    Scratch* sc = nullptr;
    st = get_scratch(ctx, stream, np, ng, nc, &sc);
    if (st != GLM_OK) return st;

    // f and g at the starting point
    st = launch_fused(ds.d, ds.plan, ds.plan.fn, 1, beta, prior->mean, nullptr, prior->prec, 1,
                      fg, sc, s);
    if (st != GLM_OK) return st;
    if (n_steps == 0) return GLM_OK;
    glmk::ChainParams cp;
    cp.beta = beta;
    cp.fg = fg;
    cp.beta_prop = beta_prop;
    cp.incs = incs;
    cp.logu = logu;
    cp.step = step;
    cp.n_steps = n_steps;
    cp.accepted = accepted;
    cp.f_trace = f_trace;
    cp.kind = 0;
    hipLaunchKernelGGL(k_mh_start, dim3(1), dim3(kT), 0, s, cp, cp_dev, K);
    GLM_HIP_CHECK(hipGetLastError());
    // one launch per step: evaluate the proposal, accept or not, propose again
    for (int t = 0; t < n_steps; ++t) {
        st = launch_fused(ds.d, ds.plan, ds.plan.fn, 1, beta_prop, prior->mean, nullptr,
                          prior->prec, 1, fg_prop, sc, s, nullptr, cp_dev);
        if (st != GLM_OK) return st;
    }
    return GLM_OK;
}

glm_status glm_hmc_run(glm_ctx* ctx, glm_dataset_id id, double* beta, double* fg, int32_t n_iter,
                       int32_t n_leap, double eps, uint64_t seed, uint64_t chain, uint32_t iter0,
                       const glm_prior* prior, uint8_t* accepted, double* f_trace, void* stream) {
    clear_error();
    if (!ctx || !beta || !fg || !prior) GLM_FAIL(GLM_EINVAL, "glm_hmc_run: NULL argument");
    if (n_iter < 0 || n_leap < 1) GLM_FAIL(GLM_EINVAL, "glm_hmc_run: n_iter < 0 or n_leap < 1");
    if ((uint64_t)iter0 + (uint64_t)n_iter > 0xFFFFFFFFull)
        GLM_FAIL(GLM_EINVAL, "glm_hmc_run: iter0 + n_iter beyond 2^32 - 1");
    if (!(eps > 0.0) || !std::isfinite(eps)) GLM_FAIL(GLM_EINVAL, "glm_hmc_run: eps must be > 0");
    if (!(prior->prec >= 0.0)) GLM_FAIL(GLM_EINVAL, "glm_hmc_run: prior precision < 0");
    std::lock_guard<std::mutex> lk(ctx->mu);
    auto it = ctx->datasets.find(id);
    if (it == ctx->datasets.end())
        GLM_FAIL(GLM_ENOTFOUND, "glm_hmc_run: unknown data set %lld", (long long)id);
    glm_status st = use_device(ctx);
    if (st != GLM_OK) return st;
    const Dataset& ds = it->second;
    const int K = ds.d.K;
    hipStream_t s = (hipStream_t)stream;

    // chain buffers: the evaluated point (K), f and g there (1 + K), momenta
    // (K), h0, the iteration and leapfrog counters, the chain parameters
    constexpr size_t kParamWords = (sizeof(glmk::ChainParams) + 7) / 8;
    SamplerBuf& sb = ctx->sampler[stream];
    const size_t need = 3 * (size_t)K + 3 + kParamWords;
    if (sb.cap < need) {
        if (sb.buf) {
            GLM_HIP_CHECK(hipStreamSynchronize(s));
            GLM_HIP_CHECK(hipFree(sb.buf));
            sb = SamplerBuf{};
        }
        if (hipMalloc((void**)&sb.buf, need * sizeof(double)) != hipSuccess)
            GLM_FAIL(GLM_ENOMEM, "glm_hmc_run: device allocation failed");
        sb.cap = need;
    }
    double* beta_prop = sb.buf;
    double* fg_prop = sb.buf + K;
    double* mom = sb.buf + 2 * K + 1;
    double* h0 = sb.buf + 3 * K + 1;
    unsigned* step = reinterpret_cast<unsigned*>(sb.buf + 3 * K + 2);
    glmk::ChainParams* cp_dev = reinterpret_cast<glmk::ChainParams*>(sb.buf + 3 * K + 3);

    size_t np, ng, nc;
    scratch_need(ds.plan, K, 1, &np, &ng, &nc);
    Scratch* sc = nullptr;
    st = get_scratch(ctx, stream, np, ng, nc, &sc);
    if (st != GLM_OK) return st;
    st = launch_fused(ds.d, ds.plan, ds.plan.fn, 1, beta, prior->mean, nullptr, prior->prec, 1,
                      fg, sc, s);
    if (st != GLM_OK) return st;
    if (n_iter == 0) return GLM_OK;
    glmk::ChainParams cp;
    cp.beta = beta;
    cp.fg = fg;
    cp.beta_prop = beta_prop;
    cp.incs = nullptr;
    cp.logu = nullptr;
    cp.step = step;
    cp.n_steps = n_iter;
    cp.accepted = accepted;
    cp.f_trace = f_trace;
    cp.kind = 1;
    cp.n_leap = n_leap;
    cp.eps = eps;
    cp.mom = mom;
    cp.h0 = h0;
    cp.seed = seed;
    cp.chain_id = chain;
    cp.iter0 = iter0;
    hipLaunchKernelGGL(k_hmc_start, dim3(1), dim3(kT), 0, s, cp, cp_dev, K);
    GLM_HIP_CHECK(hipGetLastError());
    // one launch per leapfrog position; the last block moves the chain on
    for (int64_t e = 0; e < (int64_t)n_iter * n_leap; ++e) {
        st = launch_fused(ds.d, ds.plan, ds.plan.fn, 1, beta_prop, prior->mean, nullptr,
                          prior->prec, 1, fg_prop, sc, s, nullptr, cp_dev);
        if (st != GLM_OK) return st;
    }
    return GLM_OK;
}

glm_status glm_rng_fill(glm_ctx* ctx, int32_t kind, uint64_t seed, uint64_t chain,
                        uint64_t stream_id, uint64_t offset, int64_t n, double scale, double* out,
                        void* stream) {
    clear_error();
    if (!ctx || (n > 0 && !out)) GLM_FAIL(GLM_EINVAL, "glm_rng_fill: NULL argument");
    if (kind != GLM_RNG_UNIFORM && kind != GLM_RNG_NORMAL && kind != GLM_RNG_LOG_UNIFORM)
        GLM_FAIL(GLM_EINVAL, "glm_rng_fill: unknown kind %d", kind);
    if (n < 0) GLM_FAIL(GLM_EINVAL, "glm_rng_fill: n < 0");
    if (offset > UINT64_MAX / 2 - (uint64_t)n)
        GLM_FAIL(GLM_EINVAL, "glm_rng_fill: offset + n beyond the stream");
    if (n == 0) return GLM_OK;
    std::lock_guard<std::mutex> lk(ctx->mu);
    glm_status st = use_device(ctx);
    if (st != GLM_OK) return st;
    const int64_t units = kind == GLM_RNG_NORMAL ? n / 2 + 2 : n / 4 + 2;
    const int64_t blocks = std::min<int64_t>((units + kT - 1) / kT, (int64_t)ctx->num_cu * 8);
    hipLaunchKernelGGL(k_rng_fill, dim3((unsigned)blocks), dim3(kT), 0, (hipStream_t)stream, kind,
                       seed, chain, stream_id, offset, n, scale, out);
    GLM_HIP_CHECK(hipGetLastError());
    return GLM_OK;
}

}  // extern "C"
