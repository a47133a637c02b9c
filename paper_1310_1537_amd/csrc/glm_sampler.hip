// A random-walk Metropolis chain run on the device.
//
// The paper measures that the host round trip of an offloaded log-likelihood
// (copy beta in, launch, copy the result back, wait) costs a fixed ~20 us per
// call on its GPU and argues for porting more of the sampler (Sec. 4.5).  Here
// the whole chain stays on the device: per step a proposal kernel forms
// beta' = beta + increment_t, the fused kernel evaluates f and g at beta', and
// an accept kernel compares log U_t with f(beta') - f(beta) and keeps either
// state.  The host only enqueues; nothing waits between steps.  The proposal
// increments and log-uniforms are inputs (drawn by the caller), so the chain
// is reproducible and can be replayed exactly off the device.
#include <hip/hip_runtime.h>

#include "runtime.hpp"

namespace glmrt {
namespace {

constexpr int kT = 256;

// beta' = beta + inc[t], t = the chain's step counter.
__global__ __launch_bounds__(kT) void k_mh_propose(const double* __restrict__ beta,
                                                   const double* __restrict__ inc,
                                                   const unsigned* __restrict__ step, int K,
                                                   double* __restrict__ beta_prop) {
    const int64_t t = *step;
    for (int k = threadIdx.x; k < K; k += kT) beta_prop[k] = beta[k] + inc[t * K + k];
}

// Accept iff log U_t < f(beta') - f(beta); on acceptance beta and (f, g)
// take the proposal's values.  One block.
__global__ __launch_bounds__(kT) void k_mh_accept(double* __restrict__ beta, double* __restrict__ fg,
                                                  const double* __restrict__ beta_prop,
                                                  const double* __restrict__ fg_prop,
                                                  const double* __restrict__ logu,
                                                  unsigned* __restrict__ step, int K,
                                                  uint8_t* __restrict__ accepted,
                                                  double* __restrict__ f_trace) {
    __shared__ int s_acc;
    __shared__ unsigned s_t;
    if (threadIdx.x == 0) {
        const unsigned t = *step;
        s_t = t;
        s_acc = logu[t] < fg_prop[0] - fg[0] ? 1 : 0;
    }
    __syncthreads();
    const int acc = s_acc;
    const unsigned t = s_t;
    if (acc) {
        for (int k = threadIdx.x; k < K; k += kT) beta[k] = beta_prop[k];
        for (int k = threadIdx.x; k <= K; k += kT) fg[k] = fg_prop[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (accepted) accepted[t] = (uint8_t)acc;
        if (f_trace) f_trace[t] = fg[0];
        *step = t + 1;
    }
}

__global__ void k_mh_reset(unsigned* step) { *step = 0; }

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

    // chain state buffers: beta' (K), f and g at beta' (1 + K), step counter
    SamplerBuf& sb = ctx->sampler[stream];
    const size_t need = 2 * (size_t)K + 2;
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

    size_t np, ng, nc;
    scratch_need(ds.plan, K, 1, &np, &ng, &nc);
    Scratch* sc = nullptr;
    st = get_scratch(ctx, stream, np, ng, nc, &sc);
    if (st != GLM_OK) return st;

    // f and g at the starting point
    st = launch_fused(ds.d, ds.plan, ds.plan.fn, 1, beta, prior->mean, nullptr, prior->prec, 1,
                      fg, sc, s);
    if (st != GLM_OK) return st;
    hipLaunchKernelGGL(k_mh_reset, dim3(1), dim3(1), 0, s, step);
    GLM_HIP_CHECK(hipGetLastError());
    for (int t = 0; t < n_steps; ++t) {
        hipLaunchKernelGGL(k_mh_propose, dim3(1), dim3(kT), 0, s, beta, incs, step, K, beta_prop);
        GLM_HIP_CHECK(hipGetLastError());
        st = launch_fused(ds.d, ds.plan, ds.plan.fn, 1, beta_prop, prior->mean, nullptr,
                          prior->prec, 1, fg_prop, sc, s);
        if (st != GLM_OK) return st;
        hipLaunchKernelGGL(k_mh_accept, dim3(1), dim3(kT), 0, s, beta, fg, beta_prop, fg_prop, logu,
                           step, K, accepted, f_trace);
        GLM_HIP_CHECK(hipGetLastError());
    }
    return GLM_OK;
}

}  // extern "C"
