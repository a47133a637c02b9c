// A random-walk Metropolis chain run on the device.
//
// The paper measures that the host round trip of an offloaded log-likelihood
// (copy beta in, launch, copy the result back, wait) costs a fixed ~20 us per
// call on its GPU and argues for porting more of the sampler (Sec. 4.5).  Here
// the whole chain stays on the device: one launch of the fused kernel per
// step evaluates f and g at the proposal beta' = beta + increment_t, and its
// last block compares log U_t with f(beta') - f(beta), keeps either state and
// writes the next proposal.  The host only enqueues; nothing waits between
// steps.  The proposal
// increments and log-uniforms are inputs (drawn by the caller), so the chain
// is reproducible and can be replayed exactly off the device.
#include <hip/hip_runtime.h>

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

}  // extern "C"
