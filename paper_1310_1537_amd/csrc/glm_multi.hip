// Several coefficient vectors per pass over X: the kernel instances (one
// data set per launch, and the fleet form that runs the passes of several
// data sets of one geometry in one launch), and the public entry point
// glm_logpost_grad_multi.
#include "fg_kernel.hpp"
#include "multi_inst.hpp"
#include "runtime.hpp"

namespace glmrt {

MultiInst multi_instance(int dtype, int lpr, int cpl, int nb_max, bool mx) {
    // three vectors already go faster as one matrix-core pass with a slot
    // left empty than as VALU passes of two and one (2 GB at 512 columns:
    // 467 against 800 us; at 128 columns 508 against 826)
    if (dtype == GLM_BF16 && cpl == 1 && nb_max >= 3 && mx) {
        const MultiInst m = mx_instance(lpr);
        if (m.fn) return m;
    }
    for (int nb = 8; nb >= 2; nb /= 2) {
        if (nb > nb_max) continue;
        MultiInst m;
        switch (dtype) {
        case GLM_F64: m = multi_pick_f64(lpr, cpl, nb); break;
        case GLM_F32: m = multi_pick_f32(lpr, cpl, nb); break;
        case GLM_BF16: m = multi_pick_bf16(lpr, cpl, nb); break;
        case GLM_FP8_E4M3: m = multi_pick_fp8(lpr, cpl, nb); break;
        }
        if (m.fn) return m;
    }
    return MultiInst{};
}

glm_status launch_fleet(const void* fn, int nblocks, int wpb, const glmk::FleetJob* jobs,
                        const uint16_t* blk_job, hipStream_t stream) {
    void* args[] = {&jobs, &blk_job};
    GLM_HIP_CHECK(hipLaunchKernel(fn, dim3(nblocks), dim3(wpb * 64), args, 0, stream));
    return GLM_OK;
}

}  // namespace glmrt

using namespace glmrt;

extern "C" {

glm_status glm_logpost_grad_multi(glm_ctx* ctx, glm_dataset_id id, const double* betas, int32_t nb,
                                  const glm_prior* prior, double* out, void* stream) {
    clear_error();
    if (!ctx || !betas || !prior || !out) GLM_FAIL(GLM_EINVAL, "glm_logpost_grad_multi: NULL argument");
    if (nb < 1) GLM_FAIL(GLM_EINVAL, "glm_logpost_grad_multi: nb = %d < 1", nb);
    if (!(prior->prec >= 0.0)) GLM_FAIL(GLM_EINVAL, "glm_logpost_grad_multi: prior precision < 0");
    std::lock_guard<std::mutex> lk(ctx->mu);
    auto it = ctx->datasets.find(id);
    if (it == ctx->datasets.end())
        GLM_FAIL(GLM_ENOTFOUND, "glm_logpost_grad_multi: unknown data set %lld", (long long)id);
    glm_status st = use_device(ctx);
    if (st != GLM_OK) return st;
    const Dataset& ds = it->second;
    const int K = ds.d.K;
    MultiInst mi = multi_instance(ds.d.dtype, ds.plan.lpr, ds.plan.cpl, nb, ctx->matrix_cores);
    int NB = mi.fn ? mi.NB : 1;
    const void* fn = mi.fn ? mi.fn : ds.plan.fn;
    Plan plan = ds.plan;
    if (mi.fn) plan.wpb = mi.wpb;
    size_t np, ng, nc;
    scratch_need(ds.plan, K, NB, &np, &ng, &nc);
    Scratch* s = nullptr;
    st = get_scratch(ctx, stream, np, ng, nc, &s);
    if (st != GLM_OK) return st;
    // passes of NB vectors (the last one possibly partial)
    for (int b0 = 0; b0 < nb; b0 += NB) {
        const int n = std::min(NB, nb - b0);
        st = launch_fused(ds.d, plan, fn, NB, betas + (int64_t)b0 * K,
                          prior->mean ? prior->mean + (int64_t)b0 * K : nullptr, nullptr, prior->prec,
                          n, out + (int64_t)b0 * (K + 1), s, (hipStream_t)stream);
        if (st != GLM_OK) return st;
    }
    return GLM_OK;
}

}  // extern "C"
