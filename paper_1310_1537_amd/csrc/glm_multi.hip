// Several coefficient vectors per pass over X: the kernel instances (one
// data set per launch, and the fleet form that runs the passes of several
// data sets of one geometry in one launch), and the public entry point
// glm_logpost_grad_multi.
#include <cstdlib>

#include "fg_kernel.hpp"
#include "runtime.hpp"

namespace glmrt {
namespace {

constexpr int WPB = 4;

// R = 8 row slots per lane keeps the NB copies of beta and of the gradient
// accumulators within the register file; instances with more than 32 values
// of beta or gradient per lane (NB x columns per lane) are not built.  FP32
// rows of 32 lanes with 8 vectors take 4 row slots instead, which fits two
// waves per SIMD (255 registers) and runs 8 waves per block: 9-12 % faster
// than 8 slots at one wave per SIMD.  (The other widths spill with 4 slots.)
template <int DT, int LPR, int CPL, int NB>
MultiInst minst() {
    constexpr int VE = 16 / glmk::ElemSize<DT>::v;
    if constexpr (NB * CPL * VE > 32) {
        return MultiInst{};
    } else if constexpr (DT == glmk::DT_F32 && LPR == 32 && CPL == 1 && NB == 8) {
        MultiInst m;
        m.fn = reinterpret_cast<const void*>(&glmk::fg_fused<DT, LPR, CPL, 4, 8, NB>);
        m.R = 4;
        m.NB = NB;
        m.fleet = reinterpret_cast<const void*>(&glmk::fg_fleet<DT, LPR, CPL, 4, 8, NB>);
        m.wpb = 8;
        return m;
    } else {
        return MultiInst{reinterpret_cast<const void*>(&glmk::fg_fused<DT, LPR, CPL, 8, WPB, NB>), 8, NB,
                         reinterpret_cast<const void*>(&glmk::fg_fleet<DT, LPR, CPL, 8, WPB, NB>)};
    }
}

template <int DT, int NB>
MultiInst mpick(int lpr, int cpl) {
    if (cpl == 1) {
        switch (lpr) {
        case 1: return minst<DT, 1, 1, NB>();
        case 2: return minst<DT, 2, 1, NB>();
        case 4: return minst<DT, 4, 1, NB>();
        case 8: return minst<DT, 8, 1, NB>();
        case 16: return minst<DT, 16, 1, NB>();
        case 32: return minst<DT, 32, 1, NB>();
        case 64: return minst<DT, 64, 1, NB>();
        }
    } else if (lpr == 64) {
        if (cpl == 2) return minst<DT, 64, 2, NB>();
        if (cpl == 4) return minst<DT, 64, 4, NB>();
    }
    return MultiInst{};
}

template <int DT>
MultiInst mpick_nb(int lpr, int cpl, int nb) {
    switch (nb) {
    case 8: return mpick<DT, 8>(lpr, cpl);
    case 4: return mpick<DT, 4>(lpr, cpl);
    case 2: return mpick<DT, 2>(lpr, cpl);
    }
    return MultiInst{};
}

// GLM_MFMA=0 keeps BF16 passes on the VALU kernels (for comparisons); read
// at every choice of instance, so a process can time both forms.
bool mx_enabled() {
    const char* e = std::getenv("GLM_MFMA");
    return !e || std::atoi(e) != 0;
}

}  // namespace

MultiInst multi_instance(int dtype, int lpr, int cpl, int nb_max) {
    if (dtype == GLM_BF16 && cpl == 1 && nb_max >= 4 && mx_enabled()) {
        const MultiInst m = mx_instance(lpr);
        if (m.fn) return m;
    }
    for (int nb = 8; nb >= 2; nb /= 2) {
        if (nb > nb_max) continue;
        MultiInst m;
        switch (dtype) {
        case GLM_F64: m = mpick_nb<glmk::DT_F64>(lpr, cpl, nb); break;
        case GLM_F32: m = mpick_nb<glmk::DT_F32>(lpr, cpl, nb); break;
        case GLM_BF16: m = mpick_nb<glmk::DT_BF16>(lpr, cpl, nb); break;
        case GLM_FP8_E4M3: m = mpick_nb<glmk::DT_FP8>(lpr, cpl, nb); break;
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
    MultiInst mi = multi_instance(ds.d.dtype, ds.plan.lpr, ds.plan.cpl, nb);
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
