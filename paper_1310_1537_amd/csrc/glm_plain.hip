// Plain entry points: one data set, one beta per launch.
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>

#include "fg_kernel.hpp"
#include "runtime.hpp"

namespace glmrt {

namespace {

constexpr int WPB = 4;

struct Inst {
    const void* fn;
    int R;
};

template <int DT, int LPR, int CPL>
Inst inst() {
    // 16 row slots of 16 bytes per lane per batch (64 VGPRs per tile); FP32
    // takes 8 (its FP64 gradient products keep r in FP64, and with 16 slots
    // the kernel no longer fits two waves per SIMD).  Wide FP8 rows (256 to
    // 512 columns, one chunk per lane) rotate three tiles, the load of a
    // batch going out two batches ahead: 8M x 512 random codes take 790
    // against about 810 us with two.  BF16 rows of 512 columns with 8 slots
    // and three tiles were slower on random data (1,340 against 1,265 us),
    // and FP32 and FP64 gain nothing from a third tile.
    constexpr bool WIDE = DT == glmk::DT_FP8 && CPL == 1 && LPR >= 32;
    constexpr int RE = DT == glmk::DT_F32 ? 8 : 16;
    // FP8 rows of 4 chunks per lane (4096 columns) take one row slot: with
    // the 4 of RE / CPL they spilled to scratch memory (2 GB of codes: 707
    // against 912 us; 2 slots 738).
    constexpr int R = DT == glmk::DT_FP8 && CPL == 4 ? 1 : (RE / CPL > 0 ? RE / CPL : 1);
    constexpr int NBUF = WIDE ? 3 : 2;
    return Inst{reinterpret_cast<const void*>(&glmk::fg_fused<DT, LPR, CPL, R, WPB, 1, NBUF>), R};
}

template <int DT>
Inst pick(int lpr, int cpl) {
    if (cpl == 1) {
        switch (lpr) {
        case 1: return inst<DT, 1, 1>();
        case 2: return inst<DT, 2, 1>();
        case 4: return inst<DT, 4, 1>();
        case 8: return inst<DT, 8, 1>();
        case 16: return inst<DT, 16, 1>();
        case 32: return inst<DT, 32, 1>();
        case 64: return inst<DT, 64, 1>();
        }
    } else if (lpr == 64) {
        if (cpl == 2) return inst<DT, 64, 2>();
        if (cpl == 4) return inst<DT, 64, 4>();
    }
    return Inst{nullptr, 0};
}

Inst pick_any(int dt, int lpr, int cpl) {
    switch (dt) {
    case GLM_F64: return pick<glmk::DT_F64>(lpr, cpl);
    case GLM_F32: return pick<glmk::DT_F32>(lpr, cpl);
    case GLM_BF16: return pick<glmk::DT_BF16>(lpr, cpl);
    case GLM_FP8_E4M3: return pick<glmk::DT_FP8>(lpr, cpl);
    }
    return Inst{nullptr, 0};
}

int pow2ceil(int v) {
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

}  // namespace

glm_status make_plan(glm_ctx* ctx, const glm_dataset_desc& d, Plan* plan) {
    const int es = elem_size(d.dtype);
    const int ve = 16 / es;
    // (nothing is read when N == 0)
    const bool vec_ok = d.N == 0 || ((d.ldx * es) % 16 == 0 && ((uintptr_t)d.X % 16) == 0);
    if (!vec_ok)
        GLM_FAIL(GLM_EINVAL,
                 "plan: rows must start on 16-byte boundaries (ldx*%d a multiple of 16, X "
                 "16-byte aligned)",
                 es);
    if (d.ldx * es > (1 << 21))
        GLM_FAIL(GLM_EINVAL, "plan: row stride ldx*%d = %lld bytes exceeds 2 MiB", es,
                 (long long)(d.ldx * es));
    const int nc = (d.K + ve - 1) / ve;   // chunks per row, the last possibly partial
    Plan p;
    p.kind = 0;
    p.lpr = std::min(64, pow2ceil(nc));
    p.cpl = nc <= 64 ? 1 : pow2ceil((nc + 63) / 64);
    if (p.cpl > 4) GLM_FAIL(GLM_EINVAL, "plan: K = %d too wide for dtype %d", d.K, d.dtype);
    Inst in = pick_any(d.dtype, p.lpr, p.cpl);
    if (!in.fn) GLM_FAIL(GLM_EINVAL, "plan: no kernel instance for K = %d", d.K);
    p.fn = in.fn;
    p.rows_per_lane = in.R;
    p.wpb = WPB;
    // Persistent grid: every wave streams one contiguous range of row batches.
    const int64_t wave_rows = (int64_t)in.R * (64 / p.lpr);
    const int64_t nbatch = (d.N + wave_rows - 1) / wave_rows;
    const int64_t target = (int64_t)ctx->num_cu * ctx->blocks_per_cu;
    const int64_t need = (nbatch + p.wpb - 1) / p.wpb;
    p.nblocks = (int)std::max<int64_t>(1, std::min(need, target));
    p.interleave = ctx->interleave ? 1 : 0;
    // One merge level for small grids (64 blocks or fewer, or block partials
    // of one vector that fit the merge's LDS staging), two (groups of about
    // sqrt(nblocks)) above.
    const bool one_level = p.nblocks <= 64 || (int64_t)p.nblocks * (d.K + 1) <= glmk::kStageDoubles;
    p.group = one_level ? p.nblocks : std::max(1, (int)std::ceil(std::sqrt((double)p.nblocks)));
    *plan = p;
    return GLM_OK;
}

void scratch_need(const Plan& pl, int K, int NB, size_t* n_partials, size_t* n_gpart,
                  size_t* n_counters) {
    const size_t W = (size_t)NB * (K + 1);
    const int ngroups = (pl.nblocks + pl.group - 1) / pl.group;
    *n_partials = (size_t)pl.nblocks * W;
    *n_gpart = (size_t)ngroups * W;
    *n_counters = (size_t)ngroups + 1;
}

void fused_params(const glm_dataset_desc& d, const Plan& pl, int NB, const double* betas,
                  const double* means, const double* precs, double prec, int nb, double* out,
                  double* partials, double* gpart, unsigned* counters, double* w_out,
                  const void* chain, glmk::FgParams* pp) {
    glmk::FgParams& p = *pp;
    p.X = static_cast<const unsigned char*>(d.X);
    p.ldx = d.ldx;
    p.y = d.y;
    p.N = d.N;
    p.K = d.K;
    p.scale = d.col_scale;
    p.beta = betas;
    p.mean = means;
    p.prec = prec;
    p.precs = precs;
    p.nb = nb;
    p.out = out;
    p.partials = partials;
    p.gpart = gpart;
    p.counters = counters;
    p.nblocks = pl.nblocks;
    p.group = pl.group;
    p.interleave = pl.interleave;
    p.family = d.family;
    p.w_out = NB == 1 ? w_out : nullptr;
    p.chain = NB == 1 ? static_cast<const glmk::ChainParams*>(chain) : nullptr;
}

glm_status launch_fused(const glm_dataset_desc& d, const Plan& pl, const void* fn, int NB,
                        const double* betas, const double* means, const double* precs,
                        double prec, int nb, double* out, Scratch* s, hipStream_t stream,
                        double* w_out, const void* chain) {
    glmk::FgParams p;
    fused_params(d, pl, NB, betas, means, precs, prec, nb, out, s->partials, s->gpart, s->counters,
                 w_out, chain, &p);
    void* args[] = {&p};
    GLM_HIP_CHECK(hipLaunchKernel(fn, dim3(pl.nblocks), dim3(pl.wpb * 64), args, 0, stream));
    return GLM_OK;
}

static glm_status launch_plain(glm_ctx* ctx, const Dataset& ds, const double* beta,
                               const glm_prior* prior, double* out, void* stream) {
    size_t np, ng, nc;
    scratch_need(ds.plan, ds.d.K, 1, &np, &ng, &nc);
    Scratch* s = nullptr;
    glm_status st = get_scratch(ctx, stream, np, ng, nc, &s);
    if (st != GLM_OK) return st;
    return launch_fused(ds.d, ds.plan, ds.plan.fn, 1, beta, prior->mean, nullptr, prior->prec, 1,
                        out, s, (hipStream_t)stream);
}

// ------------------------------------------------------------ static scratch
//
// The allocation-free plain call keeps its block partials, group partials and
// tickets in this file-scope device array instead of the per-stream scratch.
// Host code never passes the array's name to a kernel (on the host it is only
// a stand-in for the symbol): its device address is looked up once per device
// at context creation and kept in g_static_ptr.  Layout: kStaticTickets
// tickets (zero between calls: cleared at set-up, reset by each launch's
// merge), then the partials.
constexpr size_t kStaticBytes = size_t(4) << 20;
constexpr size_t kStaticTickets = 1024;
static __device__ __align__(256) double scratch[kStaticBytes / sizeof(double)];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
void* g_static_ptr[kMaxDevices] = {};
}  // namespace

glm_status static_scratch_setup(int device) {
    if (device < 0 || device >= kMaxDevices)
        GLM_FAIL(GLM_EINVAL, "static scratch: device %d beyond %d", device, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (g_static_ptr[device]) return GLM_OK;
    void* ptr = nullptr;
    GLM_HIP_CHECK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) GLM_FAIL(GLM_EHIP, "static scratch: no device address for device %d", device);
    GLM_HIP_CHECK(hipMemset(ptr, 0, kStaticTickets * sizeof(unsigned)));
    GLM_HIP_CHECK(hipDeviceSynchronize());
    g_static_ptr[device] = ptr;
    return GLM_OK;
}

static glm_status launch_plain_static(glm_ctx* ctx, const Dataset& ds, const double* beta,
                                      const glm_prior* prior, double* out, void* stream) {
    void* base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_static_mu);
        base = g_static_ptr[ctx->device];
    }
    if (!base) GLM_FAIL(GLM_EHIP, "glm_logpost_grad_noalloc: static scratch not set up");
    size_t np, ng, nc;
    scratch_need(ds.plan, ds.d.K, 1, &np, &ng, &nc);
    const size_t tick_bytes = kStaticTickets * sizeof(unsigned);
    const size_t need = tick_bytes + (np + ng) * sizeof(double);
    if (nc > kStaticTickets || need > kStaticBytes)
        GLM_FAIL(GLM_EINVAL,
                 "glm_logpost_grad_noalloc: this data set's launch needs %zu bytes of scratch "
                 "(%zu tickets), the static scratch holds %zu bytes (%zu tickets); use "
                 "glm_logpost_grad",
                 need, nc, kStaticBytes, kStaticTickets);
    Scratch s;
    s.counters = static_cast<unsigned*>(base);
    s.partials = reinterpret_cast<double*>(static_cast<char*>(base) + tick_bytes);
    s.gpart = s.partials + np;
    return launch_fused(ds.d, ds.plan, ds.plan.fn, 1, beta, prior->mean, nullptr, prior->prec, 1,
                        out, &s, (hipStream_t)stream);
}

}  // namespace glmrt

using namespace glmrt;

extern "C" {

glm_status glm_logpost_grad_noalloc(glm_ctx* ctx, glm_dataset_id id, const double* beta,
                                    const glm_prior* prior, double* out, void* stream) {
    clear_error();
    if (!ctx || !beta || !prior || !out)
        GLM_FAIL(GLM_EINVAL, "glm_logpost_grad_noalloc: NULL argument");
    if (!(prior->prec >= 0.0))
        GLM_FAIL(GLM_EINVAL, "glm_logpost_grad_noalloc: prior precision < 0");
    std::lock_guard<std::mutex> lk(ctx->mu);
    auto it = ctx->datasets.find(id);
    if (it == ctx->datasets.end())
        GLM_FAIL(GLM_ENOTFOUND, "glm_logpost_grad_noalloc: unknown data set %lld", (long long)id);
    glm_status st = use_device(ctx);
    if (st != GLM_OK) return st;
    return launch_plain_static(ctx, it->second, beta, prior, out, stream);
}

glm_status glm_logpost_grad(glm_ctx* ctx, glm_dataset_id id, const double* beta,
                            const glm_prior* prior, double* out, void* stream) {
    clear_error();
    if (!ctx || !beta || !prior || !out) GLM_FAIL(GLM_EINVAL, "glm_logpost_grad: NULL argument");
    if (!(prior->prec >= 0.0)) GLM_FAIL(GLM_EINVAL, "glm_logpost_grad: prior precision < 0");
    std::lock_guard<std::mutex> lk(ctx->mu);
    auto it = ctx->datasets.find(id);
    if (it == ctx->datasets.end())
        GLM_FAIL(GLM_ENOTFOUND, "glm_logpost_grad: unknown data set %lld", (long long)id);
    glm_status st = use_device(ctx);
    if (st != GLM_OK) return st;
    return launch_plain(ctx, it->second, beta, prior, out, stream);
}

glm_status glm_logpost_grad_host(glm_ctx* ctx, glm_dataset_id id, const double* beta_host,
                                 const glm_prior* prior, double* f, double* g_host) {
    clear_error();
    if (!ctx || !beta_host || !prior || !f)
        GLM_FAIL(GLM_EINVAL, "glm_logpost_grad_host: NULL argument");
    if (!(prior->prec >= 0.0)) GLM_FAIL(GLM_EINVAL, "glm_logpost_grad_host: prior precision < 0");
    std::lock_guard<std::mutex> lk(ctx->mu);
    auto it = ctx->datasets.find(id);
    if (it == ctx->datasets.end())
        GLM_FAIL(GLM_ENOTFOUND, "glm_logpost_grad_host: unknown data set %lld", (long long)id);
    glm_status st = use_device(ctx);
    if (st != GLM_OK) return st;
    const int K = it->second.d.K;
    const size_t need = 3 * (size_t)K + 1;
    if (ctx->stage_cap < need) {
        if (ctx->h_stage) hipHostFree(ctx->h_stage);
        if (ctx->d_stage) hipFree(ctx->d_stage);
        ctx->h_stage = nullptr;
        ctx->d_stage = nullptr;
        ctx->stage_cap = 0;
        // coherent: the kernel writes f and g straight into it (no copy back)
        GLM_HIP_CHECK(hipHostMalloc((void**)&ctx->h_stage, need * sizeof(double), hipHostMallocCoherent));
        GLM_HIP_CHECK(hipMalloc((void**)&ctx->d_stage, need * sizeof(double)));
        ctx->stage_cap = need;
    }
    double* hb = ctx->h_stage;
    double* db = ctx->d_stage;
    std::memcpy(hb, beta_host, K * sizeof(double));
    size_t nin = K;
    glm_prior pd = *prior;
    if (prior->mean) {
        std::memcpy(hb + K, prior->mean, K * sizeof(double));
        pd.mean = db + K;
        nin = 2 * (size_t)K;
    }
    hipStream_t s = ctx->own_stream;
    GLM_HIP_CHECK(hipMemcpyAsync(db, hb, nin * sizeof(double), hipMemcpyHostToDevice, s));
    st = launch_plain(ctx, it->second, db, &pd, hb + 2 * K, s);
    if (st != GLM_OK) return st;
    GLM_HIP_CHECK(hipStreamSynchronize(s));
    *f = hb[2 * K];
    if (g_host) std::memcpy(g_host, hb + 2 * K + 1, K * sizeof(double));
    return GLM_OK;
}

}  // extern "C"
