// Batched (hierarchical-model) entry points: group sets, their static work
// schedule and its autotuning.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <queue>
#include <string>

#include "fg_batched.hpp"
#include "runtime.hpp"

using glmk::BatchItem;

struct glm_groupset {
    glm_ctx* ctx = nullptr;
    glm_dataset_desc d{};
    int G = 0;
    std::vector<int64_t> offsets;
    // kernel instance
    const void* fn = nullptr;
    int lpr = 1, cpl = 1, R = 16, wpb = 4, batch_rows = 0;
    // schedule
    int nblocks = 1;
    int64_t tile_rows = 0;
    int n_items = 0, n_tiles = 0;
    double tuned_us = 0.0;
    // device buffers (one allocation)
    void* dev = nullptr;
    BatchItem* d_items = nullptr;
    int32_t* d_wave_items = nullptr;
    int32_t* d_tile_first = nullptr;
    int32_t* d_tile_count = nullptr;
    int32_t* d_bg_ptr = nullptr;
    int32_t* d_bg = nullptr;
    int32_t* d_group_blocks = nullptr;
    double* d_partials = nullptr;
    unsigned* d_counters = nullptr;
};

namespace glmrt {
namespace {

constexpr int WPB = 4;

// Row slots per lane: 16 slots of 16 bytes, or 8 for FP32 (its FP64
// gradient products keep r in FP64; 8 slots keep two waves per SIMD),
// divided by the chunks per lane of wide rows; FP8 rows of 4 chunks per
// lane take one slot, as in the plain kernel (4 spilled to scratch memory).
template <int DT, int CPL>
constexpr int rb() {
    return DT == glmk::DT_FP8 && CPL == 4 ? 1 : (DT == glmk::DT_F32 ? 8 : 16) / CPL;
}

struct BInst {
    const void* fn;
    int R;
};

template <int DT, int LPR, int CPL>
BInst binst() {
    constexpr int R = rb<DT, CPL>();
    return BInst{reinterpret_cast<const void*>(&glmk::fg_batched<DT, LPR, CPL, R, WPB>), R};
}

template <int DT>
BInst bpick(int lpr, int cpl) {
    if (cpl == 1) {
        switch (lpr) {
        case 1: return binst<DT, 1, 1>();
        case 2: return binst<DT, 2, 1>();
        case 4: return binst<DT, 4, 1>();
        case 8: return binst<DT, 8, 1>();
        case 16: return binst<DT, 16, 1>();
        case 32: return binst<DT, 32, 1>();
        case 64: return binst<DT, 64, 1>();
        }
    } else if (lpr == 64) {
        if (cpl == 2) return binst<DT, 64, 2>();
        if (cpl == 4) return binst<DT, 64, 4>();
    }
    return BInst{nullptr, 0};
}

BInst bpick_any(int dt, int lpr, int cpl) {
    switch (dt) {
    case GLM_F64: return bpick<glmk::DT_F64>(lpr, cpl);
    case GLM_F32: return bpick<glmk::DT_F32>(lpr, cpl);
    case GLM_BF16: return bpick<glmk::DT_BF16>(lpr, cpl);
    case GLM_FP8_E4M3: return bpick<glmk::DT_FP8>(lpr, cpl);
    }
    return BInst{nullptr, 0};
}

struct Schedule {
    std::vector<BatchItem> items;          // grouped by wave
    std::vector<int32_t> wave_items;       // waves + 1
    std::vector<int32_t> tile_first, tile_count;
    std::vector<int32_t> block_groups_ptr; // blocks + 1
    std::vector<int32_t> block_groups;     // split groups with tiles in each block
    std::vector<int32_t> group_blocks;     // per group: distinct blocks holding its tiles
    int n_tiles = 0;
};

// Splits groups longer than T rows into near-equal tiles and assigns the
// items to `waves` queues, longest first onto the least-loaded queue
// (cost = bytes of X read plus a fixed per-item overhead), then orders each
// queue by row position.
Schedule build_schedule(const std::vector<int64_t>& off, int64_t T, int waves, int wpb,
                        double row_bytes, double item_overhead_bytes) {
    Schedule s;
    const int G = (int)off.size() - 1;
    s.tile_first.assign(G, 0);
    s.tile_count.assign(G, 0);
    std::vector<BatchItem> all;
    for (int g = 0; g < G; ++g) {
        const int64_t a = off[g], n = off[g + 1] - off[g];
        if (n <= T) {
            all.push_back(BatchItem{a, a + n, g, -1});
            continue;
        }
        const int64_t m = (n + T - 1) / T;
        s.tile_first[g] = s.n_tiles;
        s.tile_count[g] = (int32_t)m;
        for (int64_t j = 0; j < m; ++j)
            all.push_back(BatchItem{a + n * j / m, a + n * (j + 1) / m, g, s.n_tiles++});
    }
    std::vector<double> cost(all.size());
    for (size_t i = 0; i < all.size(); ++i)
        cost[i] = (double)(all[i].r1 - all[i].r0) * row_bytes + item_overhead_bytes;
    std::vector<size_t> order(all.size());
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) { return cost[x] > cost[y]; });
    using QE = std::pair<double, int>;
    std::priority_queue<QE, std::vector<QE>, std::greater<QE>> heap;
    for (int w = 0; w < waves; ++w) heap.push({0.0, w});
    std::vector<std::vector<size_t>> per(waves);
    for (size_t i : order) {
        QE q = heap.top();
        heap.pop();
        per[q.second].push_back(i);
        heap.push({q.first + cost[i], q.second});
    }
    s.wave_items.assign(waves + 1, 0);
    for (int w = 0; w < waves; ++w) {
        std::sort(per[w].begin(), per[w].end(), [&](size_t x, size_t y) { return all[x].r0 < all[y].r0; });
        for (size_t i : per[w]) s.items.push_back(all[i]);
        s.wave_items[w + 1] = (int32_t)s.items.size();
    }
    // which blocks hold tiles of each split group
    const int nblocks = waves / wpb;
    std::vector<std::vector<int32_t>> bg(nblocks);
    for (int w = 0; w < waves; ++w)
        for (int i = s.wave_items[w]; i < s.wave_items[w + 1]; ++i)
            if (s.items[i].tile >= 0) bg[w / wpb].push_back(s.items[i].group);
    s.group_blocks.assign(G, 0);
    s.block_groups_ptr.assign(nblocks + 1, 0);
    for (int b = 0; b < nblocks; ++b) {
        std::sort(bg[b].begin(), bg[b].end());
        bg[b].erase(std::unique(bg[b].begin(), bg[b].end()), bg[b].end());
        for (int32_t g : bg[b]) {
            s.block_groups.push_back(g);
            s.group_blocks[g] += 1;
        }
        s.block_groups_ptr[b + 1] = (int32_t)s.block_groups.size();
    }
    return s;
}

void free_dev(glm_groupset* gs) {
    if (gs->dev) (void)hipFree(gs->dev);
    gs->dev = nullptr;
}

glm_status upload(glm_groupset* gs, const Schedule& s) {
    free_dev(gs);
    const int K1 = gs->d.K + 1;
    const size_t n_it = s.items.size(), n_w = s.wave_items.size(), G = gs->G;
    const size_t nt = std::max(1, s.n_tiles);
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t b_items = al(n_it * sizeof(BatchItem) + 1);
    const size_t b_w = al(n_w * 4);
    const size_t b_tf = al(G * 4 + 1), b_tc = al(G * 4 + 1);
    const size_t b_part = al(nt * K1 * 8);
    const size_t b_cnt = al(G * 4 + 1);
    const size_t n_bgp = s.block_groups_ptr.size(), n_bg = s.block_groups.size();
    const size_t b_bgp = al(n_bgp * 4 + 1), b_bg = al(n_bg * 4 + 1), b_gb = al(G * 4 + 1);
    const size_t total = b_items + b_w + b_tf + b_tc + b_part + b_cnt + b_bgp + b_bg + b_gb;
    hipError_t e = hipMalloc(&gs->dev, total);
    if (e != hipSuccess) GLM_FAIL(GLM_ENOMEM, "group set: device allocation of %zu bytes failed", total);
    char* p = (char*)gs->dev;
    gs->d_items = (BatchItem*)p;
    p += b_items;
    gs->d_wave_items = (int32_t*)p;
    p += b_w;
    gs->d_tile_first = (int32_t*)p;
    p += b_tf;
    gs->d_tile_count = (int32_t*)p;
    p += b_tc;
    gs->d_partials = (double*)p;
    p += b_part;
    gs->d_counters = (unsigned*)p;
    p += b_cnt;
    gs->d_bg_ptr = (int32_t*)p;
    p += b_bgp;
    gs->d_bg = (int32_t*)p;
    p += b_bg;
    gs->d_group_blocks = (int32_t*)p;
    GLM_HIP_CHECK(hipMemcpy(gs->d_items, s.items.data(), n_it * sizeof(BatchItem), hipMemcpyHostToDevice));
    GLM_HIP_CHECK(hipMemcpy(gs->d_wave_items, s.wave_items.data(), n_w * 4, hipMemcpyHostToDevice));
    GLM_HIP_CHECK(hipMemcpy(gs->d_tile_first, s.tile_first.data(), G * 4, hipMemcpyHostToDevice));
    GLM_HIP_CHECK(hipMemcpy(gs->d_tile_count, s.tile_count.data(), G * 4, hipMemcpyHostToDevice));
    GLM_HIP_CHECK(hipMemcpy(gs->d_bg_ptr, s.block_groups_ptr.data(), n_bgp * 4, hipMemcpyHostToDevice));
    if (n_bg) GLM_HIP_CHECK(hipMemcpy(gs->d_bg, s.block_groups.data(), n_bg * 4, hipMemcpyHostToDevice));
    GLM_HIP_CHECK(hipMemcpy(gs->d_group_blocks, s.group_blocks.data(), G * 4, hipMemcpyHostToDevice));
    GLM_HIP_CHECK(hipMemset(gs->d_counters, 0, G * 4));
    GLM_HIP_CHECK(hipDeviceSynchronize());
    gs->n_items = (int)n_it;
    gs->n_tiles = s.n_tiles;
    return GLM_OK;
}

glm_status apply_schedule(glm_groupset* gs, int64_t T, int bpc) {
    const int waves = gs->ctx->num_cu * bpc * gs->wpb;
    const double row_bytes = (double)gs->d.ldx * elem_size(gs->d.dtype);
    const Schedule s =
        build_schedule(gs->offsets, T, waves, gs->wpb, row_bytes, 1.0 * gs->batch_rows * row_bytes);
    glm_status st = upload(gs, s);
    if (st != GLM_OK) return st;
    gs->tile_rows = T;
    gs->nblocks = gs->ctx->num_cu * bpc;
    return GLM_OK;
}

glm_status launch_batched(glm_groupset* gs, const double* betas, const glm_prior* prior, double* out,
                          hipStream_t stream) {
    glmk::BatchedParams p;
    p.X = static_cast<const unsigned char*>(gs->d.X);
    p.ldx = gs->d.ldx;
    p.y = gs->d.y;
    p.K = gs->d.K;
    p.scale = gs->d.col_scale;
    p.betas = betas;
    p.mean = prior->mean;
    p.mean_per_group = prior->mean_per_group;
    p.prec = prior->prec;
    p.out = out;
    p.items = gs->d_items;
    p.wave_items = gs->d_wave_items;
    p.tile_first = gs->d_tile_first;
    p.tile_count = gs->d_tile_count;
    p.block_groups_ptr = gs->d_bg_ptr;
    p.block_groups = gs->d_bg;
    p.group_blocks = gs->d_group_blocks;
    p.partials = gs->d_partials;
    p.counters = gs->d_counters;
    p.family = gs->d.family;
    void* args[] = {&p};
    GLM_HIP_CHECK(hipLaunchKernel(gs->fn, dim3(gs->nblocks), dim3(gs->wpb * 64), args, 0, stream));
    return GLM_OK;
}

// Times each candidate (tile rows, blocks per CU) on the group set itself at
// beta = 0 and keeps the fastest; the choice is remembered per shape.
glm_status autotune(glm_groupset* gs) {
    const std::string key = "batched|" + gs->ctx->arch + "|" + std::to_string(gs->d.dtype) + "|" +
                            std::to_string(gs->d.K) + "|" + std::to_string(gs->G) + "|" +
                            std::to_string(gs->d.N);
    TuneEntry te;
    if (tune_cache_get(key, &te)) return apply_schedule(gs, te.a, te.b);
    const int K1 = gs->d.K + 1;
    double* dz = nullptr;
    const size_t nbeta = (size_t)gs->G * gs->d.K, nout = (size_t)gs->G * K1;
    GLM_HIP_CHECK(hipMalloc(&dz, (nbeta + nout) * sizeof(double)));
    GLM_HIP_CHECK(hipMemset(dz, 0, nbeta * sizeof(double)));
    hipEvent_t e0, e1;
    GLM_HIP_CHECK(hipEventCreate(&e0));
    GLM_HIP_CHECK(hipEventCreate(&e1));
    glm_prior pr{1.0, nullptr, 0};
    double best = 1e30;
    int64_t bestT = 0;
    int bestB = 1;
    glm_status st = GLM_OK;
    for (int mult : {2, 4, 8, 12, 16, 24, 32, 48, 64}) {
        for (int bpc : {1, 2}) {
            const int64_t T = (int64_t)gs->batch_rows * mult;
            st = apply_schedule(gs, T, bpc);
            if (st != GLM_OK) break;
            for (int w = 0; w < 3 && st == GLM_OK; ++w) st = launch_batched(gs, dz, &pr, dz + nbeta, nullptr);
            if (st != GLM_OK) break;
            const int reps = 20;   // a few microseconds separate the candidates
            GLM_HIP_CHECK(hipEventRecord(e0, nullptr));
            for (int r = 0; r < reps && st == GLM_OK; ++r) st = launch_batched(gs, dz, &pr, dz + nbeta, nullptr);
            GLM_HIP_CHECK(hipEventRecord(e1, nullptr));
            GLM_HIP_CHECK(hipEventSynchronize(e1));
            if (st != GLM_OK) break;
            float ms = 0;
            GLM_HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
            const double us = ms * 1e3 / reps;
            if (std::getenv("GLM_TUNE_VERBOSE"))
                std::fprintf(stderr, "[glm tune] batched T=%lld blocks/CU=%d items=%d tiles=%d: %.1f us\n",
                             (long long)T, bpc, gs->n_items, gs->n_tiles, us);
            if (us < best) {
                best = us;
                bestT = T;
                bestB = bpc;
            }
        }
        if (st != GLM_OK) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(dz);
    if (st != GLM_OK) return st;
    gs->tuned_us = best;
    tune_cache_put(key, TuneEntry{bestT, bestB, best});
    return apply_schedule(gs, bestT, bestB);
}

}  // namespace
}  // namespace glmrt

using namespace glmrt;

extern "C" {

glm_status glm_groupset_create(glm_ctx* ctx, const glm_dataset_desc* d, const int64_t* offsets,
                               int32_t G, int32_t tune, glm_groupset** out) {
    clear_error();
    if (!ctx || !d || !offsets || !out) GLM_FAIL(GLM_EINVAL, "glm_groupset_create: NULL argument");
    *out = nullptr;
    if (G < 1) GLM_FAIL(GLM_EINVAL, "glm_groupset_create: G = %d < 1", G);
    if (offsets[0] != 0) GLM_FAIL(GLM_EINVAL, "glm_groupset_create: offsets[0] must be 0");
    for (int g = 0; g < G; ++g)
        if (offsets[g + 1] < offsets[g])
            GLM_FAIL(GLM_EINVAL, "glm_groupset_create: offsets decrease at group %d", g);
    if (offsets[G] != d->N)
        GLM_FAIL(GLM_EINVAL, "glm_groupset_create: offsets[G] = %lld but N = %lld",
                 (long long)offsets[G], (long long)d->N);
    // same checks and kernel geometry as a plain data set
    std::lock_guard<std::mutex> lk(ctx->mu);
    glm_status st = validate_desc(*d);
    if (st != GLM_OK) return st;
    Plan plan;
    st = make_plan(ctx, *d, &plan);
    if (st != GLM_OK) return st;
    st = use_device(ctx);
    if (st != GLM_OK) return st;
    std::unique_ptr<glm_groupset> gs(new glm_groupset);
    gs->ctx = ctx;
    gs->d = *d;
    gs->G = G;
    gs->offsets.assign(offsets, offsets + G + 1);
    gs->lpr = plan.lpr;
    gs->cpl = plan.cpl;
    const BInst bi = bpick_any(d->dtype, plan.lpr, plan.cpl);
    if (!bi.fn) GLM_FAIL(GLM_EINVAL, "glm_groupset_create: no kernel instance for K = %d", d->K);
    gs->R = bi.R;
    gs->wpb = WPB;
    gs->batch_rows = bi.R * (64 / plan.lpr);
    gs->fn = bi.fn;
    if (tune)
        st = autotune(gs.get());
    else
        st = apply_schedule(gs.get(), (int64_t)gs->batch_rows * 8, 1);
    if (st != GLM_OK) {
        free_dev(gs.get());
        return st;
    }
    *out = gs.release();
    return GLM_OK;
}

glm_status glm_groupset_destroy(glm_groupset* gs) {
    clear_error();
    if (!gs) return GLM_OK;
    (void)hipSetDevice(gs->ctx->device);
    (void)hipDeviceSynchronize();
    free_dev(gs);
    delete gs;
    return GLM_OK;
}

glm_status glm_groupset_query(const glm_groupset* gs, glm_groupset_info* info) {
    clear_error();
    if (!gs || !info) GLM_FAIL(GLM_EINVAL, "glm_groupset_query: NULL argument");
    info->tile_rows = gs->tile_rows;
    info->blocks = gs->nblocks;
    info->waves = gs->nblocks * gs->wpb;
    info->items = gs->n_items;
    info->split_tiles = gs->n_tiles;
    info->tuned_us = gs->tuned_us;
    return GLM_OK;
}

glm_status glm_logpost_grad_batched(glm_ctx* ctx, glm_groupset* gs, const double* betas,
                                    const glm_prior* prior, double* out, void* stream) {
    clear_error();
    if (!ctx || !gs || !betas || !prior || !out)
        GLM_FAIL(GLM_EINVAL, "glm_logpost_grad_batched: NULL argument");
    if (gs->ctx != ctx) GLM_FAIL(GLM_EINVAL, "glm_logpost_grad_batched: group set of another context");
    if (!(prior->prec >= 0.0)) GLM_FAIL(GLM_EINVAL, "glm_logpost_grad_batched: prior precision < 0");
    glm_status st = use_device(ctx);
    if (st != GLM_OK) return st;
    return launch_batched(gs, betas, prior, out, (hipStream_t)stream);
}

}  // extern "C"
