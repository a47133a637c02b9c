// Batched evaluation for the hierarchical model (Sec. 4.1): G groups, each
// with its own rows of the stacked X / y and its own coefficient vector,
// evaluated in one launch.
//
// The host splits groups larger than T rows into near-equal tiles and
// assigns the resulting work items to waves ahead of time by a size proxy
// (longest processing time first), the static pre-allocation the paper
// proposes for uneven groups (Sec. 4.1).  A wave streams each of its items
// with the same tile machinery as the plain kernel.  An item that is a whole
// group is finished by its wave (no cross-wave traffic at all); the tiles of
// a split group write partials, and the last tile to finish (atomic ticket
// per group) adds them in tile order and applies the group's prior.
#pragma once

#include "fg_kernel.hpp"

namespace glmk {

struct BatchItem {
    int64_t r0, r1;   // rows [r0, r1) of the stacked matrix
    int32_t group;
    int32_t tile;     // -1: the whole group; else partial slot index
};

struct BatchedParams {
    const unsigned char* X;
    int64_t ldx;
    const uint8_t* y;
    int K;
    const float* scale;          // FP8 column scales
    const double* betas;         // G x K
    const double* mean;          // nullptr, K, or G x K (mean_per_group)
    int mean_per_group;
    double prec;
    double* out;                 // G x (1 + K)
    const BatchItem* items;
    const int32_t* wave_items;   // total_waves + 1 offsets into items
    const int32_t* tile_first;   // per group: first partial slot (split groups)
    const int32_t* tile_count;   // per group: number of tiles (0 = not split)
    const int32_t* block_groups_ptr;   // nblocks + 1 offsets into block_groups
    const int32_t* block_groups;       // split groups each block holds tiles of
    const int32_t* group_blocks;       // per group: number of distinct blocks holding its tiles
    double* partials;            // ntiles x (1 + K)
    unsigned* counters;          // G tickets, zero between launches
    int family;                  // response family (0 logistic, 1 Poisson)
};

template <int DT, int LPR, int CPL, int R, int WPB>
__global__ __launch_bounds__(WPB * 64) void fg_batched(BatchedParams p) {
    using WT = WaveTile<DT, LPR, CPL, R>;
    using Tile = typename WT::Tile;
    constexpr int VE = WT::VE;
    constexpr int NT = WPB * 64;
    constexpr int BATCH = WT::BATCH;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int gw = blockIdx.x * WPB + wave;
    const int K = p.K;
    const int K1 = K + 1;

    WT wt;
    wt.init(threadIdx.x & 63, K, p.ldx, p.family);
    __shared__ typename WT::rtype rbuf[WPB][WT::RBUF];

    // The wave's items are streamed as one sequence of batches, so the next
    // batch is prefetched across item boundaries too; every item yields at
    // least one batch (an empty group one empty batch).  Queue state and
    // batch descriptors are wave-uniform (scalar registers).  The item
    // descriptors are copied into LDS up to kItemsLds at a time, so moving to
    // the next item waits on LDS, not on memory: a vector-memory wait would
    // also drain the wave's tile loads in flight, and under the streaming
    // load a dependent memory access takes microseconds.
    constexpr int kItemsLds = 32;
    __shared__ BatchItem s_items[WPB][kItemsLds];
    const int lane = threadIdx.x & 63;
    const int it0 = p.wave_items[gw];
    const int it1 = p.wave_items[gw + 1];
    int ibase = -kItemsLds;   // first item (relative to it0) held in LDS
    auto item = [&](int it) {
        const int rel = it - it0;
        if (rel < ibase || rel >= ibase + kItemsLds) {   // rare: every kItemsLds items
            ibase = rel - rel % kItemsLds;
            if (lane < kItemsLds) {
                const int i = it0 + ibase + lane;
                s_items[wave][lane] = i < it1 ? p.items[i] : BatchItem{0, 0, 0, -1};
            }
            __builtin_amdgcn_wave_barrier();
        }
        const BatchItem& e = s_items[wave][rel - ibase];
        BatchItem r;
        r.r0 = ((int64_t)__builtin_amdgcn_readfirstlane((int)(e.r0 >> 32)) << 32) |
               (uint32_t)__builtin_amdgcn_readfirstlane((int)e.r0);
        r.r1 = ((int64_t)__builtin_amdgcn_readfirstlane((int)(e.r1 >> 32)) << 32) |
               (uint32_t)__builtin_amdgcn_readfirstlane((int)e.r1);
        r.group = __builtin_amdgcn_readfirstlane(e.group);
        r.tile = __builtin_amdgcn_readfirstlane(e.tile);
        return r;
    };
    int qit = it0;                                   // item of the next batch to load
    BatchItem qitem{0, 0, 0, -1};
    if (qit < it1) qitem = item(qit);
    int64_t qr = qitem.r0;                           // its first row

    // Where registers allow (CPL x VE <= 8), the coefficients and prior
    // means of the next item are loaded when an item starts (the first at
    // the start), so starting and ending an item waits on no memory; wider
    // rows load them when the item starts and ends.
    constexpr bool PF = CPL * VE <= 8;
    constexpr int PVE = PF ? VE : 1;   // prefetch array extent (unused without)
    double pb[CPL][PVE], pm[CPL][PVE];
    auto prefetch = [&](int g) {
        if constexpr (PF) {
            // buffer loads: columns past K, and a missing mean, read as zeros
            // without a branch, so the loads write the registers directly
            const double* mn =
                p.mean ? (p.mean_per_group ? p.mean + (int64_t)g * K : p.mean) : nullptr;
            const __amdgpu_buffer_rsrc_t rb = __builtin_amdgcn_make_buffer_rsrc(
                (void*)(p.betas + (int64_t)g * K), 0, K * 8, kRsrcWord3);
            const __amdgpu_buffer_rsrc_t rm = __builtin_amdgcn_make_buffer_rsrc(
                (void*)(mn ? mn : p.betas), 0, mn ? K * 8 : 0, kRsrcWord3);
#pragma unroll
            for (int i = 0; i < CPL; ++i)
#pragma unroll
                for (int e = 0; e < VE; ++e) {
                    const uint32_t off = (uint32_t)wt.col(i, e) * 8u;
                    const u32x2 wb = __builtin_amdgcn_raw_buffer_load_b64(rb, off, 0, 0);
                    const u32x2 wm = __builtin_amdgcn_raw_buffer_load_b64(rm, off, 0, 0);
                    pb[i][e] = __longlong_as_double((long long)(((unsigned long long)wb[1] << 32) | wb[0]));
                    pm[i][e] = __longlong_as_double((long long)(((unsigned long long)wm[1] << 32) | wm[0]));
                }
        }
    };

    struct Meta {
        int it;          // item index, it1 = none
        int group, tile; // its group and partial slot (-1: whole group)
        int64_t row0, r1;
        bool first, last;
    };
    auto next = [&]() {
        Meta m;
        m.it = qit;
        m.group = qitem.group;
        m.tile = qitem.tile;
        m.row0 = qr;
        m.r1 = qit < it1 ? qitem.r1 : 0;
        m.first = qit < it1 && qr == qitem.r0;
        m.last = qit < it1 && qr + BATCH >= qitem.r1;
        if (qit < it1) {
            if (qr + BATCH < qitem.r1) {
                qr += BATCH;
            } else {
                ++qit;
                if (qit < it1) {
                    qitem = item(qit);
                    qr = qitem.r0;
                }
            }
        }
        return m;
    };

    double dp[CPL][PVE];   // beta - prior mean per column of the item being computed (PF)
    int cgroup = 0, ctile = -1;
    auto compute = [&](Tile& t, const Meta& m) {
        if (m.first) {
            cgroup = m.group;
            ctile = m.tile;
            if constexpr (PF) {
#pragma unroll
                for (int i = 0; i < CPL; ++i)
#pragma unroll
                    for (int e = 0; e < VE; ++e) {
                        dp[i][e] = pb[i][e] - pm[i][e];
                        if constexpr (DT == DT_FP8)
                            wt.bd[0][i][e] = pb[i][e] * (double)p.scale[wt.col(i, e)];
                        else
                            wt.bd[0][i][e] = pb[i][e];
                        // the prefetch below may reuse the registers of pb
                        // and pm only once these are computed
                        asm volatile("" : "+v"(dp[i][e]), "+v"(wt.bd[0][i][e]));
                    }
                asm volatile("" ::: "memory");
                // unconditional (group 0 past the last item), so that the
                // loads write the prefetch registers directly and nothing
                // waits on them before the next item starts
                prefetch(m.it + 1 < it1 ? item(m.it + 1).group : 0);
            } else {
                wt.set_beta(0, p.betas + (int64_t)cgroup * K, p.scale);
            }
            wt.zero_acc();
        }
        wt.compute(t, (uint32_t)max((int64_t)0, min((int64_t)BATCH, m.r1 - m.row0)), rbuf[wave]);
        if (!m.last) return;
        // item done: whole group -> its result; tile of a split group -> its partial
        wt.wave_totals();
        const int g = cgroup;
        const double* beta = p.betas + (int64_t)g * K;
        const double* mn = p.mean ? (p.mean_per_group ? p.mean + (int64_t)g * K : p.mean) : nullptr;
        double* dst = ctile < 0 ? nullptr : p.partials + (int64_t)ctile * K1;
        double* o = p.out + (int64_t)g * K1;
        double pf = 0.0;
        if (wt.seg == 0) {
#pragma unroll
            for (int i = 0; i < CPL; ++i)
#pragma unroll
                for (int e = 0; e < VE; ++e)
                    if (wt.elem_ok(i, e)) {
                        const int k = wt.col(i, e);
                        double v = wt.g64[0][i][e];
                        if constexpr (DT == DT_FP8) v *= (double)p.scale[k];
                        if (dst) {
                            publish(dst + 1 + k, v);
                        } else {
                            double d;
                            if constexpr (PF) d = dp[i][e];
                            else d = beta[k] - (mn ? mn[k] : 0.0);
                            pf += d * d;
                            o[1 + k] = v - p.prec * d;
                        }
                    }
        }
        if (dst) {
            if (wt.lane == 0) publish(dst, wt.facc[0]);
        } else {
            for (int d = 1; d < LPR; d <<= 1) pf += __shfl_xor(pf, d, 64);
            if (wt.lane == 0) o[0] = wt.facc[0] - 0.5 * p.prec * pf;
        }
    };

    Tile ta, tb;
    Meta ma = next();
    wt.load(ta, p.X, p.y, ma.row0, ma.r1 - ma.row0);
    if (ma.it < it1) prefetch(ma.group);
    while (true) {
        const Meta mb = next();
        wt.load(tb, p.X, p.y, mb.row0, mb.r1 - mb.row0);
        if (ma.it >= it1) break;
        compute(ta, ma);
        if (mb.it >= it1) break;
        ma = next();
        wt.load(ta, p.X, p.y, ma.row0, ma.r1 - ma.row0);
        compute(tb, mb);
    }

    // Split groups: once every wave of this block is done, the block takes
    // one ticket per split group it holds tiles of; the block completing a
    // group's count adds that group's tile partials in tile order.  The
    // partials are published (written through to memory, read coherently), so
    // the tickets need no fences.
    const int q0 = p.block_groups_ptr[blockIdx.x];
    const int q1 = p.block_groups_ptr[blockIdx.x + 1];
    if (q0 == q1) return;
    // Every thread's partial stores complete before the barrier, and the
    // barrier before wave 0's tickets.
    publish_wait();
    __syncthreads();
    __shared__ unsigned s_win[NT];
    for (int qb = q0; qb < q1; qb += NT) {
        if (wave == 0) {
            for (int qq = qb + wt.lane; qq < min(q1, qb + NT); qq += 64) {
                const int g = p.block_groups[qq];
                const unsigned prev = __hip_atomic_fetch_add(&p.counters[g], 1u, __ATOMIC_RELAXED,
                                                             __HIP_MEMORY_SCOPE_AGENT);
                s_win[qq - qb] = prev == (unsigned)(p.group_blocks[g] - 1) ? 1u : 0u;
            }
        }
        __syncthreads();
        // The won groups are spread over the waves (entry j to wave
        // j mod WPB); a wave adds a group's tile partials per column in tile
        // order and its prior term with a butterfly, so groups need no block
        // barrier of their own.
        const int nq = min(NT, q1 - qb);
        for (int j = wave; j < nq; j += WPB) {
            if (!s_win[j]) continue;
            const int g = p.block_groups[qb + j];
            const int t0 = p.tile_first[g];
            const int nt = p.tile_count[g];
            const double* beta = p.betas + (int64_t)g * K;
            const double* m =
                p.mean ? (p.mean_per_group ? p.mean + (int64_t)g * K : p.mean) : nullptr;
            double* o = p.out + (int64_t)g * K1;
            double pf = 0.0, flik = 0.0;
            for (int k = wt.lane; k < K1; k += 64) {
                const double sacc = ordered_sum(p.partials + (int64_t)t0 * K1 + k, nt, K1);
                if (k == 0) {
                    flik = sacc;
                } else {
                    const double d = beta[k - 1] - (m ? m[k - 1] : 0.0);
                    pf += d * d;
                    o[k] = sacc - p.prec * d;
                }
            }
#pragma unroll
            for (int d = 32; d >= 1; d >>= 1) pf += __shfl_xor(pf, d, 64);
            if (wt.lane == 0) {
                o[0] = flik - 0.5 * p.prec * pf;
                __hip_atomic_store(&p.counters[g], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        __syncthreads();
    }
}

}  // namespace glmk
