// Fused log-posterior + gradient kernels for gfx950 (wave64).
//
// One launch streams X exactly once.  For every row tile it computes the
// linear predictor u = X beta ("LA map"), the per-row transcendental terms
// t_n = y_n u_n - softplus(u_n) and r_n = y_n - sigmoid(u_n) ("TR map"), and
// the gradient contribution sum_n r_n x_n ("second LA map") from the same
// registers -- the single-read form of the paper's cache-fused routine
// (Sec. 4.2.1, Hierarchical Loop Structure), with each wave's private
// partials merged once at the end instead of per row (Sec. 4.2.2).
//
// Work layout.  A row of X is split into 16-byte chunks (VE elements).  A
// segment of LPR lanes (a power of two) covers one row, each lane holding
// CPL chunks of it at columns (cl + i*LPR)*VE .. +VE; a wave therefore reads
// RPW = 64/LPR consecutive rows per load instruction (contiguous bytes when
// ldx == K).  Each lane keeps R such row slots in registers per batch.
//
// Per batch:
//   1. issue all R*CPL 16-byte loads (plus the y bytes of owned rows);
//   2. per-lane partial dot products in FP64: every stored value is exact in
//      FP64 (FP32, BF16 and FP8 codes alike) and is multiplied by the FP64
//      beta with FP64 FMAs, so u carries FP64 rounding only.  Without packed
//      FP32 math an FP64 FMA issues at the rate of an FP32 FMA, so the
//      conversion plus one FP64 FMA per value costs what two FP32 FMAs on a
//      hi + lo split of beta cost, at 2^-53 instead of 2^-24 per rounding;
//   3. a transposed butterfly reduction across the LPR lanes of a segment
//      leaves each lane with complete u values of R/LPR rows (or one row
//      shared by LPR/R lanes), so the TR map runs one row per lane, in FP64;
//   4. r is broadcast back through LDS and every lane adds r_j x_j into FP32
//      gradient partials over the R rows of the batch, which are then added
//      into FP64 accumulators.
// f is accumulated in FP64 from each row's t_n.  At the end the block merges
// its waves in LDS (fixed order) and writes one partial of 1 + K doubles.
//
// Cross-block merge.  Blocks can only communicate through memory (the paper
// notes the resulting two-stage reduction, Sec. 4.5).  Here it stays in one
// launch: blocks are grouped by GROUP; the last block of a group to finish
// (atomic ticket) adds the group's partials in block order, and the last
// group to finish adds the group sums in group order and the prior (a single
// group goes straight on to the final sums).  No
// floating-point atomics are used, so the result is bitwise reproducible.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "publish.hpp"
#include "rng.hpp"
#include "tr_math.hpp"

namespace glmk {

enum : int { DT_F64 = 0, DT_F32 = 1, DT_BF16 = 2, DT_FP8 = 3 };

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

template <int DT> struct ElemSize;
template <> struct ElemSize<DT_F64> { static constexpr int v = 8; };
template <> struct ElemSize<DT_F32> { static constexpr int v = 4; };
template <> struct ElemSize<DT_BF16> { static constexpr int v = 2; };
template <> struct ElemSize<DT_FP8> { static constexpr int v = 1; };

// A chain advanced by the evaluation kernel itself: the launch evaluates f
// and g at the point beta_prop (its beta), and the last block then takes the
// sampler's step and writes the next point to evaluate, so a chain costs one
// launch per evaluation.
//   kind 0, random-walk Metropolis: one evaluation per step; increments and
//     log-uniforms are inputs.
//   kind 1, Hamiltonian Monte Carlo: n_leap evaluations per iteration
//     (leapfrog positions); momenta and the accept uniform are drawn on the
//     device from the counter-based streams of rng.hpp.
struct ChainParams {
    double* beta;             // K, the chain state
    double* fg;               // 1 + K, f and g at the state
    double* beta_prop;        // K, the point being evaluated (this launch's beta)
    const double* incs;       // MH: n_steps x K proposal increments
    const double* logu;       // MH: n_steps log-uniforms
    unsigned* step;           // MH: step t; HMC: iteration t, then leapfrog position l
    int n_steps;              // MH steps or HMC iterations
    uint8_t* accepted;        // n_steps or nullptr
    double* f_trace;          // n_steps or nullptr
    int kind = 0;             // 0 MH, 1 HMC
    int n_leap = 0;           // HMC: leapfrog steps per iteration
    double eps = 0.0;         // HMC: leapfrog step
    double* mom = nullptr;    // HMC: K momenta
    double* h0 = nullptr;     // HMC: f - |p|^2 / 2 at the start of the iteration
    uint64_t seed = 0, chain_id = 0;   // HMC: generator key
    unsigned iter0 = 0;       // HMC: index of the first iteration (its random streams)
};

// Kernel parameters (passed by value).  nb coefficient vectors are
// evaluated per launch (nb <= the instance's NB; slot b's vectors at stride K,
// its result at stride 1 + K).
struct FgParams {
    const unsigned char* X;   // row-major storage, element (n,k) at X + (n*ldx + k)*es
    int64_t ldx;              // leading dimension in elements
    const uint8_t* y;         // N response bytes
    int64_t N;
    int K;
    const float* scale;       // FP8 column scales, else unused
    const double* beta;       // nb x K doubles
    const double* mean;       // nb x K doubles or nullptr (zero mean)
    double prec;              // prior precision when precs is nullptr
    const double* precs;      // nb precisions or nullptr
    int nb;                   // coefficient vectors in this launch
    double* out;              // nb x (1 + K) doubles
    double* partials;         // nblocks x NB x (1 + K)
    double* gpart;            // ngroups x NB x (1 + K)
    unsigned* counters;       // ngroups + 1 tickets, zero between launches
    int nblocks;
    int group;                // blocks per merge group
    int interleave;           // 1: wave w takes batches w, w+W, ...; 0: one contiguous range
    int family;               // response family (0 logistic, 1 Poisson)
    double* w_out;            // N Hessian row weights, or nullptr (NB == 1 only)
    const ChainParams* chain; // device copy: on-device Metropolis step, or nullptr (NB == 1)
};

// ------------------------------------------------------------ decoding

// All elements of a 16-byte chunk as float (FP32, BF16, FP8 code values).
template <int DT>
__device__ __forceinline__ void decode_chunk(const u32x4& w, float (&v)[16 / ElemSize<DT>::v]);

template <>
__device__ __forceinline__ void decode_chunk<DT_F32>(const u32x4& w, float (&v)[4]) {
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = __uint_as_float(w[e]);
}

template <>
__device__ __forceinline__ void decode_chunk<DT_BF16>(const u32x4& w, float (&v)[8]) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        v[2 * i] = __uint_as_float(w[i] << 16);
        v[2 * i + 1] = __uint_as_float(w[i] & 0xFFFF0000u);
    }
}

template <>
__device__ __forceinline__ void decode_chunk<DT_FP8>(const u32x4& w, float (&v)[16]) {
    // gfx950 converts OCP E4M3FN bytes natively, two per instruction.
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const f32x2 lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)w[i], false);
        const f32x2 hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)w[i], true);
        v[4 * i] = lo.x;
        v[4 * i + 1] = lo.y;
        v[4 * i + 2] = hi.x;
        v[4 * i + 3] = hi.y;
    }
}

__device__ __forceinline__ double chunk_elem_f64(const u32x4& w, int e) {
    const unsigned long long b =
        ((unsigned long long)w[2 * e + 1] << 32) | (unsigned long long)w[2 * e];
    return __longlong_as_double((long long)b);
}

// ------------------------------------------------------------ lane exchange
//
// One step of a transposed butterfly reduction at lane distance D (a power
// of two below 64).  Each lane holds two partial sums A (row slot i) and B
// (row slot i + H).  Lanes whose bit D is clear end with A(self) + A(partner),
// lanes whose bit D is set with B(self) + B(partner), where the partner
// differs in bit D (and possibly in lower bits, which no earlier step has
// used).  D = 32 and 16 use gfx950's permlane swaps, which exchange both
// halves in one instruction; D = 8, 4, 2, 1 use DPP row_mirror,
// row_half_mirror and quad permutations.

__device__ __forceinline__ unsigned dpp_mov(unsigned v, int ctrl) {
    switch (ctrl) {
    case 0x140: return (unsigned)__builtin_amdgcn_mov_dpp((int)v, 0x140, 0xF, 0xF, true);
    case 0x141: return (unsigned)__builtin_amdgcn_mov_dpp((int)v, 0x141, 0xF, 0xF, true);
    case 0x4E: return (unsigned)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, true);
    default: return (unsigned)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, true);
    }
}

template <int D>
constexpr int dpp_ctrl() {
    return D == 8 ? 0x140 : D == 4 ? 0x141 : D == 2 ? 0x4E : 0xB1;
}

// 32-bit words: returns the partner's copy of the half this lane keeps,
// plus this lane's kept word (both as raw bits).
template <int D>
__device__ __forceinline__ void xchg_u32(unsigned a, unsigned b, bool up, unsigned& keep,
                                         unsigned& got) {
    if constexpr (D == 32 || D == 16) {
        const u32x2 r = D == 32 ? __builtin_amdgcn_permlane32_swap(a, b, false, false)
                                : __builtin_amdgcn_permlane16_swap(a, b, false, false);
        keep = r.x;   // lanes with bit clear: own A; set: partner's B
        got = r.y;    // lanes with bit clear: partner's A; set: own B
    } else {
        const unsigned send = up ? a : b;
        keep = up ? b : a;
        got = dpp_mov(send, dpp_ctrl<D>());
    }
}

template <int D>
__device__ __forceinline__ float xstep(float a, float b, bool up) {
    unsigned k, g;
    xchg_u32<D>(__float_as_uint(a), __float_as_uint(b), up, k, g);
    return __uint_as_float(k) + __uint_as_float(g);
}

template <int D>
__device__ __forceinline__ double xstep(double a, double b, bool up) {
    const unsigned long long ua = (unsigned long long)__double_as_longlong(a);
    const unsigned long long ub = (unsigned long long)__double_as_longlong(b);
    unsigned k0, g0, k1, g1;
    xchg_u32<D>((unsigned)ua, (unsigned)ub, up, k0, g0);
    xchg_u32<D>((unsigned)(ua >> 32), (unsigned)(ub >> 32), up, k1, g1);
    const double k = __longlong_as_double((long long)(((unsigned long long)k1 << 32) | k0));
    const double g = __longlong_as_double((long long)(((unsigned long long)g1 << 32) | g0));
    return k + g;
}

// Transposed reduction over the LPR lanes of a segment (LPR a power of two,
// segments aligned).  On entry v[j] is this lane's partial of row slot j
// (j < R).  Afterwards, if R >= LPR, v[i] (i < R/LPR) holds the complete sum
// of slot cl*(R/LPR) + i; otherwise v[0] holds the sum of slot cl/(LPR/R),
// replicated on LPR/R lanes.  cl is the lane index within its segment.
template <int D, int CNT, int R, typename V>
__device__ __forceinline__ void seg_reduce(V (&v)[R], int lane) {
    if constexpr (D >= 1) {
        const bool up = (lane & D) != 0;
        if constexpr (CNT > 1) {
            constexpr int H = CNT / 2;
#pragma unroll
            for (int i = 0; i < H; ++i) v[i] = xstep<D>(v[i], v[i + H], up);
            seg_reduce<D / 2, H, R, V>(v, lane);
        } else {
            v[0] = xstep<D>(v[0], v[0], up);
            seg_reduce<D / 2, 1, R, V>(v, lane);
        }
    }
}

// Sum over the lanes that share this lane's position within its segment of
// D lanes (exact xor partners; runs once per launch).
template <int D>
__device__ __forceinline__ double cross_segment_sum(double v) {
    if constexpr (D < 64) {
        v += __shfl_xor(v, D, 64);
        return cross_segment_sum<D * 2>(v);
    } else {
        return v;
    }
}

// ------------------------------------------------------------ TR map

// Per-row terms in FP64 for the response family fam (wave-uniform):
//   logistic (0): t = y u - softplus(u), r = y - sigmoid(u), overflow-free;
//   Poisson  (1): t = y u - exp(u),      r = y - exp(u)  (y a count 0..255).
__device__ __forceinline__ void tr_map(double u, unsigned yb, int fam, double& t, double& r) {
    if (fam == 1) {
        const double yv = (double)(yb & 0xFFu);
        const double mu = exp_f64(u);
        t = yv * u - mu;
        r = yv - mu;
        return;
    }
    const double yv = (double)(yb & 1u);
    const double e = exp_f64(-fabs(u));
    const double sp = fmax(u, 0.0) + log1p_unit(e);
    const double inv = recip_1_8(1.0 + e);
    const double sig = u >= 0.0 ? inv : e * inv;
    t = yv * u - sp;
    r = yv - sig;
}

// Row weight of the Hessian (minus the second derivative of t in u):
// sigmoid(u) (1 - sigmoid(u)) = e / (1 + e)^2 with e = exp(-|u|) for the
// logistic model, exp(u) for the Poisson one.
__device__ __forceinline__ double tr_weight(double u, int fam) {
    if (fam == 1) return exp_f64(u);
    const double e = exp_f64(-fabs(u));
    const double inv = recip_1_8(1.0 + e);
    return e * inv * inv;
}

// ------------------------------------------------------------ finalisation

// sum_{t < n} a[t * stride] of published data in index order, with 16 loads
// in flight: the loads of a block are independent, the additions keep the
// fixed order (padding adds +0.0, which leaves any sum but -0.0 unchanged).
__device__ __forceinline__ double ordered_sum(const double* a, int n, int64_t stride) {
    double s = 0.0;
    for (int t = 0; t < n; t += 16) {
        double v[16];
#pragma unroll
        for (int j = 0; j < 16; ++j)
            v[j] = t + j < n ? fetch_published(a + (int64_t)(t + j) * stride) : 0.0;
#pragma unroll
        for (int j = 0; j < 16; ++j) s += v[j];
    }
    return s;
}

// Buffer descriptor word 3 for raw (untyped) buffers on gfx9-class GPUs.
constexpr int kRsrcWord3 = 0x00020000;

// The same sums (of published data) for the Q entries idx0 + q * step (q < Q) that are below lim
// (the others give 0), with the loads of all Q issued before any addition:
// one memory latency for Q entries instead of Q.  The loads go through a
// buffer descriptor spanning the n x stride doubles, so the surplus ones
// (past n, or an entry at or past lim, sent out of range) return zeros
// without a branch; each sum is added in the order of ordered_sum (padding
// included), so the results are bitwise equal.
template <int Q>
__device__ __forceinline__ void ordered_sums(const double* a, int n, int64_t stride, int idx0,
                                             int step, int lim, double (&out)[Q]) {
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        (void*)a, 0, (int)((int64_t)n * stride * 8), kRsrcWord3);
    auto load = [&](int idx, int t) {
        const uint32_t off = idx < lim ? (uint32_t)(idx + (int64_t)t * stride) * 8u : 0x80000000u;
        const u32x2 w = __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, kLoadPublished);
        return __longlong_as_double((long long)(((unsigned long long)w[1] << 32) | w[0]));
    };
    if (n == 1) {   // a single partial (one block, or one group)
#pragma unroll
        for (int q = 0; q < Q; ++q) out[q] = 0.0 + load(idx0 + q * step, 0);
        return;
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) out[q] = 0.0;
    for (int t = 0; t < n; t += 16) {
        double v[Q][16];
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
            for (int j = 0; j < 16; ++j) v[q][j] = load(idx0 + q * step, t + j);
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
            for (int j = 0; j < 16; ++j) out[q] += v[q][j];
    }
}

// The sums over n published partials (stride doubles apart) of the E entries
// idx < E, for all NT threads of a block; emit(idx, sum) is called once per
// entry by one thread (entry idx < NT by thread idx).  Loads of partials that
// other blocks wrote cost per cache line a wave touches more than per load,
// so the forms below keep each wave's lines few:
//   - more than 16 partials but a small total (n x stride <= kStageDoubles):
//     every double of the n partials is copied into LDS with contiguous
//     loads spread over the whole block, then thread (c, e) adds entry e
//     over its contiguous chunk c of the partials and the chunk sums are
//     added in chunk order (for 16 or fewer, one round of loads by the
//     threads of the entries is quicker);
//   - otherwise, when the entries leave threads idle and n needs more than
//     one round of loads, the same chunks are loaded directly;
//   - otherwise one entry per thread, or four per thread and round when
//     E > NT.
// The order of every sum is fixed by (n, stride, E, NT), so repeated calls
// agree bitwise.
constexpr int kStageDoubles = 2048;

template <int NT, typename Emit>
__device__ __forceinline__ void block_sums(const double* a, int n, int64_t stride, int E,
                                           double* s_stage, double* s_part, Emit&& emit) {
    if (n > 16 && E <= NT && (int64_t)n * stride <= kStageDoubles) {
        const int tot = n * (int)stride;
        const __amdgpu_buffer_rsrc_t rs =
            __builtin_amdgcn_make_buffer_rsrc((void*)a, 0, tot * 8, kRsrcWord3);
        constexpr int L = kStageDoubles / NT;
        double v[L];
#pragma unroll
        for (int j = 0; j < L; ++j) {
            const u32x2 w = __builtin_amdgcn_raw_buffer_load_b64(
                rs, (uint32_t)(threadIdx.x + j * NT) * 8u, 0, kLoadPublished);
            v[j] = __longlong_as_double((long long)(((unsigned long long)w[1] << 32) | w[0]));
        }
#pragma unroll
        for (int j = 0; j < L; ++j)
            if ((int)threadIdx.x + j * NT < tot) s_stage[threadIdx.x + j * NT] = v[j];
        __syncthreads();
        const int C = min(NT / E, n);
        const int t = threadIdx.x, c = t / E, e = t - c * E;
        if (c < C) {
            double sum = 0.0;
            for (int b = c * n / C; b < (c + 1) * n / C; ++b) sum += s_stage[b * (int)stride + e];
            s_part[t] = sum;
        }
        __syncthreads();
        if (t < E) {
            double sum = 0.0;
            for (int cc = 0; cc < C; ++cc) sum += s_part[cc * E + t];
            emit(t, sum);
        }
        return;
    }
    const int C = min(NT / max(E, 1), (n + 15) / 16);
    if (C >= 2) {
        const int t = threadIdx.x, c = t / E, e = t - c * E;
        if (c < C) {
            const int t0 = c * n / C, t1 = (c + 1) * n / C;
            double v[1];
            ordered_sums<1>(a + (int64_t)t0 * stride, t1 - t0, stride, e, 0, E, v);
            s_part[t] = v[0];
        }
        __syncthreads();
        if (t < E) {
            double sum = 0.0;
            for (int cc = 0; cc < C; ++cc) sum += s_part[cc * E + t];
            emit(t, sum);
        }
    } else if (E <= NT) {
        double v[1];
        ordered_sums<1>(a, n, stride, threadIdx.x, NT, E, v);
        if ((int)threadIdx.x < E) emit((int)threadIdx.x, v[0]);
    } else {
        for (int i0 = threadIdx.x; i0 < E; i0 += 4 * NT) {
            double v[4];
            ordered_sums<4>(a, n, stride, i0, NT, E, v);
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (i0 + q * NT < E) emit(i0 + q * NT, v[q]);
        }
    }
}

// Sum of one value per thread over a block of NT threads, returned to every
// thread: wave butterflies, then the wave totals in wave order.
template <int NT>
__device__ __forceinline__ double block_sum(double v) {
    __shared__ double s_w[NT / 64];
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) t += s_w[w];
    return t;
}

// Starts HMC iteration t from the chain state (beta, fg): momenta p ~ N(0, I)
// from the stream of iteration t, h0 = f - |p|^2 / 2, the first half
// momentum step and the first position step into beta_prop, leapfrog
// position 1.  Run by all NT threads of one block.
template <int NT>
__device__ __forceinline__ void hmc_begin(const ChainParams& c, unsigned t, int K) {
    double kin = 0.0;
    const double he = 0.5 * c.eps;
    for (int q = threadIdx.x; 2 * q < K; q += NT) {
        double z[2];
        polar_pair(c.seed, c.chain_id, RNG_HMC_MOMENTUM, t, (uint64_t)q, z[0], z[1]);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int k = 2 * q + h;
            if (k < K) {
                kin = fma(z[h], z[h], kin);
                const double m = z[h] + he * c.fg[1 + k];
                c.mom[k] = m;
                c.beta_prop[k] = c.beta[k] + c.eps * m;
            }
        }
    }
    kin = block_sum<NT>(kin);
    if (threadIdx.x == 0) {
        c.h0[0] = c.fg[0] - 0.5 * kin;
        c.step[0] = t;
        c.step[1] = 1;
    }
}

// One HMC evaluation's step, after f and g at beta_prop (fg_prop) are
// written: inside the trajectory a full momentum step and the next position;
// at its end the closing half momentum step, the accept test
// log U_t < (f' - |p'|^2 / 2) - h0, the state update and the start of the next
// iteration.  Run by all threads of the last block.
template <int NT>
__device__ __forceinline__ void hmc_step(const ChainParams& c, const double* fg_prop, int K) {
    __shared__ unsigned s_tl[2];
    __shared__ int s_acc;
    if (threadIdx.x == 0) {
        s_tl[0] = c.step[0];
        s_tl[1] = c.step[1];
    }
    __syncthreads();
    const unsigned t = s_tl[0], l = s_tl[1];
    if ((int)l < c.n_leap) {
        for (int k = threadIdx.x; k < K; k += NT) {
            const double m = c.mom[k] + c.eps * fg_prop[1 + k];
            c.mom[k] = m;
            c.beta_prop[k] = c.beta_prop[k] + c.eps * m;
        }
        if (threadIdx.x == 0) c.step[1] = l + 1;
        return;
    }
    double kin = 0.0;
    const double he = 0.5 * c.eps;
    for (int k = threadIdx.x; k < K; k += NT) {
        const double m = c.mom[k] + he * fg_prop[1 + k];
        kin = fma(m, m, kin);
    }
    kin = block_sum<NT>(kin);
    if (threadIdx.x == 0) {
        const double dH = (fg_prop[0] - 0.5 * kin) - c.h0[0];
        const Block4 b = philox4x64_10(0, 0, RNG_HMC_ACCEPT, t, c.seed, c.chain_id);
        s_acc = log_f64(u01(b.w[0])) < dH ? 1 : 0;
    }
    __syncthreads();
    const int acc = s_acc;
    if (acc) {
        for (int k = threadIdx.x; k <= K; k += NT) c.fg[k] = fg_prop[k];
        for (int k = threadIdx.x; k < K; k += NT) c.beta[k] = c.beta_prop[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (c.accepted) c.accepted[t - c.iter0] = (uint8_t)acc;
        if (c.f_trace) c.f_trace[t - c.iter0] = c.fg[0];
    }
    if (t + 1 - c.iter0 < (unsigned)c.n_steps) {
        hmc_begin<NT>(c, t + 1, K);
    } else if (threadIdx.x == 0) {
        c.step[0] = t + 1;
    }
}

// Accept iff log U_t < f(beta_prop) - f(beta); on acceptance the state takes
// the proposal's beta, f and g; then beta_prop = beta + incs[t + 1] and t + 1.
// Run by all threads of the last block after fg_prop (1 + K) is written.
template <int NT>
__device__ __forceinline__ void chain_step(const ChainParams& c, const double* fg_prop, int K) {
    if (c.kind == 1) {
        hmc_step<NT>(c, fg_prop, K);
        return;
    }
    __shared__ int s_acc;
    __shared__ unsigned s_t;
    if (threadIdx.x == 0) {
        const unsigned t = *c.step;
        s_t = t;
        s_acc = c.logu[t] < fg_prop[0] - c.fg[0] ? 1 : 0;
    }
    __syncthreads();
    const int acc = s_acc;
    const unsigned t = s_t;
    for (int k = threadIdx.x; k <= K; k += NT) {
        if (acc) c.fg[k] = fg_prop[k];
        if (k < K) {
            const double b = acc ? c.beta_prop[k] : c.beta[k];
            if (acc) c.beta[k] = b;
            if ((int)t + 1 < c.n_steps) c.beta_prop[k] = b + c.incs[(int64_t)(t + 1) * K + k];
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (c.accepted) c.accepted[t] = (uint8_t)acc;
        if (c.f_trace) c.f_trace[t] = acc ? fg_prop[0] : c.fg[0];
        *c.step = t + 1;
    }
}

// Called by every thread of every block after the block has published its
// partial (NB x (1 + K) doubles at partials + blk * NB * (1 + K), blk being
// the block's index among the p.nblocks blocks of this evaluation).  NT is
// the block size (a power of two).  One group of blocks: the block completing
// the count adds the block partials directly; several: the last block of each
// group adds its group's partials, and the last group's finisher adds the
// group sums.
template <int NT, int NB>
__device__ __forceinline__ void merge_partials(const FgParams& p, int blk) {
    __shared__ unsigned s_last;
    __shared__ double s_stage[kStageDoubles];   // block_sums' staging and chunk sums
    __shared__ double s_part[NT];
    const int K1 = p.K + 1;
    const int W = NB * K1;           // doubles per partial
    const int grp = blk / p.group;
    const int b0 = grp * p.group;
    const int b1 = min(p.nblocks, b0 + p.group);
    const int ngroups = (p.nblocks + p.group - 1) / p.group;

    // Every thread's partial stores complete before the barrier, and the
    // barrier before thread 0's ticket.
    publish_wait();
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned prev = __hip_atomic_fetch_add(&p.counters[grp], 1u, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT);
        s_last = (prev == (unsigned)(b1 - b0 - 1)) ? 1u : 0u;
    }
    __syncthreads();
    if (!s_last) return;

    const double* fin = p.partials;   // what the final sums add: block or group partials
    int nfin = p.nblocks;
    if (ngroups > 1) {
        double* gp = p.gpart + (int64_t)grp * W;
        block_sums<NT>(p.partials + (int64_t)b0 * W, b1 - b0, W, W, s_stage, s_part,
                       [&](int i, double v) { publish(gp + i, v); });
        if (threadIdx.x == 0)
            __hip_atomic_store(&p.counters[grp], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // second level: the last group to finish adds the group sums
        publish_wait();
        __syncthreads();
        if (threadIdx.x == 0) {
            const unsigned prev = __hip_atomic_fetch_add(&p.counters[ngroups], 1u, __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT);
            s_last = (prev == (unsigned)(ngroups - 1)) ? 1u : 0u;
        }
        __syncthreads();
        if (!s_last) return;
        fin = p.gpart;
        nfin = ngroups;
    }

    // Final sums in block or group order, plus each slot's Gaussian prior
    // N(m, prec^-1 I).  The nb x (1 + K) entries are spread over the block
    // (block_sums); each slot's squared distance to its prior mean is summed
    // per thread, then per wave (butterfly), then over the waves in order.
    __shared__ double s_flik[NB];
    __shared__ double s_pw[NT / 64][NB];
    const int nbk = p.nb * K1;
    double pf[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) pf[b] = 0.0;
    // beta_k - m_k of entry idx; entry threadIdx.x (the one this thread
    // finishes unless nb (1 + K) > NT) is loaded before the sums' loads
    auto prior_diff = [&](int idx) {
        const int b = idx / K1, k = idx - b * K1;
        const int64_t bk = (int64_t)b * p.K + k - 1;
        return k == 0 ? 0.0 : p.beta[bk] - (p.mean ? p.mean[bk] : 0.0);
    };
    const double d_own = (int)threadIdx.x < nbk ? prior_diff(threadIdx.x) : 0.0;
    auto final_entry = [&](int idx, double sum) {
        const int b = idx / K1, k = idx - b * K1;
        if (k == 0) {
            s_flik[b] = sum;   // likelihood part; prior added below
            return;
        }
        const double prec = p.precs ? p.precs[b] : p.prec;
        const double d = idx == (int)threadIdx.x ? d_own : prior_diff(idx);
        p.out[(int64_t)b * K1 + k] = sum - prec * d;
#pragma unroll
        for (int bb = 0; bb < NB; ++bb)
            if (bb == b) pf[bb] += d * d;
    };
    block_sums<NT>(fin, nfin, W, nbk, s_stage, s_part, final_entry);
    {
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            double v = pf[b];
#pragma unroll
            for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
            if (lane == 0) s_pw[wave][b] = v;
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < p.nb) {
        const int b = threadIdx.x;
        double sq = 0.0;
#pragma unroll
        for (int w = 0; w < NT / 64; ++w) sq += s_pw[w][b];
        const double prec = p.precs ? p.precs[b] : p.prec;
        p.out[(int64_t)b * K1] = s_flik[b] - 0.5 * prec * sq;
    }
    __syncthreads();
    if (p.chain) chain_step<NT>(*p.chain, p.out, p.K);
    if (threadIdx.x == 0)
        __hip_atomic_store(&p.counters[ngroups > 1 ? ngroups : 0], 0u, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

// ------------------------------------------------------------ wave tiles

// Cache policy of the streaming loads: nontemporal.
constexpr int kLoadNT = 2;

// The per-wave machinery shared by the plain, batched and several-beta
// kernels: one wave streams batches of BATCH = R * RPW consecutive rows, each
// lane holding R row slots of CPL 16-byte chunks, and accumulates f and its
// columns of the gradient for NB coefficient vectors at once (the X tile is
// read from HBM once for all of them).
template <int DT, int LPR, int CPL, int R, int NB = 1>
struct WaveTile {
    static constexpr int ES = ElemSize<DT>::v;
    static constexpr int LANES = LPR;             // lanes per row
    static constexpr int CHUNKS = CPL;            // chunks per lane per row
    static constexpr int VE = 16 / ES;            // elements per 16-byte chunk
    static constexpr int RPW = 64 / LPR;          // rows per wave-wide load
    static constexpr int BATCH = R * RPW;         // rows per batch
    static constexpr int KT = LPR * CPL * VE;     // columns an instance covers
    static constexpr bool F64 = DT == DT_F64;
    static constexpr int OWN = R >= LPR ? R / LPR : 1;   // rows owned per lane after reduction
    static constexpr int REP = R >= LPR ? 1 : LPR / R;   // lanes sharing one owned row
    static constexpr int RBUF = NB * RPW * R;     // LDS values per wave for r
    // With several coefficient vectors and rows shared by REP lanes, the REP
    // lanes of a row split its NB per-row maps between them (lane cl % REP
    // takes slots cl % REP, cl % REP + REP, ...) instead of each repeating
    // all of them; NTR is the number of maps a lane then evaluates.
    static constexpr bool SPLIT_TR = REP > 1 && NB > 1;
    static constexpr int NTR = SPLIT_TR ? (NB + REP - 1) / REP : 1;
    // The gradient products r_n x_nk in FP64 (r kept in FP64): FP64 storage,
    // and FP32 storage with one coefficient vector (the plain and hierarchical
    // kernels), where the vector ALU has room for the conversion.  Otherwise
    // (BF16, FP8, several vectors) r is rounded to FP32 and the products are
    // summed in FP32 over the R rows of a batch, then added in FP64.
    static constexpr bool G64 = F64 || (DT == DT_F32 && NB == 1);
    using rtype = typename std::conditional<G64, double, float>::type;
    // Keeping the values decoded for the dot products for the gradient
    // (instead of decoding a second time) was measured slower for FP8 and
    // BF16 rows of 512 columns at every batch height tried: the register
    // pressure costs more than the decode, so it stays off.
    static constexpr bool KEEP = false;
    // Several vectors over a small tile (at most 32 values per lane): the
    // tile is converted to FP64 once for all vectors (2 registers per value)
    // instead of once per vector; over 2 GB of FP32 rows of 32 and 128
    // columns this took passes of 8 vectors from 1243 to 1102 us and from 891
    // to 790.
    static constexpr bool CONV1 = !F64 && NB > 1 && R * CPL * VE <= 32;

    struct Tile {
        u32x4 x[R][CPL];
        unsigned yb[OWN];
    };

    int lane, seg, cl, NC, KC;
    int fam;                 // response family (wave-uniform)
    double* wout = nullptr;  // per-row Hessian weights of slot 0, or nullptr
    bool ragged;             // K * ES is not a whole number of chunks (wave-uniform)
    u32x4 xmask[CPL];        // bytes of chunk i that are columns < K (ragged K only)
    uint32_t ldb;            // row stride in bytes
    uint32_t loff[CPL];      // byte offset of this lane's chunk i in row slot 0
    uint32_t yoff[OWN];      // row slot (within a batch) of each owned row
    bool unique;             // this lane accounts its owned rows in f
    double bd[NB][CPL][VE];                   // beta (FP8: times the column scale)
    double g64[NB][CPL][VE];                  // this lane's gradient columns
    double facc[NB];
    double fk[NTR];                           // f of slot cl % REP + k * REP (SPLIT_TR)

    __device__ __forceinline__ void init(int lane_, int K, int64_t ldx, int family) {
        lane = lane_;
        fam = family;
        seg = lane / LPR;
        cl = lane % LPR;
        // A row of K columns spans NC chunks; when K * ES is not a multiple
        // of 16 the last one is partial and the bytes past column K (row
        // padding up to ldx, whatever it holds) are cleared before use.
        NC = (K + VE - 1) / VE;
        KC = K;
        ragged = (K % VE) != 0;
        ldb = (uint32_t)(ldx * ES);
#pragma unroll
        for (int i = 0; i < CPL; ++i) {
            const int c = cl + i * LPR;
            loff[i] = c < NC ? (uint32_t)seg * ldb + (uint32_t)c * 16u : 0x80000000u;
            const int vb = min(16, max(0, K * ES - c * 16));   // valid bytes of chunk i
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int nbq = min(4, max(0, vb - 4 * q));
                xmask[i][q] = nbq >= 4 ? 0xFFFFFFFFu : ((1u << (8 * nbq)) - 1u);
            }
        }
#pragma unroll
        for (int o = 0; o < OWN; ++o) {
            const int j = R >= LPR ? cl * OWN + o : cl / REP;
            yoff[o] = (uint32_t)(j * RPW + seg);
        }
        unique = R >= LPR || (cl % REP) == 0;
    }

    // Column k of this lane's chunk i, element e.
    __device__ __forceinline__ int col(int i, int e) const { return (cl + i * LPR) * VE + e; }
    __device__ __forceinline__ bool col_ok(int i) const { return cl + i * LPR < NC; }
    __device__ __forceinline__ bool elem_ok(int i, int e) const { return col(i, e) < KC; }

    // Coefficient vector of slot b (K doubles); FP8 folds the column scales in.
    // Buffer loads: columns past KC read as zeros without a branch, so every
    // load is issued before the first wait (a branch per element made the
    // FP8 form wait for each beta and scale in turn).
    __device__ __forceinline__ void set_beta(int b, const double* beta, const float* scale) {
        const __amdgpu_buffer_rsrc_t rb =
            __builtin_amdgcn_make_buffer_rsrc((void*)beta, 0, KC * 8, kRsrcWord3);
#pragma unroll
        for (int i = 0; i < CPL; ++i) {
#pragma unroll
            for (int e = 0; e < VE; ++e) {
                const u32x2 w = __builtin_amdgcn_raw_buffer_load_b64(rb, (uint32_t)col(i, e) * 8u, 0, 0);
                double v = __longlong_as_double((long long)(((unsigned long long)w[1] << 32) | w[0]));
                if constexpr (DT == DT_FP8) {
                    const __amdgpu_buffer_rsrc_t rs =
                        __builtin_amdgcn_make_buffer_rsrc((void*)scale, 0, KC * 4, kRsrcWord3);
                    v *= (double)__builtin_bit_cast(
                        float, __builtin_amdgcn_raw_buffer_load_b32(rs, (uint32_t)col(i, e) * 4u, 0, 0));
                }
                bd[b][i][e] = v;
            }
        }
    }

    __device__ __forceinline__ void zero_acc() {
#pragma unroll
        for (int b = 0; b < NB; ++b) {
#pragma unroll
            for (int i = 0; i < CPL; ++i)
#pragma unroll
                for (int e = 0; e < VE; ++e) g64[b][i][e] = 0.0;
            facc[b] = 0.0;
        }
#pragma unroll
        for (int k = 0; k < NTR; ++k) fk[k] = 0.0;
    }

    // Loads the batch of rows row0 .. row0 + BATCH - 1 of a row block whose
    // valid rows end at row0 + navail (navail <= 0: nothing valid).  Rows past
    // the end come back as zeros from the buffer range check without touching
    // memory, so the call never needs a branch.
    __device__ __forceinline__ void load(Tile& t, const unsigned char* X, const uint8_t* y,
                                         int64_t row0, int64_t navail) const {
        int64_t nvalid = min((int64_t)BATCH, navail);
        if (nvalid <= 0) {
            nvalid = 0;
            row0 = 0;
        }
        const __amdgpu_buffer_rsrc_t rx = __builtin_amdgcn_make_buffer_rsrc(
            (void*)(X + row0 * (int64_t)ldb), 0, (int)(nvalid * ldb), kRsrcWord3);
#pragma unroll
        for (int j = 0; j < R; ++j)
#pragma unroll
            for (int i = 0; i < CPL; ++i)
                t.x[j][i] = __builtin_amdgcn_raw_buffer_load_b128(
                    rx, loff[i] + (uint32_t)(j * RPW) * ldb, 0, kLoadNT);
        const __amdgpu_buffer_rsrc_t ry = __builtin_amdgcn_make_buffer_rsrc(
            (void*)(y + row0), 0, (int)nvalid, kRsrcWord3);
#pragma unroll
        for (int o = 0; o < OWN; ++o)
            t.yb[o] = __builtin_amdgcn_raw_buffer_load_b8(ry, yoff[o], 0, kLoadNT);
        // keep the math of the other tile from being scheduled ahead of
        // these loads (it would delay the prefetch by a whole compute phase)
        __builtin_amdgcn_sched_barrier(0);
    }

    // Adds the batch's rows (the first nvalid row slots are real) into f and
    // g of the first nact slots (nact is wave-uniform; the other slots are
    // skipped, so a partly filled pass costs what it carries).  rbuf: this
    // wave's LDS slice of RBUF values.
    __device__ __forceinline__ void compute(Tile& t, uint32_t nvalid, rtype* rbuf,
                                            int nact = NB, int64_t row0 = 0) {
        if (ragged) {
#pragma unroll
            for (int j = 0; j < R; ++j)
#pragma unroll
                for (int i = 0; i < CPL; ++i) t.x[j][i] &= xmask[i];
        }
        float xk[KEEP ? R : 1][CPL][KEEP ? VE : 1];   // decoded tile (KEEP)
        double xd[CONV1 ? R : 1][CPL][CONV1 ? VE : 1];  // tile in FP64 (CONV1)
        if constexpr (CONV1) {
#pragma unroll
            for (int j = 0; j < R; ++j)
#pragma unroll
                for (int i = 0; i < CPL; ++i) {
                    float xv[VE];
                    decode_chunk<DT>(t.x[j][i], xv);
#pragma unroll
                    for (int e = 0; e < VE; ++e) xd[j][i][e] = (double)xv[e];
                }
        }
        double ub[NB];   // the owned row's u per slot (SPLIT_TR)
#pragma unroll
        for (int b = 0; b < NB; ++b) ub[b] = 0.0;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            if (b >= nact) break;
            // partial dot products and the transposed reduction
            double uo[OWN];
            if constexpr (F64) {
                double v[R];
#pragma unroll
                for (int j = 0; j < R; ++j) {
                    double sacc = 0.0;
#pragma unroll
                    for (int i = 0; i < CPL; ++i)
#pragma unroll
                        for (int e = 0; e < VE; ++e)
                            sacc = fma(chunk_elem_f64(t.x[j][i], e), bd[b][i][e], sacc);
                    v[j] = sacc;
                }
                seg_reduce<LPR / 2, R, R, double>(v, lane);
#pragma unroll
                for (int o = 0; o < OWN; ++o) uo[o] = v[o];
            } else {
                double v[R];
#pragma unroll
                for (int j = 0; j < R; ++j) {
                    double sacc = 0.0;
#pragma unroll
                    for (int i = 0; i < CPL; ++i) {
                        if constexpr (CONV1) {
#pragma unroll
                            for (int e = 0; e < VE; ++e) sacc = fma(xd[j][i][e], bd[b][i][e], sacc);
                            continue;
                        }
                        // with several vectors, convert again per vector rather
                        // than keep the converted tile alive (2 registers per
                        // value): the empty asm hides that the tile is
                        // unchanged, in place (on a copy, the copy cost two
                        // moves per chunk and vector)
                        if constexpr (NB > 1) asm volatile("" : "+v"(t.x[j][i]));
                        const u32x4 raw = t.x[j][i];
                        float xv[VE];
                        decode_chunk<DT>(raw, xv);
#pragma unroll
                        for (int e = 0; e < VE; ++e) {
                            if constexpr (KEEP) xk[j][i][e] = xv[e];
                            sacc = fma((double)xv[e], bd[b][i][e], sacc);
                        }
                    }
                    v[j] = sacc;
                }
                seg_reduce<LPR / 2, R, R, double>(v, lane);
#pragma unroll
                for (int o = 0; o < OWN; ++o) uo[o] = v[o];
            }
            if constexpr (SPLIT_TR) {
                ub[b] = uo[0];
                continue;
            }
            // TR map on owned rows (FP64); r to the segment through LDS
#pragma unroll
            for (int o = 0; o < OWN; ++o) {
                double tt, rr;
                tr_map(uo[o], t.yb[o], fam, tt, rr);
                const bool ok = yoff[o] < nvalid;
                if (ok && unique) facc[b] += tt;
                if (b == 0 && wout != nullptr && ok && unique)
                    wout[row0 + yoff[o]] = tr_weight(uo[o], fam);
                if (unique) {
                    const int j = R >= LPR ? cl * OWN + o : cl / REP;
                    rbuf[(b * RPW + seg) * R + j] = ok ? (rtype)rr : (rtype)0;
                }
            }
        }
        if constexpr (SPLIT_TR) {
            // one owned row (OWN == 1), its maps split over the REP lanes
            const int sub = cl % REP;
            const int j = cl / REP;
            const bool ok = yoff[0] < nvalid;
#pragma unroll
            for (int k = 0; k < NTR; ++k) {
                const int b = sub + k * REP;
                if (b < nact) {
                    double u = ub[0];
#pragma unroll
                    for (int bb = 1; bb < NB; ++bb) u = b == bb ? ub[bb] : u;
                    double tt, rr;
                    tr_map(u, t.yb[0], fam, tt, rr);
                    if (ok) fk[k] += tt;
                    rbuf[(b * RPW + seg) * R + j] = ok ? (rtype)rr : (rtype)0;
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            if (b >= nact) break;
            rtype rs[R];
#pragma unroll
            for (int j = 0; j < R; ++j) rs[j] = rbuf[(b * RPW + seg) * R + j];
            // gradient contribution from the same registers
            if constexpr (F64) {
#pragma unroll
                for (int j = 0; j < R; ++j)
#pragma unroll
                    for (int i = 0; i < CPL; ++i)
#pragma unroll
                        for (int e = 0; e < VE; ++e)
                            g64[b][i][e] = fma(rs[j], chunk_elem_f64(t.x[j][i], e), g64[b][i][e]);
            } else if constexpr (G64) {
#pragma unroll
                for (int j = 0; j < R; ++j)
#pragma unroll
                    for (int i = 0; i < CPL; ++i) {
                        float xv[VE];
                        decode_chunk<DT>(t.x[j][i], xv);
#pragma unroll
                        for (int e = 0; e < VE; ++e)
                            g64[b][i][e] = fma(rs[j], (double)xv[e], g64[b][i][e]);
                    }
            } else {
                float g32[CPL][VE];
#pragma unroll
                for (int i = 0; i < CPL; ++i)
#pragma unroll
                    for (int e = 0; e < VE; ++e) g32[i][e] = 0.0f;
#pragma unroll
                for (int j = 0; j < R; ++j)
#pragma unroll
                    for (int i = 0; i < CPL; ++i) {
                        float xv[VE];
                        if constexpr (KEEP) {
#pragma unroll
                            for (int e = 0; e < VE; ++e) xv[e] = xk[j][i][e];
                        } else {
                            u32x4 raw = t.x[j][i];
                            // Decode again rather than keep the decoded tile of
                            // the dot-product phase alive (VE floats per 4 raw
                            // registers): the empty asm hides that raw is
                            // unchanged.
                            if constexpr (VE > 4) asm volatile("" : "+v"(raw));
                            decode_chunk<DT>(raw, xv);
                        }
#pragma unroll
                        for (int e = 0; e < VE; ++e) g32[i][e] = fmaf(rs[j], xv[e], g32[i][e]);
                    }
#pragma unroll
                for (int i = 0; i < CPL; ++i)
#pragma unroll
                    for (int e = 0; e < VE; ++e) g64[b][i][e] += (double)g32[i][e];
            }
        }
        __builtin_amdgcn_wave_barrier();
    }

    // Streams rows [r0, r1) of X / y (absolute row indices; X and y are the
    // bases of the whole matrix), batch by batch with one batch prefetched.
    __device__ __forceinline__ void stream_rows(const unsigned char* X, const uint8_t* y,
                                                int64_t r0, int64_t r1, rtype* rbuf,
                                                int nact = NB) {
        Tile ta, tb;
        load(ta, X, y, r0, r1 - r0);
        for (int64_t b = r0; b < r1; b += 2 * BATCH) {
            load(tb, X, y, b + BATCH, r1 - b - BATCH);
            compute(ta, (uint32_t)min((int64_t)BATCH, r1 - b), rbuf, nact, b);
            if (b + BATCH >= r1) break;
            load(ta, X, y, b + 2 * BATCH, r1 - b - 2 * BATCH);
            compute(tb, (uint32_t)min((int64_t)BATCH, r1 - b - BATCH), rbuf, nact, b + BATCH);
        }
    }

    // Column sums over the segments of the wave (every lane of segment 0
    // ends with its columns' totals) and the wave totals of f (every lane).
    __device__ __forceinline__ void wave_totals() {
        if constexpr (SPLIT_TR) {
            const int sub = cl % REP;
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                double v = 0.0;
#pragma unroll
                for (int k = 0; k < NTR; ++k) v = sub + k * REP == b ? fk[k] : v;
                facc[b] = v;
            }
        }
#pragma unroll
        for (int b = 0; b < NB; ++b) {
#pragma unroll
            for (int i = 0; i < CPL; ++i)
#pragma unroll
                for (int e = 0; e < VE; ++e) g64[b][i][e] = cross_segment_sum<LPR>(g64[b][i][e]);
#pragma unroll
            for (int d = 32; d >= 1; d >>= 1) facc[b] += __shfl_xor(facc[b], d, 64);
        }
    }
};

// ------------------------------------------------------------ block merge

// The waves of a block add their column totals into one LDS vector in wave
// order, the block writes its partial of NB x (1 + K) doubles and joins the
// cross-block merge.  WT is the wave tile type: every lane of segment 0 holds
// the totals of its columns col(i, e) in g64, every lane the wave's f per slot.
template <class WT, int DT, int WPB, int NB>
__device__ __forceinline__ void block_merge(const FgParams& p, const int blk, const WT& wt,
                                            const int wave) {
    constexpr int KT = WT::KT;
    constexpr int VE = WT::VE;
    constexpr int CPL = WT::CHUNKS;
    const int K1 = p.K + 1;
    // Each wave's column totals go to a slice of their own and are added in
    // wave order after one barrier; when the slices do not fit in 32 KB of
    // LDS the waves add into one vector in turn, a barrier each (the same
    // additions in the same order, so the same bits).
    constexpr bool SLICES = WPB * NB * KT * 8 <= 32768;
    __shared__ double gsh[SLICES ? WPB : 1][NB][KT];
    __shared__ double fsh[WPB][NB];
    if (wt.lane == 0)
#pragma unroll
        for (int b = 0; b < NB; ++b) fsh[wave][b] = wt.facc[b];
    if constexpr (SLICES) {
        if (wt.seg == 0) {
#pragma unroll
            for (int b = 0; b < NB; ++b)
#pragma unroll
                for (int i = 0; i < CPL; ++i)
#pragma unroll
                    for (int e = 0; e < VE; ++e) gsh[wave][b][wt.col(i, e)] = wt.g64[b][i][e];
        }
        __syncthreads();
    } else {
        for (int w = 0; w < WPB; ++w) {
            if (wave == w && wt.seg == 0) {
#pragma unroll
                for (int b = 0; b < NB; ++b)
#pragma unroll
                    for (int i = 0; i < CPL; ++i)
#pragma unroll
                        for (int e = 0; e < VE; ++e) {
                            const int k = wt.col(i, e);
                            gsh[0][b][k] = (w == 0 ? 0.0 : gsh[0][b][k]) + wt.g64[b][i][e];
                        }
            }
            __syncthreads();
        }
    }
    double* part = p.partials + (int64_t)blk * NB * K1;
    for (int b = 0; b < NB; ++b) {
        for (int k = threadIdx.x; k < p.K; k += blockDim.x) {
            double sacc;
            if constexpr (SLICES) {
                sacc = 0.0;
#pragma unroll
                for (int w = 0; w < WPB; ++w) sacc += gsh[w][b][k];
            } else {
                sacc = gsh[0][b][k];
            }
            if constexpr (DT == DT_FP8) sacc *= (double)p.scale[k];
            publish(&part[b * K1 + 1 + k], sacc);
        }
        if (threadIdx.x == 0) {
            double sacc = 0.0;
#pragma unroll
            for (int w = 0; w < WPB; ++w) sacc += fsh[w][b];
            publish(&part[b * K1], sacc);
        }
    }
    merge_partials<WPB * 64, NB>(p, blk);
}

// ------------------------------------------------------------ plain kernel

// Block blk (of p.nblocks) of the evaluation of f and g of p.nb (<= NB)
// coefficient vectors over all rows of one data set.  NBUF tiles rotate in
// the grid-strided sweep: the load of a batch is issued NBUF - 1 batches
// before it is computed.
template <int DT, int LPR, int CPL, int R, int WPB, int NB, int NBUF = 2>
__device__ __forceinline__ void fg_pass(const FgParams& p, const int blk) {
    using WT = WaveTile<DT, LPR, CPL, R, NB>;
    constexpr int BATCH = WT::BATCH;
    constexpr int VE = WT::VE;

    WT wt;
    // wave-uniform: keeps the batch bookkeeping and buffer bases in SGPRs
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    wt.init(threadIdx.x & 63, p.K, p.ldx, p.family);
    if constexpr (NB == 1) wt.wout = p.w_out;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        if (b < p.nb) {
            wt.set_beta(b, p.beta + (int64_t)b * p.K, p.scale);
        } else {
#pragma unroll
            for (int i = 0; i < CPL; ++i)
#pragma unroll
                for (int e = 0; e < VE; ++e) wt.bd[b][i][e] = 0.0;
        }
    }
    wt.zero_acc();
    const int nact = __builtin_amdgcn_readfirstlane(min(p.nb, NB));

    __shared__ typename WT::rtype rbuf[WPB][WT::RBUF];

    // This wave's batches: first, first + step, ... below last.  Either
    // grid-strided (all waves sweep memory together) or one contiguous,
    // balanced range per wave.
    const int64_t nbatch = (p.N + BATCH - 1) / BATCH;
    const int64_t tw = (int64_t)p.nblocks * WPB;
    const int64_t gw = (int64_t)blk * WPB + wave;
    if (p.interleave) {
        static_assert(NBUF >= 2, "at least double buffering");
        typename WT::Tile tl[NBUF];
        const int64_t step = tw * BATCH;
        const int64_t rend = nbatch * BATCH;
        int64_t r = gw * BATCH;
#pragma unroll
        for (int j = 0; j + 1 < NBUF; ++j) wt.load(tl[j], p.X, p.y, r + j * step, p.N - r - j * step);
        for (;; r += NBUF * step) {
#pragma unroll
            for (int j = 0; j < NBUF; ++j) {
                const int64_t rj = r + j * step;
                if (rj >= rend) goto swept;
                const int64_t rn = rj + (NBUF - 1) * step;   // loaded into the tile just freed
                wt.load(tl[(j + NBUF - 1) % NBUF], p.X, p.y, rn, p.N - rn);
                wt.compute(tl[j], (uint32_t)max((int64_t)0, min((int64_t)BATCH, p.N - rj)), rbuf[wave],
                           nact, rj);
            }
        }
    swept:;
    } else {
        const int64_t r0 = min(p.N, nbatch * gw / tw * BATCH);
        const int64_t r1 = min(p.N, nbatch * (gw + 1) / tw * BATCH);
        wt.stream_rows(p.X, p.y, r0, r1, rbuf[wave], nact);
    }
    wt.wave_totals();
    block_merge<WT, DT, WPB, NB>(p, blk, wt, wave);
}

// f and g of p.nb (<= NB) coefficient vectors over all rows of one data set
// (the grid is p.nblocks blocks).
template <int DT, int LPR, int CPL, int R, int WPB, int NB = 1, int NBUF = 2>
__global__ __launch_bounds__(WPB * 64) void fg_fused(FgParams p) {
    fg_pass<DT, LPR, CPL, R, WPB, NB, NBUF>(p, blockIdx.x);
}

// ------------------------------------------------------------ fleet kernel

// One evaluation of a fleet launch: the parameters of a several-beta pass
// over one data set and the first of its consecutive blocks in the grid.
struct FleetJob {
    FgParams p;
    int blk0;
    int pad_;
};

// Several data sets of one kernel geometry in one launch: block b works on
// job blk_job[b] as block b - blk0 of that job's own grid, so every job runs
// exactly the blocks, row ranges and merge order of a launch of its own and
// its results are bitwise those of fg_fused over the same parameters.
template <int DT, int LPR, int CPL, int R, int WPB, int NB, int NBUF = 2>
__global__ __launch_bounds__(WPB * 64) void fg_fleet(const FleetJob* jobs, const uint16_t* blk_job) {
    const int j = blk_job[blockIdx.x];
    const FgParams p = jobs[j].p;
    fg_pass<DT, LPR, CPL, R, WPB, NB, NBUF>(p, (int)blockIdx.x - jobs[j].blk0);
}

}  // namespace glmk
