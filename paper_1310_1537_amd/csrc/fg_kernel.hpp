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
//   2. per-lane partial dot products with beta split as beta_hi + beta_lo
//      (two FP32 numbers) so that no rounding of the FP64 beta leaks into u;
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
// group to finish adds the group sums in group order and the prior.  No
// floating-point atomics are used, so the result is bitwise reproducible.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

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

// Kernel parameters (passed by value).
struct FgParams {
    const unsigned char* X;   // row-major storage, element (n,k) at X + (n*ldx + k)*es
    int64_t ldx;              // leading dimension in elements
    const uint8_t* y;         // N response bytes
    int64_t N;
    int K;
    const float* scale;       // FP8 column scales, else unused
    const double* beta;       // K doubles
    const double* mean;       // K doubles or nullptr
    double prec;
    double* out;              // 1 + K doubles
    double* partials;         // nblocks x (1 + K)
    double* gpart;            // ngroups x (1 + K)
    unsigned* counters;       // ngroups + 1 tickets, zero between launches
    int nblocks;
    int group;                // blocks per merge group
    int64_t rows_per_block;   // contiguous row range of each block
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

// ------------------------------------------------------------ shuffles

struct HiLo {
    float h, l;
};

__device__ __forceinline__ float shfl_x(float v, int m) { return __shfl_xor(v, m, 64); }
__device__ __forceinline__ double shfl_x(double v, int m) { return __shfl_xor(v, m, 64); }
__device__ __forceinline__ HiLo shfl_x(HiLo v, int m) {
    return HiLo{__shfl_xor(v.h, m, 64), __shfl_xor(v.l, m, 64)};
}
__device__ __forceinline__ HiLo operator+(HiLo a, HiLo b) { return HiLo{a.h + b.h, a.l + b.l}; }

// Transposed butterfly reduction over the LPR lanes of a segment.  On entry
// v[j] is this lane's partial of row slot j (j < CNT == R).  After the steps
// with distance D = LPR/2 .. 1: if R >= LPR the lane holds the complete sums
// of slots cl*(R/LPR) + i in v[i] (i < R/LPR); otherwise v[0] holds the sum
// of slot cl / (LPR/R), replicated on LPR/R lanes.
template <int D, int CNT, int R, typename V>
__device__ __forceinline__ void seg_reduce(V (&v)[R], int lane) {
    if constexpr (D >= 1) {
        if constexpr (CNT > 1) {
            constexpr int H = CNT / 2;
            const bool up = (lane & D) != 0;
#pragma unroll
            for (int i = 0; i < H; ++i) {
                const V send = up ? v[i] : v[i + H];
                const V keep = up ? v[i + H] : v[i];
                v[i] = keep + shfl_x(send, D);
            }
            seg_reduce<D / 2, H, R, V>(v, lane);
        } else {
            v[0] = v[0] + shfl_x(v[0], D);
            seg_reduce<D / 2, 1, R, V>(v, lane);
        }
    }
}

// ------------------------------------------------------------ TR map

// t = y u - softplus(u), r = y - sigmoid(u), overflow-free, in FP64.
__device__ __forceinline__ void tr_map(double u, double yv, double& t, double& r) {
    const double e = exp(-fabs(u));
    const double sp = fmax(u, 0.0) + log1p(e);
    const double inv = 1.0 / (1.0 + e);
    const double sig = u >= 0.0 ? inv : e * inv;
    t = yv * u - sp;
    r = yv - sig;
}

// ------------------------------------------------------------ finalisation

// Called by every thread of every block after the block has written its
// partial (1 + K doubles at partials + blockIdx.x * (1 + K)).
// NT is the block size (a power of two).
template <int NT>
__device__ __forceinline__ void merge_partials(const FgParams& p) {
    __shared__ unsigned s_last;
    __shared__ double s_red[NT];
    const int K1 = p.K + 1;
    const int grp = blockIdx.x / p.group;
    const int b0 = grp * p.group;
    const int b1 = min(p.nblocks, b0 + p.group);
    const int ngroups = (p.nblocks + p.group - 1) / p.group;

    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned prev = __hip_atomic_fetch_add(&p.counters[grp], 1u, __ATOMIC_ACQ_REL,
                                                     __HIP_MEMORY_SCOPE_AGENT);
        s_last = (prev == (unsigned)(b1 - b0 - 1)) ? 1u : 0u;
    }
    __syncthreads();
    if (!s_last) return;
    __threadfence();

    for (int k = threadIdx.x; k < K1; k += blockDim.x) {
        double s = 0.0;
#pragma unroll 8
        for (int b = b0; b < b1; ++b) s += p.partials[(int64_t)b * K1 + k];
        p.gpart[(int64_t)grp * K1 + k] = s;
    }
    if (threadIdx.x == 0)
        __hip_atomic_store(&p.counters[grp], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);

    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned prev = __hip_atomic_fetch_add(&p.counters[ngroups], 1u, __ATOMIC_ACQ_REL,
                                                     __HIP_MEMORY_SCOPE_AGENT);
        s_last = (prev == (unsigned)(ngroups - 1)) ? 1u : 0u;
    }
    __syncthreads();
    if (!s_last) return;
    __threadfence();

    // Final sums in group order, plus the Gaussian prior N(mean, prec^-1 I).
    double pf = 0.0;
    for (int k = threadIdx.x; k < K1; k += blockDim.x) {
        double s = 0.0;
#pragma unroll 8
        for (int g = 0; g < ngroups; ++g) s += p.gpart[(int64_t)g * K1 + k];
        if (k == 0) {
            p.out[0] = s;   // likelihood part; prior added below
        } else {
            const double d = p.beta[k - 1] - (p.mean ? p.mean[k - 1] : 0.0);
            pf += d * d;
            p.out[k] = s - p.prec * d;
        }
    }
    s_red[threadIdx.x] = pf;
    __syncthreads();
    for (int w = NT / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s_red[threadIdx.x] += s_red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        p.out[0] = p.out[0] - 0.5 * p.prec * s_red[0];
        __hip_atomic_store(&p.counters[ngroups], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// ------------------------------------------------------------ main kernel

template <int DT, int LPR, int CPL, int R, int WPB>
__global__ __launch_bounds__(WPB * 64) void fg_fused(FgParams p) {
    constexpr int ES = ElemSize<DT>::v;
    constexpr int VE = 16 / ES;            // elements per 16-byte chunk
    constexpr int RPW = 64 / LPR;          // rows per wave-wide load
    constexpr int BATCH = R * RPW;         // rows per wave per batch
    constexpr int KT = LPR * CPL * VE;     // columns this instance can cover
    constexpr bool F64 = DT == DT_F64;
    constexpr int OWN = R >= LPR ? R / LPR : 1;   // rows owned per lane after the reduction
    constexpr int REP = R >= LPR ? 1 : LPR / R;   // lanes sharing one owned row

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int seg = lane / LPR;
    const int cl = lane % LPR;
    const int NC = p.K / VE;

    // ---- this lane's slice of beta (scale folded in for FP8) ----
    float bh[CPL][VE], bl[CPL][VE];
    double bd[CPL][VE];
#pragma unroll
    for (int i = 0; i < CPL; ++i) {
        const int c = cl + i * LPR;
#pragma unroll
        for (int e = 0; e < VE; ++e) {
            double b = 0.0;
            if (c < NC) {
                const int k = c * VE + e;
                b = p.beta[k];
                if constexpr (DT == DT_FP8) b *= (double)p.scale[k];
            }
            if constexpr (F64) {
                bd[i][e] = b;
            } else {
                bh[i][e] = (float)b;
                bl[i][e] = (float)(b - (double)bh[i][e]);
            }
        }
    }

    double g64[CPL][VE];
#pragma unroll
    for (int i = 0; i < CPL; ++i)
#pragma unroll
        for (int e = 0; e < VE; ++e) g64[i][e] = 0.0;
    double facc = 0.0;

    using rtype = typename std::conditional<F64, double, float>::type;
    __shared__ rtype rbuf[WPB][RPW][R];

    const int64_t r0 = (int64_t)blockIdx.x * p.rows_per_block;
    const int64_t r1 = min(p.N, r0 + p.rows_per_block);
    const int64_t ldb = p.ldx * ES;   // row stride in bytes

    for (int64_t base = r0 + (int64_t)wave * BATCH; base < r1; base += (int64_t)WPB * BATCH) {
        // ---- 1. loads ----
        u32x4 x[R][CPL];
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const int64_t row = base + j * RPW + seg;
            const bool rv = row < r1;
#pragma unroll
            for (int i = 0; i < CPL; ++i) {
                const int c = cl + i * LPR;
                if (rv && c < NC) {
                    x[j][i] = __builtin_nontemporal_load(
                        reinterpret_cast<const u32x4*>(p.X + row * ldb + (int64_t)c * 16));
                } else {
                    x[j][i] = u32x4{0u, 0u, 0u, 0u};
                }
            }
        }
        // y bytes of the rows this lane will own after the reduction
        double yo[OWN];
        int64_t rowo[OWN];
#pragma unroll
        for (int i = 0; i < OWN; ++i) {
            const int j = R >= LPR ? cl * OWN + i : cl / REP;
            rowo[i] = base + j * RPW + seg;
            yo[i] = rowo[i] < r1 ? (double)p.y[rowo[i]] : 0.0;
        }

        // ---- 2+3. partial dots and transposed segment reduction ----
        double uo[OWN];
        if constexpr (F64) {
            double v[R];
#pragma unroll
            for (int j = 0; j < R; ++j) {
                double s = 0.0;
#pragma unroll
                for (int i = 0; i < CPL; ++i)
#pragma unroll
                    for (int e = 0; e < VE; ++e) s = fma(chunk_elem_f64(x[j][i], e), bd[i][e], s);
                v[j] = s;
            }
            seg_reduce<LPR / 2, R, R, double>(v, lane);
#pragma unroll
            for (int i = 0; i < OWN; ++i) uo[i] = v[i];
        } else {
            HiLo v[R];
#pragma unroll
            for (int j = 0; j < R; ++j) {
                float sh = 0.0f, sl = 0.0f;
#pragma unroll
                for (int i = 0; i < CPL; ++i) {
                    float xv[VE];
                    decode_chunk<DT>(x[j][i], xv);
#pragma unroll
                    for (int e = 0; e < VE; ++e) {
                        sh = fmaf(xv[e], bh[i][e], sh);
                        sl = fmaf(xv[e], bl[i][e], sl);
                    }
                }
                v[j] = HiLo{sh, sl};
            }
            seg_reduce<LPR / 2, R, R, HiLo>(v, lane);
#pragma unroll
            for (int i = 0; i < OWN; ++i) uo[i] = (double)v[i].h + (double)v[i].l;
        }

        // ---- TR map on owned rows; r broadcast through LDS ----
        const bool unique = R >= LPR || (cl % REP) == 0;
#pragma unroll
        for (int i = 0; i < OWN; ++i) {
            double t, r;
            tr_map(uo[i], yo[i], t, r);
            const bool ok = rowo[i] < r1;
            if (ok && unique) facc += t;
            if (unique) {
                const int j = R >= LPR ? cl * OWN + i : cl / REP;
                rbuf[wave][seg][j] = ok ? (rtype)r : (rtype)0;
            }
        }
        __builtin_amdgcn_wave_barrier();
        rtype rr[R];
#pragma unroll
        for (int j = 0; j < R; ++j) rr[j] = rbuf[wave][seg][j];
        __builtin_amdgcn_wave_barrier();

        // ---- 4. gradient contribution from the same registers ----
        if constexpr (F64) {
#pragma unroll
            for (int j = 0; j < R; ++j) {
                const double rj = rr[j];
#pragma unroll
                for (int i = 0; i < CPL; ++i)
#pragma unroll
                    for (int e = 0; e < VE; ++e) g64[i][e] = fma(rj, chunk_elem_f64(x[j][i], e), g64[i][e]);
            }
        } else {
            float g32[CPL][VE];
#pragma unroll
            for (int i = 0; i < CPL; ++i)
#pragma unroll
                for (int e = 0; e < VE; ++e) g32[i][e] = 0.0f;
#pragma unroll
            for (int j = 0; j < R; ++j) {
#pragma unroll
                for (int i = 0; i < CPL; ++i) {
                    float xv[VE];
                    decode_chunk<DT>(x[j][i], xv);
#pragma unroll
                    for (int e = 0; e < VE; ++e) g32[i][e] = fmaf(rr[j], xv[e], g32[i][e]);
                }
            }
#pragma unroll
            for (int i = 0; i < CPL; ++i)
#pragma unroll
                for (int e = 0; e < VE; ++e) g64[i][e] += (double)g32[i][e];
        }
    }

    // ---- block merge: segments of a wave, then waves in LDS ----
#pragma unroll
    for (int d = LPR; d < 64; d <<= 1)
#pragma unroll
        for (int i = 0; i < CPL; ++i)
#pragma unroll
            for (int e = 0; e < VE; ++e) g64[i][e] += shfl_x(g64[i][e], d);
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) facc += shfl_x(facc, d);

    // Waves add their slices into one LDS vector in wave order.
    __shared__ double gsh[KT];
    __shared__ double fsh[WPB];
    if (lane == 0) fsh[wave] = facc;
    for (int w = 0; w < WPB; ++w) {
        if (wave == w && seg == 0) {
#pragma unroll
            for (int i = 0; i < CPL; ++i)
#pragma unroll
                for (int e = 0; e < VE; ++e) {
                    const int k = (cl + i * LPR) * VE + e;
                    gsh[k] = (w == 0 ? 0.0 : gsh[k]) + g64[i][e];
                }
        }
        __syncthreads();
    }
    double* part = p.partials + (int64_t)blockIdx.x * (p.K + 1);
    for (int k = threadIdx.x; k < p.K; k += blockDim.x) {
        double s = gsh[k];
        if constexpr (DT == DT_FP8) s *= (double)p.scale[k];
        part[1 + k] = s;
    }
    if (threadIdx.x == 0) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < WPB; ++w) s += fsh[w];
        part[0] = s;
    }
    merge_partials<WPB * 64>(p);
}

}  // namespace glmk
