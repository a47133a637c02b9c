// Log-posterior Hessian fused with f and g:
//
//     H = -X^t W X - prec I,   W = diag(w_n),
//     w_n = sigmoid(u_n) (1 - sigmoid(u_n))  (logistic),  exp(u_n)  (Poisson).
//
// The paper names the Hessian as the next quantity to add to the fused
// routine (Sec. 5.2; Hessian-based samplers and optimisers are listed in
// Sec. 4.2).  X^t W X is a dense contraction over the rows, so it runs on the
// matrix cores: FP64 MFMA (v_mfma_f64_16x16x4), products and sums in FP64.
//
// Three launches in stream order:
//   1. the fused f+g kernel, which also writes each row's w_n (N doubles);
//   2. k_hess: the K x K output is cut into 128 x 128 tiles, of which the
//      upper triangle (tile row <= tile column) is computed; each tile's rows
//      are cut into chunks (more for off-diagonal tiles, whose work per row
//      is larger); block (tile, chunk) stages 32 rows of the tile's column
//      ranges (and w) into LDS and its four waves accumulate 16 x 16 MFMA
//      blocks, four rows per instruction: on an off-diagonal tile a 64 x 64
//      quadrant (4 x 4 blocks) each, on a diagonal tile 9 of the 36 blocks on
//      or above the diagonal each; the block writes its partial tile (FP32
//      rows take k_hess_lds, the same work with the rows loaded straight
//      into LDS);
//   3. k_hess_merge: one thread per tile entry adds the tile's partials in
//      chunk order and writes the entry and its mirror image, minus prec on
//      the diagonal.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <type_traits>
#include <vector>

#include "elem.hpp"
#include "runtime.hpp"

namespace glmrt {
namespace {

constexpr int kTile = 128;    // output tile edge
constexpr int kHT = 256;      // threads per block (4 waves)
constexpr int kRsrcWord3 = 0x00020000;   // buffer descriptor word 3, raw (untyped) buffers

typedef double dv4 __attribute__((ext_vector_type(4)));
typedef unsigned uv4 __attribute__((ext_vector_type(4)));

struct HessParams {
    const void* X;
    int64_t ldx;
    const float* scale;       // FP8 column scales
    const double* w;          // N row weights
    int64_t N;
    int K;
    const int4* tiles;        // per upper-triangle tile: tile row, tile column, first block, chunks
    const int2* blocks;       // per block: tile, chunk
    double* partials;         // blocks x kTile x kTile
};

// Element e of a 16-byte chunk of stored elements, as a double.
template <int DT>
__device__ __forceinline__ double chunk_elem(const uv4& w, int e, float s) {
    if constexpr (DT == GLM_F64) {
        return __longlong_as_double((long long)(((unsigned long long)w[2 * e + 1] << 32) | w[2 * e]));
    } else if constexpr (DT == GLM_F32) {
        return (double)__uint_as_float(w[e]);
    } else if constexpr (DT == GLM_BF16) {
        return (double)__uint_as_float(((w[e >> 1] >> (16 * (e & 1))) & 0xFFFFu) << 16);
    } else {
        const unsigned byte = (w[e >> 2] >> (8 * (e & 3))) & 0xFFu;
        return glmk::Elem<GLM_FP8_E4M3>::value((unsigned char)byte, s);
    }
}

// Block (tile, chunk): sum over the chunk's rows of w_n x_n,i x_n,j for the
// tile's 128 x 128 entries; each wave owns a 64 x 64 quadrant (4 x 4 MFMA
// blocks of 16 x 16).  Rows are staged R = 32 at a time with 16-byte loads; the next R rows are loaded into registers while the
// matrix cores work on the current ones.  Thread t stages the fixed 16-byte
// column chunk t mod CW of rows t / CW + q * 256 / CW (CW chunks per staged
// row).  A chunk starting at or past column K is not read; the part of a
// chunk past K (row padding up to ldx) is zeroed.
template <int DT>
__global__ __launch_bounds__(kHT) void k_hess(HessParams p) {
    constexpr int ES = DT == GLM_F64 ? 8 : DT == GLM_F32 ? 4 : DT == GLM_BF16 ? 2 : 1;
    constexpr int VE = 16 / ES;                 // elements per chunk
    constexpr int R = 32;                       // rows per step
    constexpr int CR = kTile / VE;              // chunks per column range
    constexpr int NPMAX = R * 2 * CR / kHT;     // chunks per thread (off-diagonal tile)
    const unsigned char* X = static_cast<const unsigned char*>(p.X);
    const int2 bt = p.blocks[blockIdx.x];
    const int4 tc = p.tiles[bt.x];
    const int chunk = bt.y, nch = tc.w;
    const int i0 = tc.x * kTile, j0 = tc.y * kTile;
    const bool diag = tc.x == tc.y;
    const int64_t r0 = p.N * chunk / nch;
    const int64_t r1 = p.N * (chunk + 1) / nch;

    // xs[r][c]: c < kTile the i-range, c >= kTile the j-range (off-diagonal
    // tiles).  The row stride is 16 doubles past a multiple of 32 (64 banks of
    // 4 bytes), so the two rows that one half-wave reads in the matrix loop
    // (lanes 0-15 and 16-31, rows kk and kk + 1) fall in disjoint banks.
    // FP32 and BF16 rows are staged as FP32 (exact; half the LDS, and each
    // thread's 16-byte chunk goes in with one conflict-free 16-byte store),
    // FP64 and scaled FP8 as FP64; the matrix loop converts on the read.
    constexpr int XS = 2 * kTile + 16;
    using LT = typename std::conditional<DT == GLM_F32 || DT == GLM_BF16, float, double>::type;
    __shared__ LT xs[R][XS];
    __shared__ double ws[R];

    const int cw = diag ? CR : 2 * CR;                 // staged chunks per row
    const int nper = R * cw / kHT;                     // chunks per thread
    const int cc = threadIdx.x % cw;                   // this thread's chunk column
    const int srow = threadIdx.x / cw;                 // first staged row
    const int rstep = kHT / cw;
    const int col0 = cc < CR ? i0 + cc * VE : j0 + (cc - CR) * VE;   // first column of the chunk
    const bool chunk_ok = col0 < p.K;
    const int lcol = cc * VE;                          // LDS column of the chunk
    float cs[VE];
#pragma unroll
    for (int e = 0; e < VE; ++e)
        cs[e] = (DT == GLM_FP8_E4M3 && col0 + e < p.K) ? p.scale[col0 + e] : 1.0f;

    // loads from clamped (always valid) addresses, masked afterwards, so that
    // they are all in flight at once
    uv4 raw[NPMAX];
    double wl = 0.0;
    auto fetch = [&](int64_t r) __attribute__((always_inline)) {
#pragma unroll
        for (int q = 0; q < NPMAX; ++q) {
            const int64_t row = min(r + srow + q * rstep, r1 - 1);
            const uv4* src = reinterpret_cast<const uv4*>(X + (row * p.ldx + (chunk_ok ? col0 : 0)) * ES);
            raw[q] = (q < nper) ? *src : uv4{0u, 0u, 0u, 0u};
        }
        wl = p.w[min(r + (int64_t)(threadIdx.x % R), r1 - 1)];
    };

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);

    // Stages rows r .. r + R - 1 of the chunk into xs / ws (every thread).
    auto stage = [&](int64_t r) __attribute__((always_inline)) {
        __syncthreads();   // the previous step's MFMA reads of xs are done
#pragma unroll
        for (int q = 0; q < NPMAX; ++q) {
            if (q >= nper) break;
            const int rr = srow + q * rstep;
            const bool row_ok = r + rr < r1 && chunk_ok;
            if constexpr (std::is_same<LT, float>::value) {
                float v[VE];
#pragma unroll
                for (int e = 0; e < VE; ++e) {
                    const unsigned bits = DT == GLM_F32 ? raw[q][e]
                                                       : ((raw[q][e >> 1] >> (16 * (e & 1))) & 0xFFFFu) << 16;
                    v[e] = (row_ok && col0 + e < p.K) ? __uint_as_float(bits) : 0.0f;
                }
#pragma unroll
                for (int e = 0; e < VE; ++e) xs[rr][lcol + e] = v[e];
            } else {
#pragma unroll
                for (int e = 0; e < VE; ++e)
                    xs[rr][lcol + e] = (row_ok && col0 + e < p.K) ? chunk_elem<DT>(raw[q], e, cs[e]) : 0.0;
            }
        }
        if (threadIdx.x < R) ws[threadIdx.x] = r + threadIdx.x < r1 ? wl : 0.0;
        __syncthreads();
        if (r + R < r1) fetch(r + R);
    };

    // partial tile of this block: D[row][col] of a 16 x 16 block sits in lane
    // col + 16 (row % 4), item row / 4
    double* part = p.partials + (int64_t)blockIdx.x * kTile * kTile;
    auto store_block = [&](int bi, int bj, const dv4& d) __attribute__((always_inline)) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
            part[(16 * bi + (lane >> 4) + 4 * q) * kTile + 16 * bj + (lane & 15)] = d[q];
    };

    if (diag) {
        // The 36 blocks (I, J), I <= J, of the 8 x 8 grid: wave W takes row W
        // (J = W .. 7, 8 - W blocks) and row 7 - W (J = 7 - W .. 7, W + 1
        // blocks), 9 in all, so the four waves (and their SIMDs) carry equal
        // matrix work.  The loop is compiled once per wave index, so that the
        // compiler knows which blocks share an operand: the row 7 - W blocks'
        // columns are a subset of the row W blocks' (W <= 3), and a wave reads
        // 2 A and 8 - W B operands per four rows for its 9 matrix
        // instructions (with the wave index known only at run time it read
        // and converted one B per instruction and chose A per instruction).
        auto run = [&](auto wc) __attribute__((always_inline)) {
            constexpr int W = decltype(wc)::value;
            constexpr int NA = 8 - W;            // row W blocks
            dv4 acc[9];
#pragma unroll
            for (int s2 = 0; s2 < 9; ++s2) acc[s2] = dv4{0.0, 0.0, 0.0, 0.0};
            if (r0 < r1) fetch(r0);
            for (int64_t r = r0; r < r1; r += R) {
                stage(r);
#pragma unroll
                for (int k0 = 0; k0 < R; k0 += 4) {
                    const int kk = k0 + (lane >> 4);
                    const double wk = ws[kk];
                    const double a1 = wk * (double)xs[kk][16 * W + (lane & 15)];
                    const double a2 = wk * (double)xs[kk][16 * (7 - W) + (lane & 15)];
                    double bv[NA];   // B of block column W + s
#pragma unroll
                    for (int s = 0; s < NA; ++s) bv[s] = (double)xs[kk][16 * (W + s) + (lane & 15)];
#pragma unroll
                    for (int s = 0; s < NA; ++s)
                        acc[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, bv[s], acc[s], 0, 0, 0);
#pragma unroll
                    for (int t = 0; t <= W; ++t)
                        acc[NA + t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a2, bv[7 - 2 * W + t],
                                                                          acc[NA + t], 0, 0, 0);
                }
            }
#pragma unroll
            for (int s = 0; s < NA; ++s) store_block(W, W + s, acc[s]);
#pragma unroll
            for (int t = 0; t <= W; ++t) store_block(7 - W, 7 - W + t, acc[NA + t]);
        };
        switch (wave) {
        case 0: run(std::integral_constant<int, 0>()); break;
        case 1: run(std::integral_constant<int, 1>()); break;
        case 2: run(std::integral_constant<int, 2>()); break;
        default: run(std::integral_constant<int, 3>()); break;
        }
    } else {
        const int qi = (wave >> 1) * 64, qj = (wave & 1) * 64;   // this wave's quadrant
        dv4 acc[4][4];
#pragma unroll
        for (int ta = 0; ta < 4; ++ta)
#pragma unroll
            for (int tb = 0; tb < 4; ++tb) acc[ta][tb] = dv4{0.0, 0.0, 0.0, 0.0};
        if (r0 < r1) fetch(r0);
        for (int64_t r = r0; r < r1; r += R) {
            stage(r);
#pragma unroll
            for (int k0 = 0; k0 < R; k0 += 4) {
                // A[i][k] = w_k x_k,(i0+i), B[k][j] = x_k,(j0+j); lane: i or j = lane % 16, k = lane / 16
                const int kk = k0 + (lane >> 4);
                const double wk = ws[kk];
                double a[4], b[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    a[t] = wk * (double)xs[kk][qi + 16 * t + (lane & 15)];
                    b[t] = (double)xs[kk][kTile + qj + 16 * t + (lane & 15)];
                }
#pragma unroll
                for (int ta = 0; ta < 4; ++ta)
#pragma unroll
                    for (int tb = 0; tb < 4; ++tb)
                        acc[ta][tb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ta], b[tb], acc[ta][tb], 0, 0, 0);
            }
        }
#pragma unroll
        for (int ta = 0; ta < 4; ++ta)
#pragma unroll
            for (int tb = 0; tb < 4; ++tb) store_block(qi / 16 + ta, qj / 16 + tb, acc[ta][tb]);
    }
}

// The same work for FP32 rows, with the rows loaded straight into LDS
// (buffer_load ... lds, 16 bytes per lane; lane l's bytes land at the LDS
// address + 16 l) into two buffers: the loads of the next R rows are issued
// at the start of a step and waited for at its end, so a step costs the
// matrix loop, a handful of load instructions and one barrier, and no
// thread converts or stores anything.  One load instruction per row and
// wave: lanes 0-31 bring the tile's row range (128 floats), lanes 32-63 its
// column range; on a diagonal tile lanes 32-63 are out of range and write
// zeros into the unused half.  Each step's buffer resource covers only its
// valid rows, so rows past the chunk's end come in as zeros.  Columns past K
// are not zeroed: they feed only entries (i, j) with i >= K or j >= K, which
// the merge drops.  The partials are bitwise those of k_hess<GLM_F32> (the
// same operands in the same order).
__global__ __launch_bounds__(kHT) void k_hess_lds(HessParams p) {
    constexpr int R = 32;                        // rows per step
    constexpr int XS = 2 * kTile + 16;           // row stride (floats), as in k_hess
    __shared__ float xs[2][R][XS];
    __shared__ double ws[2][R];
    const int2 bt = p.blocks[blockIdx.x];
    const int4 tc = p.tiles[bt.x];
    const int chunk = bt.y, nch = tc.w;
    const int i0 = tc.x * kTile, j0 = tc.y * kTile;
    const bool diag = tc.x == tc.y;
    const int64_t r0 = p.N * chunk / nch;
    const int64_t r1 = p.N * (chunk + 1) / nch;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const unsigned char* X = static_cast<const unsigned char*>(p.X);
    const uint32_t ldb = (uint32_t)(p.ldx * 4);   // row pitch in bytes
    const uint32_t voff = lane < 32 ? (uint32_t)(i0 + 4 * lane) * 4u
                                    : (diag ? 0x7FFFFFF0u : (uint32_t)(j0 + 4 * (lane - 32)) * 4u);
    // rows r .. r + R - 1 (those before r1) into buffer b: wave w loads rows
    // 8w .. 8w + 7, wave 0 also the R weights (4 bytes per lane)
    auto issue = [&](int64_t r, int b) __attribute__((always_inline)) {
        const int64_t nv = min((int64_t)R, r1 - r);
        const __amdgpu_buffer_rsrc_t rx = __builtin_amdgcn_make_buffer_rsrc(
            (void*)(X + r * (int64_t)ldb), 0, (int)(nv * ldb), kRsrcWord3);
#pragma unroll
        for (int q = 0; q < R / 4; ++q) {
            const int rr = wave * (R / 4) + q;
            __builtin_amdgcn_raw_ptr_buffer_load_lds(
                rx, (__attribute__((address_space(3))) void*)&xs[b][rr][0], 16, (int)voff,
                (int)(rr * ldb), 0, 0);
        }
        if (wave == 0) {
            const __amdgpu_buffer_rsrc_t rw = __builtin_amdgcn_make_buffer_rsrc(
                (void*)(p.w + r), 0, (int)(nv * 8), kRsrcWord3);
            __builtin_amdgcn_raw_ptr_buffer_load_lds(
                rw, (__attribute__((address_space(3))) void*)&ws[b][0], 4, lane * 4, 0, 0, 0);
        }
    };
    // this wave's loads landed, then everyone's
    auto settle = [&]() __attribute__((always_inline)) {
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
    };
    double* part = p.partials + (int64_t)blockIdx.x * kTile * kTile;
    auto store_block = [&](int bi, int bj, const dv4& d) __attribute__((always_inline)) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
            part[(16 * bi + (lane >> 4) + 4 * q) * kTile + 16 * bj + (lane & 15)] = d[q];
    };
    const int64_t nsteps = r1 > r0 ? (r1 - r0 + R - 1) / R : 0;
    if (nsteps > 0) issue(r0, 0);
    settle();
    if (diag) {
        // blocks and operand sharing as in k_hess
        auto run = [&](auto wc) __attribute__((always_inline)) {
            constexpr int W = decltype(wc)::value;
            constexpr int NA = 8 - W;
            dv4 acc[9];
#pragma unroll
            for (int s2 = 0; s2 < 9; ++s2) acc[s2] = dv4{0.0, 0.0, 0.0, 0.0};
            for (int64_t st = 0; st < nsteps; ++st) {
                const int b = (int)(st & 1);
                if (st + 1 < nsteps) issue(r0 + (st + 1) * R, b ^ 1);
#pragma unroll
                for (int k0 = 0; k0 < R; k0 += 4) {
                    const int kk = k0 + (lane >> 4);
                    const double wk = ws[b][kk];
                    const double a1 = wk * (double)xs[b][kk][16 * W + (lane & 15)];
                    const double a2 = wk * (double)xs[b][kk][16 * (7 - W) + (lane & 15)];
                    double bv[NA];
#pragma unroll
                    for (int s = 0; s < NA; ++s) bv[s] = (double)xs[b][kk][16 * (W + s) + (lane & 15)];
#pragma unroll
                    for (int s = 0; s < NA; ++s)
                        acc[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, bv[s], acc[s], 0, 0, 0);
#pragma unroll
                    for (int t = 0; t <= W; ++t)
                        acc[NA + t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a2, bv[7 - 2 * W + t],
                                                                          acc[NA + t], 0, 0, 0);
                }
                settle();
            }
#pragma unroll
            for (int s = 0; s < NA; ++s) store_block(W, W + s, acc[s]);
#pragma unroll
            for (int t = 0; t <= W; ++t) store_block(7 - W, 7 - W + t, acc[NA + t]);
        };
        switch (wave) {
        case 0: run(std::integral_constant<int, 0>()); break;
        case 1: run(std::integral_constant<int, 1>()); break;
        case 2: run(std::integral_constant<int, 2>()); break;
        default: run(std::integral_constant<int, 3>()); break;
        }
    } else {
        const int qi = (wave >> 1) * 64, qj = (wave & 1) * 64;   // this wave's quadrant
        dv4 acc[4][4];
#pragma unroll
        for (int ta = 0; ta < 4; ++ta)
#pragma unroll
            for (int tb = 0; tb < 4; ++tb) acc[ta][tb] = dv4{0.0, 0.0, 0.0, 0.0};
        for (int64_t st = 0; st < nsteps; ++st) {
            const int b = (int)(st & 1);
            if (st + 1 < nsteps) issue(r0 + (st + 1) * R, b ^ 1);
#pragma unroll
            for (int k0 = 0; k0 < R; k0 += 4) {
                const int kk = k0 + (lane >> 4);
                const double wk = ws[b][kk];
                double a[4], bb[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    a[t] = wk * (double)xs[b][kk][qi + 16 * t + (lane & 15)];
                    bb[t] = (double)xs[b][kk][kTile + qj + 16 * t + (lane & 15)];
                }
#pragma unroll
                for (int ta = 0; ta < 4; ++ta)
#pragma unroll
                    for (int tb = 0; tb < 4; ++tb)
                        acc[ta][tb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ta], bb[tb], acc[ta][tb], 0, 0, 0);
            }
            settle();
        }
#pragma unroll
        for (int ta = 0; ta < 4; ++ta)
#pragma unroll
            for (int tb = 0; tb < 4; ++tb) store_block(qi / 16 + ta, qj / 16 + tb, acc[ta][tb]);
    }
}

// H entries from the partials: each thread sums one tile entry over the
// chunks in chunk order; on a diagonal tile only i <= j is taken and mirrored,
// so H is exactly symmetric.
__global__ __launch_bounds__(kHT) void k_hess_merge(const double* __restrict__ partials,
                                                    const int4* __restrict__ tiles,
                                                    int K, double prec, double* __restrict__ H) {
    const int64_t e_all = (int64_t)blockIdx.x * kHT + threadIdx.x;
    const int tile = (int)(e_all / (kTile * kTile));
    const int e = (int)(e_all % (kTile * kTile));
    const int4 tc = tiles[tile];
    const int nchunk = tc.w;
    const int i = e / kTile, j = e % kTile;
    const int gi = tc.x * kTile + i, gj = tc.y * kTile + j;
    const bool diag = tc.x == tc.y;
    if (gi >= K || gj >= K || (diag && i > j)) return;
    const double* base = partials + (int64_t)tc.z * kTile * kTile + e;
    double s = 0.0;
    for (int c = 0; c < nchunk; c += 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = c + u < nchunk ? base[(int64_t)(c + u) * kTile * kTile] : 0.0;
#pragma unroll
        for (int u = 0; u < 8; ++u) s += v[u];
    }
    const double h = -s - (gi == gj ? prec : 0.0);
    H[(int64_t)gi * K + gj] = h;
    if (gi != gj) H[(int64_t)gj * K + gi] = h;
}

// Matrix-core throughput probe: 16 independent FP64 16x16x4 accumulators per
// wave, `iters` rounds; the sum of the results is written (per lane) only so
// that the work is kept.  The first round starts from zero inside the matrix
// instruction: with the accumulators zeroed by moves the compiler kept them
// in VGPRs between rounds and copied all 128 registers to and from AGPRs
// around every round, which halved the matrix rate the probe saw.
__global__ __launch_bounds__(kHT) void k_mfma_probe(double* __restrict__ sink, int iters, double seed) {
    const double a = seed + threadIdx.x, b = seed - threadIdx.x;
    dv4 acc[16];
#pragma unroll
    for (int i = 0; i < 16; ++i)
        acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, dv4{0.0, 0.0, 0.0, 0.0}, 0, 0, 0);
    for (int it = 1; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[i], 0, 0, 0);
    }
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < 16; ++i) s += acc[i][0] + acc[i][1] + acc[i][2] + acc[i][3];
    sink[(int64_t)blockIdx.x * kHT + threadIdx.x] = s;
}

}  // namespace
}  // namespace glmrt

using namespace glmrt;

extern "C" {

glm_status glm_logpost_grad_hess(glm_ctx* ctx, glm_dataset_id id, const double* beta,
                                 const glm_prior* prior, double* out, double* H, void* stream) {
    clear_error();
    if (!ctx || !beta || !prior || !out || !H)
        GLM_FAIL(GLM_EINVAL, "glm_logpost_grad_hess: NULL argument");
    if (!(prior->prec >= 0.0)) GLM_FAIL(GLM_EINVAL, "glm_logpost_grad_hess: prior precision < 0");
    std::lock_guard<std::mutex> lk(ctx->mu);
    auto it = ctx->datasets.find(id);
    if (it == ctx->datasets.end())
        GLM_FAIL(GLM_ENOTFOUND, "glm_logpost_grad_hess: unknown data set %lld", (long long)id);
    glm_status st = use_device(ctx);
    if (st != GLM_OK) return st;
    const Dataset& ds = it->second;
    const int K = ds.d.K;
    const int64_t N = ds.d.N;
    hipStream_t s = (hipStream_t)stream;

    const int ntile = (K + kTile - 1) / kTile;
    const int nup = ntile * (ntile + 1) / 2;
    // Chunks per tile, weighted by the time per row of one of its blocks, so
    // that the blocks take about equal time: a diagonal tile's wave has 9
    // blocks of 16 x 16 against 16 on an off-diagonal one, but reads up to
    // 10 operands per four rows where the other reads 8, and its rows took
    // 0.60 of the time of an off-diagonal tile's (FP32 rows of 256 columns,
    // 512 blocks over 4M rows per tile kind); the grid fills
    // the two-blocks-per-CU slots at most (a block past them runs after all
    // the others, nearly doubling the kernel's time).
    const int64_t slots = 2 * (int64_t)ctx->num_cu;
    const int64_t maxch = std::max<int64_t>(1, (N + 31) / 32);
    constexpr double kDiagWeight = 0.60, kOffWeight = 1.0;
    const double wsum = kDiagWeight * ntile + kOffWeight * (nup - ntile);
    std::vector<int> tl;   // per tile: row, column, first block, chunks
    std::vector<int> bl;   // per block: tile, chunk
    for (int a = 0, t = 0; a < ntile; ++a)
        for (int b = a; b < ntile; ++b, ++t) {
            const double wt = a == b ? kDiagWeight : kOffWeight;
            const int nch = (int)std::min<int64_t>(
                maxch, std::max<int64_t>(1, (int64_t)std::floor((double)slots * wt / wsum)));
            tl.insert(tl.end(), {a, b, (int)(bl.size() / 2), nch});
            for (int c = 0; c < nch; ++c) bl.insert(bl.end(), {t, c});
        }
    const int nblk = (int)(bl.size() / 2);

    // per-stream buffers: w (N), partials (one tile per block), tile and block tables
    HessBuf& hb = ctx->hess[stream];
    const size_t need = (size_t)std::max<int64_t>(N, 1) + (size_t)nblk * kTile * kTile;   // doubles
    const size_t nint = tl.size() + bl.size();
    if (hb.cap < need || hb.ntick < nint) {
        if (hb.buf) {
            GLM_HIP_CHECK(hipStreamSynchronize(s));
            GLM_HIP_CHECK(hipFree(hb.buf));
            hb = HessBuf{};
        }
        const size_t cap = need * 5 / 4 + 1024;
        const size_t nt = std::max<size_t>(nint * 2, 256);
        if (hipMalloc((void**)&hb.buf, cap * sizeof(double) + nt * sizeof(int)) != hipSuccess)
            GLM_FAIL(GLM_ENOMEM, "glm_logpost_grad_hess: device allocation failed");
        hb.cap = cap;
        hb.ntick = nt;
        hb.tiles = reinterpret_cast<int*>(hb.buf + cap);
        hb.tiles_for = -1;
    }
    double* w = hb.buf;
    double* partials = hb.buf + std::max<int64_t>(N, 1);
    if (hb.tiles_for != ntile || hb.tiles_rows != maxch) {
        std::vector<int> t(tl);
        t.insert(t.end(), bl.begin(), bl.end());
        GLM_HIP_CHECK(hipMemcpyAsync(hb.tiles, t.data(), t.size() * sizeof(int), hipMemcpyHostToDevice, s));
        GLM_HIP_CHECK(hipStreamSynchronize(s));
        hb.tiles_for = ntile;
        hb.tiles_rows = maxch;
    }

    // 1. f, g and the row weights
    size_t np, ng, nc;
    scratch_need(ds.plan, K, 1, &np, &ng, &nc);
    Scratch* sc = nullptr;
    st = get_scratch(ctx, stream, np, ng, nc, &sc);
    if (st != GLM_OK) return st;
    st = launch_fused(ds.d, ds.plan, ds.plan.fn, 1, beta, prior->mean, nullptr, prior->prec, 1, out,
                      sc, s, w);
    if (st != GLM_OK) return st;

    // 2. H = -X^t W X - prec I
    HessParams p;
    p.X = ds.d.X;
    p.ldx = ds.d.ldx;
    p.scale = ds.d.col_scale;
    p.w = w;
    p.N = N;
    p.K = K;
    p.tiles = reinterpret_cast<const int4*>(hb.tiles);
    p.blocks = reinterpret_cast<const int2*>(hb.tiles + tl.size());
    p.partials = partials;
    const dim3 grid((unsigned)nblk);
    switch (ds.d.dtype) {
    case GLM_F64: hipLaunchKernelGGL(k_hess<GLM_F64>, grid, dim3(kHT), 0, s, p); break;
    case GLM_F32: hipLaunchKernelGGL(k_hess_lds, grid, dim3(kHT), 0, s, p); break;
    case GLM_BF16: hipLaunchKernelGGL(k_hess<GLM_BF16>, grid, dim3(kHT), 0, s, p); break;
    default: hipLaunchKernelGGL(k_hess<GLM_FP8_E4M3>, grid, dim3(kHT), 0, s, p); break;
    }
    GLM_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL(k_hess_merge, dim3((unsigned)((int64_t)nup * kTile * kTile / kHT)), dim3(kHT), 0,
                       s, partials, p.tiles, K, prior->prec, H);
    GLM_HIP_CHECK(hipGetLastError());
    return GLM_OK;
}

glm_status glm_probe_mfma_f64(glm_ctx* ctx, int32_t iters, double* tflops) {
    clear_error();
    if (!ctx || !tflops || iters < 1) GLM_FAIL(GLM_EINVAL, "glm_probe_mfma_f64: bad argument");
    std::lock_guard<std::mutex> lk(ctx->mu);
    glm_status st = use_device(ctx);
    if (st != GLM_OK) return st;
    const int blocks = 2 * ctx->num_cu;
    double* sink = nullptr;
    if (hipMalloc((void**)&sink, (size_t)blocks * kHT * sizeof(double)) != hipSuccess)
        GLM_FAIL(GLM_ENOMEM, "glm_probe_mfma_f64: device allocation failed");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    hipStream_t s = ctx->own_stream;
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_mfma_probe, dim3(blocks), dim3(kHT), 0, s, sink, 8, 1.0);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_mfma_probe, dim3(blocks), dim3(kHT), 0, s, sink, iters, 1.0);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(sink);
    if (e != hipSuccess) GLM_FAIL(GLM_EHIP, "glm_probe_mfma_f64: %s", hipGetErrorString(e));
    // flops: waves x rounds x 16 instructions x (16 x 16 x 4 multiply-adds x 2)
    const double flops = (double)blocks * (kHT / 64) * iters * 16.0 * 2048.0;
    *tflops = flops / (ms * 1e-3) / 1e12;
    return GLM_OK;
}

}  // extern "C"
