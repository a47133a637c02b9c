// Several coefficient vectors per pass over BF16 storage, with the linear
// predictors on the matrix cores.
//
// With NB vectors per read of X the VALU kernels spend three FMAs per element
// and vector (the split-beta dot product and the gradient), which makes them
// VALU-bound from two vectors up when X is BF16.  The linear predictors
// u = X B are a (rows x K) by (K x NB) product, a dense contraction, so here
// they run as v_mfma_f32_16x16x32_bf16.  Every vector's beta is split into
// four BF16 pieces, beta = p0 + p1 + p2 + p3 up to about 2^-32 |beta|, each
// piece the rounding of what the earlier ones leave; the 16 columns of B are
// NB = 4 vectors x 4 pieces.  Products of BF16 values are exact, each piece is
// accumulated in FP32 over K (the FP32 accumulation of the VALU kernels'
// beta_hi / beta_lo split), and the four piece sums are added in FP64.  The
// per-row map is the same FP64 one, and the gradient stays on the VALU: one
// FMA per element and vector, FP32 over the 16 rows of a batch, then FP64.
//
// Layouts.  A batch is 16 rows.  The matrix cores take from lane l row
// l % 16 and chunk (8 columns) 4s + l / 16 of slice s, which is how the batch
// is loaded: S = LPR / 4 slices of 32 columns cover the 4S >= NC chunks of a
// row.  The same registers go to an LDS tile, from which the gradient phase
// reads the layout of the VALU kernels: lane l owns chunk cl = l % LPR of
// rows l / LPR + RPW j, so the column merge is the VALU kernels' one.  Output
// register v of lane l is D[4 (l / 16) + v][l % 16]; the four lanes of a quad
// hold the four pieces of one vector and add them in piece order (all four
// get the same bits); lane l evaluates the per-row map of row
// 4 (l / 16) + l % 4 for vector (l % 16) / 4.
#pragma once

#include "fg_kernel.hpp"

namespace glmk {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Round-to-nearest-even of a float to BF16 (the bit pattern); NaN gives a
// quiet NaN, infinities stay infinite.
__device__ __forceinline__ uint32_t bf16_rne_bits(float x) {
    const uint32_t u = __float_as_uint(x);
    if ((u & 0x7FFFFFFFu) > 0x7F800000u) return 0x7FC0u;
    return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}

// v = p0 + p1 + p2 + p3 + a remainder of about 2^-32 |v|: each piece is the
// BF16 rounding of what the earlier ones leave, and every difference is exact
// in FP64 (a rounding to 8 bits of a 53-bit value differs from it by a number
// that fits in 53 bits).
__device__ __forceinline__ void bf16_pieces(double v, uint32_t (&pc)[4]) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        pc[q] = bf16_rne_bits((float)v);
        v -= (double)__uint_as_float(pc[q] << 16);
    }
}

__device__ __forceinline__ float quad_bcast(float v, int src) {
    const int ctrl = src * 0x55;   // quad_perm [src, src, src, src]
    switch (ctrl) {
    case 0x00: return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x00, 0xF, 0xF, true));
    case 0x55: return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x55, 0xF, 0xF, true));
    case 0xAA: return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xAA, 0xF, 0xF, true));
    default: return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xFF, 0xF, 0xF, true));
    }
}

template <int LPR, int NB>
struct MxTile {
    static_assert(NB == 4, "four vectors x four pieces fill the 16 columns of B");
    static_assert(LPR >= 4 && LPR <= 64, "a row spans 4 to 64 chunks");
    static constexpr int VE = 8;                 // BF16 values per 16-byte chunk
    static constexpr int CHUNKS = 1;             // gradient layout: chunks per lane and row
    static constexpr int S = LPR / 4;            // slices of 4 chunks = chunks per lane and batch
    static constexpr int RPW = 64 / LPR;         // rows per wave-wide LDS read (gradient layout)
    static constexpr int BATCH = 16;             // rows per batch
    static constexpr int KT = LPR * VE;          // columns an instance covers
    static constexpr int LROW = 4 * S + 1;       // 16-byte units per LDS tile row (one of padding)
    static constexpr int TILE_U = 16 * LROW;     // 16-byte units of a wave's LDS tile
    static constexpr int BTAB_U = 4 * S * 16;    // 16-byte units of the B table: chunk x column

    struct Tile {
        u32x4 x[S];
        unsigned yb;
    };

    int lane, seg, cl, mi, mk, NC;
    int fam;
    bool ragged;
    int last_s;          // slice holding the last (possibly partial) chunk
    u32x4 lastmask;      // valid bytes of this lane's chunk in slice last_s
    uint32_t ldb;        // row stride in bytes
    uint32_t lbase;      // byte offset of row mi, chunk mk within a batch
    int tr_row, tr_b;    // row (within a batch) and vector of this lane's per-row map
    double ftr;          // this lane's sum of t over its rows
    double g64[NB][1][VE];
    double facc[NB];     // after wave_totals: the wave's f per vector

    __device__ __forceinline__ void init(int lane_, int K, int64_t ldx, int family) {
        lane = lane_;
        fam = family;
        seg = lane / LPR;
        cl = lane % LPR;
        mi = lane & 15;
        mk = lane >> 4;
        NC = __builtin_amdgcn_readfirstlane((K + VE - 1) / VE);
        ragged = (K % VE) != 0;
        ldb = (uint32_t)(ldx * 2);
        lbase = (uint32_t)mi * ldb + (uint32_t)mk * 16u;
        tr_row = 4 * mk + (lane & 3);
        tr_b = (lane >> 2) & 3;
        last_s = __builtin_amdgcn_readfirstlane((NC - 1) >> 2);
        const int vb = mk == ((NC - 1) & 3) ? K * 2 - (NC - 1) * 16 : 16;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int nbq = min(4, max(0, vb - 4 * q));
            lastmask[q] = nbq >= 4 ? 0xFFFFFFFFu : ((1u << (8 * nbq)) - 1u);
        }
    }

    __device__ __forceinline__ int col(int, int e) const { return cl * VE + e; }

    __device__ __forceinline__ void zero_acc() {
#pragma unroll
        for (int b = 0; b < NB; ++b) {
#pragma unroll
            for (int e = 0; e < VE; ++e) g64[b][0][e] = 0.0;
            facc[b] = 0.0;
        }
        ftr = 0.0;
    }

    // Rows row0 .. row0 + 15 of a row block whose valid rows end at
    // row0 + navail; rows past the end and chunks past the row's last come
    // back as zeros from the buffer range check.
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
        for (int s = 0; s < S; ++s) {
            const uint32_t off = 4 * s + mk < NC ? lbase + 64u * s : 0x80000000u;
            t.x[s] = __builtin_amdgcn_raw_buffer_load_b128(rx, off, 0, kLoadNT);
        }
        const __amdgpu_buffer_rsrc_t ry = __builtin_amdgcn_make_buffer_rsrc(
            (void*)(y + row0), 0, (int)nvalid, kRsrcWord3);
        t.yb = __builtin_amdgcn_raw_buffer_load_b8(ry, (uint32_t)tr_row, 0, kLoadNT);
        __builtin_amdgcn_sched_barrier(0);
    }

    // First phase of a batch: the tile goes to this wave's LDS tile lt and
    // the four pieces of each vector's linear predictor come back from the
    // matrix cores (bt: the block's B table).  The tile's registers are free
    // afterwards.
    __device__ __forceinline__ f32x4 predict(Tile& t, u32x4* lt, const u32x4* bt) const {
        if (ragged) {
#pragma unroll
            for (int s = 0; s < S; ++s)
                if (s == last_s) t.x[s] &= lastmask;
        }
#pragma unroll
        for (int s = 0; s < S; ++s) lt[mi * LROW + 4 * s + mk] = t.x[s];
        f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int s = 0; s < S; ++s) {
            if (4 * s >= NC) break;
            const u32x4 bw = bt[(4 * s + mk) * 16 + mi];
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, t.x[s]),
                                                          __builtin_bit_cast(bf16x8, bw), acc, 0,
                                                          0, 0);
        }
        return acc;
    }

    // Second phase: piece sums, the per-row map and the gradient of the
    // batch's first nvalid rows for the first nact vectors.  yb: the response
    // byte of this lane's row; rb: this wave's 16 x NB residuals.
    __device__ __forceinline__ void accumulate(const f32x4 acc, unsigned yb, uint32_t nvalid,
                                               const u32x4* lt, float* rb, int nact) {
        double uq[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const float a0 = quad_bcast(acc[v], 0), a1 = quad_bcast(acc[v], 1);
            const float a2 = quad_bcast(acc[v], 2), a3 = quad_bcast(acc[v], 3);
            uq[v] = (((double)a0 + (double)a1) + (double)a2) + (double)a3;
        }
        const int p = lane & 3;
        double u = uq[0];
        u = p == 1 ? uq[1] : u;
        u = p == 2 ? uq[2] : u;
        u = p == 3 ? uq[3] : u;

        // per-row map of (tr_row, tr_b); residuals to LDS
        double tt, rr;
        tr_map(u, yb, fam, tt, rr);
        const bool ok = (uint32_t)tr_row < nvalid && tr_b < nact;
        if (ok) ftr += tt;
        rb[tr_row * NB + tr_b] = ok ? (float)rr : 0.0f;
        __builtin_amdgcn_wave_barrier();

        // gradient from the LDS tile, in the layout of the VALU kernels
        float g32[NB][VE];
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int e = 0; e < VE; ++e) g32[b][e] = 0.0f;
#pragma unroll 2
        for (int j = 0; j < S; ++j) {
            const int row = seg + RPW * j;
            const u32x4 xw = lt[row * LROW + cl];
            const f32x4 rv = *reinterpret_cast<const f32x4*>(rb + row * NB);
            float xv[VE];
            decode_chunk<DT_BF16>(xw, xv);
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                if (b >= nact) break;
#pragma unroll
                for (int e = 0; e < VE; ++e) g32[b][e] = fmaf(rv[b], xv[e], g32[b][e]);
            }
        }
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            if (b >= nact) break;
#pragma unroll
            for (int e = 0; e < VE; ++e) g64[b][0][e] += (double)g32[b][e];
        }
        __builtin_amdgcn_wave_barrier();
    }

    // Column sums over the segments (every lane of segment 0 ends with its
    // columns' totals) and the wave's f per vector (every lane).
    __device__ __forceinline__ void wave_totals() {
#pragma unroll
        for (int b = 0; b < NB; ++b) {
#pragma unroll
            for (int e = 0; e < VE; ++e) g64[b][0][e] = cross_segment_sum<LPR>(g64[b][0][e]);
            double v = tr_b == b ? ftr : 0.0;
#pragma unroll
            for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
            facc[b] = v;
        }
    }
};

// Block blk (of p.nblocks) of the evaluation of p.nb (<= NB) vectors over a
// BF16 data set whose rows span 4 * (LPR / 4) or fewer chunks (and more than
// LPR / 2 when LPR > 4).
template <int LPR, int WPB, int NB>
__device__ __forceinline__ void fg_pass_mx(const FgParams& p, const int blk) {
    using WT = MxTile<LPR, NB>;
    constexpr int BATCH = WT::BATCH;
    constexpr int NT = WPB * 64;
    __shared__ u32x4 btab[WT::BTAB_U];
    __shared__ u32x4 ltile[WPB][WT::TILE_U];
    __shared__ __attribute__((aligned(16))) float rbuf[WPB][16 * NB];
    const int nact = __builtin_amdgcn_readfirstlane(min(p.nb, NB));

    // B table: entry (chunk c, column n) holds, for columns 8c .. 8c + 7, the
    // BF16 piece n % 4 of vector n / 4 (zero past K and for inactive vectors).
    {
        uint32_t* bw = reinterpret_cast<uint32_t*>(btab);
        for (int idx = threadIdx.x; idx < 4 * WT::S * NB * 4; idx += NT) {
            const int w = idx & 3, b = (idx >> 2) % NB, c = idx / (4 * NB);
            const int k = 8 * c + 2 * w;
            uint32_t lo[4] = {0u, 0u, 0u, 0u}, hi[4] = {0u, 0u, 0u, 0u};
            if (b < nact) {
                if (k < p.K) bf16_pieces(p.beta[(int64_t)b * p.K + k], lo);
                if (k + 1 < p.K) bf16_pieces(p.beta[(int64_t)b * p.K + k + 1], hi);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) bw[(c * 16 + 4 * b + q) * 4 + w] = lo[q] | (hi[q] << 16);
        }
    }
    __syncthreads();

    WT wt;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    wt.init(threadIdx.x & 63, p.K, p.ldx, p.family);
    wt.zero_acc();

    // Grid-strided batches.  Narrow rows keep two tiles in registers (the
    // next batch loads while this one is computed); with 16 slices a single
    // tile is reloaded as soon as the matrix cores have read it, which keeps
    // the kernel within the register file.
    const int64_t nbatch = (p.N + BATCH - 1) / BATCH;
    const int64_t tw = (int64_t)p.nblocks * WPB;
    const int64_t gw = (int64_t)blk * WPB + wave;
    const int64_t step = tw * BATCH;
    const int64_t rend = nbatch * BATCH;
    auto nval = [&](int64_t r) { return (uint32_t)max((int64_t)0, min((int64_t)BATCH, p.N - r)); };
    int64_t r = gw * BATCH;
    if constexpr (WT::S >= 16) {
        typename WT::Tile ta;
        wt.load(ta, p.X, p.y, r, p.N - r);
        for (; r < rend; r += step) {
            const f32x4 acc = wt.predict(ta, ltile[wave], btab);
            const unsigned yb = ta.yb;
            wt.load(ta, p.X, p.y, r + step, p.N - r - step);
            wt.accumulate(acc, yb, nval(r), ltile[wave], rbuf[wave], nact);
        }
    } else {
        typename WT::Tile ta, tb;
        wt.load(ta, p.X, p.y, r, p.N - r);
        for (; r < rend; r += 2 * step) {
            wt.load(tb, p.X, p.y, r + step, p.N - r - step);
            wt.accumulate(wt.predict(ta, ltile[wave], btab), ta.yb, nval(r), ltile[wave],
                          rbuf[wave], nact);
            if (r + step >= rend) break;
            wt.load(ta, p.X, p.y, r + 2 * step, p.N - r - 2 * step);
            wt.accumulate(wt.predict(tb, ltile[wave], btab), tb.yb, nval(r + step), ltile[wave],
                          rbuf[wave], nact);
        }
    }
    wt.wave_totals();
    block_merge<WT, DT_BF16, WPB, NB>(p, blk, wt, wave);
}

template <int LPR, int WPB, int NB>
__global__ __launch_bounds__(WPB * 64) void fg_fused_mx(FgParams p) {
    fg_pass_mx<LPR, WPB, NB>(p, blockIdx.x);
}

// Fleet form (several data sets of one geometry per launch), as fg_fleet.
template <int LPR, int WPB, int NB>
__global__ __launch_bounds__(WPB * 64) void fg_fleet_mx(const FleetJob* jobs, const uint16_t* blk_job) {
    const int j = blk_job[blockIdx.x];
    const FgParams p = jobs[j].p;
    fg_pass_mx<LPR, WPB, NB>(p, (int)blockIdx.x - jobs[j].blk0);
}

}  // namespace glmk
