// Kernel instances of the several-beta passes, by storage type.  Each
// storage type's instances are compiled in a translation unit of their own
// (glm_multi_<type>.hip), which keeps the build parallel.
#pragma once

#include "fg_kernel.hpp"
#include "runtime.hpp"

namespace glmrt {
namespace multi_detail {

constexpr int WPB = 4;

// R = 8 row slots per lane keeps the NB copies of beta and of the gradient
// accumulators within the register file; instances with more than 32 values
// of beta or gradient per lane (NB x columns per lane) are not built.  (With
// FP64 coefficients and linear predictors, 4 slots and 8 waves per block no
// longer fit two waves per SIMD: FP32 rows of 32 lanes with 8 vectors then
// spilled to scratch and ran 144 us per vector over 2 GB against 125 with 4
// vectors.)
//
// These geometries take 4 row slots instead (times over 2 GB):
//  - FP32 rows of 512 columns (64 lanes x 2 chunks) with 2 vectors, with a
//    ring of 3 tiles (the tile then fits in FP64 once for all vectors): 309
//    us against 331 with 8 slots (with 4 vectors 8 slots stay faster, 447
//    against 480 us);
//  - FP32 rows of 1024 columns (4 chunks per lane), with a ring of 3 tiles:
//    333 us against 561 for 2 vectors (8 slots spilled to scratch memory);
//  - FP64 rows of 2 or 4 chunks per lane (256 or 512 columns): 345 against
//    810 us for 4 vectors at 512 columns (8 slots spilled), 315 against 333
//    for 2; 525 against 607 for 8 vectors at 256 columns, 320 against 377
//    for 4;
//  - BF16 rows of at most 32 columns (one chunk on at most 4 lanes; the tile
//    then fits in FP64 once): a pass of 4 vectors 2491 against 2877 us at 8
//    columns, 1158 against 1333 at 32.  (At 128 and 512 columns 8 slots stay
//    faster: 508 against 556 us and 486 against 553 for 2 vectors.)
// Elsewhere 8 slots measured faster, e.g. 8 vectors over FP64 rows of 128
// columns 570 against 749 us, over FP32 rows of 256 columns 747 against
// 1027; 2 vectors over BF16 rows of 1024 columns 489 against 551.
template <int DT, int LPR, int CPL, int NB>
MultiInst minst() {
    constexpr int VE = 16 / glmk::ElemSize<DT>::v;
    constexpr bool F32_WIDE =
        DT == glmk::DT_F32 && LPR == 64 && ((CPL == 2 && NB == 2) || CPL == 4);
    constexpr bool F64_WIDE = DT == glmk::DT_F64 && LPR == 64 && CPL >= 2;
    constexpr bool BF16_NARROW = DT == glmk::DT_BF16 && CPL == 1 && LPR <= 4;
    constexpr int R = F32_WIDE || F64_WIDE || BF16_NARROW ? 4 : 8;
    constexpr int NBUF = F32_WIDE ? 3 : 2;
    if constexpr (NB * CPL * VE > 32) {
        return MultiInst{};
    } else {
        return MultiInst{reinterpret_cast<const void*>(&glmk::fg_fused<DT, LPR, CPL, R, WPB, NB, NBUF>), R,
                         NB, reinterpret_cast<const void*>(&glmk::fg_fleet<DT, LPR, CPL, R, WPB, NB, NBUF>)};
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
inline MultiInst mpick_nb(int lpr, int cpl, int nb) {
    switch (nb) {
    case 8: return mpick<DT, 8>(lpr, cpl);
    case 4: return mpick<DT, 4>(lpr, cpl);
    case 2: return mpick<DT, 2>(lpr, cpl);
    }
    return MultiInst{};
}

}  // namespace multi_detail

// The instance of storage type dtype for rows of lpr lanes x cpl chunks with
// nb vectors per pass (nb in {2, 4, 8}); fn == nullptr if none is built.
MultiInst multi_pick_f64(int lpr, int cpl, int nb);
MultiInst multi_pick_f32(int lpr, int cpl, int nb);
MultiInst multi_pick_bf16(int lpr, int cpl, int nb);
MultiInst multi_pick_fp8(int lpr, int cpl, int nb);

}  // namespace glmrt
