// Matrix-core instances of the several-beta pass for BF16 storage
// (fg_mfma.hpp): four vectors per read of X, rows of 9 to 64 chunks (K from
// 65 to 512).  Narrower rows stay on the VALU kernels, whose batches of
// many short rows amortise the per-row map better than 16-row batches.
#include "fg_mfma.hpp"
#include "runtime.hpp"

namespace glmrt {
namespace {

// Waves per block: two per SIMD where the registers allow it (16 and 32
// lanes per row), one for 64.
template <int LPR>
constexpr int mx_wpb() {
    return LPR <= 32 ? 8 : 4;
}

template <int LPR>
MultiInst mxinst() {
    constexpr int W = mx_wpb<LPR>();
    MultiInst m;
    m.fn = reinterpret_cast<const void*>(&glmk::fg_fused_mx<LPR, W, 4>);
    m.R = 16;
    m.NB = 4;
    m.fleet = reinterpret_cast<const void*>(&glmk::fg_fleet_mx<LPR, W, 4>);
    m.wpb = W;
    return m;
}

}  // namespace

MultiInst mx_instance(int lpr) {
    switch (lpr) {
    case 16: return mxinst<16>();
    case 32: return mxinst<32>();
    case 64: return mxinst<64>();
    }
    return MultiInst{};
}

}  // namespace glmrt
