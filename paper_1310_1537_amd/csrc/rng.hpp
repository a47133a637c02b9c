// Counter-based random numbers on the device, for samplers that draw their
// own proposals, momenta and accept uniforms (the paper's batch generation of
// uniform and normal deviates, Sec. 4.4, moved onto the GPU).
//
// Generator: Philox4x64-10 (J. K. Salmon, M. A. Moraes, R. O. Dror and
// D. E. Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11).  A block
// of four 64-bit words is a keyed bijection of a four-word counter: ten rounds,
// each taking the 128-bit products of counter words 0 and 2 with two fixed odd
// multipliers and recombining them as (hi(M1 x2) ^ x1 ^ k0, lo(M1 x2),
// hi(M0 x0) ^ x3 ^ k1, lo(M0 x0)); the key words advance by Weyl constants
// between rounds.  Any value of any stream is computed from its index alone,
// so every thread draws what it needs with no shared state.
//
// Streams (key = (seed, chain); counter word 2 = purpose, word 3 = stream):
//   uniforms  value i = word i mod 4 of the block at counter (i / 4, 0, 1, s),
//             mapped to ((w >> 12) + 1/2) 2^-52, in [2^-53, 1 - 2^-53];
//   normals   Marsaglia's polar method (SIAM Review 6, 1964): pair p takes
//             attempt a from the block at counter (p, a / 2, 2, s), words
//             2 (a mod 2) and 2 (a mod 2) + 1, as u, v = 2 U - 1; the first
//             point with 0 < s = fma(u, u, v v) < 1 gives u c and v c,
//             c = sqrt(-2 log(s) / s);
//   HMC       momenta of iteration t: normals of purpose 16, stream t; accept
//             uniform of iteration t: word 0 of the block at (0, 0, 17, t).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tr_math.hpp"

namespace glmk {

enum : uint64_t { RNG_UNIFORM = 1, RNG_NORMAL = 2, RNG_HMC_MOMENTUM = 16, RNG_HMC_ACCEPT = 17 };

// At most this many polar attempts per pair (the chance that all miss the
// disc is (1 - pi/4)^256 < 10^-170); a pair that never hits returns zeros.
constexpr int kPolarMaxAttempts = 256;

struct Block4 {
    uint64_t w[4];
};

__device__ __forceinline__ Block4 philox4x64_10(uint64_t x0, uint64_t x1, uint64_t x2, uint64_t x3,
                                                uint64_t k0, uint64_t k1) {
    constexpr uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    constexpr uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += W0;
            k1 += W1;
        }
        const uint64_t hi0 = __umul64hi(M0, x0), lo0 = M0 * x0;
        const uint64_t hi1 = __umul64hi(M1, x2), lo1 = M1 * x2;
        const uint64_t y0 = hi1 ^ x1 ^ k0, y2 = hi0 ^ x3 ^ k1;
        x0 = y0;
        x1 = lo1;
        x2 = y2;
        x3 = lo0;
    }
    return Block4{{x0, x1, x2, x3}};
}

__device__ __forceinline__ double u01(uint64_t w) {
    return ((double)(w >> 12) + 0.5) * 0x1.0p-52;
}

// Normals 2p and 2p + 1 of a stream.
__device__ __forceinline__ void polar_pair(uint64_t seed, uint64_t chain, uint64_t purpose,
                                           uint64_t stream, uint64_t p, double& z0, double& z1) {
    z0 = z1 = 0.0;
    for (int a = 0; a < kPolarMaxAttempts; ++a) {
        const Block4 b = philox4x64_10(p, (uint64_t)(a >> 1), purpose, stream, seed, chain);
        const uint64_t wu = (a & 1) ? b.w[2] : b.w[0];
        const uint64_t wv = (a & 1) ? b.w[3] : b.w[1];
        const double u = 2.0 * u01(wu) - 1.0;
        const double v = 2.0 * u01(wv) - 1.0;
        const double s = fma(u, u, v * v);
        if (s > 0.0 && s < 1.0) {
            const double c = sqrt(-2.0 * log_f64(s) / s);
            z0 = u * c;
            z1 = v * c;
            return;
        }
    }
}

}  // namespace glmk
