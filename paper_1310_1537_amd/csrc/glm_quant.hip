// Storage conversions of an FP32 design matrix: BF16 and per-column-scaled
// FP8 E4M3FN.  Encoders work on the IEEE bit patterns with integer
// arithmetic, so the codes do not depend on any hardware conversion mode.
#include "runtime.hpp"

namespace glmrt {

namespace {

// Round-to-nearest-even BF16 code of a binary32 value; NaN stays a quiet NaN.
__device__ __forceinline__ uint16_t bf16_rne(float v) {
    const unsigned b = __float_as_uint(v);
    if ((b & 0x7FFFFFFFu) > 0x7F800000u) return (uint16_t)((b >> 16) | 0x0040u);
    const unsigned bias = 0x7FFFu + ((b >> 16) & 1u);
    return (uint16_t)((b + bias) >> 16);
}

// Nearest E4M3FN code (ties to even), saturating to +-448 (code 0x7E).
__device__ __forceinline__ uint8_t e4m3_rne_sat(float v) {
    const unsigned b = __float_as_uint(v);
    const unsigned sign = (b >> 24) & 0x80u;
    const unsigned a = b & 0x7FFFFFFFu;
    if (a > 0x7F800000u) return (uint8_t)(sign | 0x7Fu);      // NaN
    if (a >= 0x43E00000u) return (uint8_t)(sign | 0x7Eu);     // |v| >= 448
    const unsigned e32 = a >> 23;                              // biased binary32 exponent
    if (e32 >= 121u) {
        // normal E4M3 range (|v| >= 2^-6): keep 3 mantissa bits
        const unsigned keep = a >> 20;                         // exponent and top 3 bits
        const unsigned rest = a & 0xFFFFFu;
        const unsigned up = (rest > 0x80000u || (rest == 0x80000u && (keep & 1u))) ? 1u : 0u;
        unsigned code = keep + up - ((127u - 7u) << 3);
        if (code > 0x7Eu) code = 0x7Eu;
        return (uint8_t)(sign | code);
    }
    if (e32 == 0u) return (uint8_t)sign;                       // binary32 zero / subnormal
    // |v| < 2^-6: multiples of 2^-9.  significand * 2^(e32 - 150) * 2^9
    const unsigned sig = (a & 0x7FFFFFu) | 0x800000u;
    const unsigned sh = 141u - e32;                            // >= 21
    if (sh >= 26u) return (uint8_t)sign;                       // below half of 2^-9
    const unsigned q = sig >> sh;
    const unsigned rem = sig & ((1u << sh) - 1u);
    const unsigned half = 1u << (sh - 1u);
    const unsigned up = (rem > half || (rem == half && (q & 1u))) ? 1u : 0u;
    return (uint8_t)(sign | (q + up));
}

__global__ void k_quant_bf16(const float* X, int64_t N, int K, int64_t ldx, uint16_t* Q,
                             int64_t ldq) {
    const int64_t total = N * (int64_t)K;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t n = i / K;
        const int k = (int)(i - n * K);
        Q[n * ldq + k] = bf16_rne(X[n * ldx + k]);
    }
}

// Column max of |x| into amax (binary32 bits; all values >= 0 so the unsigned
// order of the bits is the numeric order and atomicMax is exact).
__global__ void k_col_absmax(const float* X, int64_t N, int K, int64_t ldx, unsigned* amax) {
    const int64_t rows_per = (N + gridDim.x - 1) / gridDim.x;
    const int64_t r0 = (int64_t)blockIdx.x * rows_per;
    const int64_t r1 = min(N, r0 + rows_per);
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
        unsigned m = 0u;
        for (int64_t n = r0; n < r1; ++n) m = max(m, __float_as_uint(fabsf(X[n * ldx + k])));
        if (m) atomicMax(&amax[k], m);
    }
}

__global__ void k_scales(const unsigned* amax, int K, float* scale) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < K) {
        const float a = __uint_as_float(amax[k]);
        scale[k] = a > 0.0f ? __fdiv_rn(a, 448.0f) : 1.0f;
    }
}

__global__ void k_zero_u32(unsigned* p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

__global__ void k_quant_fp8(const float* X, int64_t N, int K, int64_t ldx, const float* scale,
                            uint8_t* Q, int64_t ldq) {
    const int64_t total = N * (int64_t)K;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t n = i / K;
        const int k = (int)(i - n * K);
        Q[n * ldq + k] = e4m3_rne_sat(__fdiv_rn(X[n * ldx + k], scale[k]));
    }
}

// Row-wise forms for rows of whole 4-float chunks (K, ldx and ldq multiples
// of 4, 16-byte aligned X): one 16-byte load and one 8- or 4-byte store per
// four elements; the threads of a block take the chunks of a row, the blocks
// take rows in turn.
typedef float qfv4 __attribute__((ext_vector_type(4)));
typedef unsigned quv2 __attribute__((ext_vector_type(2)));

// Four rows per trip with their loads issued together.
constexpr int kRowUnroll = 4;

__global__ __launch_bounds__(256) void k_quant_bf16_v4(const float* X, int64_t N, int K, int64_t ldx,
                                                       uint16_t* Q, int64_t ldq) {
    const int kc = K >> 2;
    const int64_t G = gridDim.x;
    for (int c = threadIdx.x; c < kc; c += blockDim.x) {
        for (int64_t n0 = blockIdx.x; n0 < N; n0 += kRowUnroll * G) {
            qfv4 v[kRowUnroll];
#pragma unroll
            for (int u = 0; u < kRowUnroll; ++u) {
                const int64_t n = min(n0 + u * G, N - 1);
                v[u] = __builtin_nontemporal_load(reinterpret_cast<const qfv4*>(X + n * ldx) + c);
            }
#pragma unroll
            for (int u = 0; u < kRowUnroll; ++u) {
                const int64_t n = n0 + u * G;
                if (n >= N) break;
                quv2 o;
                o.x = (unsigned)bf16_rne(v[u].x) | ((unsigned)bf16_rne(v[u].y) << 16);
                o.y = (unsigned)bf16_rne(v[u].z) | ((unsigned)bf16_rne(v[u].w) << 16);
                reinterpret_cast<quv2*>(Q + n * ldq)[c] = o;
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_col_absmax_v4(const float* X, int64_t N, int K, int64_t ldx,
                                                       unsigned* amax) {
    const int kc = K >> 2;
    const int64_t G = gridDim.x;
    for (int c = threadIdx.x; c < kc; c += blockDim.x) {
        unsigned m0 = 0u, m1 = 0u, m2 = 0u, m3 = 0u;
        for (int64_t n0 = blockIdx.x; n0 < N; n0 += kRowUnroll * G) {
            qfv4 v[kRowUnroll];
#pragma unroll
            for (int u = 0; u < kRowUnroll; ++u) {
                const int64_t n = min(n0 + u * G, N - 1);   // a repeated row changes no maximum
                v[u] = __builtin_nontemporal_load(reinterpret_cast<const qfv4*>(X + n * ldx) + c);
            }
#pragma unroll
            for (int u = 0; u < kRowUnroll; ++u) {
                m0 = max(m0, __float_as_uint(fabsf(v[u].x)));
                m1 = max(m1, __float_as_uint(fabsf(v[u].y)));
                m2 = max(m2, __float_as_uint(fabsf(v[u].z)));
                m3 = max(m3, __float_as_uint(fabsf(v[u].w)));
            }
        }
        if (m0) atomicMax(&amax[4 * c], m0);
        if (m1) atomicMax(&amax[4 * c + 1], m1);
        if (m2) atomicMax(&amax[4 * c + 2], m2);
        if (m3) atomicMax(&amax[4 * c + 3], m3);
    }
}

__global__ __launch_bounds__(256) void k_quant_fp8_v4(const float* X, int64_t N, int K, int64_t ldx,
                                                      const float* scale, uint8_t* Q, int64_t ldq) {
    const int kc = K >> 2;
    const int64_t G = gridDim.x;
    for (int c = threadIdx.x; c < kc; c += blockDim.x) {
        const qfv4 s = reinterpret_cast<const qfv4*>(scale)[c];
        for (int64_t n0 = blockIdx.x; n0 < N; n0 += kRowUnroll * G) {
            qfv4 v[kRowUnroll];
#pragma unroll
            for (int u = 0; u < kRowUnroll; ++u) {
                const int64_t n = min(n0 + u * G, N - 1);
                v[u] = __builtin_nontemporal_load(reinterpret_cast<const qfv4*>(X + n * ldx) + c);
            }
#pragma unroll
            for (int u = 0; u < kRowUnroll; ++u) {
                const int64_t n = n0 + u * G;
                if (n >= N) break;
                const unsigned o = (unsigned)e4m3_rne_sat(__fdiv_rn(v[u].x, s.x)) |
                                   ((unsigned)e4m3_rne_sat(__fdiv_rn(v[u].y, s.y)) << 8) |
                                   ((unsigned)e4m3_rne_sat(__fdiv_rn(v[u].z, s.z)) << 16) |
                                   ((unsigned)e4m3_rne_sat(__fdiv_rn(v[u].w, s.w)) << 24);
                reinterpret_cast<unsigned*>(Q + n * ldq)[c] = o;
            }
        }
    }
}

bool rows_of_chunks(const void* X, int K, int64_t ldx, const void* Q, int64_t ldq, int qalign) {
    return K % 4 == 0 && ldx % 4 == 0 && ldq % 4 == 0 && (uintptr_t)X % 16 == 0 &&
           (Q == nullptr || (uintptr_t)Q % qalign == 0);
}

dim3 row_block(int K) { return dim3((unsigned)std::min(256, std::max(64, ((K / 4 + 63) / 64) * 64))); }

unsigned row_grid(const glm_ctx* ctx, int64_t N) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(N, (int64_t)ctx->num_cu * 16));
}

glm_status check_conv(glm_ctx* ctx, const void* X, int64_t N, int32_t K, int64_t ldx,
                      const void* Q, int64_t ldq, const char* who) {
    if (!ctx) GLM_FAIL(GLM_EINVAL, "%s: ctx is NULL", who);
    if (N < 0 || K < 1 || K > GLM_K_MAX || ldx < K || ldq < K)
        GLM_FAIL(GLM_EINVAL, "%s: bad shape N=%lld K=%d ldx=%lld ld=%lld", who, (long long)N, K,
                 (long long)ldx, (long long)ldq);
    if (N > 0 && (!X || !Q)) GLM_FAIL(GLM_EINVAL, "%s: NULL buffer", who);
    return use_device(ctx);
}

unsigned grid_for(int64_t total) {
    int64_t b = (total + 255) / 256;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, 65536));
}

}  // namespace
}  // namespace glmrt

using namespace glmrt;

extern "C" {

glm_status glm_quantize_bf16(glm_ctx* ctx, const float* X, int64_t N, int32_t K, int64_t ldx,
                             uint16_t* Q, int64_t ldq, void* stream) {
    clear_error();
    glm_status st = check_conv(ctx, X, N, K, ldx, Q, ldq, "glm_quantize_bf16");
    if (st != GLM_OK || N == 0) return st;
    if (rows_of_chunks(X, K, ldx, Q, ldq, 8))
        hipLaunchKernelGGL(k_quant_bf16_v4, dim3(row_grid(ctx, N)), row_block(K), 0,
                           (hipStream_t)stream, X, N, K, ldx, Q, ldq);
    else
        hipLaunchKernelGGL(k_quant_bf16, dim3(grid_for(N * K)), dim3(256), 0, (hipStream_t)stream, X,
                           N, K, ldx, Q, ldq);
    GLM_HIP_CHECK(hipGetLastError());
    return GLM_OK;
}

glm_status glm_fp8_col_scales(glm_ctx* ctx, const float* X, int64_t N, int32_t K, int64_t ldx,
                              float* scale, void* stream) {
    clear_error();
    glm_status st = check_conv(ctx, X, N, K, ldx, scale, K, "glm_fp8_col_scales");
    if (st != GLM_OK) return st;
    if (!scale) GLM_FAIL(GLM_EINVAL, "glm_fp8_col_scales: scale is NULL");
    hipStream_t s = (hipStream_t)stream;
    // the max is accumulated in the scale buffer itself (as bits), then converted
    unsigned* amax = reinterpret_cast<unsigned*>(scale);
    hipLaunchKernelGGL(k_zero_u32, dim3((K + 255) / 256), dim3(256), 0, s, amax, K);
    if (N > 0 && rows_of_chunks(X, K, ldx, nullptr, 4, 1)) {
        const unsigned nb = (unsigned)std::max<int64_t>(1, std::min<int64_t>(N, (int64_t)ctx->num_cu * 4));
        hipLaunchKernelGGL(k_col_absmax_v4, dim3(nb), row_block(K), 0, s, X, N, K, ldx, amax);
    } else if (N > 0) {
        const unsigned nb = (unsigned)std::max<int64_t>(1, std::min<int64_t>(4096, (N + 1023) / 1024));
        hipLaunchKernelGGL(k_col_absmax, dim3(nb), dim3(std::min(256, ((K + 63) / 64) * 64)), 0, s, X,
                           N, K, ldx, amax);
    }
    hipLaunchKernelGGL(k_scales, dim3((K + 255) / 256), dim3(256), 0, s, amax, K, scale);
    GLM_HIP_CHECK(hipGetLastError());
    return GLM_OK;
}

glm_status glm_quantize_fp8(glm_ctx* ctx, const float* X, int64_t N, int32_t K, int64_t ldx,
                            const float* scale, uint8_t* Q, int64_t ldq, void* stream) {
    clear_error();
    glm_status st = check_conv(ctx, X, N, K, ldx, Q, ldq, "glm_quantize_fp8");
    if (st != GLM_OK || N == 0) return st;
    if (!scale) GLM_FAIL(GLM_EINVAL, "glm_quantize_fp8: scale is NULL");
    if (rows_of_chunks(X, K, ldx, Q, ldq, 4) && (uintptr_t)scale % 16 == 0)
        hipLaunchKernelGGL(k_quant_fp8_v4, dim3(row_grid(ctx, N)), row_block(K), 0,
                           (hipStream_t)stream, X, N, K, ldx, scale, Q, ldq);
    else
        hipLaunchKernelGGL(k_quant_fp8, dim3(grid_for(N * K)), dim3(256), 0, (hipStream_t)stream, X,
                           N, K, ldx, scale, Q, ldq);
    GLM_HIP_CHECK(hipGetLastError());
    return GLM_OK;
}

}  // extern "C"
