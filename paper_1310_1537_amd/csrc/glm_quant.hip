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
    if (N > 0) {
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
    hipLaunchKernelGGL(k_quant_fp8, dim3(grid_for(N * K)), dim3(256), 0, (hipStream_t)stream, X, N,
                       K, ldx, scale, Q, ldq);
    GLM_HIP_CHECK(hipGetLastError());
    return GLM_OK;
}

}  // extern "C"
