// One stored element of X as a double, for the kernels that read X an
// element at a time (column streams, tile staging): FP64 and FP32 as they are,
// BF16 as the upper half of a binary32, FP8 E4M3FN through gfx950's native
// conversion times its column scale (exact in FP64).
#pragma once

#include <hip/hip_runtime.h>

#include "glm.h"

namespace glmk {

template <int DT> struct Elem;
template <> struct Elem<GLM_F64> {
    using T = double;
    static __device__ __forceinline__ double value(T v, float) { return v; }
};
template <> struct Elem<GLM_F32> {
    using T = float;
    static __device__ __forceinline__ double value(T v, float) { return (double)v; }
};
template <> struct Elem<GLM_BF16> {
    using T = unsigned short;
    static __device__ __forceinline__ double value(T v, float) {
        return (double)__uint_as_float((unsigned)v << 16);
    }
};
template <> struct Elem<GLM_FP8_E4M3> {
    using T = unsigned char;
    static __device__ __forceinline__ double value(T v, float s) {
        const float x = __builtin_amdgcn_cvt_pk_f32_fp8((int)v, false)[0];
        return (double)x * (double)s;
    }
};

}  // namespace glmk
