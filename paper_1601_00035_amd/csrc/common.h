// Internal helpers shared by the HIP sources of the library: status handling, complex arithmetic,
// dtype traits.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/nslgf.h"

namespace nslgf {

void set_error(const std::string& msg);

struct Status {
    int code = NSLGF_OK;
};

#define NSLGF_HIP_CHECK(expr)                                                                      \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess) {                                                                    \
            ::nslgf::set_error(std::string(#expr) + ": " + hipGetErrorString(e_));                 \
            return NSLGF_EHIP;                                                                     \
        }                                                                                          \
    } while (0)

#define NSLGF_CHECK_ARG(cond, msg)                                                                 \
    do {                                                                                           \
        if (!(cond)) {                                                                             \
            ::nslgf::set_error(msg);                                                               \
            return NSLGF_EINVAL;                                                                   \
        }                                                                                          \
    } while (0)

#define NSLGF_TRY(expr)                                                                            \
    do {                                                                                           \
        int rc_ = (expr);                                                                          \
        if (rc_ != NSLGF_OK) return rc_;                                                           \
    } while (0)

// Launch-error check after a kernel launch.
#define NSLGF_LAUNCH_CHECK() NSLGF_HIP_CHECK(hipGetLastError())

template <typename T> struct Vec2;
template <> struct Vec2<double> { using type = double2; };
template <> struct Vec2<float> { using type = float2; };
template <typename T> using cplx = typename Vec2<T>::type;

template <typename T>
__host__ __device__ __forceinline__ cplx<T> mk(T re, T im) {
    cplx<T> r;
    r.x = re;
    r.y = im;
    return r;
}
template <typename T>
__device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) { return mk<T>(a.x + b.x, a.y + b.y); }
template <typename T>
__device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) { return mk<T>(a.x - b.x, a.y - b.y); }
template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
    return mk<T>(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
template <typename T>
__device__ __forceinline__ cplx<T> cmulc(cplx<T> a, cplx<T> b) {  // a * conj(b)
    return mk<T>(fma(a.x, b.x, a.y * b.y), fma(a.y, b.x, -a.x * b.y));
}
template <typename T>
__device__ __forceinline__ cplx<T> cscale(cplx<T> a, T s) { return mk<T>(a.x * s, a.y * s); }
template <typename T>
__device__ __forceinline__ cplx<T> cconj(cplx<T> a) { return mk<T>(a.x, -a.y); }
// i * a and -i * a
template <typename T>
__device__ __forceinline__ cplx<T> cmul_i(cplx<T> a) { return mk<T>(-a.y, a.x); }
template <typename T>
__device__ __forceinline__ cplx<T> cmul_mi(cplx<T> a) { return mk<T>(a.y, -a.x); }

inline size_t dtype_size(int dtype) { return dtype == NSLGF_F32 ? 4 : 8; }

inline int ceil_div(long long a, long long b) { return (int)((a + b - 1) / b); }

}  // namespace nslgf
