// Step guard: the FP64 divergence check of a projected velocity and the non-finite test.  In the FP32
// form the stored values are widened to FP64 before they are differenced, so the check measures what
// the FP32 projection left, not the rounding of the check itself.
#include <cmath>

#include "kernels.h"

namespace nslgf {

// Over the box: acc[0] = max (as the bit pattern of a nonnegative double, so that integer maxima order
// like the values) of |Dbar u| on the cells at least `margin` (>= 1) from every face, with
//     Dbar u (i,j,k) = (u1(i,j,k) - u1(i-1,j,k) + u2(i,j,k) - u2(i,j-1,k) + u3(i,j,k) - u3(i,j,k-1)) / dx
// (Appendix A) in FP64; acc[1] += the number of non-finite values of u (3 components) and of d (if set).
template <typename T>
__global__ void __launch_bounds__(256) k_guard(const T* __restrict__ u, const T* __restrict__ d, int nx, int ny, int nz,
                                               int margin, double idx, unsigned long long* acc) {
    const long long n = (long long)nx * ny * nz;
    const long long sxy = (long long)nx * ny;
    double m = 0.0;
    unsigned long long bad = 0;
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(p % nx);
        const int j = (int)((p / nx) % ny);
        const int k = (int)(p / sxy);
        const double a = (double)u[p], b = (double)u[n + p], c = (double)u[2 * n + p];
        bad += !isfinite(a) + !isfinite(b) + !isfinite(c);
        if (d) bad += !isfinite((double)d[p]);
        if (i >= margin && i < nx - margin && j >= margin && j < ny - margin && k >= margin && k < nz - margin) {
            const double v = ((a - (double)u[p - 1]) + (b - (double)u[n + p - nx]) + (c - (double)u[2 * n + p - sxy])) * idx;
            m = fmax(m, fabs(v));  // (a NaN operand leaves m unchanged; it is counted above)
        }
    }
    // wave reduction, then one atomic per wave
    for (int off = 32; off > 0; off >>= 1) {
        m = fmax(m, __shfl_xor(m, off));
        bad += __shfl_xor(bad, off);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicMax(&acc[0], (unsigned long long)__double_as_longlong(m));
        if (bad) atomicAdd(&acc[1], bad);
    }
}

__global__ void k_guard_reset(unsigned long long* acc) {
    if (threadIdx.x < 2) acc[threadIdx.x] = 0ull;
}

int launch_guard_reset(unsigned long long* acc, hipStream_t s) {
    if (recording_unsupported()) return NSLGF_OK;
    hipLaunchKernelGGL(k_guard_reset, dim3(1), dim3(64), 0, s, acc);
    NSLGF_LAUNCH_CHECK();
    return NSLGF_OK;
}

int launch_guard(int dtype, const void* u, const void* d, int nx, int ny, int nz, int margin, double dx,
                 unsigned long long* acc, hipStream_t s) {
    if (recording_unsupported()) return NSLGF_OK;
    const long long n = (long long)nx * ny * nz;
    const int blocks = (int)std::min<long long>(2048, (n + 255) / 256);
    if (margin < 1) margin = 1;
    if (dtype == NSLGF_F32)
        hipLaunchKernelGGL(k_guard<float>, dim3(blocks), dim3(256), 0, s, (const float*)u, (const float*)d, nx, ny, nz,
                           margin, 1.0 / dx, acc);
    else
        hipLaunchKernelGGL(k_guard<double>, dim3(blocks), dim3(256), 0, s, (const double*)u, (const double*)d, nx, ny,
                           nz, margin, 1.0 / dx, acc);
    NSLGF_LAUNCH_CHECK();
    return NSLGF_OK;
}

}  // namespace nslgf
