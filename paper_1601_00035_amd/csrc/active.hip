// Sub-box transfers of the active-box driver (the grid update of Sec. 5): fields move between boxes of
// whole blocks by plain copies, and the cells a new box has beyond the old one start at zero.
#include <algorithm>

#include "kernels.h"

namespace nslgf {

// dst[c][dz + k][dy + j][dx + i] = src[c][sz + k][sy + j][sx + i] for (i, j, k) < (ex, ey, ez), c < ncomp;
// one thread per x, consecutive lanes on consecutive x (contiguous row segments on both sides).
template <typename T>
__global__ void __launch_bounds__(256) k_copy_box(const T* __restrict__ src, int snx, int sny, int snz, int sx, int sy,
                                                  int sz, T* __restrict__ dst, int dnx, int dny, int dnz, int dx, int dy,
                                                  int dz, int ex, int ey, int ez) {
    const int i = blockIdx.x * 64 + threadIdx.x;
    const int j = blockIdx.y * 4 + threadIdx.y;
    const int k = blockIdx.z % ez, c = blockIdx.z / ez;
    if (i >= ex || j >= ey) return;
    const long long s = (long long)c * snx * sny * snz + ((long long)(sz + k) * sny + (sy + j)) * snx + (sx + i);
    const long long d = (long long)c * dnx * dny * dnz + ((long long)(dz + k) * dny + (dy + j)) * dnx + (dx + i);
    dst[d] = src[s];
}

template <typename T>
__global__ void __launch_bounds__(256) k_zero(T* __restrict__ dst, long long n) {
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (long long)gridDim.x * blockDim.x)
        dst[p] = (T)0;
}

int launch_zero(int dtype, void* dst, long long n, hipStream_t s) {
    if (recording_unsupported()) return NSLGF_OK;
    if (n <= 0) return NSLGF_OK;
    const int blocks = (int)std::min<long long>(4096, (n + 255) / 256);
    if (dtype == NSLGF_F32)
        hipLaunchKernelGGL(k_zero<float>, dim3(blocks), dim3(256), 0, s, (float*)dst, n);
    else
        hipLaunchKernelGGL(k_zero<double>, dim3(blocks), dim3(256), 0, s, (double*)dst, n);
    NSLGF_LAUNCH_CHECK();
    return NSLGF_OK;
}

int launch_copy_box(int dtype, const void* src, const int sdim[3], const int soff[3], void* dst, const int ddim[3],
                    const int doff[3], const int ext[3], int ncomp, hipStream_t s) {
    if (recording_unsupported()) return NSLGF_OK;
    for (int a = 0; a < 3; ++a) {
        if (ext[a] <= 0) return NSLGF_OK;
        if (soff[a] < 0 || doff[a] < 0 || soff[a] + ext[a] > sdim[a] || doff[a] + ext[a] > ddim[a]) {
            set_error("copy_box: the extent leaves a box");
            return NSLGF_EINVAL;
        }
    }
    const dim3 grid(ceil_div(ext[0], 64), ceil_div(ext[1], 4), ext[2] * ncomp);
    if (dtype == NSLGF_F32)
        hipLaunchKernelGGL(k_copy_box<float>, grid, dim3(64, 4), 0, s, (const float*)src, sdim[0], sdim[1], sdim[2],
                           soff[0], soff[1], soff[2], (float*)dst, ddim[0], ddim[1], ddim[2], doff[0], doff[1], doff[2],
                           ext[0], ext[1], ext[2]);
    else
        hipLaunchKernelGGL(k_copy_box<double>, grid, dim3(64, 4), 0, s, (const double*)src, sdim[0], sdim[1], sdim[2],
                           soff[0], soff[1], soff[2], (double*)dst, ddim[0], ddim[1], ddim[2], doff[0], doff[1],
                           doff[2], ext[0], ext[1], ext[2]);
    NSLGF_LAUNCH_CHECK();
    return NSLGF_OK;
}

}  // namespace nslgf
