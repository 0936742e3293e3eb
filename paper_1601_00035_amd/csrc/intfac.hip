// Integrating factor E(alpha) (Sec. 2.3): the kernel of the discrete heat semigroup is the product
// of three 1D factors w[k] = e^{-2 alpha} I_k(2 alpha) (Appendix B, Eq. lgf_intfac), so
// M E(alpha) M is applied as three masked 1D convolutions, one per axis, each reading its input
// with zero extension outside the box.
#include <cmath>

#include "kernels.h"

namespace nslgf {

int if_weights(double alpha, int dtype, double* w, int wmax) {
    if (!(alpha >= 0.0) || !std::isfinite(alpha)) {
        set_error("if_apply: alpha must be a finite value >= 0");
        return -1;
    }
    if (alpha == 0.0) {
        w[0] = 1.0;
        return 0;
    }
    // I_k(2a) = sum_j a^{2j+k} / (j! (j+k)!), all terms positive; scaled by e^{-2a}
    const int kmax = 200;
    double vals[kmax + 1];
    const double ea = exp(-2.0 * alpha);
    double lead = 1.0;  // a^k / k!
    for (int k = 0; k <= kmax; ++k) {
        if (k > 0) lead *= alpha / k;
        double term = lead, sum = lead;
        for (int j = 1; j < 400; ++j) {
            term *= alpha * alpha / ((double)j * (double)(j + k));
            sum += term;
            if (term < 1e-19 * sum) break;
        }
        vals[k] = ea * sum;
    }
    // smallest radius whose two-sided tail is below a quarter of the dtype's unit roundoff times w[0]
    const double tol = (dtype == NSLGF_F32 ? 5.960464477539063e-08 : 1.1102230246251565e-16) * 0.25 * vals[0];
    double tail = 0.0;
    int r = kmax;
    for (int k = kmax; k >= 1; --k) {
        if (2.0 * (tail + vals[k]) > tol) {
            r = k;
            break;
        }
        tail += vals[k];
    }
    if (r > wmax || r >= kmax) {
        set_error("if_apply: alpha too large for the supported kernel radius");
        return -1;
    }
    for (int k = 0; k <= r; ++k) w[k] = vals[k];
    return r;
}

struct IfWeights {
    double w[kIfMaxRadius + 1];
};

// One masked 1D convolution along `axis` (0 = x, 1 = y, 2 = z); one thread per output element.
template <typename T, int AXIS>
__global__ void __launch_bounds__(256) k_if_axis(const T* __restrict__ in, T* __restrict__ out, int nx, int ny, int nz,
                                                 IfWeights wts, int radius) {
    const long long n = (long long)nx * ny * nz;
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n) return;
    const int comp = blockIdx.y;
    in += comp * n;
    out += comp * n;
    const int i = (int)(idx % nx);
    const int j = (int)((idx / nx) % ny);
    const int k = (int)(idx / ((long long)nx * ny));
    const int pos = AXIS == 0 ? i : (AXIS == 1 ? j : k);
    const int len = AXIS == 0 ? nx : (AXIS == 1 ? ny : nz);
    const long long stride = AXIS == 0 ? 1 : (AXIS == 1 ? (long long)nx : (long long)nx * ny);
    const int lo = max(-radius, -pos), hi = min(radius, len - 1 - pos);
    // sum from the outer offsets inwards (smallest weights first)
    double acc = 0.0;
    for (int d = max(-lo, hi); d >= 1; --d) {
        T s = 0;
        if (-d >= lo) s += in[idx - d * stride];
        if (d <= hi) s += in[idx + d * stride];
        acc += wts.w[d] * (double)s;
    }
    acc += wts.w[0] * (double)in[idx];
    out[idx] = (T)acc;
}

template <typename T>
static int if_axis_t(int axis, const void* in, void* out, int ncomp, int nx, int ny, int nz, const double* w,
                     int radius, hipStream_t s) {
    IfWeights wts;
    for (int k = 0; k <= kIfMaxRadius; ++k) wts.w[k] = k <= radius ? w[k] : 0.0;
    const long long n = (long long)nx * ny * nz;
    dim3 grid(ceil_div(n, 256), ncomp);
    if (axis == 0)
        hipLaunchKernelGGL((k_if_axis<T, 0>), grid, dim3(256), 0, s, (const T*)in, (T*)out, nx, ny, nz, wts, radius);
    else if (axis == 1)
        hipLaunchKernelGGL((k_if_axis<T, 1>), grid, dim3(256), 0, s, (const T*)in, (T*)out, nx, ny, nz, wts, radius);
    else
        hipLaunchKernelGGL((k_if_axis<T, 2>), grid, dim3(256), 0, s, (const T*)in, (T*)out, nx, ny, nz, wts, radius);
    NSLGF_LAUNCH_CHECK();
    return NSLGF_OK;
}

int launch_if_axis(int axis, int dtype, const void* in, void* out, int ncomp, int nx, int ny, int nz, const double* w,
                   int radius, hipStream_t s) {
    if (dtype == NSLGF_F32) return if_axis_t<float>(axis, in, out, ncomp, nx, ny, nz, w, radius, s);
    return if_axis_t<double>(axis, in, out, ncomp, nx, ny, nz, w, radius, s);
}

}  // namespace nslgf
