// Integrating factor E(alpha) (Sec. 2.3): the kernel of the discrete heat semigroup is the product
// of three 1D factors w[k] = e^{-2 alpha} I_k(2 alpha) (Appendix B, Eq. lgf_intfac), so
// M E(alpha) M is applied as three masked 1D convolutions, one per axis, each reading its input
// with zero extension outside the box.  Every pass reads and writes each element of HBM once with
// coalesced accesses: rows through LDS for x, register windows over adjacent x-columns for y and z.
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

// x pass: whole rows staged in LDS (RPW rows of length nx per workgroup), each output summing its
// 2r+1 row neighbours from LDS; global reads and writes are contiguous.
constexpr int kIfRowElems = 2048;  // LDS elements per workgroup for the row pass

template <typename T>
__global__ void __launch_bounds__(256) k_if_rows(const T* __restrict__ in, T* __restrict__ out, int nx,
                                                 long long nrows, IfWeights wts, int radius) {
    __shared__ T lds[kIfRowElems];
    const int rpw = kIfRowElems / nx;
    const long long row0 = (long long)blockIdx.x * rpw;
    const int comp = blockIdx.y;
    const long long nrow_here = min((long long)rpw, nrows - row0);
    const long long base = comp * nrows * nx + row0 * nx;
    const int cnt = (int)(nrow_here * nx);
    for (int e = threadIdx.x; e < cnt; e += blockDim.x) lds[e] = in[base + e];
    __syncthreads();
    for (int e = threadIdx.x; e < cnt; e += blockDim.x) {
        const int i = e % nx;
        const int lo = max(-radius, -i), hi = min(radius, nx - 1 - i);
        double acc = 0.0;
        for (int d = max(-lo, hi); d >= 1; --d) {
            T s = 0;
            if (-d >= lo) s += lds[e - d];
            if (d <= hi) s += lds[e + d];
            acc += wts.w[d] * (double)s;
        }
        acc += wts.w[0] * (double)lds[e];
        out[base + e] = (T)acc;
    }
}

// y or z pass: a tile of TB adjacent x-columns times the full length along the axis is staged in
// LDS; each output sums its 2r+1 neighbours along the axis.  `stride` is the element distance
// between consecutive points along the axis, `outer_stride` between the tile groups of grid y.
template <typename T, int TB>
__global__ void __launch_bounds__(256) k_if_cols(const T* __restrict__ in, T* __restrict__ out, int nx, int len,
                                                 long long stride, long long outer_stride, long long comp_stride,
                                                 IfWeights wts, int radius) {
    extern __shared__ unsigned char smem[];
    T* lds = (T*)smem;  // [len][TB]
    const int c = threadIdx.x % TB;
    const int t = threadIdx.x / TB;
    constexpr int TPC = 256 / TB;  // threads per column
    const int col = blockIdx.x * TB + c;
    const bool valid = col < nx;
    const long long base = blockIdx.z * comp_stride + (long long)blockIdx.y * outer_stride + (valid ? col : 0);
    for (int k = t; k < len; k += TPC) lds[k * TB + c] = valid ? in[base + k * stride] : (T)0;
    __syncthreads();
    if (!valid) return;
    for (int k = t; k < len; k += TPC) {
        const int lo = max(-radius, -k), hi = min(radius, len - 1 - k);
        double acc = 0.0;
        for (int d = max(-lo, hi); d >= 1; --d) {
            T s = 0;
            if (-d >= lo) s += lds[(k - d) * TB + c];
            if (d <= hi) s += lds[(k + d) * TB + c];
            acc += wts.w[d] * (double)s;
        }
        acc += wts.w[0] * (double)lds[k * TB + c];
        out[base + k * stride] = (T)acc;
    }
}

// Fixed-radius passes (radius R known at compile time).  Outputs are formed in one order on every
// axis: w[0] v[k] + sum_{d = 1..R} w[d] (v[k - d] + v[k + d]), accumulated in FP64, with v = 0
// outside the box.  Input and output must not overlap.
//
// x pass: a workgroup stages `rpb` whole rows (components are consecutive rows too) in LDS in their
// natural order with R zeros at both ends of each row; global reads and writes are contiguous and
// consecutive lanes read consecutive LDS words (no bank conflicts).
struct IfTerms {  // optional extra input terms of the x pass: v = c0 in + c1 in1 + c2 in2
    const void* in1;
    const void* in2;
    double c0, c1, c2;
};

template <typename T, int R, bool COMB>
__global__ void __launch_bounds__(256) k_if_x(const T* __restrict__ in, T* __restrict__ out, long long nrows, int len,
                                              int rpb, IfWeights wts, IfTerms terms) {
    extern __shared__ unsigned char smem[];
    T* lds = (T*)smem;  // [rpb][len + 2R]
    const int W = len + 2 * R;
    const long long row0 = (long long)blockIdx.x * rpb;
    const int nr = (int)min((long long)rpb, nrows - row0);
    const int cnt = nr * len;
    const T* src = in + row0 * len;
    T* dst = out + row0 * len;
    for (int e = threadIdx.x; e < nr * 2 * R; e += 256) {
        const int r = e / (2 * R), h = e - r * (2 * R);
        lds[r * W + (h < R ? h : len + h)] = (T)0;
    }
    if constexpr (COMB) {
        const T* s1 = (const T*)terms.in1 + row0 * len;
        const T* s2 = terms.in2 ? (const T*)terms.in2 + row0 * len : nullptr;
        for (int e = threadIdx.x; e < cnt; e += 256) {
            const int r = e / len;
            double v = terms.c0 * (double)src[e];
            v += terms.c1 * (double)s1[e];
            if (s2) v += terms.c2 * (double)s2[e];
            lds[r * W + R + (e - r * len)] = (T)v;
        }
    } else {
        for (int e = threadIdx.x; e < cnt; e += 256) {
            const int r = e / len;
            lds[r * W + R + (e - r * len)] = src[e];
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < cnt; e += 256) {
        const int r = e / len;
        const T* p = lds + r * W + R + (e - r * len);
        double acc = wts.w[0] * (double)p[0];
#pragma unroll
        for (int d = 1; d <= R; ++d) acc += wts.w[d] * (double)(p[-d] + p[d]);
        dst[e] = (T)acc;
    }
}

// y and z passes: a thread owns one x position (consecutive lanes take consecutive x, so every load
// and store of a wavefront is one contiguous row segment) and S consecutive outputs of its line; the
// S + 2R inputs go straight from memory into registers (neighbouring segments re-read their shared
// halo through the caches, not from HBM).  No LDS and no barriers.
template <typename T, int R, int S>
__global__ void __launch_bounds__(256) k_if_strided(const T* __restrict__ in, T* __restrict__ out, int nx, int len,
                                                    long long stride, int nouter, long long outer_stride,
                                                    long long comp_stride, IfWeights wts) {
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int k0 = (blockIdx.y * 4 + (threadIdx.x >> 6)) * S;
    if (x >= nx || k0 >= len) return;
    const int o = blockIdx.z % nouter, comp = blockIdx.z / nouter;
    const long long base = comp * comp_stride + (long long)o * outer_stride + x;
    T v[S + 2 * R];
#pragma unroll
    for (int j = 0; j < S + 2 * R; ++j) {
        const int k = k0 - R + j;
        v[j] = (k >= 0 && k < len) ? in[base + (long long)k * stride] : (T)0;
    }
#pragma unroll
    for (int m = 0; m < S; ++m) {
        if (k0 + m < len) {
            double acc = wts.w[0] * (double)v[m + R];
#pragma unroll
            for (int d = 1; d <= R; ++d) acc += wts.w[d] * (double)(v[m + R - d] + v[m + R + d]);
            out[base + (long long)(k0 + m) * stride] = (T)acc;
        }
    }
}

constexpr int kIfSegment = 32;  // outputs per thread of the strided passes

template <typename T, int R>
static void launch_fixed(int axis, const T* in, T* out, int ncomp, int nx, int ny, int nz, const IfWeights& wts,
                         hipStream_t s, const IfTerms* terms = nullptr) {
    const long long n = (long long)nx * ny * nz;
    if (axis == 0) {
        const long long nrows = (long long)ncomp * ny * nz;
        const int rpb = nx + 2 * R >= 2048 ? 1 : 2048 / (nx + 2 * R);  // at most 2048 LDS elements
        const size_t lds = (size_t)rpb * (nx + 2 * R) * sizeof(T);
        const dim3 grid((unsigned)ceil_div(nrows, rpb));
        if (terms)
            hipLaunchKernelGGL((k_if_x<T, R, true>), grid, dim3(256), lds, s, in, out, nrows, nx, rpb, wts, *terms);
        else
            hipLaunchKernelGGL((k_if_x<T, R, false>), grid, dim3(256), lds, s, in, out, nrows, nx, rpb, wts,
                               IfTerms{});
        return;
    }
    const int len = axis == 1 ? ny : nz;
    const long long stride = axis == 1 ? (long long)nx : (long long)nx * ny;
    const int nouter = axis == 1 ? nz : ny;
    const long long outer_stride = axis == 1 ? (long long)nx * ny : (long long)nx;
    dim3 grid(ceil_div(nx, 64), ceil_div(ceil_div(len, kIfSegment), 4), nouter * ncomp);
    hipLaunchKernelGGL((k_if_strided<T, R, kIfSegment>), grid, dim3(256), 0, s, in, out, nx, len, stride, nouter,
                       outer_stride, n, wts);
}

template <typename T>
static int if_axis_t(int axis, const void* in, void* out, int ncomp, int nx, int ny, int nz, const double* w,
                     int radius, hipStream_t s) {
    IfWeights wts;
    for (int k = 0; k <= kIfMaxRadius; ++k) wts.w[k] = k <= radius ? w[k] : 0.0;
    const long long n = (long long)nx * ny * nz;
    const T* src = (const T*)in;
    T* dst = (T*)out;
    switch (radius) {
#define NSLGF_IF_R(R_) case R_: launch_fixed<T, R_>(axis, src, dst, ncomp, nx, ny, nz, wts, s); NSLGF_LAUNCH_CHECK(); return NSLGF_OK;
        NSLGF_IF_R(1) NSLGF_IF_R(2) NSLGF_IF_R(3) NSLGF_IF_R(4) NSLGF_IF_R(5) NSLGF_IF_R(6) NSLGF_IF_R(7)
        NSLGF_IF_R(8) NSLGF_IF_R(9) NSLGF_IF_R(10) NSLGF_IF_R(11) NSLGF_IF_R(12)
#undef NSLGF_IF_R
        default: break;
    }
    // larger radii: runtime-radius passes
    if (axis == 0) {
        if (nx > kIfRowElems) {
            set_error("if_apply: rows longer than the LDS row buffer");
            return NSLGF_EUNSUPPORTED;
        }
        const long long nrows = (long long)ny * nz;
        const int rpw = kIfRowElems / nx;
        dim3 grid(ceil_div(nrows, rpw), ncomp);
        hipLaunchKernelGGL((k_if_rows<T>), grid, dim3(256), 0, s, src, dst, nx, nrows, wts, radius);
    } else {
        constexpr int TB = (int)(128 / sizeof(T));
        const int len = axis == 1 ? ny : nz;
        const long long stride = axis == 1 ? (long long)nx : (long long)nx * ny;
        const int nouter = axis == 1 ? nz : ny;
        const long long outer_stride = axis == 1 ? (long long)nx * ny : (long long)nx;
        const size_t lds = (size_t)len * TB * sizeof(T);
        dim3 grid(ceil_div(nx, TB), nouter, ncomp);
        hipLaunchKernelGGL((k_if_cols<T, TB>), grid, dim3(256), lds, s, src, dst, nx, len, stride, outer_stride, n,
                           wts, radius);
    }
    NSLGF_LAUNCH_CHECK();
    return NSLGF_OK;
}

template <typename T>
static int if_x_combined_t(const IfCombine& comb, void* out, int ncomp, int nx, int ny, int nz, const double* w,
                           int radius, hipStream_t s) {
    IfWeights wts;
    for (int k = 0; k <= kIfMaxRadius; ++k) wts.w[k] = k <= radius ? w[k] : 0.0;
    const IfTerms terms{comb.p[1], comb.p[2], comb.c[0], comb.c[1], comb.c[2]};
    const T* src = (const T*)comb.p[0];
    T* dst = (T*)out;
    switch (radius) {
#define NSLGF_IF_R(R_) case R_: launch_fixed<T, R_>(0, src, dst, ncomp, nx, ny, nz, wts, s, &terms); NSLGF_LAUNCH_CHECK(); return NSLGF_OK;
        NSLGF_IF_R(1) NSLGF_IF_R(2) NSLGF_IF_R(3) NSLGF_IF_R(4) NSLGF_IF_R(5) NSLGF_IF_R(6) NSLGF_IF_R(7)
        NSLGF_IF_R(8) NSLGF_IF_R(9) NSLGF_IF_R(10) NSLGF_IF_R(11) NSLGF_IF_R(12)
#undef NSLGF_IF_R
        default: break;
    }
    return NSLGF_EUNSUPPORTED;
}

int launch_if_x_combined(int dtype, const IfCombine& comb, void* out, int ncomp, int nx, int ny, int nz,
                         const double* w, int radius, hipStream_t s) {
    if (!comb.p[0] || !comb.p[1]) {
        set_error("if_apply: a combined input needs at least two terms");
        return NSLGF_EINVAL;
    }
    if (dtype == NSLGF_F32) return if_x_combined_t<float>(comb, out, ncomp, nx, ny, nz, w, radius, s);
    return if_x_combined_t<double>(comb, out, ncomp, nx, ny, nz, w, radius, s);
}

int launch_if_axis(int axis, int dtype, const void* in, void* out, int ncomp, int nx, int ny, int nz, const double* w,
                   int radius, hipStream_t s) {
    if (dtype == NSLGF_F32) return if_axis_t<float>(axis, in, out, ncomp, nx, ny, nz, w, radius, s);
    return if_axis_t<double>(axis, in, out, ncomp, nx, ny, nz, w, radius, s);
}

}  // namespace nslgf
