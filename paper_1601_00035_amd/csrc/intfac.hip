// Integrating factor E(alpha) (Sec. 2.3): the kernel of the discrete heat semigroup is the product
// of three 1D factors w[k] = e^{-2 alpha} I_k(2 alpha) (Appendix B, Eq. lgf_intfac), so
// M E(alpha) M is applied as three masked 1D convolutions, one per axis, each reading its input
// with zero extension outside the box.  Each pass stages whole lines in LDS so that every element
// is read from and written to HBM once, with coalesced accesses (rows for x, tiles of adjacent
// x-columns for y and z).
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

// Fixed-radius variant for every axis: a workgroup owns TB lines (adjacent x-columns for the y and
// z passes, rows for the x pass), staged in LDS as [position][line] with R zeros at both ends, so
// that consecutive lanes touch consecutive lines (no bank conflicts) while each line's global
// accesses stay contiguous across its threads.  Each thread then loads a window of S + 2R values of
// its line into registers and produces S consecutive outputs with no bounds tests.
// Line l of grid column group starts at comp * comp_stride + outer * outer_stride + l * line_stride
// and its points are `stride` apart.
template <typename T, int TB, int R, int S, bool CONTIG>
__global__ void __launch_bounds__(256) k_if_lines(const T* __restrict__ in, T* __restrict__ out, int nlines, int len,
                                                  long long stride, long long line_stride, long long outer_stride,
                                                  long long comp_stride, IfWeights wts) {
    extern __shared__ unsigned char smem[];
    T* lds = (T*)smem;  // [TPC * S + 2R][TB]
    constexpr int TPC = 256 / TB;
    constexpr int ROWS = TPC * S + 2 * R;
    const int c = threadIdx.x % TB;
    const int t = threadIdx.x / TB;
    const int line = blockIdx.x * TB + c;
    const bool valid = line < nlines;
    const long long base =
        blockIdx.z * comp_stride + (long long)blockIdx.y * outer_stride + (valid ? (long long)line * line_stride : 0);
    if (CONTIG) {
        // lines are contiguous rows: global accesses run along the row (coalesced), LDS keeps [k][c]
        for (int k = t; k < ROWS; k += TPC) lds[k * TB + c] = (T)0;
        __syncthreads();
        const long long base0 = blockIdx.z * comp_stride + (long long)blockIdx.y * outer_stride;
        for (int e = threadIdx.x; e < TB * len; e += 256) {
            const int cc = e / len, kk = e - cc * len;
            const int ln = blockIdx.x * TB + cc;
            if (ln < nlines) lds[(kk + R) * TB + cc] = in[base0 + (long long)ln * line_stride + kk];
        }
    } else {
        for (int k = t; k < ROWS; k += TPC) {
            const int kk = k - R;
            lds[k * TB + c] = (valid && kk >= 0 && kk < len) ? in[base + kk * stride] : (T)0;
        }
    }
    __syncthreads();
    const bool active = valid && t * S < len;
    T v[S + 2 * R];
    T res[S];
    if (active) {
#pragma unroll
        for (int j = 0; j < S + 2 * R; ++j) v[j] = lds[(t * S + j) * TB + c];
#pragma unroll
        for (int m = 0; m < S; ++m) {
            double acc = wts.w[0] * (double)v[m + R];
#pragma unroll
            for (int d = 1; d <= R; ++d) acc += wts.w[d] * (double)(v[m + R - d] + v[m + R + d]);
            res[m] = (T)acc;
        }
    }
    if (CONTIG) {
        __syncthreads();  // every window has been read: reuse the buffer for the outputs
        if (active) {
#pragma unroll
            for (int m = 0; m < S; ++m) lds[(t * S + m) * TB + c] = res[m];
        }
        __syncthreads();
        const long long base0 = blockIdx.z * comp_stride + (long long)blockIdx.y * outer_stride;
        for (int e = threadIdx.x; e < TB * len; e += 256) {
            const int cc = e / len, kk = e - cc * len;
            const int ln = blockIdx.x * TB + cc;
            if (ln < nlines) out[base0 + (long long)ln * line_stride + kk] = lds[kk * TB + cc];
        }
    } else if (active) {
#pragma unroll
        for (int m = 0; m < S; ++m) {
            const int k = t * S + m;
            if (k < len) out[base + k * stride] = res[m];
        }
    }
}

template <typename T, int R>
static void launch_fixed(int axis, const T* in, T* out, int ncomp, int nx, int ny, int nz, const IfWeights& wts,
                         hipStream_t s) {
    const long long n = (long long)nx * ny * nz;
    constexpr int TB = (int)(128 / sizeof(T));
    constexpr int TPC = 256 / TB;
    constexpr int S = 256 / TPC;  // the longest line (256 points) split over the threads of a line
    const size_t lds = (size_t)(TPC * S + 2 * R) * TB * sizeof(T);
    int nlines, len, nouter;
    long long stride, line_stride, outer_stride;
    if (axis == 0) {  // rows: lines are (y, z) rows of nx points
        nlines = ny * nz;
        len = nx;
        stride = 1;
        line_stride = nx;
        nouter = 1;
        outer_stride = 0;
    } else if (axis == 1) {  // lines along y: x-columns of each z-plane
        nlines = nx;
        len = ny;
        stride = nx;
        line_stride = 1;
        nouter = nz;
        outer_stride = (long long)nx * ny;
    } else {  // lines along z: x-columns of each y-row
        nlines = nx;
        len = nz;
        stride = (long long)nx * ny;
        line_stride = 1;
        nouter = ny;
        outer_stride = nx;
    }
    dim3 grid(ceil_div(nlines, TB), nouter, ncomp);
    if (axis == 0)
        hipLaunchKernelGGL((k_if_lines<T, TB, R, S, true>), grid, dim3(256), lds, s, in, out, nlines, len, stride,
                           line_stride, outer_stride, n, wts);
    else
        hipLaunchKernelGGL((k_if_lines<T, TB, R, S, false>), grid, dim3(256), lds, s, in, out, nlines, len, stride,
                           line_stride, outer_stride, n, wts);
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

int launch_if_axis(int axis, int dtype, const void* in, void* out, int ncomp, int nx, int ny, int nz, const double* w,
                   int radius, hipStream_t s) {
    if (dtype == NSLGF_F32) return if_axis_t<float>(axis, in, out, ncomp, nx, ny, nz, w, radius, s);
    return if_axis_t<double>(axis, in, out, ncomp, nx, ny, nz, w, radius, s);
}

}  // namespace nslgf
