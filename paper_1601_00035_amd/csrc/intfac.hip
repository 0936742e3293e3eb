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
// Input modes of the fused x-y pass.
enum IfInput { IF_IN_PLAIN = 0, IF_IN_COMB = 1, IF_IN_PROJ = 2 };
struct IfTerms {
    // IF_IN_COMB: v = c0 in + c1 in1 + c2 in2
    const void* in1;
    const void* in2;
    double c0, c1, c2;
    // IF_IN_PROJ: v = in - G dhat (component a of a 3-component field: the difference of dhat along axis
    // a); wnew = (v - (c_q q + c_w1 w1)) inv where wnew is given
    const void* dhat;
    const void* q;
    const void* w1;
    void* wnew;
    double idx, c_q, c_w1, inv;
};

// Fused x and y passes (fixed radius R): a workgroup owns one (component, z) plane and S consecutive
// output rows y0 .. y0 + S - 1 (the tile height, from the rows per workgroup the launch tuner sets per
// box), one thread per x (nx <= 256).  It walks the rows from y0 - R upwards,
// RB rows per step: each thread holds the raw values of the next P steps in registers (loads issued
// P steps ahead), the step's rows go through a double-buffered LDS tile with R zeros at both ends of
// each row (one barrier per step), each x-filtered value is rounded to the dtype and pushed into a
// register window of the last 2R + RB rows, and every row whose 2R + 1 neighbours are in the window
// is y-filtered and stored.  The values are the ones the separate x and y passes produce (same order
// of operations and roundings) without the intermediate field making a round trip through HBM.
// With IF_IN_COMB the raw value is the combination c0 in + c1 in1 + c2 in2, formed in FP64 and
// rounded once; with IF_IN_PROJ it is the projection r - G dhat of the stage (in the order of
// operations of the projection kernel), and the stage's new w is written on the way (each point by
// the workgroup that owns its output row).
// Workgroups are numbered so that all row blocks of one plane run on one XCD (the hardware hands
// workgroup b to XCD b mod 8) and share their halo rows through its L2.
// Arguments of one fused x-y pass (the batched form reads one table entry per problem).
struct IfXyArgs {
    const void* in;
    void* out;
    int nx, ny, nz, ntiles, S;
    IfWeights wts;
    IfTerms terms;
};
// BATCH: per consecutive logical workgroups make up one problem, whose arguments are da[problem].
template <typename T, int R, int RB, int P, int MODE, bool BATCH>
__global__ void __launch_bounds__(256) k_if_xy(IfXyArgs a0, const IfXyArgs* __restrict__ da, int per) {
    constexpr int W = 256 + 2 * R;  // LDS row length
    constexpr int NW = 2 * R + RB;  // register window (x-filtered rows)
    __shared__ T tile_lds[2][RB][W];
    const int nb = (int)gridDim.x, b = (int)blockIdx.x, xcd = b % 8;
    int lg = xcd * (nb / 8) + min(xcd, nb % 8) + b / 8;
    int pb = 0;
    if constexpr (BATCH) {
        pb = lg / per;
        lg -= pb * per;
    }
    const IfXyArgs* A = BATCH ? da + pb : nullptr;
    const T* __restrict__ in = (const T*)(BATCH ? A->in : a0.in);
    T* __restrict__ out = (T*)(BATCH ? A->out : a0.out);
    const int nx = BATCH ? A->nx : a0.nx, ny = BATCH ? A->ny : a0.ny, nz = BATCH ? A->nz : a0.nz;
    const int ntiles = BATCH ? A->ntiles : a0.ntiles, S = BATCH ? A->S : a0.S;
    const IfTerms terms = BATCH ? A->terms : a0.terms;
    auto wd = [&](int d) -> double {
        if constexpr (BATCH) return A->wts.w[d];
        else return a0.wts.w[d];
    };
    const int NSTEP = (S + 2 * R + RB - 1) / RB;
    const int tile = lg % ntiles, plane = lg / ntiles;  // plane = comp * nz + z
    const int x = threadIdx.x;
    const bool act = x < nx;
    const long long pbase = (long long)plane * nx * ny;
    const int y0 = tile * S, ylo = y0 - R;
    if (threadIdx.x < 2 * R) {
        const int h = threadIdx.x < R ? threadIdx.x : nx + threadIdx.x;
#pragma unroll
        for (int i = 0; i < RB; ++i) {
            tile_lds[0][i][h] = (T)0;
            tile_lds[1][i][h] = (T)0;
        }
    }
    const int comp = plane / nz, zpl = plane - comp * nz;
    auto raw = [&](int y) -> T {
        if (!act || y < 0 || y >= ny) return (T)0;
        const long long e = pbase + (long long)y * nx + x;
        if constexpr (MODE == IF_IN_COMB) {
            double v = terms.c0 * (double)in[e];
            v += terms.c1 * (double)((const T*)terms.in1)[e];
            if (terms.in2) v += terms.c2 * (double)((const T*)terms.in2)[e];
            return (T)v;
        } else if constexpr (MODE == IF_IN_PROJ) {
            const T* D = (const T*)terms.dhat;
            const long long c0 = ((long long)zpl * ny + y) * nx + x;  // offset within one component
            const T d0 = D[c0];
            T d1 = (T)0;
            if (comp == 0) {
                if (x + 1 < nx) d1 = D[c0 + 1];
            } else if (comp == 1) {
                if (y + 1 < ny) d1 = D[c0 + nx];
            } else {
                if (zpl + 1 < nz) d1 = D[c0 + (long long)nx * ny];
            }
            const T v = in[e] - (d1 - d0) * (T)terms.idx;
            if (terms.wnew && y >= y0 && y < y0 + S) {
                double base = terms.c_q * (double)((const T*)terms.q)[e];
                if (terms.w1) base += terms.c_w1 * (double)((const T*)terms.w1)[e];
                ((T*)terms.wnew)[e] = (T)(((double)v - base) * terms.inv);
            }
            return v;
        } else {
            return in[e];
        }
    };
    T q[P][RB];
#pragma unroll
    for (int j = 0; j < P; ++j)
#pragma unroll
        for (int i = 0; i < RB; ++i) q[j][i] = raw(ylo + j * RB + i);
    T win[NW];
#pragma unroll
    for (int i = 0; i < NW; ++i) win[i] = (T)0;
    for (int ks = 0; ks < NSTEP; ++ks) {
        T (*lt)[W] = tile_lds[ks & 1];
        if (act) {
#pragma unroll
            for (int i = 0; i < RB; ++i) lt[i][R + x] = q[0][i];
        }
#pragma unroll
        for (int j = 0; j < P - 1; ++j)
#pragma unroll
            for (int i = 0; i < RB; ++i) q[j][i] = q[j + 1][i];
#pragma unroll
        for (int i = 0; i < RB; ++i) q[P - 1][i] = raw(ylo + (ks + P) * RB + i);
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 2 * R; ++i) win[i] = win[i + RB];
#pragma unroll
        for (int i = 0; i < RB; ++i) {
            T xf = (T)0;
            if (act) {
                const T* p = &lt[i][R + x];
                double acc = wd(0) * (double)p[0];
#pragma unroll
                for (int d = 1; d <= R; ++d) acc += wd(d) * (double)(p[-d] + p[d]);
                xf = (T)acc;
            }
            win[2 * R + i] = xf;
        }
#pragma unroll
        for (int i = 0; i < RB; ++i) {
            const int kk = ks * RB + i;  // rows ylo .. ylo + kk are in; the row y = ylo + kk - R is complete
            const int y = ylo + kk - R;
            if (kk >= 2 * R && act && y < ny && y < y0 + S) {
                const T* v = win + i;
                double acc = wd(0) * (double)v[R];
#pragma unroll
                for (int d = 1; d <= R; ++d) acc += wd(d) * (double)(v[R - d] + v[R + d]);
                out[pbase + (long long)y * nx + x] = (T)acc;
            }
        }
    }
}

// y and z passes: a thread owns one x position (consecutive lanes take consecutive x, so every load
// and store of a wavefront is one contiguous row segment) and S consecutive outputs of its line; the
// S + 2R inputs go straight from memory into registers (neighbouring segments re-read their shared
// halo through the caches, not from HBM).  No LDS and no barriers.
struct IfStrArgs {
    const void* in;
    void* out;
    int nx, len, nouter;
    long long stride, outer_stride, comp_stride;
    IfWeights wts;
};
// BATCH: per consecutive values of the grid's z index make up one problem, whose arguments are da[problem].
template <typename T, int R, int S, bool BATCH>
__global__ void __launch_bounds__(256) k_if_strided(IfStrArgs a0, const IfStrArgs* __restrict__ da, int per) {
    int bz = blockIdx.z, pb = 0;
    if constexpr (BATCH) {
        pb = bz / per;
        bz -= pb * per;
    }
    const IfStrArgs* A = BATCH ? da + pb : nullptr;
    const T* __restrict__ in = (const T*)(BATCH ? A->in : a0.in);
    T* __restrict__ out = (T*)(BATCH ? A->out : a0.out);
    const int nx = BATCH ? A->nx : a0.nx, len = BATCH ? A->len : a0.len, nouter = BATCH ? A->nouter : a0.nouter;
    const long long stride = BATCH ? A->stride : a0.stride, outer_stride = BATCH ? A->outer_stride : a0.outer_stride;
    const long long comp_stride = BATCH ? A->comp_stride : a0.comp_stride;
    auto wd = [&](int d) -> double {
        if constexpr (BATCH) return A->wts.w[d];
        else return a0.wts.w[d];
    };
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int k0 = (blockIdx.y * 4 + (threadIdx.x >> 6)) * S;
    if (x >= nx || k0 >= len) return;
    const int o = bz % nouter, comp = bz / nouter;
    const long long base = comp * comp_stride + (long long)o * outer_stride + x;
    T v[S + 2 * R];
    if (k0 >= R && k0 + S + R <= len) {  // the whole window inside the line: loads without tests
#pragma unroll
        for (int j = 0; j < S + 2 * R; ++j) v[j] = in[base + (long long)(k0 - R + j) * stride];
    } else {
#pragma unroll
        for (int j = 0; j < S + 2 * R; ++j) {
            const int k = k0 - R + j;
            v[j] = (k >= 0 && k < len) ? in[base + (long long)k * stride] : (T)0;
        }
    }
    const bool full = k0 + S <= len;
#pragma unroll
    for (int m = 0; m < S; ++m) {
        if (full || k0 + m < len) {
            double acc = wd(0) * (double)v[m + R];
#pragma unroll
            for (int d = 1; d <= R; ++d) acc += wd(d) * (double)(v[m + R - d] + v[m + R + d]);
            out[base + (long long)(k0 + m) * stride] = (T)acc;
        }
    }
}

// Outputs per thread of the strided passes: 32 by default, 16 where the launch tuner finds it faster.
constexpr int kIfRowsPerStep = 4;    // rows per barrier of the fused x-y pass
constexpr int kIfPrefetch = 2;       // steps loaded ahead by the fused x-y pass

template <typename T, int R, int S>
static int batched_strided(const void* args, int nprob, dim3 g, dim3 b, hipStream_t s) {
    hipLaunchKernelGGL((k_if_strided<T, R, S, true>), dim3(g.x, g.y, g.z * nprob), b, 0, s, IfStrArgs{},
                       (const IfStrArgs*)args, (int)g.z);
    NSLGF_LAUNCH_CHECK();
    return NSLGF_OK;
}
template <typename T, int R, int MODE>
static int batched_xy(const void* args, int nprob, dim3 g, dim3 b, hipStream_t s) {
    hipLaunchKernelGGL((k_if_xy<T, R, kIfRowsPerStep, kIfPrefetch, MODE, true>), dim3(g.x * nprob), b, 0, s,
                       IfXyArgs{}, (const IfXyArgs*)args, (int)g.x);
    NSLGF_LAUNCH_CHECK();
    return NSLGF_OK;
}

template <typename T, int R, int S> static void issue_strided(const IfStrArgs& a, dim3 grid, hipStream_t s) {
    if (launch_recorder()) {
        record_launch(&batched_strided<T, R, S>, grid, dim3(256), a);
        return;
    }
    hipLaunchKernelGGL((k_if_strided<T, R, S, false>), grid, dim3(256), 0, s, a, nullptr, 0);
}

template <typename T, int R>
static void launch_fixed(int axis, const T* in, T* out, int ncomp, int nx, int ny, int nz, const IfWeights& wts,
                         hipStream_t s, int seg) {
    const long long n = (long long)nx * ny * nz;
    const int len = axis == 1 ? ny : nz;
    const long long stride = axis == 1 ? (long long)nx : (long long)nx * ny;
    const int nouter = axis == 1 ? nz : ny;
    const long long outer_stride = axis == 1 ? (long long)nx * ny : (long long)nx;
    const IfStrArgs a{in, out, nx, len, nouter, stride, outer_stride, n, wts};
    if (seg == 16)
        issue_strided<T, R, 16>(a, dim3(ceil_div(nx, 64), ceil_div(ceil_div(len, 16), 4), nouter * ncomp), s);
    else
        issue_strided<T, R, 32>(a, dim3(ceil_div(nx, 64), ceil_div(ceil_div(len, 32), 4), nouter * ncomp), s);
}

template <typename T, int R, int MODE>
static void issue_xy(const IfXyArgs& a, dim3 grid, dim3 block, hipStream_t s) {
    if (launch_recorder()) {
        record_launch(&batched_xy<T, R, MODE>, grid, block, a);
        return;
    }
    hipLaunchKernelGGL((k_if_xy<T, R, kIfRowsPerStep, kIfPrefetch, MODE, false>), grid, block, 0, s, a, nullptr, 0);
}

// rows: at most this many output rows per workgroup; the ny rows of a plane are split into
// ntiles = ceil(ny / rows) tiles of height ceil(ny / ntiles) (the last at most ntiles - 1 rows shorter,
// never empty), so that no workgroup walks far past the plane's end or carries a long tail alone (halo
// rows re-read: 2R / height).  A workgroup has one thread per x rounded up to whole wavefronts.
template <typename T, int R>
static void launch_xy(const IfCombine& cb, T* out, int ncomp, int nx, int ny, int nz, const IfWeights& wts,
                      hipStream_t s, int rows) {
    const int ntiles = ceil_div(ny, rows);
    const int height = ceil_div(ny, ntiles);
    const dim3 grid((unsigned)((long long)ntiles * nz * ncomp)), block((unsigned)(ceil_div(nx, 64) * 64));
    IfXyArgs a{cb.p[0], out, nx, ny, nz, ntiles, height, wts, IfTerms{}};
    IfTerms& terms = a.terms;
    if (cb.proj) {
        const IfProject& pj = *cb.proj;
        terms.dhat = pj.dhat;
        terms.q = pj.q;
        terms.w1 = pj.w1;
        terms.wnew = pj.wnew;
        terms.idx = pj.idx;
        terms.c_q = pj.c_q;
        terms.c_w1 = pj.c_w1;
        terms.inv = pj.inv;
        issue_xy<T, R, IF_IN_PROJ>(a, grid, block, s);
    } else if (cb.p[1]) {
        terms.in1 = cb.p[1];
        terms.in2 = cb.p[2];
        terms.c0 = cb.c[0];
        terms.c1 = cb.c[1];
        terms.c2 = cb.c[2];
        issue_xy<T, R, IF_IN_COMB>(a, grid, block, s);
    } else {
        issue_xy<T, R, IF_IN_PLAIN>(a, grid, block, s);
    }
}

template <typename T>
static int if_axis_t(int axis, const void* in, void* out, int ncomp, int nx, int ny, int nz, const double* w,
                     int radius, hipStream_t s, int seg) {
    IfWeights wts;
    for (int k = 0; k <= kIfMaxRadius; ++k) wts.w[k] = k <= radius ? w[k] : 0.0;
    const long long n = (long long)nx * ny * nz;
    const T* src = (const T*)in;
    T* dst = (T*)out;
    if (axis != 0) {
        switch (radius) {
#define NSLGF_IF_R(R_) case R_: launch_fixed<T, R_>(axis, src, dst, ncomp, nx, ny, nz, wts, s, seg); NSLGF_LAUNCH_CHECK(); return NSLGF_OK;
            NSLGF_IF_R(1) NSLGF_IF_R(2) NSLGF_IF_R(3) NSLGF_IF_R(4) NSLGF_IF_R(5) NSLGF_IF_R(6) NSLGF_IF_R(7)
            NSLGF_IF_R(8) NSLGF_IF_R(9) NSLGF_IF_R(10) NSLGF_IF_R(11) NSLGF_IF_R(12)
#undef NSLGF_IF_R
            default: break;
        }
    }
    // runtime-radius passes (every radius on x; radii above the fixed ones on y and z); no batched form
    if (recording_unsupported()) return NSLGF_OK;
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
static int if_xy_t(const IfCombine& cb, void* out, int ncomp, int nx, int ny, int nz, const double* w, int radius,
                   hipStream_t s, int rows) {
    IfWeights wts;
    for (int k = 0; k <= kIfMaxRadius; ++k) wts.w[k] = k <= radius ? w[k] : 0.0;
    T* dst = (T*)out;
    switch (radius) {
#define NSLGF_IF_R(R_) case R_: launch_xy<T, R_>(cb, dst, ncomp, nx, ny, nz, wts, s, rows); NSLGF_LAUNCH_CHECK(); return NSLGF_OK;
        NSLGF_IF_R(1) NSLGF_IF_R(2) NSLGF_IF_R(3) NSLGF_IF_R(4) NSLGF_IF_R(5) NSLGF_IF_R(6) NSLGF_IF_R(7)
        NSLGF_IF_R(8) NSLGF_IF_R(9) NSLGF_IF_R(10) NSLGF_IF_R(11) NSLGF_IF_R(12)
#undef NSLGF_IF_R
        default: break;
    }
    set_error("if_apply: no fused x-y pass for this radius");
    return NSLGF_EUNSUPPORTED;
}

int launch_if_xy(int dtype, const IfCombine& cb, void* out, int ncomp, int nx, int ny, int nz, const double* w,
                 int radius, hipStream_t s, int rows) {
    if (!cb.p[0] || (cb.p[2] && !cb.p[1]) || (cb.proj && (cb.p[1] || ncomp != 3 || !cb.proj->dhat ||
                                                          (cb.proj->wnew && !cb.proj->q)))) {
        set_error("if_apply: bad input combination");
        return NSLGF_EINVAL;
    }
    if (nx > 256) {
        set_error("if_apply: the fused x-y pass needs nx <= 256");
        return NSLGF_EUNSUPPORTED;
    }
    if (rows != 32 && rows != 64 && rows != 128 && rows != 256) {
        set_error("if_apply: the fused x-y pass takes 32, 64, 128 or 256 rows per workgroup");
        return NSLGF_EINVAL;
    }
    if (dtype == NSLGF_F32) return if_xy_t<float>(cb, out, ncomp, nx, ny, nz, w, radius, s, rows);
    return if_xy_t<double>(cb, out, ncomp, nx, ny, nz, w, radius, s, rows);
}

int launch_if_axis(int axis, int dtype, const void* in, void* out, int ncomp, int nx, int ny, int nz, const double* w,
                   int radius, hipStream_t s, int seg) {
    if (seg != 16 && seg != 32) {
        set_error("if_apply: the strided pass takes 16 or 32 outputs per thread");
        return NSLGF_EINVAL;
    }
    if (dtype == NSLGF_F32) return if_axis_t<float>(axis, in, out, ncomp, nx, ny, nz, w, radius, s, seg);
    return if_axis_t<double>(axis, in, out, ncomp, nx, ny, nz, w, radius, s, seg);
}

}  // namespace nslgf
