// Staggered-grid point operators of Appendix A on one box, and the fused IF-HERK stage kernels.
//
// Every input is read with zero extension outside the box and every output is produced on the box
// only (the mask operators of Sec. 4.1).  Components (2) and (3) of each printed operator follow from
// component (1) by the cyclic permutation (component, axis): 1 -> 2 -> 3 -> 1 with x -> y -> z -> x.
#include <cmath>

#include "kernels.h"

namespace nslgf {

// Boxes have at most 256 points per axis, so a point's offset within one component fits 32 bits.
template <typename T> struct Fld {
    const T* p;
    int nx, ny, nz;
    __device__ __forceinline__ T operator()(int i, int j, int k) const {
        return (i >= 0 && i < nx && j >= 0 && j < ny && k >= 0 && k < nz) ? p[(k * ny + j) * nx + i] : (T)0;
    }
};

// The same field read without bounds tests, for points whose neighbours are all inside the box (the
// tests would otherwise turn every load into a branch).
template <typename T> struct FldIn {
    const T* p;
    int nx, ny, nz;
    __device__ __forceinline__ T operator()(int i, int j, int k) const { return p[(k * ny + j) * nx + i]; }
};

template <typename T> struct Vec3 {
    Fld<T> c[3];
};
template <typename T> struct Vec3In {
    FldIn<T> c[3];
};
template <typename T> __device__ __forceinline__ Vec3In<T> unchecked(const Vec3<T>& v) {
    Vec3In<T> r;
    for (int q = 0; q < 3; ++q) r.c[q] = FldIn<T>{v.c[q].p, v.c[q].nx, v.c[q].ny, v.c[q].nz};
    return r;
}

template <typename T>
__device__ __forceinline__ Vec3<T> vec3(const T* p, int nx, int ny, int nz) {
    const long long n = (long long)nx * ny * nz;
    Vec3<T> v;
    for (int q = 0; q < 3; ++q) v.c[q] = Fld<T>{p + q * n, nx, ny, nz};
    return v;
}

// e = C f at edge (i, j, k), component q (0-based); the curl of the zero-extended face field, so
// it is also defined one layer outside the box.
template <typename T>
__device__ __forceinline__ T curl_at(const Vec3<T>& f, int q, int i, int j, int k, T idx) {
    if (q == 0) return (f.c[1](i, j, k) - f.c[1](i, j, k + 1) + f.c[2](i, j + 1, k) - f.c[2](i, j, k)) * idx;
    if (q == 1) return (f.c[2](i, j, k) - f.c[2](i + 1, j, k) + f.c[0](i, j, k + 1) - f.c[0](i, j, k)) * idx;
    return (f.c[0](i, j, k) - f.c[0](i, j + 1, k) + f.c[1](i + 1, j, k) - f.c[1](i, j, k)) * idx;
}

// Ntilde(f) at face (i, j, k), all three components (Eq. opr_def_nonlin and its cyclic images).
// The nine edge values of e = C f it needs (e1, e2, e3 at the cell and one step back along the
// other axes) use 24 distinct face values, each loaded once: component (1) at offsets
// (0,0,0), (0,0,+-1), (0,+-1,0), (-1,0,0), (-1,+1,0), (-1,0,+1) and the cyclic images for (2), (3).
template <typename T, class V>
__device__ __forceinline__ void nonlinear_at(const V& f, int i, int j, int k, T idx, T out[3]) {
    const auto& F1 = f.c[0];
    const auto& F2 = f.c[1];
    const auto& F3 = f.c[2];
    const T a000 = F1(i, j, k), a00p = F1(i, j, k + 1), a00m = F1(i, j, k - 1), a0p0 = F1(i, j + 1, k),
            a0m0 = F1(i, j - 1, k), am00 = F1(i - 1, j, k), amp0 = F1(i - 1, j + 1, k), am0p = F1(i - 1, j, k + 1);
    const T b000 = F2(i, j, k), bp00 = F2(i + 1, j, k), bm00 = F2(i - 1, j, k), b00p = F2(i, j, k + 1),
            b00m = F2(i, j, k - 1), b0m0 = F2(i, j - 1, k), bpm0 = F2(i + 1, j - 1, k), b0mp = F2(i, j - 1, k + 1);
    const T c000 = F3(i, j, k), cp00 = F3(i + 1, j, k), cm00 = F3(i - 1, j, k), c0p0 = F3(i, j + 1, k),
            c0m0 = F3(i, j - 1, k), c00m = F3(i, j, k - 1), cp0m = F3(i + 1, j, k - 1), c0pm = F3(i, j + 1, k - 1);
    // edge values: e1 at (i,j,k), (i,j,k-1), (i,j-1,k); e2 at (i,j,k), (i,j,k-1), (i-1,j,k);
    // e3 at (i,j,k), (i,j-1,k), (i-1,j,k)
    const T e1_0 = (b000 - b00p + c0p0 - c000) * idx;
    const T e1_km = (b00m - b000 + c0pm - c00m) * idx;
    const T e1_jm = (b0m0 - b0mp + c000 - c0m0) * idx;
    const T e2_0 = (c000 - cp00 + a00p - a000) * idx;
    const T e2_km = (c00m - cp0m + a000 - a00m) * idx;
    const T e2_im = (cm00 - c000 + am0p - am00) * idx;
    const T e3_0 = (a000 - a0p0 + bp00 - b000) * idx;
    const T e3_jm = (a0m0 - a000 + bpm0 - b0m0) * idx;
    const T e3_im = (am00 - amp0 + b000 - bm00) * idx;
    out[0] = (T)0.25 * (e2_0 * (c000 + cp00) + e2_km * (c00m + cp0m) - e3_0 * (b000 + bp00) - e3_jm * (b0m0 + bpm0));
    out[1] = (T)0.25 * (e3_0 * (a000 + a0p0) + e3_im * (am00 + amp0) - e1_0 * (c000 + c0p0) - e1_km * (c00m + c0pm));
    out[2] = (T)0.25 * (e1_0 * (b000 + b00p) + e1_jm * (b0m0 + b0mp) - e2_0 * (a000 + a00p) - e2_im * (am00 + am0p));
}

// Point kernels run on 256-thread blocks tiling (x, y) (64 x 4 by default; the launch tuner may
// pick another of kCellShape), one z plane per grid z (no integer division); launch with cell_grid /
// cell_block.  (Renumbering the blocks so that each XCD works through a contiguous range of planes
// was measured slower for the stage kernels.)
#define NSLGF_CELL_INDEX_Z(KZ)                                                                     \
    const long long n = (long long)nx * ny * nz;                                                   \
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);                                    \
    const int j = (int)(blockIdx.y * blockDim.y + threadIdx.y);                                    \
    const int kz_ = (KZ);                                                                          \
    const int k = kz_ % nz;                                                                        \
    if (i >= nx || j >= ny) return;                                                                \
    const long long idx = (long long)((k * ny + j) * nx + i);
#define NSLGF_CELL_INDEX                                                                           \
    const long long n = (long long)nx * ny * nz;                                                   \
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);                                    \
    const int j = (int)(blockIdx.y * blockDim.y + threadIdx.y);                                    \
    const int kz_ = (int)blockIdx.z;                                                               \
    const int k = kz_ % nz;                                                                        \
    if (i >= nx || j >= ny) return;                                                                \
    const long long idx = (long long)((k * ny + j) * nx + i);

static const int kCellShape[kCellShapeCount][2] = {{64, 4}, {128, 2}, {32, 8}, {256, 1}};
static dim3 cell_block(int shape) {
    const int k = (shape >= 0 && shape < kCellShapeCount) ? shape : 0;
    return dim3(kCellShape[k][0], kCellShape[k][1]);
}
static dim3 cell_grid(int nx, int ny, int nz, int ncomp = 1, int shape = 0) {
    const dim3 b = cell_block(shape);
    return dim3(ceil_div(nx, b.x), ceil_div(ny, b.y), nz * ncomp);
}

template <typename T>
__global__ void __launch_bounds__(256) k_grad(const T* c, T* f, int nx, int ny, int nz, T idx_) {
    NSLGF_CELL_INDEX
    Fld<T> C{c, nx, ny, nz};
    const T v = C(i, j, k);
    f[idx] = (C(i + 1, j, k) - v) * idx_;
    f[n + idx] = (C(i, j + 1, k) - v) * idx_;
    f[2 * n + idx] = (C(i, j, k + 1) - v) * idx_;
}

template <typename T>
__global__ void __launch_bounds__(256) k_div(const T* f, T* c, int nx, int ny, int nz, T idx_, int nbuf) {
    NSLGF_CELL_INDEX
    Vec3<T> F = vec3(f, nx, ny, nz);
    const bool in_supp = i >= nbuf && i < nx - nbuf && j >= nbuf && j < ny - nbuf && k >= nbuf && k < nz - nbuf;
    T v = (F.c[0](i, j, k) + F.c[1](i, j, k) + F.c[2](i, j, k) - F.c[0](i - 1, j, k) - F.c[1](i, j - 1, k) -
           F.c[2](i, j, k - 1)) * idx_;
    c[idx] = in_supp ? v : (T)0;
}

// e = C f on the box; with nbuf > 0 or support blocks, e = M_supp C f: edges outside the support
// domain (the box shrunk by nbuf points, or the union of the marked blocks of nb^3 cells) are set to 0.
template <typename T>
__global__ void __launch_bounds__(256) k_curl(const T* f, T* e, int nx, int ny, int nz, T idx_, int nbuf,
                                              const unsigned char* blocks, int nb) {
    NSLGF_CELL_INDEX
    Vec3<T> F = vec3(f, nx, ny, nz);
    const bool in_supp = in_domain(i, j, k, nx, ny, nz, nbuf, blocks, nb);
    for (int q = 0; q < 3; ++q) e[q * n + idx] = in_supp ? curl_at(F, q, i, j, k, idx_) : (T)0;
}

template <typename T>
__global__ void __launch_bounds__(256) k_curl_bar(const T* e, T* f, int nx, int ny, int nz, T idx_) {
    NSLGF_CELL_INDEX
    Vec3<T> Ed = vec3(e, nx, ny, nz);
    f[idx] = (Ed.c[1](i, j, k - 1) - Ed.c[1](i, j, k) + Ed.c[2](i, j, k) - Ed.c[2](i, j - 1, k)) * idx_;
    f[n + idx] = (Ed.c[2](i - 1, j, k) - Ed.c[2](i, j, k) + Ed.c[0](i, j, k) - Ed.c[0](i, j, k - 1)) * idx_;
    f[2 * n + idx] = (Ed.c[0](i, j - 1, k) - Ed.c[0](i, j, k) + Ed.c[1](i, j, k) - Ed.c[1](i - 1, j, k)) * idx_;
}

template <typename T>
__global__ void __launch_bounds__(256) k_nonlinear(const T* f, T* out, int nx, int ny, int nz, T idx_) {
    NSLGF_CELL_INDEX
    Vec3<T> F = vec3(f, nx, ny, nz);
    T r[3];
    nonlinear_at(F, i, j, k, idx_, r);
    out[idx] = r[0];
    out[n + idx] = r[1];
    out[2 * n + idx] = r[2];
}

template <typename T>
__global__ void __launch_bounds__(256) k_laplacian(const T* a, T* out, int nx, int ny, int nz, T idx2) {
    NSLGF_CELL_INDEX
    const int comp = kz_ / nz;
    Fld<T> A{a + comp * n, nx, ny, nz};
    out[comp * n + idx] = (-(T)6 * A(i, j, k) + A(i + 1, j, k) + A(i - 1, j, k) + A(i, j + 1, k) + A(i, j - 1, k) +
                           A(i, j, k + 1) + A(i, j, k - 1)) * idx2;
}

// Arguments of the stage kernels (the batched forms read one table entry per problem: per consecutive
// values of the grid's z index make up one problem).
struct StageRhsArgs {
    const void* u;
    void* q;
    const void* w1;
    const void* w2;
    void* r;
    double idx;
    StageCoef c;
    int nx, ny, nz;
};
struct StageProjArgs {
    const void* r;
    void* rout;
    const void* dhat;
    const void* q;
    const void* w1;
    const void* w2;
    double c_q, c_w1, c_w2;
    void* wnew;
    double inv, idx;
    int nx, ny, nz;
};
struct AxpbyArgs {
    void* out;
    const void* x;
    double a;
    const void* y;
    double b;
    const void* z;
    double c;
    long long n;
};

// r = c_q q + c_w1 w1 + c_w2 w2 + c_g M_soln Ntilde(u); optionally also copies u into q first
// (stage 1 starts the step with q^1 = u_k).
template <typename T, bool BATCH>
__global__ void __launch_bounds__(256) k_stage_rhs(StageRhsArgs a0, const StageRhsArgs* __restrict__ da, int per) {
    int bz = blockIdx.z, pb = 0;
    if constexpr (BATCH) {
        pb = bz / per;
        bz -= pb * per;
    }
    const StageRhsArgs& A = BATCH ? da[pb] : a0;
    const T* u = (const T*)A.u;
    T* q = (T*)A.q;
    const T* w1 = (const T*)A.w1;
    const T* w2 = (const T*)A.w2;
    T* r = (T*)A.r;
    const T idx_ = (T)A.idx;
    const StageCoef c = A.c;
    const int copy_q = c.copy_q, nx = A.nx, ny = A.ny, nz = A.nz;
    NSLGF_CELL_INDEX_Z(bz)
    Vec3<T> U = vec3(u, nx, ny, nz);
    const bool in_soln = in_domain(i, j, k, nx, ny, nz, c.nbuf, c.soln_blocks, c.nb);
    T nl[3] = {0, 0, 0};
    if (in_soln) {
        if (i >= 1 && i < nx - 1 && j >= 1 && j < ny - 1 && k >= 1 && k < nz - 1)
            nonlinear_at(unchecked(U), i, j, k, idx_, nl);
        else
            nonlinear_at(U, i, j, k, idx_, nl);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const long long p = a * n + idx;
        T qv;
        if (copy_q) {
            qv = u[p];
            q[p] = qv;
        } else {
            qv = q[p];
        }
        double v = c.c_q * (double)qv + c.c_g * (double)nl[a];
        if (w1) v += c.c_w1 * (double)w1[p];
        if (w2) v += c.c_w2 * (double)w2[p];
        r[p] = (T)v;
    }
}

// y = r - G dhat (into r); if wnew: wnew = (y - (c_q q + c_w1 w1 + c_w2 w2)) * inv
template <typename T, bool BATCH>
__global__ void __launch_bounds__(256) k_stage_project(StageProjArgs a0, const StageProjArgs* __restrict__ da,
                                                       int per) {
    int bz = blockIdx.z, pb = 0;
    if constexpr (BATCH) {
        pb = bz / per;
        bz -= pb * per;
    }
    const StageProjArgs& A = BATCH ? da[pb] : a0;
    const T* r = (const T*)A.r;
    T* rout = (T*)A.rout;
    const T* dhat = (const T*)A.dhat;
    const T* q = (const T*)A.q;
    const T* w1 = (const T*)A.w1;
    const T* w2 = (const T*)A.w2;
    const double c_q = A.c_q, c_w1 = A.c_w1, c_w2 = A.c_w2, inv = A.inv;
    T* wnew = (T*)A.wnew;
    const int nx = A.nx, ny = A.ny, nz = A.nz;
    const T idx_ = (T)A.idx;
    NSLGF_CELL_INDEX_Z(bz)
    Fld<T> D{dhat, nx, ny, nz};
    const T d0 = D(i, j, k);
    const T g[3] = {(D(i + 1, j, k) - d0) * idx_, (D(i, j + 1, k) - d0) * idx_, (D(i, j, k + 1) - d0) * idx_};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const long long p = a * n + idx;
        const T y = r[p] - g[a];
        rout[p] = y;
        if (wnew) {
            double base = c_q * (double)q[p];
            if (w1) base += c_w1 * (double)w1[p];
            if (w2) base += c_w2 * (double)w2[p];
            wnew[p] = (T)(((double)y - base) * inv);
        }
    }
}

// BATCH: the grid's y index is the problem.
template <typename T, bool BATCH>
__global__ void __launch_bounds__(256) k_axpby(AxpbyArgs a0, const AxpbyArgs* __restrict__ da) {
    const AxpbyArgs& A = BATCH ? da[blockIdx.y] : a0;
    T* out = (T*)A.out;
    const T* x = (const T*)A.x;
    const T* y = (const T*)A.y;
    const T* z = (const T*)A.z;
    const double a = A.a, b = A.b, c = A.c;
    const long long n = A.n;
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n) return;
    double v = a * (double)x[idx];
    if (y) v += b * (double)y[idx];
    if (z) v += c * (double)z[idx];
    out[idx] = (T)v;
}

// Plain streaming copy (16-byte vectors), the reference for hardware byte counters.
__global__ void __launch_bounds__(256) k_copy(const uint4* __restrict__ in, uint4* __restrict__ out, long long n16) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += (long long)gridDim.x * blockDim.x)
        out[i] = in[i];
}

int launch_copy(const void* in, void* out, size_t bytes, hipStream_t s) {
    if (recording_unsupported()) return NSLGF_OK;
    if (bytes % 16 != 0 || ((uintptr_t)in % 16) != 0 || ((uintptr_t)out % 16) != 0) {
        set_error("copy: size and pointers must be multiples of 16 bytes");
        return NSLGF_EINVAL;
    }
    const long long n16 = (long long)(bytes / 16);
    hipLaunchKernelGGL(k_copy, dim3(4096), dim3(256), 0, s, (const uint4*)in, (uint4*)out, n16);
    NSLGF_LAUNCH_CHECK();
    return NSLGF_OK;
}

template <typename T>
__global__ void __launch_bounds__(256) k_max_speed(const T* u, int nx, int ny, int nz, double* partial) {
    const long long n = (long long)nx * ny * nz;
    __shared__ double red[256];
    double m = 0.0;
    for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
         idx += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(idx % nx);
        const int j = (int)((idx / nx) % ny);
        const int k = (int)(idx / ((long long)nx * ny));
        Vec3<T> U = vec3(u, nx, ny, nz);
        const double a = 0.5 * ((double)U.c[0](i, j, k) + (double)U.c[0](i - 1, j, k));
        const double b = 0.5 * ((double)U.c[1](i, j, k) + (double)U.c[1](i, j - 1, k));
        const double c = 0.5 * ((double)U.c[2](i, j, k) + (double)U.c[2](i, j, k - 1));
        m = fmax(m, sqrt(a * a + b * b + c * c));
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// Largest |u^(q)| over the three components on the solution domain (the box shrunk by nbuf points);
// one partial maximum per workgroup.
template <typename T>
__global__ void __launch_bounds__(256) k_max_abs(const T* u, int nx, int ny, int nz, int nbuf, double* partial) {
    const long long n = (long long)nx * ny * nz;
    __shared__ double red[256];
    double m = 0.0;
    for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < 3 * n;
         idx += (long long)gridDim.x * blockDim.x) {
        const long long p = idx % n;
        const int i = (int)(p % nx);
        const int j = (int)((p / nx) % ny);
        const int k = (int)(p / ((long long)nx * ny));
        if (i >= nbuf && i < nx - nbuf && j >= nbuf && j < ny - nbuf && k >= nbuf && k < nz - nbuf)
            m = fmax(m, fabs((double)u[idx]));
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// Volume integrals of an isolated vortex ring (Sec. 6.2, Eq. int_quantities) as 15 raw sums over the
// box, one set of partial sums per workgroup (partial[blockIdx.x * kDiagnosticSums + v]):
//   0..2   S_q    = sum (x cross w)_q              (I = dx^3 S / 2)
//   3..11  M_qp   = sum (x cross w)_q x_p          (X = dx^3 sum_q I_q M_q. / (2 |I|^2))
//   12     sum |w|^2                               (E = dx^3 sum / 2)
//   13     sum u_c . (x_c cross w_c)               (K = dx^3 sum)
//   14     sum u_c . w_c                           (J = dx^3 sum)
// with w = M_supp C u: zero outside the box and on edges closer than nbuf points to a face (there the
// curl of the zero-extended velocity sees a spurious jump).  The terms of S, M and |w|^2 are taken at the edge of
// each vorticity component (edge (q) is half a cell back along axis q); K and J average u (two faces)
// and w (four edges) to the cell centres.  Point (i, j, k) with offsets -1/2 on the flagged axes sits
// at origin + (i, j, k) dx - dx/2 on those axes.
template <typename T>
__device__ __forceinline__ double edge_w(const Vec3<T>& U, int q, int i, int j, int k, int nx, int ny, int nz, T idx,
                                         int nbuf) {
    if (i < nbuf || j < nbuf || k < nbuf || i >= nx - nbuf || j >= ny - nbuf || k >= nz - nbuf) return 0.0;
    return (double)curl_at(U, q, i, j, k, idx);
}

template <typename T>
__global__ void __launch_bounds__(256) k_diagnostics(const T* u, int nx, int ny, int nz, int nbuf, T idx, double dx,
                                                     double ox, double oy, double oz, double* partial) {
    const long long n = (long long)nx * ny * nz;
    const Vec3<T> U = vec3(u, nx, ny, nz);
    double acc[kDiagnosticSums];
#pragma unroll
    for (int v = 0; v < kDiagnosticSums; ++v) acc[v] = 0.0;
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(p % nx);
        const int j = (int)((p / nx) % ny);
        const int k = (int)(p / ((long long)nx * ny));
        const double xi = ox + i * dx, yj = oy + j * dx, zk = oz + k * dx;
        const double h = 0.5 * dx;
        // the three edges (i, j, k) and their positions: edge (q) is half a cell back along q
        const double w[3] = {edge_w(U, 0, i, j, k, nx, ny, nz, idx, nbuf), edge_w(U, 1, i, j, k, nx, ny, nz, idx, nbuf),
                             edge_w(U, 2, i, j, k, nx, ny, nz, idx, nbuf)};
        const double pe[3][3] = {{xi - h, yj, zk}, {xi, yj - h, zk}, {xi, yj, zk - h}};
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int a = (q + 1) % 3, b = (q + 2) % 3;
            // (x cross w)_q = x_a w_b - x_b w_a, each term at its own edge
            const double tb = pe[b][a] * w[b], ta = pe[a][b] * w[a];
            acc[q] += tb - ta;
#pragma unroll
            for (int c = 0; c < 3; ++c) acc[3 + 3 * q + c] += tb * pe[b][c] - ta * pe[a][c];
        }
        acc[12] += w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
        // cell centre
        const double uc[3] = {0.5 * ((double)U.c[0](i, j, k) + (double)U.c[0](i - 1, j, k)),
                              0.5 * ((double)U.c[1](i, j, k) + (double)U.c[1](i, j - 1, k)),
                              0.5 * ((double)U.c[2](i, j, k) + (double)U.c[2](i, j, k - 1))};
        const double wc[3] = {
            0.25 * (w[0] + edge_w(U, 0, i, j - 1, k, nx, ny, nz, idx, nbuf) + edge_w(U, 0, i, j, k - 1, nx, ny, nz, idx, nbuf) +
                    edge_w(U, 0, i, j - 1, k - 1, nx, ny, nz, idx, nbuf)),
            0.25 * (w[1] + edge_w(U, 1, i, j, k - 1, nx, ny, nz, idx, nbuf) + edge_w(U, 1, i - 1, j, k, nx, ny, nz, idx, nbuf) +
                    edge_w(U, 1, i - 1, j, k - 1, nx, ny, nz, idx, nbuf)),
            0.25 * (w[2] + edge_w(U, 2, i - 1, j, k, nx, ny, nz, idx, nbuf) + edge_w(U, 2, i, j - 1, k, nx, ny, nz, idx, nbuf) +
                    edge_w(U, 2, i - 1, j - 1, k, nx, ny, nz, idx, nbuf))};
        const double xc[3] = {xi - h, yj - h, zk - h};
        const double xw[3] = {xc[1] * wc[2] - xc[2] * wc[1], xc[2] * wc[0] - xc[0] * wc[2],
                              xc[0] * wc[1] - xc[1] * wc[0]};
        acc[13] += uc[0] * xw[0] + uc[1] * xw[1] + uc[2] * xw[2];
        acc[14] += uc[0] * wc[0] + uc[1] * wc[1] + uc[2] * wc[2];
    }
    __shared__ double red[kDiagnosticSums][256];
#pragma unroll
    for (int v = 0; v < kDiagnosticSums; ++v) red[v][threadIdx.x] = acc[v];
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int v = 0; v < kDiagnosticSums; ++v) red[v][threadIdx.x] += red[v][threadIdx.x + s];
        __syncthreads();
    }
    if ((int)threadIdx.x < kDiagnosticSums) partial[(long long)blockIdx.x * kDiagnosticSums + threadIdx.x] = red[threadIdx.x][0];
}

// Block weights of the active domain (Sec. 4.3, Eq. weight_fun), one workgroup per block of nb^3
// cells (blocks tile the box from its origin; the last along an axis may be shorter): mu = the largest
// |(C u)^(q)| over the block's edges, nu = the largest |Dbar Ntilde(u)| over its cells (nl holds
// Ntilde(u) on the box), both over the points at least nbuf away from every box face.
template <typename T>
__global__ void __launch_bounds__(256) k_block_weights(const T* u, const T* nl, int nx, int ny, int nz, int nb, int nbuf,
                                                       T idx, double* mu, double* nu) {
    const int bxn = (nx + nb - 1) / nb, byn = (ny + nb - 1) / nb;
    const int b = (int)blockIdx.x;
    const int bi = b % bxn, bj = (b / bxn) % byn, bk = b / (bxn * byn);
    const Vec3<T> U = vec3(u, nx, ny, nz);
    const Vec3<T> F = vec3(nl, nx, ny, nz);
    double m1 = 0.0, m2 = 0.0;
    const int cells = nb * nb * nb;
    for (int c = threadIdx.x; c < cells; c += blockDim.x) {
        const int i = bi * nb + c % nb, j = bj * nb + (c / nb) % nb, k = bk * nb + c / (nb * nb);
        if (i < nbuf || j < nbuf || k < nbuf || i >= nx - nbuf || j >= ny - nbuf || k >= nz - nbuf) continue;
#pragma unroll
        for (int q = 0; q < 3; ++q) m1 = fmax(m1, fabs((double)curl_at(U, q, i, j, k, idx)));
        const T d = (F.c[0](i, j, k) - F.c[0](i - 1, j, k) + F.c[1](i, j, k) - F.c[1](i, j - 1, k) + F.c[2](i, j, k) -
                     F.c[2](i, j, k - 1)) * idx;
        m2 = fmax(m2, fabs((double)d));
    }
    __shared__ double r1[256], r2[256];
    r1[threadIdx.x] = m1;
    r2[threadIdx.x] = m2;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            r1[threadIdx.x] = fmax(r1[threadIdx.x], r1[threadIdx.x + s]);
            r2[threadIdx.x] = fmax(r2[threadIdx.x], r2[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        mu[b] = r1[0];
        nu[b] = r2[0];
    }
}

// ---------------------------------------------------------------------------------------------------
template <typename T>
static int stencil_t(int op, const void* src, void* dst, int ncomp, int nx, int ny, int nz, double dx, hipStream_t s,
                     int shape) {
    if (recording_unsupported()) return NSLGF_OK;
    const long long n = (long long)nx * ny * nz;
    const T idx_ = (T)(1.0 / dx);
    const dim3 grid = cell_grid(nx, ny, nz, 1, shape), block = cell_block(shape);
    switch (op) {
        case NSLGF_OP_GRAD: hipLaunchKernelGGL(k_grad<T>, grid, block, 0, s, (const T*)src, (T*)dst, nx, ny, nz, idx_); break;
        case NSLGF_OP_DIV: hipLaunchKernelGGL(k_div<T>, grid, block, 0, s, (const T*)src, (T*)dst, nx, ny, nz, idx_, 0); break;
        case NSLGF_OP_CURL: hipLaunchKernelGGL(k_curl<T>, grid, block, 0, s, (const T*)src, (T*)dst, nx, ny, nz, idx_, 0, nullptr, 0); break;
        case NSLGF_OP_CURL_BAR: hipLaunchKernelGGL(k_curl_bar<T>, grid, block, 0, s, (const T*)src, (T*)dst, nx, ny, nz, idx_); break;
        case NSLGF_OP_NONLINEAR: hipLaunchKernelGGL(k_nonlinear<T>, grid, block, 0, s, (const T*)src, (T*)dst, nx, ny, nz, idx_); break;
        case NSLGF_OP_LAPLACIAN:
            hipLaunchKernelGGL(k_laplacian<T>, cell_grid(nx, ny, nz, ncomp, shape), block, 0, s, (const T*)src, (T*)dst, nx,
                               ny, nz, (T)(1.0 / (dx * dx)));
            break;
        default: set_error("stencil_apply: unknown operator"); return NSLGF_EINVAL;
    }
    NSLGF_LAUNCH_CHECK();
    return NSLGF_OK;
}

int launch_stencil(int op, int dtype, const void* src, void* dst, int ncomp, int nx, int ny, int nz, double dx,
                   hipStream_t s, int shape) {
    if (dtype == NSLGF_F32) return stencil_t<float>(op, src, dst, ncomp, nx, ny, nz, dx, s, shape);
    return stencil_t<double>(op, src, dst, ncomp, nx, ny, nz, dx, s, shape);
}

// Batched launches: nprob problems' argument tables, one problem's grid (z extended by nprob).
template <typename T> static int batched_rhs(const void* args, int nprob, dim3 g, dim3 b, hipStream_t s) {
    hipLaunchKernelGGL((k_stage_rhs<T, true>), dim3(g.x, g.y, g.z * nprob), b, 0, s, StageRhsArgs{},
                       (const StageRhsArgs*)args, (int)g.z);
    NSLGF_LAUNCH_CHECK();
    return NSLGF_OK;
}
template <typename T> static int batched_proj(const void* args, int nprob, dim3 g, dim3 b, hipStream_t s) {
    hipLaunchKernelGGL((k_stage_project<T, true>), dim3(g.x, g.y, g.z * nprob), b, 0, s, StageProjArgs{},
                       (const StageProjArgs*)args, (int)g.z);
    NSLGF_LAUNCH_CHECK();
    return NSLGF_OK;
}
template <typename T> static int batched_axpby(const void* args, int nprob, dim3 g, dim3 b, hipStream_t s) {
    hipLaunchKernelGGL((k_axpby<T, true>), dim3(g.x, nprob), b, 0, s, AxpbyArgs{}, (const AxpbyArgs*)args);
    NSLGF_LAUNCH_CHECK();
    return NSLGF_OK;
}

int launch_stage_rhs(int dtype, const void* u, const void* q, const void* w1, const void* w2, void* r,
                     const StageCoef& c, int nx, int ny, int nz, double dx, hipStream_t s, int shape) {
    const StageRhsArgs a{u, (void*)q, w1, w2, r, 1.0 / dx, c, nx, ny, nz};
    const dim3 grid = cell_grid(nx, ny, nz, 1, shape), block = cell_block(shape);
    if (launch_recorder()) {
        record_launch(dtype == NSLGF_F32 ? &batched_rhs<float> : &batched_rhs<double>, grid, block, a);
        return NSLGF_OK;
    }
    if (dtype == NSLGF_F32)
        hipLaunchKernelGGL((k_stage_rhs<float, false>), grid, block, 0, s, a, nullptr, 0);
    else
        hipLaunchKernelGGL((k_stage_rhs<double, false>), grid, block, 0, s, a, nullptr, 0);
    NSLGF_LAUNCH_CHECK();
    return NSLGF_OK;
}

int launch_masked_div(int dtype, const void* r, void* sdiv, int nbuf, int nx, int ny, int nz, double dx,
                      hipStream_t s) {
    if (recording_unsupported()) return NSLGF_OK;
    const long long n = (long long)nx * ny * nz;
    if (dtype == NSLGF_F32)
        hipLaunchKernelGGL(k_div<float>, cell_grid(nx, ny, nz), cell_block(0), 0, s, (const float*)r, (float*)sdiv, nx,
                           ny, nz, (float)(1.0 / dx), nbuf);
    else
        hipLaunchKernelGGL(k_div<double>, cell_grid(nx, ny, nz), cell_block(0), 0, s, (const double*)r, (double*)sdiv, nx,
                           ny, nz, 1.0 / dx, nbuf);
    NSLGF_LAUNCH_CHECK();
    return NSLGF_OK;
}

int launch_stage_project(int dtype, const void* r, void* rout, const void* dhat, const void* q, const void* w1,
                         const void* w2, double c_q, double c_w1, double c_w2, void* wnew, double inv, int nx, int ny,
                         int nz, double dx, hipStream_t s, int shape) {
    const StageProjArgs a{r, rout, dhat, q, w1, w2, c_q, c_w1, c_w2, wnew, inv, 1.0 / dx, nx, ny, nz};
    const dim3 grid = cell_grid(nx, ny, nz, 1, shape), block = cell_block(shape);
    if (launch_recorder()) {
        record_launch(dtype == NSLGF_F32 ? &batched_proj<float> : &batched_proj<double>, grid, block, a);
        return NSLGF_OK;
    }
    if (dtype == NSLGF_F32)
        hipLaunchKernelGGL((k_stage_project<float, false>), grid, block, 0, s, a, nullptr, 0);
    else
        hipLaunchKernelGGL((k_stage_project<double, false>), grid, block, 0, s, a, nullptr, 0);
    NSLGF_LAUNCH_CHECK();
    return NSLGF_OK;
}

int launch_axpby(int dtype, void* out, const void* x, double a, const void* y, double b, const void* z, double c,
                 long long n, hipStream_t s) {
    const AxpbyArgs args{out, x, a, y, b, z, c, n};
    const dim3 grid(ceil_div(n, 256)), block(256);
    if (launch_recorder()) {
        record_launch(dtype == NSLGF_F32 ? &batched_axpby<float> : &batched_axpby<double>, grid, block, args);
        return NSLGF_OK;
    }
    if (dtype == NSLGF_F32)
        hipLaunchKernelGGL((k_axpby<float, false>), grid, block, 0, s, args, nullptr);
    else
        hipLaunchKernelGGL((k_axpby<double, false>), grid, block, 0, s, args, nullptr);
    NSLGF_LAUNCH_CHECK();
    return NSLGF_OK;
}

int launch_masked_curl(int dtype, const void* f, void* e, int nbuf, const unsigned char* blocks, int nb, int nx, int ny,
                       int nz, double dx, hipStream_t s, int shape) {
    if (recording_unsupported()) return NSLGF_OK;
    if (dtype == NSLGF_F32)
        hipLaunchKernelGGL(k_curl<float>, cell_grid(nx, ny, nz, 1, shape), cell_block(shape), 0, s, (const float*)f, (float*)e, nx, ny,
                           nz, (float)(1.0 / dx), nbuf, blocks, nb);
    else
        hipLaunchKernelGGL(k_curl<double>, cell_grid(nx, ny, nz, 1, shape), cell_block(shape), 0, s, (const double*)f, (double*)e, nx,
                           ny, nz, 1.0 / dx, nbuf, blocks, nb);
    NSLGF_LAUNCH_CHECK();
    return NSLGF_OK;
}

int launch_max_abs(int dtype, const void* u, int nbuf, int nx, int ny, int nz, double* dev_partial, int nblocks,
                   hipStream_t s) {
    if (recording_unsupported()) return NSLGF_OK;
    if (dtype == NSLGF_F32)
        hipLaunchKernelGGL(k_max_abs<float>, dim3(nblocks), dim3(256), 0, s, (const float*)u, nx, ny, nz, nbuf,
                           dev_partial);
    else
        hipLaunchKernelGGL(k_max_abs<double>, dim3(nblocks), dim3(256), 0, s, (const double*)u, nx, ny, nz, nbuf,
                           dev_partial);
    NSLGF_LAUNCH_CHECK();
    return NSLGF_OK;
}

int launch_diagnostics(int dtype, const void* u, int nbuf, int nx, int ny, int nz, double dx, const double origin[3],
                       double* dev_partial, int nblocks, hipStream_t s) {
    if (recording_unsupported()) return NSLGF_OK;
    if (dtype == NSLGF_F32)
        hipLaunchKernelGGL(k_diagnostics<float>, dim3(nblocks), dim3(256), 0, s, (const float*)u, nx, ny, nz, nbuf,
                           (float)(1.0 / dx), dx, origin[0], origin[1], origin[2], dev_partial);
    else
        hipLaunchKernelGGL(k_diagnostics<double>, dim3(nblocks), dim3(256), 0, s, (const double*)u, nx, ny, nz, nbuf,
                           1.0 / dx, dx, origin[0], origin[1], origin[2], dev_partial);
    NSLGF_LAUNCH_CHECK();
    return NSLGF_OK;
}

int launch_block_weights(int dtype, const void* u, const void* nl, int nx, int ny, int nz, int nb, int nbuf, double dx,
                         double* dev_mu, double* dev_nu, hipStream_t s) {
    if (recording_unsupported()) return NSLGF_OK;
    const long long nblocks = (long long)((nx + nb - 1) / nb) * ((ny + nb - 1) / nb) * ((nz + nb - 1) / nb);
    if (dtype == NSLGF_F32)
        hipLaunchKernelGGL(k_block_weights<float>, dim3((unsigned)nblocks), dim3(256), 0, s, (const float*)u,
                           (const float*)nl, nx, ny, nz, nb, nbuf, (float)(1.0 / dx), dev_mu, dev_nu);
    else
        hipLaunchKernelGGL(k_block_weights<double>, dim3((unsigned)nblocks), dim3(256), 0, s, (const double*)u,
                           (const double*)nl, nx, ny, nz, nb, nbuf, 1.0 / dx, dev_mu, dev_nu);
    NSLGF_LAUNCH_CHECK();
    return NSLGF_OK;
}

int launch_max_speed(int dtype, const void* u, int nx, int ny, int nz, double* dev_partial, int nblocks,
                     hipStream_t s) {
    if (recording_unsupported()) return NSLGF_OK;
    if (dtype == NSLGF_F32)
        hipLaunchKernelGGL(k_max_speed<float>, dim3(nblocks), dim3(256), 0, s, (const float*)u, nx, ny, nz, dev_partial);
    else
        hipLaunchKernelGGL(k_max_speed<double>, dim3(nblocks), dim3(256), 0, s, (const double*)u, nx, ny, nz,
                           dev_partial);
    NSLGF_LAUNCH_CHECK();
    return NSLGF_OK;
}

}  // namespace nslgf
