// Zero-padded FFT convolution passes of the LGF solve (Sec. 2.2, Eq. dpoisson_conv).
//
// The box convolution y = dx^2 g * s equals, on the box, the cyclic convolution of the zero-padded
// source with the LGF wrapped onto a padded lattice of P >= 2n - 1 points per axis.  One scalar
// solve is five passes over HBM:
//   1. rows along x: real -> half spectrum (P/2 + 1 complex), n_x inputs, the rest implicit zeros;
//   2. columns along y: forward, n_y nonzero inputs -> P outputs;
//   3. columns along z: forward (n_z nonzero inputs), times the real even kernel spectrum,
//      inverse, keeping the n_z box outputs -- all in registers, one HBM round trip;
//   4. columns along y: inverse, keeping the n_y box outputs;
//   5. rows along x: half spectrum -> real, keeping the n_x box outputs.
// Rows are contiguous; the column passes work on tiles of TB adjacent columns (one 128-byte
// segment per transform element) so that every global access is coalesced without transposes.
#include <cmath>
#include <type_traits>
#include <vector>

#include "fft.h"
#include "kernels.h"

namespace nslgf {

// ---------------------------------------------------------------------------------------------------
// Masked divergence of a face field at (x, y, z), in the order of operations of the divergence kernel.
template <typename T>
__device__ __forceinline__ T masked_div_at(const T* f, int x, int y, int z, int nx, int ny, int nz, int nbuf,
                                           const unsigned char* blocks, int nb, T idx) {
    if (!in_domain(x, y, z, nx, ny, nz, nbuf, blocks, nb)) return (T)0;
    const long long n = (long long)nx * ny * nz;
    const long long c = ((long long)z * ny + y) * nx + x;
    const T f0m = x > 0 ? f[c - 1] : (T)0;
    const T f1m = y > 0 ? f[n + c - nx] : (T)0;
    const T f2m = z > 0 ? f[2 * n + c - (long long)nx * ny] : (T)0;
    return (f[c] + f[n + c] + f[2 * n + c] - f0m - f1m - f2m) * idx;
}

// PAIRS: the real rows are read as pairs (x[2n], x[2n+1]) with one vector load each (the host sets it
// when the base is aligned, rows and components have even lengths, and n_io is even).  DIV: the rows
// are the masked divergence of RowPass::div_src, formed on load.
// Batched form (da set): the workgroups of grid z index p take the arguments da[p].
template <typename T, int LH, bool PAIRS, bool DIV>
__global__ void __launch_bounds__(256) k_row_r2c(RowPass a0, const RowPass* __restrict__ da) {
    RowPass a = a0;
    if (da) a = da[blockIdx.z];
    using P = Plan1D<LH>;
    constexpr int E = P::E, TP = LH / E, RPW = row_rpw<T, LH>();
    using RL = typename P::Fwd;
    constexpr int LD = row_lds_len<T, LH>();
    __shared__ cplx<T> lds[RPW * LD];
    const int tid = threadIdx.x;
    const int rl = tid / TP, t = tid % TP;
    const long long row = (long long)blockIdx.x * RPW + rl;
    const int comp = blockIdx.y;
    const bool valid = row < a.nrows;
    const T* in = (const T*)a.in + comp * a.in_comp + (valid ? row : 0) * a.in_row;
    cplx<T>* out = (cplx<T>*)a.out + comp * a.out_comp + (valid ? row : 0) * a.out_row;
    // the half-length root table goes to LDS (read by the transform's passes after the barrier below)
    __shared__ cplx<T> twh[LH];
    for (int m = tid; m < LH; m += RPW * TP) twh[m] = ((const cplx<T>*)a.tw_half)[m];
    const cplx<T>* twf = (const cplx<T>*)a.tw_full;
    RowAcc<T> acc{lds + rl * LD};
    cplx<T> v[E];
    constexpr int R1 = First<RL>::value;
#pragma unroll
    for (int b = 0; b < E / R1; ++b) {
        const int j = t + b * TP;
#pragma unroll
        for (int r = 0; r < R1; ++r) {
            const int m = 2 * (j + r * (LH / R1));  // z[n] = x[2n] + i x[2n+1]
            if constexpr (DIV) {
                const int y = (int)(row % a.div_ny), z = (int)(row / a.div_ny);
                const T* f = (const T*)a.div_src;
                const T idx = (T)a.div_idx;
                const T re = (valid && m < a.n_io)
                                 ? masked_div_at<T>(f, m, y, z, a.n_io, a.div_ny, a.div_nz, a.div_nbuf, a.div_blocks, a.div_nb, idx)
                                 : (T)0;
                const T im = (valid && m + 1 < a.n_io)
                                 ? masked_div_at<T>(f, m + 1, y, z, a.n_io, a.div_ny, a.div_nz, a.div_nbuf, a.div_blocks, a.div_nb,
                                                   idx)
                                 : (T)0;
                v[b * R1 + r] = mk<T>(re, im);
            } else if constexpr (PAIRS) {
                v[b * R1 + r] = (valid && m < a.n_io) ? *(const cplx<T>*)(in + m) : mk<T>((T)0, (T)0);
            } else {
                const T re = (valid && m < a.n_io) ? in[m] : (T)0;
                const T im = (valid && m + 1 < a.n_io) ? in[m + 1] : (T)0;
                v[b * R1 + r] = mk<T>(re, im);
            }
        }
    }
    __syncthreads();
    fft_regs<T, LH, false, RL>(v, t, twh, acc);
    constexpr int RLs = Last<RL>::value;
    __syncthreads();
#pragma unroll
    for (int b = 0; b < E / RLs; ++b) {
        const int j = t + b * TP;
#pragma unroll
        for (int r = 0; r < RLs; ++r) acc(j + r * (LH / RLs)) = v[b * RLs + r];
    }
    __syncthreads();
    if (valid) {
        // X[k] = E[k] + W_P^k O[k], E = (Z[k] + conj Z[-k]) / 2, O = -i (Z[k] - conj Z[-k]) / 2
        for (int k = t; k < LH; k += TP) {
            const cplx<T> zk = acc(k);
            const cplx<T> zm = acc(k == 0 ? 0 : LH - k);
            const T ex = (T)0.5 * (zk.x + zm.x), ey = (T)0.5 * (zk.y - zm.y);
            const cplx<T> o = mk<T>((T)0.5 * (zk.y + zm.y), (T)-0.5 * (zk.x - zm.x));
            const cplx<T> wo = cmul<T>(twf[k], o);
            out[k] = mk<T>(ex + wo.x, ey + wo.y);
        }
        if (t == 0) {
            const cplx<T> z0 = acc(0);
            out[LH] = mk<T>(z0.x - z0.y, (T)0);
        }
    }
}

// PAIRS: the real outputs are written as pairs with one vector store each (conditions as for r2c).
template <typename T, int LH, bool PAIRS>
__global__ void __launch_bounds__(256) k_row_c2r(RowPass a0, const RowPass* __restrict__ da) {
    RowPass a = a0;
    if (da) a = da[blockIdx.z];
    using P = Plan1D<LH>;
    constexpr int E = P::E, TP = LH / E, RPW = row_rpw<T, LH>();
    using RL = Reverse<typename P::Fwd>;
    constexpr int LD = row_lds_len<T, LH>();
    __shared__ cplx<T> lds[RPW * LD];
    const int tid = threadIdx.x;
    const int rl = tid / TP, t = tid % TP;
    const long long row = (long long)blockIdx.x * RPW + rl;
    const int comp = blockIdx.y;
    const bool valid = row < a.nrows;
    const cplx<T>* in = (const cplx<T>*)a.in + comp * a.in_comp + (valid ? row : 0) * a.in_row;
    T* out = (T*)a.out + comp * a.out_comp + (valid ? row : 0) * a.out_row;
    __shared__ cplx<T> twh[LH];  // the half-length root table, in LDS from the first barrier on
    for (int m = tid; m < LH; m += RPW * TP) twh[m] = ((const cplx<T>*)a.tw_half)[m];
    const cplx<T>* twf = (const cplx<T>*)a.tw_full;
    RowAcc<T> acc{lds + rl * LD};
    for (int k = t; k <= LH; k += TP) acc(k) = valid ? in[k] : mk<T>((T)0, (T)0);
    __syncthreads();
    cplx<T> v[E];
    constexpr int R1 = First<RL>::value;
#pragma unroll
    for (int b = 0; b < E / R1; ++b) {
        const int j = t + b * TP;
#pragma unroll
        for (int r = 0; r < R1; ++r) {
            const int k = j + r * (LH / R1);
            const cplx<T> xk = acc(k), xm = acc(LH - k);
            // Z = (X[k] + conj X[LH-k]) + i W_P^{-k} (X[k] - conj X[LH-k])
            const cplx<T> d = mk<T>(xk.x - xm.x, xk.y + xm.y);
            const cplx<T> o = cmulc<T>(d, twf[k]);
            v[b * R1 + r] = mk<T>(xk.x + xm.x - o.y, xk.y - xm.y + o.x);
        }
    }
    fft_regs<T, LH, true, RL>(v, t, twh, acc);
    constexpr int RLs = Last<RL>::value;
    if (valid) {
#pragma unroll
        for (int b = 0; b < E / RLs; ++b) {
            const int j = t + b * TP;
#pragma unroll
            for (int r = 0; r < RLs; ++r) {
                const int m = 2 * (j + r * (LH / RLs));
                if constexpr (PAIRS) {
                    if (m < a.n_io) *(cplx<T>*)(out + m) = v[b * RLs + r];
                } else {
                    if (m < a.n_io) out[m] = v[b * RLs + r].x;
                    if (m + 1 < a.n_io) out[m + 1] = v[b * RLs + r].y;
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------------------------------
// PR bit 1: n_in <= L/2, so the forward transform's first butterflies see a zero upper half; bit 2:
// n_out <= L/2, so the inverse transform's last butterflies produce only the lower half (set by the
// host; the fused pass always has both).
// Batched form (da set): one problem spans `per` consecutive values of the grid's z index (FWD, INV:
// its components) or of the logical workgroup index (CONV) and takes the arguments da[p].
template <typename T, int L, int MODE, int V = 0, int PR = 0>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(PlanV<L, V>::waves)))
k_col(ColPass a0, const ColPass* __restrict__ da, int per) {
    using P = PlanV<L, V>;
    constexpr int E = P::E, TP = L / E, TB = col_tb<T>(TP);
    using RF = typename P::Fwd;
    using RI = Reverse<RF>;
    static_assert(TB * TP <= 512, "column pass workgroup too large");
    constexpr int LD = col_lds_len<L>();
    constexpr bool SPLIT = col_split_exchange<T, L>();
    using Acc = typename std::conditional<SPLIT, ColAccS<T, TB>, ColAcc<T, TB>>::type;
    using LdsElem = typename std::conditional<SPLIT, T, cplx<T>>::type;
    __shared__ LdsElem lds[TB * LD];
    const int tid = threadIdx.x;
    const int c = tid % TB, t = tid / TB;
    int tile, outer, comp;
    ColPass a = a0;
    if constexpr (MODE == COL_CONV) {
        // One-dimensional grid, remapped so that the workgroups sharing a spectrum tile (the mirrored
        // outer indices ky and P - ky, every component) run on one XCD one after the other: the
        // hardware hands workgroup b to XCD b mod 8, so XCD x takes the x-th contiguous chunk of the
        // logical order below and the tile stays in that XCD's L2.
        const int n = (int)gridDim.x, b = (int)blockIdx.x, x = b % 8;
        int lg = x * (n / 8) + min(x, n % 8) + b / 8;
        if (da) {
            a = da[lg / per];
            lg %= per;
        }
        comp = lg % a.ncomp;
        const int rest = lg / a.ncomp;
        const int sq = rest % a.nouter;
        tile = rest / a.nouter;
        outer = (sq & 1) ? a.nouter - 1 - (sq >> 1) : (sq >> 1);
    } else {
        tile = blockIdx.x;
        outer = blockIdx.y;
        comp = blockIdx.z;
        if (da) {
            a = da[blockIdx.z / per];
            comp = blockIdx.z % per;
        }
    }
    const int col = tile * TB + c;
    const bool valid = col < a.ncols;
    const cplx<T>* in = (const cplx<T>*)a.in + comp * a.in_comp + (long long)outer * a.in_outer + (valid ? col : 0);
    cplx<T>* out = (cplx<T>*)a.out + comp * a.out_comp + (long long)outer * a.out_outer + (valid ? col : 0);
    // The fused pass reads its twiddles from a copy of the root table in LDS, made once per
    // workgroup (the barrier matters: composite radix-16/32 butterflies read the table already in
    // the first pass); the single-transform passes read them through the caches, which measured
    // faster there.
    const cplx<T>* tw;
    if constexpr (MODE == COL_CONV) {
        __shared__ cplx<T> twl[L];
        for (int m = tid; m < L; m += TB * TP) twl[m] = ((const cplx<T>*)a.tw)[m];
        __syncthreads();
        tw = twl;
    } else {
        tw = (const cplx<T>*)a.tw;
    }
    Acc acc{lds, c};
    cplx<T> v[E];
    constexpr int R1 = (MODE == COL_INV) ? First<RI>::value : First<RF>::value;
#pragma unroll
    for (int b = 0; b < E / R1; ++b) {
        const int j = t + b * TP;
#pragma unroll
        for (int r = 0; r < R1; ++r) {
            const int row = j + r * (L / R1);
            if (MODE != COL_INV && (PR & 1) && prunable<R1>() && 2 * r >= R1)
                v[b * R1 + r] = mk<T>((T)0, (T)0);  // padding (row >= L/2 >= n_in)
            else
                v[b * R1 + r] = (valid && row < a.n_in) ? in[(long long)row * a.in_row] : mk<T>((T)0, (T)0);
        }
    }
    // COL_CONV: the spectrum values this thread multiplies by are loaded now, behind the data loads,
    // so that their latency overlaps the forward transform
    constexpr int RLf = Last<RF>::value;
    T kv[MODE == COL_CONV ? E : 1];
    if constexpr (MODE == COL_CONV) {
        const int kyf = min(outer, a.outer_period - outer);
        // the spectrum is tiled by the default plan's column width KTB, which a variant's TB may divide
        constexpr int KTB = col_tb<T>(L / Plan1D<L>::E);
        static_assert(KTB % TB == 0, "column tiles must nest in the spectrum's tiles");
        const T* kh;
        if constexpr (KTB == TB) {
            kh = (const T*)a.khat + ((long long)kyf * a.khat_tiles + tile) * (L / 2 + 1) * KTB + c;
        } else {
            const unsigned kcol = (unsigned)(tile * TB + c);
            kh = (const T*)a.khat + ((long long)kyf * a.khat_tiles + kcol / KTB) * (L / 2 + 1) * KTB + kcol % KTB;
        }
#pragma unroll
        for (int b = 0; b < E / RLf; ++b) {
            const int j = t + b * TP;
#pragma unroll
            for (int r = 0; r < RLf; ++r) {
                const int kz = j + r * (L / RLf);
                kv[b * RLf + r] = kh[min(kz, L - kz) * KTB];
            }
        }
    }
    if constexpr (MODE == COL_INV) {
        fft_regs<T, L, true, RI, Acc, E, PR & 2>(v, t, tw, acc);
    } else {
        fft_regs<T, L, false, RF, Acc, E, PR & 1>(v, t, tw, acc);
    }
    if constexpr (MODE == COL_CONV) {
        const T sc = (T)a.scale;
#pragma unroll
        for (int e = 0; e < E; ++e) v[e] = cscale<T>(v[e], kv[e] * sc);
        fft_regs<T, L, true, RI, Acc, E, PR & 2>(v, t, tw, acc);
    }
    using ROut = typename std::conditional<MODE == COL_FWD, RF, RI>::type;
    constexpr int RO = Last<ROut>::value;
    if (valid) {
#pragma unroll
        for (int b = 0; b < E / RO; ++b) {
            const int j = t + b * TP;
#pragma unroll
            for (int r = 0; r < RO; ++r) {
                const int row = j + r * (L / RO);
                if (MODE != COL_FWD && (PR & 2) && prunable<RO>() && 2 * r >= RO) continue;  // not computed
                if (row < a.n_out) out[(long long)row * a.out_row] = v[b * RO + r];
            }
        }
    }
}

// ---------------------------------------------------------------------------------------------------
static const int kLengths[] = {16, 32, 48, 64, 96, 128, 160, 192, 256, 320, 384, 512};

bool fft_length_supported(int P) {
    for (int L : kLengths)
        if (L == P) return true;
    return false;
}

int next_supported_length(int n) {
    for (int L : kLengths)
        if (L >= n) return L;
    return -1;
}

template <int L> static int tb_of(int dtype) {
    constexpr int TP = L / Plan1D<L>::E;
    return dtype == NSLGF_F32 ? col_tb<float>(TP) : col_tb<double>(TP);
}

int col_tile_width(int L, int dtype) {
    switch (L) {
#define NSLGF_CASE(L_) case L_: return tb_of<L_>(dtype);
        NSLGF_CASE(16) NSLGF_CASE(32) NSLGF_CASE(48) NSLGF_CASE(64) NSLGF_CASE(96) NSLGF_CASE(128)
        NSLGF_CASE(160) NSLGF_CASE(192) NSLGF_CASE(256) NSLGF_CASE(320) NSLGF_CASE(384) NSLGF_CASE(512)
#undef NSLGF_CASE
    }
    return -1;
}

int make_twiddles(int L, int dtype, void** dev_out) {
    const size_t esz = 2 * dtype_size(dtype);
    std::vector<unsigned char> host(esz * L);
    const long double two_pi = 6.283185307179586476925286766559005768L;
    for (int m = 0; m < L; ++m) {
        // exp(-2 pi i m / L) evaluated in extended precision and rounded once to the dtype
        // (accurately rounded twiddles); the exact quarter-period values are set directly
        const long double ang = two_pi * (long double)m / (long double)L;
        long double c = cosl(ang), s = sinl(ang);
        if (m == 0) { c = 1; s = 0; }
        if (4 * m == L) { c = 0; s = 1; }
        if (2 * m == L) { c = -1; s = 0; }
        if (4 * m == 3 * L) { c = 0; s = -1; }
        if (dtype == NSLGF_F32) {
            float* p = (float*)host.data();
            p[2 * m] = (float)c;
            p[2 * m + 1] = (float)-s;
        } else {
            double* p = (double*)host.data();
            p[2 * m] = (double)c;
            p[2 * m + 1] = (double)-s;
        }
    }
    void* d = nullptr;
    if (hipMalloc(&d, host.size()) != hipSuccess) {
        set_error("hipMalloc(twiddles) failed");
        return NSLGF_ENOMEM;
    }
    NSLGF_HIP_CHECK(hipMemcpy(d, host.data(), host.size(), hipMemcpyHostToDevice));
    *dev_out = d;
    return NSLGF_OK;
}

LaunchRecorder*& launch_recorder() {
    static thread_local LaunchRecorder* r = nullptr;
    return r;
}

// Batched launches of the row and column passes: nprob problems' argument tables, one problem's grid.
template <typename T, int LH, bool PAIRS, bool DIV>
static int batched_r2c(const void* args, int nprob, dim3 g, dim3 b, hipStream_t s) {
    hipLaunchKernelGGL((k_row_r2c<T, LH, PAIRS, DIV>), dim3(g.x, g.y, nprob), b, 0, s, RowPass{}, (const RowPass*)args);
    NSLGF_LAUNCH_CHECK();
    return NSLGF_OK;
}
template <typename T, int LH, bool PAIRS>
static int batched_c2r(const void* args, int nprob, dim3 g, dim3 b, hipStream_t s) {
    hipLaunchKernelGGL((k_row_c2r<T, LH, PAIRS>), dim3(g.x, g.y, nprob), b, 0, s, RowPass{}, (const RowPass*)args);
    NSLGF_LAUNCH_CHECK();
    return NSLGF_OK;
}
template <typename T, int L, int MODE, int V, int PR>
static int batched_col(const void* args, int nprob, dim3 g, dim3 b, hipStream_t s) {
    if (MODE == COL_CONV)
        hipLaunchKernelGGL((k_col<T, L, MODE, V, PR>), dim3(g.x * nprob), b, 0, s, ColPass{}, (const ColPass*)args,
                           (int)g.x);
    else
        hipLaunchKernelGGL((k_col<T, L, MODE, V, PR>), dim3(g.x, g.y, g.z * nprob), b, 0, s, ColPass{},
                           (const ColPass*)args, (int)g.z);
    NSLGF_LAUNCH_CHECK();
    return NSLGF_OK;
}

template <typename T, int LH, bool PAIRS, bool DIV> static int issue_r2c(const RowPass& a, dim3 grid, dim3 block,
                                                                          hipStream_t s) {
    if (launch_recorder()) {
        record_launch(&batched_r2c<T, LH, PAIRS, DIV>, grid, block, a);
        return NSLGF_OK;
    }
    hipLaunchKernelGGL((k_row_r2c<T, LH, PAIRS, DIV>), grid, block, 0, s, a, nullptr);
    NSLGF_LAUNCH_CHECK();
    return NSLGF_OK;
}
template <typename T, int L, int MODE, int V, int PR> static int issue_col(const ColPass& a, dim3 grid, dim3 block,
                                                                           hipStream_t s) {
    if (launch_recorder()) {
        record_launch(&batched_col<T, L, MODE, V, PR>, grid, block, a);
        return NSLGF_OK;
    }
    hipLaunchKernelGGL((k_col<T, L, MODE, V, PR>), grid, block, 0, s, a, nullptr, 0);
    NSLGF_LAUNCH_CHECK();
    return NSLGF_OK;
}

template <typename T> static bool real_pairs(const void* p, long long row, long long comp, int n_io) {
    return ((uintptr_t)p % (2 * sizeof(T))) == 0 && row % 2 == 0 && comp % 2 == 0 && n_io % 2 == 0;
}
template <typename T, int LH> static int do_r2c(const RowPass& a, hipStream_t s) {
    constexpr int TP = LH / Plan1D<LH>::E, RPW = row_rpw<T, LH>();
    dim3 grid(ceil_div(a.nrows, RPW), a.ncomp);
    if (a.div_src) {
        if (a.ncomp != 1 || a.nrows != (long long)a.div_ny * a.div_nz) {
            set_error("row pass: the divergence input needs one component over ny * nz rows");
            return NSLGF_EINVAL;
        }
        return issue_r2c<T, LH, false, true>(a, grid, dim3(RPW * TP), s);
    }
    if (real_pairs<T>(a.in, a.in_row, a.in_comp, a.n_io)) return issue_r2c<T, LH, true, false>(a, grid, dim3(RPW * TP), s);
    return issue_r2c<T, LH, false, false>(a, grid, dim3(RPW * TP), s);
}
template <typename T, int LH> static int do_c2r(const RowPass& a, hipStream_t s) {
    constexpr int TP = LH / Plan1D<LH>::E, RPW = row_rpw<T, LH>();
    dim3 grid(ceil_div(a.nrows, RPW), a.ncomp);
    const bool pairs = real_pairs<T>(a.out, a.out_row, a.out_comp, a.n_io);
    if (launch_recorder()) {
        record_launch(pairs ? &batched_c2r<T, LH, true> : &batched_c2r<T, LH, false>, grid, dim3(RPW * TP), a);
        return NSLGF_OK;
    }
    if (pairs)
        hipLaunchKernelGGL((k_row_c2r<T, LH, true>), grid, dim3(RPW * TP), 0, s, a, nullptr);
    else
        hipLaunchKernelGGL((k_row_c2r<T, LH, false>), grid, dim3(RPW * TP), 0, s, a, nullptr);
    NSLGF_LAUNCH_CHECK();
    return NSLGF_OK;
}
template <typename T, int L, int MODE, int V = 0> static int do_col(const ColPass& a, hipStream_t s) {
    constexpr int TP = L / PlanV<L, V>::E, TB = col_tb<T>(TP);
    if (a.nouter > 65535 || a.ncomp > 65535) {
        set_error("column pass grid too large");
        return NSLGF_EINVAL;
    }
    dim3 grid(ceil_div(a.ncols, TB), a.nouter, a.ncomp);
    if (MODE == COL_CONV) grid = dim3(ceil_div(a.ncols, TB) * a.nouter * a.ncomp);
    const bool half_in = 2 * a.n_in <= L, half_out = 2 * a.n_out <= L;
    if (MODE == COL_CONV) {
        if (!half_in || !half_out) {
            set_error("column pass: the fused pass needs n_in, n_out <= L/2");
            return NSLGF_EINVAL;
        }
        return issue_col<T, L, MODE, V, 3>(a, grid, dim3(TB * TP), s);
    }
    if ((MODE == COL_FWD && half_in) || (MODE == COL_INV && half_out))
        return issue_col<T, L, MODE, V, MODE == COL_FWD ? 1 : 2>(a, grid, dim3(TB * TP), s);
    return issue_col<T, L, MODE, V, 0>(a, grid, dim3(TB * TP), s);
}

#define NSLGF_ROW_SWITCH(FN, T)                                                                    \
    switch (P) {                                                                                   \
        case 16: return FN<T, 8>(a, s);                                                            \
        case 32: return FN<T, 16>(a, s);                                                           \
        case 48: return FN<T, 24>(a, s);                                                           \
        case 64: return FN<T, 32>(a, s);                                                           \
        case 96: return FN<T, 48>(a, s);                                                           \
        case 128: return FN<T, 64>(a, s);                                                          \
        case 160: return FN<T, 80>(a, s);                                                          \
        case 192: return FN<T, 96>(a, s);                                                          \
        case 256: return FN<T, 128>(a, s);                                                         \
        case 320: return FN<T, 160>(a, s);                                                         \
        case 384: return FN<T, 192>(a, s);                                                         \
        case 512: return FN<T, 256>(a, s);                                                         \
    }

int launch_row_r2c(int P, int dtype, const RowPass& a, hipStream_t s) {
    if (dtype == NSLGF_F32) {
        NSLGF_ROW_SWITCH(do_r2c, float)
    } else {
        NSLGF_ROW_SWITCH(do_r2c, double)
    }
    set_error("unsupported padded length " + std::to_string(P));
    return NSLGF_EUNSUPPORTED;
}

int launch_row_c2r(int P, int dtype, const RowPass& a, hipStream_t s) {
    if (dtype == NSLGF_F32) {
        NSLGF_ROW_SWITCH(do_c2r, float)
    } else {
        NSLGF_ROW_SWITCH(do_c2r, double)
    }
    set_error("unsupported padded length " + std::to_string(P));
    return NSLGF_EUNSUPPORTED;
}

#define NSLGF_COL_SWITCH(T, MODE)                                                                  \
    switch (L) {                                                                                   \
        case 16: return do_col<T, 16, MODE>(a, s);                                                 \
        case 32: return do_col<T, 32, MODE>(a, s);                                                 \
        case 48: return do_col<T, 48, MODE>(a, s);                                                 \
        case 64: return do_col<T, 64, MODE>(a, s);                                                 \
        case 96: return do_col<T, 96, MODE>(a, s);                                                 \
        case 128: return do_col<T, 128, MODE>(a, s);                                               \
        case 160: return do_col<T, 160, MODE>(a, s);                                               \
        case 192: return do_col<T, 192, MODE>(a, s);                                               \
        case 256: return do_col<T, 256, MODE>(a, s);                                               \
        case 320: return do_col<T, 320, MODE>(a, s);                                               \
        case 384: return do_col<T, 384, MODE>(a, s);                                               \
        case 512: return do_col<T, 512, MODE>(a, s);                                               \
    }

template <typename T, int L, int V> static int col_modes(ColMode mode, const ColPass& a, hipStream_t s) {
    if (mode == COL_FWD) return do_col<T, L, COL_FWD, V>(a, s);
    if (mode == COL_INV) return do_col<T, L, COL_INV, V>(a, s);
    return do_col<T, L, COL_CONV, V>(a, s);
}

template <typename T, int L> static int col_variant(int variant, ColMode mode, const ColPass& a, hipStream_t s) {
    if (variant == 1) return col_modes<T, L, 1>(mode, a, s);
    if (variant == 2) return col_modes<T, L, 2>(mode, a, s);  // (in FP32 on 8-column tiles)
    return col_modes<T, L, 0>(mode, a, s);
}

template <typename T> static int col_dispatch(int L, ColMode mode, const ColPass& a, hipStream_t s, int variant) {
    if (variant > 0) {
        if (L == 512) return col_variant<T, 512>(variant, mode, a, s);
        if (L == 256) return col_variant<T, 256>(variant, mode, a, s);
    }
    if (mode == COL_FWD) {
        NSLGF_COL_SWITCH(T, COL_FWD)
    } else if (mode == COL_INV) {
        NSLGF_COL_SWITCH(T, COL_INV)
    } else {
        NSLGF_COL_SWITCH(T, COL_CONV)
    }
    set_error("unsupported transform length " + std::to_string(L));
    return NSLGF_EUNSUPPORTED;
}

int launch_col(int L, int dtype, ColMode mode, const ColPass& a, hipStream_t s, int variant) {
    return dtype == NSLGF_F32 ? col_dispatch<float>(L, mode, a, s, variant)
                              : col_dispatch<double>(L, mode, a, s, variant);
}

bool col_variant_valid(int L, int dtype, int v) {
    (void)dtype;
    if (L != 512 && L != 256) return v == 0;
    return v == 0 || v == 1 || v == 2;
}

// Column-pass plan per length, dtype and pass (the y passes or the fused z pass): a valid choice >= 0
// forces that variant; -1 (or a variant that does not exist for the length) takes the default
// measured fastest on gfx950.  FP32: the narrow plan for the y passes (13-15 % ahead of the wide one
// at both lengths), the wide plan for the fused pass (0.21 against 0.33 ms at length 512).  FP64: the
// wide plan spills its registers at length 512, where the default radices on 8 elements per thread
// (twice the waves of the default) win in both passes, and the default plan wins at 256.
int col_variant_choice(int L, int dtype, int choice, bool zpass) {
    if (choice >= 0 && col_variant_valid(L, dtype, choice)) return choice;
    if (L != 512 && L != 256) return 0;
    if (dtype == NSLGF_F32) return zpass ? 1 : 0;
    return L == 512 ? 2 : 0;
}

}  // namespace nslgf
