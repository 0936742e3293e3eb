// Pencil FFT building blocks for CDNA4 (gfx950): Stockham passes on register-held elements with
// LDS exchanges between passes.
//
// A length-L transform is split over TP = L / E threads, each holding E complex values in
// registers.  A pass of radix R with span NS (product of the earlier radices) processes the
// butterflies j = t + b * TP (b < E / R) of thread t: it reads x[j + r L/R], r < R, twiddles them by
// W_{NS R}^{r (j mod NS)}, applies the length-R DFT and writes the outputs to
// (j div NS) NS R + (j mod NS) + r NS.  Outputs of the last pass therefore sit at j + r L/R_last in
// natural order, which is also the input layout of a following transform whose first radix is
// R_last (used to fuse forward transform, spectral multiply and inverse transform without an
// exchange).  Forward transforms use e^{-2 pi i jk/L}; inverse ones e^{+2 pi i jk/L}; neither scales.
#pragma once

#include <type_traits>

#include "common.h"

namespace nslgf {

template <int... Rs> struct RList {};

template <class A, class B> struct RevImpl;
template <int... D> struct RevImpl<RList<>, RList<D...>> { using type = RList<D...>; };
template <int H, int... T, int... D> struct RevImpl<RList<H, T...>, RList<D...>> {
    using type = typename RevImpl<RList<T...>, RList<H, D...>>::type;
};
template <class A> using Reverse = typename RevImpl<A, RList<>>::type;

template <class A> struct First;
template <int H, int... T> struct First<RList<H, T...>> { static constexpr int value = H; };
template <class A> struct Last;
template <int H> struct Last<RList<H>> { static constexpr int value = H; };
template <int H, int H2, int... T> struct Last<RList<H, H2, T...>> { static constexpr int value = Last<RList<H2, T...>>::value; };

// Radix plan per length: forward radix list and elements per thread (every radix divides E).
template <int L> struct Plan1D;
#define NSLGF_FFT_PLAN(L_, E_, ...)                                                                \
    template <> struct Plan1D<L_> {                                                                \
        static constexpr int E = E_;                                                               \
        using Fwd = RList<__VA_ARGS__>;                                                            \
    };
NSLGF_FFT_PLAN(8, 8, 8)
NSLGF_FFT_PLAN(16, 4, 4, 4)
NSLGF_FFT_PLAN(24, 24, 3, 8)
NSLGF_FFT_PLAN(32, 8, 4, 8)
NSLGF_FFT_PLAN(48, 12, 3, 4, 4)
NSLGF_FFT_PLAN(64, 8, 8, 8)
NSLGF_FFT_PLAN(80, 20, 5, 4, 4)
NSLGF_FFT_PLAN(96, 12, 4, 3, 4, 2)
NSLGF_FFT_PLAN(128, 8, 2, 8, 8)
NSLGF_FFT_PLAN(160, 20, 5, 2, 4, 4)
NSLGF_FFT_PLAN(192, 12, 4, 3, 4, 4)
NSLGF_FFT_PLAN(256, 8, 4, 8, 8)
NSLGF_FFT_PLAN(320, 20, 5, 4, 4, 4)
NSLGF_FFT_PLAN(384, 12, 4, 3, 4, 4, 2)
NSLGF_FFT_PLAN(512, 16, 8, 8, 8)
#undef NSLGF_FFT_PLAN

// Column-pass plan variants of lengths 256 and 512 (the plan builder picks one per length and dtype):
//   V = 0  default plan of the length
//   V = 1  wide: radices 16 x 16 or 16 x 32, one LDS exchange per transform
//   V = 2  the default radices on fewer elements per thread (more waves per workgroup), with the
//          register budget held to four waves per SIMD
// `waves` is the minimum number of waves per SIMD the register allocation must allow.
template <int L, int V> struct PlanV {
    static constexpr int E = Plan1D<L>::E;
    using Fwd = typename Plan1D<L>::Fwd;
    static constexpr int waves = 1;
};
template <> struct PlanV<512, 1> {
    static constexpr int E = 32;
    using Fwd = RList<16, 32>;
    static constexpr int waves = 1;
};
template <> struct PlanV<256, 1> {
    static constexpr int E = 16;
    using Fwd = RList<16, 16>;
    static constexpr int waves = 1;
};
template <> struct PlanV<512, 2> {
    static constexpr int E = 8;
    using Fwd = RList<8, 8, 8>;
    static constexpr int waves = 4;
};
template <> struct PlanV<256, 2> {
    static constexpr int E = 4;
    using Fwd = RList<4, 4, 4, 4>;
    static constexpr int waves = 4;
};

// Columns per workgroup of the strided (column-tile) kernels: one 128-byte row segment at least,
// and at least one wavefront per workgroup, but at most 512 threads (plans with many threads per
// column then take 64-byte segments).
template <typename T>
__host__ __device__ constexpr int col_tb(int tp) {
    const int base = (int)(128 / (2 * sizeof(T)));
    const int tb = (tp * base >= 64) ? base : 64 / tp;
    return tb * tp > 512 ? 512 / tp : tb;
}


// ---- length-R DFTs on registers -------------------------------------------------------------
template <typename T, int R, bool INV> struct DFT;

template <typename T, bool INV> struct DFT<T, 2, INV> {
    __device__ __forceinline__ static void run(cplx<T>* v) {
        cplx<T> a = v[0], b = v[1];
        v[0] = cadd<T>(a, b);
        v[1] = csub<T>(a, b);
    }
};

template <typename T, bool INV> struct DFT<T, 4, INV> {
    __device__ __forceinline__ static void run(cplx<T>* v) {
        cplx<T> t0 = cadd<T>(v[0], v[2]), t1 = csub<T>(v[0], v[2]);
        cplx<T> t2 = cadd<T>(v[1], v[3]), t3 = csub<T>(v[1], v[3]);
        // forward: X1 = t1 - i t3, X3 = t1 + i t3; inverse swaps the sign of i
        cplx<T> it3 = INV ? cmul_i<T>(t3) : cmul_mi<T>(t3);
        v[0] = cadd<T>(t0, t2);
        v[2] = csub<T>(t0, t2);
        v[1] = cadd<T>(t1, it3);
        v[3] = csub<T>(t1, it3);
    }
};

// Second half of the radix-8 butterfly: X[k] = E[k] + W8^k O[k], X[k+4] = E[k] - W8^k O[k] from the
// length-4 DFTs E of the even and O of the odd inputs (only X[0..3] when nout = 4).
template <typename T, bool INV>
__device__ __forceinline__ void combine8(const cplx<T>* e, const cplx<T>* o, cplx<T>* v, int nout) {
    const T c = (T)0.70710678118654752440084436210484903928;
    // W8^1 = c (1 - i) forward, c (1 + i) inverse; W8^2 = -i / +i; W8^3 = -c (1 + i) / c (-1 + i)
    cplx<T> o1 = INV ? mk<T>(c * (o[1].x - o[1].y), c * (o[1].x + o[1].y))
                     : mk<T>(c * (o[1].x + o[1].y), c * (o[1].y - o[1].x));
    cplx<T> o2 = INV ? cmul_i<T>(o[2]) : cmul_mi<T>(o[2]);
    cplx<T> o3 = INV ? mk<T>(-c * (o[3].x + o[3].y), c * (o[3].x - o[3].y))
                     : mk<T>(c * (o[3].y - o[3].x), -c * (o[3].x + o[3].y));
    v[0] = cadd<T>(e[0], o[0]);
    v[1] = cadd<T>(e[1], o1);
    v[2] = cadd<T>(e[2], o2);
    v[3] = cadd<T>(e[3], o3);
    if (nout == 8) {
        v[4] = csub<T>(e[0], o[0]);
        v[5] = csub<T>(e[1], o1);
        v[6] = csub<T>(e[2], o2);
        v[7] = csub<T>(e[3], o3);
    }
}

template <typename T, bool INV> struct DFT<T, 8, INV> {
    __device__ __forceinline__ static void run(cplx<T>* v) {
        // even / odd split into two length-4 DFTs, then X[k] = E[k] +- W8^k O[k]
        cplx<T> e[4] = {v[0], v[2], v[4], v[6]};
        cplx<T> o[4] = {v[1], v[3], v[5], v[7]};
        DFT<T, 4, INV>::run(e);
        DFT<T, 4, INV>::run(o);
        combine8<T, INV>(e, o, v, 8);
    }
};

template <typename T, bool INV> struct DFT<T, 3, INV> {
    __device__ __forceinline__ static void run(cplx<T>* v) {
        const T h = (T)0.86602540378443864676372317075293618347;  // sin(2 pi / 3)
        cplx<T> s = cadd<T>(v[1], v[2]), d = csub<T>(v[1], v[2]);
        cplx<T> m = mk<T>(v[0].x - (T)0.5 * s.x, v[0].y - (T)0.5 * s.y);
        // forward: X1 = m - i h d, X2 = m + i h d
        cplx<T> ihd = INV ? cmul_i<T>(cscale<T>(d, h)) : cmul_mi<T>(cscale<T>(d, h));
        v[0] = cadd<T>(v[0], s);
        v[1] = cadd<T>(m, ihd);
        v[2] = csub<T>(m, ihd);
    }
};

template <typename T, bool INV> struct DFT<T, 5, INV> {
    __device__ __forceinline__ static void run(cplx<T>* v) {
        const T c1 = (T)0.30901699437494742410229341718281905886;   // cos(2 pi / 5)
        const T c2 = (T)-0.80901699437494742410229341718281905886;  // cos(4 pi / 5)
        const T s1 = (T)0.95105651629515357211643933337938214340;   // sin(2 pi / 5)
        const T s2 = (T)0.58778525229247312916870595463907276860;   // sin(4 pi / 5)
        cplx<T> t1 = cadd<T>(v[1], v[4]), t2 = cadd<T>(v[2], v[3]);
        cplx<T> d1 = csub<T>(v[1], v[4]), d2 = csub<T>(v[2], v[3]);
        cplx<T> a1 = mk<T>(v[0].x + c1 * t1.x + c2 * t2.x, v[0].y + c1 * t1.y + c2 * t2.y);
        cplx<T> a2 = mk<T>(v[0].x + c2 * t1.x + c1 * t2.x, v[0].y + c2 * t1.y + c1 * t2.y);
        cplx<T> b1 = mk<T>(s1 * d1.x + s2 * d2.x, s1 * d1.y + s2 * d2.y);
        cplx<T> b2 = mk<T>(s2 * d1.x - s1 * d2.x, s2 * d1.y - s1 * d2.y);
        // forward: X1 = a1 - i b1, X4 = a1 + i b1, X2 = a2 - i b2, X3 = a2 + i b2
        cplx<T> ib1 = INV ? cmul_i<T>(b1) : cmul_mi<T>(b1);
        cplx<T> ib2 = INV ? cmul_i<T>(b2) : cmul_mi<T>(b2);
        v[0] = cadd<T>(v[0], cadd<T>(t1, t2));
        v[1] = cadd<T>(a1, ib1);
        v[4] = csub<T>(a1, ib1);
        v[2] = cadd<T>(a2, ib2);
        v[3] = csub<T>(a2, ib2);
    }
};

// Composite length R = R1 * R2 DFT on registers (decimation in time, n = R2 n1 + n2,
// k = k1 + R1 k2): length-R1 DFTs over n1, internal twiddles W_R^{n2 k1} read from the root table
// of the full transform (W_R^m = tw[m * (L/R)]), length-R2 DFTs over n2.
template <typename T, int R1, int R2, bool INV> struct DFTC {
    __device__ __forceinline__ static void run(cplx<T>* v, const cplx<T>* __restrict__ tw, int lr) {
        constexpr int R = R1 * R2;
        cplx<T> y[R];
#pragma unroll
        for (int n2 = 0; n2 < R2; ++n2) {
            cplx<T> a[R1];
#pragma unroll
            for (int n1 = 0; n1 < R1; ++n1) a[n1] = v[R2 * n1 + n2];
            DFT<T, R1, INV>::run(a);
#pragma unroll
            for (int k1 = 0; k1 < R1; ++k1) {
                if (n2 * k1 == 0) {
                    y[k1 * R2 + n2] = a[k1];
                } else {
                    const cplx<T> w = tw[(n2 * k1) * lr];
                    y[k1 * R2 + n2] = INV ? cmulc<T>(a[k1], w) : cmul<T>(a[k1], w);
                }
            }
        }
#pragma unroll
        for (int k1 = 0; k1 < R1; ++k1) {
            cplx<T> b[R2];
#pragma unroll
            for (int n2 = 0; n2 < R2; ++n2) b[n2] = y[k1 * R2 + n2];
            DFT<T, R2, INV>::run(b);
#pragma unroll
            for (int k2 = 0; k2 < R2; ++k2) v[k1 + R1 * k2] = b[k2];
        }
    }
};

// Pruned butterflies of the zero-padded transforms.  DFTHalfIn: inputs R/2 .. R-1 are zero (the
// first pass of a transform whose upper half is padding).  DFTHalfOut: only outputs 0 .. R/2-1 are
// kept (the last pass of a transform whose upper half is discarded).  Even radices 2, 4, 8; the
// kept values equal the full butterfly's.
template <typename T, int R, bool INV> struct DFTHalfIn;
template <typename T, bool INV> struct DFTHalfIn<T, 2, INV> {
    __device__ __forceinline__ static void run(cplx<T>* v) { v[1] = v[0]; }
};
template <typename T, bool INV> struct DFTHalfIn<T, 4, INV> {
    __device__ __forceinline__ static void run(cplx<T>* v) {
        // (a, b, 0, 0): X0 = a + b, X2 = a - b, X1 = a - i b, X3 = a + i b (forward)
        const cplx<T> a = v[0], b = v[1];
        const cplx<T> ib = INV ? cmul_i<T>(b) : cmul_mi<T>(b);
        v[0] = cadd<T>(a, b);
        v[2] = csub<T>(a, b);
        v[1] = cadd<T>(a, ib);
        v[3] = csub<T>(a, ib);
    }
};
template <typename T, bool INV> struct DFTHalfIn<T, 8, INV> {
    __device__ __forceinline__ static void run(cplx<T>* v) {
        cplx<T> e[4] = {v[0], v[2], v[4], v[6]};  // v[4], v[6] are zero
        cplx<T> o[4] = {v[1], v[3], v[5], v[7]};  // v[5], v[7] are zero
        DFTHalfIn<T, 4, INV>::run(e);
        DFTHalfIn<T, 4, INV>::run(o);
        combine8<T, INV>(e, o, v, 8);
    }
};
template <typename T, int R, bool INV> struct DFTHalfOut;
template <typename T, bool INV> struct DFTHalfOut<T, 2, INV> {
    __device__ __forceinline__ static void run(cplx<T>* v) { v[0] = cadd<T>(v[0], v[1]); }
};
template <typename T, bool INV> struct DFTHalfOut<T, 4, INV> {
    __device__ __forceinline__ static void run(cplx<T>* v) {
        cplx<T> t0 = cadd<T>(v[0], v[2]), t1 = csub<T>(v[0], v[2]);
        cplx<T> t2 = cadd<T>(v[1], v[3]), t3 = csub<T>(v[1], v[3]);
        cplx<T> it3 = INV ? cmul_i<T>(t3) : cmul_mi<T>(t3);
        v[0] = cadd<T>(t0, t2);
        v[1] = cadd<T>(t1, it3);
    }
};
template <typename T, bool INV> struct DFTHalfOut<T, 8, INV> {
    __device__ __forceinline__ static void run(cplx<T>* v) {
        cplx<T> e[4] = {v[0], v[2], v[4], v[6]};
        cplx<T> o[4] = {v[1], v[3], v[5], v[7]};
        DFT<T, 4, INV>::run(e);
        DFT<T, 4, INV>::run(o);
        combine8<T, INV>(e, o, v, 4);
    }
};

// ---- passes -----------------------------------------------------------------------------------
// tw: root table tw[m] = exp(-2 pi i m / L), m < L (forward); the inverse conjugates it.
// PRUNE bit 1: this is the first pass and inputs r >= R/2 of every butterfly are zero; bit 2: this is
// the last pass and only outputs r < R/2 are used.  Only even radices 2, 4, 8 are pruned.
template <int R> __host__ __device__ constexpr bool prunable() { return R == 2 || R == 4 || R == 8; }

template <typename T, int L, int E, int TP, bool INV, int NS, int R, int PRUNE = 0>
__device__ __forceinline__ void pass_compute(cplx<T>* v, int t, const cplx<T>* __restrict__ tw) {
#pragma unroll
    for (int b = 0; b < E / R; ++b) {
        if constexpr (NS > 1) {
            const int j = t + b * TP;
            const int k = j % NS;
#pragma unroll
            for (int r = 1; r < R; ++r) {
                const cplx<T> w = tw[r * k * (L / (NS * R))];
                v[b * R + r] = INV ? cmulc<T>(v[b * R + r], w) : cmul<T>(v[b * R + r], w);
            }
        }
        if constexpr ((PRUNE & 1) && prunable<R>()) {
            DFTHalfIn<T, R, INV>::run(v + b * R);
        } else if constexpr ((PRUNE & 2) && prunable<R>()) {
            DFTHalfOut<T, R, INV>::run(v + b * R);
        } else if constexpr (R == 16) {
            DFTC<T, 4, 4, INV>::run(v + b * R, tw, L / 16);
        } else if constexpr (R == 32) {
            DFTC<T, 4, 8, INV>::run(v + b * R, tw, L / 32);
        } else {
            DFT<T, R, INV>::run(v + b * R);
        }
    }
}

template <typename T, int L, int E, int TP, int NS, int R, class Acc>
__device__ __forceinline__ void pass_store(const cplx<T>* v, int t, Acc& acc) {
#pragma unroll
    for (int b = 0; b < E / R; ++b) {
        const int j = t + b * TP;
        const int base = (j / NS) * NS * R + (j % NS);
#pragma unroll
        for (int r = 0; r < R; ++r) acc(base + r * NS) = v[b * R + r];
    }
}

template <typename T, int L, int E, int TP, int R, class Acc>
__device__ __forceinline__ void pass_load(cplx<T>* v, int t, Acc& acc) {
#pragma unroll
    for (int b = 0; b < E / R; ++b) {
        const int j = t + b * TP;
#pragma unroll
        for (int r = 0; r < R; ++r) v[b * R + r] = acc(j + r * (L / R));
    }
}

// Split exchange (accessors that address one real part per element): the real parts go through LDS
// first, then the imaginary parts, so the tile needs half the LDS (two more barriers per exchange; the
// same values move, the results are unchanged).
template <class Acc> struct SplitExchange : std::false_type {};

template <typename T, int L, int E, int TP, int NS, int R, int PART, class Acc>
__device__ __forceinline__ void pass_store_part(const cplx<T>* v, int t, Acc& acc) {
#pragma unroll
    for (int b = 0; b < E / R; ++b) {
        const int j = t + b * TP;
        const int base = (j / NS) * NS * R + (j % NS);
#pragma unroll
        for (int r = 0; r < R; ++r) acc(base + r * NS) = PART ? v[b * R + r].y : v[b * R + r].x;
    }
}

template <typename T, int L, int E, int TP, int R, int PART, class Acc>
__device__ __forceinline__ void pass_load_part(cplx<T>* v, int t, Acc& acc) {
#pragma unroll
    for (int b = 0; b < E / R; ++b) {
        const int j = t + b * TP;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if constexpr (PART)
                v[b * R + r].y = acc(j + r * (L / R));
            else
                v[b * R + r].x = acc(j + r * (L / R));
        }
    }
}

template <typename T, int L, int E, int TP, bool INV, int NS, int PRUNE, class RL> struct Runner;

template <typename T, int L, int E, int TP, bool INV, int NS, int PRUNE, int R>
struct Runner<T, L, E, TP, INV, NS, PRUNE, RList<R>> {
    template <class Acc>
    __device__ __forceinline__ static void run(cplx<T>* v, int t, const cplx<T>* __restrict__ tw, Acc&) {
        // a single-pass transform prunes only one side (input pruning wins)
        constexpr int P1 = (NS == 1 && (PRUNE & 1)) ? 1 : (PRUNE & 2);
        pass_compute<T, L, E, TP, INV, NS, R, P1>(v, t, tw);
    }
};

template <typename T, int L, int E, int TP, bool INV, int NS, int PRUNE, int R, int R2, int... Rest>
struct Runner<T, L, E, TP, INV, NS, PRUNE, RList<R, R2, Rest...>> {
    template <class Acc>
    __device__ __forceinline__ static void run(cplx<T>* v, int t, const cplx<T>* __restrict__ tw, Acc& acc) {
        pass_compute<T, L, E, TP, INV, NS, R, (NS == 1) ? (PRUNE & 1) : 0>(v, t, tw);
        __syncthreads();
        if constexpr (SplitExchange<Acc>::value) {
            pass_store_part<T, L, E, TP, NS, R, 0>(v, t, acc);
            __syncthreads();
            pass_load_part<T, L, E, TP, R2, 0>(v, t, acc);
            __syncthreads();
            pass_store_part<T, L, E, TP, NS, R, 1>(v, t, acc);
            __syncthreads();
            pass_load_part<T, L, E, TP, R2, 1>(v, t, acc);
        } else {
            pass_store<T, L, E, TP, NS, R>(v, t, acc);
            __syncthreads();
            pass_load<T, L, E, TP, R2>(v, t, acc);
        }
        Runner<T, L, E, TP, INV, NS * R, PRUNE, RList<R2, Rest...>>::run(v, t, tw, acc);
    }
};

// Full transform on registers: input v[b R1 + r] = x[t + b TP + r L/R1] (R1 = first radix of the
// list), output v[b Rl + r] = X[t + b TP + r L/Rl] (Rl = last radix).  PRUNE bit 1: the inputs
// x[L/2 .. L-1] are zero (the caller leaves v[b R1 + r], r >= R1/2, unset or zero); bit 2: only
// X[0 .. L/2-1] are wanted (v[b Rl + r], r >= Rl/2, are left undefined).  Either applies only when the
// first (bit 1) or last (bit 2) radix is 2, 4 or 8.
template <typename T, int L, bool INV, class RL, class Acc, int E = Plan1D<L>::E, int PRUNE = 0>
__device__ __forceinline__ void fft_regs(cplx<T>* v, int t, const cplx<T>* __restrict__ tw, Acc& acc) {
    Runner<T, L, E, L / E, INV, 1, PRUNE, RL>::run(v, t, tw, acc);
}

// LDS accessor of the column-tile kernels: element pos of column c, columns interleaved.
template <typename T, int TB>
struct ColAcc {
    cplx<T>* base;
    int c;
    __device__ __forceinline__ cplx<T>& operator()(int pos) { return base[(pos + (pos >> 4)) * TB + c]; }
};
template <int L> __host__ __device__ constexpr int col_lds_len() { return L + L / 16 + 1; }
// The same layout holding one part (real or imaginary) per element: the split exchange.
template <typename T, int TB>
struct ColAccS {
    T* base;
    int c;
    __device__ __forceinline__ T& operator()(int pos) { return base[(pos + (pos >> 4)) * TB + c]; }
};
template <typename T, int TB> struct SplitExchange<ColAccS<T, TB>> : std::true_type {};
// Column passes that use the split exchange: FP64 at lengths 320 and 384, which hold 20 and 12
// elements per thread, so a full-complex tile needs 20 KB and 12 KB of LDS per wave and a CU holds 6
// and 8 waves; halving it lets the register budget, not the LDS, set the occupancy (measured: the
// 192^3 FP64 step 3% faster; in FP32 the tiles are half as large and the extra barriers cost more
// than the occupancy gains).
template <typename T, int L> __host__ __device__ constexpr bool col_split_exchange() {
    return sizeof(T) == 8 && (L == 320 || L == 384);
}

// LDS accessor of the row kernels: one contiguous segment per row, one pad element every 2^S
// elements (S = 4; padding every 8 complex doubles measured no faster and would cost the row kernels
// a workgroup per CU once their twiddle table is in LDS).
template <typename T> __host__ __device__ constexpr int row_pad_shift() { return 4; }
template <typename T>
struct RowAcc {
    cplx<T>* base;
    __device__ __forceinline__ cplx<T>& operator()(int pos) { return base[pos + (pos >> row_pad_shift<T>())]; }
};
template <typename T, int L> __host__ __device__ constexpr int row_lds_len() {
    return L + 1 + ((L + 1) >> row_pad_shift<T>()) + 1;
}
// Rows per workgroup of the contiguous-row kernels of half length LH: up to 256 threads, and at most
// about 40 KB of LDS (row tiles and the half-length twiddle table), so that at least three workgroups
// share a CU (plans with many elements per thread, the radix-3 and radix-5 lengths, have few threads
// per row and would otherwise hold 90-110 KB).  A power of two.
template <typename T, int LH> __host__ __device__ constexpr int row_rpw() {
    constexpr int tp = LH / Plan1D<LH>::E;
    int r = tp >= 256 ? 1 : 256 / tp;
    while (r > 1 && (r * row_lds_len<T, LH>() + LH) * (int)sizeof(cplx<T>) > 40 * 1024) r /= 2;
    return r;
}

}  // namespace nslgf
