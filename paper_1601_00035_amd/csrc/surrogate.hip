// Layers of the learned surrogate (a 3D convolutional U-Net) on CDNA4 matrix cores.
//
// The 3x3x3 convolutions are implicit GEMMs on v_mfma_f32_32x32x16_bf16 (BF16 operands, FP32
// accumulation).  One wavefront owns a 32 x 32 output tile and walks the 27 taps and the input
// channels in steps of 16, gathering its A operand straight from the channels-last activation (the
// 8 BF16 values a lane supplies are contiguous channels of one voxel) and its B operand from the
// weight rows.  Operand layout of the instruction (wave64), checked by sur_mfma_selftest:
//   A (32 x 16): lane l supplies A[l % 32][8 (l / 32) + j], j < 8
//   B (16 x 32): lane l supplies B[8 (l / 32) + j][l % 32]
//   D (32 x 32): lane l holds D[8 (i / 4) + 4 (l / 32) + i % 4][l % 32] in accumulator i < 16
// The weight gradient, whose reduction index is the voxel, first copies dY and X into a blocked layout
// ([voxel / 8][channel][8]: a lane's 8 voxels of one channel are one 16-byte load) and gives each wave
// the three taps of one (dz, dy) pair, which share their row loads.  It reduces over voxels in fixed
// chunks followed by a fixed-order two-level sum, so every result is deterministic.
#include <cmath>

#include "../../include/nslgf_surrogate.h"
#include "kernels.h"

namespace nslgf {

typedef unsigned short bf16_t;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ bf16_t f2bf(float f) {
    unsigned u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (bf16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
    return (bf16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(bf16_t b) { return __uint_as_float(((unsigned)b) << 16); }

__device__ __forceinline__ bf16x8 load8(const bf16_t* p) {
    const uint4 q = *(const uint4*)p;
    return __builtin_bit_cast(bf16x8, q);
}
__device__ __forceinline__ bf16x8 zero8() { return __builtin_bit_cast(bf16x8, make_uint4(0, 0, 0, 0)); }
__device__ __forceinline__ bf16x8 pack8(const bf16_t v[8]) {
    uint4 q;
    q.x = (unsigned)v[0] | ((unsigned)v[1] << 16);
    q.y = (unsigned)v[2] | ((unsigned)v[3] << 16);
    q.z = (unsigned)v[4] | ((unsigned)v[5] << 16);
    q.w = (unsigned)v[6] | ((unsigned)v[7] << 16);
    return __builtin_bit_cast(bf16x8, q);
}

__device__ __forceinline__ int tap_dz(int t) { return t / 9 - 1; }
__device__ __forceinline__ int tap_dy(int t) { return (t / 3) % 3 - 1; }
__device__ __forceinline__ int tap_dx(int t) { return t % 3 - 1; }

// Y[v][n] = act(sum_tap sum_k X[v + SIGN off(tap)][k] Wn[tap][n][k]);  K % 16 == 0, N % 32 == 0.
template <bool RELU, int SIGN>
__global__ void __launch_bounds__(256) k_conv_mfma(const bf16_t* __restrict__ X, const bf16_t* __restrict__ Wn,
                                                   float* __restrict__ Y, int D, int H, int W, int K, int N) {
    const int wave = blockIdx.x * 4 + threadIdx.x / 64;
    const int lane = threadIdx.x % 64;
    const long long nvox = (long long)D * H * W;
    const int mtiles = (int)(nvox / 32), ntiles = N / 32;
    if (wave >= mtiles * ntiles) return;
    const int mt = wave % mtiles, nt = wave / mtiles;
    const long long v0 = (long long)mt * 32;
    const int n0 = nt * 32;
    const int m = lane % 32, half = lane / 32;
    const long long v = v0 + m;
    const int x = (int)(v % W), y = (int)((v / W) % H), z = (int)(v / ((long long)W * H));
    f32x16 acc;
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = 0.f;
    // (loading the operands several steps ahead measured slower: the gathered A rows, not load latency,
    // limit this kernel)
    for (int tap = 0; tap < 27; ++tap) {
        const int zz = z + SIGN * tap_dz(tap), yy = y + SIGN * tap_dy(tap), xx = x + SIGN * tap_dx(tap);
        const bool valid = zz >= 0 && zz < D && yy >= 0 && yy < H && xx >= 0 && xx < W;
        const long long vn = valid ? ((long long)zz * H + yy) * W + xx : 0;
        const bf16_t* xrow = X + vn * K + half * 8;
        const bf16_t* wrow = Wn + ((long long)tap * N + n0 + m) * K + half * 8;
        for (int kc = 0; kc < K; kc += 16) {
            const bf16x8 a = valid ? load8(xrow + kc) : zero8();
            const bf16x8 b = load8(wrow + kc);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
        }
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int row = 8 * (i / 4) + 4 * half + (i % 4);
        float val = acc[i];
        if (RELU) val = fmaxf(val, 0.f);
        Y[(v0 + row) * N + n0 + m] = val;
    }
}

// The same convolution with the input staged in LDS.  A workgroup (4 waves) owns a block of 2 (z) x 8 (y)
// rows of 32 voxels along x and one tile of 32 output channels (the grid's x index also walks the tiles).  For every slice of 16 input channels it copies the slice's halo (4 x 10 x 34 voxels,
// zero outside the volume) into LDS once.  Each wave owns 4 adjacent rows of one z plane: for every
// (dz, dx) of the stencil it reads the 6 halo rows those 4 rows need into registers and applies them for
// the three dy taps, so that an A operand read from LDS serves up to three taps, and a B operand (weights,
// read through the caches) serves the wave's 4 rows.  Needs W % 32 == 0, H % 8 == 0, D % 2 == 0.  The sum
// runs over slices, then dz, dx, dy in a fixed order: results are deterministic.
constexpr int kLdsBZ = 2, kLdsBY = 8, kLdsHX = 34, kLdsRows = 4;
constexpr int kLdsHalo = (kLdsBZ + 2) * (kLdsBY + 2) * kLdsHX;  // voxels of the halo block
template <bool RELU, int SIGN>
__global__ void __launch_bounds__(256) k_conv_lds(const bf16_t* __restrict__ X, const bf16_t* __restrict__ Wn,
                                                  float* __restrict__ Y, int D, int H, int W, int K, int N) {
    __shared__ uint4 halo[kLdsHalo * 2];  // [voxel][16 channels] as two 16-byte halves
    const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
    const int m = lane % 32, half = lane / 32;
    const int xt = W / 32;
    const int x0 = (blockIdx.x % xt) * 32, nb = (blockIdx.x / xt) * 32;
    const int y0 = blockIdx.y * kLdsBY, z0 = blockIdx.z * kLdsBZ;
    // this wave's rows: z = z0 + wave / 2, y = y0 + 4 (wave % 2) + r, r < 4
    const int tz = wave / 2, ty = kLdsRows * (wave % 2);
    f32x16 acc[kLdsRows][1];
#pragma unroll
    for (int r = 0; r < kLdsRows; ++r)
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[r][0][i] = 0.f;
    // this thread's halo elements (the same in every slice): offsets from the block's first voxel, in
    // BF16 elements (the host keeps 4 H W K below 2^31), and whether each lies inside the volume
    constexpr int kPer = (kLdsHalo * 2 + 255) / 256, kFirst = kPer / 2;
    const bf16_t* xblk = X + (((long long)z0 * H + y0) * W + x0) * K;
    int hoff[kPer];
    unsigned hok = 0;
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
        const int q = tid + 256 * i;
        const int hv = q / 2, hh = q % 2;
        const int hx = hv % kLdsHX, hy = (hv / kLdsHX) % (kLdsBY + 2), hz = hv / (kLdsHX * (kLdsBY + 2));
        const int xx = x0 + hx - 1, yy = y0 + hy - 1, zz = z0 + hz - 1;
        hoff[i] = (((hz - 1) * H + (hy - 1)) * W + (hx - 1)) * K + hh * 8;
        if (q < kLdsHalo * 2 && xx >= 0 && xx < W && yy >= 0 && yy < H && zz >= 0 && zz < D) hok |= 1u << i;
    }
    for (int kc = 0; kc < K; kc += 16) {
        // the slice's halo in two batches of loads, each issued whole before its LDS writes
        uint4 hr[kFirst];
#pragma unroll
        for (int i = 0; i < kFirst; ++i)
            hr[i] = (hok >> i) & 1 ? *(const uint4*)(xblk + kc + hoff[i]) : make_uint4(0, 0, 0, 0);
        __syncthreads();  // (the previous slice's reads are done)
#pragma unroll
        for (int i = 0; i < kFirst; ++i) halo[tid + 256 * i] = hr[i];
        uint4 hr2[kPer - kFirst];
#pragma unroll
        for (int i = kFirst; i < kPer; ++i)
            hr2[i - kFirst] = (hok >> i) & 1 ? *(const uint4*)(xblk + kc + hoff[i]) : make_uint4(0, 0, 0, 0);
#pragma unroll
        for (int i = kFirst; i < kPer; ++i)
            if (tid + 256 * i < kLdsHalo * 2) halo[tid + 256 * i] = hr2[i - kFirst];
        __syncthreads();
        // the weights of the next (dz, dx) are loaded while the current ones multiply
        const bf16_t* wbase = Wn + ((long long)nb + m) * K + kc + half * 8;
        auto load_b = [&](int it, bf16x8* b) {
            const int tdz = it / 3 - 1, tdx = it % 3 - 1;
#pragma unroll
            for (int tdy = -1; tdy <= 1; ++tdy) {
                const int tap = (tdz + 1) * 9 + (tdy + 1) * 3 + (tdx + 1);
                b[tdy + 1] = load8(wbase + (long long)tap * N * K);
            }
        };
        bf16x8 bcur[3], bnext[3];
        load_b(0, bcur);
#pragma unroll 1
        for (int it = 0; it < 9; ++it) {
            if (it + 1 < 9) load_b(it + 1, bnext);
            const int tdz = it / 3 - 1, tdx = it % 3 - 1;
            // halo rows ty .. ty + 5 hold the input rows y0 + ty - 1 .. y0 + ty + 4 of plane z + SIGN dz
            const int hb = ((tz + 1 + SIGN * tdz) * (kLdsBY + 2) + ty) * kLdsHX + (m + 1 + SIGN * tdx);
            bf16x8 a[kLdsRows + 2];
#pragma unroll
            for (int j = 0; j < kLdsRows + 2; ++j) a[j] = __builtin_bit_cast(bf16x8, halo[(hb + j * kLdsHX) * 2 + half]);
#pragma unroll
            for (int tdy = -1; tdy <= 1; ++tdy)
#pragma unroll
                for (int r = 0; r < kLdsRows; ++r)
                    acc[r][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[r + SIGN * tdy + 1], bcur[tdy + 1], acc[r][0], 0, 0, 0);
            if (it + 1 < 9) {
#pragma unroll
                for (int j = 0; j < 3; ++j) bcur[j] = bnext[j];
            }
        }
    }
#pragma unroll
    for (int r = 0; r < kLdsRows; ++r) {
        const long long vrow = ((long long)(z0 + tz) * H + (y0 + ty + r)) * W + x0;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int row = 8 * (i / 4) + 4 * half + (i % 4);
            float val = acc[r][0][i];
            if (RELU) val = fmaxf(val, 0.f);
            Y[(vrow + row) * N + nb + m] = val;
        }
    }
}

// Whether the LDS-staged convolution serves a volume and channel count.
static bool conv_lds_ok(int D, int H, int W, int K, int N) {
    return W % 32 == 0 && H % kLdsBY == 0 && D % kLdsBZ == 0 && N % 32 == 0 && N <= 1024 &&
           4LL * H * W * K < (1LL << 31);
}
template <bool RELU, int SIGN>
static void launch_conv_lds(const bf16_t* x, const bf16_t* w, float* y, int D, int H, int W, int K, int N,
                            hipStream_t s) {
    // one output tile per workgroup: more workgroups on the small volumes, and more tiles would hold
    // 64 more accumulator registers per lane and tile
    const dim3 grid((unsigned)(W / 32 * (N / 32)), H / kLdsBY, D / kLdsBZ);
    hipLaunchKernelGGL((k_conv_lds<RELU, SIGN>), grid, dim3(256), 0, s, x, w, y, D, H, W, K, N);
}

// Partial weight gradient of one voxel chunk: P[chunk][tap][co][ci] = sum_{v in chunk} dY[v][co] X[v+off][ci]
__global__ void __launch_bounds__(256) k_conv_wgrad(const bf16_t* __restrict__ dY, const bf16_t* __restrict__ X,
                                                    float* __restrict__ P, int D, int H, int W, int cin, int cout,
                                                    int chunk_len, int nchunks) {
    const int wave = blockIdx.x * 4 + threadIdx.x / 64;
    const int lane = threadIdx.x % 64;
    const int cotiles = cout / 32, citiles = (cin + 31) / 32;
    const int total = nchunks * 27 * cotiles * citiles;
    if (wave >= total) return;
    int r = wave;
    const int cit = r % citiles;
    r /= citiles;
    const int cot = r % cotiles;
    r /= cotiles;
    const int tap = r % 27;
    const int chunk = r / 27;
    const int m = lane % 32, half = lane / 32;
    const int co = cot * 32 + m;   // A row
    const int ci = cit * 32 + m;   // B column
    const bool ci_ok = ci < cin;
    const int dz = tap_dz(tap), dy = tap_dy(tap), dx = tap_dx(tap);
    f32x16 acc;
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = 0.f;
    const long long vstart = (long long)chunk * chunk_len;
    for (long long vb = vstart; vb < vstart + chunk_len; vb += 16) {
        bf16_t av[8], bv[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const long long v = vb + 8 * half + j;
            av[j] = dY[v * cout + co];
            const int x = (int)(v % W), y = (int)((v / W) % H), z = (int)(v / ((long long)W * H));
            const int zz = z + dz, yy = y + dy, xx = x + dx;
            const bool ok = ci_ok && zz >= 0 && zz < D && yy >= 0 && yy < H && xx >= 0 && xx < W;
            bv[j] = ok ? X[(((long long)zz * H + yy) * W + xx) * cin + ci] : (bf16_t)0;
        }
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(pack8(av), pack8(bv), acc, 0, 0, 0);
    }
    if (!ci_ok) return;
    float* out = P + ((long long)chunk * 27 + tap) * cout * cin;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int row = cot * 32 + 8 * (i / 4) + 4 * half + (i % 4);
        out[(long long)row * cin + ci] = acc[i];
    }
}

// Channels-last [nvox][C] -> blocked [nvox / 8][C][8] (BF16): within each group of 8 consecutive voxels the
// channels become the slow index, so that the weight gradient's MFMA operands (whose reduction index is
// the voxel) read 8 consecutive voxels of one channel as one 16-byte load, and the 32 channels of a
// half-wave read 512 contiguous bytes.  One thread transposes 8 voxels x 8 channels in registers.
__global__ void __launch_bounds__(256) k_to_blocked8(const bf16_t* __restrict__ x, bf16_t* __restrict__ y,
                                                     long long ngroups, int C) {
    const int cgs = C / 8;
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ngroups * cgs) return;
    const long long g = e / cgs;
    const int cg = (int)(e % cgs) * 8;
    uint4 in[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) in[j] = *(const uint4*)(x + (g * 8 + j) * C + cg);
    const bf16_t* a = (const bf16_t*)in;  // a[j * 8 + c]: voxel j, channel cg + c
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        bf16_t o[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) o[j] = a[j * 8 + c];
        *(uint4*)(y + (g * C + cg + c) * 8) = *(const uint4*)o;
    }
}

// FP32 -> BF16 cast of channels-last [nvox][C] with an optional ReLU backward and an optional blocked
// copy: val = src (0 where act is given and not > 0, as k_relu_bwd leaves it), y[v][c] = bf16(val) and
// yb[v / 8][c][v % 8] = bf16(val) (the layout of k_to_blocked8).  One thread: 8 voxels x 8 channels.
__global__ void __launch_bounds__(256) k_cast_ex(const float* __restrict__ src, const float* __restrict__ act,
                                                 bf16_t* __restrict__ y, bf16_t* __restrict__ yb, long long ngroups,
                                                 int C) {
    const int cgs = C / 8;
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ngroups * cgs) return;
    const long long g = e / cgs;
    const int cg = (int)(e % cgs) * 8;
    bf16_t o[64];  // o[j * 8 + c]: voxel j, channel cg + c
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const long long base = (g * 8 + j) * C + cg;
        const float4 v0 = *(const float4*)(src + base), v1 = *(const float4*)(src + base + 4);
        float v[8] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w};
        if (act) {
            const float4 a0 = *(const float4*)(act + base), a1 = *(const float4*)(act + base + 4);
            const float a[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
#pragma unroll
            for (int c = 0; c < 8; ++c)
                if (!(a[c] > 0.f)) v[c] = 0.f;
        }
#pragma unroll
        for (int c = 0; c < 8; ++c) o[j * 8 + c] = f2bf(v[c]);
        *(uint4*)(y + base) = *(const uint4*)(o + j * 8);
    }
    if (yb) {
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            bf16_t t[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) t[j] = o[j * 8 + c];
            *(uint4*)(yb + (g * C + cg + c) * 8) = *(const uint4*)t;
        }
    }
}

// Partial weight gradient of one voxel chunk for the three taps of one (dz, dy) pair and one (cout, cin)
// tile pair:
//     P[chunk][tap][co][ci] = sum_{v in chunk} dY[v][co] X[v + off(tap)][ci],  tap = 3 (3 (dz + 1) + dy + 1) + dx + 1,
// from blocked copies (dYb [nvox / 8][cout][8], Xb [nvox / 8][cin][8]).  One wave per (chunk, tile pair,
// (dz, dy)); per 16-voxel slice it loads its A operand (dY, 8 voxels per lane) and the three groups of X
// around x0 (x0 - 8, x0, x0 + 8) once, and forms the B operands of dx = -1, 0, +1 from them.  Small
// register footprint (three accumulators), so that many waves per SIMD hide the load latency.  Requires
// W % 8 == 0 (8-voxel groups stay inside one x row).
__global__ void __launch_bounds__(256) k_conv_wgrad_cm(const bf16_t* __restrict__ dYb, const bf16_t* __restrict__ Xb,
                                                       float* __restrict__ P, int D, int H, int W, int cin, int cout,
                                                       int chunk_len, int nwaves) {
    const int wid = blockIdx.x * 4 + threadIdx.x / 64, lane = threadIdx.x % 64;
    if (wid >= nwaves) return;
    const int cotiles = cout / 32, citiles = (cin + 31) / 32;
    int r = wid;
    const int g = r % 9;  // (dz, dy) = (g / 3 - 1, g % 3 - 1)
    r /= 9;
    const int cit = r % citiles;
    r /= citiles;
    const int cot = r % cotiles;
    const int chunk = r / cotiles;
    const int dz = g / 3 - 1, dy = g % 3 - 1;
    const int m = lane % 32, half = lane / 32;
    const int co = cot * 32 + m, ci = cit * 32 + m;
    const bool ci_ok = ci < cin;
    const bf16_t* acol = dYb + (long long)co * 8;
    const bf16_t* bcol = Xb + (long long)(ci_ok ? ci : 0) * 8;
    const long long astride = (long long)cout * 8, bstride = (long long)cin * 8;
    f32x16 acc[3];
#pragma unroll
    for (int t = 0; t < 3; ++t)
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[t][i] = 0.f;
    // the slice's first voxel as (x, y, z), advanced by 16 voxels per slice without divisions
    const int vstart = chunk * chunk_len, nslices = chunk_len / 16;
    int xs = vstart % W, ys = (vstart / W) % H, zs = vstart / (W * H);
    // operands of one slice: A (dY, 8 voxels of this lane's group) and the X groups at x0 - 8, x0, x0 + 8,
    // loaded one slice ahead of the matrix operations that use them
    auto load = [&](int sl, bf16x8& a, uint4& p, uint4& q, uint4& n) {
        int x0 = xs + 8 * half, y = ys, z = zs;
        if (x0 >= W) {  // (rows of 8 voxels: the second group starts the next row)
            x0 -= W;
            if (++y == H) {
                y = 0;
                ++z;
            }
        }
        a = load8(acol + (long long)((vstart >> 3) + 2 * sl + half) * astride);
        p = make_uint4(0, 0, 0, 0);
        q = p;
        n = p;
        const int zz = z + dz, yy = y + dy;
        if (ci_ok && zz >= 0 && zz < D && yy >= 0 && yy < H) {
            const bf16_t* blk = bcol + (long long)(((unsigned)((zz * H + yy) * W + x0)) >> 3) * bstride;
            q = *(const uint4*)blk;
            if (x0 >= 8) p = *(const uint4*)(blk - bstride);
            if (x0 + 8 < W) n = *(const uint4*)(blk + bstride);
        }
    };
    bf16x8 a_nx;
    uint4 p_nx, q_nx, n_nx;
    load(0, a_nx, p_nx, q_nx, n_nx);
    for (int sl = 0; sl < nslices; ++sl) {
        const bf16x8 a = a_nx;
        const uint4 p = p_nx, q = q_nx, n = n_nx;
        xs += 16;
        while (xs >= W) {
            xs -= W;
            if (++ys == H) {
                ys = 0;
                ++zs;
            }
        }
        if (sl + 1 < nslices) load(sl + 1, a_nx, p_nx, q_nx, n_nx);
        uint4 bm, bp;  // voxels x0 - 1 .. x0 + 6 and x0 + 1 .. x0 + 8 (zero beyond the row)
        bm.x = (q.x << 16) | (p.w >> 16);
        bm.y = (q.y << 16) | (q.x >> 16);
        bm.z = (q.z << 16) | (q.y >> 16);
        bm.w = (q.w << 16) | (q.z >> 16);
        bp.x = (q.x >> 16) | (q.y << 16);
        bp.y = (q.y >> 16) | (q.z << 16);
        bp.z = (q.z >> 16) | (q.w << 16);
        bp.w = (q.w >> 16) | (n.x << 16);
        acc[0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, __builtin_bit_cast(bf16x8, bm), acc[0], 0, 0, 0);
        acc[1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, __builtin_bit_cast(bf16x8, q), acc[1], 0, 0, 0);
        acc[2] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, __builtin_bit_cast(bf16x8, bp), acc[2], 0, 0, 0);
    }
    if (!ci_ok) return;
#pragma unroll
    for (int t = 0; t < 3; ++t) {
        float* out = P + ((long long)chunk * 27 + 3 * g + t) * cout * cin;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int row = cot * 32 + 8 * (i / 4) + 4 * half + (i % 4);
            out[(long long)row * cin + ci] = acc[t][i];
        }
    }
}

// First level of the fixed-order chunk reduction: Q[g][i] = sum of the chunks g G .. g G + G - 1.
__global__ void k_sum_chunk_groups(const float* __restrict__ P, float* __restrict__ Q, long long n, int G) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int g = blockIdx.y;
    float s = 0.f;
    for (int c = g * G; c < (g + 1) * G; ++c) s += P[(long long)c * n + i];
    Q[(long long)g * n + i] = s;
}

__global__ void k_sum_chunks(const float* __restrict__ P, float* __restrict__ dW, long long n, int nchunks) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float s = 0.f;
    for (int c = 0; c < nchunks; ++c) s += P[(long long)c * n + i];
    dW[i] = s;
}

__global__ void k_wtranspose(const bf16_t* __restrict__ w, bf16_t* __restrict__ wt, int cin, int cout) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long n = 27LL * cin * cout;
    if (i >= n) return;
    const int ci = (int)(i % cin);
    const int co = (int)((i / cin) % cout);
    const int tap = (int)(i / ((long long)cin * cout));
    wt[((long long)tap * cin + ci) * cout + co] = w[i];
}

__global__ void k_cast_bf16(const float* __restrict__ x, bf16_t* __restrict__ y, long long n) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = f2bf(x[i]);
}
__global__ void k_relu_bwd(const float* __restrict__ y, float* __restrict__ g, long long n) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && !(y[i] > 0.f)) g[i] = 0.f;
}
__global__ void k_add(const float* __restrict__ a, const float* __restrict__ b, float* __restrict__ o, long long n) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) o[i] = a[i] + b[i];
}

// coarse voxel index of fine (z, y, x)
__device__ __forceinline__ long long coarse_of(long long v, int D, int H, int W) {
    const int x = (int)(v % W), y = (int)((v / W) % H), z = (int)(v / ((long long)W * H));
    return ((long long)(z / 2) * (H / 2) + y / 2) * (W / 2) + x / 2;
}

// Fused resampling, skip sum and cast: val[v][c] = scale * coarse[parent(v)][c] + skip[v][c], parent(v)
// the voxel of the half-resolution grid that holds v (scale 1: the nearest-neighbour upsampling; scale
// 1/8: the adjoint of the 2x2x2 average pooling), then as k_cast_ex: zero where act is given and not
// > 0, y[v][c] = bf16(val), and yb[v / 8][c][v % 8] = bf16(val) when yb is given.  The product and the
// sum are rounded one at a time, as the separate passes round them.  One thread: 8 voxels x 8 channels.
__global__ void __launch_bounds__(256) k_cast_up(const float* __restrict__ coarse, float scale,
                                                 const float* __restrict__ skip, const float* __restrict__ act,
                                                 bf16_t* __restrict__ y, bf16_t* __restrict__ yb, long long ngroups,
                                                 int C, int D, int H, int W) {
    const int cgs = C / 8;
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ngroups * cgs) return;
    const long long g = e / cgs;
    const int cg = (int)(e % cgs) * 8;
    // W % 8 == 0: the 8 voxels lie in one x row, so their parents follow from the first one's
    long long crow = 0;
    int x0 = 0;
    const bool row8 = W % 8 == 0;
    if (row8) {
        const long long v0 = g * 8;
        const long long zy = v0 / W;
        x0 = (int)(v0 - zy * W);
        const int y = (int)(zy % H), z = (int)(zy / H);
        crow = ((long long)(z / 2) * (H / 2) + y / 2) * (W / 2);
    }
    bf16_t o[64];  // o[j * 8 + c]: voxel j, channel cg + c
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const long long v = g * 8 + j;
        const long long parent = row8 ? crow + (x0 + j) / 2 : coarse_of(v, D, H, W);
        const long long base = v * C + cg, cb = parent * C + cg;
        const float4 c0 = *(const float4*)(coarse + cb), c1 = *(const float4*)(coarse + cb + 4);
        const float4 s0 = *(const float4*)(skip + base), s1 = *(const float4*)(skip + base + 4);
        const float cv[8] = {c0.x, c0.y, c0.z, c0.w, c1.x, c1.y, c1.z, c1.w};
        const float sv[8] = {s0.x, s0.y, s0.z, s0.w, s1.x, s1.y, s1.z, s1.w};
        float v8[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) v8[c] = __fadd_rn(__fmul_rn(scale, cv[c]), sv[c]);
        if (act) {
            const float4 a0 = *(const float4*)(act + base), a1 = *(const float4*)(act + base + 4);
            const float a[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
#pragma unroll
            for (int c = 0; c < 8; ++c)
                if (!(a[c] > 0.f)) v8[c] = 0.f;
        }
#pragma unroll
        for (int c = 0; c < 8; ++c) o[j * 8 + c] = f2bf(v8[c]);
        *(uint4*)(y + base) = *(const uint4*)(o + j * 8);
    }
    if (yb) {
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            bf16_t t[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) t[j] = o[j * 8 + c];
            *(uint4*)(yb + (g * C + cg + c) * 8) = *(const uint4*)t;
        }
    }
}

__global__ void k_pool2_fwd(const float* __restrict__ x, float* __restrict__ y, int D, int H, int W, int c) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long nc = (long long)(D / 2) * (H / 2) * (W / 2) * c;
    if (i >= nc) return;
    const int ch = (int)(i % c);
    const long long vc = i / c;
    const int X = (int)(vc % (W / 2)), Y = (int)((vc / (W / 2)) % (H / 2)), Z = (int)(vc / ((long long)(W / 2) * (H / 2)));
    float s = 0.f;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int d = 0; d < 2; ++d) s += x[((((long long)(2 * Z + a) * H + 2 * Y + b) * W) + 2 * X + d) * c + ch];
    y[i] = 0.125f * s;
}
__global__ void k_pool2_bwd(const float* __restrict__ gy, float* __restrict__ gx, int D, int H, int W, int c) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long nf = (long long)D * H * W * c;
    if (i >= nf) return;
    const int ch = (int)(i % c);
    gx[i] = 0.125f * gy[coarse_of(i / c, D, H, W) * c + ch];
}
__global__ void k_up2_fwd(const float* __restrict__ x, float* __restrict__ y, int D, int H, int W, int c) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long nf = (long long)D * H * W * c;
    if (i >= nf) return;
    const int ch = (int)(i % c);
    y[i] = x[coarse_of(i / c, D, H, W) * c + ch];
}
__global__ void k_up2_bwd(const float* __restrict__ gy, float* __restrict__ gx, int D, int H, int W, int c) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long nc = (long long)(D / 2) * (H / 2) * (W / 2) * c;
    if (i >= nc) return;
    const int ch = (int)(i % c);
    const long long vc = i / c;
    const int X = (int)(vc % (W / 2)), Y = (int)((vc / (W / 2)) % (H / 2)), Z = (int)(vc / ((long long)(W / 2) * (H / 2)));
    float s = 0.f;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int d = 0; d < 2; ++d) s += gy[((((long long)(2 * Z + a) * H + 2 * Y + b) * W) + 2 * X + d) * c + ch];
    gx[i] = s;
}

// VEC (c = 4 * 2^sh, grad on 16 bytes): one thread per 4 channels of a voxel (grid-stride), one
// 16-byte store each, so a wave writes contiguous rows; else one thread per voxel, one value at a time.
template <bool VEC>
__global__ void __launch_bounds__(256) k_mse(const float* __restrict__ pred, const float* __restrict__ tgt,
                                             float* __restrict__ grad, double* __restrict__ partial, long long nvox,
                                             int c, int used, int sh) {
    __shared__ double red[256];
    const double inv = 2.0 / ((double)nvox * used);
    double s = 0.0;
    if constexpr (VEC) {
        const long long n4 = nvox << sh;
        for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n4; e += (long long)gridDim.x * blockDim.x) {
            const long long v = e >> sh;
            const int c0 = (int)(e & ((1 << sh) - 1)) * 4;
            float o[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int ch = c0 + k;
                o[k] = 0.f;
                if (ch < used) {
                    const double d = (double)pred[v * c + ch] - (double)tgt[v * used + ch];
                    s += d * d;
                    o[k] = (float)(inv * d);
                }
            }
            *(float4*)(grad + v * c + c0) = make_float4(o[0], o[1], o[2], o[3]);
        }
    } else {
        for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < nvox;
             v += (long long)gridDim.x * blockDim.x) {
            for (int ch = 0; ch < c; ++ch) {
                if (ch < used) {
                    const double d = (double)pred[v * c + ch] - (double)tgt[v * used + ch];
                    s += d * d;
                    grad[v * c + ch] = (float)(inv * d);
                } else {
                    grad[v * c + ch] = 0.f;
                }
            }
        }
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// Squared error with the gradient written only as its BF16 copy y[v][c] and, when yb is given, the
// blocked copy yb[v / 8][c][v % 8] (the layout of k_to_blocked8): the gradient values are those of
// k_mse, rounded as k_cast_ex rounds them.  One thread: 8 voxels x 8 channels (grid-stride); per-block
// FP64 partial sums of the squared error, in the order of this decomposition.
__global__ void __launch_bounds__(256) k_mse_cast(const float* __restrict__ pred, const float* __restrict__ tgt,
                                                  bf16_t* __restrict__ y, bf16_t* __restrict__ yb,
                                                  double* __restrict__ partial, long long nvox, int C, int used) {
    __shared__ double red[256];
    const double inv = 2.0 / ((double)nvox * used);
    const int cgs = C / 8;
    const long long ngroups = nvox / 8;
    double s = 0.0;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < ngroups * cgs;
         e += (long long)gridDim.x * blockDim.x) {
        const long long g = e / cgs;
        const int cg = (int)(e % cgs) * 8;
        bf16_t o[64];  // o[j * 8 + c]: voxel j, channel cg + c
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const long long v = g * 8 + j;
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                const int ch = cg + c;
                float gv = 0.f;
                if (ch < used) {
                    const double d = (double)pred[v * C + ch] - (double)tgt[v * used + ch];
                    s += d * d;
                    gv = (float)(inv * d);
                }
                o[j * 8 + c] = f2bf(gv);
            }
            *(uint4*)(y + v * C + cg) = *(const uint4*)(o + j * 8);
        }
        if (yb) {
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                bf16_t t[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) t[j] = o[j * 8 + c];
                *(uint4*)(yb + (g * C + cg + c) * 8) = *(const uint4*)t;
            }
        }
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void k_adam(float* __restrict__ w, bf16_t* __restrict__ wb, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, long long n, float lr, float b1, float b2, float eps, float c1, float c2) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    wb[i] = f2bf(wi);
}

__global__ void k_pack_input(const double* __restrict__ om, bf16_t* __restrict__ x, long long nvox, double scale,
                             double feat) {
    const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nvox) return;
    bf16_t out[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) out[k] = 0;
    for (int q = 0; q < 3; ++q) out[q] = f2bf((float)(om[q * nvox + v] * scale));
    out[3] = f2bf((float)feat);
    uint4* dst = (uint4*)(x + v * 16);
    dst[0] = __builtin_bit_cast(uint4, pack8(out));
    dst[1] = __builtin_bit_cast(uint4, pack8(out + 8));
}
// Input of the correction form: channels 0..2 = omega * scale, 3 = feat, 4..6 = delta * dscale.
__global__ void k_pack_input_pair(const double* __restrict__ om, const double* __restrict__ dl, bf16_t* __restrict__ x,
                                  long long nvox, double scale, double dscale, double feat) {
    const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nvox) return;
    bf16_t out[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) out[k] = 0;
    for (int q = 0; q < 3; ++q) {
        out[q] = f2bf((float)(om[q * nvox + v] * scale));
        out[4 + q] = f2bf((float)(dl[q * nvox + v] * dscale));
    }
    out[3] = f2bf((float)feat);
    uint4* dst = (uint4*)(x + v * 16);
    dst[0] = __builtin_bit_cast(uint4, pack8(out));
    dst[1] = __builtin_bit_cast(uint4, pack8(out + 8));
}
// out = ca a + cb b + cc c (c may be null), FP64, n values.
__global__ void k_combine3(const double* __restrict__ a, const double* __restrict__ b, const double* __restrict__ c,
                           double* __restrict__ out, long long n, double ca, double cb, double cc) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double r = ca * a[i] + cb * b[i];
    if (c) r += cc * c[i];
    out[i] = r;
}
__global__ void k_pack_target(const double* __restrict__ f, float* __restrict__ t, long long nvox, double scale) {
    const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nvox) return;
    for (int q = 0; q < 3; ++q) t[v * 3 + q] = (float)(f[q * nvox + v] * scale);
}
__global__ void k_unpack_update(const double* __restrict__ base, const float* __restrict__ y, double* __restrict__ out,
                                long long nvox, int c, double inv_scale) {
    const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nvox) return;
    for (int q = 0; q < 3; ++q) out[q * nvox + v] = base[q * nvox + v] + (double)y[v * c + q] * inv_scale;
}

__global__ void k_mfma_selftest(const bf16_t* A, const bf16_t* B, float* C) {
    const int l = threadIdx.x;
    const int m = l % 32, half = l / 32;
    bf16_t av[8], bv[8];
    for (int j = 0; j < 8; ++j) {
        av[j] = A[m * 16 + 8 * half + j];
        bv[j] = B[(8 * half + j) * 32 + m];
    }
    f32x16 acc;
    for (int i = 0; i < 16; ++i) acc[i] = 0.f;
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(pack8(av), pack8(bv), acc, 0, 0, 0);
    for (int i = 0; i < 16; ++i) C[(8 * (i / 4) + 4 * half + (i % 4)) * 32 + m] = acc[i];
}

static int grid1(long long n) { return ceil_div(n, 256); }

// Voxel chunks of the blocked-layout weight gradient: a power of two with chunks of at least 64 voxels
// (a multiple of 16), enough waves (chunks x tile pairs x 9) to fill the device, at most 4096 chunks.
// Voxel chunks of the weight gradient: as many as give about `target` waves (each chunk and
// (dz, dy) pair and channel-tile pair is one wave), chunks of at least 64 voxels (a multiple of 16).
// Fewer, longer chunks write fewer partials (at 128^3 with 32 -> 32 channels: 2048 chunks wrote
// 226 MB that the sums read back); measured best: about 4096 waves from 64^3 up, 2048 below.
static int wgrad_cm_chunks(long long nvox, int cin, int cout) {
    const long long pairs = (long long)(cout / 32) * ((cin + 31) / 32);
    const long long target = nvox >= 64LL * 64 * 64 ? 4096 : 2048;
    int nch = 1;
    while (nch < 4096 && nch * pairs * 9 < target && nvox % (nch * 2) == 0 && nvox / (nch * 2) >= 64 &&
           (nvox / (nch * 2)) % 16 == 0)
        nch *= 2;
    return nch;
}
static bool wgrad_cm_ok(int W, long long nvox) { return W % 8 == 0 && nvox % 16 == 0; }
static size_t align256(size_t b) { return (b + 255) / 256 * 256; }

static int wgrad_chunks(long long nvox) {
    // voxel chunks of at least 512 (a multiple of 16), at most 64 chunks
    int nch = 1;
    while (nch < 64 && nvox / (nch * 2) >= 512 && (nvox / (nch * 2)) % 16 == 0 && nvox % (nch * 2) == 0) nch *= 2;
    return nch;
}

}  // namespace nslgf

using namespace nslgf;

#define SUR_ENTER(h)                                                                               \
    do {                                                                                           \
        int rc_ = enter_handle(h);                                                                 \
        if (rc_ != NSLGF_OK) return rc_;                                                           \
    } while (0)

// The matrix-core and layout kernels move 16 bytes per access: their tensors must start on 16 bytes.
static bool a16(const void* p) { return p == nullptr || ((uintptr_t)p % 16) == 0; }

static int conv_shape_ok(int D, int H, int W, int cin, int cout) {
    NSLGF_CHECK_ARG(D >= 1 && H >= 1 && W >= 1 && (long long)D * H * W % 32 == 0, "surrogate: D*H*W must be a multiple of 32");
    NSLGF_CHECK_ARG(cin >= 16 && cin % 16 == 0 && cin <= 1024, "surrogate: cin must be a multiple of 16");
    NSLGF_CHECK_ARG(cout >= 32 && cout % 32 == 0 && cout <= 1024, "surrogate: cout must be a multiple of 32");
    return NSLGF_OK;
}

extern "C" {

int sur_conv3d_fwd(nslgf_t h, const void* x, const void* w, void* y, int D, int H, int W, int cin, int cout, int relu,
                   void* stream) {
    SUR_ENTER(h);
    NSLGF_TRY(conv_shape_ok(D, H, W, cin, cout));
    NSLGF_CHECK_ARG(x && w && y, "sur_conv3d_fwd: null pointer");
    NSLGF_CHECK_ARG(a16(x) && a16(w) && a16(y), "sur_conv3d_fwd: tensors must be 16-byte aligned");
    const long long waves = (long long)D * H * W / 32 * (cout / 32);
    hipStream_t s = (hipStream_t)stream;
    if (conv_lds_ok(D, H, W, cin, cout)) {
        if (relu)
            launch_conv_lds<true, 1>((const bf16_t*)x, (const bf16_t*)w, (float*)y, D, H, W, cin, cout, s);
        else
            launch_conv_lds<false, 1>((const bf16_t*)x, (const bf16_t*)w, (float*)y, D, H, W, cin, cout, s);
    } else if (relu)
        hipLaunchKernelGGL((k_conv_mfma<true, 1>), dim3(ceil_div(waves, 4)), dim3(256), 0, s, (const bf16_t*)x,
                           (const bf16_t*)w, (float*)y, D, H, W, cin, cout);
    else
        hipLaunchKernelGGL((k_conv_mfma<false, 1>), dim3(ceil_div(waves, 4)), dim3(256), 0, s, (const bf16_t*)x,
                           (const bf16_t*)w, (float*)y, D, H, W, cin, cout);
    NSLGF_LAUNCH_CHECK();
    return NSLGF_OK;
}

int sur_conv3d_bwd_data(nslgf_t h, const void* dy, const void* wt, void* dx, int D, int H, int W, int cin, int cout,
                        void* stream) {
    SUR_ENTER(h);
    NSLGF_TRY(conv_shape_ok(D, H, W, cin, cout));
    NSLGF_CHECK_ARG(cin % 32 == 0, "sur_conv3d_bwd_data: cin must be a multiple of 32");
    NSLGF_CHECK_ARG(dy && wt && dx, "sur_conv3d_bwd_data: null pointer");
    NSLGF_CHECK_ARG(a16(dy) && a16(wt) && a16(dx), "sur_conv3d_bwd_data: tensors must be 16-byte aligned");
    // GEMM with K = cout (inner) and N = cin (outputs), gathering dy at v - off
    const long long waves = (long long)D * H * W / 32 * (cin / 32);
    if (conv_lds_ok(D, H, W, cout, cin))
        launch_conv_lds<false, -1>((const bf16_t*)dy, (const bf16_t*)wt, (float*)dx, D, H, W, cout, cin,
                                   (hipStream_t)stream);
    else
        hipLaunchKernelGGL((k_conv_mfma<false, -1>), dim3(ceil_div(waves, 4)), dim3(256), 0, (hipStream_t)stream,
                           (const bf16_t*)dy, (const bf16_t*)wt, (float*)dx, D, H, W, cout, cin);
    NSLGF_LAUNCH_CHECK();
    return NSLGF_OK;
}

size_t sur_bwd_weight_work_bytes(int D, int H, int W, int cin, int cout) {
    if (D < 1 || H < 1 || W < 1 || cin < 1 || cout < 1) return 0;
    const long long nvox = (long long)D * H * W;
    if (wgrad_cm_ok(W, nvox)) {
        // the channel-major copies of dY and X, then what the blocked form needs
        return align256((size_t)nvox * cout * 2) + align256((size_t)nvox * cin * 2) +
               sur_bwd_weight_blocked_work_bytes(D, H, W, cin, cout);
    }
    return (size_t)wgrad_chunks(nvox) * 27 * cin * cout * sizeof(float);
}

size_t sur_bwd_weight_blocked_work_bytes(int D, int H, int W, int cin, int cout) {
    if (D < 1 || H < 1 || W < 1 || cin < 1 || cout < 1) return 0;
    const long long nvox = (long long)D * H * W;
    if (!wgrad_cm_ok(W, nvox)) return 0;
    // chunk partials, then the group sums of the partials
    const int nch = wgrad_cm_chunks(nvox, cin, cout);
    return align256((size_t)nch * 27 * cin * cout * sizeof(float)) + (size_t)(nch / 32 + 1) * 27 * cin * cout * sizeof(float);
}

// Weight gradient from the blocked copies, partials and their fixed-order sums in `work`.
static int wgrad_from_blocked(const bf16_t* dyc, const bf16_t* xc, float* dw, char* work, int D, int H, int W, int cin,
                              int cout, hipStream_t s) {
    const long long nvox = (long long)D * H * W;
    const long long n = 27LL * cin * cout;
    const int nch = wgrad_cm_chunks(nvox, cin, cout);
    const int chunk_len = (int)(nvox / nch);
    float* part = (float*)work;
    const long long nwaves = (long long)nch * (cout / 32) * ((cin + 31) / 32) * 9;
    hipLaunchKernelGGL(k_conv_wgrad_cm, dim3((unsigned)ceil_div(nwaves, 4)), dim3(256), 0, s, dyc, xc, part, D, H, W,
                       cin, cout, chunk_len, (int)nwaves);
    if (nch >= 64) {
        // two levels (groups of 32 chunks, then the groups), each in a fixed order
        const int G = 32, ng = nch / G;
        float* q = (float*)(work + align256((size_t)nch * 27 * cin * cout * sizeof(float)));
        hipLaunchKernelGGL(k_sum_chunk_groups, dim3(grid1(n), ng), dim3(256), 0, s, (const float*)part, q, n, G);
        hipLaunchKernelGGL(k_sum_chunks, dim3(grid1(n)), dim3(256), 0, s, (const float*)q, dw, n, ng);
    } else {
        hipLaunchKernelGGL(k_sum_chunks, dim3(grid1(n)), dim3(256), 0, s, (const float*)part, dw, n, nch);
    }
    NSLGF_LAUNCH_CHECK();
    return NSLGF_OK;
}

int sur_conv3d_bwd_weight(nslgf_t h, const void* dy, const void* x, void* dw, void* work, int D, int H, int W, int cin,
                          int cout, void* stream) {
    SUR_ENTER(h);
    NSLGF_TRY(conv_shape_ok(D, H, W, cin, cout));
    NSLGF_CHECK_ARG(dy && x && dw && work, "sur_conv3d_bwd_weight: null pointer");
    NSLGF_CHECK_ARG(a16(dy) && a16(x) && a16(dw) && a16(work), "sur_conv3d_bwd_weight: tensors must be 16-byte aligned");
    const long long nvox = (long long)D * H * W;
    hipStream_t s = (hipStream_t)stream;
    const long long n = 27LL * cin * cout;
    if (wgrad_cm_ok(W, nvox)) {
        char* base = (char*)work;
        bf16_t* dyc = (bf16_t*)base;
        bf16_t* xc = (bf16_t*)(base + align256((size_t)nvox * cout * 2));
        char* rest = (char*)xc + align256((size_t)nvox * cin * 2);
        hipLaunchKernelGGL(k_to_blocked8, dim3(ceil_div(nvox / 8 * (cout / 8), 256)), dim3(256), 0, s,
                           (const bf16_t*)dy, dyc, nvox / 8, cout);
        hipLaunchKernelGGL(k_to_blocked8, dim3(ceil_div(nvox / 8 * (cin / 8), 256)), dim3(256), 0, s,
                           (const bf16_t*)x, xc, nvox / 8, cin);
        return wgrad_from_blocked(dyc, xc, (float*)dw, rest, D, H, W, cin, cout, s);
    }
    const int nch = wgrad_chunks(nvox);
    const int chunk_len = (int)(nvox / nch);
    const long long waves = (long long)nch * 27 * (cout / 32) * ((cin + 31) / 32);
    hipLaunchKernelGGL(k_conv_wgrad, dim3(ceil_div(waves, 4)), dim3(256), 0, s, (const bf16_t*)dy, (const bf16_t*)x,
                       (float*)work, D, H, W, cin, cout, chunk_len, nch);
    hipLaunchKernelGGL(k_sum_chunks, dim3(grid1(n)), dim3(256), 0, s, (const float*)work, (float*)dw, n, nch);
    NSLGF_LAUNCH_CHECK();
    return NSLGF_OK;
}

int sur_conv3d_bwd_weight_blocked(nslgf_t h, const void* dyb, const void* xb, void* dw, void* work, int D, int H, int W,
                                  int cin, int cout, void* stream) {
    SUR_ENTER(h);
    NSLGF_TRY(conv_shape_ok(D, H, W, cin, cout));
    NSLGF_CHECK_ARG(dyb && xb && dw && work, "sur_conv3d_bwd_weight_blocked: null pointer");
    NSLGF_CHECK_ARG(a16(dyb) && a16(xb) && a16(dw) && a16(work), "sur_conv3d_bwd_weight_blocked: tensors must be 16-byte aligned");
    NSLGF_CHECK_ARG(wgrad_cm_ok(W, (long long)D * H * W), "sur_conv3d_bwd_weight_blocked: needs W % 8 == 0 and D*H*W % 16 == 0");
    return wgrad_from_blocked((const bf16_t*)dyb, (const bf16_t*)xb, (float*)dw, (char*)work, D, H, W, cin, cout,
                              (hipStream_t)stream);
}

int sur_cast_bf16_ex(nslgf_t h, const void* src, const void* act, void* y, void* yb, long long nvox, int c, void* stream) {
    SUR_ENTER(h);
    NSLGF_CHECK_ARG(src && y && nvox >= 0 && nvox % 8 == 0 && c > 0 && c % 8 == 0,
                    "sur_cast_bf16_ex: need src, y, nvox % 8 == 0, c % 8 == 0");
    NSLGF_CHECK_ARG(a16(src) && a16(act) && a16(y) && a16(yb), "sur_cast_bf16_ex: tensors must be 16-byte aligned");
    if (nvox == 0) return NSLGF_OK;
    hipLaunchKernelGGL(k_cast_ex, dim3(ceil_div(nvox / 8 * (c / 8), 256)), dim3(256), 0, (hipStream_t)stream,
                       (const float*)src, (const float*)act, (bf16_t*)y, (bf16_t*)yb, nvox / 8, c);
    NSLGF_LAUNCH_CHECK();
    return NSLGF_OK;
}

int sur_cast_bf16_up(nslgf_t h, const void* coarse, double scale, const void* skip, const void* act, void* y,
                     void* yb, int D, int H, int W, int c, void* stream) {
    SUR_ENTER(h);
    NSLGF_CHECK_ARG(coarse && skip && y && D > 0 && H > 0 && W > 0 && D % 2 == 0 && H % 2 == 0 && W % 2 == 0 &&
                        c > 0 && c % 8 == 0 && ((long long)D * H * W) % 8 == 0,
                    "sur_cast_bf16_up: need coarse, skip, y, even D, H, W with D*H*W % 8 == 0, c % 8 == 0");
    NSLGF_CHECK_ARG(a16(coarse) && a16(skip) && a16(act) && a16(y) && a16(yb),
                    "sur_cast_bf16_up: tensors must be 16-byte aligned");
    const long long nvox = (long long)D * H * W;
    hipLaunchKernelGGL(k_cast_up, dim3(ceil_div(nvox / 8 * (c / 8), 256)), dim3(256), 0, (hipStream_t)stream,
                       (const float*)coarse, (float)scale, (const float*)skip, (const float*)act, (bf16_t*)y,
                       (bf16_t*)yb, nvox / 8, c, D, H, W);
    NSLGF_LAUNCH_CHECK();
    return NSLGF_OK;
}

int sur_to_blocked8(nslgf_t h, const void* x, void* xb, long long nvox, int c, void* stream) {
    SUR_ENTER(h);
    NSLGF_CHECK_ARG(x && xb && x != xb && nvox >= 0 && nvox % 8 == 0 && c > 0 && c % 8 == 0,
                    "sur_to_blocked8: need x != xb, nvox % 8 == 0, c % 8 == 0");
    NSLGF_CHECK_ARG(a16(x) && a16(xb), "sur_to_blocked8: tensors must be 16-byte aligned");
    if (nvox == 0) return NSLGF_OK;
    hipLaunchKernelGGL(k_to_blocked8, dim3(ceil_div(nvox / 8 * (c / 8), 256)), dim3(256), 0, (hipStream_t)stream,
                       (const bf16_t*)x, (bf16_t*)xb, nvox / 8, c);
    NSLGF_LAUNCH_CHECK();
    return NSLGF_OK;
}

int sur_weight_transpose(nslgf_t h, const void* w, void* wt, int cin, int cout, void* stream) {
    SUR_ENTER(h);
    NSLGF_CHECK_ARG(w && wt && w != wt && cin > 0 && cout > 0, "sur_weight_transpose: bad arguments");
    const long long n = 27LL * cin * cout;
    hipLaunchKernelGGL(k_wtranspose, dim3(grid1(n)), dim3(256), 0, (hipStream_t)stream, (const bf16_t*)w, (bf16_t*)wt,
                       cin, cout);
    NSLGF_LAUNCH_CHECK();
    return NSLGF_OK;
}

#define SUR_ELEMWISE(call)                                                                         \
    SUR_ENTER(h);                                                                                  \
    NSLGF_CHECK_ARG(n >= 0, "surrogate: negative size");                                           \
    if (n == 0) return NSLGF_OK;                                                                   \
    call;                                                                                          \
    NSLGF_LAUNCH_CHECK();                                                                          \
    return NSLGF_OK;

int sur_cast_bf16(nslgf_t h, const void* x, void* y, long long n, void* stream) {
    SUR_ELEMWISE(hipLaunchKernelGGL(k_cast_bf16, dim3(grid1(n)), dim3(256), 0, (hipStream_t)stream, (const float*)x,
                                    (bf16_t*)y, n))
}
int sur_relu_bwd(nslgf_t h, const void* y, void* g, long long n, void* stream) {
    SUR_ELEMWISE(hipLaunchKernelGGL(k_relu_bwd, dim3(grid1(n)), dim3(256), 0, (hipStream_t)stream, (const float*)y,
                                    (float*)g, n))
}
int sur_add(nslgf_t h, const void* a, const void* b, void* o, long long n, void* stream) {
    SUR_ELEMWISE(hipLaunchKernelGGL(k_add, dim3(grid1(n)), dim3(256), 0, (hipStream_t)stream, (const float*)a,
                                    (const float*)b, (float*)o, n))
}

static int resample_ok(int D, int H, int W, int c) {
    NSLGF_CHECK_ARG(D >= 2 && H >= 2 && W >= 2 && D % 2 == 0 && H % 2 == 0 && W % 2 == 0 && c >= 1,
                    "surrogate: resampling needs even fine sizes");
    return NSLGF_OK;
}

int sur_pool2_fwd(nslgf_t h, const void* x, void* y, int D, int H, int W, int c, void* stream) {
    SUR_ENTER(h);
    NSLGF_TRY(resample_ok(D, H, W, c));
    const long long n = (long long)(D / 2) * (H / 2) * (W / 2) * c;
    hipLaunchKernelGGL(k_pool2_fwd, dim3(grid1(n)), dim3(256), 0, (hipStream_t)stream, (const float*)x, (float*)y, D, H,
                       W, c);
    NSLGF_LAUNCH_CHECK();
    return NSLGF_OK;
}
int sur_pool2_bwd(nslgf_t h, const void* gy, void* gx, int D, int H, int W, int c, void* stream) {
    SUR_ENTER(h);
    NSLGF_TRY(resample_ok(D, H, W, c));
    const long long n = (long long)D * H * W * c;
    hipLaunchKernelGGL(k_pool2_bwd, dim3(grid1(n)), dim3(256), 0, (hipStream_t)stream, (const float*)gy, (float*)gx, D,
                       H, W, c);
    NSLGF_LAUNCH_CHECK();
    return NSLGF_OK;
}
int sur_up2_fwd(nslgf_t h, const void* x, void* y, int D, int H, int W, int c, void* stream) {
    SUR_ENTER(h);
    NSLGF_TRY(resample_ok(D, H, W, c));
    const long long n = (long long)D * H * W * c;
    hipLaunchKernelGGL(k_up2_fwd, dim3(grid1(n)), dim3(256), 0, (hipStream_t)stream, (const float*)x, (float*)y, D, H, W,
                       c);
    NSLGF_LAUNCH_CHECK();
    return NSLGF_OK;
}
int sur_up2_bwd(nslgf_t h, const void* gy, void* gx, int D, int H, int W, int c, void* stream) {
    SUR_ENTER(h);
    NSLGF_TRY(resample_ok(D, H, W, c));
    const long long n = (long long)(D / 2) * (H / 2) * (W / 2) * c;
    hipLaunchKernelGGL(k_up2_bwd, dim3(grid1(n)), dim3(256), 0, (hipStream_t)stream, (const float*)gy, (float*)gx, D, H,
                       W, c);
    NSLGF_LAUNCH_CHECK();
    return NSLGF_OK;
}

int sur_mse(nslgf_t h, const void* pred, const void* target, void* grad, void* partial, long long nvox, int c, int used,
            void* stream) {
    SUR_ENTER(h);
    NSLGF_CHECK_ARG(pred && target && grad && partial && nvox > 0 && used >= 1 && used <= c, "sur_mse: bad arguments");
    int sh = 0;
    while (sh < 8 && (4 << sh) < c) ++sh;
    if ((4 << sh) == c && a16(grad))
        hipLaunchKernelGGL(k_mse<true>, dim3(1024), dim3(256), 0, (hipStream_t)stream, (const float*)pred,
                           (const float*)target, (float*)grad, (double*)partial, nvox, c, used, sh);
    else
        hipLaunchKernelGGL(k_mse<false>, dim3(1024), dim3(256), 0, (hipStream_t)stream, (const float*)pred,
                           (const float*)target, (float*)grad, (double*)partial, nvox, c, used, 0);
    NSLGF_LAUNCH_CHECK();
    return NSLGF_OK;
}

int sur_mse_cast(nslgf_t h, const void* pred, const void* target, void* partial, void* y, void* yb, long long nvox,
                 int c, int used, void* stream) {
    SUR_ENTER(h);
    NSLGF_CHECK_ARG(pred && target && partial && y && nvox > 0 && nvox % 8 == 0 && c > 0 && c % 8 == 0 && used >= 1 &&
                        used <= c,
                    "sur_mse_cast: need pred, target, partial, y, nvox % 8 == 0, c % 8 == 0, 1 <= used <= c");
    NSLGF_CHECK_ARG(a16(y) && a16(yb), "sur_mse_cast: tensors must be 16-byte aligned");
    hipLaunchKernelGGL(k_mse_cast, dim3(1024), dim3(256), 0, (hipStream_t)stream, (const float*)pred,
                       (const float*)target, (bf16_t*)y, (bf16_t*)yb, (double*)partial, nvox, c, used);
    NSLGF_LAUNCH_CHECK();
    return NSLGF_OK;
}

int sur_adam(nslgf_t h, void* w, void* wb, const void* g, void* m, void* v, long long n, float lr, float b1, float b2,
             float eps, int t, void* stream) {
    SUR_ENTER(h);
    NSLGF_CHECK_ARG(w && wb && g && m && v && n > 0 && t >= 1, "sur_adam: bad arguments");
    const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
    hipLaunchKernelGGL(k_adam, dim3(grid1(n)), dim3(256), 0, (hipStream_t)stream, (float*)w, (bf16_t*)wb, (const float*)g,
                       (float*)m, (float*)v, n, lr, b1, b2, eps, c1, c2);
    NSLGF_LAUNCH_CHECK();
    return NSLGF_OK;
}

int sur_pack_input(nslgf_t h, const void* om, void* x, int D, int H, int W, double scale, double feat, void* stream) {
    SUR_ENTER(h);
    NSLGF_CHECK_ARG(om && x && D > 0 && H > 0 && W > 0, "sur_pack_input: bad arguments");
    const long long nvox = (long long)D * H * W;
    hipLaunchKernelGGL(k_pack_input, dim3(grid1(nvox)), dim3(256), 0, (hipStream_t)stream, (const double*)om,
                       (bf16_t*)x, nvox, scale, feat);
    NSLGF_LAUNCH_CHECK();
    return NSLGF_OK;
}
int sur_pack_input_pair(nslgf_t h, const void* om, const void* delta, void* x, int D, int H, int W, double scale,
                        double dscale, double feat, void* stream) {
    SUR_ENTER(h);
    NSLGF_CHECK_ARG(om && delta && x && D > 0 && H > 0 && W > 0, "sur_pack_input_pair: bad arguments");
    const long long nvox = (long long)D * H * W;
    hipLaunchKernelGGL(k_pack_input_pair, dim3(grid1(nvox)), dim3(256), 0, (hipStream_t)stream, (const double*)om,
                       (const double*)delta, (bf16_t*)x, nvox, scale, dscale, feat);
    NSLGF_LAUNCH_CHECK();
    return NSLGF_OK;
}
int sur_combine3(nslgf_t h, const void* a, const void* b, const void* c, void* out, long long n, double ca, double cb,
                 double cc, void* stream) {
    SUR_ENTER(h);
    NSLGF_CHECK_ARG(a && b && out && n > 0, "sur_combine3: bad arguments");
    hipLaunchKernelGGL(k_combine3, dim3(grid1(n)), dim3(256), 0, (hipStream_t)stream, (const double*)a,
                       (const double*)b, (const double*)c, (double*)out, n, ca, cb, cc);
    NSLGF_LAUNCH_CHECK();
    return NSLGF_OK;
}
int sur_pack_target(nslgf_t h, const void* f, void* t, int D, int H, int W, double scale, void* stream) {
    SUR_ENTER(h);
    NSLGF_CHECK_ARG(f && t && D > 0 && H > 0 && W > 0, "sur_pack_target: bad arguments");
    const long long nvox = (long long)D * H * W;
    hipLaunchKernelGGL(k_pack_target, dim3(grid1(nvox)), dim3(256), 0, (hipStream_t)stream, (const double*)f, (float*)t,
                       nvox, scale);
    NSLGF_LAUNCH_CHECK();
    return NSLGF_OK;
}
int sur_unpack_update(nslgf_t h, const void* base, const void* y, void* out, int D, int H, int W, int c, double scale,
                      void* stream) {
    SUR_ENTER(h);
    NSLGF_CHECK_ARG(base && y && out && c >= 3 && scale != 0.0, "sur_unpack_update: bad arguments");
    const long long nvox = (long long)D * H * W;
    hipLaunchKernelGGL(k_unpack_update, dim3(grid1(nvox)), dim3(256), 0, (hipStream_t)stream, (const double*)base,
                       (const float*)y, (double*)out, nvox, c, 1.0 / scale);
    NSLGF_LAUNCH_CHECK();
    return NSLGF_OK;
}

int sur_mfma_selftest(nslgf_t h, const void* a, const void* b, void* c, void* stream) {
    SUR_ENTER(h);
    NSLGF_CHECK_ARG(a && b && c, "sur_mfma_selftest: null pointer");
    hipLaunchKernelGGL(k_mfma_selftest, dim3(1), dim3(64), 0, (hipStream_t)stream, (const bf16_t*)a, (const bf16_t*)b,
                       (float*)c);
    NSLGF_LAUNCH_CHECK();
    return NSLGF_OK;
}

}  // extern "C"
