// Host-side launchers of the library's kernels (internal interface between the C-ABI layer and the
// kernel translation units).  Every launcher enqueues on `stream` and returns an nslgf status.
#pragma once

#include <cstring>
#include <vector>

#include "common.h"

namespace nslgf {

// ---- batched launches ----------------------------------------------------------------------------
// While a LaunchRecorder is installed on the calling thread, the launchers of the IF-HERK stage record
// their launches (the batched form of the kernel, one problem's grid and block, the arguments) instead
// of issuing them.  Problems whose records match position by position can then run every position as
// one launch over a device table of their arguments (the kernels read their arguments from the table
// entry of the problem their workgroup belongs to).
using BatchedLaunch = int (*)(const void* args, int nprob, dim3 grid, dim3 block, hipStream_t s);
struct LaunchRec {
    BatchedLaunch fn;
    dim3 grid, block;
    std::vector<unsigned char> args;
};
struct LaunchRecorder {
    std::vector<LaunchRec> recs;
    bool ok = true;  // false once a launch without a batched form was requested
};
LaunchRecorder*& launch_recorder();  // this thread's recorder (null: launch normally)
template <class A> inline void record_launch(BatchedLaunch fn, dim3 g, dim3 b, const A& a) {
    LaunchRec r{fn, g, b, std::vector<unsigned char>(sizeof(A))};
    std::memcpy(r.args.data(), &a, sizeof(A));
    launch_recorder()->recs.push_back(std::move(r));
}
// For launchers without a batched form: true (and the recording marked unusable) while recording.
inline bool recording_unsupported() {
    if (!launch_recorder()) return false;
    launch_recorder()->ok = false;
    return true;
}

// Validates a handle and makes its device current (used by entry points outside api.hip).
int enter_handle(nslgf_t h);

// Whether cell (i, j, k) of an nx x ny x nz box lies in the domain: the box shrunk by nbuf cells, or,
// when blocks is set, the union of the blocks of nb^3 cells marked 1 there (Sec. 4.2; x fastest).
__device__ __forceinline__ bool in_domain(int i, int j, int k, int nx, int ny, int nz, int nbuf,
                                          const unsigned char* blocks, int nb) {
    if (blocks) {
        const int bx = (nx + nb - 1) / nb, by = (ny + nb - 1) / nb;
        return blocks[((k / nb) * by + j / nb) * bx + i / nb] != 0;
    }
    return i >= nbuf && i < nx - nbuf && j >= nbuf && j < ny - nbuf && k >= nbuf && k < nz - nbuf;
}

// Launch shapes of one box and dtype, chosen by the launch tuner (or the defaults): they change
// the work split only, never the arithmetic, so every choice gives bit-identical results.
constexpr int kCellShapeCount = 4;  // point-kernel workgroups 64x4, 128x2, 32x8, 256x1 (x by y threads)
struct Tuning {
    int if_rows = 128;   // output rows per workgroup of the fused x-y integrating-factor pass (32 .. 256)
    int if_seg = 32;     // outputs per thread of the strided (z) integrating-factor pass (16 or 32)
    int cell_shape = 0;  // point-kernel workgroup shape index
};

// ---- FFT passes (lgf_conv.hip) ----------------------------------------------------------------
// Supported padded lengths P (2,3,5-smooth, even) of the zero-padded convolution.
bool fft_length_supported(int P);
int next_supported_length(int n);  // smallest supported P >= n, or -1

// Columns per workgroup of the column-tile kernel of length L for dtype (used for spectrum layout).
int col_tile_width(int L, int dtype);

// Root twiddle table exp(-2 pi i m / L), m < L, of the dtype (owned by the caller; filled by host).
int make_twiddles(int L, int dtype, void** dev_out);

struct RowPass {
    const void* in;
    void* out;
    long long nrows;      // rows per component
    long long in_row;     // element stride between rows (real elements for R2C input, complex for C2R input)
    long long out_row;
    long long in_comp, out_comp;  // component strides in elements
    int ncomp;
    int n_io;             // R2C: real inputs per row (rest zero); C2R: real outputs kept per row
    const void* tw_half;  // root table of length P/2 (complex FFT)
    const void* tw_full;  // root table of length P (real pre/post processing)
    // R2C only, when div_src is set: the input rows are not read from `in` but formed on load as the
    // masked divergence M_supp Dbar f of the 3-component face field div_src (box nx = n_io, ny, nz;
    // rows are (z, y) pairs, one component; points closer than div_nbuf to a box face give 0)
    const void* div_src;
    int div_ny, div_nz, div_nbuf;
    double div_idx;  // 1 / dx
    // when set, the support is these blocks of div_nb^3 cells (1 = support block, x fastest) instead of
    // the box shrunk by div_nbuf
    const unsigned char* div_blocks;
    int div_nb;
};
int launch_row_r2c(int P, int dtype, const RowPass& a, hipStream_t s);
int launch_row_c2r(int P, int dtype, const RowPass& a, hipStream_t s);

enum ColMode { COL_FWD = 0, COL_INV = 1, COL_CONV = 2 };
struct ColPass {
    const void* in;
    void* out;
    int ncols;            // valid columns (complex elements contiguous in memory)
    int nouter;           // independent column groups (grid y)
    long long in_outer, out_outer;  // element stride between groups
    long long in_row, out_row;      // element stride between transform elements
    long long in_comp, out_comp;
    int ncomp;
    int n_in, n_out;      // nonzero inputs / kept outputs along the transform
    const void* tw;       // root table of length L
    // COL_CONV only: real spectrum laid out [Py/2+1][khat_tiles][L/2+1][TBk], TBk = col_tile_width(L,
    // dtype) (column c in tile c / TBk); outer index ky folds to min(ky, outer_period - ky).
    const void* khat;
    int khat_tiles;
    int outer_period;
    double scale;
};
// variant: plan variant of lengths 256 and 512 (0 = default; see PlanV and col_variant_choice)
int launch_col(int L, int dtype, ColMode mode, const ColPass& a, hipStream_t s, int variant = 0);
int col_variant_choice(int L, int dtype, int choice, bool zpass);
constexpr int kColVariants = 3;  // variants 0 .. kColVariants - 1 (not all exist for every length and dtype)
bool col_variant_valid(int L, int dtype, int v);

// ---- LGF table (lgf_table.hip) ------------------------------------------------------------------
// Host evaluation of g(n) with the same method as the device table builder.
double lgf_value_host(int n1, int n2, int n3);
// Builds the real FP64 even kernel g on the Px*Py*Pz padded lattice into dev_kernel (caller allocates
// Px*Py*Pz doubles).
int build_padded_lgf(int Px, int Py, int Pz, double* dev_kernel, hipStream_t s);
// Extracts the real spectrum (times `scale`) from the complex FFT of the kernel (layout
// [Pz][Py][XP] complex double) into the column-tile layout used by COL_CONV, in dtype.
int extract_spectrum(const void* spec, int Px, int Py, int Pz, long long XP, double scale, int tb, int tiles,
                     int dtype, void* khat, hipStream_t s);

// ---- integrating factor (intfac.hip) ------------------------------------------------------------
// Host: w[k] = e^{-2 alpha} I_k(2 alpha), k = 0..r (returns r, the truncation radius for the dtype).
int if_weights(double alpha, int dtype, double* w, int wmax);
constexpr int kIfMaxRadius = 63;
constexpr int kIfFixedMaxRadius = 12;  // radii with compile-time passes (larger ones run the runtime-radius passes)
int launch_if_axis(int axis, int dtype, const void* in, void* out, int ncomp, int nx, int ny, int nz,
                   const double* w, int radius, hipStream_t s, int seg = 32);
// Projection of an IF-HERK stage applied while the fused x-y pass loads (Sec. 3.2, Eq. ifherk_aux_1
// and the w^{ii} update): the input is u = r - G dhat (r the 3-component p[0]), and where wnew is
// given, wnew = (u - (c_q q + c_w1 w1)) inv is written too (w1 may be null).
struct IfProject {
    const void* dhat;
    double idx;  // 1 / dx
    const void* q;
    const void* w1;
    double c_q, c_w1;
    void* wnew;
    double inv;
};
// Input of the fused x-y pass: c[0] p[0] + c[1] p[1] + c[2] p[2] (p[1], p[2] null: p[0] alone, c
// ignored), formed in FP64 and rounded once to the dtype; or, with proj, the projection of p[0].
struct IfCombine {
    const void* p[3];
    double c[3];
    const IfProject* proj = nullptr;
};
// x and y passes in one launch (no intermediate field in HBM), for radius 1 .. kIfFixedMaxRadius and
// nx <= 256 (else NSLGF_EUNSUPPORTED, launching nothing).  out must not overlap the inputs.
int launch_if_xy(int dtype, const IfCombine& cb, void* out, int ncomp, int nx, int ny, int nz, const double* w,
                 int radius, hipStream_t s, int rows = 128);

// ---- velocity refresh cadence (refresh.hip) -----------------------------------------------------
// d_a(k) = sum_{n >= k} e^{-2a} I_n(2a) (k >= 1, a >= 0)
double if_trunc_error_host(double alpha, int k);
// largest q <= q_cap with umax d_{q beta}(n_buf + 1) <= eps
int refresh_interval_host(double beta, int n_buf, double umax, double eps, int q_cap);

// ---- active domain (domain.hip) ---------------------------------------------------------------------
// W = max(mu / max mu, nu / max nu) (W may be null), supp = W > eps_supp, soln = W > eps_soln,
// xsoln = soln dilated by n_xb blocks along every axis (arrays of bx * by * bz, x fastest)
void classify_blocks_host(const double* mu, const double* nu, int bx, int by, int bz, double eps_supp, double eps_soln,
                          int n_xb, double* W, unsigned char* supp, unsigned char* soln, unsigned char* xsoln);

// ---- stencils (stencils.hip) --------------------------------------------------------------------
int launch_stencil(int op, int dtype, const void* src, void* dst, int ncomp, int nx, int ny, int nz, double dx,
                   hipStream_t s, int shape = 0);

// Fused IF-HERK stage kernels (herk.hip)
struct StageCoef {
    double c_q;          // coefficient of q in r (1)
    double c_w1, c_w2;   // dt * a~_{i1}, dt * a~_{i2}
    double c_g;          // -a~_{ii} dt
    int nbuf;            // the nonlinear term is restricted to the box shrunk by nbuf cells, or,
    const unsigned char* soln_blocks;  // when set, to these blocks of nb^3 cells (1 = solution block, x fastest)
    int nb;
    int copy_q;          // 1: copy u into q first and use it as q (stage 1: q^1 = u_k)
};
// r = c_q q + c_w1 w1 + c_w2 w2 + c_g M_soln Ntilde(u); (w pointers may be null)
int launch_stage_rhs(int dtype, const void* u, const void* q, const void* w1, const void* w2, void* r,
                     const StageCoef& c, int nx, int ny, int nz, double dx, hipStream_t s, int shape = 0);
// s = M_supp Dbar r
int launch_masked_div(int dtype, const void* r, void* sdiv, int nbuf, int nx, int ny, int nz, double dx,
                      hipStream_t s);
// rout = r - G dhat (rout may be r); w_new = (rout - base) * inv  where base = c_q q + c_w1 w1 + c_w2 w2
// (optional)
int launch_stage_project(int dtype, const void* r, void* rout, const void* dhat, const void* q, const void* w1,
                         const void* w2, double c_q, double c_w1, double c_w2, void* wnew, double inv, int nx, int ny,
                         int nz, double dx, hipStream_t s, int shape = 0);
// out = a*x + b*y + c*z (elementwise over n elements; y, z may be null)
int launch_axpby(int dtype, void* out, const void* x, double a, const void* y, double b, const void* z, double c,
                 long long n, hipStream_t s);
// plain 16-byte-vector copy of `bytes` (multiple of 16)
int launch_copy(const void* in, void* out, size_t bytes, hipStream_t s);
// e = M_supp C f (edges closer than nbuf points to a box face set to 0, or, when blocks is set, edges
// outside the marked blocks of nb^3 cells)
int launch_masked_curl(int dtype, const void* f, void* e, int nbuf, const unsigned char* blocks, int nb, int nx, int ny,
                       int nz, double dx, hipStream_t s, int shape = 0);
// per-workgroup maxima of |u^(q)| over the three components on the box shrunk by nbuf points
int launch_max_abs(int dtype, const void* u, int nbuf, int nx, int ny, int nz, double* dev_partial, int nblocks,
                   hipStream_t s);
// 15 raw sums of the vortex-ring integrals per workgroup into dev_partial[nblocks][15] (order in
// stencils.hip), vorticity restricted to the box shrunk by nbuf; origin = coordinates of vertex (0, 0, 0)
constexpr int kDiagnosticSums = 15;
int launch_diagnostics(int dtype, const void* u, int nbuf, int nx, int ny, int nz, double dx, const double origin[3],
                       double* dev_partial, int nblocks, hipStream_t s);
// per block of nb^3 cells: mu = max |(C u)^(q)|, nu = max |Dbar nl| (nl = Ntilde(u) on the box), over the
// points at least nbuf away from every box face; dev_mu, dev_nu hold one value per block (x fastest)
int launch_block_weights(int dtype, const void* u, const void* nl, int nx, int ny, int nz, int nb, int nbuf, double dx,
                         double* dev_mu, double* dev_nu, hipStream_t s);
// step guard (guard.hip): acc[0] = max (bits of a nonnegative double) of the FP64 |Dbar u| over the cells at
// least margin (>= 1) from every face, acc[1] += non-finite values of u (and d when set); reset clears both
int launch_guard_reset(unsigned long long* acc, hipStream_t s);
int launch_guard(int dtype, const void* u, const void* d, int nx, int ny, int nz, int margin, double dx,
                 unsigned long long* acc, hipStream_t s);
// active-box transfers (active.hip): dst = 0 over n elements; and the sub-box copy of ncomp components
// from the box sdim (x, y, z sizes) at offset soff to the box ddim at offset doff, extent ext (x, y, z)
int launch_zero(int dtype, void* dst, long long n, hipStream_t s);
int launch_copy_box(int dtype, const void* src, const int sdim[3], const int soff[3], void* dst, const int ddim[3],
                    const int doff[3], const int ext[3], int ncomp, hipStream_t s);
// max over cells of the cell-centred speed
int launch_max_speed(int dtype, const void* u, int nx, int ny, int nz, double* dev_partial, int nblocks,
                     hipStream_t s);

}  // namespace nslgf
