/*
 * nslgf.h -- C ABI of the MI355X fast-LGF Navier-Stokes hot path.
 *
 * The library computes, on one GPU, the operations of the fast lattice Green's function (LGF)
 * method for viscous incompressible flow on unbounded staggered grids (Liska & Colonius):
 * the free-space LGF convolution that inverts the 7-point Laplacian, the integrating factor
 * E(alpha) of the discrete heat equation, and the stages of the integrating-factor half-explicit
 * Runge-Kutta (IF-HERK) step with its exact projection; around them, the velocity refresh and its
 * cadence, the active-domain block weights and classification, and the volume integrals of an
 * isolated vortex ring.
 *
 * Conventions shared by every call
 * --------------------------------
 * Box.  The computational box holds nx * ny * nz cells.  Every scalar field (a cell field, or one
 *   component of a face or edge field) is a dense array [nz][ny][nx] with x fastest; vector fields
 *   are three such arrays back to back, components (1), (2), (3).  Values outside the box are zero
 *   (the mask operators of Sec. 4.1); every output is produced on the box only.
 * Memory.  All field pointers are DEVICE pointers (hipMalloc / torch CUDA tensors) on the
 *   handle's device, owned by the caller, 256-byte aligned, and must not alias unless a call says
 *   so.  The library owns its tables and workspaces (allocated lazily, freed by nslgf_destroy;
 *   the plan of each box size, dtype and FFT-plan choice, with its spectrum and convolution
 *   workspaces, stays cached for the handle's lifetime).
 * Precision.  dtype NSLGF_F64 (double) or NSLGF_F32 (float) for the field data.  Tables (the LGF,
 *   its spectrum, the integrating-factor weights) are always built in FP64; the FP32 path rounds
 *   them once.
 * Streams.  `stream` is a hipStream_t passed as void* (NULL = the default stream).  Calls enqueue
 *   work and return without synchronising; results are ready in stream order.  Table builds and
 *   workspace allocations happen on first use and synchronise the stream once.
 *   Calls that return host values (max_cell_speed, max_component_abs, flow_diagnostics,
 *   block_weights, herk_run) synchronise the stream; calls without a handle run on the host only.
 * Errors.  Every call returns NSLGF_OK (0) or a negative code; nothing aborts and no exception
 *   crosses the ABI.  nslgf_last_error() gives a thread-local message for the last failure.
 *   A handle is not thread-safe: one host thread at a time per handle.
 */
#ifndef NSLGF_H
#define NSLGF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum nslgf_status {
    NSLGF_OK = 0,
    NSLGF_EINVAL = -1,       /* bad argument (size, pointer, alpha < 0, unsupported box) */
    NSLGF_ENOMEM = -2,       /* device allocation failed */
    NSLGF_EHIP = -3,         /* a HIP runtime call failed */
    NSLGF_EUNSUPPORTED = -4, /* valid request this build does not handle */
    NSLGF_ESTATE = -5,       /* stages called out of order */
    NSLGF_ENONFINITE = -6    /* a guarded step or herk_check found a non-finite value (NaN or Inf) */
};

enum nslgf_dtype { NSLGF_F64 = 0, NSLGF_F32 = 1 };

enum nslgf_scheme { NSLGF_SCHEME_A = 0, NSLGF_SCHEME_B = 1, NSLGF_SCHEME_C = 2 };

typedef struct nslgf_ctx *nslgf_t;

/* Create a handle bound to HIP device `device` (tables, plans and workspaces live there). */
int nslgf_create(nslgf_t *h, int device);
/* Free every device allocation of the handle.  Waits for the device first. */
int nslgf_destroy(nslgf_t h);
/* Message of the last failing call on this host thread ("" if none). */
const char *nslgf_last_error(void);
/* Library version string. */
const char *nslgf_version(void);

/*
 * Lattice Green's function of the 7-point Laplacian (Appendix B):
 *   g(n) = -int_0^inf e^{-6t} I_{n1}(2t) I_{n2}(2t) I_{n3}(2t) dt,  -6 g(n) + sum_neighbours g = delta_n0.
 * lgf_value evaluates g on the host with the same method the GPU table builder uses (quadrature of
 * the Bessel integral for |n| < 40, the far-field expansion beyond).  Writes *out; returns 0.
 */
int lgf_value(int n1, int n2, int n3, double *out);

/*
 * Build (or rebuild) the LGF table and its zero-padded spectrum for a box of nx*ny*nz cells
 * (Appendix B; preprocessing done once per box size).  The kernel is the LGF on the padded
 * lattice of Px*Py*Pz points, P >= 2n - 1 per axis (the smallest supported 2,3,5-smooth size), made
 * even by wrapping; its real spectrum is stored by symmetry.  `dtype` selects the precision of the
 * stored spectrum (built in FP64).  Sizes 1 <= n <= 256 per axis.  Returns NSLGF_EINVAL otherwise.
 * lgf_convolve builds the table lazily; calling this first only moves the cost.
 */
int lgf_table(nslgf_t h, int nx, int ny, int nz, int dtype, void *stream);

/*
 * LGF convolution (Sec. 2.2, Eq. dpoisson_conv): for each component q < ncomp,
 *     dst_q(n) = dx^2 * sum_{m in box} g(n - m) src_q(m),   n in box,
 * i.e. dst = L^{-1} src for the dimensional Laplacian (dx^2 L a = -6a + neighbours) with uniform
 * conditions at infinity; the sources outside the box are zero.  Computed exactly (to rounding) by
 * a zero-padded FFT convolution.  src, dst: device arrays [ncomp][nz][ny][nx] of `dtype`; src and
 * dst must not overlap.  ncomp in 1..3.
 */
int lgf_convolve(nslgf_t h, const void *src, void *dst, int ncomp, int nx, int ny, int nz, double dx,
                 int dtype, void *stream);

/*
 * Allocation-free form of lgf_convolve, for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the same operation, plan and
 * kernels (results equal lgf_convolve's bit for bit), with the two convolution workspaces taken from a
 * fixed device array of NSLGF_NOALLOC_SCRATCH_BYTES that the library holds on each device it runs on
 * until the process ends; the call makes no hipMalloc, hipFree or other allocating call.  The box's
 * plan must exist: call lgf_table(h, nx, ny, nz, dtype) first, under the same FFT-plan choice
 * (NSLGF_ESTATE otherwise).  The workspaces take
 *     ncomp * nz * (ny + Py) * XP * 2 * sizeof(dtype) bytes (+ alignment),  XP = Px/2 + 1 rounded up to 8,
 * NSLGF_EINVAL beyond the array (it holds, for example, one FP64 component of a 128^3 box or three FP32
 * components of a 96^3 box).
 * Every call on a device shares that device's array and leaves its last contents there: calls that
 * overlap in time on one device (concurrent streams, several host threads or handles) race; calls in
 * one stream are ordered and safe.  Per-kernel profiling is not recorded for this call.
 */
#define NSLGF_NOALLOC_SCRATCH_BYTES (128u << 20)
int lgf_convolve_noalloc(nslgf_t h, const void *src, void *dst, int ncomp, int nx, int ny, int nz, double dx,
                         int dtype, void *stream);

/*
 * Integrating factor (Sec. 2.3, Eqs. if_def and ddifussion_soln; kernel of Appendix B):
 *     dst_q(n) = sum_{m in box} prod_j w[|n_j - m_j|] src_q(m),  w[k] = e^{-2 alpha} I_k(2 alpha),
 * i.e. dst = M E(alpha) M src, the solution operator of the discrete heat equation over
 * alpha = kappa (t - tau) / dx^2.  The 1D kernel is truncated where its tail falls below the
 * rounding of the dtype.  alpha must be >= 0 (NSLGF_EINVAL otherwise; E(-alpha) is unbounded).
 * src == dst (in place) is allowed.  Arrays [ncomp][nz][ny][nx], ncomp in 1..6.
 */
int if_apply(nslgf_t h, const void *src, void *dst, int ncomp, int nx, int ny, int nz, double alpha,
             int dtype, void *stream);

/*
 * IF-HERK state of one box (Sec. 3.2 with the projection of Sec. 3.3, masked as in Sec. 5).
 * The caller fills the scalars and the pointers; `work` must hold nslgf_state_bytes() bytes of
 * device memory.  u: face velocity [3][nz][ny][nx] (in: u_k; out after the last stage: u_{k+1});
 * d: cell field [nz][ny][nx] (out: total pressure d_{k+1}).  n_buf >= 0 is the buffer width: the
 * nonlinear term and the pressure source are restricted to the box shrunk by n_buf cells on every
 * side (the solution and support domains of Sec. 5, Eqs. rhs_final and dpoisson_final).
 * stage_done counts the stages already applied (0 before the first stage).
 *
 * Step guard (optional, guard != 0): after the projection of every stage a check kernel takes, in FP64
 * whatever the dtype, the largest |Dbar u^i| over the cells at least `margin` cells from every box
 * face and counts the non-finite values of u^i (and of d in the last stage); margin = guard_margin
 * when > 0, else n_buf + r_i + 1 with r_i the radius of the stage's integrating factor (inside the
 * support domain the projection leaves no divergence, and H^i carries the buffer's divergence r_i
 * cells inwards).  The last stage reads the result back (one stream synchronisation), stores the
 * largest value of the three stages in div_max and returns NSLGF_ENONFINITE if any value was not
 * finite.  With block domains (supp_blocks) set, choose guard_margin so that the checked cells lie in
 * the support.
 */
typedef struct nslgf_state {
    int nx, ny, nz;
    int dtype;      /* enum nslgf_dtype */
    int scheme;     /* enum nslgf_scheme */
    int n_buf;
    double dx, dt, re, t;
    void *u;
    void *d;
    void *work;
    int stage_done; /* managed by herk_stage */
    int guard;      /* 1: check every stage's projection in FP64 and test for non-finite values */
    /* Optional active domain as unions of blocks (Sec. 4.2, 4.3): device arrays of one byte per block of
     * block^3 cells tiling the box from its origin (bx = ceil(nx / block), by, bz; x fastest; 1 = in the
     * domain).  When set they replace the box shrunk by n_buf: supp_blocks for the pressure source,
     * soln_blocks for the nonlinear term.  The caller owns them (e.g. the masks of classify_blocks,
     * copied to the device) and keeps them unchanged while steps that use them run.  block must be
     * 1..256 when either is set. */
    const unsigned char *supp_blocks;
    const unsigned char *soln_blocks;
    int block;
    int guard_margin; /* cells left out next to the box faces by the guard's divergence check (0: automatic) */
    double div_max;   /* out (guarded steps): largest FP64 |Dbar u^i| over the checked cells, all stages */
} nslgf_state;

/* Bytes of device workspace one state needs for its box and dtype. */
size_t nslgf_state_bytes(int nx, int ny, int nz, int dtype);

/*
 * One stage i (1-based, 1..3) of the IF-HERK step (Sec. 3.2):
 *     g^i = -a~_ii dt Ntilde(u^{i-1}),  r^i = q^i + dt sum_{j<i} a~_ij w^{i,j} + g^i,
 *     d^i = L^{-1} Dbar r^i (= -L^{-1} G^T r^i),  u^i = H^i (r^i - G d^i),
 *     w^{i,i} = (g^i - G d^i) / (a~_ii dt),  H^i = E((c~_i - c~_{i-1}) dt / (dx^2 Re)),
 * with the final-stage form of the footnote of Sec. 3.2 in the last stage.  The last stage also
 * writes u_{k+1} into st->u, d_{k+1} = d^s / (a~_ss dt) into st->d and advances st->t by dt.
 * Stages must be called in order 1, 2, 3 (NSLGF_ESTATE otherwise); stage 1 restarts a step.
 */
int herk_stage(nslgf_t h, nslgf_state *st, int stage, void *stream);

/* The three stages of one step (Scheme A, B or C per st->scheme). */
int herk_step(nslgf_t h, nslgf_state *st, void *stream);

/*
 * FP64 check of a state's fields (the projection's divergence check kept in FP64 for both dtypes):
 * *div_max = max |Dbar u| over the cells at least max(margin, 1) cells from every box face, the
 * difference quotients formed in FP64 from the stored values of u; non-finite values of u and d are
 * counted over the whole box.  Returns NSLGF_ENONFINITE (with *div_max set to the maximum over the
 * finite values) if there is any, else NSLGF_OK.  Synchronises `stream`.
 */
int herk_check(nslgf_t h, const nslgf_state *st, int margin, double *div_max, void *stream);

/*
 * One IF-HERK step of each of n independent states (boxes of any supported sizes and dtypes, each
 * with its own u, d and work; none may share them), as one launch: the first call captures the n
 * steps into a HIP graph (of batched passes, or of per-problem branches; see nslgf_set_batch_mode) and
 * later calls with the same states and step parameters replay it.  Results equal n herk_step calls bit
 * for bit.
 * Advances every st->t by its dt.  Builds missing LGF spectra first (synchronising the stream).
 * Guarded states are checked inside the graph and read back after it (one synchronisation); the call
 * returns NSLGF_ENONFINITE if any of them saw a non-finite value.
 */
int herk_step_batched(nslgf_t h, nslgf_state *const *sts, int n, void *stream);

/*
 * Form of the batched graph.  NSLGF_BATCH_PASSES (the default): the states whose steps launch the same
 * kernels with the same grids (boxes of one size, dtype and scheme whose integrating factors have the
 * same radii) form a group, and every kernel of the step runs as ONE launch over the whole group, reading
 * each problem's arguments from a device table; the groups run on concurrent branch streams.  Steps
 * that use a kernel without a batched form (the step guard, integrating-factor radii above 12) make the
 * call fall back to NSLGF_BATCH_PER_PROBLEM: each state's kernels on a branch stream of its own.
 * nslgf_batch_info reports the last captured graph: *groups (0 for the per-problem form) and *launches
 * (its kernel launches).  Results are identical in both forms.
 */
enum nslgf_batch_mode { NSLGF_BATCH_PASSES = 0, NSLGF_BATCH_PER_PROBLEM = 1 };
int nslgf_set_batch_mode(nslgf_t h, int mode);
int nslgf_batch_info(nslgf_t h, int *groups, int *launches);

/*
 * Vor2Vel (Sec. 4.1, Eqs. vel_vor and vel_refresh): a = -L^{-1} w per component, u = Cbar a.
 * w: edge vorticity [3][nz][ny][nx]; u: face velocity [3][nz][ny][nx] (must not overlap w).
 */
int vor2vel(nslgf_t h, const void *w, void *u, int nx, int ny, int nz, double dx, int dtype, void *stream);

/*
 * Truncation error of the masked integrating factor (Appendix D, Eq. if_finite_error): for a uniform
 * unit field on a half-space whose mask keeps the points k >= 1 along one axis, the deficit of
 * M E(alpha) M at the point k is the 1D kernel mass at distances >= k,
 *     d_alpha(k) = sum_{n >= k} e^{-2 alpha} I_n(2 alpha).
 * (The printed index of the sum is garbled; this is the sum the stated mask gives.)  Host only, no
 * handle.  NSLGF_EINVAL for alpha < 0 or not finite, k < 1, or a null out.
 */
int if_trunc_error(double alpha, int k, double *out);

/*
 * Velocity refresh cadence (Sec. 4.4 with Appendix D): q steps apply integrating factors that compose
 * to E(q beta), beta = dt / (dx^2 Re), and the solution domain starts n_buf points inside the box, so
 * the error there after q steps is estimated by umax d_{q beta}(n_buf + 1), umax the largest magnitude
 * of any velocity component on the solution domain.  *q_max = the largest q <= q_cap whose estimate
 * is <= eps (q_cap when umax or beta is 0; 0 when one step already exceeds eps).  Host only.
 * NSLGF_EINVAL for beta < 0, n_buf < 0, umax < 0, eps <= 0, q_cap < 1 or a null q_max.
 */
int refresh_interval(double beta, int n_buf, double umax, double eps, int q_cap, int *q_max);

/*
 * *out = the largest |u^(q)| over the three components of the face field u [3][nz][ny][nx] on the box
 * shrunk by n_buf points (the umax of refresh_interval).  Synchronises `stream`.
 */
int max_component_abs(nslgf_t h, const void *u, int nx, int ny, int nz, int n_buf, int dtype, double *out,
                      void *stream);

/*
 * Velocity refresh (Sec. 4.4): the velocity on the box is recomputed from the vorticity on the support
 * domain (the box shrunk by n_buf points) with Vor2Vel, in place:
 *     w = M_supp C u,  a = -L^{-1} w,  u = Cbar a.
 * u: face velocity [3][nz][ny][nx].  Uses handle-owned temporaries (two 3-component fields).
 */
int velocity_refresh(nslgf_t h, void *u, int nx, int ny, int nz, int n_buf, double dx, int dtype, void *stream);

/*
 * nsteps IF-HERK steps of st (herk_step each), refreshing the velocity with velocity_refresh after
 * every q_max steps (Sec. 4.4); q_max = refresh_interval(dt / (dx^2 Re), n_buf, umax, eps, q_cap) with
 * umax = max_component_abs of st->u, taken at the start and again after each refresh (each takes a
 * stream synchronisation).  The refresh works in st->work.  *refreshes (may be null) = the number of
 * refreshes done.  NSLGF_EINVAL for nsteps < 0, eps <= 0, q_cap < 1, or when q_max is 0 (the buffer
 * is too thin for eps; the footnote of Sec. 4.4 excludes that case).
 */
int herk_run(nslgf_t h, nslgf_state *st, int nsteps, double eps, int q_cap, int *refreshes, void *stream);

/*
 * Volume integrals of an isolated vortex ring (Sec. 6.2, Eq. int_quantities, u_inf = 0) of the face
 * velocity u [3][nz][ny][nx], with the vorticity w = M_supp C u: zero outside the box and on the edges
 * closer than n_buf points to a face (n_buf >= 1 removes the outermost edges, where the curl of the
 * zero-extended velocity sees a spurious jump):
 *     out[0..2] impulse I = 1/2 int x cross w     out[3] kinetic energy K = int u . (x cross w)
 *     out[4] enstrophy E = 1/2 int |w|^2          out[5] helicity J = int u . w
 *     out[6..8] centroid X = 1/2 int ((x cross w) . I / |I|^2) x   (NaN when I = 0)
 * Each integral is a sum over the box times dx^3.  I, E and X take every term at the edge of the
 * vorticity component it contains; K and J average u (two faces) and w (four edges) to the cell
 * centres.  origin[3] = coordinates of vertex (0, 0, 0); face (q) sits half a cell back on the two
 * other axes, edge (q) half a cell back along q.  The ring speed is the centroid's rate of change,
 * U = dX/dt (by differences of X between steps).  Sums in FP64 for both dtypes, reduced in a fixed
 * order (deterministic).  Synchronises `stream`.
 */
int flow_diagnostics(nslgf_t h, const void *u, int nx, int ny, int nz, int n_buf, double dx, const double *origin,
                     int dtype, double *out, void *stream);

/*
 * Block weights of the active domain (Sec. 4.3, Eq. weight_fun) for the face velocity u [3][nz][ny][nx]:
 * the box is tiled by blocks of nb^3 cells from its origin (Sec. 4.2; the last block along an axis may
 * be shorter), giving a block grid bx = ceil(nx/nb), by, bz; for each block (x fastest)
 *     mu = max |(C u)^(q)| over its edges and components,   nu = max |G^T Ntilde(u)| over its cells,
 * both over the points at least n_buf away from every box face (the values the finite box has
 * contaminated are left out, as the section does before taking the weights).  mu, nu: host arrays of
 * bx * by * bz doubles, owned by the caller.  Synchronises `stream`.
 */
int block_weights(nslgf_t h, const void *u, int nx, int ny, int nz, int nb, int n_buf, double dx, int dtype,
                  double *mu, double *nu, void *stream);

/*
 * Active-domain classification (Sec. 4.3, Eqs. d_supp, d_soln; Sec. 4.2, Eq. def_xsoln), host only:
 *     W = max(mu / max(mu), nu / max(nu))  (a term with a zero maximum counts as 0),
 *     supp = W > eps_supp,  soln = W > eps_soln,
 *     xsoln = every block at most n_xb blocks from a soln block along each of the three axes.
 * Arrays of bx * by * bz (x fastest), owned by the caller; W may be null; the masks get 0 or 1.
 * Comparing the masks with those of the previous step tells whether the domain must be re-initialised.
 */
int classify_blocks(const double *mu, const double *nu, int bx, int by, int bz, double eps_supp, double eps_soln,
                    int n_xb, double *W, unsigned char *supp, unsigned char *soln, unsigned char *xsoln);

/*
 * nsteps IF-HERK steps of st on an active domain of blocks (Sec. 4.3): at the beginning of every step
 * the block weights of st->u (block_weights with blocks of block^3 cells, leaving out the points
 * closer than st->n_buf to a box face) are classified (classify_blocks with eps_supp, eps_soln, n_xb)
 * into D_supp and D_soln, which restrict the step's pressure source and nonlinear term (the state's
 * supp_blocks / soln_blocks).  When either differs from the previous step's, the velocity is first
 * re-initialised from the vorticity on the new support (u = Cbar a, a = -L^{-1} M_supp C u,
 * Eq. vel_refresh); the first classification only sets the domain.  The masks of the run live in handle
 * memory; on return (also on failure) st->supp_blocks, soln_blocks and block are as on entry, so later
 * herk_step calls use the state's own domain again.  *reinits (may be null) = re-initialisations done; *edge_steps (may be
 * null) = steps whose D_xsoln reached the outermost block layer of the box (the box would have to grow
 * to hold the expanded domain).  Synchronises `stream` every step.
 */
int herk_run_adaptive(nslgf_t h, nslgf_state *st, int nsteps, int block, double eps_supp, double eps_soln, int n_xb,
                      int *reinits, int *edge_steps, void *stream);

/*
 * nsteps IF-HERK steps computed on an active box that follows the flow (Sec. 4.2 and 4.3 with the grid
 * update of Sec. 5).  st describes the whole grid G: u [3][nz][ny][nx] and d [nz][ny][nx] on G, whose
 * sizes must be multiples of block (st->work is not used: the box state lives in handle memory).  At the
 * beginning of every step, on the current box B of whole blocks (at first G):
 *   D_supp = {W > eps_supp}, D_soln = {W > eps_soln} united with D_supp (the domains are nested), from
 *   the block weights of u on B (block_weights with blocks of block^3 cells, leaving out the points
 *   closer than st->n_buf to a face of B); D_xsoln = every block of G at most n_xb blocks away from
 *   D_soln along each axis; the new box B' = the bounding box of D_xsoln (its blocks outside D_xsoln
 *   are computed too).  The first classification restricts u to B'; later, when D_supp or D_soln
 *   changed, u on B' is re-initialised from the vorticity on the new support, taken on B and copied to
 *   B' (u = Cbar a, a = -L^{-1} M_supp C u, Eq. vel_refresh).  The step runs on B' with the pressure
 *   source on D_supp and the nonlinear term on D_soln.
 * On return u and d on G hold the last box's values and zero elsewhere; st->t is advanced;
 * *reinits = re-initialisations, *regrids = box changes after the first step (both may be null);
 * box[0..5] (may be null) = the last box's first cell (x, y, z) and sizes (x, y, z).  Synchronises
 * `stream` every step.  The box state and its plans stay cached in the handle.
 */
int herk_run_active(nslgf_t h, nslgf_state *st, int nsteps, int block, double eps_supp, double eps_soln, int n_xb,
                    int *reinits, int *regrids, int *box, void *stream);

/*
 * Staggered-grid point operators of Appendix A on the box (inputs zero outside, outputs on the box):
 *   op NSLGF_OP_GRAD      G:     cells  -> faces   (src [nz][ny][nx], dst [3][...])
 *   op NSLGF_OP_DIV       Dbar:  faces  -> cells   (src [3][...],     dst [nz][ny][nx])
 *   op NSLGF_OP_CURL      C:     faces  -> edges
 *   op NSLGF_OP_CURL_BAR  Cbar:  edges  -> faces
 *   op NSLGF_OP_NONLINEAR Ntilde: faces -> faces (Eq. opr_def_nonlin, e = C f kept one layer
 *                          beyond the box)
 *   op NSLGF_OP_LAPLACIAN 7-point L per component (ncomp from 1 to 3 in `ncomp`)
 * src and dst must not overlap.
 */
enum nslgf_op {
    NSLGF_OP_GRAD = 0, NSLGF_OP_DIV = 1, NSLGF_OP_CURL = 2, NSLGF_OP_CURL_BAR = 3,
    NSLGF_OP_NONLINEAR = 4, NSLGF_OP_LAPLACIAN = 5
};
int stencil_apply(nslgf_t h, int op, const void *src, void *dst, int ncomp, int nx, int ny, int nz, double dx,
                  int dtype, void *stream);

/*
 * Maximum over cells of the cell-centred speed |u| (each face component averaged to the cell
 * centre), used for the CFL step size dt = CFL dx / max|u| (Sec. 6).  Writes one double to the
 * HOST pointer out (synchronises the stream).
 */
int max_cell_speed(nslgf_t h, const void *u, int nx, int ny, int nz, int dtype, double *out, void *stream);

/*
 * Per-kernel timing.  While enabled, every kernel the handle launches is bracketed by two HIP events
 * recorded on its launch stream; nslgf_profile_read reports, per kernel name, the number of launches
 * and their summed event-to-event duration in milliseconds (it waits for the recorded events).
 * enable = 1 starts (and clears) collection, 0 stops it.  index runs over the kernel names seen so
 * far; NSLGF_EINVAL past the last one.  name receives at most name_cap bytes, NUL-terminated.
 */
int nslgf_profile_enable(nslgf_t h, int enable);
/*
 * Radix plan of the strided (column) FFT passes of the convolution (Sec. 2.2's zero-padded FFT
 * convolution; the plan changes the order of rounding only) for padded lengths 256 and 512:
 *   0  narrow: 8 (length 256) or 16 (length 512) complex elements per thread, radix-4/8 passes,
 *      an LDS exchange between passes;
 *   1  wide: 16 or 32 elements per thread, radices 16 x 16 or 16 x 32, one exchange per transform;
 *   2  the narrow radices on 4 or 8 elements per thread (512-thread workgroups; in FP32 on tiles of
 *      8 columns, 64-byte row segments);
 *  -1  (the default) in FP32 narrow for the y passes and wide for the fused z pass; in FP64 narrow
 *      at length 256 and 2 at length 512;
 *  -2  (NSLGF_FFT_PLAN_AUTOTUNE) the autotuner: when a plan is built, every variant that exists for
 *      its y and z lengths is timed on the device on the plan's own shapes and the fastest is kept
 *      (the choice may differ between runs, so results may differ in the last bits).
 * A variant that does not exist for a dtype falls back to the default.  Applies to plans built after
 * the call (plans are cached per box, dtype and choice).  NSLGF_EINVAL outside -2 .. 2.
 */
#define NSLGF_FFT_PLAN_AUTOTUNE (-2)
int nslgf_set_fft_plan(nslgf_t h, int choice);
/* The column-plan variants (y and z passes) of the plan for this box and dtype under the handle's
 * current choice, building the plan (on `stream`) if needed; host outputs. */
int nslgf_plan_info(nslgf_t h, int nx, int ny, int nz, int dtype, void *stream, int *vy, int *vz);
/* Plain streaming copy of n elements of dtype (device pointers, no overlap, n * size a multiple of
 * 16 bytes, 16-byte aligned); the reference kernel whose hardware byte counters calibrate those of
 * the other kernels.  Profiled as "copy". */
int nslgf_copy(nslgf_t h, const void *src, void *dst, size_t n, int dtype, void *stream);
int nslgf_profile_read(nslgf_t h, int index, char *name, int name_cap, long long *calls, double *total_ms);

/*
 * Launch tuner.  Per box and dtype the library chooses the column-plan variants of the convolution
 * (see nslgf_set_fft_plan), the rows per workgroup of the fused x-y integrating-factor pass (32, 64,
 * 128, 256; a plane's rows are split into tiles of equal height up to that many), the outputs per thread
 * of the strided z pass (16, 32) and the workgroup shape of the point kernels (0: 64x4, 1: 128x2,
 * 2: 32x8, 3: 256x1 threads).  None of the launch shapes changes the arithmetic (results are
 * bit-identical); the column variants change the order of rounding only.
 *   NSLGF_TUNE_DEFAULT  the measured defaults: IF rows 32 for ny <= 128, 64 for ny <= 192, else 128;
 *                       z outputs 16 for nz <= 192, else 32; 64x4; the default column plans;
 *   NSLGF_TUNE_AUTO     the first use of a box and dtype times every choice on the device on zero fields
 *                       of that box (one synchronisation) and keeps the fastest.
 * Choices recorded for a box (tuned, or read by nslgf_tuning_load) are used in either mode, unless an
 * explicit column plan is set with nslgf_set_fft_plan.  nslgf_tuning_info returns, building or tuning
 * as needed, out[0..4] = y variant, z variant, IF rows, IF z outputs per thread, point-kernel shape.
 * nslgf_tuning_save writes every recorded choice as JSON (format "nslgf-tuning-1": one object per box
 * with nx, ny, nz, dtype "f64"/"f32", the padded lengths Px, Py, Pz, vy, vz, launch (1 if the launch
 * shapes were tuned), if_rows, if_seg, cell_shape); nslgf_tuning_load reads such a file (NSLGF_EINVAL for
 * a malformed file or an entry whose padded lengths or choices do not fit this library) and drops the
 * plans and batch graph that the loaded choices replace.
 */
enum nslgf_tune { NSLGF_TUNE_DEFAULT = 0, NSLGF_TUNE_AUTO = 1 };
int nslgf_set_tuning(nslgf_t h, int mode);
int nslgf_tuning_info(nslgf_t h, int nx, int ny, int nz, int dtype, void *stream, int *out);
int nslgf_tuning_save(nslgf_t h, const char *path);
int nslgf_tuning_load(nslgf_t h, const char *path);

#ifdef __cplusplus
}
#endif
#endif /* NSLGF_H */
