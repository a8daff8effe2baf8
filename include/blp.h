/*
 * blp.h -- C ABI of the MI355X boundary-layer-preconditioned FGMRES solver.
 *
 * Method: MacLachlan, Madden & Nhan, "A Boundary-Layer Preconditioner for
 * Singularly Perturbed Convection Diffusion" (arXiv 2108.13468).
 *
 * Problem (Sec. 1, eq. 2D):  -eps Lap u - c . grad u + r u = f  on (0,1)^2,
 * u = 0 on the boundary, eps in (0,1], c1 > 0, c2 >= 0, r >= 0 (Sec. 3).
 * Discretisation: upwind 5-point stencil (Sec. 3, 2D stencil) on the tensor
 * Shishkin mesh with N cells per axis, transition
 * tau = min(1/2, sigma eps ln(N) / clow) and N/2 uniform cells on each side
 * (Sec. 2.2 eq. tau 1D, Sec. 3 eq. tau exponential).
 *
 * Unknowns: the (N-1)^2 interior nodes (i, j), 1 <= i, j <= N-1, stored
 * x-fastest: index (j-1)(N-1) + (i-1).  Several right-hand sides are stacked
 * contiguously (stride (N-1)^2).
 *
 * Pointers: arguments documented "host" are read on the calling thread and
 * not kept; arguments documented "device" are device pointers (for example
 * torch.Tensor.data_ptr() of a CUDA/HIP tensor) read or written on the
 * stream given to blp_assemble.  The library copies every coefficient at
 * assemble time and keeps no caller pointer after a call returns.  All
 * device memory the library allocates belongs to the problem handle and is
 * freed by blp_destroy.
 *
 * Errors: every int-returning call returns BLP_OK (0), BLP_W_NOCONV (+1, a
 * solve stopped at its iteration cap; outputs hold the last iterate) or a
 * negative BLP_E_* code.  blp_strerror() names a code.  Calls on one handle
 * must not overlap in time (one host thread at a time per handle).
 */
#ifndef BLP_H
#define BLP_H

#ifdef __cplusplus
extern "C" {
#endif

#define BLP_OK 0
#define BLP_W_NOCONV 1
#define BLP_E_INVAL (-1)   /* argument outside the method's assumptions     */
#define BLP_E_NOMEM (-2)   /* device or host allocation failed              */
#define BLP_E_HIP (-3)     /* a HIP runtime call or kernel launch failed    */
#define BLP_E_STATE (-4)   /* call out of order (e.g. solve before setup)   */
#define BLP_E_NUMERIC (-5) /* NaN or Inf met in a residual norm             */
#define BLP_E_SCRATCH (-6) /* request larger than a fixed scratch buffer    */

typedef struct blp_problem blp_problem;

/* Coefficient fields.  kind:
 *   BLP_CONST     v[0]
 *   BLP_AXIS      N+1 nodal values along the field's own axis (c1 along x,
 *                 c2 along y); the paper's workloads have c1 = c1(x),
 *                 c2 = c2(y)
 *   BLP_NODAL     (N-1)^2 interior values, x-fastest (r only)
 *   BLP_BILINEAR  m x m controls on a uniform grid of [0,1]^2, x-fastest
 *                 (v[q*m + p] at (p/(m-1), q/(m-1))), hat-function
 *                 interpolation (r only)
 * All v are host pointers. */
#define BLP_CONST 0
#define BLP_AXIS 1
#define BLP_NODAL 2
#define BLP_BILINEAR 3
typedef struct {
  int kind;
  int m;
  const double *v;
} blp_field;

/* Mesh parameters.  The paper's mesh (Sec. 3 eq. tau exponential) is the
 * tensor Shishkin mesh: per axis, tau = min(1/2, sigma eps ln(N) / clow) and
 * N/2 equal cells on each side of it; clow_x <= c1 and clow_y <= c2 are the
 * lower bounds of the convection.  The workloads use sigma = 2, clow = 1; the
 * paper's Sec. 3.3 tests use sigma = 5/2.  Sec. 3 admits any fitted tensor
 * mesh with a transition point between the layer and the interior, and
 * Sec. 2.2 (remark on the general Shishkin mesh) lets the layer hold a
 * fraction q of the cells:
 *   kind         BLP_MESH_SHISHKIN: equal layer cells,
 *                tau = min(q, sigma eps ln(N) / clow);
 *                BLP_MESH_BAKHVALOV_SHISHKIN: tau = sigma eps ln(N) / clow
 *                and graded layer cells that make exp(-clow x / (sigma eps))
 *                fall in equal steps from 1 at x = 0 to 1/N at tau,
 *                x_i = -(sigma eps / clow) ln(1 - (1 - 1/N) i / (qN))
 *                (a uniform mesh when sigma eps ln(N) / clow >= q)
 *   layer_cells  qN, the cells on [0, tau] per axis (2 <= qN <= N-2;
 *                0 = N/2); the layer side of each axis (regions of Sec. 3.1)
 *                is then i <= qN, and the corner multigrid coarsens it by
 *                halving while the node count is even.
 *   y_layer      the layer at y = 0: BLP_LAYER_EXPONENTIAL (c2 > 0, as
 *                above) or BLP_LAYER_PARABOLIC (Sec. 3, the case c2 = 0:
 *                eq. tau parabolic, tau_y = min(q, sigma sqrt(eps) ln N),
 *                clow_y unused; the graded kind grades with the scale
 *                sigma sqrt(eps)).  A parabolic problem's corner block is
 *                solved by the semicoarsening multigrid of Sec. 3.2 (see
 *                blp_precondition).
 * The interior cells are equal in every case. */
#define BLP_MESH_SHISHKIN 0
#define BLP_MESH_BAKHVALOV_SHISHKIN 1
#define BLP_LAYER_EXPONENTIAL 0
#define BLP_LAYER_PARABOLIC 1
typedef struct {
  double sigma;
  double clow_x, clow_y;
  int kind;
  int layer_cells;
  int y_layer;
} blp_mesh_opts;

/* Mesh nodes of both axes: x[0..N], y[0..N] (host, N+1 doubles each), and
 * through tau (host, 2 doubles, may be NULL) the transition points tau_x,
 * tau_y.  opts may be NULL (the paper's Shishkin mesh, sigma = 2,
 * clow = 1).  Pure host computation in FP64.  Errors: BLP_E_INVAL for odd
 * N, N < 4, eps outside (0,1], non-positive sigma or clow, an unknown kind
 * or layer_cells outside its range. */
int blp_mesh(int N, double eps, const blp_mesh_opts *opts, double *x, double *y,
             double *tau);

/* Build the discrete operator on the device (Sec. 3, 2D stencil) and the
 * per-axis stencil tables; uploads r (BLP_BILINEAR controls are expanded to
 * nodal values by a kernel).  stream: a hipStream_t (NULL = default stream)
 * that every later call on this handle uses.  mesh may be NULL (see
 * blp_mesh_opts).  Errors: BLP_E_INVAL (odd N, N < 4 or N > 2048, eps
 * outside (0,1], c1 <= 0, c2 < 0, r < 0, NaN, bad field kind, bad mesh
 * options, or regions larger than the kernels hold: more than 1024 layer
 * cells or more than 1024 interior nodes per axis), BLP_E_NOMEM, BLP_E_HIP. */
int blp_assemble(int N, double eps, const blp_field *c1, const blp_field *c2,
                 const blp_field *r, const blp_mesh_opts *mesh, void *stream,
                 blp_problem **out);

/* Mesh nodes of an assembled problem (host arrays of N+1 doubles each). */
int blp_nodes(const blp_problem *p, double *x, double *y);

/* Preconditioner setup (Sec. 3.1 and 3.2; setup phase described in
 * Sec. 3.3): Thomas factorisations of the X and Y edge-layer lines (no
 * pivoting, Lemma diag_dom), the corner multigrid hierarchy and the FP32
 * copies used by the mixed-precision mode.  The hierarchy follows the
 * problem's layer at y = 0: two exponential layers, full coarsening with
 * rediscretised levels and FE rescaling; a parabolic layer, coarsening by
 * two in x only with Galerkin 9-point coarse operators of the
 * hbar_i kbar_j-rescaled corner block, operator-induced interpolation (each
 * odd column's row collapsed North-South) and its transpose as restriction,
 * built on the device in FP64.  Both smooth with downstream Gauss-Seidel,
 * one sweep before and after the coarse correction, four on the coarsest
 * level.
 *   mg_fixed  > 0: every corner solve runs exactly this many V(1,1) cycles
 *             (makes M a fixed linear operator; needed for M^T identities)
 *             = 0: stationary iteration until the corner residual of the
 *             rescaled system has dropped by mg_rtol (paper: 1e-3 for two
 *             exponential layers, 1e-2 with a parabolic one; o = NULL takes
 *             these), at most mg_maxcyc cycles.
 * The parabolic cycle has no transposed form: for such a problem every
 * transposed apply or solve (blp_prec_apply with transpose, the adjoint
 * solves) returns BLP_E_INVAL.
 * Calling it again on a preconditioned problem only replaces the options;
 * every later solve (single or batched) uses the new ones.
 * Errors: BLP_E_INVAL, BLP_E_NOMEM, BLP_E_HIP. */
typedef struct {
  int mg_fixed;
  double mg_rtol;
  int mg_maxcyc;
} blp_prec_opts;
int blp_precondition(blp_problem *p, const blp_prec_opts *opts);

/* Solver options.
 *   tol, absolute   stop when ||r|| <= tol (absolute) or <= tol ||F||
 *   scaled          1: the residual is that of the symmetrically Jacobi-
 *                   scaled system D^{-1/2} A D^{-1/2} (D = diag A), i.e.
 *                   ||D^{-1/2}(F - A u)||; 0: the plain residual ||F - A u||
 *   restart, maxit  FGMRES(restart), cap on total inner iterations
 *   precision       BLP_FP64, or BLP_MIXED: FP32 preconditioner, FP32
 *                   Krylov vectors and FP32-stored SpMV operands inside an
 *                   FP64 restarted outer loop (FP64 true residuals,
 *                   Hessenberg/Givens and solution)
 *   precond         1: boundary-layer preconditioner M; 0: none
 *   stop_on_estimate 0: a restart cycle ends when the FGMRES residual
 *                   estimate meets the tolerance, and the solve ends when the
 *                   true residual then does; 1: the estimate alone ends the
 *                   solve (the paper's Sec. 3.3 runs, which evaluate the
 *                   tolerance on FGMRES's own Euclidean residual norm); the
 *                   reported res is still the true residual */
#define BLP_FP64 0
#define BLP_MIXED 1
typedef struct {
  double tol;
  int absolute;
  int scaled;
  int restart;
  int maxit;
  int precision;
  int precond;
  int stop_on_estimate;
} blp_solve_opts;

typedef struct {
  int iterations;       /* inner iterations (preconditioner applies) */
  int restarts;         /* completed restart (outer) cycles */
  int converged;
  double res;           /* final true residual norm (per opts.scaled) */
  double norm_F;        /* norm of the right-hand side (per opts.scaled) */
  long mg_cycles_total; /* corner V-cycles over all applies */
  int mg_cycles_min, mg_cycles_max;
  double solve_ms;      /* wall time of the call */
} blp_solve_info;

/* Solve A U = F (Sec. 3.3: FGMRES, right preconditioned with M) from U = 0,
 * for nrhs right-hand sides sharing the operator.  F, U: device, nrhs
 * stacked vectors of (N-1)^2 doubles.  info: host, nrhs entries (may be
 * NULL).  hist: host, (maxit+1) doubles per right-hand side or NULL;
 * hist[0] = initial residual norm, hist[k] = residual estimate after inner
 * iteration k (FP64 mode; in mixed mode the outer true residuals are
 * recorded at restart boundaries).  Errors: BLP_E_STATE before
 * blp_precondition, BLP_E_INVAL, BLP_E_NUMERIC, BLP_E_HIP; BLP_W_NOCONV if
 * any right-hand side hit maxit. */
int blp_solve(blp_problem *p, int nrhs, const double *F, double *U,
              const blp_solve_opts *opts, blp_solve_info *info, double *hist);

/* Adjoint solve A^T Lambda = G with the transposed preconditioner M^T
 * (block lower triangular: corner cycle for A_CC^T, X lines bottom to top,
 * Y lines left to right, interior sweep from the bottom-left).  Same
 * arguments and errors as blp_solve. */
int blp_solve_adjoint(blp_problem *p, int nrhs, const double *G, double *Lambda,
                      const blp_solve_opts *opts, blp_solve_info *info,
                      double *hist);

/* Batched solves: S independent systems A_s U_s = F_s solved together
 * (the method of blp_solve for each; a batch is an execution schedule, not
 * a different method).  probs[s] is the assembled and preconditioned
 * problem of system s; one problem may appear several times (several
 * right-hand sides).  The batch owns each system's work vectors and Krylov
 * basis; the problems must outlive it and are only read.  All work runs on
 * `stream` (a hipStream_t, or NULL for the default stream).  Every kernel
 * launch covers all systems of one mesh size; the restart cycles of all
 * active systems start together and each system leaves a cycle (and the
 * launches) through its own gate when its estimate reaches the cycle
 * target, so each system follows exactly the iteration of its single solve.
 * opts (may be NULL): graphs = 1 replays the launches of one Krylov step from
 * HIP graphs captured on first use; autotune = 1 times the candidate kernel
 * variants of each mesh size once and keeps the fastest.  sweep_variant
 * (a test hook; 0 = default or the autotuner's choice): v > 0 runs every
 * triangular sweep of the batch in scheduling variant (v - 1) modulo the
 * number of variants its width has; all variants compute bit-identical
 * results.
 * Errors: BLP_E_INVAL (S < 1, NULL problem, sweep_variant < 0), BLP_E_STATE
 * (a problem not preconditioned), BLP_E_NOMEM, BLP_E_HIP. */
typedef struct blp_batch blp_batch;
typedef struct {
  int graphs;
  int autotune;
  int sweep_variant;
} blp_batch_opts;
int blp_batch_create(blp_problem *const *probs, int S, void *hip_stream,
                     const blp_batch_opts *opts, blp_batch **out);

/* F[s], U[s]: device vectors of system s ((N_s-1)^2 doubles; F and U host
 * arrays of S pointers).  info: host, S entries (may be NULL).  Same solve
 * options and errors as blp_solve (BLP_W_NOCONV if any system hit maxit);
 * also BLP_E_INVAL when the problems of the batch were preconditioned with
 * different blp_prec_opts (the corner cycle schedule is shared). */
int blp_batch_solve(blp_batch *b, const double *const *F, double *const *U,
                    const blp_solve_opts *opts, blp_solve_info *info);
/* Adjoint systems A_s^T L_s = G_s, as blp_solve_adjoint. */
int blp_batch_solve_adjoint(blp_batch *b, const double *const *G, double *const *L,
                            const blp_solve_opts *opts, blp_solve_info *info);
/* Device bytes held by the batch (work vectors, bases, launch plans). */
long long blp_batch_footprint(const blp_batch *b);
/* Text summary (NUL-terminated, truncated to len-1 bytes) of the batch's mesh
 * classes and of the kernel variants its launch plans use (the autotuner's
 * choices).  Returns the full length, or BLP_E_INVAL. */
int blp_batch_describe(const blp_batch *b, char *buf, int len);
/* Per-kernel-class timing of a batch's launches, as blp_timing (events on
 * the streams the launches run on; graphs are not replayed while it is on). */
int blp_batch_timing(blp_batch *b, int enable, double *ms, long long *launches,
                     double *bytes);
void blp_batch_destroy(blp_batch *b);

/* Single operator applications on one vector (device in/out, (N-1)^2
 * doubles), for tests: BLP_OP_A (y = A x), BLP_OP_AT (y = A^T x),
 * BLP_OP_MINV (y = M^{-1} x), BLP_OP_MINVT (y = M^{-T} x), and the FP32
 * preconditioner in FP64 arguments: BLP_OP_MINV32.  cycles (host, may be
 * NULL) receives the corner V-cycles used.  Errors: BLP_E_STATE,
 * BLP_E_INVAL, BLP_E_HIP. */
#define BLP_OP_A 0
#define BLP_OP_AT 1
#define BLP_OP_MINV 2
#define BLP_OP_MINVT 3
#define BLP_OP_MINV32 4
int blp_apply(blp_problem *p, int op, const double *x, double *y, int *cycles);

/* Right-hand side and gradient helpers for the sine-series forcing and the
 * bilinear reaction field (problem data of the workloads).
 * blp_sine_rhs:     F_ij = sum_{k<=K,l<=L} a[(l-1)K+(k-1)] sin(k pi x_i) sin(l pi y_j)
 *                   a: host K*L doubles; F: device (N-1)^2 doubles.
 * blp_sine_project: g_kl = sum_ij w_ij sin(k pi x_i) sin(l pi y_j)
 *                   (adjoint of blp_sine_rhs); w: device, g: host K*L.
 * blp_bilinear_project: G[q*m+p] = sum_ij w_ij phi_p(x_i) phi_q(y_j)
 *                   w: device (N-1)^2, G: host m*m.
 * blp_mul: out_ij = a_ij * b_ij (device vectors).
 * blp_reaction_gradient: the gradient of a misfit with respect to the
 *                   bilinear reaction controls, through the discrete adjoint:
 *                   A depends on r through its diagonal only, so
 *                   dJ/dR[q*m+p] = -sum_s sum_ij Lambda_s,ij U_s,ij phi_p(x_i) phi_q(y_j)
 *                   over the nrhs stacked pairs (Lambda_s, U_s) (device,
 *                   nrhs x (N-1)^2 each: adjoint solutions and solutions);
 *                   G: host m*m.  The sum over right-hand sides and the sign
 *                   are taken on the device. */
int blp_sine_rhs(blp_problem *p, int K, int L, const double *a, double *F);
int blp_sine_project(blp_problem *p, int K, int L, const double *w, double *g);
int blp_bilinear_project(blp_problem *p, int m, const double *w, double *G);
int blp_mul(blp_problem *p, const double *a, const double *b, double *out);
int blp_reaction_gradient(blp_problem *p, int m, int nrhs, const double *Lambda, const double *U,
                          double *G);

/* blp_sine_project without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving or optimisation
 * loops, harnesses that forbid hipMalloc).  Same arguments, result and
 * stream as blp_sine_project.  Its tables and partial sums live in a fixed
 * 4 MiB scratch array that the library holds on every GPU it runs on until
 * the process ends: K(N+1) + L(N+1) + K(N-1) + K L doubles, each part
 * rounded up to 256 bytes, must fit (K, L <= 64 always fit at N <= 2048).
 * The caller's current device must be the one the problem was assembled
 * on.  Calls on one GPU share its scratch array: calls that overlap in time
 * on one GPU (from several host threads, or on several streams) race.
 * Errors: BLP_E_INVAL, BLP_E_SCRATCH (tables larger than the scratch array),
 * BLP_E_STATE (another device current), BLP_E_HIP. */
int blp_sine_project_noalloc(blp_problem *p, int K, int L, const double *w, double *g);

/* The one-dimensional method (Sec. 2) for a batch of S independent problems
 *   -eps u'' - c u' + r u = f on (0,1), u(0) = u(1) = 0,
 * upwind stencil (eq. stencil_1d) on the layer-adapted mesh of
 * blp_mesh_opts (one axis: sigma, clow, kind, layer_cells), preconditioner
 * M of eq. block_M (A with the sub-diagonal of the interior block A_II
 * dropped, the coupling A_IL kept), unrestarted GMRES from u = 0 stopped
 * when ||F - A u||_inf <= K g(N) (Sec. 2.4).  One launch solves the whole
 * batch: one workgroup runs one problem's GMRES to the end on the device.
 *   probs[s]   N (even, 4..4096), eps in (0,1], mesh parameters, and host
 *              arrays c[0..N] (> 0) and r[0..N] (>= 0) at the nodes
 *   F[s], U[s] device, N-1 doubles each (nodes 1..N-1); host arrays of S
 *              pointers
 *   opts       maxit (1..128), left (1: M^{-1} A as the paper's MATLAB
 *              gmres; 0: A M^{-1}), K (<= 0: K = ||U^E||_inf from a direct
 *              tridiagonal solve on the device, as the paper suggests), g
 *              (<= 0: g(N) = ln(N)/N)
 *   info       host, S entries (may be NULL)
 * Device work memory and a pinned host staging buffer are kept per device
 * between calls, grown when a call needs more, and held until the process
 * ends; calls on one device run one at a time (each returns after its
 * stream has finished the batch).  Errors: BLP_E_INVAL, BLP_E_NOMEM,
 * BLP_E_HIP, BLP_E_NUMERIC; BLP_W_NOCONV if any problem reached maxit. */
typedef struct {
  int N;
  double eps;
  double sigma, clow;
  int kind, layer_cells;
  const double *c, *r;
} blp1d_problem;
typedef struct {
  int maxit;
  int left;
  double K, g;
} blp1d_opts;
typedef struct {
  int iterations, converged;
  double res_inf; /* ||F - A u||_inf at exit */
  double K;       /* the K used */
} blp1d_info;
int blp1d_solve(int S, const blp1d_problem *probs, const double *const *F, double *const *U,
                const blp1d_opts *opts, void *stream, blp1d_info *info);

/* Per-kernel-class timing with HIP events on the handle's stream.
 * enable = 1: discard earlier records and start recording an event pair
 * around every launch of the classes below; enable = 0: synchronise, stop
 * recording and write, per class, the summed kernel time in ms (ms[k]), the
 * number of launches (launches[k]) and the algorithmic bytes those launches
 * move (bytes[k]: words read and written that the algorithm needs, at the
 * precision of the launch).  Arrays have BLP_NCLASS entries; any may be NULL.
 * Classes (each the launches of one kernel family): 0 triangular sweeps
 * (interior region and every multigrid smoothing sweep; right-hand side in,
 * z out per node), 1 Gauss-Seidel right-hand-side pre-pass of the smoothing
 * sweeps (b and z in, folded right-hand side out), 2 edge-layer line solves
 * (b, z and two factor words per node), 3 other multigrid kernels (residual,
 * transfers, coarsest level, norms), 4 stencil SpMV / residual (x in, y
 * out), 5 Arnoldi and solution update, 6 layout gathers/scatters and corner
 * set-up.
 * Errors: BLP_E_INVAL, BLP_E_HIP. */
#define BLP_NCLASS 7
int blp_timing(blp_problem *p, int enable, double *ms, long long *launches,
               double *bytes);

/* Device bytes held by the handle. */
long long blp_footprint(const blp_problem *p);

void blp_destroy(blp_problem *p);
const char *blp_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif
