/*
 * blp_oracle.h -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously-correct FP64 CPU implementation of the method of
 * MacLachlan, Madden & Nhan, "A Boundary-Layer Preconditioner for Singularly
 * Perturbed Convection Diffusion" (arXiv 2108.13468): the upwind 5-point
 * discretisation on a tensor Shishkin mesh (Sec. 3, eqs. tau exponential and
 * the 2D stencil), the block upper-triangular boundary-layer preconditioner
 * (Sec. 3.1, eq. 2D blocks), the corner multigrids for two exponential
 * layers and for one parabolic and one exponential layer (Sec. 3.2) and
 * FGMRES (Sec. 3.3).
 *
 * Only tests/, the smoke check and the CPU-baseline leg of the benchmark may
 * load this library.  It shares no code, header or table with the HIP path.
 *
 * Layout: unknowns are interior nodes (i, j), 1 <= i, j <= nx (ny), stored
 * x-fastest: v[(j-1)*nx + (i-1)].
 */
#ifndef BLP_ORACLE_H
#define BLP_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

/* One axis of the Shishkin mesh (eq. tau 1D / tau exponential):
 * tau = min(1/2, sigma*eps*ln(N)/clow); N/2 uniform cells on [0,tau] and N/2
 * on [tau,1].  nodes[0..N], widths[1..N] (widths[0] is set to 0).
 * Returns tau. */
double orc_mesh_axis(int N, double eps, double sigma, double clow,
                     double *nodes, double *widths);

/* General layer-adapted axis: nl cells on the layer [0, tau], N - nl equal
 * cells on [tau, 1].  kind 0: Shishkin, tau = min(nl/N, sigma eps ln N /
 * clow), equal layer cells; kind 1: Bakhvalov-Shishkin, graded layer cells
 * equidistributing exp(-clow x / (sigma eps)) (uniform mesh when
 * sigma eps ln N / clow >= nl/N).  Returns tau. */
double orc_mesh_axis_ex(int N, double eps, double sigma, double clow, int kind, int nl,
                        double *nodes, double *widths);
/* The same with the axis's layer type: parabolic = 0 as above; parabolic = 1
 * (Sec. 3, eq. tau parabolic) uses sqrt(eps) in place of eps / clow:
 * tau = min(nl/N, sigma sqrt(eps) ln N). */
double orc_mesh_axis_layer(int N, double eps, double sigma, double clow, int kind, int nl,
                           int parabolic, double *nodes, double *widths);

/* Opaque problem: the full grid operator plus its corner multigrid levels. */
typedef struct orc_problem orc_problem;

/* Build the problem.  c1x[0..N] = c1 at x-nodes, c2y[0..N] = c2 at y-nodes,
 * r_int = r at the (N-1)^2 interior nodes (x-fastest).  All copied. */
orc_problem *orc_create(int N, double eps, double sigma, double clow_x,
                        double clow_y, const double *c1x, const double *c2y,
                        const double *r_int);
/* The same on the general mesh of orc_mesh_axis_ex (kind, nl on both axes);
 * the layer side of each axis is then i <= nl.  NULL for nl outside
 * [2, N-2] or an unknown kind. */
orc_problem *orc_create_ex(int N, double eps, double sigma, double clow_x,
                           double clow_y, int kind, int nl, const double *c1x,
                           const double *c2y, const double *r_int);
/* The same with the layer type at y = 0: ylayer 0 exponential, 1 parabolic
 * (the case c2 = 0 of Sec. 3: y-axis mesh of eq. tau parabolic, corner
 * multigrid with x-semicoarsening, see orc_par_corner_mg). */
orc_problem *orc_create_px(int N, double eps, double sigma, double clow_x,
                           double clow_y, int kind, int nl, int ylayer,
                           const double *c1x, const double *c2y, const double *r_int);
void orc_destroy(orc_problem *p);
int orc_y_layer(const orc_problem *p);

int orc_n(const orc_problem *p);             /* (N-1)^2 */
int orc_num_levels(const orc_problem *p);    /* corner multigrid levels */
int orc_level_size(const orc_problem *p, int l);
void orc_nodes(const orc_problem *p, double *x, double *y); /* N+1 each */

/* Stencil of row (i,j) of the fine operator, 1 <= i,j <= N-1:
 * out = {W, E, S, Nn, C}. */
void orc_stencil(const orc_problem *p, int i, int j, double *out5);

/* y = A x and y = A^T x on the full grid. */
void orc_apply_A(const orc_problem *p, const double *x, double *y);
void orc_apply_AT(const orc_problem *p, const double *x, double *y);

/* CSR export of A (row-major, column indices ascending).  Arrays sized by
 * the caller: rowptr n+1, col/val 5n. Returns nnz. */
int orc_csr(const orc_problem *p, int *rowptr, int *col, double *val);

/* Preconditioner options. */
typedef struct {
  int corner;      /* 0: exact corner solve (the idealised M-hat), 1: multigrid */
  int mg_fixed;    /* >0: exactly this many V-cycles; 0: adaptive rule */
  double mg_rtol;  /* adaptive rule: stop when ||b - A_CC z||_2 <= mg_rtol ||b||_2 */
  int mg_maxcyc;   /* cap on cycles for the adaptive rule */
} orc_prec_opts;

typedef struct {
  long applies;
  long mg_cycles_total;
  int mg_cycles_min, mg_cycles_max;
} orc_prec_stats;

/* z = M^{-1} b (transpose = 0) or z = M^{-T} b (transpose = 1). */
void orc_prec_apply(orc_problem *p, const orc_prec_opts *o, int transpose,
                    const double *b, double *z, orc_prec_stats *st);

/* Individual region solves of the forward preconditioner, for pins.  Each
 * reads b on its region and the already-computed z values it couples to,
 * and writes z on its region only. */
void orc_solve_I(const orc_problem *p, const double *b, double *z);
void orc_solve_Y(const orc_problem *p, const double *b, double *z);
void orc_solve_X(const orc_problem *p, const double *b, double *z);

/* Corner multigrid on level 0 (the corner block A_CC), vectors of size
 * (N/2)^2.  Returns cycles used.  transpose selects the cycle for A_CC^T. */
int orc_corner_mg(orc_problem *p, int transpose, int fixed_cycles,
                  double rtol, int maxcyc, const double *b, double *z);
/* Exact corner solve (banded LU of A_CC or A_CC^T). */
void orc_corner_exact(orc_problem *p, int transpose, const double *b, double *z);
/* Level-l operator apply, restriction (fine level l -> l+1) and
 * interpolation (coarse l+1 -> fine l), and one downstream Gauss-Seidel
 * sweep on level l, for pins. */
void orc_level_apply(const orc_problem *p, int l, const double *x, double *y);
void orc_level_restrict(const orc_problem *p, int l, const double *rf, double *bc);
void orc_level_interp(const orc_problem *p, int l, const double *zc, double *zf);
void orc_level_gs(const orc_problem *p, int l, const double *b, double *z);

/* Parabolic-case corner multigrid (Sec. 3.2): V(1,1) cycles with
 * x-semicoarsening, Galerkin 9-point coarse operators on the rescaled
 * corner block S A_CC (S = diag(hbar_i kbar_j)), operator-induced
 * interpolation, downstream Gauss-Seidel; stops when the rescaled residual
 * has fallen by rtol (or after fixed_cycles > 0 cycles).  Returns the
 * cycles used, -1 for a problem without the parabolic layer.  Level l has
 * (h >> l) x h nodes; the per-level accessors below are for pins:
 * a9[9 k + 3 (dj+1) + (di+1)] couples node k = (j-1) nx + (i-1) to
 * (i+di, j+dj); wl, wr are the weights of odd fine nodes toward coarse
 * nodes (i-1)/2 and (i+1)/2. */
int orc_par_corner_mg(orc_problem *p, int fixed_cycles, double rtol, int maxcyc,
                      const double *b, double *z);
int orc_par_num_levels(const orc_problem *p);
int orc_par_level_nx(const orc_problem *p, int l);
void orc_par_level_stencil(const orc_problem *p, int l, double *a9);
void orc_par_level_weights(const orc_problem *p, int l, double *wl, double *wr);
void orc_par_level_apply(const orc_problem *p, int l, const double *x, double *y);
void orc_par_level_gs(const orc_problem *p, int l, const double *b, double *z);
void orc_par_level_restrict(const orc_problem *p, int l, const double *rf, double *bc);
void orc_par_level_interp(const orc_problem *p, int l, const double *zc, double *zf);

/* FGMRES (Saad's flexible GMRES with modified Gram-Schmidt), right
 * preconditioned, x0 = 0. */
typedef struct {
  double tol;        /* stopping tolerance */
  int absolute;      /* 0: ||r|| <= tol ||F||; 1: ||r|| <= tol */
  int restart;       /* m */
  int maxit;         /* cap on total inner iterations */
  int precond;       /* 0: none (identity), 1: boundary-layer M */
  int transpose;     /* 0: solve A u = F; 1: solve A^T u = F with M^T */
  int scaled;        /* 1: run on D^{-1/2} A D^{-1/2} y = D^{-1/2} F, u = D^{-1/2} y
                        (D = diag A); tol, history and true_res then refer to
                        the scaled system */
  orc_prec_opts prec;
  int stop_on_estimate; /* 1: a restart cycle whose residual estimate met the
                           tolerance ends the solve without the true-residual
                           confirmation (the paper's Sec. 3.3 runs) */
} orc_gmres_opts;

typedef struct {
  int iterations;    /* inner iterations (preconditioner applies) */
  int restarts;      /* completed restart cycles */
  int converged;
  double true_res;   /* ||F - A u||_2 at exit */
  double norm_F;
  long mg_cycles_total;
  int mg_cycles_min, mg_cycles_max;
} orc_gmres_info;

/* hist (may be NULL, else length maxit+1): hist[0] = ||r0||, hist[k] =
 * residual estimate after inner iteration k. */
int orc_fgmres(orc_problem *p, const orc_gmres_opts *o, const double *F,
               double *u, orc_gmres_info *info, double *hist);

/* Problem data helpers (problem statement, Sec. 3 and the workloads). */
/* F_ij = sum_{k=1..K, l=1..L} a[(l-1)*K + (k-1)] sin(k pi x_i) sin(l pi y_j) */
void orc_sine_series(int N, const double *x, const double *y, int K, int L,
                     const double *a, double *F);
/* g_kl = sum_ij lam_ij sin(k pi x_i) sin(l pi y_j) (adjoint of the above) */
void orc_sine_project(int N, const double *x, const double *y, int K, int L,
                      const double *lam, double *g);
/* r_ij = sum_pq R[q*m+p] phi_p(x_i) phi_q(y_j), hat functions on m uniform
 * control nodes of [0,1]. */
void orc_bilinear(int N, const double *x, const double *y, int m,
                  const double *R, double *r);
/* G[q*m+p] = sum_ij w_ij phi_p(x_i) phi_q(y_j) (adjoint of the above) */
void orc_bilinear_project(int N, const double *x, const double *y, int m,
                          const double *w, double *G);

/* ---- The one-dimensional method (Sec. 2) -------------------------------- */

/* -eps u'' - c u' + r u = f on (0,1), u(0) = u(1) = 0, upwind stencil
 * (eq. stencil_1d) on a mesh with widths w[1..N] (w[k] = x_k - x_{k-1}, from
 * orc_mesh_axis_ex), c[0..N] and r[0..N] at the nodes; unknowns are nodes
 * 1..N-1; the layer set L is nodes 1..nl (transition node included). */
typedef struct orc1_problem orc1_problem;
orc1_problem *orc1_create(int N, double eps, const double *w, const double *c,
                          const double *r, int nl);
void orc1_destroy(orc1_problem *p);
int orc1_n(const orc1_problem *p);
void orc1_stencil(const orc1_problem *p, int i, double *out3); /* W, C, E of row i */
void orc1_apply_A(const orc1_problem *p, const double *v, double *y);
/* U^E = A^{-1} f (Thomas, no pivoting) */
void orc1_solve_A(const orc1_problem *p, const double *f, double *u);
/* z = M^{-1} b with M of eq. block_M; the tridiagonal M itself (rows of n) */
void orc1_prec_apply(const orc1_problem *p, const double *b, double *z);
void orc1_prec_matrix(const orc1_problem *p, double *sub, double *diag, double *sup);

typedef struct {
  double K, g;  /* stop when ||F - A u_k||_inf <= K g (Sec. 2.4) */
  int maxit;    /* no restart: at most maxit iterations */
  int left;     /* 1: M on the left (M^{-1} A); 0: on the right (A M^{-1}) */
} orc1_gmres_opts;
typedef struct {
  int iterations, converged;
  double res_inf; /* ||F - A u||_inf at exit */
} orc1_gmres_info;
/* Unrestarted preconditioned GMRES from u = 0.  hist (may be NULL, maxit+1
 * doubles): the inf-norm residual after each iteration.  Returns 0 when the
 * test was met. */
int orc1_gmres(const orc1_problem *p, const orc1_gmres_opts *o, const double *F, double *u,
               orc1_gmres_info *info, double *hist);

#ifdef __cplusplus
}
#endif
#endif
