/*
 * blp_oracle_1d.c -- TEST INFRASTRUCTURE ONLY (see blp_oracle.h).
 *
 * Plain FP64 reference for the one-dimensional method of arXiv 2108.13468,
 * Sec. 2: the upwind discretisation of -eps u'' - c u' + r u = f on a
 * layer-adapted mesh (eq. stencil_1d, eq. tau 1D), the block preconditioner
 * M of eq. block_M (A with the sub-diagonal of the interior block A_II
 * dropped, the coupling A_IL kept) and unrestarted GMRES with the residual
 * stopping test of Sec. 2.4 (||F - A U^(k)||_inf <= K g(N)).
 *
 * Readings where the paper is silent:
 *  - the unknowns are the interior nodes 1..N-1 (the block sizes of eq.
 *    block_A count them as N);
 *  - the layer set L is nodes 1..nl, the transition node nl included
 *    (Sec. 2.3), nl = N/2 on the paper's mesh;
 *  - GMRES is preconditioned on the left, as the MATLAB gmres the paper
 *    used does when given M (a right-preconditioned variant is available);
 *  - K is the caller's (the paper takes K = ||U^E||_inf) and g(N) = ln(N)/N.
 */
#include "blp_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

struct orc1_problem {
  int N, n, nl;   /* n = N - 1 unknowns; rows 1..nl form the layer set L */
  double *W, *C, *E; /* row i (1-based) at index i-1; W of row 1 and E of row n unused */
};

orc1_problem *orc1_create(int N, double eps, const double *w, const double *c,
                          const double *r, int nl) {
  if (N < 4 || nl < 1 || nl > N - 2) return NULL;
  orc1_problem *p = calloc(1, sizeof(*p));
  p->N = N;
  p->n = N - 1;
  p->nl = nl;
  p->W = calloc(p->n, sizeof(double));
  p->C = calloc(p->n, sizeof(double));
  p->E = calloc(p->n, sizeof(double));
  /* eq. stencil_1d at node i: h_i = x_i - x_{i-1}, hbar_i = (h_i + h_{i+1}) / 2
   *   W = -eps / (h_i hbar_i)
   *   C =  eps / hbar_i (1/h_i + 1/h_{i+1}) + c_i / h_{i+1} + r_i
   *   E = -eps / (h_{i+1} hbar_i) - c_i / h_{i+1} */
  for (int i = 1; i <= p->n; ++i) {
    double hi = w[i], hn = w[i + 1];
    double hb = 0.5 * (hi + hn);
    p->W[i - 1] = -eps / (hi * hb);
    p->C[i - 1] = eps / hb * (1.0 / hi + 1.0 / hn) + c[i] / hn + r[i];
    p->E[i - 1] = -eps / (hn * hb) - c[i] / hn;
  }
  return p;
}

void orc1_destroy(orc1_problem *p) {
  if (!p) return;
  free(p->W);
  free(p->C);
  free(p->E);
  free(p);
}

int orc1_n(const orc1_problem *p) { return p->n; }

void orc1_stencil(const orc1_problem *p, int i, double *out3) {
  out3[0] = p->W[i - 1];
  out3[1] = p->C[i - 1];
  out3[2] = p->E[i - 1];
}

void orc1_apply_A(const orc1_problem *p, const double *v, double *y) {
  int n = p->n;
  for (int k = 0; k < n; ++k) {
    double s = p->C[k] * v[k];
    if (k > 0) s += p->W[k] * v[k - 1];
    if (k < n - 1) s += p->E[k] * v[k + 1];
    y[k] = s;
  }
}

/* Thomas algorithm for a tridiagonal system (sub a[k] on row k, diagonal
 * d[k], super e[k]), forward elimination then back substitution, no
 * pivoting (the matrices here are diagonally dominant M-matrices). */
static void thomas(int n, const double *a, const double *d, const double *e,
                   const double *f, double *u) {
  double *cp = malloc(sizeof(double) * n), *fp = malloc(sizeof(double) * n);
  cp[0] = e[0] / d[0];
  fp[0] = f[0] / d[0];
  for (int k = 1; k < n; ++k) {
    double den = d[k] - a[k] * cp[k - 1];
    cp[k] = e[k] / den;
    fp[k] = (f[k] - a[k] * fp[k - 1]) / den;
  }
  u[n - 1] = fp[n - 1];
  for (int k = n - 2; k >= 0; --k) u[k] = fp[k] - cp[k] * u[k + 1];
  free(cp);
  free(fp);
}

void orc1_solve_A(const orc1_problem *p, const double *f, double *u) {
  thomas(p->n, p->W, p->C, p->E, f, u);
}

/* z = M^{-1} b, eq. block_M: M equals A except that the sub-diagonal of the
 * interior block A_II is dropped (rows nl+2..n); row nl+1 keeps A_IL.  M is
 * tridiagonal, so the plain definition is a Thomas solve of it. */
void orc1_prec_apply(const orc1_problem *p, const double *b, double *z) {
  int n = p->n;
  double *a = malloc(sizeof(double) * n);
  for (int k = 0; k < n; ++k) {
    int row = k + 1;
    a[k] = row >= p->nl + 2 ? 0.0 : p->W[k];
  }
  thomas(n, a, p->C, p->E, b, z);
  free(a);
}

/* M as a tridiagonal matrix (for pins): sub, diagonal, super of each row. */
void orc1_prec_matrix(const orc1_problem *p, double *sub, double *diag, double *sup) {
  for (int k = 0; k < p->n; ++k) {
    sub[k] = (k + 1 >= p->nl + 2) ? 0.0 : p->W[k];
    diag[k] = p->C[k];
    sup[k] = p->E[k];
  }
}

static double dot1(int n, const double *a, const double *b) {
  double s = 0.0;
  for (int k = 0; k < n; ++k) s += a[k] * b[k];
  return s;
}

/* Unrestarted GMRES (Arnoldi with modified Gram-Schmidt, Givens rotations
 * with rho = hypot), from u = 0, preconditioned with M on the left (the
 * Krylov space of M^{-1} A, minimising ||M^{-1}(F - A u)||_2) or on the right
 * (of A M^{-1}, minimising ||F - A u||_2).  After every iteration the iterate
 * u_k is formed and the test ||F - A u_k||_inf <= K g is applied (Sec. 2.4).
 * hist[k] (may be NULL, length maxit+1) = ||F - A u_k||_inf. */
int orc1_gmres(const orc1_problem *p, const orc1_gmres_opts *o, const double *F, double *u,
               orc1_gmres_info *info, double *hist) {
  int n = p->n, m = o->maxit;
  double **V = malloc(sizeof(double *) * (m + 1));
  for (int k = 0; k <= m; ++k) V[k] = calloc(n, sizeof(double));
  double *H = calloc((size_t)(m + 1) * m, sizeof(double));
  double *cs = calloc(m, sizeof(double)), *sn = calloc(m, sizeof(double));
  double *g = calloc(m + 1, sizeof(double)), *y = calloc(m, sizeof(double));
  double *w = malloc(sizeof(double) * n), *t = malloc(sizeof(double) * n);
  double *R = malloc(sizeof(double) * n);
  double target = o->K * o->g;
  memset(info, 0, sizeof(*info));
  for (int k = 0; k < n; ++k) u[k] = 0.0;
  double rinf = 0.0;
  for (int k = 0; k < n; ++k) rinf = fmax(rinf, fabs(F[k]));
  if (hist) hist[0] = rinf;
  info->res_inf = rinf;
  if (rinf <= target) {
    info->converged = 1;
  } else {
    /* r0 = M^{-1} F (left) or F (right) */
    if (o->left)
      orc1_prec_apply(p, F, t);
    else
      memcpy(t, F, sizeof(double) * n);
    double beta = sqrt(dot1(n, t, t));
    for (int k = 0; k < n; ++k) V[0][k] = t[k] / beta;
    g[0] = beta;
    for (int j = 0; j < m; ++j) {
      if (o->left) {
        orc1_apply_A(p, V[j], t);
        orc1_prec_apply(p, t, w);
      } else {
        orc1_prec_apply(p, V[j], t);
        orc1_apply_A(p, t, w);
      }
      for (int i = 0; i <= j; ++i) {
        double hij = dot1(n, w, V[i]);
        H[i * m + j] = hij;
        for (int k = 0; k < n; ++k) w[k] -= hij * V[i][k];
      }
      double hn = sqrt(dot1(n, w, w));
      H[(j + 1) * m + j] = hn;
      if (hn > 0.0)
        for (int k = 0; k < n; ++k) V[j + 1][k] = w[k] / hn;
      for (int i = 0; i < j; ++i) {
        double a = H[i * m + j], b = H[(i + 1) * m + j];
        H[i * m + j] = cs[i] * a + sn[i] * b;
        H[(i + 1) * m + j] = -sn[i] * a + cs[i] * b;
      }
      double a = H[j * m + j], b = H[(j + 1) * m + j];
      double rho = hypot(a, b);
      cs[j] = rho == 0.0 ? 1.0 : a / rho;
      sn[j] = rho == 0.0 ? 0.0 : b / rho;
      H[j * m + j] = rho;
      H[(j + 1) * m + j] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      /* u_{j+1} = V y (left) or M^{-1} V y (right), y from H y = g */
      for (int i = j; i >= 0; --i) {
        double s = g[i];
        for (int k = i + 1; k <= j; ++k) s -= H[i * m + k] * y[k];
        y[i] = s / H[i * m + i];
      }
      for (int k = 0; k < n; ++k) {
        double s = 0.0;
        for (int i = 0; i <= j; ++i) s += y[i] * V[i][k];
        t[k] = s;
      }
      if (o->left)
        memcpy(u, t, sizeof(double) * n);
      else
        orc1_prec_apply(p, t, u);
      orc1_apply_A(p, u, R);
      rinf = 0.0;
      for (int k = 0; k < n; ++k) rinf = fmax(rinf, fabs(F[k] - R[k]));
      info->iterations = j + 1;
      info->res_inf = rinf;
      if (hist) hist[j + 1] = rinf;
      if (rinf <= target || hn == 0.0) {
        info->converged = rinf <= target;
        break;
      }
    }
  }
  for (int k = 0; k <= m; ++k) free(V[k]);
  free(V);
  free(H);
  free(cs);
  free(sn);
  free(g);
  free(y);
  free(w);
  free(t);
  free(R);
  return info->converged ? 0 : 1;
}
