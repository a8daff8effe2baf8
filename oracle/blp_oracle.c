/*
 * blp_oracle.c -- TEST INFRASTRUCTURE ONLY (see blp_oracle.h).
 *
 * Plain FP64 reference for the boundary-layer preconditioned FGMRES method of
 * arXiv 2108.13468.  Every routine follows the paper's definitions directly,
 * with no blocking, fusion or reordering; it is meant to be checked by eye
 * against the paper.  Compiled with -O2 -ffp-contract=off.
 *
 * Readings taken where the paper is silent:
 *  - unknowns are the interior nodes 1 <= i, j <= N-1 (Sec. 3 stencil);
 *  - the layer side of each axis is i <= h, h = N/2 for the paper's meshes
 *    (transition node included in the layer, Sec. 3.1 region definition);
 *  - corner multigrid level l+1 keeps the even-numbered nodes of level l, so
 *    the transition node is always kept; the node beyond the transition node
 *    (first interior-mesh node) is a fixed zero "exterior" node at the same
 *    physical distance on every level; coarsening stops at 2 nodes per axis
 *    or an odd count;
 *  - the corner stopping rule measures the residual of the rescaled system
 *    the cycle works on (see orc_corner_mg), from z = 0, with a cycle cap.
 */
#include "blp_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Mesh (Sec. 2.2 eq. tau 1D; Sec. 3 eq. tau exponential)                    */
/* ------------------------------------------------------------------------ */

double orc_mesh_axis(int N, double eps, double sigma, double clow,
                     double *nodes, double *widths) {
  return orc_mesh_axis_ex(N, eps, sigma, clow, 0, N / 2, nodes, widths);
}

/* Layer-adapted meshes with nl cells in the layer [0, tau] and N - nl equal
 * cells on [tau, 1] (Sec. 2.2's remark on Linss's general Shishkin mesh, with
 * q = nl / N; Sec. 3 allows any fitted tensor mesh with a transition point).
 *  kind 0 (Shishkin): tau = min(q, sigma eps ln(N) / clow), equal layer cells.
 *  kind 1 (Bakhvalov-Shishkin): tau = sigma eps ln(N) / clow; the layer nodes
 *    equidistribute the layer function: exp(-clow x_i / (sigma eps)) falls
 *    linearly in i from 1 at i = 0 to 1/N at i = nl, i.e.
 *    x_i = -(sigma eps / clow) ln(1 - (1 - 1/N) i / nl).
 *    When sigma eps ln(N) / clow >= q the mesh is uniform (as the Shishkin
 *    mesh is then).
 * Widths come from closed forms, never from differences of nodes. */
double orc_mesh_axis_ex(int N, double eps, double sigma, double clow, int kind, int nl,
                        double *nodes, double *widths) {
  return orc_mesh_axis_layer(N, eps, sigma, clow, kind, nl, 0, nodes, widths);
}

/* The same for either layer type of the axis (Sec. 3, eq. tau parabolic and
 * eq. tau exponential): an exponential layer has the width scale eps / clow,
 * a parabolic one sqrt(eps) (clow unused); tau = sigma (scale) ln N, capped
 * at q as above, and the graded kind uses the same scale. */
double orc_mesh_axis_layer(int N, double eps, double sigma, double clow, int kind, int nl,
                           int parabolic, double *nodes, double *widths) {
  double q = (double)nl / N;
  double tl = parabolic ? sigma * sqrt(eps) * log((double)N)
                        : sigma * eps * log((double)N) / clow;
  double tau = tl < q ? tl : q;
  int graded = kind == 1 && tl < q;
  double hl = tau / nl;             /* Shishkin layer cells */
  double hi = (1.0 - tau) / (N - nl); /* interior cells       */
  double s = parabolic ? sigma * sqrt(eps) : sigma * eps / clow, a = (1.0 - 1.0 / N) / nl;
  widths[0] = 0.0;
  nodes[0] = 0.0;
  for (int k = 1; k <= N; ++k) {
    if (k < nl) {
      if (graded) {
        /* x_k = -s ln(1 - a k);  h_k = s ln((1 - a (k-1)) / (1 - a k)) */
        nodes[k] = -s * log1p(-a * k);
        widths[k] = s * log1p(a / (1.0 - a * k));
      } else {
        nodes[k] = k * hl;
        widths[k] = hl;
      }
    } else if (k == nl) {
      nodes[k] = tau;
      widths[k] = graded ? s * log1p(a / (1.0 - a * k)) : hl;
    } else {
      nodes[k] = tau + (k - nl) * hi;
      widths[k] = hi;
    }
  }
  return tau;
}

/* ------------------------------------------------------------------------ */
/* Grid operator: the upwind 5-point stencil of Sec. 3 on a tensor grid with  */
/* nx x ny unknowns, zero Dirichlet values outside.                          */
/* ------------------------------------------------------------------------ */

typedef struct {
  int nx, ny;
  double eps;
  double *hx, *hy; /* widths hx[1..nx+1], hy[1..ny+1]: hx[k] = x_k - x_{k-1} */
  double *c1, *c2; /* c1[1..nx] at x-nodes, c2[1..ny] at y-nodes            */
  double *r;       /* r at (i,j): r[(j-1)*nx + (i-1)]                       */
} grid;

static int gidx(const grid *g, int i, int j) { return (j - 1) * g->nx + (i - 1); }

static double gget(const grid *g, const double *v, int i, int j) {
  if (i < 1 || i > g->nx || j < 1 || j > g->ny) return 0.0;
  return v[gidx(g, i, j)];
}

/* Stencil at node (i,j), written as in the paper's 2D upwind stencil:
 *  W  = -eps/(hbar_i h_i)
 *  E  = -eps/(hbar_i h_{i+1}) - c1_ij/h_{i+1}
 *  S  = -eps/(kbar_j k_j)
 *  Nn = -eps/(kbar_j k_{j+1}) - c2_ij/k_{j+1}
 *  C  = eps/hbar_i (1/h_i + 1/h_{i+1}) + eps/kbar_j (1/k_j + 1/k_{j+1})
 *       + c1_ij/h_{i+1} + c2_ij/k_{j+1} + r_ij                             */
typedef struct { double W, E, S, Nn, C; } stencil5;

static stencil5 gstencil(const grid *g, int i, int j) {
  double hi = g->hx[i], hi1 = g->hx[i + 1];
  double kj = g->hy[j], kj1 = g->hy[j + 1];
  double hb = 0.5 * (hi + hi1), kb = 0.5 * (kj + kj1);
  double c1 = g->c1[i], c2 = g->c2[j], r = g->r[gidx(g, i, j)];
  double e = g->eps;
  stencil5 s;
  s.W = -e / (hb * hi);
  s.E = -e / (hb * hi1) - c1 / hi1;
  s.S = -e / (kb * kj);
  s.Nn = -e / (kb * kj1) - c2 / kj1;
  s.C = e / hb * (1.0 / hi + 1.0 / hi1) + e / kb * (1.0 / kj + 1.0 / kj1) +
        c1 / hi1 + c2 / kj1 + r;
  return s;
}

static void gapply(const grid *g, const double *x, double *y) {
  for (int j = 1; j <= g->ny; ++j)
    for (int i = 1; i <= g->nx; ++i) {
      stencil5 s = gstencil(g, i, j);
      y[gidx(g, i, j)] = s.C * gget(g, x, i, j) + s.W * gget(g, x, i - 1, j) +
                         s.E * gget(g, x, i + 1, j) + s.S * gget(g, x, i, j - 1) +
                         s.Nn * gget(g, x, i, j + 1);
    }
}

/* y = A^T x, by scattering each row of A: y_q += A_pq x_p. */
static void gapply_T(const grid *g, const double *x, double *y) {
  int n = g->nx * g->ny;
  for (int p = 0; p < n; ++p) y[p] = 0.0;
  for (int j = 1; j <= g->ny; ++j)
    for (int i = 1; i <= g->nx; ++i) {
      stencil5 s = gstencil(g, i, j);
      double xp = x[gidx(g, i, j)];
      y[gidx(g, i, j)] += s.C * xp;
      if (i > 1) y[gidx(g, i - 1, j)] += s.W * xp;
      if (i < g->nx) y[gidx(g, i + 1, j)] += s.E * xp;
      if (j > 1) y[gidx(g, i, j - 1)] += s.S * xp;
      if (j < g->ny) y[gidx(g, i, j + 1)] += s.Nn * xp;
    }
}

static double dot(int n, const double *a, const double *b) {
  double s = 0.0;
  for (int k = 0; k < n; ++k) s += a[k] * b[k];
  return s;
}

static double nrm2(int n, const double *a) { return sqrt(dot(n, a, a)); }

/* ------------------------------------------------------------------------ */
/* Problem                                                                   */
/* ------------------------------------------------------------------------ */

struct orc_problem {
  int N, n1, h; /* n1 = N-1 unknowns per axis, h = layer cells (N/2 by default) */
  double *xn, *yn;
  grid fine;
  int L;       /* corner multigrid levels; lev[0] is the corner block A_CC */
  grid *lev;
  int ylayer;  /* 0: exponential layer at y = 0; 1: parabolic layer (c2 = 0) */
  int PL;      /* semicoarsening levels of the parabolic corner multigrid */
  struct plevel *pl;
  double *band[2]; /* banded LU of A_CC (0) and A_CC^T (1), built lazily */
};

static grid grid_alloc(int nx, int ny, double eps) {
  grid g;
  g.nx = nx;
  g.ny = ny;
  g.eps = eps;
  g.hx = calloc(nx + 2, sizeof(double));
  g.hy = calloc(ny + 2, sizeof(double));
  g.c1 = calloc(nx + 1, sizeof(double));
  g.c2 = calloc(ny + 1, sizeof(double));
  g.r = calloc((size_t)nx * ny, sizeof(double));
  return g;
}

static void grid_free(grid *g) {
  free(g->hx);
  free(g->hy);
  free(g->c1);
  free(g->c2);
  free(g->r);
}

orc_problem *orc_create(int N, double eps, double sigma, double clow_x,
                        double clow_y, const double *c1x, const double *c2y,
                        const double *r_int) {
  return orc_create_ex(N, eps, sigma, clow_x, clow_y, 0, N / 2, c1x, c2y, r_int);
}

orc_problem *orc_create_ex(int N, double eps, double sigma, double clow_x,
                           double clow_y, int kind, int nl, const double *c1x,
                           const double *c2y, const double *r_int) {
  return orc_create_px(N, eps, sigma, clow_x, clow_y, kind, nl, 0, c1x, c2y, r_int);
}

static void par_build(orc_problem *p);

orc_problem *orc_create_px(int N, double eps, double sigma, double clow_x,
                           double clow_y, int kind, int nl, int ylayer,
                           const double *c1x, const double *c2y, const double *r_int) {
  if (N < 4 || N % 2 || nl < 2 || nl > N - 2 || kind < 0 || kind > 1 || ylayer < 0 ||
      ylayer > 1)
    return NULL;
  orc_problem *p = calloc(1, sizeof(*p));
  p->N = N;
  p->n1 = N - 1;
  p->h = nl; /* last node of the layer side of each axis */
  p->xn = calloc(N + 1, sizeof(double));
  p->yn = calloc(N + 1, sizeof(double));
  double *wx = calloc(N + 2, sizeof(double));
  double *wy = calloc(N + 2, sizeof(double));
  orc_mesh_axis_ex(N, eps, sigma, clow_x, kind, nl, p->xn, wx);
  orc_mesh_axis_layer(N, eps, sigma, clow_y, kind, nl, ylayer, p->yn, wy);
  p->ylayer = ylayer;

  p->fine = grid_alloc(p->n1, p->n1, eps);
  for (int k = 1; k <= N; ++k) {
    p->fine.hx[k] = wx[k];
    p->fine.hy[k] = wy[k];
  }
  for (int k = 1; k <= p->n1; ++k) {
    p->fine.c1[k] = c1x[k];
    p->fine.c2[k] = c2y[k];
  }
  memcpy(p->fine.r, r_int, sizeof(double) * p->n1 * p->n1);
  free(wx);
  free(wy);

  /* Corner multigrid hierarchy (Sec. 3.2, two exponential layers): full
   * coarsening by two, rediscretised coarse operators. */
  int L = 1;
  for (int m = p->h; m % 2 == 0 && m > 2; m /= 2) ++L;
  p->L = L;
  p->lev = calloc(L, sizeof(grid));
  /* level 0 = the corner block: nodes 1..h on each axis, the node beyond the
   * transition node enters only through its width h_{h+1}. */
  grid *g0 = &p->lev[0];
  *g0 = grid_alloc(p->h, p->h, eps);
  for (int k = 1; k <= p->h + 1; ++k) {
    g0->hx[k] = p->fine.hx[k];
    g0->hy[k] = p->fine.hy[k];
  }
  for (int k = 1; k <= p->h; ++k) {
    g0->c1[k] = p->fine.c1[k];
    g0->c2[k] = p->fine.c2[k];
  }
  for (int j = 1; j <= p->h; ++j)
    for (int i = 1; i <= p->h; ++i)
      g0->r[gidx(g0, i, j)] = p->fine.r[gidx(&p->fine, i, j)];
  for (int l = 1; l < L; ++l) {
    grid *f = &p->lev[l - 1], *c = &p->lev[l];
    *c = grid_alloc(f->nx / 2, f->ny / 2, eps);
    for (int k = 1; k <= c->nx; ++k) c->hx[k] = f->hx[2 * k - 1] + f->hx[2 * k];
    for (int k = 1; k <= c->ny; ++k) c->hy[k] = f->hy[2 * k - 1] + f->hy[2 * k];
    c->hx[c->nx + 1] = f->hx[f->nx + 1];
    c->hy[c->ny + 1] = f->hy[f->ny + 1];
    for (int k = 1; k <= c->nx; ++k) c->c1[k] = f->c1[2 * k];
    for (int k = 1; k <= c->ny; ++k) c->c2[k] = f->c2[2 * k];
    for (int j = 1; j <= c->ny; ++j)
      for (int i = 1; i <= c->nx; ++i)
        c->r[gidx(c, i, j)] = f->r[gidx(f, 2 * i, 2 * j)];
  }
  if (ylayer) par_build(p);
  return p;
}

static void par_free(orc_problem *p);

void orc_destroy(orc_problem *p) {
  if (!p) return;
  free(p->xn);
  free(p->yn);
  grid_free(&p->fine);
  for (int l = 0; l < p->L; ++l) grid_free(&p->lev[l]);
  free(p->lev);
  par_free(p);
  free(p->band[0]);
  free(p->band[1]);
  free(p);
}

int orc_n(const orc_problem *p) { return p->n1 * p->n1; }
int orc_num_levels(const orc_problem *p) { return p->L; }
int orc_level_size(const orc_problem *p, int l) { return p->lev[l].nx; }

void orc_nodes(const orc_problem *p, double *x, double *y) {
  memcpy(x, p->xn, sizeof(double) * (p->N + 1));
  memcpy(y, p->yn, sizeof(double) * (p->N + 1));
}

void orc_stencil(const orc_problem *p, int i, int j, double *out5) {
  stencil5 s = gstencil(&p->fine, i, j);
  out5[0] = s.W;
  out5[1] = s.E;
  out5[2] = s.S;
  out5[3] = s.Nn;
  out5[4] = s.C;
}

void orc_apply_A(const orc_problem *p, const double *x, double *y) {
  gapply(&p->fine, x, y);
}

void orc_apply_AT(const orc_problem *p, const double *x, double *y) {
  gapply_T(&p->fine, x, y);
}

int orc_csr(const orc_problem *p, int *rowptr, int *col, double *val) {
  const grid *g = &p->fine;
  int nnz = 0;
  for (int j = 1; j <= g->ny; ++j)
    for (int i = 1; i <= g->nx; ++i) {
      stencil5 s = gstencil(g, i, j);
      rowptr[gidx(g, i, j)] = nnz;
      /* ascending column order: S, W, C, E, N */
      if (j > 1) { col[nnz] = gidx(g, i, j - 1); val[nnz++] = s.S; }
      if (i > 1) { col[nnz] = gidx(g, i - 1, j); val[nnz++] = s.W; }
      col[nnz] = gidx(g, i, j); val[nnz++] = s.C;
      if (i < g->nx) { col[nnz] = gidx(g, i + 1, j); val[nnz++] = s.E; }
      if (j < g->ny) { col[nnz] = gidx(g, i, j + 1); val[nnz++] = s.Nn; }
    }
  rowptr[g->nx * g->ny] = nnz;
  return nnz;
}

/* ------------------------------------------------------------------------ */
/* Thomas algorithm without pivoting (Lemma diag_dom justifies it):          */
/* sub[k] z[k-1] + dia[k] z[k] + sup[k] z[k+1] = rhs[k], k = 0..m-1.         */
/* Forward elimination in increasing k, then back substitution.              */
/* ------------------------------------------------------------------------ */

static void thomas(int m, const double *sub, const double *dia, const double *sup,
                   const double *rhs, double *z, double *cp, double *dp) {
  cp[0] = sup[0] / dia[0];
  dp[0] = rhs[0] / dia[0];
  for (int k = 1; k < m; ++k) {
    double den = dia[k] - sub[k] * cp[k - 1];
    cp[k] = sup[k] / den;
    dp[k] = (rhs[k] - sub[k] * dp[k - 1]) / den;
  }
  z[m - 1] = dp[m - 1];
  for (int k = m - 2; k >= 0; --k) z[k] = dp[k] - cp[k] * z[k + 1];
}

/* ------------------------------------------------------------------------ */
/* Forward preconditioner: block upper-triangular M of eq. (2D blocks),      */
/* regions C (i,j <= h), X (i <= h < j), Y (j <= h < i), I (i,j > h).        */
/* Solve order: I, then Y and X, then C.                                     */
/* ------------------------------------------------------------------------ */

/* M_II: upper-triangular part of A_II (diagonal, East, North), a downstream
 * Gauss-Seidel sweep from the top-right corner of I to its bottom-left. */
void orc_solve_I(const orc_problem *p, const double *b, double *z) {
  const grid *g = &p->fine;
  int h = p->h, n1 = p->n1;
  for (int j = n1; j >= h + 1; --j)
    for (int i = n1; i >= h + 1; --i) {
      stencil5 s = gstencil(g, i, j);
      z[gidx(g, i, j)] = (b[gidx(g, i, j)] - s.E * gget(g, z, i + 1, j) -
                          s.Nn * gget(g, z, i, j + 1)) / s.C;
    }
}

/* M_YY: block Gauss-Seidel over lines of constant x (i), right to left; each
 * line is a tridiagonal solve in j (South, centre, North).  The East
 * neighbour (line i+1, already solved) and the North neighbour of the top
 * node (in I) move to the right-hand side. */
void orc_solve_Y(const orc_problem *p, const double *b, double *z) {
  const grid *g = &p->fine;
  int h = p->h, n1 = p->n1;
  double *sub = malloc(sizeof(double) * h), *dia = malloc(sizeof(double) * h);
  double *sup = malloc(sizeof(double) * h), *rhs = malloc(sizeof(double) * h);
  double *zz = malloc(sizeof(double) * h), *cp = malloc(sizeof(double) * h);
  double *dp = malloc(sizeof(double) * h);
  for (int i = n1; i >= h + 1; --i) {
    for (int j = 1; j <= h; ++j) {
      stencil5 s = gstencil(g, i, j);
      sub[j - 1] = (j > 1) ? s.S : 0.0;
      dia[j - 1] = s.C;
      sup[j - 1] = (j < h) ? s.Nn : 0.0;
      double rr = b[gidx(g, i, j)] - s.E * gget(g, z, i + 1, j);
      if (j == h) rr -= s.Nn * gget(g, z, i, h + 1);
      rhs[j - 1] = rr;
    }
    thomas(h, sub, dia, sup, rhs, zz, cp, dp);
    for (int j = 1; j <= h; ++j) z[gidx(g, i, j)] = zz[j - 1];
  }
  free(sub); free(dia); free(sup); free(rhs); free(zz); free(cp); free(dp);
}

/* M_XX: block Gauss-Seidel over lines of constant y (j), top to bottom; each
 * line is a tridiagonal solve in i (West, centre, East).  The North
 * neighbour (line j+1) and the East neighbour of the last node (in I) move
 * to the right-hand side. */
void orc_solve_X(const orc_problem *p, const double *b, double *z) {
  const grid *g = &p->fine;
  int h = p->h, n1 = p->n1;
  double *sub = malloc(sizeof(double) * h), *dia = malloc(sizeof(double) * h);
  double *sup = malloc(sizeof(double) * h), *rhs = malloc(sizeof(double) * h);
  double *zz = malloc(sizeof(double) * h), *cp = malloc(sizeof(double) * h);
  double *dp = malloc(sizeof(double) * h);
  for (int j = n1; j >= h + 1; --j) {
    for (int i = 1; i <= h; ++i) {
      stencil5 s = gstencil(g, i, j);
      sub[i - 1] = (i > 1) ? s.W : 0.0;
      dia[i - 1] = s.C;
      sup[i - 1] = (i < h) ? s.E : 0.0;
      double rr = b[gidx(g, i, j)] - s.Nn * gget(g, z, i, j + 1);
      if (i == h) rr -= s.E * gget(g, z, h + 1, j);
      rhs[i - 1] = rr;
    }
    thomas(h, sub, dia, sup, rhs, zz, cp, dp);
    for (int i = 1; i <= h; ++i) z[gidx(g, i, j)] = zz[i - 1];
  }
  free(sub); free(dia); free(sup); free(rhs); free(zz); free(cp); free(dp);
}

/* Transposed region solves (M^T is block lower triangular: C, X, Y, I). */
static void solve_X_T(const orc_problem *p, const double *b, double *z) {
  const grid *g = &p->fine;
  int h = p->h, n1 = p->n1;
  double *sub = malloc(sizeof(double) * h), *dia = malloc(sizeof(double) * h);
  double *sup = malloc(sizeof(double) * h), *rhs = malloc(sizeof(double) * h);
  double *zz = malloc(sizeof(double) * h), *cp = malloc(sizeof(double) * h);
  double *dp = malloc(sizeof(double) * h);
  for (int j = h + 1; j <= n1; ++j) {
    for (int i = 1; i <= h; ++i) {
      stencil5 s = gstencil(g, i, j);
      /* row (i,j) of M^T: entries M[(i-1,j),(i,j)] = E_{i-1,j},
       * M[(i+1,j),(i,j)] = W_{i+1,j}, M[(i,j-1),(i,j)] = Nn_{i,j-1} */
      sub[i - 1] = (i > 1) ? gstencil(g, i - 1, j).E : 0.0;
      dia[i - 1] = s.C;
      sup[i - 1] = (i < h) ? gstencil(g, i + 1, j).W : 0.0;
      rhs[i - 1] = b[gidx(g, i, j)] - gstencil(g, i, j - 1).Nn * gget(g, z, i, j - 1);
    }
    thomas(h, sub, dia, sup, rhs, zz, cp, dp);
    for (int i = 1; i <= h; ++i) z[gidx(g, i, j)] = zz[i - 1];
  }
  free(sub); free(dia); free(sup); free(rhs); free(zz); free(cp); free(dp);
}

static void solve_Y_T(const orc_problem *p, const double *b, double *z) {
  const grid *g = &p->fine;
  int h = p->h, n1 = p->n1;
  double *sub = malloc(sizeof(double) * h), *dia = malloc(sizeof(double) * h);
  double *sup = malloc(sizeof(double) * h), *rhs = malloc(sizeof(double) * h);
  double *zz = malloc(sizeof(double) * h), *cp = malloc(sizeof(double) * h);
  double *dp = malloc(sizeof(double) * h);
  for (int i = h + 1; i <= n1; ++i) {
    for (int j = 1; j <= h; ++j) {
      stencil5 s = gstencil(g, i, j);
      sub[j - 1] = (j > 1) ? gstencil(g, i, j - 1).Nn : 0.0;
      dia[j - 1] = s.C;
      sup[j - 1] = (j < h) ? gstencil(g, i, j + 1).S : 0.0;
      rhs[j - 1] = b[gidx(g, i, j)] - gstencil(g, i - 1, j).E * gget(g, z, i - 1, j);
    }
    thomas(h, sub, dia, sup, rhs, zz, cp, dp);
    for (int j = 1; j <= h; ++j) z[gidx(g, i, j)] = zz[j - 1];
  }
  free(sub); free(dia); free(sup); free(rhs); free(zz); free(cp); free(dp);
}

static void solve_I_T(const orc_problem *p, const double *b, double *z) {
  const grid *g = &p->fine;
  int h = p->h, n1 = p->n1;
  for (int j = h + 1; j <= n1; ++j)
    for (int i = h + 1; i <= n1; ++i) {
      stencil5 s = gstencil(g, i, j);
      double west = gget(g, z, i - 1, j) * gstencil(g, i - 1, j).E;
      double south = gget(g, z, i, j - 1) * gstencil(g, i, j - 1).Nn;
      z[gidx(g, i, j)] = (b[gidx(g, i, j)] - west - south) / s.C;
    }
}

/* ------------------------------------------------------------------------ */
/* Corner: exact solve (idealised M-hat) by banded LU without pivoting       */
/* (A_CC is an M-matrix), bandwidth nx.                                      */
/* ------------------------------------------------------------------------ */

static double *band_factor(const grid *g, int transpose) {
  int m = g->nx * g->ny, bw = g->nx, ld = 2 * bw + 1;
  double *ab = calloc((size_t)m * ld, sizeof(double));
#define AB(r, q) ab[(size_t)(r) * ld + ((q) - (r) + bw)]
  for (int j = 1; j <= g->ny; ++j)
    for (int i = 1; i <= g->nx; ++i) {
      stencil5 s = gstencil(g, i, j);
      int pr = gidx(g, i, j);
      double ent[5] = {s.C, s.W, s.E, s.S, s.Nn};
      int nb[5][2] = {{i, j}, {i - 1, j}, {i + 1, j}, {i, j - 1}, {i, j + 1}};
      for (int t = 0; t < 5; ++t) {
        int ii = nb[t][0], jj = nb[t][1];
        if (ii < 1 || ii > g->nx || jj < 1 || jj > g->ny) continue;
        int q = gidx(g, ii, jj);
        if (transpose)
          AB(q, pr) = ent[t];
        else
          AB(pr, q) = ent[t];
      }
    }
  for (int k = 0; k < m; ++k) {
    double piv = AB(k, k);
    int rmax = (k + bw < m - 1) ? k + bw : m - 1;
    for (int r = k + 1; r <= rmax; ++r) {
      double l = AB(r, k) / piv;
      if (l == 0.0) continue;
      AB(r, k) = l;
      for (int q = k + 1; q <= rmax; ++q) AB(r, q) -= l * AB(k, q);
    }
  }
  return ab;
#undef AB
}

static void band_solve(const grid *g, const double *ab, const double *b, double *z) {
  int m = g->nx * g->ny, bw = g->nx, ld = 2 * bw + 1;
#define AB(r, q) ab[(size_t)(r) * ld + ((q) - (r) + bw)]
  for (int k = 0; k < m; ++k) z[k] = b[k];
  for (int r = 0; r < m; ++r) {
    int q0 = (r - bw > 0) ? r - bw : 0;
    for (int q = q0; q < r; ++q) z[r] -= AB(r, q) * z[q];
  }
  for (int r = m - 1; r >= 0; --r) {
    int q1 = (r + bw < m - 1) ? r + bw : m - 1;
    for (int q = r + 1; q <= q1; ++q) z[r] -= AB(r, q) * z[q];
    z[r] /= AB(r, r);
  }
#undef AB
}

void orc_corner_exact(orc_problem *p, int transpose, const double *b, double *z) {
  if (!p->band[transpose]) p->band[transpose] = band_factor(&p->lev[0], transpose);
  band_solve(&p->lev[0], p->band[transpose], b, z);
}

/* ------------------------------------------------------------------------ */
/* Corner multigrid (Sec. 3.2, two exponential layers)                       */
/* ------------------------------------------------------------------------ */

/* Finite-element rescaling factor hbar_i kbar_j of node (i,j) on a level. */
static double fe_scale(const grid *g, int i, int j) {
  return 0.5 * (g->hx[i] + g->hx[i + 1]) * 0.5 * (g->hy[j] + g->hy[j + 1]);
}

/* 1D interpolation from level l+1 to level l: fine node k takes coarse nodes
 * idx[0..1] with weights w[0..1] (distance-weighted, i.e. linear in the mesh
 * coordinate; coarse node 0 is the Dirichlet boundary and is dropped). */
static int interp1d(const double *hf, int k, int idx[2], double w[2]) {
  if (k % 2 == 0) {
    idx[0] = k / 2;
    w[0] = 1.0;
    return 1;
  }
  int nterm = 0;
  double tot = hf[k] + hf[k + 1];
  if ((k - 1) / 2 >= 1) {
    idx[nterm] = (k - 1) / 2;
    w[nterm++] = hf[k + 1] / tot;
  }
  idx[nterm] = (k + 1) / 2;
  w[nterm++] = hf[k] / tot;
  return nterm;
}

/* zf += P zc (scaled = 0) or zf += S_f P S_c^{-1} zc (scaled = 1). */
static void mg_prolong_add(const grid *f, const grid *c, const double *zc,
                           double *zf, int scaled) {
  for (int j = 1; j <= f->ny; ++j)
    for (int i = 1; i <= f->nx; ++i) {
      int ix[2], iy[2];
      double wx[2], wy[2];
      int nx = interp1d(f->hx, i, ix, wx), ny = interp1d(f->hy, j, iy, wy);
      double s = 0.0;
      for (int a = 0; a < nx; ++a)
        for (int bb = 0; bb < ny; ++bb) {
          double v = zc[gidx(c, ix[a], iy[bb])];
          if (scaled) v /= fe_scale(c, ix[a], iy[bb]);
          s += wx[a] * wy[bb] * v;
        }
      if (scaled) s *= fe_scale(f, i, j);
      zf[gidx(f, i, j)] += s;
    }
}

/* bc = S_c^{-1} P^T S_f rf (scaled = 1) or bc = P^T rf (scaled = 0). */
static void mg_restrict(const grid *f, const grid *c, const double *rf,
                        double *bc, int scaled) {
  int nc = c->nx * c->ny;
  for (int k = 0; k < nc; ++k) bc[k] = 0.0;
  for (int j = 1; j <= f->ny; ++j)
    for (int i = 1; i <= f->nx; ++i) {
      int ix[2], iy[2];
      double wx[2], wy[2];
      int nx = interp1d(f->hx, i, ix, wx), ny = interp1d(f->hy, j, iy, wy);
      double v = rf[gidx(f, i, j)];
      if (scaled) v *= fe_scale(f, i, j);
      for (int a = 0; a < nx; ++a)
        for (int bb = 0; bb < ny; ++bb) bc[gidx(c, ix[a], iy[bb])] += wx[a] * wy[bb] * v;
    }
  if (scaled)
    for (int j = 1; j <= c->ny; ++j)
      for (int i = 1; i <= c->nx; ++i) bc[gidx(c, i, j)] /= fe_scale(c, i, j);
}

/* One pointwise Gauss-Seidel sweep in place.  Forward: downstream order,
 * from the top-right node to the bottom-left one, on A.  Transposed: the
 * transpose of that sweep, i.e. the reverse order on A^T. */
static void mg_gs(const grid *g, const double *b, double *z, int transpose) {
  if (!transpose) {
    for (int j = g->ny; j >= 1; --j)
      for (int i = g->nx; i >= 1; --i) {
        stencil5 s = gstencil(g, i, j);
        double acc = b[gidx(g, i, j)] - s.W * gget(g, z, i - 1, j) -
                     s.E * gget(g, z, i + 1, j) - s.S * gget(g, z, i, j - 1) -
                     s.Nn * gget(g, z, i, j + 1);
        z[gidx(g, i, j)] = acc / s.C;
      }
  } else {
    for (int j = 1; j <= g->ny; ++j)
      for (int i = 1; i <= g->nx; ++i) {
        stencil5 s = gstencil(g, i, j);
        double acc = b[gidx(g, i, j)];
        if (i > 1) acc -= gstencil(g, i - 1, j).E * z[gidx(g, i - 1, j)];
        if (i < g->nx) acc -= gstencil(g, i + 1, j).W * z[gidx(g, i + 1, j)];
        if (j > 1) acc -= gstencil(g, i, j - 1).Nn * z[gidx(g, i, j - 1)];
        if (j < g->ny) acc -= gstencil(g, i, j + 1).S * z[gidx(g, i, j + 1)];
        z[gidx(g, i, j)] = acc / s.C;
      }
  }
}

/* V(1,1) cycle on level l; z holds the initial guess and is updated. */
static void mg_vcycle(const orc_problem *p, int l, const double *b, double *z,
                      int transpose) {
  const grid *g = &p->lev[l];
  int n = g->nx * g->ny;
  if (l == p->L - 1) { /* coarsest: four Gauss-Seidel sweeps */
    for (int s = 0; s < 4; ++s) mg_gs(g, b, z, transpose);
    return;
  }
  const grid *c = &p->lev[l + 1];
  int nc = c->nx * c->ny;
  double *r = malloc(sizeof(double) * n);
  double *bc = malloc(sizeof(double) * nc);
  double *zc = calloc(nc, sizeof(double));
  mg_gs(g, b, z, transpose);
  if (!transpose)
    gapply(g, z, r);
  else
    gapply_T(g, z, r);
  for (int k = 0; k < n; ++k) r[k] = b[k] - r[k];
  mg_restrict(g, c, r, bc, !transpose);
  mg_vcycle(p, l + 1, bc, zc, transpose);
  mg_prolong_add(g, c, zc, z, transpose);
  mg_gs(g, b, z, transpose);
  free(r);
  free(bc);
  free(zc);
}

/* Stationary iteration with the V(1,1) cycle from z = 0.  Adaptive rule:
 * stop once the residual of the system the cycle works on has fallen by the
 * factor rtol (Sec. 3.2: 1e3 for two exponential layers).  The forward cycle
 * works on the finite-element rescaled system S A_CC z = S b
 * (S = diag(hbar_i kbar_j)), so its residual is measured as ||S (b - A z)||;
 * the transposed cycle is the same cycle for (S A_CC)^T in the variable
 * S^{-1} z, whose residual is b - A_CC^T z unscaled. */
int orc_corner_mg(orc_problem *p, int transpose, int fixed_cycles, double rtol,
                  int maxcyc, const double *b, double *z) {
  const grid *g = &p->lev[0];
  int n = g->nx * g->ny;
  for (int k = 0; k < n; ++k) z[k] = 0.0;
  if (fixed_cycles > 0) {
    for (int c = 0; c < fixed_cycles; ++c) mg_vcycle(p, 0, b, z, transpose);
    return fixed_cycles;
  }
  double *r = malloc(sizeof(double) * n);
  for (int j = 1; j <= g->ny; ++j)
    for (int i = 1; i <= g->nx; ++i)
      r[gidx(g, i, j)] = transpose ? b[gidx(g, i, j)] : fe_scale(g, i, j) * b[gidx(g, i, j)];
  double nb = nrm2(n, r);
  int cyc = 0;
  while (nb > 0.0 && cyc < maxcyc) {
    mg_vcycle(p, 0, b, z, transpose);
    ++cyc;
    if (!transpose)
      gapply(g, z, r);
    else
      gapply_T(g, z, r);
    for (int j = 1; j <= g->ny; ++j)
      for (int i = 1; i <= g->nx; ++i) {
        int q = gidx(g, i, j);
        r[q] = b[q] - r[q];
        if (!transpose) r[q] *= fe_scale(g, i, j);
      }
    if (nrm2(n, r) <= rtol * nb) break;
  }
  free(r);
  return cyc;
}

void orc_level_apply(const orc_problem *p, int l, const double *x, double *y) {
  gapply(&p->lev[l], x, y);
}
void orc_level_restrict(const orc_problem *p, int l, const double *rf, double *bc) {
  mg_restrict(&p->lev[l], &p->lev[l + 1], rf, bc, 1);
}
void orc_level_interp(const orc_problem *p, int l, const double *zc, double *zf) {
  const grid *f = &p->lev[l];
  for (int k = 0; k < f->nx * f->ny; ++k) zf[k] = 0.0;
  mg_prolong_add(f, &p->lev[l + 1], zc, zf, 0);
}
void orc_level_gs(const orc_problem *p, int l, const double *b, double *z) {
  mg_gs(&p->lev[l], b, z, 0);
}

/* ------------------------------------------------------------------------ */
/* Corner multigrid, one parabolic and one exponential layer (Sec. 3.2).    */
/*                                                                          */
/* The corner block is an anisotropic operator there (West-East couplings   */
/* of order 1/eps times the North-South ones), so the cycle coarsens by two */
/* in x only.  On the finest level each row of A_CC is multiplied by        */
/* hbar_i kbar_j (finite-element-like scaling); coarse operators are the    */
/* Galerkin products P^T A P, 9-point stencils.  Interpolation to an odd    */
/* fine node is operator induced: its row, collapsed North-South to three   */
/* points, is solved for the node's value given the two even neighbours     */
/* (which are coarse nodes); even nodes are injected; restriction is P^T.   */
/* Smoothing: pointwise Gauss-Seidel in the downstream order (top-right to  */
/* bottom-left); the coarsest level gets four sweeps.                       */
/* ------------------------------------------------------------------------ */

/* A level of the semicoarsening hierarchy: nx x ny unknowns, node (i, j) at
 * (j-1) nx + (i-1); a[9 k + 3 (dj+1) + (di+1)] = coefficient of node
 * (i+di, j+dj) in row k (zero for nodes outside the level); wl, wr = the
 * interpolation weights of odd node i toward the coarse nodes (i-1)/2 and
 * (i+1)/2 (fine nodes i-1 and i+1). */
struct plevel {
  int nx, ny;
  double *a;
  double *wl, *wr;
};

static int pidx(const struct plevel *v, int i, int j) { return (j - 1) * v->nx + (i - 1); }

static double pget(const struct plevel *v, const double *z, int i, int j) {
  if (i < 1 || i > v->nx || j < 1 || j > v->ny) return 0.0;
  return z[pidx(v, i, j)];
}

static double *pcoef(const struct plevel *v, int i, int j, int di, int dj) {
  return &v->a[9 * pidx(v, i, j) + 3 * (dj + 1) + (di + 1)];
}

/* Coarse nodes that fine node i (x index) interpolates from, with weights:
 * even i: i/2 with weight 1; odd i: (i-1)/2 (dropped when it is the
 * boundary node 0) with wl and (i+1)/2 with wr. */
static int pcols(const struct plevel *f, int i, int j, int I[2], double w[2]) {
  if (i % 2 == 0) {
    I[0] = i / 2;
    w[0] = 1.0;
    return 1;
  }
  int n = 0;
  if ((i - 1) / 2 >= 1) {
    I[n] = (i - 1) / 2;
    w[n++] = f->wl[pidx(f, i, j)];
  }
  I[n] = (i + 1) / 2;
  w[n++] = f->wr[pidx(f, i, j)];
  return n;
}

static struct plevel plevel_alloc(int nx, int ny) {
  struct plevel v;
  v.nx = nx;
  v.ny = ny;
  v.a = calloc((size_t)9 * nx * ny, sizeof(double));
  v.wl = calloc((size_t)nx * ny, sizeof(double));
  v.wr = calloc((size_t)nx * ny, sizeof(double));
  return v;
}

/* Interpolation weights of level f (toward the next coarser level) from its
 * own stencil: for odd i the row collapsed North-South,
 *   (sum_dj a_{-1,dj}) z_{i-1} + (sum_dj a_{0,dj}) z_i + (sum_dj a_{+1,dj}) z_{i+1} = 0,
 * solved for z_i. */
static void par_weights(struct plevel *f) {
  for (int j = 1; j <= f->ny; ++j)
    for (int i = 1; i <= f->nx; i += 2) {
      double w = 0.0, c = 0.0, e = 0.0;
      for (int dj = -1; dj <= 1; ++dj) {
        w += *pcoef(f, i, j, -1, dj);
        c += *pcoef(f, i, j, 0, dj);
        e += *pcoef(f, i, j, 1, dj);
      }
      f->wl[pidx(f, i, j)] = -w / c;
      f->wr[pidx(f, i, j)] = -e / c;
    }
}

/* Galerkin coarse operator A_c = P^T A_f P, by scattering each product
 * P_{p,(I,j)} A_{p,q} P_{q,(I',j')}: fine row p = (i, j) restricts to the
 * coarse nodes of pcols(i, j) (same j), its neighbour q = (i+di, j+dj)
 * interpolates from those of pcols(i+di, j+dj), and I' - I lies in -1..1. */
static void par_galerkin(const struct plevel *f, struct plevel *c) {
  for (int j = 1; j <= f->ny; ++j)
    for (int i = 1; i <= f->nx; ++i) {
      int I[2], n = 0;
      double rho[2];
      n = pcols(f, i, j, I, rho);
      for (int dj = -1; dj <= 1; ++dj)
        for (int di = -1; di <= 1; ++di) {
          int qi = i + di, qj = j + dj;
          if (qi < 1 || qi > f->nx || qj < 1 || qj > f->ny) continue;
          double a = *pcoef(f, i, j, di, dj);
          int Iq[2];
          double pi[2];
          int nq = pcols(f, qi, qj, Iq, pi);
          for (int s = 0; s < n; ++s)
            for (int t = 0; t < nq; ++t) {
              int d = Iq[t] - I[s];
              if (d < -1 || d > 1) abort(); /* cannot happen: |qi - i| <= 1 */
              *pcoef(c, I[s], j, d, dj) += rho[s] * a * pi[t];
            }
        }
    }
}

/* FE rescaling factor of fine corner node (i, j): hbar_i kbar_j. */
static double par_scale(const orc_problem *p, int i, int j) {
  const grid *g = &p->fine;
  return 0.5 * (g->hx[i] + g->hx[i + 1]) * 0.5 * (g->hy[j] + g->hy[j + 1]);
}

static void par_build(orc_problem *p) {
  int h = p->h;
  int L = 1;
  for (int m = h; m % 2 == 0 && m > 2; m /= 2) ++L;
  p->PL = L;
  p->pl = calloc(L, sizeof(struct plevel));
  /* level 0: the rows of A_CC (couplings into X, Y or I left out), each
   * multiplied by hbar_i kbar_j */
  p->pl[0] = plevel_alloc(h, h);
  struct plevel *f = &p->pl[0];
  for (int j = 1; j <= h; ++j)
    for (int i = 1; i <= h; ++i) {
      stencil5 s = gstencil(&p->fine, i, j);
      double sc = par_scale(p, i, j);
      *pcoef(f, i, j, 0, 0) = sc * s.C;
      if (i > 1) *pcoef(f, i, j, -1, 0) = sc * s.W;
      if (i < h) *pcoef(f, i, j, 1, 0) = sc * s.E;
      if (j > 1) *pcoef(f, i, j, 0, -1) = sc * s.S;
      if (j < h) *pcoef(f, i, j, 0, 1) = sc * s.Nn;
    }
  for (int l = 0; l + 1 < L; ++l) {
    par_weights(&p->pl[l]);
    p->pl[l + 1] = plevel_alloc(p->pl[l].nx / 2, h);
    par_galerkin(&p->pl[l], &p->pl[l + 1]);
  }
}

static void par_free(orc_problem *p) {
  for (int l = 0; l < p->PL; ++l) {
    free(p->pl[l].a);
    free(p->pl[l].wl);
    free(p->pl[l].wr);
  }
  free(p->pl);
  p->pl = NULL;
  p->PL = 0;
}

static void par_apply(const struct plevel *v, const double *z, double *y) {
  for (int j = 1; j <= v->ny; ++j)
    for (int i = 1; i <= v->nx; ++i) {
      double s = 0.0;
      for (int dj = -1; dj <= 1; ++dj)
        for (int di = -1; di <= 1; ++di) s += *pcoef(v, i, j, di, dj) * pget(v, z, i + di, j + dj);
      y[pidx(v, i, j)] = s;
    }
}

/* One downstream Gauss-Seidel sweep in place: rows from top to bottom, each
 * from right to left, every node solved for with its neighbours' latest
 * values. */
static void par_gs(const struct plevel *v, const double *b, double *z) {
  for (int j = v->ny; j >= 1; --j)
    for (int i = v->nx; i >= 1; --i) {
      double acc = b[pidx(v, i, j)];
      for (int dj = -1; dj <= 1; ++dj)
        for (int di = -1; di <= 1; ++di)
          if (di || dj) acc -= *pcoef(v, i, j, di, dj) * pget(v, z, i + di, j + dj);
      z[pidx(v, i, j)] = acc / *pcoef(v, i, j, 0, 0);
    }
}

/* bc = P^T rf. */
static void par_restrict(const struct plevel *f, const struct plevel *c, const double *rf,
                         double *bc) {
  for (int k = 0; k < c->nx * c->ny; ++k) bc[k] = 0.0;
  for (int j = 1; j <= f->ny; ++j)
    for (int i = 1; i <= f->nx; ++i) {
      int I[2];
      double w[2];
      int n = pcols(f, i, j, I, w);
      for (int s = 0; s < n; ++s) bc[pidx(c, I[s], j)] += w[s] * rf[pidx(f, i, j)];
    }
}

/* zf += P zc. */
static void par_prolong_add(const struct plevel *f, const struct plevel *c, const double *zc,
                            double *zf) {
  for (int j = 1; j <= f->ny; ++j)
    for (int i = 1; i <= f->nx; ++i) {
      int I[2];
      double w[2];
      int n = pcols(f, i, j, I, w);
      double s = 0.0;
      for (int t = 0; t < n; ++t) s += w[t] * zc[pidx(c, I[t], j)];
      zf[pidx(f, i, j)] += s;
    }
}

static void par_vcycle(const orc_problem *p, int l, const double *b, double *z) {
  const struct plevel *v = &p->pl[l];
  int n = v->nx * v->ny;
  if (l == p->PL - 1) {
    for (int s = 0; s < 4; ++s) par_gs(v, b, z);
    return;
  }
  const struct plevel *c = &p->pl[l + 1];
  int nc = c->nx * c->ny;
  double *r = malloc(sizeof(double) * n);
  double *bc = malloc(sizeof(double) * nc);
  double *zc = calloc(nc, sizeof(double));
  par_gs(v, b, z);
  par_apply(v, z, r);
  for (int k = 0; k < n; ++k) r[k] = b[k] - r[k];
  par_restrict(v, c, r, bc);
  par_vcycle(p, l + 1, bc, zc);
  par_prolong_add(v, c, zc, z);
  par_gs(v, b, z);
  free(r);
  free(bc);
  free(zc);
}

/* Corner solve of the parabolic case: V(1,1) cycles on the rescaled system
 * S A_CC z = S b from z = 0 until ||S b - S A_CC z||_2 <= rtol ||S b||_2
 * (Sec. 3.2: a reduction by 1e2), or a fixed number of cycles. */
static int par_corner_mg(orc_problem *p, int fixed_cycles, double rtol, int maxcyc,
                         const double *b, double *z) {
  const struct plevel *v = &p->pl[0];
  int n = v->nx * v->ny;
  double *bs = malloc(sizeof(double) * n), *r = malloc(sizeof(double) * n);
  for (int j = 1; j <= v->ny; ++j)
    for (int i = 1; i <= v->nx; ++i) bs[pidx(v, i, j)] = par_scale(p, i, j) * b[pidx(v, i, j)];
  for (int k = 0; k < n; ++k) z[k] = 0.0;
  int cyc = 0;
  if (fixed_cycles > 0) {
    for (; cyc < fixed_cycles; ++cyc) par_vcycle(p, 0, bs, z);
  } else {
    double nb = nrm2(n, bs);
    while (nb > 0.0 && cyc < maxcyc) {
      par_vcycle(p, 0, bs, z);
      ++cyc;
      par_apply(v, z, r);
      for (int k = 0; k < n; ++k) r[k] = bs[k] - r[k];
      if (nrm2(n, r) <= rtol * nb) break;
    }
  }
  free(bs);
  free(r);
  return cyc;
}

int orc_par_num_levels(const orc_problem *p) { return p->PL; }
int orc_par_level_nx(const orc_problem *p, int l) { return p->pl[l].nx; }
void orc_par_level_stencil(const orc_problem *p, int l, double *a9) {
  memcpy(a9, p->pl[l].a, sizeof(double) * 9 * p->pl[l].nx * p->pl[l].ny);
}
void orc_par_level_weights(const orc_problem *p, int l, double *wl, double *wr) {
  size_t n = (size_t)p->pl[l].nx * p->pl[l].ny;
  memcpy(wl, p->pl[l].wl, sizeof(double) * n);
  memcpy(wr, p->pl[l].wr, sizeof(double) * n);
}
void orc_par_level_apply(const orc_problem *p, int l, const double *x, double *y) {
  par_apply(&p->pl[l], x, y);
}
void orc_par_level_gs(const orc_problem *p, int l, const double *b, double *z) {
  par_gs(&p->pl[l], b, z);
}
void orc_par_level_restrict(const orc_problem *p, int l, const double *rf, double *bc) {
  par_restrict(&p->pl[l], &p->pl[l + 1], rf, bc);
}
void orc_par_level_interp(const orc_problem *p, int l, const double *zc, double *zf) {
  const struct plevel *f = &p->pl[l];
  for (int k = 0; k < f->nx * f->ny; ++k) zf[k] = 0.0;
  par_prolong_add(f, &p->pl[l + 1], zc, zf);
}
int orc_par_corner_mg(orc_problem *p, int fixed_cycles, double rtol, int maxcyc,
                      const double *b, double *z) {
  if (!p->ylayer) return -1;
  return par_corner_mg(p, fixed_cycles, rtol, maxcyc, b, z);
}
int orc_y_layer(const orc_problem *p) { return p->ylayer; }

/* ------------------------------------------------------------------------ */
/* Full preconditioner apply                                                 */
/* ------------------------------------------------------------------------ */

static void stats_add(orc_prec_stats *st, int cycles) {
  if (!st) return;
  if (st->applies == 0) {
    st->mg_cycles_min = cycles;
    st->mg_cycles_max = cycles;
  } else {
    if (cycles < st->mg_cycles_min) st->mg_cycles_min = cycles;
    if (cycles > st->mg_cycles_max) st->mg_cycles_max = cycles;
  }
  st->applies++;
  st->mg_cycles_total += cycles;
}

/* The corner solve of M: exact (the idealised M-hat) or the multigrid of the
 * problem's layer type.  The parabolic cycle has no transposed form here:
 * asked for one, it returns NaN so that the misuse cannot pass unnoticed. */
static void corner_solve(orc_problem *p, const orc_prec_opts *o, int transpose,
                         const double *bC, double *zC, orc_prec_stats *st) {
  int cyc = 0;
  if (o->corner == 0) {
    orc_corner_exact(p, transpose, bC, zC);
  } else if (p->ylayer) {
    if (transpose) {
      for (int k = 0; k < p->h * p->h; ++k) zC[k] = NAN;
    } else {
      cyc = par_corner_mg(p, o->mg_fixed, o->mg_rtol, o->mg_maxcyc, bC, zC);
    }
  } else {
    cyc = orc_corner_mg(p, transpose, o->mg_fixed, o->mg_rtol, o->mg_maxcyc, bC, zC);
  }
  stats_add(st, cyc);
}

void orc_prec_apply(orc_problem *p, const orc_prec_opts *o, int transpose,
                    const double *b, double *z, orc_prec_stats *st) {
  const grid *g = &p->fine;
  int h = p->h, n = orc_n(p);
  const grid *c = &p->lev[0];
  double *bC = malloc(sizeof(double) * h * h), *zC = malloc(sizeof(double) * h * h);
  for (int k = 0; k < n; ++k) z[k] = 0.0;
  if (!transpose) {
    orc_solve_I(p, b, z);
    orc_solve_Y(p, b, z);
    orc_solve_X(p, b, z);
    /* corner right-hand side: b_C - A_CX z_X - A_CY z_Y */
    for (int j = 1; j <= h; ++j)
      for (int i = 1; i <= h; ++i) {
        stencil5 s = gstencil(g, i, j);
        double v = b[gidx(g, i, j)];
        if (i == h) v -= s.E * gget(g, z, h + 1, j);
        if (j == h) v -= s.Nn * gget(g, z, i, h + 1);
        bC[gidx(c, i, j)] = v;
      }
    corner_solve(p, o, 0, bC, zC, st);
    for (int j = 1; j <= h; ++j)
      for (int i = 1; i <= h; ++i) z[gidx(g, i, j)] = zC[gidx(c, i, j)];
  } else {
    for (int j = 1; j <= h; ++j)
      for (int i = 1; i <= h; ++i) bC[gidx(c, i, j)] = b[gidx(g, i, j)];
    corner_solve(p, o, 1, bC, zC, st);
    for (int j = 1; j <= h; ++j)
      for (int i = 1; i <= h; ++i) z[gidx(g, i, j)] = zC[gidx(c, i, j)];
    solve_X_T(p, b, z);
    solve_Y_T(p, b, z);
    solve_I_T(p, b, z);
  }
  free(bC);
  free(zC);
}

/* ------------------------------------------------------------------------ */
/* FGMRES(m), right preconditioned, modified Gram-Schmidt, Givens rotations. */
/* ------------------------------------------------------------------------ */

/* Operator and preconditioner of the system FGMRES iterates on.  In scaled
 * mode the system is D^{-1/2} A D^{-1/2} (symmetric Jacobi scaling) and the
 * preconditioner D^{1/2} M^{-1} D^{1/2}, i.e. the same M applied to the
 * unscaled variables. */
typedef struct {
  orc_problem *p;
  const orc_gmres_opts *o;
  double *dh;   /* D^{1/2} (scaled mode) */
  double *tmp;  /* work */
  orc_prec_stats *st;
} orc_sys;

static void sys_op(orc_sys *s, const double *x, double *y) {
  int n = orc_n(s->p);
  if (!s->o->scaled) {
    (s->o->transpose ? orc_apply_AT : orc_apply_A)(s->p, x, y);
    return;
  }
  for (int k = 0; k < n; ++k) s->tmp[k] = x[k] / s->dh[k];
  (s->o->transpose ? orc_apply_AT : orc_apply_A)(s->p, s->tmp, y);
  for (int k = 0; k < n; ++k) y[k] /= s->dh[k];
}

static void sys_prec(orc_sys *s, const double *v, double *z) {
  int n = orc_n(s->p);
  if (!s->o->precond) {
    memcpy(z, v, sizeof(double) * n);
    return;
  }
  if (!s->o->scaled) {
    orc_prec_apply(s->p, &s->o->prec, s->o->transpose, v, z, s->st);
    return;
  }
  for (int k = 0; k < n; ++k) s->tmp[k] = v[k] * s->dh[k];
  orc_prec_apply(s->p, &s->o->prec, s->o->transpose, s->tmp, z, s->st);
  for (int k = 0; k < n; ++k) z[k] *= s->dh[k];
}

int orc_fgmres(orc_problem *p, const orc_gmres_opts *o, const double *Fin,
               double *u, orc_gmres_info *info, double *hist) {
  int n = orc_n(p), m = o->restart;
  double **V = malloc(sizeof(double *) * (m + 1));
  double **Z = malloc(sizeof(double *) * m);
  for (int k = 0; k <= m; ++k) V[k] = malloc(sizeof(double) * n);
  for (int k = 0; k < m; ++k) Z[k] = malloc(sizeof(double) * n);
  double *H = calloc((size_t)(m + 1) * m, sizeof(double)); /* H[i*m + j] */
  double *cs = calloc(m, sizeof(double)), *sn = calloc(m, sizeof(double));
  double *gv = calloc(m + 1, sizeof(double)), *y = calloc(m, sizeof(double));
  double *w = malloc(sizeof(double) * n), *r = malloc(sizeof(double) * n);
  double *F = malloc(sizeof(double) * n);
  orc_prec_stats st;
  memset(&st, 0, sizeof(st));
  memset(info, 0, sizeof(*info));
  orc_sys sy = {p, o, NULL, malloc(sizeof(double) * n), &st};
  if (o->scaled) {
    sy.dh = malloc(sizeof(double) * n);
    for (int j = 1; j <= p->n1; ++j)
      for (int i = 1; i <= p->n1; ++i)
        sy.dh[gidx(&p->fine, i, j)] = sqrt(gstencil(&p->fine, i, j).C);
    for (int k = 0; k < n; ++k) F[k] = Fin[k] / sy.dh[k];
  } else {
    memcpy(F, Fin, sizeof(double) * n);
  }

  double nF = nrm2(n, F);
  double target = o->absolute ? o->tol : o->tol * nF;
  for (int k = 0; k < n; ++k) u[k] = 0.0;
  for (int k = 0; k < n; ++k) r[k] = F[k];
  double beta = nrm2(n, r);
  if (hist) hist[0] = beta;
  int it = 0, conv = (beta <= target);
  int status = 0;

  while (!conv && it < o->maxit) {
    if (!(beta == beta)) { status = -1; break; } /* NaN */
    for (int k = 0; k < n; ++k) V[0][k] = r[k] / beta;
    for (int k = 0; k <= m; ++k) gv[k] = 0.0;
    gv[0] = beta;
    int j, ncol = 0, est_ok = 0;
    for (j = 0; j < m && it < o->maxit; ++j) {
      sys_prec(&sy, V[j], Z[j]);
      sys_op(&sy, Z[j], w);
      double wn0 = nrm2(n, w);
      for (int i = 0; i <= j; ++i) {
        double hij = dot(n, w, V[i]);
        H[i * m + j] = hij;
        for (int k = 0; k < n; ++k) w[k] -= hij * V[i][k];
      }
      double hn = nrm2(n, w);
      H[(j + 1) * m + j] = hn;
      int happy = (hn <= 1e-14 * wn0);
      if (!happy)
        for (int k = 0; k < n; ++k) V[j + 1][k] = w[k] / hn;
      for (int i = 0; i < j; ++i) {
        double a = H[i * m + j], bb = H[(i + 1) * m + j];
        H[i * m + j] = cs[i] * a + sn[i] * bb;
        H[(i + 1) * m + j] = -sn[i] * a + cs[i] * bb;
      }
      double a = H[j * m + j], bb = H[(j + 1) * m + j];
      double rho = hypot(a, bb);
      if (rho == 0.0) {
        cs[j] = 1.0;
        sn[j] = 0.0;
      } else {
        cs[j] = a / rho;
        sn[j] = bb / rho;
      }
      H[j * m + j] = rho;
      H[(j + 1) * m + j] = 0.0;
      gv[j + 1] = -sn[j] * gv[j];
      gv[j] = cs[j] * gv[j];
      ++it;
      ncol = j + 1;
      if (hist) hist[it] = fabs(gv[j + 1]);
      est_ok = fabs(gv[j + 1]) <= target;
      if (est_ok || happy) break;
    }
    /* back substitution H y = g, then u += Z y */
    for (int i = ncol - 1; i >= 0; --i) {
      double s = gv[i];
      for (int k = i + 1; k < ncol; ++k) s -= H[i * m + k] * y[k];
      y[i] = s / H[i * m + i];
    }
    for (int i = 0; i < ncol; ++i)
      for (int k = 0; k < n; ++k) u[k] += y[i] * Z[i][k];
    sys_op(&sy, u, w);
    for (int k = 0; k < n; ++k) r[k] = F[k] - w[k];
    beta = nrm2(n, r);
    info->restarts++;
    if (beta <= target || (o->stop_on_estimate && est_ok)) conv = 1;
  }
  info->iterations = it;
  info->converged = conv;
  info->true_res = beta;
  info->norm_F = nF;
  info->mg_cycles_total = st.mg_cycles_total;
  info->mg_cycles_min = st.mg_cycles_min;
  info->mg_cycles_max = st.mg_cycles_max;
  if (o->scaled)
    for (int k = 0; k < n; ++k) u[k] /= sy.dh[k];
  for (int k = 0; k <= m; ++k) free(V[k]);
  for (int k = 0; k < m; ++k) free(Z[k]);
  free(V); free(Z); free(H); free(cs); free(sn); free(gv); free(y); free(w); free(r);
  free(F); free(sy.tmp); free(sy.dh);
  if (status) return status;
  return conv ? 0 : 1;
}

/* ------------------------------------------------------------------------ */
/* Problem data: sine-series right-hand side and bilinear reaction field,    */
/* and their adjoints (used by the gradient).                                */
/* ------------------------------------------------------------------------ */

static const double PI = 3.14159265358979323846;

void orc_sine_series(int N, const double *x, const double *y, int K, int L,
                     const double *a, double *F) {
  int n1 = N - 1;
  for (int j = 1; j <= n1; ++j)
    for (int i = 1; i <= n1; ++i) {
      double s = 0.0;
      for (int l = 1; l <= L; ++l)
        for (int k = 1; k <= K; ++k)
          s += a[(l - 1) * K + (k - 1)] * sin(k * PI * x[i]) * sin(l * PI * y[j]);
      F[(j - 1) * n1 + (i - 1)] = s;
    }
}

void orc_sine_project(int N, const double *x, const double *y, int K, int L,
                      const double *lam, double *g) {
  int n1 = N - 1;
  for (int l = 1; l <= L; ++l)
    for (int k = 1; k <= K; ++k) {
      double s = 0.0;
      for (int j = 1; j <= n1; ++j)
        for (int i = 1; i <= n1; ++i)
          s += lam[(j - 1) * n1 + (i - 1)] * sin(k * PI * x[i]) * sin(l * PI * y[j]);
      g[(l - 1) * K + (k - 1)] = s;
    }
}

static double hat(int m, int p, double x) {
  double t = fabs(x * (m - 1) - p);
  return t < 1.0 ? 1.0 - t : 0.0;
}

void orc_bilinear(int N, const double *x, const double *y, int m,
                  const double *R, double *r) {
  int n1 = N - 1;
  for (int j = 1; j <= n1; ++j)
    for (int i = 1; i <= n1; ++i) {
      double s = 0.0;
      for (int q = 0; q < m; ++q)
        for (int pp = 0; pp < m; ++pp)
          s += R[q * m + pp] * hat(m, pp, x[i]) * hat(m, q, y[j]);
      r[(j - 1) * n1 + (i - 1)] = s;
    }
}

void orc_bilinear_project(int N, const double *x, const double *y, int m,
                          const double *w, double *G) {
  int n1 = N - 1;
  for (int q = 0; q < m; ++q)
    for (int pp = 0; pp < m; ++pp) {
      double s = 0.0;
      for (int j = 1; j <= n1; ++j)
        for (int i = 1; i <= n1; ++i)
          s += w[(j - 1) * n1 + (i - 1)] * hat(m, pp, x[i]) * hat(m, q, y[j]);
      G[q * m + pp] = s;
    }
}
