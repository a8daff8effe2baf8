// Operator kernels: the upwind 5-point stencil applied on the fly from the
// per-axis tables (no stored matrix), residuals and norms, problem-data
// helpers (sine-series forcing, bilinear reaction field) and conversions.
#pragma once
#include "common.h"

// Stencil application on the fine grid, one thread per column and a strip of
// `rows` rows per block (the x_{j-1}, x_j, x_{j+1} values roll in registers;
// x_{i+-1} come from neighbouring threads of the same coalesced row loads).
//   y = A x            (TR = false)   or   y = A^T x   (TR = true)
//   RESID: y = F - (A x)
//   SCALE: y *= 1/sqrt(C_ij)        (symmetric Jacobi scaling of the output)
// Arithmetic in FP64 whatever the storage type of x.  With RESID the kernel
// also reduces ||y||^2 (the last block writes st->beta = ||y||).  Batched:
// blockIdx.z selects the system; x is x + j * ldx.
template <typename TX>
struct SpmvArgs {
  Grid<double> g;
  const TX *x;
  long long ldx;
  double *y;
  const double *F;    // RESID
  double *partials;   // RESID: one per block of the system
  KrylovStatus *st;   // RESID
  const int *gate;
};

template <typename TX, bool TR, bool SCALE, bool RESID>
__global__ __launch_bounds__(256) void k_stencil(const SpmvArgs<TX> *A, const int *jp, int rows) {
  __shared__ double sh[16];
  __shared__ bool last;
  const SpmvArgs<TX> a = A[blockIdx.z];
  if (gated(a.gate)) return;
  const Grid<double> &g = a.g;
  const BLP_GLOBAL TX *__restrict__ x = gptr(a.x + step_of(jp) * a.ldx);
  BLP_GLOBAL double *__restrict__ y = gptr(a.y);
  const BLP_GLOBAL double *__restrict__ Fv = gptr(a.F);
  const int n = g.nx;
  const int i = blockIdx.x * blockDim.x + threadIdx.x + 1;
  const int j0 = blockIdx.y * rows + 1;
  const int j1 = min(j0 + rows - 1, g.ny);
  double acc = 0.0;
  const BLP_GLOBAL double *gW = gptr(g.W), *gE = gptr(g.E), *gS = gptr(g.S), *gN = gptr(g.N),
                         *gDy = gptr(g.Dy), *gr = gptr(g.r);
  if (i <= n) {
    const double cw = TR ? gE[i - 1] : gW[i];
    const double ce = TR ? gW[i + 1] : gE[i];
    const double dx = gptr(g.Dx)[i];
    // Neighbours outside the grid are read at the node itself and weighted
    // by zero, and the nodal r (when absent: a table entry, unused) through
    // a pointer chosen once: every load of a row is unconditional, so the
    // rows' loads overlap instead of each waiting at a branch.  For finite
    // x the weights change nothing; a non-finite x at the node already makes
    // its own term non-finite.
    const int iw = i > 1 ? i - 1 : i, ie = i < n ? i + 1 : i;
    const double mw = i > 1 ? 1.0 : 0.0, me = i < n ? 1.0 : 0.0;
    const bool nodal = gr != nullptr;
    const BLP_GLOBAL double *rp = nodal ? gr : gDy;
    const double mr = nodal ? 1.0 : 0.0, rc = nodal ? 0.0 : g.rc;
    double xs = (j0 > 1 ? 1.0 : 0.0) * (double)x[vidx(i, j0 > 1 ? j0 - 1 : j0, n)];
    double xc = (double)x[vidx(i, j0, n)];
    // rows in groups of four: the group's loads first (rows past j1 read
    // row j1 and are not stored), then its arithmetic and stores
    constexpr int RG = 4;
    for (int jb = j0; jb <= j1; jb += RG) {
      double xn[RG], xw[RG], xe[RG], cs[RG], cn[RG], dy[RG], rl[RG];
      size_t qv[RG];
#pragma unroll
      for (int u = 0; u < RG; ++u) {
        const int j = jb + u <= j1 ? jb + u : j1;
        qv[u] = vidx(i, j, n);
        xn[u] = (j < g.ny ? 1.0 : 0.0) * (double)x[vidx(i, j < g.ny ? j + 1 : j, n)];
        xw[u] = mw * (double)x[vidx(iw, j, n)];
        xe[u] = me * (double)x[vidx(ie, j, n)];
        cs[u] = TR ? gN[j - 1] : gS[j];
        cn[u] = TR ? gS[j + 1] : gN[j];
        dy[u] = gDy[j];
        rl[u] = rp[nodal ? qv[u] : (size_t)j];
      }
      double fv[RG];
#pragma unroll
      for (int u = 0; u < RG; ++u) fv[u] = RESID ? Fv[qv[u]] : 0.0;
#pragma unroll
      for (int u = 0; u < RG; ++u) {
        if (jb + u > j1) break;
        const double C = dx + dy[u] + (mr * rl[u] + rc);  // r_ij or the constant r
        double v = C * xc + cw * xw[u] + ce * xe[u] + cs[u] * xs + cn[u] * xn[u];
        if (RESID) v = fv[u] - v;
        if (SCALE) v /= sqrt(C);
        y[qv[u]] = v;
        if (RESID) acc += v * v;
        xs = xc;
        xc = xn[u];
      }
    }
  }
  if (!RESID) return;
  acc = block_sum(acc, sh);
  const unsigned int nblk = gridDim.x * gridDim.y;
  const int bid = blockIdx.y * gridDim.x + blockIdx.x;
  if (threadIdx.x == 0) publish(&a.partials[bid], acc);
  if (!arrive_last(&a.st->counter, &last, nblk)) return;
  // last block: block-wide fixed-order sum of the partials
  double s = 0.0;
  for (int b = threadIdx.x; b < (int)nblk; b += blockDim.x) s += collect(&a.partials[b]);
  s = block_sum(s, sh);
  if (threadIdx.x == 0) {
    a.st->beta = sqrt(s);
    reset_counter(&a.st->counter);
  }
}

// ||F|| (or ||F / sqrt(C)|| when SCALE) into st->beta.  Batched over
// blockIdx.y.
struct NormArgs {
  Grid<double> g;
  const double *F;
  double *partials;
  KrylovStatus *st;
  const int *gate;
};
template <bool SCALE>
__global__ __launch_bounds__(256) void k_norm(const NormArgs *A) {
  __shared__ double sh[16];
  __shared__ bool last;
  const NormArgs a = A[blockIdx.y];
  if (gated(a.gate)) return;
  const Grid<double> &g = a.g;
  const int n = g.nx;
  const size_t tot = (size_t)n * g.ny;
  double acc = 0.0;
  for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < tot;
       q += (size_t)gridDim.x * blockDim.x) {
    double v = a.F[q];
    if (SCALE) {
      const int i = (int)(q % n) + 1, j = (int)(q / n) + 1;
      v /= sqrt(g.C(i, j));
    }
    acc += v * v;
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) publish(&a.partials[blockIdx.x], acc);
  if (!arrive_last(&a.st->counter, &last, gridDim.x)) return;
  double s = 0.0;
  for (int b = threadIdx.x; b < (int)gridDim.x; b += blockDim.x) s += collect(&a.partials[b]);
  s = block_sum(s, sh);
  if (threadIdx.x == 0) {
    a.st->beta = sqrt(s);
    reset_counter(&a.st->counter);
  }
}

template <typename TA, typename TB>
__global__ void k_convert(const TA *a, TB *b, size_t n) {
  const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) b[q] = (TB)a[q];
}

template <typename T>
__global__ void k_div(const T *a, const T *d, T *out, size_t n) {
  const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) out[q] = a[q] / d[q];
}

__global__ void k_mul(const double *a, const double *b, double *out, size_t n) {
  const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) out[q] = a[q] * b[q];
}

// Per-axis function tables: tab[k*(N+1) + i] = sin((k+1) pi x_i) (kind 0) or
// the hat function phi_k(x_i) on m uniform nodes of [0,1] (kind 1).
__global__ void k_axis_table(const double *x, int N, int K, int kind, double *tab) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (i > N) return;
  double v;
  if (kind == 0) {
    v = sin((k + 1) * M_PI * x[i]);
  } else {
    const double t = fabs(x[i] * (K - 1) - k);
    v = t < 1.0 ? 1.0 - t : 0.0;
  }
  tab[(size_t)k * (N + 1) + i] = v;
}

// F_ij = sum_{l,k} a[l*K + k] tx[k][i] ty[l][j]  (separable synthesis).
__global__ void k_synth(int N, int K, int L, const double *a, const double *tx,
                        const double *ty, double *F) {
  const int n1 = N - 1;
  const int i = blockIdx.x * blockDim.x + threadIdx.x + 1;
  const int j = blockIdx.y + 1;
  if (i > n1) return;
  double s = 0.0;
  for (int l = 0; l < L; ++l) {
    double sx = 0.0;
    for (int k = 0; k < K; ++k) sx += a[l * K + k] * tx[(size_t)k * (N + 1) + i];
    s += sx * ty[(size_t)l * (N + 1) + j];
  }
  F[vidx(i, j, n1)] = s;
}

// Projection onto separable functions, stage 1: per row j and function k,
// t[k][j] = scale sum_{s < nrhs} sum_i w_s,ij (v_s,ij) tx[k][i], with the
// nrhs vectors of w (and of v, when given: the weight is then the product
// w v) stacked at stride (N-1)^2.  One block per row.
__global__ __launch_bounds__(256) void k_project_rows(int N, int K, int nrhs, double scale,
                                                      const double *w, const double *v,
                                                      const double *tx, double *t) {
  __shared__ double sh[16];
  const int n1 = N - 1;
  const size_t n = (size_t)n1 * n1;
  const int j = blockIdx.x + 1;
  for (int k = 0; k < K; ++k) {
    double acc = 0.0;
    for (int s = 0; s < nrhs; ++s)
      for (int i = threadIdx.x + 1; i <= n1; i += blockDim.x) {
        const size_t q = s * n + vidx(i, j, n1);
        acc += (v ? w[q] * v[q] : w[q]) * tx[(size_t)k * (N + 1) + i];
      }
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) t[(size_t)k * n1 + (j - 1)] = scale * acc;
  }
}

// Stage 2: g[l*K + k] = sum_j t[k][j] ty[l][j].  One block per (k, l).
__global__ __launch_bounds__(256) void k_project_cols(int N, int K, const double *t,
                                                      const double *ty, double *g) {
  __shared__ double sh[16];
  const int n1 = N - 1;
  const int k = blockIdx.x, l = blockIdx.y;
  double acc = 0.0;
  for (int j = threadIdx.x + 1; j <= n1; j += blockDim.x)
    acc += t[(size_t)k * n1 + (j - 1)] * ty[(size_t)l * (N + 1) + j];
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) g[l * K + k] = acc;
}
