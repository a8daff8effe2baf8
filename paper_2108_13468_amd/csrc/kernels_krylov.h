// FGMRES kernels (Saad's flexible GMRES; Sec. 3.3 uses it as the outer
// Krylov method).  The Arnoldi step orthogonalises by classical Gram-Schmidt
// with one reorthogonalisation (CGS2), which spans the same space as the
// modified Gram-Schmidt of the paper in exact arithmetic and needs four
// passes over the basis per step instead of 2(j+1) dependent reductions.
// Dot products are reduced deterministically: per-block partials, then the
// last block to arrive sums them in block order.  The Hessenberg column, the
// Givens rotations and the residual estimate are updated in FP64 by one
// thread of that last block.
#pragma once
#include "common.h"

// Krylov state layout (FP64, device): H[(m+1) x m] row-major, cs[m], sn[m],
// g[m+1], h1[m+1], h2[m+1], y[m].
struct KOffsets {
  int m;
  BLP_DEV double *H(double *b) const { return b; }
  BLP_DEV double *cs(double *b) const { return b + (m + 1) * m; }
  BLP_DEV double *sn(double *b) const { return cs(b) + m; }
  BLP_DEV double *g(double *b) const { return sn(b) + m; }
  BLP_DEV double *h1(double *b) const { return g(b) + m + 1; }
  BLP_DEV double *h2(double *b) const { return h1(b) + m + 1; }
};

constexpr int KCHUNK = 4096;  // elements per block in the basis kernels
constexpr int KPT = KCHUNK / 256;

// h1[i] = V_i . w (i = 0..j) and wn0 = ||w||.
template <typename TV>
__global__ __launch_bounds__(256) void k_arnoldi_dot(const TV *V, size_t ldv, int j,
                                                     const double *w, size_t n,
                                                     double *partials, double *ks,
                                                     KOffsets ko, KrylovStatus *st) {
  __shared__ double sh[16];
  __shared__ bool last;
  const size_t base = (size_t)blockIdx.x * KCHUNK + threadIdx.x;
  double wl[KPT];
#pragma unroll
  for (int e = 0; e < KPT; ++e) {
    const size_t q = base + (size_t)e * 256;
    wl[e] = q < n ? w[q] : 0.0;
  }
  const int nd = j + 2;  // j+1 dots and ||w||^2
  for (int v = 0; v <= j; ++v) {
    double acc = 0.0;
#pragma unroll
    for (int e = 0; e < KPT; ++e) {
      const size_t q = base + (size_t)e * 256;
      if (q < n) acc += (double)V[(size_t)v * ldv + q] * wl[e];
    }
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) publish(&partials[(size_t)blockIdx.x * nd + v], acc);
  }
  double acc = 0.0;
#pragma unroll
  for (int e = 0; e < KPT; ++e) acc += wl[e] * wl[e];
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) publish(&partials[(size_t)blockIdx.x * nd + j + 1], acc);
  if (!arrive_last(&st->counter, &last)) return;
  for (int v = threadIdx.x; v < nd; v += blockDim.x) {
    double s = 0.0;
    for (int b = 0; b < (int)gridDim.x; ++b) s += collect(&partials[(size_t)b * nd + v]);
    if (v <= j) ko.h1(ks)[v] = s;
    else st->wn0 = sqrt(s);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    reset_counter(&st->counter);
  }
}

// w -= sum_i V_i h[i]; then either h2 = V^T w (NORM = false) or
// hn = ||w|| with the Hessenberg/Givens update (NORM = true).
template <typename TV, bool NORM>
__global__ __launch_bounds__(256) void k_arnoldi_update(const TV *V, size_t ldv, int j,
                                                        double *w, size_t n, double *partials,
                                                        double *ks, KOffsets ko,
                                                        KrylovStatus *st) {
  __shared__ double sh[16];
  __shared__ bool last;
  __shared__ double hs[64];
  const double *hin = NORM ? ko.h2(ks) : ko.h1(ks);
  for (int v = threadIdx.x; v <= j; v += blockDim.x) hs[v] = hin[v];
  __syncthreads();
  const size_t base = (size_t)blockIdx.x * KCHUNK + threadIdx.x;
  double wl[KPT];
#pragma unroll
  for (int e = 0; e < KPT; ++e) {
    const size_t q = base + (size_t)e * 256;
    wl[e] = q < n ? w[q] : 0.0;
  }
  for (int v = 0; v <= j; ++v) {
    const double hv = hs[v];
#pragma unroll
    for (int e = 0; e < KPT; ++e) {
      const size_t q = base + (size_t)e * 256;
      if (q < n) wl[e] -= (double)V[(size_t)v * ldv + q] * hv;
    }
  }
#pragma unroll
  for (int e = 0; e < KPT; ++e) {
    const size_t q = base + (size_t)e * 256;
    if (q < n) w[q] = wl[e];
  }
  const int nd = NORM ? 1 : j + 1;
  if (!NORM) {
    for (int v = 0; v <= j; ++v) {
      double acc = 0.0;
#pragma unroll
      for (int e = 0; e < KPT; ++e) {
        const size_t q = base + (size_t)e * 256;
        if (q < n) acc += (double)V[(size_t)v * ldv + q] * wl[e];
      }
      acc = block_sum(acc, sh);
      if (threadIdx.x == 0) publish(&partials[(size_t)blockIdx.x * nd + v], acc);
    }
  } else {
    double acc = 0.0;
#pragma unroll
    for (int e = 0; e < KPT; ++e) acc += wl[e] * wl[e];
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) publish(&partials[blockIdx.x], acc);
  }
  if (!arrive_last(&st->counter, &last)) return;
  if (!NORM) {
    for (int v = threadIdx.x; v <= j; v += blockDim.x) {
      double s = 0.0;
      for (int b = 0; b < (int)gridDim.x; ++b) s += collect(&partials[(size_t)b * nd + v]);
      ko.h2(ks)[v] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      reset_counter(&st->counter);
    }
    return;
  }
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int b = 0; b < (int)gridDim.x; ++b) s += collect(&partials[b]);
    const double hn = sqrt(s);
    const int m = ko.m;
    double *H = ko.H(ks), *cs = ko.cs(ks), *sn = ko.sn(ks), *g = ko.g(ks);
    const double *h1 = ko.h1(ks);
    // Hessenberg column j = h1 + h2 (the two Gram-Schmidt passes)
    for (int v = 0; v <= j; ++v) H[v * m + j] = h1[v] + hs[v];
    H[(j + 1) * m + j] = hn;
    for (int v = 0; v < j; ++v) {
      const double a = H[v * m + j], b = H[(v + 1) * m + j];
      H[v * m + j] = cs[v] * a + sn[v] * b;
      H[(v + 1) * m + j] = -sn[v] * a + cs[v] * b;
    }
    const double a = H[j * m + j], b = H[(j + 1) * m + j];
    const double rho = hypot(a, b);
    if (rho == 0.0) {
      cs[j] = 1.0;
      sn[j] = 0.0;
    } else {
      cs[j] = a / rho;
      sn[j] = b / rho;
    }
    H[j * m + j] = rho;
    H[(j + 1) * m + j] = 0.0;
    g[j + 1] = -sn[j] * g[j];
    g[j] = cs[j] * g[j];
    st->est = fabs(g[j + 1]);
    st->hn = hn;
    st->happy = hn <= 1e-14 * st->wn0;
    reset_counter(&st->counter);
  }
}

// V_{j+1} = w / hn (or V_0 = w / beta), FP64 in, TV out.
template <typename TV>
__global__ void k_normalize(const double *w, TV *v, size_t n, const KrylovStatus *st,
                            int use_beta) {
  const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const double s = use_beta ? st->beta : st->hn;
  v[q] = (TV)(w[q] / s);
}

// Start of a restart cycle: g = (beta, 0, ..., 0).
__global__ void k_krylov_init(double *ks, KOffsets ko, const KrylovStatus *st) {
  double *g = ko.g(ks);
  for (int v = threadIdx.x; v <= ko.m; v += blockDim.x) g[v] = v == 0 ? st->beta : 0.0;
}

// u += Z y, with H y = g solved (upper triangular, ncol columns) by each
// block into shared memory.
template <typename TZ>
__global__ __launch_bounds__(256) void k_update_solution(const TZ *Z, size_t ldz, int ncol,
                                                         const double *ks, KOffsets ko,
                                                         double *u, size_t n) {
  __shared__ double y[64];
  if (threadIdx.x == 0) {
    const int m = ko.m;
    const double *H = ks, *g = ks + (m + 1) * m + 2 * m;
    for (int v = ncol - 1; v >= 0; --v) {
      double s = g[v];
      for (int k = v + 1; k < ncol; ++k) s -= H[v * m + k] * y[k];
      y[v] = s / H[v * m + v];
    }
  }
  __syncthreads();
  const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  double s = u[q];
  for (int v = 0; v < ncol; ++v) s += y[v] * (double)Z[(size_t)v * ldz + q];
  u[q] = s;
}
