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
#include <type_traits>
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
constexpr int KMAXD = 62;     // dot products per pass: j + 2 <= restart + 1 <= 61

// Basis vectors whose loads are issued together: one block per CU leaves a
// single wave per SIMD, so the loads of several vectors must be in flight at
// once to cover the memory latency.
constexpr int KVU = 4;

// Element q of a length-n vector, zero past n.  The load itself is
// unconditional (at n - 1 past the end): a load under a condition is waited
// for before the branch joins, which would serialise a thread's loads.
template <typename TV>
BLP_DEV TV load_elem(const BLP_GLOBAL TV *x, size_t n, size_t q) {
  const TV v = x[q < n ? q : n - 1];
  return q < n ? v : TV(0);
}

// Elements base + e * 256 (e < KPT) of basis vectors v0 .. v0 + NU - 1,
// zero past n.
template <typename TV, int NU>
BLP_DEV void load_basis(const BLP_GLOBAL TV *V, size_t n, size_t base, int v0, TV (&x)[NU][KPT]) {
#pragma unroll
  for (int u = 0; u < NU; ++u)
#pragma unroll
    for (int e = 0; e < KPT; ++e) x[u][e] = load_elem(V + (size_t)(v0 + u) * n, n, base + (size_t)e * 256);
}

// Block partials of the nd dot products V_v . w (v < nv) and, if with_norm,
// ||w||^2 as dot nv: each wave reduces every product by shuffles and leaves
// its partial in shared memory, then one barrier, then thread v sums the
// waves' partials of product v and publishes it (partials[bid * nd + v]).
template <typename TV>
BLP_DEV void block_dots(const BLP_GLOBAL TV *V, size_t n, size_t base, const double (&wl)[KPT], int nv,
                        bool with_norm, double (*sd)[4], double *partials, size_t bid) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  // elements past n hold zero in both factors and add +0 to each sum
  auto dots = [&](int v0, auto nu) __attribute__((always_inline)) {
    constexpr int NU = decltype(nu)::value;
    TV x[NU][KPT];
    load_basis<TV, NU>(V, n, base, v0, x);
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      double acc = 0.0;
#pragma unroll
      for (int e = 0; e < KPT; ++e) acc += (double)x[u][e] * wl[e];
      acc = wave_sum(acc);
      if (lane == 0) sd[v0 + u][wv] = acc;
    }
  };
  int v = 0;
  for (; v + KVU <= nv; v += KVU) dots(v, std::integral_constant<int, KVU>{});
  for (; v < nv; ++v) dots(v, std::integral_constant<int, 1>{});
  if (with_norm) {
    double acc = 0.0;
#pragma unroll
    for (int e = 0; e < KPT; ++e) acc += wl[e] * wl[e];
    acc = wave_sum(acc);
    if (lane == 0) sd[nv][wv] = acc;
  }
  __syncthreads();
  const int nd = nv + (with_norm ? 1 : 0);
  for (int v = threadIdx.x; v < nd; v += blockDim.x)
    publish(&partials[bid * nd + v], ((sd[v][0] + sd[v][1]) + sd[v][2]) + sd[v][3]);
}

// One system's Krylov state (batched: blockIdx.y selects the record).  The
// step index j is read from device memory (jp), so one launch sequence
// serves every step.
template <typename TV>
struct KArgs {
  TV *V, *Z;          // bases, column stride n
  size_t n;
  double *w;          // FP64 work vector
  double *partials;   // per-block reduction partials
  double *ks;         // Hessenberg / Givens state (KOffsets)
  KrylovStatus *st;
  double *u;          // iterate
  const int *gate;    // nonzero: the system is outside the current cycle
};

// h1[i] = V_i . w (i = 0..j) and wn0 = ||w||.
template <typename TV>
__global__ __launch_bounds__(256) void k_arnoldi_dot(const KArgs<TV> *A, const int *jp, KOffsets ko) {
  __shared__ double sd[KMAXD][4];
  __shared__ bool last;
  const KArgs<TV> a = A[blockIdx.y];
  const int gate = read_or_zero(a.gate), j = read_or_zero(jp);
  const size_t n = a.n;
  const BLP_GLOBAL TV *V = gptr(a.V);
  const BLP_GLOBAL double *wv = gptr(a.w);
  const size_t base = (size_t)blockIdx.x * KCHUNK + threadIdx.x;
  double wl[KPT];
#pragma unroll
  for (int e = 0; e < KPT; ++e) wl[e] = load_elem(wv, n, base + (size_t)e * 256);
  BLP_ISSUED();
  if (gate) return;
  const int nd = j + 2;  // j+1 dots and ||w||^2
  block_dots<TV>(V, n, base, wl, j + 1, true, sd, a.partials, blockIdx.x);
  if (!arrive_last(&a.st->counter, &last, gridDim.x)) return;
  // last block: wave w sums the block partials of products w, w + 4, ...
  // (lanes stride the blocks, then a fixed shuffle tree)
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int v = wid; v < nd; v += nw) {
    double s = 0.0;
    for (int b = lane; b < (int)gridDim.x; b += 64) s += collect(&a.partials[(size_t)b * nd + v]);
    s = wave_sum(s);
    if (lane == 0) {
      if (v <= j) ko.h1(a.ks)[v] = s;
      else a.st->wn0 = sqrt(s);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) reset_counter(&a.st->counter);
}

// w -= sum_i V_i h[i]; then either h2 = V^T w (NORM = false) or
// hn = ||w|| with the Hessenberg/Givens update (NORM = true).
template <typename TV, bool NORM>
__global__ __launch_bounds__(256) void k_arnoldi_update(const KArgs<TV> *A, const int *jp,
                                                        KOffsets ko) {
  __shared__ double sh[16];
  __shared__ double sd[KMAXD][4];
  __shared__ bool last;
  __shared__ double hs[64];
  const KArgs<TV> a = A[blockIdx.y];
  const int gate = read_or_zero(a.gate), j = read_or_zero(jp);
  const size_t n = a.n;
  const BLP_GLOBAL TV *V = gptr(a.V);
  BLP_GLOBAL double *w = gptr(a.w);
  double *ks = a.ks;
  KrylovStatus *st = a.st;
  const size_t base = (size_t)blockIdx.x * KCHUNK + threadIdx.x;
  double wl[KPT];
#pragma unroll
  for (int e = 0; e < KPT; ++e) wl[e] = load_elem<double>(w, n, base + (size_t)e * 256);
  const BLP_GLOBAL double *hin = gptr(NORM ? ko.h2(ks) : ko.h1(ks));
  for (int v = threadIdx.x; v <= j; v += blockDim.x) hs[v] = hin[v];
  BLP_ISSUED();
  if (gate) return;
  __syncthreads();
  // past n both wl and the basis elements are zero (and w is not stored)
  auto update = [&](int v0, auto nu) __attribute__((always_inline)) {
    constexpr int NU = decltype(nu)::value;
    TV x[NU][KPT];
    load_basis<TV, NU>(V, n, base, v0, x);
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      const double hv = hs[v0 + u];
#pragma unroll
      for (int e = 0; e < KPT; ++e) wl[e] -= (double)x[u][e] * hv;
    }
  };
  int v = 0;
  for (; v + KVU <= j + 1; v += KVU) update(v, std::integral_constant<int, KVU>{});
  for (; v <= j; ++v) update(v, std::integral_constant<int, 1>{});
#pragma unroll
  for (int e = 0; e < KPT; ++e) {
    const size_t q = base + (size_t)e * 256;
    if (q < n) w[q] = wl[e];
  }
  const int nd = NORM ? 1 : j + 1;
  if (!NORM) {
    block_dots<TV>(V, n, base, wl, j + 1, false, sd, a.partials, blockIdx.x);
  } else {
    double acc = 0.0;
#pragma unroll
    for (int e = 0; e < KPT; ++e) acc += wl[e] * wl[e];
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) publish(&a.partials[blockIdx.x], acc);
  }
  if (!arrive_last(&st->counter, &last, gridDim.x)) return;
  if (!NORM) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int v = wid; v <= j; v += nw) {
      double s = 0.0;
      for (int b = lane; b < (int)gridDim.x; b += 64) s += collect(&a.partials[(size_t)b * nd + v]);
      s = wave_sum(s);
      if (lane == 0) ko.h2(ks)[v] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) reset_counter(&st->counter);
    return;
  }
  // last block: hn = ||w|| (block-wide fixed-order sum of the partials), then
  // the Hessenberg column h1 + h2 with the previous rotations applied, the new
  // rotation and the residual estimate.  The column and the rotations are
  // staged in shared memory by the whole block; thread 0 applies them.
  __shared__ double col[66], rc[64], rs[64];
  double s = 0.0;
  for (int b = threadIdx.x; b < (int)gridDim.x; b += blockDim.x) s += collect(&a.partials[b]);
  s = block_sum(s, sh);
  const int m = ko.m;
  BLP_GLOBAL double *H = gptr(ko.H(ks)), *cs = gptr(ko.cs(ks)), *sn = gptr(ko.sn(ks)),
                    *g = gptr(ko.g(ks));
  const BLP_GLOBAL double *h1 = gptr(ko.h1(ks));
  for (int v = threadIdx.x; v <= j; v += blockDim.x) {
    col[v] = h1[v] + hs[v];
    if (v < j) {
      rc[v] = cs[v];
      rs[v] = sn[v];
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double hn = sqrt(s);
    col[j + 1] = hn;
    for (int v = 0; v < j; ++v) {
      const double a0 = col[v], b0 = col[v + 1];
      col[v] = rc[v] * a0 + rs[v] * b0;
      col[v + 1] = -rs[v] * a0 + rc[v] * b0;
    }
    const double a0 = col[j], b0 = col[j + 1];
    const double rho = hypot(a0, b0);
    const double c = rho == 0.0 ? 1.0 : a0 / rho, sj = rho == 0.0 ? 0.0 : b0 / rho;
    cs[j] = c;
    sn[j] = sj;
    col[j] = rho;
    col[j + 1] = 0.0;
    const double gj = g[j];
    g[j + 1] = -sj * gj;
    g[j] = c * gj;
    BLP_GLOBAL KrylovStatus *gs = gptr(st);
    gs->est = fabs(sj * gj);
    gs->hn = hn;
    gs->happy = hn <= 1e-14 * gs->wn0;
    reset_counter(&st->counter);
  }
  __syncthreads();
  for (int v = threadIdx.x; v <= j + 1; v += blockDim.x) H[(size_t)v * m + j] = col[v];
}

// V_{j+1} = w / hn (use_beta = 0) or V_0 = w / beta (use_beta = 1), FP64 in,
// TV out.  Batched over blockIdx.y.
template <typename TV>
__global__ void k_normalize(const KArgs<TV> *A, const int *jp, int use_beta) {
  const KArgs<TV> a = A[blockIdx.y];
  if (gated(a.gate)) return;
  const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= a.n) return;
  const double s = use_beta ? a.st->beta : a.st->hn;
  BLP_GLOBAL TV *v = gptr(a.V + (use_beta ? 0 : (size_t)(step_of(jp) + 1) * a.n));
  v[q] = (TV)(gptr(a.w)[q] / s);
}

// Start of a restart cycle: g = (beta, 0, ..., 0).  One block per system.
template <typename TV>
__global__ void k_krylov_init(const KArgs<TV> *A, KOffsets ko) {
  const KArgs<TV> a = A[blockIdx.x];
  if (gated(a.gate)) return;
  double *g = ko.g(a.ks);
  for (int v = threadIdx.x; v <= ko.m; v += blockDim.x) g[v] = v == 0 ? a.st->beta : 0.0;
}

// u += Z y, with H y = g solved (upper triangular, ncol[s] columns) by each
// block into shared memory.  Batched over blockIdx.y.
template <typename TV>
__global__ __launch_bounds__(256) void k_update_solution(const KArgs<TV> *A, const int *ncolv,
                                                         KOffsets ko) {
  __shared__ double y[64];
  const KArgs<TV> a = A[blockIdx.y];
  if (gated(a.gate)) return;
  const int ncol = ncolv[blockIdx.y];
  if (threadIdx.x == 0) {
    const int m = ko.m;
    const double *H = ko.H(a.ks), *g = ko.g(a.ks);
    for (int v = ncol - 1; v >= 0; --v) {
      double s = g[v];
      for (int k = v + 1; k < ncol; ++k) s -= H[v * m + k] * y[k];
      y[v] = s / H[v * m + v];
    }
  }
  __syncthreads();
  const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= a.n) return;
  BLP_GLOBAL double *u = gptr(a.u);
  const BLP_GLOBAL TV *Z = gptr(a.Z);
  double s = u[q];
  for (int v = 0; v < ncol; ++v) s += y[v] * (double)Z[(size_t)v * a.n + q];
  u[q] = s;
}
