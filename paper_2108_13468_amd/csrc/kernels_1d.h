// The one-dimensional method (Sec. 2) on the device: unrestarted GMRES
// preconditioned with the block preconditioner M of eq. block_M, for a batch
// of independent problems in one launch.  One workgroup solves one problem
// from start to finish: every iteration, reduction and stopping decision
// stays on the device.
//
// The workgroup also builds its problem: mesh widths from their closed
// forms, the stencil rows and the Thomas factors of A and M.  Tridiagonal
// solves (the direct solve for K = ||U^E||_inf and every M^{-1}) use the
// Thomas recurrences: forward y_k = (b_k - a_k y_{k-1}) / den_k, backward
// z_k = y_k - cp_k z_{k+1}.  Both
// are affine recurrences, evaluated as a block-wide scan: each thread
// composes the maps of a contiguous chunk, a Hillis-Steele scan over the
// threads composes the chunks, and each thread then re-runs its chunk from
// the value entering it.
#pragma once
#include "common.h"

struct OneDArgs {
  int n;                                // unknowns (nodes 1..N-1)
  int nl;                               // layer cells; layer nodes 1..nl (eq. block_M)
  // mesh (closed forms of the layer-adapted meshes): graded layer widths
  // s ln(1 + a / (1 - a k)), or equal layer widths hl; interior widths hi
  double eps, hl, hi, s, a;
  int graded;
  const double *c, *r;                  // nodal c and r (N + 1 each)
  double *W, *C, *E;                    // stencil rows (W of row 0 and E of row n-1 are 0)
  double *a_inv, *a_cp;                 // Thomas factors of A: 1/den_k, e_k/den_k
  double *m_inv, *m_cp;                 // Thomas factors of M
  const double *F;                      // right-hand side
  double *U;                            // solution
  double *V;                            // Krylov basis, (maxit + 1) x n
  double *H;                            // Hessenberg, (maxit + 1) x maxit, row-major
  double *t, *w;                        // n each
  double K, g;                          // stop when ||F - A u||_inf <= K g (K <= 0: ||U^E||_inf)
  int maxit, left;
  double *info;                         // {iterations, converged, res_inf, K}
};

constexpr int k1dThreads = 256;
constexpr int k1dMaxIt = 128;

// Block-wide sum (sum != 0) or max of |.| (sum == 0) of v; every thread gets
// the result.
BLP_DEV double oned_reduce(double v, double *sh, bool sum) {
  for (int d = 32; d >= 1; d >>= 1) {
    const double o = __shfl_xor(v, d, 64);
    v = sum ? v + o : fmax(v, o);
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wv] = v;
  __syncthreads();
  double s = sh[0];
  for (int k = 1; k < (int)(blockDim.x >> 6); ++k) s = sum ? s + sh[k] : fmax(s, sh[k]);
  return s;
}

// out_k = alpha(k) * out_prev + beta(k) in processing order (forward: k = 0..n-1,
// out_prev of k = 0 is 0; backward: k = n-1..0, out_prev of k = n-1 is 0).
// shA, shB: blockDim.x doubles of LDS each.  out may alias the storage that
// beta reads only at the same k.
template <bool BACKWARD, typename FA, typename FB>
BLP_DEV void oned_scan(int n, FA alpha, FB beta, double *out, double *shA, double *shB) {
  const int t = threadIdx.x, T = blockDim.x;
  const int L = (n + T - 1) / T;
  const int p0 = t * L, p1 = min(n, p0 + L);
  double A = 1.0, B = 0.0;
  for (int p = p0; p < p1; ++p) {
    const int k = BACKWARD ? n - 1 - p : p;
    const double a = alpha(k);
    A = a * A;
    B = a * B + beta(k);
  }
  shA[t] = A;
  shB[t] = B;
  __syncthreads();
  // inclusive scan of the compositions: entry t = map_t o ... o map_0
  for (int d = 1; d < T; d <<= 1) {
    double a1 = 1.0, b1 = 0.0;
    const double a2 = shA[t], b2 = shB[t];
    if (t >= d) {
      a1 = shA[t - d];
      b1 = shB[t - d];
    }
    __syncthreads();
    if (t >= d) {
      shA[t] = a2 * a1;
      shB[t] = a2 * b1 + b2;
    }
    __syncthreads();
  }
  double y = t > 0 ? shB[t - 1] : 0.0;  // the maps before this chunk, applied to 0
  __syncthreads();
  for (int p = p0; p < p1; ++p) {
    const int k = BACKWARD ? n - 1 - p : p;
    y = alpha(k) * y + beta(k);
    out[k] = y;
  }
  __syncthreads();
}

// out = T^{-1} b for the tridiagonal T with Thomas factors (inv, cp) and
// sub-diagonal sub (the row's W, or 0 where T drops it).  b and out may be
// the same array.
template <typename FS>
BLP_DEV void oned_solve(int n, FS sub, const double *inv, const double *cp, const double *b,
                        double *out, double *shA, double *shB) {
  oned_scan<false>(
      n, [&](int k) { return k ? -sub(k) * inv[k] : 0.0; }, [&](int k) { return b[k] * inv[k]; },
      out, shA, shB);
  oned_scan<true>(
      n, [&](int k) { return k < n - 1 ? -cp[k] : 0.0; }, [&](int k) { return out[k]; }, out, shA,
      shB);
}

BLP_DEV void oned_apply(const OneDArgs &a, const double *v, double *y) {
  for (int k = threadIdx.x; k < a.n; k += blockDim.x) {
    double s = a.C[k] * v[k];
    if (k > 0) s += a.W[k] * v[k - 1];
    if (k < a.n - 1) s += a.E[k] * v[k + 1];
    y[k] = s;
  }
  __syncthreads();
}

__global__ __launch_bounds__(k1dThreads) void k_gmres1d(const OneDArgs *A) {
  __shared__ double shA[k1dThreads], shB[k1dThreads], red[16];
  __shared__ double cs[k1dMaxIt], sn[k1dMaxIt], gv[k1dMaxIt + 1], y[k1dMaxIt];
  __shared__ int stop;
  const OneDArgs a = A[blockIdx.x];
  const int n = a.n, tid = threadIdx.x, T = blockDim.x, m = a.maxit;
  // set-up: widths (the closed forms, never differences of nodes), the
  // stencil rows of eq. stencil_1d, then the Thomas factors of A and of M
  // (a sequential recurrence, one thread; the others wait at the barrier)
  auto width = [&](int k) {  // w_k = x_k - x_{k-1}, 1 <= k <= N
#pragma clang fp contract(off)
    if (k > a.nl) return a.hi;
    return a.graded ? a.s * log1p(a.a / (1.0 - a.a * k)) : a.hl;
  };
  for (int k = tid; k < n; k += T) {
    // each product and sum rounded as written (no fused multiply-adds), as
    // the problem data are meant to be the same numbers on every path
#pragma clang fp contract(off)
    const int i = k + 1;
    const double hi = width(i), hn = width(i + 1), hb = 0.5 * (hi + hn);
    a.W[k] = i > 1 ? -a.eps / (hi * hb) : 0.0;
    a.E[k] = i < n ? -a.eps / (hn * hb) - a.c[i] / hn : 0.0;
    a.C[k] = a.eps / hb * (1.0 / hi + 1.0 / hn) + a.c[i] / hn + a.r[i];
  }
  __syncthreads();
  if (tid < 2) {
    const bool drop = tid == 1;
    double *inv = drop ? a.m_inv : a.a_inv, *cp = drop ? a.m_cp : a.a_cp;
    double prev = 0.0;
    for (int k = 0; k < n; ++k) {
#pragma clang fp contract(off)
      const double sub = (drop && k + 1 >= a.nl + 2) ? 0.0 : a.W[k];
      const double den = a.C[k] - sub * prev;
      inv[k] = 1.0 / den;
      cp[k] = a.E[k] / den;
      prev = cp[k];
    }
  }
  __syncthreads();
  auto subA = [&](int k) { return a.W[k]; };
  auto subM = [&](int k) { return k + 1 >= a.nl + 2 ? 0.0 : a.W[k]; };  // row k+1 (1-based)
  auto Minv = [&](const double *b, double *out) { oned_solve(n, subM, a.m_inv, a.m_cp, b, out, shA, shB); };

  // K = ||U^E||_inf from the direct solve when the caller leaves it open
  double K = a.K;
  if (!(K > 0.0)) {
    oned_solve(n, subA, a.a_inv, a.a_cp, a.F, a.t, shA, shB);
    double mx = 0.0;
    for (int k = tid; k < n; k += T) mx = fmax(mx, fabs(a.t[k]));
    K = oned_reduce(mx, red, false);
  }
  const double target = K * a.g;
  double mx = 0.0;
  for (int k = tid; k < n; k += T) {
    a.U[k] = 0.0;
    mx = fmax(mx, fabs(a.F[k]));
  }
  double rinf = oned_reduce(mx, red, false);
  int it = 0;
  bool conv = rinf <= target;
  if (!conv) {
    // r0 = M^{-1} F (left) or F (right), v_0 = r0 / ||r0||
    double *v0 = a.V;
    if (a.left) {
      Minv(a.F, v0);
    } else {
      for (int k = tid; k < n; k += T) v0[k] = a.F[k];
      __syncthreads();
    }
    double s = 0.0;
    for (int k = tid; k < n; k += T) s += v0[k] * v0[k];
    const double beta = sqrt(oned_reduce(s, red, true));
    for (int k = tid; k < n; k += T) v0[k] /= beta;
    if (tid == 0) gv[0] = beta;
    __syncthreads();
    for (int j = 0; j < m; ++j) {
      const double *vj = a.V + (size_t)j * n;
      double *w = a.w;
      if (a.left) {
        oned_apply(a, vj, a.t);
        Minv(a.t, w);
      } else {
        Minv(vj, a.t);
        oned_apply(a, a.t, w);
      }
      // modified Gram-Schmidt
      for (int i = 0; i <= j; ++i) {
        const double *vi = a.V + (size_t)i * n;
        double d = 0.0;
        for (int k = tid; k < n; k += T) d += w[k] * vi[k];
        const double h = oned_reduce(d, red, true);
        for (int k = tid; k < n; k += T) w[k] -= h * vi[k];
        if (tid == 0) a.H[(size_t)i * m + j] = h;
      }
      double d = 0.0;
      for (int k = tid; k < n; k += T) d += w[k] * w[k];
      const double hn = sqrt(oned_reduce(d, red, true));
      double *vn = a.V + (size_t)(j + 1) * n;
      for (int k = tid; k < n; k += T) vn[k] = hn > 0.0 ? w[k] / hn : 0.0;
      if (tid == 0) {
        // Givens rotations (rho = hypot) on column j, then y from H y = g
        double *H = a.H;
        H[(size_t)(j + 1) * m + j] = hn;
        for (int i = 0; i < j; ++i) {
          const double p = H[(size_t)i * m + j], q = H[(size_t)(i + 1) * m + j];
          H[(size_t)i * m + j] = cs[i] * p + sn[i] * q;
          H[(size_t)(i + 1) * m + j] = -sn[i] * p + cs[i] * q;
        }
        const double p = H[(size_t)j * m + j], q = H[(size_t)(j + 1) * m + j];
        const double rho = hypot(p, q);
        cs[j] = rho == 0.0 ? 1.0 : p / rho;
        sn[j] = rho == 0.0 ? 0.0 : q / rho;
        H[(size_t)j * m + j] = rho;
        H[(size_t)(j + 1) * m + j] = 0.0;
        gv[j + 1] = -sn[j] * gv[j];
        gv[j] = cs[j] * gv[j];
        for (int i = j; i >= 0; --i) {
          double s2 = gv[i];
          for (int k = i + 1; k <= j; ++k) s2 -= H[(size_t)i * m + k] * y[k];
          y[i] = s2 / H[(size_t)i * m + i];
        }
      }
      __syncthreads();
      // u = V y (left) or M^{-1} V y (right)
      double *dst = a.left ? a.U : a.t;
      for (int k = tid; k < n; k += T) {
        double s2 = 0.0;
        for (int i = 0; i <= j; ++i) s2 += y[i] * a.V[(size_t)i * n + k];
        dst[k] = s2;
      }
      __syncthreads();
      if (!a.left) Minv(a.t, a.U);
      // ||F - A u||_inf
      double r = 0.0;
      for (int k = tid; k < n; k += T) {
        double s2 = a.C[k] * a.U[k];
        if (k > 0) s2 += a.W[k] * a.U[k - 1];
        if (k < n - 1) s2 += a.E[k] * a.U[k + 1];
        r = fmax(r, fabs(a.F[k] - s2));
      }
      rinf = oned_reduce(r, red, false);
      it = j + 1;
      if (tid == 0) stop = (rinf <= target) || !(hn > 0.0);
      __syncthreads();
      if (stop) {
        conv = rinf <= target;
        break;
      }
    }
  }
  if (tid == 0) {
    a.info[0] = it;
    a.info[1] = conv ? 1.0 : 0.0;
    a.info[2] = rinf;
    a.info[3] = K;
  }
}
