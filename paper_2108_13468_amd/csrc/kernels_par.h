// Corner multigrid for one parabolic and one exponential layer (Sec. 3.2):
// with c2 = 0 the corner block couples West-East about 1/eps times more
// strongly than North-South, so the cycle coarsens by two in x only.
//
// Levels.  Level l has nx_l = h >> l columns and all h rows; node (i, j) is
// word (j - 1) nx_l + (i - 1) of every level vector (natural layout).
// Level 0 is the corner block A_CC, each row multiplied by hbar_i kbar_j;
// its five couplings come from the fine grid's axis tables (nothing is
// stored), and the rescaling is applied where it matters: the level-0
// right-hand side b is kept unscaled (Gauss-Seidel is the same for a row
// and its multiple), the residual handed to the coarser level and the norm
// of the stopping rule are those of the rescaled system.  Coarse levels are
// the Galerkin products A_{l+1} = P_l^T A_l P_l, 9-point stencils stored as
// nine planes (plane 3 (dj+1) + (di+1) holds the coupling to (i+di, j+dj)).
//
// Transfers.  P_l injects the even columns (fine node 2I is coarse node I)
// and interpolates an odd column from its two even neighbours with the
// operator-induced weights: the node's row, collapsed North-South onto row
// j, solved for the node's value,
//   wl = -(sum_dj a_{-1,dj}) / (sum_dj a_{0,dj}),  wr = -(sum_dj a_{+1,dj}) / (same),
// wl toward coarse node (i-1)/2 (absent for i = 1), wr toward (i+1)/2.
// Restriction is P^T.
//
// Smoothing.  One downstream Gauss-Seidel sweep visits the rows from top
// to bottom and each row from right to left.  A row is one first-order
// recurrence z_i = alpha_i - beta_i z_{i+1}: alpha holds the right-hand
// side less the row above (already new), the row below and the West
// neighbour (both still old), over the diagonal; beta = a_E / a_C.  One
// wave sweeps one system: each lane owns C consecutive columns, composes
// its columns' affine maps, a shuffle scan over the lanes composes the
// chunks, and each lane re-runs its chunk from the value entering it.
// Rows are strictly sequential (a row needs the whole row above), so the
// sweep is latency bound: depth ny x (scan of nx / C lanes).
#pragma once
#include "common.h"

// ---------------------------------------------------------------------------
// Set-up (FP64): level-0 couplings, interpolation weights, Galerkin products
// ---------------------------------------------------------------------------

// Rescaled level-0 coupling of (i, j) to (i + di, j + dj): hbar_i kbar_j
// times the 5-point stencil entry; zero for a node outside the corner
// block (those couplings belong to A_CX, A_CY, or the boundary).
BLP_DEV double par_coef0(const Grid<double> &g, const double *sx, const double *sy, int h, int i,
                         int j, int di, int dj) {
  const int qi = i + di, qj = j + dj;
  if (qi < 1 || qi > h || qj < 1 || qj > h) return 0.0;
  const double s = sx[i] * sy[j];
  if (di == 0 && dj == 0) return s * g.C(i, j);
  if (dj == 0) return s * (di < 0 ? g.W[i] : g.E[i]);
  if (di == 0) return s * (dj < 0 ? g.S[j] : g.N[j]);
  return 0.0;
}
// A stored level's coupling (zero outside the level).
BLP_DEV double par_coef(const double *a, int nx, int ny, int i, int j, int di, int dj) {
  const int qi = i + di, qj = j + dj;
  if (qi < 1 || qi > nx || qj < 1 || qj > ny) return 0.0;
  return a[(size_t)(3 * (dj + 1) + (di + 1)) * nx * ny + vidx(i, j, nx)];
}

// Level description for the set-up kernels: level 0 (a == nullptr) reads
// the fine grid's tables and the scaling factors; other levels their planes.
struct ParSetupLevel {
  Grid<double> g;
  const double *sx, *sy;
  const double *a;
  int nx, ny;
  BLP_DEV double coef(int i, int j, int di, int dj) const {
    return a ? par_coef(a, nx, ny, i, j, di, dj) : par_coef0(g, sx, sy, nx, i, j, di, dj);
  }
};

// Interpolation weights of the odd columns (one thread per odd node).
__global__ void k_par_weights(ParSetupLevel f, double *wl, double *wr) {
  const int i = 2 * (blockIdx.x * blockDim.x + threadIdx.x) + 1;
  const int j = blockIdx.y + 1;
  if (i > f.nx) return;
  double w = 0.0, c = 0.0, e = 0.0;
  for (int dj = -1; dj <= 1; ++dj) {
    w += f.coef(i, j, -1, dj);
    c += f.coef(i, j, 0, dj);
    e += f.coef(i, j, 1, dj);
  }
  wl[vidx(i, j, f.nx)] = -w / c;
  wr[vidx(i, j, f.nx)] = -e / c;
}

// Entry of P_l: the weight of coarse column I in fine node (i, j).
BLP_DEV double par_p(const double *wl, const double *wr, int nx, int i, int j, int I) {
  if (i < 1 || i > nx || I < 1) return 0.0;
  if (i == 2 * I) return 1.0;
  if (i == 2 * I - 1) return wr[vidx(i, j, nx)];
  if (i == 2 * I + 1) return wl[vidx(i, j, nx)];
  return 0.0;
}

// Galerkin product, one thread per coarse node (I, J): for each of the
// nine couplings (I + dI, J + dJ),
//   sum over fine rows i = 2I-1..2I+1 of row J and their neighbours
//   q = (i + di, J + dJ): P(i, J; I) A_f(i, J; q) P(q; I + dI).
__global__ void k_par_rap(ParSetupLevel f, const double *wl, const double *wr, int nxc,
                          double *ac) {
  const int I = blockIdx.x * blockDim.x + threadIdx.x + 1;
  const int J = blockIdx.y + 1;
  if (I > nxc) return;
  const int ny = f.ny;
  for (int dJ = -1; dJ <= 1; ++dJ)
    for (int dI = -1; dI <= 1; ++dI) {
      double s = 0.0;
      const int Jq = J + dJ, Iq = I + dI;
      if (Jq >= 1 && Jq <= ny && Iq >= 1 && Iq <= nxc) {
        for (int i = 2 * I - 1; i <= 2 * I + 1; ++i) {
          const double rho = par_p(wl, wr, f.nx, i, J, I);
          if (rho == 0.0) continue;
          for (int di = -1; di <= 1; ++di) {
            const double a = f.coef(i, J, di, dJ);
            if (a == 0.0) continue;
            s += rho * a * par_p(wl, wr, f.nx, i + di, Jq, Iq);
          }
        }
      }
      ac[(size_t)(3 * (dJ + 1) + (dI + 1)) * nxc * ny + vidx(I, J, nxc)] = s;
    }
}

// 1 / (centre coupling) of a level (level 0: of the unscaled stencil, which
// is what its sweep divides by).
__global__ void k_par_invc(ParSetupLevel f, double *ic) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x + 1;
  const int j = blockIdx.y + 1;
  if (i > f.nx) return;
  ic[vidx(i, j, f.nx)] = f.a ? 1.0 / f.coef(i, j, 0, 0) : 1.0 / f.g.C(i, j);
}

// ---------------------------------------------------------------------------
// The cycle (T = storage and sweep precision; residuals in FP64)
// ---------------------------------------------------------------------------

// One system's view of a level (blockIdx selects the record) and of the
// next coarser level for the transfers.
template <typename T>
struct ParArgs {
  int nx, ny;
  Grid<T> g;            // fine grid tables (level-0 couplings)
  const T *sx, *sy;     // level-0 rescaling factors hbar_i, kbar_j (1..h)
  const T *a;           // planes (coarse levels); nullptr on level 0
  const T *ic;          // 1 / centre coupling
  const T *wl, *wr;     // interpolation weights toward the next level
  T *z, *b, *t;         // iterate, right-hand side, residual
  int nxc;              // next coarser level: columns and vectors
  T *zc, *bc;
  MgCtrl *ctrl;
  double *partials;
};

// Level-0 coupling (unscaled 5-point, zero outside the corner block) and a
// stored plane entry, at storage precision.
template <typename T>
BLP_DEV T pc0(const GridG<T> &g, int h, int i, int j, int di, int dj) {
  if (dj == 0) return di < 0 ? (i > 1 ? g.W[i] : T(0)) : (i < h ? g.E[i] : T(0));
  return dj < 0 ? (j > 1 ? g.S[j] : T(0)) : (j < h ? g.N[j] : T(0));
}

// (A z)_(i,j) of a level in FP64 (level 0: unscaled), z read through the
// global space; a neighbour outside the level counts as zero.
template <typename T, bool L0>
BLP_DEV double par_apply(const ParArgs<T> &a, const GridG<T> &g, const BLP_GLOBAL T *z, int i,
                         int j) {
  const int nx = a.nx, ny = a.ny;
  double s = 0.0;
  if (L0) {
    s = (double)g.C(i, j) * (double)z[vidx(i, j, nx)];
    if (i > 1) s += (double)g.W[i] * (double)z[vidx(i - 1, j, nx)];
    if (i < nx) s += (double)g.E[i] * (double)z[vidx(i + 1, j, nx)];
    if (j > 1) s += (double)g.S[j] * (double)z[vidx(i, j - 1, nx)];
    if (j < ny) s += (double)g.N[j] * (double)z[vidx(i, j + 1, nx)];
  } else {
    const BLP_GLOBAL T *A = gptr(a.a);
    const size_t pl = (size_t)nx * ny, q = vidx(i, j, nx);
#pragma unroll
    for (int dj = -1; dj <= 1; ++dj)
#pragma unroll
      for (int di = -1; di <= 1; ++di) {
        const int qi = i + di, qj = j + dj;
        if (qi < 1 || qi > nx || qj < 1 || qj > ny) continue;
        s += (double)A[(3 * (dj + 1) + (di + 1)) * pl + q] * (double)z[vidx(qi, qj, nx)];
      }
  }
  return s;
}

// Residual handed to the next level: level 0 t = S (b - A z) (the rescaled
// system's residual), coarse levels t = b - A z.  One thread per node.
template <typename T, bool L0>
__global__ void k_par_resid(const ParArgs<T> *A) {
  const ParArgs<T> a = A[blockIdx.z];
  if (gptr(a.ctrl)->gate) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x + 1, j = blockIdx.y + 1;
  if (i > a.nx) return;
  const GridG<T> g = gview(a.g);
  const size_t q = vidx(i, j, a.nx);
  double r = (double)gptr(a.b)[q] - par_apply<T, L0>(a, g, gptr(a.z), i, j);
  if (L0) r *= (double)a.sx[i] * (double)a.sy[j];
  gptr(a.t)[q] = T(r);
}

// Coarse right-hand side bc = P^T t, one thread per coarse node, the fine
// columns 2I-1, 2I, 2I+1 added in that order.
template <typename T>
__global__ void k_par_restrict(const ParArgs<T> *A) {
  const ParArgs<T> a = A[blockIdx.z];
  if (gptr(a.ctrl)->gate) return;
  const int I = blockIdx.x * blockDim.x + threadIdx.x + 1, J = blockIdx.y + 1;
  if (I > a.nxc) return;
  const BLP_GLOBAL T *t = gptr(a.t);
  const int nx = a.nx;
  T s = gptr(a.wr)[vidx(2 * I - 1, J, nx)] * t[vidx(2 * I - 1, J, nx)];
  s += t[vidx(2 * I, J, nx)];
  if (2 * I + 1 <= nx) s += gptr(a.wl)[vidx(2 * I + 1, J, nx)] * t[vidx(2 * I + 1, J, nx)];
  gptr(a.bc)[vidx(I, J, a.nxc)] = s;
}

// Coarse-grid correction z += P zc, one thread per fine node.
template <typename T>
__global__ void k_par_prolong(const ParArgs<T> *A) {
  const ParArgs<T> a = A[blockIdx.z];
  if (gptr(a.ctrl)->gate) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x + 1, j = blockIdx.y + 1;
  if (i > a.nx) return;
  const BLP_GLOBAL T *zc = gptr(a.zc);
  const size_t q = vidx(i, j, a.nx);
  T s;
  if (i % 2 == 0) {
    s = zc[vidx(i / 2, j, a.nxc)];
  } else {
    s = T(0);
    if (i > 1) s += gptr(a.wl)[q] * zc[vidx((i - 1) / 2, j, a.nxc)];
    s += gptr(a.wr)[q] * zc[vidx((i + 1) / 2, j, a.nxc)];
  }
  gptr(a.z)[q] += s;
}

// Wave-wide suffix composition of affine maps x -> A x + B (lane L ends
// with map_L o map_{L+1} o ... o map_63).
template <typename T>
BLP_DEV void suffix_compose(T &A, T &B) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const T A2 = __shfl_down(A, d, 64), B2 = __shfl_down(B, d, 64);
    if (lane + d < 64) {
      B = A * B2 + B;
      A = A * A2;
    }
  }
}

// One downstream Gauss-Seidel sweep of a level, one wave per system; lane
// L owns columns L C + 1 .. L C + C.  zero_init: the iterate is zero on
// entry (its old values are not read).
template <typename T, int C, bool L0>
__global__ __launch_bounds__(64) void k_par_gs(const ParArgs<T> *A, int zero_init) {
  const ParArgs<T> a = A[blockIdx.x];
  if (gptr(a.ctrl)->gate) return;
  const int lane = threadIdx.x, nx = a.nx, ny = a.ny;
  const int i0 = lane * C + 1;
  const GridG<T> g = gview(a.g);
  const BLP_GLOBAL T *b = gptr(a.b);
  const BLP_GLOBAL T *ic = gptr(a.ic);
  const BLP_GLOBAL T *P = gptr(a.a);
  BLP_GLOBAL T *z = gptr(a.z);
  const size_t pl = (size_t)nx * ny;
  // per-lane x data of level 0 (constant down the columns)
  T xW[C], xE[C];
#pragma unroll
  for (int k = 0; k < C; ++k) {
    const int i = i0 + k;
    xW[k] = T(0);
    xE[k] = T(0);
    if (L0 && i <= nx) {
      xW[k] = pc0(g, nx, i, 1, -1, 0);
      xE[k] = pc0(g, nx, i, 1, 1, 0);
    }
  }
  // rows: north (new), current (old), south (old)
  T zn[C], zc[C], zs[C];
#pragma unroll
  for (int k = 0; k < C; ++k) {
    zn[k] = T(0);
    zc[k] = T(0);
    const int i = i0 + k;
    if (!zero_init && i <= nx) zc[k] = z[vidx(i, ny, nx)];
  }
  for (int j = ny; j >= 1; --j) {
#pragma unroll
    for (int k = 0; k < C; ++k) {
      const int i = i0 + k;
      zs[k] = T(0);
      if (!zero_init && j > 1 && i <= nx) zs[k] = z[vidx(i, j - 1, nx)];
    }
    // neighbours' edge values: left (column i0 - 1) and right (i0 + C)
    const T znl = __shfl_up(zn[C - 1], 1, 64), znr = __shfl_down(zn[0], 1, 64);
    const T zcl = __shfl_up(zc[C - 1], 1, 64);
    const T zsl = __shfl_up(zs[C - 1], 1, 64), zsr = __shfl_down(zs[0], 1, 64);
    T al[C], be[C];
#pragma unroll
    for (int k = 0; k < C; ++k) {
      const int i = i0 + k;
      const bool in = i <= nx;
      const int ii = in ? i : 1;
      const size_t q = vidx(ii, j, nx);
      const T nW = k ? zn[k - 1] : (lane ? znl : T(0));
      const T nE = k + 1 < C ? zn[k + 1] : (lane < 63 ? znr : T(0));
      const T sW = k ? zs[k - 1] : (lane ? zsl : T(0));
      const T sE = k + 1 < C ? zs[k + 1] : (lane < 63 ? zsr : T(0));
      const T cW = k ? zc[k - 1] : (lane ? zcl : T(0));
      T acc = b[q], aE;
      if (L0) {
        const T aS = j > 1 ? g.S[j] : T(0), aN = j < ny ? g.N[j] : T(0);
        acc -= aS * zs[k] + aN * zn[k] + xW[k] * cW;
        aE = xE[k];
      } else {
        acc -= P[0 * pl + q] * sW + P[1 * pl + q] * zs[k] + P[2 * pl + q] * sE;
        acc -= P[3 * pl + q] * cW;
        acc -= P[6 * pl + q] * nW + P[7 * pl + q] * zn[k] + P[8 * pl + q] * nE;
        aE = P[5 * pl + q];
      }
      const T d = ic[q];
      al[k] = in ? acc * d : T(0);
      be[k] = in ? aE * d : T(0);
    }
    // compose the chunk right to left: z_{i0} = Ac z_in + Bc
    T Ac = T(1), Bc = T(0);
#pragma unroll
    for (int k = C - 1; k >= 0; --k) {
      Bc = al[k] - be[k] * Bc;
      Ac = -be[k] * Ac;
    }
    suffix_compose(Ac, Bc);
    // value entering the chunk from the right: z at column i0 + C
    T zr = __shfl_down(Bc, 1, 64);
    if (lane == 63) zr = T(0);
#pragma unroll
    for (int k = C - 1; k >= 0; --k) {
      zr = al[k] - be[k] * zr;
      zn[k] = zr;
    }
#pragma unroll
    for (int k = 0; k < C; ++k) {
      const int i = i0 + k;
      if (i <= nx) z[vidx(i, j, nx)] = zn[k];
      zc[k] = zs[k];
    }
  }
}

// Stopping rule of the corner iteration: mode 0 ||S b||^2 before the first
// cycle, mode 1 ||S (b - A z)||^2 after each; the last block of a system
// compares and sets its gate (as the two-exponential-layer rule does).
template <typename T, int mode>
__global__ __launch_bounds__(256) void k_par_norm(const ParArgs<T> *A) {
  __shared__ double sh[16];
  __shared__ bool last;
  const ParArgs<T> a = A[blockIdx.y];
  MgCtrl *ctrl = a.ctrl;
  if (gptr(ctrl)->gate) return;  // uniform across the system's blocks
  const GridG<T> g = gview(a.g);
  const int nx = a.nx;
  const size_t n = (size_t)nx * a.ny;
  double acc = 0.0;
  for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
       q += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(q % nx) + 1, j = (int)(q / nx) + 1;
    double v = (double)gptr(a.b)[q];
    if (mode == 1) v -= par_apply<T, true>(a, g, gptr(a.z), i, j);
    v *= (double)a.sx[i] * (double)a.sy[j];
    acc += v * v;
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) publish(&a.partials[blockIdx.x], acc);
  if (!arrive_last(&ctrl->counter, &last, gridDim.x)) return;
  double s = 0.0;
  for (int b2 = threadIdx.x; b2 < (int)gridDim.x; b2 += blockDim.x) s += collect(&a.partials[b2]);
  s = block_sum(s, sh);
  if (threadIdx.x == 0) {
    reset_counter(&ctrl->counter);
    if (mode == 0) {
      ctrl->bnorm2 = s;
      if (s == 0.0) ctrl->gate = 1;
    } else {
      ctrl->cycles += 1;
      ctrl->res2 = s;
      if (s <= ctrl->rtol2 * ctrl->bnorm2 || ctrl->cycles >= ctrl->maxcyc) ctrl->gate = 1;
    }
  }
}

// Count a fixed-mode cycle (no norm evaluation).  One thread per system.
template <typename T>
__global__ void k_par_count(const ParArgs<T> *A) {
  MgCtrl *c = A[blockIdx.x].ctrl;
  if (threadIdx.x == 0 && !c->gate) c->cycles += 1;
}
