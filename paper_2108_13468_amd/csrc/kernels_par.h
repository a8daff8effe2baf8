// Corner multigrid for one parabolic and one exponential layer (Sec. 3.2):
// with c2 = 0 the corner block couples West-East about 1/eps times more
// strongly than North-South, so the cycle coarsens by two in x only.
//
// Levels.  Level l has nx_l = h >> l columns and all h rows.  Level 0 is the
// corner block A_CC, each row multiplied by hbar_i kbar_j; it is the same
// 5-point block as level 0 of the two-exponential-layer hierarchy, and it is
// held and smoothed as that one is (skewed vectors, the wavefront sweep
// kernels, their residual norm, which is that of the rescaled system).  The
// level-0 right-hand side b is kept unscaled (Gauss-Seidel is the same for
// a row and its multiple); the residual handed to level 1 is that of the
// rescaled system.  Coarse levels (l >= 1) are the Galerkin products
// A_{l+1} = P_l^T A_l P_l, 9-point stencils stored as nine planes (plane
// 3 (dj+1) + (di+1) holds the coupling to (i+di, j+dj)); node (i, j) is word
// (j - 1) nx_l + (i - 1) of their vectors (natural layout).
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
// to bottom and each row from right to left (on the 5-point level 0 this is
// the wavefront order's result).  On a coarse level a row is one first-order
// recurrence z_i = alpha_i - beta_i z_{i+1}: alpha holds the right-hand
// side less the row above (already new), the row below and the West
// neighbour (both still old), over the diagonal; beta = a_E / a_C.  One
// workgroup sweeps one system with a thread per column; the recurrence is
// an affine scan over the row.  Rows are strictly sequential (a row needs
// the whole row above), so the sweep is latency bound: depth ny x (one
// row's scan).
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

// 1 / (centre coupling) of a coarse level.
__global__ void k_par_invc(ParSetupLevel f, double *ic) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x + 1;
  const int j = blockIdx.y + 1;
  if (i > f.nx) return;
  ic[vidx(i, j, f.nx)] = 1.0 / f.coef(i, j, 0, 0);
}

// ---------------------------------------------------------------------------
// The cycle (T = storage and sweep precision; residuals in FP64)
// ---------------------------------------------------------------------------

// One system's view of a level (blockIdx selects the record) and of the
// next coarser level for the transfers.  Level 0's z and b are the skewed
// vectors of the two-exponential-layer level 0 (level_skew(h)).
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
};

// (A z)_(i,j) of a coarse level in FP64, z read through the global space; a
// neighbour outside the level counts as zero.
template <typename T>
BLP_DEV double par_apply(const ParArgs<T> &a, const BLP_GLOBAL T *z, int i, int j) {
  const int nx = a.nx, ny = a.ny;
  const BLP_GLOBAL T *A = gptr(a.a);
  const size_t pl = (size_t)nx * ny, q = vidx(i, j, nx);
  double s = 0.0;
#pragma unroll
  for (int dj = -1; dj <= 1; ++dj)
#pragma unroll
    for (int di = -1; di <= 1; ++di) {
      const int qi = i + di, qj = j + dj;
      if (qi < 1 || qi > nx || qj < 1 || qj > ny) continue;
      s += (double)A[(3 * (dj + 1) + (di + 1)) * pl + q] * (double)z[vidx(qi, qj, nx)];
    }
  return s;
}

// Residual of a coarse level, t = b - A z.  One thread per node.
template <typename T>
__global__ void k_par_resid(const ParArgs<T> *A) {
  const ParArgs<T> a = A[blockIdx.z];
  if (gptr(a.ctrl)->gate) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x + 1, j = blockIdx.y + 1;
  if (i > a.nx) return;
  const size_t q = vidx(i, j, a.nx);
  const double r = (double)gptr(a.b)[q] - par_apply<T>(a, gptr(a.z), i, j);
  gptr(a.t)[q] = T(r);
}

// Level 0 to level 1 in one pass: the rescaled residual S (b - A_CC z) at
// the fine columns 2I-1, 2I, 2I+1 of row J (b and z skewed, FP64
// arithmetic, couplings out of the corner block left out), restricted by
// P^T in that order.  One thread per level-1 node.
template <typename T>
__global__ void k_par_rr0(const ParArgs<T> *A) {
  const ParArgs<T> a = A[blockIdx.z];
  if (gptr(a.ctrl)->gate) return;
  const int I = blockIdx.x * blockDim.x + threadIdx.x + 1, J = blockIdx.y + 1;
  if (I > a.nxc) return;
  const int h = a.nx;
  const GridG<T> g = gview(a.g);
  const SkewT<T, false> sk = level_skew<T, false>(h);
  const BLP_GLOBAL T *z = gptr(a.z), *b = gptr(a.b);
  auto res = [&](int i) {
    double s = (double)g.C(i, J) * (double)z[sk.at(i, J)];
    if (i > 1) s += (double)g.W[i] * (double)z[sk.at(i - 1, J)];
    if (i < h) s += (double)g.E[i] * (double)z[sk.at(i + 1, J)];
    if (J > 1) s += (double)g.S[J] * (double)z[sk.at(i, J - 1)];
    if (J < h) s += (double)g.N[J] * (double)z[sk.at(i, J + 1)];
    return ((double)b[sk.at(i, J)] - s) * ((double)a.sx[i] * (double)a.sy[J]);
  };
  double s = (double)gptr(a.wr)[vidx(2 * I - 1, J, h)] * res(2 * I - 1);
  s += res(2 * I);
  if (2 * I + 1 <= h) s += (double)gptr(a.wl)[vidx(2 * I + 1, J, h)] * res(2 * I + 1);
  gptr(a.bc)[vidx(I, J, a.nxc)] = T(s);
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

// Coarse-grid correction of level 0 (skewed z) from level 1, z += P zc.
template <typename T>
__global__ void k_par_prolong0(const ParArgs<T> *A) {
  const ParArgs<T> a = A[blockIdx.z];
  if (gptr(a.ctrl)->gate) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x + 1, j = blockIdx.y + 1;
  const int h = a.nx;
  if (i > h) return;
  const BLP_GLOBAL T *zc = gptr(a.zc);
  const size_t q = vidx(i, j, h);
  T s;
  if (i % 2 == 0) {
    s = zc[vidx(i / 2, j, a.nxc)];
  } else {
    s = T(0);
    if (i > 1) s += gptr(a.wl)[q] * zc[vidx((i - 1) / 2, j, a.nxc)];
    s += gptr(a.wr)[q] * zc[vidx((i + 1) / 2, j, a.nxc)];
  }
  gptr(a.z)[level_skew<T, false>(h).at(i, j)] += s;
}

// One downstream Gauss-Seidel sweep of a coarse level, one workgroup of W waves
// (at most one per SIMD) per system; thread t owns the C consecutive
// columns t C + 1 .. t C + C (nx <= 64 W C).  Per row each thread forms its
// columns' maps z_i = alpha_i - beta_i z_{i+1} and composes them (right to
// left), a DPP scan composes the threads' maps within each wave, the
// waves' aggregates (through LDS) give the value entering each wave from
// the right, and each thread re-runs its columns from the value entering
// its chunk.  Neighbour values across chunk edges (the row above, new; this
// row and the row below, old) come by DPP within one wave, through LDS with
// several (old rows double-buffered by row parity).  The operands of a row
// (right-hand side, 1/centre, couplings, the old values below it) are
// loaded kParAhead rows ahead.  zero_init: the iterate is zero on entry
// (its old values are not read).  SW: the lanes the scan spans (a one-wave
// sweep of at most 16 columns needs only the in-row DPP steps).
constexpr int kParAhead = 4;

template <typename T, int C>
struct ParRowOps {
  T b[C], ic[C], zs[C];   // right-hand side, 1 / centre, old value one row down
  T p[9][C];              // the couplings (plane 4, the centre, unused)
};

// Neighbour value across the wave by one DPP move per 32 bits (CTRL
// wave_shr:1 0x138 or wave_shl:1 0x130); the lane without a source reads 0.
template <int CTRL>
BLP_DEV float par_shift(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
BLP_DEV double par_shift(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}

// Suffix composition of the lanes' affine maps x -> A + M x over the first
// SW lanes (the lanes at and beyond the level's width hold the constant map
// 0): at most 16 lanes need only the in-row DPP steps.
template <typename T, int SW>
BLP_DEV void par_scan_down(T &A, T &M, int lane) {
  if constexpr (SW > 16) {
    scan_affine_down(A, M, lane);
  } else {
#define BLP_PCOMBINE(CTRL)                                                   \
  {                                                                         \
    const T a_ = dpp_mov<CTRL, 0xF>(T(0), A), m_ = dpp_mov<CTRL, 0xF>(T(1), M); \
    A = A + M * a_;                                                         \
    M = M * m_;                                                             \
  }
    if constexpr (SW > 1) BLP_PCOMBINE(0x101)
    if constexpr (SW > 2) BLP_PCOMBINE(0x102)
    if constexpr (SW > 4) BLP_PCOMBINE(0x104)
    if constexpr (SW > 8) BLP_PCOMBINE(0x108)
#undef BLP_PCOMBINE
  }
}

template <typename T, int W, int C, int SW>
__global__ __launch_bounds__(64 * W) void k_par_gs(const ParArgs<T> *A, int zero_init) {
  constexpr int NT = 64 * W, NC = NT * C;
  // W > 1: the north row (new values) and the old values of row j (at
  // [j & 1]) in LDS, index = column; with the waves' aggregate maps
  __shared__ T s_new[W > 1 ? NC + 2 : 1];
  __shared__ T s_old[2][W > 1 ? NC + 2 : 1];
  __shared__ T s_agA[W], s_agM[W];
  const ParArgs<T> a = A[blockIdx.x];
  if (gptr(a.ctrl)->gate) return;  // the same for every thread of the block
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int nx = a.nx, ny = a.ny, i0 = t * C + 1;
  bool in[C];
  unsigned lob[C];  // byte offsets of the thread's columns (clamped into the level)
#pragma unroll
  for (int k = 0; k < C; ++k) {
    in[k] = i0 + k <= nx;
    lob[k] = (unsigned)((in[k] ? i0 + k : nx) - 1) * (unsigned)sizeof(T);
  }
  const BLP_GLOBAL T *B = gptr(a.b);
  const BLP_GLOBAL T *IC = gptr(a.ic);
  const BLP_GLOBAL T *P = gptr(a.a);
  BLP_GLOBAL T *Z = gptr(a.z);
  BLP_GLOBAL T *Tw = gptr(a.t);  // free during a sweep: padding lanes store here
  const int pl = nx * ny;  // at most 512 x 1024: 32-bit offsets
  if (W > 1) {
    for (int k = t; k < NC + 2; k += NT) {
      s_new[k] = T(0);
      s_old[0][k] = T(0);
      s_old[1][k] = T(0);
    }
  }
  // Row bases are uniform (scalar registers), the column offsets the
  // thread's own constants.  Operands are loaded unconditionally (row
  // indices clamped to the level; what a clamped load brings is replaced at
  // its use), so that no branch or copy waits for loads in flight.
  auto at = [&](const BLP_GLOBAL T *row, int k) {
    return *(const BLP_GLOBAL T *)((const BLP_GLOBAL char *)row + lob[k]);
  };
  auto load = [&](int j, ParRowOps<T, C> &o) {
    const int jj = j >= 1 ? j : 1, js = jj > 1 ? jj - 1 : 1;
    const int rb = (jj - 1) * nx;
#pragma unroll
    for (int k = 0; k < C; ++k) {
      o.b[k] = at(B + rb, k);
      o.ic[k] = at(IC + rb, k);
      o.zs[k] = at(Z + (js - 1) * nx, k);
    }
#pragma unroll
    for (int q = 0; q < 9; ++q)
#pragma unroll
      for (int k = 0; k < C; ++k)
        if (q != 4) o.p[q][k] = at(P + q * pl + rb, k);
  };
  T zn[C], zc[C];  // the row above (new) and this row (old), own columns
#pragma unroll
  for (int k = 0; k < C; ++k) zn[k] = T(0);
  // One row: operands in cur (loaded kParAhead rows earlier); those of row
  // j - kParAhead are loaded into nxt, the buffer row j + 1 has released.
  auto row = [&](int j, const ParRowOps<T, C> &cur, ParRowOps<T, C> &nxt) {
    T zs[C];
#pragma unroll
    for (int k = 0; k < C; ++k) zs[k] = (zero_init || j == 1 || !in[k]) ? T(0) : cur.zs[k];
    T nl, nr, sl, sr, cl;  // edge neighbours: columns i0 - 1 (l) and i0 + C (r)
    if (W > 1) {
#pragma unroll
      for (int k = 0; k < C; ++k) s_old[(j - 1) & 1][i0 + k] = zs[k];  // 0 past the level
      load(j - kParAhead, nxt);
      // the rows written above and the north row are visible; the loads of
      // later rows and the stores of earlier rows stay in flight
      lds_barrier();
      nl = s_new[i0 - 1];
      nr = s_new[i0 + C];
      sl = s_old[(j - 1) & 1][i0 - 1];
      sr = s_old[(j - 1) & 1][i0 + C];
      cl = s_old[j & 1][i0 - 1];
    } else {
      load(j - kParAhead, nxt);
      nl = par_shift<0x138>(zn[C - 1]);  // lane l-1 (lane 0: the boundary, 0)
      nr = par_shift<0x130>(zn[0]);      // lane l+1 (lane 63: beyond the level)
      sl = par_shift<0x138>(zs[C - 1]);
      sr = par_shift<0x130>(zs[0]);
      cl = par_shift<0x138>(zc[C - 1]);
    }
    T al[C], be[C];
#pragma unroll
    for (int k = 0; k < C; ++k) {
      const T nW = k ? zn[k - 1] : nl, nE = k + 1 < C ? zn[k + 1] : nr;
      const T sW = k ? zs[k - 1] : sl, sE = k + 1 < C ? zs[k + 1] : sr;
      const T cW = k ? zc[k - 1] : cl;
      T acc = cur.b[k];
      acc -= cur.p[0][k] * sW + cur.p[1][k] * zs[k] + cur.p[2][k] * sE;
      acc -= cur.p[3][k] * cW;
      acc -= cur.p[6][k] * nW + cur.p[7][k] * zn[k] + cur.p[8][k] * nE;
      const T aE = cur.p[5][k];
      al[k] = in[k] ? acc * cur.ic[k] : T(0);
      be[k] = in[k] ? aE * cur.ic[k] : T(0);
    }
    // the chunk's map x -> Am + Mm x from the value x entering at i0 + C
    T Am = T(0), Mm = T(1);
#pragma unroll
    for (int k = C - 1; k >= 0; --k) {
      Am = al[k] - be[k] * Am;
      Mm = -be[k] * Mm;
    }
    par_scan_down<T, SW>(Am, Mm, lane);
    if (W > 1) {
      if (lane == 0) {
        s_agA[w] = Am;
        s_agM[w] = Mm;
      }
      lds_barrier();
    }
    // value entering this wave: the waves to its right applied to zero
    T zin = T(0);
#pragma unroll
    for (int v = W - 1; v > 0; --v)
      if (v > w) zin = s_agA[v] + s_agM[v] * zin;
    // value entering this thread's chunk: the next lane's composed map
    // applied to zin (the wave's last lane: zin itself)
    T ar = par_shift<0x130>(Am), mr = par_shift<0x130>(Mm);
    if (lane == 63) {
      ar = T(0);
      mr = T(1);
    }
    T zr = ar + mr * zin;
    T z[C];
#pragma unroll
    for (int k = C - 1; k >= 0; --k) {
      zr = al[k] - be[k] * zr;
      z[k] = zr;
    }
    // stores are unconditional (a padding lane writes to the free vector t),
    // so that every row issues the same memory operations
    BLP_GLOBAL char *zrow = (BLP_GLOBAL char *)(Z + (j - 1) * nx);
    BLP_GLOBAL char *trow = (BLP_GLOBAL char *)(Tw + (j - 1) * nx);
#pragma unroll
    for (int k = 0; k < C; ++k) {
      *(BLP_GLOBAL T *)((in[k] ? zrow : trow) + lob[k]) = z[k];
      // every read of s_new for this row came before the barrier above
      if (W > 1) s_new[i0 + k] = in[k] ? z[k] : T(0);
      zn[k] = in[k] ? z[k] : T(0);
      zc[k] = zs[k];
    }
  };
  // operand buffers of rows ny .. ny - kParAhead + 1
  ParRowOps<T, C> r[kParAhead + 1];
#pragma unroll
  for (int u = 0; u < kParAhead; ++u) load(ny - u, r[u]);
#pragma unroll
  for (int k = 0; k < C; ++k)
    zc[k] = (zero_init || !in[k]) ? T(0) : at(Z + (ny - 1) * nx, k);
  __syncthreads();  // LDS rows zeroed, y tables in place
  if (W > 1) {
#pragma unroll
    for (int k = 0; k < C; ++k) s_old[ny & 1][i0 + k] = zc[k];
  }
  // the buffers in turn (indices fixed at compile time: no register copies
  // between rows); whole groups of kParAhead + 1 rows, then the rest
  int j = ny;
  for (; j - kParAhead >= 1; j -= kParAhead + 1) {
#pragma unroll
    for (int u = 0; u <= kParAhead; ++u)
      row(j - u, r[u], r[(u + kParAhead) % (kParAhead + 1)]);
  }
#pragma unroll
  for (int u = 0; u < kParAhead; ++u)
    if (j - u >= 1) row(j - u, r[u], r[(u + kParAhead) % (kParAhead + 1)]);
}
