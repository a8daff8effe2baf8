// Kernels of the boundary-layer preconditioner (Sec. 3.1, eq. 2D blocks) and
// of the corner multigrid (Sec. 3.2, two exponential layers).
//
// Regions of the fine grid (h = N/2, n1 = N-1): C = [1,h]^2, X = [1,h] x
// [h+1,n1], Y = [h+1,n1] x [1,h], I = [h+1,n1]^2.  Forward apply of M^{-1}:
// I (downstream sweep), then Y and X (line solves, concurrently), then C
// (multigrid).  Transposed apply of M^{-T}: C, then X and Y, then I.
#pragma once
#include "common.h"

// Lane l receives lane l-1's value (DPP wave_shr:1); lane 0 receives 0.
BLP_DEV float wave_shr1(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, false));
}
BLP_DEV double wave_shr1(double v) {
  int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x138, 0xf, 0xf, false);
  int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x138, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

// Generic DPP move with an explicit 'old' value (kept where the source lane
// is out of range or the row is masked off).  GFX9 controls: row_shr:n
// 0x110+n, row_shl:n 0x100+n, wave_shr:1 0x138, wave_shl:1 0x130,
// row_bcast:15 0x142, row_bcast:31 0x143.
template <int CTRL, int RM = 0xF>
BLP_DEV float dpp_mov(float old, float v) {
  return __int_as_float(
      __builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(v), CTRL, RM, 0xF, false));
}
template <int CTRL, int RM = 0xF>
BLP_DEV double dpp_mov(double old, double v) {
  const int lo = __builtin_amdgcn_update_dpp(__double2loint(old), __double2loint(v), CTRL, RM, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(__double2hiint(old), __double2hiint(v), CTRL, RM, 0xF, false);
  return __hiloint2double(hi, lo);
}
BLP_DEV float read_lane(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
BLP_DEV double read_lane(double v, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                          __builtin_amdgcn_readlane(__double2loint(v), l));
}

// Inclusive wave scan of affine maps x -> A + M x, composed from lane 0
// upward (lane l ends with the composition of lanes 0..l).  In-row
// Hillis-Steele steps by DPP row shifts, then the row_bcast15/31 steps carry
// the row totals across rows; the identity map (0, 1) fills missing sources.
template <typename T>
BLP_DEV void scan_affine_up(T &A, T &M) {
#define BLP_COMBINE(CTRL, RM)                                      \
  {                                                               \
    const T a_ = dpp_mov<CTRL, RM>(T(0), A), m_ = dpp_mov<CTRL, RM>(T(1), M); \
    A = A + M * a_;                                               \
    M = M * m_;                                                   \
  }
  BLP_COMBINE(0x111, 0xF)
  BLP_COMBINE(0x112, 0xF)
  BLP_COMBINE(0x114, 0xF)
  BLP_COMBINE(0x118, 0xF)
  BLP_COMBINE(0x142, 0xA)
  BLP_COMBINE(0x143, 0xC)
}

// Suffix version: lane l ends with the composition of lanes 63..l applied to
// a zero value beyond lane 63 (only A is meaningful on exit).  In-row steps
// by DPP row_shl; the three row totals cross rows through readlane.
template <typename T>
BLP_DEV void scan_affine_down(T &A, T &M, int lane) {
  BLP_COMBINE(0x101, 0xF)
  BLP_COMBINE(0x102, 0xF)
  BLP_COMBINE(0x104, 0xF)
  BLP_COMBINE(0x108, 0xF)
#undef BLP_COMBINE
  const T A48 = read_lane(A, 48);
  const T A32 = read_lane(A, 32), M32 = read_lane(M, 32);
  const T A16 = read_lane(A, 16), M16 = read_lane(M, 16);
  const T S3 = A48;
  const T S2 = A32 + M32 * S3;
  const T S1 = A16 + M16 * S2;
  const int row = lane >> 4;
  const T Sin = row == 0 ? S1 : (row == 1 ? S2 : (row == 2 ? S3 : T(0)));
  A = A + M * Sin;
}

// ---------------------------------------------------------------------------
// Wavefront-major ("skewed") layout.
//
// A downstream sweep over the rectangle [i0,i1] x [j0,j1] visits column c
// (c = 0 first: i1 - c forward, i0 + c transposed) and row t (t = 0 first:
// j1 - t forward, j0 + t transposed).  Columns are grouped in bands of 64;
// lane l = c mod 64 handles node (c, t) at step s = t + l.  In this layout
// node (c, t) is stored at ((band * (mr + 64)) + t + l) * 64 + l, so the 64
// lanes of a band read and write 64 consecutive words at every step.  Step
// index mr + 63 of each band is never a node (a sink row for idle steps).
// ---------------------------------------------------------------------------
template <bool TR>
struct Skew {
  int i0, i1, j0, j1;
  BLP_DEV int mc() const { return i1 - i0 + 1; }
  BLP_DEV int mr() const { return j1 - j0 + 1; }
  BLP_DEV int col(int i) const { return TR ? i - i0 : i1 - i; }
  BLP_DEV int row(int j) const { return TR ? j - j0 : j1 - j; }
  BLP_DEV int icol(int c) const { return TR ? i0 + c : i1 - c; }
  BLP_DEV int jrow(int t) const { return TR ? j0 + t : j1 - t; }
  BLP_DEV size_t slot(int band, int s, int lane) const {
    return ((size_t)band * (mr() + 64) + s) * 64 + lane;
  }
  BLP_DEV size_t at_ct(int c, int t) const { return slot(c >> 6, t + (c & 63), c & 63); }
  BLP_DEV size_t at(int i, int j) const { return at_ct(col(i), row(j)); }
  // slot index -> node; false on padding
  BLP_DEV bool decode(size_t q, int &i, int &j) const {
    const int lane = (int)(q & 63);
    const size_t r = q >> 6;
    const int band = (int)(r / (size_t)(mr() + 64)), s = (int)(r % (size_t)(mr() + 64));
    const int c = band * 64 + lane, t = s - lane;
    if (c >= mc() || t < 0 || t >= mr()) return false;
    i = icol(c);
    j = jrow(t);
    return true;
  }
};
inline size_t skew_size(int mc, int mr) { return (size_t)((mc + 63) / 64) * (mr + 64) * 64; }

// ---------------------------------------------------------------------------
// Downstream triangular sweep on a rectangle of a grid.
//
// Forward (TR = false) solves, from the top-right corner to the bottom-left,
//   C_ij z_ij + E_i z_{i+1,j} + N_j z_{i,j+1} = rhs_ij
// (the upper-triangular part of the block: M_II of Sec. 3.1, and the
// downstream pointwise Gauss-Seidel of Sec. 3.2, whose not-yet-updated
// neighbour terms k_gs_rhs folds into rhs beforehand).  Transposed
// (TR = true) solves the transpose from the bottom-left corner:
//   C_ij z_ij + E_{i-1} z_{i-1,j} + N_{j-1} z_{i,j-1} = rhs_ij.
// Values just outside the rectangle on its upstream sides come from zb (a
// grid vector in natural layout, e.g. already-solved neighbouring regions)
// when they lie inside the grid, else are zero.
//
// rhs, 1/C and z are in the skewed layout of the rectangle.  One workgroup;
// wave w owns band w, lane l one column.  The upstream-column value comes
// from lane l-1 by a DPP shift, the upstream-row value is the lane's own
// previous result.  Band w runs LAG = 64 + K steps behind band w-1 and takes
// the band-boundary column from an LDS ring; an LDS-only barrier every K
// steps (a superstep) orders the ring traffic.
//
// Memory pipelining: a wave that both loads and stores can only wait for all
// of its outstanding memory operations at once, so work is organised by
// supersteps with two register buffers: at the start of superstep m the wave
// stores the results of superstep m-1 and issues the loads of superstep m+1,
// then computes superstep m from registers.  Every operation outstanding at
// the next wait was issued a whole superstep earlier.  Step offsets are
// wave-uniform (scalar arithmetic); lanes add a constant lane offset.
// ---------------------------------------------------------------------------
template <typename T>
struct SweepArgs {
  Grid<T> g;
  int i0, i1, j0, j1;
  const T *b;     // skewed rhs
  const T *ic;    // skewed 1/C
  T *z;           // skewed solution
  const T *zb;    // natural-layout source of upstream boundary values, or null
  const int *gate;
};

constexpr int kSweepMaxRows = 1024;

// Workgroup barrier that waits for this wave's LDS traffic only (global
// loads and stores may stay in flight): s_waitcnt lgkmcnt(0) with vmcnt and
// expcnt at their maxima (GFX9 encoding 0xC07F), then s_barrier.
BLP_DEV void lds_barrier() {
  __builtin_amdgcn_s_waitcnt(0xC07F);
  __builtin_amdgcn_s_barrier();
}

template <typename T, bool TR, int K>
__global__ __launch_bounds__(K > 8 ? 512 : 1024) void k_sweep(SweepArgs<T> a) {
  if (a.gate && *a.gate) return;
  constexpr int LAG = 64 + K, RING = 64;
  __shared__ T ring[16][RING];
  __shared__ T bnd[kSweepMaxRows];  // upstream boundary column, by row t
  __shared__ T ycu[kSweepMaxRows];  // upstream y coupling, by row t
  const Grid<T> &g = a.g;
  const Skew<TR> sk{a.i0, a.i1, a.j0, a.j1};
  const int mc = sk.mc(), mr = sk.mr();
  const int ib = TR ? a.i0 - 1 : a.i1 + 1;
  const bool ib_in = a.zb && ib >= 1 && ib <= g.nx;
  for (int t = threadIdx.x; t < mr; t += blockDim.x) {
    const int j = sk.jrow(t);
    ycu[t] = TR ? g.N[j - 1] : g.N[j];
    bnd[t] = ib_in ? a.zb[vidx(ib, j, g.nx)] : T(0);
  }
  __syncthreads();

  const int lane = threadIdx.x & 63;
  const int band = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
  const int nb = blockDim.x >> 6;
  const int c = band * 64 + lane;
  const bool colok = c < mc;
  const int i = sk.icol(colok ? c : mc - 1);
  const T cu = colok ? (TR ? g.E[i - 1] : g.E[i]) : T(0);  // upstream x coupling
  const int jb = TR ? a.j0 - 1 : a.j1 + 1;
  T zrow = (colok && a.zb && jb >= 1 && jb <= g.ny) ? a.zb[vidx(i, jb, g.nx)] : T(0);
  T zlast = T(0);
  const int total = (nb - 1) * LAG + mr + 63;
  const int smax = mr + 63;  // steps 0..smax-1 are the band's work, smax its sink row
  // this band's storage; step s of lane l is element (s * 64 + l)
  const T *__restrict__ bb = a.b + sk.slot(band, 0, 0);
  const T *__restrict__ ib_ = a.ic + sk.slot(band, 0, 0);
  T *__restrict__ zz = a.z + sk.slot(band, 0, 0);
  auto clampstep = [&](int s) { return (s >= 0 && s < smax) ? s : smax; };

  T Ab[K], Ai[K], Bb[K], Bi[K], res[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int s = clampstep(k - band * LAG);
    Ab[k] = bb[s * 64 + lane];
    Ai[k] = ib_[s * 64 + lane];
    res[k] = T(0);
  }
  int s_prev = -(1 << 20);  // first local step of the results held in res

  // one superstep: store previous results, prefetch the next superstep into
  // (Nb, Ni), compute from (Cb, Ci) into res
  auto superstep = [&](int s0, T (&Cb)[K], T (&Ci)[K], T (&Nb)[K], T (&Ni)[K]) {
    const int sl = s0 - band * LAG;  // local step of k = 0
#pragma unroll
    for (int k = 0; k < K; ++k) zz[clampstep(s_prev + k) * 64 + lane] = res[k];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int s = clampstep(sl + K + k);
      Nb[k] = bb[s * 64 + lane];
      Ni[k] = ib_[s * 64 + lane];
    }
    // LDS operands of the superstep, read up front so that no LDS latency
    // sits on the step-to-step dependency chain (the ring rows read here were
    // written at least one superstep earlier)
    T yc[K], zb0[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int s = sl + k;
      const int t = s - lane;
      yc[k] = ycu[t < 0 ? 0 : (t >= mr ? mr - 1 : t)];
      const int su = s < 0 ? 0 : (s >= mr ? mr - 1 : s);  // lane 0's row
      zb0[k] = band == 0 ? bnd[su] : ring[band - 1][su & (RING - 1)];
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int t = sl + k - lane;
      // Values computed on idle steps only feed idle steps of the next lane,
      // and land in padding slots; only the row carry needs masking.
      T zin = wave_shr1(zlast);
      zin = lane == 0 ? zb0[k] : zin;
      const T t1 = Cb[k] - yc[k] * zrow;
      const T zv = (t1 - cu * zin) * Ci[k];
      zrow = (t >= 0) ? zv : zrow;
      res[k] = zv;
      // ring slot t mod 64: a slot is rewritten 64 rows later, i.e. 63 - K
      // steps after its reader (band + 1) has read it
      if (lane == 63) ring[band][t & (RING - 1)] = zv;
      zlast = zv;
    }
    s_prev = sl;
    lds_barrier();
  };
  for (int s0 = 0; s0 < total; s0 += 2 * K) {
    superstep(s0, Ab, Ai, Bb, Bi);
    if (s0 + K >= total) break;
    superstep(s0 + K, Bb, Bi, Ab, Ai);
  }
#pragma unroll
  for (int k = 0; k < K; ++k) zz[clampstep(s_prev + k) * 64 + lane] = res[k];
}

// Gauss-Seidel right-hand side, folded before a smoothing sweep: with the
// current iterate z (skewed), rhs = b - (downstream couplings) * z, i.e.
// forward b - W_i z_{i-1,j} - S_j z_{i,j-1}, transposed
// b - W_{i+1} z_{i+1,j} - S_{j+1} z_{i,j+1}; the sweep then solves the
// triangular system with this rhs, which is one Gauss-Seidel sweep.
template <typename T, bool TR>
__global__ void k_gs_rhs(Grid<T> g, const T *b, const T *z, T *out, size_t nslot, const int *gate) {
  if (gate && *gate) return;
  const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nslot) return;
  const int n = g.nx;
  const Skew<TR> sk{1, n, 1, n};
  int i, j;
  if (!sk.decode(q, i, j)) {
    out[q] = T(0);
    return;
  }
  const int id = TR ? i + 1 : i - 1, jd = TR ? j + 1 : j - 1;
  T v = b[q];
  if (id >= 1 && id <= n) v -= (TR ? g.W[i + 1] : g.W[i]) * z[sk.at(id, j)];
  if (jd >= 1 && jd <= g.ny) v -= (TR ? g.S[j + 1] : g.S[j]) * z[sk.at(i, jd)];
  out[q] = v;
}

// Natural <-> skewed copies of a rectangle of the fine grid; the gather can
// multiply by dh (scaled-system input).  One thread per skewed slot.
template <typename T, bool TR>
__global__ void k_gather_skew(Skew<TR> sk, const T *v, const T *dh, int ld, T *out, size_t nslot) {
  const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nslot) return;
  int i, j;
  T val = T(0);
  if (sk.decode(q, i, j)) {
    const size_t o = vidx(i, j, ld);
    val = v[o];
    if (dh) val *= dh[o];
  }
  out[q] = val;
}
template <typename T, bool TR>
__global__ void k_scatter_skew(Skew<TR> sk, const T *in, T *z, int ld, size_t nslot) {
  const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nslot) return;
  int i, j;
  if (sk.decode(q, i, j)) z[vidx(i, j, ld)] = in[q];
}

// 1/C_ij in the skewed layout of a rectangle (setup).
template <typename T, bool TR>
__global__ void k_diag_skew(Grid<double> g, Skew<TR> sk, T *ic, size_t nslot) {
  const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nslot) return;
  int i, j;
  ic[q] = sk.decode(q, i, j) ? T(1.0 / g.C(i, j)) : T(0);
}

// ---------------------------------------------------------------------------
// Edge-layer line solves (Sec. 3.1, M_YY and M_XX): block Gauss-Seidel over
// lines, each line a tridiagonal solve by the Thomas algorithm without
// pivoting (Lemma diag_dom) with factors computed at setup.
//
// Region r has L = n1 - h lines of length h.  Line q couples to line q-1
// (already solved) through a coefficient constant along the line, and, in
// the forward direction, its last node couples to the interior region.
//   Y forward:  line q <-> i = n1-q, node p <-> j = p+1; previous line i+1
//               (E_i); last node couples to (i, h+1) through N_h.
//   X forward:  line q <-> j = n1-q, node p <-> i = p+1; previous line j+1
//               (N_j); last node couples to (h+1, j) through E_h.
//   Y transposed: line q <-> i = h+1+q, previous line i-1 (E_{i-1}); line 0
//               couples to the corner values (h, j).
//   X transposed: line q <-> j = h+1+q, previous line j-1 (N_{j-1}); line 0
//               couples to the corner values (i, h).
// Thomas factors per line: forward elimination y_p = rhs_p d_p + m_p y_{p-1},
// back substitution z_p = y_p + w_p z_{p+1} (d = 1/pivot, m = -sub/pivot,
// w = -super/pivot).
//
// Operand access: node (q, p) of region r is element off[r] + q*sq[r] + p of
// b / z (Y lines are gathered into a line-major buffer first, X lines are
// rows of the natural layout), so each line is contiguous.
//
// One wave per region; lane l holds the EP contiguous nodes p = l*EP + e.
// Each of the two recurrences is an affine scan: a sequential pass over the
// lane's nodes, a DPP wave scan across the 64 lanes, and a fix-up pass.
// ---------------------------------------------------------------------------
template <typename T>
struct LineArgs {
  Grid<T> g;          // fine grid
  int h, n1;
  const T *b[2];      // operands per region
  const T *dh[2];     // scaled-system input factor (same indexing as b) or null
  T *z[2];            // outputs per region
  long long off[2], sq[2];
  const T *znat;      // natural-layout z: coupling values of C / I
  const T *fd[2], *fm[2], *fw[2];  // factors [region 0 = Y, 1 = X], (lines x h)
  const int *gate;
};

// Operands of one line held in registers (raw loads).
template <typename T, int EP>
struct LineBuf {
  T b[EP], d[EP], m[EP], w[EP], s[EP];
  T zc;  // value of the already-solved node the line's last (forward) node couples to
};

template <typename T, bool TR, int EP>
BLP_DEV void line_load(const LineArgs<T> &a, int r, int q, int lane, LineBuf<T, EP> &B) {
  const int h = a.h, n1 = a.n1;
  const int line = TR ? h + 1 + q : n1 - q;
  const T *fd = a.fd[r], *fm = a.fm[r], *fw = a.fw[r];
  const long long lb = a.off[r] + (long long)q * a.sq[r];
#pragma unroll
  for (int e = 0; e < EP; ++e) {
    int p = lane * EP + e;
    p = p < h ? p : h - 1;  // clamp: loads stay in bounds, values are masked later
    B.b[e] = a.b[r][lb + p];
    if (a.dh[r]) B.s[e] = a.dh[r][lb + p];
    const size_t f = (size_t)q * h + p;
    B.d[e] = fd[f];
    B.m[e] = fm[f];
    B.w[e] = fw[f];
  }
  if (!TR) B.zc = r == 0 ? a.znat[vidx(line, h + 1, n1)] : a.znat[vidx(h + 1, line, n1)];
}

template <typename T, bool TR, int EP>
BLP_DEV void line_solve(const LineArgs<T> &a, int r, int q, int lane,
                        const LineBuf<T, EP> &B, T (&zprev)[EP]) {
  const int h = a.h, n1 = a.n1;
  const Grid<T> &g = a.g;
  const int line = TR ? h + 1 + q : n1 - q;
  T cprev;  // coupling to the previous line (constant along the line)
  if (r == 0) cprev = TR ? g.E[line - 1] : g.E[line];
  else cprev = TR ? g.N[line - 1] : g.N[line];
  T clast = T(0);  // coupling of the last node to the interior region (forward)
  if (!TR) clast = r == 0 ? g.N[h] : g.E[h];
  T av[EP], mv[EP], y[EP], wv[EP];
  T A = T(0), M = T(1);
#pragma unroll
  for (int e = 0; e < EP; ++e) {
    const int p = lane * EP + e;
    const bool on = p < h;
    T rhs = B.b[e];
    if (a.dh[r]) rhs *= B.s[e];
    rhs -= cprev * zprev[e];
    if (!TR && p == h - 1) rhs -= clast * B.zc;
    av[e] = on ? rhs * B.d[e] : T(0);
    mv[e] = on ? B.m[e] : T(0);
    wv[e] = on ? B.w[e] : T(0);
    A = av[e] + mv[e] * A;
    M = mv[e] * M;
  }
  scan_affine_up(A, M);
  T x = dpp_mov<0x138>(T(0), A);  // value before this lane's chunk
#pragma unroll
  for (int e = 0; e < EP; ++e) {
    x = av[e] + mv[e] * x;
    y[e] = x;
  }
  A = T(0);
  M = T(1);
#pragma unroll
  for (int e = EP - 1; e >= 0; --e) {
    A = y[e] + wv[e] * A;
    M = wv[e] * M;
  }
  scan_affine_down(A, M, lane);
  T zn = dpp_mov<0x130>(T(0), A);  // value just after this lane's chunk
#pragma unroll
  for (int e = EP - 1; e >= 0; --e) {
    zn = y[e] + wv[e] * zn;
    zprev[e] = zn;
  }
}

template <typename T, int EP>
BLP_DEV void line_store(const LineArgs<T> &a, int r, int q, int lane, const T (&zl)[EP]) {
  const long long lb = a.off[r] + (long long)q * a.sq[r];
#pragma unroll
  for (int e = 0; e < EP; ++e) {
    const int p = lane * EP + e;
    if (p < a.h) a.z[r][lb + p] = zl[e];
  }
}

// One wave per region (block 0: Y, block 1: X).  The operands of line q+1
// are loaded while line q is solved (two register buffers, alternating), and
// line q's results are stored when line q+1 starts: the wave both loads and
// stores, so it can only wait for all of its outstanding memory operations at
// once, and this order makes them all a full line old at every wait.
template <typename T, bool TR, int EP>
__global__ __launch_bounds__(64) void k_lines(LineArgs<T> a) {
  if (a.gate && *a.gate) return;
  const int r = blockIdx.x;
  const int lane = threadIdx.x;
  const int h = a.h, L = a.n1 - h;
  T zprev[EP];
#pragma unroll
  for (int e = 0; e < EP; ++e) {
    const int p = lane * EP + e;
    zprev[e] = T(0);
    // transposed: the first line couples to the corner region's edge
    if (TR && p < h) zprev[e] = r == 0 ? a.znat[vidx(h, p + 1, a.n1)] : a.znat[vidx(p + 1, h, a.n1)];
  }
  LineBuf<T, EP> A_, B_;
  line_load<T, TR, EP>(a, r, 0, lane, A_);
  for (int q = 0; q < L; q += 2) {
    if (q > 0) line_store<T, EP>(a, r, q - 1, lane, zprev);
    if (q + 1 < L) line_load<T, TR, EP>(a, r, q + 1, lane, B_);
    line_solve<T, TR, EP>(a, r, q, lane, A_, zprev);
    if (q + 1 >= L) {
      line_store<T, EP>(a, r, q, lane, zprev);
      break;
    }
    line_store<T, EP>(a, r, q, lane, zprev);
    if (q + 2 < L) line_load<T, TR, EP>(a, r, q + 2, lane, A_);
    line_solve<T, TR, EP>(a, r, q + 1, lane, B_, zprev);
    if (q + 2 >= L) line_store<T, EP>(a, r, q + 1, lane, zprev);
  }
}

// Y-region lines <-> line-major buffer: element (q, p) <-> (i(q), p+1),
// i(q) = n1-q (forward) or h+1+q (transposed); the gather multiplies by dh.
template <typename T, bool TR>
__global__ void k_gather_lines(const T *v, const T *dh, int h, int n1, T *out) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const int q = blockIdx.y;
  if (p >= h) return;
  const int i = TR ? h + 1 + q : n1 - q;
  const size_t o = vidx(i, p + 1, n1);
  T val = v[o];
  if (dh) val *= dh[o];
  out[(size_t)q * h + p] = val;
}
template <typename T, bool TR>
__global__ void k_scatter_lines(const T *in, int h, int n1, T *z) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const int q = blockIdx.y;
  if (p >= h) return;
  const int i = TR ? h + 1 + q : n1 - q;
  z[vidx(i, p + 1, n1)] = in[(size_t)q * h + p];
}

// Thomas factorisation of every line (setup).  One thread per line.
template <typename T>
__global__ void k_line_factor(Grid<T> g, int h, int n1, int region, int tr, T *fd,
                              T *fm, T *fw) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  const int L = n1 - h;
  if (q >= L) return;
  const int line = tr ? h + 1 + q : n1 - q;
  T cp = T(0);
  for (int p = 0; p < h; ++p) {
    const int i = region == 0 ? line : p + 1;
    const int j = region == 0 ? p + 1 : line;
    T sub, sup;
    if (region == 0) {  // along j: S (to j-1), N (to j+1); transposed: N_{j-1}, S_{j+1}
      sub = p > 0 ? (tr ? g.N[j - 1] : g.S[j]) : T(0);
      sup = p < h - 1 ? (tr ? g.S[j + 1] : g.N[j]) : T(0);
    } else {            // along i: W (to i-1), E (to i+1); transposed: E_{i-1}, W_{i+1}
      sub = p > 0 ? (tr ? g.E[i - 1] : g.W[i]) : T(0);
      sup = p < h - 1 ? (tr ? g.W[i + 1] : g.E[i]) : T(0);
    }
    const T den = g.C(i, j) - sub * cp;
    const T inv = T(1) / den;
    cp = sup * inv;
    const size_t f = (size_t)q * h + p;
    fd[f] = inv;
    fm[f] = -sub * inv;
    fw[f] = -cp;
  }
}

// 1/C_ij and sqrt(C_ij) on a grid in natural layout (setup).
template <typename T>
__global__ void k_diag_tables(Grid<double> g, T *ic, T *dh) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x + 1;
  const int j = blockIdx.y + 1;
  if (i > g.nx) return;
  const double C = g.C(i, j);
  if (ic) ic[vidx(i, j, g.nx)] = T(1.0 / C);
  if (dh) dh[vidx(i, j, g.nx)] = T(sqrt(C));
}

// ---------------------------------------------------------------------------
// Corner multigrid (Sec. 3.2, two exponential layers).  Level l has n_l x n_l
// unknowns; its vectors z, b, t and 1/C live in the skewed layout of the
// level grid for the direction of the cycle (forward / transposed), the
// layout the level's Gauss-Seidel sweeps run in.  Per-axis level tables:
// W/E/Dx, S/N/Dy (rediscretised on the level's widths), hb (FE rescaling
// factor hbar_i, kbar_j) and, for odd fine nodes, the interpolation weights
// wl (toward the coarse node (i-1)/2) and wr (toward (i+1)/2), linear in the
// mesh coordinate.
// ---------------------------------------------------------------------------
template <typename T>
struct MgLevel {
  Grid<T> g;
  const T *ic;  // skewed 1/C for the cycle's direction
  const T *hbx, *hby;
  const T *wlx, *wrx, *wly, *wry;
  T *z, *b, *t;
  size_t nslot;
};

template <bool TR>
BLP_DEV Skew<TR> level_skew(int n) { return Skew<TR>{1, n, 1, n}; }

// (A z)_ij (forward) or (A^T z)_ij (transposed) on a level, z skewed.
template <typename T, bool TR>
BLP_DEV T level_apply(const Grid<T> &g, const Skew<TR> &sk, const T *z, int i, int j) {
  const int n = g.nx;
  const T zc = z[sk.at(i, j)];
  const T zw = i > 1 ? z[sk.at(i - 1, j)] : T(0);
  const T ze = i < n ? z[sk.at(i + 1, j)] : T(0);
  const T zs = j > 1 ? z[sk.at(i, j - 1)] : T(0);
  const T zn = j < g.ny ? z[sk.at(i, j + 1)] : T(0);
  if (!TR) return g.C(i, j) * zc + g.W[i] * zw + g.E[i] * ze + g.S[j] * zs + g.N[j] * zn;
  return g.C(i, j) * zc + g.E[i - 1] * zw + g.W[i + 1] * ze + g.N[j - 1] * zs + g.S[j + 1] * zn;
}

// t = b - A z (forward) or b - A^T z (transposed) on a level.
template <typename T, bool TR>
__global__ void k_mg_resid(MgLevel<T> L, const int *gate) {
  if (gate && *gate) return;
  const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= L.nslot) return;
  const Skew<TR> sk = level_skew<TR>(L.g.nx);
  int i, j;
  if (!sk.decode(q, i, j)) return;
  L.t[q] = L.b[q] - level_apply<T, TR>(L.g, sk, L.z, i, j);
}

// One-dimensional transfer weight from fine node i to coarse node k
// (i in {2k-1, 2k, 2k+1}).
template <typename T>
BLP_DEV T w1d(const T *wl, const T *wr, int i, int k) {
  if (i == 2 * k) return T(1);
  if (i == 2 * k - 1) return wr[i];
  return wl[i];  // i == 2k+1
}

// Coarse right-hand side: forward b_c = S_c^{-1} P^T S_f t_f (FE rescaling,
// Sec. 3.2), transposed b_c = P^T t_f.  Gathers the 3x3 fine neighbourhood.
template <typename T, bool TR>
__global__ void k_mg_restrict(MgLevel<T> F, MgLevel<T> Cc, const int *gate) {
  if (gate && *gate) return;
  const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= Cc.nslot) return;
  const int nc = Cc.g.nx, nf = F.g.nx;
  const Skew<TR> skc = level_skew<TR>(nc), skf = level_skew<TR>(nf);
  int k, m;
  if (!skc.decode(q, k, m)) return;
  T s = T(0);
  for (int jj = 2 * m - 1; jj <= 2 * m + 1; ++jj) {
    if (jj < 1 || jj > nf) continue;
    const T wy = w1d(F.wly, F.wry, jj, m);
    for (int ii = 2 * k - 1; ii <= 2 * k + 1; ++ii) {
      if (ii < 1 || ii > nf) continue;
      T v = F.t[skf.at(ii, jj)] * w1d(F.wlx, F.wrx, ii, k) * wy;
      if (!TR) v *= F.hbx[ii] * F.hby[jj];
      s += v;
    }
  }
  if (!TR) s /= Cc.hbx[k] * Cc.hby[m];
  Cc.b[q] = s;
}

// Coarse-grid correction: forward z_f += P z_c; transposed
// z_f += S_f P S_c^{-1} z_c.
template <typename T, bool TR>
__global__ void k_mg_prolong(MgLevel<T> F, MgLevel<T> Cc, const int *gate) {
  if (gate && *gate) return;
  const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= F.nslot) return;
  const int nc = Cc.g.nx, nf = F.g.nx;
  const Skew<TR> skc = level_skew<TR>(nc), skf = level_skew<TR>(nf);
  int i, j;
  if (!skf.decode(q, i, j)) return;
  int kx[2], ky[2];
  T wx[2], wy[2];
  int nxk = 0, nyk = 0;
  if (i % 2 == 0) { kx[0] = i / 2; wx[0] = T(1); nxk = 1; }
  else {
    if ((i - 1) / 2 >= 1) { kx[nxk] = (i - 1) / 2; wx[nxk++] = F.wlx[i]; }
    kx[nxk] = (i + 1) / 2; wx[nxk++] = F.wrx[i];
  }
  if (j % 2 == 0) { ky[0] = j / 2; wy[0] = T(1); nyk = 1; }
  else {
    if ((j - 1) / 2 >= 1) { ky[nyk] = (j - 1) / 2; wy[nyk++] = F.wly[j]; }
    ky[nyk] = (j + 1) / 2; wy[nyk++] = F.wry[j];
  }
  T s = T(0);
  for (int b2 = 0; b2 < nyk; ++b2)
    for (int a2 = 0; a2 < nxk; ++a2) {
      T v = Cc.z[skc.at(kx[a2], ky[b2])];
      if (TR) v /= Cc.hbx[kx[a2]] * Cc.hby[ky[b2]];
      s += wx[a2] * wy[b2] * v;
    }
  if (TR) s *= F.hbx[i] * F.hby[j];
  F.z[q] += s;
}

// Coarsest level: four downstream Gauss-Seidel sweeps (transposed: the
// transposed sweep on A^T), by one thread, from z = 0 when zero_init (a
// coarse level) or from the current iterate (when the corner block itself is
// the coarsest level).
template <typename T, bool TR>
__global__ void k_mg_coarsest(MgLevel<T> L, int zero_init, const int *gate) {
  if (gate && *gate) return;
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const Grid<T> &g = L.g;
  const int n = g.nx;
  const Skew<TR> sk = level_skew<TR>(n);
  if (zero_init)
    for (int j = 1; j <= g.ny; ++j)
      for (int i = 1; i <= n; ++i) L.z[sk.at(i, j)] = T(0);
  for (int sweep = 0; sweep < 4; ++sweep) {
    for (int jj = 0; jj < g.ny; ++jj)
      for (int ii = 0; ii < n; ++ii) {
        const int i = TR ? ii + 1 : n - ii, j = TR ? jj + 1 : g.ny - jj;
        const T *z = L.z;
        const T zw = i > 1 ? z[sk.at(i - 1, j)] : T(0);
        const T ze = i < n ? z[sk.at(i + 1, j)] : T(0);
        const T zs = j > 1 ? z[sk.at(i, j - 1)] : T(0);
        const T zn = j < g.ny ? z[sk.at(i, j + 1)] : T(0);
        T off;
        if (!TR) off = g.W[i] * zw + g.E[i] * ze + g.S[j] * zs + g.N[j] * zn;
        else off = g.E[i - 1] * zw + g.W[i + 1] * ze + g.N[j - 1] * zs + g.S[j + 1] * zn;
        const size_t q = sk.at(i, j);
        L.z[q] = (L.b[q] - off) * L.ic[q];
      }
  }
}

// Corner stopping rule (Sec. 3.2): norm of the residual of the system the
// cycle works on -- forward ||S (b - A z)||, transposed ||b - A^T z|| -- with
// mode 0 measuring ||S b|| (resp. ||b||) before the first cycle.  The last
// block compares against rtol and sets the gate.
template <typename T, bool TR>
__global__ __launch_bounds__(256) void k_mg_norm(MgLevel<T> L, MgCtrl *ctrl, int mode,
                                                 double *partials) {
  __shared__ double sh[16];
  __shared__ bool last;
  if (ctrl->gate) return;  // uniform across the grid
  const Skew<TR> sk = level_skew<TR>(L.g.nx);
  double acc = 0.0;
  for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < L.nslot;
       q += (size_t)gridDim.x * blockDim.x) {
    int i, j;
    if (!sk.decode(q, i, j)) continue;
    double v = (double)L.b[q];
    if (mode == 1) v -= (double)level_apply<T, TR>(L.g, sk, L.z, i, j);
    if (!TR) v *= (double)L.hbx[i] * (double)L.hby[j];
    acc += v * v;
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = acc;
  if (!arrive_last(&ctrl->counter, &last)) return;
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int b2 = 0; b2 < (int)gridDim.x; ++b2) s += partials[b2];
    ctrl->counter = 0;
    if (mode == 0) {
      ctrl->bnorm2 = s;
      if (s == 0.0) ctrl->gate = 1;  // zero right-hand side: z = 0, no cycle
    } else {
      ctrl->cycles += 1;
      ctrl->res2 = s;
      if (s <= ctrl->rtol2 * ctrl->bnorm2 || ctrl->cycles >= ctrl->maxcyc) ctrl->gate = 1;
    }
    __threadfence();
  }
}

// Count a fixed-mode cycle (no norm evaluation).
__global__ void k_mg_count(MgCtrl *ctrl) { ctrl->cycles += 1; }

// ---------------------------------------------------------------------------
// Corner block: right-hand side and copy-back.
// Forward: b_C = b_C - A_CX z_X - A_CY z_Y, the couplings sitting on the
// transition column (E_h to (h+1, j) in Y) and row (N_h to (i, h+1) in X).
// b_0 is written in the skewed layout of level 0.  The kernel also resets the
// corner control block.
// ---------------------------------------------------------------------------
template <typename T, bool TR>
__global__ void k_corner_rhs(Grid<T> g, int h, int n1, const T *b, const T *dh,
                             const T *z, T *b0, MgCtrl *ctrl, int maxcyc, T rtol) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x + 1;
  const int j = blockIdx.y + 1;
  if (i == 1 && j == 1 && ctrl) {
    ctrl->gate = 0;
    ctrl->cycles = 0;
    ctrl->maxcyc = maxcyc;
    ctrl->rtol2 = (double)rtol * (double)rtol;
    ctrl->counter = 0;
  }
  if (i > h) return;
  const size_t q = vidx(i, j, n1);
  T v = b[q];
  if (dh) v *= dh[q];
  if (!TR) {
    if (i == h) v -= g.E[h] * z[vidx(h + 1, j, n1)];
    if (j == h) v -= g.N[h] * z[vidx(i, h + 1, n1)];
  }
  b0[level_skew<TR>(h).at(i, j)] = v;
}

template <typename T, bool TR>
__global__ void k_corner_copy(int h, int n1, const T *z0, T *z) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x + 1;
  const int j = blockIdx.y + 1;
  if (i > h) return;
  z[vidx(i, j, n1)] = z0[level_skew<TR>(h).at(i, j)];
}

// Sample a nodal field at every f-th node: rc(k, m) = rf(f k, f m), natural
// layout (f = 1: the corner block of the fine grid; f = 2: the next level).
template <typename T>
__global__ void k_sample(const T *rf, int ldf, int f, T *rc, int nc) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x + 1;
  const int m = blockIdx.y + 1;
  if (k > nc) return;
  rc[vidx(k, m, nc)] = rf[vidx(f * k, f * m, ldf)];
}
