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

// Suffix version: lane l ends with the composition f_l o f_{l+1} o ... o
// f_63 of the affine maps of lanes l..63 (A and M both valid).  In-row steps
// by DPP row_shl; the row totals (held by lanes 16, 32, 48) cross rows
// through readlane.
template <typename T>
BLP_DEV void scan_affine_down(T &A, T &M, int lane) {
  BLP_COMBINE(0x101, 0xF)
  BLP_COMBINE(0x102, 0xF)
  BLP_COMBINE(0x104, 0xF)
  BLP_COMBINE(0x108, 0xF)
#undef BLP_COMBINE
  const T A48 = read_lane(A, 48), M48 = read_lane(M, 48);
  const T A32 = read_lane(A, 32), M32 = read_lane(M, 32);
  const T A16 = read_lane(A, 16), M16 = read_lane(M, 16);
  // suffix of the rows after row r: S3 = id, S2 = R3, S1 = R2 o R3, S0 = R1 o S1
  const T SA2 = A48, SM2 = M48;
  const T SA1 = A32 + M32 * SA2, SM1 = M32 * SM2;
  const T SA0 = A16 + M16 * SA1, SM0 = M16 * SM1;
  const int row = lane >> 4;
  const T SA = row == 0 ? SA0 : (row == 1 ? SA1 : (row == 2 ? SA2 : T(0)));
  const T SM = row == 0 ? SM0 : (row == 1 ? SM1 : (row == 2 ? SM2 : T(1)));
  A = A + M * SA;
  M = M * SM;
}

// ---------------------------------------------------------------------------
// Wavefront-major ("skewed") layout.
//
// A downstream sweep over the rectangle [i0,i1] x [j0,j1] visits column c
// (c = 0 first: i1 - c forward, i0 + c transposed) and row t (t = 0 first:
// j1 - t forward, j0 + t transposed).  Columns are grouped in bands of 64;
// lane l = c mod 64 handles node (c, t) at step s = t + l.  Steps are grouped
// in chunks of P = 16 / sizeof(word) (2 in FP64, 4 in FP32), and the P steps
// of one lane in one chunk are contiguous:
//   node (c, t) -> ((band * nck + s / P) * 64 + l) * P + s mod P,
// so one 16-byte access per lane moves P steps of a band, and the 64 lanes of
// a wave touch 1 KiB of consecutive bytes.  A band has nck chunks, a whole
// number of groups of kSkewGroup = 4 chunks: those of steps 0 .. mr + 62 (the
// last node of the band is at step mr - 1 + 63), then at least one whole
// group that holds no node (the sink that the sweep's loads past the band's
// last step read).  Slots with t < 0 or t >= mr are padding, kept at zero in
// right-hand sides and inverse diagonals.
// ---------------------------------------------------------------------------
constexpr int kSkewGroup = 4;
template <bool TR, int P>
struct Skew {
  int i0, i1, j0, j1;
  BLP_DEV int mc() const { return i1 - i0 + 1; }
  BLP_DEV int mr() const { return j1 - j0 + 1; }
  BLP_DEV int nck() const { return ((mr() + 62) / (kSkewGroup * P) + 2) * kSkewGroup; }
  BLP_DEV int col(int i) const { return TR ? i - i0 : i1 - i; }
  BLP_DEV int row(int j) const { return TR ? j - j0 : j1 - j; }
  BLP_DEV int icol(int c) const { return TR ? i0 + c : i1 - c; }
  BLP_DEV int jrow(int t) const { return TR ? j0 + t : j1 - t; }
  // s >= 0.  32-bit arithmetic: a rectangle of at most kSweepMaxRows rows
  // and kSweepMaxBands bands holds far fewer than 2^32 slots.
  BLP_DEV size_t slot(int band, int s, int lane) const {
    const unsigned us = (unsigned)s;
    return (size_t)((((unsigned)band * (unsigned)nck() + us / P) * 64u + (unsigned)lane) * P + us % P);
  }
  BLP_DEV size_t at_ct(int c, int t) const { return slot(c >> 6, t + (c & 63), c & 63); }
  BLP_DEV size_t at(int i, int j) const { return at_ct(col(i), row(j)); }
  // decode for a slot whose wave holds 64 consecutive slots starting at a
  // multiple of 64, so that every lane lies in the same band and chunk row:
  // that pair comes from one scalar division per wave instead of an integer
  // division in every lane.  Same result as decode.
  BLP_DEV bool decode_wave(size_t q, int &i, int &j) const {
    const int e = (int)(q % P);
    const unsigned r = (unsigned)(q / P);
    const int lane = (int)(r & 63u);
    const unsigned r2 = __builtin_amdgcn_readfirstlane(r >> 6), n = (unsigned)nck();
    const unsigned band = r2 / n, sc = r2 - band * n;
    const int c = (int)band * 64 + lane, t = (int)sc * P + e - lane;
    if (c >= mc() || t < 0 || t >= mr()) return false;
    i = icol(c);
    j = jrow(t);
    return true;
  }
  // slot index -> node; false on padding
  BLP_DEV bool decode(size_t q, int &i, int &j) const {
    const int e = (int)(q % P);
    const size_t r = q / P;
    const int lane = (int)(r & 63);
    const size_t r2 = r >> 6;
    const int n = nck();
    const int band = (int)(r2 / (size_t)n), s = (int)(r2 % (size_t)n) * P + e;
    const int c = band * 64 + lane, t = s - lane;
    if (c >= mc() || t < 0 || t >= mr()) return false;
    i = icol(c);
    j = jrow(t);
    return true;
  }
};
template <typename T>
constexpr int kChunk = 16 / (int)sizeof(T);
template <typename T, bool TR>
using SkewT = Skew<TR, kChunk<T>>;
template <typename T>
inline size_t skew_size(int mc, int mr) {
  constexpr int P = kChunk<T>;
  return (size_t)((mc + 63) / 64) * (((mr + 62) / (kSkewGroup * P) + 2) * kSkewGroup) * 64 * P;
}

#include "kernels_sweep.h"


// Natural <-> skewed copies of a rectangle of the fine grid (batched over
// blockIdx.y).  The gather reads v + j ldv, can multiply by dh (scaled-system
// input) and folds the couplings to the already-solved values of z + j ldz
// just outside the rectangle's upstream sides into the right-hand side
// (forward: E_i z_{i+1,j} past column i1, N_j z_{i,j+1} past row j1;
// transposed: E_{i-1} z_{i-1,j} before column i0, N_{j-1} z_{i,j-1} before
// row j0), so that the sweep runs with zero boundary values.  One thread per
// skewed slot; padding slots get zero.  The scatter writes the rectangle of
// z + j ldz from the skewed result.
template <typename T, bool TR>
struct SkewIO {
  Grid<T> g;
  SkewT<T, TR> sk;
  const T *v;
  long long ldv;
  const T *dh;
  T *z;
  long long ldz;
  T *bbuf;        // skewed right-hand side (gather output)
  const T *zbuf;  // skewed result (scatter input)
  size_t nslot;
  const int *gate;
};
// A block moves the slots of kSkewTS steps of one band (blockIdx.x: step
// tile, blockIdx.y: band, blockIdx.z: system), which are contiguous in the
// skewed layout.  Their nodes (c, s - lane) lie on mesh rows s0 - 63 ..
// s0 + kSkewTS - 1; "virtual row" r pairs row s0 - 64 + r (lanes l >= 64 - r)
// with row s0 + r (lanes l < 64 - r), so that every lane has a node and each
// half is a contiguous piece of a mesh row; lane l of virtual row r holds step
// s0 + (r + l) mod 64.  The tile passes through LDS between the two layouts.
constexpr int kSkewTS = 64, kSkewThreads = 256, kSkewUnroll = 8;
template <typename T>
inline int skew_steps(int mr) {  // steps (slots per lane) of a band
  constexpr int P = kChunk<T>;
  return ((mr + 62) / (kSkewGroup * P) + 2) * kSkewGroup * P;
}
template <typename T, bool TR>
__global__ __launch_bounds__(kSkewThreads) void k_gather_skew(const SkewIO<T, TR> *A, const int *jp) {
  __shared__ T tile[kSkewTS][65];
  constexpr int P = kChunk<T>, NW = kSkewThreads / 64, RW = kSkewTS / NW;
  const SkewIO<T, TR> a = A[blockIdx.z];  // a copy: read before the barrier
  const int gate = read_or_zero(a.gate);
  const SkewT<T, TR> sk = a.sk;
  const int mc = sk.mc(), mr = sk.mr(), ns = sk.nck() * P;
  const int band = blockIdx.y, s0 = blockIdx.x * kSkewTS;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const Grid<T> &g = a.g;
  const int ld = g.nx;
  const BLP_GLOBAL T *v = gptr(a.v + step_of(jp) * a.ldv);
  const BLP_GLOBAL T *zb = gptr(a.z + step_of(jp) * a.ldz);
  // scaling factors (absent: read v again and leave the value as it is)
  const bool scaled = a.dh != nullptr;
  const BLP_GLOBAL T *dh = gptr(scaled ? a.dh : a.v + step_of(jp) * a.ldv);
  const int c = band * 64 + lane;
  const int i = sk.icol(c < mc ? c : mc - 1);
  // wave w takes virtual rows w, w + NW, ..; kSkewUnroll of them per round,
  // loads first (node reads at clamped in-range positions)
  const BLP_GLOBAL T *gE = gptr(g.E), *gN = gptr(g.N);
#pragma unroll
  for (int r0 = 0; r0 < RW; r0 += kSkewUnroll) {
    T xs[kSkewUnroll], ys[kSkewUnroll];
#pragma unroll
    for (int u = 0; u < kSkewUnroll; ++u) {
      const int r = w + (r0 + u) * NW;
      const int t = lane >= 64 - r ? s0 - 64 + r : s0 + r;
      const size_t o = vidx(i, sk.jrow(t < 0 ? 0 : (t < mr ? t : mr - 1)), ld);
      xs[u] = v[o];
      ys[u] = dh[o];
    }
    // the loads above are issued before any value is selected (a select
    // could otherwise become a branch that holds them)
    BLP_ISSUED();
#pragma unroll
    for (int u = 0; u < kSkewUnroll; ++u) {
      const int r = w + (r0 + u) * NW;
      const int t = lane >= 64 - r ? s0 - 64 + r : s0 + r;
      const bool in = c < mc && t >= 0 && t < mr;
      T val = in ? (scaled ? xs[u] * ys[u] : xs[u]) : T(0);
      // couplings to the solved values past the rectangle's upstream sides
      // (edge nodes only)
      if (in) {
        const int j = sk.jrow(t);
        if (!TR) {
          if (i == sk.i1 && i < g.nx) val -= gE[i] * zb[vidx(i + 1, j, ld)];
          if (j == sk.j1 && j < g.ny) val -= gN[j] * zb[vidx(i, j + 1, ld)];
        } else {
          if (i == sk.i0 && i > 1) val -= gE[i - 1] * zb[vidx(i - 1, j, ld)];
          if (j == sk.j0 && j > 1) val -= gN[j - 1] * zb[vidx(i, j - 1, ld)];
        }
      }
      tile[(r + lane) & 63][lane] = val;
    }
  }
  BLP_ISSUED();
  if (gate) return;
  __syncthreads();
  // the tile's slots: o = (chunk * 64 + lane) * P + e holds step s0 + chunk P + e
  BLP_GLOBAL T *out = gptr(a.bbuf + sk.slot(band, s0, 0));
  const int no = min(kSkewTS, ns - s0) * 64;
  for (int o = tid; o < no; o += kSkewThreads) out[o] = tile[(o / (64 * P)) * P + o % P][(o / P) & 63];
}
template <typename T, bool TR>
__global__ __launch_bounds__(kSkewThreads) void k_scatter_skew(const SkewIO<T, TR> *A, const int *jp) {
  __shared__ T tile[kSkewTS][65];
  constexpr int P = kChunk<T>, NW = kSkewThreads / 64, RW = kSkewTS / NW;
  const SkewIO<T, TR> a = A[blockIdx.z];  // a copy: read before the barrier
  const int gate = read_or_zero(a.gate);
  const SkewT<T, TR> sk = a.sk;
  const int mc = sk.mc(), mr = sk.mr(), ns = sk.nck() * P;
  const int band = blockIdx.y, s0 = blockIdx.x * kSkewTS;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const BLP_GLOBAL T *in = gptr(a.zbuf + sk.slot(band, s0, 0));
  const int no = min(kSkewTS, ns - s0) * 64;
  constexpr int NO = kSkewTS * 64 / kSkewThreads;
  T x[NO];
#pragma unroll
  for (int k = 0; k < NO; ++k) {
    const int o = tid + k * kSkewThreads;
    x[k] = in[o < no ? o : no - 1];
  }
  BLP_ISSUED();
#pragma unroll
  for (int k = 0; k < NO; ++k) {
    const int o = tid + k * kSkewThreads;
    if (o < no) tile[(o / (64 * P)) * P + o % P][(o / P) & 63] = x[k];
  }
  if (gate) return;
  __syncthreads();
  BLP_GLOBAL T *z = gptr(a.z + step_of(jp) * a.ldz);
  BLP_GLOBAL T *zs = gptr(const_cast<T *>(a.zbuf) + sk.slot(band, s0, 0));
  const int ld = a.g.nx;
  const int c = band * 64 + lane;
  const int i = sk.icol(c < mc ? c : mc - 1);
  // every lane stores (all addresses first, so that no store waits for the
  // one before it to release its address registers): a node goes to z; a
  // padding slot is written back unchanged to its own place in the skewed
  // buffer, and a lane whose step lies past the band's last slot (s >= ns,
  // no slot: last tile of a band) writes the tile's first slot back
  // unchanged.  Each block owns its tile's slots and has read them above.
  T val[RW];
  BLP_GLOBAL T *dst[RW];
#pragma unroll
  for (int k = 0; k < RW; ++k) {
    const int r = w + k * NW, sl = (r + lane) & 63;
    const int t = lane >= 64 - r ? s0 - 64 + r : s0 + r;
    const bool node = c < mc && t >= 0 && t < mr;  // implies s0 + sl < ns
    const bool slot = s0 + sl < ns;
    val[k] = slot ? tile[sl][lane] : tile[0][0];
    dst[k] = node ? z + vidx(i, sk.jrow(node ? t : 0), ld)
                  : zs + (slot ? ((sl / P) * 64 + lane) * P + sl % P : 0);
  }
#pragma unroll
  for (int k = 0; k < RW; ++k) *dst[k] = val[k];
}

// 1/C_ij in the skewed layout of a rectangle (setup).
template <typename T, bool TR>
__global__ void k_diag_skew(Grid<double> g, SkewT<T, TR> sk, T *ic, size_t nslot) {
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
// Region r (0 = Y, 1 = X) has L = n1 - h lines of length h; line q couples
// to line q-1 through a coefficient constant along the line.
//   Y forward:  line q <-> i = n1-q, node p <-> j = p+1; previous line i+1
//               (E_i); node h-1 couples to (i, h+1) in I through N_h.
//   X forward:  line q <-> j = n1-q, node p <-> i = p+1; previous line j+1
//               (N_j); node h-1 couples to (h+1, j) in I through E_h.
//   Y transposed: line q <-> i = h+1+q, previous line i-1 (E_{i-1}); line 0
//               couples to the corner values (h, j) through E_h.
//   X transposed: line q <-> j = h+1+q, previous line j-1 (N_{j-1}); line 0
//               couples to the corner values (i, h) through N_h.
// The couplings to the already-solved regions (I, resp. C) are folded into
// the right-hand side by k_gather_lines, which also applies the scaled-system
// factor and writes both regions line-major with row stride hp (h rounded up
// to a multiple of 4, padding zero), so that the kernel only sees
//   T_q z_q = b_q - c_q z_{q-1},  z_{-1} = 0.
// Thomas factors per line: forward elimination y_p = rhs_p d_p + m_p y_{p-1},
// back substitution z_p = y_p + w_p z_{p+1} (d = 1/pivot, m = -sub/pivot,
// w = -super/pivot); zero in padding, so padding nodes give y = z = 0.
//
// One workgroup of W waves per region; thread g holds the EP contiguous
// nodes p = g EP + e (one or two 16-byte accesses per operand); FULL
// variants serve lines whose stride hp is exactly 64 W EP.  Each
// recurrence is an affine scan: a sequential pass over the thread's nodes, a
// DPP scan across the wave, the wave totals combined through LDS (one
// barrier per scan), and a fix-up pass.  The operands of D lines ahead are in flight
// (D + 1 register buffers rotated by unrolling); line q's results are stored
// when line q+1 starts.
// ---------------------------------------------------------------------------
template <typename T>
struct LineArgs {
  Grid<T> g;          // fine grid (line couplings)
  int h, n1, hp;
  const T *b[2];      // gathered right-hand sides [region], line-major, stride hp
  T *z[2];            // results [region], same layout
  const T *fd[2], *fm[2], *fw[2];  // factors [region], same layout
  const int *gate;
};

template <typename T, int EP>
BLP_DEV void load_ep(const BLP_GLOBAL T *p, T (&x)[EP]) {
  if constexpr (EP == 1) {
    x[0] = p[0];
  } else {
    constexpr int VW = 16 / (int)sizeof(T) < EP ? 16 / (int)sizeof(T) : EP;
    typedef T V __attribute__((ext_vector_type(VW)));
#pragma unroll
    for (int k = 0; k < EP / VW; ++k) {
      const V v = reinterpret_cast<const BLP_GLOBAL V *>(p)[k];
#pragma unroll
      for (int e = 0; e < VW; ++e) x[k * VW + e] = v[e];
    }
  }
}
template <typename T, int EP>
BLP_DEV void store_ep(BLP_GLOBAL T *p, const T (&x)[EP]) {
  if constexpr (EP == 1) {
    p[0] = x[0];
  } else {
    constexpr int VW = 16 / (int)sizeof(T) < EP ? 16 / (int)sizeof(T) : EP;
    typedef T V __attribute__((ext_vector_type(VW)));
#pragma unroll
    for (int k = 0; k < EP / VW; ++k) {
      V v;
#pragma unroll
      for (int e = 0; e < VW; ++e) v[e] = x[k * VW + e];
      reinterpret_cast<BLP_GLOBAL V *>(p)[k] = v;
    }
  }
}

template <typename T, int EP>
struct LineOps {
  T b[EP], d[EP], m[EP], w[EP];
  T c;  // coupling to the previous line
};

template <typename T, bool TR, int EP, int W, int D, bool FULL>
__global__ __launch_bounds__(64 * W) void k_lines(const LineArgs<T> *A) {
  const LineArgs<T> a = A[blockIdx.x >> 1];  // two workgroups (regions) per system
  if (gated(a.gate)) return;
  // wave totals of the forward and of the backward scan (separate, so that
  // one barrier per scan orders every write after all reads of the previous
  // use)
  __shared__ T fwA[W], fwM[W], bwA[W], bwM[W];
  const int r = blockIdx.x & 1;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int h = a.h, hp = a.hp, L = a.n1 - h;
  const Grid<T> &g = a.g;
  // this thread's nodes; threads past the line read node 0 and are masked
  // (FULL: the threads' nodes are exactly the line's hp, none is past it)
  const bool act = FULL || tid * EP < hp;
  const size_t toff = act ? (size_t)tid * EP : 0;
  // region pointers picked by selects (an index into the record's arrays by
  // the runtime region would place the record in private memory)
  const BLP_GLOBAL T *__restrict__ bp = gptr((r ? a.b[1] : a.b[0]) + toff);
  const BLP_GLOBAL T *__restrict__ dp = gptr((r ? a.fd[1] : a.fd[0]) + toff);
  const BLP_GLOBAL T *__restrict__ mp = gptr((r ? a.fm[1] : a.fm[0]) + toff);
  const BLP_GLOBAL T *__restrict__ wp = gptr((r ? a.fw[1] : a.fw[0]) + toff);
  BLP_GLOBAL T *__restrict__ zp = gptr((r ? a.z[1] : a.z[0]) + toff);
  const BLP_GLOBAL T *cc = gptr(r == 0 ? g.E : g.N);  // previous-line coupling table

  auto load = [&](int q, LineOps<T, EP> &B) {
    const int qq = q < L ? q : L - 1;  // loads past the last line stay in bounds
    const size_t o = (size_t)qq * hp;
    load_ep<T, EP>(bp + o, B.b);
    load_ep<T, EP>(dp + o, B.d);
    load_ep<T, EP>(mp + o, B.m);
    load_ep<T, EP>(wp + o, B.w);
    const int line = TR ? h + 1 + qq : a.n1 - qq;
    B.c = qq == 0 ? T(0) : (TR ? cc[line - 1] : cc[line]);
  };
  T zl[EP];  // results of the latest line (the next line's coupling values)
#pragma unroll
  for (int e = 0; e < EP; ++e) zl[e] = T(0);
  int q_prev = -1;

  auto solve = [&](int q, const LineOps<T, EP> &B) {
    if (q_prev >= 0 && act) store_ep<T, EP>(zp + (size_t)q_prev * hp, zl);
    T av[EP], y[EP];
    T A = T(0), M = T(1);
#pragma unroll
    for (int e = 0; e < EP; ++e) {
      av[e] = act ? (B.b[e] - B.c * zl[e]) * B.d[e] : T(0);
      const T m = act ? B.m[e] : T(0);
      A = av[e] + m * A;
      M = m * M;
    }
    scan_affine_up(A, M);
    T xin = dpp_mov<0x138>(T(0), A), xm = dpp_mov<0x138>(T(1), M);  // exclusive prefix
    if constexpr (W > 1) {
      if (lane == 63) {
        fwA[wv] = A;
        fwM[wv] = M;
      }
      lds_barrier();
      T x0 = T(0);
      for (int v = 0; v < wv; ++v) x0 = fwA[v] + fwM[v] * x0;
      xin = xin + xm * x0;
    }
    T x = xin;
#pragma unroll
    for (int e = 0; e < EP; ++e) {
      x = av[e] + (act ? B.m[e] : T(0)) * x;
      y[e] = x;
    }
    A = T(0);
    M = T(1);
#pragma unroll
    for (int e = EP - 1; e >= 0; --e) {
      const T w = act ? B.w[e] : T(0);
      A = y[e] + w * A;
      M = w * M;
    }
    scan_affine_down(A, M, lane);
    T zin = dpp_mov<0x130>(T(0), A), zm = dpp_mov<0x130>(T(1), M);  // exclusive suffix
    if constexpr (W > 1) {
      if (lane == 0) {
        bwA[wv] = A;
        bwM[wv] = M;
      }
      lds_barrier();
      T zr = T(0);
      for (int v = W - 1; v > wv; --v) zr = bwA[v] + bwM[v] * zr;
      zin = zin + zm * zr;
    }
    T zn = zin;
#pragma unroll
    for (int e = EP - 1; e >= 0; --e) {
      zn = y[e] + (act ? B.w[e] : T(0)) * zn;
      zl[e] = zn;
    }
    q_prev = q;
  };

  LineOps<T, EP> buf[D + 1];
#pragma unroll
  for (int u = 0; u < D; ++u) load(u, buf[u]);
  int q = 0;
  for (; q + D < L; q += D + 1) {
#pragma unroll
    for (int u = 0; u <= D; ++u) {
      load(q + u + D, buf[(u + D) % (D + 1)]);
      solve(q + u, buf[u]);
    }
  }
#pragma unroll
  for (int u = 0; u < D; ++u) {
    if (q + u < L) {
      load(q + u + D, buf[(u + D) % (D + 1)]);
      solve(q + u, buf[u]);
    }
  }
  if (act) store_ep<T, EP>(zp + (size_t)q_prev * hp, zl);
}

// Natural layout -> line-major buffers of both edge regions, and back
// (blockIdx.z = 2 * system + region).  The gather reads v + j ldv, scales by
// dh and folds in the couplings to already-solved regions (see above), read
// from z + j ldz; padding nodes p in [h, hp) get zero.  The scatter writes
// the edge regions of z + j ldz.
//
// A block moves a tile of kLineTQ lines by kLineTP nodes.  In the X region
// (r = 1) a line is a mesh row, contiguous in both layouts, and the tile is
// copied directly.  In the Y region (r = 0) a line is a mesh column: the
// tile passes through LDS so that the natural side is accessed along rows
// (consecutive lines) and the line-major side along lines (consecutive
// nodes).
constexpr int kLineTQ = 32, kLineTP = 64, kLineThreads = 256;
template <typename T>
struct LineIO {
  Grid<T> g;
  int h, n1, hp;
  const T *v;
  long long ldv;
  const T *dh;
  T *z;
  long long ldz;
  T *bL[2];        // gathered right-hand sides [Y, X]
  const T *zL[2];  // line results [Y, X]
  const int *gate;
};
// Gathered value of node p of line q in region r (p < h).
template <typename T, bool TR>
BLP_DEV T line_gather_node(const LineIO<T> &a, const BLP_GLOBAL T *v, const BLP_GLOBAL T *dh,
                           const BLP_GLOBAL T *z, int r, int q, int p) {
  const int h = a.h, n1 = a.n1;
  const int line = TR ? h + 1 + q : n1 - q;
  const int i = r == 0 ? line : p + 1, j = r == 0 ? p + 1 : line;
  const size_t k = vidx(i, j, n1);
  T val = v[k];
  if (dh) val *= dh[k];
  if (!TR) {
    if (p == h - 1) val -= r == 0 ? a.g.N[h] * z[vidx(i, h + 1, n1)] : a.g.E[h] * z[vidx(h + 1, j, n1)];
  } else if (q == 0) {
    val -= r == 0 ? a.g.E[h] * z[vidx(h, j, n1)] : a.g.N[h] * z[vidx(i, h, n1)];
  }
  return val;
}
template <typename T, bool TR>
__global__ __launch_bounds__(kLineThreads) void k_gather_lines(const LineIO<T> *A, const int *jp) {
  __shared__ T tile[kLineTP][kLineTQ + 1];
  const LineIO<T> &a = A[blockIdx.z >> 1];
  if (gated(a.gate)) return;
  const int r = blockIdx.z & 1, h = a.h, hp = a.hp, L = a.n1 - h;
  const int p0 = blockIdx.x * kLineTP, q0 = blockIdx.y * kLineTQ, tid = threadIdx.x;
  const BLP_GLOBAL T *v = gptr(a.v + step_of(jp) * a.ldv);
  const BLP_GLOBAL T *z = gptr(a.z + step_of(jp) * a.ldz);
  const BLP_GLOBAL T *dh = gptr(a.dh);
  BLP_GLOBAL T *out = gptr(a.bL[r]);
  constexpr int NE = kLineTQ * kLineTP / kLineThreads;
  if (r == 1) {
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      const int p = p0 + tid % kLineTP, q = q0 + tid / kLineTP + e * (kLineThreads / kLineTP);
      if (q < L && p < hp) out[(size_t)q * hp + p] = p < h ? line_gather_node<T, TR>(a, v, dh, z, 1, q, p) : T(0);
    }
    return;
  }
#pragma unroll
  for (int e = 0; e < NE; ++e) {
    const int ql = tid % kLineTQ, pl = tid / kLineTQ + e * (kLineThreads / kLineTQ);
    const int q = q0 + ql, p = p0 + pl;
    tile[pl][ql] = (q < L && p < h) ? line_gather_node<T, TR>(a, v, dh, z, 0, q, p) : T(0);
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < NE; ++e) {
    const int pl = tid % kLineTP, ql = tid / kLineTP + e * (kLineThreads / kLineTP);
    const int q = q0 + ql, p = p0 + pl;
    if (q < L && p < hp) out[(size_t)q * hp + p] = tile[pl][ql];
  }
}
template <typename T, bool TR>
__global__ __launch_bounds__(kLineThreads) void k_scatter_lines(const LineIO<T> *A, const int *jp) {
  __shared__ T tile[kLineTP][kLineTQ + 1];
  const LineIO<T> &a = A[blockIdx.z >> 1];
  if (gated(a.gate)) return;
  const int r = blockIdx.z & 1, h = a.h, hp = a.hp, n1 = a.n1, L = n1 - h;
  const int p0 = blockIdx.x * kLineTP, q0 = blockIdx.y * kLineTQ, tid = threadIdx.x;
  BLP_GLOBAL T *z = gptr(a.z + step_of(jp) * a.ldz);
  const BLP_GLOBAL T *zl = gptr(a.zL[r]);
  constexpr int NE = kLineTQ * kLineTP / kLineThreads;
  if (r == 1) {
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      const int p = p0 + tid % kLineTP, q = q0 + tid / kLineTP + e * (kLineThreads / kLineTP);
      const int line = TR ? h + 1 + q : n1 - q;
      if (q < L && p < h) z[vidx(p + 1, line, n1)] = zl[(size_t)q * hp + p];
    }
    return;
  }
#pragma unroll
  for (int e = 0; e < NE; ++e) {
    const int pl = tid % kLineTP, ql = tid / kLineTP + e * (kLineThreads / kLineTP);
    const int q = q0 + ql, p = p0 + pl;
    if (q < L && p < h) tile[pl][ql] = zl[(size_t)q * hp + p];
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < NE; ++e) {
    const int ql = tid % kLineTQ, pl = tid / kLineTQ + e * (kLineThreads / kLineTQ);
    const int q = q0 + ql, p = p0 + pl;
    const int line = TR ? h + 1 + q : n1 - q;
    if (q < L && p < h) z[vidx(line, p + 1, n1)] = tile[pl][ql];
  }
}

// Thomas factorisation of every line (setup), row stride hp; the padding
// stays as allocated (zero).  One thread per line.
template <typename T>
__global__ void k_line_factor(Grid<T> g, int h, int n1, int hp, int region, int tr, T *fd,
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
    const size_t f = (size_t)q * hp + p;
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

// One system's view of a level for the batched cycle kernels
// (blockIdx.y selects the record): the level, the next coarser level
// (transfers), the corner control block (its gate switches every kernel of
// the cycle off) and the norm partials.
template <typename T>
struct MgArgs {
  MgLevel<T> L, Cc;
  MgCtrl *ctrl;
  double *partials;
};

// A level with its pointers in the global space (device-side view).
template <typename T>
struct MgLevelG {
  GridG<T> g;
  const BLP_GLOBAL T *ic, *hbx, *hby, *wlx, *wrx, *wly, *wry;
  BLP_GLOBAL T *z, *b, *t;
};
template <typename T>
BLP_DEV MgLevelG<T> lview(const MgLevel<T> &L) {
  return MgLevelG<T>{gview(L.g),  gptr(L.ic),  gptr(L.hbx), gptr(L.hby), gptr(L.wlx), gptr(L.wrx),
                     gptr(L.wly), gptr(L.wry), gptr(L.z),   gptr(L.b),   gptr(L.t)};
}

template <typename T, bool TR>
BLP_DEV SkewT<T, TR> level_skew(int n) { return SkewT<T, TR>{1, n, 1, n}; }

// (A z)_ij (forward) or (A^T z)_ij (transposed) on a level, z skewed, in
// FP64 arithmetic whatever the storage precision (residuals of the FP32
// cycle would otherwise lose the digits that cancel in b - A z).  A
// neighbour outside the level is read at the node itself and counts as
// zero: every load is unconditional, so all of them are in flight together
// (a load under a condition is waited for before the branch joins).
template <typename T, bool TR>
BLP_DEV double level_apply(const GridG<T> &g, const SkewT<T, TR> &sk, const BLP_GLOBAL T *z, int i,
                           int j) {
  const int n = g.nx;
  const bool hw = i > 1, he = i < n, hs = j > 1, hn = j < g.ny;
  const double zc = z[sk.at(i, j)];
  const double lw = z[sk.at(hw ? i - 1 : i, j)], le = z[sk.at(he ? i + 1 : i, j)];
  const double ls = z[sk.at(i, hs ? j - 1 : j)], ln = z[sk.at(i, hn ? j + 1 : j)];
  const double zw = hw ? lw : 0.0, ze = he ? le : 0.0, zs = hs ? ls : 0.0, zn = hn ? ln : 0.0;
  const double C = (double)g.Dx[i] + (double)g.Dy[j] + (double)g.rr(i, j);
  if (!TR)
    return C * zc + (double)g.W[i] * zw + (double)g.E[i] * ze + (double)g.S[j] * zs +
           (double)g.N[j] * zn;
  return C * zc + (double)g.E[i - 1] * zw + (double)g.W[i + 1] * ze + (double)g.N[j - 1] * zs +
         (double)g.S[j + 1] * zn;
}

// Gauss-Seidel right-hand side, folded before a smoothing sweep: with the
// current iterate z (skewed), t = b - (downstream couplings) * z, i.e.
// forward b - W_i z_{i-1,j} - S_j z_{i,j-1}, transposed
// b - W_{i+1} z_{i+1,j} - S_{j+1} z_{i,j+1}; the sweep then solves the
// triangular system with this right-hand side, which is one Gauss-Seidel
// sweep.  FP64 arithmetic (the terms largely cancel).  Loads as in
// level_apply.
template <typename T, bool TR>
BLP_DEV double gs_rhs_value(const MgLevelG<T> &L, const SkewT<T, TR> &sk, int i, int j, size_t q) {
  const GridG<T> &g = L.g;
  const int n = g.nx;
  const int id = TR ? i + 1 : i - 1, jd = TR ? j + 1 : j - 1;
  const bool hx = id >= 1 && id <= n, hy = jd >= 1 && jd <= g.ny;
  const double zx = L.z[sk.at(hx ? id : i, j)], zy = L.z[sk.at(i, hy ? jd : j)];
  const double cx = TR ? g.W[i + 1] : g.W[i], cy = TR ? g.S[j + 1] : g.S[j];
  // an absent neighbour enters with weight zero (v - 0 z = v exactly); a
  // select between v and v - c z would be compiled into a branch holding
  // the loads
  double v = L.b[q];
  v -= (hx ? cx : 0.0) * zx;
  v -= (hy ? cy : 0.0) * zy;
  return v;
}

// The level kernels below take one skewed slot per thread; a padding slot
// evaluates node (1, 1), whose reads are in range, and discards the value.
// The system's gate is read together with the data and tested before the
// stores.
template <typename T, bool TR>
__global__ void k_gs_rhs(const MgArgs<T> *A) {
  const MgArgs<T> a = A[blockIdx.y];
  const int gate = gptr(a.ctrl)->gate;
  const size_t q = (size_t)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (q >= a.L.nslot) return;
  const MgLevelG<T> L = lview(a.L);
  const SkewT<T, TR> sk = level_skew<T, TR>(L.g.nx);
  int i = 1, j = 1;
  const bool node = sk.decode_wave(q, i, j);
  if (!node) i = j = 1;
  const double v = gs_rhs_value<T, TR>(L, sk, i, j, q);
  BLP_ISSUED();
  if (gate) return;
  L.t[q] = node ? T(v) : T(0);
}

// t = b - A z (forward) or b - A^T z (transposed) on a level.
template <typename T, bool TR>
__global__ void k_mg_resid(const MgArgs<T> *A) {
  const MgArgs<T> a = A[blockIdx.y];
  const int gate = gptr(a.ctrl)->gate;
  const size_t q = (size_t)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (q >= a.L.nslot) return;
  const MgLevelG<T> L = lview(a.L);
  const SkewT<T, TR> sk = level_skew<T, TR>(L.g.nx);
  int i = 1, j = 1;
  const bool node = sk.decode_wave(q, i, j);
  if (!node) i = j = 1;
  const double r = (double)L.b[q] - level_apply<T, TR>(L.g, sk, L.z, i, j);
  BLP_ISSUED();
  if (gate || !node) return;
  L.t[q] = T(r);
}

// Coarse right-hand side: forward b_c = S_c^{-1} P^T S_f t_f (FE rescaling,
// Sec. 3.2), transposed b_c = P^T t_f.  Gathers the 3x3 fine neighbourhood
// 2k-1 .. 2k+1 by 2m-1 .. 2m+1; a fine node past the level's edge is read
// at 2k (2m), which always exists, and left out of the sum.
template <typename T, bool TR>
BLP_DEV T restrict_value(const MgLevelG<T> &F, const MgLevelG<T> &Cc, const SkewT<T, TR> &skf, int k,
                         int m) {
  const int nf = F.g.nx;
  T s = T(0);
#pragma unroll
  for (int dj = -1; dj <= 1; ++dj) {
    const int jj = 2 * m + dj;
    const bool iny = jj >= 1 && jj <= nf;
    const int jc = iny ? jj : 2 * m;
    const T wy = dj == 0 ? T(1) : (dj < 0 ? F.wry[jc] : F.wly[jc]);
#pragma unroll
    for (int di = -1; di <= 1; ++di) {
      const int ii = 2 * k + di;
      const bool inx = ii >= 1 && ii <= nf;
      const int ic = inx ? ii : 2 * k;
      const T wx = di == 0 ? T(1) : (di < 0 ? F.wrx[ic] : F.wlx[ic]);
      T v = F.t[skf.at(ic, jc)] * wx * wy;
      if (!TR) v *= F.hbx[ic] * F.hby[jc];
      s = (inx && iny) ? s + v : s;
    }
  }
  if (!TR) s /= Cc.hbx[k] * Cc.hby[m];
  return s;
}
template <typename T, bool TR>
__global__ void k_mg_restrict(const MgArgs<T> *A) {
  const MgArgs<T> a = A[blockIdx.y];
  const int gate = gptr(a.ctrl)->gate;
  const size_t q = (size_t)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (q >= a.Cc.nslot) return;
  const MgLevelG<T> F = lview(a.L), Cc = lview(a.Cc);
  const SkewT<T, TR> skc = level_skew<T, TR>(Cc.g.nx), skf = level_skew<T, TR>(F.g.nx);
  int k = 1, m = 1;
  const bool node = skc.decode_wave(q, k, m);
  if (!node) k = m = 1;
  const T v = restrict_value<T, TR>(F, Cc, skf, k, m);
  BLP_ISSUED();
  if (gate || !node) return;
  Cc.b[q] = v;
}

// Coarse-grid correction at fine node (i, j): forward z_f + P z_c;
// transposed z_f + S_f P S_c^{-1} z_c.  Per axis a fine node has one coarse
// neighbour (even index, weight 1, or the first node) or two (odd index,
// weights wl and wr); an absent second neighbour is read at coarse node 1
// and left out.
template <typename T, bool TR>
BLP_DEV T prolong_value(const MgLevelG<T> &F, const MgLevelG<T> &Cc, const SkewT<T, TR> &skc, int i,
                        int j, size_t q) {
  auto axis = [](int x, const BLP_GLOBAL T *wl, const BLP_GLOBAL T *wr, int &k0, T &w0, int &k1, T &w1) {
    const T l = wl[x], r = wr[x];
    const bool even = x % 2 == 0, two = !even && (x - 1) / 2 >= 1;
    k0 = even ? x / 2 : (two ? (x - 1) / 2 : (x + 1) / 2);
    w0 = even ? T(1) : (two ? l : r);
    k1 = two ? (x + 1) / 2 : 1;
    w1 = two ? r : T(0);
    return two;
  };
  int kx0, kx1, ky0, ky1;
  T wx0, wx1, wy0, wy1;
  const bool tx = axis(i, F.wlx, F.wrx, kx0, wx0, kx1, wx1);
  const bool ty = axis(j, F.wly, F.wry, ky0, wy0, ky1, wy1);
  T s = T(0);
  auto term = [&](int kx, T wxv, int ky, T wyv, bool on) {
    T v = Cc.z[skc.at(kx, ky)];
    if (TR) v /= Cc.hbx[kx] * Cc.hby[ky];
    s += (on ? wxv * wyv : T(0)) * v;  // weight zero: s unchanged
  };
  term(kx0, wx0, ky0, wy0, true);
  term(kx1, wx1, ky0, wy0, tx);
  term(kx0, wx0, ky1, wy1, ty);
  term(kx1, wx1, ky1, wy1, tx && ty);
  if (TR) s *= F.hbx[i] * F.hby[j];
  return F.z[q] + s;
}

// Coarse-grid correction and Gauss-Seidel right-hand side in one pass: the
// right-hand side of gs_rhs_value for the corrected iterate z + P z_c (as
// prolong_value, rounded to the storage type), which enters only through
// the two downstream neighbours.  The corrected iterate is not stored: the
// post-smoothing sweep that follows recomputes every node of z from this
// right-hand side alone.
template <typename T, bool TR>
BLP_DEV T prolong_gs_value(const MgLevelG<T> &F, const MgLevelG<T> &Cc, const SkewT<T, TR> &skf,
                           const SkewT<T, TR> &skc, int i, int j, size_t q) {
  const GridG<T> &g = F.g;
  const int n = g.nx;
  const int id = TR ? i + 1 : i - 1, jd = TR ? j + 1 : j - 1;
  const bool hx = id >= 1 && id <= n, hy = jd >= 1 && jd <= g.ny;
  const int ic = hx ? id : i, jc = hy ? jd : j;
  const double cx = TR ? g.W[i + 1] : g.W[i], cy = TR ? g.S[j + 1] : g.S[j];
  const double px = prolong_value<T, TR>(F, Cc, skc, ic, j, skf.at(ic, j));
  const double py = prolong_value<T, TR>(F, Cc, skc, i, jc, skf.at(i, jc));
  double v = F.b[q];
  v -= (hx ? cx : 0.0) * px;  // weight zero: v unchanged
  v -= (hy ? cy : 0.0) * py;
  return T(v);
}
template <typename T, bool TR>
__global__ void k_mg_prolong_gs(const MgArgs<T> *A) {
  const MgArgs<T> a = A[blockIdx.y];
  const int gate = gptr(a.ctrl)->gate;
  const size_t q = (size_t)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (q >= a.L.nslot) return;
  const MgLevelG<T> F = lview(a.L), Cc = lview(a.Cc);
  const SkewT<T, TR> skf = level_skew<T, TR>(F.g.nx), skc = level_skew<T, TR>(Cc.g.nx);
  int i = 1, j = 1;
  const bool node = skf.decode_wave(q, i, j);
  if (!node) i = j = 1;
  const T v = prolong_gs_value<T, TR>(F, Cc, skf, skc, i, j, q);
  BLP_ISSUED();
  if (gate) return;
  F.t[q] = node ? v : T(0);
}

// Coarsest level: four downstream Gauss-Seidel sweeps (transposed: the
// transposed sweep on A^T), by one thread per system, from z = 0 when
// zero_init (a coarse level) or from the current iterate (when the corner
// block itself is the coarsest level).
template <typename T, bool TR>
BLP_DEV void coarsest_body(const MgLevelG<T> &L, int zero_init) {
  const GridG<T> &g = L.g;
  const int n = g.nx;
  const SkewT<T, TR> sk = level_skew<T, TR>(n);
  if (zero_init)
    for (int j = 1; j <= g.ny; ++j)
      for (int i = 1; i <= n; ++i) L.z[sk.at(i, j)] = T(0);
  for (int sweep = 0; sweep < 4; ++sweep) {
    for (int jj = 0; jj < g.ny; ++jj)
      for (int ii = 0; ii < n; ++ii) {
        const int i = TR ? ii + 1 : n - ii, j = TR ? jj + 1 : g.ny - jj;
        const BLP_GLOBAL T *z = L.z;
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
template <typename T, bool TR>
__global__ void k_mg_coarsest(const MgArgs<T> *A, int zero_init) {
  const MgArgs<T> a = A[blockIdx.x];
  if (a.ctrl->gate) return;
  if (threadIdx.x == 0) coarsest_body<T, TR>(lview(a.L), zero_init);
}

// ---------------------------------------------------------------------------
// The V-cycle below a level with at most kLdsN<T> nodes per axis, in one
// workgroup per system with every level held in LDS in the natural layout
// (node (i, j) at word (j - 1) n + i - 1, plus a zero padding row j = 0 and
// j = n + 1 in the iterate, right-hand side, residual and inverse diagonal):
// the axis and transfer tables, the inverse diagonal and nodal r (when
// present) of every level form a constant image, laid out once per system in
// global memory (k_coarse_image) and copied into LDS at the start of each
// cycle.  The steps and their arithmetic are those of the level-by-level
// launches (pre-smoothing sweep, residual, restriction, the coarser cycle,
// prolongation, Gauss-Seidel right-hand side, post-smoothing sweep; four
// Gauss-Seidel sweeps on the coarsest level); node loops use the whole
// workgroup, sweeps one wave (the levels have at most 64 columns).  Only the
// finest fused level touches the work vectors in global memory: its
// right-hand side (and iterate, when not zero) is read at the start and its
// iterate written back at the end, in the skewed layout of the other kernels.
// ---------------------------------------------------------------------------
template <typename T>
constexpr int kLdsN = sizeof(T) == 4 ? 64 : 32;
constexpr int kCoarseMax = 8;
template <typename T>
struct CoarseArgs {
  int nlev;                  // levels held (the last is the coarsest)
  MgLevel<T> L[kCoarseMax];  // consecutive levels, finest first
  MgCtrl *ctrl;
  T *image;                  // constant image (k_coarse_image)
};

constexpr int kCoarseThreads = 512;

// Array sizes in words, rounded up to whole 16-byte chunks: tables (n + 2),
// padded node arrays (n + 2 rows), plain node arrays (nodal r).
template <typename T>
__host__ __device__ inline int lds_round(int w) {
  constexpr int P = 16 / (int)sizeof(T);
  return (w + P - 1) / P * P;
}
// constant words of one level: twelve tables, the row couplings in sweep
// order (2n + 8 entries), the inverse diagonal, nodal r
template <typename T>
__host__ __device__ inline int lds_const_words(int n, bool nodal) {
  return 12 * lds_round<T>(n + 2) + lds_round<T>(2 * n + 8) + lds_round<T>((n + 2) * n) +
         (nodal ? lds_round<T>(n * n) : 0);
}
// work words of one level: iterate, right-hand side, residual
template <typename T>
__host__ __device__ inline int lds_work_words(int n) {
  return 3 * lds_round<T>((n + 2) * n);
}
template <typename T>
__host__ __device__ inline int lds_image_words(int n0, int nl, bool nodal) {
  int w = 0;
  for (int l = 0; l < nl; ++l) w += lds_const_words<T>(n0 >> l, nodal);
  return w;
}

template <typename T>
struct LdsLevel {
  int n;
  T *z, *b, *t, *ic;  // node (1, 1); rows j = 0 and j = n + 1 are padding
  T *r;               // nodal r (no padding), or nullptr: constant rc
  T *W, *E, *S, *N, *Dx, *Dy, *hbx, *hby, *wlx, *wrx, *wly, *wry;
  T *Y;               // Y[t]: upstream coupling of the sweep's row t (0 for t >= n)
  T rc;
  BLP_DEV int at(int i, int j) const { return (j - 1) * n + (i - 1); }
  BLP_DEV T rr(int i, int j) const { return r ? r[at(i, j)] : rc; }
};

// Level l of the fused hierarchy (n0 >> l nodes per axis): constant part in
// cbase (the image layout), work part in wbase.
template <typename T>
BLP_DEV LdsLevel<T> lds_level(T *cbase, T *wbase, int n0, int l, bool nodal, T rc) {
  int co = 0, wo = 0;
  for (int k = 0; k < l; ++k) {
    co += lds_const_words<T>(n0 >> k, nodal);
    wo += lds_work_words<T>(n0 >> k);
  }
  const int n = n0 >> l, a1 = lds_round<T>(n + 2), ap = lds_round<T>((n + 2) * n);
  LdsLevel<T> v;
  v.n = n;
  v.rc = rc;
  T *p = cbase + co;
  T **tab[12] = {&v.W, &v.E, &v.S, &v.N, &v.Dx, &v.Dy, &v.hbx, &v.hby, &v.wlx, &v.wrx, &v.wly, &v.wry};
#pragma unroll
  for (int k = 0; k < 12; ++k) { *tab[k] = p; p += a1; }
  v.Y = p; p += lds_round<T>(2 * n + 8);
  v.ic = p + n; p += ap;
  v.r = nodal ? p : nullptr;
  T *q = wbase + wo;
  v.z = q + n;
  v.b = q + ap + n;
  v.t = q + 2 * ap + n;
  return v;
}

// Constant image of one system's fused levels (setup; one block per system).
// The buffer is zero on entry (padding rows stay zero).
template <typename T, bool TR>
__global__ void k_coarse_image(const CoarseArgs<T> *A) {
  const CoarseArgs<T> &a = A[blockIdx.x];
  const int n0 = a.L[0].g.nx;
  const bool nodal = a.L[0].g.r != nullptr;
  for (int l = 0; l < a.nlev; ++l) {
    const LdsLevel<T> V = lds_level<T>(a.image, nullptr, n0, l, nodal, T(0));
    const MgLevel<T> &G = a.L[l];
    const int n = V.n;
    const T *src[12] = {G.g.W, G.g.E, G.g.S, G.g.N, G.g.Dx, G.g.Dy, G.hbx, G.hby, G.wlx, G.wrx, G.wly, G.wry};
    T *dst[12] = {V.W, V.E, V.S, V.N, V.Dx, V.Dy, V.hbx, V.hby, V.wlx, V.wrx, V.wly, V.wry};
#pragma unroll
    for (int k = 0; k < 12; ++k)
      for (int x = threadIdx.x; x < n + 2; x += blockDim.x) dst[k][x] = src[k][x];
    // sweep row t at j = 1 + t (transposed, coupling N_{j-1}) or n - t (N_j)
    for (int x = threadIdx.x; x < 2 * n + 8; x += blockDim.x)
      V.Y[x] = x < n ? (TR ? G.g.N[x] : G.g.N[n - x]) : T(0);
    const SkewT<T, TR> sk = level_skew<T, TR>(n);
    for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
      const int i = idx % n + 1, j = idx / n + 1;
      V.ic[idx] = G.ic[sk.at(i, j)];
      if (nodal) V.r[idx] = G.g.r[(size_t)(j - 1) * G.g.rld + (i - 1)];
    }
  }
}

// (A z)_ij or (A^T z)_ij in FP64 arithmetic (as level_apply).
template <typename T, bool TR>
BLP_DEV double lds_apply(const LdsLevel<T> &L, int i, int j) {
  const int n = L.n;
  const T *z = L.z;
  const double zc = z[L.at(i, j)];
  const double zw = i > 1 ? (double)z[L.at(i - 1, j)] : 0.0;
  const double ze = i < n ? (double)z[L.at(i + 1, j)] : 0.0;
  const double zs = j > 1 ? (double)z[L.at(i, j - 1)] : 0.0;
  const double zn = j < n ? (double)z[L.at(i, j + 1)] : 0.0;
  const double C = (double)L.Dx[i] + (double)L.Dy[j] + (double)L.rr(i, j);
  if (!TR)
    return C * zc + (double)L.W[i] * zw + (double)L.E[i] * ze + (double)L.S[j] * zs +
           (double)L.N[j] * zn;
  return C * zc + (double)L.E[i - 1] * zw + (double)L.W[i + 1] * ze + (double)L.N[j - 1] * zs +
         (double)L.S[j + 1] * zn;
}

// Downstream sweep on an LDS level by one wave (lane = column, as the
// skewed sweep): z = solution of the triangular system with right-hand side
// rhs (the level's b or t).  Row t of a lane's column (t = 0 first) sits at
// word o0 + t dq; outside rows 0 .. n - 1 the word is clamped to the padding
// rows (t = -1 or n), where rhs and the inverse diagonal are zero: those
// steps compute z = 0, the upstream value of the first row, and store it
// into the iterate's padding.  The row coupling of lane l at step s (row
// s - l) is the one lane l - 1 held at step s - 1, passed on by a DPP shift;
// lane 0 takes row s's from the table.  Lane 0 has no upstream column.
template <typename T, bool TR>
BLP_DEV void lds_sweep(const LdsLevel<T> &L, const T *rhs, int lane) {
  constexpr int K = 8;
  const int n = L.n;
  const bool col = lane < n;
  const int c = col ? lane : 0;
  const int i = TR ? 1 + c : n - c;
  const T cu = col ? (TR ? L.E[i - 1] : L.E[i]) : T(0);
  // row t at j = 1 + t (transposed) or n - t
  const int o0 = TR ? i - 1 : (n - 1) * n + i - 1, dq = TR ? n : -n;
  const int oa = o0 - dq, ob = o0 + n * dq;  // rows -1 and n
  const int olo = min(oa, ob), ohi = max(oa, ob);
  const int lofs = col ? lane : 4 * n;  // lanes without a column stay in the padding
  typedef typename Vec16<T>::type V16;
  constexpr int P = 16 / (int)sizeof(T);
  static_assert(K % P == 0, "whole 16-byte table reads");
  T z = T(0), yc = T(0);
  for (int s0 = 0; s0 < 2 * n - 1; s0 += K) {
    const int os = o0 + (s0 - lofs) * dq;  // row of step s0 (unclamped)
    T bv[K], iv[K], y0[K];
    int o[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      o[k] = min(max(os + k * dq, olo), ohi);
      bv[k] = rhs[o[k]];
      iv[k] = L.ic[o[k]];
    }
    // lane 0's row couplings (rows s0 .. s0 + K - 1; wave-uniform address)
    const V16 *yv = reinterpret_cast<const V16 *>(L.Y + s0);
#pragma unroll
    for (int q = 0; q < K / P; ++q) {
      const V16 v = yv[q];
#pragma unroll
      for (int e = 0; e < P; ++e) y0[q * P + e] = v[e];
    }
    T res[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      yc = dpp_mov<0x138>(y0[k], yc);         // lane l-1's previous coupling; lane 0: table
      const T zin = dpp_mov<0x138>(T(0), z);  // lane l-1's value; lane 0: none
      z = (bv[k] - yc * z - cu * zin) * iv[k];
      res[k] = z;
    }
#pragma unroll
    for (int k = 0; k < K; ++k) L.z[o[k]] = res[k];
  }
}

// Four Gauss-Seidel sweeps on an NC x NC coarsest level (as coarsest_body),
// the iterate, right-hand side, inverse diagonal and couplings in registers.
template <typename T, bool TR, int NC>
BLP_DEV void lds_coarsest_regs(const LdsLevel<T> &V, bool zero) {
  T z[NC * NC], b[NC * NC], ic[NC * NC], W[NC + 2], E[NC + 2], S[NC + 2], N[NC + 2];
#pragma unroll
  for (int q = 0; q < NC * NC; ++q) {
    z[q] = zero ? T(0) : V.z[q];
    b[q] = V.b[q];
    ic[q] = V.ic[q];
  }
#pragma unroll
  for (int k = 0; k < NC + 2; ++k) {
    W[k] = V.W[k];
    E[k] = V.E[k];
    S[k] = V.S[k];
    N[k] = V.N[k];
  }
#pragma unroll
  for (int sw = 0; sw < 4; ++sw)
#pragma unroll
    for (int jj = 0; jj < NC; ++jj)
#pragma unroll
      for (int ii = 0; ii < NC; ++ii) {
        const int i = TR ? ii + 1 : NC - ii, j = TR ? jj + 1 : NC - jj;
        const int q = (j - 1) * NC + (i - 1);
        const T zw = i > 1 ? z[q - 1] : T(0);
        const T ze = i < NC ? z[q + 1] : T(0);
        const T zs = j > 1 ? z[q - NC] : T(0);
        const T zn = j < NC ? z[q + NC] : T(0);
        T off;
        if (!TR) off = W[i] * zw + E[i] * ze + S[j] * zs + N[j] * zn;
        else off = E[i - 1] * zw + W[i + 1] * ze + N[j - 1] * zs + S[j + 1] * zn;
        z[q] = (b[q] - off) * ic[q];
      }
#pragma unroll
  for (int q = 0; q < NC * NC; ++q) V.z[q] = z[q];
}

template <typename T>
BLP_DEV T lds_w1d(const T *wl, const T *wr, int i, int k) {
  if (i == 2 * k) return T(1);
  if (i == 2 * k - 1) return wr[i];
  return wl[i];  // i == 2k+1
}

template <typename T, bool TR>
__global__ __launch_bounds__(kCoarseThreads) void k_mg_coarse(const CoarseArgs<T> *A, int zero_init) {
  extern __shared__ __align__(16) unsigned char blp_lds[];
  typedef typename Vec16<T>::type V16;
  constexpr int P = 16 / (int)sizeof(T);
  T *cbase = reinterpret_cast<T *>(blp_lds);
  const CoarseArgs<T> &a = A[blockIdx.x];
  const int gate = a.ctrl->gate;  // tested after the loads below are issued
  const int nl = a.nlev, tid = threadIdx.x, nt = blockDim.x, lane = tid & 63;
  const int n0 = a.L[0].g.nx;
  const bool nodal = a.L[0].g.r != nullptr;
  const T rc = a.L[0].g.rc;
  const int cw = lds_image_words<T>(n0, nl, nodal);
  T *wbase = cbase + cw;
  auto lev = [&](int l) { return lds_level<T>(cbase, wbase, n0, l, nodal, rc); };

  // ---- zero padding rows of every level's right-hand side and residual
  for (int l = 0; l < nl; ++l) {
    const LdsLevel<T> Vl = lev(l);
    const int n = Vl.n;
    for (int x = tid; x < 4 * n; x += nt) {
      const int r2 = x / n, i = x - r2 * n;
      T *arr = (r2 & 1) ? Vl.t : Vl.b;
      arr[(r2 < 2 ? -n : n * n) + i] = T(0);
    }
  }
  // ---- constant image into LDS, and the finest level's right-hand side
  // (and iterate) from the skewed work vectors: per round eight 16-byte
  // image loads and eight node loads per thread are in flight together
  {
    const BLP_GLOBAL V16 *src = gptr(reinterpret_cast<const V16 *>(a.image));
    V16 *dst = reinterpret_cast<V16 *>(cbase);
    const int nv = cw / P;
    const LdsLevel<T> V0 = lev(0);
    const MgLevelG<T> G = lview(a.L[0]);
    const int n = V0.n, nn = n * n;
    const SkewT<T, TR> sk = level_skew<T, TR>(n);
    for (int r0 = tid; r0 < nv || r0 < nn; r0 += 8 * nt) {
      V16 tmp[8];
      T vb[8], vz[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        tmp[u] = src[min(r0 + u * nt, nv - 1)];
        const int idx = min(r0 + u * nt, nn - 1);
        const size_t q = sk.at(idx % n + 1, idx / n + 1);
        vb[u] = G.b[q];
        vz[u] = zero_init ? T(0) : G.z[q];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (r0 + u * nt < nv) dst[r0 + u * nt] = tmp[u];
        if (r0 + u * nt < nn) {
          V0.b[r0 + u * nt] = vb[u];
          V0.z[r0 + u * nt] = vz[u];
        }
      }
    }
  }
  if (gate) return;  // the system's cycle is switched off (same in every thread)
  __syncthreads();

  // block-wide loop over the nodes of level V: out[node] = f(i, j)
  // (lane = column i - 1, wave-strided rows: the levels have at most 64 columns)
  auto nodes = [&](const LdsLevel<T> &V, T *out, auto &&f) __attribute__((always_inline)) {
    const int n = V.n;
    if (lane < n)
      for (int j = (tid >> 6) + 1; j <= n; j += nt >> 6) out[(j - 1) * n + lane] = f(lane + 1, j);
    __syncthreads();
  };
  auto sweep = [&](const LdsLevel<T> &V, const T *rhs) __attribute__((always_inline)) {
    if (tid < 64) lds_sweep<T, TR>(V, rhs, lane);
    __syncthreads();
  };
  // Gauss-Seidel right-hand side: the downstream couplings folded in
  auto gs_rhs = [&](const LdsLevel<T> &V) __attribute__((always_inline)) {
    const int n = V.n;
    nodes(V, V.t, [&](int i, int j) {
      const int id = TR ? i + 1 : i - 1, jd = TR ? j + 1 : j - 1;
      double v = V.b[V.at(i, j)];
      if (id >= 1 && id <= n) v -= (double)(TR ? V.W[i + 1] : V.W[i]) * (double)V.z[V.at(id, j)];
      if (jd >= 1 && jd <= n) v -= (double)(TR ? V.S[j + 1] : V.S[j]) * (double)V.z[V.at(i, jd)];
      return T(v);
    });
  };

  for (int l = 0; l + 1 < nl; ++l) {
    const LdsLevel<T> F = lev(l), Cc = lev(l + 1);
    if (l == 0 && !zero_init) {
      gs_rhs(F);
      sweep(F, F.t);
    } else {
      sweep(F, F.b);
    }
    nodes(F, F.t, [&](int i, int j) { return T((double)F.b[F.at(i, j)] - lds_apply<T, TR>(F, i, j)); });
    // coarse right-hand side (as restrict_value)
    const int nf = F.n;
    nodes(Cc, Cc.b, [&](int k, int m) {
      T s2 = T(0);
      for (int jj = 2 * m - 1; jj <= 2 * m + 1; ++jj) {
        if (jj < 1 || jj > nf) continue;
        const T wy = lds_w1d(F.wly, F.wry, jj, m);
        for (int ii = 2 * k - 1; ii <= 2 * k + 1; ++ii) {
          if (ii < 1 || ii > nf) continue;
          T v = F.t[F.at(ii, jj)] * lds_w1d(F.wlx, F.wrx, ii, k) * wy;
          if (!TR) v *= F.hbx[ii] * F.hby[jj];
          s2 += v;
        }
      }
      if (!TR) s2 /= Cc.hbx[k] * Cc.hby[m];
      return s2;
    });
  }
  // coarsest level: four Gauss-Seidel sweeps by one thread (as coarsest_body);
  // in registers when it has at most 4 x 4 nodes
  if (tid == 0) {
    const LdsLevel<T> V = lev(nl - 1);
    const int n = V.n;
    const bool zc = nl > 1 || zero_init;
    if (n == 2) lds_coarsest_regs<T, TR, 2>(V, zc);
    else if (n == 3) lds_coarsest_regs<T, TR, 3>(V, zc);
    else if (n == 4) lds_coarsest_regs<T, TR, 4>(V, zc);
    else {
    if (zc)
      for (int idx = 0; idx < n * n; ++idx) V.z[idx] = T(0);
    for (int sw = 0; sw < 4; ++sw) {
      for (int jj = 0; jj < n; ++jj)
        for (int ii = 0; ii < n; ++ii) {
          const int i = TR ? ii + 1 : n - ii, j = TR ? jj + 1 : n - jj;
          const T *z = V.z;
          const T zw = i > 1 ? z[V.at(i - 1, j)] : T(0);
          const T ze = i < n ? z[V.at(i + 1, j)] : T(0);
          const T zs = j > 1 ? z[V.at(i, j - 1)] : T(0);
          const T zn = j < n ? z[V.at(i, j + 1)] : T(0);
          T off;
          if (!TR) off = V.W[i] * zw + V.E[i] * ze + V.S[j] * zs + V.N[j] * zn;
          else off = V.E[i - 1] * zw + V.W[i + 1] * ze + V.N[j - 1] * zs + V.S[j + 1] * zn;
          const int q = V.at(i, j);
          V.z[q] = (V.b[q] - off) * V.ic[q];
        }
    }
    }
  }
  __syncthreads();
  for (int l = nl - 2; l >= 0; --l) {
    const LdsLevel<T> F = lev(l), Cc = lev(l + 1);
    // coarse-grid correction (as prolong_value)
    nodes(F, F.z, [&](int i, int j) {
      // up to two coarse neighbours per axis: (k0, w0) and, if two, (k1, w1)
      auto axis = [](int x, const T *wl, const T *wr, int &k0, T &w0, int &k1, T &w1) {
        if (x % 2 == 0) { k0 = x / 2; w0 = T(1); return false; }
        if ((x - 1) / 2 >= 1) {
          k0 = (x - 1) / 2; w0 = wl[x];
          k1 = (x + 1) / 2; w1 = wr[x];
          return true;
        }
        k0 = (x + 1) / 2; w0 = wr[x];
        return false;
      };
      int kx0, kx1 = 1, ky0, ky1 = 1;
      T wx0, wx1 = T(0), wy0, wy1 = T(0);
      const bool tx = axis(i, F.wlx, F.wrx, kx0, wx0, kx1, wx1);
      const bool ty = axis(j, F.wly, F.wry, ky0, wy0, ky1, wy1);
      T s2 = T(0);
      auto term = [&](int kx, T wxv, int ky, T wyv) {
        T v = Cc.z[Cc.at(kx, ky)];
        if (TR) v /= Cc.hbx[kx] * Cc.hby[ky];
        s2 += wxv * wyv * v;
      };
      term(kx0, wx0, ky0, wy0);
      if (tx) term(kx1, wx1, ky0, wy0);
      if (ty) {
        term(kx0, wx0, ky1, wy1);
        if (tx) term(kx1, wx1, ky1, wy1);
      }
      if (TR) s2 *= F.hbx[i] * F.hby[j];
      return F.z[F.at(i, j)] + s2;
    });
    gs_rhs(F);
    sweep(F, F.t);
  }

  // ---- the finest fused level's iterate back to global memory (skewed)
  {
    const LdsLevel<T> V = lev(0);
    const MgLevelG<T> G = lview(a.L[0]);
    const int n = V.n;
    const SkewT<T, TR> sk = level_skew<T, TR>(n);
    for (int idx = tid; idx < n * n; idx += nt) {
      const int i = idx % n + 1, j = idx / n + 1;
      G.z[sk.at(i, j)] = V.z[idx];
    }
  }
}

// LDS bytes of the fused cycle from level n0 down (nl levels).
template <typename T>
inline size_t coarse_lds_bytes(int n0, int nl, bool nodal) {
  size_t w = lds_image_words<T>(n0, nl, nodal);
  for (int l = 0; l < nl; ++l) w += lds_work_words<T>(n0 >> l);
  return w * sizeof(T);
}

// Corner stopping rule (Sec. 3.2): norm of the residual of the system the
// cycle works on -- forward ||S (b - A z)||, transposed ||b - A^T z|| -- with
// mode 0 measuring ||S b|| (resp. ||b||) before the first cycle.  The last
// block of each system compares against rtol and sets its gate.
template <typename T, bool TR, int mode>
__global__ __launch_bounds__(256) void k_mg_norm(const MgArgs<T> *A) {
  __shared__ double sh[16];
  __shared__ bool last;
  const MgArgs<T> a = A[blockIdx.y];
  MgCtrl *ctrl = a.ctrl;
  const int gate = gptr(ctrl)->gate;  // uniform across the system's blocks
  const MgLevelG<T> L = lview(a.L);
  const SkewT<T, TR> sk = level_skew<T, TR>(L.g.nx);
  const size_t nslot = a.L.nslot;
  // grid-stride loop, NU slots per round with their loads issued together;
  // padding slots and slots past the end evaluate node (1, 1) and add
  // nothing, so each thread sums its slots in increasing q
  constexpr int NU = 4;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  double acc = 0.0;
  const int lb = xcd_block(blockIdx.x, gridDim.x);  // logical block (partials in its order)
  for (size_t q0 = (size_t)lb * blockDim.x + threadIdx.x; q0 < nslot; q0 += NU * stride) {
    double vs[NU];
    bool on[NU];
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      const size_t q = q0 + u * stride, qc = q < nslot ? q : nslot - 1;
      int i = 1, j = 1;
      const bool node = sk.decode_wave(qc, i, j);
      if (!node) i = j = 1;
      on[u] = node & (q < nslot);
      double v = (double)L.b[qc];
      if (mode == 1) v -= level_apply<T, TR>(L.g, sk, L.z, i, j);
      if (!TR) v *= (double)L.hbx[i] * (double)L.hby[j];
      vs[u] = v;
    }
#pragma unroll
    for (int u = 0; u < NU; ++u) acc = on[u] ? acc + vs[u] * vs[u] : acc;
  }
  BLP_ISSUED();
  if (gate) return;
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) publish(&a.partials[lb], acc);
  if (!arrive_last(&ctrl->counter, &last, gridDim.x)) return;
  // last block: fixed-order sum of the partials (deterministic)
  double s = 0.0;
  for (int b2 = threadIdx.x; b2 < (int)gridDim.x; b2 += blockDim.x) s += collect(&a.partials[b2]);
  s = block_sum(s, sh);
  if (threadIdx.x == 0) {
    reset_counter(&ctrl->counter);
    if (mode == 0) {
      ctrl->bnorm2 = s;
      if (s == 0.0) ctrl->gate = 1;  // zero right-hand side: z = 0, no cycle
    } else {
      ctrl->cycles += 1;
      ctrl->res2 = s;
      if (s <= ctrl->rtol2 * ctrl->bnorm2 || ctrl->cycles >= ctrl->maxcyc) ctrl->gate = 1;
    }
  }
}

// Count a fixed-mode cycle (no norm evaluation).  One thread per system.
template <typename T>
__global__ void k_mg_count(const MgArgs<T> *A) {
  MgCtrl *c = A[blockIdx.x].ctrl;
  if (threadIdx.x == 0 && !c->gate) c->cycles += 1;
}

// ---------------------------------------------------------------------------
// Corner block: right-hand side and copy-back (blockIdx.z = system).
// Forward: b_C = b_C - A_CX z_X - A_CY z_Y, the couplings sitting on the
// transition column (E_h to (h+1, j) in Y) and row (N_h to (i, h+1) in X).
// b_0 is written in the skewed layout of level 0.  The right-hand-side kernel
// also resets the corner control block; for a gated system it closes the
// corner gate, which switches the whole cycle off.
// ---------------------------------------------------------------------------
template <typename T>
struct CornerIO {
  Grid<T> g;
  int h, n1;
  const T *v;
  long long ldv;
  const T *dh;
  T *z;
  long long ldz;
  T *b0;        // level-0 right-hand side (skewed)
  const T *z0;  // level-0 result (skewed)
  MgCtrl *ctrl;
  int maxcyc;
  double rtol;
  const int *gate;
};
template <typename T, bool TR>
__global__ void k_corner_rhs(const CornerIO<T> *A, const int *jp) {
  const CornerIO<T> a = A[blockIdx.z];
  const int i = blockIdx.x * blockDim.x + threadIdx.x + 1;
  const int j = blockIdx.y + 1;
  const bool off = gated(a.gate);
  if (i == 1 && j == 1) {
    MgCtrl *c = a.ctrl;
    c->gate = off ? 1 : 0;
    c->cycles = 0;
    c->maxcyc = a.maxcyc;
    c->rtol2 = a.rtol * a.rtol;
    c->counter = 0;
  }
  if (off) return;
  const int h = a.h, n1 = a.n1;
  if (i > h) return;
  const size_t q = vidx(i, j, n1);
  const T *v = a.v + step_of(jp) * a.ldv;
  const T *z = a.z + step_of(jp) * a.ldz;
  T val = v[q];
  if (a.dh) val *= a.dh[q];
  if (!TR) {
    if (i == h) val -= a.g.E[h] * z[vidx(h + 1, j, n1)];
    if (j == h) val -= a.g.N[h] * z[vidx(i, h + 1, n1)];
  }
  a.b0[level_skew<T, TR>(h).at(i, j)] = val;
}

template <typename T, bool TR>
__global__ void k_corner_copy(const CornerIO<T> *A, const int *jp) {
  const CornerIO<T> a = A[blockIdx.z];
  if (gated(a.gate)) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x + 1;
  const int j = blockIdx.y + 1;
  const int h = a.h;
  if (i > h) return;
  (a.z + step_of(jp) * a.ldz)[vidx(i, j, a.n1)] = a.z0[level_skew<T, TR>(h).at(i, j)];
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
