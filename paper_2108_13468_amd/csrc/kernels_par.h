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
// 3 (dj+1) + (di+1) holds the coupling to (i+di, j+dj)).  The set-up builds
// them in FP64 in natural order (node (i, j) at word (j - 1) nx_l + (i - 1));
// the cycle keeps them, 1 / centre, the weights and the level vectors in the
// skewed order of the coarse sweep (ParSkew).
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
// the wavefront order's result).  A node's new value depends on its East
// neighbour and the three nodes of the row above, all visited before it; on
// a coarse level the sweep runs as a wavefront over lanes that own M
// columns each (k_par_wave, M = 2, 4 or 8), a node (column c, row t from the
// top) at step t + c / M, so a sweep is h + nx_l / M - 1 dependent steps.
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
// Skewed layout of a coarse level
// ---------------------------------------------------------------------------

// Coarse-level vectors and planes are stored in the order the wavefront
// sweep visits them.  Columns count from the right (c = nx - i, 0 .. nx-1),
// rows from the top (t = ny - j).  Lane l of the sweep owns the M columns
// l M .. l M + M - 1 (L = ceil(nx / M) lanes) and updates row t = p - l at
// step p, so skewed row p holds every lane's M words of its row p - l: node
// (c, t) is word (t + c / M) (L + 1) M + c.  Words c >= nx of a skewed row
// (among them lane index L, which lanes past the level read and write) and
// words whose row p - c / M is outside 0 .. ny - 1 are padding; padding holds
// zero in every plane and right-hand side, so the sweep computes zero there.
struct ParSkew {
  int nx = 0, ny = 0;  // columns and rows of the level
  int L = 0, M = 0;    // sweep lanes and columns per lane
  __host__ __device__ int rs() const { return (L + 1) * M; }  // words per skewed row
  __host__ __device__ int rows() const { return ny + L - 1; }
  __host__ __device__ size_t nslot() const { return (size_t)rows() * rs(); }
  // word of node (c, t), c in 0 .. nx - 1, t in 0 .. ny - 1
  BLP_DEV size_t slot(int c, int t) const { return (size_t)(t + c / M) * rs() + c; }
  // word of natural node (i, j)
  BLP_DEV size_t at(int i, int j) const { return slot(nx - i, ny - j); }
  // word q: its skewed row p and column c, and whether it holds a node (row t)
  BLP_DEV bool node(size_t q, int &c, int &t) const {
    const int p = (int)(q / (size_t)rs());
    c = (int)(q - (size_t)p * rs());
    t = p - c / M;
    return c < nx && t >= 0 && t < ny;
  }
};

// Sweep shape of a coarse level with nx columns, for words of wb bytes: two
// columns per lane up to 128 columns (one wave), four up to 256 (one wave);
// above, up to 512 columns, FP64 takes four (two waves) and FP32 eight (one
// wave: 32-byte chunks, fewer barriers, loads still few enough to run four
// steps ahead).  The launch (par_wave_launch) assumes these shapes.
inline ParSkew par_skew(int nx, int ny, int wb) {
  ParSkew s;
  s.nx = nx;
  s.ny = ny;
  s.M = nx <= 128 ? 2 : (nx <= 256 || wb == 8 ? 4 : 8);
  s.L = (nx + s.M - 1) / s.M;
  return s;
}
constexpr int kParMaxCols = 512;

// Natural-layout level arrays (np planes of nx ny words, FP64) into the
// skewed layout (np planes of nslot words, zero-filled beforehand) in TD.
template <typename TD>
__global__ void k_par_skew(const double *src, TD *dst, ParSkew sk, int np) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x + 1, j = blockIdx.y + 1;
  if (i > sk.nx) return;
  const size_t n = (size_t)sk.nx * sk.ny, ns = sk.nslot(), q = sk.at(i, j);
  for (int k = 0; k < np; ++k) dst[k * ns + q] = TD(src[k * n + vidx(i, j, sk.nx)]);
}

// The sweep's couplings to new values over the centre, skewed: plane k
// (0..3) holds a_q / a_C of plane q = 5 + k (East, North-West, North,
// North-East), formed in FP64 from the natural planes.
template <typename TD>
__global__ void k_par_skew_sweep(const double *a, TD *dst, ParSkew sk) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x + 1, j = blockIdx.y + 1;
  if (i > sk.nx) return;
  const size_t n = (size_t)sk.nx * sk.ny, ns = sk.nslot(), q = sk.at(i, j), v = vidx(i, j, sk.nx);
  const double c = a[4 * n + v];
  for (int k = 0; k < 4; ++k) dst[k * ns + q] = TD(a[(5 + k) * n + v] / c);
}

// ---------------------------------------------------------------------------
// The cycle (T = storage and sweep precision; residuals in FP64)
// ---------------------------------------------------------------------------

// One system's view of a level (blockIdx selects the record) and of the
// next coarser level for the transfers.  Level 0's z and b are the skewed
// vectors of the two-exponential-layer level 0 (level_skew(h)), its weights
// natural; coarse levels hold everything in their skewed layout.
template <typename T>
struct ParArgs {
  int nx, ny;
  ParSkew sk, skc;      // this level's layout (coarse levels) and the next coarser level's
  Grid<T> g;            // fine grid tables (level-0 couplings)
  const T *sx, *sy;     // level-0 rescaling factors hbar_i, kbar_j (1..h)
  const T *a;           // planes, plane q at word q sk.nslot() (coarse levels)
  const T *ic;          // 1 / centre coupling (coarse levels)
  const T *sw;          // the sweep's planes over the centre (k_par_skew_sweep)
  const T *wl, *wr;     // interpolation weights toward the next level
  T *z, *b, *t;         // iterate, right-hand side, residual
  int nxc;              // next coarser level: columns and vectors
  T *zc, *bc;
  MgCtrl *ctrl;
};

// Word q of a level's skewed vectors for a flat launch over the words (and
// the system in blockIdx.y); false past the end.
BLP_DEV bool par_word(size_t n, size_t &q) {
  q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  return q < n;
}

// Right-hand side of a sweep on a nonzero iterate, t = b - (couplings to
// the old values): West (c + 1, t), South-West (c + 1, t + 1), South (c, t + 1),
// South-East (c - 1, t + 1).  One thread per word; padding keeps zero.
template <typename T>
__global__ void k_par_pre(const ParArgs<T> *A) {
  const ParArgs<T> a = A[blockIdx.y];
  if (gptr(a.ctrl)->gate) return;
  const ParSkew sk = a.sk;
  size_t q;
  int c, t;
  if (!par_word(sk.nslot(), q) || !sk.node(q, c, t)) return;
  const BLP_GLOBAL T *z = gptr(a.z), *P = gptr(a.a);
  const size_t ns = sk.nslot();
  const bool w = c + 1 < sk.nx, e = c > 0, s = t + 1 < sk.ny;
  T r = gptr(a.b)[q];
  if (s && w) r -= P[q] * z[sk.slot(c + 1, t + 1)];
  if (s) r -= P[ns + q] * z[sk.slot(c, t + 1)];
  if (s && e) r -= P[2 * ns + q] * z[sk.slot(c - 1, t + 1)];
  if (w) r -= P[3 * ns + q] * z[sk.slot(c + 1, t)];
  gptr(a.t)[q] = r;
}

// Residual of a coarse level, t = b - A z, in FP64.  One thread per word.
template <typename T>
__global__ void k_par_resid(const ParArgs<T> *A) {
  const ParArgs<T> a = A[blockIdx.y];
  if (gptr(a.ctrl)->gate) return;
  const ParSkew sk = a.sk;
  size_t q;
  int c, t;
  if (!par_word(sk.nslot(), q) || !sk.node(q, c, t)) return;
  const BLP_GLOBAL T *z = gptr(a.z), *P = gptr(a.a);
  const size_t ns = sk.nslot();
  double s = 0.0;
#pragma unroll
  for (int dj = -1; dj <= 1; ++dj)
#pragma unroll
    for (int di = -1; di <= 1; ++di) {
      const int cc = c - di, tt = t - dj;  // natural (i + di, j + dj)
      if (cc < 0 || cc >= sk.nx || tt < 0 || tt >= sk.ny) continue;
      s += (double)P[(3 * (dj + 1) + (di + 1)) * ns + q] * (double)z[sk.slot(cc, tt)];
    }
  gptr(a.t)[q] = T((double)gptr(a.b)[q] - s);
}

// Level 0 to level 1 in one pass: the rescaled residual S (b - A_CC z) at
// the fine columns 2I-1, 2I, 2I+1 of row J (b and z skewed, FP64
// arithmetic, couplings out of the corner block left out), restricted by
// P^T in that order.  One thread per level-1 word.
template <typename T>
__global__ void k_par_rr0(const ParArgs<T> *A) {
  const ParArgs<T> a = A[blockIdx.y];
  if (gptr(a.ctrl)->gate) return;
  const ParSkew cs = a.skc;
  size_t q;
  int cc, tc;
  if (!par_word(cs.nslot(), q) || !cs.node(q, cc, tc)) return;
  const int I = cs.nx - cc, J = cs.ny - tc;
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
  gptr(a.bc)[q] = T(s);
}

// Coarse right-hand side bc = P^T t, one thread per coarse word, the fine
// columns 2I-1, 2I, 2I+1 added in that order.
template <typename T>
__global__ void k_par_restrict(const ParArgs<T> *A) {
  const ParArgs<T> a = A[blockIdx.y];
  if (gptr(a.ctrl)->gate) return;
  const ParSkew cs = a.skc, fs = a.sk;
  size_t q;
  int cc, tc;
  if (!par_word(cs.nslot(), q) || !cs.node(q, cc, tc)) return;
  const int I = cs.nx - cc, J = cs.ny - tc;
  const BLP_GLOBAL T *t = gptr(a.t), *wl = gptr(a.wl), *wr = gptr(a.wr);
  size_t f = fs.at(2 * I - 1, J);
  T s = wr[f] * t[f];
  f = fs.at(2 * I, J);
  s += t[f];
  if (2 * I + 1 <= fs.nx) {
    f = fs.at(2 * I + 1, J);
    s += wl[f] * t[f];
  }
  gptr(a.bc)[q] = s;
}

// Coarse-grid correction z += P zc, one thread per fine word.
template <typename T>
__global__ void k_par_prolong(const ParArgs<T> *A) {
  const ParArgs<T> a = A[blockIdx.y];
  if (gptr(a.ctrl)->gate) return;
  const ParSkew fs = a.sk, cs = a.skc;
  size_t q;
  int c, t;
  if (!par_word(fs.nslot(), q) || !fs.node(q, c, t)) return;
  const int i = fs.nx - c, j = fs.ny - t;
  const BLP_GLOBAL T *zc = gptr(a.zc);
  T s;
  if (i % 2 == 0) {
    s = zc[cs.at(i / 2, j)];
  } else {
    s = T(0);
    if (i > 1) s += gptr(a.wl)[q] * zc[cs.at((i - 1) / 2, j)];
    s += gptr(a.wr)[q] * zc[cs.at((i + 1) / 2, j)];
  }
  gptr(a.z)[q] += s;
}

// Coarse-grid correction of level 0 (skewed z of level_skew(h)) from level
// 1, z += P zc; one thread per level-0 node.
template <typename T>
__global__ void k_par_prolong0(const ParArgs<T> *A) {
  const ParArgs<T> a = A[blockIdx.z];
  if (gptr(a.ctrl)->gate) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x + 1, j = blockIdx.y + 1;
  const int h = a.nx;
  if (i > h) return;
  const ParSkew cs = a.skc;
  const BLP_GLOBAL T *zc = gptr(a.zc);
  const size_t q = vidx(i, j, h);
  T s;
  if (i % 2 == 0) {
    s = zc[cs.at(i / 2, j)];
  } else {
    s = T(0);
    if (i > 1) s += gptr(a.wl)[q] * zc[cs.at((i - 1) / 2, j)];
    s += gptr(a.wr)[q] * zc[cs.at((i + 1) / 2, j)];
  }
  gptr(a.z)[level_skew<T, false>(h).at(i, j)] += s;
}

// One downstream Gauss-Seidel sweep of a coarse level (rows top to bottom,
// each right to left) as a wavefront.  Lane l of the workgroup's W waves
// owns columns l M .. l M + M - 1 and updates row t = p - l at step p.  The
// new values a node needs are its East neighbour (same row) and the three
// nodes above it: for the lane's first column the East value is lane
// l - 1's last column of the previous step; for its last column the
// North-West value is lane l + 1's first column, computed earlier in the
// same step.  So a step forms the first M - 1 columns right to left, then
// the last one once the next lane's first column is in: DPP moves within a
// wave, an LDS word and a barrier across waves (two barriers per step).
// The old values (West, South-West, South, South-East) are folded into the
// right-hand side beforehand (k_par_pre; on a zero iterate the right-hand
// side is b), so per node the sweep reads the right-hand side, 1 / centre
// and the couplings East, North-West, North, North-East over the centre,
// and writes the node: z = r / a_C - sum (a_q / a_C) z_q, the terms in
// values that arrive last subtracted last, so that a step's dependent
// chain is two DPP moves and two fused multiply-adds.  Every lane loads and stores at every step (padding: zeros in,
// zeros out), D steps of operands ahead in rotated register buffers; every
// step's memory operations are the same, so the waits stay counted.
// Steps of operands in flight: a step issues six loads and a store of
// M sizeof(T) bytes per lane (16-byte pieces), and the wait counter tracks
// at most 63 memory operations.
template <typename T, int M>
constexpr int par_ahead() {
  return (M * sizeof(T) <= 16) ? 8 : 4;
}

template <typename T, int M>
struct ParStepOps {
  typedef T V __attribute__((ext_vector_type(M)));
  V r, e, nw, n, ne, ic;  // right-hand side, the four sweep planes, 1 / centre
};

// Raw buffer access to one array: a lane's constant byte offset (vo) plus a
// uniform byte offset (so, a scalar register), so that stepping through
// the skewed rows costs no vector instruction.  Accesses past the array's
// bytes read zero and write nothing.
typedef unsigned int ParU2 __attribute__((ext_vector_type(2)));
typedef unsigned int ParU4 __attribute__((ext_vector_type(4)));
BLP_DEV __amdgpu_buffer_rsrc_t par_rsrc(const void *p, size_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), 0, (int)bytes, 0x00020000);
}
template <typename V>
BLP_DEV V par_ld(__amdgpu_buffer_rsrc_t r, unsigned vo, int so) {
  static_assert(sizeof(V) == 8 || sizeof(V) % 16 == 0, "chunk of 8 or 16k bytes");
  V out;
  if constexpr (sizeof(V) == 8) {
    const ParU2 x = __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 0);
    __builtin_memcpy(&out, &x, 8);
  } else {
#pragma unroll
    for (int k = 0; k < (int)sizeof(V) / 16; ++k) {
      const ParU4 x = __builtin_amdgcn_raw_buffer_load_b128(r, vo + 16 * k, so, 0);
      __builtin_memcpy(reinterpret_cast<char *>(&out) + 16 * k, &x, 16);
    }
  }
  return out;
}
template <typename V>
BLP_DEV void par_st(const V &v, __amdgpu_buffer_rsrc_t r, unsigned vo, int so) {
  if constexpr (sizeof(V) == 8) {
    ParU2 x;
    __builtin_memcpy(&x, &v, 8);
    __builtin_amdgcn_raw_buffer_store_b64(x, r, vo, so, 0);
  } else {
#pragma unroll
    for (int k = 0; k < (int)sizeof(V) / 16; ++k) {
      ParU4 x;
      __builtin_memcpy(&x, reinterpret_cast<const char *>(&v) + 16 * k, 16);
      __builtin_amdgcn_raw_buffer_store_b128(x, r, vo + 16 * k, so, 0);
    }
  }
}

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

template <typename T, int W, int M, int D>
__global__ __launch_bounds__(64 * W) void k_par_wave(const ParArgs<T> *A, int zero_init) {
  static_assert(M >= 2, "the step order needs two or more columns per lane");
  typedef typename ParStepOps<T, M>::V V;
  __shared__ T s_e[W], s_nw[W];  // a wave's last lane's last column, first lane's first
  const ParArgs<T> a = A[blockIdx.x];
  if (gptr(a.ctrl)->gate) return;  // the same for every thread of the block
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const ParSkew sk = a.sk;
  const int L = sk.L, rv = L + 1, nrow = sk.rows();  // rv: chunks per skewed row
  // lanes past the level use the padding chunk; the lane's byte offset in
  // a skewed row is its own constant, the row offset is uniform
  const unsigned lob = (unsigned)(tid < L ? tid : L) * (unsigned)sizeof(V);
  const size_t pb = sk.nslot() * sizeof(T);  // bytes per plane or vector
  const __amdgpu_buffer_rsrc_t rR = par_rsrc(zero_init ? a.b : a.t, pb);
  const __amdgpu_buffer_rsrc_t rE = par_rsrc(a.sw, pb);
  const __amdgpu_buffer_rsrc_t rNW = par_rsrc(a.sw + sk.nslot(), pb);
  const __amdgpu_buffer_rsrc_t rN = par_rsrc(a.sw + 2 * sk.nslot(), pb);
  const __amdgpu_buffer_rsrc_t rNE = par_rsrc(a.sw + 3 * sk.nslot(), pb);
  const __amdgpu_buffer_rsrc_t rIC = par_rsrc(a.ic, pb);
  const __amdgpu_buffer_rsrc_t rZ = par_rsrc(a.z, pb);
  const int rb = rv * (int)sizeof(V);  // bytes per skewed row
  auto load = [&](int u, ParStepOps<T, M> &o) {  // step u's operands (past the end: the last row)
    const int so = (u < nrow ? u : nrow - 1) * rb;
    o.r = par_ld<V>(rR, lob, so);
    o.e = par_ld<V>(rE, lob, so);
    o.nw = par_ld<V>(rNW, lob, so);
    o.n = par_ld<V>(rN, lob, so);
    o.ne = par_ld<V>(rNE, lob, so);
    o.ic = par_ld<V>(rIC, lob, so);
  };
  if (W > 1) {
    if (tid < W) {
      s_e[tid] = T(0);
      s_nw[tid] = T(0);
    }
    __syncthreads();
  }
  T zp[M];       // this lane's columns at the previous step (the row above)
  T e0p = T(0);  // the previous step's East value of column 0 (its North-East now)
#pragma unroll
  for (int k = 0; k < M; ++k) zp[k] = T(0);
  auto step = [&](int p, const ParStepOps<T, M> &cur, ParStepOps<T, M> &nxt) {
    load(p + D, nxt);
    // issued here, D steps ahead of their use: the instruction scheduler
    // may not sink them toward later steps
    __builtin_amdgcn_sched_barrier(0);
    // terms in values of earlier steps (couplings already over the centre)
    T rest[M];
#pragma unroll
    for (int k = 0; k < M; ++k)
      rest[k] = cur.r[k] * cur.ic[k] - cur.n[k] * zp[k] - cur.ne[k] * (k ? zp[k - 1] : e0p);
    // East value of column 0: lane l - 1's last column (previous step); the
    // first lane of a wave takes it from the wave before (zero for wave 0)
    T e0;
    if constexpr (W > 1) e0 = dpp_mov<0x138>(w > 0 ? s_e[w > 0 ? w - 1 : 0] : T(0), zp[M - 1]);
    else e0 = par_shift<0x138>(zp[M - 1]);
    T z[M];
    z[0] = (rest[0] - cur.nw[0] * zp[1]) - cur.e[0] * e0;
#pragma unroll
    for (int k = 1; k + 1 < M; ++k) z[k] = (rest[k] - cur.nw[k] * zp[k + 1]) - cur.e[k] * z[k - 1];
    // North-West value of the last column: lane l + 1's first column (this
    // step); the last lane of a wave takes it from the wave after
    T nwv;
    if constexpr (W > 1) {
      if (lane == 0) s_nw[w] = z[0];
      lds_barrier();
      nwv = dpp_mov<0x130>(w + 1 < W ? s_nw[w + 1 < W ? w + 1 : w] : T(0), z[0]);
    } else {
      nwv = par_shift<0x130>(z[0]);
    }
    if constexpr (M == 2) {  // the North-West value arrives last
      z[1] = (rest[1] - cur.e[1] * z[0]) - cur.nw[1] * nwv;
    } else {  // column M - 2 arrives last
      z[M - 1] = (rest[M - 1] - cur.nw[M - 1] * nwv) - cur.e[M - 1] * z[M - 2];
    }
    if constexpr (W > 1) {
      if (lane == 63) s_e[w] = z[M - 1];
      lds_barrier();
    }
    V zv;
#pragma unroll
    for (int k = 0; k < M; ++k) {
      zv[k] = z[k];
      zp[k] = z[k];
    }
    par_st<V>(zv, rZ, lob, p * rb);
    e0p = e0;
  };
  // the buffers in turn (indices fixed at compile time: no register copies
  // between steps); whole groups of D + 1 steps, then the rest
  ParStepOps<T, M> buf[D + 1];
#pragma unroll
  for (int u = 0; u < D; ++u) load(u, buf[u]);
  int p = 0;
  for (; p + D < nrow; p += D + 1) {
#pragma unroll
    for (int u = 0; u <= D; ++u) step(p + u, buf[u], buf[(u + D) % (D + 1)]);
  }
#pragma unroll
  for (int u = 0; u < D; ++u)
    if (p + u < nrow) step(p + u, buf[u], buf[(u + D) % (D + 1)]);
}
