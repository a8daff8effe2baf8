// Host side of the MI355X boundary-layer-preconditioned FGMRES solver: the C
// ABI of include/blp.h, setup of the mesh tables and the preconditioner, and
// the orchestration of the HIP kernels on the problem's stream.
//
// Method: arXiv 2108.13468 (MacLachlan, Madden, Nhan).  The host computes only
// O(N) per-axis quantities (mesh widths and stencil tables, in FP64); every
// O(N^2) step runs in the kernels of kernels_*.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <string>
#include <tuple>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <type_traits>
#include <vector>

#include "../../include/blp.h"
#include "common.h"
#include "kernels_krylov.h"
#include "kernels_op.h"
#include "kernels_prec.h"
#include "kernels_1d.h"
#include "kernels_par.h"

namespace {

#define HIP_TRY(x)                        \
  do {                                    \
    if ((x) != hipSuccess) return BLP_E_HIP; \
  } while (0)
#define BLP_TRY(x)            \
  do {                        \
    int rc_ = (x);            \
    if (rc_ < 0) return rc_;  \
  } while (0)

// Per-axis stencil tables (index 0 and n+1 are zero padding).
struct AxisTab {
  std::vector<double> W, E, D;
};

// widths w[1..n+1], coefficient c[1..n] at the nodes -> tables (Sec. 3 stencil)
AxisTab axis_tables(int n, double eps, const std::vector<double> &w, const std::vector<double> &c) {
  AxisTab t;
  t.W.assign(n + 2, 0.0);
  t.E.assign(n + 2, 0.0);
  t.D.assign(n + 2, 0.0);
  for (int i = 1; i <= n; ++i) {
    const double hl = w[i], hr = w[i + 1], hb = 0.5 * (hl + hr);
    t.W[i] = -eps / (hb * hl);
    t.E[i] = -eps / (hb * hr) - c[i] / hr;
    t.D[i] = eps / hb * (1.0 / hl + 1.0 / hr) + c[i] / hr;
  }
  return t;
}

struct LevelHost {
  int n;
  std::vector<double> wx, wy;  // widths 1..n+1
  std::vector<double> cx, cy;  // c1, c2 at nodes 1..n
  AxisTab tx, ty;
};

template <typename T>
struct LevelDev {
  int n;
  size_t nslot;  // skewed storage of the level grid
  T *W, *E, *Dx, *S, *N, *Dy, *r, rc;
  T *ic[2];      // skewed 1/C for the forward (0) and transposed (1) cycle
  T *hbx, *hby, *wlx, *wrx, *wly, *wry;
  Grid<T> grid() const { return Grid<T>{n, n, W, E, Dx, S, N, Dy, r, n, rc}; }
  // the level with one system's work vectors (skewed z, b, t)
  MgLevel<T> view(bool tr, T *z, T *b, T *t) const {
    return MgLevel<T>{grid(), ic[tr ? 1 : 0], hbx, hby, wlx, wrx, wly, wry, z, b, t, nslot};
  }
};

// A level of the parabolic-case corner hierarchy: nx columns, h rows.
// Natural-order arrays are the FP64 set-up's (a, ic; wl and wr also level
// 0's in the cycle); the coarse levels' cycle arrays are skewed (sk).
template <typename T>
struct ParLevelDev {
  int nx = 0;
  ParSkew sk;                      // coarse levels: layout of the cycle arrays
  T *a = nullptr;                  // nine coupling planes, natural (FP64, coarse levels)
  T *ic = nullptr;                 // 1 / centre coupling, natural (FP64, coarse levels)
  T *wl = nullptr, *wr = nullptr;  // weights toward the next level, natural (FP64; FP32 on level 0)
  T *sa = nullptr, *sic = nullptr; // skewed planes and 1 / centre (coarse levels)
  T *swl = nullptr, *swr = nullptr;  // skewed weights (coarse levels with a coarser one)
  T *ssw = nullptr;                // skewed sweep planes (couplings over the centre)
  T *sx = nullptr, *sy = nullptr;  // level 0: rescaling factors hbar_i, kbar_j (0..h+1)
};

template <typename T>
struct FineDev {
  T *W, *E, *Dx, *S, *N, *Dy, *r, rc;
  T *dh;          // sqrt(C), natural layout (scaled-system input)
  T *fac[4][3];   // line factors [Y fwd, X fwd, Y tr, X tr] x [d, m, w]
  T *icI[2];      // skewed 1/C of the interior region, per direction
  size_t nslotI;  // skewed size of the interior region
};

struct Batch;

// Kernel timing: an event pair around each timed launch (recorded on the
// launch's stream), resolved into per-class sums on demand.
struct Timer {
  bool on = false;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  struct Rec { int cls; hipEvent_t a, b; double bytes; };
  std::vector<Rec> recs;
  hipEvent_t next() {
    if (used == pool.size()) {
      hipEvent_t e;
      // timestamps only: no system-scope fence (the streams are synchronised
      // before the times are read), so recording does not flush caches
      if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
      pool.push_back(e);
    }
    return pool[used++];
  }
  void start() {
    recs.clear();
    used = 0;
    on = true;
  }
  // per-class sums (ms, launches, bytes); the streams must be synchronised
  int stop(double *ms, long long *launches, double *bytes, int ncls) {
    on = false;
    std::vector<double> sm(ncls, 0.0), sb(ncls, 0.0);
    std::vector<long long> sl(ncls, 0);
    for (const auto &r : recs) {
      float t = 0.f;
      if (hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) return BLP_E_HIP;
      sm[r.cls] += t;
      sb[r.cls] += r.bytes;
      sl[r.cls] += 1;
    }
    for (int k = 0; k < ncls; ++k) {
      if (ms) ms[k] = sm[k];
      if (launches) launches[k] = sl[k];
      if (bytes) bytes[k] = sb[k];
    }
    recs.clear();
    used = 0;
    return BLP_OK;
  }
  ~Timer() {
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  }
};

}  // namespace

// A batch runs one part per mesh size.  Each part is a lockstep batch of
// that size's systems with its own FGMRES loop, stream and host thread, so
// that a part whose systems need many iterations is never held back by the
// steps of another.
struct blp_batch {
  std::vector<std::unique_ptr<Batch>> parts;
  std::vector<std::vector<int>> index;  // part -> the caller's system indices
};

struct blp_problem {
  int N, n1, h;
  size_t n;
  double eps;
  hipStream_t stream;
  std::vector<double> xn, yn, wx, wy, c1, c2;  // nodes, widths (1..N), coefficients (0..N)
  int device = -1;                  // current device at assemble
  double *xd = nullptr, *yd = nullptr;  // nodes on the device (N + 1 each)
  AxisTab fx, fy;
  bool r_nodal = false;
  double rc = 0.0;
  FineDev<double> f64{};
  FineDev<float> f32{};
  bool prec_ready = false;
  blp_prec_opts popts{0, 1e-3, 20};
  std::vector<LevelDev<double>> l64;
  std::vector<LevelDev<float>> l32;
  // layer at y = 0: BLP_LAYER_EXPONENTIAL (corner levels l64/l32 above) or
  // BLP_LAYER_PARABOLIC (x-semicoarsening levels pl64/pl32)
  int ylayer = BLP_LAYER_EXPONENTIAL;
  std::vector<ParLevelDev<double>> pl64;
  std::vector<ParLevelDev<float>> pl32;
  // solves run as a batch of systems over this problem (rebuilt when the
  // number of right-hand sides changes); FP32 staging of the test hook
  Batch *own = nullptr;
  int own_S = 0;
  float *tmp32a = nullptr, *tmp32b = nullptr;
  std::vector<void *> allocs;
  long long bytes = 0;
  Timer timer;  // kernel timing (blp_timing)

  template <typename T>
  int alloc(T **p, size_t count) {
    void *q = nullptr;
    if (hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess) return BLP_E_NOMEM;
    allocs.push_back(q);
    bytes += (long long)(count * sizeof(T));
    *p = (T *)q;
    return BLP_OK;
  }
  template <typename T>
  int upload(T **p, const std::vector<double> &h) {
    BLP_TRY(alloc(p, h.size()));
    std::vector<T> tmp(h.begin(), h.end());
    HIP_TRY(hipMemcpyAsync(*p, tmp.data(), tmp.size() * sizeof(T), hipMemcpyHostToDevice, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    return BLP_OK;
  }
  Grid<double> grid64() const {
    return Grid<double>{n1, n1, f64.W, f64.E, f64.Dx, f64.S, f64.N, f64.Dy, f64.r, n1, f64.rc};
  }
  Grid<float> grid32() const {
    return Grid<float>{n1, n1, f32.W, f32.E, f32.Dx, f32.S, f32.N, f32.Dy, f32.r, n1, f32.rc};
  }
};

namespace {

// Launch context: stream and the (optional) kernel timer.
struct Ctx {
  hipStream_t stream;
  Timer *timer;
};

// Records an event pair around the launches issued on the context's stream
// during its lifetime when timing is enabled.
struct KScope {
  Timer *t;
  hipStream_t s;
  int cls;
  double bytes;
  hipEvent_t a = nullptr;
  KScope(const Ctx &c, int k, double b) : t(c.timer), s(c.stream), cls(k), bytes(b) {
    if (t && t->on && (a = t->next())) (void)hipEventRecord(a, s);
  }
  void end() {
    if (!a) return;
    hipEvent_t b = t->next();
    if (b) {
      (void)hipEventRecord(b, s);
      t->recs.push_back({cls, a, b, bytes});
    }
    a = nullptr;
  }
  ~KScope() { end(); }
};
// Timing classes: one kernel (template) each where it matters for roofline
// accounting, so that a class average is a kernel average.
enum { KC_SWEEP = 0, KC_GSRHS, KC_LINES, KC_MG, KC_SPMV, KC_KRYLOV, KC_LAYOUT };

template <typename T>
FineDev<T> &fine(blp_problem *p);
template <>
FineDev<double> &fine<double>(blp_problem *p) { return p->f64; }
template <>
FineDev<float> &fine<float>(blp_problem *p) { return p->f32; }
template <typename T>
std::vector<LevelDev<T>> &levels(blp_problem *p);
template <>
std::vector<LevelDev<double>> &levels<double>(blp_problem *p) { return p->l64; }
template <>
std::vector<LevelDev<float>> &levels<float>(blp_problem *p) { return p->l32; }
template <typename T>
std::vector<ParLevelDev<T>> &par_levels(blp_problem *p);
template <>
std::vector<ParLevelDev<double>> &par_levels<double>(blp_problem *p) { return p->pl64; }
template <>
std::vector<ParLevelDev<float>> &par_levels<float>(blp_problem *p) { return p->pl32; }
template <typename T>
Grid<T> fine_grid(blp_problem *p);
template <>
Grid<double> fine_grid<double>(blp_problem *p) { return p->grid64(); }
template <>
Grid<float> fine_grid<float>(blp_problem *p) { return p->grid32(); }

// Row stride of the line-major edge-region buffers: h rounded up to a
// multiple of 4, so that every thread's nodes are 16-byte aligned.
inline int line_stride(int h) { return (h + 3) / 4 * 4; }

inline dim3 grid2d(int nx, int ny, int bx = 256) { return dim3((nx + bx - 1) / bx, ny); }
inline unsigned blocks1d(size_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

bool finite_all(const double *v, size_t n) {
  for (size_t k = 0; k < n; ++k)
    if (!std::isfinite(v[k])) return false;
  return true;
}

// One axis of a layer-adapted mesh: nl cells on the layer [0, tau], N - nl
// equal cells on [tau, 1] (Sec. 2.2's general Shishkin construction, q =
// nl / N; Sec. 3 admits any fitted tensor mesh with a transition point).
// BLP_MESH_SHISHKIN: tau = min(q, sigma eps ln N / clow), equal layer cells.
// BLP_MESH_BAKHVALOV_SHISHKIN: tau = sigma eps ln N / clow, and the layer
// nodes make exp(-clow x / (sigma eps)) fall in equal steps from 1 to 1/N:
// x_i = -(sigma eps / clow) ln(1 - (1 - 1/N) i / nl); uniform mesh when that
// tau reaches q.  Widths are taken from the closed forms (never as
// differences of coordinates): w[k] = x_k - x_{k-1}, w[0] = w[N+1] = 0.
// A parabolic layer (eq. tau parabolic) takes the width scale sqrt(eps)
// where an exponential one takes eps / clow.  Returns tau.
double axis_mesh(int N, double eps, double sigma, double clow, int kind, int nl,
                 std::vector<double> &nodes, std::vector<double> &w, bool parabolic = false) {
  nodes.assign(N + 1, 0.0);
  w.assign(N + 2, 0.0);
  const double q = (double)nl / N;
  const double layer = parabolic ? sigma * std::sqrt(eps) * std::log((double)N)
                                 : sigma * eps * std::log((double)N) / clow;
  const double tau = std::min(q, layer);
  const bool graded = kind == BLP_MESH_BAKHVALOV_SHISHKIN && layer < q;
  const double hl = tau / nl, hi = (1.0 - tau) / (N - nl);
  const double s = parabolic ? sigma * std::sqrt(eps) : sigma * eps / clow,
               a = (1.0 - 1.0 / N) / nl;
  for (int k = 1; k <= nl; ++k) {
    w[k] = graded ? s * std::log1p(a / (1.0 - a * k)) : hl;
    nodes[k] = k == nl ? tau : (graded ? -s * std::log1p(-a * k) : k * hl);
  }
  for (int k = nl + 1; k <= N; ++k) {
    w[k] = hi;
    nodes[k] = tau + (k - nl) * hi;
  }
  return tau;
}

// Mesh options with defaults filled in (NULL: the paper's Shishkin mesh,
// sigma = 2, clow = 1, N/2 layer cells); BLP_E_INVAL when outside the
// constructions above.
int mesh_options(int N, const blp_mesh_opts *o, blp_mesh_opts *out) {
  blp_mesh_opts m{2.0, 1.0, 1.0, BLP_MESH_SHISHKIN, 0, BLP_LAYER_EXPONENTIAL};
  if (o) m = *o;
  if (m.layer_cells == 0) m.layer_cells = N / 2;
  if (!(m.sigma > 0) || !(m.clow_x > 0) || !(m.clow_y > 0)) return BLP_E_INVAL;
  if (m.kind != BLP_MESH_SHISHKIN && m.kind != BLP_MESH_BAKHVALOV_SHISHKIN) return BLP_E_INVAL;
  if (m.y_layer != BLP_LAYER_EXPONENTIAL && m.y_layer != BLP_LAYER_PARABOLIC) return BLP_E_INVAL;
  if (m.layer_cells < 2 || m.layer_cells > N - 2) return BLP_E_INVAL;
  *out = m;
  return BLP_OK;
}

// ------------------------------------------------------------------------ //
// Setup                                                                     //
// ------------------------------------------------------------------------ //

template <typename T>
int zalloc(blp_problem *p, T **q, size_t count) {
  BLP_TRY(p->alloc(q, count));
  HIP_TRY(hipMemsetAsync(*q, 0, count * sizeof(T), p->stream));
  return BLP_OK;
}

template <typename T>
int upload_level(blp_problem *p, const LevelHost &lh, LevelDev<T> &d, const LevelDev<T> *finer,
                 const T *rfine_nodal, int rfine_ld) {
  d.n = lh.n;
  const int n = lh.n;
  d.nslot = skew_size<T>(n, n);
  BLP_TRY(p->upload(&d.W, lh.tx.W));
  BLP_TRY(p->upload(&d.E, lh.tx.E));
  BLP_TRY(p->upload(&d.Dx, lh.tx.D));
  BLP_TRY(p->upload(&d.S, lh.ty.W));
  BLP_TRY(p->upload(&d.N, lh.ty.E));
  BLP_TRY(p->upload(&d.Dy, lh.ty.D));
  std::vector<double> hbx(n + 2, 0.0), hby(n + 2, 0.0), wlx(n + 2, 0.0), wrx(n + 2, 0.0),
      wly(n + 2, 0.0), wry(n + 2, 0.0);
  for (int k = 1; k <= n; ++k) {
    hbx[k] = 0.5 * (lh.wx[k] + lh.wx[k + 1]);
    hby[k] = 0.5 * (lh.wy[k] + lh.wy[k + 1]);
    wlx[k] = lh.wx[k + 1] / (lh.wx[k] + lh.wx[k + 1]);
    wrx[k] = lh.wx[k] / (lh.wx[k] + lh.wx[k + 1]);
    wly[k] = lh.wy[k + 1] / (lh.wy[k] + lh.wy[k + 1]);
    wry[k] = lh.wy[k] / (lh.wy[k] + lh.wy[k + 1]);
  }
  BLP_TRY(p->upload(&d.hbx, hbx));
  BLP_TRY(p->upload(&d.hby, hby));
  BLP_TRY(p->upload(&d.wlx, wlx));
  BLP_TRY(p->upload(&d.wrx, wrx));
  BLP_TRY(p->upload(&d.wly, wly));
  BLP_TRY(p->upload(&d.wry, wry));
  d.rc = (T)p->rc;
  d.r = nullptr;
  if (p->r_nodal) {
    BLP_TRY(p->alloc(&d.r, (size_t)n * n));
    if (finer)
      k_sample<T><<<grid2d(n, n), 256, 0, p->stream>>>(finer->r, finer->n, 2, d.r, n);
    else
      k_sample<T><<<grid2d(n, n), 256, 0, p->stream>>>(rfine_nodal, rfine_ld, 1, d.r, n);
  }
  // skewed inverse diagonals: zero in the padding slots
  BLP_TRY(zalloc(p, &d.ic[0], d.nslot));
  BLP_TRY(zalloc(p, &d.ic[1], d.nslot));
  HIP_TRY(hipGetLastError());
  return BLP_OK;
}

template <typename T>
int build_fine_prec(blp_problem *p, FineDev<T> &f) {
  const int h = p->h, n1 = p->n1;
  BLP_TRY(p->alloc(&f.dh, p->n));
  k_diag_tables<T><<<grid2d(n1, n1), 256, 0, p->stream>>>(p->grid64(), (T *)nullptr, f.dh);
  const int m = n1 - h;
  f.nslotI = skew_size<T>(m, m);
  BLP_TRY(zalloc(p, &f.icI[0], f.nslotI));
  BLP_TRY(zalloc(p, &f.icI[1], f.nslotI));
  const SkewT<T, false> skf{h + 1, n1, h + 1, n1};
  const SkewT<T, true> skt{h + 1, n1, h + 1, n1};
  k_diag_skew<T, false><<<blocks1d(f.nslotI), 256, 0, p->stream>>>(p->grid64(), skf, f.icI[0], f.nslotI);
  k_diag_skew<T, true><<<blocks1d(f.nslotI), 256, 0, p->stream>>>(p->grid64(), skt, f.icI[1], f.nslotI);
  HIP_TRY(hipGetLastError());
  return BLP_OK;
}

template <typename T>
void level_diag(blp_problem *p, const LevelDev<double> &l64, LevelDev<T> &d) {
  const SkewT<T, false> sf{1, d.n, 1, d.n};
  const SkewT<T, true> st{1, d.n, 1, d.n};
  k_diag_skew<T, false><<<blocks1d(d.nslot), 256, 0, p->stream>>>(l64.grid(), sf, d.ic[0], d.nslot);
  k_diag_skew<T, true><<<blocks1d(d.nslot), 256, 0, p->stream>>>(l64.grid(), st, d.ic[1], d.nslot);
}

int build_exp_levels(blp_problem *p, bool level0_only);
int build_par_levels(blp_problem *p);

int build_preconditioner(blp_problem *p) {
  const int h = p->h, n1 = p->n1;
  BLP_TRY(build_fine_prec(p, p->f64));
  BLP_TRY(build_fine_prec(p, p->f32));
  // ---- Thomas factors of the edge-layer lines (computed in FP64) ----------
  // (zero-filled: the padding nodes of a line keep zero factors)
  const int hp = line_stride(h);
  const size_t fl = (size_t)(n1 - h) * hp;
  for (int v = 0; v < 4; ++v) {
    for (int k = 0; k < 3; ++k) {
      BLP_TRY(zalloc(p, &p->f64.fac[v][k], fl));
      BLP_TRY(zalloc(p, &p->f32.fac[v][k], fl));
    }
    const int region = v % 2, tr = v / 2;
    k_line_factor<double><<<blocks1d(n1 - h, 64), 64, 0, p->stream>>>(
        p->grid64(), h, n1, hp, region, tr, p->f64.fac[v][0], p->f64.fac[v][1], p->f64.fac[v][2]);
    for (int k = 0; k < 3; ++k)
      k_convert<double, float><<<blocks1d(fl), 256, 0, p->stream>>>(p->f64.fac[v][k],
                                                                    p->f32.fac[v][k], fl);
  }
  // ---- corner multigrid hierarchy (Sec. 3.2) ------------------------------
  // (the parabolic hierarchy's level 0 is the same corner block, kept in the
  // two-exponential-layer layout so that its sweeps are those kernels)
  BLP_TRY(build_exp_levels(p, p->ylayer == BLP_LAYER_PARABOLIC));
  if (p->ylayer == BLP_LAYER_PARABOLIC) BLP_TRY(build_par_levels(p));
  BLP_TRY(p->alloc(&p->tmp32a, p->n));
  BLP_TRY(p->alloc(&p->tmp32b, p->n));
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(p->stream));
  return BLP_OK;
}

// Two exponential layers: full coarsening, rediscretised levels (level 0
// alone: the corner block of either hierarchy).
int build_exp_levels(blp_problem *p, bool level0_only) {
  const int h = p->h, n1 = p->n1;
  std::vector<LevelHost> LH;
  {
    LevelHost l0;
    l0.n = h;
    l0.wx.assign(h + 2, 0.0);
    l0.wy.assign(h + 2, 0.0);
    l0.cx.assign(h + 1, 0.0);
    l0.cy.assign(h + 1, 0.0);
    for (int k = 1; k <= h + 1; ++k) {
      l0.wx[k] = p->wx[k];
      l0.wy[k] = p->wy[k];
    }
    for (int k = 1; k <= h; ++k) {
      l0.cx[k] = p->c1[k];
      l0.cy[k] = p->c2[k];
    }
    LH.push_back(l0);
    // coarsen by two while the level has an even node count above 2; the
    // coarse node k is fine node 2k, so the transition node stays a node and
    // the width beyond it (to the first interior-mesh node) is unchanged.
    while (!level0_only && LH.back().n % 2 == 0 && LH.back().n > 2) {
      const LevelHost &f = LH.back();
      LevelHost c;
      c.n = f.n / 2;
      c.wx.assign(c.n + 2, 0.0);
      c.wy.assign(c.n + 2, 0.0);
      c.cx.assign(c.n + 1, 0.0);
      c.cy.assign(c.n + 1, 0.0);
      for (int k = 1; k <= c.n; ++k) {
        c.wx[k] = f.wx[2 * k - 1] + f.wx[2 * k];
        c.wy[k] = f.wy[2 * k - 1] + f.wy[2 * k];
        c.cx[k] = f.cx[2 * k];
        c.cy[k] = f.cy[2 * k];
      }
      c.wx[c.n + 1] = f.wx[f.n + 1];
      c.wy[c.n + 1] = f.wy[f.n + 1];
      LH.push_back(c);
    }
    for (LevelHost &l : LH) {
      l.tx = axis_tables(l.n, p->eps, l.wx, l.cx);
      l.ty = axis_tables(l.n, p->eps, l.wy, l.cy);
    }
  }
  p->l64.assign(LH.size(), LevelDev<double>{});
  p->l32.assign(LH.size(), LevelDev<float>{});
  for (size_t l = 0; l < LH.size(); ++l) {
    BLP_TRY(upload_level<double>(p, LH[l], p->l64[l], l ? &p->l64[l - 1] : nullptr, p->f64.r, n1));
    BLP_TRY(upload_level<float>(p, LH[l], p->l32[l], l ? &p->l32[l - 1] : nullptr, p->f32.r, n1));
    level_diag<double>(p, p->l64[l], p->l64[l]);
    level_diag<float>(p, p->l64[l], p->l32[l]);
  }
  return BLP_OK;
}

// One parabolic and one exponential layer: x-semicoarsening, Galerkin
// levels (set up in FP64 on the device, then copied to FP32).  Coarsening
// halves the columns while their count is even and above 2.
int build_par_levels(blp_problem *p) {
  const int h = p->h;
  int L = 1;
  for (int m = h; m % 2 == 0 && m > 2; m /= 2) ++L;
  std::vector<ParLevelDev<double>> &D = p->pl64;
  std::vector<ParLevelDev<float>> &F = p->pl32;
  D.assign(L, ParLevelDev<double>{});
  F.assign(L, ParLevelDev<float>{});
  std::vector<double> sx(h + 2, 0.0), sy(h + 2, 0.0);
  for (int k = 1; k <= h; ++k) {
    sx[k] = 0.5 * (p->wx[k] + p->wx[k + 1]);
    sy[k] = 0.5 * (p->wy[k] + p->wy[k + 1]);
  }
  BLP_TRY(p->upload(&D[0].sx, sx));
  BLP_TRY(p->upload(&D[0].sy, sy));
  BLP_TRY(p->upload(&F[0].sx, sx));
  BLP_TRY(p->upload(&F[0].sy, sy));
  auto to32 = [&](const double *src, float **dst, size_t n) {
    BLP_TRY(p->alloc(dst, n));
    k_convert<double, float><<<blocks1d(n), 256, 0, p->stream>>>(src, *dst, n);
    return BLP_OK;
  };
  for (int l = 0; l < L; ++l) {
    D[l].nx = F[l].nx = h >> l;
    const int nx = D[l].nx;
    const size_t n = (size_t)nx * h;
    const ParSetupLevel f{p->grid64(), D[0].sx, D[0].sy, l ? D[l].a : nullptr, nx, h};
    // level 0 is smoothed with the two-exponential-layer level-0 tables;
    // each precision has its own coarse sweep shape
    const ParSkew sk64 = l ? par_skew(nx, h, 8) : ParSkew{}, sk32 = l ? par_skew(nx, h, 4) : ParSkew{};
    auto skew = [&](const double *src, double **d64, float **d32, int np) {
      BLP_TRY(zalloc(p, d64, np * sk64.nslot()));
      BLP_TRY(zalloc(p, d32, np * sk32.nslot()));
      k_par_skew<double><<<grid2d(nx, h), 256, 0, p->stream>>>(src, *d64, sk64, np);
      k_par_skew<float><<<grid2d(nx, h), 256, 0, p->stream>>>(src, *d32, sk32, np);
      return BLP_OK;
    };
    if (l > 0) {
      if (nx > kParMaxCols) return BLP_E_INVAL;
      D[l].sk = sk64;
      F[l].sk = sk32;
      BLP_TRY(p->alloc(&D[l].ic, n));
      k_par_invc<<<grid2d(nx, h), 256, 0, p->stream>>>(f, D[l].ic);
      BLP_TRY(skew(D[l].ic, &D[l].sic, &F[l].sic, 1));
      BLP_TRY(skew(D[l].a, &D[l].sa, &F[l].sa, 9));
      BLP_TRY(zalloc(p, &D[l].ssw, 4 * sk64.nslot()));
      BLP_TRY(zalloc(p, &F[l].ssw, 4 * sk32.nslot()));
      k_par_skew_sweep<double><<<grid2d(nx, h), 256, 0, p->stream>>>(D[l].a, D[l].ssw, sk64);
      k_par_skew_sweep<float><<<grid2d(nx, h), 256, 0, p->stream>>>(D[l].a, F[l].ssw, sk32);
    }
    if (l + 1 < L) {
      BLP_TRY(zalloc(p, &D[l].wl, n));
      BLP_TRY(zalloc(p, &D[l].wr, n));
      k_par_weights<<<grid2d((nx + 1) / 2, h), 256, 0, p->stream>>>(f, D[l].wl, D[l].wr);
      if (l == 0) {
        BLP_TRY(to32(D[0].wl, &F[0].wl, n));
        BLP_TRY(to32(D[0].wr, &F[0].wr, n));
      } else {
        BLP_TRY(skew(D[l].wl, &D[l].swl, &F[l].swl, 1));
        BLP_TRY(skew(D[l].wr, &D[l].swr, &F[l].swr, 1));
      }
      const int nxc = nx / 2;
      BLP_TRY(p->alloc(&D[l + 1].a, (size_t)9 * nxc * h));
      k_par_rap<<<grid2d(nxc, h), 256, 0, p->stream>>>(f, D[l].wl, D[l].wr, nxc, D[l + 1].a);
    }
    HIP_TRY(hipGetLastError());
  }
  return BLP_OK;
}

constexpr int kRows = 16;  // rows per block of the stencil kernels

}  // namespace

namespace {
#include "engine.h"

// The problem's own batch of nrhs systems (created on first use).
int own_batch(blp_problem *p, int nrhs, Batch **out) {
  if (!p->prec_ready) return BLP_E_STATE;
  if (!p->own || p->own_S != nrhs) {
    delete p->own;
    p->own = nullptr;
    p->own_S = 0;
    std::vector<blp_problem *> probs(nrhs, p);
    std::unique_ptr<Batch> B;
    BLP_TRY(batch_create(p->stream, probs.data(), nrhs, B));
    B->timer = &p->timer;
    p->own = B.release();
    p->own_S = nrhs;
  }
  *out = p->own;
  return BLP_OK;
}

int solve_common(blp_problem *p, bool tr, int nrhs, const double *F, double *U,
                 const blp_solve_opts *o, blp_solve_info *info, double *hist) {
  if (!p || !o || !F || !U || nrhs < 1) return BLP_E_INVAL;
  if (o->precond && !p->prec_ready) return BLP_E_STATE;
  if (!p->prec_ready) {
    // unpreconditioned solves still run on the engine's systems
    BLP_TRY(build_preconditioner(p));
    p->prec_ready = true;
  }
  Batch *B = nullptr;
  BLP_TRY(own_batch(p, nrhs, &B));
  std::vector<const double *> Fs(nrhs);
  std::vector<double *> Us(nrhs), Hs(nrhs, nullptr);
  for (int k = 0; k < nrhs; ++k) {
    Fs[k] = F + (size_t)k * p->n;
    Us[k] = U + (size_t)k * p->n;
    if (hist) Hs[k] = hist + (size_t)k * (o->maxit + 1);
  }
  return batch_solve(*B, tr, Fs.data(), Us.data(), o, info, hist ? Hs.data() : nullptr);
}

// M^{-1} x (or M^{-T} x) for one vector, through a one-off plan on the
// problem's first system.
template <typename T, bool TR>
int apply_prec(blp_problem *p, const T *x, T *y, int *cycles) {
  Batch *B = nullptr;
  BLP_TRY(own_batch(p, std::max(p->own_S, 1), &B));
  std::vector<System *> sys{B->sys[0].get()};
  std::vector<IOSpec> io{IOSpec{x, 0, y, 0}};
  PrecPlan<T, TR> P;
  BLP_TRY((build_prec_plan<T, TR>(p->stream, sys, io, false, P)));
  const Ctx c{p->stream, &p->timer};
  HIP_TRY(hipMemsetAsync(B->gate, 0, sizeof(int), p->stream));
  prec_part1<T, TR>(c, P, nullptr, p->popts);
  BLP_TRY((corner_finish<T, TR>(c, P, p->popts, first_cycles(P), B->ctrl, B->ctrl_h, 1)));
  prec_part2<T, TR>(c, P, nullptr);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(B->ctrl_h, B->ctrl, sizeof(MgCtrl), hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  if (cycles) *cycles = B->ctrl_h[0].cycles;
  return BLP_OK;
}

// y = A x or A^T x.
template <bool TR>
int apply_op(blp_problem *p, const double *x, double *y) {
  SpmvArgs<double> a{p->grid64(), x, 0, y, nullptr, nullptr, nullptr, nullptr};
  Alloc mem;
  SpmvArgs<double> *d = nullptr;
  BLP_TRY(mem.put(&d, &a, 1, p->stream));
  KScope ks(Ctx{p->stream, &p->timer}, KC_SPMV, (double)p->n * 2 * sizeof(double));
  k_stencil<double, TR, false, false>
      <<<dim3((p->n1 + 255) / 256, (p->n1 + kRows - 1) / kRows, 1), 256, 0, p->stream>>>(d, nullptr, kRows);
  ks.end();
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(p->stream));
  return BLP_OK;
}

int check_field(const blp_field *f, int N, bool allow_nodal, double lo, bool strict) {
  if (!f || !f->v) return BLP_E_INVAL;
  size_t cnt;
  switch (f->kind) {
    case BLP_CONST: cnt = 1; break;
    case BLP_AXIS: cnt = (size_t)N + 1; break;
    case BLP_NODAL: if (!allow_nodal) return BLP_E_INVAL; cnt = (size_t)(N - 1) * (N - 1); break;
    case BLP_BILINEAR:
      if (!allow_nodal || f->m < 2) return BLP_E_INVAL;
      cnt = (size_t)f->m * f->m;
      break;
    default: return BLP_E_INVAL;
  }
  for (size_t k = 0; k < cnt; ++k) {
    const double v = f->v[k];
    if (!std::isfinite(v) || (strict ? !(v > lo) : !(v >= lo))) return BLP_E_INVAL;
  }
  return BLP_OK;
}

}  // namespace

// ------------------------------------------------------------------------ //
// C ABI                                                                     //
// ------------------------------------------------------------------------ //

extern "C" {

int blp_mesh(int N, double eps, const blp_mesh_opts *o, double *x, double *y, double *tau) {
  if (N < 4 || N % 2 || !(eps > 0 && eps <= 1) || !x || !y) return BLP_E_INVAL;
  blp_mesh_opts m;
  BLP_TRY(mesh_options(N, o, &m));
  std::vector<double> nodes, w;
  const double tx = axis_mesh(N, eps, m.sigma, m.clow_x, m.kind, m.layer_cells, nodes, w);
  std::memcpy(x, nodes.data(), sizeof(double) * (N + 1));
  const double ty = axis_mesh(N, eps, m.sigma, m.clow_y, m.kind, m.layer_cells, nodes, w,
                              m.y_layer == BLP_LAYER_PARABOLIC);
  std::memcpy(y, nodes.data(), sizeof(double) * (N + 1));
  if (tau) {
    tau[0] = tx;
    tau[1] = ty;
  }
  return BLP_OK;
}

int blp_assemble(int N, double eps, const blp_field *c1, const blp_field *c2, const blp_field *r,
                 const blp_mesh_opts *mesh, void *stream, blp_problem **out) {
  if (!out) return BLP_E_INVAL;
  *out = nullptr;
  if (N < 4 || N % 2 || !(eps > 0 && eps <= 1)) return BLP_E_INVAL;
  if (N > 2048) return BLP_E_INVAL;  // one sweep workgroup holds at most 16 bands of 64 columns
  BLP_TRY(check_field(c1, N, false, 0.0, true));
  BLP_TRY(check_field(c2, N, false, 0.0, false));
  BLP_TRY(check_field(r, N, true, 0.0, false));
  blp_mesh_opts m;
  BLP_TRY(mesh_options(N, mesh, &m));
  // region sizes the kernels hold: edge lines of at most 1024 nodes, an
  // interior sweep of at most 16 bands of 64 columns
  if (m.layer_cells > 1024 || N - 1 - m.layer_cells > 1024) return BLP_E_INVAL;

  blp_problem *p = new (std::nothrow) blp_problem();
  if (!p) return BLP_E_NOMEM;
  p->N = N;
  p->n1 = N - 1;
  p->h = m.layer_cells;
  p->n = (size_t)(N - 1) * (N - 1);
  p->eps = eps;
  p->stream = (hipStream_t)stream;
  if (hipGetDevice(&p->device) != hipSuccess) {
    delete p;
    return BLP_E_HIP;
  }
  axis_mesh(N, eps, m.sigma, m.clow_x, m.kind, m.layer_cells, p->xn, p->wx);
  axis_mesh(N, eps, m.sigma, m.clow_y, m.kind, m.layer_cells, p->yn, p->wy,
            m.y_layer == BLP_LAYER_PARABOLIC);
  p->ylayer = m.y_layer;
  p->c1.assign(N + 1, 0.0);
  p->c2.assign(N + 1, 0.0);
  for (int k = 0; k <= N; ++k) {
    p->c1[k] = c1->kind == BLP_CONST ? c1->v[0] : c1->v[k];
    p->c2[k] = c2->kind == BLP_CONST ? c2->v[0] : c2->v[k];
  }
  p->fx = axis_tables(p->n1, eps, p->wx, p->c1);
  p->fy = axis_tables(p->n1, eps, p->wy, p->c2);
  int rc = BLP_OK;
  auto fail = [&](int code) {
    blp_destroy(p);
    return code;
  };
  if ((rc = p->upload(&p->xd, p->xn)) || (rc = p->upload(&p->yd, p->yn)) ||
      (rc = p->upload(&p->f64.W, p->fx.W)) || (rc = p->upload(&p->f64.E, p->fx.E)) ||
      (rc = p->upload(&p->f64.Dx, p->fx.D)) || (rc = p->upload(&p->f64.S, p->fy.W)) ||
      (rc = p->upload(&p->f64.N, p->fy.E)) || (rc = p->upload(&p->f64.Dy, p->fy.D)) ||
      (rc = p->upload(&p->f32.W, p->fx.W)) || (rc = p->upload(&p->f32.E, p->fx.E)) ||
      (rc = p->upload(&p->f32.Dx, p->fx.D)) || (rc = p->upload(&p->f32.S, p->fy.W)) ||
      (rc = p->upload(&p->f32.N, p->fy.E)) || (rc = p->upload(&p->f32.Dy, p->fy.D)))
    return fail(rc);
  p->f64.r = nullptr;
  p->f32.r = nullptr;
  if (r->kind == BLP_CONST) {
    p->rc = r->v[0];
    p->f64.rc = r->v[0];
    p->f32.rc = (float)r->v[0];
  } else {
    p->r_nodal = true;
    p->f64.rc = 0.0;
    p->f32.rc = 0.0f;
    if ((rc = p->alloc(&p->f64.r, p->n)) || (rc = p->alloc(&p->f32.r, p->n))) return fail(rc);
    if (r->kind == BLP_NODAL) {
      if (hipMemcpy(p->f64.r, r->v, p->n * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
        return fail(BLP_E_HIP);
    } else {
      // bilinear controls -> nodal values (hat functions on m uniform nodes)
      const int m = r->m;
      double *xd, *yd, *tx, *ty, *R;
      if ((rc = p->upload(&xd, p->xn)) || (rc = p->upload(&yd, p->yn)) ||
          (rc = p->alloc(&tx, (size_t)m * (N + 1))) || (rc = p->alloc(&ty, (size_t)m * (N + 1))) ||
          (rc = p->upload(&R, std::vector<double>(r->v, r->v + (size_t)m * m))))
        return fail(rc);
      k_axis_table<<<dim3(blocks1d(N + 1), m), 256, 0, p->stream>>>(xd, N, m, 1, tx);
      k_axis_table<<<dim3(blocks1d(N + 1), m), 256, 0, p->stream>>>(yd, N, m, 1, ty);
      k_synth<<<grid2d(p->n1, p->n1), 256, 0, p->stream>>>(N, m, m, R, tx, ty, p->f64.r);
    }
    k_convert<double, float><<<blocks1d(p->n), 256, 0, p->stream>>>(p->f64.r, p->f32.r, p->n);
  }
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(p->stream) != hipSuccess)
    return fail(BLP_E_HIP);
  *out = p;
  return BLP_OK;
}

int blp_nodes(const blp_problem *p, double *x, double *y) {
  if (!p || !x || !y) return BLP_E_INVAL;
  std::memcpy(x, p->xn.data(), sizeof(double) * (p->N + 1));
  std::memcpy(y, p->yn.data(), sizeof(double) * (p->N + 1));
  return BLP_OK;
}

int blp_precondition(blp_problem *p, const blp_prec_opts *o) {
  if (!p) return BLP_E_INVAL;
  // default corner stopping rule (Sec. 3.2): a residual reduction by 1e3
  // for two exponential layers, by 1e2 with a parabolic layer
  blp_prec_opts po = o ? *o
                       : blp_prec_opts{0, p->ylayer == BLP_LAYER_PARABOLIC ? 1e-2 : 1e-3, 20};
  if (po.mg_fixed < 0 || (po.mg_fixed == 0 && (!(po.mg_rtol > 0 && po.mg_rtol < 1) || po.mg_maxcyc < 1)))
    return BLP_E_INVAL;
  p->popts = po;
  if (p->prec_ready) return BLP_OK;
  BLP_TRY(build_preconditioner(p));
  p->prec_ready = true;
  return BLP_OK;
}

int blp_solve(blp_problem *p, int nrhs, const double *F, double *U, const blp_solve_opts *o,
              blp_solve_info *info, double *hist) {
  return solve_common(p, false, nrhs, F, U, o, info, hist);
}

int blp_solve_adjoint(blp_problem *p, int nrhs, const double *G, double *L,
                      const blp_solve_opts *o, blp_solve_info *info, double *hist) {
  return solve_common(p, true, nrhs, G, L, o, info, hist);
}

int blp_batch_create(blp_problem *const *probs, int S, void *stream, const blp_batch_opts *o,
                     blp_batch **out) {
  if (!out) return BLP_E_INVAL;
  *out = nullptr;
  if (!probs || S < 1) return BLP_E_INVAL;
  for (int s = 0; s < S; ++s) {
    if (!probs[s]) return BLP_E_INVAL;
    if (!probs[s]->prec_ready) return BLP_E_STATE;
  }
  if (o && o->sweep_variant < 0) return BLP_E_INVAL;
  std::unique_ptr<blp_batch> b(new (std::nothrow) blp_batch());
  if (!b) return BLP_E_NOMEM;
  // one part per mesh size and corner kind (exponential / parabolic layer
  // at y = 0), largest meshes first
  std::map<int, std::vector<int>> byN;
  for (int s = 0; s < S; ++s) byN[2 * probs[s]->N + probs[s]->ylayer].push_back(s);
  const bool graphs = o && o->graphs != 0;
  for (auto it = byN.rbegin(); it != byN.rend(); ++it) {
    std::vector<blp_problem *> pp;
    for (int s : it->second) pp.push_back(probs[s]);
    std::unique_ptr<Batch> B;
    BLP_TRY(batch_create((hipStream_t)stream, pp.data(), (int)pp.size(), B));
    B->timer = &B->own_timer;
    if (o) {
      B->graphs = o->graphs != 0;
      B->autotune = o->autotune != 0;
      B->sweep_variant = o->sweep_variant;
    }
    if (graphs || byN.size() > 1) {
      // a stream of the part's own: graphs cannot be captured on the legacy
      // default stream, and parts run concurrently; default priority
      hipStream_t st = nullptr;
      HIP_TRY(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
      B->user = B->stream;
      B->stream = st;
      B->own_stream = true;
    }
    b->parts.push_back(std::move(B));
    b->index.push_back(it->second);
  }
  *out = b.release();
  return BLP_OK;
}

// Solve every part, each on its own host thread; results and records go
// back to the caller's system order.  The most severe status wins (an
// error over BLP_W_NOCONV over BLP_OK).
static int parts_solve(blp_batch *b, bool tr, const double *const *F, double *const *U,
                       const blp_solve_opts *o, blp_solve_info *info) {
  const size_t P = b->parts.size();
  std::vector<int> rc(P, BLP_OK);
  std::vector<std::vector<blp_solve_info>> inf(P);
  auto run = [&](size_t k) {
    const std::vector<int> &ix = b->index[k];
    std::vector<const double *> f(ix.size());
    std::vector<double *> u(ix.size());
    for (size_t q = 0; q < ix.size(); ++q) {
      f[q] = F[ix[q]];
      u[q] = U[ix[q]];
    }
    inf[k].assign(ix.size(), blp_solve_info{});
    rc[k] = batch_solve(*b->parts[k], tr, f.data(), u.data(), o, inf[k].data(), nullptr);
  };
  if (P == 1) {
    run(0);
  } else {
    std::vector<std::thread> th;
    try {
      for (size_t k = 1; k < P; ++k) th.emplace_back(run, k);
    } catch (...) {
      for (auto &t : th) t.join();
      return BLP_E_NOMEM;
    }
    run(0);
    for (auto &t : th) t.join();
  }
  int out = BLP_OK;
  for (size_t k = 0; k < P; ++k) {
    if (rc[k] < 0 && (out >= 0 || rc[k] < out)) out = rc[k];
    if (rc[k] == BLP_W_NOCONV && out == BLP_OK) out = BLP_W_NOCONV;
    if (info)
      for (size_t q = 0; q < b->index[k].size(); ++q) info[b->index[k][q]] = inf[k][q];
  }
  return out;
}

int blp_batch_solve(blp_batch *b, const double *const *F, double *const *U,
                    const blp_solve_opts *o, blp_solve_info *info) {
  if (!b || !F || !U) return BLP_E_INVAL;
  return parts_solve(b, false, F, U, o, info);
}

int blp_batch_solve_adjoint(blp_batch *b, const double *const *G, double *const *L,
                            const blp_solve_opts *o, blp_solve_info *info) {
  if (!b || !G || !L) return BLP_E_INVAL;
  return parts_solve(b, true, G, L, o, info);
}

long long blp_batch_footprint(const blp_batch *b) {
  long long n = 0;
  if (b)
    for (const auto &B : b->parts) n += batch_bytes(*B);
  return n;
}

int blp_batch_timing(blp_batch *b, int enable, double *ms, long long *launches, double *bytes) {
  if (!b) return BLP_E_INVAL;
  for (auto &B : b->parts) {
    HIP_TRY(hipStreamSynchronize(B->stream));
    for (hipStream_t q : B->cstream) HIP_TRY(hipStreamSynchronize(q));
  }
  if (enable) {
    for (auto &B : b->parts) B->own_timer.start();
    return BLP_OK;
  }
  // per-class sums over the parts (their launches overlap in time)
  double tms[BLP_NCLASS] = {}, tby[BLP_NCLASS] = {};
  long long tl[BLP_NCLASS] = {};
  for (auto &B : b->parts) {
    double m[BLP_NCLASS], y[BLP_NCLASS];
    long long l[BLP_NCLASS];
    BLP_TRY(B->own_timer.stop(m, l, y, BLP_NCLASS));
    for (int k = 0; k < BLP_NCLASS; ++k) {
      tms[k] += m[k];
      tl[k] += l[k];
      tby[k] += y[k];
    }
  }
  for (int k = 0; k < BLP_NCLASS; ++k) {
    if (ms) ms[k] = tms[k];
    if (launches) launches[k] = tl[k];
    if (bytes) bytes[k] = tby[k];
  }
  return BLP_OK;
}

int blp_batch_describe(const blp_batch *b, char *buf, int len) {
  if (!b || !buf || len < 1) return BLP_E_INVAL;
  std::string s;
  for (size_t k = 0; k < b->parts.size(); ++k) {
    char h[64];
    snprintf(h, sizeof h, "part %zu (own FGMRES loop):\n", k);
    s += h;
    s += describe(*b->parts[k]);
  }
  const int n = std::min((int)s.size(), len - 1);
  std::memcpy(buf, s.data(), n);
  buf[n] = 0;
  return (int)s.size();
}

void blp_batch_destroy(blp_batch *b) { delete b; }

int blp_apply(blp_problem *p, int op, const double *x, double *y, int *cycles) {
  if (!p || !x || !y) return BLP_E_INVAL;
  if (cycles) *cycles = 0;
  if (op == BLP_OP_A) return apply_op<false>(p, x, y);
  if (op == BLP_OP_AT) return apply_op<true>(p, x, y);
  if (op != BLP_OP_MINV && op != BLP_OP_MINVT && op != BLP_OP_MINV32) return BLP_E_INVAL;
  if (!p->prec_ready) return BLP_E_STATE;
  if (op == BLP_OP_MINV32) {
    k_convert<double, float><<<blocks1d(p->n), 256, 0, p->stream>>>(x, p->tmp32a, p->n);
    BLP_TRY((apply_prec<float, false>(p, p->tmp32a, p->tmp32b, cycles)));
    k_convert<float, double><<<blocks1d(p->n), 256, 0, p->stream>>>(p->tmp32b, y, p->n);
  } else if (op == BLP_OP_MINVT) {
    BLP_TRY((apply_prec<double, true>(p, x, y, cycles)));
  } else {
    BLP_TRY((apply_prec<double, false>(p, x, y, cycles)));
  }
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(p->stream));
  return BLP_OK;
}

int blp_sine_rhs(blp_problem *p, int K, int L, const double *a, double *F) {
  if (!p || K < 1 || L < 1 || !a || !F) return BLP_E_INVAL;
  const int N = p->N;
  double *xd, *yd, *tx, *ty, *ad;
  std::vector<void *> tmp;
  auto al = [&](double **q, size_t c) {
    void *v = nullptr;
    if (hipMalloc(&v, c * sizeof(double)) != hipSuccess) return false;
    tmp.push_back(v);
    *q = (double *)v;
    return true;
  };
  int rc = BLP_OK;
  if (!al(&xd, N + 1) || !al(&yd, N + 1) || !al(&tx, (size_t)K * (N + 1)) ||
      !al(&ty, (size_t)L * (N + 1)) || !al(&ad, (size_t)K * L)) {
    rc = BLP_E_NOMEM;
  } else if (hipMemcpyAsync(xd, p->xn.data(), (N + 1) * sizeof(double), hipMemcpyHostToDevice, p->stream) ||
             hipMemcpyAsync(yd, p->yn.data(), (N + 1) * sizeof(double), hipMemcpyHostToDevice, p->stream) ||
             hipMemcpyAsync(ad, a, (size_t)K * L * sizeof(double), hipMemcpyHostToDevice, p->stream)) {
    rc = BLP_E_HIP;
  } else {
    k_axis_table<<<dim3(blocks1d(N + 1), K), 256, 0, p->stream>>>(xd, N, K, 0, tx);
    k_axis_table<<<dim3(blocks1d(N + 1), L), 256, 0, p->stream>>>(yd, N, L, 0, ty);
    k_synth<<<grid2d(p->n1, p->n1), 256, 0, p->stream>>>(N, K, L, ad, tx, ty, F);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(p->stream) != hipSuccess) rc = BLP_E_HIP;
  }
  for (void *v : tmp) (void)hipFree(v);
  return rc;
}

// Scratch of the allocation-free projection (blp_sine_project_noalloc): a
// fixed array that every GPU the library runs on holds once, at its own
// address, until the process ends.  Host code never uses this name as an
// address: the device address is looked up per device (scratch_ptr) and
// passed to the kernels.  Calls that overlap on one GPU share it and race.
constexpr size_t kScratchBytes = (size_t)4 << 20;
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// This GPU's scratch address, looked up once per device with that device
// current (the caller's current device, which must be the problem's).
int scratch_ptr(int dev, double **out) {
  if (dev < 0 || dev >= kMaxDevices) return BLP_E_STATE;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *q = nullptr;
    if (hipGetSymbolAddress(&q, HIP_SYMBOL(scratch)) != hipSuccess || !q) return BLP_E_HIP;
    g_scratch_ptr[dev] = static_cast<double *>(q);
  }
  *out = g_scratch_ptr[dev];
  return BLP_OK;
}

// doubles rounded up to whole 256-byte blocks
size_t scratch_words(size_t words) { return (words + 31) / 32 * 32; }
}  // namespace

static int project(blp_problem *p, int K, int L, int kind, int nrhs, double scale, const double *w,
                   const double *v, double *g) {
  const int N = p->N, n1 = p->n1;
  double *xd, *yd, *tx, *ty, *t, *gd;
  std::vector<void *> tmp;
  auto al = [&](double **q, size_t c) {
    void *v = nullptr;
    if (hipMalloc(&v, c * sizeof(double)) != hipSuccess) return false;
    tmp.push_back(v);
    *q = (double *)v;
    return true;
  };
  int rc = BLP_OK;
  if (!al(&xd, N + 1) || !al(&yd, N + 1) || !al(&tx, (size_t)K * (N + 1)) ||
      !al(&ty, (size_t)L * (N + 1)) || !al(&t, (size_t)K * n1) || !al(&gd, (size_t)K * L)) {
    rc = BLP_E_NOMEM;
  } else if (hipMemcpyAsync(xd, p->xn.data(), (N + 1) * sizeof(double), hipMemcpyHostToDevice, p->stream) ||
             hipMemcpyAsync(yd, p->yn.data(), (N + 1) * sizeof(double), hipMemcpyHostToDevice, p->stream)) {
    rc = BLP_E_HIP;
  } else {
    k_axis_table<<<dim3(blocks1d(N + 1), K), 256, 0, p->stream>>>(xd, N, K, kind, tx);
    k_axis_table<<<dim3(blocks1d(N + 1), L), 256, 0, p->stream>>>(yd, N, L, kind, ty);
    k_project_rows<<<n1, 256, 0, p->stream>>>(N, K, nrhs, scale, w, v, tx, t);
    k_project_cols<<<dim3(K, L), 256, 0, p->stream>>>(N, K, t, ty, gd);
    if (hipMemcpyAsync(g, gd, (size_t)K * L * sizeof(double), hipMemcpyDeviceToHost, p->stream) ||
        hipGetLastError() != hipSuccess || hipStreamSynchronize(p->stream) != hipSuccess)
      rc = BLP_E_HIP;
  }
  for (void *v : tmp) (void)hipFree(v);
  return rc;
}

int blp_sine_project(blp_problem *p, int K, int L, const double *w, double *g) {
  if (!p || K < 1 || L < 1 || !w || !g) return BLP_E_INVAL;
  return project(p, K, L, 0, 1, 1.0, w, nullptr, g);
}

int blp_bilinear_project(blp_problem *p, int m, const double *w, double *G) {
  if (!p || m < 2 || !w || !G) return BLP_E_INVAL;
  return project(p, m, m, 1, 1, 1.0, w, nullptr, G);
}

namespace {
// Memory of blp1d_solve, kept per device between calls and grown on demand:
// device words (nodal c and r, work space, result records) and pinned host
// words (c and r staged for one copy in, the records for one copy out, the
// argument records).  Calls on one device take its mutex for their whole
// duration (each ends with a stream synchronisation), so they run one at a
// time and the memory is never shared by two of them.
struct OneDCache {
  std::mutex mu;
  double *dev = nullptr;
  size_t dev_words = 0;
  unsigned char *host = nullptr;  // pinned
  size_t host_bytes = 0;
};
OneDCache g_oned[kMaxDevices];

int oned_reserve(OneDCache &c, size_t dev_words, size_t host_bytes) {
  if (c.dev_words < dev_words) {
    (void)hipFree(c.dev);
    c.dev = nullptr;
    c.dev_words = 0;
    if (hipMalloc((void **)&c.dev, dev_words * sizeof(double)) != hipSuccess) return BLP_E_NOMEM;
    c.dev_words = dev_words;
  }
  if (c.host_bytes < host_bytes) {
    (void)hipHostFree(c.host);
    c.host = nullptr;
    c.host_bytes = 0;
    if (hipHostMalloc((void **)&c.host, host_bytes, hipHostMallocDefault) != hipSuccess) return BLP_E_NOMEM;
    c.host_bytes = host_bytes;
  }
  return BLP_OK;
}
}  // namespace

int blp1d_solve(int S, const blp1d_problem *probs, const double *const *F, double *const *U,
                const blp1d_opts *o, void *stream, blp1d_info *info) {
  if (S < 1 || !probs || !F || !U || !o) return BLP_E_INVAL;
  if (o->maxit < 1 || o->maxit > k1dMaxIt) return BLP_E_INVAL;
  const hipStream_t st = (hipStream_t)stream;
  const int m = o->maxit;
  // per problem: nodal c and r (copied in), device work space (stencil
  // rows, factorisations, vectors, basis, Hessenberg, built by the kernel
  // itself) and a result record of 4 words
  std::vector<size_t> off(S + 1, 0), woff(S + 1, 0);
  std::vector<blp_mesh_opts> mo(S);
  for (int s = 0; s < S; ++s) {
    const blp1d_problem &q = probs[s];
    if (q.N < 4 || q.N % 2 || q.N > 4096 || !(q.eps > 0 && q.eps <= 1) || !q.c || !q.r ||
        !F[s] || !U[s])
      return BLP_E_INVAL;
    const blp_mesh_opts in{q.sigma, q.clow, q.clow, q.kind, q.layer_cells, BLP_LAYER_EXPONENTIAL};
    BLP_TRY(mesh_options(q.N, &in, &mo[s]));
    const size_t n = (size_t)q.N - 1;
    off[s + 1] = off[s] + 2 * ((size_t)q.N + 1);
    woff[s + 1] = woff[s] + 9 * n + (size_t)(m + 1) * n + (size_t)(m + 1) * m;
  }
  int dev_id = -1;
  HIP_TRY(hipGetDevice(&dev_id));
  if (dev_id < 0 || dev_id >= kMaxDevices) return BLP_E_STATE;
  OneDCache &cache = g_oned[dev_id];
  std::lock_guard<std::mutex> lock(cache.mu);
  // device: c and r, records, work space, argument records (16-byte aligned)
  const size_t rec0 = off[S], work0 = rec0 + 4 * (size_t)S;
  const size_t args0 = (work0 + woff[S] + 1) / 2 * 2;
  const size_t argw = ((size_t)S * sizeof(OneDArgs) + sizeof(double) - 1) / sizeof(double);
  // pinned host: c and r, records, argument records (the same offsets)
  BLP_TRY(oned_reserve(cache, args0 + argw, (rec0 + 4 * (size_t)S) * sizeof(double) + argw * sizeof(double)));
  double *hc = reinterpret_cast<double *>(cache.host);
  double *hrec = hc + rec0;
  OneDArgs *hargs = reinterpret_cast<OneDArgs *>(hc + rec0 + 4 * (size_t)S);
  double *dev = cache.dev, *recs = dev + rec0, *work = dev + work0;
  OneDArgs *dargs = reinterpret_cast<OneDArgs *>(dev + args0);
  // c > 0 and r >= 0 (NaN fails both), checked without branches on the
  // copies
  for (int s = 0; s < S; ++s) {
    const blp1d_problem &q = probs[s];
    const int N = q.N;
    double *cs = hc + off[s], *rs = cs + N + 1;
    std::memcpy(cs, q.c, (N + 1) * sizeof(double));
    std::memcpy(rs, q.r, (N + 1) * sizeof(double));
    int bad = 0;
    for (int k = 0; k <= N; ++k) bad |= !(cs[k] > 0.0) | !(rs[k] >= 0.0);
    if (bad) return BLP_E_INVAL;
  }
  for (int s = 0; s < S; ++s) {
    const blp1d_problem &q = probs[s];
    const blp_mesh_opts &mm = mo[s];
    const int N = q.N, n = N - 1, nl = mm.layer_cells;
    // the constants of the closed-form widths (the same construction as
    // blp_mesh's, evaluated per cell in the kernel)
    const double qf = (double)nl / N, layer = mm.sigma * q.eps * std::log((double)N) / mm.clow_x;
    const double tau = std::min(qf, layer);
    OneDArgs a{};
    double *wk = work + woff[s];
    a.n = n;
    a.nl = nl;
    a.eps = q.eps;
    a.hl = tau / nl;
    a.hi = (1.0 - tau) / (N - nl);
    a.s = mm.sigma * q.eps / mm.clow_x;
    a.a = (1.0 - 1.0 / N) / nl;
    a.graded = mm.kind == BLP_MESH_BAKHVALOV_SHISHKIN && layer < qf;
    a.c = dev + off[s];
    a.r = dev + off[s] + N + 1;
    a.W = wk;
    a.C = wk + n;
    a.E = wk + 2 * n;
    a.a_inv = wk + 3 * n;
    a.a_cp = wk + 4 * n;
    a.m_inv = wk + 5 * n;
    a.m_cp = wk + 6 * n;
    a.t = wk + 7 * n;
    a.w = wk + 8 * n;
    a.V = wk + 9 * n;
    a.H = a.V + (size_t)(m + 1) * n;
    a.info = recs + 4 * (size_t)s;
    a.F = F[s];
    a.U = U[s];
    a.K = o->K;
    a.g = o->g > 0 ? o->g : std::log((double)N) / N;
    a.maxit = m;
    a.left = o->left != 0;
    hargs[s] = a;
  }
  int rc = BLP_OK;
  if (hipMemcpyAsync(dev, hc, rec0 * sizeof(double), hipMemcpyHostToDevice, st) ||
      hipMemcpyAsync(dargs, hargs, S * sizeof(OneDArgs), hipMemcpyHostToDevice, st)) {
    rc = BLP_E_HIP;
  } else {
    k_gmres1d<<<S, k1dThreads, 0, st>>>(dargs);
    if (hipGetLastError() != hipSuccess) rc = BLP_E_HIP;
    if (rc == BLP_OK &&
        hipMemcpyAsync(hrec, recs, 4 * (size_t)S * sizeof(double), hipMemcpyDeviceToHost, st))
      rc = BLP_E_HIP;
  }
  // the pinned buffers are reused by the next call: wait here in any case
  if (hipStreamSynchronize(st) != hipSuccess && rc == BLP_OK) rc = BLP_E_HIP;
  if (rc != BLP_OK) return rc;
  for (int s = 0; s < S; ++s) {
    const double *r = hrec + 4 * (size_t)s;
    if (info) {
      info[s].iterations = (int)r[0];
      info[s].converged = r[1] != 0.0;
      info[s].res_inf = r[2];
      info[s].K = r[3];
    }
    if (!std::isfinite(r[2])) rc = BLP_E_NUMERIC;
    else if (r[1] == 0.0 && rc == BLP_OK) rc = BLP_W_NOCONV;
  }
  return rc;
}

int blp_sine_project_noalloc(blp_problem *p, int K, int L, const double *w, double *g) {
  if (!p || K < 1 || L < 1 || !w || !g) return BLP_E_INVAL;
  const int N = p->N, n1 = p->n1;
  // tables of the two axes, row partials and the K x L result
  const size_t ntx = scratch_words((size_t)K * (N + 1)), nty = scratch_words((size_t)L * (N + 1));
  const size_t nt = scratch_words((size_t)K * n1), ng = scratch_words((size_t)K * L);
  if ((ntx + nty + nt + ng) * sizeof(double) > kScratchBytes) return BLP_E_SCRATCH;
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != p->device) return BLP_E_STATE;
  double *base = nullptr;
  BLP_TRY(scratch_ptr(dev, &base));
  // every word read below is written first in the same call: nothing to clear
  double *tx = base, *ty = tx + ntx, *t = ty + nty, *gd = t + nt;
  k_axis_table<<<dim3(blocks1d(N + 1), K), 256, 0, p->stream>>>(p->xd, N, K, 0, tx);
  k_axis_table<<<dim3(blocks1d(N + 1), L), 256, 0, p->stream>>>(p->yd, N, L, 0, ty);
  k_project_rows<<<n1, 256, 0, p->stream>>>(N, K, 1, 1.0, w, nullptr, tx, t);
  k_project_cols<<<dim3(K, L), 256, 0, p->stream>>>(N, K, t, ty, gd);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(g, gd, (size_t)K * L * sizeof(double), hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  return BLP_OK;
}

int blp_reaction_gradient(blp_problem *p, int m, int nrhs, const double *Lambda, const double *U,
                          double *G) {
  if (!p || m < 2 || nrhs < 1 || !Lambda || !U || !G) return BLP_E_INVAL;
  return project(p, m, m, 1, nrhs, -1.0, Lambda, U, G);
}

int blp_mul(blp_problem *p, const double *a, const double *b, double *out) {
  if (!p || !a || !b || !out) return BLP_E_INVAL;
  k_mul<<<blocks1d(p->n), 256, 0, p->stream>>>(a, b, out, p->n);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(p->stream));
  return BLP_OK;
}

int blp_timing(blp_problem *p, int enable, double *ms, long long *launches, double *bytes) {
  if (!p) return BLP_E_INVAL;
  HIP_TRY(hipStreamSynchronize(p->stream));
  if (enable) {
    p->timer.start();
    return BLP_OK;
  }
  return p->timer.stop(ms, launches, bytes, BLP_NCLASS);
}

long long blp_footprint(const blp_problem *p) {
  return p ? p->bytes + (p->own ? batch_bytes(*p->own) : 0) : 0;
}

void blp_destroy(blp_problem *p) {
  if (!p) return;
  (void)hipStreamSynchronize(p->stream);
  for (void *q : p->allocs) (void)hipFree(q);
  delete p->own;
  delete p;
}

const char *blp_strerror(int code) {
  switch (code) {
    case BLP_OK: return "ok";
    case BLP_W_NOCONV: return "iteration cap reached before the tolerance";
    case BLP_E_INVAL: return "invalid argument";
    case BLP_E_NOMEM: return "out of memory";
    case BLP_E_HIP: return "HIP runtime error";
    case BLP_E_STATE: return "call out of order";
    case BLP_E_NUMERIC: return "NaN or Inf in a residual";
    case BLP_E_SCRATCH: return "request exceeds the fixed scratch buffer of the allocation-free call";
    default: return "unknown error";
  }
}

}  // extern "C"
