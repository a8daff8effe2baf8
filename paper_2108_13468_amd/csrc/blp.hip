// Host side of the MI355X boundary-layer-preconditioned FGMRES solver: the C
// ABI of include/blp.h, setup of the mesh tables and the preconditioner, and
// the orchestration of the HIP kernels on the problem's stream.
//
// Method: arXiv 2108.13468 (MacLachlan, Madden, Nhan).  The host computes only
// O(N) per-axis quantities (mesh widths and stencil tables, in FP64); every
// O(N^2) step runs in the kernels of kernels_*.h.
#include <hip/hip_runtime.h>

#include <algorithm>
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
  T *z, *b, *t;  // skewed work vectors
  Grid<T> grid() const { return Grid<T>{n, n, W, E, Dx, S, N, Dy, r, n, rc}; }
  MgLevel<T> view(bool tr) const {
    return MgLevel<T>{grid(), ic[tr ? 1 : 0], hbx, hby, wlx, wrx, wly, wry, z, b, t, nslot};
  }
};

template <typename T>
struct FineDev {
  T *W, *E, *Dx, *S, *N, *Dy, *r, rc;
  T *dh;          // sqrt(C), natural layout (scaled-system input)
  T *fac[4][3];   // line factors [Y fwd, X fwd, Y tr, X tr] x [d, m, w]
  T *icI[2];      // skewed 1/C of the interior region, per direction
  T *bI, *zI;     // skewed work vectors of the interior region
  T *bL[2], *zL[2];  // line-major work vectors of the edge regions [Y, X], stride hp
  size_t nslotI;
};

}  // namespace

struct blp_problem {
  int N, n1, h;
  size_t n;
  double eps;
  hipStream_t stream;
  std::vector<double> xn, yn, wx, wy, c1, c2;  // nodes, widths (1..N), coefficients (0..N)
  AxisTab fx, fy;
  bool r_nodal = false;
  double rc = 0.0;
  FineDev<double> f64{};
  FineDev<float> f32{};
  bool prec_ready = false;
  blp_prec_opts popts{0, 1e-3, 20};
  std::vector<LevelDev<double>> l64;
  std::vector<LevelDev<float>> l32;
  MgCtrl *ctrl = nullptr;
  MgCtrl *ctrl_h = nullptr;       // pinned host mirror
  KrylovStatus *st = nullptr;
  KrylovStatus *st_h = nullptr;   // pinned host mirror
  double *mg_partials = nullptr;
  double *partials = nullptr;     // Krylov reduction partials
  size_t partials_len = 0;
  // Krylov workspace (sized at first solve, grown on demand)
  int ws_m = 0;
  int ws_prec = -1;
  void *V = nullptr, *Z = nullptr;
  double *w = nullptr, *ks = nullptr;
  float *tmp32a = nullptr, *tmp32b = nullptr;
  std::vector<void *> allocs;
  long long bytes = 0;
  std::vector<void *> ws_allocs;
  long long ws_bytes = 0;
  // kernel timing (blp_timing): event pairs per class, resolved on demand
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  struct Rec { int cls; hipEvent_t a, b; double bytes; };
  std::vector<Rec> recs;
  hipEvent_t ev_next() {
    if (ev_used == ev_pool.size()) {
      hipEvent_t e;
      // timestamps only: no system-scope fence (the stream is synchronised
      // before the times are read), so recording does not flush caches
      if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
      ev_pool.push_back(e);
    }
    return ev_pool[ev_used++];
  }

  template <typename T>
  int alloc(T **p, size_t count, bool ws = false) {
    void *q = nullptr;
    if (hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess) return BLP_E_NOMEM;
    (ws ? ws_allocs : allocs).push_back(q);
    (ws ? ws_bytes : bytes) += (long long)(count * sizeof(T));
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

// Records an event pair around the launches issued during its lifetime when
// timing is enabled.
struct KScope {
  blp_problem *p;
  int cls;
  double bytes;
  hipEvent_t a = nullptr;
  KScope(blp_problem *p_, int c, double b) : p(p_), cls(c), bytes(b) {
    if (p->timing && (a = p->ev_next())) (void)hipEventRecord(a, p->stream);
  }
  void end() {
    if (!a) return;
    hipEvent_t b = p->ev_next();
    if (b) {
      (void)hipEventRecord(b, p->stream);
      p->recs.push_back({cls, a, b, bytes});
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
Grid<T> fine_grid(blp_problem *p);
template <>
Grid<double> fine_grid<double>(blp_problem *p) { return p->grid64(); }
template <>
Grid<float> fine_grid<float>(blp_problem *p) { return p->grid32(); }

inline dim3 grid2d(int nx, int ny, int bx = 256) { return dim3((nx + bx - 1) / bx, ny); }
inline unsigned blocks1d(size_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

bool finite_all(const double *v, size_t n) {
  for (size_t k = 0; k < n; ++k)
    if (!std::isfinite(v[k])) return false;
  return true;
}

double shishkin_tau(int N, double eps, double sigma, double clow) {
  return std::min(0.5, sigma * eps * std::log((double)N) / clow);
}

// Widths of one axis: 2 tau / N on the N/2 layer cells, 2 (1 - tau) / N on the
// others, taken from the closed form (never as differences of coordinates).
void axis_mesh(int N, double tau, std::vector<double> &nodes, std::vector<double> &w) {
  nodes.assign(N + 1, 0.0);
  w.assign(N + 2, 0.0);
  const double hl = 2.0 * tau / N, hi = 2.0 * (1.0 - tau) / N;
  for (int k = 0; k <= N; ++k) nodes[k] = k <= N / 2 ? k * hl : tau + (k - N / 2) * hi;
  for (int k = 1; k <= N; ++k) w[k] = k <= N / 2 ? hl : hi;
}

// ------------------------------------------------------------------------ //
// Preconditioner apply                                                      //
// ------------------------------------------------------------------------ //

template <typename T, bool TR>
void launch_sweep(blp_problem *p, const Grid<T> &g, int i0, int i1, int j0, int j1, const T *b,
                  const T *ic, T *z, const int *gate) {
  const int nb = (i1 - i0 + 1 + 63) / 64;
  SweepArgs<T> a{g, i0, i1, j0, j1, b, ic, z, gate};
  const double pts = (double)(i1 - i0 + 1) * (j1 - j0 + 1);
  KScope ks(p, KC_SWEEP, pts * 2 * sizeof(T));
  // superstep of K steps = 4 chunks of 16 bytes per lane; D supersteps of
  // loads in flight (D + 1 register buffers of 2K words); more than 8 waves
  // leave registers for D = 1 only
  constexpr int K = 4 * kChunk<T>;
  if (nb <= 8)
    k_sweep<T, TR, K, 4><<<1, 64 * nb, 0, p->stream>>>(a);
  else
    k_sweep<T, TR, K, 1><<<1, 64 * nb, 0, p->stream>>>(a);
}

// Row stride of the line-major edge-region buffers: h rounded up to a
// multiple of 4, so that every thread's nodes are 16-byte aligned.
inline int line_stride(int h) { return (h + 3) / 4 * 4; }

template <typename T, bool TR, int EP, int W>
void launch_lines_k(blp_problem *p, const LineArgs<T> &a) {
  // D lines of operands in flight: 4 EP words per line and wave, within the
  // 63 outstanding memory operations a wave can track and its registers
  constexpr int D = EP >= 4 ? 4 : 6;
  k_lines<T, TR, EP, W, D><<<2, 64 * W, 0, p->stream>>>(a);
}

template <typename T, bool TR>
void launch_lines(blp_problem *p, const T *v, const T *dh, T *z) {
  FineDev<T> &f = fine<T>(p);
  const int h = p->h, n1 = p->n1, hp = line_stride(h);
  LineArgs<T> a;
  a.g = fine_grid<T>(p);
  a.h = h;
  a.n1 = n1;
  a.hp = hp;
  const int base = TR ? 2 : 0;
  for (int r = 0; r < 2; ++r) {
    a.b[r] = f.bL[r];
    a.z[r] = f.zL[r];
    a.fd[r] = f.fac[base + r][0];
    a.fm[r] = f.fac[base + r][1];
    a.fw[r] = f.fac[base + r][2];
  }
  a.gate = nullptr;
  const dim3 gl((hp + 255) / 256, n1 - h, 2);
  {
    KScope ks(p, KC_LAYOUT, 0.0);
    k_gather_lines<T, TR><<<gl, 256, 0, p->stream>>>(a.g, v, dh, z, h, n1, hp, f.bL[0], f.bL[1]);
  }
  KScope ks(p, KC_LINES, 2.0 * (n1 - h) * h * 4 * sizeof(T));
  // threads hold EP contiguous nodes; up to 4 waves per region
  if (hp <= 64)
    launch_lines_k<T, TR, 1, 1>(p, a);
  else if (hp <= 128)
    launch_lines_k<T, TR, 1, 2>(p, a);
  else if (hp <= 256)
    launch_lines_k<T, TR, 1, 4>(p, a);
  else if (hp <= 512)
    launch_lines_k<T, TR, 2, 4>(p, a);
  else
    launch_lines_k<T, TR, 4, 4>(p, a);
  ks.end();
  KScope ks2(p, KC_LAYOUT, 0.0);
  k_scatter_lines<T, TR><<<gl, 256, 0, p->stream>>>(f.zL[0], f.zL[1], h, n1, hp, z);
}

// Interior region: gather into the skewed layout, sweep, scatter back.
template <typename T, bool TR>
void interior_solve(blp_problem *p, const T *v, const T *dh, T *z) {
  FineDev<T> &f = fine<T>(p);
  const int h = p->h, n1 = p->n1;
  const SkewT<T, TR> sk{h + 1, n1, h + 1, n1};
  const unsigned nb = blocks1d(f.nslotI);
  {
    KScope ks(p, KC_LAYOUT, 0.0);
    k_gather_skew<T, TR><<<nb, 256, 0, p->stream>>>(fine_grid<T>(p), sk, v, dh, z, f.bI, f.nslotI);
  }
  launch_sweep<T, TR>(p, fine_grid<T>(p), h + 1, n1, h + 1, n1, f.bI, f.icI[TR ? 1 : 0], f.zI,
                      nullptr);
  KScope ks(p, KC_LAYOUT, 0.0);
  k_scatter_skew<T, TR><<<nb, 256, 0, p->stream>>>(sk, f.zI, z, n1, f.nslotI);
}

// Gauss-Seidel rhs of a level into its t vector (t is free at that point).
template <typename T, bool TR>
void gs_rhs(blp_problem *p, const LevelDev<T> &lv, const int *gate) {
  KScope ks(p, KC_GSRHS, (double)lv.n * lv.n * 3 * sizeof(T));
  k_gs_rhs<T, TR><<<blocks1d(lv.nslot), 256, 0, p->stream>>>(lv.grid(), lv.b, lv.z, lv.t, lv.nslot,
                                                             gate);
}

// One V(1,1) cycle on level l (Sec. 3.2).  zero_init: the level iterate is
// zero on entry, so the pre-smoothing sweep is the plain triangular solve.
template <typename T, bool TR>
void vcycle(blp_problem *p, int l, bool zero_init, const int *gate) {
  std::vector<LevelDev<T>> &L = levels<T>(p);
  const LevelDev<T> &lv = L[l];
  const int n = lv.n;
  if (l == (int)L.size() - 1) {
    KScope ks(p, KC_MG, (double)n * n * 2 * sizeof(T));
    k_mg_coarsest<T, TR><<<1, 64, 0, p->stream>>>(lv.view(TR), zero_init ? 1 : 0, gate);
    return;
  }
  const LevelDev<T> &cv = L[l + 1];
  const T *ic = lv.ic[TR ? 1 : 0];
  if (zero_init) {
    launch_sweep<T, TR>(p, lv.grid(), 1, n, 1, n, lv.b, ic, lv.z, gate);
  } else {
    gs_rhs<T, TR>(p, lv, gate);
    launch_sweep<T, TR>(p, lv.grid(), 1, n, 1, n, lv.t, ic, lv.z, gate);
  }
  {
    KScope ks(p, KC_MG, (double)n * n * 3 * sizeof(T));
    k_mg_resid<T, TR><<<blocks1d(lv.nslot), 256, 0, p->stream>>>(lv.view(TR), gate);
  }
  {
    KScope ks(p, KC_MG, ((double)n * n + (double)cv.n * cv.n) * sizeof(T));
    k_mg_restrict<T, TR><<<blocks1d(cv.nslot), 256, 0, p->stream>>>(lv.view(TR), cv.view(TR), gate);
  }
  vcycle<T, TR>(p, l + 1, true, gate);
  {
    KScope ks(p, KC_MG, ((double)n * n * 2 + (double)cv.n * cv.n) * sizeof(T));
    k_mg_prolong<T, TR><<<blocks1d(lv.nslot), 256, 0, p->stream>>>(lv.view(TR), cv.view(TR), gate);
  }
  gs_rhs<T, TR>(p, lv, gate);
  launch_sweep<T, TR>(p, lv.grid(), 1, n, 1, n, lv.t, ic, lv.z, gate);
}

// blocks of the corner residual-norm reduction (one partial each)
constexpr int kMgNormBlocks = 256;

// Corner solve M_CC^{-1} b_0 (level 0 b and z).  Cycles are counted in ctrl.
template <typename T, bool TR>
int corner_solve(blp_problem *p) {
  std::vector<LevelDev<T>> &L = levels<T>(p);
  const LevelDev<T> &l0 = L[0];
  const blp_prec_opts &o = p->popts;
  const int nblk = std::min(kMgNormBlocks, (int)blocks1d(l0.nslot));
  if (o.mg_fixed > 0) {
    for (int c = 0; c < o.mg_fixed; ++c) {
      vcycle<T, TR>(p, 0, c == 0, nullptr);
      k_mg_count<<<1, 1, 0, p->stream>>>(p->ctrl);
    }
    return BLP_OK;
  }
  const int *gate = &p->ctrl->gate;
  k_mg_norm<T, TR><<<nblk, 256, 0, p->stream>>>(l0.view(TR), p->ctrl, 0, p->mg_partials);
  const int first = std::min(o.mg_maxcyc, 5);
  int enq = 0;
  for (; enq < first; ++enq) {
    vcycle<T, TR>(p, 0, enq == 0, gate);
    k_mg_norm<T, TR><<<nblk, 256, 0, p->stream>>>(l0.view(TR), p->ctrl, 1, p->mg_partials);
  }
  while (enq < o.mg_maxcyc) {
    HIP_TRY(hipMemcpyAsync(p->ctrl_h, p->ctrl, sizeof(MgCtrl), hipMemcpyDeviceToHost, p->stream));
    HIP_TRY(hipStreamSynchronize(p->stream));
    if (p->ctrl_h->gate) break;
    vcycle<T, TR>(p, 0, false, gate);
    k_mg_norm<T, TR><<<nblk, 256, 0, p->stream>>>(l0.view(TR), p->ctrl, 1, p->mg_partials);
    ++enq;
  }
  return BLP_OK;
}

// z = M^{-1} (dh .* v) (forward) or M^{-T} (dh .* v) (transposed); dh may
// be null (unscaled input).  All of z is written.
template <typename T, bool TR>
int prec_apply(blp_problem *p, const T *v, const T *dh, T *z) {
  std::vector<LevelDev<T>> &L = levels<T>(p);
  const Grid<T> g = fine_grid<T>(p);
  const int h = p->h, n1 = p->n1;
  const T rtol = (T)p->popts.mg_rtol;
  if (!TR) {
    interior_solve<T, false>(p, v, dh, z);
    launch_lines<T, false>(p, v, dh, z);
    k_corner_rhs<T, false><<<grid2d(h, h), 256, 0, p->stream>>>(g, h, n1, v, dh, z, L[0].b,
                                                                 p->ctrl, p->popts.mg_maxcyc, rtol);
    BLP_TRY((corner_solve<T, false>(p)));
    k_corner_copy<T, false><<<grid2d(h, h), 256, 0, p->stream>>>(h, n1, L[0].z, z);
  } else {
    k_corner_rhs<T, true><<<grid2d(h, h), 256, 0, p->stream>>>(g, h, n1, v, dh, z, L[0].b,
                                                                p->ctrl, p->popts.mg_maxcyc, rtol);
    BLP_TRY((corner_solve<T, true>(p)));
    k_corner_copy<T, true><<<grid2d(h, h), 256, 0, p->stream>>>(h, n1, L[0].z, z);
    launch_lines<T, true>(p, v, dh, z);
    interior_solve<T, true>(p, v, dh, z);
  }
  HIP_TRY(hipGetLastError());
  return BLP_OK;
}

template <typename T>
int prec_apply_dir(blp_problem *p, bool tr, const T *v, const T *dh, T *z) {
  return tr ? prec_apply<T, true>(p, v, dh, z) : prec_apply<T, false>(p, v, dh, z);
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
  // skewed storage: zero-filled so that padding slots always hold finite values
  BLP_TRY(zalloc(p, &d.ic[0], d.nslot));
  BLP_TRY(zalloc(p, &d.ic[1], d.nslot));
  BLP_TRY(zalloc(p, &d.z, d.nslot));
  BLP_TRY(zalloc(p, &d.b, d.nslot));
  BLP_TRY(zalloc(p, &d.t, d.nslot));
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
  BLP_TRY(zalloc(p, &f.bI, f.nslotI));
  BLP_TRY(zalloc(p, &f.zI, f.nslotI));
  const SkewT<T, false> skf{h + 1, n1, h + 1, n1};
  const SkewT<T, true> skt{h + 1, n1, h + 1, n1};
  k_diag_skew<T, false><<<blocks1d(f.nslotI), 256, 0, p->stream>>>(p->grid64(), skf, f.icI[0], f.nslotI);
  k_diag_skew<T, true><<<blocks1d(f.nslotI), 256, 0, p->stream>>>(p->grid64(), skt, f.icI[1], f.nslotI);
  for (int r = 0; r < 2; ++r) {
    BLP_TRY(zalloc(p, &f.bL[r], (size_t)m * line_stride(h)));
    BLP_TRY(zalloc(p, &f.zL[r], (size_t)m * line_stride(h)));
  }
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
    while (LH.back().n % 2 == 0 && LH.back().n > 2) {
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
  if (!p->ctrl) {
    BLP_TRY(p->alloc(&p->ctrl, 1));
    HIP_TRY(hipMemsetAsync(p->ctrl, 0, sizeof(MgCtrl), p->stream));
    BLP_TRY(p->alloc(&p->mg_partials, kMgNormBlocks));
  }
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(p->stream));
  return BLP_OK;
}

// ------------------------------------------------------------------------ //
// FGMRES driver                                                             //
// ------------------------------------------------------------------------ //

int ensure_workspace(blp_problem *p, int m, int prec) {
  if (p->ws_m >= m && p->ws_prec == prec) return BLP_OK;
  HIP_TRY(hipStreamSynchronize(p->stream));
  for (void *q : p->ws_allocs) (void)hipFree(q);
  p->ws_allocs.clear();
  p->ws_bytes = 0;
  const size_t n = p->n;
  const size_t es = prec == BLP_MIXED ? sizeof(float) : sizeof(double);
  char *V = nullptr, *Z = nullptr;
  BLP_TRY(p->alloc(&V, (size_t)(m + 1) * n * es, true));
  BLP_TRY(p->alloc(&Z, (size_t)m * n * es, true));
  p->V = V;
  p->Z = Z;
  BLP_TRY(p->alloc(&p->w, n, true));
  BLP_TRY(p->alloc(&p->ks, (size_t)(m + 1) * m + 2 * m + 3 * (m + 1) + m, true));
  const size_t nblk = (n + KCHUNK - 1) / KCHUNK;
  const size_t nstencil = (size_t)((p->n1 + 255) / 256) * ((p->n1 + 15) / 16);
  p->partials_len = std::max(nblk * (size_t)(m + 2), std::max(nstencil, (size_t)1024));
  BLP_TRY(p->alloc(&p->partials, p->partials_len, true));
  BLP_TRY(p->alloc(&p->tmp32a, n, true));
  BLP_TRY(p->alloc(&p->tmp32b, n, true));
  p->ws_m = m;
  p->ws_prec = prec;
  return BLP_OK;
}

constexpr int kRows = 16;  // rows per block of the stencil kernels

template <bool TR, bool SCALE>
void launch_residual(blp_problem *p, const double *F, const double *u, double *r) {
  KScope ks(p, KC_SPMV, (double)p->n * 3 * sizeof(double));
  dim3 gr((p->n1 + 255) / 256, (p->n1 + kRows - 1) / kRows);
  k_stencil<double, double, TR, SCALE, true><<<gr, 256, 0, p->stream>>>(p->grid64(), u, r, F, kRows,
                                                                         p->partials, p->st);
}

template <typename TX, bool TR, bool SCALE>
void launch_spmv(blp_problem *p, const TX *x, double *y) {
  KScope ks(p, KC_SPMV, (double)p->n * (sizeof(TX) + sizeof(double)));
  dim3 gr((p->n1 + 255) / 256, (p->n1 + kRows - 1) / kRows);
  k_stencil<TX, double, TR, SCALE, false><<<gr, 256, 0, p->stream>>>(p->grid64(), x, y, nullptr,
                                                                      kRows, nullptr, nullptr);
}

int read_status(blp_problem *p) {
  HIP_TRY(hipMemcpyAsync(p->st_h, p->st, sizeof(KrylovStatus), hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipMemcpyAsync(p->ctrl_h, p->ctrl, sizeof(MgCtrl), hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  return BLP_OK;
}

struct CycleStats {
  long total = 0;
  int mn = 1 << 30, mx = 0, applies = 0;
  void add(int c) {
    total += c;
    mn = std::min(mn, c);
    mx = std::max(mx, c);
    ++applies;
  }
};

// Right-preconditioned FGMRES(m) from u = 0 (Saad).  In scaled mode the
// Krylov space is that of D^{-1/2} A D^{-1/2}; the preconditioned vectors Z
// are kept in the unscaled variables, so u += Z y needs no rescaling.
// TV = double: FP64 throughout.  TV = float (mixed): V, Z and the
// preconditioner in FP32, SpMV arithmetic, Hessenberg/Givens, u and the
// restart-boundary true residuals in FP64; each restart cycle reduces the
// residual by at most inner_rtol before an FP64 residual is taken.
template <typename TV, bool TR, bool SCALE>
int fgmres(blp_problem *p, const double *F, double *u, const blp_solve_opts *o,
           blp_solve_info *info, double *hist) {
  const size_t n = p->n;
  const int m = o->restart;
  const double inner_rtol = std::is_same<TV, float>::value ? 1e-4 : 0.0;
  TV *V = (TV *)p->V, *Z = (TV *)p->Z;
  FineDev<TV> &f = fine<TV>(p);
  const TV *dh = SCALE ? f.dh : nullptr;
  KOffsets ko{m};
  CycleStats cs;
  auto t0 = std::chrono::steady_clock::now();

  k_norm<SCALE><<<256, 256, 0, p->stream>>>(p->grid64(), F, p->partials, p->st);
  BLP_TRY(read_status(p));
  const double nF = p->st_h->beta;
  if (!std::isfinite(nF)) return BLP_E_NUMERIC;
  const double target = o->absolute ? o->tol : o->tol * nF;
  HIP_TRY(hipMemsetAsync(u, 0, n * sizeof(double), p->stream));
  launch_residual<TR, SCALE>(p, F, u, p->w);
  BLP_TRY(read_status(p));
  double beta = p->st_h->beta;
  if (hist) hist[0] = beta;
  int it = 0, restarts = 0;
  bool conv = beta <= target;
  while (!conv && it < o->maxit) {
    if (!std::isfinite(beta)) return BLP_E_NUMERIC;
    k_normalize<TV><<<blocks1d(n), 256, 0, p->stream>>>(p->w, V, n, p->st, 1);
    k_krylov_init<<<1, 64, 0, p->stream>>>(p->ks, ko, p->st);
    const double cyc_target = std::max(target, inner_rtol * beta);
    int ncol = 0;
    for (int j = 0; j < m && it < o->maxit; ++j) {
      TV *vj = V + (size_t)j * n, *zj = Z + (size_t)j * n;
      if (o->precond) {
        BLP_TRY(prec_apply_dir<TV>(p, TR, vj, dh, zj));
      } else if (SCALE) {
        // identity preconditioner of the scaled system; Z keeps the unscaled
        // variables, z = v / sqrt(C)
        k_div<TV><<<blocks1d(n), 256, 0, p->stream>>>(vj, f.dh, zj, n);
      } else {
        HIP_TRY(hipMemcpyAsync(zj, vj, n * sizeof(TV), hipMemcpyDeviceToDevice, p->stream));
      }
      launch_spmv<TV, TR, SCALE>(p, zj, p->w);
      const unsigned nb = (unsigned)((n + KCHUNK - 1) / KCHUNK);
      // CGS2: four passes over the j+1 basis vectors plus w traffic
      KScope ks(p, KC_KRYLOV, (double)n * ((4.0 * (j + 1)) * sizeof(TV) + 6 * sizeof(double)));
      k_arnoldi_dot<TV><<<nb, 256, 0, p->stream>>>(V, n, j, p->w, n, p->partials, p->ks, ko, p->st);
      k_arnoldi_update<TV, false><<<nb, 256, 0, p->stream>>>(V, n, j, p->w, n, p->partials, p->ks, ko,
                                                              p->st);
      k_arnoldi_update<TV, true><<<nb, 256, 0, p->stream>>>(V, n, j, p->w, n, p->partials, p->ks, ko,
                                                             p->st);
      ks.end();
      BLP_TRY(read_status(p));
      ++it;
      ncol = j + 1;
      if (o->precond) cs.add(p->ctrl_h->cycles);
      const double est = p->st_h->est;
      if (hist && !std::is_same<TV, float>::value) hist[it] = est;
      if (!std::isfinite(est)) return BLP_E_NUMERIC;
      const bool happy = p->st_h->happy != 0;
      if (!happy && j + 1 < m)
        k_normalize<TV><<<blocks1d(n), 256, 0, p->stream>>>(p->w, V + (size_t)(j + 1) * n, n, p->st, 0);
      if (est <= cyc_target || happy) break;
    }
    k_update_solution<TV><<<blocks1d(n), 256, 0, p->stream>>>(Z, n, ncol, p->ks, ko, u, n);
    launch_residual<TR, SCALE>(p, F, u, p->w);
    BLP_TRY(read_status(p));
    beta = p->st_h->beta;
    ++restarts;
    if (hist && std::is_same<TV, float>::value) hist[std::min(it, o->maxit)] = beta;
    if (beta <= target) conv = true;
  }
  HIP_TRY(hipGetLastError());
  auto t1 = std::chrono::steady_clock::now();
  if (info) {
    info->iterations = it;
    info->restarts = restarts;
    info->converged = conv ? 1 : 0;
    info->res = beta;
    info->norm_F = nF;
    info->mg_cycles_total = cs.total;
    info->mg_cycles_min = cs.applies ? cs.mn : 0;
    info->mg_cycles_max = cs.mx;
    info->solve_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
  }
  if (!std::isfinite(beta)) return BLP_E_NUMERIC;
  return conv ? BLP_OK : BLP_W_NOCONV;
}

int solve_common(blp_problem *p, bool tr, int nrhs, const double *F, double *U,
                 const blp_solve_opts *o, blp_solve_info *info, double *hist) {
  if (!p || !o || !F || !U || nrhs < 1) return BLP_E_INVAL;
  if (o->precond && !p->prec_ready) return BLP_E_STATE;
  if (!(o->tol > 0) || o->restart < 1 || o->restart > 60 || o->maxit < 1) return BLP_E_INVAL;
  if (o->precision != BLP_FP64 && o->precision != BLP_MIXED) return BLP_E_INVAL;
  BLP_TRY(ensure_workspace(p, o->restart, o->precision));
  int worst = BLP_OK;
  for (int k = 0; k < nrhs; ++k) {
    const double *Fk = F + (size_t)k * p->n;
    double *Uk = U + (size_t)k * p->n;
    blp_solve_info *ik = info ? info + k : nullptr;
    double *hk = hist ? hist + (size_t)k * (o->maxit + 1) : nullptr;
    int rc;
    const bool mixed = o->precision == BLP_MIXED, sc = o->scaled != 0;
#define BLP_DISPATCH(TV, TRB, SCB) rc = fgmres<TV, TRB, SCB>(p, Fk, Uk, o, ik, hk)
    if (mixed) {
      if (tr) { if (sc) BLP_DISPATCH(float, true, true); else BLP_DISPATCH(float, true, false); }
      else { if (sc) BLP_DISPATCH(float, false, true); else BLP_DISPATCH(float, false, false); }
    } else {
      if (tr) { if (sc) BLP_DISPATCH(double, true, true); else BLP_DISPATCH(double, true, false); }
      else { if (sc) BLP_DISPATCH(double, false, true); else BLP_DISPATCH(double, false, false); }
    }
#undef BLP_DISPATCH
    if (rc < 0) return rc;
    if (rc > worst) worst = rc;
  }
  return worst;
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

int blp_mesh(int N, double eps, double sigma, double clow, double *nodes, double *tau) {
  if (N < 4 || N % 2 || !(eps > 0 && eps <= 1) || !(sigma > 0) || !(clow > 0) || !nodes)
    return BLP_E_INVAL;
  const double t = shishkin_tau(N, eps, sigma, clow);
  std::vector<double> x, w;
  axis_mesh(N, t, x, w);
  std::memcpy(nodes, x.data(), sizeof(double) * (N + 1));
  if (tau) *tau = t;
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
  const double sigma = mesh ? mesh->sigma : 2.0;
  const double clx = mesh ? mesh->clow_x : 1.0, cly = mesh ? mesh->clow_y : 1.0;
  if (!(sigma > 0) || !(clx > 0) || !(cly > 0)) return BLP_E_INVAL;

  blp_problem *p = new (std::nothrow) blp_problem();
  if (!p) return BLP_E_NOMEM;
  p->N = N;
  p->n1 = N - 1;
  p->h = N / 2;
  p->n = (size_t)(N - 1) * (N - 1);
  p->eps = eps;
  p->stream = (hipStream_t)stream;
  axis_mesh(N, shishkin_tau(N, eps, sigma, clx), p->xn, p->wx);
  axis_mesh(N, shishkin_tau(N, eps, sigma, cly), p->yn, p->wy);
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
  if ((rc = p->upload(&p->f64.W, p->fx.W)) || (rc = p->upload(&p->f64.E, p->fx.E)) ||
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
  if ((rc = p->alloc(&p->st, 1))) return fail(rc);
  if (hipMemsetAsync(p->st, 0, sizeof(KrylovStatus), p->stream) != hipSuccess) return fail(BLP_E_HIP);
  if (hipHostMalloc((void **)&p->st_h, sizeof(KrylovStatus), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void **)&p->ctrl_h, sizeof(MgCtrl), hipHostMallocDefault) != hipSuccess)
    return fail(BLP_E_NOMEM);
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
  blp_prec_opts po = o ? *o : blp_prec_opts{0, 1e-3, 20};
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

int blp_apply(blp_problem *p, int op, const double *x, double *y, int *cycles) {
  if (!p || !x || !y) return BLP_E_INVAL;
  if (op == BLP_OP_A || op == BLP_OP_AT) {
    if (op == BLP_OP_A) launch_spmv<double, false, false>(p, x, y);
    else launch_spmv<double, true, false>(p, x, y);
  } else if (op == BLP_OP_MINV || op == BLP_OP_MINVT || op == BLP_OP_MINV32) {
    if (!p->prec_ready) return BLP_E_STATE;
    if (op == BLP_OP_MINV32) {
      BLP_TRY(ensure_workspace(p, std::max(p->ws_m, 1), p->ws_prec < 0 ? BLP_FP64 : p->ws_prec));
      k_convert<double, float><<<blocks1d(p->n), 256, 0, p->stream>>>(x, p->tmp32a, p->n);
      BLP_TRY((prec_apply<float, false>(p, p->tmp32a, nullptr, p->tmp32b)));
      k_convert<float, double><<<blocks1d(p->n), 256, 0, p->stream>>>(p->tmp32b, y, p->n);
    } else {
      BLP_TRY(prec_apply_dir<double>(p, op == BLP_OP_MINVT, x, nullptr, y));
    }
  } else {
    return BLP_E_INVAL;
  }
  HIP_TRY(hipGetLastError());
  if (cycles) {
    *cycles = 0;
    if (p->ctrl && op >= BLP_OP_MINV) {
      HIP_TRY(hipMemcpyAsync(p->ctrl_h, p->ctrl, sizeof(MgCtrl), hipMemcpyDeviceToHost, p->stream));
      HIP_TRY(hipStreamSynchronize(p->stream));
      *cycles = p->ctrl_h->cycles;
    }
  }
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

static int project(blp_problem *p, int K, int L, int kind, const double *w, double *g) {
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
    k_project_rows<<<n1, 256, 0, p->stream>>>(N, K, w, tx, t);
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
  return project(p, K, L, 0, w, g);
}

int blp_bilinear_project(blp_problem *p, int m, const double *w, double *G) {
  if (!p || m < 2 || !w || !G) return BLP_E_INVAL;
  return project(p, m, m, 1, w, G);
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
  if (enable) {
    HIP_TRY(hipStreamSynchronize(p->stream));
    p->recs.clear();
    p->ev_used = 0;
    p->timing = true;
    return BLP_OK;
  }
  HIP_TRY(hipStreamSynchronize(p->stream));
  p->timing = false;
  double sm[BLP_NCLASS] = {0}, sb[BLP_NCLASS] = {0};
  long long sl[BLP_NCLASS] = {0};
  for (const auto &r : p->recs) {
    float t = 0.f;
    HIP_TRY(hipEventElapsedTime(&t, r.a, r.b));
    sm[r.cls] += t;
    sb[r.cls] += r.bytes;
    sl[r.cls] += 1;
  }
  for (int k = 0; k < BLP_NCLASS; ++k) {
    if (ms) ms[k] = sm[k];
    if (launches) launches[k] = sl[k];
    if (bytes) bytes[k] = sb[k];
  }
  p->recs.clear();
  p->ev_used = 0;
  return BLP_OK;
}

long long blp_footprint(const blp_problem *p) { return p ? p->bytes + p->ws_bytes : 0; }

void blp_destroy(blp_problem *p) {
  if (!p) return;
  (void)hipStreamSynchronize(p->stream);
  for (void *q : p->allocs) (void)hipFree(q);
  for (void *q : p->ws_allocs) (void)hipFree(q);
  for (hipEvent_t e : p->ev_pool) (void)hipEventDestroy(e);
  if (p->st_h) (void)hipHostFree(p->st_h);
  if (p->ctrl_h) (void)hipHostFree(p->ctrl_h);
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
    default: return "unknown error";
  }
}

}  // extern "C"
