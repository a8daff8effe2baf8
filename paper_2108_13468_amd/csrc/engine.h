// Execution engine: systems, launch plans and the batched FGMRES driver.
//
// A *system* is one right-hand side being solved with one problem's
// operator and preconditioner data; it owns its work vectors (region
// buffers, corner-level vectors, Krylov basis).  A *batch* is a set of
// systems solved together: every kernel launch covers all systems of one
// mesh size (a class) at once, each workgroup reading its system's argument
// record from a device array (a launch plan, built once).  Vectors that move
// with the Krylov step are addressed as base + j * ld with j in device
// memory, so one launch sequence -- which can be captured in a HIP graph --
// serves every step.  Systems leave a restart cycle (converged, happy
// breakdown, cycle length) through a per-system gate that every kernel
// checks; a new cycle starts for all active systems together.  A single
// solve is a batch of one.
//
// Included once, from blp.hip, inside its anonymous namespace.
#pragma once

// ------------------------------------------------------------------------ //
// Device memory ownership                                                   //
// ------------------------------------------------------------------------ //

struct Alloc {
  std::vector<void *> ptrs;
  long long bytes = 0;
  template <typename T>
  int get(T **p, size_t count, hipStream_t s = nullptr, bool zero = false) {
    void *q = nullptr;
    if (hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess) return BLP_E_NOMEM;
    ptrs.push_back(q);
    bytes += (long long)(count * sizeof(T));
    *p = (T *)q;
    if (zero && hipMemsetAsync(q, 0, std::max<size_t>(count, 1) * sizeof(T), s) != hipSuccess)
      return BLP_E_HIP;
    return BLP_OK;
  }
  template <typename T>
  int put(T **p, const T *host, size_t count, hipStream_t s) {
    BLP_TRY(get(p, count));
    if (hipMemcpyAsync(*p, host, count * sizeof(T), hipMemcpyHostToDevice, s) != hipSuccess)
      return BLP_E_HIP;
    return BLP_OK;
  }
  void release() {
    for (void *q : ptrs) (void)hipFree(q);
    ptrs.clear();
    bytes = 0;
  }
  ~Alloc() { release(); }
};

// ------------------------------------------------------------------------ //
// Systems                                                                   //
// ------------------------------------------------------------------------ //

template <typename T>
struct SysWork {
  T *bI = nullptr, *zI = nullptr;                    // interior region, skewed
  T *bL[2] = {nullptr, nullptr}, *zL[2] = {nullptr, nullptr};  // edge lines [Y, X]
  std::vector<T *> z, b, t;                          // corner levels, skewed
  std::vector<T *> pz, pb, pt;  // parabolic-case corner levels 1.. (skewed; level 0 is z, b, t [0])
};

struct System {
  blp_problem *p = nullptr;  // operator and preconditioner data (not owned)
  SysWork<double> w64;
  SysWork<float> w32;
  MgCtrl *ctrl = nullptr;        // device, in the batch's array
  KrylovStatus *st = nullptr;    // device, in the batch's array
  int *gate = nullptr;           // device, in the batch's array
  double *mg_partials = nullptr;
  // Krylov workspace of the current solve (one per precision, kept, so that
  // alternating precisions neither reallocates nor invalidates plans)
  int ws_m = 0, ws_prec = -1;
  void *V = nullptr, *Z = nullptr;
  double *w = nullptr, *ks = nullptr, *partials = nullptr;
  struct KrylovWS {
    int m = 0;
    void *V = nullptr, *Z = nullptr;
    double *w = nullptr, *ks = nullptr, *partials = nullptr;
    Alloc mem;
  } kws[2];  // [0] FP64, [1] mixed
  Alloc mem;
  long long krylov_bytes() const { return kws[0].mem.bytes + kws[1].mem.bytes; }
};

template <typename T>
SysWork<T> &work(System &s);
template <>
SysWork<double> &work<double>(System &s) { return s.w64; }
template <>
SysWork<float> &work<float>(System &s) { return s.w32; }

template <typename T>
int alloc_work(System &s, hipStream_t st, SysWork<T> &w, const FineDev<T> &f,
               const std::vector<LevelDev<T>> &L) {
  blp_problem *p = s.p;
  const int h = p->h, m = p->n1 - h, hp = line_stride(h);
  BLP_TRY(s.mem.get(&w.bI, f.nslotI, st, true));
  BLP_TRY(s.mem.get(&w.zI, f.nslotI, st, true));
  for (int r = 0; r < 2; ++r) {
    BLP_TRY(s.mem.get(&w.bL[r], (size_t)m * hp, st, true));
    BLP_TRY(s.mem.get(&w.zL[r], (size_t)m * hp, st, true));
  }
  w.z.assign(L.size(), nullptr);
  w.b.assign(L.size(), nullptr);
  w.t.assign(L.size(), nullptr);
  for (size_t l = 0; l < L.size(); ++l) {
    // zero-filled: padding slots of right-hand sides must hold zero
    BLP_TRY(s.mem.get(&w.z[l], L[l].nslot, st, true));
    BLP_TRY(s.mem.get(&w.b[l], L[l].nslot, st, true));
    BLP_TRY(s.mem.get(&w.t[l], L[l].nslot, st, true));
  }
  const std::vector<ParLevelDev<T>> &PL = par_levels<T>(p);
  w.pz.assign(PL.size(), nullptr);
  w.pb.assign(PL.size(), nullptr);
  w.pt.assign(PL.size(), nullptr);
  for (size_t l = 1; l < PL.size(); ++l) {
    // zero-filled: padding words of right-hand sides must hold zero
    const size_t n = PL[l].sk.nslot();
    BLP_TRY(s.mem.get(&w.pz[l], n, st, true));
    BLP_TRY(s.mem.get(&w.pb[l], n, st, true));
    BLP_TRY(s.mem.get(&w.pt[l], n, st, true));
  }
  return BLP_OK;
}

// Krylov workspace of a system for restart length m and precision prec.
int ensure_krylov(System &s, hipStream_t st, int m, int prec) {
  System::KrylovWS &k = s.kws[prec == BLP_MIXED ? 1 : 0];
  if (k.m < m) {
    // grows only: plans built on the old buffers notice the new V (see
    // get_solve_plan) and are rebuilt
    HIP_TRY(hipStreamSynchronize(st));
    k.mem.release();
    k.m = 0;
    const size_t n = s.p->n;
    const size_t es = prec == BLP_MIXED ? sizeof(float) : sizeof(double);
    char *V = nullptr, *Z = nullptr;
    BLP_TRY(k.mem.get(&V, (size_t)(m + 1) * n * es));
    BLP_TRY(k.mem.get(&Z, (size_t)m * n * es));
    k.V = V;
    k.Z = Z;
    BLP_TRY(k.mem.get(&k.w, n));
    BLP_TRY(k.mem.get(&k.ks, (size_t)(m + 1) * m + 2 * m + 3 * (m + 1) + m, st, true));
    const size_t nblk = (n + KCHUNK - 1) / KCHUNK;
    // stencil partials: one per block at the smallest strip height tried (8 rows)
    const size_t nstencil = (size_t)((s.p->n1 + 255) / 256) * ((s.p->n1 + 7) / 8);
    BLP_TRY(k.mem.get(&k.partials, std::max(nblk * (size_t)(m + 2), std::max(nstencil, (size_t)256))));
    k.m = m;
  }
  s.V = k.V;
  s.Z = k.Z;
  s.w = k.w;
  s.ks = k.ks;
  s.partials = k.partials;
  s.ws_m = k.m;
  s.ws_prec = prec;
  return BLP_OK;
}

// ------------------------------------------------------------------------ //
// Launch plans: device arrays of per-system argument records                //
// ------------------------------------------------------------------------ //

// Where the preconditioner of one system reads its input and writes its
// output: v + j ldv and z + j ldz (ld = 0: fixed vectors).
struct IOSpec {
  const void *v;
  long long ldv;
  void *z;
  long long ldz;
};

template <typename T, bool TR>
struct PrecPlan {
  int S = 0, N = 0, h = 0, n1 = 0, hp = 0, nbI = 0;
  size_t nslotI = 0;
  std::vector<int> ln;        // level sizes
  std::vector<size_t> lslot;  // level skewed sizes
  bool scaled = false;
  SkewIO<T, TR> *ioI = nullptr;
  SweepArgs<T> *swI = nullptr;
  LineIO<T> *ioL = nullptr;
  LineArgs<T> *lnA = nullptr;
  CornerIO<T> *cr = nullptr;
  // parabolic-case corner (x-semicoarsening): level columns and records
  bool par = false;
  std::vector<int> pn;
  std::vector<ParSkew> psk;
  std::vector<ParArgs<T> *> pa;
  std::vector<MgArgs<T> *> mg;
  std::vector<SweepArgs<T> *> swb, swt;  // per level: sweep from b, from t
  // kernel variants (autotuner; 0 = default)
  int varI = 0, varLines = 0;
  std::vector<int> varL;
  // fused cycle below level lc (at most kLdsN<T> nodes per axis, held in
  // coarse_lds bytes of LDS); -1: none
  int lc = -1;
  size_t coarse_lds = 0;
  CoarseArgs<T> *coarse = nullptr;
  Alloc mem;
};

// The fused coarse cycle's dynamic LDS limit is an attribute of the kernel,
// shared by every plan and host thread: it is only ever raised, under a lock.
template <typename T, bool TR>
int raise_coarse_lds(size_t bytes) {
  static std::mutex mu;
  static size_t set = 0;
  std::lock_guard<std::mutex> lock(mu);
  if (bytes <= set) return BLP_OK;
  HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_mg_coarse<T, TR>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  set = bytes;
  return BLP_OK;
}

template <typename T, bool TR>
int build_prec_plan(hipStream_t st, const std::vector<System *> &sys, const std::vector<IOSpec> &io,
                    bool scaled, PrecPlan<T, TR> &P) {
  const int S = (int)sys.size();
  blp_problem *p0 = sys[0]->p;
  P.S = S;
  P.N = p0->N;
  P.h = p0->h;
  P.n1 = p0->n1;
  P.hp = line_stride(P.h);
  P.scaled = scaled;
  const std::vector<LevelDev<T>> &L0 = levels<T>(p0);
  const int nl = (int)L0.size();
  P.par = p0->ylayer == BLP_LAYER_PARABOLIC;
  // the parabolic corner cycle has no transposed form
  if (P.par && TR) return BLP_E_INVAL;
  for (System *y : sys)
    if ((y->p->ylayer == BLP_LAYER_PARABOLIC) != P.par) return BLP_E_INVAL;
  const std::vector<ParLevelDev<T>> &PL0 = par_levels<T>(p0);
  const int npl = (int)PL0.size();
  P.pn.resize(npl);
  P.psk.resize(npl);
  for (int l = 0; l < npl; ++l) {
    P.pn[l] = PL0[l].nx;
    P.psk[l] = PL0[l].sk;
  }
  std::vector<std::vector<ParArgs<T>>> pa(npl, std::vector<ParArgs<T>>(S));
  P.ln.resize(nl);
  P.lslot.resize(nl);
  for (int l = 0; l < nl; ++l) {
    P.ln[l] = L0[l].n;
    P.lslot[l] = L0[l].nslot;
  }
  P.nslotI = fine<T>(p0).nslotI;
  P.nbI = (P.n1 - P.h + 63) / 64;
  P.varL.assign(nl, 0);
  std::vector<SkewIO<T, TR>> ioI(S);
  std::vector<SweepArgs<T>> swI(S);
  std::vector<LineIO<T>> ioL(S);
  std::vector<LineArgs<T>> lnA(S);
  std::vector<CornerIO<T>> cr(S);
  std::vector<std::vector<MgArgs<T>>> mg(nl, std::vector<MgArgs<T>>(S));
  std::vector<std::vector<SweepArgs<T>>> swb(nl, std::vector<SweepArgs<T>>(S)), swt = swb;
  const int h = P.h, n1 = P.n1, hp = P.hp;
  // channels and launch counters of the split sweeps (interior, then one per
  // level: a level's two sweeps never run at the same time)
  std::vector<unsigned long long *> chan(nl + 1, nullptr);
  std::vector<int *> epoch(nl + 1, nullptr);
  for (int k = 0; k <= nl; ++k) {
    BLP_TRY(P.mem.get(&chan[k], (size_t)S * (kSweepMaxGroups - 1) * kChanStride<T>, st, true));
    BLP_TRY(P.mem.get(&epoch[k], (size_t)S * 2 * (kSweepMaxGroups - 1), st, true));
  }
  auto split = [&](SweepArgs<T> a, int k, int s) {
    a.chan = chan[k] + (size_t)s * (kSweepMaxGroups - 1) * kChanStride<T>;
    a.epoch = epoch[k] + 2 * (kSweepMaxGroups - 1) * s;
    return a;
  };
  for (int s = 0; s < S; ++s) {
    System &y = *sys[s];
    blp_problem *p = y.p;
    const FineDev<T> &f = fine<T>(p);
    const std::vector<LevelDev<T>> &L = levels<T>(p);
    SysWork<T> &w = work<T>(y);
    const Grid<T> g = fine_grid<T>(p);
    const T *v = (const T *)io[s].v;
    T *z = (T *)io[s].z;
    const T *dh = scaled ? f.dh : nullptr;
    ioI[s] = SkewIO<T, TR>{g, SkewT<T, TR>{h + 1, n1, h + 1, n1}, v, io[s].ldv, dh, z, io[s].ldz,
                           w.bI, w.zI, P.nslotI, y.gate};
    swI[s] = split(SweepArgs<T>{g, h + 1, n1, h + 1, n1, w.bI, f.icI[TR ? 1 : 0], w.zI, y.gate}, nl, s);
    ioL[s] = LineIO<T>{g, h, n1, hp, v, io[s].ldv, dh, z, io[s].ldz, {w.bL[0], w.bL[1]},
                       {w.zL[0], w.zL[1]}, y.gate};
    LineArgs<T> la;
    la.g = g;
    la.h = h;
    la.n1 = n1;
    la.hp = hp;
    const int base = TR ? 2 : 0;
    for (int r = 0; r < 2; ++r) {
      la.b[r] = w.bL[r];
      la.z[r] = w.zL[r];
      la.fd[r] = f.fac[base + r][0];
      la.fm[r] = f.fac[base + r][1];
      la.fw[r] = f.fac[base + r][2];
    }
    la.gate = y.gate;
    lnA[s] = la;
    // the corner right-hand side and result are level 0's skewed vectors in
    // both hierarchies
    cr[s] = CornerIO<T>{g, h, n1, v, io[s].ldv, dh, z, io[s].ldz, w.b[0], w.z[0], y.ctrl,
                        p->popts.mg_maxcyc, p->popts.mg_rtol, y.gate};
    if (P.par) {
      const std::vector<ParLevelDev<T>> &PL = par_levels<T>(p);
      for (int l = 0; l < npl; ++l) {
        const bool last = l + 1 == npl;
        ParArgs<T> r{};
        r.nx = PL[l].nx;
        r.ny = h;
        r.sk = PL[l].sk;
        r.skc = last ? ParSkew{} : PL[l + 1].sk;
        r.g = g;
        r.sx = PL[0].sx;
        r.sy = PL[0].sy;
        r.a = PL[l].sa;
        r.ic = PL[l].sic;
        r.sw = PL[l].ssw;
        r.wl = l ? PL[l].swl : PL[0].wl;
        r.wr = l ? PL[l].swr : PL[0].wr;
        r.z = l ? w.pz[l] : w.z[0];
        r.b = l ? w.pb[l] : w.b[0];
        r.t = l ? w.pt[l] : w.t[0];
        r.nxc = last ? 0 : PL[l + 1].nx;
        r.zc = last ? nullptr : w.pz[l + 1];
        r.bc = last ? nullptr : w.pb[l + 1];
        r.ctrl = y.ctrl;
        pa[l][s] = r;
      }
    }
    for (int l = 0; l < nl; ++l) {
      const MgLevel<T> lv = L[l].view(TR, w.z[l], w.b[l], w.t[l]);
      const MgLevel<T> cv =
          l + 1 < nl ? L[l + 1].view(TR, w.z[l + 1], w.b[l + 1], w.t[l + 1]) : MgLevel<T>{};
      mg[l][s] = MgArgs<T>{lv, cv, y.ctrl, y.mg_partials};
      const T *ic = L[l].ic[TR ? 1 : 0];
      swb[l][s] = split(SweepArgs<T>{lv.g, 1, L[l].n, 1, L[l].n, w.b[l], ic, w.z[l], &y.ctrl->gate}, l, s);
      swt[l][s] = split(SweepArgs<T>{lv.g, 1, L[l].n, 1, L[l].n, w.t[l], ic, w.z[l], &y.ctrl->gate}, l, s);
    }
  }
  // the coarse levels run as one fused cycle per system (two exponential
  // layers; the parabolic plan uses level 0 alone)
  P.lc = -1;
  for (int l = 0; l < (P.par ? 0 : nl); ++l)
    if (P.ln[l] <= kLdsN<T>) {
      if (nl - l <= kCoarseMax) P.lc = l;
      break;
    }
  if (P.lc >= 0) {
    bool nodal = false;
    for (int q = 0; q < S; ++q) nodal = nodal || mg[P.lc][q].L.g.r != nullptr;
    P.coarse_lds = coarse_lds_bytes<T>(P.ln[P.lc], nl - P.lc, nodal);
    BLP_TRY((raise_coarse_lds<T, TR>(P.coarse_lds)));
    // constant LDS images, one per system (zero padding rows)
    const size_t iw = (size_t)lds_image_words<T>(P.ln[P.lc], nl - P.lc, nodal);
    T *img = nullptr;
    BLP_TRY(P.mem.get(&img, iw * S, st, true));
    std::vector<CoarseArgs<T>> ca(S);
    for (int q = 0; q < S; ++q) {
      ca[q].nlev = nl - P.lc;
      for (int l = P.lc; l < nl; ++l) ca[q].L[l - P.lc] = mg[l][q].L;
      ca[q].ctrl = mg[0][q].ctrl;
      ca[q].image = img + iw * q;
    }
    BLP_TRY(P.mem.put(&P.coarse, ca.data(), S, st));
    k_coarse_image<T, TR><<<S, 256, 0, st>>>(P.coarse);
    HIP_TRY(hipGetLastError());
  }
  BLP_TRY(P.mem.put(&P.ioI, ioI.data(), S, st));
  BLP_TRY(P.mem.put(&P.swI, swI.data(), S, st));
  BLP_TRY(P.mem.put(&P.ioL, ioL.data(), S, st));
  BLP_TRY(P.mem.put(&P.lnA, lnA.data(), S, st));
  BLP_TRY(P.mem.put(&P.cr, cr.data(), S, st));
  P.pa.assign(npl, nullptr);
  for (int l = 0; l < npl; ++l) BLP_TRY(P.mem.put(&P.pa[l], pa[l].data(), S, st));
  P.mg.assign(nl, nullptr);
  P.swb.assign(nl, nullptr);
  P.swt.assign(nl, nullptr);
  for (int l = 0; l < nl; ++l) {
    BLP_TRY(P.mem.put(&P.mg[l], mg[l].data(), S, st));
    BLP_TRY(P.mem.put(&P.swb[l], swb[l].data(), S, st));
    BLP_TRY(P.mem.put(&P.swt[l], swt[l].data(), S, st));
  }
  HIP_TRY(hipStreamSynchronize(st));  // host staging vectors go out of scope
  return BLP_OK;
}

// Kernel variants the autotuner chooses between (all compute the same
// arithmetic in the same order per lane; they differ in scheduling only).
// Sweep: superstep K = 4 or 2 chunks of 16 bytes per lane, D supersteps of
// loads in flight (D + 1 register buffers of 2K words); more than 8 waves
// leave registers for D = 1 only.
// Sweep variants: G workgroups per system (G = 2 or 4 splits the bands over
// as many compute units, joined by channels in memory), K steps per
// superstep, D supersteps of loads in flight.  Above four bands the default
// takes two compute units in FP32 and four in FP64; the alternative split is
// variant 1.
inline int sweep_variants(int ncols) {
  const int nb = (ncols + 63) / 64;
  return nb == 1 ? 4 : (nb <= 4 ? 6 : (nb <= 8 ? 7 : 6));
}

template <typename T, bool TR, int K, int D, int G>
void sweep_launch_k(const Ctx &c, int S, int nb, const SweepArgs<T> *A) {
  k_sweep<T, TR, K, D, G><<<dim3(S * G), dim3(64 * ((nb + G - 1) / G)), 0, c.stream>>>(A);
}

template <typename T, bool TR>
void sweep_launch(const Ctx &c, int S, int ncols, const SweepArgs<T> *A, int var = 0) {
  const int nb = (ncols + 63) / 64;
  constexpr int P = kChunk<T>;
  if (nb == 1) {
    switch (var) {
      case 1: sweep_launch_k<T, TR, 4 * P, 2, 1>(c, S, nb, A); break;
      case 2: sweep_launch_k<T, TR, 2 * P, 4, 1>(c, S, nb, A); break;
      case 3: sweep_launch_k<T, TR, 2 * P, 2, 1>(c, S, nb, A); break;
      default: sweep_launch_k<T, TR, 4 * P, 4, 1>(c, S, nb, A); break;
    }
  } else if (nb <= 4) {
    switch (var) {
      case 1: sweep_launch_k<T, TR, 4 * P, 2, 1>(c, S, nb, A); break;
      case 2: sweep_launch_k<T, TR, 2 * P, 4, 1>(c, S, nb, A); break;
      case 3: sweep_launch_k<T, TR, 2 * P, 2, 1>(c, S, nb, A); break;
      case 4: sweep_launch_k<T, TR, 4 * P, 4, 2>(c, S, nb, A); break;
      case 5: sweep_launch_k<T, TR, 4 * P, 2, 2>(c, S, nb, A); break;
      default: sweep_launch_k<T, TR, 4 * P, 4, 1>(c, S, nb, A); break;
    }
  } else if (nb <= 8) {
    switch (var) {
      case 1: sweep_launch_k<T, TR, 4 * P, 2, 6 - (int)sizeof(T) / 2>(c, S, nb, A); break;
      case 2: sweep_launch_k<T, TR, 4 * P, 4, 1>(c, S, nb, A); break;
      case 3: sweep_launch_k<T, TR, 4 * P, 2, 1>(c, S, nb, A); break;
      case 4: sweep_launch_k<T, TR, 2 * P, 4, 1>(c, S, nb, A); break;
      case 5: sweep_launch_k<T, TR, 4 * P, 4, 2>(c, S, nb, A); break;
      case 6: sweep_launch_k<T, TR, 4 * P, 4, 4>(c, S, nb, A); break;
      default:
        // two loads in flight; FP32 on two compute units, FP64 (twice the
        // bytes per node) on four
        if (sizeof(T) == 8) sweep_launch_k<T, TR, 4 * P, 2, 4>(c, S, nb, A);
        else sweep_launch_k<T, TR, 4 * P, 2, 2>(c, S, nb, A);
        break;
    }
  } else {
    switch (var) {
      case 1: sweep_launch_k<T, TR, 4 * P, 1, 1>(c, S, nb, A); break;
      case 2: sweep_launch_k<T, TR, 2 * P, 1, 1>(c, S, nb, A); break;
      case 3: sweep_launch_k<T, TR, 4 * P, 2, 2>(c, S, nb, A); break;
      case 4: sweep_launch_k<T, TR, 4 * P, 4, 4>(c, S, nb, A); break;
      case 5: sweep_launch_k<T, TR, 4 * P, 4, 2>(c, S, nb, A); break;
      default:
        // four compute units: at most four bands, one wave per SIMD, each
        sweep_launch_k<T, TR, 4 * P, 2, 4>(c, S, nb, A);
        break;
    }
  }
}

template <typename T, bool TR, int EP, int W>
void lines_launch_k(const Ctx &c, int S, int hp, const LineArgs<T> *A) {
  // D lines of operands in flight: 4 EP words per line and thread (two
  // buffers of them fill the registers at 16 FP32 or 8 FP64 words), within
  // the 63 outstanding memory operations a wave can track
  constexpr int B = EP * (int)sizeof(T);  // bytes per operand and thread
  constexpr int D = B >= 128 ? 1 : (B >= 64 ? 2 : (B >= 16 ? 4 : 6));
  if (hp == 64 * W * EP) k_lines<T, TR, EP, W, D, true><<<2 * S, 64 * W, 0, c.stream>>>(A);
  else k_lines<T, TR, EP, W, D, false><<<2 * S, 64 * W, 0, c.stream>>>(A);
}

// Line solves: threads hold EP contiguous nodes, W waves per region (EP x
// 64 W >= hp).  A line is a chain of dependent scans, so its latency sets the
// pace: one wave (no workgroup barriers between the scan phases) is the
// default, except FP64 lines longer than 512 nodes, whose 16 nodes per
// thread would not fit the registers (four waves of four nodes measured
// 30% faster there); the other variants remain for the autotuner.
inline int lines_variants(int hp) {
  return hp <= 64 ? 1 : (hp <= 128 ? 2 : (hp <= 256 ? 3 : 4));
}

template <typename T, bool TR>
void lines_launch(const Ctx &c, int S, int hp, const LineArgs<T> *A, int var = 0) {
  if (hp <= 64) {
    lines_launch_k<T, TR, 1, 1>(c, S, hp, A);
  } else if (hp <= 128) {
    if (var == 1) lines_launch_k<T, TR, 1, 2>(c, S, hp, A);
    else lines_launch_k<T, TR, 2, 1>(c, S, hp, A);
  } else if (hp <= 256) {
    if (var == 1) lines_launch_k<T, TR, 2, 2>(c, S, hp, A);
    else if (var == 2) lines_launch_k<T, TR, 1, 4>(c, S, hp, A);
    else lines_launch_k<T, TR, 4, 1>(c, S, hp, A);
  } else if (hp <= 512) {
    if (var == 1) lines_launch_k<T, TR, 4, 2>(c, S, hp, A);
    else if (var == 2) lines_launch_k<T, TR, 2, 4>(c, S, hp, A);
    else if (var == 3) lines_launch_k<T, TR, 1, 8>(c, S, hp, A);
    else lines_launch_k<T, TR, 8, 1>(c, S, hp, A);
  } else {
    // FP64 lines of 16 nodes per thread exceed the registers: four waves
    if (var == 1) lines_launch_k<T, TR, 8, 2>(c, S, hp, A);
    else if (var == 2 || (var == 0 && sizeof(T) == 8)) lines_launch_k<T, TR, 4, 4>(c, S, hp, A);
    else if (var == 3) lines_launch_k<T, TR, 2, 8>(c, S, hp, A);
    else lines_launch_k<T, TR, 16, 1>(c, S, hp, A);
  }
}

template <typename T, bool TR>
void interior_run(const Ctx &c, const PrecPlan<T, TR> &P, const int *jp) {
  const int S = P.S, m = P.n1 - P.h;
  const dim3 gg((skew_steps<T>(m) + kSkewTS - 1) / kSkewTS, (m + 63) / 64, S);
  {
    KScope ks(c, KC_LAYOUT, 0.0);
    k_gather_skew<T, TR><<<gg, kSkewThreads, 0, c.stream>>>(P.ioI, jp);
  }
  {
    KScope ks(c, KC_SWEEP, (double)S * m * m * 2 * sizeof(T));
    sweep_launch<T, TR>(c, S, m, P.swI, P.varI);
  }
  KScope ks(c, KC_LAYOUT, 0.0);
  k_scatter_skew<T, TR><<<gg, kSkewThreads, 0, c.stream>>>(P.ioI, jp);
}

template <typename T, bool TR>
void lines_run(const Ctx &c, const PrecPlan<T, TR> &P, const int *jp) {
  const int S = P.S, L = P.n1 - P.h;
  const dim3 gl((P.hp + kLineTP - 1) / kLineTP, (L + kLineTQ - 1) / kLineTQ, 2 * S);
  {
    KScope ks(c, KC_LAYOUT, 0.0);
    k_gather_lines<T, TR><<<gl, 256, 0, c.stream>>>(P.ioL, jp);
  }
  {
    KScope ks(c, KC_LINES, (double)S * 2.0 * L * P.h * 4 * sizeof(T));
    lines_launch<T, TR>(c, S, P.hp, P.lnA, P.varLines);
  }
  KScope ks(c, KC_LAYOUT, 0.0);
  k_scatter_lines<T, TR><<<gl, 256, 0, c.stream>>>(P.ioL, jp);
}

// One V(1,1) cycle on level l for every system (Sec. 3.2).  zero_init: the
// level iterate is zero on entry, so the pre-smoothing sweep is the plain
// triangular solve.
template <typename T, bool TR>
void vcycle_run(const Ctx &c, const PrecPlan<T, TR> &P, int l, bool zero_init) {
  const int S = P.S, n = P.ln[l], nl = (int)P.ln.size();
  const double nn = (double)S * n * n;
  if (l == P.lc) {
    double pts = 0.0;
    for (int k = l; k < nl; ++k) pts += (double)S * P.ln[k] * P.ln[k];
    KScope ks(c, KC_MG, pts * 12 * sizeof(T));
    k_mg_coarse<T, TR><<<S, kCoarseThreads, P.coarse_lds, c.stream>>>(P.coarse, zero_init ? 1 : 0);
    return;
  }
  if (l == nl - 1) {
    KScope ks(c, KC_MG, nn * 2 * sizeof(T));
    k_mg_coarsest<T, TR><<<S, 64, 0, c.stream>>>(P.mg[l], zero_init ? 1 : 0);
    return;
  }
  const dim3 gl(blocks1d(P.lslot[l]), S), gc(blocks1d(P.lslot[l + 1]), S);
  const double cc = (double)S * P.ln[l + 1] * P.ln[l + 1];
  if (zero_init) {
    KScope ks(c, KC_SWEEP, nn * 2 * sizeof(T));
    sweep_launch<T, TR>(c, S, n, P.swb[l], P.varL[l]);
  } else {
    {
      KScope ks(c, KC_GSRHS, nn * 3 * sizeof(T));
      k_gs_rhs<T, TR><<<gl, 256, 0, c.stream>>>(P.mg[l]);
    }
    KScope ks(c, KC_SWEEP, nn * 2 * sizeof(T));
    sweep_launch<T, TR>(c, S, n, P.swt[l], P.varL[l]);
  }
  {
    KScope ks(c, KC_MG, nn * 3 * sizeof(T));
    k_mg_resid<T, TR><<<gl, 256, 0, c.stream>>>(P.mg[l]);
  }
  {
    KScope ks(c, KC_MG, (nn + cc) * sizeof(T));
    k_mg_restrict<T, TR><<<gc, 256, 0, c.stream>>>(P.mg[l]);
  }
  vcycle_run<T, TR>(c, P, l + 1, true);
  {
    // coarse-grid correction folded into the post-smoothing right-hand side
    // (the corrected iterate is not stored: the sweep rewrites z from t)
    KScope ks(c, KC_GSRHS, (3 * nn + cc) * sizeof(T));
    k_mg_prolong_gs<T, TR><<<gl, 256, 0, c.stream>>>(P.mg[l]);
  }
  KScope ks(c, KC_SWEEP, nn * 2 * sizeof(T));
  sweep_launch<T, TR>(c, S, n, P.swt[l], P.varL[l]);
}

// blocks of the corner residual-norm reduction (one partial each)
constexpr int kMgNormBlocks = 256;

// Parabolic case: one downstream Gauss-Seidel sweep of coarse level l for
// every system (one workgroup each, one wave per 64 lanes of M columns),
// after the pass that folds the old values into the right-hand side (none
// on a zero iterate).
template <typename T>
void par_wave_launch(const Ctx &c, int S, const ParSkew &sk, const ParArgs<T> *A, int zero_init) {
  // the shapes of par_skew: M = 2 and 8 in one wave, M = 4 in one or two
  constexpr int D2 = par_ahead<T, 2>(), D4 = par_ahead<T, 4>(), D8 = par_ahead<T, 8>();
  if (sk.M == 2) {
    k_par_wave<T, 1, 2, D2><<<S, 64, 0, c.stream>>>(A, zero_init);
  } else if (sk.M == 8) {
    if constexpr (sizeof(T) == 4) k_par_wave<T, 1, 8, D8><<<S, 64, 0, c.stream>>>(A, zero_init);
  } else if (sk.L <= 64) {
    k_par_wave<T, 1, 4, D4><<<S, 64, 0, c.stream>>>(A, zero_init);
  } else {
    k_par_wave<T, 2, 4, D4><<<S, 128, 0, c.stream>>>(A, zero_init);
  }
}

template <typename T, bool TR>
void par_gs_run(const Ctx &c, const PrecPlan<T, TR> &P, int l, int zero_init) {
  const ParSkew &sk = P.psk[l];
  const double nn = (double)P.S * sk.nx * sk.ny;
  if (!zero_init) {
    // b, four couplings and the old iterate in, the right-hand side out
    KScope ks(c, KC_GSRHS, nn * 7 * sizeof(T));
    k_par_pre<T><<<dim3(blocks1d(sk.nslot()), P.S), 256, 0, c.stream>>>(P.pa[l]);
  }
  // the right-hand side, four couplings and 1 / centre in, the iterate out
  KScope ks(c, KC_SWEEP, nn * 7 * sizeof(T));
  par_wave_launch<T>(c, P.S, sk, P.pa[l], zero_init);
}

// One Gauss-Seidel sweep of level 0: the level-0 sweep of the
// two-exponential-layer cycle (same block, same order of results), from b
// when the iterate is zero, else from the right-hand side with the old
// West and South values folded in.
template <typename T, bool TR>
void par_level0_smooth(const Ctx &c, const PrecPlan<T, TR> &P, bool zero_init) {
  const int S = P.S, n = P.ln[0];
  const double nn = (double)S * n * n;
  if (!zero_init) {
    KScope ks(c, KC_GSRHS, nn * 3 * sizeof(T));
    k_gs_rhs<T, TR><<<dim3(blocks1d(P.lslot[0]), S), 256, 0, c.stream>>>(P.mg[0]);
  }
  KScope ks(c, KC_SWEEP, nn * 2 * sizeof(T));
  sweep_launch<T, TR>(c, S, n, zero_init ? P.swb[0] : P.swt[0], P.varL[0]);
}

// One V(1,1) cycle on level l of the semicoarsening hierarchy (Sec. 3.2);
// the coarsest level gets four sweeps.  zero_init: the level iterate is
// zero on entry.
template <typename T, bool TR>
void par_vcycle_run(const Ctx &c, const PrecPlan<T, TR> &P, int l, bool zero_init) {
  const int S = P.S, nx = P.pn[l], h = P.h, nl = (int)P.pn.size();
  if (l == nl - 1) {
    for (int k = 0; k < 4; ++k) {
      if (l == 0) par_level0_smooth<T, TR>(c, P, zero_init && k == 0);
      else par_gs_run<T, TR>(c, P, l, zero_init && k == 0);
    }
    return;
  }
  const int nxc = P.pn[l + 1];
  const double nn = (double)S * nx * h, cc = (double)S * nxc * h;
  const dim3 gc(blocks1d(P.psk[l + 1].nslot()), S);  // over the next level's words
  if (l == 0) {
    par_level0_smooth<T, TR>(c, P, zero_init);
    {
      KScope ks(c, KC_MG, (2.0 * nn + cc) * sizeof(T));
      k_par_rr0<T><<<gc, 256, 0, c.stream>>>(P.pa[0]);
    }
    par_vcycle_run<T, TR>(c, P, 1, true);
    {
      KScope ks(c, KC_MG, (2.0 * nn + cc) * sizeof(T));
      k_par_prolong0<T><<<dim3((nx + 255) / 256, h, S), 256, 0, c.stream>>>(P.pa[0]);
    }
    par_level0_smooth<T, TR>(c, P, false);
    return;
  }
  const dim3 gf(blocks1d(P.psk[l].nslot()), S);  // over this level's words
  par_gs_run<T, TR>(c, P, l, zero_init);
  {
    KScope ks(c, KC_MG, nn * 12 * sizeof(T));
    k_par_resid<T><<<gf, 256, 0, c.stream>>>(P.pa[l]);
  }
  {
    KScope ks(c, KC_MG, (2.0 * nn + cc) * sizeof(T));
    k_par_restrict<T><<<gc, 256, 0, c.stream>>>(P.pa[l]);
  }
  par_vcycle_run<T, TR>(c, P, l + 1, true);
  {
    KScope ks(c, KC_MG, (2.0 * nn + cc) * sizeof(T));
    k_par_prolong<T><<<gf, 256, 0, c.stream>>>(P.pa[l]);
  }
  par_gs_run<T, TR>(c, P, l, 0);
}

template <typename T, bool TR>
void mg_norm_run(const Ctx &c, const PrecPlan<T, TR> &P, int mode) {
  const int nblk = std::min(kMgNormBlocks, (int)blocks1d(P.lslot[0]));
  KScope ks(c, KC_MG, (double)P.S * P.ln[0] * P.ln[0] * 2 * sizeof(T));
  if (mode == 1) k_mg_norm<T, TR, 1><<<dim3(nblk, P.S), 256, 0, c.stream>>>(P.mg[0]);
  else k_mg_norm<T, TR, 0><<<dim3(nblk, P.S), 256, 0, c.stream>>>(P.mg[0]);
}

// The corner right-hand side and the first cycles: fixed mode runs all its
// cycles; the adaptive rule (Sec. 3.2) enqueues the initial norm and up to
// `first` cycles with their norms, each gated per system on device.
template <typename T, bool TR>
void corner_begin(const Ctx &c, const PrecPlan<T, TR> &P, const int *jp, const blp_prec_opts &o,
                  int first) {
  const int h = P.h;
  {
    KScope ks(c, KC_LAYOUT, 0.0);
    k_corner_rhs<T, TR><<<dim3((h + 255) / 256, h, P.S), 256, 0, c.stream>>>(P.cr, jp);
  }
  if (P.par) {
    // the stopping rule is that of level 0, the same rescaled norm as for two
    // exponential layers
    if (o.mg_fixed > 0) {
      for (int k = 0; k < o.mg_fixed; ++k) {
        par_vcycle_run<T, TR>(c, P, 0, k == 0);
        k_mg_count<T><<<P.S, 64, 0, c.stream>>>(P.mg[0]);
      }
      return;
    }
    mg_norm_run<T, TR>(c, P, 0);
    for (int k = 0; k < std::min(first, o.mg_maxcyc); ++k) {
      par_vcycle_run<T, TR>(c, P, 0, k == 0);
      mg_norm_run<T, TR>(c, P, 1);
    }
    return;
  }
  if (o.mg_fixed > 0) {
    for (int k = 0; k < o.mg_fixed; ++k) {
      vcycle_run<T, TR>(c, P, 0, k == 0);
      k_mg_count<T><<<P.S, 64, 0, c.stream>>>(P.mg[0]);
    }
    return;
  }
  mg_norm_run<T, TR>(c, P, 0);
  for (int k = 0; k < std::min(first, o.mg_maxcyc); ++k) {
    vcycle_run<T, TR>(c, P, 0, k == 0);
    mg_norm_run<T, TR>(c, P, 1);
  }
}

// One more adaptive cycle and its residual norm (after the first cycles),
// on the corner hierarchy of the plan's kind.
template <typename T, bool TR>
void corner_cycle(const Ctx &c, const PrecPlan<T, TR> &P) {
  if (P.par) {
    par_vcycle_run<T, TR>(c, P, 0, false);
    mg_norm_run<T, TR>(c, P, 1);
  } else {
    vcycle_run<T, TR>(c, P, 0, false);
    mg_norm_run<T, TR>(c, P, 1);
  }
}

// Further adaptive cycles while any system's corner gate is open; ctrl_h
// mirrors the systems' control blocks (contiguous device array ctrl).
template <typename T, bool TR>
int corner_finish(const Ctx &c, const PrecPlan<T, TR> &P, const blp_prec_opts &o, int done,
                  const MgCtrl *ctrl, MgCtrl *ctrl_h, int S) {
  if (o.mg_fixed > 0) return BLP_OK;
  for (int k = done; k < o.mg_maxcyc; ++k) {
    HIP_TRY(hipMemcpyAsync(ctrl_h, ctrl, S * sizeof(MgCtrl), hipMemcpyDeviceToHost, c.stream));
    HIP_TRY(hipStreamSynchronize(c.stream));
    bool open = false;
    for (int s = 0; s < S; ++s) open = open || !ctrl_h[s].gate;
    if (!open) break;
    corner_cycle<T, TR>(c, P);
  }
  return BLP_OK;
}

template <typename T, bool TR>
void corner_end(const Ctx &c, const PrecPlan<T, TR> &P, const int *jp) {
  KScope ks(c, KC_LAYOUT, 0.0);
  k_corner_copy<T, TR><<<dim3((P.h + 255) / 256, P.h, P.S), 256, 0, c.stream>>>(P.cr, jp);
}

// Cycles the adaptive rule enqueues before it looks at the corner residuals:
// the count the rule usually takes (Sec. 3.2: five for two exponential
// layers, about three with a parabolic one).  Enqueued cycles past a
// system's stop are gated launches; a system that needs more gets them
// through the host check.
template <typename T, bool TR>
int first_cycles(const PrecPlan<T, TR> &P) {
  return P.par ? 3 : 5;
}

// Preconditioner part before the corner-cycle check: forward I, edges,
// corner right-hand side and the first cycles; transposed (M^T, block lower
// triangular) the corner right-hand side and first cycles only.
template <typename T, bool TR>
void prec_part1(const Ctx &c, const PrecPlan<T, TR> &P, const int *jp, const blp_prec_opts &o) {
  if (!TR) {
    interior_run<T, TR>(c, P, jp);
    lines_run<T, TR>(c, P, jp);
  }
  corner_begin<T, TR>(c, P, jp, o, first_cycles(P));
}
// ... and after it: corner copy-back, then (transposed) edges and interior.
template <typename T, bool TR>
void prec_part2(const Ctx &c, const PrecPlan<T, TR> &P, const int *jp) {
  corner_end<T, TR>(c, P, jp);
  if (TR) {
    lines_run<T, TR>(c, P, jp);
    interior_run<T, TR>(c, P, jp);
  }
}

// ------------------------------------------------------------------------ //
// Batches                                                                   //
// ------------------------------------------------------------------------ //

// Operator / Krylov plans of one class for one precision and direction.
template <typename TV, bool TR, bool SCALE>
struct SolvePlan {
  int S = 0;
  std::vector<int> idx;             // the batch's systems the plan covers, in record order
  PrecPlan<TV, TR> prec;
  SpmvArgs<TV> *spmv = nullptr;     // x = Z_j -> w
  SpmvArgs<double> *resid = nullptr;  // w = F - A u (scaled if SCALE), ||w||
  NormArgs *norm = nullptr;         // ||F|| (scaled if SCALE)
  KArgs<TV> *kr = nullptr;
  int rows = kRows;  // stencil strip height (autotuner)
  bool tuned = false;
  Alloc mem;
  std::vector<const double *> F;    // right-hand sides the plan is bound to
  std::vector<double *> U;
  std::vector<const void *> V;      // Krylov bases the plan was built on
  // preconditioner options the plan was built with (its corner records hold
  // the stopping rule, its captured graphs the cycle schedule)
  blp_prec_opts po{0, 0.0, 0};
  // host copies of the records that hold F and U (rebound in place when a
  // solve passes other vectors; their device arrays keep their addresses,
  // so captured graphs stay valid)
  std::vector<SpmvArgs<double>> resid_h;
  std::vector<NormArgs> norm_h;
  std::vector<KArgs<TV>> kr_h;
  // captured step (graphs mode): part 1 of the preconditioner; the rest of
  // the step (corner copy-back, remaining regions, SpMV, Arnoldi)
  hipGraphExec_t g1 = nullptr, g2 = nullptr;
  ~SolvePlan() {
    if (g1) (void)hipGraphExecDestroy(g1);
    if (g2) (void)hipGraphExecDestroy(g2);
  }
};

struct PlanBase {
  virtual ~PlanBase() {}
};
template <typename TV, bool TR, bool SCALE>
struct PlanHolder : PlanBase {
  SolvePlan<TV, TR, SCALE> plan;
};

struct Batch {
  hipStream_t stream = nullptr;
  std::vector<std::unique_ptr<System>> sys;
  std::vector<std::vector<int>> classes;  // system indices by mesh size
  MgCtrl *ctrl = nullptr, *ctrl_h = nullptr;
  KrylovStatus *st = nullptr, *st_h = nullptr;
  int *gate = nullptr, *gate_h = nullptr;
  int *jdev = nullptr;
  int *ncol = nullptr, *ncol_h = nullptr;
  Timer *timer = nullptr;  // the problem's timer (own batches) or own_timer
  Timer own_timer;
  int graphs = 0, autotune = 0;  // blp_batch_opts
  int sweep_variant = 0;          // blp_batch_opts test hook (0: default)
  hipStream_t user = nullptr;     // caller's stream when the batch runs on its own
  bool own_stream = false;
  // one stream per mesh class when there are several (default priority)
  std::vector<hipStream_t> cstream;
  std::vector<hipEvent_t> cevent;
  hipEvent_t fork_ev = nullptr;
  Alloc mem;
  // cached plans per class and kind (key: class, TV, TR, SCALE, m)
  std::map<std::tuple<int, int, int, int, int>, std::unique_ptr<PlanBase>> plans;
  // plans over the systems of a class still iterating (same key, then the
  // systems), taken when some of the class have left the iteration
  std::map<std::tuple<int, int, int, int, int>, std::map<std::vector<int>, std::unique_ptr<PlanBase>>>
      subplans;
  ~Batch() {
    if (stream) (void)hipStreamSynchronize(stream);
    subplans.clear();
    plans.clear();
    sys.clear();
    mem.release();
    for (hipStream_t q : cstream) {
      (void)hipStreamSynchronize(q);
      (void)hipStreamDestroy(q);
    }
    for (hipEvent_t e : cevent) (void)hipEventDestroy(e);
    if (fork_ev) (void)hipEventDestroy(fork_ev);
    if (own_stream) (void)hipStreamDestroy(stream);
    if (ctrl_h) (void)hipHostFree(ctrl_h);
    if (st_h) (void)hipHostFree(st_h);
    if (gate_h) (void)hipHostFree(gate_h);
    if (ncol_h) (void)hipHostFree(ncol_h);
  }
};

// A batch over the given (preconditioned) problems, one system each.
int batch_create(hipStream_t stream, blp_problem *const *probs, int S, std::unique_ptr<Batch> &out) {
  std::unique_ptr<Batch> B(new (std::nothrow) Batch());
  if (!B) return BLP_E_NOMEM;
  B->stream = stream;
  BLP_TRY(B->mem.get(&B->ctrl, S, stream, true));
  BLP_TRY(B->mem.get(&B->st, S, stream, true));
  BLP_TRY(B->mem.get(&B->gate, S, stream, true));
  BLP_TRY(B->mem.get(&B->jdev, 1, stream, true));
  BLP_TRY(B->mem.get(&B->ncol, S, stream, true));
  if (hipHostMalloc((void **)&B->ctrl_h, S * sizeof(MgCtrl), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void **)&B->st_h, S * sizeof(KrylovStatus), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void **)&B->gate_h, S * sizeof(int), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void **)&B->ncol_h, S * sizeof(int), hipHostMallocDefault) != hipSuccess)
    return BLP_E_NOMEM;
  std::map<int, std::vector<int>> byN;
  for (int s = 0; s < S; ++s) {
    blp_problem *p = probs[s];
    if (!p || !p->prec_ready) return BLP_E_STATE;
    std::unique_ptr<System> y(new (std::nothrow) System());
    if (!y) return BLP_E_NOMEM;
    y->p = p;
    y->ctrl = B->ctrl + s;
    y->st = B->st + s;
    y->gate = B->gate + s;
    BLP_TRY(y->mem.get(&y->mg_partials, kMgNormBlocks, stream, true));
    BLP_TRY(alloc_work<double>(*y, stream, y->w64, p->f64, p->l64));
    BLP_TRY(alloc_work<float>(*y, stream, y->w32, p->f32, p->l32));
    B->sys.push_back(std::move(y));
    byN[p->N].push_back(s);
  }
  // largest meshes first: their launches start first in every step
  for (auto it = byN.rbegin(); it != byN.rend(); ++it) B->classes.push_back(it->second);
  HIP_TRY(hipStreamSynchronize(stream));
  out = std::move(B);
  return BLP_OK;
}

long long batch_bytes(const Batch &B) {
  long long b = B.mem.bytes;
  for (const auto &y : B.sys) b += y->mem.bytes + y->krylov_bytes();
  return b;
}

template <typename TV, bool TR, bool SCALE>
int build_solve_plan(Batch &B, const std::vector<int> &cls, int m, const double *const *F,
                     double *const *U, SolvePlan<TV, TR, SCALE> &P) {
  hipStream_t st = B.stream;
  const int S = (int)cls.size();
  P.S = S;
  std::vector<System *> sys;
  std::vector<IOSpec> io;
  std::vector<SpmvArgs<TV>> sp(S);
  std::vector<SpmvArgs<double>> rs(S);
  std::vector<NormArgs> nm(S);
  std::vector<KArgs<TV>> kr(S);
  P.F.clear();
  P.U.clear();
  P.V.clear();
  P.idx = cls;
  P.po = B.sys[cls[0]]->p->popts;
  for (int k = 0; k < S; ++k) {
    System &y = *B.sys[cls[k]];
    blp_problem *p = y.p;
    const size_t n = p->n;
    sys.push_back(&y);
    io.push_back(IOSpec{y.V, (long long)n, y.Z, (long long)n});
    const Grid<double> g = p->grid64();
    sp[k] = SpmvArgs<TV>{g, (const TV *)y.Z, (long long)n, y.w, nullptr, nullptr, nullptr, y.gate};
    rs[k] = SpmvArgs<double>{g, U[cls[k]], 0, y.w, F[cls[k]], y.partials, y.st, y.gate};
    nm[k] = NormArgs{g, F[cls[k]], y.partials, y.st, nullptr};
    kr[k] = KArgs<TV>{(TV *)y.V, (TV *)y.Z, n, y.w, y.partials, y.ks, y.st, U[cls[k]], y.gate};
    P.F.push_back(F[cls[k]]);
    P.U.push_back(U[cls[k]]);
    P.V.push_back(y.V);
  }
  BLP_TRY((build_prec_plan<TV, TR>(st, sys, io, SCALE, P.prec)));
  BLP_TRY(P.mem.put(&P.spmv, sp.data(), S, st));
  BLP_TRY(P.mem.put(&P.resid, rs.data(), S, st));
  BLP_TRY(P.mem.put(&P.norm, nm.data(), S, st));
  BLP_TRY(P.mem.put(&P.kr, kr.data(), S, st));
  P.resid_h = rs;
  P.norm_h = nm;
  P.kr_h = kr;
  HIP_TRY(hipStreamSynchronize(st));
  return BLP_OK;
}

// Point an existing plan at other right-hand sides and iterates: only the
// residual, norm and Krylov records hold them.
template <typename TV, bool TR, bool SCALE>
int rebind_solve_plan(Batch &B, const std::vector<int> &cls, const double *const *F,
                      double *const *U, SolvePlan<TV, TR, SCALE> &P) {
  const int S = (int)cls.size();
  for (int k = 0; k < S; ++k) {
    P.resid_h[k].x = U[cls[k]];
    P.resid_h[k].F = F[cls[k]];
    P.norm_h[k].F = F[cls[k]];
    P.kr_h[k].u = U[cls[k]];
    P.F[k] = F[cls[k]];
    P.U[k] = U[cls[k]];
  }
  HIP_TRY(hipMemcpyAsync(P.resid, P.resid_h.data(), S * sizeof(SpmvArgs<double>), hipMemcpyHostToDevice,
                         B.stream));
  HIP_TRY(hipMemcpyAsync(P.norm, P.norm_h.data(), S * sizeof(NormArgs), hipMemcpyHostToDevice, B.stream));
  HIP_TRY(hipMemcpyAsync(P.kr, P.kr_h.data(), S * sizeof(KArgs<TV>), hipMemcpyHostToDevice, B.stream));
  HIP_TRY(hipStreamSynchronize(B.stream));  // the host copies may change at the next rebind
  return BLP_OK;
}

// Average time of reps launches issued by f (after one untimed launch).
template <typename Fn>
float time_launches(hipStream_t s, Fn &&f, int reps) {
  hipEvent_t a = nullptr, b = nullptr;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return 1e30f;
  f();
  (void)hipEventRecord(a, s);
  for (int r = 0; r < reps; ++r) f();
  (void)hipEventRecord(b, s);
  float ms = 1e30f;
  if (hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&ms, a, b) != hipSuccess)
    ms = 1e30f;
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return ms / reps;
}

// Autotuner: for one class, time every variant of the interior sweep, of
// each corner level's sweep, of the line solves and of the stencil strip
// height on the plan's own data and keep the fastest.  The variants compute
// the same values (sweeps bit for bit); only the schedule differs.  Runs
// once per plan, with every gate of the class open (the work vectors it
// overwrites are rewritten by the next apply).
template <typename TV, bool TR, bool SCALE>
int tune_plan(Batch &B, int cls, SolvePlan<TV, TR, SCALE> &P) {
  const hipStream_t st = B.stream;
  HIP_TRY(hipMemsetAsync(B.gate, 0, B.sys.size() * sizeof(int), st));
  HIP_TRY(hipMemsetAsync(B.ctrl, 0, B.sys.size() * sizeof(MgCtrl), st));
  const Ctx c{st, nullptr};
  PrecPlan<TV, TR> &Q = P.prec;
  const int S = Q.S, m = Q.n1 - Q.h, reps = 4;
  auto pick = [&](int nvar, auto &&launch) {
    int best = 0;
    float tbest = 1e30f;
    for (int v = 0; v < nvar; ++v) {
      const float t = time_launches(st, [&]() { launch(v); }, reps);
      if (t < tbest) {
        tbest = t;
        best = v;
      }
    }
    return best;
  };
  Q.varI = pick(sweep_variants(m), [&](int v) { sweep_launch<TV, TR>(c, S, m, Q.swI, v); });
  for (size_t l = 0; l + 1 < Q.ln.size(); ++l) {
    const int n = Q.ln[l];
    Q.varL[l] = pick(sweep_variants(n), [&](int v) { sweep_launch<TV, TR>(c, S, n, Q.swb[l], v); });
  }
  Q.varLines = pick(lines_variants(Q.hp), [&](int v) { lines_launch<TV, TR>(c, S, Q.hp, Q.lnA, v); });
  const int n1 = Q.n1;
  const int rows_c[3] = {8, 16, 32};
  const int r = pick(3, [&](int v) {
    const int rows = rows_c[v];
    k_stencil<TV, TR, SCALE, false>
        <<<dim3((n1 + 255) / 256, (n1 + rows - 1) / rows, S), 256, 0, st>>>(P.spmv, B.jdev, rows);
  });
  P.rows = rows_c[r];
  P.tuned = true;
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(st));
  (void)cls;
  return BLP_OK;
}

template <typename TV, bool TR, bool SCALE>
int get_solve_plan(Batch &B, int c, int m, const double *const *F, double *const *U,
                   SolvePlan<TV, TR, SCALE> **out) {
  const auto key = std::make_tuple(c, (int)sizeof(TV), (int)TR, (int)SCALE, m);
  auto it = B.plans.find(key);
  if (it != B.plans.end()) {
    auto *h = static_cast<PlanHolder<TV, TR, SCALE> *>(it->second.get());
    bool basis = true, same = true;
    for (size_t k = 0; k < B.classes[c].size(); ++k) {
      const int s = B.classes[c][k];
      basis = basis && h->plan.V[k] == B.sys[s]->V;
      same = same && h->plan.F[k] == F[s] && h->plan.U[k] == U[s];
    }
    // a problem preconditioned again with other options needs a new plan
    const blp_prec_opts &q = B.sys[B.classes[c][0]]->p->popts;
    const bool opts = q.mg_fixed == h->plan.po.mg_fixed && q.mg_rtol == h->plan.po.mg_rtol &&
                      q.mg_maxcyc == h->plan.po.mg_maxcyc;
    if (basis && opts) {
      if (!same) BLP_TRY((rebind_solve_plan<TV, TR, SCALE>(B, B.classes[c], F, U, h->plan)));
      *out = &h->plan;
      return BLP_OK;
    }
    B.plans.erase(it);  // built on a basis since reallocated, or with other options
  }
  std::unique_ptr<PlanHolder<TV, TR, SCALE>> h(new (std::nothrow) PlanHolder<TV, TR, SCALE>());
  if (!h) return BLP_E_NOMEM;
  BLP_TRY((build_solve_plan<TV, TR, SCALE>(B, B.classes[c], m, F, U, h->plan)));
  if (B.autotune) BLP_TRY((tune_plan<TV, TR, SCALE>(B, c, h->plan)));
  if (B.sweep_variant > 0) {
    // every sweep of the plan takes the requested variant (modulo the
    // number its width has)
    PrecPlan<TV, TR> &Q = h->plan.prec;
    const int v = B.sweep_variant - 1;
    Q.varI = v % sweep_variants(Q.n1 - Q.h);
    for (size_t l = 0; l < Q.ln.size(); ++l) Q.varL[l] = v % sweep_variants(Q.ln[l]);
  }
  *out = &h->plan;
  B.plans[key] = std::move(h);
  return BLP_OK;
}

// A plan over the systems sub of class c (those still iterating), with the
// full class plan's kernel variants.  Kernels launch one block row per
// system of their plan; a system that has left the iteration only reads its
// gate and exits, but with most of a class done those blocks dominate the
// small kernels' time, so each restart cycle takes the plan of its systems.
constexpr size_t kMaxSubPlans = 16;  // per class and kind
template <typename TV, bool TR, bool SCALE>
int get_subset_plan(Batch &B, int c, const std::vector<int> &sub, int m, const double *const *F,
                    double *const *U, const SolvePlan<TV, TR, SCALE> &full,
                    SolvePlan<TV, TR, SCALE> **out) {
  auto &mp = B.subplans[std::make_tuple(c, (int)sizeof(TV), (int)TR, (int)SCALE, m)];
  auto it = mp.find(sub);
  if (it != mp.end()) {
    auto *h = static_cast<PlanHolder<TV, TR, SCALE> *>(it->second.get());
    bool basis = true, same = true;
    for (size_t k = 0; k < sub.size(); ++k) {
      const int s = sub[k];
      basis = basis && h->plan.V[k] == B.sys[s]->V;
      same = same && h->plan.F[k] == F[s] && h->plan.U[k] == U[s];
    }
    const blp_prec_opts &q = full.po, &r = h->plan.po;
    const bool opts = q.mg_fixed == r.mg_fixed && q.mg_rtol == r.mg_rtol && q.mg_maxcyc == r.mg_maxcyc;
    if (basis && opts) {
      if (!same) BLP_TRY((rebind_solve_plan<TV, TR, SCALE>(B, sub, F, U, h->plan)));
      *out = &h->plan;
      return BLP_OK;
    }
    mp.erase(it);
  }
  if (mp.size() >= kMaxSubPlans) mp.clear();
  std::unique_ptr<PlanHolder<TV, TR, SCALE>> h(new (std::nothrow) PlanHolder<TV, TR, SCALE>());
  if (!h) return BLP_E_NOMEM;
  BLP_TRY((build_solve_plan<TV, TR, SCALE>(B, sub, m, F, U, h->plan)));
  PrecPlan<TV, TR> &Q = h->plan.prec;
  Q.varI = full.prec.varI;
  Q.varL = full.prec.varL;
  Q.varLines = full.prec.varLines;
  h->plan.rows = full.rows;
  h->plan.tuned = full.tuned;
  *out = &h->plan;
  mp[sub] = std::move(h);
  return BLP_OK;
}

// Class streams: created on first use when the batch has several classes.
int ensure_class_streams(Batch &B) {
  const int NC = (int)B.classes.size();
  if (NC < 2 || (int)B.cstream.size() == NC) return BLP_OK;
  HIP_TRY(hipEventCreateWithFlags(&B.fork_ev, hipEventDisableTiming));
  for (int k = 0; k < NC; ++k) {
    hipStream_t q = nullptr;
    hipEvent_t e = nullptr;
    HIP_TRY(hipStreamCreateWithFlags(&q, hipStreamNonBlocking));
    B.cstream.push_back(q);
    HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    B.cevent.push_back(e);
  }
  return BLP_OK;
}
hipStream_t class_stream(const Batch &B, int k) {
  return B.cstream.empty() ? B.stream : B.cstream[k];
}
// Class streams wait for the work enqueued on the batch stream so far.
int fork(Batch &B) {
  if (B.cstream.empty()) return BLP_OK;
  HIP_TRY(hipEventRecord(B.fork_ev, B.stream));
  for (hipStream_t q : B.cstream) HIP_TRY(hipStreamWaitEvent(q, B.fork_ev, 0));
  return BLP_OK;
}
// The batch stream waits for the work enqueued on every class stream.
int join(Batch &B) {
  for (size_t k = 0; k < B.cstream.size(); ++k) {
    HIP_TRY(hipEventRecord(B.cevent[k], B.cstream[k]));
    HIP_TRY(hipStreamWaitEvent(B.stream, B.cevent[k], 0));
  }
  return BLP_OK;
}

int upload_gates(Batch &B) {
  HIP_TRY(hipMemcpyAsync(B.gate, B.gate_h, B.sys.size() * sizeof(int), hipMemcpyHostToDevice,
                         B.stream));
  return BLP_OK;
}
int read_all(Batch &B) {
  const size_t S = B.sys.size();
  HIP_TRY(hipMemcpyAsync(B.st_h, B.st, S * sizeof(KrylovStatus), hipMemcpyDeviceToHost, B.stream));
  HIP_TRY(hipMemcpyAsync(B.ctrl_h, B.ctrl, S * sizeof(MgCtrl), hipMemcpyDeviceToHost, B.stream));
  HIP_TRY(hipStreamSynchronize(B.stream));
  return BLP_OK;
}

__global__ void k_set_int(int *p, int v) { *p = v; }

// Capture the launches `body` issues on stream s into an executable graph.
// The captured kernels take their step index and gates from device memory,
// so one graph serves every step; it holds kernel nodes only (no memsets).
template <typename Body>
int capture(hipStream_t s, hipGraphExec_t *out, Body &&body) {
  hipGraph_t g = nullptr;
  HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  body();
  const hipError_t e = hipStreamEndCapture(s, &g);
  if (e != hipSuccess || !g) return BLP_E_HIP;
  const hipError_t e2 = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  return e2 == hipSuccess ? BLP_OK : BLP_E_HIP;
}

// SpMV on Z_j and the CGS2 Arnoldi kernels of one class (step j in jdev).
template <typename TV, bool TR, bool SCALE>
void krylov_step(const Ctx &c, const SolvePlan<TV, TR, SCALE> &P, int n1, int j, const int *jdev,
                 const KOffsets &ko) {
  const size_t n = (size_t)n1 * n1;
  const int Sk = P.S;
  {
    KScope ks(c, KC_SPMV, (double)Sk * n * (sizeof(TV) + sizeof(double)));
    k_stencil<TV, TR, SCALE, false>
        <<<dim3((n1 + 255) / 256, (n1 + P.rows - 1) / P.rows, Sk), 256, 0, c.stream>>>(P.spmv, jdev,
                                                                                     P.rows);
  }
  const unsigned nb = (unsigned)((n + KCHUNK - 1) / KCHUNK);
  // CGS2: four passes over the j+1 basis vectors plus w traffic
  KScope ks(c, KC_KRYLOV, (double)Sk * n * ((4.0 * (j + 1)) * sizeof(TV) + 6 * sizeof(double)));
  k_arnoldi_dot<TV><<<dim3(nb, Sk), 256, 0, c.stream>>>(P.kr, jdev, ko);
  k_arnoldi_update<TV, false><<<dim3(nb, Sk), 256, 0, c.stream>>>(P.kr, jdev, ko);
  k_arnoldi_update<TV, true><<<dim3(nb, Sk), 256, 0, c.stream>>>(P.kr, jdev, ko);
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

// Right-preconditioned FGMRES(m) from u = 0 (Saad) for every system of the
// batch.  In scaled mode the Krylov space is that of D^{-1/2} A D^{-1/2}; the
// preconditioned vectors Z are kept in the unscaled variables, so u += Z y
// needs no rescaling.  TV = double: FP64 throughout.  TV = float (mixed): V,
// Z and the preconditioner in FP32; SpMV arithmetic, Hessenberg/Givens, u and
// the restart-boundary true residuals in FP64; each restart cycle reduces the
// residual by at most inner_rtol before an FP64 residual is taken.
//
// Streams: host-side decisions (gates, step index, status reads) go through
// the batch stream; with several mesh classes each class runs on a stream
// of its own between a fork (classes wait for the batch stream) and a join
// (the batch stream waits for every class), so that the classes' launches
// overlap on the GPU.  Classes without a flagged system are not launched.
template <typename TV, bool TR, bool SCALE>
int fgmres_batch(Batch &B, const double *const *F, double *const *U, const blp_solve_opts *o,
                 blp_solve_info *info, double *const *hist) {
  const int S = (int)B.sys.size(), m = o->restart, NC = (int)B.classes.size();
  // mixed: a restart cycle ends once its estimate has dropped by 1e-6 (well
  // above the FP32 basis' rounding level, so the estimate still tracks the
  // true residual; at N = 1024, eps = 1e-6 this saves the cycle that a 1e-4
  // target needs, and 1e-7 adds one back)
  const double inner_rtol = std::is_same<TV, float>::value ? 1e-6 : 0.0;
  const KOffsets ko{m};
  auto t0 = std::chrono::steady_clock::now();
  for (auto &y : B.sys) BLP_TRY(ensure_krylov(*y, B.stream, m, o->precision));
  BLP_TRY(ensure_class_streams(B));
  // per class: the full plan, the plan of the systems that started the
  // current restart cycle, and the plan the steps launch
  std::vector<SolvePlan<TV, TR, SCALE> *> P(NC), Pfull(NC), Pcyc(NC);
  for (int k = 0; k < NC; ++k) BLP_TRY((get_solve_plan<TV, TR, SCALE>(B, k, m, F, U, &P[k])));
  Pfull = P;
  // the plan over a class's systems still in the cycle, once they are at
  // most half of the plan's (fewer idle blocks, few plan switches)

  const blp_prec_opts &po = B.sys[0]->p->popts;
  // kernel timing records events between launches: no graphs then
  const bool use_graphs = B.graphs && !(B.timer && B.timer->on);
  std::vector<Ctx> cx(NC);
  for (int k = 0; k < NC; ++k) cx[k] = Ctx{class_stream(B, k), B.timer};

  std::vector<double> nF(S), target(S), beta(S), cyc_target(S);
  std::vector<int> it(S, 0), restarts(S, 0), ncol(S, 0);
  std::vector<char> active(S, 1), conv(S, 0), incyc(S, 0), est_ok(S, 0);
  std::vector<CycleStats> cs(S);
  // the plan over a class's systems still in the cycle, once they are at
  // most half of the plan's (fewer idle blocks, few plan switches)
  auto shrink = [&](int k) {
    std::vector<int> sub;
    for (int s : B.classes[k])
      if (incyc[s]) sub.push_back(s);
    if (sub.empty() || 2 * (int)sub.size() > P[k]->S) return (int)BLP_OK;
    return get_subset_plan<TV, TR, SCALE>(B, k, sub, m, F, U, *Pfull[k], &P[k]);
  };
  // classes with at least one system flagged (launches of other classes are skipped)
  auto live = [&](int k, const std::vector<char> &on) {
    for (int s : B.classes[k])
      if (on[s]) return true;
    return false;
  };
  auto set_gates = [&](const std::vector<char> &on) {
    for (int s = 0; s < S; ++s) B.gate_h[s] = on[s] ? 0 : 1;
    return upload_gates(B);
  };
  // ||F||, u = 0
  for (int s = 0; s < S; ++s) B.gate_h[s] = 0;
  BLP_TRY(upload_gates(B));
  for (int s = 0; s < S; ++s)
    HIP_TRY(hipMemsetAsync(U[s], 0, B.sys[s]->p->n * sizeof(double), B.stream));
  BLP_TRY(fork(B));
  for (int k = 0; k < NC; ++k)
    k_norm<SCALE><<<dim3(256, P[k]->S), 256, 0, cx[k].stream>>>(P[k]->norm);
  BLP_TRY(join(B));
  BLP_TRY(read_all(B));
  for (int s = 0; s < S; ++s) {
    nF[s] = B.st_h[s].beta;
    if (!std::isfinite(nF[s])) return BLP_E_NUMERIC;
    target[s] = o->absolute ? o->tol : o->tol * nF[s];
  }
  // true residual of the active systems (gates = active)
  auto residual = [&]() {
    BLP_TRY(fork(B));
    for (int k = 0; k < NC; ++k) {
      if (!live(k, active)) continue;
      const int n1 = B.sys[B.classes[k][0]]->p->n1;
      KScope ks(cx[k], KC_SPMV, (double)P[k]->S * n1 * n1 * 3 * sizeof(double));
      k_stencil<double, TR, SCALE, true>
          <<<dim3((n1 + 255) / 256, (n1 + kRows - 1) / kRows, P[k]->S), 256, 0, cx[k].stream>>>(
              P[k]->resid, nullptr, kRows);
    }
    BLP_TRY(join(B));
    return read_all(B);
  };
  BLP_TRY(residual());
  for (int s = 0; s < S; ++s) {
    beta[s] = B.st_h[s].beta;
    if (hist && hist[s]) hist[s][0] = beta[s];
    conv[s] = beta[s] <= target[s];
    active[s] = !conv[s] && it[s] < o->maxit;
  }
  while (std::any_of(active.begin(), active.end(), [](char a) { return a != 0; })) {
    for (int s = 0; s < S; ++s) {
      if (active[s] && !std::isfinite(beta[s])) return BLP_E_NUMERIC;
      incyc[s] = active[s];
      cyc_target[s] = std::max(target[s], inner_rtol * beta[s]);
      ncol[s] = 0;
      est_ok[s] = 0;
    }
    // each class runs this cycle on the plan of its systems in the cycle
    for (int k = 0; k < NC; ++k) {
      std::vector<int> sub;
      for (int s : B.classes[k])
        if (incyc[s]) sub.push_back(s);
      if (sub.empty() || (int)sub.size() == Pfull[k]->S) P[k] = Pfull[k];
      else BLP_TRY((get_subset_plan<TV, TR, SCALE>(B, k, sub, m, F, U, *Pfull[k], &P[k])));
      Pcyc[k] = P[k];
    }
    BLP_TRY(set_gates(incyc));
    BLP_TRY(fork(B));
    for (int k = 0; k < NC; ++k) {
      if (!live(k, incyc)) continue;
      const size_t n = B.sys[B.classes[k][0]]->p->n;
      k_normalize<TV><<<dim3(blocks1d(n), P[k]->S), 256, 0, cx[k].stream>>>(P[k]->kr, nullptr, 1);
      k_krylov_init<TV><<<P[k]->S, 64, 0, cx[k].stream>>>(P[k]->kr, ko);
    }
    BLP_TRY(join(B));
    for (int j = 0; j < m; ++j) {
      k_set_int<<<1, 1, 0, B.stream>>>(B.jdev, j);
      BLP_TRY(fork(B));
      if (o->precond) {
        // part 1 for every class, the corner check (further cycles while any
        // system's corner gate is open), then the rest of the step
        for (int k = 0; k < NC; ++k) {
          if (!live(k, incyc)) continue;
          if (use_graphs) {
            if (!P[k]->g1)
              BLP_TRY(capture(cx[k].stream, &P[k]->g1,
                              [&]() { prec_part1<TV, TR>(cx[k], P[k]->prec, B.jdev, po); }));
            HIP_TRY(hipGraphLaunch(P[k]->g1, cx[k].stream));
          } else {
            prec_part1<TV, TR>(cx[k], P[k]->prec, B.jdev, po);
          }
        }
        if (po.mg_fixed == 0) {
          int first = po.mg_maxcyc;
          for (int k = 0; k < NC; ++k) first = std::min(first, first_cycles(P[k]->prec));
          for (int extra = first; extra < po.mg_maxcyc; ++extra) {
            BLP_TRY(join(B));
            HIP_TRY(hipMemcpyAsync(B.ctrl_h, B.ctrl, S * sizeof(MgCtrl), hipMemcpyDeviceToHost,
                                   B.stream));
            HIP_TRY(hipStreamSynchronize(B.stream));
            // (systems outside the cycle keep their gate closed)
            bool open = false;
            for (int s = 0; s < S; ++s) open = open || (incyc[s] && !B.ctrl_h[s].gate);
            BLP_TRY(fork(B));
            if (!open) break;
            // (a class whose first enqueued cycles already reach this count
            // waits for the others)
            for (int k = 0; k < NC; ++k) {
              if (!live(k, incyc) || extra < first_cycles(P[k]->prec)) continue;
              corner_cycle<TV, TR>(cx[k], P[k]->prec);
            }
          }
        }
      } else {
        for (int k = 0; k < NC; ++k) {
          const size_t n = B.sys[B.classes[k][0]]->p->n;
          for (int q = 0; q < P[k]->S; ++q) {
            System &y = *B.sys[P[k]->idx[q]];
            TV *vj = (TV *)y.V + (size_t)j * n, *zj = (TV *)y.Z + (size_t)j * n;
            if (!incyc[P[k]->idx[q]]) continue;
            if (SCALE)
              k_div<TV><<<blocks1d(n), 256, 0, cx[k].stream>>>(vj, fine<TV>(y.p).dh, zj, n);
            else
              HIP_TRY(hipMemcpyAsync(zj, vj, n * sizeof(TV), hipMemcpyDeviceToDevice, cx[k].stream));
          }
        }
      }
      for (int k = 0; k < NC; ++k) {
        if (!live(k, incyc)) continue;
        auto rest = [&]() {
          if (o->precond) prec_part2<TV, TR>(cx[k], P[k]->prec, B.jdev);
          krylov_step<TV, TR, SCALE>(cx[k], *P[k], B.sys[B.classes[k][0]]->p->n1, j, B.jdev, ko);
        };
        if (use_graphs && o->precond) {
          if (!P[k]->g2) BLP_TRY(capture(cx[k].stream, &P[k]->g2, rest));
          HIP_TRY(hipGraphLaunch(P[k]->g2, cx[k].stream));
        } else {
          rest();
        }
      }
      BLP_TRY(join(B));
      BLP_TRY(read_all(B));
      bool any = false, left = false;
      for (int s = 0; s < S; ++s) {
        if (!incyc[s]) continue;
        ++it[s];
        ncol[s] = j + 1;
        if (o->precond) cs[s].add(B.ctrl_h[s].cycles);
        const double est = B.st_h[s].est;
        if (hist && hist[s] && !std::is_same<TV, float>::value) hist[s][it[s]] = est;
        if (!std::isfinite(est)) return BLP_E_NUMERIC;
        const bool happy = B.st_h[s].happy != 0;
        est_ok[s] = est <= target[s];
        if (est <= cyc_target[s] || happy || j + 1 >= m || it[s] >= o->maxit) {
          incyc[s] = 0;
          left = true;
        }
        any = any || incyc[s];
      }
      if (!any) break;
      // the device gates still equal incyc unless a system left the cycle
      if (left) {
        BLP_TRY(set_gates(incyc));
        for (int k = 0; k < NC; ++k) BLP_TRY(shrink(k));
      }
      BLP_TRY(fork(B));
      for (int k = 0; k < NC; ++k) {
        if (!live(k, incyc)) continue;
        const size_t n = B.sys[B.classes[k][0]]->p->n;
        k_normalize<TV><<<dim3(blocks1d(n), P[k]->S), 256, 0, cx[k].stream>>>(P[k]->kr, B.jdev, 0);
      }
      BLP_TRY(join(B));
    }
    // u += Z y and the true residual of every system of the cycle (on the
    // plan of the systems that started it); column counts in the plan's
    // record order (the kernel indexes its record's slot)
    P = Pcyc;
    BLP_TRY(set_gates(active));
    {
      int off = 0;
      for (int k = 0; k < NC; ++k)
        for (int q = 0; q < P[k]->S; ++q) B.ncol_h[off++] = ncol[P[k]->idx[q]];
      HIP_TRY(hipMemcpyAsync(B.ncol, B.ncol_h, S * sizeof(int), hipMemcpyHostToDevice, B.stream));
      BLP_TRY(fork(B));
      off = 0;
      for (int k = 0; k < NC; ++k) {
        if (live(k, active)) {
          const size_t n = B.sys[B.classes[k][0]]->p->n;
          k_update_solution<TV>
              <<<dim3(blocks1d(n), P[k]->S), 256, 0, cx[k].stream>>>(P[k]->kr, B.ncol + off, ko);
        }
        off += P[k]->S;
      }
      BLP_TRY(join(B));
    }
    BLP_TRY(residual());
    for (int s = 0; s < S; ++s) {
      if (!active[s]) continue;
      beta[s] = B.st_h[s].beta;
      ++restarts[s];
      if (hist && hist[s] && std::is_same<TV, float>::value)
        hist[s][std::min(it[s], o->maxit)] = beta[s];
      if (beta[s] <= target[s] || (o->stop_on_estimate && est_ok[s])) conv[s] = 1;
      if (!std::isfinite(beta[s])) return BLP_E_NUMERIC;
      active[s] = !conv[s] && it[s] < o->maxit;
    }
  }
  HIP_TRY(hipGetLastError());
  auto t1 = std::chrono::steady_clock::now();
  int rc = BLP_OK;
  for (int s = 0; s < S; ++s) {
    if (info) {
      blp_solve_info &I = info[s];
      I.iterations = it[s];
      I.restarts = restarts[s];
      I.converged = conv[s] ? 1 : 0;
      I.res = beta[s];
      I.norm_F = nF[s];
      I.mg_cycles_total = cs[s].total;
      I.mg_cycles_min = cs[s].applies ? cs[s].mn : 0;
      I.mg_cycles_max = cs[s].mx;
      I.solve_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    }
    if (!conv[s]) rc = BLP_W_NOCONV;
  }
  return rc;
}

int batch_solve(Batch &B, bool tr, const double *const *F, double *const *U, const blp_solve_opts *o,
                blp_solve_info *info, double *const *hist) {
  if (!o || !(o->tol > 0) || o->restart < 1 || o->restart > 60 || o->maxit < 1) return BLP_E_INVAL;
  if (o->precision != BLP_FP64 && o->precision != BLP_MIXED) return BLP_E_INVAL;
  // one corner stopping rule for the whole batch (its schedule is shared)
  const blp_prec_opts &q0 = B.sys[0]->p->popts;
  for (size_t s = 0; s < B.sys.size(); ++s) {
    if (!F[s] || !U[s]) return BLP_E_INVAL;
    const blp_prec_opts &q = B.sys[s]->p->popts;
    if (q.mg_fixed != q0.mg_fixed || q.mg_rtol != q0.mg_rtol || q.mg_maxcyc != q0.mg_maxcyc)
      return BLP_E_INVAL;
  }
  // a batch on its own stream starts after the caller's pending work (the
  // right-hand sides) and has finished when this returns
  if (B.own_stream) HIP_TRY(hipStreamSynchronize(B.user));
  const bool mixed = o->precision == BLP_MIXED, sc = o->scaled != 0;
  int rc;
#define BLP_DISPATCH(TV, TRB, SCB) rc = fgmres_batch<TV, TRB, SCB>(B, F, U, o, info, hist)
  if (mixed) {
    if (tr) { if (sc) BLP_DISPATCH(float, true, true); else BLP_DISPATCH(float, true, false); }
    else { if (sc) BLP_DISPATCH(float, false, true); else BLP_DISPATCH(float, false, false); }
  } else {
    if (tr) { if (sc) BLP_DISPATCH(double, true, true); else BLP_DISPATCH(double, true, false); }
    else { if (sc) BLP_DISPATCH(double, false, true); else BLP_DISPATCH(double, false, false); }
  }
#undef BLP_DISPATCH
  return rc;
}

// Text summary of the batch's classes and the kernel variants of its plans.
struct PlanInfo {
  int N, S, prec, tr, rows, varI, varLines;
  std::vector<int> varL;
};
template <typename TV, bool TR, bool SCALE>
bool plan_info(PlanBase *b, PlanInfo &I) {
  auto *h = dynamic_cast<PlanHolder<TV, TR, SCALE> *>(b);
  if (!h) return false;
  const auto &P = h->plan;
  I = PlanInfo{P.prec.N, P.S, (int)sizeof(TV), (int)TR, P.rows, P.prec.varI, P.prec.varLines,
               P.prec.varL};
  return true;
}
std::string describe(const Batch &B) {
  std::string out;
  char buf[256];
  for (size_t k = 0; k < B.classes.size(); ++k) {
    snprintf(buf, sizeof buf, "class %zu: N=%d systems=%zu\n", k, B.sys[B.classes[k][0]]->p->N,
             B.classes[k].size());
    out += buf;
  }
  for (const auto &kv : B.plans) {
    PlanInfo I;
    PlanBase *b = kv.second.get();
    if (!(plan_info<double, false, true>(b, I) || plan_info<double, false, false>(b, I) ||
          plan_info<double, true, true>(b, I) || plan_info<double, true, false>(b, I) ||
          plan_info<float, false, true>(b, I) || plan_info<float, false, false>(b, I) ||
          plan_info<float, true, true>(b, I) || plan_info<float, true, false>(b, I)))
      continue;
    snprintf(buf, sizeof buf, "plan N=%d systems=%d %s%s: interior sweep v%d, lines v%d, stencil rows %d, levels",
             I.N, I.S, I.prec == 8 ? "fp64" : "fp32", I.tr ? " transposed" : "", I.varI, I.varLines,
             I.rows);
    out += buf;
    for (int v : I.varL) {
      snprintf(buf, sizeof buf, " v%d", v);
      out += buf;
    }
    out += "\n";
  }
  return out;
}
