// The downstream triangular sweep (wavefront, skewed layout) of the
// interior region and of the corner levels.  Included once, from
// kernels_prec.h, after the skewed-layout definitions it uses.
#pragma once

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
// Couplings to values outside the rectangle are already folded into rhs
// (k_gather_skew), so the sweep sees zero boundary values.
//
// rhs, 1/C and z are in the skewed layout of the rectangle.  One workgroup
// (or G of them, see sweep_body); wave w owns band w, lane l one column.  The
// upstream-column value comes from lane l-1 by a DPP shift (lane 0: from the
// previous band, through an LDS ring), the upstream-row value is the lane's
// own previous result.  Steps are processed K at a time (a superstep); band
// w needs band w-1 to be 64 + K steps ahead, which per-band progress
// counters in LDS ensure.
//
// Idle steps need no masking: padding slots hold rhs = 1/C = 0, so a lane
// whose row is not yet reached computes exactly 0 (the ring starts at zero),
// which is also the correct upstream value of the first row; steps past the
// last row land in padding.  A band works only on its own supersteps (local
// steps 0 .. its last node's step, rounded up to whole supersteps) and only
// joins the barriers before and after them.
//
// Memory pipelining: every access is one 16-byte chunk per lane; the K/P
// chunks of a superstep are consecutive, so one address per array and
// superstep serves them all (immediate offsets).  At the start of superstep m
// the wave stores the results of superstep m-1 and issues the loads of
// superstep m+D (clamped to the sink group) into the register buffer that
// superstep m-1 used (D+1 buffers, rotated by full unrolling), then computes
// superstep m.  A superstep issues 3K/P memory instructions, so the wait
// before superstep m covers operations issued D supersteps earlier, as long
// as 3DK/P stays within the 63 outstanding operations the counter can track.
//
// The wave issues one instruction at a time, so the schedule keeps the
// instructions per step few: aligned 16-byte LDS accesses for the ring and
// for the row-coupling table (held in P copies shifted by one word each, so
// that every lane's K consecutive entries start on a 16-byte boundary in one
// of them), and no per-chunk address arithmetic.
// ---------------------------------------------------------------------------
template <typename T>
struct SweepArgs {
  Grid<T> g;
  int i0, i1, j0, j1;
  const T *b;     // skewed rhs
  const T *ic;    // skewed 1/C (zero in padding)
  T *z;           // skewed result
  const int *gate;
  // split sweeps (several workgroups per system): per group boundary, the
  // channel of the writer band's last-column values (kChanStride words) and
  // the writer's and reader's launch counters (2 ints); zero-initialised
  unsigned long long *chan;
  int *epoch;
};

constexpr int kSweepMaxRows = 1024;  // also bounds the rows of the coupling table
constexpr int kSweepMaxBands = 16;
constexpr int kSweepMaxGroups = 4;  // workgroups per system of a split sweep
// channel words per group boundary: one tagged 32-bit piece per word, for
// every writer step of a band (at most kSweepMaxRows + 63 + 2 x 16)
constexpr int kChanSteps = kSweepMaxRows + 128;
template <typename T>
constexpr int kChanStride = kChanSteps * (int)(sizeof(T) / 4);
// bounded wait for a channel word (each round is one memory round trip)
constexpr int kChanSpin = 1 << 13;
// ring slots per band (the upstream band may run up to about ten supersteps
// ahead before it waits for its reader) and the bounded wait for a band's
// progress counter in LDS
constexpr int kRing = 128;
constexpr int kProgSpin = 1 << 22;

// Words per copy of the row-coupling table for rows rows (entries -64 ..
// rows + 63 + K of the row index, rounded up to whole chunks).
template <typename T, int K>
BLP_DEV constexpr int yc_stride(int rows) {
  return (rows + 128 + K + kChunk<T> - 1) / kChunk<T> * kChunk<T>;
}

// Workgroup barrier that waits for this wave's LDS traffic only (global
// loads and stores may stay in flight): s_waitcnt lgkmcnt(0) with vmcnt and
// expcnt at their maxima (GFX9 encoding 0xC07F), then s_barrier.  The empty
// asm statements keep the compiler from moving memory accesses across it.
BLP_DEV void lds_barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0xC07F);
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

template <typename T>
struct Vec16;
template <>
struct Vec16<double> { typedef double type __attribute__((ext_vector_type(2))); };
template <>
struct Vec16<float> { typedef float type __attribute__((ext_vector_type(4))); };

// Channel words: a 32-bit piece of a value with the writer's launch count
// in the high half, stored and loaded as one 64-bit word (relaxed,
// device scope), so that a word read either carries this launch's count and
// its piece, or an older count.
template <typename T>
BLP_DEV void chan_put(unsigned long long *w, T v, unsigned int tag) {
  if constexpr (sizeof(T) == 4) {
    const unsigned long long x = ((unsigned long long)tag << 32) | __float_as_uint(v);
    __hip_atomic_store(gptr(w), x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  } else {
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    __hip_atomic_store(gptr(w), ((unsigned long long)tag << 32) | (u & 0xffffffffull),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(gptr(w + 1), ((unsigned long long)tag << 32) | (u >> 32),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}
template <typename T>
struct ChanWord {
  unsigned long long w[sizeof(T) / 4];
};
template <typename T>
BLP_DEV ChanWord<T> chan_get(const unsigned long long *w) {
  ChanWord<T> c;
#pragma unroll
  for (int k = 0; k < (int)(sizeof(T) / 4); ++k)
    c.w[k] = __hip_atomic_load(gptr(w + k), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return c;
}
template <typename T>
BLP_DEV bool chan_ok(const ChanWord<T> &c, unsigned int tag) {
  bool ok = true;
#pragma unroll
  for (int k = 0; k < (int)(sizeof(T) / 4); ++k) ok = ok && (unsigned int)(c.w[k] >> 32) == tag;
  return ok;
}
template <typename T>
BLP_DEV T chan_value(const ChanWord<T> &c) {
  if constexpr (sizeof(T) == 4) {
    return __uint_as_float((unsigned int)c.w[0]);
  } else {
    return __longlong_as_double((long long)((c.w[0] & 0xffffffffull) | (c.w[1] << 32)));
  }
}

// The sweep of one workgroup: wave w is band band0 + w of the rectangle's
// nbt bands (G = 1: all of them).  ring holds (waves + 1) x kRing words, ycs
// kChunk<T> x yc_stride<T, K>(rows) words and prog one int per wave, all LDS,
// ring and ycs 16-byte aligned.
//
// The bands of a workgroup synchronise pairwise, not in lockstep: after a
// superstep a band publishes the number of supersteps it has completed in
// prog; before reading its ring a band waits until its upstream band has
// completed the superstep that holds the last step it needs, and before
// overwriting ring slots a band waits until its downstream band no longer
// needs them.  A wave's LDS operations are processed in order, so a count
// read by another wave implies the ring writes issued before it.  Both
// waits are bounded (kProgSpin rounds); a wait that runs out turns the
// band's values from there on into NaN, which the solver reports as a
// non-finite residual rather than returning a wrong result.
//
// Split sweeps (G > 1 workgroups per system, group gi taking bands gi x
// waves ..): the first band of group gi > 0 gets its upstream column from
// the last band of group gi - 1 through the channel instead of the LDS ring.
// The writer stores the K values of a superstep (one per lane); the reader
// requests them with its operand loads, D supersteps ahead, checks their
// launch count when it needs them (waiting, a bounded number of rounds, for
// any not yet written) and puts them into its ring row.  Only steps whose
// row exists need a value; after kChanSpin unanswered rounds the value is
// NaN, which the solver reports.  Groups run in block order (group 0 has the
// lowest block numbers), so a reader's writer has always started.
template <typename T, bool TR, int K, int D, int G>
BLP_DEV void sweep_body(const SweepArgs<T> &a, T *ring, T *ycs, int *prog, int tid, int nthreads,
                        int gi, int gate) {
  constexpr int P = kChunk<T>, CK = K / P, RING = kRing, NW = sizeof(T) / 4;
  static_assert(K % P == 0 && 64 % K == 0 && 2 * K + P <= 64 && CK <= kSkewGroup, "superstep length");
  typedef typename Vec16<T>::type V;
  const Grid<T> &g = a.g;
  const SkewT<T, TR> sk{a.i0, a.i1, a.j0, a.j1};
  const int mc = sk.mc(), mr = sk.mr(), nck = sk.nck();
  const int nbt = (mc + 63) >> 6;                                  // bands of the rectangle
  const int nw = __builtin_amdgcn_readfirstlane(nthreads >> 6);    // waves (bands) per group
  const int band0 = gi * nw;
  const int nbg = min(nw, nbt - band0);                            // bands of this group
  const int lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);         // wave-uniform
  const int band = band0 + wv;
  const bool has = wv < nbg;
  const int c = band * 64 + lane;
  const bool colok = c < mc;
  const int i = sk.icol(colok ? c : mc - 1);
  // upstream x coupling, read through a global (not generic) pointer before
  // the barrier below: a generic load still in flight at the first use inside
  // the step loop would make every iteration wait for all loads in flight
  // (every load of this prologue is unconditional, at an in-range index:
  // a load under a condition is waited for before the branch joins)
  const BLP_GLOBAL T *gE = gptr(g.E), *gN = gptr(g.N);
  const T cuv = TR ? gE[i - 1] : gE[i];
  const T cu = colok ? cuv : T(0);
  // row-coupling table: copy q (q < P) holds at word w the upstream y
  // coupling of row w + q - 64 (zero outside rows 0 .. mr - 1; those read
  // row 0).  One load per row, four in flight per thread, each value stored
  // into every copy.
  const int ys = yc_stride<T, K>(mr);
  for (int x0 = tid; x0 < ys + P - 1; x0 += 4 * nthreads) {
    T v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int t = x0 + u * nthreads - 64;
      const bool in = t >= 0 && t < mr;
      const int j = sk.jrow(in ? t : 0);
      const T val = TR ? gN[j - 1] : gN[j];
      v[u] = in ? val : T(0);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int x = x0 + u * nthreads;
#pragma unroll
      for (int q = 0; q < P; ++q) {
        const int w = x - q;
        if (w >= 0 && w < ys) ycs[q * ys + w] = v[u];
      }
    }
  }
  for (int q = tid; q < (nw + 1) * RING; q += nthreads) ring[q] = T(0);
  for (int q = tid; q < nw; q += nthreads) prog[q] = 0;
  // the gate (the same in every thread) was read with the loads above
  BLP_ISSUED();
  if (gate) return;
  __syncthreads();

  // the rectangle's last band holds mcl columns, so its last node is at
  // local step mr + mcl - 2; other bands end at mr + 62
  const int mcl = mc - (nbt - 1) * 64;
  auto last_step = [&](int bd) { return mr - 2 + (bd == nbt - 1 ? mcl : 64); };
  // this band's storage: chunk ck of this lane is element ck * 64
  const int bs = has ? band : band0;
  const BLP_GLOBAL V *__restrict__ bb = gptr(reinterpret_cast<const V *>(a.b + sk.slot(bs, 0, 0)) + lane);
  const BLP_GLOBAL V *__restrict__ bi = gptr(reinterpret_cast<const V *>(a.ic + sk.slot(bs, 0, 0)) + lane);
  BLP_GLOBAL V *__restrict__ zz = gptr(reinterpret_cast<V *>(a.z + sk.slot(bs, 0, 0)) + lane);
  T *ring_in_w = ring + wv * RING;
  const V *ring_in = reinterpret_cast<const V *>(ring_in_w);
  V *ring_out = reinterpret_cast<V *>(ring + (wv + 1) * RING);
  // last local step of this band that holds a node, and the last superstep
  // start at or below it
  const int lastl = __builtin_amdgcn_readfirstlane(last_step(band));
  const int shi = __builtin_amdgcn_readfirstlane(lastl / K * K);
  // the coupling of this lane at local step s is that of row s - lane, word
  // s + 64 - lane of copy 0, i.e. word s + 64 - lane - q of copy q with
  // q = (64 - lane) mod P: a multiple of P for every s that is
  const int yq = (64 - lane) & (P - 1);
  const V *yc_base = reinterpret_cast<const V *>(ycs + yq * ys + 64 - lane - yq);
  // group of K / P chunks that holds no node (loads past the band's end)
  const int sink = __builtin_amdgcn_readfirstlane(nck / CK - 1);
  // channel roles (split sweeps): the first wave of groups gi > 0 reads the
  // boundary gi - 1, the last band of groups gi < G - 1 writes boundary gi
  const bool reader = G > 1 && gi > 0 && wv == 0;
  const bool writer = G > 1 && gi < G - 1 && wv == nbg - 1 && band0 + nbg < nbt;
  unsigned long long *chw = nullptr, *chr = nullptr;
  unsigned int tagw = 0, tagr = 0;
  if (G > 1) {
    // both counters are read in every wave (at boundaries that exist)
    const BLP_GLOBAL int *ep = gptr(a.epoch);
    const int ew = ep[2 * min(gi, G - 2)], er = ep[2 * max(gi - 1, 0) + 1];
    if (writer) {
      chw = a.chan + (size_t)gi * kChanStride<T>;
      tagw = (unsigned int)ew + 1u;
    }
    if (reader) {
      chr = a.chan + (size_t)(gi - 1) * kChanStride<T>;
      tagr = (unsigned int)er + 1u;
    }
  }

  auto load = [&](int u, T (&Bb)[K], T (&Bi)[K], ChanWord<T> &Bc) {  // superstep u's operands
    const int ck = (u < sink ? u : sink) * CK;
    const BLP_GLOBAL V *pb = bb + ck * 64, *pi = bi + ck * 64;
#pragma unroll
    for (int q = 0; q < CK; ++q) {
      const V vb = pb[q * 64], vi = pi[q * 64];
#pragma unroll
      for (int e = 0; e < P; ++e) {
        Bb[q * P + e] = vb[e];
        Bi[q * P + e] = vi[e];
      }
    }
    // writer steps u K + 63 + lane (lanes < K) for the reader's ring
    if (G > 1 && reader) {
      const int st = min(u * K + 63 + (lane < K ? lane : 0), kChanSteps - 1);
      Bc = chan_get<T>(chr + (size_t)st * NW);
    }
  };
  auto store = [&](int u, const T (&R)[K]) {  // superstep u's results (u < 0: sink)
    BLP_GLOBAL V *pz = zz + (u < 0 ? sink : u) * CK * 64;
#pragma unroll
    for (int q = 0; q < CK; ++q) {
      V v;
#pragma unroll
      for (int e = 0; e < P; ++e) v[e] = R[q * P + e];
      pz[q * 64] = v;
    }
  };

  // supersteps with work of this band and of its upstream band (a full band:
  // last step rows + 62), and whether a downstream band of this workgroup
  // reads this band's ring
  const int nact = has ? __builtin_amdgcn_readfirstlane((lastl + K) / K) : 0;
  const int nact_up = (mr + 62 + K) / K;
  const bool down = wv + 1 < nbg;
  T buf_b[D + 1][K], buf_i[D + 1][K], res[K];
  ChanWord<T> buf_c[D + 1];
#pragma unroll
  for (int k = 0; k < K; ++k) res[k] = T(0);
  T z = T(0);  // this lane's latest result (the next row's upstream value)
  // superstep ml of this band: local steps ml K .. ml K + K - 1
  auto superstep = [&](int ml, T (&Cb)[K], T (&Ci)[K], ChanWord<T> &Cc, T (&Nb)[K], T (&Ni)[K],
                       ChanWord<T> &Nc) {
    const int sl = ml * K;
    store(ml - 1, res);
    load(ml + D, Nb, Ni, Nc);
    if (G > 1 && reader) {
      // the writer's steps sl + 63 .. sl + 63 + K - 1 into ring slots
      // (sl - 1 ..) mod 64; a step whose row does not exist (sl + lane >= mr)
      // needs no value
      if (lane < K) {
        T v = T(0);
        if (sl + lane < mr) {
          ChanWord<T> cw = Cc;
          int spin = 0;
          while (!chan_ok<T>(cw, tagr) && spin < kChanSpin) {
            __builtin_amdgcn_s_sleep(1);
            cw = chan_get<T>(chr + (size_t)(sl + 63 + lane) * NW);
            ++spin;
          }
          v = chan_ok<T>(cw, tagr) ? chan_value<T>(cw) : __builtin_nan("");
        }
        ring_in_w[(sl + 63 + lane) & (RING - 1)] = v;
      }
    }
    // the upstream band of this workgroup has written its steps up to
    // sl + K + 62 (those of its superstep (sl + K + 62) / K); past its last
    // active superstep the values only feed padding rows
    if (wv > 0) {
      const int need = min(ml + (K + 62) / K + 1, nact_up);
      int spin = 0;
      while (__hip_atomic_load(prog + wv - 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) < need &&
             spin < kProgSpin) {
        __builtin_amdgcn_s_sleep(1);
        ++spin;
      }
      asm volatile("" ::: "memory");
      // an expired wait would read stale ring values: poison this band's
      // chain instead, so that the solver reports a non-finite residual
      if (spin >= kProgSpin) z = __builtin_nan("");
    }
    // LDS operands of the superstep, read up front so that no LDS latency
    // sits on the step-to-step dependency chain.  The writer band stores
    // its local step s (lane 63) in ring slot s mod kRing; lane 0 of this
    // band, at local step s, needs the writer's step s + 63, slot (s - 1 +
    // 64) mod kRing.  The last superstep may pass the last row of every
    // lane: any finite coupling will do there.
    T yc[K], zb0[K];
    const V *yr = yc_base + (sl > shi ? shi : sl) / P;
#pragma unroll
    for (int q = 0; q < CK; ++q) {
      const V v = yr[q];
#pragma unroll
      for (int e = 0; e < P; ++e) yc[q * P + e] = v[e];
    }
    {
      const int r0 = ((sl + 64) & (RING - 1)) / P;
      const V pv = ring_in[(r0 + RING / P - 1) & (RING / P - 1)];
      zb0[0] = pv[P - 1];
#pragma unroll
      for (int q = 0; q < CK; ++q) {
        const V v = ring_in[r0 + q];
#pragma unroll
        for (int e = 0; e < P; ++e)
          if (q * P + e + 1 < K) zb0[q * P + e + 1] = v[e];
      }
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const T zin = dpp_mov<0x138>(zb0[k], z);  // lane l-1's value; lane 0: zb0
      z = (Cb[k] - yc[k] * z - cu * zin) * Ci[k];
      res[k] = z;
    }
    // the slots written here (steps sl .. sl + K - 1) last held steps
    // sl - kRing ..; the downstream band reads this band's steps from
    // c K + 64 - P on at its superstep c, so it must have completed every
    // superstep before the first c with c K + 64 - P > sl + K - 1 - kRing
    if (down) {
      const int need = (sl + K - RING - 64 + P + K - 1) / K;
      int spin = 0;
      while (need > 0 &&
             __hip_atomic_load(prog + wv + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) < need &&
             spin < kProgSpin) {
        __builtin_amdgcn_s_sleep(1);
        ++spin;
      }
      asm volatile("" ::: "memory");
      // an expired wait would overwrite ring slots the downstream band still
      // reads: publish NaN there (and carry it on) instead
      if (spin >= kProgSpin) {
        z = __builtin_nan("");
#pragma unroll
        for (int k = 0; k < K; ++k) res[k] = z;
      }
    }
    if (lane == 63) {
      const int r0 = (sl & (RING - 1)) / P;
#pragma unroll
      for (int q = 0; q < CK; ++q) {
        V v;
#pragma unroll
        for (int e = 0; e < P; ++e) v[e] = res[q * P + e];
        ring_out[r0 + q] = v;
      }
    }
    if (G > 1 && writer && lane < K) {
      // this wave's own ring writes above are complete before its reads
      const T v = reinterpret_cast<const T *>(ring_out)[(sl + lane) & (RING - 1)];
      chan_put<T>(chw + (size_t)(sl + lane) * NW, v, tagw);
    }
    asm volatile("" ::: "memory");
    if (lane == 0) __hip_atomic_store(prog + wv, ml + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  };
  // A band works on its supersteps 0 .. nact - 1 (local steps up to its last
  // node's); its first D supersteps of operands are requested at once, and
  // the step loop follows those loads directly, so that the compiler's wait
  // counts keep D supersteps of loads in flight.
  if (!has) return;
#pragma unroll
  for (int u = 0; u < D; ++u) load(u, buf_b[u], buf_i[u], buf_c[u]);
  // whole groups of D + 1 supersteps (buffer roles fixed by unrolling), then
  // the remaining supersteps outside the loop, so that no partially executed
  // group reaches the loop back edge
  int ml = 0;
  for (; ml + D < nact; ml += D + 1) {
#pragma unroll
    for (int u = 0; u <= D; ++u)
      superstep(ml + u, buf_b[u], buf_i[u], buf_c[u], buf_b[(u + D) % (D + 1)], buf_i[(u + D) % (D + 1)],
                buf_c[(u + D) % (D + 1)]);
  }
#pragma unroll
  for (int u = 0; u < D; ++u) {
    if (ml + u < nact)
      superstep(ml + u, buf_b[u], buf_i[u], buf_c[u], buf_b[(u + D) % (D + 1)], buf_i[(u + D) % (D + 1)],
                buf_c[(u + D) % (D + 1)]);
  }
  store(nact - 1, res);
  if (G > 1 && lane == 0) {
    if (writer) gptr(a.epoch)[2 * gi] = (int)tagw;
    if (reader) gptr(a.epoch)[2 * (gi - 1) + 1] = (int)tagr;
  }
}

// G workgroups per system (blocks g x S + s: every group-0 block precedes
// every group-1 block); the rectangle's bands are split evenly.
template <typename T, bool TR, int K, int D, int G>
__global__ __launch_bounds__(D > 1 ? 512 : 1024) void k_sweep(const SweepArgs<T> *A) {
  const int S = gridDim.x / G, gi = blockIdx.x / S;
  const SweepArgs<T> a = A[blockIdx.x - gi * S];
  const int gate = read_or_zero(a.gate);  // tested once the first loads are issued
  __shared__ __align__(16) T ring[(kSweepMaxBands + 1) * kRing];
  __shared__ __align__(16) T ycs[kChunk<T> * yc_stride<T, K>(kSweepMaxRows)];
  __shared__ int prog[kSweepMaxBands];
  sweep_body<T, TR, K, D, G>(a, ring, ycs, prog, threadIdx.x, blockDim.x, gi, gate);
}
