// Device-side building blocks shared by the solver kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define BLP_DEV __device__ __forceinline__

// A tensor grid with nx x ny unknowns (nodes 1..nx, 1..ny) and the per-axis
// tables of the upwind 5-point stencil (Sec. 3, 2D stencil):
//   W_i  = -eps/(hbar_i h_i)                 (coupling to i-1)
//   E_i  = -eps/(hbar_i h_{i+1}) - c1_i/h_{i+1}  (coupling to i+1)
//   Dx_i = -(W_i + E_i)                      (x part of the diagonal)
// and likewise S_j, N_j, Dy_j along y; the diagonal is C_ij = Dx_i + Dy_j + r_ij.
// Tables hold n+2 entries with zeros at index 0 and n+1, so a coupling to a
// node outside the grid reads as zero.  This separable form holds because
// c1 depends on x alone and c2 on y alone.
template <typename T>
struct Grid {
  int nx, ny;
  const T *W, *E, *Dx;  // x tables
  const T *S, *N, *Dy;  // y tables
  const T *r;           // nodal r, r[(j-1)*rld + (i-1)], or nullptr
  int rld;
  T rc;                 // constant r when r == nullptr
  BLP_DEV T rr(int i, int j) const { return r ? r[(size_t)(j - 1) * rld + (i - 1)] : rc; }
  BLP_DEV T C(int i, int j) const { return Dx[i] + Dy[j] + rr(i, j); }
};

BLP_DEV size_t vidx(int i, int j, int ld) { return (size_t)(j - 1) * ld + (i - 1); }

// Control block of one corner solve (device memory).
struct MgCtrl {
  int gate;          // 1 once the corner iteration has stopped
  int cycles;        // V-cycles performed in the current corner solve
  double bnorm2;     // ||S b||^2 (forward) or ||b||^2 (transposed)
  double res2;       // last corner residual norm^2
  double rtol2;      // (relative tolerance)^2
  int maxcyc;
  unsigned int counter;  // arrival counter of the reduction kernels
};

// Status block of the Krylov iteration (device memory, copied to the host).
struct KrylovStatus {
  double est;        // |g_{j+1}|, residual estimate after the last step
  double hn;         // h_{j+1,j}
  double wn0;        // ||w|| before orthogonalisation
  double beta;       // norm from the last residual / norm kernel
  int happy;         // breakdown flag of the last step
  int mg_cycles;     // corner cycles of the last preconditioner apply
  unsigned int counter;
  int pad;
};

// Wave-level sum of a double (wave64).
BLP_DEV double wave_sum(double v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

// Block sum (blockDim.x multiple of 64, at most 1024); result valid in all
// threads.  sh must hold 16 doubles.
BLP_DEV double block_sum(double v, double *sh) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int k = 0; k < nw; ++k) s += sh[k];
  return s;
}

// Pointers read from argument records in memory carry no address space, so
// the compiler would access them with FLAT instructions (which also count
// against the LDS counter).  Hot loops cast them to the global space.
#define BLP_GLOBAL __attribute__((address_space(1)))
template <typename T>
BLP_DEV BLP_GLOBAL T *gptr(T *p) {
  return (BLP_GLOBAL T *)p;
}

// Ordering point for the compiler only: no memory access is moved across
// it, and nothing waits for loads in flight.  Kernels that test a gate
// issue the gate's load and their data loads before this point and test the
// gate after it, so that those loads travel together instead of the data
// loads waiting for the gate.
#define BLP_ISSUED() asm volatile("" ::: "memory")

// "Last block" pattern: every block publishes its partial, then the last
// block to arrive reads all partials.  Partials are stored and read through
// to the device coherence point (relaxed agent-scope atomic accesses), and a
// block's arrival is counted only after its own partial store has completed
// (s_waitcnt vmcnt(0) before the counter increment), which orders the two
// without a device-scope fence: on this GPU such a fence writes back the
// whole L2 of the XCD, in every block.  Only thread 0 publishes.
BLP_DEV void publish(double *p, double v) {
  __hip_atomic_store(gptr(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
BLP_DEV double collect(const double *p) {
  return __hip_atomic_load(gptr(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Returns true in the whole last of nblocks arriving blocks.
BLP_DEV bool arrive_last(unsigned int *counter, bool *sh_flag, unsigned int nblocks) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_s_waitcnt(0 | (0x7 << 4) | (0xf << 8));  // vmcnt(0)
    const unsigned int prev =
        __hip_atomic_fetch_add(gptr(counter), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    *sh_flag = (prev == nblocks - 1);
    __builtin_amdgcn_s_waitcnt(0 | (0x7 << 4) | (0xf << 8));
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  }
  __syncthreads();
  return *sh_flag;
}
// Reset of an arrival counter by the last block (for the next launch).
BLP_DEV void reset_counter(unsigned int *counter) {
  __hip_atomic_store(gptr(counter), 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// XCD-aware block order.  The chip deals workgroups to its eight XCDs in
// turn (consecutive workgroup ids on consecutive XCDs), and each XCD has an
// L2 of its own.  In the skewed level layout the neighbours of a block's
// slots lie in the slot ranges of the adjacent blocks, so with the plain
// order every line is fetched once by each of three XCDs.  xcd_block maps
// the hardware block b of nb to a logical block such that the blocks on one
// XCD (equal b mod 8) take one contiguous range: XCD x gets nb / 8 blocks,
// one more when x < nb mod 8.  It is a permutation of 0 .. nb - 1 for any
// nb, so results do not depend on it; where blockIdx.y varies too, the
// grouping by b mod 8 still holds, only on rotated XCDs.
BLP_DEV int xcd_block(int b, int nb) {
  constexpr int X = 8;
  const int x = b % X, k = b / X, q = nb / X, r = nb % X;
  return x * q + (x < r ? x : r) + k;
}

// Batched launches: blockIdx.z (or the block's system slot) selects one
// system's argument record in a device array.  Vectors that change with the
// Krylov step are addressed as base + j * ld, with j read from device memory
// (jp; null means j = 0), so that the same launches (and captured graphs)
// serve every step.
BLP_DEV long long step_of(const int *jp) { return jp ? (long long)*jp : 0; }
// Per-system gate: nonzero means the system takes no part in the launch.
BLP_DEV bool gated(const int *g) { return g && *g; }
// The same two reads without a branch (a null pointer reads this zero word),
// so that they travel with the loads that follow them.
__device__ const int blp_zero_word = 0;
BLP_DEV int read_or_zero(const int *p) { return *gptr(p ? p : &blp_zero_word); }



// Grid with its tables in the global space (device-side view).
template <typename T>
struct GridG {
  int nx, ny;
  const BLP_GLOBAL T *W, *E, *Dx, *S, *N, *Dy, *r;
  int rld;
  T rc;
  BLP_DEV T rr(int i, int j) const { return r ? r[(size_t)(j - 1) * rld + (i - 1)] : rc; }
  BLP_DEV T C(int i, int j) const { return Dx[i] + Dy[j] + rr(i, j); }
};
template <typename T>
BLP_DEV GridG<T> gview(const Grid<T> &g) {
  return GridG<T>{g.nx,       g.ny,       gptr(g.W), gptr(g.E), gptr(g.Dx), gptr(g.S),
                  gptr(g.N), gptr(g.Dy), gptr(g.r), g.rld,     g.rc};
}
