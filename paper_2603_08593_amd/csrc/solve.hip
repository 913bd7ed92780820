// sfft_solve: FP64 solve of the normal equations G theta = h.
//
// The SFFT fit ends in a dense symmetric positive-definite solve (the
// least-squares normal equations of the delta-basis kernel, paper Sec. 1).
// One persistent kernel with P co-resident workgroups (one per CU) does:
//   equilibration  A = D G D, D = diag(G)^-1/2, v = D h;
//   right-looking blocked Cholesky on 64 x 64 tiles of the matrix augmented
//   below by the right-hand side row v^T and by the identity: factorising
//   [A; v^T; I] turns those rows into z^T = (L^-1 v)^T and L^-T, so the
//   forward substitution and the inverse factor come out of the same sweep;
//   the factorisation is a dataflow between two roles. Workgroup 0 runs the
//   diagonal chain: it factors diagonal tile k (L_kk and U_k = L_kk^-T in
//   one sweep), computes the next panel tile L_(k+1),k = A_(k+1),k U_k and
//   applies its update to diagonal tile k + 1, which it keeps in LDS, then
//   factors that one. The other workgroups compute the remaining panel
//   tiles of step k and apply its remaining trailing updates, one step
//   behind the chain. The roles synchronise through per-workgroup progress
//   flags, never through a barrier of the whole team, so the chain's
//   critical path is factor -> one panel tile -> one update per step;
//   x = L^-T z as one distributed matrix-vector product; up to `refine`
//   steps of iterative refinement on r = h - G theta (FP64), each three
//   matrix-vector products (G theta, L^-1 r = (L^-T)^T r, L^-T z);
//   final backward error and pivot range.
// Workgroups synchronise through flags (release fence + relaxed store;
// relaxed polling + one acquire fence) with bounded spins: a timeout is
// reported in the status instead of hanging.
#include <algorithm>
#include <new>
#include <vector>

#include "batch.hpp"
#include "common.hpp"
#include "layout.hpp"

namespace sfft {

constexpr int kPT = 512;                    // threads per solve workgroup
constexpr int kPlainTeam = 128;             // team of the single-pair solve
constexpr long kSpinLimit = 1L << 26;
constexpr int kLD = kTile + 1;              // LDS row pitch of a tile

struct PSArgs {
  const double* G;
  const double* h;
  double* coef;
  sfft_solve_info* info;
  double* A;        // (2 Np + 64) x Np working matrix: rows [0, Np) matrix,
                    // its diagonal tiles -> L_kk; row Np: v; rows
                    // [Np + 64, 2 Np + 64): identity
  double* s;        // Np
  double* x;        // Np
  double* theta;    // Np
  double* r;        // Np
  double* rowabs;   // Np
  double* Z;        // (Np + 64) x Np: row 0: z = L^-1 v; rows [64, Np + 64): L^-T
  double* Ud;       // nt tiles of 64 x 64: U_k = L_kk^-T of each diagonal tile
  double* part;     // partial sums of gemv_upper_t
  unsigned* sync;   // [0, P): arrival flags, [P]: release flag
  unsigned* prog;   // [0, P): factorisation progress of every workgroup
  unsigned long long* stamps;   // optional 100 MHz time stamps: [0, 128) team
                                // barriers, [128 + 2k] diagonal tile k factored,
                                // [129 + 2k] the chain's step k done
  int* flags;       // [0] nonfinite (build), [1] failed pivot + 1, [2] barrier timeout
  int N, Np, nt, P, refine;
};

// Grid barrier: release fence + relaxed arrival flag per workgroup;
// workgroup 0 polls all arrival flags (relaxed loads, short sleeps), then
// releases everyone through one flag; a single acquire fence after each wait.
// Polling never uses acquire loads, which would invalidate caches on every
// iteration. Spins are bounded; a timeout is recorded in flags[2].
struct Barrier {
  unsigned gen = 0;
  int bid = 0;        // workgroup index within the solve's team
  __device__ void wait(const PSArgs& a) {
    __syncthreads();
    ++gen;
    if (threadIdx.x == 0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __hip_atomic_store(&a.sync[bid], gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (bid == 0) {
      if (threadIdx.x < a.P) {
        long spins = 0;
        while (__hip_atomic_load(&a.sync[threadIdx.x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < gen) {
          __builtin_amdgcn_s_sleep(1);
          if (++spins > kSpinLimit) { atomicOr(&a.flags[2], 1); break; }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_store(&a.sync[a.P], gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    } else if (threadIdx.x == 0) {
      long spins = 0;
      while (__hip_atomic_load(&a.sync[a.P], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < gen) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins > kSpinLimit) { atomicOr(&a.flags[2], 1); break; }
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
    if (bid == 0 && threadIdx.x == 0 && a.stamps && gen < 128)
      a.stamps[gen] = __builtin_amdgcn_s_memrealtime();
  }
};

__device__ __forceinline__ bool failed(const PSArgs& a) {
  return __hip_atomic_load(&a.flags[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}

// true when the factorisation stopped at diagonal tile k or earlier (the
// failing pivot index + 1 is recorded in flags[1])
__device__ __forceinline__ bool failed_by(const PSArgs& a, int k) {
  const int f = __hip_atomic_load(&a.flags[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return f != 0 && (f - 1) / kTile <= k;
}

// Progress flags of the factorisation, one monotonic word per workgroup.
// Workgroup 0 (diagonal chain): 2k + 1 once L_kk and U_k of step k are
// stored. Workgroups 1 .. P-1: 2k + 2 after their bulk work of step k; in
// the two-phase bulk of the batched solve also 2k + 1 after their panel
// tiles of step k. All stores of the workgroup precede the flag (barrier,
// then a release fence by the storing thread).
__device__ __forceinline__ void publish(const PSArgs& a, int bid, unsigned val) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_store(&a.prog[bid], val, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Waits until workgroup 0's flag is >= want0 and every other workgroup's
// flag is >= want (thread b polls the flag of workgroup b with relaxed
// loads; one acquire fence after its wait). Bounded: a timeout is recorded
// in flags[2] and the caller goes on.
__device__ __forceinline__ void wait_progress(const PSArgs& a, unsigned want0, unsigned want) {
  const int t = threadIdx.x;
  if (t < a.P) {
    const unsigned w = (t == 0) ? want0 : want;
    long spins = 0;
    while (__hip_atomic_load(&a.prog[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < w) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins > kSpinLimit) { atomicOr(&a.flags[2], 1); break; }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
}

// time stamp of a diagonal-chain event (workgroup 0)
__device__ __forceinline__ void stamp(const PSArgs& a, int slot) {
  if (threadIdx.x == 0 && a.stamps && slot < 256) a.stamps[slot] = __builtin_amdgcn_s_memrealtime();
}

// ---------------------------------------------------------------------------
// tile helpers (512 threads)
// ---------------------------------------------------------------------------

constexpr int kPerThread = kTile * kTile / kPT;   // tile elements per thread

// rows [r0, r0 + rows) x columns [c0, c0 + 64) of a row-major matrix with
// leading dimension ld into an LDS tile (zeros below `rows`): every global
// load of the thread is issued before the first LDS store, so one memory
// latency is paid per tile instead of one per element
__device__ __forceinline__ void tile_in(double (*T)[kLD], const double* A, int64_t ld, int64_t r0, int64_t c0,
                                        int rows = kTile) {
  double v[kPerThread];
#pragma unroll
  for (int t = 0; t < kPerThread; ++t) {
    const int idx = threadIdx.x + t * kPT;
    const int i = idx >> 6, j = idx & 63;
    v[t] = (i < rows) ? A[(r0 + i) * ld + c0 + j] : 0.0;
  }
#pragma unroll
  for (int t = 0; t < kPerThread; ++t) {
    const int idx = threadIdx.x + t * kPT;
    T[idx >> 6][idx & 63] = v[t];
  }
}

__device__ __forceinline__ void tile_out(const double (*T)[kLD], double* A, int64_t ld, int64_t r0, int64_t c0,
                                         int rows = kTile) {
  double v[kPerThread];
#pragma unroll
  for (int t = 0; t < kPerThread; ++t) {
    const int idx = threadIdx.x + t * kPT;
    v[t] = T[idx >> 6][idx & 63];
  }
#pragma unroll
  for (int t = 0; t < kPerThread; ++t) {
    const int idx = threadIdx.x + t * kPT;
    const int i = idx >> 6, j = idx & 63;
    if (i < rows) A[(r0 + i) * ld + c0 + j] = v[t];
  }
}

// the two halves of tile_in, for issuing the loads of several tiles before
// the first LDS store
__device__ __forceinline__ void tile_gather(double (&v)[kPerThread], const double* A, int64_t ld, int64_t r0,
                                            int64_t c0, int rows = kTile) {
#pragma unroll
  for (int t = 0; t < kPerThread; ++t) {
    const int idx = threadIdx.x + t * kPT;
    const int i = idx >> 6, j = idx & 63;
    v[t] = (i < rows) ? A[(r0 + i) * ld + c0 + j] : 0.0;
  }
}

__device__ __forceinline__ void tile_scatter(double (*T)[kLD], const double (&v)[kPerThread]) {
#pragma unroll
  for (int t = 0; t < kPerThread; ++t) {
    const int idx = threadIdx.x + t * kPT;
    T[idx >> 6][idx & 63] = v[t];
  }
}

__device__ __forceinline__ void load_tile(double (*T)[kLD], const double* A, int Np, int ti, int tj,
                                          int rows = kTile) {
  tile_in(T, A, Np, (int64_t)ti * kTile, (int64_t)tj * kTile, rows);
}

__device__ __forceinline__ void store_tile(const double (*T)[kLD], double* A, int Np, int ti, int tj,
                                           int rows = kTile) {
  tile_out(T, A, Np, (int64_t)ti * kTile, (int64_t)tj * kTile, rows);
}

typedef double double4_t __attribute__((ext_vector_type(4)));

// 64 x 64 x 64 tile products on the FP64 matrix cores
// (v_mfma_f64_16x16x4f64): wave w owns rows 16 (w & 3) .. +16 and columns
// 32 (w >> 2) .. +32 of the result, as two 16 x 16 blocks. Operand lanes:
// A[l % 16][l / 16], B[l / 16][l % 16]; result lane l, element q:
// row l / 16 + 4 q, column l % 16.
// TRANS_B = true: acc = X Y^T; false: acc = X Y. UPPER_Y: Y is upper
// triangular, so columns j0 .. j0 + 31 need rows k < j0 + 32 only (a wave
// pair sharing a SIMD, w and w + 4, does 24 of the 32 k-steps of the full
// product).
template <bool TRANS_B, bool UPPER_Y = false>
__device__ __forceinline__ void tile_mma(const double (*X)[kLD], const double (*Y)[kLD],
                                         double4_t acc[2]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i0 = 16 * (w & 3), j0 = 32 * (w >> 2);
  const int lr = lane & 15, lk = lane >> 4;
  acc[0] = double4_t{0.0, 0.0, 0.0, 0.0};
  acc[1] = double4_t{0.0, 0.0, 0.0, 0.0};
  const int kend = UPPER_Y ? j0 + 32 : kTile;
#pragma unroll 4
  for (int k = 0; k < kend; k += 4) {
    const double av = X[i0 + lr][k + lk];
    const double b0 = TRANS_B ? Y[j0 + lr][k + lk] : Y[k + lk][j0 + lr];
    const double b1 = TRANS_B ? Y[j0 + 16 + lr][k + lk] : Y[k + lk][j0 + 16 + lr];
    acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, b0, acc[0], 0, 0, 0);
    acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, b1, acc[1], 0, 0, 0);
  }
}

// C -= X Y^T (all 64 x 64 in LDS; C may not alias X or Y)
__device__ __forceinline__ void tile_sub_abt(double (*C)[kLD], const double (*X)[kLD],
                                             const double (*Y)[kLD]) {
  double4_t acc[2];
  tile_mma<true>(X, Y, acc);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i0 = 16 * (w & 3) + (lane >> 4), j0 = 32 * (w >> 2) + (lane & 15);
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int q = 0; q < 4; ++q) C[i0 + 4 * q][j0 + 16 * b] -= acc[b][q];
  __syncthreads();
}

// C = C U (U upper triangular, not aliasing C)
__device__ __forceinline__ void tile_mul_inplace(double (*C)[kLD], const double (*U)[kLD]) {
  double4_t acc[2];
  tile_mma<false, true>(C, U, acc);
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i0 = 16 * (w & 3) + (lane >> 4), j0 = 32 * (w >> 2) + (lane & 15);
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int q = 0; q < 4; ++q) C[i0 + 4 * q][j0 + 16 * b] = acc[b][q];
  __syncthreads();
}

// Workgroup barrier that orders LDS accesses only: unlike __syncthreads it
// does not wait for the thread's outstanding global loads, so loads issued
// before it stay in flight across it (their consumers wait for them).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// 1 / sqrt(d): hardware estimate refined by one Newton step (relative error
// far below what the iterative refinement corrects)
__device__ __forceinline__ double rsqrt64(double d) {
  const double y = __builtin_amdgcn_rsq(d);
  return y * fma(-0.5 * d * y, y, 1.5);
}

// value of x in lane `lane` (uniform result)
__device__ __forceinline__ double lane_value(double x, int lane) {
  const long long b = __builtin_bit_cast(long long, x);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}

// Column phase of block jb (wave 0; lane i = row i of T and of Y): the
// block's 8 entries of both rows stay in registers while its 8 columns are
// factored one by one; pivots and the entries of L that update the rest of
// the block come from other lanes by readlane, so the column chain never
// waits on LDS; column j of L is written to T and the block of Y to Ut.
__device__ __forceinline__ void potrf_columns(double (*T)[kLD], double (*Ut)[kLD], int jb, int& f) {
  constexpr int kB = 8;
  const int i = threadIdx.x & 63;
  const int j0 = jb * kB;
  double rb[kB], yb[kB];
#pragma unroll
  for (int c = 0; c < kB; ++c) {
    rb[c] = T[i][j0 + c];
    yb[c] = Ut[i][j0 + c];
  }
#pragma unroll
  for (int c = 0; c < kB; ++c) {
    const int j = j0 + c;
    const double d = lane_value(rb[c], j);
    const bool good = (d > 0.0) && is_finite_d(d);
    f = (f < 0 && !good) ? j : f;
    // branch-free: the estimate is always computed, then masked to 0
    const long long keep = -(long long)good;
    const double rs = __builtin_bit_cast(double, __builtin_bit_cast(long long, rsqrt64(d)) & keep);
    const double l = (i >= j) ? rb[c] * rs : 0.0;
    const double y = yb[c] * rs;
    rb[c] = l;
    yb[c] = y;
#pragma unroll
    for (int c2 = c + 1; c2 < kB; ++c2) {
      const double lm = lane_value(l, j0 + c2);     // L[j0 + c2][j]
      rb[c2] = fma(-l, lm, rb[c2]);
      yb[c2] = fma(-y, lm, yb[c2]);
    }
  }
#pragma unroll
  for (int c = 0; c < kB; ++c) {
    T[i][j0 + c] = rb[c];
    Ut[i][j0 + c] = yb[c];
  }
}

// Rank-8 update of columns m = m0, m0 + step, ... < m1 of T and of Y with
// block jb (all 64 rows; lane = row), two columns per iteration. The wave
// holds the block's rows of L in registers, so the multipliers L[m][j] come
// by readlane from lane m instead of LDS broadcasts (m is wave-uniform).
__device__ __forceinline__ void potrf_update(double (*T)[kLD], double (*Ut)[kLD], int jb, int m0, int m1,
                                             int step) {
  constexpr int kB = 8;
  const int i = threadIdx.x & 63;
  const int j0 = jb * kB;
  double li[kB], yi[kB];
#pragma unroll
  for (int c = 0; c < kB; ++c) {
    li[c] = T[i][j0 + c];
    yi[c] = Ut[i][j0 + c];
  }
  int m = m0;
  for (; m + step < m1; m += 2 * step) {
    const int m2 = m + step;
    double t = T[i][m], u = Ut[i][m], t2 = T[i][m2], u2 = Ut[i][m2];
#pragma unroll
    for (int c = 0; c < kB; ++c) {
      const double lm = lane_value(li[c], m), lm2 = lane_value(li[c], m2);   // L[m][j], L[m2][j]
      t = fma(-li[c], lm, t);
      u = fma(-yi[c], lm, u);
      t2 = fma(-li[c], lm2, t2);
      u2 = fma(-yi[c], lm2, u2);
    }
    T[i][m] = t;
    Ut[i][m] = u;
    T[i][m2] = t2;
    Ut[i][m2] = u2;
  }
  if (m < m1) {
    double t = T[i][m], u = Ut[i][m];
#pragma unroll
    for (int c = 0; c < kB; ++c) {
      const double lm = lane_value(li[c], m);
      t = fma(-li[c], lm, t);
      u = fma(-yi[c], lm, u);
    }
    T[i][m] = t;
    Ut[i][m] = u;
  }
}

// Cholesky of the 64 x 64 SPD tile T (lower, in place) and U = L^-T into Ut.
// The right-looking factorisation of the stacked [T; I] turns the identity
// rows into L^-T (I = Y L^T); Ut starts as the identity and holds Y. Blocked
// by 8 columns and software-pipelined over the 8 waves, two barriers per
// block: while wave 0 runs the column phase of block jb (potrf_columns),
// waves 1-7 apply block jb - 1's update to columns j0 + 8 .. 63; then all 8
// waves apply block jb's update to the next block's 8 columns (one each),
// which is all the next column phase waits for.
// `mid()` runs (in every thread) before block kMidBlock: the caller's point
// to start global loads that complete during the rest of the sweep (the
// sweep's barriers order LDS only, so they do not wait for those loads).
// A pivot that is not positive and finite is recorded (the first one) and
// the sweep goes on with a zero scale, so values stay finite; the caller
// discards them. Returns the failing local pivot or -1.
constexpr int kMidBlock = 7;

template <class Mid>
__device__ __forceinline__ int tile_potrf_aug(double (*T)[kLD], double (*Ut)[kLD], Mid&& mid) {
  constexpr int kB = 8, kNB = kTile / kB;
  __shared__ int fail;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (threadIdx.x == 0) fail = -1;
  for (int idx = threadIdx.x; idx < kTile * kTile; idx += kPT)
    Ut[idx >> 6][idx & 63] = ((idx >> 6) == (idx & 63)) ? 1.0 : 0.0;
  __syncthreads();
  int f = -1;
  auto block = [&](int jb) {
    const int j0 = jb * kB;
    if (w == 0) potrf_columns(T, Ut, jb, f);
    else if (jb > 0) potrf_update(T, Ut, jb - 1, j0 + kB + (w - 1), kTile, kPT / 64 - 1);
    lds_barrier();
    if (jb + 1 < kNB) {
      potrf_update(T, Ut, jb, j0 + kB + w, j0 + kB + w + 1, 1);
      lds_barrier();
    }
  };
  // two loops, so that registers loaded by mid() stay live across the second
  // without loop-carried copies (which would wait for the loads)
#pragma unroll 1
  for (int jb = 0; jb < kMidBlock; ++jb) block(jb);
  mid();
#pragma unroll 1
  for (int jb = kMidBlock; jb < kNB; ++jb) block(jb);
  for (int idx = threadIdx.x; idx < kTile * kTile; idx += kPT)
    if ((idx & 63) > (idx >> 6)) T[idx >> 6][idx & 63] = 0.0;
  if (threadIdx.x == 0) fail = f;
  __syncthreads();
  return fail;
}

// lower-triangle tile index t -> (ti, tj) with tj <= ti
__device__ __forceinline__ void tri_decode(int t, int& ti, int& tj) {
  ti = 0;
  while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
  tj = t - ti * (ti + 1) / 2;
}

// global row offset of row tile t: [0, nt) matrix, nt: the v row,
// nt + 1 + i: identity rows of block i
__device__ __forceinline__ int64_t row_off(int t, int nt, int Np) {
  return t < nt ? (int64_t)t * kTile : (t == nt ? (int64_t)Np : (int64_t)Np + kTile + (int64_t)(t - nt - 1) * kTile);
}

__device__ __forceinline__ void load_tile_r(double (*T)[kLD], const double* A, int Np, int64_t r0, int tj,
                                            int rows = kTile) {
  tile_in(T, A, Np, r0, (int64_t)tj * kTile, rows);
}
__device__ __forceinline__ void store_tile_r(const double (*T)[kLD], double* A, int Np, int64_t r0, int tj,
                                             int rows = kTile) {
  tile_out(T, A, Np, r0, (int64_t)tj * kTile, rows);
}

// Sum over j = j0 + lane + 64 u < n of x[j] y[j] (per lane, ascending j):
// the loads of 8 strides are issued together, one memory round trip per 512
// elements.
__device__ __forceinline__ double lane_dot(const double* x, const double* y, int j0, int n) {
  const int lane = threadIdx.x & 63;
  double acc = 0.0;
  for (int jb = j0; jb < n; jb += 64 * 8) {
    double xv[8], yv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int j = jb + 64 * u + lane;
      xv[u] = j < n ? x[j] : 0.0;
      yv[u] = j < n ? y[j] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) acc = fma(xv[u], yv[u], acc);
  }
  return acc;
}

// y_i = sum_j U[i][j] in_j with U = L^-T (upper triangular: j >= i); one
// row per wave; theta_i = s_i y_i, or theta_i += s_i y_i when `accumulate`.
__device__ void gemv_upper_theta(const PSArgs& a, const double* in, bool accumulate, int bid) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nw = kPT / 64;
  const double* U = a.Z + (int64_t)kTile * a.Np;
  for (int i = bid * nw + wave; i < a.Np; i += a.P * nw) {
    double acc = lane_dot(U + (int64_t)i * a.Np, in, i & ~63, a.Np);
    acc = wave_sum(acc);
    if (lane == 0) a.theta[i] = (accumulate ? a.theta[i] : 0.0) + a.s[i] * acc;
  }
}

// out_j = sum_{i <= j} U[i][j] in_i (U^T = L^-1, lower). The rows are cut
// into chunks; wave (column block cb, chunk ch) sums its chunk for the 64
// columns of the block (one column per lane, coalesced row reads, 8 rows
// per memory round trip) into part[ch][j]; after a barrier the chunks are
// added in order.
__device__ void gemv_upper_t(const PSArgs& a, const double* in, double* out, int bid, Barrier& bar) {
  const double* U = a.Z + (int64_t)kTile * a.Np;
  const int lane = threadIdx.x & 63;
  const int nw = kPT / 64;
  const int ncb = a.Np / 64;
  const int nwaves = a.P * nw;
  const int nch = nwaves >= ncb ? nwaves / ncb : 1;
  const int len = (a.Np + nch - 1) / nch;
  for (int gw = bid * nw + (threadIdx.x >> 6); gw < ncb * nch; gw += nwaves) {
    const int cb = gw % ncb, ch = gw / ncb;
    const int j = cb * 64 + lane;
    const int i0 = ch * len;
    const int i1 = min(min(i0 + len, a.Np), cb * 64 + 64);
    double acc = 0.0;
    for (int ib = i0; ib < i1; ib += 8) {
      double uv[8], iv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int i = ib + u;
        uv[u] = i < i1 ? U[(int64_t)i * a.Np + j] : 0.0;
        iv[u] = i < i1 ? in[i] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int i = ib + u;
        acc = (i < i1 && i <= j) ? fma(uv[u], iv[u], acc) : acc;
      }
    }
    a.part[(int64_t)ch * a.Np + j] = acc;
  }
  bar.wait(a);
  for (int j = bid * kPT + threadIdx.x; j < a.Np; j += a.P * kPT) {
    double s = 0.0;
    for (int cb = 0; cb < nch; cb += 8) {
      double pv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) pv[u] = (cb + u < nch) ? a.part[(int64_t)(cb + u) * a.Np + j] : 0.0;
#pragma unroll
      for (int u = 0; u < 8; ++u) s += pv[u];
    }
    out[j] = s;
  }
}

// r = D (h - G theta), one row per wave, rows spread over all workgroups
__device__ void residual(const PSArgs& a, int bid) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nw = kPT / 64;
  for (int i = bid * nw + wave; i < a.Np; i += a.P * nw) {
    if (i >= a.N) {
      if (lane == 0) a.r[i] = 0.0;
      continue;
    }
    double sacc = lane_dot(a.G + (int64_t)i * a.N, a.theta, 0, a.N);
    sacc = wave_sum(sacc);
    if (lane == 0) a.r[i] = a.s[i] * (a.h[i] - sacc);
  }
}

// The bulk work of step k, shared by `nb` workgroups (this one: `q`).
// Task (r, J) updates tile (r, J) with the panel tiles it needs, computed
// on the spot: A_rJ -= X_rk X_Jk^T with X_rk = A_rk U_k (every input tile
// has the updates of steps < k). Tasks, in row-major order: the matrix
// tiles k + 1 <= J <= r < nt except the diagonal tile (k + 1, k + 1), which
// the chain updates; the v row and the identity rows of blocks i <= k, for
// J in [k + 1, nt). Each workgroup takes a contiguous range, so consecutive
// tasks of one row share X_rk, computed once.
// The v row's and the identity rows' panel tiles are final results: their
// J = k + 1 task stores them in Z (at the last step, k = nt - 1, they are the
// only tasks), never over the input tile, which the row's other tasks of the
// step still read; the matrix panel tiles are not needed after the step.
__device__ __forceinline__ void bulk_step(const PSArgs& a, int k, int q, int nb, double (*TU)[kLD],
                                          double (*TX)[kLD], double (*TL)[kLD], double (*TC)[kLD]) {
  const int nt = a.nt, Np = a.Np;
  const int m = nt - k - 1;
  const int ntri = m * (m + 1) / 2;
  const int nrow = k + 2;                       // v row + identity rows 0..k
  const int t0 = m > 0 ? 1 : 0;
  const int ntot = m > 0 ? ntri + nrow * m : nrow;
  const int tb = t0 + (int)((int64_t)(ntot - t0) * q / nb);
  const int te = t0 + (int)((int64_t)(ntot - t0) * (q + 1) / nb);
  bool have_u = false;
  int xrow = -1;                                // row tile whose X_rk is in TX
  for (int t = tb; t < te; ++t) {
    int rt, J;
    if (m == 0) {
      rt = nt + t;                              // panel only
      J = -1;
    } else if (t < ntri) {
      int ti, tj;
      tri_decode(t, ti, tj);
      rt = k + 1 + ti;
      J = k + 1 + tj;
    } else {
      const int u = t - ntri;
      rt = nt + u / m;
      J = k + 1 + u % m;
    }
    const int rows = (rt == nt) ? 1 : kTile;
    const int64_t r0 = row_off(rt, nt, Np);
    const bool diag = (J == rt);
    const bool new_x = (rt != xrow);
    {
      // one memory round trip for all the task's tiles
      double vu[kPerThread], vx[kPerThread], vc[kPerThread], vl[kPerThread];
      if (!have_u) tile_gather(vu, a.Ud + (int64_t)k * kTile * kTile, kTile, 0, 0);
      if (new_x) tile_gather(vx, a.A, Np, r0, (int64_t)k * kTile, rows);
      if (J >= 0) {
        tile_gather(vc, a.A, Np, r0, (int64_t)J * kTile, rows);
        if (!diag) tile_gather(vl, a.A, Np, (int64_t)J * kTile, (int64_t)k * kTile);
      }
      if (!have_u) tile_scatter(TU, vu);
      if (new_x) tile_scatter(TX, vx);
      if (J >= 0) {
        tile_scatter(TC, vc);
        if (!diag) tile_scatter(TL, vl);
      }
    }
    have_u = true;
    __syncthreads();
    if (new_x) {
      tile_mul_inplace(TX, TU);                 // X_rk
      if (rt >= nt && J <= k + 1) tile_out(TX, a.Z, Np, r0 - Np, (int64_t)k * kTile, rows);
      xrow = rt;
    }
    if (J >= 0) {
      if (!diag) tile_mul_inplace(TL, TU);      // X_Jk
      tile_sub_abt(TC, TX, diag ? TX : TL);
      store_tile_r(TC, a.A, Np, r0, J, rows);
    }
    __syncthreads();
  }
}

// The bulk work of step k in two phases (the batched solve, which is bound
// by the bulk's throughput rather than by the diagonal chain). Panels: the
// tiles X_rk = A_rk U_k of the matrix rows k + 1 <= r < nt, written over
// A_rk (read by nothing after step k), and of the v row and the identity
// rows of blocks i <= k, written to Z (their final results); each computed
// once, by one workgroup. Updates, after every bulk workgroup has finished
// its panels: A_rJ -= X_rk X_Jk^T over the same task list as bulk_step,
// with both panel tiles loaded instead of computed (one tile product per
// task instead of up to three).
__device__ __forceinline__ void bulk_panels(const PSArgs& a, int k, int q, int nb, double (*TU)[kLD],
                                            double (*TX)[kLD]) {
  const int nt = a.nt, Np = a.Np;
  const int m = nt - k - 1;
  const int ntot = m + k + 2;                   // matrix rows, the v row, identity rows 0..k
  const int tb = (int)((int64_t)ntot * q / nb), te = (int)((int64_t)ntot * (q + 1) / nb);
  bool have_u = false;
  for (int t = tb; t < te; ++t) {
    const int rt = (t < m) ? k + 1 + t : nt + (t - m);
    const int rows = (rt == nt) ? 1 : kTile;
    const int64_t r0 = row_off(rt, nt, Np);
    {
      double vu[kPerThread], vx[kPerThread];
      if (!have_u) tile_gather(vu, a.Ud + (int64_t)k * kTile * kTile, kTile, 0, 0);
      tile_gather(vx, a.A, Np, r0, (int64_t)k * kTile, rows);
      if (!have_u) tile_scatter(TU, vu);
      tile_scatter(TX, vx);
    }
    have_u = true;
    __syncthreads();
    tile_mul_inplace(TX, TU);                   // X_rk
    if (rt < nt) tile_out(TX, a.A, Np, r0, (int64_t)k * kTile, rows);
    else tile_out(TX, a.Z, Np, r0 - Np, (int64_t)k * kTile, rows);
    __syncthreads();
  }
}

__device__ __forceinline__ void bulk_updates(const PSArgs& a, int k, int q, int nb, double (*TX)[kLD],
                                             double (*TL)[kLD], double (*TC)[kLD]) {
  const int nt = a.nt, Np = a.Np;
  const int m = nt - k - 1;
  if (m == 0) return;
  const int ntri = m * (m + 1) / 2;
  const int nrow = k + 2;
  const int ntot = ntri + nrow * m;
  const int tb = 1 + (int)((int64_t)(ntot - 1) * q / nb);
  const int te = 1 + (int)((int64_t)(ntot - 1) * (q + 1) / nb);
  int xrow = -1;
  for (int t = tb; t < te; ++t) {
    int rt, J;
    if (t < ntri) {
      int ti, tj;
      tri_decode(t, ti, tj);
      rt = k + 1 + ti;
      J = k + 1 + tj;
    } else {
      const int u = t - ntri;
      rt = nt + u / m;
      J = k + 1 + u % m;
    }
    const int rows = (rt == nt) ? 1 : kTile;
    const int64_t r0 = row_off(rt, nt, Np);
    const bool diag = (J == rt);
    const bool new_x = (rt != xrow);
    {
      double vx[kPerThread], vc[kPerThread], vl[kPerThread];
      if (new_x) {
        if (rt < nt) tile_gather(vx, a.A, Np, r0, (int64_t)k * kTile, rows);
        else tile_gather(vx, a.Z, Np, r0 - Np, (int64_t)k * kTile, rows);
      }
      tile_gather(vc, a.A, Np, r0, (int64_t)J * kTile, rows);
      if (!diag) tile_gather(vl, a.A, Np, (int64_t)J * kTile, (int64_t)k * kTile);
      if (new_x) tile_scatter(TX, vx);
      tile_scatter(TC, vc);
      if (!diag) tile_scatter(TL, vl);
    }
    xrow = rt;
    __syncthreads();
    tile_sub_abt(TC, TX, diag ? TX : TL);
    store_tile_r(TC, a.A, Np, r0, J, rows);
    __syncthreads();
  }
}

template <bool TWO_PHASE>
__device__ __forceinline__ void solve_body(const PSArgs& a, const int bid) {
  extern __shared__ __align__(16) double smem[];
  double (*T0)[kLD] = reinterpret_cast<double (*)[kLD]>(smem);
  double (*T1)[kLD] = reinterpret_cast<double (*)[kLD]>(smem + kTile * kLD);
  double (*T2)[kLD] = reinterpret_cast<double (*)[kLD]>(smem + 2 * kTile * kLD);
  double (*T3)[kLD] = reinterpret_cast<double (*)[kLD]>(smem + 3 * kTile * kLD);
  __shared__ double red[kPT / 64];
  Barrier bar;
  bar.bid = bid;
  const int N = a.N, Np = a.Np, nt = a.nt, P = a.P;
  double* v = a.A + (int64_t)Np * Np;                     // row Np: v
  double* U = a.A + ((int64_t)Np + kTile) * Np;           // identity rows

  // ---- equilibrate: A = D G D (identity padding), v = D h, rowabs, identity rows
  {
    double* sv = smem;                                    // D, computed by every workgroup
    for (int j = threadIdx.x; j < Np; j += kPT) {
      double sj = 1.0;
      if (j < N) {
        const double gjj = a.G[(int64_t)j * N + j];
        sj = (gjj > 0.0 && is_finite_d(gjj)) ? 1.0 / sqrt(gjj) : 0.0;
      }
      sv[j] = sj;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int i = bid * (kPT / 64) + wave; i < Np; i += P * (kPT / 64)) {
      const double si = sv[i];
      double ra = 0.0;
      for (int jb = 0; jb < Np; jb += 64 * 8) {
        double gv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int j = jb + 64 * u + lane;
          gv[u] = (i < N && j < N) ? a.G[(int64_t)i * N + j] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int j = jb + 64 * u + lane;
          if (j >= Np) continue;
          double val;
          if (i < N && j < N) {
            ra += fabs(gv[u]);
            val = si * gv[u] * sv[j];
          } else {
            val = (i == j) ? 1.0 : 0.0;
          }
          a.A[(int64_t)i * Np + j] = val;
          // identity rows: only the tiles on and right of the diagonal are read
          if (j >= (i & ~63)) U[(int64_t)i * Np + j] = (i == j) ? 1.0 : 0.0;
        }
      }
      ra = wave_sum(ra);
      if (lane == 0) {
        a.s[i] = si;
        v[i] = (i < N) ? si * a.h[i] : 0.0;
        a.rowabs[i] = ra;
      }
    }
  }
  bar.wait(a);

  // ---- factorisation of [A; v^T; I]: diagonal chain (workgroup 0) and the
  // bulk work of the others one step behind; with P = 1 workgroup 0 takes
  // both roles in turn.
  const int q = (P > 1) ? bid - 1 : 0;        // index among the bulk workgroups
  const int nb = (P > 1) ? P - 1 : 1;
  if (bid == 0) {
    load_tile(T0, a.A, Np, 0, 0);
    __syncthreads();
  }
  for (int k = 0; k < nt; ++k) {
    if (bid == 0) {
      // T0: diagonal tile k with every update of steps < k. Before the last
      // block of its factorisation, once the bulk work of step k - 1 is
      // complete (late, so that the bulk rarely holds the chain up), the
      // two tiles of row k + 1 that the chain needs next are loaded into
      // registers (they arrive while the sweep goes on).
      if (P == 1 && k > 0) {
        load_tile(T0, a.A, Np, k, k);
        __syncthreads();
      }
      const bool ahead = k + 1 < nt;
      double xr[kPerThread], dr[kPerThread];
      const int f = tile_potrf_aug(T0, T2, [&]() {
        if (!ahead) return;
        if (P > 1) wait_progress(a, 0, 2 * k);
#pragma unroll
        for (int t = 0; t < kPerThread; ++t) {
          const int idx = threadIdx.x + t * kPT;
          const int64_t row = (int64_t)(k + 1) * kTile + (idx >> 6);
          xr[t] = a.A[row * Np + (int64_t)k * kTile + (idx & 63)];
          dr[t] = a.A[row * Np + (int64_t)(k + 1) * kTile + (idx & 63)];
        }
      });
      stamp(a, 128 + 2 * k);
      if (f >= 0) {
        if (threadIdx.x == 0) atomicCAS(&a.flags[1], 0, k * kTile + f + 1);
        publish(a, 0, 2 * k + 1);
        break;
      }
      store_tile(T0, a.A, Np, k, k);
      tile_out(T2, a.Ud + (int64_t)k * kTile * kTile, kTile, 0, 0);
      publish(a, 0, 2 * k + 1);
      if (ahead) {
#pragma unroll
        for (int t = 0; t < kPerThread; ++t) {
          const int idx = threadIdx.x + t * kPT;
          T1[idx >> 6][idx & 63] = xr[t];
          T0[idx >> 6][idx & 63] = dr[t];
        }
        __syncthreads();
        tile_mul_inplace(T1, T2);                 // L_(k+1),k = A_(k+1),k U_k
        tile_sub_abt(T0, T1, T1);                 // diagonal tile k + 1, step k
        if (P == 1) {
          store_tile(T0, a.A, Np, k + 1, k + 1);
          __syncthreads();
        }
      }
      stamp(a, 129 + 2 * k);
    }
    if (P == 1 || bid > 0) {
      // U_k stored; the bulk work of step k - 1 complete
      if (P > 1) wait_progress(a, 2 * k + 1, 2 * k);
      if (failed_by(a, k)) break;
      if constexpr (TWO_PHASE) {
        bulk_panels(a, k, q, nb, T0, T1);
        // every panel tile of step k written before any update reads it
        if (P > 1) {
          publish(a, bid, 2 * k + 1);
          wait_progress(a, 2 * k + 1, 2 * k + 1);
        }
        bulk_updates(a, k, q, nb, T1, T2, T3);
      } else {
        bulk_step(a, k, q, nb, T0, T1, T2, T3);
      }
      if (P > 1) publish(a, bid, 2 * k + 2);
    }
  }
  bar.wait(a);
  const bool bad = failed(a);
  // ---- theta = D L^-T z, refinement
  if (!bad) {
    gemv_upper_theta(a, a.Z, false, bid);
    bar.wait(a);
    for (int it = 0; it < a.refine; ++it) {
      residual(a, bid);                  // r = D (h - G theta)
      bar.wait(a);
      gemv_upper_t(a, a.r, a.x, bid, bar);   // x = L^-1 r
      bar.wait(a);
      gemv_upper_theta(a, a.x, true, bid);   // theta += D L^-T x
      bar.wait(a);
    }
    residual(a, bid);
    bar.wait(a);
  }
  // ---- final report (workgroup 0)
  if (bid == 0) {
    double rmax = 0.0, tmax = 0.0, hmax = 0.0, gmax = 0.0, pmin = 1e308, pmax = 0.0;
    for (int i = threadIdx.x; i < N; i += kPT) {
      hmax = fmax(hmax, fabs(a.h[i]));
      if (!bad) {
        const double si = a.s[i];
        rmax = fmax(rmax, si > 0.0 ? fabs(a.r[i] / si) : 0.0);
        tmax = fmax(tmax, fabs(a.theta[i]));
        gmax = fmax(gmax, a.rowabs[i]);
        const double pv = a.A[(int64_t)i * Np + i];
        pmin = fmin(pmin, pv);
        pmax = fmax(pmax, pv);
      }
      a.coef[i] = bad ? __builtin_nan("") : a.theta[i];
    }
    auto bmax = [&](double val) {
      for (int off = 32; off > 0; off >>= 1) val = fmax(val, __shfl_xor(val, off, 64));
      __syncthreads();
      if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = val;
      __syncthreads();
      double mm = red[0];
      for (int w = 1; w < kPT / 64; ++w) mm = fmax(mm, red[w]);
      return mm;
    };
    rmax = bmax(rmax);
    tmax = bmax(tmax);
    hmax = bmax(hmax);
    gmax = bmax(gmax);
    pmax = bmax(pmax);
    pmin = -bmax(-pmin);
    if (threadIdx.x == 0) {
      sfft_solve_info inf{};
      inf.nonfinite = a.flags[0];
      inf.failed_pivot = -1;
      if (bad) {
        inf.status = SFFT_ERR_NOT_SPD;
        inf.failed_pivot = a.flags[1] - 1;
        inf.backward_err = __builtin_nan("");
      } else {
        inf.status = SFFT_OK;
        inf.backward_err = rmax / (gmax * tmax + hmax);
        inf.min_pivot = pmin;
        inf.max_pivot = pmax;
        inf.refine_iters = a.refine;
      }
      if (a.flags[2]) inf.status = SFFT_ERR_INTERNAL;
      if (inf.nonfinite) inf.status = SFFT_ERR_NONFINITE;
      *a.info = inf;
    }
  }
}

__global__ __launch_bounds__(kPT) void k_solve_persistent(PSArgs a) { solve_body<false>(a, blockIdx.x); }

// T teams of P co-resident workgroups; team t solves items t, t + T, ...
// (a static work queue over items ordered by decreasing size, every item
// planned with the same P)
__global__ __launch_bounds__(kPT) void k_solve_batch(const PSArgs* args, const int* order, int n, int P, int T) {
  const int team = blockIdx.x / P, bid = blockIdx.x % P;
  for (int q = team; q < n; q += T) solve_body<true>(args[order[q]], bid);
}

// clears the arrival / release / progress flags and the time stamps
__global__ void k_solve_reset(unsigned* sync, int nsync, int* flags) {
  for (int i = threadIdx.x; i < nsync; i += blockDim.x) sync[i] = 0u;
  if (threadIdx.x == 0) { flags[1] = 0; flags[2] = 0; }
}

size_t solve_shmem_bytes() {
  return sizeof(double) * (4 * kTile * kLD);
}

int solve_workgroups(int nt) {
  // one bulk task per workgroup in the widest step (step 0: the lower
  // triangle of the trailing matrix less its first tile, the v row and one
  // identity row), plus the chain's workgroup; at most kPlainTeam
  const int m = nt - 1;
  const int widest = m > 0 ? m * (m + 1) / 2 - 1 + 2 * m : 2;
  const int p = widest + 1;
  return p < kPlainTeam ? p : kPlainTeam;
}

hipError_t prepare_solve_attributes() {
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_solve_persistent),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)solve_shmem_bytes());
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_solve_batch),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)solve_shmem_bytes());
}

static PSArgs make_solve_args(const sfft_desc& d, const double* G, const double* h, double* coef,
                              int max_refine, sfft_solve_info* info, unsigned char* ws, int P) {
  const Geometry g = make_geometry(d);
  const Layout l = make_layout(g);
  PSArgs a{};
  a.G = G; a.h = h; a.coef = coef; a.info = info;
  a.A = reinterpret_cast<double*>(ws + l.A);
  a.s = reinterpret_cast<double*>(ws + l.s);
  a.x = reinterpret_cast<double*>(ws + l.x);
  a.theta = reinterpret_cast<double*>(ws + l.theta);
  a.r = reinterpret_cast<double*>(ws + l.rvec);
  a.rowabs = reinterpret_cast<double*>(ws + l.rowabs);
  a.Z = reinterpret_cast<double*>(ws + l.Z);
  a.Ud = reinterpret_cast<double*>(ws + l.Ud);
  a.part = reinterpret_cast<double*>(ws + l.part);
  a.sync = reinterpret_cast<unsigned*>(ws + l.sync);
  a.prog = a.sync + kSyncWords / 2;
  a.stamps = reinterpret_cast<unsigned long long*>(ws + l.sync + kSyncWords * sizeof(unsigned));
  a.flags = reinterpret_cast<int*>(ws + l.flags);
  a.N = g.N; a.nt = l.nt; a.Np = l.nt * kTile; a.refine = max_refine;
  a.P = P > 0 ? P : solve_workgroups(l.nt);
  return a;
}

hipError_t launch_solve(const sfft_desc& d, const double* G, const double* h, double* coef,
                        int max_refine, sfft_solve_info* info, unsigned char* ws, int num_cus, int team,
                        const Prof* pf, hipStream_t st) {
  PSArgs a = make_solve_args(d, G, h, coef, max_refine, info, ws, 0);
  // a caller-chosen smaller team leaves CUs to work on other streams (the
  // diagonal chain, not the team size, bounds the solve's duration)
  if (team >= 2 && team < a.P) a.P = team;
  // a plain launch (no cooperative-launch overhead, capturable in a graph):
  // the LDS footprint allows one solve workgroup per CU and P is at most half
  // the CUs, so every workgroup becomes resident while the others wait; the
  // waits are bounded anyway
  const int cus = num_cus > 0 ? num_cus : 256;
  if (a.P > cus / 2) a.P = cus / 2 > 0 ? cus / 2 : 1;
  prof_begin(pf, SFFT_PROF_SOLVE, st);
  hipLaunchKernelGGL(k_solve_reset, dim3(1), dim3(256), 0, st, a.sync, kSyncClear, a.flags);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_solve_persistent, dim3(a.P), dim3(kPT), solve_shmem_bytes(), st, a);
  e = hipGetLastError();
  prof_end(pf, SFFT_PROF_SOLVE, st);
  return e;
}

// ---- batched solve: n teams of P workgroups in one launch ----

__global__ void k_solve_reset_batch(const PSArgs* args) {
  const PSArgs& a = args[blockIdx.x];
  for (int i = threadIdx.x; i < kSyncClear; i += blockDim.x) a.sync[i] = 0u;
  if (threadIdx.x == 0) { a.flags[1] = 0; a.flags[2] = 0; }
}

struct SolveBatch {
  std::vector<PSArgs> args;
  std::vector<int> order;     // items by decreasing number of unknowns
  PSArgs* dev = nullptr;
  int* dorder = nullptr;
  int P = 1, T = 1;
};

// Team size P and team count T: every workgroup of every team must be
// co-resident (one solve workgroup per CU), so T * P <= number of CUs;
// T <= n. P = 0 picks P = CUs / n (one team per item when they fit).
SolveBatch* solve_batch_create(const SolveItem* items, int n, int max_refine, int P, int num_cus,
                               hipError_t* err) {
  const int cus = num_cus > 0 ? num_cus : 256;
  if (P <= 0) P = std::max(1, cus / n);
  if (P > kMaxTeam) P = kMaxTeam;
  if (P < 1 || P > cus) { *err = hipErrorInvalidValue; return nullptr; }
  SolveBatch* b = new (std::nothrow) SolveBatch();
  if (!b) { *err = hipErrorOutOfMemory; return nullptr; }
  b->P = P;
  b->T = std::min(n, cus / P);
  for (int k = 0; k < n; ++k) {
    const SolveItem& it = items[k];
    b->args.push_back(make_solve_args(it.d, it.G, it.h, it.coef, max_refine, it.info, it.ws, P));
    b->order.push_back(k);
  }
  std::stable_sort(b->order.begin(), b->order.end(),
                   [&](int x, int y) { return b->args[x].N > b->args[y].N; });
  *err = hipSuccess;
  return b;
}

size_t solve_batch_dev_bytes(const SolveBatch* b) {
  return align256(b->args.size() * sizeof(PSArgs)) + align256(b->order.size() * sizeof(int));
}

hipError_t solve_batch_upload(SolveBatch* b, unsigned char* dev) {
  b->dev = reinterpret_cast<PSArgs*>(dev);
  b->dorder = reinterpret_cast<int*>(dev + align256(b->args.size() * sizeof(PSArgs)));
  hipError_t e = hipMemcpy(dev, b->args.data(), b->args.size() * sizeof(PSArgs), hipMemcpyHostToDevice);
  if (e != hipSuccess) return e;
  return hipMemcpy(b->dorder, b->order.data(), b->order.size() * sizeof(int), hipMemcpyHostToDevice);
}

hipError_t solve_batch_launch(const SolveBatch* b, const Prof* pf, hipStream_t st) {
  const int n = (int)b->args.size();
  prof_begin(pf, SFFT_PROF_SOLVE, st);
  hipLaunchKernelGGL(k_solve_reset_batch, dim3(n), dim3(256), 0, st, (const PSArgs*)b->dev);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // a plain launch (capturable in a graph): T * P <= CUs with one workgroup
  // per CU keeps every team resident; the barrier spins are bounded anyway
  hipLaunchKernelGGL(k_solve_batch, dim3(b->T * b->P), dim3(kPT), solve_shmem_bytes(), st,
                     (const PSArgs*)b->dev, (const int*)b->dorder, n, b->P, b->T);
  prof_end(pf, SFFT_PROF_SOLVE, st);
  return hipGetLastError();
}

int solve_batch_team(const SolveBatch* b) { return b->P; }

void solve_batch_destroy(SolveBatch* b) { delete b; }

}  // namespace sfft
