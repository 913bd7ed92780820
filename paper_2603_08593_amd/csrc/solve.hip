// sfft_solve: FP64 solve of the normal equations G theta = h.
//
// The SFFT fit ends in a dense symmetric positive-definite solve (the
// least-squares normal equations of the delta-basis kernel, paper Sec. 1).
// One persistent cooperative kernel with P co-resident workgroups does:
//   equilibration  A = D G D, D = diag(G)^-1/2, v = D h;
//   right-looking blocked Cholesky on 64 x 64 tiles of the matrix augmented
//   below by the right-hand side row v^T and by the identity: factorising
//   [A; v^T; I] turns those rows into z^T = (L^-1 v)^T and L^-T, so the
//   forward substitution and the inverse factor come out of the same sweep
//   with no extra synchronisation; look-ahead: the workgroup that owns the
//   next diagonal tile updates and factors it first while the others apply
//   the remaining trailing updates;
//   x = L^-T z as one distributed matrix-vector product; up to `refine`
//   steps of iterative refinement on r = h - G theta (FP64), each three
//   matrix-vector products (G theta, L^-1 r = (L^-T)^T r, L^-T z);
//   final backward error and pivot range.
// Workgroups synchronise through a flag barrier (one arrival flag per
// workgroup, one release flag) with bounded spins: a timeout is reported in
// the status instead of hanging.
#include <algorithm>
#include <new>
#include <vector>

#include "batch.hpp"
#include "common.hpp"
#include "layout.hpp"

namespace sfft {

constexpr int kPT = 512;                    // threads per solve workgroup
constexpr long kSpinLimit = 1L << 26;
constexpr int kLD = kTile + 1;              // LDS row pitch of a tile

struct PSArgs {
  const double* G;
  const double* h;
  double* coef;
  sfft_solve_info* info;
  double* A;        // (2 Np + 64) x Np: rows [0, Np) matrix -> L; row Np: v -> z;
                    // rows [Np + 64, 2 Np + 64): identity -> L^-T
  double* s;        // Np
  double* x;        // Np
  double* theta;    // Np
  double* r;        // Np
  double* rowabs;   // Np
  double* Ud;       // nt tiles of 64 x 64: U_k = L_kk^-T of each diagonal tile
  double* part;     // partial sums of gemv_upper_t
  unsigned* sync;   // [0, P): arrival flags, [P]: release flag
  unsigned long long* stamps;   // optional: 100 MHz time stamp of each barrier
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
    if (bid == 0 && threadIdx.x == 0 && a.stamps && gen < 256)
      a.stamps[gen] = __builtin_amdgcn_s_memrealtime();
  }
};

__device__ __forceinline__ bool failed(const PSArgs& a) {
  return __hip_atomic_load(&a.flags[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
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
// TRANS_B = true: acc = X Y^T; false: acc = X Y.
template <bool TRANS_B>
__device__ __forceinline__ void tile_mma(const double (*X)[kLD], const double (*Y)[kLD],
                                         double4_t acc[2]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i0 = 16 * (w & 3), j0 = 32 * (w >> 2);
  const int lr = lane & 15, lk = lane >> 4;
  acc[0] = double4_t{0.0, 0.0, 0.0, 0.0};
  acc[1] = double4_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
  for (int k = 0; k < kTile; k += 4) {
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

// C = X U (U upper triangular; C may not alias X or U)
__device__ __forceinline__ void tile_mul_ab(double (*C)[kLD], const double (*X)[kLD],
                                            const double (*U)[kLD]) {
  double4_t acc[2];
  tile_mma<false>(X, U, acc);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i0 = 16 * (w & 3) + (lane >> 4), j0 = 32 * (w >> 2) + (lane & 15);
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int q = 0; q < 4; ++q) C[i0 + 4 * q][j0 + 16 * b] = acc[b][q];
  __syncthreads();
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

// Cholesky of the 64 x 64 SPD tile T (lower, in place) and U = L^-T into Ut.
// The right-looking factorisation of the stacked [T; I] turns the identity
// rows into L^-T (I = Y L^T); Ut starts as the identity and holds Y. Blocked
// by 8 columns, two workgroup barriers per block:
//   panel: wave 0 (lane i = row i of T and of Y) keeps the block's 8 entries
//   of both rows in registers and factors the 8 columns one by one; pivots
//   and the entries of L that update the rest of the block come from other
//   lanes by readlane, so the column chain never waits on LDS; column j of L
//   is written to T and the block of Y to Ut;
//   trailing update: every wave applies the block's rank-8 update to its
//   share of the later columns (wave w: columns j0 + 8 + w, + 8, ...) for all
//   64 rows of T and of Y, reading the block of L as broadcasts.
// A pivot that is not positive and finite is recorded (the first one) and
// the sweep goes on with a zero scale, so values stay finite; the caller
// discards them. Returns the failing local pivot or -1.
__device__ __forceinline__ int tile_potrf_aug(double (*T)[kLD], double (*Ut)[kLD]) {
  constexpr int kB = 8;
  __shared__ int fail;
  const int i = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (threadIdx.x == 0) fail = -1;
  for (int idx = threadIdx.x; idx < kTile * kTile; idx += kPT)
    Ut[idx >> 6][idx & 63] = ((idx >> 6) == (idx & 63)) ? 1.0 : 0.0;
  __syncthreads();
  int f = -1;
#pragma unroll 1
  for (int jb = 0; jb < kTile / kB; ++jb) {
    const int j0 = jb * kB;
    if (w == 0) {
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
        const double rs = good ? rsqrt64(d) : 0.0;
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
    __syncthreads();
    if (j0 + kB < kTile) {
      double li[kB], yi[kB];
#pragma unroll
      for (int c = 0; c < kB; ++c) {
        li[c] = T[i][j0 + c];
        yi[c] = Ut[i][j0 + c];
      }
      for (int m = j0 + kB + w; m < kTile; m += kPT / 64) {
        double t = T[i][m], u = Ut[i][m];
#pragma unroll
        for (int c = 0; c < kB; ++c) {
          const double lm = T[m][j0 + c];                 // broadcast
          t = fma(-li[c], lm, t);
          u = fma(-yi[c], lm, u);
        }
        T[i][m] = t;
        Ut[i][m] = u;
      }
      __syncthreads();
    }
  }
  if (w == 0) {
    for (int k = i + 1; k < kTile; ++k) T[i][k] = 0.0;
    if (i == 0) fail = f;
  }
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

// out_i = sum_j U[i][j] in_j with U = L^-T stored in the identity rows
// (upper triangular: j >= i); one row per wave.
__device__ void gemv_upper(const PSArgs& a, const double* in, double* out, int bid) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nw = kPT / 64;
  const double* U = a.A + ((int64_t)a.Np + kTile) * a.Np;
  for (int i = bid * nw + wave; i < a.Np; i += a.P * nw) {
    const double* Ur = U + (int64_t)i * a.Np;
    double acc = 0.0;
#pragma unroll 4
    for (int j = (i & ~63) + lane; j < a.Np; j += 64) acc = fma(Ur[j], in[j], acc);
    acc = wave_sum(acc);
    if (lane == 0) out[i] = acc;
  }
}

// out_j = sum_{i <= j} U[i][j] in_i (U^T = L^-1, lower). The rows are cut
// into chunks; wave (column block cb, chunk ch) sums its chunk for the 64
// columns of the block (one column per lane, coalesced row reads) into
// part[ch][j]; after a barrier the chunks are added in order.
__device__ void gemv_upper_t(const PSArgs& a, const double* in, double* out, int bid, Barrier& bar) {
  const double* U = a.A + ((int64_t)a.Np + kTile) * a.Np;
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
#pragma unroll 8
    for (int i = i0; i < i1; ++i) {
      const double u = U[(int64_t)i * a.Np + j];
      acc = (i <= j) ? fma(u, in[i], acc) : acc;
    }
    a.part[(int64_t)ch * a.Np + j] = acc;
  }
  bar.wait(a);
  for (int j = bid * kPT + threadIdx.x; j < a.Np; j += a.P * kPT) {
    double s = 0.0;
    for (int ch = 0; ch < nch; ++ch) s += a.part[(int64_t)ch * a.Np + j];
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
    const double* Gr = a.G + (int64_t)i * a.N;
    double sacc = 0.0;
#pragma unroll 4
    for (int j = lane; j < a.N; j += 64) sacc = fma(Gr[j], a.theta[j], sacc);
    sacc = wave_sum(sacc);
    if (lane == 0) a.r[i] = a.s[i] * (a.h[i] - sacc);
  }
}

__device__ __forceinline__ void solve_body(const PSArgs& a, const int bid) {
  extern __shared__ __align__(16) double smem[];
  double (*T0)[kLD] = reinterpret_cast<double (*)[kLD]>(smem);
  double (*T1)[kLD] = reinterpret_cast<double (*)[kLD]>(smem + kTile * kLD);
  double (*T2)[kLD] = reinterpret_cast<double (*)[kLD]>(smem + 2 * kTile * kLD);
  __shared__ double red[kPT / 64];
  Barrier bar;
  bar.bid = bid;
  const int N = a.N, Np = a.Np, nt = a.nt, P = a.P;
  double* v = a.A + (int64_t)Np * Np;                     // row Np: v, then z
  double* U = a.A + ((int64_t)Np + kTile) * Np;           // identity rows, then L^-T

  // ---- equilibrate: A = D G D (identity padding), v = D h, rowabs, identity rows
  {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int i = bid * (kPT / 64) + wave; i < Np; i += P * (kPT / 64)) {
      double si = 1.0;
      if (i < N) {
        const double gii = a.G[(int64_t)i * N + i];
        si = (gii > 0.0 && is_finite_d(gii)) ? 1.0 / sqrt(gii) : 0.0;
      }
      double ra = 0.0;
      for (int j = lane; j < Np; j += 64) {
        double val;
        if (i < N && j < N) {
          const double gjj = a.G[(int64_t)j * N + j];
          const double sj = (gjj > 0.0 && is_finite_d(gjj)) ? 1.0 / sqrt(gjj) : 0.0;
          const double g = a.G[(int64_t)i * N + j];
          ra += fabs(g);
          val = si * g * sj;
        } else {
          val = (i == j) ? 1.0 : 0.0;
        }
        a.A[(int64_t)i * Np + j] = val;
        U[(int64_t)i * Np + j] = (i == j) ? 1.0 : 0.0;
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

  // ---- factorisation of [A; v^T; I]
  // Step k: workgroup 0 applies the last update to diagonal tile k (from the
  // panel of step k - 1) and factors it, storing L_kk and U_k = L_kk^-T,
  // while the others apply the remaining trailing updates of step k - 1
  // (look-ahead); then every workgroup takes panel tiles of column tile k.
  for (int k = 0; k < nt; ++k) {
    if (bid == 0) {
      load_tile(T0, a.A, Np, k, k);
      if (k > 0) load_tile(T1, a.A, Np, k, k - 1);
      __syncthreads();
      if (k > 0) tile_sub_abt(T0, T1, T1);
      const int f = tile_potrf_aug(T0, T2);
      if (f >= 0) {
        if (threadIdx.x == 0) atomicCAS(&a.flags[1], 0, k * kTile + f + 1);
      } else {
        store_tile(T0, a.A, Np, k, k);
        tile_out(T2, a.Ud + (int64_t)k * kTile * kTile, kTile, 0, 0);
      }
      __syncthreads();
    }
    // trailing update of step kp = k - 1 on column tiles J in [k, nt): rows
    // of the matrix (J <= I < nt), the v row and the identity rows i <= kp;
    // item 0, tile (k, k), is workgroup 0's
    if (k > 0 && (P == 1 || bid > 0)) {
      const int kp = k - 1;
      const int m = nt - k;
      const int ntri = m * (m + 1) / 2;
      const int nv = m;
      const int naug = k * m;
      const int ntot = ntri + nv + naug;
      const int first = (P > 1) ? bid - 1 : 0;
      const int stride = (P > 1) ? P - 1 : 1;
      for (int t = 1 + first; t < ntot; t += stride) {
        int rt, J;
        if (t < ntri) {
          int ti, tj;
          tri_decode(t, ti, tj);
          rt = k + ti;
          J = k + tj;
        } else if (t < ntri + nv) {
          rt = nt;
          J = k + (t - ntri);
        } else {
          const int u = t - ntri - nv;
          rt = nt + 1 + u / m;
          J = k + u % m;
        }
        const int rows = (rt == nt) ? 1 : kTile;
        const int64_t r0 = row_off(rt, nt, Np);
        load_tile_r(T0, a.A, Np, r0, J, rows);
        load_tile_r(T1, a.A, Np, r0, kp, rows);
        load_tile(T2, a.A, Np, J, kp);
        __syncthreads();
        tile_sub_abt(T0, T1, T2);
        store_tile_r(T0, a.A, Np, r0, J, rows);
        __syncthreads();
      }
    }
    bar.wait(a);
    if (failed(a)) break;
    // panel: row tiles k+1 .. nt-1 (matrix), nt (v row), nt+1+i for i <= k
    // (identity rows with nonzero entries in column tile k)
    {
      const int nmat = nt - k - 1;
      const int npanel = nmat + 1 + (k + 1);
      bool loaded = false;
      for (int t = bid; t < npanel; t += P) {
        int rt;
        if (t < nmat) rt = k + 1 + t;
        else if (t == nmat) rt = nt;
        else rt = nt + 1 + (t - nmat - 1);
        const int rows = (rt == nt) ? 1 : kTile;
        const int64_t r0 = row_off(rt, nt, Np);
        if (!loaded) {
          tile_in(T1, a.Ud + (int64_t)k * kTile * kTile, kTile, 0, 0);
          loaded = true;
        }
        load_tile_r(T0, a.A, Np, r0, k, rows);
        __syncthreads();
        tile_mul_ab(T2, T0, T1);          // X = A_rk L_kk^-T
        store_tile_r(T2, a.A, Np, r0, k, rows);
        __syncthreads();
      }
    }
    bar.wait(a);
  }
  const bool bad = failed(a);
  // ---- x = L^-T z, theta = D x, refinement
  if (!bad) {
    gemv_upper(a, v, a.x, bid);
    bar.wait(a);
    for (int i = bid * kPT + threadIdx.x; i < Np; i += P * kPT) a.theta[i] = a.s[i] * a.x[i];
    bar.wait(a);
    for (int it = 0; it < a.refine; ++it) {
      residual(a, bid);                  // r = D (h - G theta)
      bar.wait(a);
      gemv_upper_t(a, a.r, a.x, bid, bar);   // x = L^-1 r
      bar.wait(a);
      gemv_upper(a, a.x, a.r, bid);      // r = L^-T x
      bar.wait(a);
      for (int i = bid * kPT + threadIdx.x; i < Np; i += P * kPT) a.theta[i] += a.s[i] * a.r[i];
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

__global__ __launch_bounds__(kPT) void k_solve_persistent(PSArgs a) { solve_body(a, blockIdx.x); }

// T teams of P co-resident workgroups; team t solves items t, t + T, ...
// (a static work queue over items ordered by decreasing size, every item
// planned with the same P)
__global__ __launch_bounds__(kPT) void k_solve_batch(const PSArgs* args, const int* order, int n, int P, int T) {
  const int team = blockIdx.x / P, bid = blockIdx.x % P;
  for (int q = team; q < n; q += T) solve_body(args[order[q]], bid);
}

// clears the arrival / release flags and the barrier time stamps
__global__ void k_solve_reset(unsigned* sync, int nsync, int* flags) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nsync) sync[i] = 0u;
  if (i == 0) { flags[1] = 0; flags[2] = 0; }
}

size_t solve_shmem_bytes() {
  return sizeof(double) * (3 * kTile * kLD);
}

int solve_workgroups(int nt) {
  // about one trailing-update tile per workgroup in the first steps, at most 64
  const int widest = nt * (nt + 1) / 2 + nt;
  return widest < 64 ? (widest > 1 ? widest : 1) : 64;
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
  a.Ud = reinterpret_cast<double*>(ws + l.Ud);
  a.part = reinterpret_cast<double*>(ws + l.part);
  a.sync = reinterpret_cast<unsigned*>(ws + l.sync);
  a.stamps = reinterpret_cast<unsigned long long*>(ws + l.sync + 512);
  a.flags = reinterpret_cast<int*>(ws + l.flags);
  a.N = g.N; a.nt = l.nt; a.Np = l.nt * kTile; a.refine = max_refine;
  a.P = P > 0 ? P : solve_workgroups(l.nt);
  return a;
}

hipError_t launch_solve(const sfft_desc& d, const double* G, const double* h, double* coef,
                        int max_refine, sfft_solve_info* info, unsigned char* ws,
                        const Prof* pf, hipStream_t st) {
  PSArgs a = make_solve_args(d, G, h, coef, max_refine, info, ws, 0);
  prof_begin(pf, SFFT_PROF_SOLVE, st);
  hipLaunchKernelGGL(k_solve_reset, dim3(1), dim3(640), 0, st, a.sync, 640, a.flags);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  void* args[] = {&a};
  e = hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_solve_persistent), dim3(a.P),
                                 dim3(kPT), args, (unsigned)solve_shmem_bytes(), st);
  prof_end(pf, SFFT_PROF_SOLVE, st);
  return e;
}

// ---- batched solve: n teams of P workgroups in one launch ----

__global__ void k_solve_reset_batch(const PSArgs* args) {
  const PSArgs& a = args[blockIdx.x];
  for (int i = threadIdx.x; i < 640; i += blockDim.x) a.sync[i] = 0u;
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
  if (P > 64) P = 64;
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
