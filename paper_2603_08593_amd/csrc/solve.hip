// sfft_solve kernels: FP64 solve of the normal equations G theta = h.
//
// The paper's SFFT fit ends in a dense symmetric positive-definite linear
// solve (least-squares normal equations, paper Sec. 1). Here: equilibrate
// with D = diag(G)^-1/2 (A = D G D), blocked right-looking Cholesky on
// 64 x 64 tiles (diagonal factor, panel substitution, trailing update),
// inverses of the diagonal factors, blocked forward/backward substitution,
// then iterative refinement on the residual h - G theta in FP64.
// Matrices are padded to a multiple of 64 with an identity block.
#include "common.hpp"
#include "layout.hpp"

namespace sfft {

struct SolveArgs {
  const double* G;
  const double* h;
  double* coef;
  sfft_solve_info* info;
  double* A;        // Np x Np
  double* s;        // Np
  double* b;        // Np
  double* theta;    // Np
  double* x;        // Np
  double* rvec;     // Np
  double* rowabs;   // Np (row sums of |G|), later reused
  double* Linv;     // nt x 64 x 64
  int* flags;       // [0] nonfinite (from build), [1] failed pivot + 1 (0 = none)
  int N, Np, nt;
};

__global__ void k_solve_init(SolveArgs a) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    a.flags[1] = 0;
    sfft_solve_info inf{};
    inf.status = SFFT_OK;
    inf.failed_pivot = -1;
    inf.refine_iters = 0;
    inf.nonfinite = a.flags[0];
    inf.backward_err = 0.0;
    inf.min_pivot = 0.0;
    inf.max_pivot = 0.0;
    *a.info = inf;
  }
}

// one workgroup per row: A = D G D, b = D h, rowabs = sum_j |G_ij|
__global__ __launch_bounds__(256) void k_equil(SolveArgs a) {
  __shared__ double scratch[8];
  const int i = blockIdx.x;
  const int N = a.N, Np = a.Np;
  double si = 1.0;
  if (i < N) {
    const double gii = a.G[(int64_t)i * N + i];
    si = (gii > 0.0 && is_finite_d(gii)) ? 1.0 / sqrt(gii) : 0.0;
  }
  double ra = 0.0;
  for (int j = threadIdx.x; j < Np; j += blockDim.x) {
    double v;
    if (i < N && j < N) {
      const double gjj = a.G[(int64_t)j * N + j];
      const double sj = (gjj > 0.0 && is_finite_d(gjj)) ? 1.0 / sqrt(gjj) : 0.0;
      const double g = a.G[(int64_t)i * N + j];
      ra += fabs(g);
      v = si * g * sj;
    } else {
      v = (i == j) ? 1.0 : 0.0;
    }
    a.A[(int64_t)i * Np + j] = v;
  }
  ra = block_sum(ra, scratch);
  if (threadIdx.x == 0) {
    a.s[i] = si;
    a.b[i] = (i < N) ? si * a.h[i] : 0.0;
    a.rowabs[i] = ra;
    a.theta[i] = 0.0;
  }
}

// Cholesky of diagonal tile k in LDS (right-looking, 256 threads).
__global__ __launch_bounds__(256) void k_potrf_tile(SolveArgs a, int k) {
  if (a.flags[1] != 0) return;
  __shared__ double T[kTile][kTile + 1];
  __shared__ int failed;
  const int tid = threadIdx.x;
  const int64_t o = (int64_t)k * kTile;
  for (int idx = tid; idx < kTile * kTile; idx += 256) {
    const int i = idx / kTile, j = idx % kTile;
    T[i][j] = a.A[(o + i) * a.Np + o + j];
  }
  if (tid == 0) failed = -1;
  __syncthreads();
  for (int j = 0; j < kTile; ++j) {
    const double d = T[j][j];
    if (!(d > 0.0) || !is_finite_d(d)) {
      if (tid == 0) failed = j;
      break;
    }
    const double dsq = sqrt(d);
    if (tid < kTile && tid > j) T[tid][j] /= dsq;
    __syncthreads();
    if (tid == j) T[j][j] = dsq;
    const int i = tid & (kTile - 1);
    if (i > j) {
      const double tij = T[i][j];
      for (int l = j + 1 + (tid >> 6); l <= i; l += 4) T[i][l] = fma(-tij, T[l][j], T[i][l]);
    }
    __syncthreads();
  }
  __syncthreads();
  if (failed >= 0) {
    if (tid == 0) {
      a.flags[1] = (int)(o + failed) + 1;
    }
    return;
  }
  for (int idx = tid; idx < kTile * kTile; idx += 256) {
    const int i = idx / kTile, j = idx % kTile;
    a.A[(o + i) * a.Np + o + j] = (i >= j) ? T[i][j] : 0.0;
  }
}

// Panel: L_ik = A_ik L_kk^-T for row tiles i > k (one workgroup per tile);
// each row by forward substitution, 4 lanes per row.
__global__ __launch_bounds__(256) void k_trsm_panel(SolveArgs a, int k) {
  if (a.flags[1] != 0) return;
  __shared__ double Lk[kTile][kTile + 1];
  __shared__ double X[kTile][kTile + 1];
  const int tid = threadIdx.x;
  const int64_t o = (int64_t)k * kTile;
  const int64_t oi = (int64_t)(k + 1 + blockIdx.x) * kTile;
  for (int idx = tid; idx < kTile * kTile; idx += 256) {
    const int i = idx / kTile, j = idx % kTile;
    Lk[i][j] = a.A[(o + i) * a.Np + o + j];
    X[i][j] = a.A[(oi + i) * a.Np + o + j];
  }
  __syncthreads();
  const int row = tid >> 2, part = tid & 3;
  for (int j = 0; j < kTile; ++j) {
    double s = 0.0;
    for (int l = part; l < j; l += 4) s = fma(Lk[j][l], X[row][l], s);
    s += __shfl_xor(s, 1, 64);
    s += __shfl_xor(s, 2, 64);
    if (part == 0) X[row][j] = (X[row][j] - s) / Lk[j][j];
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  for (int idx = tid; idx < kTile * kTile; idx += 256) {
    const int i = idx / kTile, j = idx % kTile;
    a.A[(oi + i) * a.Np + o + j] = X[i][j];
  }
}

// Trailing update A_ij -= L_ik L_jk^T for k < j <= i (one workgroup per tile).
__global__ __launch_bounds__(256) void k_syrk_tile(SolveArgs a, int k) {
  if (a.flags[1] != 0) return;
  __shared__ double Li[kTile][kTile + 1];
  __shared__ double Lj[kTile][kTile + 1];
  // decode lower-triangular tile index t -> (ti, tj), tj <= ti, both in [k+1, nt)
  int t = blockIdx.x;
  int ti = 0;
  while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
  const int tj = t - ti * (ti + 1) / 2;
  const int I = k + 1 + ti, J = k + 1 + tj;
  const int tid = threadIdx.x;
  const int64_t o = (int64_t)k * kTile, oi = (int64_t)I * kTile, oj = (int64_t)J * kTile;
  for (int idx = tid; idx < kTile * kTile; idx += 256) {
    const int i = idx / kTile, j = idx % kTile;
    Li[i][j] = a.A[(oi + i) * a.Np + o + j];
    Lj[i][j] = a.A[(oj + i) * a.Np + o + j];
  }
  __syncthreads();
  // each thread: 4 rows x 4 cols
  const int r0 = (tid >> 4) * 4, c0 = (tid & 15) * 4;
  double acc[4][4] = {};
  for (int l = 0; l < kTile; ++l) {
    double av[4], bv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) { av[u] = Li[r0 + u][l]; bv[u] = Lj[c0 + u][l]; }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[u][v] = fma(av[u], bv[v], acc[u][v]);
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t idx = (oi + r0 + u) * a.Np + oj + c0 + v;
      a.A[idx] -= acc[u][v];
    }
}

// Inverse of every diagonal factor L_kk (one workgroup per tile), rows of
// the inverse in sequence: X_i = (e_i - sum_{l<i} L_il X_l) / L_ii.
__global__ __launch_bounds__(256) void k_tile_inverse(SolveArgs a) {
  if (a.flags[1] != 0) return;
  __shared__ double Lk[kTile][kTile + 1];
  __shared__ double X[kTile][kTile + 1];
  __shared__ double part[4][kTile];
  const int k = blockIdx.x, tid = threadIdx.x;
  const int64_t o = (int64_t)k * kTile;
  for (int idx = tid; idx < kTile * kTile; idx += 256) {
    const int i = idx / kTile, j = idx % kTile;
    Lk[i][j] = a.A[(o + i) * a.Np + o + j];
    X[i][j] = 0.0;
  }
  __syncthreads();
  const int j = tid & 63, q = tid >> 6;
  for (int i = 0; i < kTile; ++i) {
    double s = 0.0;
    if (j < i)
      for (int l = j + q; l < i; l += 4) s = fma(Lk[i][l], X[l][j], s);
    part[q][j] = s;
    __syncthreads();
    if (tid < kTile && j <= i) {
      const double tot = part[0][j] + part[1][j] + part[2][j] + part[3][j];
      X[i][j] = ((i == j ? 1.0 : 0.0) - tot) / Lk[i][i];
    }
    __syncthreads();
  }
  double* out = a.Linv + (int64_t)k * kTile * kTile;
  for (int idx = tid; idx < kTile * kTile; idx += 256) out[idx] = X[idx / kTile][idx % kTile];
}

// x = A^-1 rhs with A = L L^T: blocked forward then backward substitution
// using the diagonal inverses. One workgroup of 1024 threads. `mode` 0:
// theta = s .* x;  mode 1: theta += s .* x (refinement update).
// rhs_scaled: the right-hand side in the equilibrated system.
__global__ __launch_bounds__(1024) void k_trsv(SolveArgs a, const double* rhs, int mode) {
  if (a.flags[1] != 0) return;
  extern __shared__ double vbuf[];     // Np
  __shared__ double blk[kTile];
  const int tid = threadIdx.x, Np = a.Np, nt = a.nt;
  for (int i = tid; i < Np; i += 1024) vbuf[i] = rhs[i];
  __syncthreads();
  const int lane = tid & 63, wid = tid >> 6;    // 16 waves
  // forward: z_k = Linv_kk (v_k - sum_{j<k} L_kj z_j); the sum is applied eagerly
  for (int k = 0; k < nt; ++k) {
    const double* Li = a.Linv + (int64_t)k * kTile * kTile;
    // row i of the block: wave w handles rows w, w+16, ...
    for (int i = wid; i < kTile; i += 16) {
      double s = Li[i * kTile + lane] * vbuf[k * kTile + lane];
      s = wave_sum(s);
      if (lane == 0) blk[i] = s;
    }
    __syncthreads();
    if (tid < kTile) vbuf[k * kTile + tid] = blk[tid];
    __syncthreads();
    // v_i -= L_i,k z_k for rows i beyond block k
    for (int i = (k + 1) * kTile + tid; i < Np; i += 1024) {
      const double* Lr = a.A + (int64_t)i * Np + (int64_t)k * kTile;
      double s = 0.0;
#pragma unroll 8
      for (int l = 0; l < kTile; ++l) s = fma(Lr[l], vbuf[k * kTile + l], s);
      vbuf[i] -= s;
    }
    __syncthreads();
  }
  // backward: x_k = Linv_kk^T (z_k - sum_{i>k} L_ik^T x_i)
  for (int k = nt - 1; k >= 0; --k) {
    const double* Li = a.Linv + (int64_t)k * kTile * kTile;
    for (int i = wid; i < kTile; i += 16) {
      // (Linv^T v)_i = sum_l Linv[l][i] v_l
      double s = Li[lane * kTile + i] * vbuf[k * kTile + lane];
      s = wave_sum(s);
      if (lane == 0) blk[i] = s;
    }
    __syncthreads();
    if (tid < kTile) vbuf[k * kTile + tid] = blk[tid];
    __syncthreads();
    // v_j -= L_kj^T x_k for columns j < block k: v_j -= sum_l L[k*64+l][j] x_l
    for (int jcol = tid; jcol < k * kTile; jcol += 1024) {
      double s = 0.0;
#pragma unroll 8
      for (int l = 0; l < kTile; ++l)
        s = fma(a.A[(int64_t)(k * kTile + l) * Np + jcol], vbuf[k * kTile + l], s);
      vbuf[jcol] -= s;
    }
    __syncthreads();
  }
  for (int i = tid; i < Np; i += 1024) {
    const double v = a.s[i] * vbuf[i];
    if (mode == 0) a.theta[i] = v;
    else a.theta[i] += v;
  }
}

// residual: rvec = D (h - G theta) (equilibrated), rowabs kept; one row per wave
__global__ __launch_bounds__(256) void k_residual(SolveArgs a) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= a.Np) return;
  if (i >= a.N) {
    if (lane == 0) a.rvec[i] = 0.0;
    return;
  }
  double s = 0.0;
  const double* Gr = a.G + (int64_t)i * a.N;
  for (int j = lane; j < a.N; j += 64) s = fma(Gr[j], a.theta[j], s);
  s = wave_sum(s);
  if (lane == 0) a.rvec[i] = a.s[i] * (a.h[i] - s);
}

// final: coefficients, backward error, pivot range, status
__global__ __launch_bounds__(1024) void k_solve_final(SolveArgs a, int refine) {
  __shared__ double sc[16];
  const int tid = threadIdx.x;
  const int N = a.N;
  const bool failed = a.flags[1] != 0;
  double rmax = 0.0, tmax = 0.0, hmax = 0.0, gmax = 0.0, pmin = 1e308, pmax = 0.0;
  for (int i = tid; i < N; i += 1024) {
    const double si = a.s[i];
    // rvec holds D (h - G theta) from the last k_residual call
    const double ri = (si > 0.0) ? fabs(a.rvec[i] / si) : 0.0;
    rmax = fmax(rmax, ri);
    tmax = fmax(tmax, fabs(a.theta[i]));
    hmax = fmax(hmax, fabs(a.h[i]));
    gmax = fmax(gmax, a.rowabs[i]);
    if (!failed) {
      const double p = a.A[(int64_t)i * a.Np + i];
      pmin = fmin(pmin, p);
      pmax = fmax(pmax, p);
    }
    a.coef[i] = failed ? __builtin_nan("") : a.theta[i];
  }
  auto bmax = [&](double v) {
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    __syncthreads();
    if ((tid & 63) == 0) sc[tid >> 6] = v;
    __syncthreads();
    double m = sc[0];
    for (int w = 1; w < 16; ++w) m = fmax(m, sc[w]);
    return m;
  };
  rmax = bmax(rmax);
  tmax = bmax(tmax);
  hmax = bmax(hmax);
  gmax = bmax(gmax);
  pmax = bmax(pmax);
  pmin = -bmax(-pmin);
  if (tid == 0) {
    sfft_solve_info* inf = a.info;
    // a non-finite input pixel is the root cause of any later failure
    if (failed) {
      inf->status = SFFT_ERR_NOT_SPD;
      inf->failed_pivot = a.flags[1] - 1;
      inf->backward_err = __builtin_nan("");
    } else {
      inf->backward_err = rmax / (gmax * tmax + hmax);
      inf->min_pivot = pmin;
      inf->max_pivot = pmax;
      inf->refine_iters = refine;
    }
    if (inf->nonfinite) inf->status = SFFT_ERR_NONFINITE;
  }
}

hipError_t launch_solve(const sfft_desc& d, const double* G, const double* h, double* coef,
                        int max_refine, sfft_solve_info* info, unsigned char* ws,
                        const Prof* pf, hipStream_t st) {
  const Geometry g = make_geometry(d);
  const Layout l = make_layout(g);
  SolveArgs a{};
  a.G = G; a.h = h; a.coef = coef; a.info = info;
  a.A = reinterpret_cast<double*>(ws + l.A);
  a.s = reinterpret_cast<double*>(ws + l.s);
  a.b = reinterpret_cast<double*>(ws + l.b);
  a.theta = reinterpret_cast<double*>(ws + l.theta);
  a.x = reinterpret_cast<double*>(ws + l.x);
  a.rvec = reinterpret_cast<double*>(ws + l.rvec);
  a.rowabs = reinterpret_cast<double*>(ws + l.rowabs);
  a.Linv = reinterpret_cast<double*>(ws + l.Linv);
  a.flags = reinterpret_cast<int*>(ws + l.flags);
  a.N = g.N; a.nt = l.nt; a.Np = l.nt * kTile;
  hipError_t e;
#define SFFT_CHECK_LAUNCH() do { if ((e = hipGetLastError()) != hipSuccess) return e; } while (0)
  prof_begin(pf, SFFT_PROF_SOLVE, st);
  hipLaunchKernelGGL(k_solve_init, dim3(1), dim3(64), 0, st, a);
  SFFT_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_equil, dim3(a.Np), dim3(256), 0, st, a);
  SFFT_CHECK_LAUNCH();
  for (int k = 0; k < a.nt; ++k) {
    hipLaunchKernelGGL(k_potrf_tile, dim3(1), dim3(256), 0, st, a, k);
    SFFT_CHECK_LAUNCH();
    const int rest = a.nt - k - 1;
    if (rest > 0) {
      hipLaunchKernelGGL(k_trsm_panel, dim3(rest), dim3(256), 0, st, a, k);
      SFFT_CHECK_LAUNCH();
      hipLaunchKernelGGL(k_syrk_tile, dim3(rest * (rest + 1) / 2), dim3(256), 0, st, a, k);
      SFFT_CHECK_LAUNCH();
    }
  }
  hipLaunchKernelGGL(k_tile_inverse, dim3(a.nt), dim3(256), 0, st, a);
  SFFT_CHECK_LAUNCH();
  const size_t sh = sizeof(double) * a.Np;
  hipLaunchKernelGGL(k_trsv, dim3(1), dim3(1024), sh, st, a, (const double*)a.b, 0);
  SFFT_CHECK_LAUNCH();
  for (int it = 0; it < max_refine; ++it) {
    hipLaunchKernelGGL(k_residual, dim3((a.Np + 3) / 4), dim3(256), 0, st, a);
    SFFT_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_trsv, dim3(1), dim3(1024), sh, st, a, (const double*)a.rvec, 1);
    SFFT_CHECK_LAUNCH();
  }
  hipLaunchKernelGGL(k_residual, dim3((a.Np + 3) / 4), dim3(256), 0, st, a);
  SFFT_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_solve_final, dim3(1), dim3(1024), 0, st, a, max_refine);
  SFFT_CHECK_LAUNCH();
  prof_end(pf, SFFT_PROF_SOLVE, st);
#undef SFFT_CHECK_LAUNCH
  return hipSuccess;
}

}  // namespace sfft
