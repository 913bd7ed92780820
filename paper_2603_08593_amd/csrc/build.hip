// sfft_build_system kernels: normal equations of the delta-basis fit.
//
// Method (paper Sec. 1, Sec. 2.3.2): SFFT assembles the least-squares
// normal equations of the spatially varying delta-basis kernel in the
// Fourier domain. Every kernel-kernel block entry is a periodic
// cross-correlation C_ij(D) = sum_u P_i(u) P_j(u + D) of two
// polynomial-weighted reference images P_i = p_i R', every kernel-science
// entry is C_{P_i,S'}(d). Here each correlation is computed as
//   row pass   : DFT along x of xt^a R' (a = 0..DK) and of S' (one row per
//                step, radix-8 Stockham in LDS, two real rows packed into one
//                complex transform);
//   column pass: for every k_x column, the correlation along y restricted to
//                lags |Dy| <= L-1, computed blockwise (blocks of T rows with
//                an (L-1)-row halo, 128-point FFTs, products accumulated
//                over blocks, one inverse per column);
//   x-inverse  : pruned inverse DFT over k_x at lags |Dx| <= L-1.
// The kernel-background block and the background blocks are exact
// polynomial moments of R' and S' with periodic seam corrections (they need
// no transform).
#include "common.hpp"
#include "layout.hpp"

namespace sfft {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------

__global__ void k_fill_i32(int* p, int n, int v) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__device__ __forceinline__ double ipow(double x, int n) {
  double r = 1.0;
  for (int k = 0; k < n; ++k) r *= x;
  return r;
}

__device__ __forceinline__ int pad8(int i) { return i + (i >> 3); }
__device__ __forceinline__ int pad16(int i) { return i + (i >> 4); }

// ---------------------------------------------------------------------------
// Stockham FFT of length N (power of two, <= 4096) in LDS, 256 threads.
// buf uses the padded index pad8(i); tw[m] = exp(-2 pi i m / N).
// Output in natural order.
// ---------------------------------------------------------------------------

template <typename T, int R, bool INV, int NQ>
__device__ __forceinline__ void stockham_pass(cx<T>* buf, const cx<T>* tw, int N, int Ns) {
  constexpr int MAXB = (NQ / R) > 0 ? (NQ / R) : 1;
  const int nb = N / R;
  const int tstride = N / (Ns * R);
  cx<T> v[MAXB][R];
#pragma unroll
  for (int t = 0; t < MAXB; ++t) {
    const int j = threadIdx.x + t * kRowThreads;
    if (j < nb) {
      const int k = j & (Ns - 1);
#pragma unroll
      for (int r = 0; r < R; ++r) v[t][r] = buf[pad8(j + r * nb)];
      if (Ns > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          cx<T> w = tw[r * k * tstride];
          if (INV) w.im = -w.im;
          v[t][r] = cmul(v[t][r], w);
        }
      }
      dft_r<T, R, INV>(v[t]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int t = 0; t < MAXB; ++t) {
    const int j = threadIdx.x + t * kRowThreads;
    if (j < nb) {
      const int k = j & (Ns - 1);
      const int base = (j - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[pad8(base + r * Ns)] = v[t][r];
    }
  }
  __syncthreads();
}

template <typename T, bool INV, int NQ>
__device__ void fft_lds(cx<T>* buf, const cx<T>* tw, int N, int logN) {
  int Ns = 1;
  int rem = logN;
  while (rem >= 3) {
    stockham_pass<T, 8, INV, NQ>(buf, tw, N, Ns);
    Ns *= 8;
    rem -= 3;
  }
  if (rem == 2) stockham_pass<T, 4, INV, NQ>(buf, tw, N, Ns);
  else if (rem == 1) stockham_pass<T, 2, INV, NQ>(buf, tw, N, Ns);
}

// ---------------------------------------------------------------------------
// Row pass
// ---------------------------------------------------------------------------

struct RowArgs {
  const void* R;
  const void* S;
  int64_t ld;
  int W, H, DK, DB, r, logW;
  double cR, cS, sx;
  void* F;            // cx<T>[nsig][H][pitchK]
  int64_t pitchK, planeK;
  double* MR;         // [DK+DB+1][H]
  double* MS;         // [DB+1][H]
  double* ER;         // [H][2r]
  int* flags;
  const void* twW;    // cx<T>[W]
};

// NQ: row elements per thread, max(1, W / 256)
template <typename T, typename TIN, int NQ>
__global__ __launch_bounds__(kRowThreads) void k_row_pass(RowArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int W = a.W;
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* tw = buf + (W + W / 8);
  double* red = reinterpret_cast<double*>(tw + W);   // [kRowThreads/64][16]
  const cx<T>* twg = static_cast<const cx<T>*>(a.twW);
  for (int i = threadIdx.x; i < W; i += kRowThreads) tw[i] = twg[i];
  constexpr int MAXQ = NQ;
  const int nm = a.DK + a.DB + 1;
  const int nsig = a.DK + 2;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  cx<T>* F = static_cast<cx<T>*>(a.F);

  for (int y = blockIdx.x; y < a.H; y += gridDim.x) {
    double rp[MAXQ], sp[MAXQ];
    double mr[9], ms[5];
#pragma unroll
    for (int m = 0; m < 9; ++m) mr[m] = 0.0;
#pragma unroll
    for (int m = 0; m < 5; ++m) ms[m] = 0.0;
    bool bad = false;
#pragma unroll
    for (int q = 0; q < MAXQ; ++q) {
      const int x = threadIdx.x + q * kRowThreads;
      rp[q] = 0.0;
      sp[q] = 0.0;
      if (x < W) {
        const double rv = load_pix<TIN>(a.R, (int64_t)y * a.ld + x) - a.cR;
        const double sv = load_pix<TIN>(a.S, (int64_t)y * a.ld + x) - a.cS;
        bad |= !(is_finite_d(rv) && is_finite_d(sv));
        rp[q] = rv;
        sp[q] = sv;
        const double xt = (double)x * a.sx - 1.0;
        double pw = 1.0;
#pragma unroll
        for (int m = 0; m < 9; ++m) {
          if (m < nm) mr[m] = fma(pw, rv, mr[m]);
          if (m <= a.DB && m < 5) ms[m] = fma(pw, sv, ms[m]);
          pw *= xt;
        }
        if (x < a.r) a.ER[(int64_t)y * 2 * a.r + x] = rv;
        if (x >= W - a.r) a.ER[(int64_t)y * 2 * a.r + a.r + (x - (W - a.r))] = rv;
      }
    }
    if (bad) atomicOr(a.flags, 1);
    // moments: wave sums, then one value per (wave, moment) in LDS
#pragma unroll
    for (int m = 0; m < 9; ++m) {
      if (m < nm) {
        double v = wave_sum(mr[m]);
        if (lane == 0) red[wid * 16 + m] = v;
      }
    }
#pragma unroll
    for (int m = 0; m < 5; ++m) {
      if (m <= a.DB) {
        double v = wave_sum(ms[m]);
        if (lane == 0) red[wid * 16 + 9 + m] = v;
      }
    }
    __syncthreads();
    if (threadIdx.x < 16) {
      const int m = threadIdx.x;
      double s = 0.0;
      for (int w = 0; w < kRowThreads / 64; ++w) s += red[w * 16 + m];
      if (m < nm) a.MR[(int64_t)m * a.H + y] = s;
      else if (m >= 9 && m - 9 <= a.DB) a.MS[(int64_t)(m - 9) * a.H + y] = s;
    }
    // transforms: real signals s_a = xt^a R' (a <= DK), s_{DK+1} = S',
    // packed two per complex transform
    for (int f = 0; 2 * f < nsig; ++f) {
      const int s0 = 2 * f, s1 = 2 * f + 1;
#pragma unroll
      for (int q = 0; q < MAXQ; ++q) {
        const int x = threadIdx.x + q * kRowThreads;
        if (x < W) {
          const double xt = (double)x * a.sx - 1.0;
          const double v0 = (s0 <= a.DK) ? ipow(xt, s0) * rp[q] : sp[q];
          double v1 = 0.0;
          if (s1 < nsig) v1 = (s1 <= a.DK) ? ipow(xt, s1) * rp[q] : sp[q];
          buf[pad8(x)] = cx<T>{(T)v0, (T)v1};
        }
      }
      __syncthreads();
      fft_lds<T, false, NQ>(buf, tw, W, a.logW);
      const int half = W / 2;
      for (int kx = threadIdx.x; kx <= half; kx += kRowThreads) {
        const cx<T> z1 = buf[pad8(kx)];
        const cx<T> z2 = cconj(buf[pad8((W - kx) & (W - 1))]);
        const cx<T> A = cscale(cadd(z1, z2), (T)0.5);
        const cx<T> d = csub(z1, z2);
        const cx<T> B = {d.im * (T)0.5, -d.re * (T)0.5};
        F[(int64_t)s0 * a.planeK + (int64_t)y * a.pitchK + kx] = A;
        if (s1 < nsig) F[(int64_t)s1 * a.planeK + (int64_t)y * a.pitchK + kx] = B;
      }
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------
// Column pass: blocked correlation along y for 4 adjacent k_x columns
// ---------------------------------------------------------------------------

struct ColArgs {
  const void* F;
  int64_t pitchK, planeK;
  int H, nkx, h, T, ngroups, DK;
  double sy;
  cx<double>* strips;   // [NP][2h+1][nkx]
  const void* tw128;    // cx<T>[128], exp(-2 pi i m / 128)
};

template <int NK> struct PairCount { static constexpr int NKK = NK * (NK + 1) / 2, NP = NKK + NK; };

// layout of the kernel-term spectra: exponents (a, b) of term g
__device__ __forceinline__ void mono_ab(int g, int& a, int& b) {
  // order: d = 0..: b = 0..d, a = d - b
  int d = 0, start = 0;
  while (g >= start + d + 1) { start += d + 1; ++d; }
  b = g - start;
  a = d - b;
}

template <typename T, int NK>
__global__ __launch_bounds__(kColThreads) void k_col_pass(ColArgs a) {
  constexpr int NS = 2 * NK + 1;
  constexpr int NKK = PairCount<NK>::NKK;
  constexpr int NP = PairCount<NK>::NP;
  constexpr int SPAD = 136;
  // column stride (complex elements) congruent to 4 mod 16: stage-1 writes
  // of 4 columns x 4 butterflies hit distinct LDS banks
  constexpr int CS0 = NS * SPAD;
  constexpr int CS = CS0 + ((4 - (CS0 % 16)) + 16) % 16;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* spec = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* tw = spec + kColsPerWG * CS;
  const cx<T>* twg = static_cast<const cx<T>*>(a.tw128);
  if (threadIdx.x < kTP) tw[threadIdx.x] = twg[threadIdx.x];

  // XCD-aware group index: workgroups that share an XCD (id mod 8) take
  // adjacent column groups, so their 64-byte row segments share L2 lines.
  const int per_xcd = (a.ngroups + 7) / 8;
  const int grp = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (grp >= a.ngroups) return;
  const int kx0 = grp * kColsPerWG;
  const cx<T>* F = static_cast<const cx<T>*>(a.F);
  const int tid = threadIdx.x;
  const int H = a.H, h = a.h;

  cx<T> acc[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) acc[p] = cx<T>{(T)0, (T)0};
  __syncthreads();

  for (int yb = 0; yb < H; yb += a.T) {
    const int Tb = min(a.T, H - yb);
    // ---- stage 1: gather weighted rows, radix-16 over rows j + 8q
    if (tid < kColsPerWG * NS * 8) {
      const int c = tid & 3;
      const int rest = tid >> 2;
      const int j = rest & 7;
      const int s = rest >> 3;            // 0..NS-1
      const int kx = kx0 + c;
      const bool colok = kx < a.nkx;
      int base, bpow;
      bool is_u;
      if (s < NK) { int ea, eb; mono_ab(s, ea, eb); base = ea; bpow = eb; is_u = true; }
      else if (s < 2 * NK) { int ea, eb; mono_ab(s - NK, ea, eb); base = ea; bpow = eb; is_u = false; }
      else { base = a.DK + 1; bpow = 0; is_u = false; }
      const cx<T>* Fb = F + (int64_t)base * a.planeK + kx;
      cx<T> v[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int m = j + 8 * q;
        const int o = (m < kTP - h) ? m : m - kTP;
        const bool in = is_u ? (o >= 0 && o < Tb) : (o >= -h && o < Tb + h);
        int y = yb + o;
        y = (y < 0) ? y + H : ((y >= H) ? y - H : y);
        cx<T> val = {(T)0, (T)0};
        if (in && colok) {
          val = Fb[(int64_t)y * a.pitchK];
          if (bpow > 0) {
            const double yt = (double)y * a.sy - 1.0;
            const double wgt = ipow(yt, bpow);
            val = cscale(val, (T)wgt);
          }
        }
        v[q] = val;
      }
      dft16<T, false>(v);
      cx<T>* dst = spec + c * CS + s * SPAD;
#pragma unroll
      for (int r = 0; r < 16; ++r) dst[pad16(16 * j + r)] = v[r];
    }
    __syncthreads();
    // ---- stage 2: radix-8, Ns = 16 (twiddle exp(-2 pi i r j / 128)).
    // As the last Stockham stage it reads and writes the same 8 slots
    // (j + 16 r), so each butterfly is updated in place.
    {
      constexpr int NB2 = kColsPerWG * NS * 16;
      for (int t = tid; t < NB2; t += kColThreads) {
        const int j = t & 15;
        const int cs = t >> 4;
        const int c = cs % kColsPerWG, s = cs / kColsPerWG;
        cx<T>* p = spec + c * CS + s * SPAD;
        cx<T> v[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          cx<T> x = p[pad16(j + 16 * r)];
          if (r > 0) x = cmul(x, tw[r * j]);
          v[r] = x;
        }
        dft8<T, false>(v);
#pragma unroll
        for (int r = 0; r < 8; ++r) p[pad16(j + 16 * r)] = v[r];
      }
      __syncthreads();
    }
    // ---- products: thread (column, k_y)
    {
      const int c = tid >> 7, k = tid & 127;
      const cx<T>* src = spec + c * CS + pad16(k);
      cx<T> U[NK], V[NK + 1];
#pragma unroll
      for (int i = 0; i < NK; ++i) U[i] = src[i * SPAD];
#pragma unroll
      for (int i = 0; i <= NK; ++i) V[i] = src[(NK + i) * SPAD];
      int p = 0;
#pragma unroll
      for (int i = 0; i < NK; ++i)
#pragma unroll
        for (int jj = i; jj < NK; ++jj) { cmac_conj(acc[p], U[i], V[jj]); ++p; }
#pragma unroll
      for (int i = 0; i < NK; ++i) cmac_conj(acc[NKK + i], U[i], V[NK]);
    }
    __syncthreads();
  }

  // ---- per-column inverse transforms of the accumulated products
  for (int p0 = 0; p0 < NP; p0 += NS) {
    const int np = min(NS, NP - p0);
    {
      const int c = tid >> 7, k = tid & 127;
      cx<T>* dst = spec + c * CS + pad16(k);
#pragma unroll
      for (int p = 0; p < NP; ++p)
        if (p >= p0 && p < p0 + np) dst[(p - p0) * SPAD] = acc[p];
    }
    __syncthreads();
    // stage A: radix-16, Ns = 1
    {
      cx<T> v[16];
      const bool act = tid < kColsPerWG * np * 8;
      int c = 0, s = 0, j = 0;
      if (act) {
        c = tid & 3;
        const int rest = tid >> 2;
        j = rest & 7;
        s = rest >> 3;
        const cx<T>* src = spec + c * CS + s * SPAD;
#pragma unroll
        for (int q = 0; q < 16; ++q) v[q] = src[pad16(j + 8 * q)];
        dft16<T, true>(v);
      }
      __syncthreads();
      if (act) {
        cx<T>* dst = spec + c * CS + s * SPAD;
#pragma unroll
        for (int r = 0; r < 16; ++r) dst[pad16(16 * j + r)] = v[r];
      }
      __syncthreads();
    }
    // stage B: radix-8, Ns = 16, inverse twiddles, in place per butterfly
    {
      const int nb2 = kColsPerWG * np * 16;
      for (int t = tid; t < nb2; t += kColThreads) {
        const int j = t & 15;
        const int cs = t >> 4;
        const int c = cs % kColsPerWG, s = cs / kColsPerWG;
        cx<T>* p = spec + c * CS + s * SPAD;
        cx<T> v[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          cx<T> x = p[pad16(j + 16 * r)];
          if (r > 0) x = cmul(x, cconj(tw[r * j]));
          v[r] = x;
        }
        dft8<T, true>(v);
#pragma unroll
        for (int r = 0; r < 8; ++r) p[pad16(j + 16 * r)] = v[r];
      }
      __syncthreads();
    }
    // write lags |dy| <= h of each inverse, scaled by 1/128
    {
      const int ndy = 2 * h + 1;
      const int total = kColsPerWG * np * ndy;
      for (int t = tid; t < total; t += kColThreads) {
        const int c = t % kColsPerWG;
        const int rest = t / kColsPerWG;
        const int dyi = rest % ndy;
        const int s = rest / ndy;
        const int kx = kx0 + c;
        if (kx < a.nkx) {
          const int idx = (dyi - h) & (kTP - 1);
          const cx<T> vv = spec[c * CS + s * SPAD + pad16(idx)];
          const double sc = 1.0 / kTP;
          a.strips[((int64_t)(p0 + s) * ndy + dyi) * a.nkx + kx] =
              cx<double>{(double)vv.re * sc, (double)vv.im * sc};
        }
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Pruned inverse along x: C_p(dx, dy) = (1/W) sum_kx w_kx Re(e^{2 pi i kx dx / W} c_p(kx, dy))
// ---------------------------------------------------------------------------

struct XinvArgs {
  const cx<double>* strips;
  double* C;            // [NP][2h+1][2h+1]
  const cx<double>* twW;  // exp(-2 pi i m / W), FP64
  int W, nkx, h, r, NKK, NP;
};

__global__ __launch_bounds__(256) void k_strip_xinv(XinvArgs a) {
  __shared__ double red[4][32];
  const int ndy = 2 * a.h + 1;
  const int p = blockIdx.x / ndy, dyi = blockIdx.x % ndy;
  const bool ks = p >= a.NKK;
  const int lim = ks ? a.r : a.h;
  if (abs(dyi - a.h) > lim) return;
  const int ndx = 2 * lim + 1;
  double acc[32];
#pragma unroll
  for (int t = 0; t < 32; ++t) acc[t] = 0.0;
  const cx<double>* row = a.strips + ((int64_t)p * ndy + dyi) * a.nkx;
  for (int kx = threadIdx.x; kx < a.nkx; kx += blockDim.x) {
    const cx<double> c = row[kx];
    const double wk = (kx == 0 || 2 * kx == a.W) ? 1.0 : 2.0;
#pragma unroll
    for (int t = 0; t < 32; ++t) {
      if (t < ndx) {
        const int dx = t - lim;
        const int idx = (int)(((int64_t)kx * (dx + a.W)) % a.W);
        const cx<double> w = a.twW[idx];   // (cos, -sin)
        acc[t] = fma(wk, w.re * c.re + w.im * c.im, acc[t]);
      }
    }
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int t = 0; t < 32; ++t) {
    if (t < ndx) {
      double v = wave_sum(acc[t]);
      if (lane == 0) red[wid][t] = v;
    }
  }
  __syncthreads();
  if (threadIdx.x < ndx) {
    const int t = threadIdx.x;
    const double s = red[0][t] + red[1][t] + red[2][t] + red[3][t];
    const int dx = t - lim;
    a.C[((int64_t)p * ndy + dyi) * ndy + (dx + a.h)] = s / (double)a.W;
  }
}

// ---------------------------------------------------------------------------
// Polynomial moments
// ---------------------------------------------------------------------------

struct MomArgs {
  const double* MR;   // [nm][H]
  const double* MS;   // [DB+1][H]
  const double* ER;   // [H][2r]
  double* mom;
  int W, H, DK, DB, r;
  double sx, sy;
};

// One workgroup per moment scalar; fixed-order block sums.
__global__ __launch_bounds__(256) void k_moments(MomArgs a) {
  __shared__ double scratch[8];
  const int nm = a.DK + a.DB + 1;
  const int nM2 = nm * nm, nE = 2 * a.r * nm, nMS = (a.DB + 1) * (a.DB + 1);
  const int np = 2 * a.DB + 1;
  int id = blockIdx.x;
  double s = 0.0;
  if (id < nM2) {
    const int m = id / nm, n = id % nm;
    for (int y = threadIdx.x; y < a.H; y += blockDim.x)
      s += ipow((double)y * a.sy - 1.0, n) * a.MR[(int64_t)m * a.H + y];
  } else if ((id -= nM2) < nE) {
    const int e = id / nm, n = id % nm;
    for (int y = threadIdx.x; y < a.H; y += blockDim.x)
      s += ipow((double)y * a.sy - 1.0, n) * a.ER[(int64_t)y * 2 * a.r + e];
  } else if ((id -= nE) < nMS) {
    const int ac = id / (a.DB + 1), bc = id % (a.DB + 1);
    for (int y = threadIdx.x; y < a.H; y += blockDim.x)
      s += ipow((double)y * a.sy - 1.0, bc) * a.MS[(int64_t)ac * a.H + y];
  } else if ((id -= nMS) < np) {
    for (int x = threadIdx.x; x < a.W; x += blockDim.x) s += ipow((double)x * a.sx - 1.0, id);
  } else {
    id -= np;
    for (int y = threadIdx.x; y < a.H; y += blockDim.x) s += ipow((double)y * a.sy - 1.0, id);
  }
  s = block_sum(s, scratch);
  if (threadIdx.x == 0) a.mom[blockIdx.x] = s;
}

// ---------------------------------------------------------------------------
// Kernel-background block, background block, background RHS
// ---------------------------------------------------------------------------

struct KbArgs {
  const double* mom;
  const double* MR;
  const double* ER;
  double* G;
  double* hv;
  int W, H, L, r, DK, DB, nK, nB, N;
  double sx, sy;
};

__device__ __forceinline__ double binom(int n, int k) {
  double b = 1.0;
  for (int t = 1; t <= k; ++t) b = b * (double)(n - k + t) / (double)t;
  return b;
}

__global__ __launch_bounds__(256) void k_kb_assemble(KbArgs a) {
  const int L2 = a.L * a.L;
  const int nKL = a.nK * L2;
  const int nm = a.DK + a.DB + 1;
  const double* M2 = a.mom;
  const double* E = M2 + nm * nm;
  const double* MSy = E + 2 * a.r * nm;
  const double* Px = MSy + (a.DB + 1) * (a.DB + 1);
  const double* Py = Px + 2 * a.DB + 1;
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  const int nkb = nKL * a.nB;
  if (tid < nkb) {
    const int c = tid % a.nB;
    const int row = tid / a.nB;
    const int i = row / L2, d = row % L2;
    const int dy = d / a.L - a.r, dx = d % a.L - a.r;
    int ai, bi, ac, bc;
    mono_ab(i, ai, bi);
    mono_ab(c, ac, bc);
    const int W = a.W, H = a.H, r = a.r;
    // x-seam columns of this dx: (ux, edge slot e)
    int xs0 = 0, xs1 = 0;   // ux range [xs0, xs1)
    if (dx > 0) { xs0 = W - dx; xs1 = W; }
    else if (dx < 0) { xs0 = 0; xs1 = -dx; }
    auto eslot = [&](int ux) { return ux < r ? ux : r + (ux - (W - r)); };
    auto dX = [&](int ux) {
      int w = ux + dx;
      w = (w < 0) ? w + W : (w >= W ? w - W : w);
      return ipow((double)w * a.sx - 1.0, ac) - ipow(-1.0 + a.sx * (double)(ux + dx), ac);
    };
    double tot = 0.0;
    for (int l = 0; l <= bc; ++l) {
      const int n = bi + l;
      double inner = 0.0;
      for (int k = 0; k <= ac; ++k)
        inner += binom(ac, k) * ipow(a.sx * dx, ac - k) * M2[(ai + k) * nm + n];
      for (int ux = xs0; ux < xs1; ++ux)
        inner += ipow((double)ux * a.sx - 1.0, ai) * dX(ux) * E[eslot(ux) * nm + n];
      tot += binom(bc, l) * ipow(a.sy * dy, bc - l) * inner;
    }
    int ys0 = 0, ys1 = 0;
    if (dy > 0) { ys0 = H - dy; ys1 = H; }
    else if (dy < 0) { ys0 = 0; ys1 = -dy; }
    for (int uy = ys0; uy < ys1; ++uy) {
      int w = uy + dy;
      w = (w < 0) ? w + H : (w >= H ? w - H : w);
      const double dY = ipow((double)w * a.sy - 1.0, bc) - ipow(-1.0 + a.sy * (double)(uy + dy), bc);
      double I = 0.0;
      for (int k = 0; k <= ac; ++k)
        I += binom(ac, k) * ipow(a.sx * dx, ac - k) * a.MR[(int64_t)(ai + k) * H + uy];
      for (int ux = xs0; ux < xs1; ++ux)
        I += ipow((double)ux * a.sx - 1.0, ai) * dX(ux) * a.ER[(int64_t)uy * 2 * r + eslot(ux)];
      tot += ipow((double)uy * a.sy - 1.0, bi) * dY * I;
    }
    a.G[(int64_t)row * a.N + nKL + c] = tot;
    a.G[(int64_t)(nKL + c) * a.N + row] = tot;
  } else if (tid < nkb + a.nB * a.nB) {
    const int t = tid - nkb;
    const int c = t / a.nB, c2 = t % a.nB;
    int ac, bc, ac2, bc2;
    mono_ab(c, ac, bc);
    mono_ab(c2, ac2, bc2);
    a.G[(int64_t)(nKL + c) * a.N + nKL + c2] = Px[ac + ac2] * Py[bc + bc2];
    if (c2 == 0) a.hv[nKL + c] = MSy[ac * (a.DB + 1) + bc];
  }
}

// ---------------------------------------------------------------------------
// Kernel-kernel block and kernel RHS from the correlation lags
// ---------------------------------------------------------------------------

struct GatherArgs {
  const double* C;    // [NP][2h+1][2h+1]
  double* G;
  double* hv;
  int L, r, h, nK, NKK, N;
};

__device__ __forceinline__ int pair_index(int i, int j, int nK) {
  return i * nK - i * (i - 1) / 2 + (j - i);
}

__global__ __launch_bounds__(256) void k_gather_kk(GatherArgs a) {
  const int L2 = a.L * a.L;
  const int nKL = a.nK * L2;
  const int row = blockIdx.y;
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  const int ndy = 2 * a.h + 1;
  const int i = row / L2, d = row % L2;
  const int dy = d / a.L - a.r, dx = d % a.L - a.r;
  if (col < nKL) {
    const int j = col / L2, d2 = col % L2;
    const int dy2 = d2 / a.L - a.r, dx2 = d2 % a.L - a.r;
    int p, Dy, Dx;
    if (i <= j) { p = pair_index(i, j, a.nK); Dy = dy - dy2; Dx = dx - dx2; }
    else { p = pair_index(j, i, a.nK); Dy = dy2 - dy; Dx = dx2 - dx; }
    a.G[(int64_t)row * a.N + col] = a.C[((int64_t)p * ndy + (Dy + a.h)) * ndy + (Dx + a.h)];
  }
  if (col == 0) {
    const int p = a.NKK + i;
    a.hv[row] = a.C[((int64_t)p * ndy + (dy + a.h)) * ndy + (dx + a.h)];
  }
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------

hipError_t prepare_kernel_attributes() {
  static const hipError_t once = [] {
    const int lim = 160 * 1024;
    hipError_t e = hipSuccess;
    auto set = [&](const void* f) {
      if (e == hipSuccess) e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    };
    set(reinterpret_cast<const void*>(&k_row_pass<double, double, 1>));
    set(reinterpret_cast<const void*>(&k_row_pass<double, double, 2>));
    set(reinterpret_cast<const void*>(&k_row_pass<double, double, 4>));
    set(reinterpret_cast<const void*>(&k_row_pass<double, double, 8>));
    set(reinterpret_cast<const void*>(&k_row_pass<double, double, 16>));
    set(reinterpret_cast<const void*>(&k_row_pass<double, float, 1>));
    set(reinterpret_cast<const void*>(&k_row_pass<double, float, 2>));
    set(reinterpret_cast<const void*>(&k_row_pass<double, float, 4>));
    set(reinterpret_cast<const void*>(&k_row_pass<double, float, 8>));
    set(reinterpret_cast<const void*>(&k_row_pass<double, float, 16>));
    set(reinterpret_cast<const void*>(&k_row_pass<float, double, 1>));
    set(reinterpret_cast<const void*>(&k_row_pass<float, double, 2>));
    set(reinterpret_cast<const void*>(&k_row_pass<float, double, 4>));
    set(reinterpret_cast<const void*>(&k_row_pass<float, double, 8>));
    set(reinterpret_cast<const void*>(&k_row_pass<float, double, 16>));
    set(reinterpret_cast<const void*>(&k_row_pass<float, float, 1>));
    set(reinterpret_cast<const void*>(&k_row_pass<float, float, 2>));
    set(reinterpret_cast<const void*>(&k_row_pass<float, float, 4>));
    set(reinterpret_cast<const void*>(&k_row_pass<float, float, 8>));
    set(reinterpret_cast<const void*>(&k_row_pass<float, float, 16>));
    set(reinterpret_cast<const void*>(&k_col_pass<double, 1>));
    set(reinterpret_cast<const void*>(&k_col_pass<double, 3>));
    set(reinterpret_cast<const void*>(&k_col_pass<double, 6>));
    set(reinterpret_cast<const void*>(&k_col_pass<float, 1>));
    set(reinterpret_cast<const void*>(&k_col_pass<float, 3>));
    set(reinterpret_cast<const void*>(&k_col_pass<float, 6>));
    return e;
  }();
  return once;
}

template <typename T>
static hipError_t launch_row(const Geometry& g, const sfft_desc& d, const void* R, const void* S,
                             unsigned char* ws, const Layout& l, const BuildPlan& p,
                             hipStream_t st) {
  RowArgs a{};
  a.R = R; a.S = S; a.ld = d.ld; a.W = g.W; a.H = g.H; a.DK = g.DK; a.DB = g.DB; a.r = g.r;
  int lw = 0;
  while ((1 << lw) < g.W) ++lw;
  a.logW = lw;
  a.cR = d.ref_pedestal; a.cS = d.sci_pedestal;
  a.sx = g.W > 1 ? 2.0 / (double)(g.W - 1) : 0.0;
  a.F = ws + l.F; a.pitchK = g.pitchK; a.planeK = g.planeK;
  a.MR = reinterpret_cast<double*>(ws + l.MR);
  a.MS = reinterpret_cast<double*>(ws + l.MS);
  a.ER = reinterpret_cast<double*>(ws + l.ER);
  a.flags = reinterpret_cast<int*>(ws + l.flags);
  a.twW = p.twW;
  const size_t shmem = sizeof(cx<T>) * (size_t)(g.W + g.W / 8 + g.W) + sizeof(double) * 64;
  int grid = g.H < 4 * p.num_cus ? g.H : 4 * p.num_cus;
  const bool f32 = d.image_dtype == SFFT_F32;
#define SFFT_ROW(NQ)                                                                          \
  do {                                                                                        \
    if (f32) hipLaunchKernelGGL((k_row_pass<T, float, NQ>), dim3(grid), dim3(kRowThreads),   \
                                shmem, st, a);                                               \
    else hipLaunchKernelGGL((k_row_pass<T, double, NQ>), dim3(grid), dim3(kRowThreads),      \
                            shmem, st, a);                                                   \
  } while (0)
  const int nq = g.W / kRowThreads;
  if (nq <= 1) SFFT_ROW(1);
  else if (nq == 2) SFFT_ROW(2);
  else if (nq == 4) SFFT_ROW(4);
  else if (nq == 8) SFFT_ROW(8);
  else SFFT_ROW(16);
#undef SFFT_ROW
  return hipGetLastError();
}

template <typename T, int NK>
static hipError_t launch_col(const Geometry& g, unsigned char* ws, const Layout& l,
                             const BuildPlan& p, hipStream_t st) {
  ColArgs a{};
  a.F = ws + l.F; a.pitchK = g.pitchK; a.planeK = g.planeK;
  a.H = g.H; a.nkx = g.nkx; a.h = g.h; a.T = g.T; a.DK = g.DK;
  a.ngroups = (g.nkx + kColsPerWG - 1) / kColsPerWG;
  a.sy = g.H > 1 ? 2.0 / (double)(g.H - 1) : 0.0;
  a.strips = reinterpret_cast<cx<double>*>(ws + l.strips);
  a.tw128 = p.tw128;
  constexpr int NS = 2 * NK + 1;
  constexpr int CS0 = NS * 136;
  constexpr int CS = CS0 + ((4 - (CS0 % 16)) + 16) % 16;
  const size_t shmem = sizeof(cx<T>) * ((size_t)kColsPerWG * CS + kTP);
  const int grid = 8 * ((a.ngroups + 7) / 8);
  hipLaunchKernelGGL((k_col_pass<T, NK>), dim3(grid), dim3(kColThreads), shmem, st, a);
  return hipGetLastError();
}

hipError_t launch_build(const sfft_desc& d, const void* R, const void* S, double* G, double* hv,
                        unsigned char* ws, const BuildPlan& p, const Prof* pf, hipStream_t st) {
  const Geometry g = make_geometry(d);
  const Layout l = make_layout(g);
  hipError_t e;
  prof_begin(pf, SFFT_PROF_BUILD, st);
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st,
                     reinterpret_cast<int*>(ws + l.flags), 64, 0);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  prof_begin(pf, SFFT_PROF_ROW_PASS, st);
  e = g.fp32 ? launch_row<float>(g, d, R, S, ws, l, p, st)
             : launch_row<double>(g, d, R, S, ws, l, p, st);
  prof_end(pf, SFFT_PROF_ROW_PASS, st);
  if (e != hipSuccess) return e;
  prof_begin(pf, SFFT_PROF_COL_PASS, st);
  switch (g.nK) {
    case 1: e = g.fp32 ? launch_col<float, 1>(g, ws, l, p, st) : launch_col<double, 1>(g, ws, l, p, st); break;
    case 3: e = g.fp32 ? launch_col<float, 3>(g, ws, l, p, st) : launch_col<double, 3>(g, ws, l, p, st); break;
    case 6: e = g.fp32 ? launch_col<float, 6>(g, ws, l, p, st) : launch_col<double, 6>(g, ws, l, p, st); break;
    default: return hipErrorInvalidValue;
  }
  prof_end(pf, SFFT_PROF_COL_PASS, st);
  if (e != hipSuccess) return e;
  XinvArgs xa{};
  xa.strips = reinterpret_cast<const cx<double>*>(ws + l.strips);
  xa.C = reinterpret_cast<double*>(ws + l.C);
  xa.twW = static_cast<const cx<double>*>(p.twW64);
  xa.W = g.W; xa.nkx = g.nkx; xa.h = g.h; xa.r = g.r; xa.NKK = g.NKK; xa.NP = g.NP;
  prof_begin(pf, SFFT_PROF_XINV, st);
  hipLaunchKernelGGL(k_strip_xinv, dim3(g.NP * (2 * g.h + 1)), dim3(256), 0, st, xa);
  prof_end(pf, SFFT_PROF_XINV, st);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  MomArgs ma{};
  ma.MR = reinterpret_cast<const double*>(ws + l.MR);
  ma.MS = reinterpret_cast<const double*>(ws + l.MS);
  ma.ER = reinterpret_cast<const double*>(ws + l.ER);
  ma.mom = reinterpret_cast<double*>(ws + l.mom);
  ma.W = g.W; ma.H = g.H; ma.DK = g.DK; ma.DB = g.DB; ma.r = g.r;
  ma.sx = g.W > 1 ? 2.0 / (double)(g.W - 1) : 0.0;
  ma.sy = g.H > 1 ? 2.0 / (double)(g.H - 1) : 0.0;
  hipLaunchKernelGGL(k_moments, dim3(l.nmom), dim3(256), 0, st, ma);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  KbArgs ka{};
  ka.mom = ma.mom; ka.MR = ma.MR; ka.ER = ma.ER; ka.G = G; ka.hv = hv;
  ka.W = g.W; ka.H = g.H; ka.L = g.L; ka.r = g.r; ka.DK = g.DK; ka.DB = g.DB;
  ka.nK = g.nK; ka.nB = g.nB; ka.N = g.N; ka.sx = ma.sx; ka.sy = ma.sy;
  const int nkb = g.nK * g.L * g.L * g.nB + g.nB * g.nB;
  hipLaunchKernelGGL(k_kb_assemble, dim3((nkb + 255) / 256), dim3(256), 0, st, ka);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  GatherArgs ga{};
  ga.C = xa.C; ga.G = G; ga.hv = hv; ga.L = g.L; ga.r = g.r; ga.h = g.h;
  ga.nK = g.nK; ga.NKK = g.NKK; ga.N = g.N;
  const int nKL = g.nK * g.L * g.L;
  hipLaunchKernelGGL(k_gather_kk, dim3((nKL + 255) / 256, nKL), dim3(256), 0, st, ga);
  prof_end(pf, SFFT_PROF_BUILD, st);
  return hipGetLastError();
}

}  // namespace sfft
