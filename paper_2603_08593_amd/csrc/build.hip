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
#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "common.hpp"
#include "layout.hpp"
#include "batch.hpp"

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
// Stockham FFT of length N = 2^a 3^b 5^c (<= 4096) in LDS, 256 threads,
// stages of radix 8, 4, 2, 3, 5 (host-chosen plan). buf uses the padded index
// pad8(i). Twiddles exp(-2 pi i m / N) come from two small tables,
// twl[m mod 64] * twh[m div 64] (one complex product), so the transform's LDS
// footprint stays close to its data.
// ---------------------------------------------------------------------------

template <typename T>
__device__ __forceinline__ cx<T> twiddle(const cx<T>* twl, const cx<T>* twh, int m) {
  return cmul(twl[m & 63], twh[m >> 6]);
}

struct FftPlan {
  int nstages;
  int radix[12];
};

// POW2: N and Ns are powers of two, so the butterfly's position within its
// group is a mask instead of a division
template <typename T, int R, bool INV, int NQ, bool POW2>
__device__ __forceinline__ void stockham_pass(cx<T>* buf, const cx<T>* twl, const cx<T>* twh, int N, int Ns) {
  constexpr int MAXB = (NQ * kRowThreads + R * kRowThreads - 1) / (R * kRowThreads);
  const int nb = N / R;
  const int tstride = N / (Ns * R);
  cx<T> v[MAXB][R];
#pragma unroll
  for (int t = 0; t < MAXB; ++t) {
    const int j = threadIdx.x + t * kRowThreads;
    if (j < nb) {
      const int k = POW2 ? (j & (Ns - 1)) : j % Ns;
#pragma unroll
      for (int r = 0; r < R; ++r) v[t][r] = buf[pad8(j + r * nb)];
      if (Ns > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          cx<T> w = twiddle(twl, twh, r * k * tstride);
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
      const int k = POW2 ? (j & (Ns - 1)) : j % Ns;
      const int base = (j - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[pad8(base + r * Ns)] = v[t][r];
    }
  }
  __syncthreads();
}

template <typename T, bool INV, int NQ, bool MIXED>
__device__ void fft_lds(cx<T>* buf, const cx<T>* twl, const cx<T>* twh, int N, const FftPlan& plan) {
  int Ns = 1;
  for (int s = 0; s < plan.nstages; ++s) {
    const int R = plan.radix[s];
    if (R == 8) stockham_pass<T, 8, INV, NQ, !MIXED>(buf, twl, twh, N, Ns);
    else if (R == 4) stockham_pass<T, 4, INV, NQ, !MIXED>(buf, twl, twh, N, Ns);
    else if (R == 2) stockham_pass<T, 2, INV, NQ, !MIXED>(buf, twl, twh, N, Ns);
    else if constexpr (MIXED) {
      if (R == 3) stockham_pass<T, 3, INV, NQ, false>(buf, twl, twh, N, Ns);
      else stockham_pass<T, 5, INV, NQ, false>(buf, twl, twh, N, Ns);
    }
    Ns *= R;
  }
}

// radix plan: as many 8s as possible, then 4 or 2, then 3s and 5s (order
// 0), or those stages reversed (order 1). A Stockham pass takes any radix at
// any position, so both orders give the DFT; they group its sums
// differently and touch LDS with different strides per stage.
inline FftPlan make_fft_plan(int n, int order = 0) {
  FftPlan p{};
  int twos = 0, threes = 0, fives = 0;
  while (n % 2 == 0) { n /= 2; ++twos; }
  while (n % 3 == 0) { n /= 3; ++threes; }
  while (n % 5 == 0) { n /= 5; ++fives; }
  while (twos >= 3) { p.radix[p.nstages++] = 8; twos -= 3; }
  if (twos == 2) p.radix[p.nstages++] = 4;
  if (twos == 1) p.radix[p.nstages++] = 2;
  for (int i = 0; i < threes; ++i) p.radix[p.nstages++] = 3;
  for (int i = 0; i < fives; ++i) p.radix[p.nstages++] = 5;
  if (order == 1)
    for (int i = 0, j = p.nstages - 1; i < j; ++i, --j) {
      const int t = p.radix[i];
      p.radix[i] = p.radix[j];
      p.radix[j] = t;
    }
  return p;
}

// ---------------------------------------------------------------------------
// Row pass
// ---------------------------------------------------------------------------

struct RowArgs {
  const void* R;
  const void* S;
  int64_t ld;
  int W, H, DK, DB, r;
  FftPlan plan;
  double cR, cS, sx;
  void* F;            // cx<T>[nsig][H][pitchK]
  int64_t pitchK, planeK;
  double* MR;         // [DK+DB+1][H]
  double* MS;         // [DB+1][H]
  double* ER;         // [H][2r]
  int* flags;
  const void* twW;    // cx<T>[W]
  double* edge;       // [nsig][2][H]: real k_x = 0 and k_x = W/2 values
  int sci;            // row pass: 1: transform S'; 0: its spectrum is already
                      // in the workspace (a second template against it)
  // masked fit: R' and S' are taken as zero where mask[y * mask_ld + x] == 0
  // (null: no mask); R' also on the `frame`-pixel border (output-pixel
  // convention: frame = r, else 0)
  const unsigned char* mask;
  int64_t mask_ld;
  int frame;
};

// mask and frame of a build: whether R' and S' at (x, y) enter the fit
__device__ __forceinline__ void pixel_mask(const RowArgs& a, int x, int y, bool& mr, bool& ms) {
  ms = true;
  if (a.mask) ms = a.mask[(int64_t)y * a.mask_ld + x] != 0;
  mr = ms && (a.frame == 0 || (x >= a.frame && x < a.W - a.frame && y >= a.frame && y < a.H - a.frame));
}

// NQ: row elements per thread, max(1, ceil(W / 256)); MIXED: W has factors 3 or 5
// MASK: the build applies a mask or the output-pixel frame (RowArgs::mask,
// ::frame); a separate instantiation, so that the plain path carries none of it
template <typename T, typename TIN, int NQ, bool MIXED, bool PF, bool MASK = false>
__device__ __forceinline__ void row_pass_body(const RowArgs& a, const VB vb) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int W = a.W;
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* twl = buf + (W + W / 8);
  cx<T>* twh = twl + 64;
  const cx<T>* twg = static_cast<const cx<T>*>(a.twW);
  for (int i = threadIdx.x; i < 64; i += kRowThreads) twl[i] = twg[i < W ? i : 0];
  for (int i = threadIdx.x; 64 * i < W; i += kRowThreads) twh[i] = twg[64 * i];
  constexpr int MAXQ = NQ;
  // signals transformed: xt^a R' (a <= DK), then S' unless it is reused
  const int nsig = a.DK + 1 + a.sci;
  cx<T>* F = static_cast<cx<T>*>(a.F);

  // Row moments, edge pixels and the input check are done by k_row_moments.
  // PF: the pixels of the workgroup's next row are loaded while the current
  // row is transformed; without it the memory latency is left to the other
  // workgroups on the CU (both launches use PF = true).
  const TIN* Rg = static_cast<const TIN*>(a.R);
  const TIN* Sg = static_cast<const TIN*>(a.S);
  TIN rn[MAXQ], sn[MAXQ];
  if constexpr (PF) {
#pragma unroll
    for (int q = 0; q < MAXQ; ++q) {
      const int x = threadIdx.x + q * kRowThreads;
      const bool in = x < W && vb.x < a.H;
      rn[q] = in ? Rg[(int64_t)vb.x * a.ld + x] : (TIN)0;
      sn[q] = (in && a.sci) ? Sg[(int64_t)vb.x * a.ld + x] : (TIN)0;
    }
  }

  for (int y = vb.x; y < a.H; y += vb.nx) {
    TIN rc[MAXQ], sc[MAXQ];
    // PF: the current row was loaded one step ahead; the next one is loaded
    // now. Otherwise the current row is loaded here.
    const int yl = PF ? y + vb.nx : y;
#pragma unroll
    for (int q = 0; q < MAXQ; ++q) {
      if constexpr (PF) {
        rc[q] = rn[q];
        sc[q] = sn[q];
      }
      const int x = threadIdx.x + q * kRowThreads;
      const bool in = x < W && yl < a.H;
      const TIN rv = in ? Rg[(int64_t)yl * a.ld + x] : (TIN)0;
      const TIN sv = (in && a.sci) ? Sg[(int64_t)yl * a.ld + x] : (TIN)0;
      if constexpr (PF) {
        rn[q] = rv;
        sn[q] = sv;
      } else {
        rc[q] = rv;
        sc[q] = sv;
      }
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
          double rv = (double)rc[q] - a.cR, sv = (double)sc[q] - a.cS;
          if (MASK) {
            bool mr, ms;
            pixel_mask(a, x, y, mr, ms);
            rv = mr ? rv : 0.0;
            sv = ms ? sv : 0.0;
          }
          const double v0 = (s0 <= a.DK) ? ipow(xt, s0) * rv : sv;
          double v1 = 0.0;
          if (s1 < nsig) v1 = (s1 <= a.DK) ? ipow(xt, s1) * rv : sv;
          buf[pad8(x)] = cx<T>{(T)v0, (T)v1};
        }
      }
      __syncthreads();
      fft_lds<T, false, NQ, MIXED>(buf, twl, twh, W, a.plan);
      const int half = W / 2;
      for (int kx = threadIdx.x; kx <= half; kx += kRowThreads) {
        const cx<T> z1 = buf[pad8(kx)];
        const cx<T> z2 = cconj(buf[pad8(kx == 0 ? 0 : W - kx)]);
        const cx<T> A = cscale(cadd(z1, z2), (T)0.5);
        const cx<T> d = csub(z1, z2);
        const cx<T> B = {d.im * (T)0.5, -d.re * (T)0.5};
        F[(int64_t)s0 * a.planeK + (int64_t)y * a.pitchK + kx] = A;
        if (s1 < nsig) F[(int64_t)s1 * a.planeK + (int64_t)y * a.pitchK + kx] = B;
        if (kx == 0 || kx == half) {
          const int e = (kx == 0) ? 0 : 1;
          a.edge[((int64_t)s0 * 2 + e) * a.H + y] = (double)A.re;
          if (s1 < nsig) a.edge[((int64_t)s1 * 2 + e) * a.H + y] = (double)B.re;
        }
      }
      __syncthreads();
    }
  }
}

template <typename T, typename TIN, int NQ, bool MIXED, bool MASK>
__global__ __launch_bounds__(kRowThreads, NQ >= 16 ? 2 : 3) void k_row_pass(RowArgs a) {
  row_pass_body<T, TIN, NQ, MIXED, true, MASK>(a, vb_grid());
}

template <typename T, typename TIN, int NQ, bool MIXED>
__global__ __launch_bounds__(kRowThreads, 2) void k_row_pass_batch(const RowArgs* args, const BatchTab* tab,
                                                                  int n) {
  int item;
  VB vb;
  if (batch_locate(tab, n, item, vb)) row_pass_body<T, TIN, NQ, MIXED, true>(args[item], vb);
}

// ---------------------------------------------------------------------------
// Column pass: blocked correlation along y for 4 adjacent k_x columns,
// k_x in [1, W/2). The real k_x = 0 and k_x = W/2 columns are correlated
// directly in k_strip_xinv.
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
template <int NK> struct BaseCount { static constexpr int value = (NK == 1 ? 0 : (NK == 3 ? 1 : 2)) + 2; };

// layout of the kernel-term spectra: exponents (a, b) of term g
__device__ __forceinline__ void mono_ab(int g, int& a, int& b) {
  // order: d = 0..: b = 0..d, a = d - b
  int d = 0, start = 0;
  while (g >= start + d + 1) { start += d + 1; ++d; }
  b = g - start;
  a = d - b;
}

template <int NK>
constexpr int col_spec_stride() {
  // column stride (complex elements) congruent to 4 mod 16: stage-1 writes
  // of 4 columns x 4 butterflies hit distinct LDS banks
  return (2 * NK + 1) * 136 + ((4 - (((2 * NK + 1) * 136) % 16)) + 16) % 16;
}

// FP64 spectra: the staged rows go from global memory straight into LDS
// (16-byte elements, one per lane; each wave's 64 elements of one base are
// contiguous), with no registers in between, issued as soon as the previous
// block's rows have been read, so the loads overlap the rest of the block.
// The compiler keeps such a load in flight across other LDS accesses only
// when it can tell them apart, so this form keeps every LDS array static.
// (FP32 elements are 8 bytes, a size the direct loads do not have: the FP32
// form stages through registers.)
template <typename T>
constexpr bool col_direct() { return sizeof(T) == 8; }

template <typename T, int NK>
constexpr size_t col_pass_shmem() {
  // dynamic LDS of the register-staged form: spectra, twiddles, staged
  // rows, then the row weight table: [window (U, V)][power 0..DK][row] of T
  if constexpr (col_direct<T>()) return 0;
  return sizeof(cx<T>) * ((size_t)kColsPerWG * col_spec_stride<NK>() + kTP +
                          (size_t)BaseCount<NK>::value * kTP * kColsPerWG) +
         sizeof(T) * 2 * (BaseCount<NK>::value - 1) * kTP;
}

// LDS arrays of the column pass: static for the direct-staged form, carved
// from the dynamic allocation otherwise
template <typename T, int NK>
__device__ __forceinline__ void col_lds(cx<T>*& spec, cx<T>*& tw, cx<T>*& raw, T*& wtab) {
  constexpr int NBASE = BaseCount<NK>::value;
  constexpr int CS = col_spec_stride<NK>();
  if constexpr (col_direct<T>()) {
    __shared__ __align__(16) cx<T> s_spec[kColsPerWG * CS];
    __shared__ __align__(16) cx<T> s_tw[kTP];
    __shared__ __align__(16) cx<T> s_raw[NBASE * kTP * kColsPerWG];
    __shared__ __align__(16) T s_wtab[2 * (NBASE - 1) * kTP];
    spec = s_spec; tw = s_tw; raw = s_raw; wtab = s_wtab;
  } else {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    spec = reinterpret_cast<cx<T>*>(smem_raw);
    tw = spec + kColsPerWG * CS;
    raw = tw + kTP;
    wtab = reinterpret_cast<T*>(raw + NBASE * kTP * kColsPerWG);
  }
}

__device__ __forceinline__ void wait_vm_all() { __builtin_amdgcn_s_waitcnt(0x0F70); }   // vmcnt(0)

// Workgroup barrier for the LDS data that ds instructions wrote: the wave
// waits for its own LDS accesses (lgkmcnt(0)), not for its direct global ->
// LDS loads, which stay in flight across it (a memory fence would wait for
// them, as they write LDS; their data is waited for explicitly before a full
// barrier). The signal fences keep the compiler from moving memory accesses
// across the barrier.
__device__ __forceinline__ void col_lds_barrier() {
  __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0); vmcnt and expcnt not waited
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

template <typename T, int NK>
__device__ __forceinline__ void col_pass_body(const ColArgs& a, const VB vb) {
  constexpr int NS = 2 * NK + 1;
  constexpr int NKK = PairCount<NK>::NKK;
  constexpr int NP = PairCount<NK>::NP;
  constexpr int NBASE = BaseCount<NK>::value;
  constexpr int SPAD = 136;
  constexpr int CS = col_spec_stride<NK>();
  constexpr bool DIRECT = col_direct<T>();
  cx<T>* spec;
  cx<T>* tw;
  cx<T>* raw;                                // staged rows: [base][m][column]
  T* wtab;
  col_lds<T, NK>(spec, tw, raw, wtab);
  constexpr int NPOW = NBASE - 1;            // powers yt^0 .. yt^DK
  const cx<T>* twg = static_cast<const cx<T>*>(a.tw128);
  const int tid = threadIdx.x;
  if (tid < kTP) tw[tid] = twg[tid];

  // XCD-aware group index: workgroups that share an XCD (id mod 8) take
  // adjacent column groups, so their 64-byte row segments share L2 lines.
  const int per_xcd = (a.ngroups + 7) / 8;
  const int grp = (vb.x & 7) * per_xcd + (vb.x >> 3);
  if (grp >= a.ngroups) return;
  const int kx0 = 1 + grp * kColsPerWG;
  const int kxend = a.nkx - 1;               // exclusive: W/2 is done elsewhere
  const cx<T>* F = static_cast<const cx<T>*>(a.F);
  const int H = a.H, h = a.h;

  // stage-2 twiddles of this thread's butterfly column j = tid & 15: held in
  // registers unless the accumulators already fill the register file
  constexpr bool kRegTw = !(sizeof(T) == 8 && NK >= 6);
  cx<T> tw2[kRegTw ? 8 : 1];
  if constexpr (kRegTw) {
    const int j2 = tid & 15;
#pragma unroll
    for (int r = 0; r < 8; ++r) tw2[r] = twg[r * j2];
  }
  auto twid = [&](int r, int j) -> cx<T> {
    if constexpr (kRegTw) return tw2[r];
    else return tw[r * j];
  };

  // staged rows: element (base u, window row m = tid >> 2, column c = tid & 3)
  // at raw[(u * kTP + m) * kColsPerWG + c] = raw[u * kTP * kColsPerWG + tid]
  const int fm = tid >> 2, fc = tid & 3;
  cx<T> pre[DIRECT ? 1 : NBASE];
  auto fetch = [&](int yb) {
    const int o = (fm < kTP - h) ? fm : fm - kTP;
    int y = yb + o;
    y = (y < 0) ? y + H : ((y >= H) ? y - H : y);
    const int kx = kx0 + fc;
    if constexpr (DIRECT) {
      // lane l of the wave writes LDS at the wave's base + 16 l; lanes past
      // the last column load nothing and keep their zeros
      if (kx < kxend) {
        const cx<T>* src = F + (int64_t)y * a.pitchK + kx;
        cx<T>* dst = raw + (tid & ~63);
#pragma unroll
        for (int u = 0; u < NBASE; ++u)
          __builtin_amdgcn_global_load_lds(static_cast<const void*>(src + (int64_t)u * a.planeK),
                                           (__attribute__((address_space(3))) void*)(dst + u * kTP * kColsPerWG),
                                           16, 0, 0);
      }
    } else {
#pragma unroll
      for (int u = 0; u < NBASE; ++u)
        pre[u] = (kx < kxend) ? F[(int64_t)u * a.planeK + (int64_t)y * a.pitchK + kx] : cx<T>{(T)0, (T)0};
    }
  };
  auto commit = [&]() {
    if constexpr (!DIRECT) {
#pragma unroll
      for (int u = 0; u < NBASE; ++u) raw[(u * kTP + fm) * kColsPerWG + fc] = pre[u];
    }
  };
  if constexpr (DIRECT) {
    if (kx0 + fc >= kxend) {
#pragma unroll
      for (int u = 0; u < NBASE; ++u) raw[u * kTP * kColsPerWG + tid] = cx<T>{(T)0, (T)0};
    }
  }

  // weight of window row m for the block starting at yb: yt(y)^b inside the
  // window (kernel side: the T rows of the block; science side: the block
  // plus its h-row halo), 0 outside
  auto fill_weights = [&](int yb) {
    const int Tb = min(a.T, H - yb);
    for (int m = tid; m < kTP; m += kColThreads) {
      const int o = (m < kTP - h) ? m : m - kTP;
      int y = yb + o;
      y = (y < 0) ? y + H : ((y >= H) ? y - H : y);
      const double yt = (double)y * a.sy - 1.0;
      const bool inu = (o >= 0 && o < Tb), inv = (o >= -h && o < Tb + h);
      double pw = 1.0;
#pragma unroll
      for (int b = 0; b < NPOW; ++b) {
        wtab[b * kTP + m] = inu ? (T)pw : (T)0;
        wtab[(NPOW + b) * kTP + m] = inv ? (T)pw : (T)0;
        pw *= yt;
      }
    }
  };

  cx<T> acc[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) acc[p] = cx<T>{(T)0, (T)0};
  fetch(0);
  commit();
  fill_weights(0);
  if constexpr (DIRECT) wait_vm_all();
  __syncthreads();

  for (int yb = 0; yb < H; yb += a.T) {
    // ---- stage 1: weighted rows j + 8q from the staging buffer, radix-16
    if (tid < kColsPerWG * NS * 8) {
      const int c = tid & 3;
      const int rest = tid >> 2;
      const int j = rest & 7;
      const int s = rest >> 3;            // 0..NS-1
      int base, bpow;
      bool is_u;
      if (s < NK) { int ea, eb; mono_ab(s, ea, eb); base = ea; bpow = eb; is_u = true; }
      else if (s < 2 * NK) { int ea, eb; mono_ab(s - NK, ea, eb); base = ea; bpow = eb; is_u = false; }
      else { base = NBASE - 1; bpow = 0; is_u = false; }
      const cx<T>* src = raw + (base * kTP) * kColsPerWG + c;
      const T* wrow = wtab + (is_u ? bpow : NPOW + bpow) * kTP;
      cx<T> v[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int m = j + 8 * q;
        v[q] = cscale(src[m * kColsPerWG], wrow[m]);
      }
      dft16<T, false>(v);
      cx<T>* dst = spec + c * CS + s * SPAD;
#pragma unroll
      for (int r = 0; r < 16; ++r) dst[pad16(16 * j + r)] = v[r];
    }
    const bool more = yb + a.T < H;
    if constexpr (!DIRECT) {
      if (more) fetch(yb + a.T);           // in flight during stage 2
    }
    __syncthreads();
    if constexpr (DIRECT) {
      if (more) fetch(yb + a.T);           // raw is read: in flight during stage 2 and the products
    }
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
          if (r > 0) x = cmul(x, twid(r, j));
          v[r] = x;
        }
        dft8<T, false>(v);
#pragma unroll
        for (int r = 0; r < 8; ++r) p[pad16(j + 16 * r)] = v[r];
      }
      if constexpr (DIRECT) col_lds_barrier();   // the next rows stay in flight
      else __syncthreads();
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
    if (more) {
      commit();
      fill_weights(yb + a.T);
    }
    if constexpr (DIRECT) wait_vm_all();
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
          if (r > 0) x = cmul(x, cconj(twid(r, j)));
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
        if (kx < kxend) {
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

template <typename T, int NK>
__global__ __launch_bounds__(kColThreads) void k_col_pass(ColArgs a) {
  col_pass_body<T, NK>(a, vb_grid());
}

template <typename T, int NK>
__global__ __launch_bounds__(kColThreads) void k_col_pass_batch(const ColArgs* args, const BatchTab* tab, int n) {
  int item;
  VB vb;
  if (batch_locate(tab, n, item, vb)) col_pass_body<T, NK>(args[item], vb);
}

// ---------------------------------------------------------------------------
// Pruned inverse along x:
//   C_p(dx, dy) = (1/W) [ c_p(0, dy) + (-1)^dx c_p(W/2, dy)
//                         + 2 sum_{kx=1}^{W/2-1} Re(e^{2 pi i kx dx / W} c_p(kx, dy)) ]
// The k_x = 0 and k_x = W/2 columns are real sequences along y; their
// correlations c_p(0, dy), c_p(W/2, dy) are formed here by direct sums.
// ---------------------------------------------------------------------------

struct XinvArgs {
  const cx<double>* strips;
  double* C;              // [NP][2h+1][2h+1]
  const cx<double>* twW;  // exp(-2 pi i m / W), FP64
  const double* edge;     // [nsig][2][H]: real k_x = 0 and k_x = W/2 row-spectrum values
  int W, H, nkx, h, r, NKK, NP, nK, DK;
  double sy;
};

__device__ __forceinline__ void strip_xinv_body(const XinvArgs& a, const VB vb) {
  __shared__ double red[4][34];
  const int ndy = 2 * a.h + 1;
  const int p = vb.x / ndy, dyi = vb.x % ndy;
  const bool ks = p >= a.NKK;
  const int lim = ks ? a.r : a.h;
  if (abs(dyi - a.h) > lim) return;
  const int ndx = 2 * lim + 1;
  const int dy = dyi - a.h;
  // terms of the pair: u-side term iu, v-side term jv (or S)
  int iu, jv;
  if (!ks) {
    int rem = p;
    iu = 0;
    while (rem >= a.nK - iu) { rem -= a.nK - iu; ++iu; }
    jv = iu + rem;
  } else {
    iu = p - a.NKK;
    jv = -1;
  }
  int au, bu, av, bv;
  mono_ab(iu, au, bu);
  if (jv >= 0) mono_ab(jv, av, bv);
  else { av = a.DK + 1; bv = 0; }
  // direct real correlations of the k_x = 0 and k_x = W/2 columns
  double sdc = 0.0, snq = 0.0;
  const double* eu = a.edge + (int64_t)au * 2 * a.H;
  const double* ev = a.edge + (int64_t)av * 2 * a.H;
  // 4 rows per thread per round, their loads issued together
  constexpr int kU = 4;
  for (int yb = threadIdx.x; yb < a.H; yb += kU * blockDim.x) {
    double u0[kU], u1[kU], v0[kU], v1[kU];
    int ys[kU], y2s[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int y = yb + u * blockDim.x;
      const bool in = y < a.H;
      int y2 = y + dy;
      y2 = (y2 < 0) ? y2 + a.H : (y2 >= a.H ? y2 - a.H : y2);
      ys[u] = y;
      y2s[u] = y2;
      u0[u] = in ? eu[y] : 0.0;
      u1[u] = in ? eu[a.H + y] : 0.0;
      v0[u] = in ? ev[y2] : 0.0;
      v1[u] = in ? ev[a.H + y2] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const double wu = ipow((double)ys[u] * a.sy - 1.0, bu);
      const double wv = ipow((double)y2s[u] * a.sy - 1.0, bv);
      sdc = fma(wu * u0[u], wv * v0[u], sdc);
      snq = fma(wu * u1[u], wv * v1[u], snq);
    }
  }
  double acc[32];
#pragma unroll
  for (int t = 0; t < 32; ++t) acc[t] = 0.0;
  const cx<double>* row = a.strips + ((int64_t)p * ndy + dyi) * a.nkx;
  for (int kx = 1 + threadIdx.x; kx < a.nkx - 1; kx += blockDim.x) {
    const cx<double> c = row[kx];
    // e(dx) = exp(+2 pi i kx dx / W): start at dx = -lim, step by exp(+2 pi i kx / W)
    const cx<double> w0 = a.twW[(int)(((int64_t)kx * lim) % a.W)];   // exp(-2 pi i kx lim / W)
    const cx<double> w1 = a.twW[kx];
    const cx<double> step = {w1.re, -w1.im};
    cx<double> e = w0;
#pragma unroll
    for (int t = 0; t < 32; ++t) {
      if (t < ndx) {
        acc[t] = fma(2.0, e.re * c.re - e.im * c.im, acc[t]);
        e = cmul(e, step);
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
  {
    double v = wave_sum(sdc);
    if (lane == 0) red[wid][32] = v;
    v = wave_sum(snq);
    if (lane == 0) red[wid][33] = v;
  }
  __syncthreads();
  if (threadIdx.x < ndx) {
    const int t = threadIdx.x;
    const int dx = t - lim;
    const double s = red[0][t] + red[1][t] + red[2][t] + red[3][t];
    const double dc = red[0][32] + red[1][32] + red[2][32] + red[3][32];
    const double nq = red[0][33] + red[1][33] + red[2][33] + red[3][33];
    const double tot = s + dc + ((dx & 1) ? -nq : nq);
    a.C[((int64_t)p * ndy + dyi) * ndy + (dx + a.h)] = tot / (double)a.W;
  }
}

__global__ __launch_bounds__(256) void k_strip_xinv(XinvArgs a) { strip_xinv_body(a, vb_grid()); }

__global__ __launch_bounds__(256) void k_strip_xinv_batch(const XinvArgs* args, const BatchTab* tab, int n) {
  int item;
  VB vb;
  if (batch_locate(tab, n, item, vb)) strip_xinv_body(args[item], vb);
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
__device__ __forceinline__ void moments_body(const MomArgs& a, const VB vb) {
  __shared__ double scratch[8];
  const int nm = a.DK + a.DB + 1;
  const int nM2 = nm * nm, nE = 2 * a.r * nm, nMS = (a.DB + 1) * (a.DB + 1);
  const int np = 2 * a.DB + 1;
  int id = vb.x;
  double s = 0.0;
  // sum over y of yt^n src[y * stride]: 8 rows per thread per round, their
  // loads issued together (rows ascending per thread)
  auto ysum = [&](const double* src, int64_t stride, int n) {
    for (int yb = threadIdx.x; yb < a.H; yb += 8 * blockDim.x) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int y = yb + u * blockDim.x;
        v[u] = y < a.H ? src[(int64_t)y * stride] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int y = yb + u * blockDim.x;
        if (y < a.H) s += ipow((double)y * a.sy - 1.0, n) * v[u];
      }
    }
  };
  if (id < nM2) {
    const int m = id / nm, n = id % nm;
    ysum(a.MR + (int64_t)m * a.H, 1, n);
  } else if ((id -= nM2) < nE) {
    const int e = id / nm, n = id % nm;
    ysum(a.ER + e, 2 * a.r, n);
  } else if ((id -= nE) < nMS) {
    const int ac = id / (a.DB + 1), bc = id % (a.DB + 1);
    ysum(a.MS + (int64_t)ac * a.H, 1, bc);
  } else if ((id -= nMS) < np) {
    for (int x = threadIdx.x; x < a.W; x += blockDim.x) s += ipow((double)x * a.sx - 1.0, id);
  } else {
    id -= np;
    for (int y = threadIdx.x; y < a.H; y += blockDim.x) s += ipow((double)y * a.sy - 1.0, id);
  }
  s = block_sum(s, scratch);
  if (threadIdx.x == 0) a.mom[vb.x] = s;
}

__global__ __launch_bounds__(256) void k_moments(MomArgs a) { moments_body(a, vb_grid()); }

__global__ __launch_bounds__(256) void k_moments_batch(const MomArgs* args, const BatchTab* tab, int n) {
  int item;
  VB vb;
  if (batch_locate(tab, n, item, vb)) moments_body(args[item], vb);
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

// binomial coefficient (exact in integers for the small degrees used here)
__device__ __forceinline__ double binom(int n, int k) {
  int b = 1;
  for (int t = 1; t <= k; ++t) b = b * (n - k + t) / t;
  return (double)b;
}

__device__ __forceinline__ void kb_assemble_body(const KbArgs& a, const VB vb) {
  const int L2 = a.L * a.L;
  const int nKL = a.nK * L2;
  const int nm = a.DK + a.DB + 1;
  // the moment block and the seam rows (y < r, y >= H - r) of the per-row
  // moments and edge pixels, staged in LDS: every entry reads them many times
  constexpr int kMaxNm = 7, kMaxR2 = 14;
  __shared__ double smom[kMaxNm * kMaxNm + kMaxR2 * kMaxNm + 25 + 18];
  __shared__ double sMR[kMaxNm * kMaxR2];
  __shared__ double sER[kMaxR2 * kMaxR2];
  {
    const int r2 = 2 * a.r;
    const int nmomv = nm * nm + r2 * nm + (a.DB + 1) * (a.DB + 1) + 2 * (2 * a.DB + 1);
    for (int i = threadIdx.x; i < nmomv; i += blockDim.x) smom[i] = a.mom[i];
    for (int i = threadIdx.x; i < nm * r2; i += blockDim.x) {
      const int m = i / r2, sj = i % r2;
      const int uy = sj < a.r ? sj : a.H - a.r + (sj - a.r);
      sMR[i] = a.MR[(int64_t)m * a.H + uy];
    }
    for (int i = threadIdx.x; i < r2 * r2; i += blockDim.x) {
      const int sj = i / r2, e = i % r2;
      const int uy = sj < a.r ? sj : a.H - a.r + (sj - a.r);
      sER[i] = a.ER[(int64_t)uy * r2 + e];
    }
    __syncthreads();
  }
  auto yseam = [&](int uy) { return uy < a.r ? uy : a.r + (uy - (a.H - a.r)); };
  const double* M2 = smom;
  const double* E = M2 + nm * nm;
  const double* MSy = E + 2 * a.r * nm;
  const double* Px = MSy + (a.DB + 1) * (a.DB + 1);
  const double* Py = Px + 2 * a.DB + 1;
  // one wave per kernel-background entry: the entry is a sum of products
  // (the moment terms and the x- and y-seam corrections); lane t takes terms
  // t, t + 64, ... of the flattened list, then a fixed-order wave sum. The
  // last wave forms the background block and the background RHS.
  const int lane = threadIdx.x & 63;
  const int entry = vb.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  const int nkb = nKL * a.nB;
  if (entry < nkb) {
    const int c = entry % a.nB;
    const int row = entry / a.nB;
    const int i = row / L2, d = row % L2;
    const int dy = d / a.L - a.r, dx = d % a.L - a.r;
    int ai, bi, ac, bc;
    mono_ab(i, ai, bi);
    mono_ab(c, ac, bc);
    const int W = a.W, H = a.H, r = a.r;
    // x-seam columns [xs0, xs1) of this dx and y-seam rows [ys0, ys1) of dy
    int xs0 = 0, xs1 = 0;
    if (dx > 0) { xs0 = W - dx; xs1 = W; }
    else if (dx < 0) { xs0 = 0; xs1 = -dx; }
    int ys0 = 0, ys1 = 0;
    if (dy > 0) { ys0 = H - dy; ys1 = H; }
    else if (dy < 0) { ys0 = 0; ys1 = -dy; }
    const int nxs = xs1 - xs0, nys = ys1 - ys0;
    auto eslot = [&](int ux) { return ux < r ? ux : r + (ux - (W - r)); };
    auto dX = [&](int ux) {
      int w = ux + dx;
      w = (w < 0) ? w + W : (w >= W ? w - W : w);
      return ipow((double)w * a.sx - 1.0, ac) - ipow(-1.0 + a.sx * (double)(ux + dx), ac);
    };
    auto yw = [&](int uy) {
      int w = uy + dy;
      w = (w < 0) ? w + H : (w >= H ? w - H : w);
      const double dY = ipow((double)w * a.sy - 1.0, bc) - ipow(-1.0 + a.sy * (double)(uy + dy), bc);
      return ipow((double)uy * a.sy - 1.0, bi) * dY;
    };
    // terms: (l, k) moments; (l, ux) x-seam; (uy, k) y-seam; (uy, ux) corner
    const int nA = (bc + 1) * (ac + 1), nBx = (bc + 1) * nxs, nC = nys * (ac + 1), nD = nys * nxs;
    double part = 0.0;
    for (int t = lane; t < nA + nBx + nC + nD; t += 64) {
      if (t < nA) {
        const int l = t / (ac + 1), k = t % (ac + 1);
        part += binom(bc, l) * ipow(a.sy * dy, bc - l) * binom(ac, k) * ipow(a.sx * dx, ac - k) *
                M2[(ai + k) * nm + bi + l];
      } else if (t < nA + nBx) {
        const int u = t - nA, l = u / nxs, ux = xs0 + u % nxs;
        part += binom(bc, l) * ipow(a.sy * dy, bc - l) * ipow((double)ux * a.sx - 1.0, ai) * dX(ux) *
                E[eslot(ux) * nm + bi + l];
      } else if (t < nA + nBx + nC) {
        const int u = t - nA - nBx, uy = ys0 + u / (ac + 1), k = u % (ac + 1);
        part += yw(uy) * binom(ac, k) * ipow(a.sx * dx, ac - k) * sMR[(ai + k) * 2 * r + yseam(uy)];
      } else {
        const int u = t - nA - nBx - nC, uy = ys0 + u / nxs, ux = xs0 + u % nxs;
        part += yw(uy) * ipow((double)ux * a.sx - 1.0, ai) * dX(ux) * sER[yseam(uy) * 2 * r + eslot(ux)];
      }
    }
    const double tot = wave_sum(part);
    if (lane == 0) {
      a.G[(int64_t)row * a.N + nKL + c] = tot;
      a.G[(int64_t)(nKL + c) * a.N + row] = tot;
    }
  } else if (entry == nkb) {
    for (int t = lane; t < a.nB * a.nB; t += 64) {
      const int c = t / a.nB, c2 = t % a.nB;
      int ac, bc, ac2, bc2;
      mono_ab(c, ac, bc);
      mono_ab(c2, ac2, bc2);
      a.G[(int64_t)(nKL + c) * a.N + nKL + c2] = Px[ac + ac2] * Py[bc + bc2];
      if (c2 == 0) a.hv[nKL + c] = MSy[ac * (a.DB + 1) + bc];
    }
  }
}

__global__ __launch_bounds__(256) void k_kb_assemble(KbArgs a) { kb_assemble_body(a, vb_grid()); }

__global__ __launch_bounds__(256) void k_kb_assemble_batch(const KbArgs* args, const BatchTab* tab, int n) {
  int item;
  VB vb;
  if (batch_locate(tab, n, item, vb)) kb_assemble_body(args[item], vb);
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

__device__ __forceinline__ void gather_kk_body(const GatherArgs& a, const VB vb) {
  const int L2 = a.L * a.L;
  const int nKL = a.nK * L2;
  const int row = vb.y;
  const int col = vb.x * blockDim.x + threadIdx.x;
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

__global__ __launch_bounds__(256) void k_gather_kk(GatherArgs a) { gather_kk_body(a, vb_grid()); }

__global__ __launch_bounds__(256) void k_gather_kk_batch(const GatherArgs* args, const BatchTab* tab, int n) {
  int item;
  VB vb;
  if (batch_locate(tab, n, item, vb)) gather_kk_body(args[item], vb);
}

// ---------------------------------------------------------------------------
// Background refit for a given kernel (learned form): the least-squares
// background given fixed kernel coefficients a is b = G_bb^-1 (h_b - G_kb^T a),
// with G_kb, G_bb and h_b exactly the blocks the build assembles from
// polynomial moments; only the row moments are needed, not the spectra.
// ---------------------------------------------------------------------------

// Row moments MR[m][y] = sum_x xt^m R'(x, y) (m <= DK + DB) and
// MS[m][y] = sum_x xt^m S'(x, y) (m <= DB), the r edge pixels of R' of every
// row, and the non-finite input flag. A wave takes 2 rows; the 32 lanes of a
// row read 4 consecutive pixels each per 128-pixel span (one 16-byte load
// when the rows are 16-byte aligned), four spans in flight at a time, keep
// partial sums in registers and add them over the 32 lanes at the end.
constexpr int kMomRowsPerWave = 2;
constexpr int kMomRowsPerWG = kMomRowsPerWave * (kRowThreads / 64);

template <typename TIN, bool MASK = false>
__device__ __forceinline__ void row_moments_body(const RowArgs& a, const VB vb) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int rr = lane >> 5, cc = lane & 31;
  const int y = vb.x * kMomRowsPerWG + wave * kMomRowsPerWave + rr;
  const int W = a.W;
  const int nm = a.DK + a.DB + 1;
  // every power up to the largest supported degree (DK <= 2, DB <= 4) is
  // accumulated without predicates; only the first nm / DB + 1 are stored
  constexpr int kMR = 7, kMS = 5;
  double mr[kMR], ms[kMS];
#pragma unroll
  for (int m = 0; m < kMR; ++m) mr[m] = 0.0;
#pragma unroll
  for (int m = 0; m < kMS; ++m) ms[m] = 0.0;
  bool bad = false;
  auto accumulate = [&](int x, double rv, double sv) {
    if (MASK) {
      // pixels outside the mask are not part of the fit (nor of the check)
      bool mr, ms;
      pixel_mask(a, x, y, mr, ms);
      rv = mr ? rv : 0.0;
      sv = ms ? sv : 0.0;
    }
    bad |= !(is_finite_d(rv) && is_finite_d(sv));
    const double xt = (double)x * a.sx - 1.0;
    double pw = 1.0;
#pragma unroll
    for (int m = 0; m < kMR; ++m) {
      mr[m] = fma(pw, rv, mr[m]);
      if (m < kMS) ms[m] = fma(pw, sv, ms[m]);
      pw *= xt;
    }
  };
  // edge pixels x < r and x >= W - r of the row, for the seam corrections
  if (y < a.H) {
    const TIN* Rr = static_cast<const TIN*>(a.R) + (int64_t)y * a.ld;
    for (int e = cc; e < 2 * a.r; e += 32) {
      const int x = e < a.r ? e : W - 2 * a.r + e;
      double ev = (double)Rr[x] - a.cR;
      if (MASK) {
        bool mr, ms;
        pixel_mask(a, x, y, mr, ms);
        ev = mr ? ev : 0.0;
      }
      a.ER[(int64_t)y * 2 * a.r + e] = ev;
    }
  }
  if (y < a.H) {
    const TIN* Rr = static_cast<const TIN*>(a.R) + (int64_t)y * a.ld;
    const TIN* Sr = static_cast<const TIN*>(a.S) + (int64_t)y * a.ld;
    const bool vec = sizeof(TIN) == 4 && ((reinterpret_cast<uintptr_t>(Rr) | reinterpret_cast<uintptr_t>(Sr)) & 15) == 0;
    // 4 spans of 128 pixels per round; the next round's loads are issued
    // before this round's pixels are accumulated
    TIN rv[4][4], sv[4][4], rn[4][4], sn[4][4];
    auto load = [&](int x00, TIN (&rr)[4][4], TIN (&ss)[4][4]) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int x0 = x00 + u * 128 + cc * 4;
        if (vec && x0 + 3 < W) {
          const float4 r4 = *reinterpret_cast<const float4*>(Rr + x0);
          const float4 s4 = *reinterpret_cast<const float4*>(Sr + x0);
          rr[u][0] = r4.x; rr[u][1] = r4.y; rr[u][2] = r4.z; rr[u][3] = r4.w;
          ss[u][0] = s4.x; ss[u][1] = s4.y; ss[u][2] = s4.z; ss[u][3] = s4.w;
        } else {
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            rr[u][k] = (x0 + k < W) ? Rr[x0 + k] : (TIN)0;
            ss[u][k] = (x0 + k < W) ? Sr[x0 + k] : (TIN)0;
          }
        }
      }
    };
    load(0, rn, sn);
    for (int x00 = 0; x00 < W; x00 += 4 * 128) {
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          rv[u][k] = rn[u][k];
          sv[u][k] = sn[u][k];
        }
      if (x00 + 4 * 128 < W) load(x00 + 4 * 128, rn, sn);
      if (x00 + 4 * 128 <= W) {
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int k = 0; k < 4; ++k)
            accumulate(x00 + u * 128 + cc * 4 + k, (double)rv[u][k] - a.cR, (double)sv[u][k] - a.cS);
      } else {
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const int x = x00 + u * 128 + cc * 4 + k;
            if (x < W) accumulate(x, (double)rv[u][k] - a.cR, (double)sv[u][k] - a.cS);
          }
      }
    }
  }
  if (bad) atomicOr(a.flags, 1);
  // sum over the 32 lanes of each row (fixed order: butterfly 16, 8, 4, 2, 1)
#pragma unroll
  for (int m = 0; m < kMR; ++m) {
    if (m < nm) {
      double v = mr[m];
#pragma unroll
      for (int o = 16; o > 0; o >>= 1) v += __shfl_xor(v, o, 32);
      if (cc == 0 && y < a.H) a.MR[(int64_t)m * a.H + y] = v;
    }
  }
#pragma unroll
  for (int m = 0; m < kMS; ++m) {
    if (m <= a.DB) {
      double v = ms[m];
#pragma unroll
      for (int o = 16; o > 0; o >>= 1) v += __shfl_xor(v, o, 32);
      if (cc == 0 && y < a.H) a.MS[(int64_t)m * a.H + y] = v;
    }
  }
}

template <typename TIN, bool MASK>
__global__ __launch_bounds__(kRowThreads) void k_row_moments(RowArgs a) {
  row_moments_body<TIN, MASK>(a, vb_grid());
}

__global__ __launch_bounds__(kRowThreads) void k_row_moments_batch(const RowArgs* args, const BatchTab* tab,
                                                                  int n) {
  int item;
  VB vb;
  if (batch_locate(tab, n, item, vb)) row_moments_body<float>(args[item], vb);
}

inline int row_moments_grid(int H) { return (H + kMomRowsPerWG - 1) / kMomRowsPerWG; }

// b = G_bb^-1 (h_b - G_kb^T a): one workgroup; FP64 dot products in a fixed
// order, Cholesky of the (at most 15 x 15) background block by one thread
__global__ __launch_bounds__(256) void k_bg_refit(const double* G, const double* hv, double* coef, int N,
                                                  int nKL, int nB) {
  __shared__ double red[4];
  __shared__ double rhs[15];
  __shared__ double M[15][15];
  for (int c = 0; c < nB; ++c) {
    double s = 0.0;
    for (int row = threadIdx.x; row < nKL; row += 256) s += G[(int64_t)row * N + nKL + c] * coef[row];
    s = block_sum(s, red);
    if (threadIdx.x == 0) rhs[c] = hv[nKL + c] - s;
  }
  for (int t = threadIdx.x; t < nB * nB; t += 256)
    M[t / nB][t % nB] = G[(int64_t)(nKL + t / nB) * N + nKL + t % nB];
  __syncthreads();
  if (threadIdx.x == 0) {
    // Cholesky M = L L^T in place (lower), then two substitutions
    bool ok = true;
    for (int j = 0; j < nB && ok; ++j) {
      double d = M[j][j];
      for (int k = 0; k < j; ++k) d -= M[j][k] * M[j][k];
      if (!(d > 0.0)) { ok = false; break; }
      M[j][j] = sqrt(d);
      for (int i = j + 1; i < nB; ++i) {
        double v = M[i][j];
        for (int k = 0; k < j; ++k) v -= M[i][k] * M[j][k];
        M[i][j] = v / M[j][j];
      }
    }
    double y[15];
    for (int i = 0; i < nB; ++i) {
      double v = rhs[i];
      for (int k = 0; k < i; ++k) v -= M[i][k] * y[k];
      y[i] = ok ? v / M[i][i] : 0.0;
    }
    for (int i = nB - 1; i >= 0; --i) {
      double v = y[i];
      for (int k = i + 1; k < nB; ++k) v -= M[k][i] * y[k];
      coef[nKL + i] = ok ? v / M[i][i] : __builtin_nan("");
      y[i] = ok ? v / M[i][i] : 0.0;
    }
  }
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------

template <typename T, typename TIN, bool MASK, class Set>
static void set_row_attrs(Set& set) {
  set(reinterpret_cast<const void*>(&k_row_pass<T, TIN, 1, false, MASK>));
  set(reinterpret_cast<const void*>(&k_row_pass<T, TIN, 1, true, MASK>));
  set(reinterpret_cast<const void*>(&k_row_pass<T, TIN, 2, false, MASK>));
  set(reinterpret_cast<const void*>(&k_row_pass<T, TIN, 2, true, MASK>));
  set(reinterpret_cast<const void*>(&k_row_pass<T, TIN, 4, false, MASK>));
  set(reinterpret_cast<const void*>(&k_row_pass<T, TIN, 4, true, MASK>));
  set(reinterpret_cast<const void*>(&k_row_pass<T, TIN, 8, false, MASK>));
  set(reinterpret_cast<const void*>(&k_row_pass<T, TIN, 8, true, MASK>));
  set(reinterpret_cast<const void*>(&k_row_pass<T, TIN, 16, false, MASK>));
  set(reinterpret_cast<const void*>(&k_row_pass<T, TIN, 16, true, MASK>));
}

hipError_t prepare_kernel_attributes() {
  static const hipError_t once = [] {
    const int lim = 160 * 1024;
    hipError_t e = hipSuccess;
    auto set = [&](const void* f) {
      if (e == hipSuccess) e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    };
    set_row_attrs<double, double, false>(set);
    set_row_attrs<double, float, false>(set);
    set_row_attrs<float, double, false>(set);
    set_row_attrs<float, float, false>(set);
    set_row_attrs<double, double, true>(set);
    set_row_attrs<double, float, true>(set);
    set_row_attrs<float, double, true>(set);
    set_row_attrs<float, float, true>(set);
    // (the FP64 column pass has only static LDS, see col_direct)
    set(reinterpret_cast<const void*>(&k_col_pass<float, 1>));
    set(reinterpret_cast<const void*>(&k_col_pass<float, 3>));
    set(reinterpret_cast<const void*>(&k_col_pass<float, 6>));
    set(reinterpret_cast<const void*>(&k_row_pass_batch<float, float, 8, true>));
    set(reinterpret_cast<const void*>(&k_col_pass_batch<float, 1>));
    set(reinterpret_cast<const void*>(&k_col_pass_batch<float, 3>));
    set(reinterpret_cast<const void*>(&k_col_pass_batch<float, 6>));
    return e;
  }();
  return once;
}

// ---- argument builders (shared by the single-pair and batched launches) ----

static RowArgs make_row_args(const Geometry& g, const sfft_desc& d, const void* R, const void* S,
                             unsigned char* ws, const Layout& l, const BuildPlan& p) {
  RowArgs a{};
  a.R = R; a.S = S; a.ld = d.ld; a.W = g.W; a.H = g.H; a.DK = g.DK; a.DB = g.DB; a.r = g.r;
  a.plan = make_fft_plan(g.W, p.radix_order);
  a.cR = d.ref_pedestal; a.cS = d.sci_pedestal;
  a.sx = g.W > 1 ? 2.0 / (double)(g.W - 1) : 0.0;
  a.F = ws + l.F; a.pitchK = g.pitchK; a.planeK = g.planeK;
  a.MR = reinterpret_cast<double*>(ws + l.MR);
  a.MS = reinterpret_cast<double*>(ws + l.MS);
  a.ER = reinterpret_cast<double*>(ws + l.ER);
  a.flags = reinterpret_cast<int*>(ws + l.flags);
  a.twW = p.twW;
  a.edge = reinterpret_cast<double*>(ws + l.edge);
  a.sci = 1;
  a.mask = nullptr;
  a.mask_ld = 0;
  a.frame = 0;
  return a;
}

template <typename T>
static size_t row_shmem(int W) {
  return sizeof(cx<T>) * (size_t)(W + W / 8 + 64 + (W + 63) / 64) + sizeof(double) * 64;
}

static ColArgs make_col_args(const Geometry& g, unsigned char* ws, const Layout& l, const BuildPlan& p) {
  ColArgs a{};
  a.F = ws + l.F; a.pitchK = g.pitchK; a.planeK = g.planeK;
  a.H = g.H; a.nkx = g.nkx; a.h = g.h; a.T = g.T; a.DK = g.DK;
  a.ngroups = (g.nkx - 2 + kColsPerWG - 1) / kColsPerWG;
  a.sy = g.H > 1 ? 2.0 / (double)(g.H - 1) : 0.0;
  a.strips = reinterpret_cast<cx<double>*>(ws + l.strips);
  a.tw128 = p.tw128;
  return a;
}

static int col_grid(const ColArgs& a) { return 8 * ((a.ngroups + 7) / 8); }

static XinvArgs make_xinv_args(const Geometry& g, unsigned char* ws, const Layout& l, const BuildPlan& p) {
  XinvArgs xa{};
  xa.strips = reinterpret_cast<const cx<double>*>(ws + l.strips);
  xa.C = reinterpret_cast<double*>(ws + l.C);
  xa.twW = static_cast<const cx<double>*>(p.twW64);
  xa.W = g.W; xa.nkx = g.nkx; xa.h = g.h; xa.r = g.r; xa.NKK = g.NKK; xa.NP = g.NP;
  xa.H = g.H; xa.nK = g.nK; xa.DK = g.DK;
  xa.sy = g.H > 1 ? 2.0 / (double)(g.H - 1) : 0.0;
  xa.edge = reinterpret_cast<const double*>(ws + l.edge);
  return xa;
}

static MomArgs make_mom_args(const Geometry& g, unsigned char* ws, const Layout& l) {
  MomArgs ma{};
  ma.MR = reinterpret_cast<const double*>(ws + l.MR);
  ma.MS = reinterpret_cast<const double*>(ws + l.MS);
  ma.ER = reinterpret_cast<const double*>(ws + l.ER);
  ma.mom = reinterpret_cast<double*>(ws + l.mom);
  ma.W = g.W; ma.H = g.H; ma.DK = g.DK; ma.DB = g.DB; ma.r = g.r;
  ma.sx = g.W > 1 ? 2.0 / (double)(g.W - 1) : 0.0;
  ma.sy = g.H > 1 ? 2.0 / (double)(g.H - 1) : 0.0;
  return ma;
}

static KbArgs make_kb_args(const Geometry& g, const MomArgs& ma, double* G, double* hv) {
  KbArgs ka{};
  ka.mom = ma.mom; ka.MR = ma.MR; ka.ER = ma.ER; ka.G = G; ka.hv = hv;
  ka.W = g.W; ka.H = g.H; ka.L = g.L; ka.r = g.r; ka.DK = g.DK; ka.DB = g.DB;
  ka.nK = g.nK; ka.nB = g.nB; ka.N = g.N; ka.sx = ma.sx; ka.sy = ma.sy;
  return ka;
}

// one wave per kernel-background entry plus one for the background block
static int kb_grid(const Geometry& g) { return (g.nK * g.L * g.L * g.nB + 1 + 3) / 4; }

static GatherArgs make_gather_args(const Geometry& g, const XinvArgs& xa, double* G, double* hv) {
  GatherArgs ga{};
  ga.C = xa.C; ga.G = G; ga.hv = hv; ga.L = g.L; ga.r = g.r; ga.h = g.h;
  ga.nK = g.nK; ga.NKK = g.NKK; ga.N = g.N;
  return ga;
}

template <typename T>
static hipError_t launch_row(const Geometry& g, const sfft_desc& d, const void* R, const void* S,
                             unsigned char* ws, const Layout& l, const BuildPlan& p,
                             hipStream_t st, bool reuse_sci, const unsigned char* mask, int64_t mask_ld,
                             int frame) {
  RowArgs a = make_row_args(g, d, R, S, ws, l, p);
  a.sci = reuse_sci ? 0 : 1;
  a.mask = mask;
  a.mask_ld = mask_ld;
  a.frame = frame;
  const size_t shmem = row_shmem<T>(g.W);
  // one resident wave of workgroups (3 per CU for rows up to 2048 pixels)
  const int per_cu = (g.W + kRowThreads - 1) / kRowThreads >= 16 ? 2 : 3;
  int grid = g.H < per_cu * p.num_cus ? g.H : per_cu * p.num_cus;
  const bool f32 = d.image_dtype == SFFT_F32;
  const bool mixed = (g.W % 3 == 0) || (g.W % 5 == 0);
  const bool masked = mask != nullptr || frame > 0;
#define SFFT_ROW_M(NQ, M)                                                                            \
  do {                                                                                               \
    if (mixed) {                                                                                     \
      if (f32) hipLaunchKernelGGL((k_row_pass<T, float, NQ, true, M>), dim3(grid), dim3(kRowThreads), \
                                  shmem, st, a);                                                    \
      else hipLaunchKernelGGL((k_row_pass<T, double, NQ, true, M>), dim3(grid), dim3(kRowThreads),    \
                              shmem, st, a);                                                        \
    } else {                                                                                         \
      if (f32) hipLaunchKernelGGL((k_row_pass<T, float, NQ, false, M>), dim3(grid),                  \
                                  dim3(kRowThreads), shmem, st, a);                                  \
      else hipLaunchKernelGGL((k_row_pass<T, double, NQ, false, M>), dim3(grid), dim3(kRowThreads),  \
                              shmem, st, a);                                                        \
    }                                                                                                \
  } while (0)
#define SFFT_ROW(NQ)                     \
  do {                                   \
    if (masked) SFFT_ROW_M(NQ, true);    \
    else SFFT_ROW_M(NQ, false);          \
  } while (0)
  const int nq = (g.W + kRowThreads - 1) / kRowThreads;
  if (nq <= 1) SFFT_ROW(1);
  else if (nq == 2) SFFT_ROW(2);
  else if (nq <= 4) SFFT_ROW(4);
  else if (nq <= 8) SFFT_ROW(8);
  else SFFT_ROW(16);
#undef SFFT_ROW
#undef SFFT_ROW_M
  return hipGetLastError();
}

template <typename T, int NK>
static hipError_t launch_col(const Geometry& g, unsigned char* ws, const Layout& l,
                             const BuildPlan& p, hipStream_t st) {
  const ColArgs a = make_col_args(g, ws, l, p);
  hipLaunchKernelGGL((k_col_pass<T, NK>), dim3(col_grid(a)), dim3(kColThreads), (col_pass_shmem<T, NK>()), st, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Output-pixel convention. With the kernel polynomial evaluated at the output
// pixel, design column (i, d) is p_i(x) R'(x - d). Where R'(u) is nonzero
// only at least r pixels from every edge, x = u + d never wraps and
// p_i(u + d) = sum_m T_d[m][i] p_m(u) exactly (binomial expansion in the
// shifted normalised coordinates, xt(u + dx) = xt(u) + 2 dx / (W - 1)):
//   T_d[(a', b')][(a, b)] = C(a, a') C(b, b') ex^(a - a') ey^(b - b'),
//   ex = 2 dx / (W - 1), ey = 2 dy / (H - 1), a' <= a, b' <= b.
// So the output-pixel design is the input-pixel one times the block-diagonal
// T (identity on the background), and its normal equations are
// G_out = T^T G T, h_out = T^T h. The build zeroes R' on the r-pixel frame
// (RowArgs::frame), assembles the input-pixel system, copies it aside and
// forms G_out, h_out entry by entry (at most (n(DK))^2 terms each).
// ---------------------------------------------------------------------------

struct OutpixArgs {
  const double* Gi;   // input-pixel G (copy), N x N
  const double* hi;   // input-pixel h (copy)
  double* G;
  double* hv;
  int N, L, r, nK, W, H;
  int ea[6], eb[6];   // monomial exponents (DK <= 2)
};

__device__ __forceinline__ double binom_small(int n, int k) {
  // n <= 2
  return (k == 0 || k == n) ? 1.0 : (double)n;
}

// T_d[m][i] for unknown block d (tap index) and monomials m, i
__device__ __forceinline__ double outpix_t(const OutpixArgs& a, int d, int m, int i) {
  const int am = a.ea[m], bm = a.eb[m], ai = a.ea[i], bi = a.eb[i];
  if (am > ai || bm > bi) return 0.0;
  const int dx = d % a.L - a.r, dy = d / a.L - a.r;
  const double ex = a.W > 1 ? 2.0 * dx / (double)(a.W - 1) : 0.0;
  const double ey = a.H > 1 ? 2.0 * dy / (double)(a.H - 1) : 0.0;
  double v = binom_small(ai, am) * binom_small(bi, bm);
  for (int k = am; k < ai; ++k) v *= ex;
  for (int k = bm; k < bi; ++k) v *= ey;
  return v;
}

// one thread per entry of G_out (and of h_out on row N); fixed summation order
__global__ __launch_bounds__(256) void k_outpix_transform(OutpixArgs a) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t total = (int64_t)a.N * a.N + a.N;
  if (idx >= total) return;
  const int LL = a.L * a.L, nKL = a.nK * LL;
  if (idx >= (int64_t)a.N * a.N) {
    const int p = (int)(idx - (int64_t)a.N * a.N);
    double v;
    if (p >= nKL) {
      v = a.hi[p];
    } else {
      const int i = p / LL, d = p % LL;
      v = 0.0;
      for (int m = 0; m < a.nK; ++m) {
        const double t = outpix_t(a, d, m, i);
        if (t != 0.0) v = fma(t, a.hi[m * LL + d], v);
      }
    }
    a.hv[p] = v;
    return;
  }
  const int p = (int)(idx / a.N), q = (int)(idx % a.N);
  const int ip = p < nKL ? p / LL : -1, dp = p % LL;
  const int iq = q < nKL ? q / LL : -1, dq = q % LL;
  double v = 0.0;
  for (int m = 0; m < (ip >= 0 ? a.nK : 1); ++m) {
    const double tp = ip >= 0 ? outpix_t(a, dp, m, ip) : 1.0;
    if (tp == 0.0) continue;
    const int row = ip >= 0 ? m * LL + dp : p;
    double u = 0.0;
    for (int n = 0; n < (iq >= 0 ? a.nK : 1); ++n) {
      const double tq = iq >= 0 ? outpix_t(a, dq, n, iq) : 1.0;
      if (tq == 0.0) continue;
      const int col = iq >= 0 ? n * LL + dq : q;
      u = fma(tq, a.Gi[(int64_t)row * a.N + col], u);
    }
    v = fma(tp, u, v);
  }
  a.G[(int64_t)p * a.N + q] = v;
}

// The science image's row spectrum (the last plane of F) and its DC /
// Nyquist values survive a solve and a subtract in the same workspace when
// the solve and subtract regions end before that plane; a build for another
// reference against the same science image (and science pedestal) can then
// skip its transform (the row moments still read the science image, cheaply,
// and check it for non-finite pixels).
bool sci_reusable(const sfft_desc& d) {
  const Geometry g = make_geometry(d);
  const Layout l = make_layout(g);
  const size_t sci_plane = l.F + (size_t)(g.nsig - 1) * g.planeK * g.cxsize;
  return l.solve_end <= sci_plane && l.sub_end <= sci_plane;
}

hipError_t launch_build_masked(const sfft_desc& d, const void* R, const void* S, const unsigned char* mask,
                               int64_t mask_ld, double* G, double* hv, unsigned char* ws, const BuildPlan& p,
                               const Prof* pf, hipStream_t st, bool reuse_sci);

hipError_t launch_build(const sfft_desc& d, const void* R, const void* S, double* G, double* hv,
                        unsigned char* ws, const BuildPlan& p, const Prof* pf, hipStream_t st,
                        bool reuse_sci) {
  return launch_build_masked(d, R, S, nullptr, 0, G, hv, ws, p, pf, st, reuse_sci);
}

hipError_t launch_build_masked(const sfft_desc& d, const void* R, const void* S, const unsigned char* mask,
                               int64_t mask_ld, double* G, double* hv, unsigned char* ws, const BuildPlan& p,
                               const Prof* pf, hipStream_t st, bool reuse_sci) {
  const Geometry g = make_geometry(d);
  const Layout l = make_layout(g);
  const bool outpix = d.convention == 1;
  hipError_t e;
  prof_begin(pf, SFFT_PROF_BUILD, st);
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, reinterpret_cast<int*>(ws + l.flags), 64, 0);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  {
    RowArgs ra = make_row_args(g, d, R, S, ws, l, p);
    ra.sci = reuse_sci ? 0 : 1;
    ra.mask = mask;
    ra.mask_ld = mask_ld;
    ra.frame = outpix ? g.r : 0;
    const bool masked = mask != nullptr || outpix;
    const dim3 mg(row_moments_grid(g.H));
    if (d.image_dtype == SFFT_F32) {
      if (masked) hipLaunchKernelGGL((k_row_moments<float, true>), mg, dim3(kRowThreads), 0, st, ra);
      else hipLaunchKernelGGL((k_row_moments<float, false>), mg, dim3(kRowThreads), 0, st, ra);
    } else {
      if (masked) hipLaunchKernelGGL((k_row_moments<double, true>), mg, dim3(kRowThreads), 0, st, ra);
      else hipLaunchKernelGGL((k_row_moments<double, false>), mg, dim3(kRowThreads), 0, st, ra);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  prof_begin(pf, SFFT_PROF_ROW_PASS, st);
  e = g.fp32 ? launch_row<float>(g, d, R, S, ws, l, p, st, reuse_sci, mask, mask_ld, outpix ? g.r : 0)
             : launch_row<double>(g, d, R, S, ws, l, p, st, reuse_sci, mask, mask_ld, outpix ? g.r : 0);
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
  const XinvArgs xa = make_xinv_args(g, ws, l, p);
  prof_begin(pf, SFFT_PROF_XINV, st);
  hipLaunchKernelGGL(k_strip_xinv, dim3(g.NP * (2 * g.h + 1)), dim3(256), 0, st, xa);
  prof_end(pf, SFFT_PROF_XINV, st);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const MomArgs ma = make_mom_args(g, ws, l);
  hipLaunchKernelGGL(k_moments, dim3(l.nmom), dim3(256), 0, st, ma);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const KbArgs ka = make_kb_args(g, ma, G, hv);
  hipLaunchKernelGGL(k_kb_assemble, dim3(kb_grid(g)), dim3(256), 0, st, ka);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const GatherArgs ga = make_gather_args(g, xa, G, hv);
  const int nKL = g.nK * g.L * g.L;
  hipLaunchKernelGGL(k_gather_kk, dim3((nKL + 255) / 256, nKL), dim3(256), 0, st, ga);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (outpix && g.DK > 0) {
    // the input-pixel system is copied aside into the solve's matrix region
    // (N^2 + N doubles fit in it; every build kernel that used it is done)
    double* Gi = reinterpret_cast<double*>(ws + l.A);
    double* hi = Gi + (int64_t)g.N * g.N;
    if ((e = hipMemcpyAsync(Gi, G, sizeof(double) * g.N * g.N, hipMemcpyDeviceToDevice, st)) != hipSuccess)
      return e;
    if ((e = hipMemcpyAsync(hi, hv, sizeof(double) * g.N, hipMemcpyDeviceToDevice, st)) != hipSuccess) return e;
    OutpixArgs oa{};
    oa.Gi = Gi; oa.hi = hi; oa.G = G; oa.hv = hv;
    oa.N = g.N; oa.L = g.L; oa.r = g.r; oa.nK = g.nK; oa.W = g.W; oa.H = g.H;
    const MonoTable mt = make_monos(g.DK);
    for (int i = 0; i < g.nK; ++i) { oa.ea[i] = mt.a[i]; oa.eb[i] = mt.b[i]; }
    const int64_t total = (int64_t)g.N * g.N + g.N;
    hipLaunchKernelGGL(k_outpix_transform, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, oa);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  prof_end(pf, SFFT_PROF_BUILD, st);
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// Batched build: every phase is one launch over all items of the batch. A
// flat grid is split into per-item block ranges (BatchTab); the argument
// structures of every item live in device memory owned by the batch plan.
// Items share the compute precision (FP32 spectra), the image type (FP32),
// the kernel degree and a row length of at most 2048 (one row-pass
// instantiation, radix 2/3/4/5/8).
// ---------------------------------------------------------------------------

struct BuildBatchHost {
  int n = 0, nK = 0;
  std::vector<RowArgs> row;
  std::vector<ColArgs> col;
  std::vector<XinvArgs> xinv;
  std::vector<MomArgs> mom;
  std::vector<KbArgs> kb;
  std::vector<GatherArgs> gat;
  std::vector<int*> flags;
  std::vector<BatchTab> trm, trow, tcol, txinv, tmom, tkb, tgat;
  int brm = 0, brow = 0, bcol = 0, bxinv = 0, bmom = 0, bkb = 0, bgat = 0;   // total blocks per phase
  size_t row_shmem = 0;
};

struct BuildBatchDev {
  RowArgs* row;
  ColArgs* col;
  XinvArgs* xinv;
  MomArgs* mom;
  KbArgs* kb;
  GatherArgs* gat;
  int* const* flags;
  BatchTab *trm, *trow, *tcol, *txinv, *tmom, *tkb, *tgat;
};

struct BuildBatch {
  BuildBatchHost h;
  BuildBatchDev d{};
};

__global__ void k_fill_flags_batch(int* const* flags, int n) {
  const int i = blockIdx.x;
  if (i < n && threadIdx.x < 64) flags[i][threadIdx.x] = 0;
}

static void tab_push(std::vector<BatchTab>& t, int& total, int nx, int ny) {
  BatchTab b{};
  b.start = total; b.nx = nx; b.ny = ny;
  t.push_back(b);
  total += nx * ny;
}

static hipError_t plan_build_batch(const BuildItem* items, int n, const BuildPlan* plans, int rows_per_block,
                                   BuildBatchHost& h) {
  h = BuildBatchHost{};
  h.n = n;
  for (int k = 0; k < n; ++k) {
    const BuildItem& it = items[k];
    const Geometry g = make_geometry(it.d);
    const Layout l = make_layout(g);
    if (!g.fp32 || it.d.image_dtype != SFFT_F32 || g.W > 2048) return hipErrorInvalidValue;
    if (k > 0 && g.nK != h.nK) return hipErrorInvalidValue;
    h.nK = g.nK;
    h.row.push_back(make_row_args(g, it.d, it.R, it.S, it.ws, l, plans[k]));
    tab_push(h.trm, h.brm, row_moments_grid(g.H), 1);
    const int rpb = rows_per_block > 0 ? rows_per_block : 4;
    tab_push(h.trow, h.brow, (g.H + rpb - 1) / rpb, 1);
    h.row_shmem = std::max(h.row_shmem, row_shmem<float>(g.W));
    const ColArgs ca = make_col_args(g, it.ws, l, plans[k]);
    h.col.push_back(ca);
    tab_push(h.tcol, h.bcol, col_grid(ca), 1);
    const XinvArgs xa = make_xinv_args(g, it.ws, l, plans[k]);
    h.xinv.push_back(xa);
    tab_push(h.txinv, h.bxinv, g.NP * (2 * g.h + 1), 1);
    const MomArgs ma = make_mom_args(g, it.ws, l);
    h.mom.push_back(ma);
    tab_push(h.tmom, h.bmom, l.nmom, 1);
    h.kb.push_back(make_kb_args(g, ma, it.G, it.hv));
    tab_push(h.tkb, h.bkb, kb_grid(g), 1);
    h.gat.push_back(make_gather_args(g, xa, it.G, it.hv));
    const int nKL = g.nK * g.L * g.L;
    tab_push(h.tgat, h.bgat, (nKL + 255) / 256, nKL);
    h.flags.push_back(reinterpret_cast<int*>(it.ws + l.flags));
  }
  return hipSuccess;
}

hipError_t build_batch_launch(const BuildBatch* b, const Prof* pf, hipStream_t st) {
  const BuildBatchHost& h = b->h;
  const BuildBatchDev& d = b->d;
  hipError_t e;
  prof_begin(pf, SFFT_PROF_BUILD, st);
  hipLaunchKernelGGL(k_fill_flags_batch, dim3(h.n), dim3(64), 0, st, d.flags, h.n);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_row_moments_batch, dim3(h.brm), dim3(kRowThreads), 0, st, d.row, d.trm, h.n);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  prof_begin(pf, SFFT_PROF_ROW_PASS, st);
  hipLaunchKernelGGL((k_row_pass_batch<float, float, 8, true>), dim3(h.brow), dim3(kRowThreads), h.row_shmem,
                     st, d.row, d.trow, h.n);
  prof_end(pf, SFFT_PROF_ROW_PASS, st);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  prof_begin(pf, SFFT_PROF_COL_PASS, st);
  switch (h.nK) {
    case 1: hipLaunchKernelGGL((k_col_pass_batch<float, 1>), dim3(h.bcol), dim3(kColThreads),
                               (col_pass_shmem<float, 1>()), st, d.col, d.tcol, h.n); break;
    case 3: hipLaunchKernelGGL((k_col_pass_batch<float, 3>), dim3(h.bcol), dim3(kColThreads),
                               (col_pass_shmem<float, 3>()), st, d.col, d.tcol, h.n); break;
    case 6: hipLaunchKernelGGL((k_col_pass_batch<float, 6>), dim3(h.bcol), dim3(kColThreads),
                               (col_pass_shmem<float, 6>()), st, d.col, d.tcol, h.n); break;
    default: return hipErrorInvalidValue;
  }
  prof_end(pf, SFFT_PROF_COL_PASS, st);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  prof_begin(pf, SFFT_PROF_XINV, st);
  hipLaunchKernelGGL(k_strip_xinv_batch, dim3(h.bxinv), dim3(256), 0, st, d.xinv, d.txinv, h.n);
  prof_end(pf, SFFT_PROF_XINV, st);
  hipLaunchKernelGGL(k_moments_batch, dim3(h.bmom), dim3(256), 0, st, d.mom, d.tmom, h.n);
  hipLaunchKernelGGL(k_kb_assemble_batch, dim3(h.bkb), dim3(256), 0, st, d.kb, d.tkb, h.n);
  hipLaunchKernelGGL(k_gather_kk_batch, dim3(h.bgat), dim3(256), 0, st, d.gat, d.tgat, h.n);
  prof_end(pf, SFFT_PROF_BUILD, st);
  return hipGetLastError();
}

hipError_t launch_bg_refit(const sfft_desc& d, const void* R, const void* S, double* coef, double* G,
                           double* hv, unsigned char* ws, const BuildPlan& p, hipStream_t st) {
  const Geometry g = make_geometry(d);
  const Layout l = make_layout(g);
  const RowArgs ra = make_row_args(g, d, R, S, ws, l, p);
  if (d.image_dtype == SFFT_F32)
    hipLaunchKernelGGL((k_row_moments<float, false>), dim3(row_moments_grid(g.H)), dim3(kRowThreads), 0, st, ra);
  else
    hipLaunchKernelGGL((k_row_moments<double, false>), dim3(row_moments_grid(g.H)), dim3(kRowThreads), 0, st, ra);
  hipError_t e;
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const MomArgs ma = make_mom_args(g, ws, l);
  hipLaunchKernelGGL(k_moments, dim3(l.nmom), dim3(256), 0, st, ma);
  const KbArgs ka = make_kb_args(g, ma, G, hv);
  hipLaunchKernelGGL(k_kb_assemble, dim3(kb_grid(g)), dim3(256), 0, st, ka);
  hipLaunchKernelGGL(k_bg_refit, dim3(1), dim3(256), 0, st, (const double*)G, (const double*)hv, coef, g.N,
                     g.nK * g.L * g.L, g.nB);
  return hipGetLastError();
}

// device copies of the host tables, carved from one allocation
static size_t dev_bytes(const BuildBatchHost& h) {
  const size_t n = (size_t)h.n;
  size_t o = 0;
  auto add = [&](size_t b) { o = align256(o) + b; };
  add(n * sizeof(RowArgs)); add(n * sizeof(ColArgs)); add(n * sizeof(XinvArgs)); add(n * sizeof(MomArgs));
  add(n * sizeof(KbArgs)); add(n * sizeof(GatherArgs)); add(n * sizeof(int*));
  for (int t = 0; t < 7; ++t) add(n * sizeof(BatchTab));
  return align256(o);
}

static hipError_t upload(const BuildBatchHost& h, unsigned char* dev, BuildBatchDev& d) {
  std::vector<unsigned char> blob(dev_bytes(h));
  size_t o = 0;
  auto put = [&](const void* src, size_t b) {
    o = align256(o);
    std::memcpy(blob.data() + o, src, b);
    unsigned char* p = dev + o;
    o += b;
    return p;
  };
  const size_t n = (size_t)h.n;
  d.row = reinterpret_cast<RowArgs*>(put(h.row.data(), n * sizeof(RowArgs)));
  d.col = reinterpret_cast<ColArgs*>(put(h.col.data(), n * sizeof(ColArgs)));
  d.xinv = reinterpret_cast<XinvArgs*>(put(h.xinv.data(), n * sizeof(XinvArgs)));
  d.mom = reinterpret_cast<MomArgs*>(put(h.mom.data(), n * sizeof(MomArgs)));
  d.kb = reinterpret_cast<KbArgs*>(put(h.kb.data(), n * sizeof(KbArgs)));
  d.gat = reinterpret_cast<GatherArgs*>(put(h.gat.data(), n * sizeof(GatherArgs)));
  d.flags = reinterpret_cast<int* const*>(put(h.flags.data(), n * sizeof(int*)));
  d.trm = reinterpret_cast<BatchTab*>(put(h.trm.data(), n * sizeof(BatchTab)));
  d.trow = reinterpret_cast<BatchTab*>(put(h.trow.data(), n * sizeof(BatchTab)));
  d.tcol = reinterpret_cast<BatchTab*>(put(h.tcol.data(), n * sizeof(BatchTab)));
  d.txinv = reinterpret_cast<BatchTab*>(put(h.txinv.data(), n * sizeof(BatchTab)));
  d.tmom = reinterpret_cast<BatchTab*>(put(h.tmom.data(), n * sizeof(BatchTab)));
  d.tkb = reinterpret_cast<BatchTab*>(put(h.tkb.data(), n * sizeof(BatchTab)));
  d.tgat = reinterpret_cast<BatchTab*>(put(h.tgat.data(), n * sizeof(BatchTab)));
  return hipMemcpy(dev, blob.data(), blob.size(), hipMemcpyHostToDevice);
}

BuildBatch* build_batch_create(const BuildItem* items, int n, const BuildPlan* plans, int rows_per_block,
                               hipError_t* err) {
  BuildBatch* b = new (std::nothrow) BuildBatch();
  if (!b) { *err = hipErrorOutOfMemory; return nullptr; }
  *err = plan_build_batch(items, n, plans, rows_per_block, b->h);
  if (*err != hipSuccess) { delete b; return nullptr; }
  return b;
}

size_t build_batch_dev_bytes(const BuildBatch* b) { return dev_bytes(b->h); }

hipError_t build_batch_upload(BuildBatch* b, unsigned char* dev) { return upload(b->h, dev, b->d); }

void build_batch_destroy(BuildBatch* b) { delete b; }

}  // namespace sfft
