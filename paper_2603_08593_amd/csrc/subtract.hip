// sfft_subtract kernels: convolve the reference with the fitted spatially
// varying kernel, subtract from the science image, and accumulate the chi2
// judge (paper Sec. 2.3.2: difference image; Sec. 1: delta-basis kernel).
//
// D(x) = S'(x) - sum_d w_d(x - d) R'(x - d) - sum_c b_c q_c(x), where the
// kernel value w_d(u) = sum_m c_m(d, u_y) xt(u_x)^m is evaluated at the input
// pixel u by Horner in xt, with c_m(d, u_y) = sum_b a_((m,b),d) yt(u_y)^b
// formed once per (tap, input row) and shared by a thread's 8 pixels.
// Output tiles of 64 x 32 pixels; the reference tile with an r-pixel halo is
// staged in LDS in FP64; accumulation in FP64. The chi2 judge's kappa2(x)
// polynomial depends on the coefficients only: a one-workgroup kernel forms
// it once per launch.
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "batch.hpp"
#include "common.hpp"
#include "layout.hpp"

namespace sfft {

struct SubArgs {
  const void* R;
  const void* S;
  void* D;
  int64_t ld;
  const double* coef;
  double* partials;
  double* k2;         // kappa2 polynomial: K2[e][f], e, f <= 2 DK
  int W, H, N, DB, want_chi2, L, DK;
  double cR, cS, sx, sy;
};

__device__ __forceinline__ int mono_index(int a, int b) {
  const int d = a + b;
  return d * (d + 1) / 2 + b;
}

// a * b + c, rounded twice (never contracted into one fused operation)
__device__ __forceinline__ double mul_add_nc(double a, double b, double c) {
#pragma clang fp contract(off)
  return a * b + c;
}

// kappa2(x) = sum_d (sum_i a_(i,d) p_i(x))^2 = sum_{e,f} K2[e][f] xt^e yt^f:
// Q[i][j] = sum_d a_(i,d) a_(j,d), K2[ai+aj][bi+bj] += Q[i][j]. One
// workgroup of 256 threads: the kernel coefficients are staged in LDS, each
// Q entry is summed as 7 fixed chunks (one thread each) added in order.
constexpr int kK2Threads = 256;
constexpr int kK2Chunks = 7;

__device__ __forceinline__ void kappa2_body(const SubArgs& a) {
  __shared__ double cf[6 * 225];
  __shared__ double part[36 * kK2Chunks];
  __shared__ double Q[36];
  const int DK = a.DK, NK = (DK + 1) * (DK + 2) / 2, LL = a.L * a.L, NE = 2 * DK + 1;
  const int t = threadIdx.x;
  for (int i = t; i < NK * LL; i += kK2Threads) cf[i] = a.coef[i];
  __syncthreads();
  const int len = (LL + kK2Chunks - 1) / kK2Chunks;
  if (t < NK * NK * kK2Chunks) {
    const int q = t / kK2Chunks, ch = t % kK2Chunks;
    const int i = q / NK, j = q % NK;
    double sacc = 0.0;
    const int d1 = min(LL, (ch + 1) * len);
    for (int dd = ch * len; dd < d1; ++dd) sacc = fma(cf[i * LL + dd], cf[j * LL + dd], sacc);
    part[t] = sacc;
  }
  __syncthreads();
  if (t < NK * NK) {
    double sacc = 0.0;
    for (int ch = 0; ch < kK2Chunks; ++ch) sacc += part[t * kK2Chunks + ch];
    Q[t] = sacc;
  }
  __syncthreads();
  if (t < NE * NE) {
    const int e = t / NE, f = t % NE;
    double sacc = 0.0;
    int i = 0;
    for (int di = 0; di <= DK; ++di)
      for (int bi = 0; bi <= di; ++bi, ++i) {
        int j = 0;
        for (int dj = 0; dj <= DK; ++dj)
          for (int bj = 0; bj <= dj; ++bj, ++j)
            if ((di - bi) + (dj - bj) == e && bi + bj == f) sacc += Q[i * NK + j];
      }
    a.k2[t] = sacc;
  }
}

__global__ __launch_bounds__(kK2Threads) void k_kappa2(SubArgs a) { kappa2_body(a); }
__global__ __launch_bounds__(kK2Threads) void k_kappa2_batch(const SubArgs* args) { kappa2_body(args[blockIdx.x]); }

// OUTPIX: the kernel polynomial is evaluated at the output pixel x (the
// output-pixel convention) instead of the input pixel x - d: the Horner
// coordinates are those of the output row and pixel.
//
// TY: output tile height (the tile is kSubTX = 64 pixels wide, one thread per
// 8 pixels of a row, so the workgroup has 8 * TY threads).
template <int L, int DK, typename TIO, bool OUTPIX = false, int TY = kSubTY>
__device__ __forceinline__ void subtract_body(const SubArgs& a, const VB vb) {
  constexpr int r = (L - 1) / 2;
  constexpr int NK = (DK + 1) * (DK + 2) / 2;
  constexpr int TX = kSubTX, P = 8;
  constexpr int NT = TX * TY / P;
  constexpr int RW = TX + 2 * r, RH = TY + 2 * r;
  constexpr int NQ = P + 2 * r;
  // LDS tile with each run of 8 columns skewed by one slot (column lx at
  // lx + lx / 8) and a row pitch of 8 mod 16 doubles: the threads of a wave
  // read their windows (8 pixels apart, 8 rows) from distinct banks
  constexpr int RWP = ((RW - 1 + (RW - 1) / 8 + 1 + 7) / 16) * 16 + 8;
  __shared__ double Rt[RH][RWP];
  auto col = [](int lx) { return lx + (lx >> 3); };
  static_assert(P == 8, "the skewed window offsets assume 8 pixels per thread");
  __shared__ double red[NT / 64];
  const int tid = threadIdx.x;
  const int W = a.W, H = a.H;
  // the fitted coefficients are read-only for the whole launch: reading them
  // through the constant address space lets uniform reads use scalar loads
  const __attribute__((address_space(4))) double* coef =
      (const __attribute__((address_space(4))) double*)a.coef;
  const int x0 = vb.x * TX, y0 = vb.y * TY;
  // tiles whose halo stays inside the image need no periodic wrap
  const bool inner = x0 >= r && x0 + RW - r <= W && y0 >= r && y0 + RH - r <= H;
  if (inner) {
    const TIO* Rb = static_cast<const TIO*>(a.R) + (int64_t)(y0 - r) * a.ld + (x0 - r);
    for (int i = tid; i < RH * RW; i += NT) {
      const int ly = i / RW, lx = i - (i / RW) * RW;
      Rt[ly][col(lx)] = (double)Rb[(int64_t)ly * a.ld + lx] - a.cR;
    }
  } else {
    for (int i = tid; i < RH * RW; i += NT) {
      const int ly = i / RW, lx = i - (i / RW) * RW;
      int yy = y0 + ly - r, xx = x0 + lx - r;
      yy = (yy < 0) ? yy + H : yy;
      yy = (yy >= H) ? yy - H : yy;
      yy = (yy >= H) ? yy - H : yy;
      xx = (xx < 0) ? xx + W : xx;
      xx = (xx >= W) ? xx - W : xx;
      xx = (xx >= W) ? xx - W : xx;
      Rt[ly][col(lx)] = (double)static_cast<const TIO*>(a.R)[(int64_t)yy * a.ld + xx] - a.cR;
    }
  }
  __syncthreads();
  const int tx = tid & 7, ty = tid >> 3;
  const int y = y0 + ty;
  const int xb = x0 + P * tx;
  double xq[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    int ux = xb + q - r;
    if (!inner) {
      ux = (ux < 0) ? ux + W : ux;
      ux = (ux >= W) ? ux - W : ux;
      ux = (ux >= W) ? ux - W : ux;
    }
    xq[q] = (double)ux * a.sx - 1.0;
  }
  double acc[P];
#pragma unroll
  for (int p = 0; p < P; ++p) acc[p] = 0.0;
  // output-pixel convention: xt of the thread's own pixels (no wrap needed;
  // values of pixels past the image are never stored)
  double xo[OUTPIX ? P : 1];
#pragma unroll
  for (int p = 0; p < (OUTPIX ? P : 1); ++p) xo[p] = (double)(xb + p) * a.sx - 1.0;
#pragma unroll 1
  for (int dyi = 0; dyi < L; ++dyi) {
    const int lr = ty + (L - 1 - dyi);           // local row of u_y = y - dy
    int uy = y - (dyi - r);
    uy = (uy < 0) ? uy + H : uy;
    uy = (uy >= H) ? uy - H : uy;
    uy = (uy >= H) ? uy - H : uy;
    const double yt = OUTPIX ? (double)y * a.sy - 1.0 : (double)uy * a.sy - 1.0;
    double win[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) win[q] = Rt[lr][9 * tx + q + (q >> 3)];   // col(8 tx + q)
#pragma unroll
    for (int dxi = 0; dxi < L; ++dxi) {
      const int tap = dyi * L + dxi;
      // c_m = sum_b a_((m,b),d) yt^b by Horner in yt; the coefficients are
      // uniform across the workgroup and come through the scalar cache
      double cm[DK + 1];
#pragma unroll
      for (int m = 0; m <= DK; ++m) {
        double s = coef[mono_index(m, DK - m) * L * L + tap];
        if (DK - m - 1 >= 0) {
          // first step as a separate multiply and add: a fused step would
          // read two scalar operands, which one VALU instruction cannot
          s = mul_add_nc(s, yt, coef[mono_index(m, DK - m - 1) * L * L + tap]);
#pragma unroll
          for (int b = DK - m - 2; b >= 0; --b) s = fma(s, yt, coef[mono_index(m, b) * L * L + tap]);
        }
        cm[m] = s;
      }
      // Horner in xt for all P pixels stage by stage: P independent chains
      double w[P];
#pragma unroll
      for (int p = 0; p < P; ++p) w[p] = cm[DK];
#pragma unroll
      for (int m = DK - 1; m >= 0; --m)
#pragma unroll
        for (int p = 0; p < P; ++p) w[p] = fma(w[p], OUTPIX ? xo[OUTPIX ? p : 0] : xq[p + (L - 1 - dxi)], cm[m]);
#pragma unroll
      for (int p = 0; p < P; ++p) acc[p] = fma(w[p], win[p + (L - 1 - dxi)], acc[p]);
    }
  }
  // background, difference, chi2. The thread's indices are formed again
  // here, behind an empty asm statement, so that the compiler does not keep
  // per-pixel column indices live (spilled) across the tap loop.
  int tid_e = tid;
  asm volatile("" : "+v"(tid_e));
  const int te_x = tid_e & 7, te_y = tid_e >> 3;
  const int ye = y0 + te_y, xbe = x0 + P * te_x;
  const double yto = (double)ye * a.sy - 1.0;
  const double* bg = a.coef + NK * L * L;
  const int DB = a.DB;
  double chi = 0.0;
  if (ye < H) {
    // per-row background polynomial in xt: coefficients e_k(yt)
    double ek[5] = {0, 0, 0, 0, 0};
    {
      int c = 0;
      for (int d = 0; d <= DB; ++d)
        for (int b = 0; b <= d; ++b, ++c) {
          double ypw = 1.0;
          for (int t = 0; t < b; ++t) ypw *= yto;
          ek[d - b] = fma(bg[c], ypw, ek[d - b]);
        }
    }
    double kk[2 * DK + 1];
    if (a.want_chi2) {
      const __attribute__((address_space(4))) double* K2 =
          (const __attribute__((address_space(4))) double*)a.k2;
#pragma unroll
      for (int e = 0; e <= 2 * DK; ++e) {
        double s = 0.0;
#pragma unroll
        for (int f = 2 * DK; f >= 0; --f) s = fma(s, yto, K2[e * (2 * DK + 1) + f]);
        kk[e] = s;
      }
    }
    // the thread's 8 pixels of S and D as two 16-byte accesses when the
    // images are FP32, the row segment is 16-byte aligned and inside the image
    const TIO* srow = static_cast<const TIO*>(a.S) + (int64_t)ye * a.ld + xbe;
    TIO* drow = static_cast<TIO*>(a.D) + (int64_t)ye * a.ld + xbe;
    constexpr bool kF32 = sizeof(TIO) == 4;
    const bool vec = kF32 && xbe + P <= W &&
                     ((reinterpret_cast<uintptr_t>(srow) | reinterpret_cast<uintptr_t>(drow)) & 15) == 0;
    double sv8[P], dv8[P];
    if (vec) {
      const float4 s0 = reinterpret_cast<const float4*>(srow)[0];
      const float4 s1 = reinterpret_cast<const float4*>(srow)[1];
      sv8[0] = s0.x; sv8[1] = s0.y; sv8[2] = s0.z; sv8[3] = s0.w;
      sv8[4] = s1.x; sv8[5] = s1.y; sv8[6] = s1.z; sv8[7] = s1.w;
    } else {
#pragma unroll
      for (int p = 0; p < P; ++p) sv8[p] = (xbe + p < W) ? (double)srow[p] : 0.0;
    }
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const int x = xbe + p;
      dv8[p] = 0.0;
      if (x < W) {
        const double xt = (double)x * a.sx - 1.0;
        double bgv = 0.0;
        for (int k = DB; k >= 0; --k) bgv = fma(bgv, xt, ek[k]);
        const double sv = sv8[p];
        const double dv = (sv - a.cS) - acc[p] - bgv;
        dv8[p] = dv;
        if (!vec) drow[p] = (TIO)dv;
        if (a.want_chi2 && x >= r && x < W - r && ye >= r && ye < H - r) {
          double k2v = 0.0;
#pragma unroll
          for (int e = 2 * DK; e >= 0; --e) k2v = fma(k2v, xt, kk[e]);
          const double rv = Rt[te_y + r][9 * te_x + (p + r) + ((p + r) >> 3)] + a.cR;   // col(8 te_x + p + r)
          const double var = fmax(sv, 1.0) + k2v * fmax(rv, 1.0);
          // 1 / var: hardware estimate and two Newton steps (var >= 1)
          double iv = __builtin_amdgcn_rcp(var);
          iv = fma(fma(-var, iv, 1.0), iv, iv);
          iv = fma(fma(-var, iv, 1.0), iv, iv);
          chi = fma(dv * dv, iv, chi);
        }
      }
    }
    if (vec) {
      reinterpret_cast<float4*>(drow)[0] = float4{(float)dv8[0], (float)dv8[1], (float)dv8[2], (float)dv8[3]};
      reinterpret_cast<float4*>(drow)[1] = float4{(float)dv8[4], (float)dv8[5], (float)dv8[6], (float)dv8[7]};
    }
  }
  if (a.want_chi2) {
    chi = wave_sum(chi);
    if ((tid & 63) == 0) red[tid >> 6] = chi;
    __syncthreads();
    if (tid == 0) {
      double t = red[0];
#pragma unroll
      for (int w = 1; w < NT / 64; ++w) t += red[w];
      a.partials[vb.y * vb.nx + vb.x] = t;
    }
  }
}

// Four waves per SIMD (at most 128 registers) for the shapes whose kernels
// (single-pair and batched) fit in them without spilling (checked on the
// compiler's output: DK = 0, and DK = 2 with 7 <= L <= 11); otherwise the
// compiler's choice
template <int L, int DK>
constexpr int subtract_waves() { return (DK == 0 || (DK == 2 && L >= 7 && L <= 11)) ? 4 : 1; }

// XCD-aware tile columns: consecutive workgroups of a launch go to the 8
// XCDs in turn, so workgroup column bx takes tile column (bx mod 8) * per +
// bx / 8 (per = ceil(tile columns / 8)): each XCD works through a strip of
// per adjacent tile columns over all tile rows, and the reference halo that
// neighbouring tiles share stays in that XCD's L2. The grid has 8 * per
// workgroup columns; the surplus ones exit.
template <int L, int DK, typename TIO, bool OUTPIX>
__global__ __launch_bounds__(kSubThreads, (subtract_waves<L, DK>())) void k_subtract(SubArgs a) {
  const int gx = (a.W + kSubTX - 1) / kSubTX;
  const int per = (gx + 7) >> 3;
  const int tx = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
  if (tx >= gx) return;
  subtract_body<L, DK, TIO, OUTPIX>(a, VB{tx, (int)blockIdx.y, gx, (int)gridDim.y});
}

// batched items (FP32 images), tiles of 64 x TY pixels
template <int L, int DK, int TY>
__global__ __launch_bounds__(kSubTX * TY / 8, (subtract_waves<L, DK>())) void k_subtract_batch(const SubArgs* args, const BatchTab* tab, int n) {
  int item;
  VB vb;
  if (batch_locate(tab, n, item, vb)) subtract_body<L, DK, float, false, TY>(args[item], vb);
}

__global__ __launch_bounds__(1024) void k_chi2_final(const double* partials, int n, double dof,
                                                     double* out) {
  __shared__ double scratch[16];
  double s = 0.0;
  // fixed assignment of partials to threads, fixed tree: reproducible
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += partials[i];
  s = block_sum(s, scratch);
  if (threadIdx.x == 0) *out = s / dof;
}

template <int L, int DK>
static hipError_t launch_sub_ldk(const SubArgs& a, bool f32, bool outpix, dim3 grid, hipStream_t st) {
  if (outpix) {
    if (f32) hipLaunchKernelGGL((k_subtract<L, DK, float, true>), grid, dim3(kSubThreads), 0, st, a);
    else hipLaunchKernelGGL((k_subtract<L, DK, double, true>), grid, dim3(kSubThreads), 0, st, a);
  } else {
    if (f32) hipLaunchKernelGGL((k_subtract<L, DK, float, false>), grid, dim3(kSubThreads), 0, st, a);
    else hipLaunchKernelGGL((k_subtract<L, DK, double, false>), grid, dim3(kSubThreads), 0, st, a);
  }
  return hipGetLastError();
}

template <int L>
static hipError_t launch_sub_l(const SubArgs& a, int DK, bool f32, bool outpix, dim3 grid, hipStream_t st) {
  // DK = 0: the two conventions coincide (the polynomial is a constant)
  switch (DK) {
    case 0: return launch_sub_ldk<L, 0>(a, f32, false, grid, st);
    case 1: return launch_sub_ldk<L, 1>(a, f32, outpix, grid, st);
    case 2: return launch_sub_ldk<L, 2>(a, f32, outpix, grid, st);
    default: return hipErrorInvalidValue;
  }
}

static SubArgs make_sub_args(const sfft_desc& d, const void* R, const void* S, const double* coef, void* D,
                             bool want_chi2, double* partials, double* k2) {
  const Geometry g = make_geometry(d);
  SubArgs a{};
  a.R = R; a.S = S; a.D = D; a.ld = d.ld; a.coef = coef;
  a.partials = partials;
  a.k2 = k2;
  a.W = g.W; a.H = g.H; a.N = g.N; a.DB = g.DB; a.want_chi2 = want_chi2; a.L = g.L; a.DK = g.DK;
  a.cR = d.ref_pedestal; a.cS = d.sci_pedestal;
  a.sx = g.W > 1 ? 2.0 / (double)(g.W - 1) : 0.0;
  a.sy = g.H > 1 ? 2.0 / (double)(g.H - 1) : 0.0;
  return a;
}

static double chi2_dof(const Geometry& g) {
  const double inner = (double)(g.W - 2 * g.r) * (double)(g.H - 2 * g.r);
  return inner - (double)g.N;
}

hipError_t launch_subtract(const sfft_desc& d, const void* R, const void* S, const double* coef,
                           void* D, double* chi2, unsigned char* ws, const Prof* pf,
                           hipStream_t st) {
  const Geometry g = make_geometry(d);
  const Layout l = make_layout(g);
  const SubArgs a = make_sub_args(d, R, S, coef, D, chi2 != nullptr,
                                  reinterpret_cast<double*>(ws + l.partials),
                                  reinterpret_cast<double*>(ws + l.k2));
  hipError_t e;
  const dim3 grid(8 * (((g.W + kSubTX - 1) / kSubTX + 7) / 8), (g.H + kSubTY - 1) / kSubTY);
  const bool f32 = d.image_dtype == SFFT_F32;
  prof_begin(pf, SFFT_PROF_SUBTRACT, st);
  if (chi2) {
    hipLaunchKernelGGL(k_kappa2, dim3(1), dim3(kK2Threads), 0, st, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  switch (g.L) {
    case 1: e = launch_sub_l<1>(a, g.DK, f32, d.convention == 1, grid, st); break;
    case 3: e = launch_sub_l<3>(a, g.DK, f32, d.convention == 1, grid, st); break;
    case 5: e = launch_sub_l<5>(a, g.DK, f32, d.convention == 1, grid, st); break;
    case 7: e = launch_sub_l<7>(a, g.DK, f32, d.convention == 1, grid, st); break;
    case 9: e = launch_sub_l<9>(a, g.DK, f32, d.convention == 1, grid, st); break;
    case 11: e = launch_sub_l<11>(a, g.DK, f32, d.convention == 1, grid, st); break;
    case 13: e = launch_sub_l<13>(a, g.DK, f32, d.convention == 1, grid, st); break;
    case 15: e = launch_sub_l<15>(a, g.DK, f32, d.convention == 1, grid, st); break;
    default: return hipErrorInvalidValue;
  }
  prof_end(pf, SFFT_PROF_SUBTRACT, st);
  if (e != hipSuccess) return e;
  if (chi2) {
    hipLaunchKernelGGL(k_chi2_final, dim3(1), dim3(1024), 0, st,
                       (const double*)a.partials, l.npartials, chi2_dof(g), chi2);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

// ---- allocation-free subtract ---------------------------------------------
// For callers that cannot allocate (code under stream capture, serving loops):
// the chi2 partial sums and the kappa2 coefficients live in this file-scope
// device array instead of a caller workspace. Each device holds its own copy;
// its address is looked up once per device (sfft_create, with the device
// current) and only that address is used on the host. Calls on one device
// share the array, so calls that overlap on one device race; every call
// rewrites all the entries it reads (one partial per output tile, the kappa2
// coefficients), so nothing needs clearing between calls.
constexpr int kNoAllocMaxPartials = 1 << 16;   // 64 x 32 tiles: up to 2^27 pixels
constexpr int kNoAllocK2 = 128;
constexpr int kNoAllocMaxDevices = 64;
static __device__ __align__(256) double scratch[kNoAllocMaxPartials + kNoAllocK2];
static double* g_noalloc_ptr[kNoAllocMaxDevices] = {};
static std::mutex g_noalloc_mu;

hipError_t noalloc_prepare(int device) {
  if (device < 0 || device >= kNoAllocMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (g_noalloc_ptr[device]) return hipSuccess;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_noalloc_ptr[device] = static_cast<double*>(ptr);
  return hipSuccess;
}

int noalloc_max_partials() { return kNoAllocMaxPartials; }

hipError_t launch_subtract_noalloc(int device, const sfft_desc& d, const void* R, const void* S,
                                   const double* coef, void* D, double* chi2, hipStream_t st) {
  if (device < 0 || device >= kNoAllocMaxDevices) return hipErrorInvalidDevice;
  double* base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    base = g_noalloc_ptr[device];
  }
  if (!base) return hipErrorNotInitialized;
  const Geometry g = make_geometry(d);
  const int np = subtract_blocks(g);
  if (np > kNoAllocMaxPartials) return hipErrorInvalidValue;
  const SubArgs a = make_sub_args(d, R, S, coef, D, chi2 != nullptr, base, base + kNoAllocMaxPartials);
  hipError_t e;
  const dim3 grid(8 * (((g.W + kSubTX - 1) / kSubTX + 7) / 8), (g.H + kSubTY - 1) / kSubTY);
  const bool f32 = d.image_dtype == SFFT_F32;
  if (chi2) {
    hipLaunchKernelGGL(k_kappa2, dim3(1), dim3(kK2Threads), 0, st, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  switch (g.L) {
    case 1: e = launch_sub_l<1>(a, g.DK, f32, d.convention == 1, grid, st); break;
    case 3: e = launch_sub_l<3>(a, g.DK, f32, d.convention == 1, grid, st); break;
    case 5: e = launch_sub_l<5>(a, g.DK, f32, d.convention == 1, grid, st); break;
    case 7: e = launch_sub_l<7>(a, g.DK, f32, d.convention == 1, grid, st); break;
    case 9: e = launch_sub_l<9>(a, g.DK, f32, d.convention == 1, grid, st); break;
    case 11: e = launch_sub_l<11>(a, g.DK, f32, d.convention == 1, grid, st); break;
    case 13: e = launch_sub_l<13>(a, g.DK, f32, d.convention == 1, grid, st); break;
    case 15: e = launch_sub_l<15>(a, g.DK, f32, d.convention == 1, grid, st); break;
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  if (chi2) {
    hipLaunchKernelGGL(k_chi2_final, dim3(1), dim3(1024), 0, st, (const double*)a.partials, np,
                       chi2_dof(g), chi2);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

// ---- batched subtract: one launch per kernel size L in the batch (the
// kernel-size loop is unrolled at compile time), then one chi2 launch ----

struct Chi2Item {
  const double* partials;
  double* out;
  double dof;
  int n;
};

__global__ __launch_bounds__(1024) void k_chi2_final_batch(const Chi2Item* items) {
  __shared__ double scratch[16];
  const Chi2Item& it = items[blockIdx.x];
  double s = 0.0;
  for (int i = threadIdx.x; i < it.n; i += blockDim.x) s += it.partials[i];
  s = block_sum(s, scratch);
  if (threadIdx.x == 0) *it.out = s / it.dof;
}

struct SubBatch {
  int n = 0, DK = 0;
  int tile_rows = kSubTY;                    // output tile height: 16, 32 or 64
  std::vector<int> Ls;                       // distinct kernel sizes
  std::vector<std::vector<SubArgs>> args;    // per size
  std::vector<std::vector<BatchTab>> tabs;   // per size
  std::vector<int> blocks;                   // per size
  std::vector<Chi2Item> chi;
  std::vector<SubArgs*> dargs;
  std::vector<BatchTab*> dtabs;
  Chi2Item* dchi = nullptr;
};

SubBatch* sub_batch_create(const SubItem* items, int n, int tile_rows, hipError_t* err) {
  if (tile_rows != 16 && tile_rows != 32 && tile_rows != 64) {
    *err = hipErrorInvalidValue;
    return nullptr;
  }
  SubBatch* b = new (std::nothrow) SubBatch();
  if (!b) { *err = hipErrorOutOfMemory; return nullptr; }
  b->n = n;
  b->tile_rows = tile_rows;
  for (int k = 0; k < n; ++k) {
    const SubItem& it = items[k];
    const Geometry g = make_geometry(it.d);
    if ((k > 0 && g.DK != b->DK) || it.d.image_dtype != SFFT_F32 || !it.chi2) {
      delete b;
      *err = hipErrorInvalidValue;
      return nullptr;
    }
    b->DK = g.DK;
    int slot = -1;
    for (size_t q = 0; q < b->Ls.size(); ++q)
      if (b->Ls[q] == g.L) slot = (int)q;
    if (slot < 0) {
      slot = (int)b->Ls.size();
      b->Ls.push_back(g.L);
      b->args.emplace_back();
      b->tabs.emplace_back();
      b->blocks.push_back(0);
    }
    const Layout l = make_layout(g);
    b->args[slot].push_back(make_sub_args(it.d, it.R, it.S, it.coef, it.D, true,
                                          reinterpret_cast<double*>(it.ws + l.partials),
                                          reinterpret_cast<double*>(it.ws + l.k2)));
    BatchTab t{};
    t.start = b->blocks[slot];
    t.nx = (g.W + kSubTX - 1) / kSubTX;
    t.ny = (g.H + tile_rows - 1) / tile_rows;
    b->tabs[slot].push_back(t);
    b->blocks[slot] += t.nx * t.ny;
    Chi2Item c{};
    c.partials = reinterpret_cast<const double*>(it.ws + l.partials);
    c.out = it.chi2;
    c.dof = chi2_dof(g);
    c.n = subtract_blocks(g, tile_rows);   // within the workspace's room (tile_rows >= kSubTYMin)
    b->chi.push_back(c);
  }
  *err = hipSuccess;
  return b;
}

size_t sub_batch_dev_bytes(const SubBatch* b) {
  size_t o = 0;
  for (size_t q = 0; q < b->Ls.size(); ++q) {
    o = align256(o) + b->args[q].size() * sizeof(SubArgs);
    o = align256(o) + b->tabs[q].size() * sizeof(BatchTab);
  }
  o = align256(o) + b->chi.size() * sizeof(Chi2Item);
  return align256(o);
}

hipError_t sub_batch_upload(SubBatch* b, unsigned char* dev) {
  std::vector<unsigned char> blob(sub_batch_dev_bytes(b));
  size_t o = 0;
  auto put = [&](const void* src, size_t bytes) {
    o = align256(o);
    std::memcpy(blob.data() + o, src, bytes);
    unsigned char* p = dev + o;
    o += bytes;
    return p;
  };
  b->dargs.clear();
  b->dtabs.clear();
  for (size_t q = 0; q < b->Ls.size(); ++q) {
    b->dargs.push_back(reinterpret_cast<SubArgs*>(put(b->args[q].data(), b->args[q].size() * sizeof(SubArgs))));
    b->dtabs.push_back(reinterpret_cast<BatchTab*>(put(b->tabs[q].data(), b->tabs[q].size() * sizeof(BatchTab))));
  }
  b->dchi = reinterpret_cast<Chi2Item*>(put(b->chi.data(), b->chi.size() * sizeof(Chi2Item)));
  return hipMemcpy(dev, blob.data(), blob.size(), hipMemcpyHostToDevice);
}

template <int L, int TY>
static void sub_batch_lt(const SubBatch* b, int q, hipStream_t st) {
  const int n = (int)b->args[q].size();
  const dim3 grid(b->blocks[q]), block(kSubTX * TY / 8);
  const SubArgs* args = b->dargs[q];
  const BatchTab* tab = b->dtabs[q];
  if (b->DK == 0) hipLaunchKernelGGL((k_subtract_batch<L, 0, TY>), grid, block, 0, st, args, tab, n);
  else if (b->DK == 1) hipLaunchKernelGGL((k_subtract_batch<L, 1, TY>), grid, block, 0, st, args, tab, n);
  else hipLaunchKernelGGL((k_subtract_batch<L, 2, TY>), grid, block, 0, st, args, tab, n);
}

template <int L>
static void sub_batch_l(const SubBatch* b, int q, hipStream_t st) {
  if (b->tile_rows == 16) sub_batch_lt<L, 16>(b, q, st);
  else if (b->tile_rows == 64) sub_batch_lt<L, 64>(b, q, st);
  else sub_batch_lt<L, 32>(b, q, st);
}

hipError_t sub_batch_launch(const SubBatch* b, const Prof* pf, hipStream_t st) {
  prof_begin(pf, SFFT_PROF_SUBTRACT, st);
  for (size_t q = 0; q < b->Ls.size(); ++q)
    hipLaunchKernelGGL(k_kappa2_batch, dim3((unsigned)b->args[q].size()), dim3(kK2Threads), 0, st,
                       (const SubArgs*)b->dargs[q]);
  for (size_t q = 0; q < b->Ls.size(); ++q) {
    switch (b->Ls[q]) {
      case 1: sub_batch_l<1>(b, (int)q, st); break;
      case 3: sub_batch_l<3>(b, (int)q, st); break;
      case 5: sub_batch_l<5>(b, (int)q, st); break;
      case 7: sub_batch_l<7>(b, (int)q, st); break;
      case 9: sub_batch_l<9>(b, (int)q, st); break;
      case 11: sub_batch_l<11>(b, (int)q, st); break;
      case 13: sub_batch_l<13>(b, (int)q, st); break;
      case 15: sub_batch_l<15>(b, (int)q, st); break;
      default: return hipErrorInvalidValue;
    }
  }
  prof_end(pf, SFFT_PROF_SUBTRACT, st);
  hipLaunchKernelGGL(k_chi2_final_batch, dim3(b->n), dim3(1024), 0, st, (const Chi2Item*)b->dchi);
  return hipGetLastError();
}

void sub_batch_destroy(SubBatch* b) { delete b; }

}  // namespace sfft
