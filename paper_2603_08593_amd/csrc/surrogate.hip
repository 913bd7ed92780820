// Learned form of the fit: a small convolutional network predicts the kernel
// and background coefficients from star-stamp pairs (the paper's pipeline
// pairs the image differencing with learned models, Sec. 2.3; this network
// and its training are this library's own). Hand-written kernels for the
// stamp extraction, the forward pass (FP32 or bfloat16 storage with FP32
// accumulation), the backward pass, the mean-squared loss and Adam.
//
// Data layout: stamps [n][2][32][32] FP32 (reference, science), positions
// [n][2] (xt, yt) of the stamp centres, n = n_pairs * n_stamps with the
// stamps of one pair contiguous; activations NCHW; linear weights [out][in].
// Every reduction runs in a fixed order: results are bit-reproducible.
#include <cmath>

#include "common.hpp"
#include "layout.hpp"
#include "surrogate.hpp"

namespace sfft {

struct bf16s {
  unsigned short v;
};

__device__ __forceinline__ unsigned short rne16(float x) {
  const unsigned u = __builtin_bit_cast(unsigned, x);
  return (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float ldv(const float* p, int64_t i) { return p[i]; }
__device__ __forceinline__ float ldv(const bf16s* p, int64_t i) {
  return __builtin_bit_cast(float, (unsigned)p[i].v << 16);
}
__device__ __forceinline__ void stv(float* p, int64_t i, float x) { p[i] = x; }
__device__ __forceinline__ void stv(bf16s* p, int64_t i, float x) { p[i].v = rne16(x); }

// ---------------------------------------------------------------------------
// stamp extraction: window [cx - 16, cx + 16) x [cy - 16, cy + 16) (periodic),
// minus the mean of the window's border, divided by the reference window's
// sky-subtracted sum (1 if not positive), times `scale`
// ---------------------------------------------------------------------------
template <typename TIN>
__global__ __launch_bounds__(256) void k_extract_stamps(const void* R, const void* S, int64_t ld, int W,
                                                        int H, const int32_t* centers, float* out,
                                                        float* pos, float scale, double sx, double sy) {
  __shared__ double red[8];
  const int n = blockIdx.x, tid = threadIdx.x;
  const int cx = centers[2 * n], cy = centers[2 * n + 1];
  constexpr int Z = kNetStamp;
  double r[4], s[4];
  double br = 0.0, bs = 0.0;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int p = tid + 256 * e, yy = p / Z, xx = p % Z;
    int Y = (cy - Z / 2 + yy) % H, X = (cx - Z / 2 + xx) % W;
    Y = Y < 0 ? Y + H : Y;
    X = X < 0 ? X + W : X;
    r[e] = (double)static_cast<const TIN*>(R)[(int64_t)Y * ld + X];
    s[e] = (double)static_cast<const TIN*>(S)[(int64_t)Y * ld + X];
    const bool border = yy == 0 || yy == Z - 1 || xx == 0 || xx == Z - 1;
    if (border) { br += r[e]; bs += s[e]; }
  }
  const double nb = 4.0 * (Z - 1);
  const double skyr = block_sum(br, red) / nb;
  const double skys = block_sum(bs, red) / nb;
  double fr = 0.0;
#pragma unroll
  for (int e = 0; e < 4; ++e) fr += r[e] - skyr;
  double f = block_sum(fr, red);
  f = f > 0.0 ? f : 1.0;
  const double k = (double)scale / f;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int p = tid + 256 * e;
    out[(int64_t)n * 2 * Z * Z + p] = (float)((r[e] - skyr) * k);
    out[(int64_t)n * 2 * Z * Z + Z * Z + p] = (float)((s[e] - skys) * k);
  }
  if (tid == 0) {
    pos[2 * n] = (float)((double)cx * sx - 1.0);
    pos[2 * n + 1] = (float)((double)cy * sy - 1.0);
  }
}

// ---------------------------------------------------------------------------
// convolution 3x3, zero padding 1, stride ST, bias, ReLU: one workgroup per
// (stamp, block of COB output channels); the padded input stack and the
// block's weights are staged in LDS; a thread computes 8 channels of a pixel
// ---------------------------------------------------------------------------
template <int CI, int CO, int HI, int ST, int COB, typename T>
__global__ __launch_bounds__(256) void k_conv_fwd(const T* in, const T* w, const T* bias, T* out) {
  constexpr int HO = (HI - 1) / ST + 1, HP = HI + 2;
  extern __shared__ float sm[];
  float* xin = sm;
  float* wsm = sm + CI * HP * HP;
  const int n = blockIdx.x, cb = blockIdx.y, tid = threadIdx.x;
  for (int idx = tid; idx < CI * HP * HP; idx += 256) {
    const int ci = idx / (HP * HP), rem = idx - ci * HP * HP;
    const int y = rem / HP - 1, x = rem % HP - 1;
    xin[idx] = (y >= 0 && y < HI && x >= 0 && x < HI)
                   ? ldv(in, ((int64_t)n * CI + ci) * HI * HI + y * HI + x) : 0.0f;
  }
  for (int idx = tid; idx < COB * CI * 9; idx += 256) wsm[idx] = ldv(w, (int64_t)cb * COB * CI * 9 + idx);
  __syncthreads();
  constexpr int NG = COB / 8;
  for (int it = tid; it < NG * HO * HO; it += 256) {
    const int g = it / (HO * HO), p = it - g * HO * HO, oy = p / HO, ox = p % HO;
    float acc[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) acc[c] = ldv(bias, cb * COB + g * 8 + c);
    for (int ci = 0; ci < CI; ++ci) {
      const float* xp = xin + ci * HP * HP + (ST * oy) * HP + ST * ox;
      float v[9];
#pragma unroll
      for (int ky = 0; ky < 3; ++ky)
#pragma unroll
        for (int kx = 0; kx < 3; ++kx) v[ky * 3 + kx] = xp[ky * HP + kx];
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const float* wc = wsm + ((g * 8 + c) * CI + ci) * 9;
#pragma unroll
        for (int t = 0; t < 9; ++t) acc[c] = fmaf(wc[t], v[t], acc[c]);
      }
    }
#pragma unroll
    for (int c = 0; c < 8; ++c)
      stv(out, ((int64_t)n * CO + cb * COB + g * 8 + c) * HO * HO + p, fmaxf(acc[c], 0.0f));
  }
}

// gradient with respect to the input of a convolution: gin = conv^T(gout * (aout > 0));
// one workgroup per (stamp, block of CIB input channels)
template <int CI, int CO, int HI, int ST, int CIB>
__global__ __launch_bounds__(256) void k_conv_bwd_data(const float* gout, const float* aout, const float* w,
                                                       float* gin) {
  constexpr int HO = (HI - 1) / ST + 1;
  extern __shared__ float sm[];
  float* gz = sm;                    // [CO][HO][HO]
  float* wsm = sm + CO * HO * HO;    // [CO][CIB][9]
  const int n = blockIdx.x, cb = blockIdx.y, tid = threadIdx.x;
  for (int idx = tid; idx < CO * HO * HO; idx += 256) {
    const int64_t gi = (int64_t)n * CO * HO * HO + idx;
    gz[idx] = aout[gi] > 0.0f ? gout[gi] : 0.0f;
  }
  for (int idx = tid; idx < CO * CIB * 9; idx += 256) {
    const int co = idx / (CIB * 9), rem = idx - co * CIB * 9;
    wsm[idx] = w[((int64_t)co * CI + cb * CIB) * 9 + rem];
  }
  __syncthreads();
  constexpr int NG = CIB / 8;
  for (int it = tid; it < NG * HI * HI; it += 256) {
    const int g = it / (HI * HI), p = it - g * HI * HI, y = p / HI, x = p % HI;
    float acc[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) acc[c] = 0.0f;
#pragma unroll
    for (int ky = 0; ky < 3; ++ky) {
      const int ty = y + 1 - ky;
      if (ty < 0 || ty % ST != 0 || ty / ST >= HO) continue;
#pragma unroll
      for (int kx = 0; kx < 3; ++kx) {
        const int tx = x + 1 - kx;
        if (tx < 0 || tx % ST != 0 || tx / ST >= HO) continue;
        const int o = (ty / ST) * HO + tx / ST;
        for (int co = 0; co < CO; ++co) {
          const float v = gz[co * HO * HO + o];
          const float* wc = wsm + (co * CIB + g * 8) * 9 + ky * 3 + kx;
#pragma unroll
          for (int c = 0; c < 8; ++c) acc[c] = fmaf(wc[c * 9], v, acc[c]);
        }
      }
    }
#pragma unroll
    for (int c = 0; c < 8; ++c) gin[((int64_t)n * CI + cb * CIB + g * 8 + c) * HI * HI + p] = acc[c];
  }
}

// weight and bias gradients of a convolution, partial over a chunk of
// kNetChunk stamps: part_w[chunk][co][ci][9], part_b[chunk][co]; one
// workgroup per (chunk, block of 8 output channels). Thread t owns the
// (ci, tap) pairs t, t + 256, ... and, when there are fewer than 256 pairs,
// one slice of the pixels; slices are added in a fixed order.
template <int CI, int CO, int HI, int ST>
__global__ __launch_bounds__(256) void k_conv_bwd_w(const float* ain, const float* gout, const float* aout,
                                                    float* part_w, float* part_b, int ns) {
  constexpr int HO = (HI - 1) / ST + 1, HP = HI + 2;
  constexpr int NPAIR = CI * 9;
  constexpr int NPP = NPAIR < 256 ? NPAIR : 256;       // pair lanes
  constexpr int NSL = 256 / NPP;                        // pixel slices
  constexpr int PPT = (NPAIR + 255) / 256;              // pairs per thread
  extern __shared__ float sm[];
  float* xin = sm;                         // [CI][HP][HP]
  float* gz = sm + CI * HP * HP;           // [8][HO][HO]
  float* red = gz + 8 * HO * HO;           // [NSL][NPP][8]
  const int kc = blockIdx.x, cb = blockIdx.y, tid = threadIdx.x;
  const int lane_pair = tid % NPP, slice = tid / NPP;
  const bool active = slice < NSL;
  float acc[PPT][8];
#pragma unroll
  for (int q = 0; q < PPT; ++q)
#pragma unroll
    for (int c = 0; c < 8; ++c) acc[q][c] = 0.0f;
  float bacc = 0.0f;
  const int n0 = kc * kNetChunk, n1 = min(ns, n0 + kNetChunk);
  for (int n = n0; n < n1; ++n) {
    for (int idx = tid; idx < CI * HP * HP; idx += 256) {
      const int ci = idx / (HP * HP), rem = idx - ci * HP * HP;
      const int y = rem / HP - 1, x = rem % HP - 1;
      xin[idx] = (y >= 0 && y < HI && x >= 0 && x < HI) ? ain[((int64_t)n * CI + ci) * HI * HI + y * HI + x] : 0.0f;
    }
    for (int idx = tid; idx < 8 * HO * HO; idx += 256) {
      const int64_t gi = ((int64_t)n * CO + cb * 8) * HO * HO + idx;
      gz[idx] = aout[gi] > 0.0f ? gout[gi] : 0.0f;
    }
    __syncthreads();
    if (active) {
#pragma unroll
      for (int q = 0; q < PPT; ++q) {
        const int pr = lane_pair + 256 * q;
        if (pr < NPAIR) {
          const int ci = pr / 9, t = pr % 9, ky = t / 3, kx = t % 3;
          const float* xp = xin + ci * HP * HP + ky * HP + kx;
          for (int p = slice; p < HO * HO; p += NSL) {
            const int oy = p / HO, ox = p % HO;
            const float v = xp[(ST * oy) * HP + ST * ox];
#pragma unroll
            for (int c = 0; c < 8; ++c) acc[q][c] = fmaf(v, gz[c * HO * HO + p], acc[q][c]);
          }
        }
      }
    }
    if (tid < 8) {
      float sb = 0.0f;
      for (int p = 0; p < HO * HO; ++p) sb += gz[tid * HO * HO + p];
      bacc += sb;
    }
    __syncthreads();
  }
  // fixed-order sum over the pixel slices
  if (NSL > 1) {
    if (active)
#pragma unroll
      for (int c = 0; c < 8; ++c) red[(slice * NPP + lane_pair) * 8 + c] = acc[0][c];
    __syncthreads();
    if (tid < NPP) {
      for (int c = 0; c < 8; ++c) {
        float s = 0.0f;
        for (int sl = 0; sl < NSL; ++sl) s += red[(sl * NPP + tid) * 8 + c];
        acc[0][c] = s;
      }
    }
  }
  if (slice == 0) {
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
      const int pr = lane_pair + 256 * q;
      if (pr < NPAIR)
#pragma unroll
        for (int c = 0; c < 8; ++c)
          part_w[((int64_t)kc * CO + cb * 8 + c) * NPAIR + pr] = acc[q][c];
    }
  }
  if (tid < 8) part_b[(int64_t)kc * CO + cb * 8 + tid] = bacc;
}

// out[i] = sum over chunks (fixed order) of part[chunk * n + i]
__global__ void k_sum_chunks(const float* part, int nchunk, int n, float* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float s = 0.0f;
  for (int k = 0; k < nchunk; ++k) s += part[(int64_t)k * n + i];
  out[i] = s;
}

// ---------------------------------------------------------------------------
// C[i][j] = epi(sum_k A(i,k) B(k,j) + bias[j]); A(i,k) = TA ? A[k][i] : A[i][k],
// B(k,j) = TB ? B[j][k] : B[k][j]; epi: optional ReLU, optional mask
// (zero where mask <= 0). 64 x 64 tiles, k in chunks of 16, 4 x 4 per thread.
// ---------------------------------------------------------------------------
template <bool TA, bool TB, typename T, typename TO>
__global__ __launch_bounds__(256) void k_gemm(const T* A, const T* B, TO* C, int M, int N, int K, int lda,
                                              int ldb, int ldc, const T* bias, int relu,
                                              const float* mask) {
  __shared__ float As[16][65];
  __shared__ float Bs[16][65];
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
  float acc[4][4] = {};
  for (int k0 = 0; k0 < K; k0 += 16) {
    for (int idx = tid; idx < 16 * 64; idx += 256) {
      const int kk = idx / 64, ii = idx % 64;
      const int i = i0 + ii, k = k0 + kk;
      float av = 0.0f;
      if (i < M && k < K) av = TA ? ldv(A, (int64_t)k * lda + i) : ldv(A, (int64_t)i * lda + k);
      As[kk][ii] = av;
      const int j = j0 + ii;
      float bv = 0.0f;
      if (j < N && k < K) bv = TB ? ldv(B, (int64_t)j * ldb + k) : ldv(B, (int64_t)k * ldb + j);
      Bs[kk][ii] = bv;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      float a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) { a[u] = As[kk][ty + 16 * u]; b[u] = Bs[kk][tx + 16 * u]; }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = fmaf(a[u], b[v], acc[u][v]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int i = i0 + ty + 16 * u;
    if (i >= M) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int j = j0 + tx + 16 * v;
      if (j >= N) continue;
      float c = acc[u][v] + (bias ? ldv(bias, j) : 0.0f);
      if (relu) c = fmaxf(c, 0.0f);
      if (mask && !(mask[(int64_t)i * ldc + j] > 0.0f)) c = 0.0f;
      stv(C, (int64_t)i * ldc + j, c);
    }
  }
}

// column sums (bias gradients), one thread per column, rows in order
__global__ void k_colsum(const float* G, int M, int N, float* out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  float s = 0.0f;
  for (int i = 0; i < M; ++i) s += G[(int64_t)i * N + j];
  out[j] = s;
}

__device__ __forceinline__ void mono6(float x, float y, float* m) {
  m[0] = 1.0f; m[1] = x; m[2] = y; m[3] = x * x; m[4] = x * y; m[5] = y * y;
}

// u[b][i*128 + c] = (1/S) sum_s p_i(pos_s) h[b*S + s][c]
template <typename T>
__global__ __launch_bounds__(256) void k_pool_fwd(const T* h, const float* pos, T* u, int S) {
  const int b = blockIdx.x;
  for (int o = threadIdx.x; o < kNetU; o += 256) {
    const int i = o / kNetH, c = o % kNetH;
    float s = 0.0f;
#pragma unroll 8
    for (int t = 0; t < S; ++t) {
      const int n = b * S + t;
      float m[6];
      mono6(pos[2 * n], pos[2 * n + 1], m);
      s = fmaf(m[i], ldv(h, (int64_t)n * kNetH + c), s);
    }
    stv(u, (int64_t)b * kNetU + o, s / (float)S);
  }
}

// gh[n][c] = (h > 0) (1/S) sum_i p_i(pos_n) gu[b][i*128 + c]
__global__ __launch_bounds__(128) void k_pool_bwd(const float* gu, const float* pos, const float* h, float* gh,
                                                  int S) {
  const int n = blockIdx.x, b = n / S, c = threadIdx.x;
  float m[6];
  mono6(pos[2 * n], pos[2 * n + 1], m);
  float s = 0.0f;
#pragma unroll
  for (int i = 0; i < kNetMono; ++i) s = fmaf(m[i], gu[(int64_t)b * kNetU + i * kNetH + c], s);
  gh[(int64_t)n * kNetH + c] = h[(int64_t)n * kNetH + c] > 0.0f ? s / (float)S : 0.0f;
}

// loss = mean (pred - t)^2 (FP64 sum, fixed order), gpred = 2 (pred - t) / count
__global__ __launch_bounds__(1024) void k_mse(const float* pred, const float* target, int count, float* gpred,
                                              double* loss) {
  __shared__ double red[16];
  double s = 0.0;
  for (int i = threadIdx.x; i < count; i += 1024) {
    const float d = pred[i] - target[i];
    s += (double)d * d;
    gpred[i] = 2.0f * d / (float)count;
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) *loss = s / count;
}

__global__ void k_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

__global__ void k_to_bf16(const float* x, bf16s* y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i].v = rne16(x[i]);
}

__global__ void k_destandardize(const float* pred, const double* mean, const double* scale, int n_pairs,
                                int n_out, double* coef) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)n_pairs * n_out) return;
  const int j = (int)(i % n_out);
  coef[i] = mean[j] + scale[j] * (double)pred[i];
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

template <int CI, int CO, int HI, int ST, int COB>
constexpr size_t conv_fwd_lds() { return sizeof(float) * (CI * (HI + 2) * (HI + 2) + COB * CI * 9); }
template <int CI, int CO, int HI, int ST, int CIB>
constexpr size_t conv_bwd_data_lds() {
  return sizeof(float) * (CO * ((HI - 1) / ST + 1) * ((HI - 1) / ST + 1) + CO * CIB * 9);
}
template <int CI, int CO, int HI, int ST>
constexpr size_t conv_bwd_w_lds() {
  constexpr int HO = (HI - 1) / ST + 1;
  constexpr int NPP = CI * 9 < 256 ? CI * 9 : 256;
  return sizeof(float) * (CI * (HI + 2) * (HI + 2) + 8 * HO * HO + (256 / NPP) * NPP * 8);
}

#define SFFT_CONV_CFG1 2, 16, 32, 1
#define SFFT_CONV_CFG2 16, 32, 32, 2
#define SFFT_CONV_CFG3 32, 64, 16, 2
#define SFFT_CONV_CFG4 64, 64, 8, 2

template <typename T>
static hipError_t set_fwd_attrs() {
  hipError_t e;
#define SFFT_SET(K, L)                                                                              \
  if ((e = hipFuncSetAttribute(reinterpret_cast<const void*>(&K), hipFuncAttributeMaxDynamicSharedMemorySize, \
                               (int)(L))) != hipSuccess)                                            \
    return e;
  SFFT_SET((k_conv_fwd<SFFT_CONV_CFG1, 16, T>), (conv_fwd_lds<SFFT_CONV_CFG1, 16>()));
  SFFT_SET((k_conv_fwd<SFFT_CONV_CFG2, 32, T>), (conv_fwd_lds<SFFT_CONV_CFG2, 32>()));
  SFFT_SET((k_conv_fwd<SFFT_CONV_CFG3, 64, T>), (conv_fwd_lds<SFFT_CONV_CFG3, 64>()));
  SFFT_SET((k_conv_fwd<SFFT_CONV_CFG4, 32, T>), (conv_fwd_lds<SFFT_CONV_CFG4, 32>()));
  // narrow batches (inference on a few pairs): more workgroups per layer
  SFFT_SET((k_conv_fwd<SFFT_CONV_CFG1, 8, T>), (conv_fwd_lds<SFFT_CONV_CFG1, 8>()));
  SFFT_SET((k_conv_fwd<SFFT_CONV_CFG2, 8, T>), (conv_fwd_lds<SFFT_CONV_CFG2, 8>()));
  SFFT_SET((k_conv_fwd<SFFT_CONV_CFG3, 32, T>), (conv_fwd_lds<SFFT_CONV_CFG3, 32>()));
  SFFT_SET((k_conv_fwd<SFFT_CONV_CFG4, 16, T>), (conv_fwd_lds<SFFT_CONV_CFG4, 16>()));
  return hipSuccess;
}

hipError_t prepare_surrogate_attributes() {
  hipError_t e;
  if ((e = set_fwd_attrs<float>()) != hipSuccess) return e;
  if ((e = set_fwd_attrs<bf16s>()) != hipSuccess) return e;
  SFFT_SET((k_conv_bwd_data<SFFT_CONV_CFG2, 16>), (conv_bwd_data_lds<SFFT_CONV_CFG2, 16>()));
  SFFT_SET((k_conv_bwd_data<SFFT_CONV_CFG3, 32>), (conv_bwd_data_lds<SFFT_CONV_CFG3, 32>()));
  SFFT_SET((k_conv_bwd_data<SFFT_CONV_CFG4, 32>), (conv_bwd_data_lds<SFFT_CONV_CFG4, 32>()));
  SFFT_SET((k_conv_bwd_w<SFFT_CONV_CFG1>), (conv_bwd_w_lds<SFFT_CONV_CFG1>()));
  SFFT_SET((k_conv_bwd_w<SFFT_CONV_CFG2>), (conv_bwd_w_lds<SFFT_CONV_CFG2>()));
  SFFT_SET((k_conv_bwd_w<SFFT_CONV_CFG3>), (conv_bwd_w_lds<SFFT_CONV_CFG3>()));
  SFFT_SET((k_conv_bwd_w<SFFT_CONV_CFG4>), (conv_bwd_w_lds<SFFT_CONV_CFG4>()));
#undef SFFT_SET
  return hipSuccess;
}

// C = A B^T (+ bias, ReLU) for few rows of A (inference): one wave per
// output element, lanes over k (coalesced rows of A and of B), FP32
// accumulation, butterfly sum over the wave
template <typename T, typename TO>
__global__ __launch_bounds__(256) void k_gemm_rows(const T* A, const T* B, TO* C, int M, int N, int K, int lda,
                                                   int ldb, int ldc, const T* bias, int relu) {
  const int64_t wv = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (wv >= (int64_t)M * N) return;            // whole waves only
  const int i = (int)(wv / N), j = (int)(wv % N);
  float acc = 0.0f;
#pragma unroll 4
  for (int k = lane; k < K; k += 64) acc = fmaf(ldv(A, (int64_t)i * lda + k), ldv(B, (int64_t)j * ldb + k), acc);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if (lane == 0) {
    float c = acc + (bias ? ldv(bias, j) : 0.0f);
    if (relu) c = fmaxf(c, 0.0f);
    stv(C, (int64_t)i * ldc + j, c);
  }
}

template <bool TA, bool TB, typename T, typename TO>
static void gemm(const T* A, const T* B, TO* C, int M, int N, int K, int lda, int ldb, int ldc, const T* bias,
                 int relu, const float* mask, hipStream_t st) {
  if (!TA && TB && !mask && M <= 1024) {
    const int64_t waves = (int64_t)M * N;
    hipLaunchKernelGGL((k_gemm_rows<T, TO>), dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, st, A, B, C, M, N,
                       K, lda, ldb, ldc, bias, relu);
    return;
  }
  const dim3 grid((N + 63) / 64, (M + 63) / 64);
  hipLaunchKernelGGL((k_gemm<TA, TB, T, TO>), grid, dim3(256), 0, st, A, B, C, M, N, K, lda, ldb, ldc, bias,
                     relu, mask);
}

hipError_t launch_extract_stamps(const sfft_desc& d, const void* R, const void* S, const int32_t* centers,
                                 int n, float* stamps, float* pos, hipStream_t st) {
  const double sx = d.width > 1 ? 2.0 / (double)(d.width - 1) : 0.0;
  const double sy = d.height > 1 ? 2.0 / (double)(d.height - 1) : 0.0;
  if (d.image_dtype == SFFT_F32)
    hipLaunchKernelGGL(k_extract_stamps<float>, dim3(n), dim3(256), 0, st, R, S, d.ld, d.width, d.height,
                       centers, stamps, pos, 100.0f, sx, sy);
  else
    hipLaunchKernelGGL(k_extract_stamps<double>, dim3(n), dim3(256), 0, st, R, S, d.ld, d.width, d.height,
                       centers, stamps, pos, 100.0f, sx, sy);
  return hipGetLastError();
}

// forward pass with storage type T; x: stamps as T; params as T; pred FP32
template <typename T>
static void forward_t(const T* P, const T* x, const float* pos, int n_pairs, int n_stamps, int n_out,
                      const NetWs& w, unsigned char* ws, float* pred, hipStream_t st) {
  const NetLayout L = net_layout(n_out);
  const int ns = n_pairs * n_stamps;
  T* a1 = reinterpret_cast<T*>(ws + w.a[1]);
  T* a2 = reinterpret_cast<T*>(ws + w.a[2]);
  T* a3 = reinterpret_cast<T*>(ws + w.a[3]);
  T* a4 = reinterpret_cast<T*>(ws + w.a[4]);
  T* h = reinterpret_cast<T*>(ws + w.h);
  T* u = reinterpret_cast<T*>(ws + w.u);
  T* g = reinterpret_cast<T*>(ws + w.g);
  if (ns < 1024) {
    // few stamps (inference on one or a few pairs): split the output channels
    // over more workgroups so that the layers fill the GPU (same arithmetic)
    hipLaunchKernelGGL((k_conv_fwd<SFFT_CONV_CFG1, 8, T>), dim3(ns, 2), dim3(256),
                       (conv_fwd_lds<SFFT_CONV_CFG1, 8>()), st, x, P + L.cw[0], P + L.cb[0], a1);
    hipLaunchKernelGGL((k_conv_fwd<SFFT_CONV_CFG2, 8, T>), dim3(ns, 4), dim3(256),
                       (conv_fwd_lds<SFFT_CONV_CFG2, 8>()), st, a1, P + L.cw[1], P + L.cb[1], a2);
    hipLaunchKernelGGL((k_conv_fwd<SFFT_CONV_CFG3, 32, T>), dim3(ns, 2), dim3(256),
                       (conv_fwd_lds<SFFT_CONV_CFG3, 32>()), st, a2, P + L.cw[2], P + L.cb[2], a3);
    hipLaunchKernelGGL((k_conv_fwd<SFFT_CONV_CFG4, 16, T>), dim3(ns, 4), dim3(256),
                       (conv_fwd_lds<SFFT_CONV_CFG4, 16>()), st, a3, P + L.cw[3], P + L.cb[3], a4);
  } else {
    hipLaunchKernelGGL((k_conv_fwd<SFFT_CONV_CFG1, 16, T>), dim3(ns, 1), dim3(256),
                       (conv_fwd_lds<SFFT_CONV_CFG1, 16>()), st, x, P + L.cw[0], P + L.cb[0], a1);
    hipLaunchKernelGGL((k_conv_fwd<SFFT_CONV_CFG2, 32, T>), dim3(ns, 1), dim3(256),
                       (conv_fwd_lds<SFFT_CONV_CFG2, 32>()), st, a1, P + L.cw[1], P + L.cb[1], a2);
    hipLaunchKernelGGL((k_conv_fwd<SFFT_CONV_CFG3, 64, T>), dim3(ns, 1), dim3(256),
                       (conv_fwd_lds<SFFT_CONV_CFG3, 64>()), st, a2, P + L.cw[2], P + L.cb[2], a3);
    hipLaunchKernelGGL((k_conv_fwd<SFFT_CONV_CFG4, 32, T>), dim3(ns, 2), dim3(256),
                       (conv_fwd_lds<SFFT_CONV_CFG4, 32>()), st, a3, P + L.cw[3], P + L.cb[3], a4);
  }
  gemm<false, true, T, T>(a4, P + L.fc1w, h, ns, kNetH, kNetF, kNetF, kNetF, kNetH, P + L.fc1b, 1, nullptr, st);
  hipLaunchKernelGGL((k_pool_fwd<T>), dim3(n_pairs), dim3(256), 0, st, h, pos, u, n_stamps);
  gemm<false, true, T, T>(u, P + L.fc2w, g, n_pairs, kNetG, kNetU, kNetU, kNetU, kNetG, P + L.fc2b, 1, nullptr,
                          st);
  gemm<false, true, T, float>(g, P + L.fc3w, pred, n_pairs, n_out, kNetG, kNetG, kNetG, n_out, P + L.fc3b, 0,
                              nullptr, st);
}

hipError_t launch_surrogate_forward(const float* params, const float* stamps, const float* pos, int n_pairs,
                                    int n_stamps, int n_out, bool bf16, float* pred, unsigned char* ws,
                                    hipStream_t st) {
  const NetWs w = net_ws(n_pairs, n_stamps, n_out);
  if (!bf16) {
    forward_t<float>(params, stamps, pos, n_pairs, n_stamps, n_out, w, ws, pred, st);
  } else {
    const NetLayout L = net_layout(n_out);
    bf16s* pb = reinterpret_cast<bf16s*>(ws + w.pbf);
    bf16s* xb = reinterpret_cast<bf16s*>(ws + w.xbf);
    const int64_t nx = (int64_t)n_pairs * n_stamps * 2 * kNetStamp * kNetStamp;
    hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)((L.total + 255) / 256)), dim3(256), 0, st, params, pb, L.total);
    hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)((nx + 255) / 256)), dim3(256), 0, st, stamps, xb, nx);
    forward_t<bf16s>(pb, xb, pos, n_pairs, n_stamps, n_out, w, ws, pred, st);
  }
  return hipGetLastError();
}

template <int CI, int CO, int HI, int ST>
static void conv_wgrad(const float* ain, const float* gout, const float* aout, float* grad_w, float* grad_b,
                       int ns, const NetWs& w, unsigned char* ws, hipStream_t st) {
  float* part = reinterpret_cast<float*>(ws + w.part);
  float* part_b = part + (size_t)w.nchunk * CO * CI * 9;
  hipLaunchKernelGGL((k_conv_bwd_w<CI, CO, HI, ST>), dim3(w.nchunk, CO / 8), dim3(256),
                     (conv_bwd_w_lds<CI, CO, HI, ST>()), st, ain, gout, aout, part, part_b, ns);
  const int nw = CO * CI * 9;
  hipLaunchKernelGGL(k_sum_chunks, dim3((nw + 255) / 256), dim3(256), 0, st, (const float*)part, w.nchunk, nw,
                     grad_w);
  hipLaunchKernelGGL(k_sum_chunks, dim3(1), dim3(256), 0, st, (const float*)part_b, w.nchunk, CO, grad_b);
}

// forward (FP32) + mean-squared loss + backward: grads (flat, parameter layout), loss (device double)
hipError_t launch_surrogate_grad(const float* P, const float* x, const float* pos, const float* target,
                                 int n_pairs, int n_stamps, int n_out, float* grads, double* loss,
                                 unsigned char* ws, hipStream_t st) {
  const NetWs w = net_ws(n_pairs, n_stamps, n_out);
  const NetLayout L = net_layout(n_out);
  const int ns = n_pairs * n_stamps;
  float* pred = reinterpret_cast<float*>(ws + w.pred);
  forward_t<float>(P, x, pos, n_pairs, n_stamps, n_out, w, ws, pred, st);
  float* a[5];
  float* ga[5];
  for (int k = 1; k <= 4; ++k) {
    a[k] = reinterpret_cast<float*>(ws + w.a[k]);
    ga[k] = reinterpret_cast<float*>(ws + w.ga[k]);
  }
  float* h = reinterpret_cast<float*>(ws + w.h);
  float* gh = reinterpret_cast<float*>(ws + w.gh);
  float* u = reinterpret_cast<float*>(ws + w.u);
  float* gu = reinterpret_cast<float*>(ws + w.gu);
  float* g = reinterpret_cast<float*>(ws + w.g);
  float* gg = reinterpret_cast<float*>(ws + w.gg);
  float* gpred = reinterpret_cast<float*>(ws + w.gpred);
  const int count = n_pairs * n_out;
  hipLaunchKernelGGL(k_mse, dim3(1), dim3(1024), 0, st, (const float*)pred, target, count, gpred, loss);
  // fc3
  gemm<true, false, float, float>(gpred, g, grads + L.fc3w, n_out, kNetG, n_pairs, n_out, kNetG, kNetG, nullptr,
                                  0, nullptr, st);
  hipLaunchKernelGGL(k_colsum, dim3((n_out + 255) / 256), dim3(256), 0, st, (const float*)gpred, n_pairs, n_out,
                     grads + L.fc3b);
  gemm<false, false, float, float>(gpred, P + L.fc3w, gg, n_pairs, kNetG, n_out, n_out, kNetG, kNetG, nullptr, 0,
                                   g, st);
  // fc2
  gemm<true, false, float, float>(gg, u, grads + L.fc2w, kNetG, kNetU, n_pairs, kNetG, kNetU, kNetU, nullptr, 0,
                                  nullptr, st);
  hipLaunchKernelGGL(k_colsum, dim3((kNetG + 255) / 256), dim3(256), 0, st, (const float*)gg, n_pairs, kNetG,
                     grads + L.fc2b);
  gemm<false, false, float, float>(gg, P + L.fc2w, gu, n_pairs, kNetU, kNetG, kNetG, kNetU, kNetU, nullptr, 0,
                                   nullptr, st);
  // pooling, fc1
  hipLaunchKernelGGL(k_pool_bwd, dim3(ns), dim3(kNetH), 0, st, (const float*)gu, pos, (const float*)h, gh,
                     n_stamps);
  gemm<true, false, float, float>(gh, a[4], grads + L.fc1w, kNetH, kNetF, ns, kNetH, kNetF, kNetF, nullptr, 0,
                                  nullptr, st);
  hipLaunchKernelGGL(k_colsum, dim3(1), dim3(kNetH), 0, st, (const float*)gh, ns, kNetH, grads + L.fc1b);
  gemm<false, false, float, float>(gh, P + L.fc1w, ga[4], ns, kNetF, kNetH, kNetH, kNetF, kNetF, nullptr, 0,
                                   nullptr, st);
  // conv4 .. conv1: weight gradients from (input, grad of output, output); data gradients below
  conv_wgrad<SFFT_CONV_CFG4>(a[3], ga[4], a[4], grads + L.cw[3], grads + L.cb[3], ns, w, ws, st);
  hipLaunchKernelGGL((k_conv_bwd_data<SFFT_CONV_CFG4, 32>), dim3(ns, 2), dim3(256),
                     (conv_bwd_data_lds<SFFT_CONV_CFG4, 32>()), st, (const float*)ga[4], (const float*)a[4],
                     P + L.cw[3], ga[3]);
  conv_wgrad<SFFT_CONV_CFG3>(a[2], ga[3], a[3], grads + L.cw[2], grads + L.cb[2], ns, w, ws, st);
  hipLaunchKernelGGL((k_conv_bwd_data<SFFT_CONV_CFG3, 32>), dim3(ns, 1), dim3(256),
                     (conv_bwd_data_lds<SFFT_CONV_CFG3, 32>()), st, (const float*)ga[3], (const float*)a[3],
                     P + L.cw[2], ga[2]);
  conv_wgrad<SFFT_CONV_CFG2>(a[1], ga[2], a[2], grads + L.cw[1], grads + L.cb[1], ns, w, ws, st);
  hipLaunchKernelGGL((k_conv_bwd_data<SFFT_CONV_CFG2, 16>), dim3(ns, 1), dim3(256),
                     (conv_bwd_data_lds<SFFT_CONV_CFG2, 16>()), st, (const float*)ga[2], (const float*)a[2],
                     P + L.cw[1], ga[1]);
  conv_wgrad<SFFT_CONV_CFG1>(x, ga[1], a[1], grads + L.cw[0], grads + L.cb[0], ns, w, ws, st);
  return hipGetLastError();
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, int step, float lr, float b1,
                       float b2, float eps, hipStream_t st) {
  const double c1 = 1.0 / (1.0 - std::pow((double)b1, step));
  const double c2 = 1.0 / (1.0 - std::pow((double)b2, step));
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, g, m, v, n, lr, b1, b2, eps,
                     (float)c1, (float)c2);
  return hipGetLastError();
}

hipError_t launch_destandardize(const float* pred, const double* mean, const double* scale, int n_pairs,
                                int n_out, double* coef, hipStream_t st) {
  const int64_t n = (int64_t)n_pairs * n_out;
  hipLaunchKernelGGL(k_destandardize, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, pred, mean, scale,
                     n_pairs, n_out, coef);
  return hipGetLastError();
}

}  // namespace sfft
