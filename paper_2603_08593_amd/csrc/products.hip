// Products made from difference images.
//
// Multi-template combine (paper Sec. 2.3.2, image differencing against each
// of the N_TEMP templates of Sec. 2.2.1): every difference image is scaled to
// a common photometric zero point, 10^(0.4 (zp_common - zp_t)), and the stack
// is median-combined pixel by pixel (the mean of the two middle values for an
// even count; NaN if any input is NaN). One pass over the stack: each thread
// holds its pixels' values of every template in registers and sorts them
// with a compare-exchange network; the kernel is bound by HBM (n reads and
// one write per pixel).
//
// Aperture photometry (paper Sec. 2.3.3, differential photometry and the
// 5-sigma limiting magnitude from apertures at random background
// positions; Sec. 2.4.3, forced photometry at fixed positions): the flux in
// a circle of radius r is sum over pixels of value x (area of the pixel
// square inside the circle), pixel centres at integer coordinates, pixels
// outside the image contributing nothing. The area is exact: the integral
// over x of the chord length inside the pixel's y range, split at the
// points where the chord meets the pixel's edges and integrated in closed
// form (antiderivative of sqrt(r^2 - u^2), in a form that stays accurate where
// the circle meets the pixel edge tangentially). One wave per aperture, lanes over
// the pixels of its bounding box, a fixed-order wave sum in FP64.
#include <cmath>

#include "common.hpp"
#include "products.hpp"

namespace sfft {

// ---------------------------------------------------------------------------
// median combine
// ---------------------------------------------------------------------------

constexpr int kCombThreads = 256;
constexpr int kCombPix = 4;     // pixels per thread (consecutive in a row)

template <int NT>
__device__ __forceinline__ void sort_net(double* v) {
  // odd-even transposition sort: NT rounds of compare-exchange
#pragma unroll
  for (int rnd = 0; rnd < NT; ++rnd) {
#pragma unroll
    for (int i = rnd & 1; i + 1 < NT; i += 2) {
      const double lo = fmin(v[i], v[i + 1]);
      const double hi = fmax(v[i], v[i + 1]);
      v[i] = lo;
      v[i + 1] = hi;
    }
  }
}

// VEC: FP32 images whose rows start 16-byte aligned; a thread's 4 pixels of
// every template are one 16-byte load each
template <typename T, int NT, bool VEC>
__global__ __launch_bounds__(kCombThreads) void k_median_combine(CombineArgs a) {
  const int y = blockIdx.y;
  const int x0 = (blockIdx.x * kCombThreads + threadIdx.x) * kCombPix;
  if (x0 >= a.W) return;
  const int64_t row = (int64_t)y * a.ld;
  double v[kCombPix][NT];
  // every template's loads are issued before any is used
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const T* D = static_cast<const T*>(a.D[t]) + row;
    if (VEC && x0 + kCombPix <= a.W) {
      const float4 q = *reinterpret_cast<const float4*>(D + x0);
      v[0][t] = q.x;
      v[1][t] = q.y;
      v[2][t] = q.z;
      v[3][t] = q.w;
    } else {
#pragma unroll
      for (int p = 0; p < kCombPix; ++p) {
        const int x = x0 + p;
        v[p][t] = x < a.W ? (double)D[x] : 0.0;
      }
    }
  }
  T* out = static_cast<T*>(a.out) + row;
  T res[kCombPix];
#pragma unroll
  for (int p = 0; p < kCombPix; ++p) {
    bool nan = false;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      v[p][t] *= a.scale[t];
      nan |= !(v[p][t] == v[p][t]);
    }
    sort_net<NT>(v[p]);
    double m = (NT & 1) ? v[p][NT / 2] : 0.5 * (v[p][NT / 2 - 1] + v[p][NT / 2]);
    if (nan) m = __builtin_nan("");
    res[p] = (T)m;
  }
  if (VEC && x0 + kCombPix <= a.W) {
    *reinterpret_cast<float4*>(out + x0) = float4{(float)res[0], (float)res[1], (float)res[2], (float)res[3]};
  } else {
#pragma unroll
    for (int p = 0; p < kCombPix; ++p)
      if (x0 + p < a.W) out[x0 + p] = res[p];
  }
}

template <typename T, bool VEC>
static hipError_t launch_combine_t(const CombineArgs& a, int n, hipStream_t st) {
  const dim3 grid((unsigned)((a.W + kCombThreads * kCombPix - 1) / (kCombThreads * kCombPix)), (unsigned)a.H);
  const dim3 blk(kCombThreads);
  switch (n) {
#define SFFT_COMB_CASE(K) \
    case K: hipLaunchKernelGGL((k_median_combine<T, K, VEC>), grid, blk, 0, st, a); break;
    SFFT_COMB_CASE(1) SFFT_COMB_CASE(2) SFFT_COMB_CASE(3) SFFT_COMB_CASE(4)
    SFFT_COMB_CASE(5) SFFT_COMB_CASE(6) SFFT_COMB_CASE(7) SFFT_COMB_CASE(8)
    SFFT_COMB_CASE(9) SFFT_COMB_CASE(10) SFFT_COMB_CASE(11) SFFT_COMB_CASE(12)
    SFFT_COMB_CASE(13) SFFT_COMB_CASE(14) SFFT_COMB_CASE(15) SFFT_COMB_CASE(16)
#undef SFFT_COMB_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_median_combine(const CombineArgs& a, int n, bool f32, hipStream_t st) {
  if (n < 1 || n > kMaxTemplates) return hipErrorInvalidValue;
  if (!f32) return launch_combine_t<double, false>(a, n, st);
  bool aligned = (a.ld % 4) == 0 && (reinterpret_cast<uintptr_t>(a.out) & 15) == 0;
  for (int t = 0; t < n; ++t) aligned = aligned && (reinterpret_cast<uintptr_t>(a.D[t]) & 15) == 0;
  return aligned ? launch_combine_t<float, true>(a, n, st) : launch_combine_t<float, false>(a, n, st);
}

// ---------------------------------------------------------------------------
// aperture photometry
// ---------------------------------------------------------------------------

// integral of sqrt(r^2 - t^2) dt from 0 to u, |u| <= r, as (u s + r^2 theta) / 2
// with s = sqrt((r - u)(r + u)) and theta = atan2(u, s): near u = +-r both
// terms are steep in u, and asin(u / r) would amplify the rounding of u / r
// (by r / s); s and theta from the exact u do not
__device__ __forceinline__ double chord_prim(double u, double r, double r2) {
  const double s = sqrt(fmax((r - u) * (r + u), 0.0));
  return 0.5 * (u * s + r2 * atan2(u, s));
}

// area of [x0, x1] x [y0, y1] (coordinates relative to the circle centre)
// inside the circle of radius r
__device__ double rect_circle_area(double x0, double x1, double y0, double y1, double r) {
  const double r2 = r * r;
  const double a = fmax(x0, -r), b = fmin(x1, r);
  if (!(a < b)) return 0.0;
  // x where the chord's ends cross y0 or y1
  double c[4];
  int nc = 0;
  if (fabs(y0) < r) {
    const double t = sqrt((r - fabs(y0)) * (r + fabs(y0)));
    c[nc++] = -t;
    c[nc++] = t;
  }
  if (fabs(y1) < r) {
    const double t = sqrt((r - fabs(y1)) * (r + fabs(y1)));
    c[nc++] = -t;
    c[nc++] = t;
  }
  for (int i = 1; i < nc; ++i)
    for (int j = i; j > 0 && c[j - 1] > c[j]; --j) {
      const double tmp = c[j];
      c[j] = c[j - 1];
      c[j - 1] = tmp;
    }
  double area = 0.0;
  double lo = a;
  for (int k = 0; k <= nc; ++k) {
    double hi = b;
    if (k < nc) {
      if (!(c[k] > lo)) continue;
      hi = fmin(c[k], b);
    }
    if (hi > lo) {
      // on (lo, hi) the chord's top is either y1 or the circle and its
      // bottom either y0 or the circle, the same throughout
      const double m = 0.5 * (lo + hi);
      const double sm = sqrt(fmax(r2 - m * m, 0.0));
      const bool top_c = sm < y1, bot_c = -sm > y0;
      const double top = top_c ? sm : y1, bot = bot_c ? -sm : y0;
      if (top > bot) {
        const double sint = chord_prim(hi, r, r2) - chord_prim(lo, r, r2);
        const double w = hi - lo;
        area += (top_c ? sint : y1 * w) - (bot_c ? -sint : y0 * w);
      }
      lo = hi;
    }
    if (lo >= b) break;
  }
  return area;
}

constexpr int kApThreads = 256;   // 4 apertures per workgroup, one wave each

template <typename T>
__global__ __launch_bounds__(kApThreads) void k_aperture(ApArgs a) {
  const int lane = threadIdx.x & 63;
  const int k = blockIdx.x * (kApThreads / 64) + (threadIdx.x >> 6);
  if (k >= a.n) return;
  const double cx = a.xy[2 * k], cy = a.xy[2 * k + 1];
  const double r = a.radius;
  // a non-finite centre gives NaN, a circle clear of the image 0 (and the
  // pixel box below stays at most 2r + 2 wide)
  const bool fin = is_finite_d(cx) && is_finite_d(cy);
  const bool near = fin && cx > -r - 1.0 && cx < a.W + r && cy > -r - 1.0 && cy < a.H + r;
  if (!near) {
    if (lane == 0) {
      const double v = fin ? 0.0 : __builtin_nan("");
      a.flux[k] = v;
      if (a.mag) a.mag[k] = __builtin_nan("");
      if (a.mag_err) a.mag_err[k] = __builtin_nan("");
    }
    return;
  }
  // pixels whose square can meet the circle
  const int px0 = (int)ceil(cx - r - 0.5), px1 = (int)floor(cx + r + 0.5);
  const int py0 = (int)ceil(cy - r - 0.5), py1 = (int)floor(cy + r + 0.5);
  const int bw = px1 - px0 + 1, bh = py1 - py0 + 1;
  const T* img = static_cast<const T*>(a.img);
  double s = 0.0;
  for (int c = lane; c < bw * bh; c += 64) {
    const int px = px0 + c % bw, py = py0 + c / bw;
    if (px < 0 || px >= a.W || py < 0 || py >= a.H) continue;
    const double w = rect_circle_area(px - 0.5 - cx, px + 0.5 - cx, py - 0.5 - cy, py + 0.5 - cy, r);
    if (w > 0.0) s = fma(w, (double)img[(int64_t)py * a.ld + px], s);
  }
  s = wave_sum(s);
  if (lane == 0) {
    a.flux[k] = s;
    if (a.mag) a.mag[k] = s > 0.0 ? a.zp - 2.5 * log10(s) : __builtin_nan("");
    if (a.mag_err) {
      const double sig = a.sigma ? *a.sigma : __builtin_nan("");
      a.mag_err[k] = s != 0.0 ? (2.5 / 2.302585092994045684017991454684364) * sig / fabs(s)
                              : __builtin_nan("");
    }
  }
}

hipError_t launch_aperture(const ApArgs& a, bool f32, hipStream_t st) {
  const dim3 grid((unsigned)((a.n + kApThreads / 64 - 1) / (kApThreads / 64)));
  if (f32) hipLaunchKernelGGL(k_aperture<float>, grid, dim3(kApThreads), 0, st, a);
  else hipLaunchKernelGGL(k_aperture<double>, grid, dim3(kApThreads), 0, st, a);
  return hipGetLastError();
}

// sigma = sample standard deviation of the n fluxes, m_lim = zp - 2.5
// log10(nsigma sigma); out = {sigma, m_lim, mean}. One workgroup, fixed order.
__global__ __launch_bounds__(1024) void k_limiting_mag(const double* flux, int n, double zp, double nsigma,
                                                       double* out) {
  __shared__ double red[16];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += flux[i];
  const double mean = block_sum(s, red) / (double)n;
  double q = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double d = flux[i] - mean;
    q = fma(d, d, q);
  }
  const double ss = block_sum(q, red);
  if (threadIdx.x == 0) {
    const double sigma = sqrt(ss / (double)(n - 1));
    out[0] = sigma;
    out[1] = zp - 2.5 * log10(nsigma * sigma);
    out[2] = mean;
  }
}

hipError_t launch_limiting_mag(const double* flux, int n, double zp, double nsigma, double* out,
                               hipStream_t st) {
  hipLaunchKernelGGL(k_limiting_mag, dim3(1), dim3(1024), 0, st, flux, n, zp, nsigma, out);
  return hipGetLastError();
}

}  // namespace sfft
