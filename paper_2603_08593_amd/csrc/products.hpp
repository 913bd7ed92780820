// Argument blocks of the difference-image product kernels (products.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sfft {

constexpr int kMaxTemplates = 16;

// median of n zero-point-scaled difference images (all W x H, pitch ld)
struct CombineArgs {
  const void* D[kMaxTemplates];
  double scale[kMaxTemplates];
  void* out;
  int64_t ld;
  int W, H;
};

// circular-aperture sums at n positions xy[k] = (x, y)
struct ApArgs {
  const void* img;
  int64_t ld;
  int W, H;
  const double* xy;
  int n;
  double radius;
  double* flux;            // [n]
  double* mag;             // [n] or null: zp - 2.5 log10(flux), NaN for flux <= 0
  double* mag_err;         // [n] or null: (2.5 / ln 10) sigma / |flux|
  const double* sigma;     // device scalar (background aperture scatter) or null
  double zp;
};

hipError_t launch_median_combine(const CombineArgs& a, int n, bool f32, hipStream_t st);
hipError_t launch_aperture(const ApArgs& a, bool f32, hipStream_t st);
hipError_t launch_limiting_mag(const double* flux, int n, double zp, double nsigma, double* out,
                               hipStream_t st);

}  // namespace sfft
