// Layer table, workspace plan and argument blocks of the real-bogus scorer
// (realbogus.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace sfft {

constexpr int kRbStamp = 32;
constexpr int kRbMaxN = 16384;     // candidates per call

// flat FP32 parameter layout: each conv weight [out][in][ky][kx] (1x1:
// [out][in]) then its bias, in the order stem, b1a, b1b, b2a, b2b, b2p, b3a,
// b3b, b3p; then fc1 [64][128] + bias [64], fc2 [1][64] + bias [1]
constexpr int kRbConvOut[9] = {32, 32, 32, 64, 64, 64, 128, 128, 128};
constexpr int kRbConvIn[9] = {3, 32, 32, 32, 64, 32, 64, 128, 64};
constexpr int kRbConvK[9] = {3, 3, 3, 3, 3, 1, 3, 3, 1};

constexpr int rb_conv_woff(int l) {
  int o = 0;
  for (int i = 0; i < l; ++i) o += kRbConvOut[i] * kRbConvIn[i] * kRbConvK[i] * kRbConvK[i] + kRbConvOut[i];
  return o;
}
constexpr int rb_conv_boff(int l) {
  return rb_conv_woff(l) + kRbConvOut[l] * kRbConvIn[l] * kRbConvK[l] * kRbConvK[l];
}
constexpr int kRbFc1W = rb_conv_woff(9);
constexpr int kRbFc1B = kRbFc1W + 64 * 128;
constexpr int kRbFc2W = kRbFc1B + 64;
constexpr int kRbFc2B = kRbFc2W + 64;
constexpr int kRbNumParams = kRbFc2B + 1;

// the seven GEMMs: a 3x3 conv, plus a 1x1 stride-2 projection shortcut
// appended to its k range (blocks 2 and 3)
struct RbGemm {
  int co, ci, cinp, stride;     // output channels, input channels (padded to 8k), stride
  int cip, cipp;                // projection input channels (padded), 0 if none
  int w_off, b_off, wp_off, bp_off;
};
constexpr int kRbGemms = 7;
constexpr RbGemm kRbGemm[kRbGemms] = {
    {32, 3, 8, 1, 0, 0, rb_conv_woff(0), rb_conv_boff(0), -1, -1},
    {32, 32, 32, 1, 0, 0, rb_conv_woff(1), rb_conv_boff(1), -1, -1},
    {32, 32, 32, 1, 0, 0, rb_conv_woff(2), rb_conv_boff(2), -1, -1},
    {64, 32, 32, 2, 0, 0, rb_conv_woff(3), rb_conv_boff(3), -1, -1},
    {64, 64, 64, 1, 32, 32, rb_conv_woff(4), rb_conv_boff(4), rb_conv_woff(5), rb_conv_boff(5)},
    {128, 64, 64, 2, 0, 0, rb_conv_woff(6), rb_conv_boff(6), -1, -1},
    {128, 128, 128, 1, 64, 64, rb_conv_woff(7), rb_conv_boff(7), rb_conv_woff(8), rb_conv_boff(8)},
};

struct RbPlan {
  int n;
  int KP[kRbGemms];             // padded k length of each GEMM (multiple of 32)
  size_t w[kRbGemms], bias[kRbGemms];
  size_t act[2];                // stage outputs (bf16 NHWC): stage 1 then stage 3, stage 2
  size_t total;
};
RbPlan rb_plan(int n);

struct RbExtractArgs {
  const void* img[3];           // science, template, difference
  int64_t ld;
  int W, H;
  const int32_t* centers;       // [n][2] = (x, y)
  int n;
  float offset[3], scale[3];
  float* stamps;                // [n][3][32][32]
};

hipError_t launch_rb_score(const float* params, const float* stamps, int n, float* logits, float* probs,
                           unsigned char* ws, hipStream_t st);
hipError_t launch_rb_extract(const RbExtractArgs& a, bool f32, hipStream_t st);
hipError_t prepare_rb_attributes();   // dynamic LDS limit of the fused stage-1 kernel

}  // namespace sfft
