// Real-bogus scorer inference (paper Sec. 2.3.4): a rotation-invariant
// convolutional network with residual connections scores three-channel
// (science, template, difference) stamps of candidates. Layer sizes (not
// published; the reading documented with the C declarations): per rotated copy
// of a 32 x 32 stamp, stem conv 3 -> 32, residual block 32, strided residual
// blocks 64 and 128 with 1x1 projections, global average pool; the four
// copies' features averaged; linear 128 -> 64, ReLU, linear 64 -> 1.
//
// The convolutions run as implicit GEMMs on the bf16 matrix cores
// (v_mfma_f32_16x16x32_bf16): rows = output pixels of all copies (NHWC
// activations, bf16), columns = output channels, k = (tap, input channel)
// with the input channels padded to a multiple of 8 so that every lane's 8
// consecutive k values are one 16-byte load of one pixel; a block's 1x1
// projection shortcut is appended to the same k range (one accumulator), an
// identity shortcut is added in the epilogue. FP32 accumulation; bias,
// shortcut, ReLU and the rounding to bf16 in the epilogue. The network runs
// as two fused kernels (stem and blocks 1 and 2; block 3 and the first
// pooling step), one stamp copy per workgroup with the activations in LDS.
#include <cmath>
#include <cstring>
#include <vector>

#include "common.hpp"
#include "layout.hpp"
#include "realbogus.hpp"

namespace sfft {

typedef __bf16 bf16x8_rb __attribute__((ext_vector_type(8)));
typedef float floatx4_rb __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short f32_to_bf16_rne(float f) {
  const unsigned u = __builtin_bit_cast(unsigned, f);
  return (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_to_f32(unsigned short h) {
  return __builtin_bit_cast(float, (unsigned)h << 16);
}

// The convolution GEMMs put the weights in the matrix-core instruction's
// first operand and the activations in its second, so lane (g, l16) of a
// 16 x 16 result tile holds output channels 4 g .. 4 g + 3 of pixel l16:
// four adjacent channels of one pixel, stored as one 8-byte access.
typedef __bf16 bf16x2_rb __attribute__((ext_vector_type(2)));
typedef float floatx2_rb __attribute__((ext_vector_type(2)));

// two floats to a pair of bf16 (round to nearest even, the rounding of
// f32_to_bf16_rne), low half first
__device__ __forceinline__ unsigned bf16x2_rne(float lo, float hi) {
  return __builtin_bit_cast(unsigned, __builtin_convertvector(floatx2_rb{lo, hi}, bf16x2_rb));
}
// bias, optional residual (4 bf16 at r), ReLU, packed to 4 bf16
__device__ __forceinline__ uint2 rb_act4(const floatx4_rb& acc, const float (&b)[4], const uint2* r) {
  float v[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) v[i] = acc[i] + b[i];
  if (r) {
    const uint2 x = *r;
    v[0] += __builtin_bit_cast(float, x.x << 16);
    v[1] += __builtin_bit_cast(float, x.x & 0xFFFF0000u);
    v[2] += __builtin_bit_cast(float, x.y << 16);
    v[3] += __builtin_bit_cast(float, x.y & 0xFFFF0000u);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) v[i] = fmaxf(v[i], 0.0f);
  return uint2{bf16x2_rne(v[0], v[1]), bf16x2_rne(v[2], v[3])};
}

// ---------------------------------------------------------------------------
// weights: FP32 [out][in][ky][kx] (+ projection [out][in]) -> bf16 [out][KP]
// with k = tap * CINP + c for the 3x3 part and 9 CINP + c for the projection
// ---------------------------------------------------------------------------

struct RbPackArgs {
  const float* w;        // main conv weights [co][ci][3][3]
  const float* b;        // main bias [co]
  const float* wp;       // projection [co][cip] or null
  const float* bp;       // projection bias or null
  unsigned short* out;   // [co][KP]
  float* bias;           // [co]
  int co, ci, cinp, cip, cipp, KP;
};

__global__ __launch_bounds__(256) void k_rb_pack(RbPackArgs a) {
  const int64_t total = (int64_t)a.co * a.KP;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256) {
    const int o = (int)(i / a.KP), k = (int)(i % a.KP);
    float v = 0.0f;
    if (k < 9 * a.cinp) {
      const int tap = k / a.cinp, c = k % a.cinp;
      if (c < a.ci) v = a.w[((int64_t)o * a.ci + c) * 9 + tap];
    } else if (a.wp && k < 9 * a.cinp + a.cipp) {
      const int c = k - 9 * a.cinp;
      if (c < a.cip) v = a.wp[(int64_t)o * a.cip + c];
    }
    a.out[i] = f32_to_bf16_rne(v);
    if (k == 0) a.bias[o] = a.b[o] + (a.bp ? a.bp[o] : 0.0f);
  }
}

// ---------------------------------------------------------------------------
// Stage 1 fused (stem, block-1 conv a, block-1 conv b + identity shortcut,
// then block 2 below): the layers keep their activations in LDS, one copy
// per workgroup, and only block 2's output goes to memory. Layer by layer,
// every 32-channel 32 x 32 map of 4096 candidates is ~1 GB written and read
// back (each layer then bound by memory traffic); here the stamp (12 KB)
// and block 2's output (32 KB) are the only traffic besides the
// L2-resident weights.
// Maps are 34 x 34 pixels (a zero border of one pixel, so the 3 x 3 taps
// need no bounds checks), bf16, 32 channels as four planes of 8-channel
// groups (16 bytes per pixel in each plane): 16 consecutive pixels of one
// group are 256 contiguous bytes, on distinct banks, and a tap's pixel
// offset is a constant added to a per-lane base, which the LDS instruction
// takes as its immediate offset. The input map holds 8 channels per pixel
// (plane 0 alone). Every output is the sum of its k chunks in
// order, one v_mfma_f32_16x16x32_bf16 per chunk and output tile, then the
// epilogue (bias, shortcut, ReLU, rounding to bf16) in FP32: the rounding
// points the FP64 oracle reproduces.
// ---------------------------------------------------------------------------

constexpr int kRbFusedThreads = 512;   // fused stages: 8 waves, two per SIMD
constexpr int kRbMapSide = 34;
constexpr int kRbMapPix = kRbMapSide * kRbMapSide;
constexpr size_t kRbMapBytes = (size_t)kRbMapPix * 64;          // 32 channels of bf16
constexpr size_t kRbStage1Lds = 2 * kRbMapBytes;

constexpr int kRbPlane = kRbMapPix * 16;                        // bytes of one channel group

// zero the one-pixel border of np consecutive planes (side x side pixels of
// `groups` 16-byte groups each); the layers write every interior pixel of
// their maps, so only the borders that the 3 x 3 taps read need clearing
__device__ __forceinline__ void rb_zero_border(unsigned char* base, int np, int side, int plane_bytes,
                                               int groups = 1) {
  const int nb = 4 * side - 4;
  for (int i = threadIdx.x; i < np * nb * groups; i += kRbFusedThreads) {
    const int q = i % groups, rest = i / groups;
    const int pl = rest / nb, k = rest - pl * nb;
    int y, x;
    if (k < side) { y = 0; x = k; }
    else if (k < 2 * side) { y = side - 1; x = k - side; }
    else { const int e = k - 2 * side; y = 1 + (e >> 1); x = (e & 1) ? side - 1 : 0; }
    *reinterpret_cast<uint4*>(base + pl * plane_bytes + ((y * side + x) * groups + q) * 16) = uint4{0u, 0u, 0u, 0u};
  }
}

__device__ __forceinline__ int rb_map_off(int p, int cg) {      // bytes, 32-channel map
  return cg * kRbPlane + p * 16;
}

// one layer: out = relu(conv3x3(in) + bias [+ res]) on the 32 x 32 interior;
// CIN8: the input map has 8 channels per pixel (the stem)
template <bool CIN8, bool RES>
__device__ __forceinline__ void rb_stage1_layer(const unsigned char* in, unsigned char* out,
                                                const unsigned short* w, const float* bias, int KP) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l16 = lane & 15, g = lane >> 4;
  constexpr int NKC = CIN8 ? 3 : 9;            // k chunks: KP = 96 (stem), 288
  const int cin = CIN8 ? 8 : 32;
  // the lane's weights of every k chunk and the biases of its result
  // channels 16 t + 4 g + i, held in registers for the 2 passes
  float bias4[2][4];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i) bias4[t][i] = bias[16 * t + 4 * g + i];
  uint4 Bw[NKC][2];
#pragma unroll
  for (int kc = 0; kc < NKC; ++kc)
#pragma unroll
    for (int t = 0; t < 2; ++t)
      Bw[kc][t] = *reinterpret_cast<const uint4*>(w + (int64_t)(16 * t + l16) * KP + kc * 32 + 8 * g);
  // wave w: row tiles 8 w .. 8 w + 7 of the 64 (16 pixels each), 4 per pass
  for (int pass = 0; pass < 2; ++pass) {
    const int mt0 = 8 * wave + 4 * pass;
    floatx4_rb acc[4][2];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int t = 0; t < 2; ++t) acc[m][t] = floatx4_rb{0.f, 0.f, 0.f, 0.f};
    auto load_a = [&](int kc, uint4 (&A)[4]) {
      const int k0 = kc * 32 + 8 * g;
      const int tap = k0 / cin, c0 = k0 - tap * cin;
      const int ky = tap / 3, kx = tap - ky * 3;
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int P = 16 * (mt0 + m) + l16;                      // output pixel, row-major 32 x 32
        const int p = ((P >> 5) + ky) * kRbMapSide + (P & 31) + kx;
        if (tap >= 9) A[m] = uint4{0u, 0u, 0u, 0u};               // k padding
        else if (CIN8) A[m] = *reinterpret_cast<const uint4*>(in + p * 16);
        else A[m] = *reinterpret_cast<const uint4*>(in + rb_map_off(p, c0 >> 3));
      }
    };
    uint4 A[4], An[4];
    load_a(0, A);
#pragma unroll
    for (int kc = 0; kc < NKC; ++kc) {
      if (kc + 1 < NKC) load_a(kc + 1, An);
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int m = 0; m < 4; ++m)
          acc[m][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_rb, Bw[kc][t]),
                                                              __builtin_bit_cast(bf16x8_rb, A[m]), acc[m][t],
                                                              0, 0, 0);
      if (kc + 1 < NKC) {
#pragma unroll
        for (int m = 0; m < 4; ++m) A[m] = An[m];
      }
    }
    // epilogue: lane (g, l16), element i -> channel 16 t + 4 g + i of pixel 16 m + l16
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int P = 16 * (mt0 + m) + l16;
      const int p = ((P >> 5) + 1) * kRbMapSide + (P & 31) + 1;
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int co = 16 * t + 4 * g;
        uint2* dst = reinterpret_cast<uint2*>(out + rb_map_off(p, co >> 3) + 2 * (co & 7));
        *dst = rb_act4(acc[m][t], bias4[t], RES ? dst : nullptr);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Block 2 (stride-2 conv a 32 -> 64, conv b 64 -> 64 with the 1x1 stride-2
// projection of the block input appended to its k range), run by the first
// fused kernel after block 1 on the same copy. LDS: the block input is block
// 1's output map (34 x 34 x 32), conv a's output an 18 x 18 map of 64
// channels over the other map's space (a zero border; eight planes of
// 8-channel groups, 16 bytes per pixel in each, as block 1's maps); conv b's
// output goes to memory. Wave w computes the output channels 32 (w & 1) ..
// + 31 of half the pixels, with that half's weights in registers.
// ---------------------------------------------------------------------------

constexpr int kRbMap16Side = 18;
constexpr size_t kRbMap16Bytes = (size_t)kRbMap16Side * kRbMap16Side * 128;   // 64 channels of bf16
static_assert(kRbMap16Bytes <= kRbMapBytes, "block 2's conv a map fits over block 1's second map");

constexpr int kRbPlane16 = kRbMap16Side * kRbMap16Side * 16;    // bytes of one channel group

__device__ __forceinline__ int rb_map16_off(int p, int cg) {    // bytes, 64-channel map
  return cg * kRbPlane16 + p * 16;
}

// one GEMM of block 2: 256 output pixels (16 x 16) x 64 channels; wave w:
// channel half h = w & 1, pixels 64 (w >> 1) .. + 63.
// CONV_A: input the 34 x 34 block-input map (stride 2); else the 18 x 18 map
// (stride 1) plus the projection chunk from the block-input map.
template <bool CONV_A, int NKC>
__device__ __forceinline__ void rb_stage2_gemm(const unsigned char* in32, const unsigned char* in64,
                                               unsigned char* out64, unsigned short* gout,
                                               const unsigned short* w, const float* bias, int KP) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l16 = lane & 15, g = lane >> 4;
  const int h = wave & 1;
  float bias4[2][4];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i) bias4[t][i] = bias[32 * h + 16 * t + 4 * g + i];
  uint4 Bw[NKC][2];
#pragma unroll
  for (int kc = 0; kc < NKC; ++kc)
#pragma unroll
    for (int t = 0; t < 2; ++t)
      Bw[kc][t] = *reinterpret_cast<const uint4*>(w + (int64_t)(32 * h + 16 * t + l16) * KP + kc * 32 + 8 * g);
  {
    const int mt0 = 4 * (wave >> 1);
    floatx4_rb acc[4][2];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int t = 0; t < 2; ++t) acc[m][t] = floatx4_rb{0.f, 0.f, 0.f, 0.f};
    auto load_a = [&](int kc, uint4 (&A)[4]) {
      const int k0 = kc * 32 + 8 * g;
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int P = 16 * (mt0 + m) + l16;                     // output pixel, row-major 16 x 16
        const int oy = P >> 4, ox = P & 15;
        if (CONV_A) {                                          // 3 x 3, stride 2, 32 input channels
          const int tap = k0 >> 5, c0 = k0 & 31;
          const int ky = tap / 3, kx = tap - ky * 3;
          const int p = (2 * oy + ky) * kRbMapSide + 2 * ox + kx;
          A[m] = *reinterpret_cast<const uint4*>(in32 + rb_map_off(p, c0 >> 3));
        } else if (k0 < 9 * 64) {                              // 3 x 3, stride 1, 64 channels
          const int tap = k0 >> 6, c0 = k0 & 63;
          const int ky = tap / 3, kx = tap - ky * 3;
          const int p = (oy + ky) * kRbMap16Side + ox + kx;
          A[m] = *reinterpret_cast<const uint4*>(in64 + rb_map16_off(p, c0 >> 3));
        } else {                                               // projection: block input at (2 oy, 2 ox)
          const int c0 = k0 - 9 * 64;
          const int p = (2 * oy + 1) * kRbMapSide + 2 * ox + 1;
          A[m] = *reinterpret_cast<const uint4*>(in32 + rb_map_off(p, c0 >> 3));
        }
      }
    };
    uint4 A[4], An[4];
    load_a(0, A);
#pragma unroll
    for (int kc = 0; kc < NKC; ++kc) {
      if (kc + 1 < NKC) load_a(kc + 1, An);
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int m = 0; m < 4; ++m)
          acc[m][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_rb, Bw[kc][t]),
                                                              __builtin_bit_cast(bf16x8_rb, A[m]), acc[m][t],
                                                              0, 0, 0);
      if (kc + 1 < NKC) {
#pragma unroll
        for (int m = 0; m < 4; ++m) A[m] = An[m];
      }
    }
    // lane (g, l16), element i -> channel 32 h + 16 t + 4 g + i of pixel 16 m + l16
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int P = 16 * (mt0 + m) + l16;
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int co = 32 * h + 16 * t + 4 * g;
        const uint2 b = rb_act4(acc[m][t], bias4[t], nullptr);
        if (CONV_A) {
          const int p = ((P >> 4) + 1) * kRbMap16Side + (P & 15) + 1;
          *reinterpret_cast<uint2*>(out64 + rb_map16_off(p, co >> 3) + 2 * (co & 7)) = b;
        } else {
          *reinterpret_cast<uint2*>(gout + (int64_t)P * 64 + co) = b;
        }
      }
    }
  }
}

struct RbStage1Args {
  const float* stamps;                    // [n][3][32][32]: science, template, difference
  const unsigned short* w[5];             // packed weights of stem, b1a, b1b, b2a, b2b (+ projection)
  const float* bias[5];
  int KP[5];
  unsigned short* y;                      // [copies][16][16][64]: block 2 output
  int copies;
};

__global__ __launch_bounds__(kRbFusedThreads, 1) void k_rb_stage1(RbStage1Args a) {
  extern __shared__ __align__(16) unsigned char rbm[];
  unsigned char* M0 = rbm;                       // stem output, then block output (in place)
  unsigned char* M1 = rbm + kRbMapBytes;         // input (8 channels), then conv a output
  const int c = blockIdx.x;
  if (c >= a.copies) return;
  const int tid = threadIdx.x;
  // the borders of both maps (M0 and M1 are 8 consecutive planes), then the
  // copy's input into M1's first plane
  rb_zero_border(rbm, 8, kRbMapSide, kRbPlane);
  __syncthreads();
  // the copy's input: copy c is candidate c / 4 turned by (c mod 4) quarter
  // turns (numpy's rot90 on the two image axes: one turn maps
  // out[i][j] = s[j][31 - i]), so that a quarter turn of a stamp only
  // permutes its copies; pixel (r, j) of the copy holds the three stamp
  // channels in bf16 and five zero channels (16 bytes)
  {
    const int rot = c & 3;
    const float* stp = a.stamps + (int64_t)(c >> 2) * 3 * kRbStamp * kRbStamp;
    constexpr int e = kRbStamp - 1;
    for (int i = tid; i < kRbStamp * kRbStamp; i += kRbFusedThreads) {
      const int r = i / kRbStamp, j = i % kRbStamp;
      int sy, sx;
      switch (rot) {
        case 0: sy = r; sx = j; break;
        case 1: sy = j; sx = e - r; break;
        case 2: sy = e - r; sx = e - j; break;
        default: sy = e - j; sx = r; break;
      }
      const int o = sy * kRbStamp + sx;
      uint4 pk;
      pk.x = f32_to_bf16_rne(stp[o]) | ((unsigned)f32_to_bf16_rne(stp[kRbStamp * kRbStamp + o]) << 16);
      pk.y = f32_to_bf16_rne(stp[2 * kRbStamp * kRbStamp + o]);
      pk.z = 0u;
      pk.w = 0u;
      reinterpret_cast<uint4*>(M1)[(r + 1) * kRbMapSide + j + 1] = pk;
    }
  }
  __syncthreads();
  rb_stage1_layer<true, false>(M1, M0, a.w[0], a.bias[0], a.KP[0]);
  __syncthreads();
  // M1 becomes a 32-channel map: conv a writes every interior pixel of its
  // four planes, and their borders are still zero (the input sat in the
  // interior of the first plane)
  rb_stage1_layer<false, false>(M0, M1, a.w[1], a.bias[1], a.KP[1]);
  __syncthreads();
  rb_stage1_layer<false, true>(M1, M0, a.w[2], a.bias[2], a.KP[2]);
  __syncthreads();
  // block 2 on the same copy: M0 (block 1's output, zero border) is its
  // input map; conv a's output (18 x 18 x 64, zero border) goes over M1
  rb_zero_border(M1, 8, kRbMap16Side, kRbPlane16);
  __syncthreads();
  rb_stage2_gemm<true, 9>(M0, nullptr, M1, nullptr, a.w[3], a.bias[3], a.KP[3]);
  __syncthreads();
  rb_stage2_gemm<false, 19>(M0, M1, nullptr, a.y + (int64_t)c * 16 * 16 * 64, a.w[4], a.bias[4], a.KP[4]);
}

// ---------------------------------------------------------------------------
// Stage 3: block 3 (conv a: 3 x 3 stride 2, 64 -> 128; conv b: 3 x 3, 128 ->
// 128 plus the 1 x 1 stride-2 projection of the block input) for one stamp
// copy per workgroup: the block input (18 x 18 x 64, zero border) and the
// conv a output (10 x 10 x 128, zero border) stay in LDS, and the block
// output goes to global memory for the head. Wave w owns output channels
// 16 w .. 16 w + 15 for all 64 output pixels (four matrix-core tiles), with
// its k-chunks of weights in registers.
// ---------------------------------------------------------------------------

constexpr int kRbMap8Side = 10;
constexpr size_t kRbMap8Bytes = (size_t)kRbMap8Side * kRbMap8Side * 256;   // 128 channels of bf16
constexpr size_t kRbStage3Lds = kRbMap16Bytes + kRbMap8Bytes;

// 128-channel map: 16 groups of 8 channels (16 bytes) per pixel; the group
// slot is cg ^ ((x + 8 (y & 1)) mod 16), so the 16 pixels that a
// quarter-wave reads (two rows of 8) take distinct banks
__device__ __forceinline__ int rb_map8_off(int y, int x, int cg) {
  return (y * kRbMap8Side + x) * 256 + ((cg ^ ((x + 8 * (y & 1)) & 15)) << 4);
}

// block 3's output in LDS: [pixel][channel] bf16 with a pitch of 136
// channels (272 bytes, 16 bytes past a multiple of 256), so the 16 pixels
// that a quarter-wave's 8-byte stores cover start on distinct banks
constexpr int kRbYPitch = 136;
static_assert(64 * kRbYPitch * 2 <= (int)kRbMap16Bytes, "block 3's output fits over its input map");

// one GEMM of stage 3: 64 output pixels (8 x 8) x 128 channels.
// CONV_A: input the 18 x 18 block-input map (stride 2); else the 10 x 10
// map (stride 1) plus the projection chunk from the block-input map.
template <bool CONV_A, int NKC>
__device__ __forceinline__ void rb_stage3_gemm(const unsigned char* in64, const unsigned char* in128,
                                               unsigned char* out128, unsigned short* yout,
                                               const unsigned short* w, const float* bias, int KP) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l16 = lane & 15, g = lane >> 4;
  const int co = 16 * wave + l16;           // weight row of this lane
  const int co4 = 16 * wave + 4 * g;        // its result channels co4 .. co4 + 3
  float bias4[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) bias4[i] = bias[co4 + i];
  uint4 Bw[NKC];
#pragma unroll
  for (int kc = 0; kc < NKC; ++kc)
    Bw[kc] = *reinterpret_cast<const uint4*>(w + (int64_t)co * KP + kc * 32 + 8 * g);
  floatx4_rb acc[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) acc[m] = floatx4_rb{0.f, 0.f, 0.f, 0.f};
  auto load_a = [&](int kc, uint4 (&A)[4]) {
    const int k0 = kc * 32 + 8 * g;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int P = 16 * m + l16;                              // output pixel, row-major 8 x 8
      const int oy = P >> 3, ox = P & 7;
      if (CONV_A) {                                          // 3 x 3, stride 2, 64 input channels
        const int tap = k0 >> 6, c0 = k0 & 63;
        const int ky = tap / 3, kx = tap - ky * 3;
        const int p = (2 * oy + ky) * kRbMap16Side + 2 * ox + kx;
        A[m] = *reinterpret_cast<const uint4*>(in64 + rb_map16_off(p, c0 >> 3));
      } else if (k0 < 9 * 128) {                             // 3 x 3, stride 1, 128 channels
        const int tap = k0 >> 7, c0 = k0 & 127;
        const int ky = tap / 3, kx = tap - ky * 3;
        A[m] = *reinterpret_cast<const uint4*>(in128 + rb_map8_off(oy + ky, ox + kx, c0 >> 3));
      } else {                                               // projection: block input at (2 oy, 2 ox)
        const int c0 = k0 - 9 * 128;
        const int p = (2 * oy + 1) * kRbMap16Side + 2 * ox + 1;
        A[m] = *reinterpret_cast<const uint4*>(in64 + rb_map16_off(p, c0 >> 3));
      }
    }
  };
  uint4 A[4], An[4];
  load_a(0, A);
#pragma unroll
  for (int kc = 0; kc < NKC; ++kc) {
    if (kc + 1 < NKC) load_a(kc + 1, An);
#pragma unroll
    for (int m = 0; m < 4; ++m)
      acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_rb, Bw[kc]),
                                                       __builtin_bit_cast(bf16x8_rb, A[m]), acc[m], 0, 0, 0);
    if (kc + 1 < NKC) {
#pragma unroll
      for (int m = 0; m < 4; ++m) A[m] = An[m];
    }
  }
  // conv b: its output overwrites LDS that the other waves may still read,
  // so it waits for them
  if (!CONV_A) __syncthreads();
  // lane (g, l16), element i -> channel co4 + i of pixel 16 m + l16
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const int P = 16 * m + l16;
    const uint2 b = rb_act4(acc[m], bias4, nullptr);
    if (CONV_A)
      *reinterpret_cast<uint2*>(out128 + rb_map8_off((P >> 3) + 1, (P & 7) + 1, co4 >> 3) + 2 * (co4 & 7)) = b;
    else
      *reinterpret_cast<uint2*>(yout + P * kRbYPitch + co4) = b;
  }
}

struct RbStage3Args {
  const unsigned short* x;                // [copies][16][16][64]: block 2 output
  const unsigned short* w[2];             // packed weights of block 3 conv a, conv b (+ projection)
  const float* bias[2];
  int KP[2];
  float* feat;                            // [copies][128]: per-channel sums of the block output
  int copies;
};

__global__ __launch_bounds__(kRbFusedThreads, 1) void k_rb_stage3(RbStage3Args a) {
  extern __shared__ __align__(16) unsigned char rbm[];
  unsigned char* M64 = rbm;                      // block input, 18 x 18 x 64
  unsigned char* M128 = rbm + kRbMap16Bytes;     // conv a output, 10 x 10 x 128
  const int c = blockIdx.x;
  if (c >= a.copies) return;
  const int tid = threadIdx.x;
  // borders only: the block input's planes (their interiors are filled
  // below) and conv a's output map (conv a writes every interior pixel)
  rb_zero_border(M64, 8, kRbMap16Side, kRbPlane16);
  rb_zero_border(M128, 1, kRbMap8Side, 0, 16);
  __syncthreads();
  const uint4* src = reinterpret_cast<const uint4*>(a.x + (int64_t)c * 16 * 16 * 64);
  for (int i = tid; i < 16 * 16 * 8; i += kRbFusedThreads) {
    const int P = i >> 3, cg = i & 7;
    const int p = ((P >> 4) + 1) * kRbMap16Side + (P & 15) + 1;
    *reinterpret_cast<uint4*>(M64 + rb_map16_off(p, cg)) = src[i];
  }
  __syncthreads();
  rb_stage3_gemm<true, 18>(M64, nullptr, M128, nullptr, a.w[0], a.bias[0], a.KP[0]);
  __syncthreads();
  // the block output (bf16, [pixel][channel]) goes over the block-input map
  // (free once conv b is done); then each channel's 64 pixels are summed in
  // pixel order in FP32, the first step of the head's average pooling
  unsigned short* Y = reinterpret_cast<unsigned short*>(M64);
  rb_stage3_gemm<false, 38>(M64, M128, nullptr, Y, a.w[1], a.bias[1], a.KP[1]);
  __syncthreads();
  if (tid < 128) {
    float sr = 0.0f;
    for (int px = 0; px < 64; ++px) sr += bf16_to_f32(Y[px * kRbYPitch + tid]);
    a.feat[(int64_t)c * 128 + tid] = sr;
  }
}

// ---------------------------------------------------------------------------
// head: mean over the 8 x 8 pixels (from the per-copy channel sums of
// stage 3) and the 4 copies, linear 128 -> 64, ReLU, linear 64 -> 1, sigmoid.
// One workgroup of 128 threads per candidate, FP32, fixed order.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(128) void k_rb_head(const float* feat, const float* w1, const float* b1,
                                                 const float* w2, const float* b2, int n, float* logits,
                                                 float* probs) {
  __shared__ float f[128];
  __shared__ float hbuf[64];
  const int k = blockIdx.x, c = threadIdx.x;
  if (k >= n) return;
  // feat: each copy's per-channel sum over its 8 x 8 pixels (stage 3)
  float s = 0.0f;
  for (int rot = 0; rot < 4; ++rot) s += feat[(int64_t)(4 * k + rot) * 128 + c] * (1.0f / 64.0f);
  f[c] = s * 0.25f;
  __syncthreads();
  if (c < 64) {
    float v = b1[c];
    for (int j = 0; j < 128; ++j) v = fmaf(w1[c * 128 + j], f[j], v);
    hbuf[c] = fmaxf(v, 0.0f);
  }
  __syncthreads();
  if (c == 0) {
    float v = b2[0];
    for (int j = 0; j < 64; ++j) v = fmaf(w2[j], hbuf[j], v);
    logits[k] = v;
    if (probs) probs[k] = 1.0f / (1.0f + expf(-v));
  }
}

// ---------------------------------------------------------------------------
// stamp extraction: (I_c - offset_c) * scale_c on the 32 x 32 window
// [cx - 16, cx + 16) x [cy - 16, cy + 16), periodic
// ---------------------------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(256) void k_rb_extract(RbExtractArgs a) {
  const int64_t total = (int64_t)a.n * 3 * kRbStamp * kRbStamp;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= total) return;
  const int j = (int)(i % kRbStamp), r = (int)((i / kRbStamp) % kRbStamp);
  const int c = (int)((i / (kRbStamp * kRbStamp)) % 3), k = (int)(i / (3 * kRbStamp * kRbStamp));
  int y = a.centers[2 * k + 1] - kRbStamp / 2 + r, x = a.centers[2 * k] - kRbStamp / 2 + j;
  y %= a.H;
  if (y < 0) y += a.H;
  x %= a.W;
  if (x < 0) x += a.W;
  const T* img = static_cast<const T*>(a.img[c]);
  a.stamps[i] = (float)(((double)img[(int64_t)y * a.ld + x] - (double)a.offset[c]) * (double)a.scale[c]);
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

RbPlan rb_plan(int n) {
  RbPlan p{};
  p.n = n;
  const int64_t copies = 4 * (int64_t)n;
  size_t o = 0;
  auto take = [&](size_t bytes) { const size_t at = o; o = align256(o + bytes); return at; };
  for (int l = 0; l < kRbGemms; ++l) {
    const RbGemm& gm = kRbGemm[l];
    const int kp = (9 * gm.cinp + gm.cipp + 31) / 32 * 32;
    p.KP[l] = kp;
    p.w[l] = take((size_t)gm.co * kp * 2);
    p.bias[l] = take((size_t)gm.co * 4);
  }
  p.act[0] = take((size_t)copies * 16 * 16 * 64 * 2);   // block 2 output (bf16)
  p.act[1] = take((size_t)copies * 128 * 4);            // block 3 channel sums (FP32)
  p.total = o;
  return p;
}

hipError_t launch_rb_score(const float* params, const float* stamps, int n, float* logits, float* probs,
                           unsigned char* ws, hipStream_t st) {
  const RbPlan p = rb_plan(n);
  hipError_t e;
  // pack the weights of every GEMM (main conv + projection)
  for (int l = 0; l < kRbGemms; ++l) {
    const RbGemm& gm = kRbGemm[l];
    RbPackArgs pa{};
    pa.w = params + gm.w_off;
    pa.b = params + gm.b_off;
    pa.wp = gm.wp_off >= 0 ? params + gm.wp_off : nullptr;
    pa.bp = gm.bp_off >= 0 ? params + gm.bp_off : nullptr;
    pa.out = reinterpret_cast<unsigned short*>(ws + p.w[l]);
    pa.bias = reinterpret_cast<float*>(ws + p.bias[l]);
    pa.co = gm.co; pa.ci = gm.ci; pa.cinp = gm.cinp; pa.cip = gm.cip; pa.cipp = gm.cipp; pa.KP = p.KP[l];
    const int64_t total = (int64_t)gm.co * p.KP[l];
    hipLaunchKernelGGL(k_rb_pack, dim3((unsigned)std::min<int64_t>((total + 255) / 256, 4096)), dim3(256), 0,
                       st, pa);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  const int64_t copies = 4 * (int64_t)n;
  unsigned short* A2 = reinterpret_cast<unsigned short*>(ws + p.act[0]);   // blocks 1-2 out: [copies][16][16][64]
  float* feat = reinterpret_cast<float*>(ws + p.act[1]);                    // block 3 out: [copies][128]
  {
    RbStage1Args sa{};
    sa.stamps = stamps;
    for (int l = 0; l < 5; ++l) {
      sa.w[l] = reinterpret_cast<const unsigned short*>(ws + p.w[l]);
      sa.bias[l] = reinterpret_cast<const float*>(ws + p.bias[l]);
      sa.KP[l] = p.KP[l];
    }
    sa.y = A2;
    sa.copies = (int)copies;
    if (sa.KP[0] != 96 || sa.KP[1] != 288 || sa.KP[2] != 288 || sa.KP[3] != 288 || sa.KP[4] != 608)
      return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_rb_stage1, dim3((unsigned)copies), dim3(kRbFusedThreads), kRbStage1Lds, st, sa);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  {
    RbStage3Args sa{};
    sa.x = A2;
    for (int l = 0; l < 2; ++l) {
      sa.w[l] = reinterpret_cast<const unsigned short*>(ws + p.w[5 + l]);
      sa.bias[l] = reinterpret_cast<const float*>(ws + p.bias[5 + l]);
      sa.KP[l] = p.KP[5 + l];
    }
    sa.feat = feat;
    sa.copies = (int)copies;
    if (sa.KP[0] != 576 || sa.KP[1] != 1216) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_rb_stage3, dim3((unsigned)copies), dim3(kRbFusedThreads), kRbStage3Lds, st, sa);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_rb_head, dim3(n), dim3(128), 0, st, feat, params + kRbFc1W, params + kRbFc1B,
                     params + kRbFc2W, params + kRbFc2B, n, logits, probs);
  return hipGetLastError();
}

hipError_t prepare_rb_attributes() {
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_rb_stage1),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)kRbStage1Lds);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_rb_stage3),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)kRbStage3Lds);
}

hipError_t launch_rb_extract(const RbExtractArgs& a, bool f32, hipStream_t st) {
  const int64_t total = (int64_t)a.n * 3 * 32 * 32;
  const dim3 grid((unsigned)((total + 255) / 256));
  if (f32) hipLaunchKernelGGL(k_rb_extract<float>, grid, dim3(256), 0, st, a);
  else hipLaunchKernelGGL(k_rb_extract<double>, grid, dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace sfft
