// sfft_build_system_stamps: the normal equations of the kernel fit restricted
// to square star stamps, with the Gram sums on matrix cores (precision form:
// every FP32 operand split exactly into three bfloat16 terms, the six term
// products of order <= 2 accumulated in FP32 over short runs and in FP64
// beyond them).
//
// The design row of a stamp pixel x holds p_i(x - d) R'(x - d) for every
// kernel unknown (i, d) and q_c(x) for every background unknown; appending
// S'(x) as one more column makes G_s = A^T A and h_s = A^T S' two parts of
// one Gram matrix of the augmented [A | S'] (paper Sec. 1: delta-basis kernel
// by least squares; the stamp selection is the usual star-based SFFT mode).
//
// Two kernels. k_stamp_planes evaluates every source plane of every stamp
// once (kernel planes p_i R' with an r-pixel halo, background planes and S'
// over the stamp), splits each FP32 value into (hi, mid, lo) bfloat16 terms
// and stores them in the operand layout of stamps.hpp (pairs of pixels
// x, x + P per word, so that every kernel offset reads whole words).
// k_stamp_gram cuts the augmented Gram (N + 1 columns, padded to 64-tiles)
// into upper-triangular 64 x 64 tiles; workgroup (tile, group) sums its tile
// over one group of stamps: per stamp it copies the planes its 128 unknowns
// read into LDS, then each of its 4 waves accumulates the whole tile over
// every 4th 32-pixel chunk with v_mfma_f32_16x16x32_bf16 (hi*hi, hi*mid,
// mid*hi, hi*lo, lo*hi, mid*mid), flushing its FP32 accumulators into FP64
// ones every 8 chunks; the waves' tiles are added in FP64 in a fixed order
// and written as one partial per group; a third kernel adds the groups in
// order and scatters G and h.
#include "common.hpp"
#include "layout.hpp"
#include "stamps.hpp"

namespace sfft {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

struct StampArgs {
  const void* R;
  const void* S;
  int64_t ld;
  const int32_t* centers;   // [nst][2] = (x, y)
  int nst, W, H, DK, DB;
  double cR, cS, sx, sy;
  StampGeom g;
  int ngroups, ntri;
  double* partials;         // [ngroups][ntri][64][64]
  unsigned* planes;         // [nst][stamp_dw] split planes
  int* flags;
};

__global__ void k_stamp_clear(int* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// round-to-nearest-even FP32 -> bfloat16 bits (finite inputs)
__device__ __forceinline__ unsigned bf16_bits(float v) {
  const unsigned u = __builtin_bit_cast(unsigned, v);
  return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}

__device__ __forceinline__ float bf16_value(unsigned b) { return __builtin_bit_cast(float, b << 16); }

// v = hi + mid + lo exactly (every difference below is exact in FP32)
__device__ __forceinline__ void split3(float v, unsigned (&t)[kStParts]) {
  t[0] = bf16_bits(v);
  const float r1 = v - bf16_value(t[0]);
  t[1] = bf16_bits(r1);
  t[2] = bf16_bits(r1 - bf16_value(t[1]));
}

// FP32 value of plane p at image pixel (Y, X) (already wrapped)
template <typename TIN>
__device__ __forceinline__ float plane_value(const StampArgs& a, int p, int Y, int X, int nK, int nB) {
  const double xt = (double)X * a.sx - 1.0, yt = (double)Y * a.sy - 1.0;
  if (p == nK + nB) return (float)((double)static_cast<const TIN*>(a.S)[(int64_t)Y * a.ld + X] - a.cS);
  int q = p < nK ? p : p - nK;
  int d = 0;
  while ((d + 1) * (d + 2) / 2 <= q) ++d;
  const int b = q - d * (d + 1) / 2, ea = d - b;
  double m = 1.0;
  for (int t = 0; t < ea; ++t) m *= xt;
  for (int t = 0; t < b; ++t) m *= yt;
  if (p < nK) m *= (double)static_cast<const TIN*>(a.R)[(int64_t)Y * a.ld + X] - a.cR;
  return (float)m;
}

__device__ __forceinline__ int wrap(int v, int n) {
  v %= n;
  return v < 0 ? v + n : v;
}

// Split planes of one (stamp, plane) per workgroup. Kernel plane word (yy, w)
// holds the pixels (cy - half - r + yy, cx - half + w - r) and (.., + P);
// compact plane word (y, m) the pixels (cy - half + y, cx - half + m) and
// (.., + P), zero outside the stamp.
template <typename TIN>
__global__ __launch_bounds__(256) void k_stamp_planes(StampArgs a) {
  const StampGeom& g = a.g;
  const int s = blockIdx.x, p = blockIdx.y;
  const int cx = a.centers[2 * s], cy = a.centers[2 * s + 1];
  unsigned* out = a.planes + (int64_t)s * g.stamp_dw + stamp_plane_offset(g, p);
  const bool halo = p < g.nK;
  const int rows = halo ? g.hrows : g.crows, pitch = halo ? g.hpitch : g.cpitch;
  const int nw = rows * pitch;
  const int ry = halo ? g.r : 0, rx = halo ? g.r : 0;
  int nonfinite = 0;
  for (int i = threadIdx.x; i < nw; i += 256) {
    const int yy = i / pitch, w = i - yy * pitch;
    const int y = yy - ry;                      // stamp row
    const int x0 = w - rx, x1 = x0 + g.P;       // stamp columns of the two halves
    const int Y = wrap(cy - g.half + y, a.H);
    float v0 = 0.f, v1 = 0.f;
    if (halo || (y < g.size && x0 < g.size)) v0 = plane_value<TIN>(a, p, Y, wrap(cx - g.half + x0, a.W), g.nK, g.nB);
    if (halo || (y < g.size && x1 < g.size)) v1 = plane_value<TIN>(a, p, Y, wrap(cx - g.half + x1, a.W), g.nK, g.nB);
    nonfinite |= !(v0 - v0 == 0.0f) || !(v1 - v1 == 0.0f);
    unsigned t0[kStParts], t1[kStParts];
    split3(v0, t0);
    split3(v1, t1);
#pragma unroll
    for (int q = 0; q < kStParts; ++q) out[q * nw + i] = t0[q] | (t1[q] << 16);
  }
  if (nonfinite) atomicOr(&a.flags[0], 1);
}

// plane of unknown u, and its kernel offset (dy, dx) (0 for non-kernel planes)
__device__ __forceinline__ void decode_unknown(const StampGeom& g, int u, int& p, int& dy, int& dx) {
  const int L2 = g.L * g.L;
  dy = 0; dx = 0;
  if (u < g.nK * L2) {
    p = u / L2;
    const int d = u - p * L2;
    dy = d / g.L - g.r;
    dx = d - (d / g.L) * g.L - g.r;
  } else if (u < g.N) {
    p = g.nK + (u - g.nK * L2);
  } else {
    p = g.nK + g.nB;          // S' column (u == N) and padding columns
  }
}

__device__ __forceinline__ void tri_tile(int t, int nt, int& ti, int& tj) {
  ti = 0;
  while (t >= nt - ti) { t -= nt - ti; ++ti; }
  tj = ti + t;
}

// operand of one 16-row block: the three split terms of the lane's 4 words
struct Operand {
  bf16x8 t[kStParts];
};

__device__ __forceinline__ void read_operand(const unsigned* lds, int base, int pstride, Operand& o) {
#pragma unroll
  for (int q = 0; q < kStParts; ++q) {
    const unsigned* ptr = lds + base + q * pstride;
    unsigned w[4] = {ptr[0], ptr[1], ptr[2], ptr[3]};
    o.t[q] = __builtin_bit_cast(bf16x8, w);
  }
}

__device__ __forceinline__ void mask_operand(Operand& o, const unsigned (&msk)[4]) {
#pragma unroll
  for (int q = 0; q < kStParts; ++q) {
    unsigned w[4];
    __builtin_memcpy(w, &o.t[q], sizeof w);
#pragma unroll
    for (int j = 0; j < 4; ++j) w[j] &= msk[j];
    o.t[q] = __builtin_bit_cast(bf16x8, w);
  }
}

// acc += sum of the six term products of order <= 2 (smallest first)
__device__ __forceinline__ floatx4 mma6(const Operand& A, const Operand& B, floatx4 acc) {
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.t[1], B.t[1], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.t[0], B.t[2], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.t[2], B.t[0], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.t[0], B.t[1], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.t[1], B.t[0], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.t[0], B.t[0], acc, 0, 0, 0);
  return acc;
}

__global__ __launch_bounds__(kStThreads, 1) void k_stamp_gram(StampArgs a) {
  extern __shared__ __align__(16) unsigned lds[];
  __shared__ int slot_off[kStMaxPlanes];
  __shared__ int used[kStMaxPlanes];
  __shared__ int copy_plane[kStMaxPlanes];
  __shared__ int ncopy;
  const StampGeom& g = a.g;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tile = blockIdx.x % a.ntri, group = blockIdx.x / a.ntri;
  int ti, tj;
  tri_tile(tile, g.nt, ti, tj);
  const int r0 = ti * kStT, c0 = tj * kStT;
  const int nplanes = g.nK + g.nB + 1;

  // ---- planes this tile reads, and their LDS slots
  if (tid < kStMaxPlanes) used[tid] = 0;
  __syncthreads();
  if (tid < 2 * kStT) {
    int p, dy, dx;
    decode_unknown(g, (tid < kStT ? r0 : c0 - kStT) + tid, p, dy, dx);
    used[p] = 1;
  }
  __syncthreads();
  if (tid == 0) {
    int o = 0, n = 0;
    for (int p = 0; p < nplanes; ++p) {
      slot_off[p] = o;
      if (used[p]) {
        o += p < g.nK ? g.halo_dw : g.comp_dw;
        copy_plane[n++] = p;
      }
    }
    ncopy = n;
  }
  __syncthreads();

  // ---- per-lane operand addresses (words, part 0) and part strides
  const int l16 = lane & 15, grp = lane >> 4;
  int abase[4], apitch[4], apst[4], bbase[4], bpitch[4], bpst[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const int u = (side == 0 ? r0 : c0) + 16 * m + l16;
      int p, dy, dx;
      decode_unknown(g, u, p, dy, dx);
      int base, pitch, pst;
      if (p < g.nK) {
        pitch = g.hpitch;
        pst = g.hrows * g.hpitch;
        base = slot_off[p] + (g.r - dy) * pitch + (g.r - dx);
      } else {
        pitch = g.cpitch;
        pst = g.crows * g.cpitch;
        base = slot_off[p];
      }
      if (side == 0) { abase[m] = base; apitch[m] = pitch; apst[m] = pst; }
      else { bbase[m] = base; bpitch[m] = pitch; bpst[m] = pst; }
    }
  }
  const bool diag = ti == tj;

  floatx4 acc[4][4];
  doublex4 acc64[4][4];
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int n = 0; n < 4; ++n) {
      acc[m][n] = floatx4{0.f, 0.f, 0.f, 0.f};
      acc64[m][n] = doublex4{0.0, 0.0, 0.0, 0.0};
    }
  auto flush = [&]() {
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int n = 0; n < 4; ++n) {
#pragma unroll
        for (int q = 0; q < 4; ++q) acc64[m][n][q] += (double)acc[m][n][q];
        acc[m][n] = floatx4{0.f, 0.f, 0.f, 0.f};
      }
  };

  const int s_begin = (int)((int64_t)group * a.nst / a.ngroups);
  const int s_end = (int)((int64_t)(group + 1) * a.nst / a.ngroups);
  for (int s = s_begin; s < s_end; ++s) {
    // ---- copy the used planes of this stamp into LDS: direct global -> LDS
    // loads (16 bytes per lane; lane l of a wave writes its wave's LDS base
    // + 16 l), all of the stamp's issued before one wait, so the copy costs
    // about one memory latency instead of one per 16 KB
    const unsigned* src = a.planes + (int64_t)s * g.stamp_dw;
    for (int c = 0; c < ncopy; ++c) {
      const int p = copy_plane[c];
      const uint4* s4 = reinterpret_cast<const uint4*>(src + stamp_plane_offset(g, p));
      uint4* d4 = reinterpret_cast<uint4*>(lds + slot_off[p]);
      const int n4 = (p < g.nK ? g.halo_dw : g.comp_dw) / 4;
      for (int i0 = 0; i0 < n4; i0 += kStThreads) {
        const int idx = i0 + tid;
        if (idx < n4)
          __builtin_amdgcn_global_load_lds(static_cast<const void*>(s4 + idx),
                                           (__attribute__((address_space(3))) void*)(d4 + i0 + (tid & ~63)), 16, 0,
                                           0);
      }
    }
    __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): this wave's copies have landed
    __syncthreads();

    // ---- Gram over this stamp's 32-pixel chunks (every 4th chunk per wave)
    int it = 0;
    for (int ch = wave; ch < g.kchunks; ch += kStThreads / 64, ++it) {
      const int wi = ch * 16 + grp * 4;
      const int y = wi / g.P, m0 = wi - y * g.P;
      // valid halves of this lane's 4 words: low x = m0 + j, high x = m0 + j + P
      unsigned msk[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const bool row = y < g.size;
        msk[j] = ((row && m0 + j < g.size) ? 0x0000FFFFu : 0u) |
                 ((row && m0 + j + g.P < g.size) ? 0xFFFF0000u : 0u);
      }
      Operand A[4], B[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) read_operand(lds, abase[m] + y * apitch[m] + m0, apst[m], A[m]);
#pragma unroll
      for (int n = 0; n < 4; ++n) {
        if (diag) B[n] = A[n];
        else read_operand(lds, bbase[n] + y * bpitch[n] + m0, bpst[n], B[n]);
        mask_operand(B[n], msk);
      }
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int n = 0; n < 4; ++n) {
          if (diag && m > n) continue;          // below the diagonal of a diagonal tile
          acc[m][n] = mma6(A[m], B[n], acc[m][n]);
        }
      if ((it % kStFlushChunks) == kStFlushChunks - 1) flush();
    }
    if ((it % kStFlushChunks) != 0) flush();
    __syncthreads();
  }

  // ---- add the 4 waves' tiles in FP64, fixed order, into LDS; write the partial
  double* tileacc = reinterpret_cast<double*>(lds);
  for (int w = 0; w < kStThreads / 64; ++w) {
    if (wave == w) {
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int n = 0; n < 4; ++n)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int row = 16 * m + 4 * grp + q, col = 16 * n + l16;
            const double v = acc64[m][n][q];
            tileacc[row * kStT + col] = (w == 0) ? v : tileacc[row * kStT + col] + v;
          }
    }
    __syncthreads();
  }
  double* out = a.partials + ((int64_t)group * a.ntri + tile) * (kStT * kStT);
  for (int i = tid; i < kStT * kStT; i += kStThreads) out[i] = tileacc[i];
}

// G[a][b] = G[b][a] = sum over groups (fixed order) for a <= b < N;
// h[a] from the S' column b == N.
__global__ __launch_bounds__(256) void k_stamp_finalize(const double* partials, int ngroups, int ntri,
                                                        int nt, int N, double* G, double* h) {
  const int tile = blockIdx.x;
  int ti, tj;
  tri_tile(tile, nt, ti, tj);
  for (int i = threadIdx.x; i < kStT * kStT; i += 256) {
    const int a = ti * kStT + i / kStT, b = tj * kStT + i % kStT;
    if (a > b || a >= N || b > N) continue;
    double s = 0.0;
    for (int gi = 0; gi < ngroups; ++gi) s += partials[((int64_t)gi * ntri + tile) * (kStT * kStT) + i];
    if (b == N) {
      h[a] = s;
    } else {
      G[(int64_t)a * N + b] = s;
      G[(int64_t)b * N + a] = s;
    }
  }
}

hipError_t prepare_stamp_attributes() {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_stamp_gram),
                             hipFuncAttributeMaxDynamicSharedMemorySize, kStMaxLds);
}

hipError_t launch_stamps(const sfft_desc& d, const void* R, const void* S, const int32_t* centers,
                         int nst, int size, double* G, double* hv, unsigned char* ws, int num_cus,
                         const Prof* pf, hipStream_t st) {
  const StampGeom g = make_stamp_geom(d, size);
  const StampPlan pl = make_stamp_plan(g, nst, num_cus);
  StampArgs a{};
  a.R = R; a.S = S; a.ld = d.ld; a.centers = centers; a.nst = nst;
  a.W = d.width; a.H = d.height; a.DK = d.dk; a.DB = d.db;
  a.cR = d.ref_pedestal; a.cS = d.sci_pedestal;
  a.sx = d.width > 1 ? 2.0 / (double)(d.width - 1) : 0.0;
  a.sy = d.height > 1 ? 2.0 / (double)(d.height - 1) : 0.0;
  a.g = g;
  a.ngroups = pl.ngroups;
  a.ntri = pl.ntri;
  a.partials = reinterpret_cast<double*>(ws + kStPartialsOffset);
  a.planes = reinterpret_cast<unsigned*>(ws + pl.planes_off);
  a.flags = reinterpret_cast<int*>(ws);
  hipLaunchKernelGGL(k_stamp_clear, dim3(1), dim3(64), 0, st, a.flags, 64);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  prof_begin(pf, SFFT_PROF_STAMP_GRAM, st);
  const dim3 pgrid(nst, g.nK + g.nB + 1);
  if (d.image_dtype == SFFT_F32)
    hipLaunchKernelGGL(k_stamp_planes<float>, pgrid, dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL(k_stamp_planes<double>, pgrid, dim3(256), 0, st, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_stamp_gram, dim3(pl.ntri * pl.ngroups), dim3(kStThreads), pl.lds_bytes, st, a);
  prof_end(pf, SFFT_PROF_STAMP_GRAM, st);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_stamp_finalize, dim3(pl.ntri), dim3(256), 0, st, (const double*)a.partials,
                     pl.ngroups, pl.ntri, g.nt, g.N, G, hv);
  return hipGetLastError();
}

}  // namespace sfft
