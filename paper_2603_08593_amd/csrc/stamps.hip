// sfft_build_system_stamps: the normal equations of the kernel fit restricted
// to square star stamps, with the Gram sums on matrix cores (precision form:
// products of FP32 operands split into two bfloat16 halves, accumulated in
// FP32 inside a workgroup and in FP64 across workgroups).
//
// The design row of a stamp pixel x holds p_i(x - d) R'(x - d) for every
// kernel unknown (i, d) and q_c(x) for every background unknown; appending
// S'(x) as one more column makes G_s = A^T A and h_s = A^T S' two parts of
// one Gram matrix of the augmented [A | S'] (paper Sec. 1: delta-basis kernel
// by least squares; the stamp selection is the usual star-based SFFT mode).
//
// Work decomposition: the augmented Gram (N+1 columns, padded to 64-tiles) is
// cut into upper-triangular 64 x 64 tiles; workgroup (tile, group) sums the
// tile over one group of stamps. For each stamp it fills LDS with the few
// source planes its 128 unknowns read (kernel planes p_i R' over the stamp
// plus an r-pixel halo, stored twice with a one-element shift so every 8-pixel
// operand run is a 4-byte-aligned read; background and S' planes over the
// stamp only), as bfloat16 (hi, lo) pairs. Each of the 8 waves accumulates the
// whole 64 x 64 tile over every 8th 32-pixel chunk with
// v_mfma_f32_16x16x32_bf16 (hi*hi + hi*lo + lo*hi); the waves' tiles are
// added in FP64 in a fixed order and written as one partial per group; a
// second kernel adds the groups in order and scatters G and h.
#include "common.hpp"
#include "layout.hpp"
#include "stamps.hpp"

namespace sfft {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

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

template <typename TIN>
__global__ __launch_bounds__(kStThreads) void k_stamp_gram(StampArgs a) {
  extern __shared__ __align__(16) unsigned lds[];
  __shared__ int slot_off[kStMaxPlanes];
  __shared__ int used[kStMaxPlanes];
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
    int o = 0;
    for (int p = 0; p < nplanes; ++p) {
      slot_off[p] = o;
      if (used[p]) o += p < g.nK ? g.halo_dw : g.comp_dw;
    }
  }
  __syncthreads();

  // ---- per-lane operand bases (dwords): hi and lo copy for each 16-row block
  const int l16 = lane & 15, grp = lane >> 4;
  int abase[4], alo[4], bbase[4], blo[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const int u = (side == 0 ? r0 : c0) + 16 * m + l16;
      int p, dy, dx;
      decode_unknown(g, u, p, dy, dx);
      int base, lo;
      if (p < g.nK) {
        const int par = (g.r - dx) & 1;
        base = slot_off[p] + par * g.hrows * g.pitch + (g.r - dy) * g.pitch + (g.r - dx - par) / 2;
        lo = 2 * g.hrows * g.pitch;
      } else {
        base = slot_off[p];
        lo = g.crows * g.pitch;
      }
      if (side == 0) { abase[m] = base; alo[m] = lo; }
      else { bbase[m] = base; blo[m] = lo; }
    }
  }
  const bool diag = ti == tj;

  floatx4 acc[4][4];
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int n = 0; n < 4; ++n) acc[m][n] = floatx4{0.f, 0.f, 0.f, 0.f};

  const int s_begin = (int)((int64_t)group * a.nst / a.ngroups);
  const int s_end = (int)((int64_t)(group + 1) * a.nst / a.ngroups);
  int nonfinite = 0;
  for (int s = s_begin; s < s_end; ++s) {
    const int cx = a.centers[2 * s], cy = a.centers[2 * s + 1];
    // ---- fill the used planes for this stamp
    for (int p = 0; p < nplanes; ++p) {
      if (!used[p]) continue;
      unsigned* hi = lds + slot_off[p];
      if (p < g.nK) {
        // halo plane: element (yy, xx) is pixel (cy - half - r + yy, cx - half - r + xx);
        // copy 0 word m = (e[2m], e[2m+1]), copy 1 word m = (e[2m+1], e[2m+2])
        unsigned* lo = hi + 2 * g.hrows * g.pitch;
        const int y0 = cy - g.half - g.r, x0 = cx - g.half - g.r;
        for (int i = tid; i < g.hrows * g.pitch; i += kStThreads) {
          const int yy = i / g.pitch, m = i - yy * g.pitch;
          const int Y = wrap(y0 + yy, a.H);
          float v[3];
#pragma unroll
          for (int e = 0; e < 3; ++e) v[e] = plane_value<TIN>(a, p, Y, wrap(x0 + 2 * m + e, a.W), g.nK, g.nB);
          unsigned h[3], l[3];
#pragma unroll
          for (int e = 0; e < 3; ++e) {
            nonfinite |= !(v[e] - v[e] == 0.0f);
            h[e] = bf16_bits(v[e]);
            l[e] = bf16_bits(v[e] - __builtin_bit_cast(float, h[e] << 16));
          }
          hi[i] = h[0] | (h[1] << 16);
          hi[g.hrows * g.pitch + i] = h[1] | (h[2] << 16);
          lo[i] = l[0] | (l[1] << 16);
          lo[g.hrows * g.pitch + i] = l[1] | (l[2] << 16);
        }
      } else {
        // compact plane: element (yy, xx) is pixel (cy - half + yy, cx - half + xx)
        unsigned* lo = hi + g.crows * g.pitch;
        const int y0 = cy - g.half, x0 = cx - g.half;
        for (int i = tid; i < g.crows * g.pitch; i += kStThreads) {
          const int yy = i / g.pitch, m = i - yy * g.pitch;
          const int Y = wrap(y0 + yy, a.H);
          float v[2];
#pragma unroll
          for (int e = 0; e < 2; ++e) v[e] = plane_value<TIN>(a, p, Y, wrap(x0 + 2 * m + e, a.W), g.nK, g.nB);
          unsigned h[2], l[2];
#pragma unroll
          for (int e = 0; e < 2; ++e) {
            nonfinite |= !(v[e] - v[e] == 0.0f);
            h[e] = bf16_bits(v[e]);
            l[e] = bf16_bits(v[e] - __builtin_bit_cast(float, h[e] << 16));
          }
          hi[i] = h[0] | (h[1] << 16);
          lo[i] = l[0] | (l[1] << 16);
        }
      }
    }
    __syncthreads();

    // ---- Gram over this stamp's 32-pixel chunks (every 8th chunk per wave)
    for (int ch = wave; ch < g.kchunks; ch += kStThreads / 64) {
      const int kk = ch * 32 + grp * 8;
      const int y = kk / g.rowpad, xs = kk - y * g.rowpad;
      const int pix = y * g.pitch + (xs >> 1);
      // valid elements of this lane's 8-pixel run: x < size and y < size
      const int nv = (y < g.size) ? min(max(g.size - xs, 0), 8) : 0;
      unsigned msk[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int e0 = 2 * q;
        msk[q] = (e0 < nv ? 0x0000FFFFu : 0u) | (e0 + 1 < nv ? 0xFFFF0000u : 0u);
      }
      bf16x8 ah[4], al[4], bh[4], bl[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const unsigned* ph = lds + abase[m] + pix;
        const unsigned* pl = ph + alo[m];
        unsigned th[4] = {ph[0], ph[1], ph[2], ph[3]};
        unsigned tl[4] = {pl[0], pl[1], pl[2], pl[3]};
        ah[m] = __builtin_bit_cast(bf16x8, th);
        al[m] = __builtin_bit_cast(bf16x8, tl);
        if (!diag) {
          const unsigned* qh = lds + bbase[m] + pix;
          const unsigned* ql = qh + blo[m];
#pragma unroll
          for (int q = 0; q < 4; ++q) { th[q] = qh[q]; tl[q] = ql[q]; }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) { th[q] &= msk[q]; tl[q] &= msk[q]; }
        bh[m] = __builtin_bit_cast(bf16x8, th);
        bl[m] = __builtin_bit_cast(bf16x8, tl);
      }
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int n = 0; n < 4; ++n) {
          acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[m], bh[n], acc[m][n], 0, 0, 0);
          acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[m], bl[n], acc[m][n], 0, 0, 0);
          acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[m], bh[n], acc[m][n], 0, 0, 0);
        }
    }
    __syncthreads();
  }
  if (nonfinite) atomicOr(&a.flags[0], 1);

  // ---- add the 8 waves' tiles in FP64, fixed order, into LDS; write the partial
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
            const double v = (double)acc[m][n][q];
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
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_stamp_gram<float>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, kStMaxLds);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_stamp_gram<double>),
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
  a.flags = reinterpret_cast<int*>(ws);
  hipLaunchKernelGGL(k_stamp_clear, dim3(1), dim3(64), 0, st, a.flags, 64);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  prof_begin(pf, SFFT_PROF_STAMP_GRAM, st);
  if (d.image_dtype == SFFT_F32)
    hipLaunchKernelGGL(k_stamp_gram<float>, dim3(pl.ntri * pl.ngroups), dim3(kStThreads), pl.lds_bytes, st, a);
  else
    hipLaunchKernelGGL(k_stamp_gram<double>, dim3(pl.ntri * pl.ngroups), dim3(kStThreads), pl.lds_bytes, st, a);
  prof_end(pf, SFFT_PROF_STAMP_GRAM, st);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_stamp_finalize, dim3(pl.ntri), dim3(256), 0, st, (const double*)a.partials,
                     pl.ngroups, pl.ntri, g.nt, g.N, G, hv);
  return hipGetLastError();
}

}  // namespace sfft
