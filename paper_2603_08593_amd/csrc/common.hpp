// Shared device helpers of the SFFT library: complex arithmetic, in-register
// small DFTs (radix 2/4/8/16, either sign), block reductions, launch checks.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "sfft.h"

namespace sfft {

template <typename T>
struct __attribute__((aligned(2 * sizeof(T)))) cx {
  T re, im;
};

template <typename T>
__device__ __forceinline__ cx<T> cadd(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ cx<T> csub(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__device__ __forceinline__ cx<T> cscale(cx<T> a, T s) { return {a.re * s, a.im * s}; }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// conj(a) * b
template <typename T>
__device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
  return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
// acc += conj(a) * b
template <typename T>
__device__ __forceinline__ void cmac_conj(cx<T>& acc, cx<T> a, cx<T> b) {
  acc.re = fma(a.re, b.re, fma(a.im, b.im, acc.re));
  acc.im = fma(a.re, b.im, fma(-a.im, b.re, acc.im));
}
template <typename T>
__device__ __forceinline__ cx<T> cconj(cx<T> a) { return {a.re, -a.im}; }
// multiply by -i (forward) or +i (inverse)
template <typename T, bool INV>
__device__ __forceinline__ cx<T> rot90(cx<T> a) {
  return INV ? cx<T>{-a.im, a.re} : cx<T>{a.im, -a.re};
}

// ---------------------------------------------------------------------------
// In-register DFTs, X_k = sum_n v_n exp(-+2 pi i n k / R), unscaled.
// INV = false: forward sign (-), INV = true: inverse sign (+).
// ---------------------------------------------------------------------------

template <typename T, bool INV>
__device__ __forceinline__ void dft2(cx<T>& a, cx<T>& b) {
  cx<T> t = a;
  a = cadd(t, b);
  b = csub(t, b);
}

template <typename T, bool INV>
__device__ __forceinline__ void dft4(cx<T>& a0, cx<T>& a1, cx<T>& a2, cx<T>& a3) {
  cx<T> t0 = cadd(a0, a2), t1 = csub(a0, a2);
  cx<T> t2 = cadd(a1, a3), t3 = rot90<T, INV>(csub(a1, a3));
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  a1 = cadd(t1, t3);
  a3 = csub(t1, t3);
}

// multiply by w8^k, w8 = exp(-+2 pi i / 8)
template <typename T, bool INV, int K>
__device__ __forceinline__ cx<T> w8(cx<T> a) {
  const T h = (T)0.70710678118654752440084436210485;
  if (K == 0) return a;
  if (K == 2) return rot90<T, INV>(a);
  if (K == 1) return INV ? cx<T>{(a.re - a.im) * h, (a.re + a.im) * h}
                         : cx<T>{(a.re + a.im) * h, (a.im - a.re) * h};
  // K == 3
  return INV ? cx<T>{-(a.re + a.im) * h, (a.re - a.im) * h}
             : cx<T>{(a.im - a.re) * h, -(a.re + a.im) * h};
}

template <typename T, bool INV>
__device__ __forceinline__ void dft8(cx<T>* v) {
  // even / odd split
  cx<T> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  cx<T> o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4<T, INV>(e0, e1, e2, e3);
  dft4<T, INV>(o0, o1, o2, o3);
  o1 = w8<T, INV, 1>(o1);
  o2 = w8<T, INV, 2>(o2);
  o3 = w8<T, INV, 3>(o3);
  v[0] = cadd(e0, o0); v[4] = csub(e0, o0);
  v[1] = cadd(e1, o1); v[5] = csub(e1, o1);
  v[2] = cadd(e2, o2); v[6] = csub(e2, o2);
  v[3] = cadd(e3, o3); v[7] = csub(e3, o3);
}

template <typename T, bool INV>
__device__ __forceinline__ void dft16(cx<T>* v) {
  cx<T> e[8], o[8];
#pragma unroll
  for (int n = 0; n < 8; ++n) { e[n] = v[2 * n]; o[n] = v[2 * n + 1]; }
  dft8<T, INV>(e);
  dft8<T, INV>(o);
  // w16^k = cos(2 pi k / 16) -+ i sin(2 pi k / 16)
  const T c1 = (T)0.92387953251128675612818318939679;
  const T s1 = (T)0.38268343236508977172845998403040;
  const T h = (T)0.70710678118654752440084436210485;
  const T sg = INV ? (T)1 : (T)-1;
  const cx<T> w[8] = {{(T)1, (T)0}, {c1, sg * s1}, {h, sg * h}, {s1, sg * c1},
                      {(T)0, sg}, {-s1, sg * c1}, {-h, sg * h}, {-c1, sg * s1}};
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    cx<T> t = (k == 0) ? o[k] : cmul(o[k], w[k]);
    v[k] = cadd(e[k], t);
    v[k + 8] = csub(e[k], t);
  }
}

template <typename T, bool INV>
__device__ __forceinline__ void dft3(cx<T>* v) {
  const T hs = (T)0.86602540378443864676372317075294;   // sin(2 pi / 3)
  const cx<T> t1 = cadd(v[1], v[2]);
  const cx<T> m = {v[0].re - (T)0.5 * t1.re, v[0].im - (T)0.5 * t1.im};
  const cx<T> d = csub(v[1], v[2]);
  // forward: -i hs d; inverse: +i hs d
  const cx<T> t2 = INV ? cx<T>{-hs * d.im, hs * d.re} : cx<T>{hs * d.im, -hs * d.re};
  v[0] = cadd(v[0], t1);
  v[1] = cadd(m, t2);
  v[2] = csub(m, t2);
}

template <typename T, bool INV>
__device__ __forceinline__ void dft5(cx<T>* v) {
  const T c1 = (T)0.30901699437494742410229341718282;    // cos(2 pi / 5)
  const T c2 = (T)-0.80901699437494742410229341718282;   // cos(4 pi / 5)
  const T s1 = (T)0.95105651629515357211643933337938;    // sin(2 pi / 5)
  const T s2 = (T)0.58778525229247312916870595463907;    // sin(4 pi / 5)
  const cx<T> b1 = cadd(v[1], v[4]), b2 = cadd(v[2], v[3]);
  const cx<T> d1 = csub(v[1], v[4]), d2 = csub(v[2], v[3]);
  const cx<T> a0 = v[0];
  const cx<T> p1 = {a0.re + c1 * b1.re + c2 * b2.re, a0.im + c1 * b1.im + c2 * b2.im};
  const cx<T> p2 = {a0.re + c2 * b1.re + c1 * b2.re, a0.im + c2 * b1.im + c1 * b2.im};
  const cx<T> q1 = {s1 * d1.re + s2 * d2.re, s1 * d1.im + s2 * d2.im};
  const cx<T> q2 = {s2 * d1.re - s1 * d2.re, s2 * d1.im - s1 * d2.im};
  // forward: X1 = p1 - i q1, X4 = p1 + i q1, X2 = p2 - i q2, X3 = p2 + i q2
  const cx<T> iq1 = INV ? cx<T>{-q1.im, q1.re} : cx<T>{q1.im, -q1.re};
  const cx<T> iq2 = INV ? cx<T>{-q2.im, q2.re} : cx<T>{q2.im, -q2.re};
  v[0] = cadd(a0, cadd(b1, b2));
  v[1] = cadd(p1, iq1);
  v[4] = csub(p1, iq1);
  v[2] = cadd(p2, iq2);
  v[3] = csub(p2, iq2);
}

template <typename T, int R, bool INV>
__device__ __forceinline__ void dft_r(cx<T>* v) {
  if constexpr (R == 2) dft2<T, INV>(v[0], v[1]);
  else if constexpr (R == 3) dft3<T, INV>(v);
  else if constexpr (R == 5) dft5<T, INV>(v);
  else if constexpr (R == 4) dft4<T, INV>(v[0], v[1], v[2], v[3]);
  else if constexpr (R == 8) dft8<T, INV>(v);
  else if constexpr (R == 16) dft16<T, INV>(v);
}

// ---------------------------------------------------------------------------
// Reductions (fixed order: results are bit-reproducible run to run)
// ---------------------------------------------------------------------------

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum of `v` over the block; every thread gets the result. `scratch` holds
// at least blockDim.x / 64 doubles. Contains __syncthreads.
__device__ __forceinline__ double block_sum(double v, double* scratch) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) scratch[wid] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < nw; ++w) s += scratch[w];
  return s;
}

__device__ __forceinline__ bool is_finite_d(double v) { return (v - v) == 0.0; }

template <typename T>
__device__ __forceinline__ double load_pix(const void* p, int64_t idx) {
  return (double)static_cast<const T*>(p)[idx];
}

// ---------------------------------------------------------------------------
// Virtual block index: a kernel body sees (x, y) within its own grid
// (nx, ny); the single-problem kernel passes blockIdx / gridDim, the batched
// kernel maps its flat block index to (item, local block) through a table of
// per-item block ranges.
// ---------------------------------------------------------------------------

struct VB {
  int x, y, nx, ny;
};

__device__ __forceinline__ VB vb_grid() {
  return VB{(int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x, (int)gridDim.y};
}

struct BatchTab {
  int start, nx, ny, pad;   // first flat block of the item, its grid
};

// Locates the item of flat block blockIdx.x (tab sorted by start, n >= 1).
// Returns false for blocks past the item's own grid.
__device__ __forceinline__ bool batch_locate(const BatchTab* tab, int n, int& item, VB& vb) {
  const int b = (int)blockIdx.x;
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tab[mid].start <= b) lo = mid;
    else hi = mid - 1;
  }
  item = lo;
  const int local = b - tab[lo].start;
  const int nx = tab[lo].nx, ny = tab[lo].ny;
  vb = VB{local % nx, local / nx, nx, ny};
  return local < nx * ny;
}

// polynomial monomial tables: exponent pairs of the layout order, up to D = 4
struct MonoTable {
  int n;
  int a[15];
  int b[15];
};

inline MonoTable make_monos(int D) {
  MonoTable t{};
  t.n = 0;
  for (int d = 0; d <= D; ++d)
    for (int b = 0; b <= d; ++b) {
      t.a[t.n] = d - b;
      t.b[t.n] = b;
      ++t.n;
    }
  return t;
}

inline int n_mono(int D) { return (D + 1) * (D + 2) / 2; }

}  // namespace sfft
