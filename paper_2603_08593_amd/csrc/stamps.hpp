// Geometry and launch plan of the stamp Gram kernels (host and device).
#pragma once

#include "layout.hpp"

namespace sfft {

constexpr int kStT = 64;                  // Gram tile side
constexpr int kStThreads = 256;           // 4 waves per workgroup, one per SIMD
constexpr int kStParts = 3;               // bfloat16 terms per FP32 operand (hi, mid, lo)
constexpr int kStFlushChunks = 8;         // FP32 accumulation run before each FP64 flush
constexpr int kStMaxPlanes = 32;          // kernel + background planes + S'
constexpr int kStMaxLds = 159 * 1024;     // dynamic LDS limit (the CU has 160 KiB; static use is small)
constexpr size_t kStPartialsOffset = 256; // after the status flags
constexpr int kStMaxSize = 127;
constexpr int kStMaxStamps = 1 << 16;

// Operand layout. The K index of the Gram runs over stamp pixels; a stamp
// row is padded to `rowpad` (a multiple of 8) pixels and stored as P =
// rowpad / 2 words, word m holding the pixels x = m (low half) and x = m + P
// (high half) as bfloat16. A 16-lane group of an MFMA operand reads 4
// consecutive words (8 pixels). A shift of the source plane by dx moves both
// halves of every word together, so any kernel offset reads whole words.
// Kernel planes p_i R' carry an r-pixel halo (hrows x hpitch words, word w
// holding x = w - r and w - r + P), background and S' planes only the stamp
// (crows x cpitch words, zero outside it). Each plane holds kStParts copies
// (hi, mid, lo) one after the other.
struct StampGeom {
  int size, half, rowpad, P, kchunks;   // kchunks: 16-word (32-pixel) chunks per stamp
  int L, r, nK, nB, N, Naug, nt;        // Naug = N + 1 (S' column); nt = tiles per side
  int ymax, hrows, hpitch, crows, cpitch;
  int halo_dw, comp_dw;                 // words of one plane (all parts), multiples of 4
  int64_t stamp_dw;                     // words of every plane of one stamp
};

inline int round4(int v) { return (v + 3) / 4 * 4; }

inline StampGeom make_stamp_geom(const sfft_desc& d, int size) {
  StampGeom g{};
  g.size = size;
  g.half = size / 2;
  g.rowpad = (size + 7) / 8 * 8;
  g.P = g.rowpad / 2;
  g.kchunks = (size * g.P + 15) / 16;
  g.L = d.L;
  g.r = (d.L - 1) / 2;
  g.nK = (d.dk + 1) * (d.dk + 2) / 2;
  g.nB = (d.db + 1) * (d.db + 2) / 2;
  g.N = g.nK * d.L * d.L + g.nB;
  g.Naug = g.N + 1;
  g.nt = (g.Naug + kStT - 1) / kStT;
  g.ymax = (g.kchunks * 16 - 1) / g.P;                   // last stamp row a chunk touches
  g.hrows = g.ymax + 2 * g.r + 1;
  g.hpitch = g.P + 2 * g.r;
  g.crows = g.ymax + 1;
  g.cpitch = g.P;
  g.halo_dw = round4(kStParts * g.hrows * g.hpitch);
  g.comp_dw = round4(kStParts * g.crows * g.cpitch);
  g.stamp_dw = (int64_t)g.nK * g.halo_dw + (int64_t)(g.nB + 1) * g.comp_dw;
  return g;
}

// word offset of plane p inside one stamp's block
__host__ __device__ inline int64_t stamp_plane_offset(const StampGeom& g, int p) {
  return p < g.nK ? (int64_t)p * g.halo_dw : (int64_t)g.nK * g.halo_dw + (int64_t)(p - g.nK) * g.comp_dw;
}

// plane of unknown u (host copy of the device decode)
inline int stamp_plane_of(const StampGeom& g, int u) {
  const int L2 = g.L * g.L;
  if (u < g.nK * L2) return u / L2;
  if (u < g.N) return g.nK + (u - g.nK * L2);
  return g.nK + g.nB;
}

struct StampPlan {
  int ntri, ngroups;
  size_t lds_bytes;     // largest LDS need over all tiles
  size_t planes_off;    // byte offset of the split planes in the workspace
  size_t ws_bytes;      // flags + partial tiles + split planes
};

inline StampPlan make_stamp_plan(const StampGeom& g, int nst, int num_cus) {
  StampPlan p{};
  p.ntri = g.nt * (g.nt + 1) / 2;
  size_t worst = 0;
  const int nplanes = g.nK + g.nB + 1;
  for (int ti = 0; ti < g.nt; ++ti)
    for (int tj = ti; tj < g.nt; ++tj) {
      bool used[kStMaxPlanes] = {};
      for (int k = 0; k < kStT; ++k) {
        used[stamp_plane_of(g, ti * kStT + k)] = true;
        used[stamp_plane_of(g, tj * kStT + k)] = true;
      }
      size_t w = 0;
      for (int q = 0; q < nplanes; ++q)
        if (used[q]) w += (size_t)(q < g.nK ? g.halo_dw : g.comp_dw);
      if (w > worst) worst = w;
    }
  p.lds_bytes = 4 * worst;
  if (p.lds_bytes < sizeof(double) * kStT * kStT) p.lds_bytes = sizeof(double) * kStT * kStT;
  // one workgroup per CU (its registers fill the CU's four SIMDs); stamp
  // groups minimise (rounds of resident workgroups) x (stamps per group)
  const int slots = num_cus > 0 ? num_cus : 256;
  int best = 1;
  long best_cost = -1;
  for (int ng = 1; ng <= nst && ng <= 64; ++ng) {
    const long rounds = ((long)p.ntri * ng + slots - 1) / slots;
    const long cost = rounds * ((nst + ng - 1) / ng);
    if (best_cost < 0 || cost < best_cost) { best_cost = cost; best = ng; }
  }
  p.ngroups = best;
  p.planes_off = align256(kStPartialsOffset + sizeof(double) * (size_t)best * p.ntri * kStT * kStT);
  p.ws_bytes = p.planes_off + sizeof(unsigned) * (size_t)nst * (size_t)g.stamp_dw;
  return p;
}

}  // namespace sfft
