// Geometry and launch plan of the stamp Gram kernels (host and device).
#pragma once

#include "layout.hpp"

namespace sfft {

constexpr int kStT = 64;                  // Gram tile side
constexpr int kStThreads = 512;           // 8 waves per workgroup
constexpr int kStMaxPlanes = 32;          // kernel + background planes + S'
constexpr int kStMaxLds = 159 * 1024;     // dynamic LDS limit (the CU has 160 KiB; static use is small)
constexpr size_t kStPartialsOffset = 256; // after the status flags
constexpr int kStMaxSize = 127;
constexpr int kStMaxStamps = 1 << 16;

struct StampGeom {
  int size, half, rowpad, kchunks;   // stamp side, side/2, row length padded to 8, 32-pixel chunks
  int L, r, nK, nB, N, Naug, nt;     // Naug = N + 1 (S' column); nt = tiles per side
  int hrows, crows, pitch;           // LDS plane rows (halo / compact) and words per row
  int halo_dw, comp_dw;              // words of one halo / compact plane (hi and lo halves)
};

inline StampGeom make_stamp_geom(const sfft_desc& d, int size) {
  StampGeom g{};
  g.size = size;
  g.half = size / 2;
  g.rowpad = (size + 7) / 8 * 8;
  g.kchunks = (size * g.rowpad + 31) / 32;
  g.L = d.L;
  g.r = (d.L - 1) / 2;
  g.nK = (d.dk + 1) * (d.dk + 2) / 2;
  g.nB = (d.db + 1) * (d.db + 2) / 2;
  g.N = g.nK * d.L * d.L + g.nB;
  g.Naug = g.N + 1;
  g.nt = (g.Naug + kStT - 1) / kStT;
  const int ymax = (g.kchunks * 32 - 8) / g.rowpad;      // last pixel row a chunk touches
  g.hrows = ymax + 2 * g.r + 1;
  g.crows = ymax + 1;
  g.pitch = g.rowpad / 2 + g.r + 1;
  g.halo_dw = 4 * g.hrows * g.pitch;                     // (hi, lo) x (two shifted copies)
  g.comp_dw = 2 * g.crows * g.pitch;                     // (hi, lo)
  return g;
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
  size_t ws_bytes;      // flags + partial tiles
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
  // stamp groups: minimise (rounds of resident workgroups) x (stamps per group)
  const int per_cu = p.lds_bytes > 0 ? (int)((size_t)kStMaxLds / p.lds_bytes) : 1;
  const int slots = (num_cus > 0 ? num_cus : 256) * (per_cu < 1 ? 1 : (per_cu > 2 ? 2 : per_cu));
  int best = 1;
  long best_cost = -1;
  for (int ng = 1; ng <= nst && ng <= 64; ++ng) {
    const long rounds = ((long)p.ntri * ng + slots - 1) / slots;
    const long cost = rounds * ((nst + ng - 1) / ng);
    if (best_cost < 0 || cost < best_cost) { best_cost = cost; best = ng; }
  }
  p.ngroups = best;
  p.ws_bytes = kStPartialsOffset + sizeof(double) * (size_t)best * p.ntri * kStT * kStT;
  return p;
}

}  // namespace sfft
