// Workspace layout and problem geometry shared by the host API and kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "sfft.h"

namespace sfft {

constexpr int kTP = 128;        // length of the blocked y-correlation FFT
constexpr int kColsPerWG = 4;   // k_x columns per column-pass workgroup
constexpr int kColThreads = 512;
constexpr int kRowThreads = 256;
constexpr int kTile = 64;       // Cholesky tile
constexpr int kSubTX = 64, kSubTY = 32;   // subtract output tile (single-pair launch)
constexpr int kSubTYMin = 16;             // smallest tile height a batch may choose
constexpr int kSubThreads = kSubTX * kSubTY / 8;   // 8 pixels of a row per thread
constexpr int kMaxW = 4096;
// solve synchronisation words: [0, 256) barrier flags, [256, 512) progress
// flags, then 256 64-bit time stamps
constexpr int kSyncWords = 512;
constexpr int kMaxTeam = 128;   // workgroups of one solve
constexpr int kSyncClear = kSyncWords + 2 * 256;

struct Geometry {
  int W, H, L, r, h, DK, DB, nK, nB, N, NKK, NP, nkx, TP, T, nsig;
  int64_t pitchK;     // complex elements per row-spectrum row
  int64_t planeK;     // complex elements per row-spectrum plane
  bool fp32;
  size_t cxsize;      // bytes of one spectrum element
};

inline Geometry make_geometry(const sfft_desc& d) {
  Geometry g{};
  g.W = d.width; g.H = d.height; g.L = d.L; g.r = (d.L - 1) / 2; g.h = d.L - 1;
  g.DK = d.dk; g.DB = d.db;
  g.nK = (d.dk + 1) * (d.dk + 2) / 2;
  g.nB = (d.db + 1) * (d.db + 2) / 2;
  g.N = g.nK * d.L * d.L + g.nB;
  g.NKK = g.nK * (g.nK + 1) / 2;
  g.NP = g.NKK + g.nK;
  g.nkx = d.width / 2 + 1;
  g.TP = kTP;
  g.T = kTP - 2 * g.h;
  g.nsig = d.dk + 2;
  g.pitchK = ((int64_t)g.nkx + 7) / 8 * 8;
  g.planeK = g.pitchK * d.height;
  g.fp32 = d.compute == SFFT_COMPUTE_FP32;
  g.cxsize = g.fp32 ? 8 : 16;
  return g;
}

struct BuildPlan {
  const void* twW;      // exp(-2 pi i m / W) in the build precision
  const void* twW64;    // same table in FP64
  const void* tw128;    // exp(-2 pi i m / 128) in the build precision
  int num_cus;
  int radix_order;      // row FFT stage order: 0 largest radix first, 1 reversed
};

// caller-provided timing events per sfft_prof_slot
struct Prof {
  void* start[SFFT_PROF_MAX];
  void* stop[SFFT_PROF_MAX];
};

inline void prof_begin(const Prof* p, int slot, hipStream_t st) {
  if (p && p->start[slot]) (void)hipEventRecord(static_cast<hipEvent_t>(p->start[slot]), st);
}
inline void prof_end(const Prof* p, int slot, hipStream_t st) {
  if (p && p->stop[slot]) (void)hipEventRecord(static_cast<hipEvent_t>(p->stop[slot]), st);
}

inline size_t align256(size_t x) { return (x + 255) / 256 * 256; }

struct Layout {
  // build
  size_t flags, F, MR, MS, ER, edge, strips, C, mom, build_end;
  // solve (overlaps the build region after `flags`)
  size_t A, Z, s, b, theta, x, rvec, rowabs, Ud, part, sync, solve_end;
  // subtract
  size_t partials, k2, sub_end;
  size_t total;
  int nmom;           // doubles in the moment block
  int nt;             // Cholesky tiles per side
  int npartials;      // subtract tiles of the single-pair launch
};

// moment block (doubles): M2[(DK+DB+1)^2], E[2r*(DK+DB+1)], MSy[(DB+1)^2],
// Px[2DB+1], Py[2DB+1]
inline int moment_count(const Geometry& g) {
  const int nm = g.DK + g.DB + 1;
  return nm * nm + 2 * g.r * nm + (g.DB + 1) * (g.DB + 1) + 2 * (2 * g.DB + 1);
}

inline int subtract_blocks(const Geometry& g, int tile_rows = kSubTY) {
  return ((g.W + kSubTX - 1) / kSubTX) * ((g.H + tile_rows - 1) / tile_rows);
}

inline Layout make_layout(const Geometry& g) {
  Layout l{};
  size_t o = 0;
  l.flags = o; o += 256;
  const size_t base = o;
  l.F = o; o = align256(o + (size_t)g.nsig * g.planeK * g.cxsize);
  const int nm = g.DK + g.DB + 1;
  l.MR = o; o = align256(o + sizeof(double) * nm * g.H);
  l.MS = o; o = align256(o + sizeof(double) * (g.DB + 1) * g.H);
  l.ER = o; o = align256(o + sizeof(double) * (2 * g.r > 0 ? 2 * g.r : 1) * g.H);
  l.edge = o; o = align256(o + sizeof(double) * g.nsig * 2 * g.H);
  l.strips = o; o = align256(o + (size_t)16 * g.NP * (2 * g.h + 1) * g.nkx);
  l.C = o; o = align256(o + sizeof(double) * g.NP * (2 * g.h + 1) * (2 * g.h + 1));
  l.nmom = moment_count(g);
  l.mom = o; o = align256(o + sizeof(double) * l.nmom);
  l.build_end = o;
  // solve region
  const int N = g.N;
  l.nt = (N + kTile - 1) / kTile;
  const size_t Np = (size_t)l.nt * kTile;
  o = base;
  // matrix rows, the right-hand-side row (padded to a tile) and identity rows
  l.A = o; o = align256(o + sizeof(double) * (2 * Np + kTile) * Np);
  // outputs of the augmented rows: z and L^-T
  l.Z = o; o = align256(o + sizeof(double) * (Np + kTile) * Np);
  l.s = o; o = align256(o + sizeof(double) * Np);
  l.b = o; o = align256(o + sizeof(double) * Np);
  l.theta = o; o = align256(o + sizeof(double) * Np);
  l.x = o; o = align256(o + sizeof(double) * Np);
  l.rvec = o; o = align256(o + sizeof(double) * Np);
  l.rowabs = o; o = align256(o + sizeof(double) * Np);
  l.Ud = o; o = align256(o + sizeof(double) * Np * kTile);
  // partial sums of the transposed triangular product: (row chunks) x Np,
  // at most max(Np, kMaxTeam workgroups x 8 waves x 64 columns)
  const size_t npart = (size_t)kMaxTeam * 8 * 64;
  l.part = o; o = align256(o + sizeof(double) * (Np > npart ? Np : npart));
  l.sync = o; o = align256(o + sizeof(unsigned) * kSyncClear);
  l.solve_end = o;
  // subtract region
  o = base;
  // chi2 partials, one per subtract tile: room for the smallest tile height
  l.npartials = subtract_blocks(g);
  l.partials = o; o = align256(o + sizeof(double) * subtract_blocks(g, kSubTYMin));
  // coefficients of the chi2 judge's kappa2 polynomial, (2 DK + 1)^2
  l.k2 = o; o = align256(o + sizeof(double) * 81);
  l.sub_end = o;
  size_t t = l.build_end;
  if (l.solve_end > t) t = l.solve_end;
  if (l.sub_end > t) t = l.sub_end;
  l.total = t;
  return l;
}

}  // namespace sfft
