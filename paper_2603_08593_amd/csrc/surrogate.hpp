// Parameter and workspace layout of the learned form's network (host and
// device). The network: per stamp 4 convolutions 3x3 (2->16 s1, 16->32 s2,
// 32->64 s2, 64->64 s2, ReLU), linear 1024->128 ReLU; position-weighted
// pooling of the stamps of a pair over the 6 DK = 2 monomials; linear
// 768->512 ReLU; linear 512->n_out.
#pragma once

#include <stddef.h>
#include <stdint.h>

namespace sfft {

constexpr int kNetStamp = 32;
constexpr int kNetMono = 6;
constexpr int kNetCin[4] = {2, 16, 32, 64};
constexpr int kNetCout[4] = {16, 32, 64, 64};
constexpr int kNetHin[4] = {32, 32, 16, 8};
constexpr int kNetStride[4] = {1, 2, 2, 2};
constexpr int kNetF = 1024;        // conv4 output per stamp (64 x 4 x 4)
constexpr int kNetH = 128;         // per-stamp feature
constexpr int kNetU = kNetMono * kNetH;
constexpr int kNetG = 512;
constexpr int kNetChunk = 32;      // stamps per weight-gradient partial

inline int net_hout(int k) { return (kNetHin[k] - 1) / kNetStride[k] + 1; }

struct NetLayout {
  int64_t cw[4], cb[4];
  int64_t fc1w, fc1b, fc2w, fc2b, fc3w, fc3b, total;
};

inline NetLayout net_layout(int n_out) {
  NetLayout l{};
  int64_t o = 0;
  for (int k = 0; k < 4; ++k) {
    l.cw[k] = o; o += (int64_t)kNetCout[k] * kNetCin[k] * 9;
    l.cb[k] = o; o += kNetCout[k];
  }
  l.fc1w = o; o += (int64_t)kNetH * kNetF;
  l.fc1b = o; o += kNetH;
  l.fc2w = o; o += (int64_t)kNetG * kNetU;
  l.fc2b = o; o += kNetG;
  l.fc3w = o; o += (int64_t)n_out * kNetG;
  l.fc3b = o; o += n_out;
  l.total = o;
  return l;
}

// workspace (bytes, 256-aligned): activations a1..a4 and their gradients,
// h, u, g, pred and gradients, weight-gradient partials, loss, bf16 params
struct NetWs {
  size_t a[5], ga[5], h, gh, u, gu, g, gg, pred, gpred, part, loss, pbf, xbf, total;
  int nchunk;
};

inline size_t net_align(size_t x) { return (x + 255) / 256 * 256; }

inline NetWs net_ws(int n_pairs, int n_stamps, int n_out) {
  NetWs w{};
  const size_t ns = (size_t)n_pairs * n_stamps;
  size_t o = 0;
  for (int k = 1; k <= 4; ++k) {
    const size_t n = ns * kNetCout[k - 1] * net_hout(k - 1) * net_hout(k - 1);
    w.a[k] = o; o = net_align(o + 4 * n);
    w.ga[k] = o; o = net_align(o + 4 * n);
  }
  w.h = o; o = net_align(o + 4 * ns * kNetH);
  w.gh = o; o = net_align(o + 4 * ns * kNetH);
  w.u = o; o = net_align(o + 4 * (size_t)n_pairs * kNetU);
  w.gu = o; o = net_align(o + 4 * (size_t)n_pairs * kNetU);
  w.g = o; o = net_align(o + 4 * (size_t)n_pairs * kNetG);
  w.gg = o; o = net_align(o + 4 * (size_t)n_pairs * kNetG);
  w.pred = o; o = net_align(o + 4 * (size_t)n_pairs * n_out);
  w.gpred = o; o = net_align(o + 4 * (size_t)n_pairs * n_out);
  w.nchunk = (int)((ns + kNetChunk - 1) / kNetChunk);
  w.part = o; o = net_align(o + 4 * (size_t)w.nchunk * (64 * 64 * 9 + 64));
  w.loss = o; o = net_align(o + 8);
  w.pbf = o; o = net_align(o + 2 * (size_t)net_layout(n_out).total);
  w.xbf = o; o = net_align(o + 2 * ns * 2 * kNetStamp * kNetStamp);
  w.total = o;
  return w;
}

}  // namespace sfft
