// Host side of the C ABI declared in include/sfft.h: handle and plan tables,
// argument validation, workspace sizing and kernel dispatch.
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <sstream>
#include <string>
#include <mutex>
#include <new>
#include <vector>
#include <algorithm>

#include "common.hpp"
#include "layout.hpp"
#include "batch.hpp"
#include "stamps.hpp"
#include "surrogate.hpp"
#include "products.hpp"
#include "realbogus.hpp"

namespace sfft {

hipError_t launch_build(const sfft_desc& d, const void* R, const void* S, double* G, double* hv,
                        unsigned char* ws, const BuildPlan& p, const Prof* pf, hipStream_t st,
                        bool reuse_sci = false);
bool sci_reusable(const sfft_desc& d);
hipError_t launch_build_masked(const sfft_desc& d, const void* R, const void* S, const unsigned char* mask,
                               int64_t mask_ld, double* G, double* hv, unsigned char* ws, const BuildPlan& p,
                               const Prof* pf, hipStream_t st, bool reuse_sci);
hipError_t launch_solve(const sfft_desc& d, const double* G, const double* h, double* coef,
                        int max_refine, sfft_solve_info* info, unsigned char* ws, int num_cus, int team,
                        const Prof* pf, hipStream_t st);
hipError_t launch_subtract(const sfft_desc& d, const void* R, const void* S, const double* coef,
                           void* D, double* chi2, unsigned char* ws, const Prof* pf,
                           hipStream_t st);
hipError_t noalloc_prepare(int device);
int noalloc_max_partials();
hipError_t launch_subtract_noalloc(int device, const sfft_desc& d, const void* R, const void* S,
                                   const double* coef, void* D, double* chi2, hipStream_t st);
hipError_t launch_stamps(const sfft_desc& d, const void* R, const void* S, const int32_t* centers,
                         int nst, int size, double* G, double* hv, unsigned char* ws, int num_cus,
                         const Prof* pf, hipStream_t st);
hipError_t launch_bg_refit(const sfft_desc& d, const void* R, const void* S, double* coef, double* G,
                           double* hv, unsigned char* ws, const BuildPlan& p, hipStream_t st);
hipError_t prepare_kernel_attributes();
hipError_t prepare_solve_attributes();
hipError_t prepare_stamp_attributes();
hipError_t prepare_surrogate_attributes();
hipError_t launch_extract_stamps(const sfft_desc& d, const void* R, const void* S, const int32_t* centers,
                                 int n, float* stamps, float* pos, hipStream_t st);
hipError_t launch_surrogate_forward(const float* params, const float* stamps, const float* pos, int n_pairs,
                                    int n_stamps, int n_out, bool bf16, float* pred, unsigned char* ws,
                                    hipStream_t st);
hipError_t launch_surrogate_grad(const float* P, const float* x, const float* pos, const float* target,
                                 int n_pairs, int n_stamps, int n_out, float* grads, double* loss,
                                 unsigned char* ws, hipStream_t st);
hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, int step, float lr, float b1,
                       float b2, float eps, hipStream_t st);
hipError_t launch_destandardize(const float* pred, const double* mean, const double* scale, int n_pairs,
                                int n_out, double* coef, hipStream_t st);

struct Twiddles {
  void* w64 = nullptr;    // cx<double>[n]
  void* w32 = nullptr;    // cx<float>[n]
};

}  // namespace sfft

struct sfft_handle_s {
  int device = 0;
  int num_cus = 0;
  std::map<int, sfft::Twiddles> tw;   // keyed by transform length
  sfft::Prof prof{};                  // timing events per sfft_prof_slot
  int solve_team = 0;                 // workgroups of the single-pair solve (0: default)
  int radix_order = 0;                // stage order of the single-pair row FFTs
  std::map<std::string, sfft_batch_knobs> tuned;   // batch key -> tuned configuration
  char arch[64] = {0};
};

struct sfft_batch_s {
  sfft_handle handle = nullptr;
  std::vector<sfft_batch_item> items;
  int max_refine = 2;
  sfft_batch_knobs knobs{4, 0, sfft::kSubTY, 0};   // team: the value in use (0 resolved)
  std::string key;
  sfft::BuildBatch* build = nullptr;
  sfft::SolveBatch* solve = nullptr;
  sfft::SubBatch* sub = nullptr;
  void* dev = nullptr;
  size_t dev_bytes = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

using namespace sfft;

// exp(-2 pi i m / n), m = 0..n-1, in FP64 on the host
hipError_t get_twiddles(sfft_handle hd, int n, Twiddles& out) {
  auto it = hd->tw.find(n);
  if (it != hd->tw.end()) { out = it->second; return hipSuccess; }
  std::vector<double> h64(2 * (size_t)n);
  std::vector<float> h32(2 * (size_t)n);
  for (int m = 0; m < n; ++m) {
    const long double ang = -2.0L * 3.141592653589793238462643383279502884L * (long double)m / (long double)n;
    h64[2 * m] = (double)std::cos(ang);
    h64[2 * m + 1] = (double)std::sin(ang);
    h32[2 * m] = (float)h64[2 * m];
    h32[2 * m + 1] = (float)h64[2 * m + 1];
  }
  Twiddles t;
  hipError_t e;
  if ((e = hipMalloc(&t.w64, sizeof(double) * 2 * n)) != hipSuccess) return e;
  if ((e = hipMalloc(&t.w32, sizeof(float) * 2 * n)) != hipSuccess) { (void)hipFree(t.w64); return e; }
  if ((e = hipMemcpy(t.w64, h64.data(), sizeof(double) * 2 * n, hipMemcpyHostToDevice)) != hipSuccess) return e;
  if ((e = hipMemcpy(t.w32, h32.data(), sizeof(float) * 2 * n, hipMemcpyHostToDevice)) != hipSuccess) return e;
  hd->tw[n] = t;
  out = t;
  return hipSuccess;
}

bool is_smooth235(int v) {
  if (v <= 0) return false;
  for (int f : {2, 3, 5})
    while (v % f == 0) v /= f;
  return v == 1;
}

sfft_status check_device(sfft_handle hd) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return SFFT_ERR_HIP;
  return dev == hd->device ? SFFT_OK : SFFT_ERR_INVALID_ARG;
}

}  // namespace

extern "C" {

const char* sfft_status_string(sfft_status s) {
  switch (s) {
    case SFFT_OK: return "SFFT_OK";
    case SFFT_ERR_INVALID_ARG: return "SFFT_ERR_INVALID_ARG";
    case SFFT_ERR_UNSUPPORTED: return "SFFT_ERR_UNSUPPORTED";
    case SFFT_ERR_WORKSPACE: return "SFFT_ERR_WORKSPACE";
    case SFFT_ERR_NONFINITE: return "SFFT_ERR_NONFINITE";
    case SFFT_ERR_NOT_SPD: return "SFFT_ERR_NOT_SPD";
    case SFFT_ERR_HIP: return "SFFT_ERR_HIP";
    case SFFT_ERR_INTERNAL: return "SFFT_ERR_INTERNAL";
  }
  return "SFFT_ERR_UNKNOWN";
}

int64_t sfft_num_unknowns(const sfft_desc* d) {
  if (!d || d->L < 1 || (d->L % 2) == 0 || d->dk < 0 || d->dk > 4 || d->db < 0 || d->db > 4)
    return -1;
  const int64_t nk = (int64_t)(d->dk + 1) * (d->dk + 2) / 2;
  const int64_t nb = (int64_t)(d->db + 1) * (d->db + 2) / 2;
  return nk * d->L * d->L + nb;
}

}  // extern "C"

// argument rules plus the limits of the solve and subtract kernels
static sfft_status validate_core(const sfft_desc* d) {
  if (!d) return SFFT_ERR_INVALID_ARG;
  if (d->width < 1 || d->height < 1 || d->ld < d->width) return SFFT_ERR_INVALID_ARG;
  if (d->L < 1 || (d->L % 2) == 0) return SFFT_ERR_INVALID_ARG;
  if (d->L > d->width || d->L > d->height) return SFFT_ERR_INVALID_ARG;
  if (d->dk < 0 || d->dk > 4 || d->db < 0 || d->db > 4) return SFFT_ERR_INVALID_ARG;
  if (d->image_dtype != SFFT_F32 && d->image_dtype != SFFT_F64) return SFFT_ERR_INVALID_ARG;
  if (d->compute != SFFT_COMPUTE_FP64 && d->compute != SFFT_COMPUTE_FP32) return SFFT_ERR_INVALID_ARG;
  if (d->convention != SFFT_CONV_INPUT_PIXEL && d->convention != SFFT_CONV_OUTPUT_PIXEL)
    return SFFT_ERR_INVALID_ARG;
  if (!std::isfinite(d->ref_pedestal) || !std::isfinite(d->sci_pedestal)) return SFFT_ERR_INVALID_ARG;
  if (d->L > 15 || d->dk > 2) return SFFT_ERR_UNSUPPORTED;
  if ((int64_t)d->height * d->ld > ((int64_t)1 << 40)) return SFFT_ERR_UNSUPPORTED;
  return SFFT_OK;
}

extern "C" {

sfft_status sfft_validate(const sfft_desc* d) {
  const sfft_status s = validate_core(d);
  if (s != SFFT_OK) return s;
  if (!is_smooth235(d->width) || (d->width & 1) || d->width < 16 || d->width > kMaxW)
    return SFFT_ERR_UNSUPPORTED;
  if (d->width < 2 * d->L || d->height < 2 * d->L) return SFFT_ERR_UNSUPPORTED;
  return SFFT_OK;
}

sfft_status sfft_create(sfft_handle* out) {
  if (!out) return SFFT_ERR_INVALID_ARG;
  *out = nullptr;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return SFFT_ERR_HIP;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return SFFT_ERR_HIP;
  if (prepare_kernel_attributes() != hipSuccess) return SFFT_ERR_HIP;
  if (prepare_solve_attributes() != hipSuccess) return SFFT_ERR_HIP;
  if (prepare_stamp_attributes() != hipSuccess || prepare_surrogate_attributes() != hipSuccess ||
      prepare_rb_attributes() != hipSuccess) {
    (void)hipGetLastError();
    return SFFT_ERR_HIP;
  }
  // device address of the allocation-free subtract's scratch array, once per device
  if (noalloc_prepare(dev) != hipSuccess) {
    (void)hipGetLastError();
    return SFFT_ERR_HIP;
  }
  sfft_handle h = new (std::nothrow) sfft_handle_s();
  if (!h) return SFFT_ERR_INTERNAL;
  h->device = dev;
  h->num_cus = cus;
  hipDeviceProp_t prop{};
  if (hipGetDeviceProperties(&prop, dev) == hipSuccess)
    std::snprintf(h->arch, sizeof h->arch, "%s", prop.gcnArchName);
  *out = h;
  return SFFT_OK;
}

sfft_status sfft_destroy(sfft_handle h) {
  if (!h) return SFFT_ERR_INVALID_ARG;
  for (auto& kv : h->tw) {
    if (kv.second.w64) (void)hipFree(kv.second.w64);
    if (kv.second.w32) (void)hipFree(kv.second.w32);
  }
  delete h;
  return SFFT_OK;
}

sfft_status sfft_workspace_size(sfft_handle h, const sfft_desc* d, size_t* bytes) {
  if (!h || !bytes) return SFFT_ERR_INVALID_ARG;
  const sfft_status s = sfft_validate(d);
  if (s != SFFT_OK) return s;
  *bytes = make_layout(make_geometry(*d)).total;
  return SFFT_OK;
}

static sfft_status check_ws(void* ws, size_t ws_bytes, size_t need) {
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255) != 0) return SFFT_ERR_WORKSPACE;
  if (ws_bytes < need) return SFFT_ERR_WORKSPACE;
  return SFFT_OK;
}

sfft_status sfft_build_system(sfft_handle h, const sfft_desc* d, const void* ref, const void* sci,
                              double* G, double* hv, void* ws, size_t ws_bytes, void* stream) {
  if (!h) return SFFT_ERR_INVALID_ARG;
  sfft_status s = sfft_validate(d);
  if (s != SFFT_OK) return s;
  if (!ref || !sci || !G || !hv) return SFFT_ERR_INVALID_ARG;
  if ((s = check_ws(ws, ws_bytes, make_layout(make_geometry(*d)).total)) != SFFT_OK) return s;
  if ((s = check_device(h)) != SFFT_OK) return s;
  Twiddles tw, t128;
  if (get_twiddles(h, d->width, tw) != hipSuccess) return SFFT_ERR_HIP;
  if (get_twiddles(h, kTP, t128) != hipSuccess) return SFFT_ERR_HIP;
  const bool f32 = d->compute == SFFT_COMPUTE_FP32;
  BuildPlan p{f32 ? tw.w32 : tw.w64, tw.w64, f32 ? t128.w32 : t128.w64, h->num_cus, h->radix_order};
  const hipError_t e = launch_build(*d, ref, sci, G, hv, static_cast<unsigned char*>(ws), p,
                                    &h->prof, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? SFFT_OK : SFFT_ERR_HIP;
}

sfft_status sfft_build_system_masked(sfft_handle h, const sfft_desc* d, const void* ref, const void* sci,
                                     const uint8_t* mask, int64_t mask_ld, double* G, double* hv, void* ws,
                                     size_t ws_bytes, void* stream) {
  if (!h) return SFFT_ERR_INVALID_ARG;
  sfft_status s = sfft_validate(d);
  if (s != SFFT_OK) return s;
  if (!ref || !sci || !G || !hv || !mask || mask_ld < d->width) return SFFT_ERR_INVALID_ARG;
  if ((s = check_ws(ws, ws_bytes, make_layout(make_geometry(*d)).total)) != SFFT_OK) return s;
  if ((s = check_device(h)) != SFFT_OK) return s;
  Twiddles tw, t128;
  if (get_twiddles(h, d->width, tw) != hipSuccess) return SFFT_ERR_HIP;
  if (get_twiddles(h, kTP, t128) != hipSuccess) return SFFT_ERR_HIP;
  const bool f32 = d->compute == SFFT_COMPUTE_FP32;
  BuildPlan p{f32 ? tw.w32 : tw.w64, tw.w64, f32 ? t128.w32 : t128.w64, h->num_cus, h->radix_order};
  const hipError_t e = launch_build_masked(*d, ref, sci, mask, mask_ld, G, hv, static_cast<unsigned char*>(ws), p,
                                           &h->prof, static_cast<hipStream_t>(stream), false);
  return e == hipSuccess ? SFFT_OK : SFFT_ERR_HIP;
}

sfft_status sfft_solve(sfft_handle h, const sfft_desc* d, const double* G, const double* hv,
                       double* coef, int32_t max_refine, sfft_solve_info* info, void* ws,
                       size_t ws_bytes, void* stream) {
  if (!h) return SFFT_ERR_INVALID_ARG;
  sfft_status s = validate_core(d);
  if (s != SFFT_OK) return s;
  if (!G || !hv || !coef || !info || max_refine < 0 || max_refine > 8) return SFFT_ERR_INVALID_ARG;
  if ((s = check_ws(ws, ws_bytes, make_layout(make_geometry(*d)).solve_end)) != SFFT_OK) return s;
  if ((s = check_device(h)) != SFFT_OK) return s;
  const hipError_t e = launch_solve(*d, G, hv, coef, max_refine, info,
                                    static_cast<unsigned char*>(ws), h->num_cus, h->solve_team, &h->prof,
                                    static_cast<hipStream_t>(stream));
  return e == hipSuccess ? SFFT_OK : SFFT_ERR_HIP;
}

sfft_status sfft_set_solve_team(sfft_handle h, int32_t team) {
  if (!h || team < 0 || team == 1 || team > kMaxTeam) return SFFT_ERR_INVALID_ARG;
  h->solve_team = team;
  return SFFT_OK;
}

sfft_status sfft_get_solve_team(sfft_handle h, int32_t* team) {
  if (!h || !team) return SFFT_ERR_INVALID_ARG;
  *team = h->solve_team;
  return SFFT_OK;
}

sfft_status sfft_set_radix_order(sfft_handle h, int32_t order) {
  if (!h || order < 0 || order > 1) return SFFT_ERR_INVALID_ARG;
  h->radix_order = order;
  return SFFT_OK;
}

sfft_status sfft_get_radix_order(sfft_handle h, int32_t* order) {
  if (!h || !order) return SFFT_ERR_INVALID_ARG;
  *order = h->radix_order;
  return SFFT_OK;
}

sfft_status sfft_subtract(sfft_handle h, const sfft_desc* d, const void* ref, const void* sci,
                          const double* coef, void* diff, double* chi2, void* ws, size_t ws_bytes,
                          void* stream) {
  if (!h) return SFFT_ERR_INVALID_ARG;
  sfft_status s = validate_core(d);
  if (s != SFFT_OK) return s;
  if (!ref || !sci || !coef || !diff || diff == ref || diff == sci) return SFFT_ERR_INVALID_ARG;
  if ((s = check_ws(ws, ws_bytes, make_layout(make_geometry(*d)).sub_end)) != SFFT_OK) return s;
  if ((s = check_device(h)) != SFFT_OK) return s;
  const hipError_t e = launch_subtract(*d, ref, sci, coef, diff, chi2,
                                       static_cast<unsigned char*>(ws), &h->prof,
                                       static_cast<hipStream_t>(stream));
  return e == hipSuccess ? SFFT_OK : SFFT_ERR_HIP;
}

sfft_status sfft_subtract_noalloc(sfft_handle h, const sfft_desc* d, const void* ref, const void* sci,
                                  const double* coef, void* diff, double* chi2, void* stream) {
  if (!h) return SFFT_ERR_INVALID_ARG;
  sfft_status s = validate_core(d);
  if (s != SFFT_OK) return s;
  if (!ref || !sci || !coef || !diff || diff == ref || diff == sci) return SFFT_ERR_INVALID_ARG;
  if (subtract_blocks(make_geometry(*d)) > noalloc_max_partials()) return SFFT_ERR_WORKSPACE;
  if ((s = check_device(h)) != SFFT_OK) return s;
  const hipError_t e = launch_subtract_noalloc(h->device, *d, ref, sci, coef, diff, chi2,
                                               static_cast<hipStream_t>(stream));
  return e == hipSuccess ? SFFT_OK : SFFT_ERR_HIP;
}

// The stamp form needs no FFT: any width; the solve and subtract limits stay.
static sfft_status validate_stamps(const sfft_desc* d, int32_t n, int32_t size) {
  sfft_status s = validate_core(d);
  if (s != SFFT_OK) return s;
  if (d->convention != SFFT_CONV_INPUT_PIXEL) return SFFT_ERR_UNSUPPORTED;
  if (n < 1 || n > kStMaxStamps || size < 1 || (size % 2) == 0 || size > kStMaxSize)
    return SFFT_ERR_INVALID_ARG;
  if (size > d->width || size > d->height) return SFFT_ERR_INVALID_ARG;
  const StampGeom g = make_stamp_geom(*d, size);
  if (g.nK + g.nB + 1 > kStMaxPlanes) return SFFT_ERR_UNSUPPORTED;
  if (make_stamp_plan(g, n, 256).lds_bytes > (size_t)kStMaxLds) return SFFT_ERR_UNSUPPORTED;
  return SFFT_OK;
}

static size_t stamps_ws_total(const sfft_desc& d, int32_t n, int32_t size, int num_cus) {
  const StampGeom g = make_stamp_geom(d, size);
  const size_t sw = make_stamp_plan(g, n, num_cus).ws_bytes;
  const Layout l = make_layout(make_geometry(d));
  size_t t = sw;
  if (l.solve_end > t) t = l.solve_end;
  if (l.sub_end > t) t = l.sub_end;
  return t;
}

sfft_status sfft_stamps_workspace_size(sfft_handle h, const sfft_desc* d, int32_t n_stamps,
                                       int32_t size, size_t* bytes) {
  if (!h || !bytes) return SFFT_ERR_INVALID_ARG;
  const sfft_status s = validate_stamps(d, n_stamps, size);
  if (s != SFFT_OK) return s;
  *bytes = stamps_ws_total(*d, n_stamps, size, h->num_cus);
  return SFFT_OK;
}

sfft_status sfft_build_system_stamps(sfft_handle h, const sfft_desc* d, const void* ref,
                                     const void* sci, const int32_t* centers, int32_t n_stamps,
                                     int32_t size, double* G, double* hv, void* ws,
                                     size_t ws_bytes, void* stream) {
  if (!h) return SFFT_ERR_INVALID_ARG;
  sfft_status s = validate_stamps(d, n_stamps, size);
  if (s != SFFT_OK) return s;
  if (!ref || !sci || !centers || !G || !hv) return SFFT_ERR_INVALID_ARG;
  if ((s = check_ws(ws, ws_bytes, stamps_ws_total(*d, n_stamps, size, h->num_cus))) != SFFT_OK)
    return s;
  if ((s = check_device(h)) != SFFT_OK) return s;
  const hipError_t e = launch_stamps(*d, ref, sci, centers, n_stamps, size, G, hv,
                                     static_cast<unsigned char*>(ws), h->num_cus, &h->prof,
                                     static_cast<hipStream_t>(stream));
  return e == hipSuccess ? SFFT_OK : SFFT_ERR_HIP;
}

sfft_status sfft_refit_background(sfft_handle h, const sfft_desc* d, const void* ref, const void* sci,
                                  double* coef, double* G, double* hv, void* ws, size_t ws_bytes,
                                  void* stream) {
  if (!h) return SFFT_ERR_INVALID_ARG;
  sfft_status s = validate_core(d);
  if (s != SFFT_OK) return s;
  if (!ref || !sci || !coef || !G || !hv) return SFFT_ERR_INVALID_ARG;
  if (d->convention != SFFT_CONV_INPUT_PIXEL) return SFFT_ERR_UNSUPPORTED;
  if ((s = check_ws(ws, ws_bytes, make_layout(make_geometry(*d)).build_end)) != SFFT_OK) return s;
  if ((s = check_device(h)) != SFFT_OK) return s;
  BuildPlan p{nullptr, nullptr, nullptr, h->num_cus, 0};
  const hipError_t e = launch_bg_refit(*d, ref, sci, coef, G, hv, static_cast<unsigned char*>(ws), p,
                                       static_cast<hipStream_t>(stream));
  return e == hipSuccess ? SFFT_OK : SFFT_ERR_HIP;
}

// ---- multi-template differencing and photometry ---------------------------

static sfft_status validate_image(const sfft_desc* d) {
  if (!d) return SFFT_ERR_INVALID_ARG;
  if (d->width < 1 || d->height < 1 || d->ld < d->width) return SFFT_ERR_INVALID_ARG;
  if (d->image_dtype != SFFT_F32 && d->image_dtype != SFFT_F64) return SFFT_ERR_INVALID_ARG;
  if ((int64_t)d->height * d->ld > ((int64_t)1 << 40)) return SFFT_ERR_UNSUPPORTED;
  return SFFT_OK;
}

static bool zp_ok(const double* zp, int n, double zp_common) {
  if (!zp || !std::isfinite(zp_common)) return false;
  for (int t = 0; t < n; ++t)
    if (!std::isfinite(zp[t])) return false;
  return true;
}

static CombineArgs make_combine(const sfft_desc& d, const void* const* diffs, int n, const double* zp,
                                double zp_common, void* out) {
  CombineArgs a{};
  for (int t = 0; t < n; ++t) {
    a.D[t] = diffs[t];
    a.scale[t] = std::pow(10.0, 0.4 * (zp_common - zp[t]));
  }
  a.out = out;
  a.ld = d.ld;
  a.W = d.width;
  a.H = d.height;
  return a;
}

sfft_status sfft_median_combine(sfft_handle h, const sfft_desc* d, const void* const* diffs, int32_t n,
                                const double* zp, double zp_common, void* out, void* stream) {
  if (!h) return SFFT_ERR_INVALID_ARG;
  sfft_status s = validate_image(d);
  if (s != SFFT_OK) return s;
  if (!diffs || !out || n < 1 || n > kMaxTemplates || !zp_ok(zp, n, zp_common)) return SFFT_ERR_INVALID_ARG;
  for (int t = 0; t < n; ++t)
    if (!diffs[t]) return SFFT_ERR_INVALID_ARG;
  if ((s = check_device(h)) != SFFT_OK) return s;
  const CombineArgs a = make_combine(*d, diffs, n, zp, zp_common, out);
  const hipError_t e = launch_median_combine(a, n, d->image_dtype == SFFT_F32, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? SFFT_OK : SFFT_ERR_HIP;
}

sfft_status sfft_difference_multi(sfft_handle h, const sfft_desc* d, const void* const* refs, const void* sci,
                                  int32_t n, const double* ref_pedestals, const double* zp, double zp_common,
                                  int32_t max_refine, double* G, double* hv, double* coefs,
                                  sfft_solve_info* infos, double* chi2s, void* const* diffs, void* combined,
                                  void* ws, size_t ws_bytes, void* stream) {
  if (!h) return SFFT_ERR_INVALID_ARG;
  sfft_status s = sfft_validate(d);
  if (s != SFFT_OK) return s;
  if (!refs || !sci || !G || !hv || !coefs || !infos || !chi2s || !diffs || !combined) return SFFT_ERR_INVALID_ARG;
  if (n < 1 || n > kMaxTemplates || max_refine < 0 || max_refine > 8 || !zp_ok(zp, n, zp_common))
    return SFFT_ERR_INVALID_ARG;
  for (int t = 0; t < n; ++t) {
    if (!refs[t] || !diffs[t] || diffs[t] == sci || diffs[t] == combined) return SFFT_ERR_INVALID_ARG;
    if (ref_pedestals && !std::isfinite(ref_pedestals[t])) return SFFT_ERR_INVALID_ARG;
    for (int u = 0; u < n; ++u)
      if (diffs[t] == refs[u] || (u != t && diffs[t] == diffs[u])) return SFFT_ERR_INVALID_ARG;
  }
  if (combined == sci) return SFFT_ERR_INVALID_ARG;
  if ((s = check_ws(ws, ws_bytes, make_layout(make_geometry(*d)).total)) != SFFT_OK) return s;
  if ((s = check_device(h)) != SFFT_OK) return s;
  Twiddles tw, t128;
  if (get_twiddles(h, d->width, tw) != hipSuccess) return SFFT_ERR_HIP;
  if (get_twiddles(h, kTP, t128) != hipSuccess) return SFFT_ERR_HIP;
  const bool f32 = d->compute == SFFT_COMPUTE_FP32;
  const BuildPlan p{f32 ? tw.w32 : tw.w64, tw.w64, f32 ? t128.w32 : t128.w64, h->num_cus, h->radix_order};
  hipStream_t st = static_cast<hipStream_t>(stream);
  unsigned char* w = static_cast<unsigned char*>(ws);
  const int64_t N = sfft_num_unknowns(d);
  // the science image's row spectrum and moments are computed once, by the
  // first template's build, when they survive the solve and subtract
  const bool reuse = sci_reusable(*d);
  for (int t = 0; t < n; ++t) {
    sfft_desc dt = *d;
    if (ref_pedestals) dt.ref_pedestal = ref_pedestals[t];
    hipError_t e = launch_build(dt, refs[t], sci, G, hv, w, p, &h->prof, st, reuse && t > 0);
    if (e == hipSuccess)
      e = launch_solve(dt, G, hv, coefs + t * N, max_refine, infos + t, w, h->num_cus, h->solve_team,
                       &h->prof, st);
    if (e == hipSuccess)
      e = launch_subtract(dt, refs[t], sci, coefs + t * N, diffs[t], chi2s + t, w, &h->prof, st);
    if (e != hipSuccess) return SFFT_ERR_HIP;
  }
  const CombineArgs a = make_combine(*d, diffs, n, zp, zp_common, combined);
  const hipError_t e = launch_median_combine(a, n, d->image_dtype == SFFT_F32, st);
  return e == hipSuccess ? SFFT_OK : SFFT_ERR_HIP;
}

static bool ap_args_ok(const double* xy, int32_t n, double radius) {
  return xy && n >= 1 && n <= (1 << 24) && std::isfinite(radius) && radius > 0.0 && radius <= 64.0;
}

sfft_status sfft_aperture_flux(sfft_handle h, const sfft_desc* d, const void* image, const double* xy, int32_t n,
                               double radius, double* flux, void* stream) {
  return sfft_forced_photometry(h, d, image, xy, n, radius, 0.0, nullptr, flux, nullptr, nullptr, stream);
}

sfft_status sfft_forced_photometry(sfft_handle h, const sfft_desc* d, const void* image, const double* xy,
                                   int32_t n, double radius, double zp, const double* sigma, double* flux,
                                   double* mag, double* mag_err, void* stream) {
  if (!h) return SFFT_ERR_INVALID_ARG;
  sfft_status s = validate_image(d);
  if (s != SFFT_OK) return s;
  if (!image || !flux || !ap_args_ok(xy, n, radius) || !std::isfinite(zp)) return SFFT_ERR_INVALID_ARG;
  if (mag_err && !sigma) return SFFT_ERR_INVALID_ARG;
  if ((s = check_device(h)) != SFFT_OK) return s;
  ApArgs a{};
  a.img = image; a.ld = d->ld; a.W = d->width; a.H = d->height; a.xy = xy; a.n = n; a.radius = radius;
  a.flux = flux; a.mag = mag; a.mag_err = mag_err; a.sigma = sigma; a.zp = zp;
  const hipError_t e = launch_aperture(a, d->image_dtype == SFFT_F32, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? SFFT_OK : SFFT_ERR_HIP;
}

sfft_status sfft_limiting_magnitude(sfft_handle h, const sfft_desc* d, const void* image, const double* xy,
                                    int32_t n, double radius, double zp, double nsigma, double* flux,
                                    double* result, void* stream) {
  if (!h) return SFFT_ERR_INVALID_ARG;
  if (n < 2 || !result || !std::isfinite(nsigma) || !(nsigma > 0.0)) return SFFT_ERR_INVALID_ARG;
  sfft_status s = sfft_forced_photometry(h, d, image, xy, n, radius, zp, nullptr, flux, nullptr, nullptr, stream);
  if (s != SFFT_OK) return s;
  const hipError_t e = launch_limiting_mag(flux, n, zp, nsigma, result, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? SFFT_OK : SFFT_ERR_HIP;
}

// ---- real-bogus scorer ----------------------------------------------------

int64_t sfft_rb_num_params(void) { return kRbNumParams; }

sfft_status sfft_rb_workspace_size(int32_t n, size_t* bytes) {
  if (!bytes || n < 1 || n > kRbMaxN) return SFFT_ERR_INVALID_ARG;
  *bytes = rb_plan(n).total;
  return SFFT_OK;
}

sfft_status sfft_rb_extract(sfft_handle h, const sfft_desc* d, const void* sci, const void* ref, const void* diff,
                            const int32_t* centers, int32_t n, const float* offsets, const float* scales,
                            float* stamps, void* stream) {
  if (!h) return SFFT_ERR_INVALID_ARG;
  sfft_status s = validate_image(d);
  if (s != SFFT_OK) return s;
  if (!sci || !ref || !diff || !centers || !offsets || !scales || !stamps || n < 1 || n > (1 << 20))
    return SFFT_ERR_INVALID_ARG;
  for (int c = 0; c < 3; ++c)
    if (!std::isfinite(offsets[c]) || !std::isfinite(scales[c])) return SFFT_ERR_INVALID_ARG;
  if ((s = check_device(h)) != SFFT_OK) return s;
  RbExtractArgs a{};
  a.img[0] = sci; a.img[1] = ref; a.img[2] = diff;
  a.ld = d->ld; a.W = d->width; a.H = d->height; a.centers = centers; a.n = n; a.stamps = stamps;
  for (int c = 0; c < 3; ++c) { a.offset[c] = offsets[c]; a.scale[c] = scales[c]; }
  const hipError_t e = launch_rb_extract(a, d->image_dtype == SFFT_F32, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? SFFT_OK : SFFT_ERR_HIP;
}

sfft_status sfft_rb_score(sfft_handle h, const float* params, const float* stamps, int32_t n, float* logits,
                          float* probs, void* ws, size_t ws_bytes, void* stream) {
  if (!h || !params || !stamps || !logits || n < 1 || n > kRbMaxN) return SFFT_ERR_INVALID_ARG;
  sfft_status s;
  if ((s = check_ws(ws, ws_bytes, rb_plan(n).total)) != SFFT_OK) return s;
  if ((s = check_device(h)) != SFFT_OK) return s;
  const hipError_t e = launch_rb_score(params, stamps, n, logits, probs, static_cast<unsigned char*>(ws),
                                       static_cast<hipStream_t>(stream));
  return e == hipSuccess ? SFFT_OK : SFFT_ERR_HIP;
}

// ---- learned form -------------------------------------------------------

static bool net_shape_ok(int32_t n_pairs, int32_t n_stamps, int32_t n_out) {
  return n_pairs >= 1 && n_pairs <= 4096 && n_stamps >= 1 && n_stamps <= 1024 && n_out >= 1 &&
         n_out <= 65536 && (int64_t)n_pairs * n_stamps <= (1 << 20);
}

int64_t sfft_surrogate_num_params(int32_t n_out) {
  if (n_out < 1 || n_out > 65536) return -1;
  return net_layout(n_out).total;
}

sfft_status sfft_surrogate_workspace_size(int32_t n_pairs, int32_t n_stamps, int32_t n_out, size_t* bytes) {
  if (!bytes || !net_shape_ok(n_pairs, n_stamps, n_out)) return SFFT_ERR_INVALID_ARG;
  *bytes = net_ws(n_pairs, n_stamps, n_out).total;
  return SFFT_OK;
}

sfft_status sfft_extract_stamps(sfft_handle h, const sfft_desc* d, const void* ref, const void* sci,
                                const int32_t* centers, int32_t n, float* stamps, float* pos,
                                void* stream) {
  if (!h) return SFFT_ERR_INVALID_ARG;
  sfft_status s = validate_core(d);
  if (s != SFFT_OK) return s;
  if (!ref || !sci || !centers || !stamps || !pos || n < 1 || n > (1 << 20)) return SFFT_ERR_INVALID_ARG;
  if (d->width < kNetStamp || d->height < kNetStamp) return SFFT_ERR_INVALID_ARG;
  if ((s = check_device(h)) != SFFT_OK) return s;
  const hipError_t e = launch_extract_stamps(*d, ref, sci, centers, n, stamps, pos,
                                             static_cast<hipStream_t>(stream));
  return e == hipSuccess ? SFFT_OK : SFFT_ERR_HIP;
}

sfft_status sfft_surrogate_forward(sfft_handle h, const float* params, const float* stamps, const float* pos,
                                   int32_t n_pairs, int32_t n_stamps, int32_t n_out, int32_t precision,
                                   float* pred, void* ws, size_t ws_bytes, void* stream) {
  if (!h || !params || !stamps || !pos || !pred) return SFFT_ERR_INVALID_ARG;
  if (!net_shape_ok(n_pairs, n_stamps, n_out)) return SFFT_ERR_INVALID_ARG;
  if (precision != SFFT_NET_FP32 && precision != SFFT_NET_BF16) return SFFT_ERR_INVALID_ARG;
  sfft_status s;
  if ((s = check_ws(ws, ws_bytes, net_ws(n_pairs, n_stamps, n_out).total)) != SFFT_OK) return s;
  if ((s = check_device(h)) != SFFT_OK) return s;
  const hipError_t e = launch_surrogate_forward(params, stamps, pos, n_pairs, n_stamps, n_out,
                                                precision == SFFT_NET_BF16, pred,
                                                static_cast<unsigned char*>(ws), static_cast<hipStream_t>(stream));
  return e == hipSuccess ? SFFT_OK : SFFT_ERR_HIP;
}

sfft_status sfft_surrogate_grad(sfft_handle h, const float* params, const float* stamps, const float* pos,
                                const float* target, int32_t n_pairs, int32_t n_stamps, int32_t n_out,
                                float* grads, double* loss, void* ws, size_t ws_bytes, void* stream) {
  if (!h || !params || !stamps || !pos || !target || !grads || !loss) return SFFT_ERR_INVALID_ARG;
  if (!net_shape_ok(n_pairs, n_stamps, n_out)) return SFFT_ERR_INVALID_ARG;
  sfft_status s;
  if ((s = check_ws(ws, ws_bytes, net_ws(n_pairs, n_stamps, n_out).total)) != SFFT_OK) return s;
  if ((s = check_device(h)) != SFFT_OK) return s;
  const hipError_t e = launch_surrogate_grad(params, stamps, pos, target, n_pairs, n_stamps, n_out, grads, loss,
                                             static_cast<unsigned char*>(ws), static_cast<hipStream_t>(stream));
  return e == hipSuccess ? SFFT_OK : SFFT_ERR_HIP;
}

sfft_status sfft_surrogate_adam(sfft_handle h, float* params, const float* grads, float* m, float* v, int64_t n,
                                int32_t step, float lr, float beta1, float beta2, float eps, void* stream) {
  if (!h || !params || !grads || !m || !v || n < 1 || step < 1) return SFFT_ERR_INVALID_ARG;
  if (!(lr > 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
    return SFFT_ERR_INVALID_ARG;
  sfft_status s;
  if ((s = check_device(h)) != SFFT_OK) return s;
  const hipError_t e = launch_adam(params, grads, m, v, n, step, lr, beta1, beta2, eps,
                                   static_cast<hipStream_t>(stream));
  return e == hipSuccess ? SFFT_OK : SFFT_ERR_HIP;
}

sfft_status sfft_surrogate_destandardize(sfft_handle h, const float* pred, const double* mean,
                                         const double* scale, int32_t n_pairs, int32_t n_out, double* coef,
                                         void* stream) {
  if (!h || !pred || !mean || !scale || !coef || n_pairs < 1 || n_out < 1) return SFFT_ERR_INVALID_ARG;
  sfft_status s;
  if ((s = check_device(h)) != SFFT_OK) return s;
  const hipError_t e = launch_destandardize(pred, mean, scale, n_pairs, n_out, coef,
                                            static_cast<hipStream_t>(stream));
  return e == hipSuccess ? SFFT_OK : SFFT_ERR_HIP;
}

// ---- batched form ---------------------------------------------------------

static void batch_release(sfft_batch b) {
  if (b->exec) { (void)hipGraphExecDestroy(b->exec); b->exec = nullptr; }
  if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
  if (b->build) { build_batch_destroy(b->build); b->build = nullptr; }
  if (b->solve) { solve_batch_destroy(b->solve); b->solve = nullptr; }
  if (b->sub) { sub_batch_destroy(b->sub); b->sub = nullptr; }
  if (b->dev) { (void)hipFree(b->dev); b->dev = nullptr; }
  b->dev_bytes = 0;
}

static bool knobs_valid(const sfft_batch_knobs& k) {
  return k.rows_per_block >= 1 && k.rows_per_block <= 64 && k.radix_order >= 0 && k.radix_order <= 1 &&
         (k.tile_rows == 16 || k.tile_rows == 32 || k.tile_rows == 64) && k.team >= 0 && k.team <= kMaxTeam;
}

// (re)build the per-phase tables for the given configuration and upload them
static sfft_status batch_plan(sfft_batch b, const sfft_batch_knobs& kn) {
  batch_release(b);
  const int n = (int)b->items.size();
  std::vector<BuildItem> bi(n);
  std::vector<SolveItem> si(n);
  std::vector<SubItem> ui(n);
  std::vector<BuildPlan> plans(n);
  for (int k = 0; k < n; ++k) {
    const sfft_batch_item& it = b->items[k];
    Twiddles tw, t128;
    if (get_twiddles(b->handle, it.desc.width, tw) != hipSuccess) return SFFT_ERR_HIP;
    if (get_twiddles(b->handle, kTP, t128) != hipSuccess) return SFFT_ERR_HIP;
    plans[k] = BuildPlan{tw.w32, tw.w64, t128.w32, b->handle->num_cus, kn.radix_order};
    unsigned char* ws = static_cast<unsigned char*>(it.ws);
    bi[k] = BuildItem{it.desc, it.ref, it.sci, it.G, it.h, ws};
    si[k] = SolveItem{it.desc, it.G, it.h, it.coef, it.info, ws};
    ui[k] = SubItem{it.desc, it.ref, it.sci, it.coef, it.diff, it.chi2, ws};
  }
  hipError_t e;
  b->build = build_batch_create(bi.data(), n, plans.data(), kn.rows_per_block, &e);
  if (!b->build) return e == hipErrorInvalidValue ? SFFT_ERR_UNSUPPORTED : SFFT_ERR_HIP;
  b->solve = solve_batch_create(si.data(), n, b->max_refine, kn.team, b->handle->num_cus, &e);
  if (!b->solve) return e == hipErrorInvalidValue ? SFFT_ERR_UNSUPPORTED : SFFT_ERR_HIP;
  b->sub = sub_batch_create(ui.data(), n, kn.tile_rows, &e);
  if (!b->sub) return e == hipErrorInvalidValue ? SFFT_ERR_UNSUPPORTED : SFFT_ERR_HIP;
  const size_t o1 = align256(build_batch_dev_bytes(b->build));
  const size_t o2 = o1 + align256(solve_batch_dev_bytes(b->solve));
  b->dev_bytes = o2 + align256(sub_batch_dev_bytes(b->sub));
  if (hipMalloc(&b->dev, b->dev_bytes) != hipSuccess) { b->dev = nullptr; return SFFT_ERR_HIP; }
  unsigned char* d = static_cast<unsigned char*>(b->dev);
  if (build_batch_upload(b->build, d) != hipSuccess || solve_batch_upload(b->solve, d + o1) != hipSuccess ||
      sub_batch_upload(b->sub, d + o2) != hipSuccess)
    return SFFT_ERR_HIP;
  b->knobs = kn;
  b->knobs.team = solve_batch_team(b->solve);
  return SFFT_OK;
}

static std::string batch_key(sfft_handle h, const std::vector<sfft_batch_item>& items) {
  std::map<std::string, int> count;
  for (const auto& it : items) {
    const sfft_desc& d = it.desc;
    char buf[128];
    std::snprintf(buf, sizeof buf, "%dx%d:L%d:DK%d:DB%d:%s", d.width, d.height, d.L, d.dk, d.db,
                  d.compute == SFFT_COMPUTE_FP32 ? "fp32" : "fp64");
    count[buf] += 1;
  }
  std::ostringstream os;
  os << h->arch;
  for (const auto& kv : count) os << "|" << kv.second << "*" << kv.first;
  return os.str();
}

static const char* tune_cache_path() { return std::getenv("SFFT_TUNE_CACHE"); }

// cache lines: "<key> <rows per block> <team> <radix order> <tile rows>";
// lines with only the first two values (an older cache) take the defaults
// of the others
static bool tune_cache_lookup(sfft_handle h, const std::string& key, sfft_batch_knobs& kn) {
  auto it = h->tuned.find(key);
  if (it != h->tuned.end()) { kn = it->second; return true; }
  const char* path = tune_cache_path();
  if (!path) return false;
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char line[4096];
  bool found = false;
  while (std::fgets(line, sizeof line, f)) {
    char k[3900];
    sfft_batch_knobs c{4, 0, kSubTY, 0};
    const int got = std::sscanf(line, "%3899s %d %d %d %d", k, &c.rows_per_block, &c.team, &c.radix_order,
                                &c.tile_rows);
    if (got >= 3 && key == k) {
      if (got < 5) { c.radix_order = 0; c.tile_rows = kSubTY; }
      if (knobs_valid(c)) { kn = c; found = true; }
    }
  }
  std::fclose(f);
  if (found) h->tuned[key] = kn;
  return found;
}

static void tune_cache_store(sfft_handle h, const std::string& key, const sfft_batch_knobs& kn) {
  h->tuned[key] = kn;
  const char* path = tune_cache_path();
  if (!path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%s %d %d %d %d\n", key.c_str(), kn.rows_per_block, kn.team, kn.radix_order, kn.tile_rows);
  std::fclose(f);
}

sfft_status sfft_batch_create(sfft_handle h, const sfft_batch_item* items, int32_t n, int32_t max_refine,
                              sfft_batch* out) {
  if (!h || !items || !out || n < 1 || n > 4096 || max_refine < 0 || max_refine > 8) return SFFT_ERR_INVALID_ARG;
  *out = nullptr;
  sfft_status s;
  if ((s = check_device(h)) != SFFT_OK) return s;
  for (int k = 0; k < n; ++k) {
    const sfft_batch_item& it = items[k];
    if ((s = sfft_validate(&it.desc)) != SFFT_OK) return s;
    if (!it.ref || !it.sci || !it.diff || !it.G || !it.h || !it.coef || !it.info || !it.chi2)
      return SFFT_ERR_INVALID_ARG;
    if (it.diff == it.ref || it.diff == it.sci) return SFFT_ERR_INVALID_ARG;
    if ((s = check_ws(it.ws, it.ws_bytes, make_layout(make_geometry(it.desc)).total)) != SFFT_OK) return s;
    if (it.desc.compute != SFFT_COMPUTE_FP32 || it.desc.image_dtype != SFFT_F32 || it.desc.width > 2048)
      return SFFT_ERR_UNSUPPORTED;
    if (it.desc.dk != items[0].desc.dk || it.desc.convention != SFFT_CONV_INPUT_PIXEL) return SFFT_ERR_UNSUPPORTED;
  }
  sfft_batch b = new (std::nothrow) sfft_batch_s();
  if (!b) return SFFT_ERR_INTERNAL;
  b->handle = h;
  b->items.assign(items, items + n);
  b->max_refine = max_refine;
  b->key = batch_key(h, b->items);
  sfft_batch_knobs kn{4, 0, kSubTY, 0};
  (void)tune_cache_lookup(h, b->key, kn);
  if ((s = batch_plan(b, kn)) != SFFT_OK) {
    batch_release(b);
    delete b;
    return s;
  }
  *out = b;
  return SFFT_OK;
}

static sfft_status batch_launch(sfft_batch b, hipStream_t st, const Prof* pf) {
  if (build_batch_launch(b->build, pf, st) != hipSuccess) return SFFT_ERR_HIP;
  if (solve_batch_launch(b->solve, pf, st) != hipSuccess) return SFFT_ERR_HIP;
  if (sub_batch_launch(b->sub, pf, st) != hipSuccess) return SFFT_ERR_HIP;
  return SFFT_OK;
}

sfft_status sfft_batch_run(sfft_batch b, void* stream) {
  if (!b) return SFFT_ERR_INVALID_ARG;
  sfft_status s;
  if ((s = check_device(b->handle)) != SFFT_OK) return s;
  return batch_launch(b, static_cast<hipStream_t>(stream), &b->handle->prof);
}

sfft_status sfft_batch_run_graph(sfft_batch b, void* stream) {
  if (!b || !stream) return SFFT_ERR_INVALID_ARG;
  sfft_status s;
  if ((s = check_device(b->handle)) != SFFT_OK) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (!b->exec) {
    if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) return SFFT_ERR_HIP;
    const sfft_status ls = batch_launch(b, st, nullptr);
    hipGraph_t g = nullptr;
    const hipError_t ce = hipStreamEndCapture(st, &g);
    if (ls != SFFT_OK || ce != hipSuccess || !g) {
      if (g) (void)hipGraphDestroy(g);
      return ls != SFFT_OK ? ls : SFFT_ERR_HIP;
    }
    b->graph = g;
    if (hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess) {
      b->exec = nullptr;
      return SFFT_ERR_HIP;
    }
  }
  return hipGraphLaunch(b->exec, st) == hipSuccess ? SFFT_OK : SFFT_ERR_HIP;
}

// Autotuner. The three phases run one after another and each knob acts on
// one phase only (rows per workgroup and radix order: the build; team: the
// solve; tile rows: the subtract), so the knobs are searched group by group
// with the others held: build knobs first, then the team, then the tile.
// Each candidate runs the whole batch twice on the stream, timed by events
// on the second run; the fastest is kept and recorded in the handle (and in
// $SFFT_TUNE_CACHE when set).
sfft_status sfft_batch_tune(sfft_batch b, void* stream, int32_t* rows_per_block, int32_t* team) {
  if (!b) return SFFT_ERR_INVALID_ARG;
  sfft_status s;
  if ((s = check_device(b->handle)) != SFFT_OK) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int n = (int)b->items.size();
  const int cus = b->handle->num_cus > 0 ? b->handle->num_cus : 256;
  // solve team sizes: one team per item (CUs / n) and larger teams that
  // work through a queue of items (fewer concurrent teams)
  std::vector<int> teams;
  const int one_each = std::max(1, std::min(64, cus / n));
  teams.push_back(one_each);
  for (int t : {4, 8, 16, 32, 64})
    if (t > one_each && t <= cus) teams.push_back(t);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return SFFT_ERR_HIP;
  if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return SFFT_ERR_HIP; }
  auto time_knobs = [&](const sfft_batch_knobs& kn, float& ms) -> sfft_status {
    sfft_status r;
    if ((r = batch_plan(b, kn)) != SFFT_OK) return r;
    for (int rep = 0; rep < 2; ++rep) {
      if (hipEventRecord(e0, st) != hipSuccess) return SFFT_ERR_HIP;
      if ((r = batch_launch(b, st, nullptr)) != SFFT_OK) return r;
      if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return SFFT_ERR_HIP;
      if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return SFFT_ERR_HIP;
    }
    return SFFT_OK;
  };
  sfft_batch_knobs best{4, 0, kSubTY, teams.back()};
  float best_ms = 1e30f;
  auto consider = [&](const sfft_batch_knobs& kn) -> sfft_status {
    float ms = 0.f;
    const sfft_status r = time_knobs(kn, ms);
    if (r == SFFT_OK && ms < best_ms) { best_ms = ms; best = kn; }
    return r;
  };
  const sfft_batch_knobs start = best;
  for (int rpb : {2, 4, 8, 16})
    for (int ro : {0, 1}) {
      sfft_batch_knobs kn = start;
      kn.rows_per_block = rpb;
      kn.radix_order = ro;
      if (s == SFFT_OK) s = consider(kn);
    }
  for (size_t i = 0; s == SFFT_OK && i < teams.size(); ++i) {
    sfft_batch_knobs kn = best;
    kn.team = teams[i];
    s = consider(kn);
  }
  for (int tr : {16, 32, 64}) {
    if (s != SFFT_OK) break;
    sfft_batch_knobs kn = best;
    kn.tile_rows = tr;
    s = consider(kn);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (s != SFFT_OK) return s;
  if ((s = batch_plan(b, best)) != SFFT_OK) return s;
  tune_cache_store(b->handle, b->key, b->knobs);
  if (rows_per_block) *rows_per_block = b->knobs.rows_per_block;
  if (team) *team = b->knobs.team;
  return SFFT_OK;
}

sfft_status sfft_batch_plan(sfft_batch b, int32_t rows_per_block, int32_t team) {
  if (!b) return SFFT_ERR_INVALID_ARG;
  sfft_batch_knobs kn = b->knobs;
  kn.rows_per_block = rows_per_block;
  kn.team = team;
  return sfft_batch_set_knobs(b, &kn);
}

sfft_status sfft_batch_set_knobs(sfft_batch b, const sfft_batch_knobs* knobs) {
  if (!b || !knobs || !knobs_valid(*knobs)) return SFFT_ERR_INVALID_ARG;
  sfft_status s;
  if ((s = check_device(b->handle)) != SFFT_OK) return s;
  if (hipDeviceSynchronize() != hipSuccess) return SFFT_ERR_HIP;   // tables in use by queued work
  return batch_plan(b, *knobs);
}

sfft_status sfft_batch_get_knobs(sfft_batch b, sfft_batch_knobs* knobs) {
  if (!b || !knobs) return SFFT_ERR_INVALID_ARG;
  *knobs = b->knobs;
  return SFFT_OK;
}

sfft_status sfft_batch_set_pedestals(sfft_batch b, const double* ref_pedestals, const double* sci_pedestals) {
  if (!b || !ref_pedestals || !sci_pedestals) return SFFT_ERR_INVALID_ARG;
  const int n = (int)b->items.size();
  for (int k = 0; k < n; ++k)
    if (!std::isfinite(ref_pedestals[k]) || !std::isfinite(sci_pedestals[k])) return SFFT_ERR_INVALID_ARG;
  sfft_status s;
  if ((s = check_device(b->handle)) != SFFT_OK) return s;
  if (hipDeviceSynchronize() != hipSuccess) return SFFT_ERR_HIP;   // tables in use by queued work
  for (int k = 0; k < n; ++k) {
    b->items[k].desc.ref_pedestal = ref_pedestals[k];
    b->items[k].desc.sci_pedestal = sci_pedestals[k];
  }
  return batch_plan(b, b->knobs);
}

sfft_status sfft_batch_destroy(sfft_batch b) {
  if (!b) return SFFT_ERR_INVALID_ARG;
  batch_release(b);
  delete b;
  return SFFT_OK;
}

sfft_status sfft_profile_events(sfft_handle h, int32_t slot, void* start_event, void* stop_event) {
  if (!h || slot <= 0 || slot >= SFFT_PROF_MAX) return SFFT_ERR_INVALID_ARG;
  if ((start_event == nullptr) != (stop_event == nullptr)) return SFFT_ERR_INVALID_ARG;
  h->prof.start[slot] = start_event;
  h->prof.stop[slot] = stop_event;
  return SFFT_OK;
}

}  // extern "C"
