// avm_api.cpp -- C-ABI of libavm (declared in include/avm.h): argument
// validation, device memory, streams and the host side of the two
// scheduling modes.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <thread>
#include <type_traits>
#include <vector>

#include "avm.h"
#include "avm_internal.hpp"

using namespace avm;

namespace {

thread_local std::string g_err;

avm_status fail(avm_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) return fail(AVM_E_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// Physical constants: speed of light, electron rest energy.
constexpr double kCcmPerNs = 29.9792458;
constexpr double kCmPerS = 299792458.0;
constexpr double kMeC2eV = 510998.95;

double k_a() { return (kCcmPerNs * kCcmPerNs) / kMeC2eV; }       // (cm/ns^2) / (V/cm)
double k_b() { return 1e-9 * (kCmPerS * kCmPerS) / kMeC2eV; }    // rad / (ns T)

// Makes `dev` current for the lifetime of the guard.
struct DeviceGuard {
  int prev = -1;
  hipError_t err = hipSuccess;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    err = hipSetDevice(dev);
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

template <class T>
hipError_t dmalloc(T** p, size_t n) {
  return hipMalloc(reinterpret_cast<void**>(p), sizeof(T) * (n ? n : 1));
}

}  // namespace

struct avm_gas {
  int device = 0;
  double e_max = 0, density = 0, gamma = 0;
  int32_t n_bins = 0, n_ch = 0, band_bins = 0, n_bands = 1;
  double *cum = nullptr, *cum0 = nullptr, *total = nullptr, *band_gamma = nullptr,
         *band_inv = nullptr, *band_edge = nullptr;
  ChanDev* ch = nullptr;
  // FP32 copies for the FP32-mixed path
  float *cum_f = nullptr, *cum0_f = nullptr, *total_f = nullptr, *band_gamma_f = nullptr,
        *band_inv_f = nullptr, *band_edge_f = nullptr;
  ChanP<float>* ch_f = nullptr;
  double* sct = nullptr;     // azimuth table
  double* binmax = nullptr;  // per-bin maxima, kept for rebuilding the bands
  std::vector<ChanDev> host_ch;        // channel records as on the device
  std::vector<ChanP<float>> host_ch_f;
  uint64_t version = 0;      // bumped whenever the device tables change
  GasDev dev{};
};

struct avm_field {
  int device = 0;
  double B[3] = {0, 0, 0};
  double* E = nullptr;
  float *Er = nullptr, *Ephi = nullptr;
  FieldDev dev{};
};

struct avm_run {
  const avm_gas* gas = nullptr;
  const avm_field* field = nullptr;
  avm_run_opts opts{};
  uint64_t n_prim = 0;
  uint32_t n_aval = 0;
  int prim_on_device = 0;
  const PrimaryRec* prim_dev_user = nullptr;
  PrimaryRec* prim_dev = nullptr;   // library copy (host primaries)
  PrimaryRec* prim_host = nullptr;  // pinned staging
  void* store_mem = nullptr;
  Store S{};
  Store* store_dev = nullptr;  // device copy of S (the transport kernels read it there)
  uint32_t *list0 = nullptr, *list1 = nullptr;
  Counters* ctr = nullptr;
  AvalStats* stats = nullptr;
  Totals* tot = nullptr;
  Totals* tot_host = nullptr;      // pinned
  Counters* ctr_host = nullptr;    // pinned
  hipStream_t stream = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr, ev_done = nullptr;
  int executed = 0, synced = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  uint64_t graph_version = 0;  // gas version the graph was captured with
  double* signal = nullptr;     // induced signal [n_aval][n_bins] (avm_run_set_signal)
  SignalDev sigdev{};
  uint32_t iterations = 0;
  double plain_ms = 0.0;
  int grid = 0, block = persistent_block();
  int clock_khz = 100000;  // wall_clock64() rate
};

extern "C" {

const char* avm_last_error(void) { return g_err.c_str(); }
int32_t avm_abi_version(void) { return AVM_ABI_VERSION; }

int32_t avm_device_count(void) {
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess) return 0;
  return n;
}

// ---------------------------------------------------------------------------
// gas
// ---------------------------------------------------------------------------
static void gas_free(avm_gas* g) {
  if (!g) return;
  (void)hipFree(g->cum);
  (void)hipFree(g->cum0);
  (void)hipFree(g->total);
  (void)hipFree(g->band_gamma);
  (void)hipFree(g->band_inv);
  (void)hipFree(g->band_edge);
  (void)hipFree(g->ch);
  (void)hipFree(g->cum_f);
  (void)hipFree(g->cum0_f);
  (void)hipFree(g->total_f);
  (void)hipFree(g->band_gamma_f);
  (void)hipFree(g->band_inv_f);
  (void)hipFree(g->band_edge_f);
  (void)hipFree(g->ch_f);
  (void)hipFree(g->sct);
  (void)hipFree(g->binmax);
  delete g;
}

avm_status avm_gas_create(int32_t device, double e_max_eV, int32_t n_bins, double density_cm3,
                          int32_t n_channels, const avm_channel* ch, int32_t band_bins,
                          avm_gas** out) {
  g_err.clear();
  if (!out) return fail(AVM_E_ARG, "avm_gas_create: out is NULL");
  *out = nullptr;
  if (!ch || n_channels < 1) return fail(AVM_E_ARG, "avm_gas_create: need at least one channel");
  if (n_bins < 1 || n_bins > (1 << 28)) return fail(AVM_E_ARG, "avm_gas_create: n_bins out of range");
  if (!(e_max_eV > 0.0) || !std::isfinite(e_max_eV)) return fail(AVM_E_ARG, "avm_gas_create: e_max must be > 0");
  if (!(density_cm3 >= 0.0) || !std::isfinite(density_cm3)) return fail(AVM_E_ARG, "avm_gas_create: bad density");
  if (band_bins < 0) return fail(AVM_E_ARG, "avm_gas_create: band_bins < 0");
  std::vector<ChanDev> cd(n_channels);
  std::vector<ChanP<float>> cf(n_channels);
  std::vector<int32_t> vk(n_channels);
  const size_t nn = (size_t)n_bins + 1;
  std::vector<double> sig(nn * n_channels);
  for (int c = 0; c < n_channels; ++c) {
    const avm_channel& x = ch[c];
    if (!x.values) return fail(AVM_E_ARG, "channel %d: values is NULL", c);
    if (x.kind < 0 || x.kind > 3) return fail(AVM_E_ARG, "channel %d: bad kind", c);
    if (!(x.e_lo_eV <= x.e_hi_eV)) return fail(AVM_E_ARG, "channel %d: empty window", c);
    if (!(x.loss_eV >= 0.0) || !std::isfinite(x.loss_eV)) return fail(AVM_E_ARG, "channel %d: bad loss", c);
    if ((x.kind == AVM_CH_EXCITATION || x.kind == AVM_CH_IONISATION) && !(x.e_lo_eV >= x.loss_eV))
      return fail(AVM_E_ARG, "channel %d: window opens below the energy loss", c);
    if (x.kind == AVM_CH_ELASTIC && (!(x.mass_ratio >= 0.0) || !std::isfinite(x.mass_ratio)))
      return fail(AVM_E_ARG, "channel %d: bad mass ratio", c);
    if (x.kind == AVM_CH_ELASTIC && x.angular == AVM_ANG_SCREENED_RUTHERFORD && !(x.screening_eV > 0.0))
      return fail(AVM_E_ARG, "channel %d: screened Rutherford needs screening_eV > 0", c);
    if (x.kind == AVM_CH_IONISATION && x.split == AVM_SPLIT_OPAL_BEATY && !(x.split_w_eV > 0.0))
      return fail(AVM_E_ARG, "channel %d: Opal-Beaty split needs w > 0", c);
    if (x.values_kind != AVM_VALUES_SIGMA && x.values_kind != AVM_VALUES_RATE)
      return fail(AVM_E_ARG, "channel %d: bad values_kind", c);
    for (size_t k = 0; k < nn; ++k) {
      const double v = x.values[k];
      if (!(v >= 0.0) || !std::isfinite(v)) return fail(AVM_E_ARG, "channel %d node %zu: bad value", c, k);
      sig[(size_t)c * nn + k] = v;
    }
    ChanDev& d = cd[c];
    d.kind = x.kind;
    d.angular = x.kind == AVM_CH_ELASTIC ? x.angular : 0;
    d.split = x.kind == AVM_CH_IONISATION ? x.split : 0;
    d.loss = x.loss_eV;
    d.e_lo = x.e_lo_eV;
    d.e_hi = x.e_hi_eV;
    const double mu = x.kind == AVM_CH_ELASTIC ? x.mass_ratio : 0.0;
    d.mu = mu;
    d.el_loss = 2.0 * mu / ((1.0 + mu) * (1.0 + mu));
    d.mu2p1 = 1.0 + mu * mu;
    d.two_mu = 2.0 * mu;
    d.split_w = x.split_w_eV;
    d.atan_scale = x.split_w_eV > 0.0 ? 1.0 / (2.0 * x.split_w_eV) : 0.0;
    d.inv_screen8 = x.screening_eV > 0.0 ? 8.0 / x.screening_eV : 0.0;
    ChanP<float>& q = cf[c];
    q.kind = d.kind;
    q.angular = d.angular;
    q.split = d.split;
    q.e_lo = d.e_lo;
    q.e_hi = d.e_hi;
    q.loss = (float)d.loss;
    q.mu = (float)d.mu;
    q.el_loss = (float)d.el_loss;
    q.mu2p1 = (float)d.mu2p1;
    q.two_mu = (float)d.two_mu;
    q.split_w = (float)d.split_w;
    q.atan_scale = (float)d.atan_scale;
    q.inv_screen8 = (float)d.inv_screen8;
    vk[c] = x.values_kind;
  }
  DeviceGuard dg(device);
  if (dg.err != hipSuccess) return fail(AVM_E_HIP, "hipSetDevice(%d): %s", device, hipGetErrorString(dg.err));
  avm_gas* g = new (std::nothrow) avm_gas();
  if (!g) return fail(AVM_E_NOMEM, "host allocation");
  g->device = device;
  g->e_max = e_max_eV;
  g->density = density_cm3;
  g->n_bins = n_bins;
  g->n_ch = n_channels;
  g->band_bins = band_bins;
  g->n_bands = band_bins > 0 ? (n_bins + band_bins - 1) / band_bins : 1;
  double *d_sig = nullptr, *d_gamma = nullptr;
  int32_t* d_vk = nullptr;
  hipStream_t st = nullptr;
  avm_status rc = AVM_OK;
  auto cleanup = [&]() {
    (void)hipFree(d_sig);
    (void)hipFree(d_gamma);
    (void)hipFree(d_vk);
    if (st) (void)hipStreamDestroy(st);
  };
  auto try_hip = [&](hipError_t e, const char* what) {
    if (e != hipSuccess && rc == AVM_OK) rc = fail(e == hipErrorOutOfMemory ? AVM_E_NOMEM : AVM_E_HIP, "%s: %s", what, hipGetErrorString(e));
    return e == hipSuccess;
  };
  bool ok = try_hip(hipStreamCreateWithFlags(&st, hipStreamNonBlocking), "hipStreamCreate") &&
            try_hip(dmalloc(&d_sig, sig.size()), "hipMalloc") && try_hip(dmalloc(&d_vk, n_channels), "hipMalloc") &&
            try_hip(dmalloc(&g->binmax, (size_t)n_bins), "hipMalloc") && try_hip(dmalloc(&d_gamma, 1), "hipMalloc") &&
            try_hip(dmalloc(&g->cum, nn * n_channels), "hipMalloc") && try_hip(dmalloc(&g->total, nn), "hipMalloc") &&
            try_hip(dmalloc(&g->cum0, nn), "hipMalloc") &&
            try_hip(dmalloc(&g->band_gamma, (size_t)g->n_bands), "hipMalloc") &&
            try_hip(dmalloc(&g->band_inv, (size_t)g->n_bands), "hipMalloc") &&
            try_hip(dmalloc(&g->band_edge, (size_t)g->n_bands), "hipMalloc") &&
            try_hip(dmalloc(&g->ch, (size_t)n_channels), "hipMalloc") &&
            try_hip(dmalloc(&g->ch_f, (size_t)n_channels), "hipMalloc") &&
            try_hip(dmalloc(&g->cum_f, nn * n_channels), "hipMalloc") &&
            try_hip(dmalloc(&g->cum0_f, nn), "hipMalloc") && try_hip(dmalloc(&g->total_f, nn), "hipMalloc") &&
            try_hip(dmalloc(&g->band_gamma_f, (size_t)g->n_bands), "hipMalloc") &&
            try_hip(dmalloc(&g->band_inv_f, (size_t)g->n_bands), "hipMalloc") &&
            try_hip(dmalloc(&g->band_edge_f, (size_t)g->n_bands), "hipMalloc") &&
            try_hip(dmalloc(&g->sct, (size_t)(2 * kAzN)), "hipMalloc");
  if (ok)
    ok = try_hip(hipMemcpyAsync(d_sig, sig.data(), sizeof(double) * sig.size(), hipMemcpyHostToDevice, st), "H2D") &&
         try_hip(hipMemcpyAsync(d_vk, vk.data(), sizeof(int32_t) * vk.size(), hipMemcpyHostToDevice, st), "H2D") &&
         try_hip(hipMemcpyAsync(g->ch, cd.data(), sizeof(ChanDev) * cd.size(), hipMemcpyHostToDevice, st), "H2D") &&
         try_hip(hipMemcpyAsync(g->ch_f, cf.data(), sizeof(ChanP<float>) * cf.size(), hipMemcpyHostToDevice, st), "H2D") &&
         try_hip(launch_build_rates(d_sig, d_vk, n_channels, n_bins, e_max_eV, density_cm3, k_a(), g->cum,
                                    g->total, g->binmax, st), "rate-table kernels") &&
         try_hip(launch_build_bands(g->binmax, n_bins, band_bins, g->n_bands, e_max_eV, g->band_gamma,
                                    g->band_inv, g->band_edge, d_gamma, st), "band kernels") &&
         // cumulative column 0, contiguous (staged in LDS by the transport)
         try_hip(hipMemcpy2DAsync(g->cum0, sizeof(double), g->cum, sizeof(double) * n_channels,
                                  sizeof(double), nn, hipMemcpyDeviceToDevice, st), "column copy") &&
         try_hip(launch_tables_f32(g->cum, g->total, g->cum0, nn * n_channels, (int)nn, g->band_gamma,
                                   g->band_edge, g->n_bands, g->cum_f, g->total_f, g->cum0_f,
                                   g->band_gamma_f, g->band_inv_f, g->band_edge_f, st), "FP32 tables") &&
         try_hip(launch_azimuth_table(g->sct, st), "azimuth table");
  double gamma = 0.0;
  if (ok)
    ok = try_hip(hipMemcpyAsync(&gamma, d_gamma, sizeof(double), hipMemcpyDeviceToHost, st), "D2H") &&
         try_hip(hipStreamSynchronize(st), "hipStreamSynchronize");
  cleanup();
  if (!ok) {
    gas_free(g);
    return rc;
  }
  if (!(gamma > 0.0) || !std::isfinite(gamma)) {
    gas_free(g);
    return fail(AVM_E_ARG, "avm_gas_create: the table has no collisions (majorant %g)", gamma);
  }
  g->gamma = gamma;
  g->host_ch = cd;
  g->host_ch_f = cf;
  GasDev& D = g->dev;
  D.cum = g->cum;
  D.cum0 = g->cum0;
  D.total = g->total;
  D.band_gamma = g->band_gamma;
  D.band_inv = g->band_inv;
  D.band_edge = g->band_edge;
  D.ch = g->ch;
  D.scale = (double)n_bins / e_max_eV;
  D.gamma = gamma;
  D.inv_gamma = 1.0 / gamma;
  D.band_scale = band_bins > 0 ? (double)n_bins / (e_max_eV * (double)band_bins) : 0.0;
  D.n_bins = n_bins;
  D.n_ch = n_channels;
  D.n_bands = g->n_bands;
  D.band_bins = band_bins;
  D.cum_f = g->cum_f;
  D.cum0_f = g->cum0_f;
  D.total_f = g->total_f;
  D.band_gamma_f = g->band_gamma_f;
  D.band_inv_f = g->band_inv_f;
  D.band_edge_f = g->band_edge_f;
  D.ch_f = g->ch_f;
  D.sct = g->sct;
  float gf = (float)gamma;
  if ((double)gf < gamma) gf = std::nextafter(gf, INFINITY);  // a majorant stays a majorant
  D.gamma_f = gf;
  D.inv_gamma_f = 1.0f / gf;
  D.scale_f = (float)D.scale;
  D.x_top = (double)n_bins;
  D.x_top_f = (float)n_bins;
  D.band_scale_f = (float)D.band_scale;
  *out = g;
  return AVM_OK;
}

avm_status avm_gas_get_info(const avm_gas* g, avm_gas_info* out) {
  if (!g || !out) return fail(AVM_E_ARG, "avm_gas_get_info: NULL argument");
  out->gamma = g->gamma;
  out->e_max_eV = g->e_max;
  out->n_bins = g->n_bins;
  out->n_channels = g->n_ch;
  out->n_bands = g->n_bands;
  out->band_bins = g->band_bins;
  return AVM_OK;
}

avm_status avm_gas_get_tables(const avm_gas* g, double* cumulative, double* band_gamma,
                              double* band_edge_eV) {
  if (!g) return fail(AVM_E_ARG, "avm_gas_get_tables: gas is NULL");
  DeviceGuard dg(g->device);
  if (cumulative)
    HIP_TRY(hipMemcpy(cumulative, g->cum, sizeof(double) * ((size_t)g->n_bins + 1) * g->n_ch, hipMemcpyDeviceToHost));
  if (band_gamma) HIP_TRY(hipMemcpy(band_gamma, g->band_gamma, sizeof(double) * g->n_bands, hipMemcpyDeviceToHost));
  if (band_edge_eV) HIP_TRY(hipMemcpy(band_edge_eV, g->band_edge, sizeof(double) * g->n_bands, hipMemcpyDeviceToHost));
  return AVM_OK;
}

avm_status avm_gas_set_band_bins(avm_gas* g, int32_t band_bins) {
  g_err.clear();
  if (!g) return fail(AVM_E_ARG, "avm_gas_set_band_bins: gas is NULL");
  if (band_bins < 0) return fail(AVM_E_ARG, "avm_gas_set_band_bins: band_bins < 0");
  DeviceGuard dg(g->device);
  if (dg.err != hipSuccess) return fail(AVM_E_HIP, "hipSetDevice: %s", hipGetErrorString(dg.err));
  const int32_t nb = band_bins > 0 ? (g->n_bins + band_bins - 1) / band_bins : 1;
  double *bg = nullptr, *bi = nullptr, *be = nullptr, *gam = nullptr;
  float *bgf = nullptr, *bif = nullptr, *bef = nullptr;
  hipStream_t st = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
  if (e == hipSuccess) e = dmalloc(&bg, (size_t)nb);
  if (e == hipSuccess) e = dmalloc(&bi, (size_t)nb);
  if (e == hipSuccess) e = dmalloc(&be, (size_t)nb);
  if (e == hipSuccess) e = dmalloc(&gam, 1);
  if (e == hipSuccess) e = dmalloc(&bgf, (size_t)nb);
  if (e == hipSuccess) e = dmalloc(&bif, (size_t)nb);
  if (e == hipSuccess) e = dmalloc(&bef, (size_t)nb);
  if (e == hipSuccess) e = launch_build_bands(g->binmax, g->n_bins, band_bins, nb, g->e_max, bg, bi, be, gam, st);
  if (e == hipSuccess)
    e = launch_tables_f32(nullptr, nullptr, nullptr, 0, 0, bg, be, nb, nullptr, nullptr, nullptr, bgf, bif, bef, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (st) (void)hipStreamDestroy(st);
  (void)hipFree(gam);
  if (e != hipSuccess) {
    for (void* q : {(void*)bg, (void*)bi, (void*)be, (void*)bgf, (void*)bif, (void*)bef}) (void)hipFree(q);
    return fail(e == hipErrorOutOfMemory ? AVM_E_NOMEM : AVM_E_HIP, "avm_gas_set_band_bins: %s", hipGetErrorString(e));
  }
  for (void* q : {(void*)g->band_gamma, (void*)g->band_inv, (void*)g->band_edge, (void*)g->band_gamma_f,
                  (void*)g->band_inv_f, (void*)g->band_edge_f})
    (void)hipFree(q);
  g->band_gamma = bg;
  g->band_inv = bi;
  g->band_edge = be;
  g->band_gamma_f = bgf;
  g->band_inv_f = bif;
  g->band_edge_f = bef;
  g->band_bins = band_bins;
  g->n_bands = nb;
  GasDev& D = g->dev;
  D.band_gamma = bg;
  D.band_inv = bi;
  D.band_edge = be;
  D.band_gamma_f = bgf;
  D.band_inv_f = bif;
  D.band_edge_f = bef;
  D.n_bands = nb;
  D.band_bins = band_bins;
  D.band_scale = band_bins > 0 ? (double)g->n_bins / (g->e_max * (double)band_bins) : 0.0;
  D.band_scale_f = (float)D.band_scale;
  g->version += 1;
  return AVM_OK;
}

avm_status avm_gas_set_penning(avm_gas* g, int32_t channel, double probability, double energy_eV) {
  g_err.clear();
  if (!g) return fail(AVM_E_ARG, "avm_gas_set_penning: gas is NULL");
  if (channel < 0 || channel >= g->n_ch) return fail(AVM_E_ARG, "avm_gas_set_penning: no channel %d", channel);
  if (g->host_ch[channel].kind != AVM_CH_EXCITATION)
    return fail(AVM_E_ARG, "avm_gas_set_penning: channel %d is not an excitation", channel);
  if (!(probability >= 0.0 && probability <= 1.0))
    return fail(AVM_E_ARG, "avm_gas_set_penning: probability outside [0, 1]");
  if (!(energy_eV >= 0.0) || !std::isfinite(energy_eV))
    return fail(AVM_E_ARG, "avm_gas_set_penning: energy must be finite and >= 0");
  DeviceGuard dg(g->device);
  if (dg.err != hipSuccess) return fail(AVM_E_HIP, "hipSetDevice: %s", hipGetErrorString(dg.err));
  ChanDev d = g->host_ch[channel];
  ChanP<float> f = g->host_ch_f[channel];
  d.pen_prob = probability;
  d.pen_e = energy_eV;
  f.pen_prob = (float)probability;
  f.pen_e = (float)energy_eV;
  HIP_TRY(hipMemcpy(g->ch + channel, &d, sizeof d, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(g->ch_f + channel, &f, sizeof f, hipMemcpyHostToDevice));
  g->host_ch[channel] = d;
  g->host_ch_f[channel] = f;
  g->version += 1;
  return AVM_OK;
}

void avm_gas_destroy(avm_gas* g) {
  if (!g) return;
  DeviceGuard dg(g->device);
  gas_free(g);
}

// ---------------------------------------------------------------------------
// fields
// ---------------------------------------------------------------------------
static void field_free(avm_field* f) {
  if (!f) return;
  (void)hipFree(f->E);
  (void)hipFree(f->Er);
  (void)hipFree(f->Ephi);
  delete f;
}

static void set_bfield(avm_field* f, const double* B) {
  FieldDev& D = f->dev;
  if (B) {
    f->B[0] = B[0];
    f->B[1] = B[1];
    f->B[2] = B[2];
  }
  const double bb = f->B[0] * f->B[0] + f->B[1] * f->B[1] + f->B[2] * f->B[2];
  D.has_b = bb > 0.0;
  if (D.has_b) {
    const double bm = std::sqrt(bb);
    for (int i = 0; i < 3; ++i) {
      D.bh[i] = f->B[i] / bm;
      D.Bv[i] = f->B[i];
    }
    D.omega = k_b() * bm;
    D.inv_omega = 1.0 / D.omega;
    D.wd_scale = (k_a() / k_b()) / bb;
  }
}

static bool finite3(const double* B) {
  return !B || (std::isfinite(B[0]) && std::isfinite(B[1]) && std::isfinite(B[2]));
}

avm_status avm_field_slab(int32_t device, double z_lo_cm, double z_hi_cm, uint32_t n_E,
                          const double* E_vcm, const double* B_T, avm_field** out) {
  g_err.clear();
  if (!out) return fail(AVM_E_ARG, "avm_field_slab: out is NULL");
  *out = nullptr;
  if (!E_vcm || n_E < 1) return fail(AVM_E_ARG, "avm_field_slab: need n_E >= 1 field vectors");
  if (!(z_lo_cm < z_hi_cm) || !std::isfinite(z_lo_cm) || !std::isfinite(z_hi_cm))
    return fail(AVM_E_ARG, "avm_field_slab: need finite z_lo < z_hi");
  if (!finite3(B_T)) return fail(AVM_E_ARG, "avm_field_slab: B not finite");
  if (B_T && (B_T[0] != 0.0 || B_T[1] != 0.0))
    return fail(AVM_E_UNSUPPORTED, "avm_field_slab: B must be zero or along z");
  for (size_t i = 0; i < 3 * (size_t)n_E; ++i)
    if (!std::isfinite(E_vcm[i])) return fail(AVM_E_ARG, "avm_field_slab: E not finite");
  DeviceGuard dg(device);
  if (dg.err != hipSuccess) return fail(AVM_E_HIP, "hipSetDevice(%d): %s", device, hipGetErrorString(dg.err));
  avm_field* f = new (std::nothrow) avm_field();
  if (!f) return fail(AVM_E_NOMEM, "host allocation");
  f->device = device;
  hipError_t e = dmalloc(&f->E, 3 * (size_t)n_E);
  if (e == hipSuccess) e = hipMemcpy(f->E, E_vcm, sizeof(double) * 3 * n_E, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    field_free(f);
    return fail(AVM_E_HIP, "avm_field_slab: %s", hipGetErrorString(e));
  }
  FieldDev& D = f->dev;
  D.kind = FIELD_SLAB;
  D.n_E = n_E;
  D.z_lo = z_lo_cm;
  D.z_hi = z_hi_cm;
  D.E = f->E;
  set_bfield(f, B_T);
  *out = f;
  return AVM_OK;
}

avm_status avm_field_polar_map(int32_t device, double a_cm, double b_cm, int32_t n_r, int32_t n_phi,
                               const float* E_r, const float* E_phi, const double* B_T,
                               avm_field** out) {
  g_err.clear();
  if (!out) return fail(AVM_E_ARG, "avm_field_polar_map: out is NULL");
  *out = nullptr;
  if (!E_r || !E_phi) return fail(AVM_E_ARG, "avm_field_polar_map: map is NULL");
  if (!(a_cm > 0.0) || !(b_cm > a_cm) || !std::isfinite(b_cm)) return fail(AVM_E_ARG, "avm_field_polar_map: need 0 < a < b");
  if (n_r < 2 || n_phi < 1 || (int64_t)n_r * n_phi > (1 << 28)) return fail(AVM_E_ARG, "avm_field_polar_map: bad map size");
  if (!finite3(B_T)) return fail(AVM_E_ARG, "avm_field_polar_map: B not finite");
  const size_t n = (size_t)n_r * n_phi;
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(E_r[i]) || !std::isfinite(E_phi[i])) return fail(AVM_E_ARG, "avm_field_polar_map: map not finite");
  DeviceGuard dg(device);
  if (dg.err != hipSuccess) return fail(AVM_E_HIP, "hipSetDevice(%d): %s", device, hipGetErrorString(dg.err));
  avm_field* f = new (std::nothrow) avm_field();
  if (!f) return fail(AVM_E_NOMEM, "host allocation");
  f->device = device;
  hipError_t e = dmalloc(&f->Er, n);
  if (e == hipSuccess) e = dmalloc(&f->Ephi, n);
  if (e == hipSuccess) e = hipMemcpy(f->Er, E_r, sizeof(float) * n, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(f->Ephi, E_phi, sizeof(float) * n, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    field_free(f);
    return fail(AVM_E_HIP, "avm_field_polar_map: %s", hipGetErrorString(e));
  }
  FieldDev& D = f->dev;
  D.kind = FIELD_POLAR;
  D.a = a_cm;
  D.b = b_cm;
  D.a2 = a_cm * a_cm;
  D.b2 = b_cm * b_cm;
  D.inv_dlog = (double)(n_r - 1) / std::log(b_cm / a_cm);
  D.ln_a = std::log(a_cm);
  D.n_r = n_r;
  D.n_phi = n_phi;
  D.Er = f->Er;
  D.Ephi = f->Ephi;
  set_bfield(f, B_T);
  *out = f;
  return AVM_OK;
}

void avm_field_destroy(avm_field* f) {
  if (!f) return;
  DeviceGuard dg(f->device);
  field_free(f);
}

// ---------------------------------------------------------------------------
// runs
// ---------------------------------------------------------------------------
static void run_free(avm_run* r) {
  if (!r) return;
  (void)hipFree(r->store_mem);
  (void)hipFree(r->store_dev);
  (void)hipFree(r->signal);
  (void)hipFree(r->list0);
  (void)hipFree(r->list1);
  (void)hipFree(r->ctr);
  (void)hipFree(r->stats);
  (void)hipFree(r->tot);
  (void)hipFree(r->prim_dev);
  if (r->prim_host) (void)hipHostFree(r->prim_host);
  if (r->tot_host) (void)hipHostFree(r->tot_host);
  if (r->ctr_host) (void)hipHostFree(r->ctr_host);
  if (r->ev0) (void)hipEventDestroy(r->ev0);
  if (r->ev1) (void)hipEventDestroy(r->ev1);
  if (r->ev_done) (void)hipEventDestroy(r->ev_done);
  if (r->graph_exec) (void)hipGraphExecDestroy(r->graph_exec);
  if (r->graph) (void)hipGraphDestroy(r->graph);
  delete r;
}

// Carves the structure-of-arrays electron store out of one allocation.
static size_t layout_store(Store& S, char* base, uint64_t cap) {
  size_t off = 0;
  auto take = [&](auto** p, size_t elem) {
    off = (off + 255) & ~size_t(255);
    if (base) *p = reinterpret_cast<std::remove_pointer_t<decltype(p)>>(base + off);
    off += elem * cap;
  };
  take(&S.x0, 8); take(&S.y0, 8); take(&S.z0, 8); take(&S.t0, 8);
  take(&S.vx0, 8); take(&S.vy0, 8); take(&S.vz0, 8); take(&S.e0, 8);
  take(&S.eid, 8); take(&S.parent, 8); take(&S.aval, 4); take(&S.qready, 4); take(&S.qslot, 4);
  take(&S.end, sizeof(avm_end_record));
  take(&S.vx1, 8); take(&S.vy1, 8); take(&S.vz1, 8);
  take(&S.k1, 4); take(&S.band1, 4);
  S.capacity = cap;
  return off;
}

// Grid of the persistent kernel: blocks per CU from the occupancy limit,
// capped by the requested resident waves per CU, times the CU count.
static hipError_t persistent_grid(const avm_gas* gas, const avm_field* field, const avm_run_opts& o,
                                  int signal, int block, int32_t waves_per_cu, int* grid,
                                  int* blocks_per_cu_max) {
  int per_cu = 0, n_cu = 0, dev = 0;
  hipError_t e = persistent_occupancy(o.precision == AVM_FP32_MIXED, o.majorant == AVM_MAJORANT_BANDED,
                                      field->dev.kind, signal, tables_fit_lds(gas->dev), block, &per_cu);
  if (e == hipSuccess) e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  if (per_cu < 1) per_cu = 1;
  if (blocks_per_cu_max) *blocks_per_cu_max = per_cu;
  const int waves_per_block = block / 64;
  if (waves_per_cu > 0) {
    const int want = (waves_per_cu + waves_per_block - 1) / waves_per_block;
    per_cu = want < per_cu ? want : per_cu;
  }
  *grid = per_cu * n_cu;
  return hipSuccess;
}

static hipError_t batched_grid(const avm_run* r, int32_t waves_per_cu, int* grid, int* blocks_per_cu_max) {
  return persistent_grid(r->gas, r->field, r->opts, r->signal != nullptr, r->block, waves_per_cu, grid,
                         blocks_per_cu_max);
}

// Checks the run options against the gas, field and sizes, and fills in
// their defaults (shared by avm_run_create and avm_run_noalloc).
static avm_status check_opts(const char* fn, const avm_gas* gas, const avm_field* field, uint64_t n_prim,
                             uint32_t n_aval, avm_run_opts& o) {
  if (field->dev.kind == FIELD_SLAB && field->dev.n_E > 1 && n_aval > field->dev.n_E)
    return fail(AVM_E_ARG, "%s: %u avalanches but %u field vectors", fn, n_aval, field->dev.n_E);
  if (o.precision != AVM_FP64 && o.precision != AVM_FP32_MIXED) return fail(AVM_E_ARG, "%s: bad precision", fn);
  if (o.mode != AVM_MODE_PLAIN && o.mode != AVM_MODE_BATCHED) return fail(AVM_E_ARG, "%s: bad mode", fn);
  if (o.majorant != AVM_MAJORANT_GLOBAL && o.majorant != AVM_MAJORANT_BANDED) return fail(AVM_E_ARG, "%s: bad majorant", fn);
  if (o.majorant == AVM_MAJORANT_BANDED && gas->n_bands < 2)
    return fail(AVM_E_ARG, "%s: banded majorant needs a gas built with band_bins > 0", fn);
  if (o.majorant == AVM_MAJORANT_BANDED && field->dev.has_b && field->dev.kind == FIELD_SLAB)
    return fail(AVM_E_UNSUPPORTED, "%s: banded majorant with B needs the polar-map geometry", fn);
  if (o.k_max == 0) o.k_max = (1u << 30) - 1u;
  if (o.k_max > (1u << 30) - 1u) return fail(AVM_E_ARG, "%s: k_max > 2^30-1", fn);
  if (std::isnan(o.t_max_ns)) return fail(AVM_E_ARG, "%s: t_max is NaN", fn);
  if (o.capacity < n_prim) return fail(AVM_E_ARG, "%s: capacity %llu < %llu primaries", fn, (unsigned long long)o.capacity, (unsigned long long)n_prim);
  if (o.capacity > 0xFFFFFFF0ull) return fail(AVM_E_ARG, "%s: capacity above 2^32-16", fn);
  if (o.flights_per_pass <= 0) o.flights_per_pass = default_flights_per_pass(o.precision);
  if (o.waves_per_cu < 0) return fail(AVM_E_ARG, "%s: waves_per_cu < 0", fn);
  if (!(o.band_lookahead >= 0.0f) || !std::isfinite(o.band_lookahead))
    return fail(AVM_E_ARG, "%s: band_lookahead must be finite and >= 0", fn);
  if (o.graph && o.mode != AVM_MODE_BATCHED)
    return fail(AVM_E_ARG, "%s: graph capture needs the batched mode (the plain mode reads the host)", fn);
  return AVM_OK;
}

// Transport parameters of a run: seed, limits, constants, the device time
// budget (wall_clock64 ticks at `clock_khz`), the band lookahead.
static RunParams run_params_of(const avm_run_opts& o, int clock_khz) {
  RunParams P{};
  P.key0 = (uint32_t)o.seed;
  P.key1 = (uint32_t)(o.seed >> 32);
  P.k_max = o.k_max;
  P.banded = o.majorant == AVM_MAJORANT_BANDED;
  P.t_max = o.t_max_ns;
  P.k_a = k_a();
  P.two_ka = 2.0 * P.k_a;
  P.inv_2ka = 1.0 / P.two_ka;
  P.k_a_f = (float)P.k_a;
  P.two_ka_f = (float)P.two_ka;
  P.inv_2ka_f = (float)P.inv_2ka;
  // device time budget of one transport kernel: the caller's timeout, else
  // a hard cap; a kernel past it stops and the run reports AVM_E_TIMEOUT
  const double budget_s = o.timeout_s > 0.0 ? o.timeout_s : 600.0;
  P.budget_ticks = (uint64_t)(budget_s * 1e3 * (double)clock_khz);
  P.look = o.majorant == AVM_MAJORANT_BANDED ? (double)o.band_lookahead : 0.0;
  return P;
}

avm_status avm_run_create(const avm_gas* gas, const avm_field* field, const avm_primary* prim,
                          int32_t prim_on_device, uint64_t n_prim, uint32_t n_aval,
                          const avm_run_opts* opts, avm_run** out) {
  g_err.clear();
  if (!out) return fail(AVM_E_ARG, "avm_run_create: out is NULL");
  *out = nullptr;
  if (!gas || !field || !opts) return fail(AVM_E_ARG, "avm_run_create: NULL gas, field or opts");
  if (gas->device != field->device) return fail(AVM_E_ARG, "avm_run_create: gas and field on different devices");
  if (n_prim && !prim) return fail(AVM_E_ARG, "avm_run_create: primaries are NULL");
  if (n_aval == 0 && n_prim) return fail(AVM_E_ARG, "avm_run_create: n_aval = 0");
  avm_run_opts o = *opts;
  if (o.capacity == 0) o.capacity = n_prim * 64 > (1u << 20) ? n_prim * 64 : (1u << 20);
  const avm_status cs = check_opts("avm_run_create", gas, field, n_prim, n_aval, o);
  if (cs != AVM_OK) return cs;
  if (!prim_on_device)
    for (uint64_t i = 0; i < n_prim; ++i) {
      const avm_primary& p = prim[i];
      if (p.avalanche >= n_aval) return fail(AVM_E_ARG, "primary %llu: avalanche %u >= n_aval", (unsigned long long)i, p.avalanche);
      if (!std::isfinite(p.x) || !std::isfinite(p.y) || !std::isfinite(p.z) || !std::isfinite(p.t) ||
          !(p.e >= 0.0) || !std::isfinite(p.e) || !std::isfinite(p.dx) || !std::isfinite(p.dy) || !std::isfinite(p.dz))
        return fail(AVM_E_ARG, "primary %llu: non-finite or negative value", (unsigned long long)i);
    }
  DeviceGuard dg(gas->device);
  if (dg.err != hipSuccess) return fail(AVM_E_HIP, "hipSetDevice: %s", hipGetErrorString(dg.err));
  avm_run* r = new (std::nothrow) avm_run();
  if (!r) return fail(AVM_E_NOMEM, "host allocation");
  r->gas = gas;
  r->field = field;
  r->opts = o;
  r->n_prim = n_prim;
  r->n_aval = n_aval;
  r->prim_on_device = prim_on_device;
  r->stream = static_cast<hipStream_t>(o.hip_stream);
  const uint64_t cap = o.capacity;
  const size_t bytes = layout_store(r->S, nullptr, cap);
  hipError_t e = hipMalloc(&r->store_mem, bytes);
  if (e == hipSuccess) layout_store(r->S, static_cast<char*>(r->store_mem), cap);
  if (e == hipSuccess) e = hipMemset(r->S.qready, 0, sizeof(uint32_t) * cap);
  if (e == hipSuccess) e = dmalloc(&r->stats, n_aval ? n_aval : 1);
  if (e == hipSuccess) e = dmalloc(&r->tot, 1);
  r->S.stats = r->stats;
  r->S.tot = r->tot;
  if (e == hipSuccess) e = dmalloc(&r->store_dev, 1);
  if (e == hipSuccess) e = hipMemcpy(r->store_dev, &r->S, sizeof(Store), hipMemcpyHostToDevice);
  if (e == hipSuccess && o.mode == AVM_MODE_PLAIN) e = dmalloc(&r->list0, cap);
  if (e == hipSuccess && o.mode == AVM_MODE_PLAIN) e = dmalloc(&r->list1, cap);
  if (e == hipSuccess) e = dmalloc(&r->ctr, 1);
  if (e == hipSuccess) e = hipMemset(r->ctr, 0, sizeof(Counters));
  if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&r->tot_host), sizeof(Totals), hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&r->ctr_host), sizeof(Counters), hipHostMallocDefault);
  if (e == hipSuccess && !prim_on_device && n_prim) {
    e = dmalloc(&r->prim_dev, n_prim);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&r->prim_host), sizeof(PrimaryRec) * n_prim, hipHostMallocDefault);
    if (e == hipSuccess) std::memcpy(r->prim_host, prim, sizeof(PrimaryRec) * n_prim);
  }
  if (e == hipSuccess) {
    int dev = 0, khz = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && khz > 0)
      r->clock_khz = khz;
  }
  if (e == hipSuccess) e = hipEventCreate(&r->ev0);
  if (e == hipSuccess) e = hipEventCreate(&r->ev1);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&r->ev_done, hipEventDisableTiming);
  if (e == hipSuccess && o.mode == AVM_MODE_BATCHED) e = batched_grid(r, o.waves_per_cu, &r->grid, nullptr);
  if (e != hipSuccess) {
    const avm_status st = e == hipErrorOutOfMemory ? AVM_E_NOMEM : AVM_E_HIP;
    run_free(r);
    return fail(st, "avm_run_create: %s", hipGetErrorString(e));
  }
  if (prim_on_device) r->prim_dev_user = reinterpret_cast<const PrimaryRec*>(prim);
  *out = r;
  return AVM_OK;
}

static RunParams run_params(const avm_run* r) { return run_params_of(r->opts, r->clock_khz); }

// The batched run's device work, in stream order: primaries (if on the
// host), reset, primary load, persistent transport (which also adds up the
// statistics as electrons terminate), result copies.
static avm_status enqueue_batched(avm_run* r, hipStream_t st, bool timed) {
  const PrimaryRec* pd = r->prim_dev_user;
  if (!r->prim_on_device && r->n_prim) {
    HIP_TRY(hipMemcpyAsync(r->prim_dev, r->prim_host, sizeof(PrimaryRec) * r->n_prim, hipMemcpyHostToDevice, st));
    pd = r->prim_dev;
  }
  HIP_TRY(launch_reset(r->ctr, r->n_prim, r->stats, r->n_aval, r->tot, st));
  HIP_TRY(launch_load_primaries(pd, r->n_prim, r->S, k_a(), r->n_aval, r->list0, r->ctr, 0, st));
  const RunParams P = run_params(r);
  if (r->signal) HIP_TRY(launch_zero(r->signal, (size_t)r->n_aval * (size_t)r->sigdev.n_bins, st));
  if (timed) HIP_TRY(hipEventRecord(r->ev0, st));
  HIP_TRY(launch_persistent(r->opts.precision == AVM_FP32_MIXED, r->opts.majorant == AVM_MAJORANT_BANDED,
                            r->field->dev.kind, r->gas->dev, r->field->dev, P, r->store_dev, r->ctr,
                            r->opts.flights_per_pass, r->signal ? &r->sigdev : nullptr, r->grid,
                            r->block, st));
  if (timed) HIP_TRY(hipEventRecord(r->ev1, st));
  HIP_TRY(hipMemcpyAsync(r->tot_host, r->tot, sizeof(Totals), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(r->ctr_host, r->ctr, sizeof(Counters), hipMemcpyDeviceToHost, st));
  return AVM_OK;
}

avm_status avm_run_execute(avm_run* r) {
  g_err.clear();
  if (!r) return fail(AVM_E_ARG, "avm_run_execute: run is NULL");
  if (r->opts.majorant == AVM_MAJORANT_BANDED && r->gas->n_bands < 2)
    return fail(AVM_E_STATE, "avm_run_execute: banded majorant but the gas has no bands now");
  DeviceGuard dg(r->gas->device);
  hipStream_t st = r->stream;
  r->executed = 1;
  r->synced = 0;
  if (r->opts.mode == AVM_MODE_BATCHED) {
    if (r->graph_exec && r->graph_version != r->gas->version) {
      // the gas tables moved since the capture: capture again
      (void)hipGraphExecDestroy(r->graph_exec);
      (void)hipGraphDestroy(r->graph);
      r->graph_exec = nullptr;
      r->graph = nullptr;
    }
    if (!r->opts.graph) {
      avm_status s = enqueue_batched(r, st, true);
      if (s != AVM_OK) return s;
    } else {
      if (!r->graph_exec) {
        // capture once on a private stream, replay on the run's stream
        hipStream_t cs = nullptr;
        HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        avm_status s = e == hipSuccess ? enqueue_batched(r, cs, false) : AVM_E_HIP;
        hipGraph_t g = nullptr;
        const hipError_t e2 = hipStreamEndCapture(cs, &g);
        (void)hipStreamDestroy(cs);
        if (e != hipSuccess) return fail(AVM_E_HIP, "hipStreamBeginCapture: %s", hipGetErrorString(e));
        if (s != AVM_OK) {
          if (g) (void)hipGraphDestroy(g);
          return s;
        }
        if (e2 != hipSuccess) return fail(AVM_E_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e2));
        r->graph = g;
        r->graph_version = r->gas->version;
        HIP_TRY(hipGraphInstantiate(&r->graph_exec, g, nullptr, nullptr, 0));
      }
      HIP_TRY(hipEventRecord(r->ev0, st));
      HIP_TRY(hipGraphLaunch(r->graph_exec, st));
      HIP_TRY(hipEventRecord(r->ev1, st));
    }
    r->iterations = 1;
    HIP_TRY(hipEventRecord(r->ev_done, st));
    return AVM_OK;
  }
  // plain mode: the paper's loop -- transport every active electron to its
  // next ionisation or termination, then rebuild the active list, until
  // none is left; the host reads the list size after each iteration
  const PrimaryRec* pd = r->prim_dev_user;
  if (!r->prim_on_device && r->n_prim) {
    HIP_TRY(hipMemcpyAsync(r->prim_dev, r->prim_host, sizeof(PrimaryRec) * r->n_prim, hipMemcpyHostToDevice, st));
    pd = r->prim_dev;
  }
  HIP_TRY(launch_reset(r->ctr, r->n_prim, r->stats, r->n_aval, r->tot, st));
  HIP_TRY(launch_load_primaries(pd, r->n_prim, r->S, k_a(), r->n_aval, r->list0, r->ctr, 1, st));
  const RunParams P = run_params(r);
  const int banded = r->opts.majorant == AVM_MAJORANT_BANDED;
  const int fk = r->field->dev.kind;
  const int fp32 = r->opts.precision == AVM_FP32_MIXED;
  uint64_t n_active = r->n_prim;
  uint32_t *A = r->list0, *B = r->list1;
  r->iterations = 0;
  r->plain_ms = 0.0;
  while (n_active > 0) {
    HIP_TRY(hipMemsetAsync(&r->ctr->next, 0, sizeof(unsigned long long), st));
    HIP_TRY(hipEventRecord(r->ev0, st));
    HIP_TRY(launch_generation(fp32, banded, fk, r->gas->dev, r->field->dev, P, r->store_dev, A, (uint32_t)n_active, B, r->ctr, st));
    HIP_TRY(hipEventRecord(r->ev1, st));
    HIP_TRY(hipMemcpyAsync(r->ctr_host, r->ctr, sizeof(Counters), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, r->ev0, r->ev1));
    r->plain_ms += ms;
    r->iterations += 1;
    n_active = r->ctr_host->next;
    if (r->ctr_host->timeout) break;
    uint32_t* t = A;
    A = B;
    B = t;
  }
  HIP_TRY(hipMemcpyAsync(r->tot_host, r->tot, sizeof(Totals), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(r->ctr_host, r->ctr, sizeof(Counters), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipEventRecord(r->ev_done, st));
  return AVM_OK;
}

avm_status avm_run_sync(avm_run* r) {
  g_err.clear();
  if (!r) return fail(AVM_E_ARG, "avm_run_sync: run is NULL");
  if (!r->executed) return fail(AVM_E_STATE, "avm_run_sync: run not executed");
  DeviceGuard dg(r->gas->device);
  if (r->opts.timeout_s > 0.0) {
    const auto t0 = std::chrono::steady_clock::now();
    for (;;) {
      const hipError_t q = hipEventQuery(r->ev_done);
      if (q == hipSuccess) break;
      if (q != hipErrorNotReady) return fail(AVM_E_HIP, "hipEventQuery: %s", hipGetErrorString(q));
      const double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      if (el > r->opts.timeout_s) return fail(AVM_E_TIMEOUT, "avm_run_sync: run still busy after %.1f s", el);
      std::this_thread::sleep_for(std::chrono::microseconds(200));
    }
  } else {
    HIP_TRY(hipEventSynchronize(r->ev_done));
  }
  r->synced = 1;
  if (r->ctr_host->timeout) return fail(AVM_E_TIMEOUT, "avm_run_sync: a transport kernel exceeded its time budget");
  if (r->ctr_host->err) return fail(AVM_E_ARG, "avm_run_sync: %llu primaries had an avalanche id >= n_aval", r->ctr_host->err);
  if (r->ctr_host->tail > r->S.capacity)
    return fail(AVM_E_CAPACITY, "avm_run_sync: %llu electrons requested, capacity %llu", r->ctr_host->tail, (unsigned long long)r->S.capacity);
  return AVM_OK;
}

avm_status avm_run_counts(const avm_run* r, avm_counts* out) {
  if (!r || !out) return fail(AVM_E_ARG, "avm_run_counts: NULL argument");
  if (!r->synced) return fail(AVM_E_STATE, "avm_run_counts: call avm_run_sync first");
  std::memset(out, 0, sizeof *out);
  const Totals& T = *r->tot_host;
  out->n_endpoints = T.c[0];
  out->n_ion = T.c[1];
  out->n_att = T.c[2];
  out->n_real = T.c[3];
  out->n_null = T.c[4];
  out->n_masked = T.c[5];
  out->n_band = T.c[6];
  out->n_overflow = T.c[7];
  for (int i = 0; i < 9; ++i) out->n_status[i] = T.status[i];
  out->n_requested = r->ctr_host->tail;
  out->truncated = r->ctr_host->tail > r->S.capacity;
  return AVM_OK;
}

avm_status avm_run_avalanche_counts(const avm_run* r, uint32_t first, uint32_t n, avm_counts* out) {
  if (!r || (!out && n)) return fail(AVM_E_ARG, "avm_run_avalanche_counts: NULL argument");
  if (!r->synced) return fail(AVM_E_STATE, "avm_run_avalanche_counts: call avm_run_sync first");
  if ((uint64_t)first + n > r->n_aval) return fail(AVM_E_ARG, "avm_run_avalanche_counts: range beyond n_aval");
  if (n == 0) return AVM_OK;
  DeviceGuard dg(r->gas->device);
  std::vector<AvalStats> h(n);
  HIP_TRY(hipMemcpy(h.data(), r->stats + first, sizeof(AvalStats) * n, hipMemcpyDeviceToHost));
  for (uint32_t i = 0; i < n; ++i) {
    avm_counts& c = out[i];
    std::memset(&c, 0, sizeof c);
    c.n_endpoints = h[i].c[0];
    c.n_ion = h[i].c[1];
    c.n_att = h[i].c[2];
    c.n_real = h[i].c[3];
    c.n_null = h[i].c[4];
    c.n_masked = h[i].c[5];
    c.n_band = h[i].c[6];
    c.n_overflow = h[i].c[7];
  }
  return AVM_OK;
}

avm_status avm_run_num_endpoints(const avm_run* r, uint64_t* n) {
  if (!r || !n) return fail(AVM_E_ARG, "avm_run_num_endpoints: NULL argument");
  if (!r->synced) return fail(AVM_E_STATE, "avm_run_num_endpoints: call avm_run_sync first");
  *n = r->ctr_host->tail < r->S.capacity ? r->ctr_host->tail : r->S.capacity;
  return AVM_OK;
}

avm_status avm_run_endpoints(const avm_run* r, uint64_t first, uint64_t n, avm_endpoint* out) {
  if (!r || (!out && n)) return fail(AVM_E_ARG, "avm_run_endpoints: NULL argument");
  uint64_t total = 0;
  avm_status s = avm_run_num_endpoints(r, &total);
  if (s != AVM_OK) return s;
  if (first > total || n > total - first) return fail(AVM_E_ARG, "avm_run_endpoints: range beyond the stored endpoints");
  if (n == 0) return AVM_OK;
  DeviceGuard dg(r->gas->device);
  const Store& S = r->S;
  std::vector<double> d(n);
  std::vector<uint64_t> q(n);
  std::vector<uint32_t> u(n);
  auto getd = [&](const double* src, size_t off) -> avm_status {
    HIP_TRY(hipMemcpy(d.data(), src + first, sizeof(double) * n, hipMemcpyDeviceToHost));
    for (uint64_t i = 0; i < n; ++i) std::memcpy(reinterpret_cast<char*>(&out[i]) + off, &d[i], 8);
    return AVM_OK;
  };
  auto getq = [&](const uint64_t* src, size_t off) -> avm_status {
    HIP_TRY(hipMemcpy(q.data(), src + first, sizeof(uint64_t) * n, hipMemcpyDeviceToHost));
    for (uint64_t i = 0; i < n; ++i) std::memcpy(reinterpret_cast<char*>(&out[i]) + off, &q[i], 8);
    return AVM_OK;
  };
  auto getu = [&](const uint32_t* src, size_t off) -> avm_status {
    HIP_TRY(hipMemcpy(u.data(), src + first, sizeof(uint32_t) * n, hipMemcpyDeviceToHost));
    for (uint64_t i = 0; i < n; ++i) std::memcpy(reinterpret_cast<char*>(&out[i]) + off, &u[i], 4);
    return AVM_OK;
  };
#define AVM_GET(fn, arr, field) \
  if ((s = fn(S.arr, offsetof(avm_endpoint, field))) != AVM_OK) return s
  AVM_GET(getd, x0, x0); AVM_GET(getd, y0, y0); AVM_GET(getd, z0, z0); AVM_GET(getd, t0, t0);
  AVM_GET(getd, e0, e0);
  AVM_GET(getq, eid, eid); AVM_GET(getq, parent, parent);
  AVM_GET(getu, aval, avalanche);
#undef AVM_GET
  std::vector<avm_end_record> rec(n);
  HIP_TRY(hipMemcpy(rec.data(), S.end + first, sizeof(avm_end_record) * n, hipMemcpyDeviceToHost));
  for (uint64_t i = 0; i < n; ++i) {
    const avm_end_record& c = rec[i];
    avm_endpoint& o = out[i];
    o.x1 = c.x1; o.y1 = c.y1; o.z1 = c.z1; o.t1 = c.t1; o.e1 = c.e1;
    o.status = c.status; o.n_real = c.n_real; o.n_ion = c.n_ion; o.n_null = c.n_null;
    o.n_masked = c.n_masked; o.n_band = c.n_band; o.n_overflow = c.n_overflow; o.trace = c.trace;
  }
  return AVM_OK;
}

avm_status avm_run_endpoint_arrays(const avm_run* r, avm_endpoint_arrays* out) {
  if (!r || !out) return fail(AVM_E_ARG, "avm_run_endpoint_arrays: NULL argument");
  const Store& S = r->S;
  out->x0 = S.x0; out->y0 = S.y0; out->z0 = S.z0; out->t0 = S.t0; out->e0 = S.e0;
  out->eid = S.eid; out->parent = S.parent; out->avalanche = S.aval; out->end = S.end;
  return AVM_OK;
}

avm_status avm_run_set_signal(avm_run* r, double t0_ns, double dt_ns, int32_t n_bins) {
  g_err.clear();
  if (!r) return fail(AVM_E_ARG, "avm_run_set_signal: run is NULL");
  if (r->opts.mode != AVM_MODE_BATCHED)
    return fail(AVM_E_UNSUPPORTED, "avm_run_set_signal: the induced signal needs the batched mode");
  if (r->executed && !r->synced) return fail(AVM_E_STATE, "avm_run_set_signal: the run is executing");
  if (n_bins < 1) return fail(AVM_E_ARG, "avm_run_set_signal: n_bins < 1");
  if (!(dt_ns > 0.0) || !std::isfinite(dt_ns) || !std::isfinite(t0_ns))
    return fail(AVM_E_ARG, "avm_run_set_signal: need finite t0 and dt > 0");
  DeviceGuard dg(r->gas->device);
  if (dg.err != hipSuccess) return fail(AVM_E_HIP, "hipSetDevice: %s", hipGetErrorString(dg.err));
  double* buf = nullptr;
  const size_t n = (size_t)(r->n_aval ? r->n_aval : 1) * (size_t)n_bins;
  hipError_t e = dmalloc(&buf, n);
  if (e != hipSuccess) return fail(e == hipErrorOutOfMemory ? AVM_E_NOMEM : AVM_E_HIP, "avm_run_set_signal: %s", hipGetErrorString(e));
  (void)hipFree(r->signal);
  r->signal = buf;
  SignalDev& Q = r->sigdev;
  Q.out = buf;
  Q.t0 = t0_ns;
  Q.dt = dt_ns;
  Q.n_bins = n_bins;
  const FieldDev& F = r->field->dev;
  if (F.kind == FIELD_SLAB) {
    Q.w0 = F.z_lo;
    Q.w1 = F.z_hi - F.z_lo;
  } else {
    Q.w0 = std::log(F.b);
    Q.w1 = std::log(F.b / F.a);
  }
  e = batched_grid(r, r->opts.waves_per_cu, &r->grid, nullptr);
  if (e != hipSuccess) return fail(AVM_E_HIP, "avm_run_set_signal: %s", hipGetErrorString(e));
  if (r->graph_exec) {  // captured with the old kernel arguments
    (void)hipGraphExecDestroy(r->graph_exec);
    (void)hipGraphDestroy(r->graph);
    r->graph_exec = nullptr;
    r->graph = nullptr;
  }
  r->synced = 0;
  r->executed = 0;
  return AVM_OK;
}

avm_status avm_run_signal(const avm_run* r, uint32_t first, uint32_t n, double* out) {
  if (!r || (!out && n)) return fail(AVM_E_ARG, "avm_run_signal: NULL argument");
  if (!r->signal) return fail(AVM_E_STATE, "avm_run_signal: no signal requested (avm_run_set_signal)");
  if (!r->synced) return fail(AVM_E_STATE, "avm_run_signal: call avm_run_sync first");
  if ((uint64_t)first + n > r->n_aval) return fail(AVM_E_ARG, "avm_run_signal: avalanches beyond n_aval");
  if (!n) return AVM_OK;
  DeviceGuard dg(r->gas->device);
  const size_t nb = (size_t)r->sigdev.n_bins;
  HIP_TRY(hipMemcpy(out, r->signal + (size_t)first * nb, sizeof(double) * nb * n, hipMemcpyDeviceToHost));
  return AVM_OK;
}

avm_status avm_run_set_seed(avm_run* r, uint64_t seed) {
  g_err.clear();
  if (!r) return fail(AVM_E_ARG, "avm_run_set_seed: run is NULL");
  if (r->executed && !r->synced) return fail(AVM_E_STATE, "avm_run_set_seed: the run is executing");
  if (r->opts.seed == seed) return AVM_OK;
  r->opts.seed = seed;
  if (r->graph_exec) {  // captured with the old seed in the kernel arguments
    DeviceGuard dg(r->gas->device);
    (void)hipGraphExecDestroy(r->graph_exec);
    (void)hipGraphDestroy(r->graph);
    r->graph_exec = nullptr;
    r->graph = nullptr;
  }
  r->synced = 0;
  r->executed = 0;
  return AVM_OK;
}

avm_status avm_run_timing(const avm_run* r, double* transport_ms, uint32_t* iterations) {
  if (!r) return fail(AVM_E_ARG, "avm_run_timing: run is NULL");
  if (!r->synced) return fail(AVM_E_STATE, "avm_run_timing: call avm_run_sync first");
  if (transport_ms) {
    if (r->opts.mode == AVM_MODE_PLAIN) {
      *transport_ms = r->plain_ms;
    } else {
      float ms = 0.f;
      DeviceGuard dg(r->gas->device);
      HIP_TRY(hipEventElapsedTime(&ms, r->ev0, r->ev1));
      *transport_ms = ms;
    }
  }
  if (iterations) *iterations = r->iterations;
  return AVM_OK;
}

void avm_run_destroy(avm_run* r) {
  if (!r) return;
  DeviceGuard dg(r->gas->device);
  if (r->executed && !r->synced) (void)hipEventSynchronize(r->ev_done);
  run_free(r);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// no-allocation runs: validation and launch parameters (the entry point
// itself is in avm_noalloc.hip, beside its scratch array)
// ---------------------------------------------------------------------------
avm_status avm::set_error(avm_status st, const char* msg) {
  g_err = msg ? msg : "";
  return st;
}

avm_status avm::noalloc_setup(const avm_gas* gas, const avm_field* field, uint64_t n_prim, uint32_t n_aval,
                              const avm_run_opts* opts, uint64_t max_electrons, NoallocSetup* out) {
  g_err.clear();
  if (!gas || !field || !opts || !out) return fail(AVM_E_ARG, "avm_run_noalloc: NULL argument");
  if (gas->device != field->device) return fail(AVM_E_ARG, "avm_run_noalloc: gas and field on different devices");
  if (n_aval == 0 && n_prim) return fail(AVM_E_ARG, "avm_run_noalloc: n_aval = 0");
  avm_run_opts o = *opts;
  if (o.mode != AVM_MODE_BATCHED) return fail(AVM_E_ARG, "avm_run_noalloc: only the batched mode allocates nothing");
  if (o.graph) return fail(AVM_E_ARG, "avm_run_noalloc: graph must be 0 (a caller may capture the call itself)");
  if (o.capacity == 0) return fail(AVM_E_ARG, "avm_run_noalloc: capacity must be the length of the output arrays");
  if (o.capacity > max_electrons)
    return fail(AVM_E_ARG, "avm_run_noalloc: capacity %llu above the scratch limit %llu",
                (unsigned long long)o.capacity, (unsigned long long)max_electrons);
  const avm_status cs = check_opts("avm_run_noalloc", gas, field, n_prim, n_aval, o);
  if (cs != AVM_OK) return cs;
  DeviceGuard dg(gas->device);
  if (dg.err != hipSuccess) return fail(AVM_E_HIP, "hipSetDevice: %s", hipGetErrorString(dg.err));
  NoallocSetup& S = *out;
  S.device = gas->device;
  S.gas = gas->dev;
  S.field = field->dev;
  int khz = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, gas->device) != hipSuccess || khz <= 0)
    khz = 100000;
  S.params = run_params_of(o, khz);
  S.fp32 = o.precision == AVM_FP32_MIXED;
  S.banded = o.majorant == AVM_MAJORANT_BANDED;
  S.field_kind = field->dev.kind;
  S.flights_per_pass = o.flights_per_pass;
  S.block = persistent_block();
  S.k_a = k_a();
  HIP_TRY(persistent_grid(gas, field, o, 0, S.block, o.waves_per_cu, &S.grid, nullptr));
  return AVM_OK;
}

// ---------------------------------------------------------------------------
// autotuning
// ---------------------------------------------------------------------------
namespace {

struct Fnv {
  uint64_t h = 0xcbf29ce484222325ull;
  void bytes(const void* p, size_t n) {
    const unsigned char* c = static_cast<const unsigned char*>(p);
    for (size_t i = 0; i < n; ++i) {
      h ^= c[i];
      h *= 0x100000001b3ull;
    }
  }
  template <class T>
  void val(const T& v) { bytes(&v, sizeof v); }
};

template <class T>
hipError_t hash_device(Fnv& f, const T* p, size_t n) {
  if (!p || !n) return hipSuccess;
  std::vector<T> h(n);
  const hipError_t e = hipMemcpy(h.data(), p, sizeof(T) * n, hipMemcpyDeviceToHost);
  if (e == hipSuccess) f.bytes(h.data(), sizeof(T) * n);
  return e;
}

// Key of a tuning problem: device, gas tables, field, primaries, options
// that change the work (not the seed).
hipError_t tune_key(const avm_gas* g, const avm_field* fl, const avm_primary* prim, int32_t on_dev,
                    uint64_t n_prim, uint32_t n_aval, const avm_run_opts& o, uint32_t flags, uint64_t* key) {
  Fnv f;
  int dev = 0;
  hipDeviceProp_t prop{};
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipGetDeviceProperties(&prop, dev);
  if (e != hipSuccess) return e;
  f.bytes(prop.gcnArchName, std::strlen(prop.gcnArchName));
  f.val(prop.multiProcessorCount);
  f.val(g->n_bins); f.val(g->n_ch); f.val(g->e_max); f.val(g->density);
  e = hash_device(f, g->cum, ((size_t)g->n_bins + 1) * (size_t)g->n_ch);
  if (e == hipSuccess) e = hash_device(f, g->ch, (size_t)g->n_ch);
  const FieldDev& F = fl->dev;
  f.val(F.kind); f.val(F.n_E); f.val(F.z_lo); f.val(F.z_hi); f.val(F.a); f.val(F.b);
  f.val(F.n_r); f.val(F.n_phi); f.bytes(fl->B, sizeof fl->B);
  if (e == hipSuccess) e = hash_device(f, F.E, (size_t)F.n_E * 3);
  if (e == hipSuccess) e = hash_device(f, F.Er, (size_t)F.n_r * (size_t)F.n_phi);
  if (e == hipSuccess) e = hash_device(f, F.Ephi, (size_t)F.n_r * (size_t)F.n_phi);
  f.val(n_prim); f.val(n_aval);
  if (e == hipSuccess && n_prim) {
    if (on_dev)
      e = hash_device(f, reinterpret_cast<const PrimaryRec*>(prim), n_prim);
    else
      f.bytes(prim, sizeof(avm_primary) * n_prim);
  }
  f.val(o.precision); f.val(o.majorant); f.val(o.mode); f.val(o.k_max); f.val(o.t_max_ns);
  f.val(flags);
  if (!((flags & AVM_TUNE_BANDS) && o.majorant == AVM_MAJORANT_BANDED && !fl->dev.has_b)) {
    // bands not tuned, so part of the problem: the caller's band width and lookahead
    f.val(g->band_bins);
    f.val(o.band_lookahead);
  }
  *key = f.h;
  return e;
}

// Version of the cache lines: raised whenever the transport kernel changes
// enough that an earlier timing no longer ranks the candidates right, so
// that lines from an older library are ignored (and a new choice appended).
constexpr int kTuneLineVersion = 5;

bool cache_lookup(const char* path, uint64_t key, int* fpp, int* wpc, int* bb, float* look, double* ms) {
  if (!path) return false;
  std::FILE* fp = std::fopen(path, "r");
  if (!fp) return false;
  char line[256];
  bool found = false;
  while (std::fgets(line, sizeof line, fp)) {
    unsigned long long k = 0;
    int a = 0, b = 0, c = 0;
    int v = 0;
    float l = 0.0f;
    double t = 0.0;
    if (std::sscanf(line, "avm_tune %d %llx %d %d %d %f %lf", &v, &k, &a, &b, &c, &l, &t) == 7 &&
        v == kTuneLineVersion && k == key) {
      *fpp = a; *wpc = b; *bb = c; *look = l; *ms = t;
      found = true;  // the last matching line wins
    }
  }
  std::fclose(fp);
  return found;
}

}  // namespace

extern "C" avm_status avm_autotune(avm_gas* gas, const avm_field* field, const avm_primary* prim,
                                   int32_t prim_on_device, uint64_t n_prim, uint32_t n_aval,
                                   const avm_run_opts* base, uint32_t flags, const char* cache_path,
                                   avm_tune_result* out) {
  g_err.clear();
  if (!gas || !field || !base || !out) return fail(AVM_E_ARG, "avm_autotune: NULL argument");
  if (base->mode != AVM_MODE_BATCHED) return fail(AVM_E_ARG, "avm_autotune: only the batched mode has launch parameters");
  if (flags & ~AVM_TUNE_BANDS) return fail(AVM_E_ARG, "avm_autotune: unknown flags 0x%x", flags);
  std::memset(out, 0, sizeof *out);
  avm_run_opts o = *base;
  o.graph = 0;
  if (o.flights_per_pass <= 0) o.flights_per_pass = default_flights_per_pass(o.precision);  // as a run
  const bool tune_bands = (flags & AVM_TUNE_BANDS) && o.majorant == AVM_MAJORANT_BANDED && !field->dev.has_b;
  const int32_t bb0 = gas->band_bins;
  DeviceGuard dg(gas->device);
  if (dg.err != hipSuccess) return fail(AVM_E_HIP, "hipSetDevice: %s", hipGetErrorString(dg.err));
  uint64_t key = 0;
  HIP_TRY(tune_key(gas, field, prim, prim_on_device, n_prim, n_aval, o, flags, &key));
  out->key = key;
  {
    int fpp = 0, wpc = 0, bb = 0;
    float look = 0.0f;
    double ms = 0.0;
    if (cache_lookup(cache_path, key, &fpp, &wpc, &bb, &look, &ms)) {
      if (tune_bands && bb != gas->band_bins) {
        const avm_status st = avm_gas_set_band_bins(gas, bb);
        if (st != AVM_OK) return st;
      }
      out->flights_per_pass = fpp;
      out->waves_per_cu = wpc;
      out->band_bins = gas->band_bins;
      out->band_lookahead = look;
      out->from_cache = 1;
      out->best_ms = ms;
      out->start_ms = ms;
      return AVM_OK;
    }
  }
  avm_run* r = nullptr;
  avm_status st = avm_run_create(gas, field, prim, prim_on_device, n_prim, n_aval, &o, &r);
  if (st != AVM_OK) return st;
  int max_blocks = 1;
  {
    int grid = 0;
    const hipError_t e = batched_grid(r, 0, &grid, &max_blocks);
    if (e != hipSuccess) {
      avm_run_destroy(r);
      return fail(AVM_E_HIP, "avm_autotune: %s", hipGetErrorString(e));
    }
  }
  struct Trial { int fpp, wpc, bb; float look; double ms; };
  std::vector<Trial> done;
  bool warm = false;
  // best of two timed executions (after one warm-up execution of the run)
  auto measure = [&](int fpp, int wpc, int bb, float look, double* ms) -> avm_status {
    if (fpp < 1) return fail(AVM_E_ARG, "avm_autotune: flights per pass %d < 1", fpp);
    for (const Trial& t : done)
      if (t.fpp == fpp && t.wpc == wpc && t.bb == bb && t.look == look) {
        *ms = t.ms;
        return AVM_OK;
      }
    if (bb != gas->band_bins) {
      const avm_status s = avm_gas_set_band_bins(gas, bb);
      if (s != AVM_OK) return s;
    }
    r->opts.flights_per_pass = fpp;
    r->opts.waves_per_cu = wpc;
    r->opts.band_lookahead = look;
    const hipError_t e = batched_grid(r, wpc, &r->grid, nullptr);
    if (e != hipSuccess) return fail(AVM_E_HIP, "avm_autotune: %s", hipGetErrorString(e));
    double best = INFINITY;
    for (int rep = warm ? 0 : -1; rep < 2; ++rep) {
      avm_status s = avm_run_execute(r);
      if (s == AVM_OK) s = avm_run_sync(r);
      if (s != AVM_OK) return s;
      double t = 0.0;
      s = avm_run_timing(r, &t, nullptr);
      if (s != AVM_OK) return s;
      if (rep >= 0 && t < best) best = t;
    }
    warm = true;
    done.push_back({fpp, wpc, bb, look, best});
    *ms = best;
    return AVM_OK;
  };
  const int fpps[] = {8, 16, 24, 32, 40, 48, 64, 128};
  std::vector<int> bands = {bb0};
  if (tune_bands)
    for (int b : {25, 50, 100, 200, 400})
      if (b < gas->n_bins && b != bb0) bands.push_back(b);
  std::vector<int> wpcs = {0};
  for (int j = 1; j < max_blocks; ++j) wpcs.push_back(j * (r->block / 64));
  std::vector<float> looks = {o.band_lookahead};
  if (tune_bands)
    for (float l : {0.0f, 0.5f, 1.0f, 2.0f})
      if (l != o.band_lookahead) looks.push_back(l);
  Trial best{o.flights_per_pass, o.waves_per_cu, bb0, o.band_lookahead, INFINITY};
  st = measure(best.fpp, best.wpc, best.bb, best.look, &best.ms);
  if (st == AVM_OK) out->start_ms = best.ms;
  auto consider = [&](int fpp, int wpc, int bb, float look) {
    if (st != AVM_OK) return;
    double ms = 0.0;
    st = measure(fpp, wpc, bb, look, &ms);
    if (st == AVM_OK && ms < best.ms) best = {fpp, wpc, bb, look, ms};
  };
  // coordinate search: flights per pass, band width, lookahead, band width
  // again at the chosen lookahead, flights per pass around the best,
  // resident waves
  for (int f : fpps) consider(f, best.wpc, best.bb, best.look);
  for (int b : bands) consider(best.fpp, best.wpc, b, best.look);
  for (float l : looks) consider(best.fpp, best.wpc, best.bb, l);
  for (int b : bands) consider(best.fpp, best.wpc, b, best.look);
  const int f0 = best.fpp;
  for (int f : {f0 - 4, f0 + 4})
    if (f >= 4 && f <= 256) consider(f, best.wpc, best.bb, best.look);
  for (int w : wpcs) consider(best.fpp, w, best.bb, best.look);
  avm_run_destroy(r);
  if (st == AVM_OK && best.bb != gas->band_bins) st = avm_gas_set_band_bins(gas, best.bb);
  if (st != AVM_OK) {
    const std::string msg = g_err;
    if (gas->band_bins != bb0) (void)avm_gas_set_band_bins(gas, bb0);
    g_err = msg;
    return st;
  }
  out->flights_per_pass = best.fpp;
  out->waves_per_cu = best.wpc;
  out->band_bins = best.bb;
  out->band_lookahead = best.look;
  out->trials = (int32_t)done.size();
  out->best_ms = best.ms;
  if (cache_path) {
    std::FILE* fp = std::fopen(cache_path, "a");
    if (!fp) return fail(AVM_E_ARG, "avm_autotune: cannot append to %s", cache_path);
    std::fprintf(fp, "avm_tune %d %016llx %d %d %d %.3f %.6f\n", kTuneLineVersion,
                 (unsigned long long)key, best.fpp, best.wpc, best.bb, (double)best.look, best.ms);
    std::fclose(fp);
  }
  return AVM_OK;
}
