// avm_noalloc.hip -- avm_run_noalloc: the batched transport of
// avm_run_execute for callers that cannot allocate device memory.  The
// caller passes the primaries and every output array; the run's working
// memory (counters, queue entries, the start velocities of queued
// electrons, the store descriptor and the totals) lives in `scratch`, one
// static device array per GPU, set up once per device.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>

#include "avm_internal.hpp"

using namespace avm;

namespace {

// Layout of the scratch array (byte offsets, each 256-aligned).  The
// per-electron arrays have a fixed place for the largest capacity, so a
// queue entry's ready word is never another array's old bytes: it holds
// zero or the epoch of an earlier call, never the current one.
constexpr uint64_t kMaxE = AVM_NOALLOC_MAX_ELECTRONS;
constexpr size_t kOffCtr = 0;
constexpr size_t kOffTot = 2048;
constexpr size_t kOffStore = 2304;
constexpr size_t kOffQready = 4096;
constexpr size_t kOffQslot = kOffQready + 4 * kMaxE;
constexpr size_t kOffVx = kOffQslot + 4 * kMaxE;
constexpr size_t kOffVy = kOffVx + 8 * kMaxE;
constexpr size_t kOffVz = kOffVy + 8 * kMaxE;
constexpr size_t kScratchBytes = kOffVz + 8 * kMaxE;
static_assert(sizeof(Counters) <= kOffTot - kOffCtr, "counters overlap the totals");
static_assert(sizeof(Totals) <= kOffStore - kOffTot, "totals overlap the store descriptor");
static_assert(sizeof(Store) <= kOffQready - kOffStore, "store descriptor overlaps the queue");

__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};  // device address of `scratch` per device (set up once)

__global__ void k_clear_words(uint32_t* p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

// The device address of this device's scratch array (the array's name is a
// host-side stand-in in host code, never a device address).  The first call
// on a device looks it up (with the device current) and clears the queue's
// ready words on stream s, ahead of the run's own kernels.
hipError_t scratch_ptr(int dev, hipStream_t s, unsigned char** out) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_clear_words, dim3(1024), dim3(256), 0, s,
                       reinterpret_cast<uint32_t*>(static_cast<unsigned char*>(p) + kOffQready), (size_t)kMaxE);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    g_ptr[dev] = p;
  }
  *out = static_cast<unsigned char*>(g_ptr[dev]);
  return hipSuccess;
}

// The store descriptor, written into scratch by a kernel (its value comes
// as a kernel argument, so nothing is copied from host memory).
__global__ void k_put_store(Store S, Store* dst) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *dst = S;
}

// Totals and error flags of the finished run into the caller's records.
__global__ void k_finish(const Counters* ctr, const Totals* tot, uint64_t capacity, avm_counts* out,
                         uint32_t* flags) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  avm_counts c;
  std::memset(&c, 0, sizeof c);
  c.n_endpoints = tot->c[0];
  c.n_ion = tot->c[1];
  c.n_att = tot->c[2];
  c.n_real = tot->c[3];
  c.n_null = tot->c[4];
  c.n_masked = tot->c[5];
  c.n_band = tot->c[6];
  c.n_overflow = tot->c[7];
  for (int i = 0; i < 9; ++i) c.n_status[i] = tot->status[i];
  c.n_requested = ctr->tail;
  c.truncated = ctr->tail > capacity ? 1u : 0u;
  *out = c;
  *flags = (ctr->timeout ? AVM_NOALLOC_TIMEOUT : 0u) | (ctr->err ? AVM_NOALLOC_BAD_AVALANCHE : 0u) |
           (c.truncated ? AVM_NOALLOC_TRUNCATED : 0u);
}

}  // namespace

extern "C" avm_status avm_run_noalloc(const avm_gas* gas, const avm_field* field, const avm_primary* prim,
                                      uint64_t n_prim, uint32_t n_aval, const avm_run_opts* opts,
                                      const avm_noalloc_out* out) {
  if (!out) return set_error(AVM_E_ARG, "avm_run_noalloc: out is NULL");
  if (n_prim && !prim) return set_error(AVM_E_ARG, "avm_run_noalloc: primaries are NULL");
  const void* arrays[] = {out->x0, out->y0, out->z0, out->t0, out->e0, out->eid, out->parent,
                          out->avalanche, out->end, out->aval_counts, out->counts, out->flags};
  for (const void* a : arrays)
    if (!a) return set_error(AVM_E_ARG, "avm_run_noalloc: an output array is NULL");
  NoallocSetup su{};
  const avm_status st = noalloc_setup(gas, field, n_prim, n_aval, opts, kMaxE, &su);
  if (st != AVM_OK) return st;
  int prev = -1;
  if (hipGetDevice(&prev) != hipSuccess) prev = -1;
  hipError_t e = hipSetDevice(su.device);
  hipStream_t s = static_cast<hipStream_t>(opts->hip_stream);
  unsigned char* base = nullptr;
  if (e == hipSuccess) e = scratch_ptr(su.device, s, &base);
  if (e == hipSuccess) {
    Counters* ctr = reinterpret_cast<Counters*>(base + kOffCtr);
    Totals* tot = reinterpret_cast<Totals*>(base + kOffTot);
    Store* sdev = reinterpret_cast<Store*>(base + kOffStore);
    Store S{};
    S.x0 = out->x0; S.y0 = out->y0; S.z0 = out->z0; S.t0 = out->t0; S.e0 = out->e0;
    S.vx0 = reinterpret_cast<double*>(base + kOffVx);
    S.vy0 = reinterpret_cast<double*>(base + kOffVy);
    S.vz0 = reinterpret_cast<double*>(base + kOffVz);
    S.eid = out->eid; S.parent = out->parent; S.aval = out->avalanche;
    S.qready = reinterpret_cast<uint32_t*>(base + kOffQready);
    S.qslot = reinterpret_cast<uint32_t*>(base + kOffQslot);
    S.end = out->end;
    S.stats = reinterpret_cast<AvalStats*>(out->aval_counts);
    S.tot = tot;
    S.capacity = opts->capacity;
    // descriptor; counters (a new epoch), totals and the caller's
    // per-avalanche counters cleared; primaries loaded; transport (which
    // adds up the statistics); totals and flags out
    hipLaunchKernelGGL(k_put_store, dim3(1), dim3(64), 0, s, S, sdev);
    e = hipGetLastError();
    if (e == hipSuccess) e = launch_reset(ctr, n_prim, S.stats, n_aval, tot, s);
    if (e == hipSuccess)
      e = launch_load_primaries(reinterpret_cast<const PrimaryRec*>(prim), n_prim, S, su.k_a, n_aval, nullptr,
                                ctr, 0, s);
    if (e == hipSuccess)
      e = launch_persistent(su.fp32, su.banded, su.field_kind, su.gas, su.field, su.params, sdev, ctr,
                            su.flights_per_pass, nullptr, su.grid, su.block, s);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(k_finish, dim3(1), dim3(64), 0, s, ctr, tot, (uint64_t)opts->capacity, out->counts,
                         out->flags);
      e = hipGetLastError();
    }
  }
  if (prev >= 0) (void)hipSetDevice(prev);
  if (e != hipSuccess) return set_error(AVM_E_HIP, hipGetErrorString(e));
  return AVM_OK;
}
