// avm_internal.hpp -- host-side structures shared by the C-ABI layer and the
// kernel launchers of libavm (not installed; the public interface is avm.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "avm.h"
#include "avm_device.hpp"

namespace avm {

static_assert(sizeof(avm_end_record) == 72 && alignof(avm_end_record) == 8, "end record layout");

// Flights a lane makes between two visits of its wave to the queue when the
// caller leaves it at 0, by precision.  Same-box sweeps on the slab
// workloads: in FP64, 40 is 1.6-1.8 % faster than 32 (44 no better); in
// FP32-mixed, whose flight steps are shorter, 48 is 1-2.6 % faster than 40
// (56 no better).  The wire chamber is flat from 24 to 48 in both.
constexpr int32_t kDefaultFlightsPerPass = 40;
constexpr int32_t kDefaultFlightsPerPassF32 = 48;
inline int32_t default_flights_per_pass(int32_t precision) {
  return precision == AVM_FP32_MIXED ? kDefaultFlightsPerPassF32 : kDefaultFlightsPerPass;
}

// Per-avalanche statistics (and totals, with the status histogram).
struct AvalStats {
  unsigned long long c[8];  // endpoints, ionisations, attachments, real, null, masked, band cuts, overflows
};
struct Totals {
  unsigned long long c[8];       // as AvalStats
  unsigned long long status[9];
  unsigned long long _pad[7];
};

// Device store of a run, indexed by slot.  Slot s holds the s-th electron
// created: its start record (arrays, written when it is created) and its
// end record (one 72-byte record, written when it terminates).  The plain
// mode also keeps the state of live electrons between transport iterations
// in the end record (x1..t1 = current position) and in vx1..band1.  In device code
// the pointers are typed as global memory (same 64-bit layout), so accesses
// are global instructions with a scalar base rather than FLAT ones (only in
// the translation unit of the kernels, which defines AVM_KERNELS_TU; host
// code elsewhere sees plain pointers).
#if defined(__HIP_DEVICE_COMPILE__) && defined(AVM_KERNELS_TU)
#define AVM_GLB __attribute__((address_space(1)))
#else
#define AVM_GLB
#endif
struct Store {
  // start arrays (vx0..vz0: only for primaries and queued electrons, which
  // the claiming wave reads back)
  AVM_GLB double *x0, *y0, *z0, *t0, *vx0, *vy0, *vz0, *e0;
  AVM_GLB uint64_t *eid, *parent;
  AVM_GLB uint32_t* aval;
  AVM_GLB uint32_t* qready;  // batched: queue entry q published when qready[q] == epoch
  AVM_GLB uint32_t* qslot;   // batched: slot of queue entry q
  // end records, one per slot (plain mode: also the live position, time,
  // counters and running decision trace between iterations)
  AVM_GLB avm_end_record* end;
  AVM_GLB double *vx1, *vy1, *vz1;  // plain mode: live velocity
  AVM_GLB uint32_t *k1, *band1;      // plain mode: live flight index and band
  // statistics, added to by the transport kernels as electrons terminate
  AVM_GLB AvalStats* stats;  // [n_aval]
  AVM_GLB Totals* tot;
  uint64_t capacity;
};

// Device counters of a run.  The ones every wave of the persistent kernel
// updates or polls sit on separate 256-byte blocks: device-scope atomics are
// performed at the memory side, and counters sharing a line serialise there.
struct Counters {
  alignas(256) unsigned long long tail;   // slots requested (electrons created, incl. dropped)
  alignas(256) unsigned long long qhead;  // batched: queue entries claimed by lanes
  alignas(256) unsigned long long qtail;  // batched: queue entries published or being published
  alignas(256) unsigned long long ended;  // batched: electrons terminated or dropped, as flushed by waves
  alignas(256) unsigned long long next;   // plain: size of the next active list
  unsigned long long err;                 // bad primary avalanche id
  unsigned long long timeout;             // a transport kernel ran out of its time budget
  unsigned long long epoch;               // run counter (bumped by every reset; tags queue entries)
};

struct PrimaryRec {
  double x, y, z, t, e, dx, dy, dz;
  uint32_t aval, _pad;
};

// Everything the no-allocation entry point (avm_noalloc.hip) launches with:
// validated options turned into the kernels' parameter blocks.
struct NoallocSetup {
  int device;
  GasDev gas;
  FieldDev field;
  RunParams params;
  int fp32, banded, field_kind, flights_per_pass, grid, block;
  double k_a;
};

// ---- host side (avm_api.cpp) ----
// Validates a no-allocation run and fills `out` (message set on error).
avm_status noalloc_setup(const avm_gas* gas, const avm_field* field, uint64_t n_prim, uint32_t n_aval,
                         const avm_run_opts* opts, uint64_t max_electrons, NoallocSetup* out);
// Sets the thread's error text (avm_last_error) and returns st.
avm_status set_error(avm_status st, const char* msg);

// ---- launchers (avm_kernels.hip) ----
hipError_t launch_build_rates(const double* sigma, const int32_t* values_kind, int n_ch, int n_bins,
                              double e_max, double density, double k_a, double* cum, double* total,
                              double* binmax, hipStream_t st);
hipError_t launch_build_bands(const double* binmax, int n_bins, int band_bins, int n_bands,
                              double e_max, double* band_gamma, double* band_inv, double* band_edge,
                              double* gamma_out, hipStream_t st);
hipError_t launch_load_primaries(const PrimaryRec* prim, uint64_t n, const Store& S, double k_a,
                                 uint32_t n_aval, uint32_t* active, Counters* ctr, int plain,
                                 hipStream_t st);
hipError_t launch_reset(Counters* ctr, uint64_t n_prim, AvalStats* stats, uint32_t n_aval,
                        Totals* tot, hipStream_t st);
hipError_t launch_generation(int fp32, int banded, int field_kind, const GasDev& G,
                             const FieldDev& F, const RunParams& P, const Store* S,
                             const uint32_t* active, uint32_t n_active, uint32_t* next,
                             Counters* ctr, hipStream_t st);
hipError_t launch_persistent(int fp32, int banded, int field_kind, const GasDev& G,
                             const FieldDev& F, const RunParams& P, const Store* S, Counters* ctr,
                             int flights_per_pass, const SignalDev* signal, int grid, int block,
                             hipStream_t st);
hipError_t launch_zero(double* p, size_t n, hipStream_t st);
int persistent_block();  // threads per block of the persistent kernel
hipError_t persistent_occupancy(int fp32, int banded, int field_kind, int signal, int fit, int block,
                                int* blocks_per_cu);
hipError_t launch_azimuth_table(double* sct, hipStream_t st);
hipError_t launch_tables_f32(const double* cum, const double* total, const double* cum0,
                             size_t n_cum, int n_nodes, const double* bg, const double* be,
                             int n_bands, float* cum_f, float* total_f, float* cum0_f, float* bg_f,
                             float* bi_f, float* be_f, hipStream_t st);

}  // namespace avm
