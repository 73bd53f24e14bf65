// avm_kernels.hip -- gfx950 kernels of libavm: rate-table builder, primary
// load, the plain generation-synchronous transport iteration, the batched
// persistent transport kernel with its device work queue, and the
// statistics reduction.
#define AVM_KERNELS_TU 1  // device pointers of the run store typed as global memory
#include "avm_internal.hpp"

namespace avm {

namespace {

constexpr int kBlock = 256;        // set-up, plain and statistics kernels
// Persistent kernel: one block per CU of AVM_PBLOCK threads (16 waves, 4 per
// SIMD: the register budget is then 128 VGPRs), sharing one LDS copy of
// the hot tables.
#ifndef AVM_PBLOCK
#define AVM_PBLOCK 1024
#endif
constexpr int kPBlock = AVM_PBLOCK;
constexpr int kLdsBytes = 24576;   // bytes of each table slice staged in LDS

// ---------------------------------------------------------------------------
// wave-level helpers (wave64)
// ---------------------------------------------------------------------------

// Each active lane with `pred` gets a distinct index from *ctr; one atomic
// per wave (ballot -> popcount -> mbcnt prefix -> broadcast of the base).
__device__ __forceinline__ unsigned long long wave_alloc(unsigned long long* ctr, bool pred) {
  const uint64_t mask = __ballot(pred);
  if (mask == 0) return 0;
  const uint32_t prefix =
      __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
  const int leader = __builtin_ctzll(mask);
  unsigned long long base = 0;
  if (pred && prefix == 0)
    base = __hip_atomic_fetch_add(ctr, (unsigned long long)__popcll(mask), __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
  base = __shfl(base, leader);
  return base + prefix;
}

template <class R>
AVM_FN R energy(const RunParams& P, R vx, R vy, R vz) {
  return dot3<R>(vx, vy, vz, vx, vy, vz) * Sel<R>::inv_2ka(P);
}

// ---------------------------------------------------------------------------
// rate-table builder
// ---------------------------------------------------------------------------

// One thread per node k: nu_c(e_k) = N sigma_c(e_k) sqrt(2 k_a e_k) (or the
// rate itself), cumulative over channels in order, total = last column.
__global__ void k_build_rates(const double* __restrict__ sigma, const int32_t* __restrict__ vkind,
                              int n_ch, int n_bins, double e_max, double density, double k_a,
                              double* __restrict__ cum, double* __restrict__ total) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k > n_bins) return;
  const double e_k = ((double)k * e_max) / (double)n_bins;
  const double speed = sqrt(2.0 * k_a * e_k);
  const size_t nn = (size_t)n_bins + 1;
  double acc = 0.0;
  for (int c = 0; c < n_ch; ++c) {
    const double v = sigma[(size_t)c * nn + k];
    const double nu = vkind[c] ? v : (density * v) * speed;
    acc = acc + nu;
    cum[(size_t)k * n_ch + c] = acc;
  }
  total[k] = acc;
}

// Linear interpolation inside bin k never exceeds max(total_k, total_k+1).
__global__ void k_bin_max(const double* __restrict__ total, int n_bins, double* __restrict__ binmax) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_bins) return;
  const double a = total[k], b = total[k + 1];
  binmax[k] = a > b ? a : b;
}

// One block per band: maximum of the per-bin maxima inside the band.
__global__ void k_band_local_max(const double* __restrict__ binmax, int n_bins, int band_bins,
                                 double* __restrict__ local) {
  const int b = blockIdx.x;
  const int k0 = band_bins > 0 ? b * band_bins : 0;
  const int k1 = band_bins > 0 ? min(n_bins, (b + 1) * band_bins) : n_bins;
  double m = 0.0;
  for (int k = k0 + (int)threadIdx.x; k < k1; k += blockDim.x) m = fmax(m, binmax[k]);
  __shared__ double red[kBlock];
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) local[b] = red[0];
}

// Prefix maximum over bands (a band's majorant bounds every slower energy
// too), the global majorant, inverses and band edges.  A band whose prefix
// maximum is zero (no collisions below its edge) takes the global majorant.
__global__ void k_band_prefix(double* __restrict__ local, int n_bins, int band_bins, int n_bands,
                              double e_max, double* __restrict__ band_gamma,
                              double* __restrict__ band_inv, double* __restrict__ band_edge,
                              double* __restrict__ gamma_out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double run = 0.0;
  for (int b = 0; b < n_bands; ++b) {
    run = fmax(run, local[b]);
    band_gamma[b] = run;
  }
  const double g = run;
  for (int b = 0; b < n_bands; ++b) {
    if (b == n_bands - 1) {
      band_gamma[b] = g;
      band_edge[b] = __builtin_inf();
    } else {
      if (!(band_gamma[b] > 0.0)) band_gamma[b] = g;
      band_edge[b] = ((double)((b + 1) * band_bins) * e_max) / (double)n_bins;
    }
    band_inv[b] = 1.0 / band_gamma[b];
  }
  *gamma_out = g;
}

// ---------------------------------------------------------------------------
// run set-up
// ---------------------------------------------------------------------------
__global__ void k_reset(Counters* ctr, uint64_t n_prim, AvalStats* stats, uint32_t n_aval,
                        Totals* tot) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    ctr->tail = n_prim;
    ctr->qhead = 0;
    ctr->qtail = n_prim;
    ctr->ended = 0;
    ctr->next = 0;
    ctr->err = 0;
    ctr->timeout = 0;
    // a new run tag: queue entries of earlier runs no longer count as ready
    unsigned long long ep = (ctr->epoch + 1ull) & 0xFFFFFFFFull;
    ctr->epoch = ep == 0 ? 1ull : ep;
    for (int j = 0; j < 8; ++j) tot->c[j] = 0;
    for (int j = 0; j < 9; ++j) tot->status[j] = 0;
  }
  if (i < n_aval)
    for (int j = 0; j < 8; ++j) stats[i].c[j] = 0;
}

// Primaries -> slots [0, n): start record, zeroed end record, published.
__global__ void k_load_primaries(const PrimaryRec* __restrict__ prim, uint64_t n, Store S,
                                 double k_a, uint32_t n_aval, uint32_t* active, Counters* ctr,
                                 int plain) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t epoch = (uint32_t)ctr->epoch;
  const PrimaryRec p = prim[i];
  uint32_t a = p.aval;
  if (a >= n_aval) {
    __hip_atomic_fetch_add(&ctr->err, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    a = 0;
  }
  double dx = p.dx, dy = p.dy, dz = p.dz;
  const double nrm = sqrt(dx * dx + dy * dy + dz * dz);
  if (nrm > 0.0) {
    dx = dx / nrm;
    dy = dy / nrm;
    dz = dz / nrm;
  } else {
    dx = 0.0;
    dy = 0.0;
    dz = 1.0;
  }
  const double sp = sqrt(2.0 * k_a * p.e);
  S.x0[i] = p.x; S.y0[i] = p.y; S.z0[i] = p.z; S.t0[i] = p.t;
  S.vx0[i] = sp * dx; S.vy0[i] = sp * dy; S.vz0[i] = sp * dz;
  S.e0[i] = p.e;
  S.eid[i] = 0x8000000000000000ull | (unsigned long long)i;
  S.parent[i] = 0;
  S.aval[i] = a;
  if (plain) {
    S.end[i] = avm_end_record{p.x, p.y, p.z, p.t, 0.0, 0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};
    S.vx1[i] = sp * dx; S.vy1[i] = sp * dy; S.vz1[i] = sp * dz;
    S.k1[i] = 0; S.band1[i] = 0;
    active[i] = (uint32_t)i;
  }
  S.qslot[i] = (uint32_t)i;
  S.qready[i] = epoch;
}

template <class R>
AVM_FN void slab_field(const FieldDev& F, uint32_t aval, Elec<R>& e) {
  const double* E = F.E + 3 * (size_t)(F.n_E == 1 ? 0u : aval);
  e.Ex = (R)E[0];
  e.Ey = (R)E[1];
  e.Ez = (R)E[2];
}

// Null collisions of a terminated electron: every flight that went on
// advanced k, so nulls are what the other outcomes leave (an attachment
// ends the electron without advancing k).
template <class R>
AVM_FN uint32_t null_count(const Elec<R>& e, uint32_t status) {
  return e.k - e.n_masked - e.n_band - e.n_real + (status == ST_ATTACHED ? 1u : 0u);
}

// The end record of a terminated electron: 72 contiguous bytes.
template <class R>
AVM_FN void write_end(const Store& S, uint32_t s, const Elec<R>& e, const RunParams& P,
                      uint32_t status) {
  S.end[s] = avm_end_record{e.x, e.y, e.z, e.t, (double)energy<R>(P, e.vx, e.vy, e.vz), status,
                            e.n_real, e.n_ion, null_count(e, status), e.n_masked, e.n_band, e.n_over,
                            e.trace};
}

template <class R>
AVM_FN void write_start(const Store& S, uint64_t s, const Elec<R>& parent, const Child<R>& c) {
  S.x0[s] = parent.x; S.y0[s] = parent.y; S.z0[s] = parent.z; S.t0[s] = parent.t;
  S.e0[s] = (double)c.e;
  S.eid[s] = c.eid;
  S.parent[s] = parent.eid;
  S.aval[s] = parent.aval;
}

// ---------------------------------------------------------------------------
// statistics at termination
// ---------------------------------------------------------------------------
// Block totals in LDS (flushed to the run's totals when the block ends):
// the eight counters of AvalStats, then the status histogram.
constexpr int kTally = 17;

// Wave-wide sum (the device library's DPP reduction: row shifts and
// broadcasts, no LDS round trips).
extern "C" __device__ __attribute__((const)) unsigned long long __ockl_wfred_add_u64(unsigned long long);

// Sum of v over the lanes with `in` (every lane of the wave calls it).
AVM_FN unsigned long long group_sum(bool in, uint32_t v) {
  return __ockl_wfred_add_u64(in ? (unsigned long long)v : 0ull);
}

// Adds one counter of a group of lanes to its avalanche (device atomic) and
// to the block's totals (LDS); called by every lane, acted on by the leader.
AVM_FN void tally_add(bool leader, AVM_GLB unsigned long long* dst, AVM_LDS unsigned long long* blk,
                      unsigned long long v) {
  if (leader && v) {
    __hip_atomic_fetch_add(dst, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_fetch_add(blk, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
}

// Adds the electrons this wave terminated (lanes with `ended`, status
// `status`) to the statistics: the lanes are grouped by avalanche, and each
// group's sums go to its avalanche's counters with one atomic per non-zero
// counter, and to the block's totals in LDS.  The counters are summed one
// at a time, so only one sum is live.
template <class R>
AVM_FN void tally_ends(bool ended, uint32_t status, const Elec<R>& e, const Store& S,
                       AVM_LDS unsigned long long* blk) {
  uint64_t m = __ballot(ended);
  if (!m) return;
  const uint32_t lane = __lane_id();
  while (m) {
    const int lead = __builtin_ctzll(m);
    const uint32_t a = __builtin_amdgcn_readlane(e.aval, lead);
    const bool in = ended && e.aval == a;
    const uint64_t g = __ballot(in);
    m &= ~g;
    const bool L = lane == (uint32_t)lead;
    AVM_GLB unsigned long long* dst = S.stats[a].c;
    tally_add(L, dst + 0, blk + 0, __popcll(g));
    tally_add(L, dst + 1, blk + 1, group_sum(in, e.n_ion));
    tally_add(L, dst + 2, blk + 2, __popcll(__ballot(in && status == ST_ATTACHED)));
    tally_add(L, dst + 3, blk + 3, group_sum(in, e.n_real));
    tally_add(L, dst + 4, blk + 4, group_sum(in, in ? null_count(e, status) : 0u));
    if (__ballot(in && e.n_masked)) tally_add(L, dst + 5, blk + 5, group_sum(in, e.n_masked));
    if (__ballot(in && e.n_band)) tally_add(L, dst + 6, blk + 6, group_sum(in, e.n_band));
    if (__ballot(in && e.n_over)) tally_add(L, dst + 7, blk + 7, group_sum(in, e.n_over));
  }
  // status histogram: one LDS add per status present
  m = __ballot(ended);
  while (m) {
    const uint32_t st = __builtin_amdgcn_readlane(status, __builtin_ctzll(m));
    const uint64_t g = __ballot(ended && status == st);
    m &= ~g;
    if (lane == (uint32_t)__builtin_ctzll(g))
      __hip_atomic_fetch_add(blk + 8 + (st < 9 ? st : 8), (unsigned long long)__popcll(g), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_WORKGROUP);
  }
}

// Per-wave statistics accumulator of the persistent kernel, in LDS: the
// counters (as AvalStats) of the electrons the wave terminated for one
// avalanche, `tag`.  They go to the avalanche's counters in device memory
// (and to the block's totals) only when the wave ends electrons of another
// avalanche while holding none of this one, or when the wave leaves.
struct WaveAcc {
  unsigned long long c[8];
  uint32_t tag, _pad;
};
constexpr uint32_t kNoTag = 0xFFFFFFFFu;  // avalanche ids are below n_aval <= 2^32 - 1

// Lanes 0..7 add counter `lane` of the accumulator to its avalanche and to
// the block's totals, and clear it (every lane of the wave calls it).
AVM_FN void acc_flush(AVM_LDS WaveAcc* W, const Store& S, AVM_LDS unsigned long long* blk) {
  const uint32_t tag = __builtin_amdgcn_readfirstlane(W->tag);
  if (tag == kNoTag) return;
  const uint32_t lane = __lane_id();
  if (lane < 8) {
    const unsigned long long v = W->c[lane];
    if (v) {
      __hip_atomic_fetch_add(&S.stats[tag].c[lane], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(blk + lane, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    W->c[lane] = 0ull;
  }
}

// The persistent kernel's form of tally_ends: the ended lanes of the
// accumulator's avalanche add their counters to it in LDS (one LDS atomic
// per counter and lane); when no ended lane belongs to it, the accumulator
// is flushed and taken over by the avalanche of the first ended lane; lanes
// of any further avalanche add to device memory directly.  The status
// histogram goes to the block's totals.
template <class R>
AVM_FN void tally_ends_acc(bool ended, uint32_t status, const Elec<R>& e, const Store& S,
                           AVM_LDS WaveAcc* W, AVM_LDS unsigned long long* blk) {
  const uint64_t m = __ballot(ended);
  if (!m) return;
  uint32_t tag = __builtin_amdgcn_readfirstlane(W->tag);
  if (__ballot(ended && e.aval == tag) == 0) {
    acc_flush(W, S, blk);
    tag = __builtin_amdgcn_readlane(e.aval, __builtin_ctzll(m));
    if (__lane_id() == 0) W->tag = tag;
  }
  // counter j of this lane's electron (formed where it is used, one at a time)
  const auto val = [&](int j) -> uint32_t {
    switch (j) {
      case 0: return 1u;
      case 1: return e.n_ion;
      case 2: return status == ST_ATTACHED ? 1u : 0u;
      case 3: return e.n_real;
      case 4: return null_count(e, status);
      case 5: return e.n_masked;
      case 6: return e.n_band;
      default: return e.n_over;
    }
  };
  if (ended && e.aval == tag) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const uint32_t x = val(j);
      if (x) __hip_atomic_fetch_add(&W->c[j], (unsigned long long)x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    }
  } else if (ended) {
    AVM_GLB unsigned long long* dst = S.stats[e.aval].c;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const uint32_t x = val(j);
      if (x) {
        __hip_atomic_fetch_add(dst + j, (unsigned long long)x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(blk + j, (unsigned long long)x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      }
    }
  }
  if (ended)
    __hip_atomic_fetch_add(blk + 8 + (status < 9 ? status : 8), 1ull, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_WORKGROUP);
}

// A block's totals go to the run's totals (after the block's last tally).
AVM_FN void flush_tally(const AVM_LDS unsigned long long* blk, AVM_GLB Totals* tot) {
  const int i = threadIdx.x;
  if (i < kTally && blk[i]) {
    AVM_GLB unsigned long long* dst = i < 8 ? tot->c + i : tot->status + (i - 8);
    __hip_atomic_fetch_add(dst, blk[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Counters, band and (slab) field of an electron whose position, velocity,
// id and avalanche are set.
template <class R, bool kBanded, int kField, class TV>
AVM_FN void load_elec_tail(const GasDev& G, const TV& T, const FieldDev& F,
                           const RunParams& P, Elec<R>& e) {
  e.k = 0;
  e.n_real = 0; e.n_ion = 0; e.n_masked = 0; e.n_band = 0; e.n_over = 0;
  e.trace = 0;
  e.band = kBanded ? band_of<R>(G, T, energy<R>(P, e.vx, e.vy, e.vz)) : G.n_bands - 1;
  e.Ex = R(0); e.Ey = R(0); e.Ez = R(0);
  if (kField == FIELD_SLAB) slab_field<R>(F, e.aval, e);
}

// ---------------------------------------------------------------------------
// plain mode: one transport iteration of the paper's loop (Fig. 2)
// ---------------------------------------------------------------------------
// Every active electron is carried until it ionises or terminates.  The
// survivors and the new secondaries form the next active list (the paper's
// stack processing: inactive removed, new added), appended with one atomic
// per wave.
template <class R, bool kBanded, int kField>
__global__ void __launch_bounds__(kBlock) k_generation(GasDev G, FieldDev F, RunParams P,
                                                       const Store* __restrict__ Sg,
                                                       const uint32_t* __restrict__ active,
                                                       uint32_t n_active, uint32_t* __restrict__ next,
                                                       Counters* ctr) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  const bool mine = i < n_active;
  const TabView<R> T = global_view<R>(G);
  const Store& S = *Sg;
  __shared__ unsigned long long s_tally[kTally];
  if (threadIdx.x < kTally) s_tally[threadIdx.x] = 0;
  __syncthreads();
  uint32_t term = 0;
  bool ionised = false;
  uint32_t slot = 0;
  Elec<R> e;
  Child<R> child;
  if (mine) {
    slot = active[i];
    const avm_end_record live = S.end[slot];
    e.x = live.x1; e.y = live.y1; e.z = live.z1; e.t = live.t1;
    e.vx = (R)S.vx1[slot]; e.vy = (R)S.vy1[slot]; e.vz = (R)S.vz1[slot];
    e.eid = S.eid[slot];
    e.aval = S.aval[slot];
    e.k = S.k1[slot];
    e.band = kBanded ? (e.k == 0 ? band_of<R>(G, T, energy<R>(P, e.vx, e.vy, e.vz)) : (int32_t)S.band1[slot])
                     : G.n_bands - 1;
    e.n_real = live.n_real; e.n_ion = live.n_ion;
    e.n_masked = live.n_masked; e.n_band = live.n_band; e.n_over = live.n_overflow;
    e.trace = live.trace;
    e.Ex = R(0); e.Ey = R(0); e.Ez = R(0);
    if (kField == FIELD_SLAB) slab_field<R>(F, e.aval, e);
    uint32_t status = 0;
    int32_t r;
    const uint64_t t_start = wall_clock64();
    uint32_t n = 0;
    do {
      r = flight_step<R, kBanded, kField>(e, G, T, F, P, child, status);
      if (r == STEP_CONTINUE && (++n & 4095u) == 0 && wall_clock64() - t_start > P.budget_ticks) {
        // out of time: stop this electron, flag the run
        __hip_atomic_store(&ctr->timeout, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        status = ST_ERROR;
        r = STEP_DONE;
      }
    } while (r == STEP_CONTINUE);
    if (kField == FIELD_POLAR && r == STEP_EXIT) {
      // the crossing of the flight that left the volume (the lanes of the
      // wave that got here search together)
      status = finish_exit<R, kBanded>(e, F, P, child.pen);
      r = STEP_DONE;
    }
    if (r == STEP_DONE) {
      write_end(S, slot, e, P, status);
      term = status;
    } else {
      complete_ionisation<R, kBanded>(e, G, T, P, child);
      ionised = true;
      S.end[slot] = avm_end_record{e.x, e.y, e.z, e.t, 0.0, 0u, e.n_real, e.n_ion, 0u, e.n_masked,
                                   e.n_band, e.n_over, e.trace};
      S.vx1[slot] = (double)e.vx; S.vy1[slot] = (double)e.vy; S.vz1[slot] = (double)e.vz;
      S.k1[slot] = e.k; S.band1[slot] = (uint32_t)e.band;
    }
  }
  // stack processing for this wave: slots for the secondaries, then the
  // next active list (surviving parents and stored secondaries)
  const unsigned long long cs = wave_alloc(&ctr->tail, ionised);
  const bool stored = ionised && cs < S.capacity;
  if (stored) {
    write_start<R>(S, cs, e, child);
    S.end[cs] = avm_end_record{e.x, e.y, e.z, e.t, 0.0, 0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};
    S.vx1[cs] = (double)child.vx; S.vy1[cs] = (double)child.vy; S.vz1[cs] = (double)child.vz;
    S.k1[cs] = 0; S.band1[cs] = 0;
  }
  const unsigned long long np = wave_alloc(&ctr->next, ionised);
  if (ionised) next[np] = slot;
  const unsigned long long nc = wave_alloc(&ctr->next, stored);
  if (stored) next[nc] = (uint32_t)cs;
  tally_ends<R>(term != 0, term, e, S, (AVM_LDS unsigned long long*)s_tally);
  __syncthreads();
  flush_tally((const AVM_LDS unsigned long long*)s_tally, S.tot);
}

// ---------------------------------------------------------------------------
// batched mode: persistent kernel fed by a device work queue
// ---------------------------------------------------------------------------
// Device-coherent accesses (scope: agent, relaxed) for the data handed from
// one wave to another: they are performed at the device's point of
// coherence, so they need no L2 write-back or invalidation (which the
// release/acquire forms would issue on every XCD-local L2).
AVM_FN void st_coh(AVM_GLB double* p, double v) {
  __hip_atomic_store(reinterpret_cast<AVM_GLB unsigned long long*>(p), __builtin_bit_cast(unsigned long long, v),
                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
AVM_FN void st_coh(AVM_GLB uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
AVM_FN void st_coh(AVM_GLB uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
AVM_FN double ld_coh(const AVM_GLB double* p) {
  return __builtin_bit_cast(double, __hip_atomic_load(reinterpret_cast<const AVM_GLB unsigned long long*>(p),
                                                      __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}
template <class T>
AVM_FN T ld_coh_int(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// wait until every store this wave issued has been acknowledged
AVM_FN void wait_stores() { __builtin_amdgcn_s_waitcnt(0x0F70); /* vmcnt(0) */ }

// Child records handed from a lane to an idle lane of the same wave.
struct Xfer {
  double x[64], y[64], z[64], t[64], vx[64], vy[64], vz[64];
  uint64_t eid[64];
  uint32_t slot[64], aval[64];
};

// Back-off of a wave with no electron: repeated s_sleep(AVM_IDLE_NAP)
// (64 cycles each per unit), up to AVM_IDLE_MAX_NAPS in a row (16 x 63:
// up to ~27 us; measured 8-12 % faster than one short nap on the
// 1000-avalanche benchmark, where most waves are idle while the avalanches
// start and end).
// Waves carrying electrons issue ahead of waves that only poll the queue.
#ifndef AVM_BUSY_PRIO
#define AVM_BUSY_PRIO 1
#endif
#ifndef AVM_IDLE_NAP
#define AVM_IDLE_NAP 16
#endif
#ifndef AVM_IDLE_MAX_NAPS
#define AVM_IDLE_MAX_NAPS 63
#endif

// Occupancy target of the persistent kernel (waves per SIMD); the register
// budget follows from it.
#ifndef AVM_PERSISTENT_WAVES_PER_EU
#define AVM_PERSISTENT_WAVES_PER_EU (AVM_PBLOCK / 256)
#endif

// Every lane carries one electron at a time through up to `flights_per_pass`
// flights; a lane stops early when its electron ends or ionises (the
// secondary waits in registers).  After the flights, the lanes whose
// electron ended write their endpoint records together, and the lanes that
// ionised finish their collisions together.  Then the wave, in lockstep:
//   1. allocates storage slots for its new secondaries (one atomic on
//      `tail`, which so counts every electron created, before any of them
//      can be seen by another wave);
//   2. hands secondaries to its own idle lanes through LDS (ballot/mbcnt
//      ranks: the k-th secondary goes to the k-th idle lane);
//   3. publishes the remaining secondaries on the global queue (one atomic
//      on qtail; records written device-coherent, then the entry's ready
//      word after the record stores are acknowledged);
//   4. counts its terminated (and dropped) electrons locally;
//   5. lets its still-idle lanes claim queue entries (one atomic on qhead)
//      and picks up entries whose ready word shows the run's epoch.
// A wave that holds no electron adds its local count to `ended` (one
// atomic), so `ended` never exceeds the number of electrons terminated.
// Reading `ended` and then `tail` and finding them equal means every
// electron created by the first read had terminated by then, and none was
// created in between: no electron exists and none can appear, and the wave
// leaves.
//
// kSignal: the electrons also deposit their induced signal (Shockley-Ramo,
// binned in time) on the readout electrode.  kFit: every band and channel
// fits the LDS copies, and the flights read them without index tests.
template <class R, bool kBanded, int kField, bool kSignal, bool kFit>
__global__ void __launch_bounds__(kPBlock)
    __attribute__((amdgpu_waves_per_eu(AVM_PERSISTENT_WAVES_PER_EU, AVM_PERSISTENT_WAVES_PER_EU)))
    k_persistent(GasDev G, FieldDev F, RunParams P, const Store* __restrict__ Sg, Counters* ctr,
                 int flights_per_pass, SignalDev Q) {
  const uint32_t epoch = (uint32_t)ctr->epoch;
  constexpr unsigned long long kNone = ~0ull;
  __shared__ Xfer xfer_all[kPBlock / 64];
  // hot table slices: total rate and cumulative column 0 on the lowest
  // nodes, and the band tables, one copy per block
  constexpr int kLdsNodes = kLdsBytes / (int)sizeof(R);
  __shared__ R s_tot[kLdsNodes], s_cum0[kLdsNodes];
  __shared__ R s_bg[kLdsBands], s_bi[kLdsBands], s_be[kLdsBands];
  __shared__ ChanP<R> s_ch[kLdsChannels];
  __shared__ double s_sct[2 * kAzN];
  __shared__ unsigned long long s_tally[kTally];
  __shared__ WaveAcc wacc_all[kPBlock / 64];
  if (threadIdx.x < kTally) s_tally[threadIdx.x] = 0;
  if ((threadIdx.x & 63u) < 8u) wacc_all[threadIdx.x >> 6].c[threadIdx.x & 63u] = 0ull;
  if ((threadIdx.x & 63u) == 0u) wacc_all[threadIdx.x >> 6].tag = kNoTag;
  const TabView<R> Tg = global_view<R>(G);
  const int n_lo = G.n_bins + 1 < kLdsNodes ? G.n_bins + 1 : kLdsNodes;
  for (int k = threadIdx.x; k < n_lo; k += kPBlock) {
    s_tot[k] = Tg.tot[k];
    s_cum0[k] = Tg.cum0[k];
  }
  // the first kLdsBands bands and kLdsChannels channels (the accessors read
  // higher indices from the global arrays)
  const int n_lb = G.n_bands < kLdsBands ? G.n_bands : kLdsBands;
  for (int b = threadIdx.x; b < n_lb; b += kPBlock) {
    s_bg[b] = Tg.bgam[b];
    s_bi[b] = Tg.binv[b];
    s_be[b] = Tg.bedge[b];
  }
  const int n_lc = G.n_ch < kLdsChannels ? G.n_ch : kLdsChannels;
  if ((int)threadIdx.x < n_lc) s_ch[threadIdx.x] = Tg.ch[threadIdx.x];
  for (int k = threadIdx.x; k < 2 * kAzN; k += kPBlock) s_sct[k] = G.sct[k];
  __syncthreads();
  using View = std::conditional_t<kFit, TabFit<R>, TabLds<R>>;
  const View T{(const AVM_LDS R*)s_tot, (const AVM_LDS R*)s_cum0, n_lo, (const AVM_LDS R*)s_bg,
               (const AVM_LDS R*)s_bi, (const AVM_LDS R*)s_be, (const AVM_LDS ChanP<R>*)s_ch,
               (const AVM_LDS double*)s_sct};
  Xfer& X = xfer_all[threadIdx.x >> 6];
  const uint32_t lane = __lane_id();
  bool has = false, cp = false;
  unsigned long long n_gone = 0;  // electrons this wave terminated or dropped, not yet in `ended`
  int idle_naps = 0;  // a wave with no electron backs off, longer the longer it stays idle
  unsigned long long claim = kNone;
  uint32_t slot = 0;
  Elec<R> e;
  Child<R> child;
  const uint64_t t_start = wall_clock64();
  for (;;) {
    if (wall_clock64() - t_start > P.budget_ticks) {
      // out of time (every wave checks on every pass, so all of them leave)
      __hip_atomic_store(&ctr->timeout, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      break;
    }
    // ---- transport pass
    uint32_t term = 0;  // status of this lane's electron if it terminated in this pass
    bool xp = false;    // the electron's last flight left the volume (polar map)
    for (int f = 0; f < flights_per_pass && has && !cp && !xp; ++f) {
      uint32_t status = 0;
      const int32_t r = flight_step<R, kBanded, kField, kSignal>(e, G, T, F, P, child, status, &Q);
      if (r == STEP_IONISED) {
        cp = true;
      } else if (r == STEP_DONE) {
        has = false;
        term = status;
      } else if (kField == FIELD_POLAR && r == STEP_EXIT) {
        xp = true;
      }
    }
    // ---- boundary crossings of this pass, found together
    if (kField == FIELD_POLAR && xp) {
      term = finish_exit<R, kBanded, kSignal>(e, F, P, child.pen, &Q);
      has = false;
    }
    // ---- endpoints of this pass, written together (the state of a
    // terminated electron stays in place until the exchange)
    if (term) {
      if (kSignal) signal_end<R, kField>(Q, e);
      write_end<R>(pinned(Sg), slot, e, P, term);
    }
    tally_ends_acc<R>(term != 0, term, e, pinned(Sg), (AVM_LDS WaveAcc*)&wacc_all[threadIdx.x >> 6],
                      (AVM_LDS unsigned long long*)s_tally);
    // ---- ionisations of this pass, finished together
    // (the secondary is born where its parent stands: e.x, e.y, e.z, e.t)
    if (cp) complete_ionisation<R, kBanded>(e, G, T, P, child);
    // ---- exchange (wave in lockstep from here)
    const Store& S = pinned(Sg);
    // 1. storage slots for all secondaries of this pass (dropped beyond the
    //    capacity; the stored ones are the lowest-ranked, slots are handed
    //    out in lane order)
    const unsigned long long cs = wave_alloc(&ctr->tail, cp);
    const bool stored = cp && cs < S.capacity;
    const uint64_t m_child = __ballot(stored);
    // 4. terminations and dropped secondaries of this pass
    n_gone += __popcll(__ballot(term != 0)) + __popcll(__ballot(cp && !stored));
    const uint64_t m_idle = __ballot(!has && claim == kNone);
    const uint32_t n_child = __popcll(m_child), n_idle = __popcll(m_idle);
    const uint32_t n_match = n_child < n_idle ? n_child : n_idle;
    const uint32_t rank_c = __builtin_amdgcn_mbcnt_hi((uint32_t)(m_child >> 32),
                                                      __builtin_amdgcn_mbcnt_lo((uint32_t)m_child, 0u));
    const uint32_t rank_i = __builtin_amdgcn_mbcnt_hi((uint32_t)(m_idle >> 32),
                                                      __builtin_amdgcn_mbcnt_lo((uint32_t)m_idle, 0u));
    const bool local = stored && rank_c < n_match;
    // 3. queue entries for the secondaries no idle lane of this wave takes
    const unsigned long long q = wave_alloc(&ctr->qtail, stored && !local);
    if (stored) {
      // start record: the electron's output; queued ones are also read by
      // other waves, so those go out device-coherent
      if (local) {
        // (the start velocity goes through LDS: only queued electrons need
        // it in memory)
        S.x0[cs] = e.x; S.y0[cs] = e.y; S.z0[cs] = e.z; S.t0[cs] = e.t;
        S.eid[cs] = child.eid;
        S.aval[cs] = e.aval;
        X.x[rank_c] = e.x; X.y[rank_c] = e.y; X.z[rank_c] = e.z; X.t[rank_c] = e.t;
        X.vx[rank_c] = (double)child.vx; X.vy[rank_c] = (double)child.vy;
        X.vz[rank_c] = (double)child.vz;
        X.eid[rank_c] = child.eid;
        X.slot[rank_c] = (uint32_t)cs;
        X.aval[rank_c] = e.aval;
      } else {
        st_coh(&S.x0[cs], e.x); st_coh(&S.y0[cs], e.y); st_coh(&S.z0[cs], e.z); st_coh(&S.t0[cs], e.t);
        st_coh(&S.vx0[cs], (double)child.vx); st_coh(&S.vy0[cs], (double)child.vy);
        st_coh(&S.vz0[cs], (double)child.vz);
        st_coh(&S.eid[cs], child.eid);
        st_coh(&S.aval[cs], e.aval);
        st_coh(&S.qslot[q], (uint32_t)cs);
      }
      S.e0[cs] = (double)child.e;
      S.parent[cs] = e.eid;
    }
    // publish queue entries once their records are acknowledged
    wait_stores();
    if (stored && !local) st_coh(&S.qready[q], epoch);
    // 2. idle lanes of this wave take the local secondaries
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const bool take = (m_idle >> lane & 1) && rank_i < n_match;
    if (take) {
      e.x = X.x[rank_i]; e.y = X.y[rank_i]; e.z = X.z[rank_i]; e.t = X.t[rank_i];
      e.vx = (R)X.vx[rank_i]; e.vy = (R)X.vy[rank_i]; e.vz = (R)X.vz[rank_i];
      e.eid = X.eid[rank_i];
      e.aval = X.aval[rank_i];
      slot = X.slot[rank_i];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    cp = false;
    // 5. still-idle lanes claim queue entries while the queue has some
    const bool want = !has && claim == kNone && !take;
    const uint64_t m_want = __ballot(want);
    if (m_want) {
      const unsigned long long qt = ld_coh_int(&ctr->qtail);
      const unsigned long long qh = ld_coh_int(&ctr->qhead);
      const unsigned long long avail = qt > qh ? qt - qh : 0ull;
      const uint32_t n_want = __popcll(m_want);
      const uint32_t n_take = avail < n_want ? (uint32_t)avail : n_want;
      if (n_take) {
        const uint32_t rk = __builtin_amdgcn_mbcnt_hi((uint32_t)(m_want >> 32),
                                                      __builtin_amdgcn_mbcnt_lo((uint32_t)m_want, 0u));
        unsigned long long base = 0;
        if (want && rk == 0)
          base = __hip_atomic_fetch_add(&ctr->qhead, (unsigned long long)n_take, __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT);
        base = __shfl(base, __builtin_ctzll(m_want));
        if (want && rk < n_take) claim = base + rk;
      }
    }
    if (take) {
      load_elec_tail<R, kBanded, kField>(G, T, F, P, e);
      if (kSignal) signal_birth<R, kField>(Q, e);
      has = true;
    } else if (!has && claim != kNone) {
      if (claim < S.capacity && ld_coh_int(&S.qready[claim]) == epoch) {
        slot = ld_coh_int(&S.qslot[claim]);
        e.x = ld_coh(&S.x0[slot]); e.y = ld_coh(&S.y0[slot]); e.z = ld_coh(&S.z0[slot]);
        e.t = ld_coh(&S.t0[slot]);
        e.vx = (R)ld_coh(&S.vx0[slot]); e.vy = (R)ld_coh(&S.vy0[slot]);
        e.vz = (R)ld_coh(&S.vz0[slot]);
        e.eid = ld_coh_int(&S.eid[slot]);
        e.aval = ld_coh_int(&S.aval[slot]);
        load_elec_tail<R, kBanded, kField>(G, T, F, P, e);
        if (kSignal) signal_birth<R, kField>(Q, e);
        has = true;
        claim = kNone;
      }
    }
    if (__ballot(has) == 0) {
      // no electron in this wave: flush the local count, then test for the
      // end.  (A pending claim is no electron: below qtail its entry is
      // counted in `tail` and not ended; at or beyond qtail -- lanes may
      // claim past it, reading qtail and qhead apart from the claim -- it
      // names an entry that does not exist yet.)
      if (n_gone != 0) {
        if (lane == (uint32_t)__builtin_ctzll(__ballot(1)))
          __hip_atomic_fetch_add(&ctr->ended, n_gone, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        n_gone = 0;
      }
      // `tail` is read after `ended` has arrived: its address depends on the
      // value read (n_end < 2^63, so the offset is zero)
      const unsigned long long n_end = ld_coh_int(&ctr->ended);
      if (n_end == ld_coh_int(&ctr->tail + (n_end >> 63))) break;
    }
    if (__ballot(has) == 0) {
      // nothing to carry: leave the SIMD to busy waves for a while before
      // polling the queue again (the polls and the exchange code would
      // otherwise take their issue slots)
#if AVM_BUSY_PRIO
      __builtin_amdgcn_s_setprio(0);
#endif
      idle_naps = idle_naps < AVM_IDLE_MAX_NAPS ? 2 * idle_naps + 1 : AVM_IDLE_MAX_NAPS;
      for (int i = 0; i < idle_naps; ++i) __builtin_amdgcn_s_sleep(AVM_IDLE_NAP);
    } else {
#if AVM_BUSY_PRIO
      __builtin_amdgcn_s_setprio(2);
#endif
      idle_naps = 0;
    }
  }
  // the wave's accumulated statistics go out; once every wave of the block
  // has left the loop, the block's totals
  acc_flush((AVM_LDS WaveAcc*)&wacc_all[threadIdx.x >> 6], pinned(Sg), (AVM_LDS unsigned long long*)s_tally);
  __syncthreads();
  flush_tally((const AVM_LDS unsigned long long*)s_tally, pinned(Sg).tot);
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_build_rates(const double* sigma, const int32_t* values_kind, int n_ch, int n_bins,
                              double e_max, double density, double k_a, double* cum, double* total,
                              double* binmax, hipStream_t st) {
  const int nn = n_bins + 1;
  hipLaunchKernelGGL(k_build_rates, dim3((nn + kBlock - 1) / kBlock), dim3(kBlock), 0, st, sigma,
                     values_kind, n_ch, n_bins, e_max, density, k_a, cum, total);
  hipLaunchKernelGGL(k_bin_max, dim3((n_bins + kBlock - 1) / kBlock), dim3(kBlock), 0, st, total,
                     n_bins, binmax);
  return hipGetLastError();
}

hipError_t launch_build_bands(const double* binmax, int n_bins, int band_bins, int n_bands,
                              double e_max, double* band_gamma, double* band_inv, double* band_edge,
                              double* gamma_out, hipStream_t st) {
  // band_gamma doubles as the per-band scratch of the local maxima
  hipLaunchKernelGGL(k_band_local_max, dim3(n_bands), dim3(kBlock), 0, st, binmax, n_bins,
                     band_bins, band_gamma);
  hipLaunchKernelGGL(k_band_prefix, dim3(1), dim3(64), 0, st, band_gamma, n_bins, band_bins,
                     n_bands, e_max, band_gamma, band_inv, band_edge, gamma_out);
  return hipGetLastError();
}

hipError_t launch_reset(Counters* ctr, uint64_t n_prim, AvalStats* stats, uint32_t n_aval,
                        Totals* tot, hipStream_t st) {
  const uint64_t n = n_aval > 0 ? n_aval : 1;
  hipLaunchKernelGGL(k_reset, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, ctr,
                     n_prim, stats, n_aval, tot);
  return hipGetLastError();
}

hipError_t launch_load_primaries(const PrimaryRec* prim, uint64_t n, const Store& S, double k_a,
                                 uint32_t n_aval, uint32_t* active, Counters* ctr, int plain,
                                 hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_load_primaries, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                     st, prim, n, S, k_a, n_aval, active, ctr, plain);
  return hipGetLastError();
}

template <class R, bool B, int FK>
static void gen_one(const GasDev& G, const FieldDev& F, const RunParams& P, const Store* S,
                    const uint32_t* active, uint32_t n_active, uint32_t* next, Counters* ctr,
                    hipStream_t st) {
  hipLaunchKernelGGL((k_generation<R, B, FK>), dim3((n_active + kBlock - 1) / kBlock), dim3(kBlock),
                     0, st, G, F, P, S, active, n_active, next, ctr);
}

template <class R>
static void gen_prec(int banded, int fk, const GasDev& G, const FieldDev& F, const RunParams& P,
                     const Store* S, const uint32_t* active, uint32_t n_active, uint32_t* next,
                     Counters* ctr, hipStream_t st) {
  if (banded) {
    if (fk == FIELD_SLAB)
      gen_one<R, true, FIELD_SLAB>(G, F, P, S, active, n_active, next, ctr, st);
    else
      gen_one<R, true, FIELD_POLAR>(G, F, P, S, active, n_active, next, ctr, st);
  } else {
    if (fk == FIELD_SLAB)
      gen_one<R, false, FIELD_SLAB>(G, F, P, S, active, n_active, next, ctr, st);
    else
      gen_one<R, false, FIELD_POLAR>(G, F, P, S, active, n_active, next, ctr, st);
  }
}

hipError_t launch_generation(int fp32, int banded, int field_kind, const GasDev& G,
                             const FieldDev& F, const RunParams& P, const Store* S,
                             const uint32_t* active, uint32_t n_active, uint32_t* next,
                             Counters* ctr, hipStream_t st) {
  if (n_active == 0) return hipSuccess;
  if (fp32)
    gen_prec<float>(banded, field_kind, G, F, P, S, active, n_active, next, ctr, st);
  else
    gen_prec<double>(banded, field_kind, G, F, P, S, active, n_active, next, ctr, st);
  return hipGetLastError();
}

template <class R, bool SIG, bool FIT>
static const void* pick_persistent_fit(int banded, int fk) {
  if (banded)
    return fk == FIELD_SLAB ? reinterpret_cast<const void*>(&k_persistent<R, true, FIELD_SLAB, SIG, FIT>)
                            : reinterpret_cast<const void*>(&k_persistent<R, true, FIELD_POLAR, SIG, FIT>);
  return fk == FIELD_SLAB ? reinterpret_cast<const void*>(&k_persistent<R, false, FIELD_SLAB, SIG, FIT>)
                          : reinterpret_cast<const void*>(&k_persistent<R, false, FIELD_POLAR, SIG, FIT>);
}

template <class R, bool SIG>
static const void* pick_persistent_sig(int banded, int fk, int fit) {
  return fit ? pick_persistent_fit<R, SIG, true>(banded, fk) : pick_persistent_fit<R, SIG, false>(banded, fk);
}

static const void* pick_persistent(int fp32, int banded, int fk, int signal, int fit) {
  if (fp32)
    return signal ? pick_persistent_sig<float, true>(banded, fk, fit)
                  : pick_persistent_sig<float, false>(banded, fk, fit);
  return signal ? pick_persistent_sig<double, true>(banded, fk, fit)
                : pick_persistent_sig<double, false>(banded, fk, fit);
}

int persistent_block() { return kPBlock; }

hipError_t persistent_occupancy(int fp32, int banded, int field_kind, int signal, int fit, int block,
                                int* blocks_per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(
      blocks_per_cu, pick_persistent(fp32, banded, field_kind, signal, fit), block, 0);
}

hipError_t launch_persistent(int fp32, int banded, int field_kind, const GasDev& G,
                             const FieldDev& F, const RunParams& P, const Store* S, Counters* ctr,
                             int flights_per_pass, const SignalDev* signal, int grid, int block,
                             hipStream_t st) {
  SignalDev Q{};
  if (signal) Q = *signal;
  const void* fn = pick_persistent(fp32, banded, field_kind, signal != nullptr, tables_fit_lds(G));
  void* args[] = {const_cast<GasDev*>(&G), const_cast<FieldDev*>(&F), const_cast<RunParams*>(&P),
                  const_cast<Store**>(&S), &ctr, &flights_per_pass, &Q};
  return hipLaunchKernel(fn, dim3(grid), dim3(block), args, 0, st);
}

// Zero fill (a kernel, so that it can be captured into a graph).
__global__ void k_zero(double* __restrict__ p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

hipError_t launch_zero(double* p, size_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  size_t blocks = (n + kBlock - 1) / kBlock;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(kBlock), 0, st, p, n);
  return hipGetLastError();
}

// FP32 copies of the rate tables: rates rounded to nearest, majorants
// rounded up and band edges rounded down (so they stay bounds), inverse
// majorants from the rounded-up values.
__global__ void k_tables_f32(const double* __restrict__ cum, const double* __restrict__ total,
                             const double* __restrict__ cum0, size_t n_cum, int n_nodes,
                             const double* __restrict__ bg, const double* __restrict__ be, int n_bands,
                             float* __restrict__ cum_f, float* __restrict__ total_f,
                             float* __restrict__ cum0_f, float* __restrict__ bg_f,
                             float* __restrict__ bi_f, float* __restrict__ be_f) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_cum) cum_f[i] = (float)cum[i];
  if (i < (size_t)n_nodes) {
    total_f[i] = (float)total[i];
    cum0_f[i] = (float)cum0[i];
  }
  if (i < (size_t)n_bands) {
    const float g = __double2float_ru(bg[i]);
    bg_f[i] = g;
    bi_f[i] = 1.0f / g;
    be_f[i] = __double2float_rd(be[i]);
  }
}

// The azimuth table: sin and cos of 2 pi j / kAzN, j = 0 .. kAzN - 1, from
// sincospi_pos at the exact argument j / (kAzN / 2).
__global__ void k_azimuth_table(double* __restrict__ sct) {
  const int j = (int)threadIdx.x;
  if (j < kAzN) {
    double sn, cs;
    sincospi_pos((double)j / (double)(kAzN / 2), &sn, &cs);
    sct[2 * j] = sn;
    sct[2 * j + 1] = cs;
  }
}

hipError_t launch_azimuth_table(double* sct, hipStream_t st) {
  hipLaunchKernelGGL(k_azimuth_table, dim3(1), dim3(kAzN), 0, st, sct);
  return hipGetLastError();
}

hipError_t launch_tables_f32(const double* cum, const double* total, const double* cum0,
                             size_t n_cum, int n_nodes, const double* bg, const double* be,
                             int n_bands, float* cum_f, float* total_f, float* cum0_f, float* bg_f,
                             float* bi_f, float* be_f, hipStream_t st) {
  size_t n = n_cum;
  if ((size_t)n_nodes > n) n = n_nodes;
  if ((size_t)n_bands > n) n = n_bands;
  hipLaunchKernelGGL(k_tables_f32, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st,
                     cum, total, cum0, n_cum, n_nodes, bg, be, n_bands, cum_f, total_f, cum0_f, bg_f,
                     bi_f, be_f);
  return hipGetLastError();
}


}  // namespace avm
