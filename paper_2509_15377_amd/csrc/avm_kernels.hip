// avm_kernels.hip -- gfx950 kernels of libavm: rate-table builder, primary
// load, the plain generation-synchronous transport iteration, the batched
// persistent transport kernel with its device work queue, and the
// statistics reduction.
#include "avm_internal.hpp"

namespace avm {

namespace {

constexpr int kBlock = 256;

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

__device__ __forceinline__ double energy(const RunParams& P, double vx, double vy, double vz) {
  return dot3(vx, vy, vz, vx, vy, vz) * P.inv_2ka;
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
    ctr->head = 0;
    ctr->live = n_prim;
    ctr->next = 0;
    ctr->err = 0;
    ctr->timeout = 0;
    for (int j = 0; j < 8; ++j) tot->c[j] = 0;
    for (int j = 0; j < 9; ++j) tot->status[j] = 0;
  }
  if (i < n_aval) stats[i] = AvalStats{0, 0, 0, 0, 0, 0, 0, 0};
}

// Primaries -> slots [0, n): start record, zeroed end record, published.
__global__ void k_load_primaries(const PrimaryRec* __restrict__ prim, uint64_t n, Store S,
                                 uint32_t epoch, double k_a, uint32_t n_aval, uint32_t* active,
                                 Counters* ctr, int plain) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
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
    S.x1[i] = p.x; S.y1[i] = p.y; S.z1[i] = p.z; S.t1[i] = p.t;
    S.vx1[i] = sp * dx; S.vy1[i] = sp * dy; S.vz1[i] = sp * dz;
    S.k1[i] = 0; S.band1[i] = 0;
    S.n_real[i] = 0; S.n_ion[i] = 0; S.n_null[i] = 0; S.n_masked[i] = 0;
    S.n_band[i] = 0; S.n_over[i] = 0; S.status[i] = 0;
    active[i] = (uint32_t)i;
  }
  S.ready[i] = epoch;
}

__device__ __forceinline__ void slab_field(const FieldDev& F, uint32_t aval, Elec& e) {
  const double* E = F.E + 3 * (size_t)(F.n_E == 1 ? 0u : aval);
  e.Ex = E[0];
  e.Ey = E[1];
  e.Ez = E[2];
}

__device__ __forceinline__ void write_end(const Store& S, uint32_t s, const Elec& e,
                                          const RunParams& P, uint32_t status) {
  S.x1[s] = e.x; S.y1[s] = e.y; S.z1[s] = e.z; S.t1[s] = e.t;
  S.e1[s] = energy(P, e.vx, e.vy, e.vz);
  S.status[s] = status;
  S.n_real[s] = e.n_real; S.n_ion[s] = e.n_ion; S.n_null[s] = e.n_null;
  S.n_masked[s] = e.n_masked; S.n_band[s] = e.n_band; S.n_over[s] = e.n_over;
}

__device__ __forceinline__ void write_start(const Store& S, uint64_t s, const Elec& parent,
                                            const Child& c) {
  S.x0[s] = parent.x; S.y0[s] = parent.y; S.z0[s] = parent.z; S.t0[s] = parent.t;
  S.vx0[s] = c.vx; S.vy0[s] = c.vy; S.vz0[s] = c.vz;
  S.e0[s] = c.e;
  S.eid[s] = c.eid;
  S.parent[s] = parent.eid;
  S.aval[s] = parent.aval;
}

// A fresh electron from its start record.
template <bool kBanded, int kField>
__device__ __forceinline__ void load_fresh(const Store& S, const GasDev& G, const FieldDev& F,
                                           const RunParams& P, uint64_t s, Elec& e) {
  e.x = S.x0[s]; e.y = S.y0[s]; e.z = S.z0[s]; e.t = S.t0[s];
  e.vx = S.vx0[s]; e.vy = S.vy0[s]; e.vz = S.vz0[s];
  e.eid = S.eid[s];
  e.aval = S.aval[s];
  e.k = 0;
  e.n_real = 0; e.n_ion = 0; e.n_null = 0; e.n_masked = 0; e.n_band = 0; e.n_over = 0;
  e.band = kBanded ? band_of(G, energy(P, e.vx, e.vy, e.vz)) : G.n_bands - 1;
  e.Ex = 0.0; e.Ey = 0.0; e.Ez = 0.0;
  if (kField == FIELD_SLAB) slab_field(F, e.aval, e);
}

// ---------------------------------------------------------------------------
// plain mode: one transport iteration of the paper's loop (Fig. 2)
// ---------------------------------------------------------------------------
// Every active electron is carried until it ionises or terminates.  The
// survivors and the new secondaries form the next active list (the paper's
// stack processing: inactive removed, new added), appended with one atomic
// per wave.
template <bool kBanded, int kField>
__global__ void __launch_bounds__(kBlock) k_generation(GasDev G, FieldDev F, RunParams P, Store S,
                                                       const uint32_t* __restrict__ active,
                                                       uint32_t n_active, uint32_t* __restrict__ next,
                                                       Counters* ctr) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  const bool mine = i < n_active;
  bool ionised = false;
  uint32_t slot = 0;
  Elec e;
  Child child;
  if (mine) {
    slot = active[i];
    e.x = S.x1[slot]; e.y = S.y1[slot]; e.z = S.z1[slot]; e.t = S.t1[slot];
    e.vx = S.vx1[slot]; e.vy = S.vy1[slot]; e.vz = S.vz1[slot];
    e.eid = S.eid[slot];
    e.aval = S.aval[slot];
    e.k = S.k1[slot];
    e.band = kBanded ? (e.k == 0 ? band_of(G, energy(P, e.vx, e.vy, e.vz)) : (int32_t)S.band1[slot])
                     : G.n_bands - 1;
    e.n_real = S.n_real[slot]; e.n_ion = S.n_ion[slot]; e.n_null = S.n_null[slot];
    e.n_masked = S.n_masked[slot]; e.n_band = S.n_band[slot]; e.n_over = S.n_over[slot];
    e.Ex = 0.0; e.Ey = 0.0; e.Ez = 0.0;
    if (kField == FIELD_SLAB) slab_field(F, e.aval, e);
    uint32_t status = 0;
    int32_t r;
    const uint64_t t_start = wall_clock64();
    uint32_t n = 0;
    do {
      r = flight_step<kBanded, kField>(e, G, F, P, child, status);
      if (r == STEP_CONTINUE && (++n & 4095u) == 0 && wall_clock64() - t_start > P.budget_ticks) {
        // out of time: stop this electron, flag the run
        __hip_atomic_store(&ctr->timeout, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        status = ST_ERROR;
        r = STEP_DONE;
      }
    } while (r == STEP_CONTINUE);
    if (r == STEP_DONE) {
      write_end(S, slot, e, P, status);
    } else {
      ionised = true;
      S.x1[slot] = e.x; S.y1[slot] = e.y; S.z1[slot] = e.z; S.t1[slot] = e.t;
      S.vx1[slot] = e.vx; S.vy1[slot] = e.vy; S.vz1[slot] = e.vz;
      S.k1[slot] = e.k; S.band1[slot] = (uint32_t)e.band;
      S.n_real[slot] = e.n_real; S.n_ion[slot] = e.n_ion; S.n_null[slot] = e.n_null;
      S.n_masked[slot] = e.n_masked; S.n_band[slot] = e.n_band; S.n_over[slot] = e.n_over;
    }
  }
  // stack processing for this wave: slots for the secondaries, then the
  // next active list (surviving parents and stored secondaries)
  const unsigned long long cs = wave_alloc(&ctr->tail, ionised);
  const bool stored = ionised && cs < S.capacity;
  if (stored) {
    write_start(S, cs, e, child);
    S.x1[cs] = e.x; S.y1[cs] = e.y; S.z1[cs] = e.z; S.t1[cs] = e.t;
    S.vx1[cs] = child.vx; S.vy1[cs] = child.vy; S.vz1[cs] = child.vz;
    S.k1[cs] = 0; S.band1[cs] = 0;
    S.n_real[cs] = 0; S.n_ion[cs] = 0; S.n_null[cs] = 0; S.n_masked[cs] = 0;
    S.n_band[cs] = 0; S.n_over[cs] = 0; S.status[cs] = 0;
  }
  const unsigned long long np = wave_alloc(&ctr->next, ionised);
  if (ionised) next[np] = slot;
  const unsigned long long nc = wave_alloc(&ctr->next, stored);
  if (stored) next[nc] = (uint32_t)cs;
}

// ---------------------------------------------------------------------------
// batched mode: persistent kernel fed by a device work queue
// ---------------------------------------------------------------------------
// The queue is the slot store itself: slots are handed out in order by
// `tail` (creation) and claimed in order by `head`; slot s is published
// by a release store of the run's epoch into ready[s] after its start record
// is written, and read after an acquire load observes it.  `live` counts
// electrons created and not yet terminated: it is raised before a slot is
// published and lowered after an end record is written, so live == 0 means
// no electron exists and none can appear -- every lane then leaves.
template <bool kBanded, int kField>
__global__ void __launch_bounds__(kBlock) k_persistent(GasDev G, FieldDev F, RunParams P, Store S,
                                                       Counters* ctr, uint32_t epoch,
                                                       int flights_per_pass) {
  constexpr unsigned long long kNone = ~0ull;
  bool has = false, done = false;
  unsigned long long claim = kNone;
  uint32_t slot = 0;
  Elec e;
  const uint64_t t_start = wall_clock64();
  for (;;) {
    if (wall_clock64() - t_start > P.budget_ticks) {
      // out of time (every wave checks on every pass, so all of them leave)
      __hip_atomic_store(&ctr->timeout, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      break;
    }
    if (!has && !done) {
      if (claim == kNone)
        claim = __hip_atomic_fetch_add(&ctr->head, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (claim < S.capacity &&
          __hip_atomic_load(&S.ready[claim], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == epoch) {
        slot = (uint32_t)claim;
        claim = kNone;
        load_fresh<kBanded, kField>(S, G, F, P, slot, e);
        has = true;
      } else if (__hip_atomic_load(&ctr->live, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
        done = true;
      }
    }
    if (__ballot(!done) == 0) break;
    if (__ballot(has) == 0) {
      __builtin_amdgcn_s_sleep(4);
      continue;
    }
    for (int f = 0; f < flights_per_pass && has; ++f) {
      Child child;
      uint32_t status = 0;
      const int32_t r = flight_step<kBanded, kField>(e, G, F, P, child, status);
      if (r == STEP_IONISED) {
        const unsigned long long cs =
            __hip_atomic_fetch_add(&ctr->tail, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (cs < S.capacity) {
          __hip_atomic_fetch_add(&ctr->live, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          write_start(S, cs, e, child);
          __hip_atomic_store(&S.ready[cs], epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
      } else if (r == STEP_DONE) {
        write_end(S, slot, e, P, status);
        __hip_atomic_fetch_add(&ctr->live, ~0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        has = false;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// statistics
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_stats(Store S, const Counters* ctr, AvalStats* stats,
                                                  Totals* tot) {
  __shared__ unsigned long long blk[17];
  if (threadIdx.x < 17) blk[threadIdx.x] = 0;
  __syncthreads();
  const unsigned long long n = ctr->tail < S.capacity ? ctr->tail : S.capacity;
  for (unsigned long long s = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; s < n;
       s += (unsigned long long)gridDim.x * blockDim.x) {
    const uint32_t a = S.aval[s];
    const uint32_t st = S.status[s];
    const unsigned long long v[8] = {1ull, S.n_ion[s], st == ST_ATTACHED ? 1ull : 0ull, S.n_real[s],
                                     S.n_null[s], S.n_masked[s], S.n_band[s], S.n_over[s]};
    unsigned long long* dst = &stats[a].n_endpoints;
    for (int j = 0; j < 8; ++j) {
      if (v[j]) {
        __hip_atomic_fetch_add(dst + j, v[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        atomicAdd(&blk[j], v[j]);
      }
    }
    atomicAdd(&blk[8 + (st < 9 ? st : 8)], 1ull);
  }
  __syncthreads();
  if (threadIdx.x < 8) {
    if (blk[threadIdx.x])
      __hip_atomic_fetch_add(&tot->c[threadIdx.x], blk[threadIdx.x], __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
  } else if (threadIdx.x < 17) {
    if (blk[threadIdx.x])
      __hip_atomic_fetch_add(&tot->status[threadIdx.x - 8], blk[threadIdx.x], __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
  }
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

hipError_t launch_load_primaries(const PrimaryRec* prim, uint64_t n, const Store& S, uint32_t epoch,
                                 double k_a, uint32_t n_aval, uint32_t* active, Counters* ctr,
                                 int plain, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_load_primaries, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                     st, prim, n, S, epoch, k_a, n_aval, active, ctr, plain);
  return hipGetLastError();
}

template <bool B, int FK>
static void gen_one(const GasDev& G, const FieldDev& F, const RunParams& P, const Store& S,
                    const uint32_t* active, uint32_t n_active, uint32_t* next, Counters* ctr,
                    hipStream_t st) {
  hipLaunchKernelGGL((k_generation<B, FK>), dim3((n_active + kBlock - 1) / kBlock), dim3(kBlock), 0,
                     st, G, F, P, S, active, n_active, next, ctr);
}

hipError_t launch_generation(int banded, int field_kind, const GasDev& G, const FieldDev& F,
                             const RunParams& P, const Store& S, const uint32_t* active,
                             uint32_t n_active, uint32_t* next, Counters* ctr, hipStream_t st) {
  if (n_active == 0) return hipSuccess;
  if (banded) {
    if (field_kind == FIELD_SLAB)
      gen_one<true, FIELD_SLAB>(G, F, P, S, active, n_active, next, ctr, st);
    else
      gen_one<true, FIELD_POLAR>(G, F, P, S, active, n_active, next, ctr, st);
  } else {
    if (field_kind == FIELD_SLAB)
      gen_one<false, FIELD_SLAB>(G, F, P, S, active, n_active, next, ctr, st);
    else
      gen_one<false, FIELD_POLAR>(G, F, P, S, active, n_active, next, ctr, st);
  }
  return hipGetLastError();
}

template <bool B, int FK>
static const void* persistent_fn() {
  return reinterpret_cast<const void*>(&k_persistent<B, FK>);
}

static const void* pick_persistent(int banded, int field_kind) {
  if (banded) return field_kind == FIELD_SLAB ? persistent_fn<true, FIELD_SLAB>() : persistent_fn<true, FIELD_POLAR>();
  return field_kind == FIELD_SLAB ? persistent_fn<false, FIELD_SLAB>() : persistent_fn<false, FIELD_POLAR>();
}

hipError_t persistent_occupancy(int banded, int field_kind, int block, int* blocks_per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, pick_persistent(banded, field_kind),
                                                      block, 0);
}

template <bool B, int FK>
static void pers_one(const GasDev& G, const FieldDev& F, const RunParams& P, const Store& S,
                     Counters* ctr, uint32_t epoch, int fpp, int grid, int block, hipStream_t st) {
  hipLaunchKernelGGL((k_persistent<B, FK>), dim3(grid), dim3(block), 0, st, G, F, P, S, ctr, epoch,
                     fpp);
}

hipError_t launch_persistent(int banded, int field_kind, const GasDev& G, const FieldDev& F,
                             const RunParams& P, const Store& S, Counters* ctr, uint32_t epoch,
                             int flights_per_pass, int grid, int block, hipStream_t st) {
  if (banded) {
    if (field_kind == FIELD_SLAB)
      pers_one<true, FIELD_SLAB>(G, F, P, S, ctr, epoch, flights_per_pass, grid, block, st);
    else
      pers_one<true, FIELD_POLAR>(G, F, P, S, ctr, epoch, flights_per_pass, grid, block, st);
  } else {
    if (field_kind == FIELD_SLAB)
      pers_one<false, FIELD_SLAB>(G, F, P, S, ctr, epoch, flights_per_pass, grid, block, st);
    else
      pers_one<false, FIELD_POLAR>(G, F, P, S, ctr, epoch, flights_per_pass, grid, block, st);
  }
  return hipGetLastError();
}

hipError_t launch_stats(const Store& S, const Counters* ctr, AvalStats* stats, Totals* tot,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_stats, dim3(2048), dim3(kBlock), 0, st, S, ctr, stats, tot);
  return hipGetLastError();
}

}  // namespace avm
