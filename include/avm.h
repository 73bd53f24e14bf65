/*
 * avm.h -- C-ABI of the MI355X (gfx950) microscopic electron-avalanche
 * transport library, libavm.so.
 *
 * What the library computes is the paper's AvalancheMicroscopic method
 * (Sec. 2 and its Fig. 2; user interface in Sec. 3.2): electrons are carried
 * collision by collision through a gas in an electric (and optional
 * magnetic) field; every ionisation adds a secondary electron; the run ends
 * when every electron has a non-zero status; the result is one endpoint per
 * electron (start and end position, time and energy, status) and the
 * per-avalanche gain (electrons after the avalanche / initial electrons,
 * Sec. 2).  Free flights are null-collision flights (Skullerud, cited in
 * Sec. 1) against a majorant rate taken from an energy-binned rate table.
 *
 * Conventions.
 *  - Units: cm, ns, eV, V/cm, tesla, cm^2, cm^-3.
 *  - Every call returns avm_status.  Nothing aborts or throws across the
 *    ABI.  On error no handle is created and no output is written, except
 *    AVM_E_CAPACITY (the run completed, but secondaries beyond the capacity
 *    were dropped; see avm_counts.truncated).  avm_last_error() returns a
 *    thread-local description of the last failing call on this thread.
 *  - Handles are owned by the library and released with *_destroy.  A handle
 *    is not thread-safe; distinct handles may be used from distinct threads.
 *  - Input arrays are caller-owned host memory, copied during the call,
 *    unless a parameter says "device pointer".
 *  - All device work of a run is enqueued on the run's HIP stream.
 */
#ifndef AVM_H
#define AVM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define AVM_ABI_VERSION 3

typedef enum {
  AVM_OK = 0,
  AVM_E_ARG = 1,         /* invalid argument (message says which)                   */
  AVM_E_NOMEM = 2,       /* host or device allocation failed                        */
  AVM_E_HIP = 3,         /* a HIP runtime call failed (message carries its text)    */
  AVM_E_CAPACITY = 4,    /* run finished but electrons beyond capacity were dropped */
  AVM_E_UNSUPPORTED = 5, /* valid request this library does not implement           */
  AVM_E_TIMEOUT = 6,     /* the run did not finish within the requested wall time   */
  AVM_E_STATE = 7        /* call out of order (e.g. results before a run)           */
} avm_status;

/* Thread-local text of the last error on the calling thread ("" if none). */
const char* avm_last_error(void);
int32_t avm_abi_version(void);
/* Number of HIP devices visible (0 when none); never fails. */
int32_t avm_device_count(void);

/* ------------------------------------------------------------------------ */
/* Gas: energy-binned rate table                                             */
/* ------------------------------------------------------------------------ */
typedef enum { AVM_CH_ELASTIC = 0, AVM_CH_EXCITATION = 1, AVM_CH_IONISATION = 2, AVM_CH_ATTACHMENT = 3 } avm_channel_kind;
typedef enum { AVM_ANG_ISOTROPIC = 0, AVM_ANG_SCREENED_RUTHERFORD = 1 } avm_angular;
typedef enum { AVM_SPLIT_UNIFORM = 0, AVM_SPLIT_OPAL_BEATY = 1 } avm_split;
typedef enum { AVM_VALUES_SIGMA = 0, AVM_VALUES_RATE = 1 } avm_values_kind;

/* One collision channel, tabulated at the n_bins+1 nodes e_k = k E_max / n_bins. */
typedef struct {
  int32_t kind;        /* avm_channel_kind                                               */
  int32_t angular;     /* elastic only: avm_angular                                      */
  int32_t split;       /* ionisation only: avm_split                                     */
  int32_t values_kind; /* AVM_VALUES_SIGMA: cm^2 (rate = N sigma v); AVM_VALUES_RATE: 1/ns */
  double loss_eV;      /* excitation threshold / ionisation potential (0 otherwise)      */
  double e_lo_eV;      /* the channel acts only for e in [e_lo, e_hi); interpolated rate */
  double e_hi_eV;      /*   outside the window is a "masked" null collision (INFINITY ok) */
  double mass_ratio;   /* elastic: electron mass / target mass                           */
  double split_w_eV;   /* Opal-Beaty w: dsigma/de_s ~ 1/(1 + (e_s/w)^2) on [0, (e-I)/2] */
  double screening_eV; /* screened Rutherford: eta(e) = screening / (8 e)               */
  const double* values;/* host pointer, n_bins+1 node values (>= 0, finite); copied      */
} avm_channel;

typedef struct avm_gas avm_gas;

/* Paper: Sec. 1 (null-collision free flights after Skullerud need a bound
 * of the collision rate) and Sec. 2 with Fig. 2 (the loop asks whether a
 * collision happens and of which kind); Sec. 3.1 (the gas data are
 * prepared once, before the transport, and moved to the device).
 * Build the rate table on `device` (rate-table builder kernels): rates at the
 * nodes, cumulative rates over channels (in the given order), per-bin maxima
 * max(nu_k, nu_k+1) -- exact bounds of the linear interpolation -- the global
 * majorant Gamma and, with band_bins > 0, band majorants Gamma_b = max of the
 * per-bin maxima below the band's upper edge (bands of band_bins bins).
 * Errors: AVM_E_ARG for n_channels < 1, n_bins < 1, e_max <= 0, negative or
 * non-finite values, an excitation/ionisation window opening below its loss,
 * or a table with no collisions at all.  Not timed work (done once per gas). */
avm_status avm_gas_create(int32_t device, double e_max_eV, int32_t n_bins, double density_cm3,
                          int32_t n_channels, const avm_channel* channels, int32_t band_bins,
                          avm_gas** out);

typedef struct {
  double gamma;       /* global majorant, 1/ns */
  double e_max_eV;
  int32_t n_bins, n_channels, n_bands, band_bins;
} avm_gas_info;

/* The majorant and table sizes of a gas (Sec. 1: the null-collision bound).
 * Errors: AVM_E_ARG for NULL arguments. */
avm_status avm_gas_get_info(const avm_gas* gas, avm_gas_info* out);
/* Copy the device tables to host buffers (any may be NULL):
 * cumulative [(n_bins+1) * n_channels] node-major; band_gamma and band_edge_eV
 * [n_bands] (the last edge is +INFINITY). */
avm_status avm_gas_get_tables(const avm_gas* gas, double* cumulative, double* band_gamma,
                              double* band_edge_eV);
/* Sec. 1 (the null-collision bound, here per energy band; an extension).
 * Rebuild the band majorants with a new band width (band_bins > 0; 0 drops
 * the bands, leaving the global majorant only).  The per-bin maxima are kept
 * from avm_gas_create, so the bands are the ones avm_gas_create would build
 * with this band_bins.  The gas must not be in use by a run that has been
 * executed and not yet synced; runs created earlier use the new bands from
 * their next execute (a captured graph is captured again).  Errors:
 * AVM_E_ARG for band_bins < 0. */
avm_status avm_gas_set_band_bins(avm_gas* gas, int32_t band_bins);
/* Penning transfer of an excitation channel (a synthetic extension; real
 * transfer probabilities need gas data): each excitation in `channel` is
 * followed, with `probability`, by an extra electron of energy `energy_eV`
 * born where the excitation happened, isotropic; the exciting electron is
 * scattered as for any excitation.  The decision takes the first uniform of
 * the flight's random block j = 2; the new electron's direction and id come
 * from blocks 2 and 3 as for an ionisation secondary, and it counts as a
 * secondary (n_ion).  Probability 0 switches it off.  The gas must not be
 * in use by an executing run.  Errors: AVM_E_ARG for a channel that is not
 * an excitation, a probability outside [0, 1], a negative or non-finite
 * energy. */
avm_status avm_gas_set_penning(avm_gas* gas, int32_t channel, double probability, double energy_eV);
void avm_gas_destroy(avm_gas* gas);

/* ------------------------------------------------------------------------ */
/* Fields                                                                    */
/* ------------------------------------------------------------------------ */
typedef struct avm_field avm_field;

/* Paper: Fig. 2 (the field at the electron is looked up for every flight)
 * and Sec. 3.1 (field data are moved to the device once, before the first
 * transport); the analytic slab and the polar map stand in for the field
 * maps of the case studies (Sec. 4).
 * Parallel-plate slab z_lo <= z < z_hi (x, y unbounded), uniform field.
 * E_vcm: host pointer to n_E field vectors [n_E][3]; n_E == 1 applies one
 * field to every avalanche, otherwise avalanche a uses vector a.
 * B_T: uniform magnetic field (may be NULL); it must be zero or along z.
 * Electrons leaving through z_lo get status 1, through z_hi status 2. */
avm_status avm_field_slab(int32_t device, double z_lo_cm, double z_hi_cm, uint32_t n_E,
                          const double* E_vcm, const double* B_T, avm_field** out);

/* Coaxial wire (radius a) inside a tube (radius b), field from a polar map:
 * E_r and E_phi are host float arrays [n_r][n_phi] sampled at
 * r_i = a (b/a)^(i/(n_r-1)), phi_j = 2 pi j / n_phi; the field is bilinear
 * in (ln r, phi), clamped in r, periodic in phi.  B_T: uniform (may be NULL).
 * Electrons reaching rho <= a get status 4, rho >= b status 5 (bisection of
 * the flight on the inside/outside predicate). */
avm_status avm_field_polar_map(int32_t device, double a_cm, double b_cm, int32_t n_r,
                               int32_t n_phi, const float* E_r, const float* E_phi,
                               const double* B_T, avm_field** out);
void avm_field_destroy(avm_field* field);

/* ------------------------------------------------------------------------ */
/* Runs                                                                      */
/* ------------------------------------------------------------------------ */
/* A primary electron: position, time, kinetic energy, direction (normalised
 * by the library; ignored at zero energy, where (0,0,1) is used), avalanche. */
typedef struct {
  double x, y, z, t, e, dx, dy, dz;
  uint32_t avalanche, _pad;
} avm_primary; /* 72 bytes */

/* FP64: every step in double precision.  FP32_MIXED: velocities, flight
 * times, energies, table interpolation and scattering in single precision,
 * position and time accumulated in double, boundary crossings solved in
 * double, and a collision decision whose single-precision margin is below
 * 2^-18 taken again in double; it draws the same random blocks as FP64
 * (24-bit uniforms from the same words), so the two are paired runs. */
typedef enum { AVM_FP64 = 0, AVM_FP32_MIXED = 1 } avm_precision;
typedef enum { AVM_MAJORANT_GLOBAL = 0, AVM_MAJORANT_BANDED = 1 } avm_majorant;
typedef enum {
  AVM_MODE_PLAIN = 0,  /* generation-synchronous loop of Fig. 2: one kernel per
                          transport iteration, host reads the active count */
  AVM_MODE_BATCHED = 1 /* one persistent kernel over every avalanche, fed by a
                          device work queue; no host round trip */
} avm_mode;

typedef struct {
  uint64_t seed;          /* Philox key                                                  */
  int32_t precision;      /* avm_precision                                               */
  int32_t majorant;       /* avm_majorant (banded needs B = 0 and band_bins > 0)          */
  int32_t mode;           /* avm_mode                                                    */
  int32_t flights_per_pass; /* batched: flights between queue visits (0: 40 FP64, 48 FP32) */
  double t_max_ns;        /* time limit (INFINITY: none) -> status 6                     */
  uint64_t capacity;      /* electrons the run can hold (primaries included), >= n_prim  */
  uint32_t k_max;         /* flights per electron before status 7; 0: 2^30-1             */
  int32_t waves_per_cu;   /* batched: resident waves per CU (0: occupancy limit)          */
  double timeout_s;       /* avm_run_sync wall-time limit (0: none) -> AVM_E_TIMEOUT      */
  void* hip_stream;       /* hipStream_t for all of the run's work (NULL: null stream)    */
  int32_t graph;          /* batched: 1 = capture the run's device work (reset, primary  */
                          /*   load, transport with its statistics, result copies) into  */
                          /*   a HIP graph on the first execute and replay it afterwards */
  float band_lookahead;   /* banded: before each flight the band is raised to the band   */
                          /*   of the energy after this many mean free times of the      */
                          /*   current band (flight energy; with B its helical bound);   */
                          /*   the restart rule keeps sampling exact; 0: none; >= 0      */
} avm_run_opts;

/* One electron's record (the endpoint getter of paper Sec. 3.2: start and
 * end position, time and energy, status).  status: 1 left z_lo, 2 left
 * z_hi, 3 attached, 4 hit the wire, 5 reached the tube, 6 time limit,
 * 7 flight limit, 8 numerical error.  eid: primaries 2^63 | index,
 * secondaries 63-bit ids drawn from the parent's random stream; parent = 0
 * for primaries.  trace: the electron's decision trace, a running 32-bit
 * hash over its real collisions, masked nulls and band cuts in flight
 * order -- from 0, each such event at flight index k maps h to
 * rotl(h, 5) ^ (k 2^18 + code), code = c for a real collision in channel c,
 * 2^16 + c for a masked null at channel c, 2^17 for a band cut -- so that
 * runs can be compared decision by decision (null collisions enter through
 * n_null). */
typedef struct {
  double x0, y0, z0, t0, e0, x1, y1, z1, t1, e1;
  uint64_t eid, parent;
  uint32_t avalanche, status, n_real, n_ion, n_null, n_masked, n_band, n_overflow;
  uint32_t trace, _pad;
} avm_endpoint; /* 136 bytes */

/* Counters of a run (or of a range of avalanches).  gain of avalanche a =
 * n_endpoints / number of its primaries. */
typedef struct {
  uint64_t n_endpoints; /* electrons, primaries included                          */
  uint64_t n_ion;       /* ionisations = secondaries created                      */
  uint64_t n_att;       /* attachments                                            */
  uint64_t n_real;      /* real collisions (elastic+excitation+ionisation+attach) */
  uint64_t n_null;      /* null collisions                                        */
  uint64_t n_masked;    /* null because the chosen channel's window excludes e    */
  uint64_t n_band;      /* flights cut at a band edge (banded majorant)            */
  uint64_t n_overflow;  /* lookups above the table's last node                    */
  uint64_t n_status[9]; /* electrons per status code                              */
  uint64_t n_requested; /* electrons the run tried to create (> capacity: truncated) */
  uint32_t truncated, _pad;
} avm_counts;

typedef struct avm_run avm_run;

/* Paper: Sec. 2 and Fig. 2 (every electron transported flight by flight
 * until it terminates; ionisations add electrons); Sec. 3.2 (the run mode
 * and the device are chosen by the user; initial electrons in, endpoints
 * out).
 * Prepare a run: validates, allocates the electron store (capacity
 * electrons, ~200 bytes each) on the gas's device.  prim: n_prim records,
 * a host pointer, or a device pointer when prim_on_device = 1 (it must stay
 * valid until avm_run_sync returns).  n_aval: number of avalanches (every
 * primary's avalanche id must be < n_aval, and < n_E for per-avalanche slab
 * fields).  Gas and field must stay alive for the run's lifetime. */
avm_status avm_run_create(const avm_gas* gas, const avm_field* field, const avm_primary* prim,
                          int32_t prim_on_device, uint64_t n_prim, uint32_t n_aval,
                          const avm_run_opts* opts, avm_run** out);
/* Paper: Sec. 2 (the loop of Fig. 2; the paper's generation-synchronous
 * stack processing is the PLAIN mode, the idle-thread problem of Fig. 1 is
 * what the BATCHED mode removes).
 * Enqueue the run on its stream.  BATCHED: asynchronous.  PLAIN: returns
 * when the generation loop has finished (it reads the active count back
 * after every transport iteration, as the paper's stack processing does). */
avm_status avm_run_execute(avm_run* run);
/* Wait for the run, then fetch the totals.  AVM_E_CAPACITY if truncated;
 * AVM_E_TIMEOUT when the device time budget (timeout_s) ran out;
 * AVM_E_ARG when a device primary had a bad avalanche id. */
avm_status avm_run_sync(avm_run* run);
/* Totals of the last execute (Sec. 2: gain = electrons after the avalanche
 * over initial electrons).  AVM_E_STATE before avm_run_sync. */
avm_status avm_run_counts(const avm_run* run, avm_counts* out);
/* Per-avalanche counters for avalanches [first, first+n) (n_status and
 * n_requested are zero in these records). */
avm_status avm_run_avalanche_counts(const avm_run* run, uint32_t first, uint32_t n,
                                    avm_counts* out);
/* Endpoint getters of Sec. 3.2 (the number of endpoints; each endpoint's
 * start and end position, time, energy and status).
 * Number of endpoints stored (= min(n_requested, capacity)). */
avm_status avm_run_num_endpoints(const avm_run* run, uint64_t* n);
/* Copy endpoints [first, first+n) in storage order to host memory. */
avm_status avm_run_endpoints(const avm_run* run, uint64_t first, uint64_t n, avm_endpoint* out);

/* The end of one electron (written once, when it terminates): position,
 * time and energy, status, counters and decision trace, as in
 * avm_endpoint.  Kept as one record per electron so that a termination
 * writes 72 contiguous bytes. */
typedef struct {
  double x1, y1, z1, t1, e1;
  uint32_t status, n_real, n_ion, n_null, n_masked, n_band, n_overflow, trace;
} avm_end_record; /* 72 bytes */

/* Device pointers to the endpoints, indexed by storage slot, valid until
 * avm_run_destroy: the start of each electron as arrays (structure of
 * arrays, written when it is created), its end as records. */
typedef struct {
  const double *x0, *y0, *z0, *t0, *e0;
  const uint64_t *eid, *parent;
  const uint32_t* avalanche;
  const avm_end_record* end;
} avm_endpoint_arrays;
avm_status avm_run_endpoint_arrays(const avm_run* run, avm_endpoint_arrays* out);

/* Sec. 3.3 (each event of a validation run draws its own random numbers).
 * The seed of the following executes: the same primaries and options with
 * other random streams, without a new run (a captured graph is captured
 * again on the next execute).  Results of the last execute are no longer
 * available.  Errors: AVM_E_ARG for a NULL run; AVM_E_STATE while the run
 * executes. */
avm_status avm_run_set_seed(avm_run* run, uint64_t seed);
/* Sec. 4 (the GPU run time measured against the CPU run).
 * Kernel time of the last execute (ms, HIP events on the run's stream
 * around the transport kernels; plain mode: summed over iterations; graph
 * mode: the whole replayed graph) and the number of transport iterations
 * (plain) or 1 (batched). */
avm_status avm_run_timing(const avm_run* run, double* transport_ms, uint32_t* iterations);
void avm_run_destroy(avm_run* run);

/* ------------------------------------------------------------------------ */
/* Induced signal                                                            */
/* ------------------------------------------------------------------------ */
/* Request the induced signal on the readout electrode for the following
 * executes (paper Sec. 3.2: the induced signal is read out once the
 * avalanche has been simulated).  Shockley-Ramo: a point charge q at r
 * induces -q phi_w(r) on an electrode with weighting potential phi_w.
 * Readout electrode: the z_hi plane of a slab, phi_w = (z - z_lo) /
 * (z_hi - z_lo); the wire of the coaxial geometry, phi_w = ln(b/rho) /
 * ln(b/a).  Bin j covers [t0 + j dt, t0 + (j+1) dt); the value of bin j of
 * avalanche a is the change of induced charge during the bin, in units of
 * the elementary charge, from the avalanche's electrons (charge -1): the sum
 * over them of phi_w(r(end of the bin)) - phi_w(r(start of the bin)), each
 * electron's times clamped to its own life (the position at a bin edge comes
 * from the flight formula).  Ions are not transported.  Batched mode only
 * (AVM_E_UNSUPPORTED otherwise); allocates n_aval x n_bins doubles on the
 * device; the deposits are device atomics, so sums are exact up to the
 * order of rounding.  Errors: AVM_E_ARG for n_bins < 1, dt <= 0, non-finite
 * values; AVM_E_STATE while the run executes. */
avm_status avm_run_set_signal(avm_run* run, double t0_ns, double dt_ns, int32_t n_bins);
/* Copy the signal rows of avalanches [first, first+n) after avm_run_sync:
 * out[(a - first) n_bins + j].  AVM_E_STATE without a requested signal or
 * before sync. */
avm_status avm_run_signal(const avm_run* run, uint32_t first, uint32_t n, double* out);

/* ------------------------------------------------------------------------ */
/* Autotuning of the batched launch                                          */
/* ------------------------------------------------------------------------ */
#define AVM_TUNE_BANDS 1u /* also choose the gas's band width (banded majorant) */

typedef struct {
  int32_t flights_per_pass; /* chosen flights between queue visits                     */
  int32_t waves_per_cu;     /* chosen resident waves per CU (0: occupancy limit)        */
  int32_t band_bins;        /* band width the gas is left with                          */
  int32_t trials;           /* configurations timed (0 when taken from the cache)       */
  int32_t from_cache;       /* 1 when cache_path already held this workload's choice    */
  float band_lookahead;     /* chosen band lookahead (banded; results depend on it)     */
  double best_ms;           /* transport-kernel ms of the chosen configuration (cache:  */
                            /*   as recorded)                                           */
  double start_ms;          /* transport-kernel ms of the starting configuration        */
  uint64_t key;             /* workload key (device, gas table, field, sizes, options)  */
} avm_tune_result;

/* No counterpart in the paper (its launch is fixed); the batched launch's
 * parameters and the band width decide how many threads idle (Fig. 1).
 * Choose flights_per_pass, waves_per_cu and (with AVM_TUNE_BANDS and the
 * banded majorant) the gas's band width and the band lookahead for a
 * batched run of these
 * primaries: a coordinate search over candidate values, each timed on the
 * device (HIP events around the transport kernel, best of two executions
 * after one warm-up).  The trials run the given primaries in full, so for a
 * large workload pass a representative subset.  base: the run options the
 * result applies to (mode must be AVM_MODE_BATCHED; seed, precision,
 * majorant, limits, capacity and stream are used as given; graph is
 * ignored).  cache_path (may be NULL): a text file of earlier choices; a
 * line with this workload's key is used without trials, a new choice is
 * appended.  The gas is left with the chosen band width.  Results of runs
 * depend on the band width and lookahead (other random draws), not on
 * flights_per_pass or waves_per_cu.  Errors: AVM_E_ARG as avm_run_create, or a mode other than
 * batched; any error of the trial runs. */
avm_status avm_autotune(avm_gas* gas, const avm_field* field, const avm_primary* prim,
                        int32_t prim_on_device, uint64_t n_prim, uint32_t n_aval,
                        const avm_run_opts* base, uint32_t flags, const char* cache_path,
                        avm_tune_result* out);

/* ------------------------------------------------------------------------ */
/* Batched transport that allocates nothing                                   */
/* ------------------------------------------------------------------------ */
/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The same
 * transport as avm_run_execute in the batched mode (same kernels, same
 * results for the same inputs and options), with the caller's arrays as
 * the outputs.  Its working memory -- run counters, queue entries, the
 * start velocities of queued electrons, the store descriptor and the
 * totals -- is one static device array of the library per GPU, of
 * 32 bytes x AVM_NOALLOC_MAX_ELECTRONS + 4 KiB (128 MiB), which each GPU the
 * library runs on holds until the process ends.  Every call on a GPU shares
 * that GPU's array, so calls that overlap on one GPU (on different streams,
 * or from different threads) race and give wrong results: serialise them.
 * Nothing is allocated or freed, on the host or the device, after the
 * first call on a device (which looks up the array's device address).
 *
 * prim: device pointer, n_prim records (as avm_run_create with
 *   prim_on_device = 1; a bad avalanche id sets AVM_NOALLOC_BAD_AVALANCHE).
 * opts: mode must be AVM_MODE_BATCHED and graph 0; capacity is the length of
 *   every per-electron output array (1 <= capacity <=
 *   AVM_NOALLOC_MAX_ELECTRONS, and >= n_prim); hip_stream is where the work
 *   is enqueued; timeout_s bounds the transport kernel on the device (the
 *   flag AVM_NOALLOC_TIMEOUT), nothing waits on the host.
 * out: device pointers, caller-owned.  The per-electron arrays and end
 *   records are indexed by storage slot as in avm_endpoint_arrays (slots
 *   [0, min(n_requested, capacity)) are written); aval_counts [n_aval][8]
 *   receives the per-avalanche counters (endpoints, ionisations, attachments, real,
 *   null, masked, band cuts, overflows) and is cleared first; counts
 *   receives one avm_counts record of totals, flags one word of
 *   AVM_NOALLOC_* bits.
 * Asynchronous: returns once the work is enqueued; results are valid after
 * the stream has reached this point.  Errors (nothing enqueued): AVM_E_ARG
 * for NULL arguments or arrays, a capacity outside the limits, options as
 * avm_run_create, a mode other than batched, graph != 0; AVM_E_HIP for a
 * failing launch. */
#define AVM_NOALLOC_MAX_ELECTRONS 4194304u
#define AVM_NOALLOC_TIMEOUT 1u        /* the transport kernel ran out of its time budget */
#define AVM_NOALLOC_BAD_AVALANCHE 2u  /* a primary's avalanche id was >= n_aval          */
#define AVM_NOALLOC_TRUNCATED 4u      /* electrons beyond capacity were dropped           */

typedef struct {
  double *x0, *y0, *z0, *t0, *e0;
  uint64_t *eid, *parent;
  uint32_t* avalanche;
  avm_end_record* end;   /* [capacity]                         */
  uint64_t* aval_counts; /* [n_aval][8]                       */
  avm_counts* counts;    /* one record                         */
  uint32_t* flags;       /* one word of AVM_NOALLOC_* bits     */
} avm_noalloc_out;

avm_status avm_run_noalloc(const avm_gas* gas, const avm_field* field, const avm_primary* prim,
                           uint64_t n_prim, uint32_t n_aval, const avm_run_opts* opts,
                           const avm_noalloc_out* out);

#ifdef __cplusplus
}
#endif
#endif
