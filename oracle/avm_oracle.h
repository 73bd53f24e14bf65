/*
 * avm_oracle.h -- plain, slow, FP64 CPU oracle for microscopic
 * electron-avalanche transport.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is what the HIP implementation is
 * checked against; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no source, header, table or
 * constant with the HIP implementation.
 *
 * What it computes (paper Sec. 2 and its Fig. 2: each electron is checked
 * for still being inside the volume, takes a random free flight in the local
 * field, may collide, and on an ionisation or attachment changes the electron
 * count, until every electron has a non-zero status; null-collision free
 * flights after Skullerud, cited in Sec. 1): every electron of every
 * avalanche is transported flight by flight
 * through a gas described by an energy-binned rate table with linear
 * interpolation between nodes, with a majorant rate Gamma >= nu(e) that turns
 * the flight law into "exponential with rate Gamma, real with probability
 * nu/Gamma".  Ionisation pushes a secondary electron; attachment and leaving
 * the volume terminate one.  The readings taken where the paper is silent are
 * listed in the design notes of the repository, and in the comments of
 * avm_oracle.c next to the code they govern.
 *
 * Parity pins: every function here is pinned by a CPU test against a closed
 * form, an invariant, brute force or an independent library (rocRAND's
 * Philox for the generator); the polar map's azimuthal interpolation,
 * periodic wrap and E_phi rotation against a field with a closed form, the
 * scattering samplers as the transport calls them against a brute-force
 * integrator, the ionisation energy split against the energy balance of
 * every single event.  Nothing here is "parity unpinned" except the
 * physical correctness of the synthetic gas models, which are definitions.
 *
 * Planted mistakes: compiled with one of the ORC_PLANT_* macros (only the
 * pin tests do this, into a separate library) the oracle carries one known
 * mistake, so that a test can show that its pin catches it.
 */
#ifndef AVM_ORACLE_H
#define AVM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_OK = 0, ORC_E_ARG = 1, ORC_E_NOMEM = 2 };

/* channel kind / angular model / energy split / node value kind */
enum { ORC_ELASTIC = 0, ORC_EXCITATION = 1, ORC_IONISATION = 2, ORC_ATTACHMENT = 3 };
enum { ORC_ISOTROPIC = 0, ORC_SCREENED_RUTHERFORD = 1 };
enum { ORC_SPLIT_UNIFORM = 0, ORC_SPLIT_OPAL_BEATY = 1 };
enum { ORC_VALUES_SIGMA = 0, ORC_VALUES_RATE = 1 };

/* electron status codes (non-zero = terminated) */
enum {
  ORC_ST_ACTIVE = 0, ORC_ST_LOW = 1, ORC_ST_HIGH = 2, ORC_ST_ATTACHED = 3,
  ORC_ST_WIRE = 4, ORC_ST_TUBE = 5, ORC_ST_TIME = 6, ORC_ST_ABANDONED = 7,
  ORC_ST_ERROR = 8
};

typedef struct {
  int32_t kind, angular, split, values_kind;
  double loss_eV, e_lo_eV, e_hi_eV, mass_ratio, split_w_eV, screening_eV;
  const double* values; /* n_bins+1 node values: cm^2 or 1/ns */
} orc_channel;

typedef struct orc_gas orc_gas;
typedef struct orc_field orc_field;

/* Build the rate table: nu at the nodes, cumulative rates, per-bin maxima,
 * band majorants (band_bins bins per band; 0 = a single band). */
int orc_gas_create(double e_max_eV, int32_t n_bins, double density_cm3, int32_t n_ch,
                   const orc_channel* ch, int32_t band_bins, orc_gas** out);
void orc_gas_destroy(orc_gas*);
/* Penning transfer of excitation channel c: with probability prob an
 * excitation is followed by an extra electron of energy energy_eV born
 * where it happened, isotropic (random blocks j = 2, 3 of the flight, as
 * for an ionisation; it counts as a secondary in n_ion). */
int orc_gas_set_penning(orc_gas*, int32_t channel, double prob, double energy_eV);
double orc_gas_gamma(const orc_gas*);
int32_t orc_gas_n_bands(const orc_gas*);
/* Gamma_b and the upper edge (eV) of band b (edge = +inf for the last band). */
int orc_gas_band(const orc_gas*, int32_t b, double* gamma_b, double* edge_eV);
/* Replace Gamma (and every band majorant) by a larger value (tests only). */
int orc_gas_set_gamma(orc_gas*, double gamma);
/* Interpolated per-channel rates at energy e; returns 1 if e is above the
 * table (rates then frozen at the last node). */
int orc_gas_rates(const orc_gas*, double e_eV, double* nu_ch, double* nu_total);
/* Copy of the cumulative table, node-major [(n_bins+1)][n_ch]. */
int orc_gas_cumulative(const orc_gas*, double* out);
int32_t orc_gas_band_of(const orc_gas*, double e_eV);

/* Slab z_lo <= z < z_hi with one uniform field vector per avalanche
 * (n_E == 1: the same field for every avalanche); B must be zero or along z. */
int orc_field_slab(double z_lo, double z_hi, uint32_t n_E, const double* E_vcm,
                   const double B_T[3], orc_field** out);
/* Coaxial wire (radius a) and tube (radius b) with a polar map of (E_r, E_phi)
 * float32 [n_r][n_phi] at r_i = a (b/a)^(i/(n_r-1)), phi_j = 2 pi j / n_phi. */
int orc_field_polar(double a, double b, int32_t n_r, int32_t n_phi, const float* E_r,
                    const float* E_phi, const double B_T[3], orc_field** out);
void orc_field_destroy(orc_field*);
int orc_field_eval(const orc_field*, const double r[3], uint32_t aval, double E[3]);

typedef struct {
  double x, y, z, t, e, dx, dy, dz;
  uint32_t aval, _pad;
} orc_primary; /* 72 bytes */

/* trace: the electron's decision trace, a running 32-bit hash over its
 * real collisions, masked nulls and band cuts, in flight order: starting
 * from 0, each such event at flight index k maps h to
 * rotl(h, 5) ^ (k * 2^18 + code) (mod 2^32), with code = c for a real
 * collision in channel c, 2^16 + c for a masked null whose chosen channel
 * is c, 2^17 for a band cut (channel indices below 2^16).  Two runs whose
 * electron made the same decisions give the same trace; null collisions
 * enter through n_null. */
typedef struct {
  double x0, y0, z0, t0, e0, x1, y1, z1, t1, e1;
  uint64_t eid, parent;
  uint32_t aval, status, n_real, n_ion, n_null, n_masked, n_band, n_overflow;
  uint32_t trace, _pad;
} orc_endpoint; /* 136 bytes */

typedef struct {
  uint64_t seed;
  int32_t banded;      /* 0: global majorant; 1: banded majorant (with B: helical bound) */
  int32_t fifo;        /* 0: LIFO stack per avalanche; 1: FIFO queue */
  double t_max_ns;     /* +inf: no time limit */
  uint32_t k_max;      /* flight index limit (<= 2^30-1) */
  int32_t n_threads;   /* 0: all online cores */
  /* banded majorant: before each flight the band is raised to the band of
   * the energy the electron would have after band_lookahead mean free times
   * 1/Gamma_b of its current band (without B the exact flight energy, with B
   * the helical bound); chosen from the state at the flight start, so the
   * restart rule keeps the sampling exact.  0: no lookahead. */
  double band_lookahead;
} orc_opts;

typedef struct orc_result orc_result;

/* Transport every primary whose index is listed in `sel` (NULL: all).  The
 * primary with array index i gets the electron id 2^63 | ids[i] (ids NULL:
 * ids[i] = i).  Endpoints are returned grouped by avalanche. */
int orc_run(const orc_gas*, const orc_field*, const orc_primary* prim, const uint64_t* ids,
            uint64_t n_prim, const orc_opts*, orc_result** out, int32_t* threads_used);

/* Induced signal on the readout electrode (the step after transport, paper
 * Sec. 3.2: induced signals are read out as usual once the avalanche is
 * simulated).  Shockley-Ramo: a point charge q at r induces -q phi_w(r) on
 * the electrode whose weighting potential is phi_w, so moving from r to r'
 * changes the induced charge by -q [phi_w(r') - phi_w(r)].  Readout
 * electrode: the z_hi plane of a slab, phi_w = (z - z_lo) / (z_hi - z_lo);
 * the wire of the coaxial geometry, phi_w = ln(b/rho) / ln(b/a).  Bin j
 * covers [T_j, T_j+1) with T_j = t0 + j dt; out[a n_bins + j] receives the
 * change of induced charge during bin j, in units of the elementary charge,
 * from the electrons (q = -1) of avalanche a: the sum of
 * phi_w(r(T_j+1)) - phi_w(r(T_j)) over them, each electron's times clamped
 * to its own lifetime (its motion before birth and after termination
 * contributes nothing).  Ions are not transported.  `out` holds
 * n_rows x n_bins values, n_rows > every avalanche id; it is accumulated
 * into (zero it first). */
typedef struct {
  double t0_ns, dt_ns;
  int32_t n_bins;
  uint32_t n_rows;
  double* out;
} orc_signal;

int orc_run_signal(const orc_gas*, const orc_field*, const orc_primary* prim, const uint64_t* ids,
                   uint64_t n_prim, const orc_opts*, const orc_signal* sig, orc_result** out,
                   int32_t* threads_used);
/* Weighting potential of the readout electrode at r (see above). */
double orc_weighting(const orc_field*, const double r[3]);
uint64_t orc_result_count(const orc_result*);
int orc_result_copy(const orc_result*, orc_endpoint* out);
void orc_result_destroy(orc_result*);

/* ---- single steps, exported for the pins ---- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double orc_u53(uint32_t w_hi, uint32_t w_lo);
float orc_u24(uint32_t w);
double orc_cos_screened_rutherford(double u, double e_eV, double screening_eV);
double orc_split_energy(int32_t split, double u, double e_avail, double w_eV);
void orc_rotate(const double d[3], double cos_t, double phi, double out[3]);
void orc_elastic(double e_eV, double mass_ratio, double cos_chi, double* e_out, double* cos_lab);
/* First exit time of z(s) = z0 + vz s + az s^2/2 from [z_lo, z_hi) within
 * (0, T]; returns 0 (none), ORC_ST_LOW or ORC_ST_HIGH. */
int orc_slab_exit(double z0, double vz, double az, double z_lo, double z_hi, double T,
                  double* s_exit);
/* Smallest s >= 0 with |v + a s|^2 = 2 k_a e_edge (-1 if none). */
double orc_band_root(const double v[3], const double a[3], double e_edge);
/* Free flight over time s in a field frozen at E, optional B. */
void orc_propagate(const double r0[3], const double v0[3], const double E[3], const double B[3],
                   double s, double r[3], double v[3]);
/* Helical-flight energy bound for the banded majorant with B:
 * out = {vp, ap, p, q, m} with 2 k_a e(s) <= (vp + ap s)^2 + min(p + q s, m)^2. */
void orc_helical_bound(const double v[3], const double E[3], const double B[3], double out[5]);
/* Smallest s >= 0 at which that bound reaches e_edge (0: already; +inf: never). */
double orc_helical_bound_root(const double b[5], double e_edge);
/* Decisions (all runs of the process) that saw an interpolated total rate
 * above the majorant in use; never expected to be non-zero. */
uint64_t orc_majorant_violations(void);
void orc_reset_majorant_violations(void);
double orc_k_a(void);
double orc_k_b(void);

#ifdef __cplusplus
}
#endif
#endif
