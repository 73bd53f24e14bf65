/*
 * avm_oracle.c -- plain FP64 CPU oracle for microscopic electron-avalanche
 * transport.  TEST INFRASTRUCTURE ONLY (see avm_oracle.h): loaded by the
 * tests, the smoke check and the benchmark's CPU-baseline leg, never by the
 * product path.
 *
 * Built with -O2 -ffp-contract=off and no fast-math, so every expression is
 * evaluated exactly as written, one IEEE-754 double operation at a time.
 * Nothing is blocked, fused or reordered: each electron is carried through
 * the paper's loop (Fig. 2) one flight at a time, exactly as the comments
 * state.  Avalanches are independent, so whole avalanches are spread over
 * threads; inside an avalanche the electrons are processed from a LIFO stack
 * (or a FIFO queue), which the random-number protocol makes irrelevant.
 */
#define _GNU_SOURCE
#include "avm_oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

/* ------------------------------------------------------------------------ */
/* Units and constants: cm, ns, eV, V/cm, T.                                */
/* dv/dt = -k_a E - k_b (v x B) for an electron; e = |v|^2 / (2 k_a).       */
/* ------------------------------------------------------------------------ */
static const double C_CM_PER_NS = 29.9792458;     /* speed of light */
static const double C_M_PER_S = 299792458.0;
static const double ME_C2_EV = 510998.95;         /* electron rest energy */
static const double TWO_PI = 6.283185307179586;

double orc_k_a(void) { return (C_CM_PER_NS * C_CM_PER_NS) / ME_C2_EV; } /* (cm/ns^2)/(V/cm) */
double orc_k_b(void) { return 1e-9 * (C_M_PER_S * C_M_PER_S) / ME_C2_EV; } /* rad/(ns T) */

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as  */
/* easy as 1, 2, 3", SC'11): ten rounds of two 32x32->64 multiplications,   */
/* key bumped by the Weyl constants between rounds.                          */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t y0 = hi1 ^ x1 ^ k0;
    uint32_t y2 = hi0 ^ x3 ^ k1;
    x0 = y0;
    x1 = lo1;
    x2 = y2;
    x3 = lo0;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* 53-bit uniform in (0, 1]: 27 high bits of w_hi, 26 high bits of w_lo. */
double orc_u53(uint32_t w_hi, uint32_t w_lo)
{
  uint64_t m = ((uint64_t)(w_hi >> 5) << 26) + (uint64_t)(w_lo >> 6);
  return (double)(m + 1) * (1.0 / 9007199254740992.0);
}

/* 24-bit uniform in (0, 1] from the high bits of one word. */
float orc_u24(uint32_t w) { return (float)((w >> 8) + 1u) * (1.0f / 16777216.0f); }

/* One random block of an event: counter (4k + j, aval, eid_lo, eid_hi),
 * key (seed_lo, seed_hi).  k is the electron's flight index, j selects the
 * block inside the event: 0 flight, 1 scattering, 2 and 3 ionisation. */
static void draw(uint64_t seed, uint32_t aval, uint64_t eid, uint32_t k, uint32_t j, uint32_t w[4])
{
  uint32_t ctr[4] = {4u * k + j, aval, (uint32_t)eid, (uint32_t)(eid >> 32)};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  orc_philox4x32_10(ctr, key, w);
}

/* ------------------------------------------------------------------------ */
/* Gas rate table                                                            */
/* ------------------------------------------------------------------------ */
struct orc_gas {
  int32_t n_bins, n_ch;
  double e_max, scale; /* scale = n_bins / e_max */
  int32_t *kind, *angular, *split;
  double *loss, *e_lo, *e_hi, *mass_ratio, *split_w, *screening;
  double *cum;    /* [(n_bins+1)][n_ch] cumulative rates, 1/ns */
  double *total;  /* [n_bins+1] total rate at the nodes */
  double *binmax; /* [n_bins] max(total_k, total_k+1) */
  double gamma;   /* global majorant */
  int32_t band_bins, n_bands;
  double *band_gamma; /* [n_bands] */
  double *band_edge;  /* [n_bands] upper energy edge; +inf for the last */
  double *penning_prob, *penning_e; /* [n_ch] Penning transfer of excitations */
};

static void gas_free(orc_gas* g)
{
  if (!g) return;
  free(g->kind); free(g->angular); free(g->split);
  free(g->loss); free(g->e_lo); free(g->e_hi); free(g->mass_ratio); free(g->split_w);
  free(g->screening); free(g->cum); free(g->total); free(g->binmax);
  free(g->band_gamma); free(g->band_edge);
  free(g->penning_prob); free(g->penning_e);
  free(g);
}

void orc_gas_destroy(orc_gas* g) { gas_free(g); }

int orc_gas_create(double e_max_eV, int32_t n_bins, double density_cm3, int32_t n_ch,
                   const orc_channel* ch, int32_t band_bins, orc_gas** out)
{
  if (!out || !ch || n_ch < 1 || n_bins < 1 || !(e_max_eV > 0.0) || !isfinite(e_max_eV) ||
      !(density_cm3 >= 0.0) || band_bins < 0)
    return ORC_E_ARG;
  for (int c = 0; c < n_ch; ++c) {
    if (!ch[c].values || ch[c].kind < 0 || ch[c].kind > 3) return ORC_E_ARG;
    if (!(ch[c].e_lo_eV <= ch[c].e_hi_eV) || !(ch[c].loss_eV >= 0.0)) return ORC_E_ARG;
    if ((ch[c].kind == ORC_EXCITATION || ch[c].kind == ORC_IONISATION) &&
        !(ch[c].e_lo_eV >= ch[c].loss_eV))
      return ORC_E_ARG;
    for (int32_t k = 0; k <= n_bins; ++k)
      if (!(ch[c].values[k] >= 0.0) || !isfinite(ch[c].values[k])) return ORC_E_ARG;
  }
  orc_gas* g = (orc_gas*)calloc(1, sizeof(orc_gas));
  if (!g) return ORC_E_NOMEM;
  size_t nn = (size_t)n_bins + 1;
  g->n_bins = n_bins;
  g->n_ch = n_ch;
  g->e_max = e_max_eV;
  g->scale = (double)n_bins / e_max_eV;
  g->kind = calloc(n_ch, sizeof(int32_t));
  g->angular = calloc(n_ch, sizeof(int32_t));
  g->split = calloc(n_ch, sizeof(int32_t));
  g->loss = calloc(n_ch, sizeof(double));
  g->e_lo = calloc(n_ch, sizeof(double));
  g->e_hi = calloc(n_ch, sizeof(double));
  g->mass_ratio = calloc(n_ch, sizeof(double));
  g->split_w = calloc(n_ch, sizeof(double));
  g->screening = calloc(n_ch, sizeof(double));
  g->penning_prob = calloc(n_ch, sizeof(double));
  g->penning_e = calloc(n_ch, sizeof(double));
  g->cum = calloc(nn * (size_t)n_ch, sizeof(double));
  g->total = calloc(nn, sizeof(double));
  g->binmax = calloc((size_t)n_bins, sizeof(double));
  if (!g->kind || !g->angular || !g->split || !g->loss || !g->e_lo || !g->e_hi ||
      !g->mass_ratio || !g->split_w || !g->screening || !g->cum || !g->total || !g->binmax ||
      !g->penning_prob || !g->penning_e) {
    gas_free(g);
    return ORC_E_NOMEM;
  }
  for (int c = 0; c < n_ch; ++c) {
    g->kind[c] = ch[c].kind;
    g->angular[c] = ch[c].angular;
    g->split[c] = ch[c].split;
    g->loss[c] = ch[c].loss_eV;
    g->e_lo[c] = ch[c].e_lo_eV;
    g->e_hi[c] = ch[c].e_hi_eV;
    g->mass_ratio[c] = ch[c].mass_ratio;
    g->split_w[c] = ch[c].split_w_eV;
    g->screening[c] = ch[c].screening_eV;
  }
  const double k_a = orc_k_a();
  /* nu_c(e_k) = N sigma_c(e_k) v(e_k), v = sqrt(2 k_a e); cumulative over the
   * channels in the caller's order; total = last cumulative column. */
  for (int32_t k = 0; k <= n_bins; ++k) {
    double e_k = ((double)k * e_max_eV) / (double)n_bins;
    double speed = sqrt(2.0 * k_a * e_k);
    double acc = 0.0;
    for (int c = 0; c < n_ch; ++c) {
      double nu;
      if (ch[c].values_kind == ORC_VALUES_RATE)
        nu = ch[c].values[k];
      else
        nu = (density_cm3 * ch[c].values[k]) * speed;
      acc = acc + nu;
      g->cum[(size_t)k * n_ch + c] = acc;
    }
    g->total[k] = acc;
  }
  /* Linear interpolation inside bin k never exceeds the larger end node. */
  double gmax = 0.0;
  for (int32_t k = 0; k < n_bins; ++k) {
    g->binmax[k] = g->total[k] > g->total[k + 1] ? g->total[k] : g->total[k + 1];
    if (g->binmax[k] > gmax) gmax = g->binmax[k];
  }
  if (!(gmax > 0.0) || !isfinite(gmax)) {
    gas_free(g);
    return ORC_E_ARG; /* no collisions at all */
  }
  g->gamma = gmax;
  /* Bands of band_bins bins: Gamma_b is the maximum over every bin below the
   * band's upper edge (a prefix maximum), so it also bounds the rate of an
   * electron that slows down.  The last band reaches to +inf with Gamma. */
  g->band_bins = band_bins;
  g->n_bands = band_bins > 0 ? (n_bins + band_bins - 1) / band_bins : 1;
  g->band_gamma = calloc((size_t)g->n_bands, sizeof(double));
  g->band_edge = calloc((size_t)g->n_bands, sizeof(double));
  if (!g->band_gamma || !g->band_edge) {
    gas_free(g);
    return ORC_E_NOMEM;
  }
  for (int32_t b = 0; b < g->n_bands; ++b) {
    if (b == g->n_bands - 1) {
      g->band_gamma[b] = g->gamma;
      g->band_edge[b] = INFINITY;
      continue;
    }
    int32_t kend = (b + 1) * band_bins; /* bins [0, kend) */
    double m = 0.0;
    for (int32_t k = 0; k < kend; ++k)
      if (g->binmax[k] > m) m = g->binmax[k];
    /* a band with no collisions at all below its edge keeps the global
     * majorant (any bound >= the rate is valid; a zero one is not usable) */
    g->band_gamma[b] = m > 0.0 ? m : g->gamma;
    g->band_edge[b] = ((double)kend * e_max_eV) / (double)n_bins;
  }
  *out = g;
  return ORC_OK;
}

/* Penning transfer (reading): an excitation in channel c is followed, with
 * probability prob, by an extra electron of energy energy_eV born where the
 * excitation happened (the excitation energy ionising another molecule).
 * Excitation channels only. */
int orc_gas_set_penning(orc_gas* g, int32_t c, double prob, double energy_eV)
{
  if (!g || c < 0 || c >= g->n_ch || g->kind[c] != ORC_EXCITATION) return ORC_E_ARG;
  if (!(prob >= 0.0 && prob <= 1.0) || !(energy_eV >= 0.0) || !isfinite(energy_eV)) return ORC_E_ARG;
  g->penning_prob[c] = prob;
  g->penning_e[c] = energy_eV;
  return ORC_OK;
}

double orc_gas_gamma(const orc_gas* g) { return g->gamma; }
int32_t orc_gas_n_bands(const orc_gas* g) { return g->n_bands; }

int orc_gas_band(const orc_gas* g, int32_t b, double* gamma_b, double* edge_eV)
{
  if (b < 0 || b >= g->n_bands) return ORC_E_ARG;
  if (gamma_b) *gamma_b = g->band_gamma[b];
  if (edge_eV) *edge_eV = g->band_edge[b];
  return ORC_OK;
}

int orc_gas_set_gamma(orc_gas* g, double gamma)
{
  if (!(gamma >= g->gamma) || !isfinite(gamma)) return ORC_E_ARG;
  g->gamma = gamma;
  for (int32_t b = 0; b < g->n_bands; ++b) g->band_gamma[b] = gamma;
  return ORC_OK;
}

/* Band of energy e: the smallest b whose upper edge lies above e. */
int32_t orc_gas_band_of(const orc_gas* g, double e)
{
  int32_t lo = 0, hi = g->n_bands - 1; /* answer in [lo, hi] */
  while (lo < hi) {
    int32_t mid = lo + (hi - lo) / 2;
    if (e < g->band_edge[mid])
      hi = mid;
    else
      lo = mid + 1;
  }
  return lo;
}

/* Position in the table: x = e N / E_max, node k = floor(x), fraction
 * f = x - k.  Above the last node the rates stay at the last node's values. */
static int lookup(const orc_gas* g, double e, int32_t* k, double* f)
{
  double x = e * g->scale;
  if (!(x < (double)g->n_bins)) {
    *k = g->n_bins;
    *f = 0.0;
    return 1;
  }
  double fl = floor(x);
  *k = (int32_t)fl;
  *f = x - fl;
  return 0;
}

/* Linear interpolation written with non-negative weights, (1-f) a + f b,
 * which is monotone in a and b after rounding: interpolated cumulative rates
 * then stay ordered across channels. */
static double lerp(double a, double b, double f) { return (1.0 - f) * a + f * b; }

static double cum_at(const orc_gas* g, int32_t k, double f, int over, int c)
{
  if (over) return g->cum[(size_t)k * g->n_ch + c];
  return lerp(g->cum[(size_t)k * g->n_ch + c], g->cum[(size_t)(k + 1) * g->n_ch + c], f);
}

static double total_at(const orc_gas* g, int32_t k, double f, int over)
{
  if (over) return g->total[k];
  return lerp(g->total[k], g->total[k + 1], f);
}

int orc_gas_rates(const orc_gas* g, double e, double* nu_ch, double* nu_total)
{
  int32_t k;
  double f;
  int over = lookup(g, e, &k, &f);
  double prev = 0.0;
  for (int c = 0; c < g->n_ch; ++c) {
    double cc = cum_at(g, k, f, over, c);
    if (nu_ch) nu_ch[c] = cc - prev;
    prev = cc;
  }
  if (nu_total) *nu_total = total_at(g, k, f, over);
  return over;
}

int orc_gas_cumulative(const orc_gas* g, double* out)
{
  memcpy(out, g->cum, sizeof(double) * ((size_t)g->n_bins + 1) * (size_t)g->n_ch);
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Fields                                                                    */
/* ------------------------------------------------------------------------ */
enum { FIELD_SLAB = 0, FIELD_POLAR = 1 };

struct orc_field {
  int kind;
  double z_lo, z_hi;
  uint32_t n_E;
  double* E; /* n_E * 3 */
  double a, b;
  int32_t n_r, n_phi;
  float *Er, *Ephi;
  double B[3];
};

void orc_field_destroy(orc_field* f)
{
  if (!f) return;
  free(f->E);
  free(f->Er);
  free(f->Ephi);
  free(f);
}

static int b_valid(const double B[3]) { return isfinite(B[0]) && isfinite(B[1]) && isfinite(B[2]); }

int orc_field_slab(double z_lo, double z_hi, uint32_t n_E, const double* E_vcm,
                   const double B_T[3], orc_field** out)
{
  static const double zero[3] = {0.0, 0.0, 0.0};
  if (!B_T) B_T = zero;
  if (!out || !E_vcm || n_E < 1 || !(z_lo < z_hi) || !b_valid(B_T)) return ORC_E_ARG;
  if (B_T[0] != 0.0 || B_T[1] != 0.0) return ORC_E_ARG; /* B along z only */
  for (size_t i = 0; i < 3 * (size_t)n_E; ++i)
    if (!isfinite(E_vcm[i])) return ORC_E_ARG;
  orc_field* f = (orc_field*)calloc(1, sizeof(orc_field));
  if (!f) return ORC_E_NOMEM;
  f->kind = FIELD_SLAB;
  f->z_lo = z_lo;
  f->z_hi = z_hi;
  f->n_E = n_E;
  f->E = malloc(sizeof(double) * 3 * (size_t)n_E);
  if (!f->E) {
    free(f);
    return ORC_E_NOMEM;
  }
  memcpy(f->E, E_vcm, sizeof(double) * 3 * (size_t)n_E);
  memcpy(f->B, B_T, sizeof(f->B));
  *out = f;
  return ORC_OK;
}

int orc_field_polar(double a, double b, int32_t n_r, int32_t n_phi, const float* E_r,
                    const float* E_phi, const double B_T[3], orc_field** out)
{
  static const double zero[3] = {0.0, 0.0, 0.0};
  if (!B_T) B_T = zero;
  if (!out || !E_r || !E_phi || !(a > 0.0) || !(b > a) || !isfinite(b) || n_r < 2 || n_phi < 1 ||
      !b_valid(B_T))
    return ORC_E_ARG;
  size_t n = (size_t)n_r * (size_t)n_phi;
  for (size_t i = 0; i < n; ++i)
    if (!isfinite(E_r[i]) || !isfinite(E_phi[i])) return ORC_E_ARG;
  orc_field* f = (orc_field*)calloc(1, sizeof(orc_field));
  if (!f) return ORC_E_NOMEM;
  f->kind = FIELD_POLAR;
  f->a = a;
  f->b = b;
  f->n_r = n_r;
  f->n_phi = n_phi;
  f->Er = malloc(sizeof(float) * n);
  f->Ephi = malloc(sizeof(float) * n);
  if (!f->Er || !f->Ephi) {
    orc_field_destroy(f);
    return ORC_E_NOMEM;
  }
  memcpy(f->Er, E_r, sizeof(float) * n);
  memcpy(f->Ephi, E_phi, sizeof(float) * n);
  memcpy(f->B, B_T, sizeof(f->B));
  *out = f;
  return ORC_OK;
}

/* E at r: slab -> the avalanche's uniform vector; polar map -> bilinear in
 * (ln rho, phi), clamped in rho, periodic in phi, rotated to Cartesian. */
int orc_field_eval(const orc_field* f, const double r[3], uint32_t aval, double E[3])
{
  if (f->kind == FIELD_SLAB) {
    const double* e = f->E + 3 * (size_t)(f->n_E == 1 ? 0 : aval);
    E[0] = e[0];
    E[1] = e[1];
    E[2] = e[2];
    return ORC_OK;
  }
  double rho = sqrt(r[0] * r[0] + r[1] * r[1]);
  if (!(rho > 0.0)) {
    E[0] = E[1] = E[2] = 0.0;
    return ORC_OK;
  }
  double u = log(rho / f->a) / log(f->b / f->a) * (double)(f->n_r - 1);
  if (u < 0.0) u = 0.0;
  if (u > (double)(f->n_r - 1)) u = (double)(f->n_r - 1);
  int32_t i = (int32_t)floor(u);
  if (i > f->n_r - 2) i = f->n_r - 2;
  double fr = u - (double)i;
  double phi = atan2(r[1], r[0]);
  if (phi < 0.0) phi += TWO_PI;
  double w = phi / TWO_PI * (double)f->n_phi;
  double wf = floor(w);
  double fp = w - wf;
  int32_t j0 = ((int32_t)wf) % f->n_phi;
  int32_t j1 = (j0 + 1) % f->n_phi;
#if defined(ORC_PLANT_PHI_SWAP)
  { int32_t tmp = j0; j0 = j1; j1 = tmp; }
#elif defined(ORC_PLANT_PHI_WRAP)
  j1 = j0 + 1 < f->n_phi ? j0 + 1 : j0;
#endif
  const float* ER = f->Er;
  const float* EP = f->Ephi;
  int32_t np = f->n_phi;
  double er = (1.0 - fr) * (1.0 - fp) * (double)ER[i * np + j0] + (1.0 - fr) * fp * (double)ER[i * np + j1] +
              fr * (1.0 - fp) * (double)ER[(i + 1) * np + j0] + fr * fp * (double)ER[(i + 1) * np + j1];
  double ep = (1.0 - fr) * (1.0 - fp) * (double)EP[i * np + j0] + (1.0 - fr) * fp * (double)EP[i * np + j1] +
              fr * (1.0 - fp) * (double)EP[(i + 1) * np + j0] + fr * fp * (double)EP[(i + 1) * np + j1];
  double c = r[0] / rho, s = r[1] / rho;
#if defined(ORC_PLANT_EPHI_SIGN)
  E[0] = er * c + ep * s;
#else
  E[0] = er * c - ep * s;
#endif
  E[1] = er * s + ep * c;
  E[2] = 0.0;
  return ORC_OK;
}

/* Status of a position: 0 inside the drift volume, else the exit code. */
static int region_status(const orc_field* f, const double r[3])
{
  if (f->kind == FIELD_SLAB) {
    if (r[2] < f->z_lo) return ORC_ST_LOW;
    if (r[2] >= f->z_hi) return ORC_ST_HIGH;
    return 0;
  }
  double rho2 = r[0] * r[0] + r[1] * r[1];
  if (rho2 <= f->a * f->a) return ORC_ST_WIRE;
  if (rho2 >= f->b * f->b) return ORC_ST_TUBE;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Free flight with the field frozen at the flight start                     */
/* ------------------------------------------------------------------------ */
static double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

static void cross3(const double a[3], const double b[3], double c[3])
{
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

/* E only: r(s) = r0 + v0 s + a s^2/2, v(s) = v0 + a s with a = -k_a E.
 * With B: exact solution of dv/dt = -k_a E - k_b v x B for constant E, B.
 * Along B the motion is uniformly accelerated; across B it is the E x B drift
 * w = (k_a/k_b) (E x B)/|B|^2 plus a circle of frequency k_b |B| traversed by
 * u0 = v0_perp - w. */
void orc_propagate(const double r0[3], const double v0[3], const double E[3], const double B[3],
                   double s, double r[3], double v[3])
{
  const double k_a = orc_k_a(), k_b = orc_k_b();
  double acc[3] = {-k_a * E[0], -k_a * E[1], -k_a * E[2]};
  double bb = B ? dot3(B, B) : 0.0;
  if (bb == 0.0) {
    for (int i = 0; i < 3; ++i) {
      r[i] = r0[i] + v0[i] * s + 0.5 * acc[i] * s * s;
      v[i] = v0[i] + acc[i] * s;
    }
    return;
  }
  double bmag = sqrt(bb);
  double bh[3] = {B[0] / bmag, B[1] / bmag, B[2] / bmag};
  double omega = k_b * bmag;
  double vpar = dot3(v0, bh);
  double apar = dot3(acc, bh);
  double exb[3];
  cross3(E, B, exb);
  double wd[3];
  for (int i = 0; i < 3; ++i) wd[i] = (k_a / k_b) * exb[i] / bb;
  double u0[3];
  for (int i = 0; i < 3; ++i) u0[i] = (v0[i] - vpar * bh[i]) - wd[i];
  double bxu[3];
  cross3(bh, u0, bxu);
  double ph = omega * s;
  double cs = cos(ph), sn = sin(ph);
  double sh = sin(0.5 * ph);
  double omc = 2.0 * sh * sh; /* 1 - cos(omega s) without cancellation */
  double along = vpar * s + 0.5 * apar * s * s;
  for (int i = 0; i < 3; ++i) {
    r[i] = r0[i] + along * bh[i] + wd[i] * s + (sn / omega) * u0[i] + (omc / omega) * bxu[i];
    v[i] = (vpar + apar * s) * bh[i] + wd[i] + cs * u0[i] + sn * bxu[i];
  }
}

/* Bound of the energy along a helical flight (frozen E, B != 0), for the
 * banded majorant.  Along B the speed is |v_par + a_par s| <= vp + ap s with
 * vp = |v_par|, ap = |a_par|.  Across B the velocity is w + R(omega s) u0
 * (w the E x B drift, u0 = v_perp - w turned by the angle omega s): it moves
 * away from v_perp by |R u0 - u0| = 2 |u0| sin(omega s / 2) <= |u0| omega s,
 * and its length never exceeds |w| + |u0|.  So, with p = |v_perp|,
 * q = |u0| omega and m = |w| + |u0| (>= p),
 *   2 k_a e(s) <= (vp + ap s)^2 + min(p + q s, m)^2,
 * which is exact at s = 0 and grows with s. */
void orc_helical_bound(const double v[3], const double E[3], const double B[3], double out[5])
{
  const double k_a = orc_k_a(), k_b = orc_k_b();
  double bb = dot3(B, B);
  double bmag = sqrt(bb);
  double bh[3] = {B[0] / bmag, B[1] / bmag, B[2] / bmag};
  double acc[3] = {-k_a * E[0], -k_a * E[1], -k_a * E[2]};
  double vpar = dot3(v, bh), apar = dot3(acc, bh);
  double exb[3];
  cross3(E, B, exb);
  double wd[3], u0[3], vperp[3];
  for (int i = 0; i < 3; ++i) {
    wd[i] = (k_a / k_b) * exb[i] / bb;
    vperp[i] = v[i] - vpar * bh[i];
    u0[i] = vperp[i] - wd[i];
  }
  double un = sqrt(dot3(u0, u0));
  out[0] = fabs(vpar);
  out[1] = fabs(apar);
  out[2] = sqrt(dot3(vperp, vperp));
  out[3] = un * (k_b * bmag);
  out[4] = sqrt(dot3(wd, wd)) + un;
}

/* Smallest s >= 0 at which the helical energy bound (b = the five numbers
 * above) reaches e_edge: 0 if it is there already, +inf if never. */
double orc_helical_bound_root(const double b[5], double e_edge)
{
  const double vp = b[0], ap = b[1], p = b[2], q = b[3], m = b[4];
  const double T = 2.0 * orc_k_a() * e_edge;
  const double c = T - (vp * vp + p * p);
  if (!(c > 0.0)) return 0.0;
  /* unsaturated branch: (ap^2 + q^2) s^2 + 2 (vp ap + p q) s - c = 0 */
  const double A = ap * ap + q * q, Bq = 2.0 * (vp * ap + p * q);
  if (A == 0.0 && Bq == 0.0) return INFINITY;
  const double s1 = 2.0 * c / (Bq + sqrt(Bq * Bq + 4.0 * A * c));
  if (q == 0.0 || p + q * s1 <= m) return s1;
  /* saturated: (vp + ap s)^2 + m^2 = T, reached after p + q s = m */
  if (ap == 0.0 || !(T > m * m)) return INFINITY;
  return (sqrt(T - m * m) - vp) / ap;
}

/* Real roots of A s^2 + B s + C = 0, ascending; the numerically stable form
 * q = -(B + sgn(B) sqrt(disc))/2, roots q/A and C/q. */
static int quad_roots(double A, double B, double C, double out[2])
{
  if (A == 0.0) {
    if (B == 0.0) return 0;
    out[0] = -C / B;
    return 1;
  }
  double disc = B * B - 4.0 * A * C;
  if (disc < 0.0) return 0;
  double sq = sqrt(disc);
  double q = -0.5 * (B + (B >= 0.0 ? sq : -sq));
  double r1, r2;
  if (q == 0.0) {
    r1 = 0.0;
    r2 = 0.0;
  } else {
    r1 = q / A;
    r2 = C / q;
  }
  if (r1 > r2) {
    double t = r1;
    r1 = r2;
    r2 = t;
  }
  out[0] = r1;
  out[1] = r2;
  return 2;
}

/* First time in (0, T] at which z(s) = z0 + vz s + az s^2/2, starting inside
 * [z_lo, z_hi), reaches z_hi, or drops below z_lo (a crossing with dz/ds < 0;
 * s = 0 counts when the electron sits on z_lo moving down). */
int orc_slab_exit(double z0, double vz, double az, double z_lo, double z_hi, double T,
                  double* s_exit)
{
  double best = INFINITY;
  int side = 0;
  double rt[2];
  int n = quad_roots(0.5 * az, vz, z0 - z_hi, rt);
  for (int i = 0; i < n; ++i)
    if (rt[i] > 0.0 && rt[i] < best) {
      best = rt[i];
      side = ORC_ST_HIGH;
      break; /* ascending: the first positive root is the first arrival */
    }
  n = quad_roots(0.5 * az, vz, z0 - z_lo, rt);
  for (int i = 0; i < n; ++i) {
    double s = rt[i];
    if (s < 0.0) continue;
    double slope = az * s + vz;
    if (slope < 0.0 || (s == 0.0 && slope == 0.0 && az < 0.0)) {
      if (s < best) {
        best = s;
        side = ORC_ST_LOW;
      }
      break;
    }
  }
  if (side && best <= T) {
    *s_exit = best;
    return side;
  }
  return 0;
}

/* Smallest s >= 0 at which the energy of v + a s reaches e_edge. */
double orc_band_root(const double v[3], const double a[3], double e_edge)
{
  const double k_a = orc_k_a();
  double C = dot3(v, v) - 2.0 * k_a * e_edge;
  if (C >= 0.0) return 0.0;
  double rt[2];
  int n = quad_roots(dot3(a, a), 2.0 * dot3(v, a), C, rt);
  for (int i = 0; i < n; ++i)
    if (rt[i] >= 0.0) return rt[i];
  return -1.0;
}

/* ------------------------------------------------------------------------ */
/* Scattering                                                                */
/* ------------------------------------------------------------------------ */

/* Screened Rutherford, dsigma/dOmega ~ (1 - cos chi + 2 eta)^-2 with
 * eta = screening / (8 e): inverse CDF 1 - cos chi = 2 u / (1 + (1 - u)/eta),
 * written with 1/eta = 8 e / screening so that e = 0 gives the isotropic
 * limit 1 - 2u. */
double orc_cos_screened_rutherford(double u, double e, double screening)
{
  double inv_eta = 8.0 * e / screening;
  return 1.0 - 2.0 * u / (1.0 + (1.0 - u) * inv_eta);
}

/* Energy of the secondary electron out of e_avail = e - I. */
double orc_split_energy(int32_t split, double u, double e_avail, double w)
{
  if (split == ORC_SPLIT_OPAL_BEATY) /* dsigma/de_s ~ 1/(1+(e_s/w)^2) on [0, e_avail/2] */
    return w * tan(u * atan(e_avail / (2.0 * w)));
  return u * e_avail;
}

/* Direction cosines of d turned by polar angle theta and azimuth phi.  The
 * transverse length s = sin(angle of d to z) is taken as sqrt(dx^2 + dy^2)
 * rather than sqrt(1 - dz^2): equal for a unit vector, but without the
 * cancellation near the poles that would make |d'| != 1 (and change the
 * electron's energy when the speed is re-applied). */
void orc_rotate(const double d[3], double cos_t, double phi, double out[3])
{
  double st2 = 1.0 - cos_t * cos_t;
  double sin_t = st2 > 0.0 ? sqrt(st2) : 0.0;
  double cp = cos(phi), sp = sin(phi);
  double s = sqrt(d[0] * d[0] + d[1] * d[1]);
  if (s > 1e-12) {
    out[0] = d[0] * cos_t + sin_t * (d[0] * d[2] * cp - d[1] * sp) / s;
    out[1] = d[1] * cos_t + sin_t * (d[1] * d[2] * cp + d[0] * sp) / s;
    out[2] = d[2] * cos_t - s * sin_t * cp;
  } else {
    out[0] = sin_t * cp;
    out[1] = sin_t * sp;
    out[2] = (d[2] < 0.0 ? -1.0 : 1.0) * cos_t;
  }
}

/* Elastic collision with an atom at rest (m/M = mass_ratio): centre-of-mass
 * angle chi -> energy after the collision and laboratory deflection. */
void orc_elastic(double e, double mu, double cos_chi, double* e_out, double* cos_lab)
{
  double loss = 2.0 * mu * (1.0 - cos_chi) / ((1.0 + mu) * (1.0 + mu));
  *e_out = e * (1.0 - loss);
  *cos_lab = (mu + cos_chi) / sqrt(1.0 + mu * mu + 2.0 * mu * cos_chi);
}

/* ------------------------------------------------------------------------ */
/* Transport                                                                 */
/* ------------------------------------------------------------------------ */
typedef struct {
  double r[3], v[3], t;
  double r0[3], t0, e0;
  uint64_t eid, parent;
  uint32_t aval;
} elec;

typedef struct {
  elec* a;
  size_t n, cap, head;
} estack;

static int estack_push(estack* s, const elec* e)
{
  if (s->n == s->cap) {
    size_t nc = s->cap ? 2 * s->cap : 64;
    elec* na = realloc(s->a, nc * sizeof(elec));
    if (!na) return ORC_E_NOMEM;
    s->a = na;
    s->cap = nc;
  }
  s->a[s->n++] = *e;
  return ORC_OK;
}

typedef struct {
  orc_endpoint* a;
  size_t n, cap;
} evec;

static int evec_push(evec* v, const orc_endpoint* e)
{
  if (v->n == v->cap) {
    size_t nc = v->cap ? 2 * v->cap : 64;
    orc_endpoint* na = realloc(v->a, nc * sizeof(orc_endpoint));
    if (!na) return ORC_E_NOMEM;
    v->a = na;
    v->cap = nc;
  }
  v->a[v->n++] = *e;
  return ORC_OK;
}

typedef struct {
  const orc_gas* g;
  const orc_field* f;
  const orc_opts* o;
  const orc_signal* sig; /* NULL: no induced signal */
} ctx_t;

/* ---- induced signal (Shockley-Ramo, readout electrode as in the header) -- */
double orc_weighting(const orc_field* f, const double r[3])
{
  if (f->kind == FIELD_SLAB) return (r[2] - f->z_lo) / (f->z_hi - f->z_lo);
  return log(f->b / sqrt(r[0] * r[0] + r[1] * r[1])) / log(f->b / f->a);
}

static double edge_time(const orc_signal* s, int64_t j) { return s->t0_ns + (double)j * s->dt_ns; }

/* Index of the first bin edge strictly after t; edges beyond T_n_bins are
 * irrelevant, so the answer is capped at n_bins + 1. */
static int64_t first_edge_after(const orc_signal* s, double t)
{
  if (t < edge_time(s, 0)) return 0;
  if (!(t < edge_time(s, s->n_bins))) return (int64_t)s->n_bins + 1;
  int64_t j = (int64_t)floor((t - s->t0_ns) / s->dt_ns) + 1;
  if (j < 1) j = 1;
  if (j > s->n_bins) j = s->n_bins;
  while (!(edge_time(s, j) > t)) j++;
  while (j > 0 && edge_time(s, j - 1) > t) j--;
  return j;
}

static void deposit(const orc_signal* s, uint32_t aval, int64_t bin, double dq)
{
  if (bin >= 0 && bin < s->n_bins) s->out[(size_t)aval * (size_t)s->n_bins + (size_t)bin] += dq;
}

/* The flight from (r_s, v_s) at time t_s, in the frozen field E, ends at
 * r_e at time t_e: it is cut at every bin edge T in (t_s, t_e], the
 * position at T coming from the flight formula, and each piece adds the
 * change of the weighting potential over it to its bin. */
static void signal_flight(const ctx_t* cx, uint32_t aval, const double r_s[3], const double v_s[3],
                          const double E[3], double t_s, double t_e, const double r_e[3])
{
  const orc_signal* s = cx->sig;
  if (!s) return;
  double phi_a = orc_weighting(cx->f, r_s);
  int64_t j = first_edge_after(s, t_s);
  while (j <= s->n_bins && edge_time(s, j) <= t_e) {
    double T = edge_time(s, j);
    double rr[3], vv[3];
    orc_propagate(r_s, v_s, E, cx->f->B, T - t_s, rr, vv);
    double phi_b = orc_weighting(cx->f, rr);
    deposit(s, aval, j - 1, phi_b - phi_a);
    phi_a = phi_b;
    j++;
  }
  deposit(s, aval, j - 1, orc_weighting(cx->f, r_e) - phi_a);
}

static double energy_of(const double v[3]) { return dot3(v, v) / (2.0 * orc_k_a()); }

/* One event of the decision trace (see orc_endpoint): rotate left by 5,
 * then mix in the flight index and the event code. */
static uint32_t trace_step(uint32_t h, uint32_t k, uint32_t code)
{
  return ((h << 5) | (h >> 27)) ^ ((k << 18) + code);
}
enum { TRACE_MASKED = 1u << 16, TRACE_BAND = 1u << 17 };

/* Decisions that saw an interpolated total rate above the majorant in use
 * (a majorant that is not one; counted for the pins, never expected). */
static uint64_t g_majorant_violations = 0;
uint64_t orc_majorant_violations(void) { return __atomic_load_n(&g_majorant_violations, __ATOMIC_RELAXED); }
void orc_reset_majorant_violations(void) { __atomic_store_n(&g_majorant_violations, 0, __ATOMIC_RELAXED); }

/* Set v to speed sqrt(2 k_a e) along unit vector d. */
static void set_velocity(double v[3], double e, const double d[3])
{
  double sp = sqrt(2.0 * orc_k_a() * e);
  v[0] = sp * d[0];
  v[1] = sp * d[1];
  v[2] = sp * d[2];
}

static void direction_of(const double v[3], double d[3])
{
  double s = sqrt(dot3(v, v));
  if (s == 0.0) {
    d[0] = 0.0;
    d[1] = 0.0;
    d[2] = 1.0;
  } else {
    d[0] = v[0] / s;
    d[1] = v[1] / s;
    d[2] = v[2] / s;
  }
}

/* Push a secondary electron of energy e_s born at the parent's position and
 * time, direction isotropic from (uC, uP), id `child`. */
static int push_secondary(estack* st, const elec* parent, double e_s, double uC, double uP, uint64_t child)
{
  double ct = 1.0 - 2.0 * uC;
  double st2 = 1.0 - ct * ct;
  double stt = st2 > 0.0 ? sqrt(st2) : 0.0;
  double ph2 = TWO_PI * uP;
  double ds[3] = {stt * cos(ph2), stt * sin(ph2), ct};
  elec s;
  s.r[0] = parent->r[0]; s.r[1] = parent->r[1]; s.r[2] = parent->r[2];
  set_velocity(s.v, e_s, ds);
  s.t = parent->t;
  s.r0[0] = parent->r[0]; s.r0[1] = parent->r[1]; s.r0[2] = parent->r[2];
  s.t0 = parent->t;
  s.e0 = e_s;
  s.eid = child;
  s.parent = parent->eid;
  s.aval = parent->aval;
  return estack_push(st, &s);
}

/* Carry one electron through the loop of Fig. 2 until it terminates.  Each
 * pass checks the position, takes the field at r and a random flight time,
 * looks for a boundary, the time limit or a band edge within the flight,
 * decides between a real and a null collision and scatters; an ionisation
 * pushes the secondary onto `st`. */
static int transport(const ctx_t* cx, elec e, estack* st, orc_endpoint* ep)
{
  const orc_gas* g = cx->g;
  const orc_field* f = cx->f;
  const orc_opts* o = cx->o;
  const double k_a = orc_k_a();
  const int banded = o->banded && g->n_bands > 1;
  const int helical = banded && dot3(f->B, f->B) != 0.0;
  memset(ep, 0, sizeof(*ep));
  ep->x0 = e.r0[0];
  ep->y0 = e.r0[1];
  ep->z0 = e.r0[2];
  ep->t0 = e.t0;
  ep->e0 = e.e0;
  ep->eid = e.eid;
  ep->parent = e.parent;
  ep->aval = e.aval;
  uint32_t k = 0;
  int32_t band = banded ? orc_gas_band_of(g, energy_of(e.v)) : g->n_bands - 1;
  int status = 0;
  for (;;) {
    /* still inside the volume? */
    status = region_status(f, e.r);
    if (status) break;
    if (k >= o->k_max) {
      status = ORC_ST_ABANDONED;
      break;
    }
    if (e.t >= o->t_max_ns) {
      status = ORC_ST_TIME;
      break;
    }
    uint32_t w[4];
    draw(o->seed, e.aval, e.eid, k, 0, w);
    double u1 = orc_u53(w[0], w[1]);
    double u2 = orc_u53(w[2], w[3]);
    double E[3];
    orc_field_eval(f, e.r, e.aval, E);
    /* with B the band must bound the energy over the whole flight: raise it
     * until the helical bound at the flight start lies below its edge */
    double hb[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (helical) orc_helical_bound(e.v, E, f->B, hb);
    if (banded && o->band_lookahead > 0.0 && band < g->n_bands - 1) {
      /* lookahead: the band of the energy after band_lookahead mean free
       * times of the current band (the flight energy, or its helical bound) */
      double s_look = o->band_lookahead / g->band_gamma[band];
      double e_look;
      if (helical) {
        double vpar = hb[0] + hb[1] * s_look;
        double vperp = hb[2] + hb[3] * s_look < hb[4] ? hb[2] + hb[3] * s_look : hb[4];
        e_look = (vpar * vpar + vperp * vperp) / (2.0 * k_a);
      } else {
        double rr[3], vv[3];
        orc_propagate(e.r, e.v, E, f->B, s_look, rr, vv);
        e_look = energy_of(vv);
      }
      int32_t bl = orc_gas_band_of(g, e_look);
      if (bl > band) band = bl;
    }
    if (helical)
      while (band < g->n_bands - 1 && (hb[0] * hb[0] + hb[2] * hb[2]) / (2.0 * k_a) >= g->band_edge[band])
        band++;
    double gam = banded ? g->band_gamma[band] : g->gamma;
    double tau = -log(u1) / gam;
    /* the flight ends at the earliest of: the collision candidate, the band
     * edge (banded majorant), the time limit */
    double tau_end = tau;
    int cut = 0; /* 1 band edge, 2 time limit */
    if (helical && band < g->n_bands - 1) {
      /* cut where the energy bound reaches the edge: Gamma_b holds before */
      double tc = orc_helical_bound_root(hb, g->band_edge[band]);
      if (tc < tau_end) {
        tau_end = tc;
        cut = 1;
      }
    } else if (banded && band < g->n_bands - 1) {
      double rr[3], vv[3];
      orc_propagate(e.r, e.v, E, f->B, tau, rr, vv);
      if (energy_of(vv) >= g->band_edge[band]) {
        double acc[3] = {-k_a * E[0], -k_a * E[1], -k_a * E[2]};
        double tc = orc_band_root(e.v, acc, g->band_edge[band]);
        if (tc < 0.0) tc = 0.0;
        if (tc < tau_end) {
          tau_end = tc;
          cut = 1;
        }
      }
    }
    double t_left = o->t_max_ns - e.t;
    if (t_left < tau_end) {
      tau_end = t_left;
      cut = 2;
    }
    /* boundary first passage within (0, tau_end] */
    double rn[3], vn[3];
    double s_exit = 0.0;
    int side = 0;
    if (f->kind == FIELD_SLAB) {
      double acc_z = -k_a * E[2];
      side = orc_slab_exit(e.r[2], e.v[2], acc_z, f->z_lo, f->z_hi, tau_end, &s_exit);
      if (side) {
        orc_propagate(e.r, e.v, E, f->B, s_exit, rn, vn);
        rn[2] = side == ORC_ST_HIGH ? f->z_hi : f->z_lo;
      }
    } else {
      orc_propagate(e.r, e.v, E, f->B, tau_end, rn, vn);
      if (region_status(f, rn)) {
        /* bisection on the inside/outside predicate; excursions that leave
         * and re-enter within one flight are not detected */
        double lo = 0.0, hi = tau_end;
        for (int it = 0; it < 60; ++it) {
          double mid = 0.5 * (lo + hi);
          double rm[3], vm[3];
          orc_propagate(e.r, e.v, E, f->B, mid, rm, vm);
          if (region_status(f, rm))
            hi = mid;
          else
            lo = mid;
        }
        s_exit = hi;
        orc_propagate(e.r, e.v, E, f->B, s_exit, rn, vn);
        side = region_status(f, rn);
        if (!side) side = ORC_ST_TUBE; /* unreachable: hi stays outside */
        double rho = sqrt(rn[0] * rn[0] + rn[1] * rn[1]);
        double target = side == ORC_ST_WIRE ? f->a : f->b;
        rn[0] = rn[0] * (target / rho);
        rn[1] = rn[1] * (target / rho);
      }
    }
    if (side) {
      signal_flight(cx, e.aval, e.r, e.v, E, e.t, e.t + s_exit, rn);
      e.r[0] = rn[0]; e.r[1] = rn[1]; e.r[2] = rn[2];
      e.v[0] = vn[0]; e.v[1] = vn[1]; e.v[2] = vn[2];
      e.t = e.t + s_exit;
      status = side;
      break;
    }
    orc_propagate(e.r, e.v, E, f->B, tau_end, rn, vn);
    signal_flight(cx, e.aval, e.r, e.v, E, e.t, e.t + tau_end, rn);
    e.r[0] = rn[0]; e.r[1] = rn[1]; e.r[2] = rn[2];
    e.v[0] = vn[0]; e.v[1] = vn[1]; e.v[2] = vn[2];
    e.t = e.t + tau_end;
    if (cut == 2) {
      status = ORC_ST_TIME;
      break;
    }
    if (cut == 1) {
      /* restart the flight at the band edge with the next band's majorant;
       * the band index is advanced explicitly, never re-derived from the
       * rounded energy at the edge */
      band = band + 1;
      ep->n_band++;
      ep->trace = trace_step(ep->trace, k, TRACE_BAND);
      k++;
      continue;
    }
    /* collision? */
    double en = energy_of(e.v);
    if (!isfinite(en)) {
      status = ORC_ST_ERROR;
      break;
    }
    int32_t kb;
    double fb;
    int over = lookup(g, en, &kb, &fb);
    if (over) ep->n_overflow++;
    double nu_tot = total_at(g, kb, fb, over);
    if (nu_tot > gam) __atomic_fetch_add(&g_majorant_violations, 1, __ATOMIC_RELAXED);
    double r_sel = u2 * gam;
    if (r_sel >= nu_tot) {
      ep->n_null++;
      k++;
      if (banded) band = orc_gas_band_of(g, en);
      continue;
    }
    int c = 0;
    while (c < g->n_ch - 1 && !(r_sel < cum_at(g, kb, fb, over, c))) c++;
    if (en < g->e_lo[c] || en >= g->e_hi[c]) {
      ep->n_masked++;
      ep->trace = trace_step(ep->trace, k, TRACE_MASKED + (uint32_t)c);
      k++;
      if (banded) band = orc_gas_band_of(g, en);
      continue;
    }
    ep->n_real++;
    ep->trace = trace_step(ep->trace, k, (uint32_t)c);
    if (g->kind[c] == ORC_ATTACHMENT) {
      status = ORC_ST_ATTACHED;
      break;
    }
    double d[3], dn[3];
    direction_of(e.v, d);
    draw(o->seed, e.aval, e.eid, k, 1, w);
    double uA = orc_u53(w[0], w[1]);
    double uB = orc_u53(w[2], w[3]);
    double phi = TWO_PI * uB;
    double e_new;
    if (g->kind[c] == ORC_ELASTIC) {
#if defined(ORC_PLANT_SR_ISOTROPIC)
      double cos_chi = 1.0 - 2.0 * uA;
#else
      double cos_chi = g->angular[c] == ORC_SCREENED_RUTHERFORD
                           ? orc_cos_screened_rutherford(uA, en, g->screening[c])
                           : 1.0 - 2.0 * uA;
#endif
      double cos_lab;
      orc_elastic(en, g->mass_ratio[c], cos_chi, &e_new, &cos_lab);
      orc_rotate(d, cos_lab, phi, dn);
    } else if (g->kind[c] == ORC_EXCITATION) {
      e_new = en - g->loss[c];
      orc_rotate(d, 1.0 - 2.0 * uA, phi, dn);
      if (g->penning_prob[c] > 0.0) {
        /* Penning transfer: blocks j = 2, 3 as for an ionisation */
        uint32_t w2[4], w3[4];
        draw(o->seed, e.aval, e.eid, k, 2, w2);
        if (orc_u53(w2[0], w2[1]) < g->penning_prob[c]) {
          draw(o->seed, e.aval, e.eid, k, 3, w3);
          uint64_t child = (((uint64_t)w3[3] << 32) | (uint64_t)w3[2]) & 0x7FFFFFFFFFFFFFFFull;
          if (push_secondary(st, &e, g->penning_e[c], orc_u53(w2[2], w2[3]), orc_u53(w3[0], w3[1]), child) != ORC_OK)
            return ORC_E_NOMEM;
          ep->n_ion++;
        }
      }
    } else { /* ionisation */
      double e_avail = en - g->loss[c];
      uint32_t w2[4], w3[4];
      draw(o->seed, e.aval, e.eid, k, 2, w2);
      draw(o->seed, e.aval, e.eid, k, 3, w3);
      double uS = orc_u53(w2[0], w2[1]);
      double uC = orc_u53(w2[2], w2[3]);
      double uP = orc_u53(w3[0], w3[1]);
      uint64_t child = (((uint64_t)w3[3] << 32) | (uint64_t)w3[2]) & 0x7FFFFFFFFFFFFFFFull;
#if defined(ORC_PLANT_OB_AVAIL)
      double e_s = orc_split_energy(g->split[c], uS, en, g->split_w[c]);
#else
      double e_s = orc_split_energy(g->split[c], uS, e_avail, g->split_w[c]);
#endif
#if defined(ORC_PLANT_ION_KEEP)
      e_new = e_avail;
#else
      e_new = e_avail - e_s;
#endif
      orc_rotate(d, 1.0 - 2.0 * uA, phi, dn);
      /* the secondary starts where the ionisation happened, isotropically */
      if (push_secondary(st, &e, e_s, uC, uP, child) != ORC_OK) return ORC_E_NOMEM;
      ep->n_ion++;
    }
    set_velocity(e.v, e_new, dn);
    k++;
    if (banded) band = orc_gas_band_of(g, e_new);
  }
  ep->x1 = e.r[0];
  ep->y1 = e.r[1];
  ep->z1 = e.r[2];
  ep->t1 = e.t;
  ep->e1 = energy_of(e.v);
  ep->status = (uint32_t)status;
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Runs: avalanches spread over threads                                      */
/* ------------------------------------------------------------------------ */
struct orc_result {
  uint64_t n;
  orc_endpoint* a;
};

typedef struct {
  const ctx_t* cx;
  const orc_primary* prim;
  const uint64_t* ids;
  const uint64_t* order;     /* primary indices grouped by avalanche */
  const uint64_t* group_off; /* n_groups+1 offsets into order */
  uint64_t n_groups;
  evec* out;                 /* one per group */
  uint64_t next;             /* shared work counter */
  int err;
} pool_t;

static void primary_to_elec(const orc_primary* p, uint64_t id, elec* e)
{
  memset(e, 0, sizeof(*e));
  e->r[0] = p->x; e->r[1] = p->y; e->r[2] = p->z;
  e->t = p->t;
  double d[3] = {p->dx, p->dy, p->dz};
  double n = sqrt(dot3(d, d));
  if (n > 0.0) {
    d[0] = d[0] / n; d[1] = d[1] / n; d[2] = d[2] / n;
  } else {
    d[0] = 0.0; d[1] = 0.0; d[2] = 1.0;
  }
  set_velocity(e->v, p->e, d);
  e->r0[0] = p->x; e->r0[1] = p->y; e->r0[2] = p->z;
  e->t0 = p->t;
  e->e0 = p->e;
  e->eid = 0x8000000000000000ull | id;
  e->parent = 0;
  e->aval = p->aval;
}

static void* worker(void* arg)
{
  pool_t* P = (pool_t*)arg;
  estack st = {0};
  for (;;) {
    uint64_t gidx = __atomic_fetch_add(&P->next, 1, __ATOMIC_RELAXED);
    if (gidx >= P->n_groups) break;
    if (__atomic_load_n(&P->err, __ATOMIC_RELAXED)) break;
    st.n = 0;
    st.head = 0;
    for (uint64_t q = P->group_off[gidx]; q < P->group_off[gidx + 1]; ++q) {
      uint64_t i = P->order[q];
      elec e;
      primary_to_elec(&P->prim[i], P->ids ? P->ids[i] : i, &e);
      if (estack_push(&st, &e) != ORC_OK) {
        __atomic_store_n(&P->err, ORC_E_NOMEM, __ATOMIC_RELAXED);
        break;
      }
    }
    while (st.n > st.head) {
      elec e;
      if (P->cx->o->fifo)
        e = st.a[st.head++];
      else
        e = st.a[--st.n];
      orc_endpoint ep;
      if (transport(P->cx, e, &st, &ep) != ORC_OK || evec_push(&P->out[gidx], &ep) != ORC_OK) {
        __atomic_store_n(&P->err, ORC_E_NOMEM, __ATOMIC_RELAXED);
        break;
      }
      if (P->cx->o->fifo && st.head == st.n) {
        st.head = 0;
        st.n = 0;
      }
    }
  }
  free(st.a);
  return NULL;
}

static int cmp_u64_by_aval(const void* a, const void* b, void* arg)
{
  const orc_primary* p = (const orc_primary*)arg;
  uint64_t ia = *(const uint64_t*)a, ib = *(const uint64_t*)b;
  if (p[ia].aval != p[ib].aval) return p[ia].aval < p[ib].aval ? -1 : 1;
  return ia < ib ? -1 : (ia > ib ? 1 : 0);
}

int orc_run(const orc_gas* g, const orc_field* f, const orc_primary* prim, const uint64_t* ids,
            uint64_t n_prim, const orc_opts* o, orc_result** out, int32_t* threads_used)
{
  return orc_run_signal(g, f, prim, ids, n_prim, o, NULL, out, threads_used);
}

int orc_run_signal(const orc_gas* g, const orc_field* f, const orc_primary* prim, const uint64_t* ids,
                   uint64_t n_prim, const orc_opts* o, const orc_signal* sig, orc_result** out,
                   int32_t* threads_used)
{
  if (!g || !f || !o || !out || (!prim && n_prim)) return ORC_E_ARG;
  if (sig) {
    if (sig->n_bins < 1 || !(sig->dt_ns > 0.0) || !isfinite(sig->dt_ns) || !isfinite(sig->t0_ns) || !sig->out)
      return ORC_E_ARG;
    for (uint64_t i = 0; i < n_prim; ++i)
      if (prim[i].aval >= sig->n_rows) return ORC_E_ARG;
  }
  if (o->k_max > (1u << 30) - 1u) return ORC_E_ARG;
  if (!(o->band_lookahead >= 0.0) || !isfinite(o->band_lookahead)) return ORC_E_ARG;
  if (f->kind == FIELD_SLAB && f->n_E > 1)
    for (uint64_t i = 0; i < n_prim; ++i)
      if (prim[i].aval >= f->n_E) return ORC_E_ARG;
  ctx_t cx = {g, f, o, sig};
  uint64_t* order = malloc(sizeof(uint64_t) * (n_prim ? n_prim : 1));
  uint64_t* goff = malloc(sizeof(uint64_t) * (n_prim + 1));
  if (!order || !goff) {
    free(order);
    free(goff);
    return ORC_E_NOMEM;
  }
  for (uint64_t i = 0; i < n_prim; ++i) order[i] = i;
  qsort_r(order, n_prim, sizeof(uint64_t), cmp_u64_by_aval, (void*)prim);
  uint64_t ng = 0;
  for (uint64_t q = 0; q < n_prim; ++q)
    if (q == 0 || prim[order[q]].aval != prim[order[q - 1]].aval) goff[ng++] = q;
  goff[ng] = n_prim;
  evec* outs = calloc(ng ? ng : 1, sizeof(evec));
  if (!outs) {
    free(order);
    free(goff);
    return ORC_E_NOMEM;
  }
  pool_t P = {&cx, prim, ids, order, goff, ng, outs, 0, 0};
  int nt = o->n_threads > 0 ? o->n_threads : (int)sysconf(_SC_NPROCESSORS_ONLN);
  if (nt < 1) nt = 1;
  if ((uint64_t)nt > ng) nt = ng ? (int)ng : 1;
  pthread_t* th = malloc(sizeof(pthread_t) * nt);
  int started = 0;
  if (th)
    for (int i = 0; i < nt; ++i)
      if (pthread_create(&th[i], NULL, worker, &P) == 0) started++;
  if (started == 0) worker(&P);
  for (int i = 0; i < started; ++i) pthread_join(th[i], NULL);
  free(th);
  if (threads_used) *threads_used = started ? started : 1;
  int rc = P.err;
  orc_result* R = NULL;
  if (!rc) {
    R = calloc(1, sizeof(orc_result));
    uint64_t total = 0;
    for (uint64_t i = 0; i < ng; ++i) total += outs[i].n;
    if (R) R->a = malloc(sizeof(orc_endpoint) * (total ? total : 1));
    if (!R || !R->a) {
      rc = ORC_E_NOMEM;
    } else {
      uint64_t p = 0;
      for (uint64_t i = 0; i < ng; ++i) {
        memcpy(R->a + p, outs[i].a, sizeof(orc_endpoint) * outs[i].n);
        p += outs[i].n;
      }
      R->n = total;
    }
  }
  for (uint64_t i = 0; i < ng; ++i) free(outs[i].a);
  free(outs);
  free(order);
  free(goff);
  if (rc) {
    if (R) free(R->a);
    free(R);
    return rc;
  }
  *out = R;
  return ORC_OK;
}

uint64_t orc_result_count(const orc_result* r) { return r ? r->n : 0; }

int orc_result_copy(const orc_result* r, orc_endpoint* out)
{
  if (!r || !out) return ORC_E_ARG;
  memcpy(out, r->a, sizeof(orc_endpoint) * r->n);
  return ORC_OK;
}

void orc_result_destroy(orc_result* r)
{
  if (!r) return;
  free(r->a);
  free(r);
}
