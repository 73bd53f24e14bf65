// avm_device.hpp -- device side of microscopic electron-avalanche transport
// for gfx950 (CDNA4, wave64).
//
// One call of `flight_step` is one pass of the AvalancheMicroscopic loop of
// the paper's Fig. 2 for one electron held in registers: check that it is
// still inside the volume, take the local field and a random flight time,
// decide whether a real collision ends the flight, and, for a real one,
// which channel (an ionisation or an attachment changes the electron
// count).  The free flight is a null-collision flight (Skullerud, cited in
// Sec. 1): exponential with the majorant rate, real with probability
// nu(e)/majorant.  Both the plain (generation-synchronous) and the batched
// (persistent) kernels call this same function, so for a given electron they
// produce the same bits.
//
// Everything random is drawn from Philox4x32-10 (Salmon et al., SC'11) with
// key (seed_lo, seed_hi) and counter (4k + j, avalanche, eid_lo, eid_hi),
// k = flight index of the electron, j = block within the event (0 flight,
// 1 scattering, 2-3 ionisation): results do not depend on which lane, wave
// or kernel carries an electron.
//
// Precision is a template parameter R of the step:
//   R = double: FP64 throughout (53-bit uniforms);
//   R = float : FP32-mixed -- velocities, flight times, energies, table
//               interpolation and scattering in FP32 (24-bit uniforms from the
//               high word of the same Philox output, so an FP32 run and an
//               FP64 run see common random numbers); position and time are
//               accumulated in FP64; boundary crossings are solved in FP64;
//               a collision decision whose FP32 margin is below 2^-18 is
//               taken again in FP64.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

// Device functions.  AVM_HOST_DEBUG (never set by the library build) makes
// them callable from host code too, for CPU debugging builds of the kernels'
// arithmetic.
#ifdef AVM_HOST_DEBUG
#define AVM_FN __host__ __device__ inline
#else
#define AVM_FN __device__ __forceinline__
#endif

// Channel search: 2 (binary) or 4 (four-way steps, then binary).
#ifndef AVM_SEARCH_WAYS
#define AVM_SEARCH_WAYS 2
#endif

namespace avm {

// electron status codes (non-zero: terminated)
enum : uint32_t {
  ST_ACTIVE = 0, ST_LOW = 1, ST_HIGH = 2, ST_ATTACHED = 3, ST_WIRE = 4,
  ST_TUBE = 5, ST_TIME = 6, ST_ABANDONED = 7, ST_ERROR = 8
};
enum : int32_t { CH_ELASTIC = 0, CH_EXCITATION = 1, CH_IONISATION = 2, CH_ATTACHMENT = 3 };

// Per-channel scattering parameters, in the step's precision R.
template <class R>
struct ChanP {
  int32_t kind, angular, split, _pad;
  double e_lo, e_hi;    // validity window (compared in FP64)
  R loss;
  R mu;                 // m/M
  R el_loss;            // 2 mu / (1 + mu)^2
  R mu2p1;              // 1 + mu^2
  R two_mu;             // 2 mu
  R split_w;            // Opal-Beaty w
  R atan_scale;         // 1 / (2 w)
  R inv_screen8;        // 8 / screening (1/eta = 8 e / screening)
  R pen_prob;           // excitation: Penning transfer probability
  R pen_e;              // excitation: energy of the transfer electron
};
using ChanDev = ChanP<double>;

// Rate tables of one gas on the device.  FP64 tables serve the FP64 path and
// the FP64 re-evaluation of close FP32 decisions; FP32 copies serve the
// FP32-mixed path (majorants rounded up, band edges rounded down, so the
// FP32 bounds stay bounds).
struct GasDev {
  const double* cum;        // [(n_bins+1) * n_ch] node-major cumulative rates, 1/ns
  const double* cum0;       // [n_bins+1] cumulative column 0 (the first channel's rate)
  const double* total;      // [n_bins+1] total rate at the nodes
  const double* band_gamma; // [n_bands]
  const double* band_inv;   // [n_bands] 1 / Gamma_b
  const double* band_edge;  // [n_bands] upper edge (eV), +inf for the last
  const ChanDev* ch;        // [n_ch]
  const float* cum_f;       // FP32 copies of the above
  const float* cum0_f;
  const float* total_f;
  const float* band_gamma_f;
  const float* band_inv_f;
  const float* band_edge_f;
  const ChanP<float>* ch_f;
  const double* sct;        // [kAzN][2] sin and cos of 2 pi j / kAzN (azimuth table, FP64)
  double scale;             // n_bins / E_max
  double gamma, inv_gamma;
  double band_scale;        // n_bins / (E_max * band_bins): first guess of the band
  float gamma_f, inv_gamma_f, scale_f, band_scale_f;
  int32_t n_bins, n_ch, n_bands, band_bins;
  double x_top;             // n_bins as a double (the table's end in bin units)
  float x_top_f;            // n_bins as a float
};

// Where the hot tables are read from.  TabView: the global arrays (`tot`
// and `cum0` hold nodes [0, n_lo) of the total rate and of cumulative
// column 0).  TabLds: the persistent kernel's LDS copies -- the first n_lo
// nodes of those two, the first kLdsBands bands and the first kLdsChannels
// channels -- with reads of higher band or channel indices going to the
// global arrays.  Both sources hold the same values, so results do not
// depend on the view.
template <class R>
struct TabView {
  const R* tot;
  const R* cum0;
  int32_t n_lo;
  const R* bgam;
  const R* binv;
  const R* bedge;
  const ChanP<R>* ch;  // channel parameters
  const double* sct;   // azimuth table (GasDev::sct)
};

constexpr int kLdsBands = 512;    // band tables staged in LDS (the first this many)
constexpr int kLdsChannels = 64;  // channel parameters staged in LDS (the first this many)

// Every band and channel of the gas fits the LDS copies (host side: selects
// the persistent kernel's kFit instance).
inline bool tables_fit_lds(const GasDev& G) { return G.n_bands <= kLdsBands && G.n_ch <= kLdsChannels; }

// Pointers into LDS, typed as such in device code: loads through them are
// DS instructions (a pointer that may hold either an LDS or a global address
// is read with the slower FLAT instructions).
#if defined(__HIP_DEVICE_COMPILE__)
#define AVM_LDS __attribute__((address_space(3)))
#else
#define AVM_LDS
#endif

template <class R>
struct TabLds {
  const AVM_LDS R* tot;
  const AVM_LDS R* cum0;
  int32_t n_lo;
  const AVM_LDS R* bgam;
  const AVM_LDS R* binv;
  const AVM_LDS R* bedge;
  const AVM_LDS ChanP<R>* ch;
  const AVM_LDS double* sct;
};

// The same LDS copies when every band and channel is staged (the persistent
// kernel's kFit instances): the accessors read them without an index test.
// With the per-lane test each read carries a divergent global path, and the
// waits the compiler places where the two paths join also hold up the LDS
// reads that follow.
template <class R>
struct TabFit {
  const AVM_LDS R* tot;
  const AVM_LDS R* cum0;
  int32_t n_lo;
  const AVM_LDS R* bgam;
  const AVM_LDS R* binv;
  const AVM_LDS R* bedge;
  const AVM_LDS ChanP<R>* ch;
  const AVM_LDS double* sct;
};

enum FieldKind : int32_t { FIELD_SLAB = 0, FIELD_POLAR = 1 };

struct FieldDev {
  int32_t kind;
  uint32_t n_E;
  double z_lo, z_hi;
  const double* E;          // slab: [n_E][3]
  double a, b, a2, b2;      // polar: wire and tube radii (and squares)
  double inv_dlog;          // (n_r - 1) / ln(b/a)
  double ln_a;
  int32_t n_r, n_phi;
  const float* Er;          // [n_r][n_phi]
  const float* Ephi;
  // magnetic field: unit vector, |B|-derived constants
  int32_t has_b, _pad;
  double bh[3];
  double omega, inv_omega;  // k_b |B|
  double wd_scale;          // (k_a / k_b) / |B|^2
  double Bv[3];
};

struct RunParams {
  uint32_t key0, key1;      // seed
  uint32_t k_max;
  int32_t banded;
  double t_max;
  double k_a, two_ka, inv_2ka;
  float k_a_f, two_ka_f, inv_2ka_f, _padf;
  uint64_t budget_ticks;    // wall_clock64() ticks a transport kernel may run
  double look;              // banded: band lookahead in mean free times (0: none)
};

// Induced signal on the readout electrode (Shockley-Ramo): bin j of
// avalanche a, out[a n_bins + j], accumulates the change of the weighting
// potential phi_w of the avalanche's electrons while they move during
// [T_j, T_j+1), T_j = t0 + j dt (the change of induced charge in units of
// the elementary charge, electrons carrying -1).  Readout electrode: the
// z_hi plane of a slab, phi_w = (z - z_lo) / (z_hi - z_lo); the wire of the
// coaxial geometry, phi_w = ln(b/rho) / ln(b/a).
struct SignalDev {
  double* out;
  double t0, dt;
  double w0, w1;   // slab: phi_w = (z - w0) / w1; coaxial wire: (w0 - ln rho) / w1
  int32_t n_bins;
  int32_t _pad;
};

// ---------------------------------------------------------------------------
// Philox4x32-10 and uniform maps
// ---------------------------------------------------------------------------
struct Block { uint32_t w0, w1, w2, w3; };

// Marks a wave-uniform value as redefined here (it stays in a scalar
// register).  Work derived from it cannot be hoisted out of the enclosing
// loop, where the derived values would stay live across the whole loop and
// be spilled to VGPR lanes; recomputing them costs a few scalar adds.
AVM_FN uint32_t pin_uniform(uint32_t v) {
#if defined(__HIP_DEVICE_COMPILE__)
  asm volatile("" : "+s"(v));
#endif
  return v;
}

// The object p points to, through an address the compiler cannot see
// through: loads of its fields stay where they are used instead of being
// hoisted out of loops (for rarely used parameter blocks).
template <class T>
AVM_FN const T& pinned(const T* p) {
  return *(p + pin_uniform(0u));
}

// a ^ b ^ c in one instruction (gfx950's three-input bitwise operation,
// truth table 0x96)
AVM_FN uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
#else
  return a ^ b ^ c;
#endif
}

AVM_FN Block philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1) {
  k0 = pin_uniform(k0);  // the round keys are formed here, not kept live
  k1 = pin_uniform(k1);
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
    const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
    const uint32_t n0 = xor3(hi1, c1, k0);
    const uint32_t n2 = xor3(hi0, c3, k1);
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return Block{c0, c1, c2, c3};
}

AVM_FN Block draw(const RunParams& p, uint32_t aval, uint64_t eid, uint32_t k, uint32_t j) {
  return philox(4u * k + j, aval, (uint32_t)eid, (uint32_t)(eid >> 32), p.key0, p.key1);
}


// 53-bit uniform in (0, 1]: ((hi >> 5) 2^26 + (lo >> 6) + 1) 2^-53, every
// intermediate an exact integer in binary64.
AVM_FN double u53(uint32_t hi, uint32_t lo) {
  return __builtin_fma((double)(hi >> 5), 67108864.0, (double)((lo >> 6) + 1u)) *
         1.1102230246251565e-16;
}
// 24-bit uniform in (0, 1] from the high word alone, exact in binary32.
AVM_FN float u24(uint32_t hi) { return (float)((hi >> 8) + 1u) * 5.9604644775390625e-8f; }

// ---------------------------------------------------------------------------
// FP64 logarithm and sin/cos of pi x for the transport loop
// ---------------------------------------------------------------------------
// Both are written for the arguments the loop gives them (a uniform in
// (0, 1] for the flight time, 2u in (0, 2] for an azimuth): no handling of
// zero, negative, infinite or NaN arguments, and under half the
// instructions of the general library routines.  Their polynomials are the
// Taylor series of the functions, truncated where the next term is below
// 2^-60 of the result; the constants are those coefficients rounded to
// binary64.  Polynomials run in Horner's form with the coefficient as the
// addend, which the hardware takes from a scalar register (no vector moves
// for the constants).  Errors, measured on 2e7 arguments against extended
// precision: log 0.84 ulp, sincospi 1.05 ulp.

// a * b + c with the constant c taken from a scalar register pair by the
// three-operand FMA.  (The compiler's two-operand form wants the addend in
// the destination vector register: two vector moves per constant, as many
// issue cycles as the FMA itself.)
AVM_FN double fma_k(double a, double b, double c) {
#if defined(__HIP_DEVICE_COMPILE__)
  double r;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(c));
  return r;
#else
  return __builtin_fma(a, b, c);
#endif
}

// Approximate 1/d (device: the hardware reciprocal); callers refine it.
AVM_FN double rcp_seed(double d) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rcp(d);
#else
  return 1.0 / d;
#endif
}

// Square root of x >= 0 (0 for x <= 0) in the range the loop uses: the
// hardware reciprocal square root refined by one coupled Goldschmidt step
// and two Newton corrections of the root (Markstein's scheme).  Correctly
// rounded: no difference from the IEEE square root on 1e8 arguments over
// 1e-12..1e2, even from a seed with 3e-5 relative error; it skips the
// rescaling and special-value handling of the general routine.
AVM_FN double sqrt_nn(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y, h = 0.5 * y;
  const double r = __builtin_fma(-g, h, 0.5);
  g = __builtin_fma(g, r, g);
  h = __builtin_fma(h, r, h);
  double d = __builtin_fma(-g, g, x);
  g = __builtin_fma(d, h, g);
  d = __builtin_fma(-g, g, x);
  g = __builtin_fma(d, h, g);
  return x > 0.0 ? g : 0.0;
#else
  return x > 0.0 ? sqrt(x) : 0.0;
#endif
}

// 1 / sqrt(x) for a positive normal x: the hardware estimate y0 refined by
// the binomial series of (1 - e)^(-1/2) = 1 + e/2 + 3e^2/8 + ... with
// e = 1 - x y0^2 (no handling of zero, infinite or negative arguments).
AVM_FN double rsqrt_pos(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  const double y = __builtin_amdgcn_rsq(x);
  const double e = __builtin_fma(y * -x, y, 1.0);
  return __builtin_fma(y * e, __builtin_fma(e, 0.375, 0.5), y);
#else
  return 1.0 / sqrt(x);
#endif
}

// Natural logarithm of a positive normal x.  x = 2^k m with m in
// [sqrt(1/2), sqrt(2)) and f = m - 1; with s = f / (2 + f),
// log(1 + f) = 2 atanh(s) = f - f^2/2 + s (f^2/2 + R), R = sum_{i>=1}
// 2 s^{2i} / (2i + 1) (ten terms: |s| < 0.172, split into even and odd
// powers of s^2 for two independent chains).  k ln 2 is added in two parts,
// the first with 42 significant bits so that k times it is exact (the
// reduction of Cody and Waite, Software Manual for the Elementary
// Functions, 1980).  s needs only ~2^-40 relative accuracy (it scales a
// term below f^2/2); one Newton step and one residual correction on the
// reciprocal give far more, whatever the seed's accuracy beyond 2^-24.
AVM_FN double log_pos(double x) {
  int k;
  double m = frexp(x, &k);  // [1/2, 1)
  const bool low = m < 0x1.6a09e667f3bcdp-1;
  m = low ? m + m : m;
  k = low ? k - 1 : k;
  const double f = m - 1.0;  // exact
  const double d = 2.0 + f;
  double r = rcp_seed(d);
  r = __builtin_fma(r, __builtin_fma(-d, r, 1.0), r);
  double s = f * r;
  s = __builtin_fma(__builtin_fma(-s, d, f), r, s);
  const double z = s * s, w = z * z;
  // 2 / (2i + 1): i odd in E, i even in O
  double E = __builtin_fma(0x1.af286bca1af28p-4, w, 0x1.1111111111111p-3);
  double O = __builtin_fma(0x1.8618618618618p-4, w, 0x1.e1e1e1e1e1e1ep-4);
  E = fma_k(E, w, 0x1.745d1745d1746p-3);
  O = fma_k(O, w, 0x1.3b13b13b13b14p-3);
  E = fma_k(E, w, 0x1.2492492492492p-2);
  O = fma_k(O, w, 0x1.c71c71c71c71cp-3);
  E = fma_k(E, w, 0x1.5555555555555p-1);
  O = fma_k(O, w, 0x1.999999999999ap-2);
  const double R = z * __builtin_fma(z, O, E);
  const double hfsq = 0.5 * f * f;
  const double dk = (double)k;
  const double t = __builtin_fma(s, hfsq + R, dk * 0x1.ef35793c76730p-45);  // + k ln2 (low part)
  return __builtin_fma(dk, 0x1.62e42fefa3800p-1, f - (hfsq - t));         // + k ln2 (high part)
}

// v with its sign flipped when bit 1 of n is set
AVM_FN double flip_if_bit1(double v, uint32_t n) {
  return __builtin_bit_cast(double, __builtin_bit_cast(uint64_t, v) ^ ((uint64_t)(n & 2u) << 62));
}

// sin(pi x) and cos(pi x) for moderate |x|: t = 2x = q + r with q the
// nearest integer (r in [-1/2, 1/2], exact), so the angle is
// q pi/2 + theta with theta = (pi/2) r in [-pi/4, pi/4]; sin theta and
// cos theta from their series in r (terms to r^17 and r^18; the leading
// pi/2 in two parts); q mod 4 picks the quadrant.
AVM_FN void sincospi_pos(double x, double* sp, double* cp) {
  const double t = x + x;
  const double q = rint(t);
  const double r = t - q;
  const uint32_t n = (uint32_t)(int32_t)q;
  const double r2 = r * r;
  // (-1)^j (pi/2)^(2j+1) / (2j+1)!, j = 8..1, and (-1)^j (pi/2)^(2j) / (2j)!, j = 9..1
  double ps = __builtin_fma(0x1.aaec32af93359p-38, r2, -0x1.6fadb9f155744p-31);
  double pc = __builtin_fma(-0x1.2a0c591af8314p-41, r2, 0x1.20c62c2f2d7f5p-34);
  ps = fma_k(ps, r2, 0x1.e8f434d018d63p-25);
  pc = fma_k(pc, r2, -0x1.b6e24f44b128fp-28);
  ps = fma_k(ps, r2, -0x1.e3074fde8871fp-19);
  pc = fma_k(pc, r2, 0x1.f9d38a3763cc3p-22);
  ps = fma_k(ps, r2, 0x1.50783487ee782p-13);
  pc = fma_k(pc, r2, -0x1.a6d1f2a204a8cp-16);
  ps = fma_k(ps, r2, -0x1.32d2cce62bd86p-8);
  pc = fma_k(pc, r2, 0x1.e1f506891babbp-11);
  ps = fma_k(ps, r2, 0x1.466bc6775aae2p-4);
  pc = fma_k(pc, r2, -0x1.55d3c7e3cbffap-6);
  ps = fma_k(ps, r2, -0x1.4abbce625be53p-1);
  pc = fma_k(pc, r2, 0x1.03c1f081b5ac4p-2);
  pc = fma_k(pc, r2, -0x1.3bd3cc9be45dep+0);
  const double sn = __builtin_fma(r, 0x1.921fb54442d18p+0, r * fma_k(r2, ps, 0x1.1a62633145c07p-54));
  const double cs = __builtin_fma(r2, pc, 1.0);
  const bool odd = n & 1u;
  // sin is negative in quadrants 2, 3 and cos in quadrants 1, 2
  *sp = flip_if_bit1(odd ? cs : sn, n);
  *cp = flip_if_bit1(odd ? sn : cs, n + 1u);
}

// ---------------------------------------------------------------------------
// precision-generic arithmetic
// ---------------------------------------------------------------------------
template <class R> struct M;
template <> struct M<double> {
  AVM_FN static double uni(uint32_t hi, uint32_t lo) { return u53(hi, lo); }
  AVM_FN static double fma(double a, double b, double c) { return __builtin_fma(a, b, c); }
  AVM_FN static double sqrt_(double x) { return sqrt_nn(x); }
  AVM_FN static double rsqrt_(double x) { return rsqrt_pos(x); }
  AVM_FN static double log_(double x) { return log_pos(x); }
  AVM_FN static double floor_(double x) { return floor(x); }
  AVM_FN static double tan_(double x) { return tan(x); }
  AVM_FN static double atan_(double x) { return atan(x); }
  AVM_FN static void sincospi_(double x, double* s, double* c) { sincospi_pos(x, s, c); }
  AVM_FN static double abs_(double x) { return fabs(x); }
  AVM_FN static double inf() { return __builtin_inf(); }
  // the sampling and scattering forms (flight-time logarithm, scattering
  // and emission angles, speeds): the accurate ones in FP64
  AVM_FN static double log_s(double x) { return log_pos(x); }
  AVM_FN static double sqrt_s(double x) { return sqrt_nn(x); }
  AVM_FN static double rsqrt_s(double x) { return rsqrt_pos(x); }
};
template <> struct M<float> {
  AVM_FN static float uni(uint32_t hi, uint32_t) { return u24(hi); }
  AVM_FN static float fma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
  AVM_FN static float sqrt_(float x) { return sqrtf(x); }
  AVM_FN static float rsqrt_(float x) { return rsqrtf(x); }
  AVM_FN static float log_(float x) { return logf(x); }
  AVM_FN static float floor_(float x) { return floorf(x); }
  AVM_FN static float tan_(float x) { return tanf(x); }
  AVM_FN static float atan_(float x) { return atanf(x); }
  AVM_FN static void sincospi_(float x, float* s, float* c) { sincospif(x, s, c); }
  AVM_FN static float abs_(float x) { return fabsf(x); }
  AVM_FN static float inf() { return __builtin_inff(); }
  // the sampling and scattering forms in FP32-mixed: the hardware
  // approximations (log2, square root and reciprocal square root to about
  // 1 ulp; sin and cos of 2 pi u with u in turns), whose errors enter only
  // sampled flight times, angles and speeds; the library forms above stay
  // where a bound depends on the result (band crossings, helical steps)
#ifdef AVM_HOST_DEBUG
  AVM_FN static float log_s(float x) { return logf(x); }
  AVM_FN static float sqrt_s(float x) { return sqrtf(x); }
  AVM_FN static float rsqrt_s(float x) { return 1.0f / sqrtf(x); }
  AVM_FN static void sincos2pi_s(float u, float* s, float* c) { sincospif(u + u, s, c); }
#else
  AVM_FN static float log_s(float x) { return __builtin_amdgcn_logf(x) * 0.693147180559945309f; }
  AVM_FN static float sqrt_s(float x) { return __builtin_amdgcn_sqrtf(x); }
  AVM_FN static float rsqrt_s(float x) { return __builtin_amdgcn_rsqf(x); }
  AVM_FN static void sincos2pi_s(float u, float* s, float* c) {
    const float t = u - floorf(u);  // [0, 1) turns
    *s = __builtin_amdgcn_sinf(t);
    *c = __builtin_amdgcn_cosf(t);
  }
#endif
};

template <class R>
AVM_FN R dot3(R ax, R ay, R az, R bx, R by, R bz) {
  return M<R>::fma(az, bz, M<R>::fma(ay, by, ax * bx));
}

// Interpolation (1-f) a + f b with non-negative weights: monotone in a and
// b after rounding, so interpolated cumulative rates stay ordered.
template <class R>
AVM_FN R lerp(R a, R b, R g1, R f) { return M<R>::fma(f, b, g1 * a); }

// Entries of the azimuth table: sin and cos of 2 pi j / kAzN.
constexpr int kAzN = 256;

// sin and cos of an azimuth 2 pi u, u in [0, 1].  FP64: the nearest table
// angle 2 pi j / kAzN and the series of the remainder
// theta = 2 pi (u - j / kAzN), |theta| <= pi / kAzN (sine to theta^7,
// cosine to theta^6), combined by the addition theorem; the table holds
// sincospi_pos values, so the result is within about 1.6 ulp.  (The
// general sincospi_pos takes 19 polynomial terms.)  FP32-mixed: the
// hardware sine and cosine of the angle in turns.
template <class TV>
AVM_FN void azimuth(const TV& T, double u, double* sp, double* cp) {
  const double x = u * (double)kAzN;  // exact
  const double jr = rint(x);
  const double t = x - jr;            // [-1/2, 1/2], exact
  const int j = (int)jr & (kAzN - 1);
  const double sa = T.sct[2 * j], ca = T.sct[2 * j + 1];
  // theta = t (2 pi / kAzN), the constant in two parts
  const double th = __builtin_fma(t, 0x1.921fb54442d18p-6, t * 0x1.1a62633145c07p-60);
  const double z = th * th;
  const double sm = th * z * fma_k(__builtin_fma(z, -0x1.a01a01a01a01ap-13, 0x1.1111111111111p-7), z,
                                   -0x1.5555555555555p-3);
  const double cm = z * fma_k(__builtin_fma(z, -0x1.6c16c16c16c17p-10, 0x1.5555555555555p-5), z, -0.5);
  *sp = sa + __builtin_fma(ca, th, __builtin_fma(ca, sm, sa * cm));
  *cp = ca + __builtin_fma(-sa, th, __builtin_fma(-sa, sm, ca * cm));
}
template <class TV>
AVM_FN void azimuth(const TV&, float u, float* sp, float* cp) { M<float>::sincos2pi_s(u, sp, cp); }

// Direction of (dx, dy, dz) turned by polar angle theta (cos_t) and azimuth
// phi = 2 pi u_phi.  The transverse length s = sqrt(dx^2 + dy^2) avoids the
// cancellation of sqrt(1 - dz^2) next to the poles, so |d'| = 1 to rounding.
template <class R, class TV>
AVM_FN void turn(const TV& T, R dx, R dy, R dz, R cos_t, R u_phi, R& ox, R& oy, R& oz) {
  const R st2 = M<R>::fma(-cos_t, cos_t, R(1));
  const R sin_t = st2 > R(0) ? M<R>::sqrt_s(st2) : R(0);
  R sp, cp;
  azimuth(T, u_phi, &sp, &cp);
  const R q = M<R>::fma(dx, dx, dy * dy);
  const R tiny = sizeof(R) == 8 ? R(1e-24) : R(1e-12);
  if (q > tiny) {
    const R inv_s = M<R>::rsqrt_s(q);
    const R s = q * inv_s;
    const R a = sin_t * inv_s;
    ox = M<R>::fma(dx, cos_t, a * M<R>::fma(dx * dz, cp, -dy * sp));
    oy = M<R>::fma(dy, cos_t, a * M<R>::fma(dy * dz, cp, dx * sp));
    oz = M<R>::fma(dz, cos_t, -s * sin_t * cp);
  } else {
    ox = sin_t * cp;
    oy = sin_t * sp;
    oz = (dz < R(0) ? R(-1) : R(1)) * cos_t;
  }
}

// Real roots of A s^2 + B s + C = 0 in ascending order (stable form).
template <class R>
AVM_FN int roots2(R A, R B, R C, R& r1, R& r2) {
  if (A == R(0)) {
    if (B == R(0)) return 0;
    r1 = -C / B;
    return 1;
  }
  const R disc = B * B - R(4) * A * C;
  if (disc < R(0)) return 0;
  const R sq = M<R>::sqrt_(disc);
  const R q = R(-0.5) * (B + (B >= R(0) ? sq : -sq));
  if (q == R(0)) {
    r1 = R(0);
    r2 = R(0);
  } else {
    r1 = q / A;
    r2 = C / q;
  }
  if (r1 > r2) {
    const R t = r1;
    r1 = r2;
    r2 = t;
  }
  return 2;
}

// First exit time in (0, T] of z(s) = z0 + vz s + az s^2 / 2 from the slab
// [zlo, zhi): arrival at zhi, or a crossing below zlo with dz/ds < 0 (s = 0
// counts when sitting on zlo moving down).  A cheap bound on the extremes of
// the parabola over [0, T] rules out the common no-exit case before any root
// is taken.  FP64 in both precisions.
AVM_FN uint32_t slab_exit(double z0, double vz, double az, double zlo, double zhi, double T,
                          double& s_exit) {
  const double zT = __builtin_fma(0.5 * az * T, T, __builtin_fma(vz, T, z0));
  // margin: a relative 1e-12 of the coordinates keeps the filter conservative
  const double m = 1e-12 * (fabs(z0) + fabs(zhi) + fabs(zlo) + fabs(vz * T) + fabs(az * T * T));
  const double lo = zlo + m, hi = zhi - m;
  bool inside = (z0 > zT ? z0 : zT) < hi && (z0 < zT ? z0 : zT) > lo;
  // the vertex s* = -vz/az lies in (0, T) iff vz az < 0 and |vz| < |az| T;
  // there z = z0 - vz^2 / (2 az), a minimum for az > 0 (to stay above lo)
  // and a maximum for az < 0 (to stay below hi): compared after multiplying
  // by 2 az, without a division
  if (inside && vz * az < 0.0 && fabs(vz) < fabs(az) * T)
    inside = 2.0 * az * (z0 - (az > 0.0 ? lo : hi)) > vz * vz;
  if (inside) return 0;
  double best = __builtin_inf();
  uint32_t side = 0;
  double r1 = 0.0, r2 = 0.0;
  int n = roots2<double>(0.5 * az, vz, z0 - zhi, r1, r2);
  if (n >= 1 && r1 > 0.0) {
    best = r1;
    side = ST_HIGH;
  } else if (n == 2 && r2 > 0.0) {
    best = r2;
    side = ST_HIGH;
  }
  n = roots2<double>(0.5 * az, vz, z0 - zlo, r1, r2);
  for (int i = 0; i < n; ++i) {
    const double s = i == 0 ? r1 : r2;
    if (s < 0.0) continue;
    const double slope = az * s + vz;
    if (slope < 0.0 || (s == 0.0 && slope == 0.0 && az < 0.0)) {
      if (s < best) {
        best = s;
        side = ST_LOW;
      }
      break;
    }
  }
  if (side && best <= T) {
    s_exit = best;
    return side;
  }
  return 0;
}

// ---------------------------------------------------------------------------
// fields
// ---------------------------------------------------------------------------
// Polar map: bilinear in (ln rho, phi), clamped in rho, periodic in phi,
// rotated to Cartesian.
template <class R>
AVM_FN void polar_field(const FieldDev& F, double x, double y, R& Ex, R& Ey) {
  const double r2 = x * x + y * y;
  if (!(r2 > 0.0)) {
    Ex = R(0);
    Ey = R(0);
    return;
  }
  // ln rho = ln(rho^2) / 2, and 1/rho from one reciprocal square root
  double u = (0.5 * log_pos(r2) - F.ln_a) * F.inv_dlog;
  const double umax = (double)(F.n_r - 1);
  u = u < 0.0 ? 0.0 : (u > umax ? umax : u);
  int i = (int)floor(u);
  i = i > F.n_r - 2 ? F.n_r - 2 : i;
  const R fr = (R)(u - (double)i);
  double phi = atan2(y, x);
  if (phi < 0.0) phi += 6.283185307179586;
  const double w = phi * (0.15915494309189535 * (double)F.n_phi);
  const double wf = floor(w);
  const R fp = (R)(w - wf);
  int j0 = (int)wf;
  j0 = j0 >= F.n_phi ? j0 - F.n_phi : j0;
  const int j1 = j0 + 1 == F.n_phi ? 0 : j0 + 1;
  const int np = F.n_phi;
  const R w00 = (R(1) - fr) * (R(1) - fp), w01 = (R(1) - fr) * fp;
  const R w10 = fr * (R(1) - fp), w11 = fr * fp;
  const float* A = F.Er;
  const float* B = F.Ephi;
  const R er = w00 * (R)A[i * np + j0] + w01 * (R)A[i * np + j1] + w10 * (R)A[(i + 1) * np + j0] +
               w11 * (R)A[(i + 1) * np + j1];
  const R ep = w00 * (R)B[i * np + j0] + w01 * (R)B[i * np + j1] + w10 * (R)B[(i + 1) * np + j0] +
               w11 * (R)B[(i + 1) * np + j1];
  const double inv = rsqrt_pos(r2);
  const R c = (R)(x * inv), s = (R)(y * inv);
  Ex = er * c - ep * s;
  Ey = er * s + ep * c;
}

// ---------------------------------------------------------------------------
// electron state and one pass of the transport loop
// ---------------------------------------------------------------------------
template <class R>
struct Elec {
  double x, y, z, t;  // accumulators: FP64 in both precisions
  R vx, vy, vz;
  uint64_t eid;
  uint32_t aval, k;
  int32_t band;
  // counters (null collisions are not counted here: every flight that goes
  // on advances k, so k = n_null + n_masked + n_band + n_real - [attached])
  uint32_t n_real, n_ion, n_masked, n_band, n_over;
  uint32_t trace;  // decision trace (trace_step)
  R Ex, Ey, Ez;  // slab: the avalanche's field, loaded once per electron
  // induced signal: weighting potential where the current bin piece began,
  // time and index of the next bin edge
  double sphi, snext;
  int32_t sj;
};

template <class R>
struct Child {
  R vx, vy, vz, e;
  uint64_t eid;
  R pen;      // pending ionisation: energy at the collision; pending
              // boundary exit: the flight's end time (STEP_EXIT)
  int32_t pc; // pending ionisation: channel
};

enum : int32_t { STEP_CONTINUE = 0, STEP_IONISED = 1, STEP_DONE = 2, STEP_EXIT = 3 };

// Decision trace of an electron: a running 32-bit hash over its real
// collisions, masked nulls and band cuts in flight order, so that two runs
// can be told apart by the decisions an electron made (null collisions
// enter through n_null).  Each event at flight index k maps h to
// rotl(h, 5) ^ (k 2^18 + code), code = c for a real collision in channel
// c, 2^16 + c for a masked null at channel c, 2^17 for a band cut.
enum : uint32_t { TRACE_MASKED = 1u << 16, TRACE_BAND = 1u << 17 };
AVM_FN uint32_t trace_step(uint32_t h, uint32_t k, uint32_t code) {
  return ((h << 5) | (h >> 27)) ^ ((k << 18) + code);
}

// Precision-selected members of the gas and run parameters.
template <class R> struct Sel;
template <> struct Sel<double> {
  AVM_FN static double scale(const GasDev& G) { return G.scale; }
  AVM_FN static double x_top(const GasDev& G) { return G.x_top; }
  AVM_FN static double band_scale(const GasDev& G) { return G.band_scale; }
  AVM_FN static double gamma(const GasDev& G) { return G.gamma; }
  AVM_FN static double inv_gamma(const GasDev& G) { return G.inv_gamma; }
  AVM_FN static const ChanP<double>* ch(const GasDev& G) { return G.ch; }
  AVM_FN static const double* total(const GasDev& G) { return G.total; }
  AVM_FN static const double* cum0(const GasDev& G) { return G.cum0; }
  AVM_FN static const double* cum(const GasDev& G) { return G.cum; }
  AVM_FN static const double* bgam(const GasDev& G) { return G.band_gamma; }
  AVM_FN static const double* binv(const GasDev& G) { return G.band_inv; }
  AVM_FN static const double* bedge(const GasDev& G) { return G.band_edge; }
  AVM_FN static double k_a(const RunParams& P) { return P.k_a; }
  AVM_FN static double two_ka(const RunParams& P) { return P.two_ka; }
  AVM_FN static double inv_2ka(const RunParams& P) { return P.inv_2ka; }
};
template <> struct Sel<float> {
  AVM_FN static float scale(const GasDev& G) { return G.scale_f; }
  AVM_FN static float x_top(const GasDev& G) { return G.x_top_f; }
  AVM_FN static float band_scale(const GasDev& G) { return G.band_scale_f; }
  AVM_FN static float gamma(const GasDev& G) { return G.gamma_f; }
  AVM_FN static float inv_gamma(const GasDev& G) { return G.inv_gamma_f; }
  AVM_FN static const ChanP<float>* ch(const GasDev& G) { return G.ch_f; }
  AVM_FN static const float* total(const GasDev& G) { return G.total_f; }
  AVM_FN static const float* cum0(const GasDev& G) { return G.cum0_f; }
  AVM_FN static const float* cum(const GasDev& G) { return G.cum_f; }
  AVM_FN static const float* bgam(const GasDev& G) { return G.band_gamma_f; }
  AVM_FN static const float* binv(const GasDev& G) { return G.band_inv_f; }
  AVM_FN static const float* bedge(const GasDev& G) { return G.band_edge_f; }
  AVM_FN static float k_a(const RunParams& P) { return P.k_a_f; }
  AVM_FN static float two_ka(const RunParams& P) { return P.two_ka_f; }
  AVM_FN static float inv_2ka(const RunParams& P) { return P.inv_2ka_f; }
};

// The global-memory tables of precision R (no LDS copies).
template <class R> AVM_FN TabView<R> global_view(const GasDev& G);
template <> AVM_FN TabView<double> global_view<double>(const GasDev& G) {
  return TabView<double>{G.total, G.cum0, G.n_bins + 1, G.band_gamma, G.band_inv, G.band_edge, G.ch, G.sct};
}
template <> AVM_FN TabView<float> global_view<float>(const GasDev& G) {
  return TabView<float>{G.total_f, G.cum0_f, G.n_bins + 1, G.band_gamma_f, G.band_inv_f,
                        G.band_edge_f, G.ch_f, G.sct};
}

// Band tables and channel parameters through either view.  Beyond the LDS
// copies the global pointer is read from the kernel argument where it is
// used (pinned), so it does not occupy registers across the loop.
template <class R>
AVM_FN R band_gamma(const GasDev&, const TabView<R>& T, int32_t b) { return T.bgam[b]; }
template <class R>
AVM_FN R band_inv(const GasDev&, const TabView<R>& T, int32_t b) { return T.binv[b]; }
template <class R>
AVM_FN R band_edge(const GasDev&, const TabView<R>& T, int32_t b) { return T.bedge[b]; }
template <class R>
AVM_FN ChanP<R> chan(const GasDev&, const TabView<R>& T, int32_t c) { return T.ch[c]; }
template <class R>
AVM_FN R band_gamma(const GasDev& G, const TabLds<R>& T, int32_t b) {
  return b < kLdsBands ? T.bgam[b] : Sel<R>::bgam(pinned(&G))[b];
}
template <class R>
AVM_FN R band_inv(const GasDev& G, const TabLds<R>& T, int32_t b) {
  return b < kLdsBands ? T.binv[b] : Sel<R>::binv(pinned(&G))[b];
}
template <class R>
AVM_FN R band_edge(const GasDev& G, const TabLds<R>& T, int32_t b) {
  return b < kLdsBands ? T.bedge[b] : Sel<R>::bedge(pinned(&G))[b];
}
template <class R>
AVM_FN ChanP<R> chan(const GasDev& G, const TabLds<R>& T, int32_t c) {
  if (c < kLdsChannels) return T.ch[c];
  return Sel<R>::ch(pinned(&G))[c];
}
template <class R>
AVM_FN R band_gamma(const GasDev&, const TabFit<R>& T, int32_t b) { return T.bgam[b]; }
template <class R>
AVM_FN R band_inv(const GasDev&, const TabFit<R>& T, int32_t b) { return T.binv[b]; }
template <class R>
AVM_FN R band_edge(const GasDev&, const TabFit<R>& T, int32_t b) { return T.bedge[b]; }
template <class R>
AVM_FN ChanP<R> chan(const GasDev&, const TabFit<R>& T, int32_t c) { return T.ch[c]; }

template <class R, class TV>
AVM_FN int32_t band_of(const GasDev& G, const TV& T, R e) {
  const int32_t nb = G.n_bands;
  int32_t b = (int32_t)(e * Sel<R>::band_scale(G));
  b = b < 0 ? 0 : (b > nb - 1 ? nb - 1 : b);
  // the first guess is the band or a neighbour: both of its edges are read
  // at once (the last band's edge is infinite), and the rare further steps
  // follow one at a time
  const R hi = band_edge(G, T, b);
  const R lo = band_edge(G, T, b > 0 ? b - 1 : 0);
  if (b < nb - 1 && !(e < hi)) {
    ++b;
    while (b < nb - 1 && !(e < band_edge(G, T, b))) ++b;
  } else if (b > 0 && e < lo) {
    --b;
    while (b > 0 && e < band_edge(G, T, b - 1)) --b;
  }
  return b;
}

// band_of() that also hands back the band's majorant, its inverse and its
// upper edge: read together with the edges of the first guess, so a flight
// whose lookahead lands in the guessed band waits for one LDS round trip.
template <class R, class TV>
AVM_FN int32_t band_of_tabs(const GasDev& G, const TV& T, R e, R& gam, R& inv, R& edge) {
  const int32_t nb = G.n_bands;
  int32_t b = (int32_t)(e * Sel<R>::band_scale(G));
  b = b < 0 ? 0 : (b > nb - 1 ? nb - 1 : b);
  const int32_t guess = b;
  const R hi = band_edge(G, T, b);
  const R lo = band_edge(G, T, b > 0 ? b - 1 : 0);
  gam = band_gamma(G, T, b);
  inv = band_inv(G, T, b);
  edge = hi;
  if (b < nb - 1 && !(e < hi)) {
    ++b;
    while (b < nb - 1 && !(e < band_edge(G, T, b))) ++b;
  } else if (b > 0 && e < lo) {
    --b;
    while (b > 0 && e < band_edge(G, T, b - 1)) --b;
  }
  if (b != guess) {
    gam = band_gamma(G, T, b);
    inv = band_inv(G, T, b);
    edge = band_edge(G, T, b);
  }
  return b;
}

// Termination status of a position outside the drift region, 0 inside
// (the geometry is the kernel's kField, the same as F.kind).
template <class R, int kField>
AVM_FN uint32_t region_status(const FieldDev& F, const Elec<R>& e) {
  if (kField == FIELD_SLAB) {
    if (e.z < F.z_lo) return ST_LOW;
    if (e.z >= F.z_hi) return ST_HIGH;
    return 0;
  }
  const double r2 = e.x * e.x + e.y * e.y;
  if (r2 <= F.a2) return ST_WIRE;
  if (r2 >= F.b2) return ST_TUBE;
  return 0;
}

// Free flight of duration s from (r, v) with the field frozen at E: the
// displacement is formed in R and added to the FP64 position.  kMayHaveB =
// false compiles the B = 0 case only (the banded majorant requires B = 0).
template <class R, bool kMayHaveB = true>
AVM_FN void propagate(const FieldDev& F, const Elec<R>& e, R ax, R ay, R az, R Ex, R Ey, R Ez, R s,
                      double& rx, double& ry, double& rz, R& ux, R& uy, R& uz) {
  using Mr = M<R>;
  if (!kMayHaveB || !F.has_b) {
    const R hs2 = R(0.5) * s * s;
    rx = e.x + (double)Mr::fma(ax, hs2, e.vx * s);
    ry = e.y + (double)Mr::fma(ay, hs2, e.vy * s);
    rz = e.z + (double)Mr::fma(az, hs2, e.vz * s);
    ux = Mr::fma(ax, s, e.vx);
    uy = Mr::fma(ay, s, e.vy);
    uz = Mr::fma(az, s, e.vz);
    return;
  }
  // constant E and B: uniform acceleration along B, E x B drift plus
  // gyration across it
  const R bx = (R)F.bh[0], by = (R)F.bh[1], bz = (R)F.bh[2];
  const R Bx = (R)F.Bv[0], By = (R)F.Bv[1], Bz = (R)F.Bv[2];
  const R wds = (R)F.wd_scale;
  const R vpar = dot3<R>(e.vx, e.vy, e.vz, bx, by, bz);
  const R apar = dot3<R>(ax, ay, az, bx, by, bz);
  const R wx = wds * (Ey * Bz - Ez * By);
  const R wy = wds * (Ez * Bx - Ex * Bz);
  const R wz = wds * (Ex * By - Ey * Bx);
  const R u0x = (e.vx - vpar * bx) - wx;
  const R u0y = (e.vy - vpar * by) - wy;
  const R u0z = (e.vz - vpar * bz) - wz;
  const R cx = by * u0z - bz * u0y;
  const R cy = bz * u0x - bx * u0z;
  const R cz = bx * u0y - by * u0x;
  // sin and cos of the phase ph = omega s, and 1 - cos(ph) without
  // cancellation, from one sin/cos pair of the half phase:
  // sin(ph) = 2 sh ch, 1 - cos(ph) = 2 sh^2 (sh, ch of ph / 2)
  const R ph = (R)F.omega * s;
  R sh, ch;
  Mr::sincospi_(ph * R(0.15915494309189535), &sh, &ch);
  const R sn = R(2) * sh * ch;
  const R omc = R(2) * sh * sh;
  const R cs = R(1) - omc;
  const R along = vpar * s + R(0.5) * apar * s * s;
  const R io = (R)F.inv_omega;
  const R a1 = sn * io, a2 = omc * io;
  rx = e.x + (double)(along * bx + wx * s + a1 * u0x + a2 * cx);
  ry = e.y + (double)(along * by + wy * s + a1 * u0y + a2 * cy);
  rz = e.z + (double)(along * bz + wz * s + a1 * u0z + a2 * cz);
  const R vp = vpar + apar * s;
  ux = vp * bx + wx + cs * u0x + sn * cx;
  uy = vp * by + wy + cs * u0y + sn * cy;
  uz = vp * bz + wz + cs * u0z + sn * cz;
}

// ---- induced signal ----
// Weighting potential of the readout electrode at (x, y, z).
template <int kField>
AVM_FN double weighting(const SignalDev& Q, double x, double y, double z) {
  if (kField == FIELD_SLAB) return (z - Q.w0) / Q.w1;
  return (Q.w0 - 0.5 * log(x * x + y * y)) / Q.w1;
}

// Time of bin edge j (edges past the last bin are never reached).
AVM_FN double signal_edge(const SignalDev& Q, int32_t j) {
  return j <= Q.n_bins ? Q.t0 + (double)j * Q.dt : __builtin_inf();
}

// Adds dq to bin j of avalanche `aval`; bins outside [0, n_bins) are dropped.
AVM_FN void signal_deposit(const SignalDev& Q, uint32_t aval, int32_t j, double dq) {
  if (j >= 0 && j < Q.n_bins) {
#ifdef AVM_HOST_DEBUG
    Q.out[(size_t)aval * (size_t)Q.n_bins + (size_t)j] += dq;
#else
    unsafeAtomicAdd(Q.out + (size_t)aval * (size_t)Q.n_bins + (size_t)j, dq);
#endif
  }
}

// Signal state of an electron at its birth (current position and time): the
// weighting potential there and the first bin edge strictly after it.
template <class R, int kField>
AVM_FN void signal_birth(const SignalDev& Q, Elec<R>& e) {
  e.sphi = weighting<kField>(Q, e.x, e.y, e.z);
  int32_t j;
  if (e.t < Q.t0) {
    j = 0;
  } else if (!(e.t < signal_edge(Q, Q.n_bins))) {
    j = Q.n_bins + 1;
  } else {
    j = (int32_t)floor((e.t - Q.t0) / Q.dt) + 1;
    j = j < 1 ? 1 : (j > Q.n_bins ? Q.n_bins : j);
    while (!(signal_edge(Q, j) > e.t)) ++j;
    while (j > 0 && signal_edge(Q, j - 1) > e.t) --j;
  }
  e.sj = j;
  e.snext = signal_edge(Q, j);
}

// Bin edges passed during the flight that starts from state e and ends at
// t_e: at each, the position from the flight formula closes the current
// piece (its potential change goes to the bin the edge ends).  The pieces
// between edges are closed lazily: consecutive flights chain, so the change
// over a run of flights is the difference of its end points.
template <class R, bool kMayHaveB, int kField>
AVM_FN void signal_flight(const SignalDev& Q, const FieldDev& F, Elec<R>& e, R ax, R ay, R az, R Ex,
                          R Ey, R Ez, double t_e) {
  while (e.snext <= t_e) {
    double mx, my, mz;
    R wx, wy, wz;
    propagate<R, kMayHaveB>(F, e, ax, ay, az, Ex, Ey, Ez, (R)(e.snext - e.t), mx, my, mz, wx, wy, wz);
    const double phi = weighting<kField>(Q, mx, my, mz);
    signal_deposit(Q, e.aval, e.sj - 1, phi - e.sphi);
    e.sphi = phi;
    e.sj += 1;
    e.snext = signal_edge(Q, e.sj);
  }
}

// At termination: the last piece, up to the end point.
template <class R, int kField>
AVM_FN void signal_end(const SignalDev& Q, const Elec<R>& e) {
  signal_deposit(Q, e.aval, e.sj - 1, weighting<kField>(Q, e.x, e.y, e.z) - e.sphi);
}

// ---- banded majorant with a magnetic field ----
// Along a helical flight the energy is not convex in time, so the band rule
// uses a bound that grows with time.  Along B the speed is at most
// vp + ap s (vp = |v_par|, ap = |a_par|); across B the velocity is the drift
// w plus u0 = v_perp - w turned by omega s, which moves away from v_perp by
// at most |u0| omega s and is never longer than |w| + |u0|.  With p =
// |v_perp|, q = |u0| omega, m = |w| + |u0|:
//   2 k_a e(s) <= (vp + ap s)^2 + min(p + q s, m)^2,
// exact at s = 0.  Evaluated in FP64 in both precisions.
struct HelixBound {
  double vp, ap, p, q, m;
};

AVM_FN HelixBound helix_bound(const FieldDev& F, const RunParams& P, double vx, double vy, double vz,
                              double Ex, double Ey, double Ez) {
  const double bx = F.bh[0], by = F.bh[1], bz = F.bh[2];
  const double vpar = vx * bx + vy * by + vz * bz;
  const double apar = -P.k_a * (Ex * bx + Ey * by + Ez * bz);
  const double wx = F.wd_scale * (Ey * F.Bv[2] - Ez * F.Bv[1]);
  const double wy = F.wd_scale * (Ez * F.Bv[0] - Ex * F.Bv[2]);
  const double wz = F.wd_scale * (Ex * F.Bv[1] - Ey * F.Bv[0]);
  const double px = vx - vpar * bx, py = vy - vpar * by, pz = vz - vpar * bz;
  const double ux = px - wx, uy = py - wy, uz = pz - wz;
  const double un = sqrt_nn(ux * ux + uy * uy + uz * uz);
  return HelixBound{fabs(vpar), fabs(apar), sqrt_nn(px * px + py * py + pz * pz), un * F.omega,
                    sqrt_nn(wx * wx + wy * wy + wz * wz) + un};
}

// Smallest s >= 0 at which the bound reaches energy e_edge (0 if it is
// there already, +inf if it never gets there).
AVM_FN double helix_root(const HelixBound& h, const RunParams& P, double e_edge) {
  const double T = P.two_ka * e_edge;
  const double c = T - (h.vp * h.vp + h.p * h.p);
  if (!(c > 0.0)) return 0.0;
  // unsaturated branch: (ap^2 + q^2) s^2 + 2 (vp ap + p q) s - c = 0
  const double A = h.ap * h.ap + h.q * h.q, B = 2.0 * (h.vp * h.ap + h.p * h.q);
  if (A == 0.0 && B == 0.0) return __builtin_inf();
  const double s1 = 2.0 * c / (B + sqrt(B * B + 4.0 * A * c));
  if (h.q == 0.0 || h.p + h.q * s1 <= h.m) return s1;
  // saturated: (vp + ap s)^2 + m^2 = T, reached after p + q s = m
  if (h.ap == 0.0 || !(T > h.m * h.m)) return __builtin_inf();
  return (sqrt(T - h.m * h.m) - h.vp) / h.ap;
}

// A duration in R no longer than s (a cut time must not overshoot).
template <class R> AVM_FN R down_to(double s);
template <> AVM_FN double down_to<double>(double s) { return s; }
template <> AVM_FN float down_to<float>(double s) {
#ifdef AVM_HOST_DEBUG
  float f = (float)s;
  return (double)f > s ? nextafterf(f, 0.0f) : f;
#else
  return __double2float_rd(s);
#endif
}

// Smallest s >= 0 at which |v + a s|^2 reaches 2 k_a edge (energy at the band
// edge).  The energy starts below the edge (C < 0), so with A = |a|^2 > 0 the
// quadratic has one positive root; its stable form needs one division (the
// same bits as the positive root of the general stable solver).
template <class R>
AVM_FN R band_crossing(const RunParams& P, const Elec<R>& e, R ax, R ay, R az, R edge) {
  const R C = dot3<R>(e.vx, e.vy, e.vz, e.vx, e.vy, e.vz) - Sel<R>::two_ka(P) * edge;
  if (C >= R(0)) return R(0);
  const R A = dot3<R>(ax, ay, az, ax, ay, az);
  if (A == R(0)) return R(0);
  const R B = R(2) * dot3<R>(e.vx, e.vy, e.vz, ax, ay, az);
  const R sq = M<R>::sqrt_(B * B - R(4) * A * C);
  // the stable form of the positive root, with one division
  const bool pos = B > R(0);
  return (pos ? R(-2) * C : sq - B) / (pos ? B + sq : R(2) * A);
}

// New velocity after a real collision: the old direction turned by
// (cos_t, phi = 2 pi uB), speed from the new energy.  (The caller advances
// the flight index.)
template <class R, class TV>
AVM_FN void scatter_to(Elec<R>& e, const RunParams& P, const TV& T, R cos_t, R uB, R e_new) {
  const R v2 = dot3<R>(e.vx, e.vy, e.vz, e.vx, e.vy, e.vz);
  R dx = R(0), dy = R(0), dz = R(1);
  if (v2 > R(0)) {
    const R inv = M<R>::rsqrt_s(v2);
    dx = e.vx * inv;
    dy = e.vy * inv;
    dz = e.vz * inv;
  }
  R ox, oy, oz;
  turn<R>(T, dx, dy, dz, cos_t, uB, ox, oy, oz);
  const R sp1 = M<R>::sqrt_s(Sel<R>::two_ka(P) * e_new);
  e.vx = sp1 * ox;
  e.vy = sp1 * oy;
  e.vz = sp1 * oz;
}

// Collision decision at energy en with selection value r_sel: -1 null,
// -2 - c masked null (the chosen channel c's window excludes en), otherwise
// the channel: the smallest c with r_sel < interpolated cumulative rate c
// (channel 0 first -- the elastic channel dominates -- then a binary search
// over the rest; interpolated cumulative rates are non-decreasing in c).
// `close` tells whether r_sel lies within a relative 2^-18 of a rate it was
// compared with, or en within a relative 2^-18 of the window edge it was
// compared with (tested by multiplying with the power of two, which is
// exact, instead of dividing); `over` tells whether en lies above the table.
constexpr double kCloseRel = 3.814697265625e-6;  // 2^-18
template <class R, class TV>
AVM_FN int decide(const GasDev& G, const TV& T, R en, R r_sel, bool& close, bool& over) {
  using Mr = M<R>;
  const R x = en * Sel<R>::scale(G);
  int32_t kb;
  R f;
  over = !(x < Sel<R>::x_top(G));
  if (over) {
    kb = G.n_bins;
    f = R(0);
  } else {
    const R fl = Mr::floor_(x);
    kb = (int32_t)fl;
    f = x - fl;
  }
  const R g1 = R(1) - f;
  const bool in_lo = kb + 1 < T.n_lo;  // both nodes in the fast copy
  const R* tot = Sel<R>::total(G);
  const R* cz = Sel<R>::cum0(G);
  R nu_tot, c0;
  if (in_lo) {
    nu_tot = lerp<R>(T.tot[kb], T.tot[kb + 1], g1, f);
    c0 = lerp<R>(T.cum0[kb], T.cum0[kb + 1], g1, f);
  } else {
    nu_tot = over ? tot[kb] : lerp<R>(tot[kb], tot[kb + 1], g1, f);
    c0 = over ? cz[kb] : lerp<R>(cz[kb], cz[kb + 1], g1, f);
  }
  R mg = Mr::abs_(r_sel - nu_tot);
  if (r_sel >= nu_tot) {
    close = mg <= R(kCloseRel) * r_sel;
    return -1;
  }
  int c = 0;
  R dm = Mr::abs_(r_sel - c0);
  mg = dm < mg ? dm : mg;
  if (!(r_sel < c0)) {
    const int nc = G.n_ch;
    const R* row0 = Sel<R>::cum(G) + (size_t)kb * nc;
    const R* row1 = over ? row0 : row0 + nc;
    int lo = 1, hi = nc - 1;  // answer in [lo, hi]
#if AVM_SEARCH_WAYS == 4
    // four-way steps while the range is wide: three probes per step, their
    // gathers issued together (fewer dependent round trips to L2)
    while (hi - lo >= 4) {
      const int p1 = lo + ((hi - lo) >> 2), p2 = lo + ((hi - lo) >> 1), p3 = lo + (3 * (hi - lo) >> 2);
      const R a1 = row0[p1], a2 = row0[p2], a3 = row0[p3];
      const R b1 = row1[p1], b2 = row1[p2], b3 = row1[p3];
      const R c1 = over ? a1 : lerp<R>(a1, b1, g1, f);
      const R c2 = over ? a2 : lerp<R>(a2, b2, g1, f);
      const R c3 = over ? a3 : lerp<R>(a3, b3, g1, f);
      const R d1 = Mr::abs_(r_sel - c1), d2 = Mr::abs_(r_sel - c2), d3 = Mr::abs_(r_sel - c3);
      mg = d1 < mg ? d1 : mg;
      mg = d2 < mg ? d2 : mg;
      mg = d3 < mg ? d3 : mg;
      if (r_sel < c1) {
        hi = p1;
      } else if (r_sel < c2) {
        lo = p1 + 1;
        hi = p2;
      } else if (r_sel < c3) {
        lo = p2 + 1;
        hi = p3;
      } else {
        lo = p3 + 1;
      }
    }
#endif
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      const R cm = over ? row0[mid] : lerp<R>(row0[mid], row1[mid], g1, f);
      dm = Mr::abs_(r_sel - cm);
      mg = dm < mg ? dm : mg;
      if (r_sel < cm)
        hi = mid;
      else
        lo = mid + 1;
    }
    c = lo;
  }
  close = mg <= R(kCloseRel) * r_sel;
  const ChanP<R> cw = chan(G, T, c);
  const double e_lo = cw.e_lo;
  const double e_hi = cw.e_hi;
  const double ed = (double)en;
  if (sizeof(R) == 4) {
    const double dl = fabs(ed - e_lo), dh = fabs(ed - e_hi);
    const double d = dl < dh ? dl : dh;
    close = close || d <= kCloseRel * (ed > 1e-30 ? ed : 1e-30);
  }
  if (ed < e_lo || ed >= e_hi) return -2 - c;
  return c;
}

// One pass of the loop for electron `e`.  Returns STEP_DONE with `status`
// set when the electron terminates, STEP_IONISED (with the channel and
// energy in `child`) when the collision is an ionisation -- the caller then
// finishes it with complete_ionisation() before the next pass -- otherwise
// STEP_CONTINUE.
template <class R, bool kBanded, int kField, bool kSignal = false, class TV>
AVM_FN int32_t flight_step(Elec<R>& e, const GasDev& G, const TV& T, const FieldDev& F,
                           const RunParams& P, Child<R>& child, uint32_t& status,
                           const SignalDev* Q = nullptr) {
  using Mr = M<R>;
  constexpr bool kMixed = sizeof(R) == 4;
  // still inside the volume, with flights and time left?
  uint32_t st0 = region_status<R, kField>(F, e);
  st0 = st0 ? st0 : (e.k >= P.k_max ? (uint32_t)ST_ABANDONED : (e.t >= P.t_max ? (uint32_t)ST_TIME : 0u));
  if (st0) {
    status = st0;
    return STEP_DONE;
  }
  const Block w = draw(P, e.aval, e.eid, e.k, 0);
  const R u1 = Mr::uni(w.w0, w.w1);
  const R u2 = Mr::uni(w.w2, w.w3);
  R Ex = e.Ex, Ey = e.Ey, Ez = e.Ez;
  if (kField == FIELD_POLAR) {
    polar_field<R>(F, e.x, e.y, Ex, Ey);
    Ez = R(0);
  }
  const R ka = Sel<R>::k_a(P);
  const R ax = -ka * Ex, ay = -ka * Ey, az = -ka * Ez;
  // banded with B (polar-map geometry): raise the band until the helical
  // energy bound at the flight start lies below its edge
  constexpr bool kMayHaveB = !kBanded || kField == FIELD_POLAR;
  const bool helical = kBanded && kMayHaveB && F.has_b;
  HelixBound hb{};
  if (helical)
    hb = helix_bound(F, P, (double)e.vx, (double)e.vy, (double)e.vz, (double)Ex, (double)Ey, (double)Ez);
  // the current band's tables are read first, and the logarithm (which does
  // not depend on the band) is formed while they arrive
  const int32_t band0 = e.band;
  const R gam0 = kBanded ? band_gamma(G, T, band0) : Sel<R>::gamma(G);
  const R inv0 = kBanded ? band_inv(G, T, band0) : Sel<R>::inv_gamma(G);
  const R edge0 = kBanded ? band_edge(G, T, band0) : R(0);
  const R nlog = -Mr::log_s(u1);
  // the flight's band: its majorant, inverse and upper edge
  R gam = gam0, inv_gam = inv0, edge = edge0;
  if (kBanded && P.look > 0.0 && e.band < G.n_bands - 1) {
    // lookahead: raise the band to the band of the energy after `look` mean
    // free times of the current band (the flight energy, or its helical
    // bound); the choice uses only the state at the flight start
    const double s_look = P.look * (double)inv0;
    R e_look;
    if (helical) {
      const double vpar = hb.vp + hb.ap * s_look;
      const double lin = hb.p + hb.q * s_look;
      const double vperp = lin < hb.m ? lin : hb.m;
      e_look = (R)((vpar * vpar + vperp * vperp) * P.inv_2ka);
    } else {
      const R sl = (R)s_look;
      const R fx = Mr::fma(ax, sl, e.vx), fy = Mr::fma(ay, sl, e.vy), fz = Mr::fma(az, sl, e.vz);
      e_look = dot3<R>(fx, fy, fz, fx, fy, fz) * Sel<R>::inv_2ka(P);
    }
    R gl, il, el;
    const int32_t bl = band_of_tabs<R>(G, T, e_look, gl, il, el);
    if (bl > e.band) {
      e.band = bl;
      gam = gl;
      inv_gam = il;
      edge = el;
    }
  }
  if (helical) {
    const int32_t b1 = e.band;
    while (e.band < G.n_bands - 1 && (hb.vp * hb.vp + hb.p * hb.p) * P.inv_2ka >= (double)band_edge(G, T, e.band))
      e.band += 1;
    if (e.band != b1) {
      gam = band_gamma(G, T, e.band);
      inv_gam = band_inv(G, T, e.band);
    }
  }
  const R tau = nlog * inv_gam;
  R tau_end = tau;
  int cut = 0;  // 1: band edge, 2: time limit
  if (helical) {
    if (e.band < G.n_bands - 1) {
      // cut where the energy bound reaches the edge: Gamma_b holds before
      const double tc = helix_root(hb, P, (double)band_edge(G, T, e.band));
      if (tc < (double)tau_end) {
        tau_end = down_to<R>(tc);
        cut = 1;
      }
    }
  } else if (kBanded && e.band < G.n_bands - 1) {
    const R fx = Mr::fma(ax, tau, e.vx), fy = Mr::fma(ay, tau, e.vy), fz = Mr::fma(az, tau, e.vz);
    if (dot3<R>(fx, fy, fz, fx, fy, fz) * Sel<R>::inv_2ka(P) >= edge) {
      const R tc = band_crossing<R>(P, e, ax, ay, az, edge);
      if (tc < tau_end) {
        tau_end = tc;
        cut = 1;
      }
    }
  }
  const double t_left = P.t_max - e.t;
  if (t_left < (double)tau_end) {
    tau_end = (R)t_left;
    cut = 2;
  }
  // boundary first passage within (0, tau_end]
  double rx, ry, rz;
  R ux, uy, uz;
  double s_exit = (double)tau_end;
  uint32_t side = 0;
  if (kField == FIELD_SLAB) {
    side = slab_exit(e.z, (double)e.vz, (double)az, F.z_lo, F.z_hi, (double)tau_end, s_exit);
    propagate<R, kMayHaveB>(F, e, ax, ay, az, Ex, Ey, Ez, side ? (R)s_exit : tau_end, rx, ry, rz, ux, uy, uz);
    if (side) rz = side == ST_HIGH ? F.z_hi : F.z_lo;
  } else {
    propagate<R, kMayHaveB>(F, e, ax, ay, az, Ex, Ey, Ez, tau_end, rx, ry, rz, ux, uy, uz);
    const double r2 = rx * rx + ry * ry;
    if (r2 <= F.a2 || r2 >= F.b2) {
      // the flight ends on the wire or beyond the tube: the electron stops
      // here, unchanged, and the caller finds the crossing with
      // finish_exit() after the pass, for all such lanes of the wave at once
      child.pen = tau_end;
      return STEP_EXIT;
    }
  }
  if (kSignal) signal_flight<R, kMayHaveB, kField>(*Q, F, e, ax, ay, az, Ex, Ey, Ez,
                                                   e.t + (side ? s_exit : (double)tau_end));
  e.x = rx; e.y = ry; e.z = rz;
  e.vx = ux; e.vy = uy; e.vz = uz;
  e.t = e.t + (side ? s_exit : (double)tau_end);
  // the rest runs to a single exit: the outcome is kept in `st` (a
  // termination status) and `ret`, so the paths share one join
  uint32_t st = side ? side : (cut == 2 ? (uint32_t)ST_TIME : 0u);
  int32_t ret = STEP_CONTINUE;
  if (st == 0) {
    if (kBanded && cut == 1) {
      // restart at the band edge with the next majorant; the band index is
      // advanced explicitly, never re-derived from the rounded energy
      e.band += 1;
      e.n_band += 1;
      e.trace = trace_step(e.trace, e.k, TRACE_BAND);
    } else {
      // collision?
      const R en = dot3<R>(e.vx, e.vy, e.vz, e.vx, e.vy, e.vz) * Sel<R>::inv_2ka(P);
      if (!(en < Mr::inf())) {
        st = ST_ERROR;
      } else {
        bool close, over;
        int c = decide<R>(G, T, en, u2 * gam, close, over);
        if (kMixed && close) {
          // too close to call in FP32: decide again in FP64 for this state
          const double vx = (double)e.vx, vy = (double)e.vy, vz = (double)e.vz;
          const double en64 = dot3<double>(vx, vy, vz, vx, vy, vz) * P.inv_2ka;
          bool close64;
          c = decide<double>(G, global_view<double>(G), en64, u53(w.w2, w.w3) * (double)gam, close64, over);
        }
        if (over) e.n_over += 1;
        R e_band = en;  // energy whose band the next flight starts in
        if (c < 0) {
          if (c != -1) {
            e.n_masked += 1;
            e.trace = trace_step(e.trace, e.k, TRACE_MASKED + (uint32_t)(-2 - c));
          }
        } else {
          e.n_real += 1;
          e.trace = trace_step(e.trace, e.k, (uint32_t)c);
          const ChanP<R> ch = chan(G, T, c);
          const int32_t kind = ch.kind;
          if (kind == CH_ATTACHMENT) {
            st = ST_ATTACHED;
          } else if (kind == CH_IONISATION) {
            // finished by complete_ionisation() (the caller batches it)
            child.pen = en;
            child.pc = c;
            ret = STEP_IONISED;
          } else {
            const Block w1 = draw(P, e.aval, e.eid, e.k, 1);
            const R uA = Mr::uni(w1.w0, w1.w1);
            const R uB = Mr::uni(w1.w2, w1.w3);
            R e_new = en, cos_t = R(1);
            if (kind == CH_ELASTIC) {
              const R cchi = ch.angular ? R(1) - R(2) * uA / Mr::fma(R(1) - uA, en * ch.inv_screen8, R(1))
                                        : R(1) - R(2) * uA;
              e_new = en * (R(1) - ch.el_loss * (R(1) - cchi));
              cos_t = (ch.mu + cchi) * Mr::rsqrt_s(Mr::fma(ch.two_mu, cchi, ch.mu2p1));
            } else {  // excitation
              if (ch.pen_prob > R(0)) {
                // Penning transfer, decided by the first uniform of block 2:
                // the excitation and its transfer electron are finished with
                // the ionisations after the pass
                const Block w2 = draw(P, e.aval, e.eid, e.k, 2);
                if (Mr::uni(w2.w0, w2.w1) < ch.pen_prob) {
                  child.pen = en;
                  child.pc = c;
                  ret = STEP_IONISED;
                }
              }
              e_new = en - ch.loss;
              cos_t = R(1) - R(2) * uA;
            }
            if (ret == STEP_CONTINUE) {
              scatter_to<R>(e, P, T, cos_t, uB, e_new);
              e_band = e_new;
            }
          }
        }
        // one band search for the null and the real-collision paths
        if (kBanded && st == 0 && ret == STEP_CONTINUE) e.band = band_of<R>(G, T, e_band);
      }
    }
  }
  // every flight that goes on (null or masked collision, band cut, real
  // collision) advances the flight index; an ionisation's is advanced when
  // it is completed (its blocks j = 1..3 belong to this index)
  if (st == 0 && ret == STEP_CONTINUE) e.k += 1;
  status = st;
  return st ? STEP_DONE : ret;
}

// The flight of a STEP_EXIT (polar-map geometry): the electron stands at
// the flight start; its flight of duration tau_end (child.pen) ends on the
// wire or beyond the tube.  Finds the time the boundary is crossed,
// between the flight start (inside) and its end (outside): a bracket
// [lo, hi] on the inside/outside predicate, shrunk at false-position points
// of g(s) = R^2 - rho(s)^2 (wire) or rho(s)^2 - R^2 (tube), negative
// inside, with the Illinois halving of the stale end's value, and at the
// midpoint when the interpolant leaves the bracket; it stops when the
// bracket is a few ulps wide (excursions that leave and re-enter within one
// flight are not detected).  Moves the electron to the crossing (on the
// boundary surface) and returns its status, ST_WIRE or ST_TUBE.  The lanes
// of a wave that ended a pass this way search together.
template <class R, bool kBanded, bool kSignal = false>
AVM_FN uint32_t finish_exit(Elec<R>& e, const FieldDev& F, const RunParams& P, R tau_end,
                            const SignalDev* Q = nullptr) {
  constexpr bool kMayHaveB = true;  // polar-map geometry
  R Ex = e.Ex, Ey = e.Ey, Ez = e.Ez;
  polar_field<R>(F, e.x, e.y, Ex, Ey);
  Ez = R(0);
  const R ka = Sel<R>::k_a(P);
  const R ax = -ka * Ex, ay = -ka * Ey, az = -ka * Ez;
  double rx, ry, rz;
  R ux, uy, uz;
  propagate<R, kMayHaveB>(F, e, ax, ay, az, Ex, Ey, Ez, tau_end, rx, ry, rz, ux, uy, uz);
  const double r2 = rx * rx + ry * ry;
  const bool to_wire = r2 <= F.a2;
  const double R2 = to_wire ? F.a2 : F.b2;
  const double sg = to_wire ? -1.0 : 1.0;
  const double q0 = e.x * e.x + e.y * e.y;
  double lo = 0.0, hi = (double)tau_end;
  double glo = sg * (q0 - R2), ghi = sg * (r2 - R2);
  int last = 0;
  // a few ulps of the flight time in the step's precision (the trial
  // times are rounded to R for the flight formula)
  const double eps = sizeof(R) == 4 ? 2.4e-7 : 4.5e-16;
  for (int it = 0; it < 60 && hi - lo > eps * hi; ++it) {
    double c = (lo * ghi - hi * glo) / (ghi - glo);
    if (!(c > lo && c < hi)) c = 0.5 * (lo + hi);
    double mx, my, mz;
    R wx_, wy_, wz_;
    propagate<R, kMayHaveB>(F, e, ax, ay, az, Ex, Ey, Ez, (R)c, mx, my, mz, wx_, wy_, wz_);
    const double m2 = mx * mx + my * my;
    const double gc = sg * (m2 - R2);
    if (m2 <= F.a2 || m2 >= F.b2) {
      hi = c;
      ghi = gc > 0.0 ? gc : 0.0;
      if (last < 0) glo *= 0.5;
      last = -1;
    } else {
      lo = c;
      glo = gc < 0.0 ? gc : -0.0;
      if (last > 0) ghi *= 0.5;
      last = 1;
    }
  }
  const double s_exit = hi;
  propagate<R, kMayHaveB>(F, e, ax, ay, az, Ex, Ey, Ez, (R)s_exit, rx, ry, rz, ux, uy, uz);
  const double q2 = rx * rx + ry * ry;
  const uint32_t side = q2 <= F.a2 ? ST_WIRE : ST_TUBE;
  const double sc = (side == ST_WIRE ? F.a : F.b) / sqrt(q2);
  rx = rx * sc;
  ry = ry * sc;
  if (kSignal) signal_flight<R, kMayHaveB, FIELD_POLAR>(*Q, F, e, ax, ay, az, Ex, Ey, Ez, e.t + s_exit);
  e.x = rx; e.y = ry; e.z = rz;
  e.vx = ux; e.vy = uy; e.vz = uz;
  e.t = e.t + s_exit;
  return side;
}

// Finishes an ionisation (or a Penning transfer) decided by flight_step
// (blocks j = 1..3 of the electron's flight k): energy split (transfer: the
// channel's transfer energy, the electron keeps e - threshold), the
// electron's new direction, the secondary's energy, direction and id.
template <class R, bool kBanded, class TV>
AVM_FN void complete_ionisation(Elec<R>& e, const GasDev& G, const TV& T,
                                const RunParams& P, Child<R>& child) {
  using Mr = M<R>;
  const int c = child.pc;
  const ChanP<R> ch = chan(G, T, c);
  const R avail = child.pen - ch.loss;
  const Block w1 = draw(P, e.aval, e.eid, e.k, 1);
  const Block w2 = draw(P, e.aval, e.eid, e.k, 2);
  const Block w3 = draw(P, e.aval, e.eid, e.k, 3);
  const R uA = Mr::uni(w1.w0, w1.w1);
  const R uB = Mr::uni(w1.w2, w1.w3);
  const R uS = Mr::uni(w2.w0, w2.w1);
  const R uC = Mr::uni(w2.w2, w2.w3);
  const R uP = Mr::uni(w3.w0, w3.w1);
  R es, e_new;
  if (ch.kind == CH_EXCITATION) {
    // Penning transfer after an excitation: the electron keeps e - threshold
    es = ch.pen_e;
    e_new = avail;
  } else {
    es = ch.split ? ch.split_w * Mr::tan_(uS * Mr::atan_(avail * ch.atan_scale)) : uS * avail;
    e_new = avail - es;
  }
  const R ct = R(1) - R(2) * uC;
  const R st2 = Mr::fma(-ct, ct, R(1));
  const R stt = st2 > R(0) ? Mr::sqrt_s(st2) : R(0);
  R sp, cp;
  azimuth(T, uP, &sp, &cp);
  const R vs = Mr::sqrt_s(Sel<R>::two_ka(P) * es);
  child.vx = vs * (stt * cp);
  child.vy = vs * (stt * sp);
  child.vz = vs * ct;
  child.e = es;
  child.eid = (((uint64_t)w3.w3 << 32) | (uint64_t)w3.w2) & 0x7FFFFFFFFFFFFFFFull;
  e.n_ion += 1;
  scatter_to<R>(e, P, T, R(1) - R(2) * uA, uB, e_new);
  e.k += 1;
  if (kBanded) e.band = band_of<R>(G, T, e_new);
}

}  // namespace avm
