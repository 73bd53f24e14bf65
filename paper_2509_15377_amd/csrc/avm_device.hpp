// avm_device.hpp -- device side of microscopic electron-avalanche transport
// for gfx950 (CDNA4, wave64).
//
// One call of `flight_step` is one pass of the AvalancheMicroscopic loop of
// the paper's Fig. 2 ("position valid? -> find E and add a random time step
// -> collision? -> ionisation or attachment?") for one electron held in
// registers.  The free flight is a null-collision flight (Skullerud, cited in
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

namespace avm {

// electron status codes (non-zero: terminated)
enum : uint32_t {
  ST_ACTIVE = 0, ST_LOW = 1, ST_HIGH = 2, ST_ATTACHED = 3, ST_WIRE = 4,
  ST_TUBE = 5, ST_TIME = 6, ST_ABANDONED = 7, ST_ERROR = 8
};
enum : int32_t { CH_ELASTIC = 0, CH_EXCITATION = 1, CH_IONISATION = 2, CH_ATTACHMENT = 3 };

// Per-channel scattering parameters (device copy, read on real collisions).
struct ChanDev {
  int32_t kind, angular, split, _pad;
  double loss, e_lo, e_hi;
  double mu;            // m/M
  double el_loss;       // 2 mu / (1 + mu)^2
  double mu2p1;         // 1 + mu^2
  double two_mu;        // 2 mu
  double split_w;       // Opal-Beaty w
  double atan_scale;    // 1 / (2 w)
  double inv_screen8;   // 8 / screening (1/eta = 8 e / screening)
};

struct GasDev {
  const double* cum;        // [(n_bins+1) * n_ch] node-major cumulative rates, 1/ns
  const double* total;      // [n_bins+1] total rate at the nodes
  const double* band_gamma; // [n_bands]
  const double* band_inv;   // [n_bands] 1 / Gamma_b
  const double* band_edge;  // [n_bands] upper edge (eV), +inf for the last
  const ChanDev* ch;        // [n_ch]
  double scale;             // n_bins / E_max
  double gamma, inv_gamma;
  double band_scale;        // n_bins / (E_max * band_bins): first guess of the band
  int32_t n_bins, n_ch, n_bands, band_bins;
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
  uint64_t budget_ticks;    // wall_clock64() ticks a transport kernel may run
};

// ---------------------------------------------------------------------------
// Philox4x32-10
// ---------------------------------------------------------------------------
struct Block { uint32_t w0, w1, w2, w3; };

AVM_FN Block philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
    const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
    const uint32_t n0 = hi1 ^ c1 ^ k0;
    const uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return Block{c0, c1, c2, c3};
}

AVM_FN Block draw(const RunParams& p, uint32_t aval, uint64_t eid, uint32_t k,
                                      uint32_t j) {
  return philox(4u * k + j, aval, (uint32_t)eid, (uint32_t)(eid >> 32), p.key0, p.key1);
}

// 53-bit uniform in (0, 1]: ((hi >> 5) 2^26 + (lo >> 6) + 1) 2^-53, every
// intermediate an exact integer in binary64.
AVM_FN double u53(uint32_t hi, uint32_t lo) {
  return __builtin_fma((double)(hi >> 5), 67108864.0, (double)((lo >> 6) + 1u)) *
         1.1102230246251565e-16;
}

// ---------------------------------------------------------------------------
// geometry helpers
// ---------------------------------------------------------------------------
AVM_FN double dot3(double ax, double ay, double az, double bx, double by,
                                       double bz) {
  return ax * bx + ay * by + az * bz;
}

// Direction of (vx, vy, vz) turned by polar angle theta (cos_t) and azimuth
// phi.  The transverse length s = sqrt(dx^2 + dy^2) avoids the cancellation
// of sqrt(1 - dz^2) next to the poles, so |d'| = 1 to rounding.
AVM_FN void turn(double dx, double dy, double dz, double cos_t, double phi,
                                     double& ox, double& oy, double& oz) {
  const double st2 = 1.0 - cos_t * cos_t;
  const double sin_t = st2 > 0.0 ? sqrt(st2) : 0.0;
  double sp, cp;
  sincos(phi, &sp, &cp);
  const double s = sqrt(dx * dx + dy * dy);
  if (s > 1e-12) {
    const double inv_s = 1.0 / s;
    ox = dx * cos_t + sin_t * (dx * dz * cp - dy * sp) * inv_s;
    oy = dy * cos_t + sin_t * (dy * dz * cp + dx * sp) * inv_s;
    oz = dz * cos_t - s * sin_t * cp;
  } else {
    ox = sin_t * cp;
    oy = sin_t * sp;
    oz = (dz < 0.0 ? -1.0 : 1.0) * cos_t;
  }
}

// Real roots of A s^2 + B s + C = 0 in ascending order (stable form).
AVM_FN int roots2(double A, double B, double C, double& r1, double& r2) {
  if (A == 0.0) {
    if (B == 0.0) return 0;
    r1 = -C / B;
    return 1;
  }
  const double disc = B * B - 4.0 * A * C;
  if (disc < 0.0) return 0;
  const double sq = sqrt(disc);
  const double q = -0.5 * (B + (B >= 0.0 ? sq : -sq));
  if (q == 0.0) {
    r1 = 0.0;
    r2 = 0.0;
  } else {
    r1 = q / A;
    r2 = C / q;
  }
  if (r1 > r2) {
    const double t = r1;
    r1 = r2;
    r2 = t;
  }
  return 2;
}

// First exit time in (0, T] of z(s) = z0 + vz s + az s^2 / 2 from the slab
// [zlo, zhi): arrival at zhi, or a crossing below zlo with dz/ds < 0 (s = 0
// counts when sitting on zlo moving down).  A cheap bound on the extremes of
// the parabola over [0, T] rules out the common no-exit case before any root
// is taken.
AVM_FN uint32_t slab_exit(double z0, double vz, double az, double zlo,
                                              double zhi, double T, double& s_exit) {
  const double zT = z0 + vz * T + 0.5 * az * T * T;
  double zmin = z0 < zT ? z0 : zT;
  double zmax = z0 > zT ? z0 : zT;
  if (az != 0.0) {
    const double sv = -vz / az;  // vertex
    if (sv > 0.0 && sv < T) {
      const double zv = z0 + vz * sv + 0.5 * az * sv * sv;
      zmin = zmin < zv ? zmin : zv;
      zmax = zmax > zv ? zmax : zv;
    }
  }
  // margin: a relative 1e-12 of the coordinates keeps the filter conservative
  const double m = 1e-12 * (fabs(z0) + fabs(zhi) + fabs(zlo) + fabs(vz * T) + fabs(az * T * T));
  if (zmax < zhi - m && zmin > zlo + m) return 0;
  double best = __builtin_inf();
  uint32_t side = 0;
  double r1 = 0.0, r2 = 0.0;
  int n = roots2(0.5 * az, vz, z0 - zhi, r1, r2);
  if (n >= 1 && r1 > 0.0) {
    best = r1;
    side = ST_HIGH;
  } else if (n == 2 && r2 > 0.0) {
    best = r2;
    side = ST_HIGH;
  }
  n = roots2(0.5 * az, vz, z0 - zlo, r1, r2);
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
AVM_FN void polar_field(const FieldDev& F, double x, double y, double& Ex,
                                            double& Ey) {
  const double rho = sqrt(x * x + y * y);
  if (!(rho > 0.0)) {
    Ex = 0.0;
    Ey = 0.0;
    return;
  }
  double u = (log(rho) - F.ln_a) * F.inv_dlog;
  const double umax = (double)(F.n_r - 1);
  u = u < 0.0 ? 0.0 : (u > umax ? umax : u);
  int i = (int)floor(u);
  i = i > F.n_r - 2 ? F.n_r - 2 : i;
  const double fr = u - (double)i;
  double phi = atan2(y, x);
  if (phi < 0.0) phi += 6.283185307179586;
  const double w = phi * (0.15915494309189535 * (double)F.n_phi);
  const double wf = floor(w);
  const double fp = w - wf;
  int j0 = (int)wf;
  j0 = j0 >= F.n_phi ? j0 - F.n_phi : j0;
  const int j1 = j0 + 1 == F.n_phi ? 0 : j0 + 1;
  const int np = F.n_phi;
  const double w00 = (1.0 - fr) * (1.0 - fp), w01 = (1.0 - fr) * fp;
  const double w10 = fr * (1.0 - fp), w11 = fr * fp;
  const float* R = F.Er;
  const float* P = F.Ephi;
  const double er = w00 * (double)R[i * np + j0] + w01 * (double)R[i * np + j1] +
                    w10 * (double)R[(i + 1) * np + j0] + w11 * (double)R[(i + 1) * np + j1];
  const double ep = w00 * (double)P[i * np + j0] + w01 * (double)P[i * np + j1] +
                    w10 * (double)P[(i + 1) * np + j0] + w11 * (double)P[(i + 1) * np + j1];
  const double inv = 1.0 / rho;
  const double c = x * inv, s = y * inv;
  Ex = er * c - ep * s;
  Ey = er * s + ep * c;
}

// ---------------------------------------------------------------------------
// electron state and one pass of the transport loop
// ---------------------------------------------------------------------------
struct Elec {
  double x, y, z, t, vx, vy, vz;
  uint64_t eid;
  uint32_t aval, k;
  int32_t band;
  uint32_t n_real, n_ion, n_null, n_masked, n_band, n_over;
  double Ex, Ey, Ez;  // slab: the avalanche's field, loaded once per electron
};

struct Child {
  double vx, vy, vz, e;
  uint64_t eid;
};

enum : int32_t { STEP_CONTINUE = 0, STEP_IONISED = 1, STEP_DONE = 2 };

AVM_FN int32_t band_of(const GasDev& G, double e) {
  int32_t b = (int32_t)(e * G.band_scale);
  b = b < 0 ? 0 : (b > G.n_bands - 1 ? G.n_bands - 1 : b);
  while (b < G.n_bands - 1 && !(e < G.band_edge[b])) ++b;
  while (b > 0 && e < G.band_edge[b - 1]) --b;
  return b;
}

AVM_FN uint32_t region_status(const FieldDev& F, const Elec& e) {
  if (F.kind == FIELD_SLAB) {
    if (e.z < F.z_lo) return ST_LOW;
    if (e.z >= F.z_hi) return ST_HIGH;
    return 0;
  }
  const double r2 = e.x * e.x + e.y * e.y;
  if (r2 <= F.a2) return ST_WIRE;
  if (r2 >= F.b2) return ST_TUBE;
  return 0;
}

// Free flight of duration s from (r, v) with the field frozen at E.
AVM_FN void propagate(const FieldDev& F, const RunParams& P, const Elec& e,
                                          double ax, double ay, double az, double Ex, double Ey,
                                          double Ez, double s, double& rx, double& ry, double& rz,
                                          double& ux, double& uy, double& uz) {
  if (!F.has_b) {
    const double hs2 = 0.5 * s * s;
    rx = e.x + e.vx * s + ax * hs2;
    ry = e.y + e.vy * s + ay * hs2;
    rz = e.z + e.vz * s + az * hs2;
    ux = e.vx + ax * s;
    uy = e.vy + ay * s;
    uz = e.vz + az * s;
    return;
  }
  // constant E and B: uniform acceleration along B, E x B drift plus
  // gyration across it
  const double bx = F.bh[0], by = F.bh[1], bz = F.bh[2];
  const double vpar = dot3(e.vx, e.vy, e.vz, bx, by, bz);
  const double apar = dot3(ax, ay, az, bx, by, bz);
  const double wx = F.wd_scale * (Ey * F.Bv[2] - Ez * F.Bv[1]);
  const double wy = F.wd_scale * (Ez * F.Bv[0] - Ex * F.Bv[2]);
  const double wz = F.wd_scale * (Ex * F.Bv[1] - Ey * F.Bv[0]);
  const double u0x = (e.vx - vpar * bx) - wx;
  const double u0y = (e.vy - vpar * by) - wy;
  const double u0z = (e.vz - vpar * bz) - wz;
  const double cx = by * u0z - bz * u0y;
  const double cy = bz * u0x - bx * u0z;
  const double cz = bx * u0y - by * u0x;
  const double ph = F.omega * s;
  double sn, cs;
  sincos(ph, &sn, &cs);
  const double sh = sin(0.5 * ph);
  const double omc = 2.0 * sh * sh;
  const double along = vpar * s + 0.5 * apar * s * s;
  const double a1 = sn * F.inv_omega, a2 = omc * F.inv_omega;
  rx = e.x + along * bx + wx * s + a1 * u0x + a2 * cx;
  ry = e.y + along * by + wy * s + a1 * u0y + a2 * cy;
  rz = e.z + along * bz + wz * s + a1 * u0z + a2 * cz;
  const double vp = vpar + apar * s;
  ux = vp * bx + wx + cs * u0x + sn * cx;
  uy = vp * by + wy + cs * u0y + sn * cy;
  uz = vp * bz + wz + cs * u0z + sn * cz;
}

// Smallest s >= 0 at which |v + a s|^2 reaches 2 k_a edge (energy at the band edge).
AVM_FN double band_crossing(const RunParams& P, const Elec& e, double ax,
                                                double ay, double az, double edge) {
  const double C = dot3(e.vx, e.vy, e.vz, e.vx, e.vy, e.vz) - P.two_ka * edge;
  if (C >= 0.0) return 0.0;
  double r1 = 0.0, r2 = 0.0;
  const int n = roots2(dot3(ax, ay, az, ax, ay, az), 2.0 * dot3(e.vx, e.vy, e.vz, ax, ay, az), C,
                       r1, r2);
  if (n >= 1 && r1 >= 0.0) return r1;
  if (n == 2 && r2 >= 0.0) return r2;
  return 0.0;
}

// One pass of the loop for electron `e`.  Returns STEP_DONE with `status`
// set when the electron terminates, STEP_IONISED with `child` filled when an
// ionisation spawned a secondary (the electron itself continues), otherwise
// STEP_CONTINUE.
template <bool kBanded, int kField>
AVM_FN int32_t flight_step(Elec& e, const GasDev& G, const FieldDev& F,
                                               const RunParams& P, Child& child,
                                               uint32_t& status) {
  // position valid?
  status = region_status(F, e);
  if (status) return STEP_DONE;
  if (e.k >= P.k_max) {
    status = ST_ABANDONED;
    return STEP_DONE;
  }
  if (e.t >= P.t_max) {
    status = ST_TIME;
    return STEP_DONE;
  }
  const Block w = draw(P, e.aval, e.eid, e.k, 0);
  const double u1 = u53(w.w0, w.w1);
  const double u2 = u53(w.w2, w.w3);
  double Ex = e.Ex, Ey = e.Ey, Ez = e.Ez;
  if (kField == FIELD_POLAR) {
    polar_field(F, e.x, e.y, Ex, Ey);
    Ez = 0.0;
  }
  const double ax = -P.k_a * Ex, ay = -P.k_a * Ey, az = -P.k_a * Ez;
  const double gam = kBanded ? G.band_gamma[e.band] : G.gamma;
  const double inv_gam = kBanded ? G.band_inv[e.band] : G.inv_gamma;
  const double tau = -log(u1) * inv_gam;
  double tau_end = tau;
  int cut = 0;  // 1: band edge, 2: time limit
  if (kBanded && e.band < G.n_bands - 1) {
    const double fx = e.vx + ax * tau, fy = e.vy + ay * tau, fz = e.vz + az * tau;
    const double edge = G.band_edge[e.band];
    if (dot3(fx, fy, fz, fx, fy, fz) * P.inv_2ka >= edge) {
      const double tc = band_crossing(P, e, ax, ay, az, edge);
      if (tc < tau_end) {
        tau_end = tc;
        cut = 1;
      }
    }
  }
  const double t_left = P.t_max - e.t;
  if (t_left < tau_end) {
    tau_end = t_left;
    cut = 2;
  }
  // boundary first passage within (0, tau_end]
  double rx, ry, rz, ux, uy, uz;
  double s_exit = tau_end;
  uint32_t side = 0;
  if (kField == FIELD_SLAB) {
    side = slab_exit(e.z, e.vz, az, F.z_lo, F.z_hi, tau_end, s_exit);
    propagate(F, P, e, ax, ay, az, Ex, Ey, Ez, side ? s_exit : tau_end, rx, ry, rz, ux, uy, uz);
    if (side) rz = side == ST_HIGH ? F.z_hi : F.z_lo;
  } else {
    propagate(F, P, e, ax, ay, az, Ex, Ey, Ez, tau_end, rx, ry, rz, ux, uy, uz);
    const double r2 = rx * rx + ry * ry;
    if (r2 <= F.a2 || r2 >= F.b2) {
      // bisection on the inside/outside predicate (excursions that leave
      // and re-enter within one flight are not detected)
      double lo = 0.0, hi = tau_end;
      for (int it = 0; it < 60; ++it) {
        const double mid = 0.5 * (lo + hi);
        double mx, my, mz, wx_, wy_, wz_;
        propagate(F, P, e, ax, ay, az, Ex, Ey, Ez, mid, mx, my, mz, wx_, wy_, wz_);
        const double m2 = mx * mx + my * my;
        if (m2 <= F.a2 || m2 >= F.b2)
          hi = mid;
        else
          lo = mid;
      }
      s_exit = hi;
      propagate(F, P, e, ax, ay, az, Ex, Ey, Ez, s_exit, rx, ry, rz, ux, uy, uz);
      const double q2 = rx * rx + ry * ry;
      side = q2 <= F.a2 ? ST_WIRE : ST_TUBE;
      const double sc = (side == ST_WIRE ? F.a : F.b) / sqrt(q2);
      rx = rx * sc;
      ry = ry * sc;
    }
  }
  e.x = rx; e.y = ry; e.z = rz;
  e.vx = ux; e.vy = uy; e.vz = uz;
  if (side) {
    e.t = e.t + s_exit;
    status = side;
    return STEP_DONE;
  }
  e.t = e.t + tau_end;
  if (cut == 2) {
    status = ST_TIME;
    return STEP_DONE;
  }
  if (kBanded && cut == 1) {
    // restart at the band edge with the next majorant; the band index is
    // advanced explicitly, never re-derived from the rounded energy
    e.band += 1;
    e.n_band += 1;
    e.k += 1;
    return STEP_CONTINUE;
  }
  // collision?
  const double en = dot3(e.vx, e.vy, e.vz, e.vx, e.vy, e.vz) * P.inv_2ka;
  if (!(en < __builtin_inf())) {
    status = ST_ERROR;
    return STEP_DONE;
  }
  const double x = en * G.scale;
  int32_t kb;
  double f;
  const bool over = !(x < (double)G.n_bins);
  if (over) {
    kb = G.n_bins;
    f = 0.0;
    e.n_over += 1;
  } else {
    const double fl = floor(x);
    kb = (int32_t)fl;
    f = x - fl;
  }
  const double g1 = 1.0 - f;
  const double nu_tot = over ? G.total[kb] : g1 * G.total[kb] + f * G.total[kb + 1];
  const double r_sel = u2 * gam;
  if (r_sel >= nu_tot) {
    e.n_null += 1;
    e.k += 1;
    if (kBanded) e.band = band_of(G, en);
    return STEP_CONTINUE;
  }
  // channel: the smallest c with r_sel < interpolated cumulative rate c.
  // Channel 0 first (the elastic channel dominates), then a binary search
  // over the rest; the interpolated cumulative rates are non-decreasing in c.
  const int nc = G.n_ch;
  const double* row0 = G.cum + (size_t)kb * nc;
  const double* row1 = over ? row0 : row0 + nc;
  auto cum_at = [&](int c) -> double { return over ? row0[c] : g1 * row0[c] + f * row1[c]; };
  int c = 0;
  if (!(r_sel < cum_at(0))) {
    int lo = 1, hi = nc - 1;  // answer in [lo, hi]
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (r_sel < cum_at(mid))
        hi = mid;
      else
        lo = mid + 1;
    }
    c = lo;
  }
  const ChanDev& ch = G.ch[c];
  if (en < ch.e_lo || en >= ch.e_hi) {
    e.n_masked += 1;
    e.k += 1;
    if (kBanded) e.band = band_of(G, en);
    return STEP_CONTINUE;
  }
  e.n_real += 1;
  if (ch.kind == CH_ATTACHMENT) {
    status = ST_ATTACHED;
    return STEP_DONE;
  }
  // direction before the collision
  const double sp0 = sqrt(dot3(e.vx, e.vy, e.vz, e.vx, e.vy, e.vz));
  double dx = 0.0, dy = 0.0, dz = 1.0;
  if (sp0 > 0.0) {
    const double inv = 1.0 / sp0;
    dx = e.vx * inv;
    dy = e.vy * inv;
    dz = e.vz * inv;
  }
  const Block w1 = draw(P, e.aval, e.eid, e.k, 1);
  const double uA = u53(w1.w0, w1.w1);
  const double uB = u53(w1.w2, w1.w3);
  const double phi = 6.283185307179586 * uB;
  double e_new, cos_t;
  int32_t ret = STEP_CONTINUE;
  if (ch.kind == CH_ELASTIC) {
    const double cchi = ch.angular ? 1.0 - 2.0 * uA / (1.0 + (1.0 - uA) * (en * ch.inv_screen8))
                                   : 1.0 - 2.0 * uA;
    e_new = en * (1.0 - ch.el_loss * (1.0 - cchi));
    cos_t = (ch.mu + cchi) / sqrt(ch.mu2p1 + ch.two_mu * cchi);
  } else if (ch.kind == CH_EXCITATION) {
    e_new = en - ch.loss;
    cos_t = 1.0 - 2.0 * uA;
  } else {
    const double avail = en - ch.loss;
    const Block w2 = draw(P, e.aval, e.eid, e.k, 2);
    const Block w3 = draw(P, e.aval, e.eid, e.k, 3);
    const double uS = u53(w2.w0, w2.w1);
    const double uC = u53(w2.w2, w2.w3);
    const double uP = u53(w3.w0, w3.w1);
    const double es = ch.split ? ch.split_w * tan(uS * atan(avail * ch.atan_scale)) : uS * avail;
    e_new = avail - es;
    cos_t = 1.0 - 2.0 * uA;
    const double ct = 1.0 - 2.0 * uC;
    const double st2 = 1.0 - ct * ct;
    const double stt = st2 > 0.0 ? sqrt(st2) : 0.0;
    double sp, cp;
    sincos(6.283185307179586 * uP, &sp, &cp);
    const double vs = sqrt(P.two_ka * es);
    child.vx = vs * (stt * cp);
    child.vy = vs * (stt * sp);
    child.vz = vs * ct;
    child.e = es;
    child.eid = (((uint64_t)w3.w3 << 32) | (uint64_t)w3.w2) & 0x7FFFFFFFFFFFFFFFull;
    e.n_ion += 1;
    ret = STEP_IONISED;
  }
  double ox, oy, oz;
  turn(dx, dy, dz, cos_t, phi, ox, oy, oz);
  const double sp1 = sqrt(P.two_ka * e_new);
  e.vx = sp1 * ox;
  e.vy = sp1 * oy;
  e.vz = sp1 * oz;
  e.k += 1;
  if (kBanded) e.band = band_of(G, e_new);
  return ret;
}

}  // namespace avm
