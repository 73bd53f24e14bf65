"""Seeded synthetic workloads for microscopic electron-avalanche transport.

This module only *describes inputs*: gas cross-sections sampled at the
energy nodes of a rate table, field descriptions and primary electrons.  It
holds none of the transport method's arithmetic (no rates, no majorants, no
flights, no random numbers drawn by the method), so both the FP64 oracle and
the HIP path are fed from here without sharing any of the method.

The paper (Sec. 4, case studies) measures on ANSYS GEM field maps with
Magboltz gas data, neither of which is available; the synthetic gases and
fields below stand in for them.  Five workloads are defined:

* ``toy``      - toy gas (elastic + 1 excitation + ionisation), 100 um slab,
                 30 kV/cm, 200 avalanches of one electron at rest.
* ``argon``    - argon-like gas (elastic with a Ramsauer dip and screened
                 Rutherford anisotropy, 30 excitations, ionisation with an
                 Opal-Beaty split), 128 um slab, 40 kV/cm, 1000 avalanches.
* ``batched``  - the argon-like gas, 8192 avalanches, one field per avalanche
                 drawn uniformly in 25-55 kV/cm.
* ``highgain`` - the argon-like gas plus an attachment channel below 2 eV,
                 55 kV/cm, 256 avalanches.
* ``wire``     - proportional counter (wire 25 um, tube 5 mm, 1500 V)
                 sampled to a 512 x 64 polar field map, 0.5 T axial B,
                 2048 avalanches from rho = 1 mm.

Units: cm, ns, eV, V/cm, T, cm^2, cm^-3.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

# Channel kinds, angular models, energy-split models, value kinds.  The same
# integers are used by the C-ABI and by the oracle's own C interface.
ELASTIC, EXCITATION, IONISATION, ATTACHMENT = 0, 1, 2, 3
ISOTROPIC, SCREENED_RUTHERFORD = 0, 1
SPLIT_UNIFORM, SPLIT_OPAL_BEATY = 0, 1
VALUES_SIGMA, VALUES_RATE = 0, 1

HARTREE_EV = 27.211386245988  # screening energy of the screened-Rutherford model
PENNING_QUENCHER_EV = 10.5    # ionisation potential of the synthetic Penning quencher
GAS_DENSITY = 2.5e19          # cm^-3, ~1 bar at room temperature


@dataclasses.dataclass
class Channel:
    kind: int
    values: np.ndarray            # n_bins+1 node values (cm^2, or 1/ns if values_kind==RATE)
    angular: int = ISOTROPIC
    split: int = SPLIT_UNIFORM
    values_kind: int = VALUES_SIGMA
    loss_eV: float = 0.0          # excitation threshold / ionisation potential
    e_lo_eV: float = 0.0          # validity window [e_lo, e_hi)
    e_hi_eV: float = math.inf
    mass_ratio: float = 0.0       # elastic: m_e / M
    split_w_eV: float = 0.0       # Opal-Beaty w
    screening_eV: float = 0.0     # screened Rutherford: eta(e) = screening / (8 e)
    penning_prob: float = 0.0     # excitation: probability of a Penning transfer electron
    penning_energy_eV: float = 0.0  # excitation: energy of that electron


@dataclasses.dataclass
class Gas:
    e_max_eV: float
    n_bins: int
    density_cm3: float
    channels: List[Channel]
    band_bins: int = 0            # 0: one band (global majorant only)


@dataclasses.dataclass
class SlabField:
    z_lo_cm: float
    z_hi_cm: float
    E_vcm: np.ndarray             # shape (n_aval, 3) or (1, 3): field vector per avalanche
    B_T: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(3))


@dataclasses.dataclass
class PolarMapField:
    a_cm: float                   # wire radius
    b_cm: float                   # tube radius
    E_r: np.ndarray               # float32 [n_r][n_phi], V/cm
    E_phi: np.ndarray             # float32 [n_r][n_phi], V/cm
    B_T: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(3))


@dataclasses.dataclass
class Workload:
    name: str
    gas: Gas
    field: object
    primaries: np.ndarray         # structured array, PRIMARY_DTYPE
    n_aval: int
    seed: int
    description: str


# One primary electron: start position, time and kinetic energy, direction of
# motion (normalised by the consumer; ignored at zero energy) and avalanche
# id.  Layout matches the primary record of the C-ABI (72 bytes).
PRIMARY_DTYPE = np.dtype([
    ("x", "<f8"), ("y", "<f8"), ("z", "<f8"), ("t", "<f8"), ("e", "<f8"),
    ("dx", "<f8"), ("dy", "<f8"), ("dz", "<f8"),
    ("aval", "<u4"), ("_pad", "<u4"),
], align=True)
assert PRIMARY_DTYPE.itemsize == 72


def energy_nodes(e_max_eV: float, n_bins: int) -> np.ndarray:
    """Node energies k*E_max/N, k = 0..N (integer product, then a divide)."""
    k = np.arange(n_bins + 1, dtype=np.float64)
    return (k * e_max_eV) / float(n_bins)


def primaries_at_rest(n: int, x=0.0, y=0.0, z=0.0) -> np.ndarray:
    p = np.zeros(n, dtype=PRIMARY_DTYPE)
    p["x"], p["y"], p["z"] = x, y, z
    p["dz"] = 1.0
    p["aval"] = np.arange(n, dtype=np.uint32)
    return p


# ---------------------------------------------------------------------------
# Gases
# ---------------------------------------------------------------------------

def toy_gas(e_max_eV: float = 200.0, n_bins: int = 2000, band_bins: int = 0) -> Gas:
    """Toy gas: constant isotropic elastic 1e-15 cm^2 (m/M = 1.37e-5), one
    excitation at 11.5 eV with a 2e-17 cm^2 step, ionisation at 15.7 eV rising
    linearly to 3e-16 cm^2 at 100 eV then flat, uniform energy split."""
    e = energy_nodes(e_max_eV, n_bins)
    el = np.full_like(e, 1e-15)
    ex = np.where(e >= 11.5, 2e-17, 0.0)
    ion = np.where(e >= 15.7, 3e-16 * np.minimum((e - 15.7) / (100.0 - 15.7), 1.0), 0.0)
    chans = [
        Channel(ELASTIC, el, angular=ISOTROPIC, mass_ratio=1.37e-5),
        Channel(EXCITATION, ex, loss_eV=11.5, e_lo_eV=11.5),
        Channel(IONISATION, ion, loss_eV=15.7, e_lo_eV=15.7, split=SPLIT_UNIFORM),
    ]
    return Gas(e_max_eV, n_bins, GAS_DENSITY, chans, band_bins)


def argon_like_gas(e_max_eV: float = 400.0, n_bins: int = 20000,
                   attachment: bool = False, band_bins: int = 0,
                   penning: Optional[float] = None) -> Gas:
    """Synthetic argon-like gas.

    * elastic 7e-16*(e/10)^0.5/(1+(0.25/e)^2) cm^2 times a Ramsauer dip
      1-0.9*exp(-(e-0.23)^2/(2*0.1^2)), screened-Rutherford anisotropy with
      eta = E_H/(8e), m/M = 1.37e-5;
    * 30 excitations with thresholds 11.5 + i*3.5/29 eV, sigma =
      5e-18*ln(x)/x for x = e/thr > 1;
    * ionisation at 15.7 eV, linear to 3e-16 cm^2 at 100 eV then flat,
      Opal-Beaty split with w = 10 eV;
    * optionally attachment 1e-18 cm^2 for e < 2 eV;
    * optionally Penning transfer: every excitation level passes its energy
      on with probability ``penning`` to a quencher of ionisation potential
      10.5 eV, freeing an electron of energy thr - 10.5 eV (synthetic: no
      transfer data are available here).
    """
    e = energy_nodes(e_max_eV, n_bins)
    with np.errstate(divide="ignore", invalid="ignore"):
        base = 7e-16 * np.sqrt(e / 10.0) / (1.0 + (0.25 / e) ** 2)
    base[e == 0.0] = 0.0
    ramsauer = 1.0 - 0.9 * np.exp(-((e - 0.23) ** 2) / (2.0 * 0.1 ** 2))
    chans = [Channel(ELASTIC, base * ramsauer, angular=SCREENED_RUTHERFORD,
                     mass_ratio=1.37e-5, screening_eV=HARTREE_EV)]
    for i in range(30):
        thr = 11.5 + i * 3.5 / 29.0
        x = e / thr
        with np.errstate(divide="ignore", invalid="ignore"):
            s = np.where(x > 1.0, 5e-18 * np.log(x) / x, 0.0)
        chans.append(Channel(EXCITATION, s, loss_eV=thr, e_lo_eV=thr,
                             penning_prob=0.0 if penning is None else float(penning),
                             penning_energy_eV=thr - PENNING_QUENCHER_EV))
    ion = np.where(e >= 15.7, 3e-16 * np.minimum((e - 15.7) / (100.0 - 15.7), 1.0), 0.0)
    chans.append(Channel(IONISATION, ion, loss_eV=15.7, e_lo_eV=15.7,
                         split=SPLIT_OPAL_BEATY, split_w_eV=10.0))
    if attachment:
        att = np.where(e < 2.0, 1e-18, 0.0)
        chans.append(Channel(ATTACHMENT, att, e_lo_eV=0.0, e_hi_eV=2.0))
    return Gas(e_max_eV, n_bins, GAS_DENSITY, chans, band_bins)


def constant_rate_gas(nu_per_ns: float, mass_ratio: float = 0.0,
                      e_max_eV: float = 1000.0, n_bins: int = 100) -> Gas:
    """One isotropic elastic channel with a rate that is the same at every
    node (given directly as a rate, 1/ns): the constant-collision-frequency
    model of the Langevin closed forms."""
    vals = np.full(n_bins + 1, float(nu_per_ns))
    ch = Channel(ELASTIC, vals, angular=ISOTROPIC, values_kind=VALUES_RATE,
                 mass_ratio=mass_ratio)
    return Gas(e_max_eV, n_bins, GAS_DENSITY, [ch], 0)


# ---------------------------------------------------------------------------
# Fields
# ---------------------------------------------------------------------------

def slab(gap_cm: float, E_z_vcm, B_T=(0.0, 0.0, 0.0)) -> SlabField:
    """Parallel-plate gap [0, gap).  ``E_z_vcm`` is the magnitude of the field
    that accelerates electrons towards +z, one value or one per avalanche; the
    field vector is therefore (0, 0, -E)."""
    E = np.atleast_1d(np.asarray(E_z_vcm, dtype=np.float64))
    vec = np.zeros((E.size, 3))
    vec[:, 2] = -E
    return SlabField(0.0, float(gap_cm), vec, np.asarray(B_T, dtype=np.float64))


def wire_polar_map(a_cm=25e-4, b_cm=0.5, volts=1500.0, n_r=512, n_phi=64,
                   B_T=(0.0, 0.0, 0.5)) -> PolarMapField:
    """E = V/(r ln(b/a)) radially outward, sampled at log-spaced radii
    r_i = a (b/a)^(i/(n_r-1)) and n_phi azimuths, stored as float32."""
    i = np.arange(n_r, dtype=np.float64)
    r = a_cm * (b_cm / a_cm) ** (i / (n_r - 1))
    er = volts / (r * math.log(b_cm / a_cm))
    E_r = np.repeat(er[:, None], n_phi, axis=1).astype(np.float32)
    E_phi = np.zeros((n_r, n_phi), dtype=np.float32)
    return PolarMapField(a_cm, b_cm, E_r, E_phi, np.asarray(B_T, dtype=np.float64))


def wire_crossed_map(a_cm=25e-4, b_cm=0.5, volts=1500.0, E0_vcm=500.0, n_r=512, n_phi=64,
                     B_T=(0.0, 0.0, 0.5)) -> PolarMapField:
    """The wire field plus a uniform transverse field E0 along +x, sampled in
    polar components at the same nodes: E_r = V/(r ln(b/a)) + E0 cos(phi),
    E_phi = -E0 sin(phi) (float32).  It depends on phi and has E_phi != 0,
    and its Cartesian closed form is V/(r^2 ln(b/a)) (x, y) + (E0, 0)."""
    i = np.arange(n_r, dtype=np.float64)
    r = a_cm * (b_cm / a_cm) ** (i / (n_r - 1))
    phi = 2.0 * math.pi * np.arange(n_phi, dtype=np.float64) / n_phi
    er = volts / (r * math.log(b_cm / a_cm))
    E_r = (er[:, None] + E0_vcm * np.cos(phi)[None, :]).astype(np.float32)
    E_phi = np.repeat((-E0_vcm * np.sin(phi))[None, :], n_r, axis=0).astype(np.float32)
    return PolarMapField(a_cm, b_cm, E_r, E_phi, np.asarray(B_T, dtype=np.float64))


# ---------------------------------------------------------------------------
# The five workloads
# ---------------------------------------------------------------------------

def toy(n_aval: int = 200, band_bins: int = 0) -> Workload:
    return Workload("toy", toy_gas(band_bins=band_bins), slab(100e-4, 30e3),
                    primaries_at_rest(n_aval), n_aval, 1,
                    "toy gas, 100 um slab, 30 kV/cm, 1 primary at rest per avalanche")


def argon(n_aval: int = 1000, band_bins: int = 0) -> Workload:
    return Workload("argon", argon_like_gas(band_bins=band_bins), slab(128e-4, 40e3),
                    primaries_at_rest(n_aval), n_aval, 2,
                    "argon-like gas, 128 um slab, 40 kV/cm, 1 primary at rest per avalanche")


def batched(n_aval: int = 8192, band_bins: int = 0) -> Workload:
    E = np.random.default_rng(3).uniform(25e3, 55e3, 8192)[:n_aval]
    return Workload("batched", argon_like_gas(band_bins=band_bins), slab(128e-4, E),
                    primaries_at_rest(n_aval), n_aval, 3,
                    "argon-like gas, 128 um slab, per-avalanche E ~ U(25,55) kV/cm")


def highgain(n_aval: int = 256, band_bins: int = 0) -> Workload:
    return Workload("highgain", argon_like_gas(attachment=True, band_bins=band_bins),
                    slab(128e-4, 55e3), primaries_at_rest(n_aval), n_aval, 4,
                    "argon-like gas + attachment below 2 eV, 128 um slab, 55 kV/cm")


def wire(n_aval: int = 2048, band_bins: int = 0) -> Workload:
    phi = np.random.default_rng(5).uniform(0.0, 2.0 * math.pi, 2048)[:n_aval]
    p = primaries_at_rest(n_aval)
    p["x"] = 0.1 * np.cos(phi)
    p["y"] = 0.1 * np.sin(phi)
    return Workload("wire", argon_like_gas(band_bins=band_bins), wire_polar_map(), p, n_aval, 5,
                    "argon-like gas, wire counter 25 um / 5 mm / 1500 V polar map, 0.5 T axial B")


def wire_crossed(n_aval: int = 256, band_bins: int = 0, rho_cm: float = 0.1) -> Workload:
    """The wire chamber with an extra uniform transverse field of 500 V/cm
    (a phi-dependent map with E_phi != 0), primaries at rest on a circle of
    radius rho_cm at uniform azimuths (default_rng(7))."""
    phi = np.random.default_rng(7).uniform(0.0, 2.0 * math.pi, n_aval)
    p = primaries_at_rest(n_aval)
    p["x"] = rho_cm * np.cos(phi)
    p["y"] = rho_cm * np.sin(phi)
    return Workload("wire_crossed", argon_like_gas(band_bins=band_bins), wire_crossed_map(), p,
                    n_aval, 7, "argon-like gas, wire counter polar map plus 500 V/cm along x, 0.5 T axial B")


def penning(n_aval: int = 500, band_bins: int = 0, prob: float = 0.05) -> Workload:
    return Workload("penning", argon_like_gas(band_bins=band_bins, penning=prob), slab(128e-4, 40e3),
                    primaries_at_rest(n_aval), n_aval, 6,
                    f"argon-like gas with Penning transfer p = {prob} (quencher 10.5 eV), 128 um slab, 40 kV/cm")


WORKLOADS = {"toy": toy, "argon": argon, "batched": batched, "highgain": highgain, "wire": wire,
             "penning": penning}


def subset_primaries(prim: np.ndarray, modulus: int, residue: int = 0) -> np.ndarray:
    """Indices of the primaries whose avalanche id is congruent to ``residue``
    modulo ``modulus`` (avalanche-deterministic subsets replay exactly)."""
    return np.nonzero((prim["aval"] % modulus) == residue)[0]
