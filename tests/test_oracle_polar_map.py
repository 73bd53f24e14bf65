"""Pin of the oracle's polar field map (orc_field_eval) on a map that
depends on the azimuth and has E_phi != 0: the wire field plus a uniform
transverse field E0 along x, sampled in polar components.  Its Cartesian
closed form is known, so:

* at the map nodes the oracle returns the closed form to the float32
  rounding of the stored values;
* anywhere in the map it stays within the error bound of bilinear
  interpolation, h^2/8 max|f''| per direction (h the node spacing in
  ln rho and in phi), computed from the closed form's second derivatives;
* the same holds across the periodic seam phi -> 2 pi.

Planted mistakes in the azimuthal branch (neighbours swapped, no periodic
wrap, wrong sign of the E_phi rotation term) each break these bounds by a
large factor."""
import math

import numpy as np
import pytest

from paper_2509_15377_amd import workloads as W

A, B, V, E0 = 25e-4, 0.5, 1500.0, 500.0
NR, NPHI = 512, 64
L = math.log(B / A)


def _exact(x, y):
    r2 = x * x + y * y
    return V / (r2 * L) * x + E0, V / (r2 * L) * y


def _bound(rho):
    """Bilinear-interpolation error bound of each polar component at radius
    rho (cell's inner node bounds the radial second derivative), plus the
    float32 rounding of the stored node values."""
    du = L / (NR - 1)
    dphi = 2.0 * math.pi / NPHI
    r_in = A * np.exp(np.floor(np.log(rho / A) / du) * du)
    e_line = V / (r_in * L)
    interp = du * du / 8.0 * e_line + dphi * dphi / 8.0 * E0
    rounding = 2.0 ** -24 * (e_line + 2.0 * E0)
    # both components: the Cartesian error is at most sqrt(2) times either
    return math.sqrt(2.0) * (interp + rounding) * 1.001 + 1e-9


def _excess(O, rho, phi):
    """Largest ratio |E_oracle - E_exact| / bound over the points."""
    f = O.Field(W.wire_crossed_map(A, B, V, E0, NR, NPHI))
    worst = 0.0
    for r, p in zip(rho, phi):
        x, y = r * math.cos(p), r * math.sin(p)
        Ex, Ey, Ez = f.eval([x, y, 0.0])
        ex, ey = _exact(x, y)
        err = math.hypot(Ex - ex, Ey - ey)
        worst = max(worst, err / _bound(r))
        assert Ez == 0.0
    return worst


def _nodes():
    i = np.array([0, 1, 7, 100, 255, 400, 510])
    j = np.arange(NPHI)
    rho = A * (B / A) ** (i / (NR - 1))
    rr, pp = np.meshgrid(rho * (1.0 + 1e-12), 2.0 * math.pi * j / NPHI)
    return rr.ravel(), pp.ravel()


def _between(seed=3, n=4000):
    rng = np.random.default_rng(seed)
    rho = A * (B / A) ** rng.uniform(0.0, 0.999, n)
    return rho, rng.uniform(0.0, 2.0 * math.pi, n)


def _seam(n=400):
    rng = np.random.default_rng(4)
    dphi = 2.0 * math.pi / NPHI
    rho = A * (B / A) ** rng.uniform(0.0, 0.999, n)
    # the last cell [phi_63, 2 pi): its upper neighbour is node 0
    return rho, 2.0 * math.pi - dphi * rng.uniform(1e-6, 0.999, n)


def test_nodes_reproduce_the_closed_form(oracle_mod):
    rho, phi = _nodes()
    f = oracle_mod.Field(W.wire_crossed_map(A, B, V, E0, NR, NPHI))
    for r, p in zip(rho, phi):
        x, y = r * math.cos(p), r * math.sin(p)
        Ex, Ey, _ = f.eval([x, y, 0.0])
        ex, ey = _exact(x, y)
        mag = V / (r * L) + E0
        # float32 node values and node positions known to ~1e-12
        assert math.hypot(Ex - ex, Ey - ey) <= 4.0 * 2.0 ** -24 * mag + 1e-9 * mag, (r, p)


def test_bilinear_error_bound_everywhere(oracle_mod):
    assert _excess(oracle_mod, *_between()) <= 1.0


def test_periodic_seam(oracle_mod):
    assert _excess(oracle_mod, *_seam()) <= 1.0


def test_field_without_phi_dependence_is_unchanged(oracle_mod):
    """E0 = 0 is the plain wire map: purely radial, E_phi = 0."""
    f = oracle_mod.Field(W.wire_crossed_map(A, B, V, 0.0, NR, NPHI))
    g = oracle_mod.Field(W.wire_polar_map(A, B, V, NR, NPHI))
    for r, p in zip(*_between(5, 200)):
        x, y = r * math.cos(p), r * math.sin(p)
        assert np.array_equal(f.eval([x, y, 0.0]), g.eval([x, y, 0.0]))


@pytest.mark.parametrize("macro,points", [
    ("ORC_PLANT_PHI_SWAP", "between"),
    ("ORC_PLANT_EPHI_SIGN", "between"),
    ("ORC_PLANT_PHI_WRAP", "seam"),
])
def test_planted_mistakes_break_the_bound(oracle_mod, macro, points):
    pts = _between() if points == "between" else _seam()
    with oracle_mod.planted(macro):
        assert _excess(oracle_mod, *pts) > 10.0
