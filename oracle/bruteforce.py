"""Brute-force companion of the oracle: small-time-step integration of the
same tabulated gas model WITHOUT null collisions.

TEST INFRASTRUCTURE ONLY.  It shares nothing with the oracle's C code: the
rate table is interpolated with numpy from the node cross-sections, the
scattering directions are built from an orthonormal frame (not from the
direction-cosine update), the random numbers come from numpy.

Each electron moves along exact parabolic sub-steps of length dt in its
(uniform) field; at the end of a sub-step it collides with probability
1 - exp(-nu_real(e) dt), where nu_real is the sum of the linearly
interpolated channel rates that are valid at e (the masked-null rule of the
tabulated model), and the channel is chosen in proportion to its rate.  The
result converges to the exact transport as dt -> 0 (first order), which is
what the null-collision method (Skullerud, cited in Sec. 1) samples exactly.

Supported: slab fields along z; elastic scattering with target recoil,
isotropic or screened Rutherford (dsigma/dOmega ~ (1 - cos chi + 2 eta)^-2,
eta = screening / (8 e), sampled by rejection from a 1/(1 - cos chi + 2 eta)
envelope, not by the oracle's inverse CDF); excitation; ionisation with a
uniform or an Opal-Beaty split (dsigma/de_s ~ 1/(1 + (e_s/w)^2) on
[0, (e - I)/2], sampled by rejection from a uniform proposal); attachment.
The total valid rate at the sub-step ends comes from one piecewise-linear
table whose breakpoints are the nodes and both sides of every channel's
window edge (exact for the masked, linearly interpolated model).
"""
from __future__ import annotations

import numpy as np

C_CM_PER_NS = 29.9792458
ME_C2_EV = 510998.95
K_A = C_CM_PER_NS ** 2 / ME_C2_EV

ELASTIC, EXCITATION, IONISATION, ATTACHMENT = 0, 1, 2, 3


def _iso_dirs(rng, n):
    c = rng.uniform(-1.0, 1.0, n)
    p = rng.uniform(0.0, 2 * np.pi, n)
    s = np.sqrt(np.maximum(0.0, 1.0 - c * c))
    return np.stack([s * np.cos(p), s * np.sin(p), c], axis=1)


def _turn(rng, d, cos_t):
    """Turn unit vectors d by polar angle theta (cos_t) about a uniform
    azimuth, using an explicit orthonormal frame (e1, e2, d)."""
    n = d.shape[0]
    helper = np.zeros_like(d)
    use_x = np.abs(d[:, 0]) < 0.9
    helper[use_x, 0] = 1.0
    helper[~use_x, 1] = 1.0
    e1 = np.cross(d, helper)
    e1 /= np.linalg.norm(e1, axis=1)[:, None]
    e2 = np.cross(d, e1)
    phi = rng.uniform(0.0, 2 * np.pi, n)
    s = np.sqrt(np.maximum(0.0, 1.0 - cos_t * cos_t))
    return (cos_t[:, None] * d + (s * np.cos(phi))[:, None] * e1
            + (s * np.sin(phi))[:, None] * e2)


def _screened_rutherford(rng, eta):
    """cos chi with density ~ (1 - cos chi + 2 eta)^-2 on [-1, 1]: x = 1 -
    cos chi + 2 eta is drawn from the envelope ~ 1/x on [2 eta, 2 + 2 eta]
    (x = 2 eta (1 + 1/eta)^U) and kept with probability 2 eta / x."""
    out = np.empty(eta.size)
    todo = np.arange(eta.size)
    while todo.size:
        et = eta[todo]
        x = 2.0 * et * np.power(1.0 + 1.0 / et, rng.random(todo.size))
        ok = rng.random(todo.size) * x < 2.0 * et
        out[todo[ok]] = 1.0 + 2.0 * et[ok] - x[ok]
        todo = todo[~ok]
    return out


def _opal_beaty(rng, avail, w):
    """Secondary energy with density ~ 1/(1 + (e_s/w)^2) on [0, avail/2]:
    uniform proposal, kept with probability 1/(1 + (e_s/w)^2)."""
    out = np.empty(avail.size)
    todo = np.arange(avail.size)
    while todo.size:
        es = 0.5 * avail[todo] * rng.random(todo.size)
        ok = rng.random(todo.size) * (1.0 + (es / w[todo]) ** 2) < 1.0
        out[todo[ok]] = es[ok]
        todo = todo[~ok]
    return out


def _valid_rate_table(e_nodes, nu_nodes, e_lo, e_hi):
    """Breakpoints and values of the total valid rate: linear between nodes,
    stepping at the window edges (both sides of each edge are breakpoints,
    the lower one the largest double below the edge)."""
    pts = [e_nodes]
    for lo, hi in zip(e_lo, e_hi):
        for edge in (lo, hi):
            if 0.0 < edge <= e_nodes[-1]:
                pts.append(np.array([np.nextafter(edge, -np.inf), edge]))
    xs = np.unique(np.concatenate(pts))
    tot = np.zeros(xs.size)
    for c in range(len(nu_nodes)):
        valid = (xs >= e_lo[c]) & (xs < e_hi[c])
        tot += np.where(valid, np.interp(xs, e_nodes, nu_nodes[c]), 0.0)
    return xs, tot


def simulate(gas, z_hi, E_z, n_aval, dt, rng, block=128, max_electrons=10 ** 7):
    """Avalanches from one electron at rest at z = 0 in the slab [0, z_hi)
    with field magnitude E_z accelerating towards +z.  Returns per-electron
    arrays (aval, z, t, e, status) with status 1 (z < 0), 2 (z >= z_hi) or
    3 (attached), and the birth energies of the secondaries (``sec_e``).

    The sub-steps of every active electron are evaluated ``block`` at a time
    (positions, energies and collision draws of sub-steps 1..block in closed
    form), then each electron is advanced to its first event in the block:
    the same discrete process as one sub-step at a time."""
    e_nodes = (np.arange(gas.n_bins + 1, dtype=np.float64) * gas.e_max_eV) / gas.n_bins
    speed = np.sqrt(2.0 * K_A * e_nodes)
    nu_nodes, kinds, e_lo, e_hi, loss, mu, ang, scr, split, sw = [], [], [], [], [], [], [], [], [], []
    for ch in gas.channels:
        if ch.values_kind == 1:
            nu_nodes.append(np.asarray(ch.values, dtype=np.float64))
        else:
            nu_nodes.append(gas.density_cm3 * np.asarray(ch.values, dtype=np.float64) * speed)
        kinds.append(ch.kind)
        e_lo.append(ch.e_lo_eV)
        e_hi.append(ch.e_hi_eV)
        loss.append(ch.loss_eV)
        mu.append(ch.mass_ratio)
        ang.append(ch.angular)
        scr.append(ch.screening_eV)
        split.append(ch.split)
        sw.append(ch.split_w_eV)
        if getattr(ch, "penning_prob", 0.0):
            raise NotImplementedError("brute force: no Penning transfer")
    kinds = np.asarray(kinds)
    loss = np.asarray(loss)
    mu = np.asarray(mu)
    ang = np.asarray(ang)
    scr = np.asarray(scr, dtype=np.float64)
    split = np.asarray(split)
    sw = np.asarray(sw, dtype=np.float64)
    if any(h > e_nodes[-1] and np.isfinite(h) for h in e_hi):
        raise NotImplementedError("brute force: window edges above the table")
    xs_tab, tot_tab = _valid_rate_table(e_nodes, nu_nodes, e_lo, e_hi)
    nch = len(kinds)
    acc = K_A * E_z  # along +z
    s = dt * np.arange(1, block + 1, dtype=np.float64)  # sub-step ends

    def rates(e):
        """Per-channel valid rates (only at collisions)."""
        nu = np.zeros(e.shape + (nch,))
        for c in range(nch):
            r = np.interp(e, e_nodes, nu_nodes[c])  # constant above the last node
            nu[..., c] = np.where((e >= e_lo[c]) & (e < e_hi[c]), r, 0.0)
        return nu

    pos = np.zeros((n_aval, 3))
    vel = np.zeros((n_aval, 3))
    t = np.zeros(n_aval)
    aval = np.arange(n_aval)
    out = {k: [] for k in ("aval", "z", "t", "e", "status")}
    sec_e = []

    def emit(sel, z, tt, e, st):
        out["aval"].append(aval[sel]); out["z"].append(z); out["t"].append(tt)
        out["e"].append(e); out["status"].append(np.full(z.size, st))

    while pos.shape[0] > 0:
        n = pos.shape[0]
        if n > max_electrons:
            raise RuntimeError("too many electrons")
        # sub-step ends j = 1..block for every electron (exact parabolas)
        zj = pos[:, 2:3] + vel[:, 2:3] * s + 0.5 * acc * s * s
        vzj = vel[:, 2:3] + acc * s
        vperp2 = vel[:, 0:1] ** 2 + vel[:, 1:2] ** 2
        ej = 0.5 * (vperp2 + vzj * vzj) / K_A
        p = -np.expm1(-np.interp(ej, xs_tab, tot_tab) * dt)
        coll = rng.random((n, block)) < p
        outj = (zj >= z_hi) | (zj < 0.0)
        big = block + 1
        j_out = np.where(outj.any(axis=1), outj.argmax(axis=1), big)
        j_col = np.where(coll.any(axis=1), coll.argmax(axis=1), big)
        # electrons leaving the slab in this block (exit before collision)
        leave = j_out < big
        leave &= j_out <= j_col
        keep = np.ones(n, dtype=bool)
        if np.any(leave):
            li = np.nonzero(leave)[0]
            jj = j_out[li]
            z_end = zj[li, jj]
            z_prev = np.where(jj > 0, zj[li, np.maximum(jj - 1, 0)], pos[li, 2])
            hi = z_end >= z_hi
            zb = np.where(hi, z_hi, 0.0)
            den = np.where(z_end != z_prev, z_end - z_prev, 1.0)
            frac = np.clip((zb - z_prev) / den, 0.0, 1.0)
            t_x = t[li] + (jj + frac) * dt
            e_x = ej[li, jj]
            for st, m in ((2, hi), (1, ~hi)):
                if np.any(m):
                    emit(li[m], zb[m], t_x[m], e_x[m], st)
            keep[li] = False
        # electrons colliding in this block
        col = (j_col < big) & ~leave
        ci = np.nonzero(col)[0]
        # electrons with no event: advance by the whole block
        idle = keep & ~col
        if np.any(idle):
            ii = np.nonzero(idle)[0]
            S = s[-1]
            pos[ii, 0] += vel[ii, 0] * S
            pos[ii, 1] += vel[ii, 1] * S
            pos[ii, 2] = zj[ii, -1]
            vel[ii, 2] = vzj[ii, -1]
            t[ii] += S
        sec = None
        if ci.size:
            jj = j_col[ci]
            S = s[jj]
            pos[ci, 0] += vel[ci, 0] * S
            pos[ci, 1] += vel[ci, 1] * S
            pos[ci, 2] = zj[ci, jj]
            vel[ci, 2] = vzj[ci, jj]
            t[ci] += S
            e_i = ej[ci, jj]
            nu_i = rates(e_i)
            cum = np.cumsum(nu_i, axis=1)
            pick = rng.random(ci.size) * cum[:, -1]
            ch = np.minimum((cum <= pick[:, None]).sum(axis=1), nch - 1)
            kind = kinds[ch]
            sp = np.sqrt(np.sum(vel[ci] ** 2, axis=1))
            d = np.where(sp[:, None] > 0, vel[ci] / np.where(sp > 0, sp, 1.0)[:, None],
                         np.array([0.0, 0.0, 1.0]))
            new_e = e_i.copy()
            new_d = d.copy()
            m = kind == ELASTIC
            if np.any(m):
                mu_i = mu[ch[m]]
                cchi = rng.uniform(-1.0, 1.0, m.sum())
                sr = ang[ch[m]] != 0
                if np.any(sr):
                    eta = scr[ch[m]][sr] / (8.0 * e_i[m][sr])
                    cchi[sr] = _screened_rutherford(rng, eta)
                v_in = np.sqrt(2 * K_A * e_i[m])
                vcm = mu_i / (1 + mu_i) * v_in
                urel = v_in / (1 + mu_i)
                vz = vcm + urel * cchi
                vt = urel * np.sqrt(np.maximum(0.0, 1 - cchi * cchi))
                vout = np.sqrt(vz * vz + vt * vt)
                cos_lab = np.where(vout > 0, vz / np.where(vout > 0, vout, 1.0), 1.0)
                new_e[m] = 0.5 * vout * vout / K_A
                new_d[m] = _turn(rng, d[m], cos_lab)
            m = kind == EXCITATION
            if np.any(m):
                new_e[m] = e_i[m] - loss[ch[m]]
                new_d[m] = _iso_dirs(rng, m.sum())
            m = kind == IONISATION
            if np.any(m):
                avail = e_i[m] - loss[ch[m]]
                es = rng.random(m.sum()) * avail
                ob = split[ch[m]] != 0
                if np.any(ob):
                    es[ob] = _opal_beaty(rng, avail[ob], sw[ch[m]][ob])
                sec_e.append(es.copy())
                new_e[m] = avail - es
                new_d[m] = _iso_dirs(rng, m.sum())
                sv = np.sqrt(2 * K_A * es)[:, None] * _iso_dirs(rng, m.sum())
                src = ci[m]
                sec = (pos[src].copy(), sv, t[src].copy(), aval[src].copy())
            vel[ci] = np.sqrt(2 * K_A * np.maximum(new_e, 0.0))[:, None] * new_d
            m = kind == ATTACHMENT
            if np.any(m):
                a = ci[m]
                emit(a, pos[a, 2].copy(), t[a].copy(), e_i[m], 3)
                keep[a] = False
        pos, vel, t, aval = pos[keep], vel[keep], t[keep], aval[keep]
        if sec is not None:
            pos = np.concatenate([pos, sec[0]])
            vel = np.concatenate([vel, sec[1]])
            t = np.concatenate([t, sec[2]])
            aval = np.concatenate([aval, sec[3]])

    res = {k: np.concatenate(v) if v else np.zeros(0) for k, v in out.items()}
    res["sec_e"] = np.concatenate(sec_e) if sec_e else np.zeros(0)
    return res
