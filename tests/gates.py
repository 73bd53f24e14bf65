"""Accuracy gates of the FP32-mixed path against a reference run of the
same avalanches (the FP64 GPU path or the FP64 oracle): mean gain within
1 %, drift velocity within 0.5 %, KS p > 0.01 on the endpoint and
arrival-time distributions."""
import numpy as np
from scipy import stats


def _drift(ep):
    m = ep["status"] == 2
    return (ep["z1"][m] - ep["z0"][m]).sum() / (ep["t1"][m] - ep["t0"][m]).sum()


def statistical_gates(ref, got, label, n_aval):
    """The FP32-mixed accuracy gates against a reference run of the same
    avalanches (FP64 GPU or the oracle): mean gain within 1 %, drift velocity
    within 0.5 %, KS p > 0.01 on the arrival time, energy and x of the
    electrons reaching the anode (pooled) and on the per-avalanche gain and
    mean arrival time (independent samples).  Returns the numbers."""
    def per_aval(ep):
        n = np.bincount(ep["aval"], minlength=n_aval).astype(float)
        t = np.bincount(ep["aval"], weights=ep["t1"], minlength=n_aval)
        keep = n > 0
        return n[keep], t[keep] / n[keep]
    gr, tr = per_aval(ref)
    gg, tg = per_aval(got)
    rel = abs(gg.mean() - gr.mean()) / gr.mean()
    vr, vg = _drift(ref), _drift(got)
    dv = abs(vg - vr) / vr
    mr, mg = ref["status"] == 2, got["status"] == 2
    ks = {k: stats.ks_2samp(ref[k][mr], got[k][mg]).pvalue for k in ("t1", "e1", "x1")}
    ks["gain"] = stats.ks_2samp(gr, gg).pvalue
    ks["mean_t"] = stats.ks_2samp(tr, tg).pvalue
    print(f"{label}: mean gain {gr.mean():.2f} -> {gg.mean():.2f} (rel {rel:.2e}), drift rel {dv:.2e}, KS {ks}")
    assert rel < 0.01, label
    assert dv < 0.005, label
    for k, pv in ks.items():
        assert pv > 0.01, (label, k)
    return rel, dv, ks
