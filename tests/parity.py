"""Comparison of a GPU state with the oracle's (test helper).

Metric (max relative cell error): for the strictly positive components
(rho, E) the pointwise |g - o| / |o|; for the momenta |g - o| divided by the
largest |o| of that component in the box, and a momentum component that is
identically zero in the oracle must be identically zero on the GPU.  The
fraction of bitwise-equal values is reported alongside.
"""
import numpy as np


def compare(g, o):
    g = np.asarray(g, dtype=np.float64)
    o = np.asarray(o, dtype=np.float64)
    assert g.shape == o.shape
    worst = 0.0
    for c in range(5):
        gc, oc = g[c], o[c]
        if c in (0, 4):
            err = np.max(np.abs(gc - oc) / np.abs(oc)) if oc.size else 0.0
        else:
            scale = np.max(np.abs(oc)) if oc.size else 0.0
            if scale == 0.0:
                err = 0.0 if np.all(gc == 0.0) else np.inf
            else:
                err = np.max(np.abs(gc - oc)) / scale
        worst = max(worst, float(err))
    bitwise = float(np.mean(g.view(np.int64) == o.view(np.int64))) if g.size else 1.0
    return worst, bitwise
