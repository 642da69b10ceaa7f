"""The seeded input generators: determinism, shapes, value ranges, recipes."""
import math

import numpy as np

from paper_2007_05218_amd import inputs


def _prim(U, box):
    v = inputs.valid(U, box)
    rho = v[0]
    u, w3, w = v[1] / rho, v[2] / rho, v[3] / rho
    p = 0.4 * (v[4] - 0.5 * rho * (u * u + w3 * w3 + w * w))
    return rho, u, w3, w, p


def test_level_deterministic_and_ranges():
    s1, b1, _ = inputs.level(nboxes=12, seed=2)
    s2, b2, _ = inputs.level(nboxes=12, seed=2)
    assert [b["n"] for b in b1] == [b["n"] for b in b2]
    for a, b, box in zip(s1, s2, b1):
        assert np.array_equal(a, b)
        assert set(box["n"]) <= {16, 32, 64}
        assert box["dx"] == (1 / 64,) * 3
        rho, u, v, w, p = _prim(a, box)
        assert rho.min() >= 0.5 - 1e-12 and rho.max() <= 2.0 + 1e-12
        assert p.min() >= 0.5 - 1e-9 and p.max() <= 2.0 + 1e-9
        assert max(np.abs(u).max(), np.abs(v).max(), np.abs(w).max()) <= 0.5 + 1e-12
    full = inputs.level_shapes(512, seed=2)
    cells = sum(a * b * c for a, b, c in full)
    assert 2.4e7 < cells < 2.9e7


def test_smooth_is_periodic():
    U, box, _ = inputs.smooth((16, 32, 24), seed=4)
    # the field continued one period further equals itself: check by the
    # discrete Fourier spectrum having only integer modes (no leakage)
    rho = inputs.valid(U, box)[0]
    F = np.abs(np.fft.fftn(rho - rho.mean()))
    k = np.argsort(F.ravel())[::-1]
    assert F.ravel()[k[16]] < 1e-9 * F.ravel()[k[0]]


def test_kh_recipe():
    U, box, prm = inputs.kh(32, seed=1)
    rho, u, v, w, p = _prim(U, box)
    y = (np.arange(32) + 0.5) / 32
    inner = np.abs(y - 0.5) < 0.25
    assert np.all(rho[:, inner, :] == 2.0) and np.all(rho[:, ~inner, :] == 1.0)
    assert np.all(u[:, inner, :] == 0.5) and np.all(u[:, ~inner, :] == -0.5)
    assert np.allclose(p, 2.5) and np.abs(v).max() < 0.01 and np.abs(w).max() < 0.01
    assert prm["gamma"] == 1.4 and prm["cfl"] == 0.5


def test_rt_hydrostatic():
    U, box, prm = inputs.rt(32, seed=4)
    rho, u, v, w, p = _prim(U, box)
    assert prm["grav"] == (0.0, 0.0, -0.1)
    assert box["bc_lo"] == (0, 0, 2)
    # column-wise hydrostatic: p jumps only by g rho dz between cells of one fluid
    dz = 1 / 32
    dp = np.diff(p, axis=0)
    same = rho[1:] == rho[:-1]
    assert np.allclose(dp[same], (-0.1 * rho[1:] * dz)[same], rtol=1e-9)
    assert np.all(u == 0) and np.all(w == 0)


def test_sod_recipe():
    U, box, prm = inputs.sod(32)
    rho, u, v, w, p = _prim(U, box)
    assert box["bc_lo"] == (1, 1, 1)
    assert np.all(rho[:, :, :16] == 1.0) and np.all(rho[:, :, 16:] == 0.125)
    assert np.allclose(p[:, :, :16], 1.0) and np.allclose(p[:, :, 16:], 0.1)


def test_request_stream():
    reqs = inputs.request_stream(2000, rate=10.0, seed=3)
    ns = np.array([r["n"] for r in reqs])
    assert ns.min() >= 32 and ns.max() <= 192
    steps = np.array([r["steps"] for r in reqs])
    assert steps.min() >= 10 and steps.max() <= 200
    gaps = np.diff([r["arrival"] for r in reqs])
    assert abs(gaps.mean() - 0.1) < 0.01
    fams = {r["family"] for r in reqs}
    assert fams == set(inputs.FAMILIES)
    # log-uniform: median near sqrt(32*192)
    assert abs(np.median(ns) - math.sqrt(32 * 192)) < 8
