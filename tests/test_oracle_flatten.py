"""Shock flattening in the oracle (Colella & Woodward 1984, Sec. 4), pinned
without the GPU: worked examples of the coefficient, no effect where there is
no shock (bitwise), full flattening turns the scheme first order, the
coefficient marks a strong shock and nothing else, and the flattened Sedov
blast still follows the self-similar solution."""
import math

import numpy as np
import pytest

import exact_riemann as er
import sedov_exact
from paper_2007_05218_amd import inputs


def test_coefficient_worked_examples(orc):
    # a pressure step at rest: no convergence, no flattening
    assert orc.flatten_1d([1, 1, 1, 1, .1, .1, .1], [0] * 7) == 1.0
    # a converging flow with the jump inside one cell: for the centre,
    # p[i+1]-p[i-1] = .1-1 and p[i+2]-p[i-2] = .1-1, z = 1 -> chi = 1
    assert orc.flatten_1d([1, 1, 1, .55, .1, .1, .1], [1, 1, 1, .5, 0, 0, 0]) == 0.0
    # the same jump diverging (an expansion): no flattening
    assert orc.flatten_1d([1, 1, 1, .55, .1, .1, .1], [0, 0, 0, .5, 1, 1, 1]) == 1.0
    # a weak jump (|dp| = .02 < .33 min(p)): no flattening
    assert orc.flatten_1d([1, 1, 1, .99, .98, .98, .98], [1, 1, 1, .5, 0, 0, 0]) == 1.0
    # a wider front: centre z = .72/.9 = .8 -> chi = 10 (.8 - .75) = .5; the
    # neighbours have z = .5/.86 and .4/.76 (< .75) -> chi = 0
    f = orc.flatten_1d([1, 1, .86, .5, .14, .1, .1], [1, 1, 1, .5, 0, 0, 0])
    assert f == pytest.approx(0.5, abs=1e-12)
    # the cell behind a shock (its lower-pressure neighbour is in the shock)
    # is flattened with it; the cell ahead of it is not
    p = [1, 1, 1, 1, .55, .1, .1, .1]
    u = [1, 1, 1, 1, .5, 0, 0, 0]
    assert orc.flatten_1d(p[1:], u[1:]) == 0.0   # centre = the shock cell
    assert orc.flatten_1d(p[:7], u[:7]) == 0.0   # centre = the cell behind it
    ahead = [1, 1, .55, .1, .1, .1, .1]
    assert orc.flatten_1d(ahead, [1, 1, .5, 0, 0, 0, 0]) == 1.0


def test_flattening_limits_the_parabola_toward_the_mean(orc):
    a5 = [0.0, 0.1, 0.3, 0.8, 0.9]
    aL, aR = orc.ppm_parabola(a5)
    assert orc.ppm_parabola_flat(a5, 1.0) == (aL, aR)
    fL, fR = orc.ppm_parabola_flat(a5, 0.0)
    assert fL == fR == 0.3
    hL, hR = orc.ppm_parabola_flat(a5, 0.5)
    assert min(aL, 0.3) <= hL <= max(aL, 0.3) and min(aR, 0.3) <= hR <= max(aR, 0.3)
    # continuous at f = 1, and the face values approach the mean steadily as
    # f falls (a monotone profile the limiter leaves alone)
    nL, nR = orc.ppm_parabola_flat(a5, 0.999)
    assert abs(nL - aL) < 1e-3 and abs(nR - aR) < 1e-3
    dev = [abs(l - 0.3) + abs(r - 0.3)
           for l, r in (orc.ppm_parabola_flat(a5, f) for f in (0.999, 0.75, 0.5, 0.25, 0.0))]
    assert all(a > b for a, b in zip(dev, dev[1:])), dev


def _run(orc, U, box, prm, steps):
    ob, op = orc.box_from(box), orc.params_from(prm)
    err = 0
    for _ in range(steps):
        orc.fill_ghosts(U, ob)
        dt = orc.estimate_dt(U, ob, op)
        Un = U.copy()
        err |= orc.advance_box(U, Un, ob, op, dt)
        U = Un
    return U, err


@pytest.mark.parametrize("make", [
    lambda: inputs.advect((16, 16, 8), kvec=(1, 1, 0), vel=(1.0, 1.0, 0.0)),
    lambda: inputs.kh(16, seed=1),
])
def test_no_shock_no_effect_bitwise(orc, make):
    # smooth advection and a shear layer at uniform pressure: no cell meets
    # the shock test, so flattening changes nothing, bit for bit
    U, box, prm = make()
    a, ea = _run(orc, U.copy(), box, prm, 4)
    b, eb = _run(orc, U.copy(), box, dict(prm, flatten=1), 4)
    assert ea == eb and np.array_equal(inputs.valid(a, box), inputs.valid(b, box))


def _advect_l1(orc, n, flatten, tend=1.0):
    U, box, prm = inputs.advect((n, 4, 4), kvec=(1, 0, 0), vel=(1.0, 0.0, 0.0))
    prm = dict(prm, flatten=flatten)
    ob, op = orc.box_from(box), orc.params_from(prm)
    U0 = inputs.valid(U, box)[0].copy()
    t = 0.0
    while t < tend - 1e-12:
        orc.fill_ghosts(U, ob)
        dt = min(orc.estimate_dt(U, ob, op), tend - t)
        Un = U.copy()
        assert orc.advance_box(U, Un, ob, op, dt) == 0
        U = Un
        t += dt
    return np.mean(np.abs(inputs.valid(U, box)[0] - U0))


def test_full_flattening_is_first_order(orc):
    # coefficient 0 everywhere (the oracle's test mode 2) reduces every
    # parabola to the cell average: the scheme becomes first order on a
    # smooth wave, while PPM proper is second order
    full = [_advect_l1(orc, n, 2) for n in (32, 64)]
    none = [_advect_l1(orc, n, 0) for n in (32, 64)]
    o_full = math.log(full[0] / full[1], 2)
    o_none = math.log(none[0] / none[1], 2)
    assert 0.8 <= o_full <= 1.2, full
    assert o_none >= 1.8, none
    assert full[1] > 5 * none[1]


def test_coefficient_marks_a_strong_shock_only(orc):
    # a shock tube with a pressure ratio of 1000 (the Sod tube's own shock,
    # spread over three cells, stays just below the steepness threshold):
    # the cells with a coefficient below one sit at the shock, within two
    # cells of the exact front, and none at the contact or in the rarefaction
    n = 128
    U, box, prm = inputs.sod((n, 4, 4), axis=0)
    x, _, _ = inputs.cell_centres(box)
    left = np.broadcast_to(x < 0.5, (4, 4, n))
    U = inputs.from_primitive(box, np.where(left, 1.0, 0.125), 0.0, 0.0, 0.0,
                              np.where(left, 100.0, 0.1))
    U, err = _run_to(orc, U, box, dict(prm, flatten=1), 0.025)
    assert err == 0
    orc.fill_ghosts(U, orc.box_from(box))
    g = box["ng"]
    row = U[:, g + 2, g + 2, :]
    rho = row[0]
    u = row[1] / rho
    p = 0.4 * (row[4] - 0.5 * row[1] ** 2 / rho)
    cells = range(3, n + 2 * g - 3)
    f = np.array([orc.flatten_1d(p[i - 3:i + 4], u[i - 3:i + 4]) for i in cells])
    xc = (np.array(cells) - g + 0.5) / n
    w = er.waves(1.0, 0.0, 100.0, 0.125, 0.0, 0.1)
    xs = 0.5 + w["right_shock"] * 0.025
    flagged = xc[f < 1.0]
    assert flagged.size >= 1
    assert np.all(np.abs(flagged - xs) <= 2.0 / n), (flagged, xs)


def test_flattened_sod_converges(orc):
    # with flattening the tube still converges to the exact solution, at a
    # first-order rate, and no less accurately than 1.3x the unflattened L1
    def l1(n, flatten):
        U, box, prm = inputs.sod((n, 4, 4), axis=0)
        U, err = _run_to(orc, U, box, dict(prm, flatten=flatten), 0.2)
        assert err == 0
        rho = inputs.valid(U, box)[0, 2, 2, :]
        xc = (np.arange(n) + 0.5) / n
        ex = er.cell_average(xc, 1.0 / n, 0.2, 0.5, (1.0, 0.0, 1.0), (0.125, 0.0, 0.1))
        return np.sum(np.abs(rho - ex)) / n
    e = [l1(n, 1) for n in (32, 64, 128)]
    assert e[0] > e[1] > e[2]
    assert math.log(e[1] / e[2], 2) >= 0.6, e
    assert e[2] <= 1.3 * l1(128, 0)


def _run_to(orc, U, box, prm, tend):
    ob, op = orc.box_from(box), orc.params_from(prm)
    t, err = 0.0, 0
    while t < tend - 1e-12:
        orc.fill_ghosts(U, ob)
        dt = min(orc.estimate_dt(U, ob, op), tend - t)
        Un = U.copy()
        err |= orc.advance_box(U, Un, ob, op, dt)
        U = Un
        t += dt
    return U, err


def test_flattened_sedov_follows_similarity(orc):
    n = 32
    U, box, prm = inputs.sedov(n)
    prm = dict(prm, flatten=1)
    x, y, z = inputs.cell_centres(box)
    r = np.broadcast_to(np.sqrt((x - 0.5) ** 2 + (y - 0.5) ** 2 + (z - 0.5) ** 2), (n,) * 3)
    m0, e0 = (inputs.valid(U, box)[c].sum() for c in (0, 4))
    U, err = _run_to(orc, U, box, prm, 0.04)
    assert err & 7 == 0
    V = inputs.valid(U, box)
    assert V[0].sum() == pytest.approx(m0, rel=1e-13)
    assert V[4].sum() == pytest.approx(e0, rel=1e-13)
    R = sedov_exact.measured_radius(V[0], r, n, 0.5)
    assert R == pytest.approx(sedov_exact.shock_radius(0.04), rel=0.10)


def test_flattening_needs_four_ghost_layers(orc):
    U, box, prm = inputs.sod((16, 4, 4), axis=0, ng=3)
    ob = orc.box_from(box)
    with pytest.raises(ValueError):
        orc.advance_box(U, U.copy(), ob, orc.params_from(dict(prm, flatten=1)), 1e-3)
