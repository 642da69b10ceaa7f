"""The oracle's ghost exchange between the boxes of a tiled level, and the
Sedov blast, pinned on the CPU: the level fill of one box equals the oracle's
box fill, every ghost cell equals a brute-force lookup, a level of boxes steps
exactly like the domain as one box, and the blast follows the self-similar
solution while conserving mass and energy."""
import itertools
import math

import numpy as np
import pytest

import sedov_exact
from oracle import level as olev
from paper_2007_05218_amd import inputs

P, O, R = inputs.BC_PERIODIC, inputs.BC_OUTFLOW, inputs.BC_REFLECT
BCS = [((P, P, P), (P, P, P)), ((O, O, R), (O, O, R)), ((P, R, O), (P, O, R))]


def _random_domain(n, ng, bc_lo, bc_hi, seed):
    box = inputs.box_desc(n, ng, bc_lo=bc_lo, bc_hi=bc_hi)
    rng = np.random.default_rng(seed)
    U = np.zeros(inputs.state_shape(box))
    inputs.valid(U, box)[...] = rng.uniform(0.5, 2.0, size=inputs.valid(U, box).shape)
    inputs.valid(U, box)[1:4] -= 1.25
    return U, box


@pytest.mark.parametrize("bcs", BCS)
def test_single_box_level_equals_box_fill(orc, bcs):
    # a level of one box covering the domain is the box's own ghost fill
    U, box = _random_domain((9, 7, 6), 4, bcs[0], bcs[1], seed=1)
    (G,) = olev.fill_ghosts_level([U], [box], [(0, 0, 0)], box["n"], *bcs)
    V = U.copy()
    orc.fill_ghosts(V, orc.box_from(box))
    assert np.array_equal(G, V)


def _brute_src(g, D, bl, bh):
    if g < 0:
        return {P: g + D, O: 0, R: -1 - g}[bl], bl == R
    if g >= D:
        return {P: g - D, O: D - 1, R: 2 * D - 1 - g}[bh], bh == R
    return g, False


@pytest.mark.parametrize("bcs", BCS)
def test_level_fill_brute_force(bcs):
    # every ghost cell of every box, looked up cell by cell
    ng = 3
    U, dbox = _random_domain((7, 6, 5), ng, bcs[0], bcs[1], seed=2)
    cuts = ([0, 3, 7], [0, 2, 6], [0, 5])
    states, boxes, lo, til = inputs.tile(U, dbox, cuts)
    dom = til["dom"]
    out = olev.fill_ghosts_level(states, boxes, lo, dom, til["bc_lo"], til["bc_hi"])
    for G, b, l, S in zip(out, boxes, lo, states):
        n = b["n"]
        assert np.array_equal(inputs.valid(G, b), inputs.valid(S, b))
        for k, j, i in itertools.product(*(range(-ng, n[d] + ng) for d in (2, 1, 0))):
            if 0 <= i < n[0] and 0 <= j < n[1] and 0 <= k < n[2]:
                continue
            s, flip = zip(*(_brute_src(l[d] + c, dom[d], bcs[0][d], bcs[1][d])
                            for d, c in enumerate((i, j, k))))
            owner = [m for m, (bb, ll) in enumerate(zip(boxes, lo))
                     if all(ll[d] <= s[d] < ll[d] + bb["n"][d] for d in range(3))]
            assert len(owner) == 1
            o = owner[0]
            src = states[o][:, ng + s[2] - lo[o][2], ng + s[1] - lo[o][1], ng + s[0] - lo[o][0]]
            want = src * np.array([1.0, -1.0 if flip[0] else 1.0, -1.0 if flip[1] else 1.0,
                                   -1.0 if flip[2] else 1.0, 1.0])
            assert np.array_equal(G[:, k + ng, j + ng, i + ng], want), (b["n"], l, i, j, k)


def test_tiling_rejects_gaps_and_overlaps():
    U, box = _random_domain((6, 6, 6), 3, (P,) * 3, (P,) * 3, seed=3)
    states, boxes, lo, til = inputs.tile(U, box, ([0, 3, 6], [0, 6], [0, 6]))
    with pytest.raises(ValueError):
        olev.assemble(states[:1], boxes[:1], lo[:1], til["dom"])
    with pytest.raises(ValueError):
        olev.assemble(states, boxes, [lo[0], lo[0]], til["dom"])


def _oracle_level_run(orc, states, boxes, lo, til, prm, steps):
    op = orc.params_from(prm)
    obs = [orc.box_from(b) for b in boxes]
    err, dts = 0, []
    for _ in range(steps):
        # the timestep reads valid cells only (its own per-box fill is then
        # replaced by the level's)
        dt = min(orc.estimate_dt(U, ob, op) for U, ob in zip(states, obs))
        states = olev.fill_ghosts_level(states, boxes, lo, til["dom"], til["bc_lo"],
                                        til["bc_hi"])
        new = []
        for U, ob in zip(states, obs):
            Un = U.copy()
            err |= orc.advance_box(U, Un, ob, op, dt)
            new.append(Un)
        states = new
        dts.append(dt)
    return states, err, dts


@pytest.mark.parametrize("case", ["rt", "sod"])
def test_level_steps_like_the_domain(orc, case):
    # boxes of uneven sizes advanced with the level's ghost exchange give,
    # bit for bit, the domain advanced as one box
    if case == "rt":
        U, box, prm = inputs.rt((20, 16, 24), seed=4)
        cuts = ([0, 5, 12, 20], [0, 9, 16], [0, 7, 24])
    else:
        U, box, prm = inputs.sod((24, 12, 12), axis=0)
        cuts = ([0, 8, 13, 24], [0, 12], [0, 4, 12])
    states, boxes, lo, til = inputs.tile(U, box, cuts)
    steps = 3
    got, err, dts = _oracle_level_run(orc, states, boxes, lo, til, prm, steps)
    ob, op = orc.box_from(box), orc.params_from(prm)
    D = U.copy()
    derr = 0
    for s in range(steps):
        orc.fill_ghosts(D, ob)
        assert orc.estimate_dt(D, ob, op) == dts[s]
        Dn = D.copy()
        derr |= orc.advance_box(D, Dn, ob, op, dts[s])
        D = Dn
    assert err == derr
    whole = inputs.valid(D, box)
    for G, b, l in zip(got, boxes, lo):
        n = b["n"]
        part = whole[:, l[2]:l[2] + n[2], l[1]:l[1] + n[1], l[0]:l[0] + n[0]]
        assert np.array_equal(inputs.valid(G, b), part)


def test_sedov_similarity_constant():
    # E = alpha rho0 R^5 / t^2: Sedov's value for gamma = 1.4 as tabulated by
    # Kamm & Timmes (2007), alpha = 0.851072
    assert sedov_exact.alpha(1.4) == pytest.approx(0.851072, abs=2e-6)


def test_sedov_oracle_follows_similarity(orc):
    # the oracle's blast: mass and energy conserved to roundoff while the
    # shock is inside the box (the outflow faces see gas at rest), and the
    # shock radius close to the self-similar one, R ~ t^(2/5), at 32^3
    n = 32
    U, box, prm = inputs.sedov(n)
    ob, op = orc.box_from(box), orc.params_from(prm)
    x, y, z = inputs.cell_centres(box)
    r = np.broadcast_to(np.sqrt((x - 0.5) ** 2 + (y - 0.5) ** 2 + (z - 0.5) ** 2), (n,) * 3)
    m0, e0 = (inputs.valid(U, box)[c].sum() for c in (0, 4))
    t, err, radii = 0.0, 0, {}
    marks = [0.01, 0.04]
    while marks:
        orc.fill_ghosts(U, ob)
        dt = orc.estimate_dt(U, ob, op)
        Un = U.copy()
        err |= orc.advance_box(U, Un, ob, op, dt)
        U = Un
        t += dt
        if t >= marks[0]:
            marks.pop(0)
            radii[t] = sedov_exact.measured_radius(inputs.valid(U, box)[0], r, n, 0.5)
    assert err & 7 == 0
    V = inputs.valid(U, box)
    assert V[0].sum() == pytest.approx(m0, rel=1e-13)
    assert V[4].sum() == pytest.approx(e0, rel=1e-13)
    (t1, r1), (t2, r2) = sorted(radii.items())
    for tt, rr in radii.items():
        assert rr == pytest.approx(sedov_exact.shock_radius(tt), rel=0.10)
    assert math.log(r2 / r1) / math.log(t2 / t1) == pytest.approx(0.4, abs=0.04)
