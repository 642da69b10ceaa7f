"""Shock flattening on the GPU (k_flatten + the flattened trace kernel)
against the oracle with flattening on: strong shock tubes along each axis, the
Sedov blast as one box, as a tiled level and batched, a ragged box; no effect
without shocks; the flattened blast follows the self-similar solution."""
import numpy as np
import pytest

import sedov_exact
from parity import compare
from paper_2007_05218_amd import inputs

pytestmark = pytest.mark.gpu
TOL = 1e-11


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_2007_05218_amd import hydro
    hydro.lib()
    return hydro


def _gpu_run(hydro, U, box, prm, steps):
    import torch
    B = hydro.Box(U, box, prm)
    B.run(steps)
    torch.cuda.synchronize()
    return B.state(), int(B.err.item())


def _oracle_run(orc, U, box, prm, steps):
    U = U.copy()
    ob, op = orc.box_from(box), orc.params_from(prm)
    err = 0
    for _ in range(steps):
        orc.fill_ghosts(U, ob)
        dt = orc.estimate_dt(U, ob, op)
        Un = U.copy()
        err |= orc.advance_box(U, Un, ob, op, dt)
        U = Un
    return U, err


def _strong_tube(n, axis):
    U, box, prm = inputs.sod(n, axis=axis)
    c = inputs.cell_centres(box)[axis]
    shp = (box["n"][2], box["n"][1], box["n"][0])
    left = np.broadcast_to(c < 0.5, shp)
    U = inputs.from_primitive(box, np.where(left, 1.0, 0.125), 0.0, 0.0, 0.0,
                              np.where(left, 100.0, 0.1))
    return U, box, dict(prm, flatten=1)


CASES = {
    "tube_x": lambda: _strong_tube((48, 8, 8), 0),
    "tube_y": lambda: _strong_tube((8, 48, 8), 1),
    "tube_z": lambda: _strong_tube((8, 8, 48), 2),
    "sedov32": lambda: (lambda U, b, p: (U, b, dict(p, flatten=1)))(*inputs.sedov(32)),
    "sedov_ragged": lambda: (lambda U, b, p: (U, b, dict(p, flatten=1)))(
        *inputs.sedov((37, 29, 23))),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_flattened_parity_20_steps(gpu, orc, case):
    U, box, prm = CASES[case]()
    print("flattened parity", case, box["n"], flush=True)
    g, gerr = _gpu_run(gpu, U, box, prm, 20)
    o, oerr = _oracle_run(orc, U, box, prm, 20)
    assert gerr == oerr
    err, bw = compare(inputs.valid(g, box), inputs.valid(o, box))
    assert err <= TOL and bw == 1.0, (err, bw)
    # and flattening did act: the unflattened run differs
    u, _ = _gpu_run(gpu, U, box, dict(prm, flatten=0), 20)
    assert not np.array_equal(inputs.valid(u, box), inputs.valid(g, box))


def test_no_shock_no_effect_bitwise(gpu):
    U, box, prm = inputs.kh(48, seed=1)
    a, ea = _gpu_run(gpu, U, box, prm, 10)
    b, eb = _gpu_run(gpu, U, box, dict(prm, flatten=1), 10)
    assert ea == eb and np.array_equal(inputs.valid(a, box), inputs.valid(b, box))


def test_flattened_sedov_level_matches_oracle(gpu, orc):
    # 8 boxes of 32^3 tiling the 64^3 blast, batched with the ghost exchange,
    # against the oracle's 64^3 box, 20 steps
    import torch
    states, boxes, prm, lo, til = inputs.sedov_level(64, 32)
    prm = dict(prm, flatten=1)
    U, box, _ = inputs.sedov(64)
    tiling = gpu.Tiling(boxes, lo, til["dom"], til["bc_lo"], til["bc_hi"])
    lev = gpu.Level(states, boxes, prm, shared_dt=True, tiling=tiling)
    lev.run(20)
    torch.cuda.synchronize()
    o, oerr = _oracle_run(orc, U, box, prm, 20)
    assert int(lev.err.item()) == oerr
    W = inputs.valid(o, box)
    for G, b, l in zip(lev.states(), boxes, lo):
        n = b["n"]
        part = W[:, l[2]:l[2] + n[2], l[1]:l[1] + n[1], l[0]:l[0] + n[0]]
        err, bw = compare(inputs.valid(G, b), part)
        assert err <= TOL and bw == 1.0


def test_flattened_batch_equals_single_boxes(gpu):
    # independent boxes batched in one launch per stage equal their
    # single-box advances, bit for bit, with flattening on
    import torch
    cases = [CASES[k]() for k in ("tube_x", "tube_y", "sedov32", "sedov_ragged")]
    states = [c[0] for c in cases]
    boxes = [c[1] for c in cases]
    prm = cases[0][2]
    lev = gpu.Level(states, boxes, prm, shared_dt=False)
    lev.run(5)
    torch.cuda.synchronize()
    for G, (U, box, p) in zip(lev.states(), cases):
        g, _ = _gpu_run(gpu, U, box, prm, 5)
        assert np.array_equal(inputs.valid(G, box), inputs.valid(g, box))


def test_flattened_sedov_follows_similarity(gpu):
    import torch
    n = 128
    U, box, prm = inputs.sedov(n)
    B = gpu.Box(U, box, dict(prm, flatten=1))
    x, y, z = inputs.cell_centres(box)
    r = np.broadcast_to(np.sqrt((x - 0.5) ** 2 + (y - 0.5) ** 2 + (z - 0.5) ** 2), (n,) * 3)
    t = 0.0
    while t < 0.04:
        B.step()
        t += B.dt.item()
    torch.cuda.synchronize()
    assert int(B.err.item()) & 7 == 0
    R = sedov_exact.measured_radius(inputs.valid(B.state(), box)[0], r, n, 0.5)
    assert R == pytest.approx(sedov_exact.shock_radius(t), rel=0.04)


@pytest.mark.parametrize("flatten", [0, 1])
def test_full_size_sedov_level_sampled(gpu, orc, flatten):
    # the benchmark's Sedov configuration (256^3 as 64 boxes of 64^3, with and
    # without flattening): the tenth step, from the state the GPU reached in
    # nine (the blast has started and flattening acts), against the oracle's
    # 256^3 box on sampled regions, several of them straddling box boundaries
    import torch
    n, bs = 256, 64
    states, boxes, prm, lo, til = inputs.sedov_level(n, bs)
    prm = dict(prm, flatten=flatten)
    print("sedov level 256 flatten", flatten, flush=True)
    tiling = gpu.Tiling(boxes, lo, til["dom"], til["bc_lo"], til["bc_hi"])
    lev = gpu.Level(states, boxes, prm, shared_dt=True, tiling=tiling)

    def domain():
        D = np.zeros((5, n, n, n))
        for G, b, l in zip(lev.states(), boxes, lo):
            m = b["n"]
            D[:, l[2]:l[2] + m[2], l[1]:l[1] + m[1], l[0]:l[0] + m[0]] = inputs.valid(G, b)
        return D

    lev.run(9)
    torch.cuda.synchronize()
    U, box, _ = inputs.sedov(n)
    inputs.valid(U, box)[...] = domain()
    lev.step()
    torch.cuda.synchronize()
    gdt = lev.dt_min.item()
    D = domain()
    del lev
    tiling.close()
    torch.cuda.empty_cache()
    ob, op = orc.box_from(box), orc.params_from(prm)
    orc.fill_ghosts(U, ob)
    odt = orc.estimate_dt(U, ob, op)
    assert gdt == odt
    ng = box["ng"]
    Unew = np.empty_like(U)
    regions = [((124, 124, 124), (132, 132, 132)),   # the blast, across 8 boxes
               ((60, 120, 126), (68, 128, 130)),     # a box face in x
               ((0, 0, 0), (4, 4, 4)), ((252, 252, 252), (256, 256, 256)),
               ((126, 62, 60), (130, 66, 68))]       # box faces in y and z
    for rlo, rhi in regions:
        orc.advance_region(U, Unew, ob, op, odt, rlo, rhi)
        o = Unew[:, ng + rlo[2]:ng + rhi[2], ng + rlo[1]:ng + rhi[1], ng + rlo[0]:ng + rhi[0]]
        g = D[:, rlo[2]:rhi[2], rlo[1]:rhi[1], rlo[0]:rhi[0]]
        err, bw = compare(g, o)
        print("region", rlo, rhi, err, bw, flush=True)
        assert err <= TOL and bw == 1.0
