"""A level of boxes tiling one domain (hydro_level_create,
hydro_fill_ghosts_level): the GPU ghost exchange equals the oracle's bit for
bit, a tiled level advances exactly like the domain as one box, and the Sedov
blast run as a tiled level matches the oracle and follows the self-similar
solution."""
import numpy as np
import pytest

import sedov_exact
from oracle import level as olev
from parity import compare
from paper_2007_05218_amd import inputs

pytestmark = pytest.mark.gpu
TOL = 1e-11
P, O, R = inputs.BC_PERIODIC, inputs.BC_OUTFLOW, inputs.BC_REFLECT


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_2007_05218_amd import hydro
    hydro.lib()
    return hydro


LAYOUTS = [
    # domain, ghost depth, boundary kinds (low, high), cuts per axis
    ((32, 32, 32), 4, ((P, P, P), (P, P, P)), ([0, 16, 32], [0, 16, 32], [0, 16, 32])),
    ((40, 24, 36), 4, ((P, O, R), (P, R, O)), ([0, 8, 13, 40], [0, 24], [0, 5, 20, 36])),
    ((19, 17, 23), 3, ((O, P, R), (R, P, R)), ([0, 3, 19], [0, 10, 17], [0, 23])),
    ((48, 16, 16), 4, ((R, R, R), (R, R, R)), ([0, 16, 32, 48], [0, 16], [0, 16])),
]


@pytest.mark.parametrize("lay", range(len(LAYOUTS)))
def test_level_fill_matches_oracle(gpu, lay):
    import torch
    dom, ng, (bl, bh), cuts = LAYOUTS[lay]
    print("level fill layout", dom, ng, bl, bh, flush=True)
    box = inputs.box_desc(dom, ng, bc_lo=bl, bc_hi=bh)
    rng = np.random.default_rng(10 + lay)
    U = np.zeros(inputs.state_shape(box))
    inputs.valid(U, box)[...] = rng.standard_normal(inputs.valid(U, box).shape)
    states, boxes, lo, til = inputs.tile(U, box, cuts)
    want = olev.fill_ghosts_level(states, boxes, lo, til["dom"], til["bc_lo"], til["bc_hi"])
    # ghosts start as NaN so a ghost cell the kernel misses cannot compare equal
    dev = []
    for S, b in zip(states, boxes):
        T = np.full_like(S, np.nan)
        inputs.valid(T, b)[...] = inputs.valid(S, b)
        dev.append(torch.as_tensor(T).cuda())
    til_h = gpu.Tiling(boxes, lo, til["dom"], til["bc_lo"], til["bc_hi"])
    gpu.fill_ghosts_level(til_h, gpu.pointer_array(dev))
    torch.cuda.synchronize()
    for G, W in zip(dev, want):
        assert np.array_equal(G.cpu().numpy(), W)
    til_h.close()


def test_level_fill_mixed_ghost_depths(gpu):
    # boxes of one level may carry different ghost depths (3 and 4 here)
    import torch
    dom = (24, 20, 16)
    box = inputs.box_desc(dom, 4, bc_lo=(P, R, O), bc_hi=(P, O, R))
    rng = np.random.default_rng(21)
    U = np.zeros(inputs.state_shape(box))
    inputs.valid(U, box)[...] = rng.standard_normal(inputs.valid(U, box).shape)
    states, boxes, lo, til = inputs.tile(U, box, ([0, 10, 24], [0, 20], [0, 7, 16]))
    for i in (1, 2):  # re-cut two boxes with three ghost layers
        b = dict(boxes[i], ng=3)
        W = np.zeros(inputs.state_shape(b))
        inputs.valid(W, b)[...] = inputs.valid(states[i], boxes[i])
        states[i], boxes[i] = W, b
    want = olev.fill_ghosts_level(states, boxes, lo, til["dom"], til["bc_lo"], til["bc_hi"])
    dev = []
    for S, b in zip(states, boxes):
        T = np.full_like(S, np.nan)
        inputs.valid(T, b)[...] = inputs.valid(S, b)
        dev.append(torch.as_tensor(T).cuda())
    tl = gpu.Tiling(boxes, lo, til["dom"], til["bc_lo"], til["bc_hi"])
    gpu.fill_ghosts_level(tl, gpu.pointer_array(dev))
    torch.cuda.synchronize()
    for G, W in zip(dev, want):
        assert np.array_equal(G.cpu().numpy(), W)
    tl.close()


def _domain_run(gpu, U, box, prm, steps):
    import torch
    B = gpu.Box(U, box, prm)
    B.run(steps)
    torch.cuda.synchronize()
    return B.state(), int(B.err.item())


@pytest.mark.parametrize("case", ["rt", "sod"])
def test_tiled_level_equals_domain_box(gpu, orc, case):
    # 20 steps of uneven boxes with the level's ghost exchange equal 20 steps
    # of the domain as one box, bit for bit, and the oracle's domain run
    import torch
    if case == "rt":
        U, box, prm = inputs.rt((40, 32, 48), seed=4)
        cuts = ([0, 16, 23, 40], [0, 9, 32], [0, 16, 29, 48])
    else:
        U, box, prm = inputs.sod((48, 20, 16), axis=0)
        cuts = ([0, 20, 26, 48], [0, 20], [0, 8, 16])
    print("tiled level", case, box["n"], flush=True)
    states, boxes, lo, til = inputs.tile(U, box, cuts)
    tiling = gpu.Tiling(boxes, lo, til["dom"], til["bc_lo"], til["bc_hi"])
    lev = gpu.Level(states, boxes, prm, shared_dt=True, tiling=tiling)
    lev.run(20)
    torch.cuda.synchronize()
    got = lev.states()
    whole, derr = _domain_run(gpu, U, box, prm, 20)
    assert int(lev.err.item()) == derr
    W = inputs.valid(whole, box)
    for G, b, l in zip(got, boxes, lo):
        n = b["n"]
        assert np.array_equal(inputs.valid(G, b),
                              W[:, l[2]:l[2] + n[2], l[1]:l[1] + n[1], l[0]:l[0] + n[0]])
    D = U.copy()
    ob, op = orc.box_from(box), orc.params_from(prm)
    for _ in range(20):
        orc.fill_ghosts(D, ob)
        dt = orc.estimate_dt(D, ob, op)
        Dn = D.copy()
        orc.advance_box(D, Dn, ob, op, dt)
        D = Dn
    err, bw = compare(W, inputs.valid(D, box))
    assert err <= TOL and bw == 1.0


def test_sedov_level_matches_oracle(gpu, orc):
    # the paper's blast problem as 8 boxes of 32^3 tiling a 64^3 domain, 20
    # steps, against the oracle's 64^3 box
    import torch
    states, boxes, prm, lo, til = inputs.sedov_level(64, 32)
    U, box, _ = inputs.sedov(64)
    tiling = gpu.Tiling(boxes, lo, til["dom"], til["bc_lo"], til["bc_hi"])
    lev = gpu.Level(states, boxes, prm, shared_dt=True, tiling=tiling)
    lev.run(20)
    torch.cuda.synchronize()
    D = U.copy()
    ob, op = orc.box_from(box), orc.params_from(prm)
    oerr = 0
    for _ in range(20):
        orc.fill_ghosts(D, ob)
        dt = orc.estimate_dt(D, ob, op)
        Dn = D.copy()
        oerr |= orc.advance_box(D, Dn, ob, op, dt)
        D = Dn
    assert int(lev.err.item()) == oerr
    W = inputs.valid(D, box)
    for G, b, l in zip(lev.states(), boxes, lo):
        n = b["n"]
        part = W[:, l[2]:l[2] + n[2], l[1]:l[1] + n[1], l[0]:l[0] + n[0]]
        err, bw = compare(inputs.valid(G, b), part)
        assert err <= TOL and bw == 1.0


def test_sedov_gpu_follows_similarity(gpu):
    # 128^3 blast as 8 boxes of 64^3: shock radius within 4% of the
    # self-similar one at t = 0.01 and t = 0.04; mass and energy conserved
    import torch
    n = 128
    states, boxes, prm, lo, til = inputs.sedov_level(n, 64)
    tiling = gpu.Tiling(boxes, lo, til["dom"], til["bc_lo"], til["bc_hi"])
    lev = gpu.Level(states, boxes, prm, shared_dt=True, tiling=tiling)
    U0, dbox, _ = inputs.sedov(n)
    m0, e0 = (inputs.valid(U0, dbox)[c].sum() for c in (0, 4))
    x, y, z = inputs.cell_centres(dbox)
    r = np.broadcast_to(np.sqrt((x - 0.5) ** 2 + (y - 0.5) ** 2 + (z - 0.5) ** 2), (n,) * 3)
    t, marks, radii = 0.0, [0.01, 0.04], {}
    while marks:
        lev.step()
        t += lev.dt_min.item()
        if t >= marks[0]:
            marks.pop(0)
            D = np.zeros((5, n, n, n))
            for G, b, l in zip(lev.states(), boxes, lo):
                m = b["n"]
                D[:, l[2]:l[2] + m[2], l[1]:l[1] + m[1], l[0]:l[0] + m[0]] = inputs.valid(G, b)
            radii[t] = sedov_exact.measured_radius(D[0], r, n, 0.5)
    torch.cuda.synchronize()
    assert int(lev.err.item()) & 7 == 0
    assert D[0].sum() == pytest.approx(m0, rel=1e-12)
    assert D[4].sum() == pytest.approx(e0, rel=1e-12)
    for tt, rr in radii.items():
        assert rr == pytest.approx(sedov_exact.shock_radius(tt), rel=0.04), (tt, rr)


def test_tiled_flattened_level_graph_replay(gpu):
    # two steps of a tiled level (ghost exchange, flattening, batched
    # advance) captured in a HIP graph; every replay equals the eager steps
    import torch
    states, boxes, prm, lo, til = inputs.sedov_level(64, 32)
    prm = dict(prm, flatten=1)

    def make():
        tiling = gpu.Tiling(boxes, lo, til["dom"], til["bc_lo"], til["bc_hi"])
        return gpu.Level(states, boxes, prm, shared_dt=True, tiling=tiling), tiling

    eager, t1 = make()
    refs = []
    for _ in range(3):
        eager.run(2)
        torch.cuda.synchronize()
        refs.append(eager.states())
    lev, t2 = make()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    snap = [u.clone() for u in lev.U]
    with torch.cuda.stream(s):  # warm-up outside the graph
        lev.step()
        lev.step()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for u, v in zip(lev.U, snap):
        u.copy_(v)
    lev.invalidate_dt()
    lev.err.zero_()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        lev.step()
        lev.step()
    for rep in range(3):
        g.replay()
        junk = torch.ones(1000, device="cuda").sum()
        torch.cuda.synchronize()
        assert junk.item() == 1000.0
        for a, b, box in zip([u.cpu().numpy() for u in lev.U], refs[rep], boxes):
            assert np.array_equal(inputs.valid(a, box), inputs.valid(b, box)), rep
    assert int(lev.err.item()) & 7 == 0


def test_sedov_shock_radius_converges(gpu):
    # the blast front converges to the self-similar radius as the grid is
    # refined (64^3, 128^3, 256^3, each as boxes of 64^3 tiling the domain)
    import torch
    errs = []
    for n in (64, 128, 256):
        states, boxes, prm, lo, til = inputs.sedov_level(n, 64)
        tiling = gpu.Tiling(boxes, lo, til["dom"], til["bc_lo"], til["bc_hi"])
        lev = gpu.Level(states, boxes, prm, shared_dt=True, tiling=tiling)
        t = 0.0
        while t < 0.03:
            lev.step()
            t += lev.dt_min.item()
        torch.cuda.synchronize()
        assert int(lev.err.item()) & 7 == 0
        D = np.zeros((n, n, n))
        for G, b, l in zip(lev.states(), boxes, lo):
            m = b["n"]
            D[l[2]:l[2] + m[2], l[1]:l[1] + m[1], l[0]:l[0] + m[0]] = inputs.valid(G, b)[0]
        x = (np.arange(n) + 0.5) / n
        r = np.sqrt((x[None, None, :] - 0.5) ** 2 + (x[None, :, None] - 0.5) ** 2 +
                    (x[:, None, None] - 0.5) ** 2)
        R = sedov_exact.measured_radius(D, r, n, 0.5)
        errs.append(abs(R / sedov_exact.shock_radius(t) - 1.0))
        print("sedov n=%d t=%.4f R=%.4f err=%.4f" % (n, t, R, errs[-1]), flush=True)
        del lev
        tiling.close()
        torch.cuda.empty_cache()
    assert errs[0] > errs[1] > errs[2] and errs[2] < 0.015, errs


def test_level_fill_rejects_a_mismatched_pointer_count(gpu):
    # argument errors are returned before anything is launched
    import ctypes
    import torch
    U, box, prm = inputs.sedov(32)
    states, boxes, lo, til = inputs.tile(U, box, ([0, 16, 32], [0, 32], [0, 32]))
    tl = gpu.Tiling(boxes, lo, til["dom"], til["bc_lo"], til["bc_hi"])
    dev = [torch.as_tensor(st).cuda() for st in states]
    ptrs = gpu.pointer_array(dev)
    L = gpu.lib()
    assert L.hydro_fill_ghosts_level(1, ctypes.c_void_p(ptrs.data_ptr()), tl.handle,
                                     None) == gpu.HYDRO_EINVAL
    assert L.hydro_fill_ghosts_level(2, None, tl.handle, None) == gpu.HYDRO_EINVAL
    tl.close()
