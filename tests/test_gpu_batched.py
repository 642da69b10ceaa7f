"""Batched level (advance_boxes): every box matches the oracle and matches its
own single-box advance bitwise, with a shared (level-wide) or per-box dt."""
import numpy as np
import pytest

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


def _oracle_level(orc, states, boxes, prm, steps, shared=True):
    states = [u.copy() for u in states]
    obs = [orc.box_from(b) for b in boxes]
    op = orc.params_from(prm)
    err = 0
    for _ in range(steps):
        dts = []
        for U, ob in zip(states, obs):
            orc.fill_ghosts(U, ob)
            dts.append(orc.estimate_dt(U, ob, op))
        dmin = min(dts)
        new = []
        for U, ob, dt in zip(states, obs, dts):
            Un = U.copy()
            err |= orc.advance_box(U, Un, ob, op, dmin if shared else dt)
            new.append(Un)
        states = new
    return states, err


@pytest.mark.parametrize("shared", [True, False])
def test_level_matches_oracle(gpu, orc, shared):
    import torch
    states, boxes, prm = inputs.level(nboxes=24, seed=5)
    lev = gpu.Level(states, boxes, prm, shared_dt=shared)
    lev.run(20)
    torch.cuda.synchronize()
    gs = lev.states()
    os_, oerr = _oracle_level(orc, states, boxes, prm, 20, shared)
    assert int(lev.err.item()) == oerr
    for g, o, b in zip(gs, os_, boxes):
        err, bw = compare(inputs.valid(g, b), inputs.valid(o, b))
        assert err <= TOL and bw == 1.0, (b["n"], err, bw)


def test_full_level_batched_equals_per_box(gpu, orc):
    # the 512-box level: one batched step == 512 single-box steps, bitwise;
    # a few boxes also against the oracle
    import torch
    states, boxes, prm = inputs.level(nboxes=512, seed=2)
    lev = gpu.Level(states, boxes, prm, shared_dt=True)
    lev.step()
    torch.cuda.synchronize()
    dmin = lev.dt_min.item()
    per = lev.dt.cpu().numpy()
    gs = lev.states()
    assert dmin == per.min()
    dt = torch.tensor([dmin], dtype=torch.float64, device="cuda")
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    for b in range(len(boxes)):
        U = torch.tensor(states[b], device="cuda")
        Un = torch.empty_like(U)
        d1 = torch.zeros(1, dtype=torch.float64, device="cuda")
        gpu.estimate_dt(U, boxes[b], prm, d1)
        ws = gpu.alloc_workspace(boxes[b])
        gpu.advance_box(U, Un, boxes[b], prm, dt, ws, err)
        torch.cuda.synchronize()
        assert d1.item() == per[b]
        assert np.array_equal(inputs.valid(Un.cpu().numpy(), boxes[b]),
                              inputs.valid(gs[b], boxes[b])), b
    assert int(err.item()) == int(lev.err.item())
    op = orc.params_from(prm)
    for b in [0, 17, 255, 511]:
        U = states[b].copy()
        ob = orc.box_from(boxes[b])
        orc.fill_ghosts(U, ob)
        Un = U.copy()
        orc.advance_box(U, Un, ob, op, dmin)
        e, bw = compare(inputs.valid(gs[b], boxes[b]), inputs.valid(Un, boxes[b]))
        assert e <= TOL and bw == 1.0


def test_tile_shapes_do_not_change_results(gpu):
    # every cell's arithmetic is independent of the tile it is computed in
    import torch
    from paper_2007_05218_amd import autotune
    states, boxes, prm = inputs.level(nboxes=12, seed=8)
    shapes = {tuple(b["n"]) for b in boxes}
    res = []
    for tb in [(8, 8), (16, 64), (32, 16, 8, 32), (16, 4, 32, 128), (16, 8, 18, 32),
               (18, 16, 18, 4), (18, 4, 16, 8)]:
        table = {autotune.shape_key(n): tb for n in shapes}
        lev = gpu.Level(states, boxes, prm, shared_dt=True,
                        autotune_json=autotune.table_json(table))
        lev.run(3)
        torch.cuda.synchronize()
        res.append((lev.states(), int(lev.err.item())))
    for other, err in res[1:]:
        assert err == res[0][1]
        for a, b, box in zip(res[0][0], other, boxes):
            assert np.array_equal(inputs.valid(a, box), inputs.valid(b, box))


@pytest.mark.parametrize("flatten", [0, 1])
def test_flux_rows_of_18_match_oracle(gpu, orc, flatten):
    # tiles 18 columns wide for both kernels (the trace kernel's 18 x 14 with
    # four idle threads, the flux kernel's rows of 18 lanes, three to a
    # wavefront, ten idle lanes) on ragged boxes, 16 and 32 wide among them:
    # the oracle's bits, and those of the built-in tiles
    import torch
    from paper_2007_05218_amd import autotune
    shapes = [(16, 16, 16), (32, 16, 8), (17, 9, 20), (5, 33, 7), (4, 18, 4), (16, 40, 4)]
    states, boxes = [], []
    for i, n in enumerate(shapes):
        U, b, prm = inputs.smooth(n, seed=40 + i, dx=(1.0 / 64,) * 3)
        states.append(U)
        boxes.append(b)
    prm = dict(prm, grav=(0.0, -0.1, 0.05), flatten=flatten)
    table = {autotune.shape_key(n): (18, z, 18, z) for n, z in zip(shapes, (8, 3, 16, 2, 4, 1))}
    res = []
    for js in (None, autotune.table_json(table)):
        lev = gpu.Level(states, boxes, prm, shared_dt=True, autotune_json=js)
        lev.run(6)
        torch.cuda.synchronize()
        res.append((lev.states(), int(lev.err.item())))
    os_, oerr = _oracle_level(orc, states, boxes, prm, 6)
    assert res[1][1] == res[0][1] == oerr
    for a, b, o, box in zip(res[0][0], res[1][0], os_, boxes):
        assert np.array_equal(inputs.valid(a, box), inputs.valid(b, box)), box["n"]
        err, bw = compare(inputs.valid(b, box), inputs.valid(o, box))
        assert err <= TOL and bw == 1.0, (box["n"], err, bw)


def _seg_split(N, zs):
    # the kernels' z-segments of N planes, no longer than zs, made equal
    m = -(-N // zs)
    seg = -(-N // m)
    return [min(seg, N - i * seg) for i in range(m)]


@pytest.mark.parametrize("flatten", [0, 1])
def test_equal_z_segments_match_oracle(gpu, orc, flatten):
    # segment lengths that do not divide a box's planes: both kernels split
    # the planes into equal segments no longer than the length asked for
    # (trace kernel: the n2 + 2 traced planes; flux kernel: the n2 planes),
    # one plane per segment, and one segment for the whole box
    import torch
    from paper_2007_05218_amd import autotune
    cases = [((20, 18, 30), (16, 20, 16, 20)),   # trace 32 -> 16 + 16, flux 30 -> 15 + 15
             ((17, 21, 23), (16, 7, 18, 5)),     # 25 -> 7 7 7 4, 23 -> 5 5 5 5 3
             ((9, 12, 13), (8, 1, 16, 1)),       # a plane per segment
             ((14, 10, 11), (32, 64, 8, 64)),    # one segment
             ((16, 16, 16), (18, 17, 18, 9))]    # 18 -> 9 + 9, 16 -> 8 + 8
    for n, t in cases:
        assert _seg_split(n[2] + 2, t[1]) and _seg_split(n[2], t[3])
    states, boxes = [], []
    for i, (n, _) in enumerate(cases):
        U, b, prm = inputs.smooth(n, seed=70 + i, dx=(1.0 / 64,) * 3)
        states.append(U)
        boxes.append(b)
    prm = dict(prm, grav=(0.02, 0.0, -0.1), flatten=flatten)
    table = {autotune.shape_key(n): t for n, t in cases}
    lev = gpu.Level(states, boxes, prm, shared_dt=True, autotune_json=autotune.table_json(table))
    lev.run(5)
    torch.cuda.synchronize()
    g, gerr = lev.states(), int(lev.err.item())
    os_, oerr = _oracle_level(orc, states, boxes, prm, 5)
    assert gerr == oerr
    for a, o, box in zip(g, os_, boxes):
        err, bw = compare(inputs.valid(a, box), inputs.valid(o, box))
        assert err <= TOL and bw == 1.0, (box["n"], err, bw)


def test_autotuner_runs(gpu):
    from paper_2007_05218_amd import autotune
    boxes = [inputs.box_desc((16, 32, 16)), inputs.box_desc((32, 16, 64))]
    table, timings = autotune.tune(boxes, max_boxes_per_class=4, min_cells_per_class=1,
                                   reps=1)
    assert set(timings) == {"16x32x16", "32x16x64"} and set(table) <= set(timings)
    for k, (tbx1, tzs1, tbx2, tzs2) in table.items():
        assert (tbx1, tzs1) == autotune.BUILTIN or (tbx1 in (8, 16, 18, 32) and tzs1 >= 1)
        assert (tbx2, tzs2) == autotune.BUILTIN or (tbx2 in (8, 16, 18, 32) and tzs2 >= 1)
        assert (tbx1, tzs1, tbx2, tzs2) != autotune.BUILTIN * 2
    gpu.Plan(boxes, autotune.table_json(table)).close()
    # a table keeping one kernel's built-in tile is accepted
    gpu.Plan(boxes, autotune.table_json({"16x32x16": (16, 8) + autotune.BUILTIN})).close()
    # the level-wide check keeps the table only if the level runs faster with it
    states = [inputs.smooth(b["n"], seed=i)[0] for i, b in enumerate(boxes)]
    kept, ms_builtin, ms_table = autotune.validate(
        states, boxes, inputs.params_desc(), {"16x32x16": (8, 4, 8, 4)}, steps=1, rounds=1)
    assert ms_builtin > 0 and ms_table > 0
    assert kept == ({"16x32x16": (8, 4, 8, 4)} if ms_table < ms_builtin else {})


def test_batched_fused_next_timesteps(gpu):
    # advance_boxes' dt_next / dt_next_min equal estimate_dt_boxes of the new
    # states, bit for bit, with per-box and with shared timesteps
    import torch
    states, boxes, prm = inputs.level(nboxes=12, seed=5)
    plan = gpu.Plan(boxes)
    U = [torch.as_tensor(u).cuda() for u in states]
    Un = [torch.empty_like(u) for u in U]
    pa, pb = gpu.pointer_array(U), gpu.pointer_array(Un)
    ws = torch.empty(max(plan.ws_bytes, 256), dtype=torch.uint8, device="cuda")
    nb = len(boxes)
    dt, dtn, dte = (torch.zeros(nb, dtype=torch.float64, device="cuda") for _ in range(3))
    dmin, dnmin, demin = (torch.zeros(1, dtype=torch.float64, device="cuda") for _ in range(3))
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    for shared in (True, False):
        gpu.estimate_dt_boxes(plan, pa, prm, dt, dmin)
        gpu.advance_boxes(plan, pa, pb, prm, dmin if shared else dt, ws, err,
                          dt_stride=0 if shared else 1, dt_next=dtn, dt_next_min=dnmin)
        gpu.estimate_dt_boxes(plan, pb, prm, dte, demin)
        torch.cuda.synchronize()
        assert torch.equal(dtn, dte) and dnmin.item() == demin.item()
        assert dnmin.item() == dte.min().item()
        pa, pb = pb, pa
    plan.close()
