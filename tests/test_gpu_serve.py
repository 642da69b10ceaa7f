"""Serving and graph capture on the GPU: each served result equals the same run
alone (bitwise), and a captured batched step replays to the eager result."""
import numpy as np
import pytest

from parity import compare
from paper_2007_05218_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_2007_05218_amd import hydro
    hydro.lib()
    return hydro


def test_served_equals_alone(gpu, orc):
    import torch
    from paper_2007_05218_amd.serve import GpuExecutor, Server
    specs = inputs.request_stream(10, rate=400.0, seed=7, nmin=16, nmax=40, smin=4, smax=14)
    ex = GpuExecutor(keep_results=True)
    srv = Server(ex, budget_bytes=20e9, max_active=6)
    done = srv.run(specs)
    assert len(done) == 10 and ex.error_bits() == 0
    assert srv.peak_active > 1  # the runs really were batched together
    for r in done:
        U, box, prm = inputs.request_state({"family": r.family, "n": r.n, "seed": r.seed})
        B = gpu.Box(U, box, prm)
        B.run(r.steps)
        torch.cuda.synchronize()
        alone = B.state()
        assert np.array_equal(inputs.valid(alone, box), inputs.valid(r.result, box)), r.id
    # and one of them against the oracle
    r = done[0]
    U, box, prm = inputs.request_state({"family": r.family, "n": r.n, "seed": r.seed})
    o, _, _ = orc.run(U, orc.box_from(box), orc.params_from(prm), r.steps)
    err, bw = compare(inputs.valid(r.result, box), inputs.valid(o, box))
    assert err <= 1e-11 and bw == 1.0
    m = srv.metrics()
    assert m["p50_s"] > 0 and m["p99_s"] >= m["p50_s"]
    # requests that bring their initial states give the same results
    for s in specs:
        s["state"] = inputs.request_state(s)
    ex2 = GpuExecutor(keep_results=True)
    done2 = Server(ex2, budget_bytes=20e9, max_active=6).run(specs)
    for a, b in zip(done, done2):
        assert np.array_equal(a.result, b.result), a.id


def test_graph_replay_equals_eager(gpu):
    import torch
    states, boxes, prm = inputs.level(nboxes=6, seed=9)
    eager = gpu.Level(states, boxes, prm, shared_dt=True)
    refs = []
    for _ in range(3):
        eager.run(2)
        torch.cuda.synchronize()
        refs.append(eager.states())

    lev = gpu.Level(states, boxes, prm, shared_dt=True)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    # capture two steps so the state ends in the buffers it started in
    snap = [u.clone() for u in lev.U]
    with torch.cuda.stream(s):
        lev.step()
        lev.step()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for u, v in zip(lev.U, snap):
        u.copy_(v)
    lev.invalidate_dt()  # the restored states' timesteps are not the carried ones
    lev.err.zero_()
    with torch.cuda.graph(g):
        lev.step()
        lev.step()
    for rep in range(3):
        g.replay()
        # unrelated eager work between replays
        junk = torch.ones(1000, device="cuda").sum()
        torch.cuda.synchronize()
        assert junk.item() == 1000.0
        got = [u.cpu().numpy() for u in lev.U]
        for a, b, box in zip(got, refs[rep], boxes):
            assert np.array_equal(inputs.valid(a, box), inputs.valid(b, box)), rep
    assert int(lev.err.item()) == 0


def test_capacity_plan_updates_are_stream_ordered(gpu):
    # one plan made with a capacity, refilled for several lists of boxes with
    # no host synchronisation in between (more updates than it has staging
    # buffers): every list's step equals the same step with a fixed plan
    import torch
    states, boxes, prm = inputs.level(nboxes=12, seed=4)
    lists = [[0, 1, 2, 3, 4], [2, 5, 6], [7, 8, 9, 10, 11, 0, 3], [4], [1, 9, 5, 11],
             [6, 7], [10, 2, 8]]
    cap = gpu.Plan.with_capacity(8)
    assert gpu.lib().hydro_plan_boxes(cap.handle) == 0
    U = [torch.as_tensor(u).cuda() for u in states]
    ws = torch.empty(max(gpu.workspace_bytes(boxes), 256), dtype=torch.uint8, device="cuda")
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    # every buffer first, so that the loop below enqueues only
    outs = [[torch.empty_like(U[b]) for b in sel] for sel in lists]
    ptrs = [(gpu.pointer_array([U[b] for b in sel]), gpu.pointer_array(Un))
            for sel, Un in zip(lists, outs)]
    dts = [torch.zeros(len(sel), dtype=torch.float64, device="cuda") for sel in lists]
    torch.cuda.synchronize()
    for sel, (pa, pb), dt in zip(lists, ptrs, dts):
        cap.update([boxes[b] for b in sel])
        assert cap.ws_bytes == gpu.workspace_bytes([boxes[b] for b in sel])
        gpu.estimate_dt_boxes(cap, pa, prm, dt)
        gpu.advance_boxes(cap, pa, pb, prm, dt, ws, err, dt_stride=1)
    torch.cuda.synchronize()
    assert int(err.item()) == 0
    for sel, got in zip(lists, outs):
        fixed = gpu.Plan([boxes[b] for b in sel])
        Un = [torch.empty_like(U[b]) for b in sel]
        pa, pb = gpu.pointer_array([U[b] for b in sel]), gpu.pointer_array(Un)
        dt = torch.zeros(len(sel), dtype=torch.float64, device="cuda")
        gpu.estimate_dt_boxes(fixed, pa, prm, dt)
        gpu.advance_boxes(fixed, pa, pb, prm, dt, ws, err, dt_stride=1)
        torch.cuda.synchronize()
        for b, x, y in zip(sel, got, Un):
            assert np.array_equal(inputs.valid(x.cpu().numpy(), boxes[b]),
                                  inputs.valid(y.cpu().numpy(), boxes[b])), (sel, b)
        fixed.close()
    # refused updates leave the plan as it was
    with pytest.raises(gpu.HydroError):
        cap.update(boxes[:9])  # beyond the capacity
    bad = dict(boxes[0], n=(0, 4, 4))
    with pytest.raises(gpu.HydroError):
        cap.update([boxes[1], bad])
    assert gpu.lib().hydro_plan_boxes(cap.handle) == len(lists[-1])
    cap.close()
