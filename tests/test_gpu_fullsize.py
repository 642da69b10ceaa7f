"""GPU parity at the workloads' own sizes and step counts, through the C ABI,
in the launch configuration the benchmark times (ghost fill + advance with
the carried timestep, one box or one batched launch per stage).

* Kelvin-Helmholtz 256^3: 20 steps, every cell against the oracle stepped
  20 times on the whole box (its own timesteps).
* Rayleigh-Taylor 512^3: 20 steps of the timestep the oracle gives the
  initial state; the oracle steps windows of the box, each the compared
  region (32 x 32 columns through the whole height, both walls included,
  crossing tile and z-segment edges) widened by the scheme's reach of three
  cells per step that is left, with the cells near a window's edge left out
  step by step.  The GPU's own timestep of the result is checked to equal
  estimate_dt of it.
* The 512-box level: 20 steps with the level-wide timestep, every box
  against the per-box oracle stepped the same way.
* Serving: 24 requests of the serving stream (sides 32..192, 10..200 steps,
  all three families), many in flight at once; each result equals the same
  run alone, bit for bit.
"""
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


def _free_gpu():
    import gc
    import torch
    gc.collect()
    torch.cuda.empty_cache()


def test_kh256_twenty_steps_whole_box(gpu, orc):
    import torch
    U, box, prm = inputs.kh(256, seed=1)
    print("KH 256^3: 20 GPU steps", flush=True)
    B = gpu.Box(U, box, prm)
    gdts = []
    for _ in range(20):
        B.step()
        gdts.append(B.dt.item())
    torch.cuda.synchronize()
    g, gerr = B.state(), int(B.err.item())
    del B
    _free_gpu()
    print("KH 256^3: 20 oracle steps", flush=True)
    o, odts, oerr = orc.run(U.copy(), orc.box_from(box), orc.params_from(prm), 20, slab=64)
    assert gdts == odts and gerr == oerr == 0
    err, bw = compare(inputs.valid(g, box), inputs.valid(o, box))
    print("KH 256^3 after 20 steps: max rel err %.3e, bitwise %.6f" % (err, bw), flush=True)
    assert err <= TOL and bw == 1.0


# 32 x 32 columns: across the periodic corner, in the middle, at the high x edge
RT_REGIONS = [(-16, -16), (250, 301), (480, 100)]
RT_STEPS = 20
REACH = 3  # cells one step of the scheme reads beyond a cell, per axis


def test_rt512_twenty_steps_on_windows(gpu, orc):
    import torch
    U, box, prm = inputs.rt(512, seed=4)
    n, ng = box["n"], box["ng"]
    ob, op = orc.box_from(box), orc.params_from(prm)
    U0 = U.copy()
    orc.fill_ghosts(U0, ob)
    dt0 = orc.estimate_dt(U0, ob, op)
    del U0

    print("RT 512^3: 20 GPU steps of dt %.9e" % dt0, flush=True)
    Ud = torch.as_tensor(U).cuda()
    Un = torch.empty_like(Ud)
    ws = gpu.alloc_workspace(box)
    dt = torch.tensor([dt0], dtype=torch.float64, device="cuda")
    dtn = torch.zeros(1, dtype=torch.float64, device="cuda")
    dte = torch.zeros(1, dtype=torch.float64, device="cuda")
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    for _ in range(RT_STEPS):
        gpu.fill_ghosts(Ud, box)
        gpu.advance_box(Ud, Un, box, prm, dt, ws, err, dt_next=dtn)
        Ud, Un = Un, Ud
    gpu.estimate_dt(Ud, box, prm, dte)
    torch.cuda.synchronize()
    assert int(err.item()) == 0
    assert dtn.item() == dte.item() and dtn.item() > 0.0
    del Un, ws
    g = inputs.valid(Ud.cpu().numpy(), box)
    del Ud
    _free_gpu()

    V = inputs.valid(U, box)
    side = 32
    M = REACH * RT_STEPS
    for rx, ry in RT_REGIONS:
        print("RT 512^3: oracle window at x %d, y %d" % (rx, ry), flush=True)
        xi = np.arange(rx - M, rx + side + M) % n[0]
        yi = np.arange(ry - M, ry + side + M) % n[1]
        W = side + 2 * M
        # the window as a box of its own: the full height with the walls,
        # outflow across x and y (wrong data near those faces, which the
        # shrinking output regions never reach)
        wbox = inputs.box_desc((W, W, n[2]), ng, dx=box["dx"],
                               bc_lo=(inputs.BC_OUTFLOW, inputs.BC_OUTFLOW, inputs.BC_REFLECT))
        wob = orc.box_from(wbox)
        Wa = np.zeros(inputs.state_shape(wbox))
        inputs.valid(Wa, wbox)[...] = V[:, :, yi][:, :, :, xi]
        Wb = Wa.copy()
        werr = 0
        for s in range(1, RT_STEPS + 1):
            m = REACH * s
            orc.fill_ghosts(Wa, wob)
            werr |= orc.advance_region(Wa, Wb, wob, op, dt0, (m, m, 0), (W - m, W - m, n[2]))
            Wa, Wb = Wb, Wa
        assert werr == 0
        o = inputs.valid(Wa, wbox)[:, :, M:M + side, M:M + side]
        gr = g[:, :, yi[M:M + side]][:, :, :, xi[M:M + side]]
        e, bw = compare(gr, o)
        print("  region max rel err %.3e, bitwise %.6f" % (e, bw), flush=True)
        assert e <= TOL and bw == 1.0


def test_level512_twenty_steps(gpu, orc):
    import torch
    states, boxes, prm = inputs.level(nboxes=512, seed=2)
    print("level of 512 boxes: 20 GPU steps", flush=True)
    lev = gpu.Level(states, boxes, prm, shared_dt=True)
    gdts = []
    for _ in range(20):
        lev.step()
        gdts.append(lev.dt_min.item())
    torch.cuda.synchronize()
    gs, gerr = lev.states(), int(lev.err.item())
    del lev
    _free_gpu()
    print("level of 512 boxes: 20 oracle steps", flush=True)
    obs = [orc.box_from(b) for b in boxes]
    op = orc.params_from(prm)
    cur = [u.copy() for u in states]
    oerr = 0
    for step in range(20):
        cur, dmin, e = orc.level_step(cur, obs, op)
        oerr |= e
        assert dmin == gdts[step], step
        print("  oracle step %d" % (step + 1), flush=True)
    assert gerr == oerr == 0
    worst = 0.0
    for g, o, b in zip(gs, cur, boxes):
        e, bw = compare(inputs.valid(g, b), inputs.valid(o, b))
        worst = max(worst, e)
        assert e <= TOL and bw == 1.0, (b["n"], e, bw)
    print("level after 20 steps: max rel err %.3e over 512 boxes" % worst, flush=True)


def test_serving_stream_results_equal_runs_alone(gpu):
    import torch
    from paper_2007_05218_amd.serve import GpuExecutor, Server
    # the serving workload's stream (sides 32..192, 10..200 steps, all three
    # families), arriving fast enough that many runs share the GPU
    specs = inputs.request_stream(24, rate=200.0, seed=3)
    assert min(s["n"] for s in specs) >= 32 and max(s["n"] for s in specs) <= 192
    assert {s["family"] for s in specs} == {"sod", "kh", "smooth"}
    ex = GpuExecutor(keep_results=True, max_active=16)
    srv = Server(ex, budget_bytes=200e9, max_active=16)
    print("serving 24 requests", flush=True)
    done = srv.run(specs)
    assert len(done) == 24 and ex.error_bits() == 0
    print("peak active %d, iterations %d" % (srv.peak_active, srv.iterations), flush=True)
    assert srv.peak_active >= 8
    for r in done:
        U, box, prm = inputs.request_state({"family": r.family, "n": r.n, "seed": r.seed})
        B = gpu.Box(U, box, prm)
        B.run(r.steps)
        torch.cuda.synchronize()
        assert int(B.err.item()) == 0
        assert np.array_equal(inputs.valid(B.state(), box), inputs.valid(r.result, box)), r.id
        del B
    ex.close()
