#!/usr/bin/env python3
"""Throughput benchmark of the FP64 CTU-PPM + HLLC hydro step on one MI355X.

A step is the whole hot path on one box: ghost fill + CFL timestep reduction
(estimate_dt) and the advance (advance_box), all on the device, inputs
resident in HBM before timing starts.  The headline workload is the 512^3
Rayleigh-Taylor box (FP64, gamma = 1.4, g = -0.1 z, reflecting z walls);
`value` = valid cells x timed steps / device time (HIP events on the stream
the library launches on), in cell-updates per second.

Also reported on the same JSON line:
  roofline      the dominant kernel's achieved FP64 rate (algorithmic flops
                per cell-update, counted by the oracle's operation-counting
                build, x cells / the kernel's average device time per step,
                from HIP events the library records around it) against
                MI355X's published FP64 vector peak (78.6 TFLOP/s), with the
                single add/multiply issue rate (39.3 T/s) as a labelled
                second figure; per kernel also its HBM rates (algorithmic
                bytes and the committed FETCH_SIZE + WRITE_SIZE counters, per
                launch, over its time) against 8 TB/s and the practical roof
                of a plain copy kernel timed in the same run; and, from the
                committed counters, the instructions each kernel executed and
                the step's cell-updates/s against the roof its FP64 VALU
                instructions set
  cpu_baseline  the CPU oracle timed on the host on a bounded sample of the
                same workload (rank 0, N = 1 only), with the CPU model and
                one-thread rates on the Sod 32^3 tube and the KH box at 64^3
  also          secondary workloads: the 256^3 Kelvin-Helmholtz box, also
                with two passively advected species; the
                paper's Sedov blast at its per-node size (256^3 as 64 boxes of
                64^3 tiling the domain, with the ghost exchange between boxes,
                and as one box); the 512-box batched level (one launch per
                stage for all boxes) against the same boxes launched one by
                one (on one stream, and dealt to 8 streams); the serving loop
                (p50/p99 latency and cell-updates/s at 80% load, and its
                saturated capacity batched vs one request at a time)

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workloads ...]
(defaults: 50 timed steps after 3 warm-up steps, every workload)
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X's published dense FP64 vector peak (an FMA counted as two flops)
PEAK_FP64 = 78.6e12
# the same units' issue rate of single adds or multiplies (the arithmetic
# contract forbids contracting them into FMAs): 256 CUs x 64 FP64 lanes per
# clock x 2.4 GHz -- reported beside the published peak, labelled
PEAK_FP64_NOFMA = 256 * 64 * 2.4e9
HBM_PEAK = 8.0e12
# oracle stages computed by each kernel group of the library's advance
KERNEL_STAGES = {"trace": ["prim", "trace"],
                 "flux_update": ["flux1", "corner_flux2", "final_flux3", "update"]}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "rt512_traffic.json")
KERNEL_SYMBOL = {"trace": "k_trace_fused<false>", "flux_update": "k_flux_fused<false>"}
# each kernel's algorithmic HBM bytes per cell-update (its inputs read once,
# its outputs written once): the trace kernel reads the state (40 B) and
# writes the 30 traced face states (240 B) of a cell; the flux kernel reads
# those and the state and writes the new state (320 B)
ALG_BYTES = {"trace": 280.0, "flux_update": 320.0}


# the sources the profiled step kernels are built from
STEP_SOURCES = ("flux_fused.h", "hydro.hip", "hydro_common.h", "trace_fused.h")


def source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in STEP_SOURCES:
        with open(os.path.join(ROOT, "paper_2007_05218_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_counters(kernel):
    """Per-launch counters of `kernel` from the committed counter profile, if
    it was taken on the current kernel sources; else None."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != source_hash():
        return None
    return t.get("kernels", {}).get(KERNEL_SYMBOL.get(kernel, kernel))


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` (FETCH_SIZE + WRITE_SIZE, scaled),
    from the committed counter profile; None if it is stale."""
    k = measured_counters(kernel)
    if not k or k.get("fetch_bytes") is None or k.get("write_bytes") is None:
        return None
    return k["fetch_bytes"] + k["write_bytes"]


# FP64 VALU instructions a wave issues: add, multiply, FMA, transcendental
FP64_INSTS = ("SQ_INSTS_VALU_ADD_F64", "SQ_INSTS_VALU_MUL_F64", "SQ_INSTS_VALU_FMA_F64",
              "SQ_INSTS_VALU_TRANS_F64")
# lane-instruction issue rate of the chip: 256 CUs x 4 SIMDs x 16 lanes per clock
LANE_ISSUE_PER_S = 256 * 64 * 2.4e9


def executed_valu(kernel, ncell):
    """From the committed counters (None if stale): FP64 VALU and all VALU
    lane-instructions per cell-update of one launch over ncell cells, and the
    FP64 flops the hardware executed per cell-update (an FMA counted twice)."""
    k = measured_counters(kernel)
    if not k or any(c not in k for c in FP64_INSTS + ("SQ_INSTS_VALU", "SQ_INSTS_VALU_FLOPS_FP64")):
        return None
    return {"fp64_valu_instr_per_cu": 64 * sum(k[c] for c in FP64_INSTS) / ncell,
            "valu_instr_per_cu": 64 * k["SQ_INSTS_VALU"] / ncell,
            "executed_fp64_flops_per_cu": 64 * k["SQ_INSTS_VALU_FLOPS_FP64"] / ncell}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workloads", default="rt512,kh256,species,sedov,level,serve",
                    help="comma list of rt512, kh256, sedov, level, serve, copy (a plain 2 GiB "
                         "device copy, the reference for HBM traffic counters)")
    ap.add_argument("--serve-requests", type=int, default=1000)
    ap.add_argument("--serve-warmup", type=int, default=50)
    ap.add_argument("--serve-states", type=int, default=96,
                    help="distinct initial states the serving stream's requests cycle through")
    ap.add_argument("--level-steps", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    return ap.parse_args()


def time_box(hydro, torch, U, box, prm, steps, warmup, B=None):
    B = B if B is not None else hydro.Box(U, box, prm)
    for _ in range(warmup):
        B.step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(steps):
        B.step()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    # per-stage device time, in a separate pass with the library's stage events
    timer = hydro.StageTimer()
    for _ in range(steps):
        with timer:
            B.step()
    err = int(B.err.item())
    del B
    torch.cuda.empty_cache()
    return ms, wall, timer, err


def time_species(hydro, torch, inputs, steps, warmup, ns=2, n=256):
    """KH n^3 with ns passively advected species (advance_box_species) against
    the same box without them; the species pass's time and the bytes it must
    move at least, as a bandwidth: the twelve exported mass fluxes and the six
    traced densities over the index box [-1, n]^3 and the gas state, each read
    once, the partial densities read and written once."""
    U, box, prm = inputs.kh(n, seed=1)
    S = inputs.species(U, box, ns, seed=3)
    B = hydro.SpeciesBox(U, S, box, prm)
    ms, _, timer, err = time_box(hydro, torch, None, box, prm, steps, warmup, B=B)
    del B
    torch.cuda.empty_cache()
    ms0, _, _, _ = time_box(hydro, torch, U, box, prm, steps, warmup)
    ncell = n ** 3
    st = {k: v / max(timer.calls, 1) for k, v in timer.total_ms.items()}
    sp_ms = st.get("species", 0.0)
    e = (n + 2) ** 3
    pass_bytes = (12 + 6) * 8 * e + 5 * 8 * ncell + 2 * 8 * ns * ncell
    # the Sedov blast as a tiled level (256^3 in 64^3 boxes) with the same
    # species count: both ghost exchanges and the batched species step
    states, boxes, prm_s, lo, til = inputs.sedov_level(256, 64)
    U0, box0, _ = inputs.sedov(256)
    S0 = inputs.species(U0, box0, ns, seed=8)
    sst, _, _, _ = inputs.tile(S0, box0, [inputs.even_cuts(256, 64)] * 3)
    del U0, S0
    tiling = hydro.Tiling(boxes, lo, til["dom"], til["bc_lo"], til["bc_hi"])
    lev = hydro.Level(states, boxes, prm_s, shared_dt=True, tiling=tiling, species=sst)
    for _ in range(warmup):
        lev.step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        lev.step()
    e1.record()
    torch.cuda.synchronize()
    ms_lev = e0.elapsed_time(e1) / steps
    err |= int(lev.err.item())
    del lev
    tiling.close()
    torch.cuda.empty_cache()
    return {"species": ns, "cu_per_s": ncell * steps / (ms * 1e-3),
            "sedov256_tiled_level_cu_per_s": 256 ** 3 / (ms_lev * 1e-3),
            "sedov256_tiled_level_ms_per_step": ms_lev,
            "ms_per_step": ms / steps, "ms_per_step_without_species": ms0 / steps,
            "stage_ms": {k: round(v, 3) for k, v in st.items()},
            "species_pass_ms": sp_ms,
            "species_pass_min_GB": pass_bytes / 1e9,
            "species_pass_GBps": pass_bytes / (sp_ms * 1e-3) / 1e9 if sp_ms > 0 else None,
            "err": err}


def _time_level_once(hydro, torch, states, boxes, prm, steps, warmup, table=None):
    lev = hydro.Level(states, boxes, prm, shared_dt=True, autotune_json=table)
    for _ in range(warmup):
        lev.step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        lev.step()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    del lev
    torch.cuda.empty_cache()
    return ms


def time_level(hydro, torch, inputs, steps, warmup):
    from paper_2007_05218_amd import autotune
    states, boxes, prm = inputs.level(nboxes=512, seed=2)
    cells = sum(b["n"][0] * b["n"][1] * b["n"][2] for b in boxes)
    t0 = time.perf_counter()
    table, _ = autotune.tune(boxes, prm, log=log)
    table, ms_b, ms_t = autotune.validate(states, boxes, prm, table)
    log("tile table validated on the level: built-in %s ms, tuned %s ms per step -> %s"
        % (ms_b, ms_t, "tuned" if table else "built-in"))
    tune_s = time.perf_counter() - t0
    js = autotune.table_json(table) if table else None
    ms_default = _time_level_once(hydro, torch, states, boxes, prm, steps, warmup)
    ms_batched = _time_level_once(hydro, torch, states, boxes, prm, steps, warmup, js)
    # the batched step captured in a HIP graph (two steps per graph, so the
    # states end in the buffers they started in), replayed
    lev = hydro.Level(states, boxes, prm, shared_dt=True, autotune_json=js)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        lev.step()
        lev.step()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        lev.step()
        lev.step()
    graph.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = max(1, steps // 2)
    e0.record()
    for _ in range(reps):
        graph.replay()
    e1.record()
    torch.cuda.synchronize()
    ms_graph = e0.elapsed_time(e1) / (2 * reps)
    del graph, lev
    torch.cuda.empty_cache()
    # the same boxes, one library call per box and stage (one stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    Us = [torch.tensor(u, device="cuda") for u in states]
    Uns = [torch.empty_like(u) for u in Us]
    ws = hydro.alloc_workspace(max(boxes, key=lambda b: hydro.workspace_bytes(b)))
    dts = torch.zeros(len(boxes), dtype=torch.float64, device="cuda")
    err = torch.zeros(1, dtype=torch.int32, device="cuda")

    def per_box_step():
        for b in range(len(boxes)):
            hydro.estimate_dt(Us[b], boxes[b], prm, dts[b:b + 1])
        dmin = dts.min().reshape(1)
        for b in range(len(boxes)):
            hydro.advance_box(Us[b], Uns[b], boxes[b], prm, dmin, ws, err)
        for b in range(len(boxes)):
            Us[b], Uns[b] = Uns[b], Us[b]

    for _ in range(warmup):
        per_box_step()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        per_box_step()
    e1.record()
    torch.cuda.synchronize()
    ms_per_box = e0.elapsed_time(e1)
    # the paper's remedy for small boxes (Sec. IV-A): one call per box as
    # above, the boxes dealt round-robin to 8 streams, each with its own
    # workspace
    streams = [torch.cuda.Stream() for _ in range(8)]
    wss = [ws] + [hydro.alloc_workspace(max(boxes, key=lambda b: hydro.workspace_bytes(b)))
                  for _ in streams[1:]]

    def per_box_streams_step():
        cur = torch.cuda.current_stream()
        for s in streams:
            s.wait_stream(cur)
        for b in range(len(boxes)):
            hydro.estimate_dt(Us[b], boxes[b], prm, dts[b:b + 1], stream=streams[b % 8])
        for s in streams:
            cur.wait_stream(s)
        dmin = dts.min().reshape(1)
        for s in streams:
            s.wait_stream(cur)
        for b in range(len(boxes)):
            hydro.advance_box(Us[b], Uns[b], boxes[b], prm, dmin, wss[b % 8], err,
                              stream=streams[b % 8])
        for s in streams:
            cur.wait_stream(s)
        for b in range(len(boxes)):
            Us[b], Uns[b] = Uns[b], Us[b]

    for _ in range(warmup):
        per_box_streams_step()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        per_box_streams_step()
    e1.record()
    torch.cuda.synchronize()
    ms_streams = e0.elapsed_time(e1)
    del Us, Uns, ws, wss, streams
    torch.cuda.empty_cache()
    return {"workload": "level512: 512 periodic boxes, sides from {16,32,64} per axis, "
                        "smooth random fields, dx=1/64, shared dt, seed 2",
            "boxes": len(boxes), "cells": cells, "steps": steps,
            "batched_cu_per_s": cells * steps / (ms_batched * 1e-3),
            "batched_untuned_cu_per_s": cells * steps / (ms_default * 1e-3),
            "per_box_cu_per_s": cells * steps / (ms_per_box * 1e-3),
            "per_box_8_streams_cu_per_s": cells * steps / (ms_streams * 1e-3),
            "batched_ms_per_step": ms_batched / steps, "per_box_ms_per_step": ms_per_box / steps,
            "batched_graph_ms_per_step": ms_graph,
            "autotune_s": tune_s, "tile_table": table}


def time_sedov(hydro, torch, inputs, steps, warmup, n=256, bs=64):
    """The paper's blast problem at its per-node size (Sec. IV-A: 256^3 cells
    per node in 64^3 boxes): the domain as a tiled level of (n/bs)^3 boxes
    (ghost exchange between boxes + batched advance), its ghost exchange on
    its own, and the same domain advanced as one box."""
    states, boxes, prm, lo, til = inputs.sedov_level(n, bs)
    tiling = hydro.Tiling(boxes, lo, til["dom"], til["bc_lo"], til["bc_hi"])
    lev = hydro.Level(states, boxes, prm, shared_dt=True, tiling=tiling)
    for _ in range(warmup):
        lev.step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        lev.step()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    e0.record()
    for _ in range(steps):
        hydro.fill_ghosts_level(tiling, lev.pa)
    e1.record()
    torch.cuda.synchronize()
    ms_fill = e0.elapsed_time(e1) / steps
    err = int(lev.err.item())
    del lev
    tiling.close()
    torch.cuda.empty_cache()
    ghosts = sum((b["n"][0] + 2 * b["ng"]) * (b["n"][1] + 2 * b["ng"]) * (b["n"][2] + 2 * b["ng"])
                 - b["n"][0] * b["n"][1] * b["n"][2] for b in boxes)
    # the same tiled level with shock flattening (Colella-Woodward) on
    prm_f = dict(prm, flatten=1)
    tiling = hydro.Tiling(boxes, lo, til["dom"], til["bc_lo"], til["bc_hi"])
    lev = hydro.Level(states, boxes, prm_f, shared_dt=True, tiling=tiling)
    for _ in range(warmup):
        lev.step()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        lev.step()
    e1.record()
    torch.cuda.synchronize()
    ms_flat = e0.elapsed_time(e1) / steps
    timer = hydro.StageTimer()
    for _ in range(steps):
        with timer:
            lev.step()
    flat_stage = {k: v / max(timer.calls, 1) for k, v in timer.total_ms.items()}
    err |= int(lev.err.item())
    del lev
    tiling.close()
    torch.cuda.empty_cache()
    U, box, _ = inputs.sedov(n)
    ms1, _, _, err1 = time_box(hydro, torch, U, box, prm, steps, warmup)
    cells = n ** 3
    return {"workload": "sedov%d: point blast (rho 1, p 1e-5, E 1 in r < 2 dx), unit cube, "
                        "outflow, gamma 1.4, CFL 0.5, as %d boxes of %d^3 tiling the domain"
                        % (n, len(boxes), bs),
            "cells": cells, "boxes": len(boxes), "steps": steps,
            "tiled_cu_per_s": cells / (ms * 1e-3), "tiled_ms_per_step": ms,
            "level_fill_ms": ms_fill,
            "level_fill_GB_per_s": 80.0 * ghosts / (ms_fill * 1e-3) / 1e9,
            "level_fill_bytes": 80 * ghosts,
            "tiled_flattened_cu_per_s": cells / (ms_flat * 1e-3),
            "tiled_flattened_ms_per_step": ms_flat,
            "tiled_flattened_stage_ms": flat_stage,
            "one_box_cu_per_s": cells / (ms1 / steps * 1e-3), "one_box_ms_per_step": ms1 / steps,
            "err_bits": err | err1,
            "paper_context": "Castro Sedov: 130 zones/us per Summit node (6 V100) at 256^3 "
                             "cells per node in 64^3 boxes; about 25 zones/us per V100 under "
                             "optimal conditions (other hardware, precision not stated)"}


def time_serving(torch, inputs, nreq, warm, nstates, seed=3):
    """Continuous-batching server: saturated capacity (all requests at t=0),
    the same with one request at a time, then a Poisson stream at 80% load of
    `warm` warm-up requests followed by `nreq` measured ones.  Every request
    arrives with its initial state (the client's payload): `nstates` distinct
    runs of the serving stream (family, side and seed), built and pinned in
    host memory before the timed runs, which the stream's requests cycle
    through, each with its own arrival time and step count.  The server's
    work starts at admission, with the upload of that state."""
    from paper_2007_05218_amd.serve import GpuExecutor, Server
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor
    base = inputs.request_stream(nstates, rate=1.0, seed=seed + 7)
    with ThreadPoolExecutor(8) as pool:
        built = list(pool.map(inputs.request_state, base))
    payloads = [(torch.from_numpy(U).pin_memory(), box, prm) for U, box, prm in built]
    del built

    def attach(specs):
        for i, s in enumerate(specs):
            k = i % nstates
            s.update(n=base[k]["n"], family=base[k]["family"], seed=base[k]["seed"],
                     state=payloads[k])
        return specs

    cap = {}
    for name, slots in (("batched", 64), ("one_at_a_time", 1)):
        probe = attach(inputs.request_stream(24, rate=0.0, seed=seed + 100))
        srv = Server(GpuExecutor(max_active=64), budget_bytes=200e9, max_active=slots)
        srv.run(probe)
        cap[name] = srv.metrics()["cu_per_s"]
        srv.ex.close()
    sample = attach(inputs.request_stream(20000, rate=1.0, seed=seed + 1))
    ework = float(np.mean([r["n"] ** 3 * r["steps"] for r in sample]))
    lam = 0.8 * cap["batched"] / ework
    specs = attach(inputs.request_stream(nreq + warm, rate=lam, seed=seed))
    ex = GpuExecutor(max_active=64)
    srv = Server(ex, budget_bytes=200e9, max_active=64)
    t0 = time.perf_counter()
    # (a ROCTx range around the measured loop, for API traces of it)
    torch.cuda.nvtx.range_push("serve loop")
    srv.run(specs)
    torch.cuda.nvtx.range_pop()
    wall = time.perf_counter() - t0
    ex.close()
    m = srv.metrics(skip=warm)
    m.update({"workload": "serve: Poisson arrivals at 80%% of saturated capacity, cubic n "
                          "log-uniform in [32,192], steps uniform in [10,200], families "
                          "sod/kh/smooth, 200 GB HBM budget, seed %d; %d warm-up + %d "
                          "measured requests cycling through %d distinct initial states"
                          % (seed, warm, nreq, nstates),
              "rate_per_s": lam, "mean_work_cu": ework, "warmup_requests": warm,
              "loop_wall_s": wall,
              "capacity_batched_cu_per_s": cap["batched"],
              "capacity_one_at_a_time_cu_per_s": cap["one_at_a_time"]})
    return m


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(inputs, U, box, prm, seconds):
    """The oracle on z-slabs of the workload's first step until ~`seconds`
    of host time have been spent, on all the threads OpenMP gives it; then on
    one thread the Sod 32^3 tube for 20 steps and one step of the
    Kelvin-Helmholtz box at 64^3."""
    from oracle import build, oracle as orc
    build.build(force=False)
    ob, op = orc.box_from(box), orc.params_from(prm)
    U = U.copy()
    orc.fill_ghosts(U, ob)
    dt = orc.estimate_dt(U, ob, op)
    ops = {k: orc.opcount_cell(U, ob, op, dt, N=16, stage=v) for k, v in KERNEL_STAGES.items()}
    ops["step"] = orc.opcount_cell(U, ob, op, dt, N=16)
    n = box["n"]
    Unew = U.copy()
    slab = 4
    cells = 0
    threads = orc.num_threads()
    t0 = time.perf_counter()
    z = 0
    while time.perf_counter() - t0 < seconds and z < n[2]:
        hi = min(n[2], z + slab)
        orc.advance_region(U, Unew, ob, op, dt, (0, 0, z), (n[0], n[1], hi))
        cells += n[0] * n[1] * (hi - z)
        z = hi
    el = time.perf_counter() - t0
    del Unew
    one = {}
    orc.set_num_threads(1)
    try:
        for name, (Ui, bi, pi), steps in (("sod32_20_steps", inputs.sod(32), 20),
                                          ("kh64_1_step", inputs.kh(64, seed=1), 1)):
            obi, opi = orc.box_from(bi), orc.params_from(pi)
            t1 = time.perf_counter()
            orc.run(Ui, obi, opi, steps)
            one[name + "_cu_per_s"] = bi["n"][0] * bi["n"][1] * bi["n"][2] * steps / (
                time.perf_counter() - t1)
    finally:
        orc.set_num_threads(threads)
    return ({"value": cells / el, "unit": "cell-updates/s", "cores": threads,
             "kind": "oracle",
             "sample": "first step of the %dx%dx%d workload on %d z-slabs of %d cells "
                       "(%d cell-updates, %.1f s)" % (n[0], n[1], n[2], z // slab, slab,
                                                      cells, el),
             "cpu_model": cpu_model(), "one_thread": one}, ops)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    from paper_2007_05218_amd import hydro, inputs
    hydro.lib()
    work = [w.strip() for w in args.workloads.split(",") if w.strip()]
    rank = int(os.environ.get("RANK", "0"))

    # the practical HBM roof: a plain elementwise kernel over 2 GiB (2 GiB
    # read and 2 GiB written per launch), timed with events
    a = torch.empty(2 ** 28, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    torch.neg(a, out=b)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 1 if "copy" in work else 10  # one launch only under the counters
    e0.record()
    for _ in range(reps):
        torch.neg(a, out=b)
    e1.record()
    torch.cuda.synchronize()
    copy_gbps = 2 * a.numel() * 8 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    # and the practical write roof: a fill of the same 2 GiB (write only; the
    # trace kernel's traffic is four fifths writes)
    e0.record()
    for _ in range(reps):
        b.fill_(2.0)
    e1.record()
    torch.cuda.synchronize()
    write_gbps = a.numel() * 8 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    log("copy: 2 GiB read + 2 GiB written per launch, %.0f GB/s; fill of 2 GiB, %.0f GB/s"
        % (copy_gbps, write_gbps))
    log("building RT 512^3 input")
    U, box, prm = inputs.rt(512, seed=4)
    ncell = box["n"][0] * box["n"][1] * box["n"][2]
    log("timing RT 512^3: %d warmup + %d steps" % (args.warmup, args.steps))
    ms, wall, timer, err = time_box(hydro, torch, U, box, prm, args.steps, args.warmup)
    value = ncell * args.steps / (ms * 1e-3)
    log("RT512: %.3f ms/step, %.3e cu/s, err=%d" % (ms / args.steps, value, err))
    stage_ms = {k: v / max(timer.calls, 1) for k, v in timer.total_ms.items()}
    log("stage ms/step:", json.dumps({k: round(v, 3) for k, v in stage_ms.items()}))

    cpu = None
    ops = None
    if rank == 0 and not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        cpu, ops = cpu_baseline(inputs, U, box, prm, args.cpu_seconds)
        log("cpu baseline:", json.dumps(cpu), "ops/cell-update:", json.dumps(ops))
    def flops(o):
        return o["add"] + o["mul"] + o["div"] + o["sqrt"]

    # dominant kernel group and its roofline: algorithmic FP64 operations of
    # the oracle stages it computes, per cell-update, x cells / its device time
    adv = {k: v for k, v in stage_ms.items() if k in KERNEL_STAGES}
    dom = max(adv, key=adv.get)
    roof = None
    if ops:
        step_s = ms / args.steps * 1e-3

        def valu_entry(k, kms):
            # executed instructions from the committed counters: the FP64
            # flops the hardware ran per second against the 78.6 T peak, and
            # the lane-instruction issue rate against the chip's
            ex = executed_valu(k, ncell)
            if not ex:
                return None
            return dict(ex, **{
                "executed_fp64_TFLOPs": ex["executed_fp64_flops_per_cu"] * ncell / (kms * 1e-3) / 1e12,
                "executed_fp64_frac": ex["executed_fp64_flops_per_cu"] * ncell / (kms * 1e-3)
                / PEAK_FP64,
                "valu_issue_frac": ex["valu_instr_per_cu"] * ncell / (kms * 1e-3) / LANE_ISSUE_PER_S})

        def kernel_entry(k):
            kms = stage_ms[k]
            ach = flops(ops[k]) * ncell / (kms * 1e-3)
            traffic = measured_traffic(k)
            alg = ALG_BYTES[k] * ncell / (kms * 1e-3)
            return ach, traffic, {
                "ms": kms, "achieved_TFLOPs": ach / 1e12, "frac": ach / PEAK_FP64,
                "frac_of_issue_peak_no_fma": ach / PEAK_FP64_NOFMA,
                "flops_per_cell_update": flops(ops[k]),
                "algorithmic_bytes_per_cell_update": ALG_BYTES[k],
                "algorithmic_GBps": alg / 1e9, "algorithmic_frac_of_8TBps": alg / HBM_PEAK,
                "counter_bytes_per_launch": traffic,
                "counter_GBps": traffic / (kms * 1e-3) / 1e9 if traffic else None,
                "counter_frac_of_8TBps": traffic / (kms * 1e-3) / HBM_PEAK if traffic else None,
                "counter_valu": valu_entry(k, kms)}

        ach, traffic, dom_entry = kernel_entry(dom)
        roof = {"bound": "alu", "achieved": ach / 1e12, "peak": PEAK_FP64 / 1e12,
                "unit": "TFLOP/s", "frac": ach / PEAK_FP64, "traffic": traffic,
                "kernel": KERNEL_SYMBOL[dom], "kernel_ms": stage_ms[dom],
                "flops_per_cell_update": flops(ops[dom]),
                "issue_peak_no_fma_TFLOPs": PEAK_FP64_NOFMA / 1e12,
                "frac_of_issue_peak_no_fma": ach / PEAK_FP64_NOFMA,
                "kernels": {KERNEL_SYMBOL[k]: (dom_entry if k == dom else kernel_entry(k)[2])
                            for k in adv},
                "practical_hbm_copy_GBps": copy_gbps,
                "practical_hbm_write_GBps": write_gbps,
                "step": {"flops_per_cell_update": flops(ops["step"]),
                         "achieved_TFLOPs": flops(ops["step"]) * ncell / step_s / 1e12,
                         "frac": flops(ops["step"]) * ncell / step_s / PEAK_FP64,
                         "frac_of_issue_peak_no_fma":
                             flops(ops["step"]) * ncell / step_s / PEAK_FP64_NOFMA,
                         "algorithmic_GBps_80B_per_cu": 80.0 * value / 1e9,
                         "hbm_frac_80B_per_cu": 80.0 * value / HBM_PEAK}}
        # the step against its VALU roof: the FP64 VALU instructions the
        # advance kernels issue per cell-update (counters), at one lane-
        # instruction per lane and clock, bounds cell-updates/s
        exs = [executed_valu(k, ncell) for k in adv]
        if all(exs):
            fp64_i = sum(e["fp64_valu_instr_per_cu"] for e in exs)
            all_i = sum(e["valu_instr_per_cu"] for e in exs)
            roof["step"].update({
                "fp64_valu_instr_per_cu": fp64_i, "valu_instr_per_cu": all_i,
                "fp64_valu_roof_cu_per_s": LANE_ISSUE_PER_S / fp64_i,
                "frac_of_fp64_valu_roof": value / (LANE_ISSUE_PER_S / fp64_i),
                "valu_roof_cu_per_s": LANE_ISSUE_PER_S / all_i,
                "frac_of_valu_roof": value / (LANE_ISSUE_PER_S / all_i)})

    also = {}
    if "kh256" in work:
        U2, box2, prm2 = inputs.kh(256, seed=1)
        n2 = 256 ** 3
        log("timing KH 256^3")
        ms2, _, t2, e2 = time_box(hydro, torch, U2, box2, prm2, args.steps, args.warmup)
        also["kh256"] = {"cu_per_s": n2 * args.steps / (ms2 * 1e-3),
                         "ms_per_step": ms2 / args.steps, "err": e2}
        del U2
    if "species" in work:
        log("timing KH 256^3 with 2 passively advected species")
        also["kh256_species2"] = time_species(hydro, torch, inputs, args.steps, args.warmup)
        log("species:", json.dumps(also["kh256_species2"]))
    if "sedov" in work:
        log("timing the Sedov blast, 256^3 as 64 boxes of 64^3 and as one box")
        also["sedov256"] = time_sedov(hydro, torch, inputs, args.steps, args.warmup)
        log("sedov:", json.dumps(also["sedov256"]))
    if "level" in work:
        log("timing the 512-box level, batched vs per-box")
        also["level512"] = time_level(hydro, torch, inputs, args.level_steps, 1)
    if "serve" in work:
        log("serving %d + %d requests" % (args.serve_warmup, args.serve_requests))
        also["serve"] = time_serving(torch, inputs, args.serve_requests, args.serve_warmup,
                                     args.serve_states)
        log("serve:", json.dumps(also["serve"]))

    out = {"metric": "FP64 hydro cell-updates/s (whole step: ghost fill + CFL dt + CTU-PPM-HLLC advance)",
           "value": value, "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms / args.steps, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "rt512: Rayleigh-Taylor 512^3 box, FP64 SoA, 4 ghosts, "
                                  "gamma 1.4, g=-0.1 z, CFL 0.5, seed 4",
                      "cells": ncell, "parallelism": "single GPU"},
           "stage_ms_per_step": stage_ms, "err_bits": err,
           "roofline": roof, "cpu_baseline": cpu, "also": also}
    if rank == 0:
        print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
