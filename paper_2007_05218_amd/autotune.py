"""Tile-shape autotuner for batched levels of boxes.

The two fused kernels of the step (the trace kernel and the flux kernel)
each process a box in tiles of columns marching over z-segments of tzs
planes, tile width tbx in {8, 16, 18, 32}: the trace kernel tbx x 256/tbx
columns, the flux kernel rows of tbx lanes, 64/tbx whole rows per
wavefront.  Width 18 leaves threads idle, but a flux-kernel row of 18 lanes
computes 16 columns, so it covers a box 16 cells wide with one tile row and
one 32 cells wide with two, where rows of 16 lanes (14 columns each) need
two and three.
The best tile depends on the box shape: narrow boxes waste halo columns in
wide tiles, short boxes want short z-segments to expose enough blocks, tall
ones long segments to amortise the two warm-up planes.  The paper finds the
same trade-off at the level of AMReX box sizes and tunes it empirically
(Sec. IV-A, the best/worst box-width sweep); here it is tuned per box-shape
class on the GPU, by timing a batched step of boxes of that class with each
candidate tile (the library's stage events give each kernel's own time, so
the two kernels are tuned independently in the same runs), and the winners
are written as the JSON table that hydro_plan_create accepts.  Results never
depend on the tile (every cell's arithmetic is the same), only the speed
does.
"""
import json

from . import hydro, inputs

TBX = (8, 16, 18, 32)
TZS = (8, 16, 32, 64, 128)
STAGES = ("trace", "flux_update")


def shape_key(n):
    return "%dx%dx%d" % tuple(n)


def table_json(table):
    """JSON text of a {shape: (tbx, tzs) or (tbx1, tzs1, tbx2, tzs2)} table in
    the plan's format."""
    return json.dumps({k: [int(x) for x in v] for k, v in sorted(table.items())})


def candidates(n):
    """Table entries to time for shape n: (tbx, tzs), for both kernels."""
    zs = sorted({z for z in TZS if z < n[2]} | {n[2]})
    return [(b, z) for b in TBX for z in zs]


def _kernel_tile(entry, kernel):
    """The (tbx, tzs) a table entry gives one kernel (0: trace, 1: flux), or
    BUILTIN."""
    if len(entry) == 2:
        return tuple(entry)
    return tuple(entry[2 * kernel:2 * kernel + 2])


BUILTIN = (0, 0)  # table entry keeping a kernel's built-in tile
MARGIN = 0.03     # a tuned tile must beat the built-in one by this fraction


def _time_class(n, tiles, prm, nboxes, reps, torch):
    """{tile: (trace-kernel ms, flux-kernel ms)} for a batch of boxes of shape
    n; the tile BUILTIN times the library's built-in choice."""
    # a few distinct synthetic states, repeated to fill the batch
    distinct = [inputs.smooth(n, seed=1000 + i, dx=(1.0 / 64,) * 3)[:2]
                for i in range(min(nboxes, 8))]
    states = [distinct[i % len(distinct)][0] for i in range(nboxes)]
    boxes = [distinct[i % len(distinct)][1] for i in range(nboxes)]
    out = {}
    for tb in tiles:
        lev = hydro.Level(states, boxes, prm, shared_dt=True,
                          autotune_json=None if tb == BUILTIN else table_json({shape_key(n): tb}))
        lev.step()  # warm-up (and first touch of the workspace)
        torch.cuda.synchronize()
        timer = hydro.StageTimer()
        for _ in range(reps):
            with timer:
                lev.step()
        out[tb] = tuple(timer.total_ms[s] / reps for s in STAGES)
        del lev
    return out


def _pick(t, kernel):
    """The fastest tile for one kernel (0: trace, 1: flux), kept only if it
    beats the built-in choice by MARGIN (timing noise must not replace a good
    built-in tile with an equal one).  Entries that leave this kernel at its
    built-in tile do not compete for it."""
    own = [k for k in t if k == BUILTIN or _kernel_tile(k, kernel) != BUILTIN]
    best = min(own, key=lambda k: t[k][kernel])
    if best != BUILTIN and t[best][kernel] < (1.0 - MARGIN) * t[BUILTIN][kernel]:
        return _kernel_tile(best, kernel), t[best][kernel]
    return BUILTIN, t[BUILTIN][kernel]


def tune(boxes, prm=None, max_boxes_per_class=4096, min_cells_per_class=2 ** 23, reps=3,
         log=None):
    """Tune every box shape of ``boxes``.  Each class is timed on a batch of
    synthetic boxes of that shape (enough boxes to keep the GPU saturated, as
    a level's launch does: at least ``min_cells_per_class`` cells, at most
    ``max_boxes_per_class`` boxes) with the built-in tiles and every candidate; the
    trace and flux kernels each get their fastest tile when it beats the
    built-in one by MARGIN.  Returns ({shape: (tbx1, tzs1, tbx2, tzs2)} for
    the shapes where a kernel changed (0, 0 = built-in), timings)."""
    import torch
    prm = prm or inputs.params_desc()
    shapes = sorted({tuple(b["n"]) for b in boxes})
    table, timings = {}, {}
    for n in shapes:
        cells = n[0] * n[1] * n[2]
        nb = max(1, min(max_boxes_per_class, -(-min_cells_per_class // cells)))
        t = _time_class(n, [BUILTIN] + candidates(n), prm, nb, reps, torch)
        (b1, ms1), (b2, ms2) = _pick(t, 0), _pick(t, 1)
        if (b1, b2) != (BUILTIN, BUILTIN):
            table[shape_key(n)] = (b1[0], b1[1], b2[0], b2[1])
        timings[shape_key(n)] = {",".join("%d" % x for x in k): v for k, v in t.items()}
        if log:
            log("tiles %s: trace %s (%.3f ms, built-in %.3f), flux %s (%.3f ms, built-in %.3f), "
                "%d boxes" % (shape_key(n), b1, ms1, t[BUILTIN][0], b2, ms2,
                              t[BUILTIN][1], nb))
    return table, timings


def validate(states, boxes, prm, table, steps=4, rounds=3):
    """Time the whole level with the built-in tiles and with ``table``
    (alternating, ``rounds`` times ``steps`` steps each) and keep the table
    only if the level is faster with it: per-class timings need not add up
    to the level's (its classes share the GPU in one launch).  Returns
    (table or {}, ms per step built-in, ms per step with the table)."""
    import torch
    if not table:
        return {}, None, None
    levels = [hydro.Level(states, boxes, prm, shared_dt=True),
              hydro.Level(states, boxes, prm, shared_dt=True, autotune_json=table_json(table))]
    best = [float("inf"), float("inf")]
    for lev in levels:
        lev.step()
    for _ in range(rounds):
        for i, lev in enumerate(levels):
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            lev.run(steps)
            e1.record()
            torch.cuda.synchronize()
            best[i] = min(best[i], e0.elapsed_time(e1) / steps)
    del levels
    torch.cuda.empty_cache()
    return (table if best[1] < best[0] else {}), best[0], best[1]
