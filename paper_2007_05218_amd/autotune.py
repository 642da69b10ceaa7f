"""Tile-shape autotuner for batched levels of boxes.

The two fused kernels of the step process a box in tiles of 256 columns
(tbx x 256/tbx, tbx in {8, 16, 32}) marching over z-segments of tzs planes.
The best tile depends on the box shape: narrow boxes waste halo columns in
wide tiles, short boxes want short z-segments to expose enough blocks, tall
ones long segments to amortise the two warm-up planes.  The paper finds the
same trade-off at the level of AMReX box sizes and tunes it empirically
(Sec. IV-A, the best/worst box-width sweep); here it is tuned per box-shape
class on the GPU, by timing a batched step of boxes of that class with each
candidate tile, and the winners are written as the JSON table that
hydro_plan_create accepts.  Results never depend on the tile (every cell's
arithmetic is the same), only the speed does.
"""
import json

from . import hydro, inputs

TBX = (8, 16, 32)
TZS = (8, 16, 32, 64, 128)


def shape_key(n):
    return "%dx%dx%d" % tuple(n)


def table_json(table):
    """JSON text of a {shape: (tbx, tzs)} table in the plan's format."""
    return json.dumps({k: [int(v[0]), int(v[1])] for k, v in sorted(table.items())})


def candidates(n):
    zs = sorted({z for z in TZS if z < n[2]} | {n[2]})
    return [(b, z) for b in TBX for z in zs]


def _time_class(n, tiles, prm, nboxes, reps, torch):
    states, boxes = [], []
    for i in range(nboxes):
        U, box, _ = inputs.smooth(n, seed=1000 + i, dx=(1.0 / 64,) * 3)
        states.append(U)
        boxes.append(box)
    out = {}
    for tb in tiles:
        lev = hydro.Level(states, boxes, prm, shared_dt=True,
                          autotune_json=table_json({shape_key(n): tb}))
        lev.step()  # warm-up (and first-touch of the workspace)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            lev.step()
        e1.record()
        torch.cuda.synchronize()
        out[tb] = e0.elapsed_time(e1) / reps
        del lev
    return out


def tune(boxes, prm=None, max_boxes_per_class=64, min_cells_per_class=2 ** 21, reps=3,
         log=None):
    """Tune every box shape of ``boxes``.  Each class is timed on a batch of
    synthetic boxes of that shape (enough boxes to fill the GPU, at most
    ``max_boxes_per_class``).  Returns ({shape: (tbx, tzs)}, timings)."""
    import torch
    prm = prm or inputs.params_desc()
    shapes = sorted({tuple(b["n"]) for b in boxes})
    table, timings = {}, {}
    for n in shapes:
        cells = n[0] * n[1] * n[2]
        nb = max(1, min(max_boxes_per_class, -(-min_cells_per_class // cells)))
        t = _time_class(n, candidates(n), prm, nb, reps, torch)
        best = min(t, key=t.get)
        table[shape_key(n)] = best
        timings[shape_key(n)] = {"%d,%d" % k: v for k, v in t.items()}
        if log:
            log("tile %s: best %s (%.3f ms for %d boxes)" % (shape_key(n), best, t[best], nb))
    return table, timings
