"""Tile-shape autotuner for batched levels of boxes.

The two fused kernels of the step (the trace kernel and the flux kernel)
each process a box in tiles of 256 columns (tbx x 256/tbx, tbx in
{8, 16, 32}) marching over z-segments of tzs planes.
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

TBX = (8, 16, 32)
TZS = (8, 16, 32, 64, 128)
STAGES = ("trace", "flux_update")


def shape_key(n):
    return "%dx%dx%d" % tuple(n)


def table_json(table):
    """JSON text of a {shape: (tbx, tzs) or (tbx1, tzs1, tbx2, tzs2)} table in
    the plan's format."""
    return json.dumps({k: [int(x) for x in v] for k, v in sorted(table.items())})


def candidates(n):
    zs = sorted({z for z in TZS if z < n[2]} | {n[2]})
    return [(b, z) for b in TBX for z in zs]


def _time_class(n, tiles, prm, nboxes, reps, torch):
    """{tile: (trace-kernel ms, flux-kernel ms)} for a batch of boxes of shape n."""
    states, boxes = [], []
    for i in range(nboxes):
        U, box, _ = inputs.smooth(n, seed=1000 + i, dx=(1.0 / 64,) * 3)
        states.append(U)
        boxes.append(box)
    out = {}
    for tb in tiles:
        lev = hydro.Level(states, boxes, prm, shared_dt=True,
                          autotune_json=table_json({shape_key(n): tb}))
        lev.step()  # warm-up (and first touch of the workspace)
        torch.cuda.synchronize()
        timer = hydro.StageTimer()
        for _ in range(reps):
            with timer:
                lev.step()
        out[tb] = tuple(timer.total_ms[s] / reps for s in STAGES)
        del lev
    return out


def tune(boxes, prm=None, max_boxes_per_class=64, min_cells_per_class=2 ** 21, reps=3,
         log=None):
    """Tune every box shape of ``boxes``.  Each class is timed on a batch of
    synthetic boxes of that shape (enough boxes to fill the GPU, at most
    ``max_boxes_per_class``); the trace and flux kernels each get their
    fastest tile.  Returns ({shape: (tbx1, tzs1, tbx2, tzs2)}, timings)."""
    import torch
    prm = prm or inputs.params_desc()
    shapes = sorted({tuple(b["n"]) for b in boxes})
    table, timings = {}, {}
    for n in shapes:
        cells = n[0] * n[1] * n[2]
        nb = max(1, min(max_boxes_per_class, -(-min_cells_per_class // cells)))
        t = _time_class(n, candidates(n), prm, nb, reps, torch)
        b1 = min(t, key=lambda k: t[k][0])
        b2 = min(t, key=lambda k: t[k][1])
        table[shape_key(n)] = (b1[0], b1[1], b2[0], b2[1])
        timings[shape_key(n)] = {"%d,%d" % k: v for k, v in t.items()}
        if log:
            log("tiles %s: trace %s (%.3f ms), flux %s (%.3f ms), %d boxes"
                % (shape_key(n), b1, t[b1][0], b2, t[b2][1], nb))
    return table, timings
