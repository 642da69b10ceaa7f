"""The C ABI library: it loads, exports every entry point include/hydro.h
declares, and validates arguments synchronously (no GPU needed; no call
here launches a kernel)."""
import ctypes as C
import os
import re

import pytest

from paper_2007_05218_amd import hydro, inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "hydro.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b([A-Za-z_][A-Za-z0-9_]*)\s*\(", src)
    skip = {"defined", "sizeof"}
    return sorted({n for n in names if n not in skip and not n.isupper()})


def test_library_exports_every_declared_symbol():
    L = hydro.lib()
    decl = _declared()
    assert set(decl) == set(hydro.EXPORTS), decl
    for name in decl:
        assert hasattr(L, name), name


def test_struct_layouts():
    assert C.sizeof(hydro.HydroBox) == 64
    assert C.sizeof(hydro.HydroParams) == 48
    assert hydro.HydroParams.flatten.offset == 40
    assert hydro.HydroBox.dx.offset == 16
    assert hydro.HydroBox.bc_lo.offset == 40


def test_state_and_workspace_sizes():
    U, box, prm = inputs.sod(32)
    assert hydro.state_elems(box) == U.size == 5 * 40 ** 3
    ws = hydro.workspace_bytes(box)
    # the traced face states (3 directions x 2 faces x 5 components) of the
    # traced region, one cell beyond the 32^3 valid cells
    assert ws >= 30 * 34 ** 3 * 8 and ws % 256 == 0
    boxes = [inputs.box_desc((16, 32, 64)), inputs.box_desc((64, 16, 16))]
    assert hydro.workspace_bytes(boxes) == sum(hydro.workspace_bytes(b) for b in boxes)


@pytest.mark.parametrize("bad", [
    dict(n=(0, 8, 8)), dict(ng=2), dict(ng=9), dict(dx=(0.0, 1.0, 1.0)),
    dict(n=(3, 8, 8), bc_lo=(0, 0, 0), bc_hi=(0, 0, 0)),  # periodic axis shorter than ng
    dict(bc_lo=(0, 1, 1), bc_hi=(1, 1, 1)),               # unpaired periodic
    dict(bc_lo=(5, 1, 1), bc_hi=(5, 1, 1)),
    dict(n=(6000, 12000, 1)),  # a component beyond 32-bit byte offsets
    dict(n=(3000, 3000, 1)),   # a workspace plane beyond 32-bit byte offsets
])
def test_invalid_boxes_rejected(bad):
    d = inputs.box_desc((8, 8, 8), bc_lo=(1, 1, 1))
    d.update(bad)
    assert hydro.state_elems(d) == 0
    assert hydro.workspace_bytes(d) == 0
    L = hydro.lib()
    b = hydro.make_box(d)
    p = hydro.make_params(inputs.params_desc())
    fake = C.c_void_p(256)
    assert L.estimate_dt(fake, C.byref(b), C.byref(p), fake, None) == hydro.HYDRO_EINVAL
    assert L.hydro_fill_ghosts(fake, C.byref(b), None) == hydro.HYDRO_EINVAL
    assert L.advance_box(fake, C.c_void_p(1 << 40), C.byref(b), C.byref(p), fake, None, fake,
                         1 << 40, fake, None) == hydro.HYDRO_EINVAL
    arr = (hydro.HydroBox * 1)(b)
    h = C.c_void_p()
    assert L.hydro_plan_create(arr, 1, None, C.byref(h)) == hydro.HYDRO_EINVAL


@pytest.mark.parametrize("bad", [dict(gamma=1.0), dict(cfl=0.0), dict(cfl=1.5),
                                 dict(gamma=float("nan")), dict(flatten=2), dict(flatten=-1)])
def test_invalid_params_rejected(bad):
    d = inputs.box_desc((8, 8, 8), bc_lo=(1, 1, 1))
    p = inputs.params_desc()
    p.update(bad)
    L = hydro.lib()
    fake = C.c_void_p(256)
    assert L.estimate_dt(fake, C.byref(hydro.make_box(d)), C.byref(hydro.make_params(p)),
                         fake, None) == hydro.HYDRO_EINVAL


def test_null_and_overlap_rejected():
    d = inputs.box_desc((8, 8, 8), bc_lo=(1, 1, 1))
    L = hydro.lib()
    b = hydro.make_box(d)
    p = hydro.make_params(inputs.params_desc())
    a = C.c_void_p(1 << 30)
    ws = C.c_void_p(1 << 34)
    nbytes = hydro.workspace_bytes(d)
    # U_new overlapping U
    assert L.advance_box(a, C.c_void_p((1 << 30) + 8), C.byref(b), C.byref(p), a, None, ws,
                         nbytes, a, None) == hydro.HYDRO_EINVAL
    # workspace misaligned
    assert L.advance_box(a, C.c_void_p(1 << 32), C.byref(b), C.byref(p), a, None,
                         C.c_void_p((1 << 34) + 8), nbytes, a, None) == hydro.HYDRO_EINVAL
    # workspace too small
    assert L.advance_box(a, C.c_void_p(1 << 32), C.byref(b), C.byref(p), a, None, ws,
                         nbytes - 256, a, None) == hydro.HYDRO_ENOWS
    # next-step timestep overlapping the one in use
    assert L.advance_box(a, C.c_void_p(1 << 32), C.byref(b), C.byref(p), C.c_void_p(1 << 36),
                         C.c_void_p((1 << 36) + 4), ws, nbytes, a, None) == hydro.HYDRO_EINVAL
    assert L.estimate_dt(None, C.byref(b), C.byref(p), a, None) == hydro.HYDRO_EINVAL
    assert L.advance_boxes(1, a, a, None, C.byref(p), a, 1, None, None, ws, nbytes, a,
                           None) == hydro.HYDRO_EINVAL
    assert L.hydro_fill_ghosts_boxes(1, a, None, None) == hydro.HYDRO_EINVAL
    # workspace overlapping the old or the new state
    ub = 5 * 16 ** 3 * 8
    assert L.advance_box(a, C.c_void_p(1 << 32), C.byref(b), C.byref(p), C.c_void_p(1 << 36),
                         None, C.c_void_p((1 << 30) + ub - 256), nbytes, a,
                         None) == hydro.HYDRO_EINVAL
    assert L.advance_box(a, C.c_void_p(1 << 32), C.byref(b), C.byref(p), C.c_void_p(1 << 36),
                         None, C.c_void_p((1 << 32) - 256), nbytes, a,
                         None) == hydro.HYDRO_EINVAL
    # flattening reads the fourth ghost layer: a box with three is refused
    d3 = inputs.box_desc((8, 8, 8), ng=3, bc_lo=(1, 1, 1))
    b3 = hydro.make_box(d3)
    pf = hydro.make_params(inputs.params_desc(flatten=1))
    n3 = hydro.workspace_bytes(d3)
    assert L.advance_box(a, C.c_void_p(1 << 32), C.byref(b3), C.byref(pf), a, None, ws,
                         n3, a, None) == hydro.HYDRO_EINVAL


def test_status_strings():
    L = hydro.lib()
    for s in range(4):
        assert L.hydro_status_string(s).startswith(b"HYDRO_")


@pytest.mark.parametrize("js", ['{"16x16x16": [12, 8]}', '{"16x16x16": [16, 0]}', '{16x16x16: [16, 8]}',
                                '{"16x16": [16, 8]}', '["16x16x16"]', '{"16x16x16": [16, 8]} x',
                                '{"16x16x16": [16, 8, 32]}', '{"16x16x16": [16, 8, 32, 8, 8]}',
                                '{"16x16x16": [16, 8, 24, 8]}', '{"16x16x16": [16, 8, 0, 8]}',
                                '{"16x16x16": [0, 4, 16, 8]}', '{"16x16x16": [20, 8]}',
                                '{"16x16x16": [18, 0, 16, 8]}', '{"16x16x16": [16, 8, 20, 8]}'])
def test_plan_rejects_bad_tile_tables(js):
    # the table is parsed before any device allocation, so this needs no GPU
    L = hydro.lib()
    arr = (hydro.HydroBox * 1)(hydro.make_box(inputs.box_desc((16, 16, 16))))
    h = C.c_void_p()
    assert L.hydro_plan_create(arr, 1, js.encode(), C.byref(h)) == hydro.HYDRO_EINVAL


def test_autotune_table_format():
    from paper_2007_05218_amd import autotune
    js = autotune.table_json({"16x32x64": (16, 32), "64x64x64": (32, 64, 16, 32)})
    assert js == '{"16x32x64": [16, 32], "64x64x64": [32, 64, 16, 32]}'
    c = autotune.candidates((16, 32, 64))
    assert (8, 64) in c and (32, 8) in c and (18, 64) in c
    assert all(t[0] in (8, 16, 18, 32) for t in c)
    # a four-entry tile gives each kernel its own pair
    assert autotune._kernel_tile((0, 0, 18, 8), 0) == autotune.BUILTIN
    assert autotune._kernel_tile((0, 0, 18, 8), 1) == (18, 8)
    assert autotune._kernel_tile((16, 8), 1) == (16, 8)


def test_autotune_pick_keeps_builtin_unless_clearly_faster():
    # timings {entry: (trace ms, flux ms)}: each kernel takes its fastest
    # entry only when it beats the built-in tile by the margin, and an entry
    # that leaves a kernel at its built-in tile does not compete for it
    from paper_2007_05218_amd import autotune
    B = autotune.BUILTIN
    t = {B: (1.00, 2.00), (16, 8): (0.99, 1.50), (32, 8): (0.80, 2.10),
         (0, 0, 18, 16): (0.50, 1.40)}
    assert autotune._pick(t, 0) == ((32, 8), 0.80)   # 20 % faster trace
    assert autotune._pick(t, 1) == ((18, 16), 1.40)  # flux-only entry wins the flux
    t = {B: (1.00, 2.00), (16, 8): (0.98, 1.99)}     # within the margin
    assert autotune._pick(t, 0) == (B, 1.00)
    assert autotune._pick(t, 1) == (B, 2.00)


def _level_args(layout):
    """(boxes, lo, dom, bc_lo, bc_hi) of a tiling, possibly broken."""
    boxes = [inputs.box_desc(n) for n in layout["n"]]
    return boxes, layout["lo"], layout["dom"], layout.get("bc_lo", (0, 0, 0)), \
        layout.get("bc_hi", layout.get("bc_lo", (0, 0, 0)))


GOOD = {"n": [(8, 16, 16), (8, 16, 16)], "lo": [(0, 0, 0), (8, 0, 0)], "dom": (16, 16, 16)}


@pytest.mark.parametrize("bad", [
    dict(lo=[(0, 0, 0), (4, 0, 0)]),                      # overlap (and a gap)
    dict(n=[(8, 16, 16), (4, 16, 16)], lo=[(0, 0, 0), (8, 0, 0)]),  # gap
    dict(lo=[(0, 0, 0), (9, 0, 0)]),                      # box beyond the domain
    dict(lo=[(0, 0, 0), (-8, 0, 0)]),                     # negative corner
    dict(dom=(16, 16, 0)),
    dict(bc_lo=(0, 1, 1), bc_hi=(1, 1, 1)),               # unpaired periodic
    dict(bc_lo=(0, 4, 0), bc_hi=(0, 4, 0)),               # unknown boundary kind
    dict(n=[(1, 16, 16), (2, 16, 16)], lo=[(0, 0, 0), (1, 0, 0)], dom=(3, 16, 16)),  # ng > dom
    # owner map beyond 2^24 cells (no common divisor > 1)
    dict(n=[(257, 256, 256)], lo=[(0, 0, 0)], dom=(257, 256, 256)),
])
def test_level_rejects_bad_tilings(bad):
    # validated before any device allocation, so no GPU is needed
    lay = dict(GOOD)
    lay.update(bad)
    boxes, lo, dom, bl, bh = _level_args(lay)
    if bad.get("dom") == (3, 16, 16):
        boxes = [inputs.box_desc(n, bc_lo=(1, 1, 1)) for n in lay["n"]]
    L = hydro.lib()
    arr = (hydro.HydroBox * len(boxes))(*[hydro.make_box(b) for b in boxes])
    flat = (C.c_int32 * (3 * len(boxes)))(*[v for l in lo for v in l])
    i3 = C.c_int32 * 3
    h = C.c_void_p(123)
    assert L.hydro_level_create(arr, flat, len(boxes), i3(*dom), i3(*bl), i3(*bh),
                                C.byref(h)) == hydro.HYDRO_EINVAL
    assert h.value is None
    # a null handle and a mismatched box count are refused by the fill
    assert L.hydro_fill_ghosts_level(1, C.c_void_p(8), None, None) == hydro.HYDRO_EINVAL


def test_species_sizes_and_rejections():
    d = inputs.box_desc((8, 8, 8), bc_lo=(1, 1, 1))
    assert hydro.species_workspace_bytes(d, 0) == 0
    assert hydro.species_workspace_bytes(d, 9) == 0
    # the twelve mass-flux fields of the gas step over the 10^3 index box,
    # each padded to 256 B, whatever the species count
    field = -(-10 ** 3 // 32) * 32 * 8
    assert hydro.species_workspace_bytes(d, 1) == 12 * field
    assert hydro.species_workspace_bytes(d, 3) == 12 * field
    L = hydro.lib()
    b = hydro.make_box(d)
    p = hydro.make_params(inputs.params_desc())
    a = C.c_void_p(1 << 30)
    ws = C.c_void_p(1 << 34)
    nws = hydro.workspace_bytes(d)
    S, Sn, sws = C.c_void_p(1 << 38), C.c_void_p(1 << 39), C.c_void_p(1 << 40)
    nsws = hydro.species_workspace_bytes(d, 2)

    def call(S_, Sn_, ns, sws_, nb, U=a, Un=C.c_void_p(1 << 32)):
        return L.advance_box_species(U, Un, S_, Sn_, ns, C.byref(b), C.byref(p), a, None, ws, nws,
                                     sws_, nb, a, None)
    assert call(None, Sn, 2, sws, nsws) == hydro.HYDRO_EINVAL
    assert call(S, Sn, 0, sws, nsws) == hydro.HYDRO_EINVAL
    assert call(S, Sn, 9, sws, nsws) == hydro.HYDRO_EINVAL
    assert call(S, C.c_void_p((1 << 38) + 8), 2, sws, nsws) == hydro.HYDRO_EINVAL   # S overlap
    assert call(S, Sn, 2, C.c_void_p((1 << 40) + 8), nsws) == hydro.HYDRO_EINVAL    # misaligned
    assert call(S, Sn, 2, C.c_void_p(1 << 38), nsws) == hydro.HYDRO_EINVAL          # sws over S
    assert call(S, Sn, 2, sws, nsws - 256) == hydro.HYDRO_ENOWS
    assert call(S, Sn, 2, sws, nsws, Un=C.c_void_p((1 << 30) + 8)) == hydro.HYDRO_EINVAL
    assert call(S, ws, 2, sws, nsws) == hydro.HYDRO_EINVAL                      # S_new over ws
    assert call(C.c_void_p(1 << 32), Sn, 2, sws, nsws) == hydro.HYDRO_EINVAL    # S over U_new
    assert call(ws, Sn, 2, sws, nsws) == hydro.HYDRO_EINVAL                     # S over ws
    assert call(S, Sn, 2, sws, nsws, U=ws) == hydro.HYDRO_EINVAL                # U over ws
    assert call(S, Sn, 2, sws, nsws, Un=ws) == hydro.HYDRO_EINVAL               # U_new over ws
    assert call(S, Sn, 2, sws, nsws, U=None) == hydro.HYDRO_EINVAL              # before sizes
    assert call(S, Sn, 2, sws, 0, U=None) == hydro.HYDRO_EINVAL
    assert L.hydro_fill_ghosts_species(None, 2, C.byref(b), None) == hydro.HYDRO_EINVAL
    assert L.hydro_fill_ghosts_species(S, 9, C.byref(b), None) == hydro.HYDRO_EINVAL


def test_batched_species_sizes_and_rejections():
    boxes = [inputs.box_desc((8, 8, 8), bc_lo=(1, 1, 1)), inputs.box_desc((16, 4, 8), bc_lo=(1, 1, 1))]
    assert hydro.species_workspace_bytes_boxes(boxes, 2) == sum(
        hydro.species_workspace_bytes(b, 2) for b in boxes)
    assert hydro.species_workspace_bytes_boxes(boxes, 0) == 0
    L = hydro.lib()
    p = hydro.make_params(inputs.params_desc())
    a = C.c_void_p(1 << 30)
    # no plan
    assert L.advance_boxes_species(2, a, a, a, a, 2, None, C.byref(p), a, 1, None, None, a,
                                   1 << 20, C.c_void_p(1 << 36), 1 << 20, a,
                                   None) == hydro.HYDRO_EINVAL
    assert L.hydro_fill_ghosts_boxes_species(2, a, 2, None, None) == hydro.HYDRO_EINVAL
    assert L.hydro_fill_ghosts_level_species(2, a, 2, None, None) == hydro.HYDRO_EINVAL


def test_capacity_plan_argument_errors():
    # checked before any device allocation or copy: no GPU needed
    L = hydro.lib()
    h = C.c_void_p(123)
    assert L.hydro_plan_create_capacity(0, None, C.byref(h)) == hydro.HYDRO_EINVAL
    assert L.hydro_plan_create_capacity((1 << 20) + 1, None, C.byref(h)) == hydro.HYDRO_EINVAL
    assert L.hydro_plan_create_capacity(4, b'{"16x16x16": [12, 8]}', C.byref(h)) == \
        hydro.HYDRO_EINVAL
    arr = (hydro.HydroBox * 1)(hydro.make_box(inputs.box_desc((16, 16, 16))))
    assert L.hydro_plan_update(None, arr, 1, None) == hydro.HYDRO_EINVAL
    assert L.hydro_plan_boxes(None) == -1
    assert L.hydro_plan_workspace_bytes(None) == 0
