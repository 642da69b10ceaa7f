"""advance_box_noalloc: the step without a workspace argument, for callers
that cannot allocate (its workspace is the library's static per-GPU array).

Through the C ABI: two calls in a row, the second on a smaller box, each
equal bit for bit to advance_box on the same input (new state, next-step
timestep, error bits); a box whose workspace exceeds the static array is
refused before anything is enqueued."""
import ctypes as C

import numpy as np
import pytest

from paper_2007_05218_amd import hydro, inputs


def test_noalloc_argument_errors_need_no_gpu():
    L = hydro.lib()
    p = hydro.make_params(inputs.params_desc())
    a = C.c_void_p(1 << 30)
    small = hydro.make_box(inputs.box_desc((8, 8, 8), bc_lo=(1, 1, 1)))
    assert L.advance_box_noalloc(None, C.c_void_p(1 << 32), C.byref(small), C.byref(p), a, None,
                                 a, None) == hydro.HYDRO_EINVAL
    assert L.advance_box_noalloc(a, C.c_void_p((1 << 30) + 8), C.byref(small), C.byref(p), a,
                                 None, a, None) == hydro.HYDRO_EINVAL
    # 78^3 fits the static array, 79^3 does not: refused before any HIP call
    assert hydro.workspace_bytes(inputs.box_desc((78,) * 3)) <= hydro.NOALLOC_WS_BYTES
    big = inputs.box_desc((79,) * 3)
    assert hydro.workspace_bytes(big) > hydro.NOALLOC_WS_BYTES
    assert L.advance_box_noalloc(a, C.c_void_p(1 << 36), C.byref(hydro.make_box(big)),
                                 C.byref(p), a, None, a, None) == hydro.HYDRO_ENOWS


def _both(U_host, box, prm):
    """advance_box (own workspace) and advance_box_noalloc on the same input."""
    import torch
    dev = "cuda:0"
    U = torch.as_tensor(U_host).to(dev).contiguous()
    dt = torch.zeros(1, dtype=torch.float64, device=dev)
    hydro.estimate_dt(U, box, prm, dt)
    out = []
    for noalloc in (False, True):
        Un = torch.full_like(U, float("nan"))
        dtn = torch.zeros(1, dtype=torch.float64, device=dev)
        err = torch.zeros(1, dtype=torch.int32, device=dev)
        if noalloc:
            hydro.advance_box_noalloc(U, Un, box, prm, dt, err, dt_next=dtn)
        else:
            ws = hydro.alloc_workspace(box, dev)
            ws.fill_(0xFF)
            hydro.advance_box(U, Un, box, prm, dt, ws, err, dt_next=dtn)
        torch.cuda.synchronize()
        out.append((inputs.valid(Un.cpu().numpy(), box), dtn.item(), int(err.item())))
    return out


@pytest.mark.gpu
def test_noalloc_equals_advance_box_two_calls():
    import torch
    assert torch.cuda.is_available()
    # a ragged KH box spanning several tiles and z-segments, then a smaller
    # Rayleigh-Taylor box with gravity and reflecting walls
    cases = [inputs.kh((70, 44, 76), seed=3), inputs.rt((20, 18, 24), seed=4)]
    for U, box, prm in cases:
        print("noalloc case", box["n"], flush=True)
        (a, dta, ea), (b, dtb, eb) = _both(U, box, prm)
        assert ea == eb
        assert dta == dtb
        assert np.array_equal(a, b)
    with pytest.raises(hydro.HydroError) as ex:
        big = inputs.box_desc((80, 80, 80))
        Ub = torch.zeros(hydro.state_elems(big), dtype=torch.float64, device="cuda:0")
        d = torch.zeros(1, dtype=torch.float64, device="cuda:0")
        e = torch.zeros(1, dtype=torch.int32, device="cuda:0")
        hydro.advance_box_noalloc(Ub, torch.zeros_like(Ub), big, inputs.params_desc(), d, e)
    assert ex.value.status == hydro.HYDRO_ENOWS
