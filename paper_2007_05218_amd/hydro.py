"""Python binding of the C ABI in include/hydro.h (argument marshalling only).

Every function here forwards to ``libhydro.so``; all arithmetic of the hydro
step runs in its HIP kernels.  PyTorch provides device memory and streams:
state arrays are CUDA float64 tensors of shape (5, n2+2ng, n1+2ng, n0+2ng)
(see inputs.state_shape), timesteps and error words are small device
tensors, and every call is enqueued on torch's current stream unless a
stream is given.

There is no CPU fallback: importing this module without the built library,
or calling it without a GPU, raises.
"""
import ctypes as C
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhydro.so")

HYDRO_OK, HYDRO_EINVAL, HYDRO_EHIP, HYDRO_ENOWS = 0, 1, 2, 3
ERR_NONFINITE, ERR_RHO, ERR_P, ERR_FALLBACK = 1, 2, 4, 8

EXPORTS = ("hydro_state_elems", "hydro_workspace_bytes", "hydro_fill_ghosts", "estimate_dt",
           "advance_box", "estimate_dt_boxes", "advance_boxes", "hydro_plan_create",
           "hydro_plan_destroy", "hydro_status_string", "hydro_stage_count",
           "hydro_stage_name", "hydro_set_stage_events", "hydro_fill_ghosts_boxes",
           "hydro_level_create", "hydro_level_destroy", "hydro_fill_ghosts_level",
           "hydro_species_workspace_bytes", "hydro_fill_ghosts_species", "advance_box_species",
           "hydro_species_workspace_bytes_boxes", "hydro_fill_ghosts_boxes_species",
           "advance_boxes_species", "hydro_fill_ghosts_level_species", "advance_box_noalloc",
           "hydro_plan_create_capacity", "hydro_plan_update", "hydro_plan_boxes",
           "hydro_plan_workspace_bytes")


class HydroBox(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("ng", C.c_int32), ("dx", C.c_double * 3),
                ("bc_lo", C.c_int32 * 3), ("bc_hi", C.c_int32 * 3)]


class HydroParams(C.Structure):
    _fields_ = [("gamma", C.c_double), ("cfl", C.c_double), ("grav", C.c_double * 3),
                ("flatten", C.c_int32)]


class HydroError(RuntimeError):
    def __init__(self, fn, status):
        self.status = status
        msg = lib().hydro_status_string(status).decode()
        super().__init__("%s: %s" % (fn, msg))


_lib = None


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libhydro.so is not built: run paper_2007_05218_amd/build.py "
                               "(or __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        bp = C.POINTER(HydroBox)
        pp = C.POINTER(HydroParams)
        L.hydro_state_elems.argtypes = [bp]
        L.hydro_state_elems.restype = C.c_size_t
        L.hydro_workspace_bytes.argtypes = [bp, C.c_int]
        L.hydro_workspace_bytes.restype = C.c_size_t
        L.hydro_fill_ghosts.argtypes = [vp, bp, vp]
        L.estimate_dt.argtypes = [vp, bp, pp, vp, vp]
        L.advance_box.argtypes = [vp, vp, bp, pp, vp, vp, vp, C.c_size_t, vp, vp]
        L.advance_box_noalloc.argtypes = [vp, vp, bp, pp, vp, vp, vp, vp]
        L.estimate_dt_boxes.argtypes = [C.c_int, vp, vp, pp, vp, vp, vp]
        L.advance_boxes.argtypes = [C.c_int, vp, vp, vp, pp, vp, C.c_int, vp, vp, vp,
                                    C.c_size_t, vp, vp]
        L.hydro_plan_create.argtypes = [bp, C.c_int, C.c_char_p, C.POINTER(vp)]
        L.hydro_plan_create_capacity.argtypes = [C.c_int, C.c_char_p, C.POINTER(vp)]
        L.hydro_plan_update.argtypes = [vp, bp, C.c_int, vp]
        L.hydro_plan_boxes.argtypes = [vp]
        L.hydro_plan_boxes.restype = C.c_int
        L.hydro_plan_workspace_bytes.argtypes = [vp]
        L.hydro_plan_workspace_bytes.restype = C.c_size_t
        L.hydro_plan_destroy.argtypes = [vp]
        L.hydro_plan_destroy.restype = None
        L.hydro_stage_count.argtypes = []
        L.hydro_stage_count.restype = C.c_int
        L.hydro_stage_name.argtypes = [C.c_int]
        L.hydro_stage_name.restype = C.c_char_p
        L.hydro_set_stage_events.argtypes = [C.POINTER(vp)]
        L.hydro_set_stage_events.restype = C.c_int
        L.hydro_status_string.argtypes = [C.c_int]
        L.hydro_status_string.restype = C.c_char_p
        L.hydro_fill_ghosts_boxes.argtypes = [C.c_int, vp, vp, vp]
        i3 = C.POINTER(C.c_int32)
        L.hydro_level_create.argtypes = [bp, i3, C.c_int, i3, i3, i3, C.POINTER(vp)]
        L.hydro_level_destroy.argtypes = [vp]
        L.hydro_level_destroy.restype = None
        L.hydro_fill_ghosts_level.argtypes = [C.c_int, vp, vp, vp]
        L.hydro_species_workspace_bytes.argtypes = [bp, C.c_int]
        L.hydro_species_workspace_bytes.restype = C.c_size_t
        L.hydro_fill_ghosts_species.argtypes = [vp, C.c_int, bp, vp]
        L.advance_box_species.argtypes = [vp, vp, vp, vp, C.c_int, bp, pp, vp, vp, vp,
                                          C.c_size_t, vp, C.c_size_t, vp, vp]
        L.hydro_species_workspace_bytes_boxes.argtypes = [bp, C.c_int, C.c_int]
        L.hydro_species_workspace_bytes_boxes.restype = C.c_size_t
        L.hydro_fill_ghosts_boxes_species.argtypes = [C.c_int, vp, C.c_int, vp, vp]
        L.advance_boxes_species.argtypes = [C.c_int, vp, vp, vp, vp, C.c_int, vp, pp, vp,
                                            C.c_int, vp, vp, vp, C.c_size_t, vp, C.c_size_t,
                                            vp, vp]
        L.hydro_fill_ghosts_level_species.argtypes = [C.c_int, vp, C.c_int, vp, vp]
        for f in ("hydro_fill_ghosts", "estimate_dt", "advance_box", "estimate_dt_boxes",
                  "advance_boxes", "hydro_plan_create", "hydro_fill_ghosts_boxes",
                  "hydro_level_create", "hydro_fill_ghosts_level", "hydro_fill_ghosts_species",
                  "advance_box_species", "hydro_fill_ghosts_boxes_species",
                  "advance_boxes_species", "hydro_fill_ghosts_level_species",
                  "advance_box_noalloc", "hydro_plan_create_capacity", "hydro_plan_update"):
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def _check(fn, st):
    if st != HYDRO_OK:
        raise HydroError(fn, st)


def make_box(desc):
    """HydroBox from a box description dict (inputs.box_desc)."""
    return HydroBox((C.c_int32 * 3)(*desc["n"]), desc["ng"], (C.c_double * 3)(*desc["dx"]),
                    (C.c_int32 * 3)(*desc["bc_lo"]), (C.c_int32 * 3)(*desc["bc_hi"]))


def make_params(desc):
    return HydroParams(desc["gamma"], desc["cfl"], (C.c_double * 3)(*desc["grav"]),
                       int(desc.get("flatten", 0)))


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t, dtype=torch.float64):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise ValueError("expected a contiguous CUDA %s tensor" % dtype)
    return C.c_void_p(t.data_ptr())


def state_elems(box):
    return int(lib().hydro_state_elems(C.byref(make_box(box))))


def workspace_bytes(boxes):
    if isinstance(boxes, dict):
        boxes = [boxes]
    arr = (HydroBox * len(boxes))(*[make_box(b) for b in boxes])
    return int(lib().hydro_workspace_bytes(arr, len(boxes)))


def _check_state(U, box):
    if U.numel() != state_elems(box):
        raise ValueError("state tensor has %d elements, box needs %d"
                         % (U.numel(), state_elems(box)))


def fill_ghosts(U, box, stream=None):
    _check_state(U, box)
    _check("hydro_fill_ghosts", lib().hydro_fill_ghosts(_ptr(U), C.byref(make_box(box)),
                                                        _stream(stream)))


def estimate_dt(U, box, prm, dt, stream=None):
    """Fill U's ghosts and write the CFL timestep to the 1-element device tensor dt."""
    _check_state(U, box)
    _check("estimate_dt", lib().estimate_dt(_ptr(U), C.byref(make_box(box)),
                                            C.byref(make_params(prm)), _ptr(dt),
                                            _stream(stream)))


def advance_box(U, Unew, box, prm, dt, ws, err, stream=None, dt_next=None):
    """One step of length dt[0] from U (ghosts filled) into the valid cells of
    Unew; with ``dt_next`` (1-element device tensor) also Unew's CFL timestep."""
    _check_state(U, box)
    _check_state(Unew, box)
    _check("advance_box", lib().advance_box(_ptr(U), _ptr(Unew), C.byref(make_box(box)),
                                            C.byref(make_params(prm)), _ptr(dt),
                                            _ptr(dt_next) if dt_next is not None else None,
                                            _ptr(ws, torch.uint8), ws.numel(),
                                            _ptr(err, torch.int32), _stream(stream)))


NOALLOC_WS_BYTES = 128 << 20  # HYDRO_NOALLOC_WS_BYTES


def advance_box_noalloc(U, Unew, box, prm, dt, err, stream=None, dt_next=None):
    """advance_box without a workspace: the library's static per-GPU array of
    NOALLOC_WS_BYTES holds the traced states (boxes needing more raise
    HydroError with HYDRO_ENOWS).  Calls overlapping in time on one GPU race."""
    _check_state(U, box)
    _check_state(Unew, box)
    _check("advance_box_noalloc", lib().advance_box_noalloc(
        _ptr(U), _ptr(Unew), C.byref(make_box(box)), C.byref(make_params(prm)), _ptr(dt),
        _ptr(dt_next) if dt_next is not None else None, _ptr(err, torch.int32),
        _stream(stream)))


def alloc_workspace(boxes, device="cuda"):
    return torch.empty(max(workspace_bytes(boxes), 256), dtype=torch.uint8, device=device)


class Box:
    """A single box on the GPU: state ping-pong buffers, workspace, dt and error
    words, all device-resident; ``step()`` enqueues one whole step
    (ghost fill + dt + advance) with no host synchronisation."""

    def __init__(self, U_host, box, prm, device="cuda"):
        self.box = dict(box)
        self.prm = dict(prm)
        self.U = torch.as_tensor(U_host, dtype=torch.float64).to(device).contiguous()
        self.Unew = torch.empty_like(self.U)
        self.ws = alloc_workspace(self.box, device)
        self.dt = torch.zeros(1, dtype=torch.float64, device=device)
        self.dt_next = torch.zeros(1, dtype=torch.float64, device=device)
        self.err = torch.zeros(1, dtype=torch.int32, device=device)
        self.t = torch.zeros(1, dtype=torch.float64, device=device)
        self.have_dt = False  # dt_next holds the current state's timestep

    def step(self, stream=None):
        """Ghost fill + CFL timestep + advance.  The timestep of a state the
        previous step produced comes from that step's advance (bitwise the
        estimate_dt value), so only the ghost fill runs before the advance;
        ``self.dt`` is the timestep of the step just taken."""
        if self.have_dt:
            fill_ghosts(self.U, self.box, stream)
            self.dt, self.dt_next = self.dt_next, self.dt
        else:
            estimate_dt(self.U, self.box, self.prm, self.dt, stream)
        advance_box(self.U, self.Unew, self.box, self.prm, self.dt, self.ws, self.err, stream,
                    dt_next=self.dt_next)
        self.U, self.Unew = self.Unew, self.U
        self.have_dt = True

    def invalidate_dt(self):
        """Call after changing ``self.U`` directly: the next step computes its
        timestep from the state instead of taking the carried one."""
        self.have_dt = False

    def run(self, steps, stream=None):
        for _ in range(steps):
            self.step(stream)

    def state(self):
        """Host copy of the current state (ghosts as last filled)."""
        return self.U.cpu().numpy()


# ---- passively advected species: S is a CUDA float64 tensor of shape
# (nspec,) + the state's spatial shape holding the partial densities rho X_s

def species_workspace_bytes(box, nspec):
    return int(lib().hydro_species_workspace_bytes(C.byref(make_box(box)), int(nspec)))


def _check_species(S, box):
    per = state_elems(box) // 5
    if S.numel() % per or not 1 <= S.numel() // per:
        raise ValueError("species tensor of %d elements does not fit the box" % S.numel())
    return S.numel() // per


def fill_ghosts_species(S, box, stream=None):
    ns = _check_species(S, box)
    _check("hydro_fill_ghosts_species", lib().hydro_fill_ghosts_species(
        _ptr(S), ns, C.byref(make_box(box)), _stream(stream)))


def advance_box_species(U, Unew, S, Snew, box, prm, dt, ws, sws, err, stream=None,
                        dt_next=None):
    """advance_box plus the species: Snew's valid cells from S (ghosts filled)."""
    _check_state(U, box)
    _check_state(Unew, box)
    ns = _check_species(S, box)
    if _check_species(Snew, box) != ns:
        raise ValueError("S and Snew differ in species count")
    _check("advance_box_species", lib().advance_box_species(
        _ptr(U), _ptr(Unew), _ptr(S), _ptr(Snew), ns, C.byref(make_box(box)),
        C.byref(make_params(prm)), _ptr(dt), _ptr(dt_next) if dt_next is not None else None,
        _ptr(ws, torch.uint8), ws.numel(), _ptr(sws, torch.uint8), sws.numel(),
        _ptr(err, torch.int32), _stream(stream)))


class SpeciesBox(Box):
    """A Box that also carries nspec passively advected species (partial
    densities S, host array of shape (nspec,) + the state's spatial shape)."""

    def __init__(self, U_host, S_host, box, prm, device="cuda"):
        super().__init__(U_host, box, prm, device)
        self.S = torch.as_tensor(S_host, dtype=torch.float64).to(device).contiguous()
        self.Snew = torch.empty_like(self.S)
        self.sws = torch.empty(max(species_workspace_bytes(self.box, self.S.shape[0]), 256),
                               dtype=torch.uint8, device=device)

    def step(self, stream=None):
        if self.have_dt:
            fill_ghosts(self.U, self.box, stream)
            self.dt, self.dt_next = self.dt_next, self.dt
        else:
            estimate_dt(self.U, self.box, self.prm, self.dt, stream)
        fill_ghosts_species(self.S, self.box, stream)
        advance_box_species(self.U, self.Unew, self.S, self.Snew, self.box, self.prm, self.dt,
                            self.ws, self.sws, self.err, stream, dt_next=self.dt_next)
        self.U, self.Unew = self.Unew, self.U
        self.S, self.Snew = self.Snew, self.S
        self.have_dt = True

    def species(self):
        """Host copy of the current partial densities."""
        return self.S.cpu().numpy()


class Plan:
    """A plan for a list of boxes: validated boxes, per-stage work lists on the
    device.  Owns one small device buffer.  ``Plan(boxes)`` is fixed
    (hydro_plan_create); ``Plan.with_capacity(n)`` starts empty and takes a
    new list of up to n boxes with ``update`` (hydro_plan_update: an
    asynchronous copy on the stream, no device allocation)."""

    def __init__(self, boxes, autotune_json=None):
        self.boxes = [dict(b) for b in boxes]
        arr = (HydroBox * len(boxes))(*[make_box(b) for b in boxes])
        h = C.c_void_p()
        js = autotune_json.encode() if autotune_json else None
        _check("hydro_plan_create", lib().hydro_plan_create(arr, len(boxes), js, C.byref(h)))
        self.handle = h
        self.nb = len(boxes)
        self.capacity = self.nb
        self.ws_bytes = workspace_bytes(self.boxes)

    @classmethod
    def with_capacity(cls, capacity, autotune_json=None):
        self = cls.__new__(cls)
        h = C.c_void_p()
        js = autotune_json.encode() if autotune_json else None
        _check("hydro_plan_create_capacity",
               lib().hydro_plan_create_capacity(int(capacity), js, C.byref(h)))
        self.handle = h
        self.boxes = []
        self.nb = 0
        self.capacity = int(capacity)
        self.ws_bytes = 0
        return self

    def update(self, boxes, stream=None):
        """Replace the list of boxes (stream-ordered with the batched calls)."""
        arr = (HydroBox * len(boxes))(*[make_box(b) for b in boxes])
        _check("hydro_plan_update", lib().hydro_plan_update(self.handle, arr, len(boxes),
                                                            _stream(stream)))
        self.boxes = [dict(b) for b in boxes]
        self.nb = len(boxes)
        self.ws_bytes = int(lib().hydro_plan_workspace_bytes(self.handle))

    def close(self):
        if self.handle:
            lib().hydro_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pointer_array(tensors, device="cuda"):
    """Device int64 tensor holding the data pointers of ``tensors``."""
    return torch.tensor([t.data_ptr() for t in tensors], dtype=torch.int64, device=device)


def estimate_dt_boxes(plan, U_ptrs, prm, dt, dt_min=None, stream=None):
    """Fill every box's ghosts; dt[b] = box b's CFL step; dt_min[0] = min over boxes."""
    _check("estimate_dt_boxes", lib().estimate_dt_boxes(
        plan.nb, _ptr(U_ptrs, torch.int64), plan.handle, C.byref(make_params(prm)), _ptr(dt),
        _ptr(dt_min) if dt_min is not None else None, _stream(stream)))


def advance_boxes(plan, U_ptrs, Unew_ptrs, prm, dt, ws, err, dt_stride=1, stream=None,
                  dt_next=None, dt_next_min=None):
    """Advance every box of the plan by dt[b] (dt_stride=1) or dt[0]
    (dt_stride=0); with ``dt_next`` also every new state's CFL timestep, and
    with ``dt_next_min`` their minimum."""
    _check("advance_boxes", lib().advance_boxes(
        plan.nb, _ptr(U_ptrs, torch.int64), _ptr(Unew_ptrs, torch.int64), plan.handle,
        C.byref(make_params(prm)), _ptr(dt), dt_stride,
        _ptr(dt_next) if dt_next is not None else None,
        _ptr(dt_next_min) if dt_next_min is not None else None,
        _ptr(ws, torch.uint8), ws.numel(), _ptr(err, torch.int32), _stream(stream)))


def species_workspace_bytes_boxes(boxes, nspec):
    arr = (HydroBox * len(boxes))(*[make_box(b) for b in boxes])
    return int(lib().hydro_species_workspace_bytes_boxes(arr, len(boxes), int(nspec)))


def fill_ghosts_boxes_species(plan, S_ptrs, nspec, stream=None):
    """Species ghost fill of every box of the plan (one launch)."""
    _check("hydro_fill_ghosts_boxes_species", lib().hydro_fill_ghosts_boxes_species(
        plan.nb, _ptr(S_ptrs, torch.int64), int(nspec), plan.handle, _stream(stream)))


def advance_boxes_species(plan, U_ptrs, Unew_ptrs, S_ptrs, Snew_ptrs, nspec, prm, dt, ws, sws,
                          err, dt_stride=1, stream=None, dt_next=None, dt_next_min=None):
    """advance_boxes plus the species of every box."""
    _check("advance_boxes_species", lib().advance_boxes_species(
        plan.nb, _ptr(U_ptrs, torch.int64), _ptr(Unew_ptrs, torch.int64),
        _ptr(S_ptrs, torch.int64), _ptr(Snew_ptrs, torch.int64), int(nspec), plan.handle,
        C.byref(make_params(prm)), _ptr(dt), dt_stride,
        _ptr(dt_next) if dt_next is not None else None,
        _ptr(dt_next_min) if dt_next_min is not None else None,
        _ptr(ws, torch.uint8), ws.numel(), _ptr(sws, torch.uint8), sws.numel(),
        _ptr(err, torch.int32), _stream(stream)))


def fill_ghosts_boxes(plan, U_ptrs, stream=None):
    """Ghost fill of every box of the plan (one launch)."""
    _check("hydro_fill_ghosts_boxes", lib().hydro_fill_ghosts_boxes(
        plan.nb, _ptr(U_ptrs, torch.int64), plan.handle, _stream(stream)))


class Tiling:
    """The boxes of a level tiling one domain (hydro_level_create): box b's
    valid cell (0,0,0) sits at domain index ``lo[b]``; ``dom`` is the domain's
    cell count and ``bc_lo``/``bc_hi`` its boundary kinds.  Owns one small
    device buffer."""

    def __init__(self, boxes, lo, dom, bc_lo, bc_hi):
        self.boxes = [dict(b) for b in boxes]
        self.lo = [tuple(int(v) for v in l) for l in lo]
        self.dom = tuple(int(v) for v in dom)
        self.bc_lo, self.bc_hi = tuple(bc_lo), tuple(bc_hi)
        arr = (HydroBox * len(boxes))(*[make_box(b) for b in boxes])
        flat = (C.c_int32 * (3 * len(boxes)))(*[v for l in self.lo for v in l])
        i3 = C.c_int32 * 3
        h = C.c_void_p()
        _check("hydro_level_create", lib().hydro_level_create(
            arr, flat, len(boxes), i3(*self.dom), i3(*self.bc_lo), i3(*self.bc_hi),
            C.byref(h)))
        self.handle = h
        self.nb = len(boxes)

    def close(self):
        if self.handle:
            lib().hydro_level_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fill_ghosts_level(tiling, U_ptrs, stream=None):
    """Ghost exchange between the boxes of a tiled level (one launch)."""
    _check("hydro_fill_ghosts_level", lib().hydro_fill_ghosts_level(
        tiling.nb, _ptr(U_ptrs, torch.int64), tiling.handle, _stream(stream)))


def fill_ghosts_level_species(tiling, S_ptrs, nspec, stream=None):
    """Species ghost exchange between the boxes of a tiled level (one launch)."""
    _check("hydro_fill_ghosts_level_species", lib().hydro_fill_ghosts_level_species(
        tiling.nb, _ptr(S_ptrs, torch.int64), int(nspec), tiling.handle, _stream(stream)))


class Level:
    """A list of boxes advanced together (a level of boxes): states and
    workspace on the device, one launch per stage for all boxes.
    ``shared_dt`` advances every box by the level-wide minimum timestep.
    Without ``tiling`` the boxes are independent (each fills its own ghosts
    from its boundary kinds); with a ``Tiling`` of the same boxes they tile one
    domain, the ghosts come from the neighbouring boxes (hydro_fill_ghosts_level)
    and the timestep is shared.  ``species`` (optional): one host array of
    partial densities per box (shape (nspec,) + the box's spatial shape),
    advanced with the gas (advance_boxes_species)."""

    def __init__(self, states, boxes, prm, shared_dt=True, device="cuda", autotune_json=None,
                 tiling=None, species=None):
        if tiling is not None and (not shared_dt or tiling.nb != len(boxes)):
            raise ValueError("a tiled level needs a tiling of its boxes and a shared timestep")
        self.tiling = tiling
        self.prm = dict(prm)
        self.plan = Plan(boxes, autotune_json)
        self.U = [torch.as_tensor(u, dtype=torch.float64).to(device).contiguous() for u in states]
        self.Unew = [torch.empty_like(u) for u in self.U]
        self.pa = pointer_array(self.U, device)
        self.pb = pointer_array(self.Unew, device)
        self.ws = torch.empty(max(self.plan.ws_bytes, 256), dtype=torch.uint8, device=device)
        self.dt = torch.zeros(len(states), dtype=torch.float64, device=device)
        self.dt_min = torch.zeros(1, dtype=torch.float64, device=device)
        self.dt_next = torch.zeros(len(states), dtype=torch.float64, device=device)
        self.dt_next_min = torch.zeros(1, dtype=torch.float64, device=device)
        self.err = torch.zeros(1, dtype=torch.int32, device=device)
        self.shared_dt = shared_dt
        self.have_dt = False  # dt_next / dt_next_min hold the current states' timesteps
        self.S = None
        if species is not None:
            self.S = [torch.as_tensor(x, dtype=torch.float64).to(device).contiguous()
                      for x in species]
            self.nspec = self.S[0].shape[0]
            if len(self.S) != len(self.U) or any(x.shape[0] != self.nspec for x in self.S):
                raise ValueError("one species array per box, all with the same count")
            self.Snew = [torch.empty_like(x) for x in self.S]
            self.sa = pointer_array(self.S, device)
            self.sb = pointer_array(self.Snew, device)
            self.sws = torch.empty(max(species_workspace_bytes_boxes(self.plan.boxes,
                                                                     self.nspec), 256),
                                   dtype=torch.uint8, device=device)

    def step(self, stream=None):
        """Ghost fill + timesteps + advance of every box (the timesteps of
        states the previous step produced come from that step's advance)."""
        if self.have_dt:
            if self.tiling is None:
                fill_ghosts_boxes(self.plan, self.pa, stream)
            self.dt, self.dt_next = self.dt_next, self.dt
            self.dt_min, self.dt_next_min = self.dt_next_min, self.dt_min
        else:
            # (the timestep reads valid cells only; its per-box ghost fill is
            # replaced below for a tiled level)
            estimate_dt_boxes(self.plan, self.pa, self.prm, self.dt, self.dt_min, stream)
        if self.tiling is not None:
            fill_ghosts_level(self.tiling, self.pa, stream)
        dt, stride = (self.dt_min, 0) if self.shared_dt else (self.dt, 1)
        dtnm = self.dt_next_min if self.shared_dt else None
        if self.S is None:
            advance_boxes(self.plan, self.pa, self.pb, self.prm, dt, self.ws, self.err,
                          dt_stride=stride, stream=stream, dt_next=self.dt_next,
                          dt_next_min=dtnm)
        else:
            if self.tiling is not None:
                fill_ghosts_level_species(self.tiling, self.sa, self.nspec, stream)
            else:
                fill_ghosts_boxes_species(self.plan, self.sa, self.nspec, stream)
            advance_boxes_species(self.plan, self.pa, self.pb, self.sa, self.sb, self.nspec,
                                  self.prm, dt, self.ws, self.sws, self.err, dt_stride=stride,
                                  stream=stream, dt_next=self.dt_next, dt_next_min=dtnm)
            self.S, self.Snew = self.Snew, self.S
            self.sa, self.sb = self.sb, self.sa
        self.U, self.Unew = self.Unew, self.U
        self.pa, self.pb = self.pb, self.pa
        self.have_dt = True

    def invalidate_dt(self):
        """Call after changing the states directly: the next step computes the
        timesteps from them instead of taking the carried ones."""
        self.have_dt = False

    def run(self, steps, stream=None):
        for _ in range(steps):
            self.step(stream)

    def states(self):
        return [u.cpu().numpy() for u in self.U]

    def species(self):
        return [x.cpu().numpy() for x in self.S]


class StageTimer:
    """Per-stage device time of library calls (hydro_set_stage_events): wrap
    each profiled call in ``with timer:``; totals accumulate in ms per stage."""

    def __init__(self):
        L = lib()
        self.names = [L.hydro_stage_name(s).decode() for s in range(L.hydro_stage_count())]
        self.events = [torch.cuda.Event(enable_timing=True) for _ in range(2 * len(self.names))]
        s = torch.cuda.current_stream()
        for e in self.events:  # torch creates the HIP event on first record
            e.record(s)
        torch.cuda.synchronize()
        self.total_ms = {n: 0.0 for n in self.names}
        self.calls = 0

    def __enter__(self):
        for e in self.events:
            e.record()
        torch.cuda.synchronize()
        arr = (C.c_void_p * len(self.events))(*[e.cuda_event for e in self.events])
        _check("hydro_set_stage_events", lib().hydro_set_stage_events(arr))
        return self

    def __exit__(self, *exc):
        lib().hydro_set_stage_events(None)
        torch.cuda.synchronize()
        for i, n in enumerate(self.names):
            a, b = self.events[2 * i], self.events[2 * i + 1]
            ms = a.elapsed_time(b)
            if ms > 0:
                self.total_ms[n] += ms
        self.calls += 1
        return False
