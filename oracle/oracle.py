"""ctypes binding of the FP64 CPU oracle (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this module.  Arrays are numpy float64 in the box layout: shape
(5, n2+2ng, n1+2ng, n0+2ng), C order, components (rho, rho u, rho v, rho w, E).
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

BC_PERIODIC, BC_OUTFLOW, BC_REFLECT = 0, 1, 2
ERR_NONFINITE, ERR_RHO, ERR_P, ERR_FALLBACK = 1, 2, 4, 8


class OrcBox(C.Structure):
    _fields_ = [("n", C.c_int * 3), ("ng", C.c_int), ("dx", C.c_double * 3),
                ("bc_lo", C.c_int * 3), ("bc_hi", C.c_int * 3)]


class OrcParams(C.Structure):
    _fields_ = [("gamma", C.c_double), ("cfl", C.c_double), ("grav", C.c_double * 3),
                ("flatten", C.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build()
        _lib = _load(path)
    return _lib


class using:
    """Context manager: route every oracle call to the library at ``path``
    (a variant build, e.g. a deliberately broken one in a test)."""

    def __init__(self, path):
        self.path = path

    def __enter__(self):
        global _lib
        self.saved = lib()
        _lib = _load(self.path)
        return self

    def __exit__(self, *exc):
        global _lib
        _lib = self.saved
        return False


def _load(path):
    if True:
        L = C.CDLL(path)
        dp = C.POINTER(C.c_double)
        bp = C.POINTER(OrcBox)
        pp = C.POINTER(OrcParams)
        ip = C.POINTER(C.c_int)
        L.orc_state_elems.argtypes = [bp]
        L.orc_state_elems.restype = C.c_longlong
        L.orc_fill_ghosts.argtypes = [dp, bp]
        L.orc_estimate_dt.argtypes = [dp, bp, pp, dp]
        L.orc_advance_region.argtypes = [dp, dp, bp, pp, C.c_double, ip, ip, ip]
        L.orc_advance_box.argtypes = [dp, dp, bp, pp, C.c_double, ip]
        L.orc_advance_region_species.argtypes = [dp, dp, dp, dp, C.c_int, bp, pp, C.c_double,
                                                 ip, ip, ip]
        L.orc_fill_ghosts_species.argtypes = [dp, C.c_int, bp]
        L.orc_ppm_parabola.argtypes = [dp, dp]
        L.orc_ppm_parabola_flat.argtypes = [dp, C.c_double, dp]
        L.orc_flatten_1d.argtypes = [dp, dp]
        L.orc_flatten_1d.restype = C.c_double
        L.orc_ppm_integrals.argtypes = [dp, C.c_double, C.c_double, dp, dp]
        L.orc_trace.argtypes = [dp, C.c_int, C.c_double, C.c_double, dp, dp]
        L.orc_hllc.argtypes = [dp, dp, C.c_int, C.c_double, dp]
        L.orc_prim_of_cons.argtypes = [dp, C.c_double, dp]
        L.orc_cons_of_prim.argtypes = [dp, C.c_double, dp]
        L.orc_num_threads.restype = C.c_int
        L.orc_set_num_threads.argtypes = [C.c_int]
        L.orc_set_num_threads.restype = None
        L.orc_accept_state.argtypes = [dp, dp, C.c_double, dp]
        L.orc_accept_state.restype = C.c_int
        for f in ("orc_ppm_parabola", "orc_ppm_parabola_flat", "orc_ppm_integrals", "orc_trace", "orc_hllc",
                  "orc_prim_of_cons", "orc_cons_of_prim"):
            getattr(L, f).restype = None
        return L


def _dp(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def make_box(n, ng=4, dx=None, bc_lo=(0, 0, 0), bc_hi=None):
    n = tuple(int(v) for v in n)
    if dx is None:
        dx = tuple(1.0 / v for v in n)
    if bc_hi is None:
        bc_hi = bc_lo
    return OrcBox((C.c_int * 3)(*n), ng, (C.c_double * 3)(*dx),
                  (C.c_int * 3)(*bc_lo), (C.c_int * 3)(*bc_hi))


def box_from(desc):
    """OrcBox from a box description dict (keys n, ng, dx, bc_lo, bc_hi)."""
    return make_box(desc["n"], desc["ng"], desc["dx"], desc["bc_lo"], desc["bc_hi"])


def make_params(gamma=1.4, cfl=0.5, grav=(0.0, 0.0, 0.0), flatten=0):
    return OrcParams(gamma, cfl, (C.c_double * 3)(*grav), flatten)


def params_from(desc):
    return make_params(desc["gamma"], desc["cfl"], desc["grav"], desc.get("flatten", 0))


def fill_ghosts(U, box):
    if lib().orc_fill_ghosts(_dp(U), C.byref(box)) != 0:
        raise ValueError("orc_fill_ghosts: invalid box")


def estimate_dt(U, box, prm):
    dt = C.c_double()
    if lib().orc_estimate_dt(_dp(U), C.byref(box), C.byref(prm), C.byref(dt)) != 0:
        raise ValueError("orc_estimate_dt: invalid arguments")
    return dt.value


def advance_region(U, Unew, box, prm, dt, lo, hi):
    err = C.c_int(0)
    lo_a = (C.c_int * 3)(*lo)
    hi_a = (C.c_int * 3)(*hi)
    rc = lib().orc_advance_region(_dp(U), _dp(Unew), C.byref(box), C.byref(prm),
                                  dt, lo_a, hi_a, C.byref(err))
    if rc == -2:
        raise MemoryError("oracle: out of memory")
    if rc != 0:
        raise ValueError("orc_advance_region: invalid arguments")
    return err.value


def advance_box(U, Unew, box, prm, dt):
    return advance_region(U, Unew, box, prm, dt, (0, 0, 0), tuple(box.n))


# ---- passively advected species: S has shape (nspec, ...) in the state
# layout and holds the partial densities rho X_s

def fill_ghosts_species(S, box):
    if lib().orc_fill_ghosts_species(_dp(S), S.shape[0], C.byref(box)) != 0:
        raise ValueError("orc_fill_ghosts_species: invalid arguments")


def advance_region_species(U, Unew, S, Snew, box, prm, dt, lo, hi):
    err = C.c_int(0)
    lo_a = (C.c_int * 3)(*lo)
    hi_a = (C.c_int * 3)(*hi)
    assert S.shape == Snew.shape and S.shape[1:] == U.shape[1:]
    rc = lib().orc_advance_region_species(_dp(U), _dp(Unew), _dp(S), _dp(Snew), S.shape[0],
                                          C.byref(box), C.byref(prm), dt, lo_a, hi_a,
                                          C.byref(err))
    if rc == -2:
        raise MemoryError("oracle: out of memory")
    if rc != 0:
        raise ValueError("orc_advance_region_species: invalid arguments")
    return err.value


def advance_box_species(U, Unew, S, Snew, box, prm, dt):
    return advance_region_species(U, Unew, S, Snew, box, prm, dt, (0, 0, 0), tuple(box.n))


def step_species(U, S, box, prm):
    """One whole step of the gas and its species: ghost fill of both, CFL dt
    (from the gas), advance.  Returns (Unew, Snew, dt, err)."""
    U = np.ascontiguousarray(U)
    S = np.ascontiguousarray(S)
    fill_ghosts(U, box)
    fill_ghosts_species(S, box)
    dt = estimate_dt(U, box, prm)
    Unew, Snew = U.copy(), S.copy()
    err = advance_box_species(U, Unew, S, Snew, box, prm, dt)
    return Unew, Snew, dt, err


def step(U, box, prm, slab=None):
    """One whole step: ghost fill, CFL dt, advance.  Returns (Unew, dt, err).

    ``slab`` (optional) bounds memory by advancing the box in z-slabs of that
    many cells; every cell's result is independent of the region it is
    computed in, so the answer is identical."""
    U = np.ascontiguousarray(U)
    fill_ghosts(U, box)
    dt = estimate_dt(U, box, prm)
    Unew = U.copy()
    n = tuple(box.n)
    if slab is None or slab >= n[2]:
        err = advance_box(U, Unew, box, prm, dt)
    else:
        err = 0
        for z0 in range(0, n[2], slab):
            err |= advance_region(U, Unew, box, prm, dt, (0, 0, z0),
                                  (n[0], n[1], min(n[2], z0 + slab)))
    return Unew, dt, err


def run(U, box, prm, steps, slab=None):
    """``steps`` whole steps; returns (U, list of dt, err)."""
    dts = []
    err = 0
    for _ in range(steps):
        U, dt, e = step(U, box, prm, slab)
        dts.append(dt)
        err |= e
    return U, dts, err


def ppm_parabola(a5):
    a = np.ascontiguousarray(a5, dtype=np.float64)
    out = np.zeros(2)
    lib().orc_ppm_parabola(_dp(a), _dp(out))
    return out[0], out[1]


def ppm_parabola_flat(a5, f):
    a = np.ascontiguousarray(a5, dtype=np.float64)
    out = np.zeros(2)
    lib().orc_ppm_parabola_flat(_dp(a), f, _dp(out))
    return out[0], out[1]


def flatten_1d(p7, un7):
    """Shock-flattening coefficient of the centre of a 7-cell pencil."""
    p = np.ascontiguousarray(p7, dtype=np.float64)
    u = np.ascontiguousarray(un7, dtype=np.float64)
    return lib().orc_flatten_1d(_dp(p), _dp(u))


def ppm_integrals(a5, lam, dtdx):
    a = np.ascontiguousarray(a5, dtype=np.float64)
    ip, im = C.c_double(), C.c_double()
    lib().orc_ppm_integrals(_dp(a), lam, dtdx, C.byref(ip), C.byref(im))
    return ip.value, im.value


def trace(q5, d, gamma, dtdx):
    q = np.ascontiguousarray(q5, dtype=np.float64).reshape(5, 5)
    qhi, qlo = np.zeros(5), np.zeros(5)
    lib().orc_trace(_dp(q), d, gamma, dtdx, _dp(qhi), _dp(qlo))
    return qhi, qlo


def hllc(qL, qR, d, gamma):
    a = np.ascontiguousarray(qL, dtype=np.float64)
    b = np.ascontiguousarray(qR, dtype=np.float64)
    F = np.zeros(5)
    lib().orc_hllc(_dp(a), _dp(b), d, gamma, _dp(F))
    return F


def prim_of_cons(U, gamma):
    a = np.ascontiguousarray(U, dtype=np.float64)
    q = np.zeros(5)
    lib().orc_prim_of_cons(_dp(a), gamma, _dp(q))
    return q


def cons_of_prim(q, gamma):
    a = np.ascontiguousarray(q, dtype=np.float64)
    U = np.zeros(5)
    lib().orc_cons_of_prim(_dp(a), gamma, _dp(U))
    return U


def accept_state(V, q, gamma):
    """The corrected-state rule: returns (state, flag), state the primitive
    form of the conserved V, or q with flag ERR_FALLBACK when V's density or
    pressure is not positive."""
    a = np.ascontiguousarray(V, dtype=np.float64)
    b = np.ascontiguousarray(q, dtype=np.float64)
    out = np.zeros(5)
    flag = lib().orc_accept_state(_dp(a), _dp(b), gamma, _dp(out))
    return out, flag


def num_threads():
    return lib().orc_num_threads()


def set_num_threads(n):
    """OpenMP threads of the later oracle calls made from this host thread."""
    lib().orc_set_num_threads(int(n))


def level_step(states, boxes, prm, workers=8):
    """One step of independent boxes with the level-wide timestep: ghost fill
    and CFL timestep of every box, their minimum, the advance of every box by
    it.  Several boxes at once on a pool of host threads (each oracle call
    releases the GIL), the OpenMP threads shared among them.  Returns (new
    states, the timestep, error bits); the states passed get their ghosts
    filled."""
    from concurrent.futures import ThreadPoolExecutor
    per = max(1, max(1, num_threads()) // workers)

    def dt_of(i):
        set_num_threads(per)
        fill_ghosts(states[i], boxes[i])
        return estimate_dt(states[i], boxes[i], prm)

    with ThreadPoolExecutor(workers) as pool:
        dt = min(pool.map(dt_of, range(len(states))))

        def one(i):
            set_num_threads(per)
            Un = states[i].copy()
            return Un, advance_box(states[i], Un, boxes[i], prm, dt)

        res = list(pool.map(one, range(len(states))))
    err = 0
    for _, e in res:
        err |= e
    return [r[0] for r in res], dt, err


# stage -> (mark index, work units of the stage per cell-update of an
# unbounded box: 1 primitive conversion, 3 traced cells (one per direction),
# 3 round-1 faces, 6 round-2 faces, 3 round-3 faces, 1 update)
STAGES = {"prim": (1, 1), "trace": (4, 3), "flux1": (5, 3), "corner_flux2": (6, 6),
          "final_flux3": (7, 3), "update": (8, 1)}


def _stage_units(N, stage):
    """Work units the oracle's stage regions hold for an N^3 output region."""
    n1, n2, n6 = N + 1, N + 2, N + 6
    return {"prim": n6 ** 3, "trace": 3 * n2 ** 3, "flux1": 3 * n1 * n2 * n2,
            "corner_flux2": 6 * n1 * N * n2, "final_flux3": 3 * n1 * N * N,
            "update": N ** 3}[stage]


def opcount_cell(U, box, prm, dt, N=16, stage=None):
    """Algorithmic operations (add, mul, div, sqrt, cmp) of one cell-update,
    counted by the operation-counting build of the oracle on the data of U
    (ghosts filled): each stage's average cost per work unit over an N^3
    output region, times its work units per cell of an unbounded box (no
    halo recomputation).  ``stage``: None for the whole step, a stage name or
    a list of names (see STAGES)."""
    path = _build.OPC_LIB
    if not os.path.exists(path):
        _build.build()
    L = C.CDLL(path)
    L.orc_opcount_region.argtypes = [C.POINTER(C.c_double), C.POINTER(OrcBox),
                                     C.POINTER(OrcParams), C.c_double, C.c_int,
                                     C.POINTER(C.c_double)]
    ops = np.zeros((9, 5))
    rc = L.orc_opcount_region(_dp(np.ascontiguousarray(U)), C.byref(box), C.byref(prm), dt, N,
                              _dp(ops))
    if rc != 0:
        raise RuntimeError("orc_opcount_region failed")
    names = list(STAGES) if stage is None else ([stage] if isinstance(stage, str) else stage)
    tot = np.zeros(5)
    for s in names:
        k, per_cell = STAGES[s]
        tot += ops[k] / _stage_units(N, s) * per_cell
    return dict(zip(("add", "mul", "div", "sqrt", "cmp"), tot.tolist()))
