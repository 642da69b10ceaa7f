"""Seeded synthetic initial conditions for the hydro workloads.

This module only builds inputs: box descriptions and host FP64 state arrays.
It holds none of the hydro scheme's arithmetic and imports nothing but numpy,
so the GPU library and the CPU oracle can both be fed from it.

Layout of a state array: numpy float64, shape (5, n2+2ng, n1+2ng, n0+2ng),
C order (x fastest), components (rho, rho*u, rho*v, rho*w, E); ghost cells are
zero and are filled by the boundary fill of whichever path advances the box.
Initial values are point values at cell centres x_i = (i + 1/2) dx.

Workloads (the paper's Sec. IV uses blast-wave and bubble problems whose
inputs are not available; these synthetic families stand in for them):
  sod      Sod shock tube along one axis, outflow boundaries
  kh       Kelvin-Helmholtz shear layer, periodic, seeded v,w noise
  rt       Rayleigh-Taylor, heavy over light in hydrostatic balance under
           g = -0.1 z, seeded phase of a single-mode interface, reflecting z walls
  smooth   sum of seeded Fourier modes, periodic (the batched AMR-like level)
  advect   a smooth density wave carried by a uniform flow, periodic
  sedov    point blast in the unit cube, outflow boundaries (the paper's
           Sec. IV hydro benchmark problem), also as a domain tiled by boxes
"""
import math

import numpy as np

BC_PERIODIC, BC_OUTFLOW, BC_REFLECT = 0, 1, 2
GAMMA = 1.4
CFL = 0.5
NG = 4


def box_desc(n, ng=NG, dx=None, bc_lo=(BC_PERIODIC,) * 3, bc_hi=None):
    """A box description: valid cells n, ghost layers, cell widths, boundary kinds."""
    n = tuple(int(v) for v in n)
    if dx is None:
        dx = tuple(1.0 / v for v in n)
    if bc_hi is None:
        bc_hi = tuple(bc_lo)
    return {"n": n, "ng": int(ng), "dx": tuple(float(v) for v in dx),
            "bc_lo": tuple(int(v) for v in bc_lo), "bc_hi": tuple(int(v) for v in bc_hi)}


def params_desc(gamma=GAMMA, cfl=CFL, grav=(0.0, 0.0, 0.0), flatten=0):
    """Method parameters; ``flatten`` = 1 switches shock flattening on."""
    return {"gamma": float(gamma), "cfl": float(cfl), "grav": tuple(float(g) for g in grav),
            "flatten": int(flatten)}


def state_shape(box):
    n, ng = box["n"], box["ng"]
    return (5, n[2] + 2 * ng, n[1] + 2 * ng, n[0] + 2 * ng)


def cell_centres(box):
    """Broadcastable (x, y, z) cell-centre coordinates of the valid cells."""
    n, dx = box["n"], box["dx"]
    x = (np.arange(n[0]) + 0.5) * dx[0]
    y = (np.arange(n[1]) + 0.5) * dx[1]
    z = (np.arange(n[2]) + 0.5) * dx[2]
    return x[None, None, :], y[None, :, None], z[:, None, None]


def from_primitive(box, rho, u, v, w, p, gamma=GAMMA):
    """State array of a box whose valid cells hold the given primitive fields."""
    n, ng = box["n"], box["ng"]
    shp = (n[2], n[1], n[0])
    rho, u, v, w, p = (np.broadcast_to(np.asarray(a, dtype=np.float64), shp)
                       for a in (rho, u, v, w, p))
    U = np.zeros(state_shape(box))
    sl = (slice(ng, ng + n[2]), slice(ng, ng + n[1]), slice(ng, ng + n[0]))
    U[0][sl] = rho
    U[1][sl] = rho * u
    U[2][sl] = rho * v
    U[3][sl] = rho * w
    U[4][sl] = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)
    return U


def valid(U, box):
    """View of the valid cells of a state array, shape (5, n2, n1, n0)."""
    n, ng = box["n"], box["ng"]
    return U[:, ng:ng + n[2], ng:ng + n[1], ng:ng + n[0]]


# ---------------------------------------------------------------------------
# workload families
# ---------------------------------------------------------------------------

def sod(n=32, axis=0, mirror=False, ng=NG):
    """Sod tube along ``axis``: (rho, p) = (1, 1) below the midplane, (0.125, 0.1)
    above; at rest; outflow on all faces.  ``mirror`` swaps the two sides."""
    nn = (n, n, n) if np.isscalar(n) else tuple(n)
    box = box_desc(nn, ng, bc_lo=(BC_OUTFLOW,) * 3)
    xc = cell_centres(box)[axis]
    left = xc < 0.5
    if mirror:
        left = ~left
    rho = np.where(left, 1.0, 0.125)
    p = np.where(left, 1.0, 0.1)
    return from_primitive(box, rho, 0.0, 0.0, 0.0, p), box, params_desc()


def kh(n=256, seed=1, ng=NG):
    """Kelvin-Helmholtz: rho = 2, u = +0.5 for |y - 0.5| < 0.25, else rho = 1,
    u = -0.5; p = 2.5; v, w i.i.d. uniform in (-0.01, 0.01) per cell."""
    nn = (n, n, n) if np.isscalar(n) else tuple(n)
    box = box_desc(nn, ng, bc_lo=(BC_PERIODIC,) * 3)
    rng = np.random.default_rng(seed)
    shp = (nn[2], nn[1], nn[0])
    v = rng.uniform(-0.01, 0.01, size=shp)
    w = rng.uniform(-0.01, 0.01, size=shp)
    _, y, _ = cell_centres(box)
    inner = np.abs(y - 0.5) < 0.25
    rho = np.broadcast_to(np.where(inner, 2.0, 1.0), shp)
    u = np.broadcast_to(np.where(inner, 0.5, -0.5), shp)
    return from_primitive(box, rho, u, v, w, 2.5), box, params_desc()


def rt(n=512, seed=4, ng=NG, gz=-0.1):
    """Rayleigh-Taylor: interface z_i = 0.5 + 0.01 cos(2 pi (x + px)) cos(2 pi (y + py))
    with seeded phases px, py in [0, 1); rho = 2 above, 1 below; column-wise
    hydrostatic p = 2.5 + gz rho (z - z_i); at rest; periodic x, y; reflecting z."""
    nn = (n, n, n) if np.isscalar(n) else tuple(n)
    box = box_desc(nn, ng, bc_lo=(BC_PERIODIC, BC_PERIODIC, BC_REFLECT))
    rng = np.random.default_rng(seed)
    px, py = rng.uniform(0.0, 1.0, size=2)
    x, y, z = cell_centres(box)
    zi = 0.5 + 0.01 * np.cos(2 * np.pi * (x + px)) * np.cos(2 * np.pi * (y + py))
    rho = np.where(z > zi, 2.0, 1.0)
    p = 2.5 + gz * rho * (z - zi)
    return (from_primitive(box, rho, 0.0, 0.0, 0.0, p), box,
            params_desc(grav=(0.0, 0.0, gz)))


def _modes(rng, n, L, xyz):
    """Normalised sum of 8 random Fourier modes, values in [-1, 1]."""
    K = [max(1, v // 16) for v in n]
    S = 0.0
    asum = 0.0
    for _ in range(8):
        while True:
            k = [int(rng.integers(-K[d], K[d] + 1)) for d in range(3)]
            if any(k):
                break
        a = rng.uniform(0.5, 1.0)
        ph = rng.uniform(0.0, 2 * np.pi)
        # a cos(k.x + ph) as the real part of a product of one-dimensional
        # complex exponentials (one multiply per cell instead of a cosine)
        e = [np.exp(1j * (2 * np.pi * k[d] / L[d]) * xyz[d]) for d in range(3)]
        S = S + (a * np.exp(1j * ph)) * (e[2] * e[1]) * e[0]
        asum += a
    return np.real(S) / asum


def smooth(n, seed, dx=None, ng=NG):
    """Smooth random periodic box: rho, p = 1.25 + 0.75 S, each u_d = 0.5 S_d,
    every S an independent normalised 8-mode Fourier sum (seeds spawned from
    ``seed``)."""
    nn = (n, n, n) if np.isscalar(n) else tuple(int(v) for v in n)
    box = box_desc(nn, ng, dx=dx, bc_lo=(BC_PERIODIC,) * 3)
    L = [nn[d] * box["dx"][d] for d in range(3)]
    xyz = cell_centres(box)
    ss = seed if isinstance(seed, np.random.SeedSequence) else np.random.SeedSequence(seed)
    kids = ss.spawn(5)
    fields = [_modes(np.random.default_rng(s), nn, L, xyz) for s in kids]
    shp = (nn[2], nn[1], nn[0])
    rho = np.broadcast_to(1.25 + 0.75 * fields[0], shp)
    p = np.broadcast_to(1.25 + 0.75 * fields[1], shp)
    u, v, w = (np.broadcast_to(0.5 * f, shp) for f in fields[2:])
    return from_primitive(box, rho, u, v, w, p), box, params_desc()


def advect(n, kvec=(1, 1, 1), vel=(1.0, 1.0, 1.0), amp=0.1, ng=NG):
    """rho = 1 + amp sin(2 pi k.x), uniform velocity ``vel``, p = 1, periodic.
    The exact solution at time t is the initial density shifted by vel*t."""
    nn = (n, n, n) if np.isscalar(n) else tuple(n)
    box = box_desc(nn, ng, bc_lo=(BC_PERIODIC,) * 3)
    x, y, z = cell_centres(box)
    rho = 1.0 + amp * np.sin(2 * np.pi * (kvec[0] * x + kvec[1] * y + kvec[2] * z))
    return from_primitive(box, rho, vel[0], vel[1], vel[2], 1.0), box, params_desc()


def uniform(n, rho=1.0, vel=(0.3, -0.2, 0.1), p=1.0, bc=BC_PERIODIC, ng=NG):
    nn = (n, n, n) if np.isscalar(n) else tuple(n)
    box = box_desc(nn, ng, bc_lo=(bc,) * 3)
    return from_primitive(box, rho, vel[0], vel[1], vel[2], p), box, params_desc()


def species(U, box, nspec=2, seed=5):
    """Partial densities rho X_s (shape (nspec,) + the state's spatial shape,
    ghosts included) of nspec mass fractions that sum to one: species 0 is
    the gas denser than the box's mean density (a sharp interface wherever
    the flow has one), the others share the rest in proportions set by
    seeded smooth random fields, 1 + 0.5 S_s."""
    ng, n = box["ng"], box["n"]
    rho = U[0]
    X = np.empty((nspec,) + rho.shape)
    heavy = (rho > rho[ng:ng + n[2], ng:ng + n[1], ng:ng + n[0]].mean()).astype(np.float64)
    if nspec == 1:
        X[0] = heavy
    else:
        X[0] = heavy
        full = box_desc(tuple(v + 2 * ng for v in n), 0, dx=box["dx"])
        L = [full["n"][d] * box["dx"][d] for d in range(3)]
        xyz = cell_centres(full)
        kids = np.random.SeedSequence(seed).spawn(nspec - 1)
        w = [np.broadcast_to(1.0 + 0.5 * _modes(np.random.default_rng(k), full["n"], L, xyz),
                             rho.shape) for k in kids]
        tot = sum(w)
        for s in range(1, nspec):
            X[s] = (1.0 - heavy) * (w[s - 1] / tot)
    return np.ascontiguousarray(rho[None] * X)


def sedov(n=64, r0_cells=2.0, p_amb=1e-5, e_blast=1.0, ng=NG):
    """Point blast (Sedov-Taylor) in the unit cube: rho = 1, at rest, pressure
    p_amb, except the cells whose centres lie within r0_cells cell widths of
    the cube's centre, which share the energy e_blast evenly as pressure
    (p = (gamma - 1) e_blast / deposited volume); outflow on all faces."""
    nn = (n, n, n) if np.isscalar(n) else tuple(n)
    box = box_desc(nn, ng, bc_lo=(BC_OUTFLOW,) * 3)
    x, y, z = cell_centres(box)
    shp = (nn[2], nn[1], nn[0])
    r = np.broadcast_to(np.sqrt((x - 0.5) ** 2 + (y - 0.5) ** 2 + (z - 0.5) ** 2), shp)
    dep = r < r0_cells * min(box["dx"])
    vol = dep.sum() * box["dx"][0] * box["dx"][1] * box["dx"][2]
    p = np.where(dep, (GAMMA - 1.0) * e_blast / vol, p_amb)
    return from_primitive(box, 1.0, 0.0, 0.0, 0.0, p), box, params_desc()


# ---------------------------------------------------------------------------
# a domain split into boxes that tile it
# ---------------------------------------------------------------------------

def tile(U, box, cuts):
    """Split the state U of a domain box (or its species array) into boxes
    that tile it: ``cuts[d]``
    lists the cut positions along axis d (first 0, last n_d).  Returns
    (states, boxes, lo, tiling): box states with zero ghost cells, box
    descriptions (the domain's cell widths and ghost depth; their own
    boundary kinds, periodic or outflow for boxes thinner than the ghost
    depth, are not the domain's), each box's lower corner, and the
    arguments of a tiling (dom, bc_lo, bc_hi)."""
    n, ng = box["n"], box["ng"]
    for d in range(3):
        c = list(cuts[d])
        if c[0] != 0 or c[-1] != n[d] or any(b <= a for a, b in zip(c, c[1:])):
            raise ValueError("cuts must increase from 0 to n along every axis")
    V = valid(U, box)
    states, boxes, lo = [], [], []
    for k0, k1 in zip(cuts[2], cuts[2][1:]):
        for j0, j1 in zip(cuts[1], cuts[1][1:]):
            for i0, i1 in zip(cuts[0], cuts[0][1:]):
                nb = (i1 - i0, j1 - j0, k1 - k0)
                bc = tuple(BC_PERIODIC if m >= ng else BC_OUTFLOW for m in nb)
                b = box_desc(nb, ng, dx=box["dx"], bc_lo=bc)
                W = np.zeros((U.shape[0],) + state_shape(b)[1:])  # gas or species
                valid(W, b)[...] = V[:, k0:k1, j0:j1, i0:i1]
                states.append(W)
                boxes.append(b)
                lo.append((i0, j0, k0))
    return states, boxes, lo, {"dom": tuple(n), "bc_lo": box["bc_lo"], "bc_hi": box["bc_hi"]}


def even_cuts(n, bs):
    """Cuts of n cells into boxes of bs cells (the last one shorter if bs does
    not divide n)."""
    return list(range(0, n, bs)) + [n]


def sedov_level(n=256, bs=64, ng=NG):
    """The Sedov blast on an n^3 domain held as (n/bs)^3 boxes of bs^3 cells
    (the paper's per-node Sedov runs use 64^3 boxes, Sec. IV-A).  Returns
    (states, boxes, params, lo, tiling arguments)."""
    U, box, prm = sedov(n, ng=ng)
    c = even_cuts(n, bs)
    states, boxes, lo, til = tile(U, box, (c, c, c))
    return states, boxes, prm, lo, til


# ---------------------------------------------------------------------------
# the batched AMR-like level and the serving stream
# ---------------------------------------------------------------------------

def level_shapes(nboxes=512, seed=2, sides=(16, 32, 64)):
    """Box shapes of the batched level: each side drawn from ``sides``."""
    rng = np.random.default_rng(seed)
    return [tuple(int(v) for v in rng.choice(sides, size=3)) for _ in range(nboxes)]


def level(nboxes=512, seed=2, dx=1.0 / 64, sides=(16, 32, 64), ng=NG):
    """The batched level: ``nboxes`` independent periodic boxes with smooth
    random fields, all with cell width ``dx``.  Returns (states, boxes, params)."""
    shapes = level_shapes(nboxes, seed, sides)
    kids = np.random.SeedSequence(seed).spawn(nboxes)
    states, boxes = [], []
    for shp, kid in zip(shapes, kids):
        U, box, prm = smooth(shp, kid, dx=(dx, dx, dx), ng=ng)
        states.append(U)
        boxes.append(box)
    return states, boxes, params_desc()


FAMILIES = ("sod", "kh", "smooth")


def request_stream(count, rate, seed=3, nmin=32, nmax=192, smin=10, smax=200):
    """Serving requests: Poisson arrival times of the given rate (per second),
    cubic side log-uniform in [nmin, nmax] rounded to an integer, step count
    uniform in [smin, smax], initial-condition family uniform over FAMILIES,
    and a per-request seed.  Returns a list of dicts (no state arrays)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for r in range(count):
        t += rng.exponential(1.0 / rate) if rate > 0 else 0.0
        n = int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))
        steps = int(rng.integers(smin, smax + 1))
        fam = FAMILIES[int(rng.integers(0, len(FAMILIES)))]
        out.append({"id": r, "arrival": t, "n": n, "steps": steps, "family": fam,
                    "seed": int(rng.integers(0, 2**31 - 1))})
    return out


def request_state(req, ng=NG):
    """Initial state, box and params of one serving request."""
    fam, n, seed = req["family"], req["n"], req["seed"]
    if fam == "sod":
        return sod(n, axis=seed % 3, ng=ng)
    if fam == "kh":
        return kh(n, seed=seed, ng=ng)
    if fam == "smooth":
        return smooth(n, seed, ng=ng)
    raise ValueError(fam)
