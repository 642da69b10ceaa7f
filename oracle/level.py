"""Oracle of the ghost exchange between the boxes of a level that tile one
domain (test infrastructure only: imported by the tests, never by the product
path).

Definition (Sec. II: a level's boxes cover the problem domain and each box's
stencil reads neighbour data from the boxes next to it): assemble the
domain's valid cells from the boxes, extend the domain by its ghost layers
axis by axis under its boundary kinds -- periodic wraps, outflow repeats the
edge cell, reflect mirrors and negates the normal momentum -- and give every
box the part of that extended domain its own ghosted array covers.  Written
with whole-array numpy copies (np.pad), so it shares nothing with the GPU
kernel's per-cell owner lookup.
"""
import numpy as np

BC_PERIODIC, BC_OUTFLOW, BC_REFLECT = 0, 1, 2
_MODE = {BC_PERIODIC: "wrap", BC_OUTFLOW: "edge", BC_REFLECT: "symmetric"}


def _valid(U, box):
    g = box["ng"]
    n0, n1, n2 = box["n"]
    return U[:, g:g + n2, g:g + n1, g:g + n0]


def assemble(states, boxes, lo, dom):
    """The domain's valid cells, shape (5, D2, D1, D0), from the boxes;
    raises if the boxes do not tile the domain exactly."""
    D = np.full((5, dom[2], dom[1], dom[0]), np.nan)
    hit = np.zeros((dom[2], dom[1], dom[0]), dtype=np.int64)
    for U, b, l in zip(states, boxes, lo):
        n0, n1, n2 = b["n"]
        sl = (slice(l[2], l[2] + n2), slice(l[1], l[1] + n1), slice(l[0], l[0] + n0))
        D[(slice(None),) + sl] = _valid(U, b)
        hit[sl] += 1
    if not np.all(hit == 1):
        raise ValueError("the boxes do not tile the domain")
    return D


def extend(D, ng, bc_lo, bc_hi):
    """The domain extended by ng ghost layers on every side: axis by axis
    (x, y, z), each side by its own boundary kind."""
    P = D
    for d in range(3):
        ax = 3 - d  # array axis of domain axis d
        if bc_lo[d] == BC_PERIODIC:  # (paired with a periodic high side)
            width = [(0, 0)] * 4
            width[ax] = (ng, ng)
            P = np.pad(P, width, mode="wrap")
            continue
        # one side at a time: each copies from its own end of the axis
        for side, bc in ((0, bc_lo[d]), (1, bc_hi[d])):
            width = [(0, 0)] * 4
            width[ax] = (ng, 0) if side == 0 else (0, ng)
            P = np.pad(P, width, mode=_MODE[bc])
            if bc == BC_REFLECT:
                sl = [slice(None)] * 4
                sl[0] = 1 + d
                sl[ax] = slice(0, ng) if side == 0 else slice(P.shape[ax] - ng, None)
                P[tuple(sl)] *= -1.0
    return P


def fill_ghosts_level(states, boxes, lo, dom, bc_lo, bc_hi):
    """New list of box states whose ghost cells hold the level's values (valid
    cells unchanged)."""
    ng = max(b["ng"] for b in boxes)
    P = extend(assemble(states, boxes, lo, dom), ng, bc_lo, bc_hi)
    out = []
    for U, b, l in zip(states, boxes, lo):
        g = b["ng"]
        n0, n1, n2 = b["n"]
        o = [l[d] + ng - g for d in range(3)]
        V = P[:, o[2]:o[2] + n2 + 2 * g, o[1]:o[1] + n1 + 2 * g, o[0]:o[0] + n0 + 2 * g]
        out.append(np.ascontiguousarray(V))
    return out
