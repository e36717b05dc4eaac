"""Oracle: mesh validation, per-cell geometry and side pairing.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Paper passages followed
  * Appendix A (RT0 basis): side j of triangle e is opposite node j; the
    outward unit normal of side j is n_j.
  * Sec. 3.2.2, eq. cs1_discr: the normal derivative across side j is
    approximated by the two-point difference (u_e - u_ep) / d_{e,ep} with
    d_{e,ep} the signed distance between the circumcenters of e and ep,
    positive when the pair is Delaunay.
  * Sec. 3.1: the mesh satisfies the (extended) Delaunay property, which is
    what makes the corrector matrices M-matrices.

Canonical transmissibility (a reading stated in the design notes): the
segment joining the circumcenters of two triangles that share a side is the
perpendicular bisector of that side, so d_{e,ep} = (l/2)(cot t_e + cot t_ep)
with t the angle opposite the shared side, and T = l/d = 2/(cot t_e + cot t_ep).
For a boundary side the circumcenter-to-midpoint distance is (l/2) cot t,
so T_b = 2/cot t.  cot t is evaluated as dot(u, v)/cross(u, v) with u, v
the edge vectors leaving the vertex.  The circumcenter form is computed too
and serves as a self-check.
"""
from __future__ import annotations

import numpy as np

# status codes shared in meaning (not in code) with the library
OK = 0
INVALID_ARG = -1
BAD_MESH = -2
NOT_DELAUNAY = -3
SINGULAR = -4
NONFINITE = -5


class MeshError(Exception):
    def __init__(self, status: int, msg: str):
        super().__init__(msg)
        self.status = status


def cell_geometry(xy: np.ndarray, tri: np.ndarray) -> dict:
    """Area, cotangents of the three angles and side vectors of every cell.

    cot[e, j]  cotangent of the angle at node j (opposite side j)
    t[e, j]    side-j vector, from node j+1 to node j+2 (CCW traversal)
    area[e]    half the cross product at node 0
    """
    xy = np.asarray(xy, np.float64)
    tri = np.asarray(tri, np.int64)
    P = xy[tri]  # [n, 3, 2]
    n = tri.shape[0]
    cot = np.empty((n, 3))
    cross = np.empty((n, 3))
    t = np.empty((n, 3, 2))
    for j in range(3):
        a = P[:, j]
        b = P[:, (j + 1) % 3]
        c = P[:, (j + 2) % 3]
        ux, uy = b[:, 0] - a[:, 0], b[:, 1] - a[:, 1]
        vx, vy = c[:, 0] - a[:, 0], c[:, 1] - a[:, 1]
        dot = ux * vx + uy * vy
        cr = ux * vy - uy * vx
        cross[:, j] = cr
        with np.errstate(divide="ignore", invalid="ignore"):
            cot[:, j] = dot / cr
        t[:, j, 0] = c[:, 0] - b[:, 0]
        t[:, j, 1] = c[:, 1] - b[:, 1]
    area = 0.5 * cross[:, 0]
    return {"cot": cot, "cross": cross, "t": t, "area": area}


def pair_sides(tri: np.ndarray, n_nodes: int) -> dict:
    """Pair every side (e, j) with the side (ep, jp) holding the same two nodes.

    Returns nbr[e, j] (ep or -1 on the boundary) and nbr_side[e, j] (jp or -1).
    Raises MeshError(BAD_MESH) when a side is shared by more than two cells or
    by two cells that traverse it in the same direction.
    """
    tri = np.asarray(tri, np.int64)
    n = tri.shape[0]
    a = np.stack([tri[:, (j + 1) % 3] for j in range(3)], axis=1).ravel()
    b = np.stack([tri[:, (j + 2) % 3] for j in range(3)], axis=1).ravel()
    lo = np.minimum(a, b)
    hi = np.maximum(a, b)
    key = lo * np.int64(n_nodes) + hi
    order = np.argsort(key, kind="stable")
    ks = key[order]
    nbr = np.full(3 * n, -1, np.int64)
    # runs of equal keys
    start = np.flatnonzero(np.r_[True, ks[1:] != ks[:-1]])
    length = np.diff(np.r_[start, ks.size])
    if np.any(length > 2):
        raise MeshError(BAD_MESH, "a side is shared by more than two triangles")
    pairs = start[length == 2]
    s0 = order[pairs]
    s1 = order[pairs + 1]
    if np.any(a[s0] == a[s1]):
        raise MeshError(BAD_MESH, "two triangles traverse a shared side in the same direction")
    nbr[s0] = s1
    nbr[s1] = s0
    nbr = nbr.reshape(n, 3)
    cell = np.where(nbr >= 0, nbr // 3, -1)
    side = np.where(nbr >= 0, nbr % 3, -1)
    return {"nbr": cell, "nbr_side": side}


def build(xy: np.ndarray, tri: np.ndarray, side_tag: np.ndarray) -> dict:
    """Validate the mesh and compute everything the assembly needs.

    side_tag[e, j] is a bit mask for boundary sides: bit 0 = Dirichlet side of
    CP1, bit 1 = Dirichlet side of CP2; other boundary sides are Neumann.
    Tags on interior sides are ignored.
    """
    xy = np.asarray(xy, np.float64)
    tri = np.asarray(tri, np.int64)
    side_tag = np.asarray(side_tag, np.int64).reshape(tri.shape)
    n_nodes = xy.shape[0]
    if tri.ndim != 2 or tri.shape[1] != 3 or tri.shape[0] == 0 or n_nodes == 0:
        raise MeshError(INVALID_ARG, "empty mesh or bad shapes")
    if tri.min() < 0 or tri.max() >= n_nodes:
        raise MeshError(INVALID_ARG, "node index out of range")
    if np.any(side_tag < 0) or np.any(side_tag > 3):
        raise MeshError(INVALID_ARG, "side tag outside 0..3")
    if not np.all(np.isfinite(xy)):
        raise MeshError(NONFINITE, "non-finite node coordinates")
    if np.any((tri[:, 0] == tri[:, 1]) | (tri[:, 1] == tri[:, 2]) | (tri[:, 0] == tri[:, 2])):
        raise MeshError(BAD_MESH, "repeated node in a triangle")
    g = cell_geometry(xy, tri)
    if np.any(~(g["cross"] > 0)):
        raise MeshError(BAD_MESH, "triangle with non-positive area (clockwise or degenerate)")
    p = pair_sides(tri, n_nodes)
    nbr = p["nbr"]
    interior = nbr >= 0
    e_idx = np.repeat(np.arange(tri.shape[0])[:, None], 3, axis=1)
    cot = g["cot"]
    # interior faces: T_f = 2 / (cot_e + cot_ep)
    cot_sum = np.where(interior, cot + cot[np.maximum(nbr, 0), np.maximum(p["nbr_side"], 0)], np.nan)
    if np.any(interior & ~(cot_sum > 0)):
        raise MeshError(NOT_DELAUNAY, "interior side with non-positive circumcenter distance")
    tag = np.where(interior, 0, side_tag)
    dirichlet_any = (~interior) & (tag != 0)
    if np.any(dirichlet_any & ~(cot > 0)):
        raise MeshError(NOT_DELAUNAY, "Dirichlet side with non-positive circumcenter-to-side distance")
    T = np.where(interior, 2.0 / np.where(interior, cot_sum, 1.0), np.where(cot > 0, 2.0 / np.where(cot > 0, cot, 1.0), 0.0))
    return {
        "n": tri.shape[0],
        "xy": xy,
        "tri": tri,
        "area": g["area"],
        "cot": cot,
        "t": g["t"],
        "nbr": nbr,
        "nbr_side": p["nbr_side"],
        "interior": interior,
        "tag": tag,
        "T": T,  # per (cell, side): T_f for interior sides, T_b for boundary sides (0 if cot<=0)
        "cell": e_idx,
    }


def circumcenters(xy: np.ndarray, tri: np.ndarray) -> np.ndarray:
    """Circumcenter of every triangle (textbook closed form)."""
    P = np.asarray(xy, np.float64)[np.asarray(tri, np.int64)]
    ax, ay = P[:, 0, 0], P[:, 0, 1]
    bx, by = P[:, 1, 0] - ax, P[:, 1, 1] - ay
    cx, cy = P[:, 2, 0] - ax, P[:, 2, 1] - ay
    d = 2.0 * (bx * cy - by * cx)
    b2 = bx * bx + by * by
    c2 = cx * cx + cy * cy
    ux = (cy * b2 - by * c2) / d
    uy = (bx * c2 - cx * b2) / d
    return np.stack([ax + ux, ay + uy], axis=1)


def circumcenter_distances(geo: dict) -> dict:
    """Signed distances the paper defines (Sec. 3.2.2): d_{e,ep} for interior
    sides, circumcenter-to-midpoint distance for boundary sides, both measured
    along the outward normal of side j of e.  Used to cross-check T = l/d."""
    xy, tri = geo["xy"], geo["tri"]
    cc = circumcenters(xy, tri)
    t = geo["t"]
    l = np.sqrt(t[..., 0] ** 2 + t[..., 1] ** 2)
    nx, ny = t[..., 1] / l, -t[..., 0] / l
    nbr = geo["nbr"]
    other = cc[np.maximum(nbr, 0)]
    d_int = (other[..., 0] - cc[:, None, 0]) * nx + (other[..., 1] - cc[:, None, 1]) * ny
    P = xy[tri]
    mid = np.stack([0.5 * (P[:, (j + 1) % 3] + P[:, (j + 2) % 3]) for j in range(3)], axis=1)
    d_b = (mid[..., 0] - cc[:, None, 0]) * nx + (mid[..., 1] - cc[:, None, 1]) * ny
    d = np.where(geo["interior"], d_int, d_b)
    return {"d": d, "l": l}
