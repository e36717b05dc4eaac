"""Seeded synthetic Delaunay triangle meshes shaped like the paper's test cases.

These generators only place points and triangulate them (scipy's Qhull
Delaunay); they hold none of the corrector method's arithmetic.  Both the
CPU oracle and the GPU library consume their output unchanged.

Conventions (Appendix A of the paper): triangle ``e`` has nodes 0,1,2 in
counter-clockwise order and side ``j`` is the side opposite node ``j``,
i.e. the segment from node ``j+1`` to node ``j+2`` (indices mod 3).

Every mesh is returned as a dict with
  xy    float64 [N, 2]  node coordinates
  tri   int32   [n, 3]  CCW node indices
  group int8    [n, 3]  boundary group of side j (0 = not on a boundary
                        line; other values are workload specific)
"""
from __future__ import annotations

import math

import numpy as np
from scipy.spatial import Delaunay

# boundary groups of rectangular domains
G_NONE, G_LEFT, G_RIGHT, G_BOTTOM, G_TOP = 0, 1, 2, 3, 4


def _triangulate(pts: np.ndarray, with_neighbors: bool = False):
    """Delaunay triangulation with CCW orientation; refuses coplanar points.
    With with_neighbors, also returns nbr[e, j]: the triangle across the side
    opposite node j (-1 on the hull)."""
    d = Delaunay(pts)
    if len(d.coplanar):
        raise RuntimeError(f"Qhull dropped {len(d.coplanar)} coplanar points")
    tri = d.simplices.astype(np.int64)
    nbr = d.neighbors.astype(np.int64)
    p = pts[tri]
    s = (p[:, 1, 0] - p[:, 0, 0]) * (p[:, 2, 1] - p[:, 0, 1]) - (
        p[:, 1, 1] - p[:, 0, 1]
    ) * (p[:, 2, 0] - p[:, 0, 0])
    cw = s < 0
    tri[cw, 1], tri[cw, 2] = tri[cw, 2].copy(), tri[cw, 1].copy()
    nbr[cw, 1], nbr[cw, 2] = nbr[cw, 2].copy(), nbr[cw, 1].copy()
    tri = np.ascontiguousarray(tri.astype(np.int32))
    return (tri, nbr) if with_neighbors else tri


def _split_encroached(pts, x0, x1, y0, y1, margin=0.1, max_rounds=20):
    """Triangulate; while some node sees a rectangle-boundary side under an
    angle wider than arccot(margin) (the node encroaches the side's diametral
    circle), add the side's midpoint as a boundary node and re-triangulate."""
    for _ in range(max_rounds):
        tri, nbr = _triangulate(pts, with_neighbors=True)
        P = pts[tri]
        add = []
        for j in range(3):
            a = P[:, (j + 1) % 3]
            b = P[:, (j + 2) % 3]
            c = P[:, j]
            on = (((a[:, 0] == x0) & (b[:, 0] == x0)) | ((a[:, 0] == x1) & (b[:, 0] == x1))
                  | ((a[:, 1] == y0) & (b[:, 1] == y0)) | ((a[:, 1] == y1) & (b[:, 1] == y1)))
            ux, uy = a[:, 0] - c[:, 0], a[:, 1] - c[:, 1]
            vx, vy = b[:, 0] - c[:, 0], b[:, 1] - c[:, 1]
            dot = ux * vx + uy * vy
            cr = np.abs(ux * vy - uy * vx)
            bad = on & (dot <= margin * cr)
            if np.any(bad):
                mid = 0.5 * (a[bad] + b[bad])
                # keep the midpoint exactly on the boundary line
                mid[a[bad, 0] == b[bad, 0], 0] = a[bad][a[bad, 0] == b[bad, 0], 0]
                mid[a[bad, 1] == b[bad, 1], 1] = a[bad][a[bad, 1] == b[bad, 1], 1]
                add.append(mid)
        if not add:
            return pts, tri
        pts = np.concatenate([pts] + add)
        pts = np.unique(pts, axis=0)
    raise RuntimeError("boundary refinement did not terminate")


def _side_quality(pts, tri, nbr):
    """Cot sum of the two angles facing every interior side (Delaunay: > 0;
    small values mean nearly cocircular quadrilaterals) and the four nodes of
    the quadrilateral around that side."""
    P = pts[tri]
    cot = np.empty((tri.shape[0], 3))
    for j in range(3):
        a, b, c = P[:, j], P[:, (j + 1) % 3], P[:, (j + 2) % 3]
        ux, uy = b[:, 0] - a[:, 0], b[:, 1] - a[:, 1]
        vx, vy = c[:, 0] - a[:, 0], c[:, 1] - a[:, 1]
        cot[:, j] = (ux * vx + uy * vy) / (ux * vy - uy * vx)
    e, j = np.nonzero(nbr >= 0)
    keep = e < nbr[e, j]  # each interior side once
    e, j = e[keep], j[keep]
    ep = nbr[e, j]
    jp = np.argmax(nbr[ep] == e[:, None], axis=1)
    cs = cot[e, j] + cot[ep, jp]
    quad = np.stack([tri[e, j], tri[e, (j + 1) % 3], tri[e, (j + 2) % 3], tri[ep, jp]], 1)
    return cs, quad


def _untangle_cocircular(pts, movable, hl, x0, x1, y0, y1, seed, min_cot_sum=0.02, max_rounds=40):
    """Mesh quality pass: each round triangulates once, splits encroached
    boundary sides (as _split_encroached) and, for every interior side whose
    facing angles are nearly supplementary (cot sum < min_cot_sum, i.e.
    T = l/d > 2/min_cot_sum), deletes one movable node of its quadrilateral
    (the one on the finest local spacing, then the lowest index), until
    neither is left.  Deleting a node changes the local triangulation
    decisively, so a few rounds suffice."""
    for _ in range(max_rounds):
        tri, nbr = _triangulate(pts, with_neighbors=True)
        P = pts[tri]
        add = []
        for j in range(3):
            a, b, c = P[:, (j + 1) % 3], P[:, (j + 2) % 3], P[:, j]
            on = (((a[:, 0] == x0) & (b[:, 0] == x0)) | ((a[:, 0] == x1) & (b[:, 0] == x1))
                  | ((a[:, 1] == y0) & (b[:, 1] == y0)) | ((a[:, 1] == y1) & (b[:, 1] == y1)))
            ux, uy = a[:, 0] - c[:, 0], a[:, 1] - c[:, 1]
            vx, vy = b[:, 0] - c[:, 0], b[:, 1] - c[:, 1]
            bad = on & (ux * vx + uy * vy <= 0.1 * np.abs(ux * vy - uy * vx))
            if np.any(bad):
                mid = 0.5 * (a[bad] + b[bad])
                vert = a[bad, 0] == b[bad, 0]
                mid[vert, 0] = a[bad][vert, 0]
                mid[~vert, 1] = a[bad][~vert, 1]
                add.append(mid)
        cs, quad = _side_quality(pts, tri, nbr)
        drop = set()
        for qd in quad[cs < min_cot_sum].tolist():
            cand = [v for v in qd if movable[v]]
            if cand and not drop.intersection(qd):
                drop.add(min(cand, key=lambda v: (hl[v], v)))
        if not add and not drop:
            return pts, tri
        keep = np.ones(len(pts), bool)
        keep[list(drop)] = False
        pts, movable, hl = pts[keep], movable[keep], hl[keep]
        if add:
            mid = np.concatenate(add)
            pts = np.concatenate([pts, mid])
            movable = np.concatenate([movable, np.zeros(len(mid), bool)])
            hl = np.concatenate([hl, np.full(len(mid), hl.min())])
            _, first = np.unique(pts, axis=0, return_index=True)
            first = np.sort(first)
            pts, movable, hl = pts[first], movable[first], hl[first]
    raise RuntimeError("mesh quality pass did not converge")


def _rect_groups(xy, tri, x0, x1, y0, y1) -> np.ndarray:
    """Group of each side that lies on a side of the rectangle (exact coords)."""
    n = tri.shape[0]
    group = np.zeros((n, 3), np.int8)
    for j in range(3):
        a = xy[tri[:, (j + 1) % 3]]
        b = xy[tri[:, (j + 2) % 3]]
        group[(a[:, 0] == x0) & (b[:, 0] == x0), j] = G_LEFT
        group[(a[:, 0] == x1) & (b[:, 0] == x1), j] = G_RIGHT
        group[(a[:, 1] == y0) & (b[:, 1] == y0), j] = G_BOTTOM
        group[(a[:, 1] == y1) & (b[:, 1] == y1), j] = G_TOP
    return group


def square_jittered_grid(npts: int = 64, jitter: float = 0.3, seed: int = 1) -> dict:
    """Unit square, npts x npts grid, interior nodes jittered by U[-jitter*h, jitter*h]
    per coordinate (boundary nodes fixed), Delaunay triangulated."""
    h = 1.0 / (npts - 1)
    g = np.linspace(0.0, 1.0, npts)
    X, Y = np.meshgrid(g, g, indexing="xy")
    X = X.ravel().copy()
    Y = Y.ravel().copy()
    interior = (X > 0) & (X < 1) & (Y > 0) & (Y < 1)
    rng = np.random.default_rng(seed)
    m = int(interior.sum())
    X[interior] += rng.uniform(-jitter * h, jitter * h, m)
    Y[interior] += rng.uniform(-jitter * h, jitter * h, m)
    xy = np.stack([X, Y], axis=1)
    tri = _triangulate(xy)
    return {"xy": xy, "tri": tri, "group": _rect_groups(xy, tri, 0.0, 1.0, 0.0, 1.0)}


def _dist_to_segments(px, py, segs):
    d = np.full(px.shape, np.inf)
    for (ax, ay, bx, by) in segs:
        vx, vy = bx - ax, by - ay
        t = ((px - ax) * vx + (py - ay) * vy) / (vx * vx + vy * vy)
        t = np.clip(t, 0.0, 1.0)
        dx = px - (ax + t * vx)
        dy = py - (ay + t * vy)
        d = np.minimum(d, np.sqrt(dx * dx + dy * dy))
    return d


def graded_lattice(
    n_rows: int,
    L: float,
    H: float,
    seed: int,
    jitter: float = 0.15,
    level_of=None,
    max_level: int = 0,
    quality: bool = True,
) -> dict:
    """Jittered triangular lattice on [0,L]x[0,H] with nested local refinement.

    The finest lattice has 2**max_level * n_rows rows; a point of the finest
    lattice is kept if it belongs to the (nested) lattice of the refinement
    level that ``level_of(x, y)`` assigns to its location, so points of
    different levels never come closer than the finest spacing.  Column spacing
    is stretched slightly so both x=0 and x=L fall on lattice columns; boundary
    rows at y=0 and y=H are lattice rows.  Boundary nodes are not jittered and
    neither are nodes within one local spacing of the boundary, so boundary
    triangles stay acute at the node opposite the boundary side.  With
    `quality`, nodes of nearly cocircular quadrilaterals (which the level
    transitions create) are removed until every interior side has a cot sum
    >= 0.02, i.e. a transmissibility l/d <= 100, as a quality mesh generator
    would guarantee.
    """
    f = 2 ** max_level
    rows_f = n_rows * f
    sy_f = H / rows_f
    n_cols0 = max(2, int(round(L * math.sqrt(3.0) * n_rows / (2.0 * H))))
    cols_f = n_cols0 * f
    hx_f = L / cols_f

    J = np.arange(rows_f + 1)
    I = np.arange(cols_f + 1)
    JJ, II = np.meshgrid(J, I, indexing="ij")
    JJ = JJ.ravel()
    II = II.ravel()
    x = II * hx_f + (JJ % 2) * (hx_f / 2)
    y = JJ * sy_f
    # boundary rows/columns land exactly on the domain edges
    x[(II == cols_f) & (JJ % 2 == 0)] = L
    y[JJ == rows_f] = H
    inside = x <= L
    JJ, II, x, y = JJ[inside], II[inside], x[inside], y[inside]

    lev = np.zeros(x.shape, np.int64) if level_of is None else level_of(x, y).astype(np.int64)
    lev = np.minimum(lev, max_level)
    keep = np.zeros(x.shape, bool)
    for l in range(max_level + 1):
        s = 2 ** (max_level - l)  # finest rows per level-l row
        jl = JJ // s
        on_row = (JJ % s) == 0
        # level-l point: I*hx_f == i*hx_l + (jl%2)*hx_l/2 with hx_l = s*hx_f,
        # and the finest lattice's own odd-row offset must vanish (J even unless s==1)
        if s == 1:
            on_col = np.ones(x.shape, bool)
        else:
            on_col = ((II - (jl % 2) * (s // 2)) % s) == 0
        keep |= (lev == l) & on_row & on_col
    px, py, plev, pJ = x[keep], y[keep], lev[keep], JJ[keep]

    # left/right boundary nodes on rows whose level lattice has no node there
    extra = []
    for xb in (0.0, L):
        for l in range(max_level + 1):
            s = 2 ** (max_level - l)
            rows = np.arange(0, rows_f + 1, s)
            yb = rows * sy_f
            yb[rows == rows_f] = H
            lb = np.minimum(
                (np.zeros(yb.shape, np.int64) if level_of is None else level_of(np.full(yb.shape, xb), yb).astype(np.int64)),
                max_level,
            )
            yb = yb[lb == l]
            extra.append(np.stack([np.full(yb.shape, xb), yb], axis=1))
    extra = np.concatenate(extra)
    pts = np.concatenate([np.stack([px, py], axis=1), extra])
    lev_all = np.concatenate([plev, np.zeros(len(extra), np.int64)])
    # drop duplicates (boundary rows that already had a lattice node at x=0 / x=L)
    _, idx = np.unique(np.round(pts / (hx_f * 1e-3)).astype(np.int64), axis=0, return_index=True)
    idx = np.sort(idx)
    pts = pts[idx]
    lev_all = lev_all[idx]
    # lattice nodes too close to x=0 / x=L (closer than a quarter of the local spacing)
    hl = hx_f * (2.0 ** (max_level - lev_all))
    on_b = (pts[:, 0] == 0.0) | (pts[:, 0] == L)
    ok = on_b | ((pts[:, 0] >= 0.25 * hl) & (pts[:, 0] <= L - 0.25 * hl))
    pts, lev_all, hl = pts[ok], lev_all[ok], hl[ok]

    rng = np.random.default_rng(seed)
    near_b = (
        (pts[:, 0] < 1.01 * hl) | (pts[:, 0] > L - 1.01 * hl)
        | (pts[:, 1] < 1.01 * hl) | (pts[:, 1] > H - 1.01 * hl)
    )
    jit = ~near_b
    m = int(jit.sum())
    pts = pts.copy()
    pts[jit, 0] += rng.uniform(-jitter, jitter, m) * hl[jit]
    pts[jit, 1] += rng.uniform(-jitter, jitter, m) * hl[jit]
    if quality:
        on_line = (pts[:, 0] == 0.0) | (pts[:, 0] == L) | (pts[:, 1] == 0.0) | (pts[:, 1] == H)
        pts, tri = _untangle_cocircular(pts, ~on_line, hl, 0.0, L, 0.0, H, seed)
    else:
        pts, tri = _split_encroached(pts, 0.0, L, 0.0, H)
    return {"xy": pts, "tri": tri, "group": _rect_groups(pts, tri, 0.0, L, 0.0, H)}


BLOCK = (1.5, 2.5, 0.5)  # porous block [1.5,2.5] x [0,0.5] on the channel floor


def block_interface_distance(x, y, block=BLOCK):
    """Distance to the exposed sides (left, top, right) of the porous block."""
    x0, x1, yt = block
    segs = [(x0, 0.0, x0, yt), (x0, yt, x1, yt), (x1, yt, x1, 0.0)]
    return _dist_to_segments(np.asarray(x, float), np.asarray(y, float), segs)


def channel_mesh(n_rows: int, seed: int, jitter: float = 0.15, bands=(0.05, 0.10)) -> dict:
    """4x1 channel with a porous block on its floor; spacing h outside, h/2 in the
    band bands[0]..bands[1] from the block's exposed sides, h/4 within bands[0]."""
    b2, b1 = bands

    def level_of(x, y):
        d = block_interface_distance(x, y)
        return np.where(d < b2, 2, np.where(d < b1, 1, 0))

    return graded_lattice(n_rows, 4.0, 1.0, seed, jitter=jitter, level_of=level_of, max_level=2)


def unit_square_lattice(target_cells: int, seed: int, jitter: float = 0.15) -> dict:
    """Jittered triangular lattice on the unit square with about target_cells triangles."""
    # r rows of spacing sqrt(3)/2 h on the unit square give h = 2 / (sqrt(3) r),
    # about 1/h points per row and two triangles per point: sqrt(3) r^2 triangles
    n_rows = max(2, int(round(math.sqrt(target_cells / math.sqrt(3.0)))))
    return graded_lattice(n_rows, 1.0, 1.0, seed, jitter=jitter)


def centroids(mesh: dict) -> np.ndarray:
    p = mesh["xy"][mesh["tri"]]
    return p.mean(axis=1)
