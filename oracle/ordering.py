"""Oracle: reverse Cuthill-McKee renumbering and the CSR sparsity pattern.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper does not say how its sparse matrices are stored (Sec. 3.2.2 only
states they are sparse and symmetric).  The library stores them in CSR with
rows in reverse Cuthill-McKee order; because the CPU oracle and the GPU
library are written independently, the order is pinned down completely:

  graph      vertices are the cells in their input order, edges are interior
             sides; deg(v) is the number of interior sides of v
  components processed in increasing order of their smallest cell index
  start      George-Liu pseudo-peripheral node: r = the minimum-degree vertex
             of the component (ties: smaller index); repeat { BFS from r;
             x = minimum-degree vertex of the last level (ties: smaller index);
             if ecc(x) > ecc(r) then r = x else stop }
  CM sweep   breadth-first from r; the unvisited neighbours of the vertex
             being expanded are appended sorted by (degree, index)
  reverse    the concatenated list of all components is reversed as a whole;
             perm[new] = old
  CSR        row i = new index i; the diagonal is included; columns ascending;
             32-bit indices
"""
from __future__ import annotations

import numpy as np


def _adjacency(nbr: np.ndarray):
    nbr = np.asarray(nbr, np.int64)
    adj = [[int(u) for u in row if u >= 0] for row in nbr.tolist()]
    deg = [len(a) for a in adj]
    return adj, deg


def _levels(adj, root):
    """BFS level structure from root (list of lists)."""
    seen = {root}
    cur = [root]
    levels = []
    while cur:
        levels.append(cur)
        nxt = []
        for v in cur:
            for u in adj[v]:
                if u not in seen:
                    seen.add(u)
                    nxt.append(u)
        cur = nxt
    return levels


def _min_deg(vertices, deg):
    best = None
    for v in vertices:
        if best is None or deg[v] < deg[best] or (deg[v] == deg[best] and v < best):
            best = v
    return best


def rcm(nbr: np.ndarray) -> np.ndarray:
    """Reverse Cuthill-McKee permutation, perm[new] = old (int32)."""
    adj, deg = _adjacency(nbr)
    n = len(adj)
    visited = [False] * n
    order = []
    for s in range(n):
        if visited[s]:
            continue
        comp = [v for lev in _levels(adj, s) for v in lev]
        r = _min_deg(comp, deg)
        lev_r = _levels(adj, r)
        while True:
            x = _min_deg(lev_r[-1], deg)
            lev_x = _levels(adj, x)
            if len(lev_x) > len(lev_r):
                r, lev_r = x, lev_x
            else:
                break
        visited[r] = True
        queue = [r]
        head = 0
        while head < len(queue):
            v = queue[head]
            head += 1
            cand = [u for u in adj[v] if not visited[u]]
            cand.sort(key=lambda u: (deg[u], u))
            for u in cand:
                visited[u] = True
                queue.append(u)
        order.extend(queue)
    order.reverse()
    return np.asarray(order, np.int32)


def csr_pattern(nbr: np.ndarray, perm: np.ndarray):
    """CSR row pointers and ascending column indices in the permuted order."""
    nbr = np.asarray(nbr, np.int64)
    perm = np.asarray(perm, np.int64)
    n = nbr.shape[0]
    inv = np.empty(n, np.int64)
    inv[perm] = np.arange(n)
    row_ptr = np.zeros(n + 1, np.int64)
    cols = []
    for i in range(n):
        c = [i] + [int(inv[u]) for u in nbr[perm[i]] if u >= 0]
        c.sort()
        cols.append(c)
        row_ptr[i + 1] = row_ptr[i] + len(c)
    col = np.fromiter((c for row in cols for c in row), np.int64, count=int(row_ptr[-1]))
    return row_ptr.astype(np.int32), col.astype(np.int32)


def bandwidth(row_ptr: np.ndarray, col: np.ndarray) -> int:
    rows = np.repeat(np.arange(len(row_ptr) - 1), np.diff(row_ptr))
    return int(np.max(np.abs(col.astype(np.int64) - rows))) if col.size else 0
