"""Pins for the oracle's reverse Cuthill-McKee order and CSR pattern."""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import reverse_cuthill_mckee

from conftest import load_rcm_graphs
from oracle import geometry, ordering
from synth import meshes


@pytest.mark.parametrize("name", ["g_two_components", "g_branch", "g_lollipop"])
def test_rcm_hand_derived_orders(name):
    nbr, perm = load_rcm_graphs()[name]
    assert np.array_equal(ordering.rcm(nbr), perm)


def _mesh_geo(m):
    return geometry.build(m["xy"], m["tri"], np.zeros(m["tri"].shape, np.int8))


def test_rcm_is_a_permutation_with_small_bandwidth():
    m = meshes.square_jittered_grid(40, 0.3, 3)
    geo = _mesh_geo(m)
    perm = ordering.rcm(geo["nbr"])
    n = geo["n"]
    assert np.array_equal(np.sort(perm), np.arange(n))
    row_ptr, col = ordering.csr_pattern(geo["nbr"], perm)
    bw = ordering.bandwidth(row_ptr, col)
    e, j = np.nonzero(geo["interior"])
    G = sp.csr_matrix((np.ones(len(e)), (e, geo["nbr"][e, j])), shape=(n, n))
    p2 = reverse_cuthill_mckee(G, symmetric_mode=True)
    inv2 = np.empty(n, np.int64)
    inv2[p2] = np.arange(n)
    bw2 = int(np.max(np.abs(inv2[e] - inv2[geo["nbr"][e, j]])))
    assert bw <= 2 * bw2
    assert bw < n // 4


def test_csr_pattern_canonical_form():
    m = meshes.channel_mesh(10, 2)
    geo = _mesh_geo(m)
    perm = ordering.rcm(geo["nbr"])
    row_ptr, col = ordering.csr_pattern(geo["nbr"], perm)
    n = geo["n"]
    assert row_ptr.dtype == np.int32 and col.dtype == np.int32
    assert row_ptr[0] == 0 and np.all(np.diff(row_ptr) >= 1) and np.all(np.diff(row_ptr) <= 4)
    nb = int((~geo["interior"]).sum())
    assert row_ptr[-1] == 4 * n - nb  # nnz = n + 2 * interior sides
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    for i in range(n):
        c = col[row_ptr[i]: row_ptr[i + 1]]
        assert np.all(np.diff(c) > 0) and i in c
    S = sp.csr_matrix((np.ones(col.size), (rows, col)), shape=(n, n))
    assert (S != S.T).nnz == 0
    # pattern is the permuted adjacency
    inv = np.empty(n, np.int64)
    inv[perm] = np.arange(n)
    e, j = np.nonzero(geo["interior"])
    assert np.all(S[inv[e], inv[geo["nbr"][e, j]]] == 1)


def test_rcm_handles_several_components_in_index_order():
    # two disjoint strips of two triangles each, listed interleaved
    nbr = np.array([[2, -1, -1], [3, -1, -1], [0, -1, -1], [1, -1, -1]])
    perm = ordering.rcm(nbr)
    # component {0,2} first (CM 0,2), then {1,3} (CM 1,3); reversed
    assert perm.tolist() == [3, 1, 2, 0]
