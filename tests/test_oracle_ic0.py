"""Pins for the oracle's IC(0) preconditioner (the paper's choice, Sec. 3.2.2
and 3.2.3; CPU context only)."""
import math

import numpy as np
import scipy.sparse as sp

from oracle import assemble as asm
from oracle import geometry, ic0, ordering
from oracle import pcg as opcg
from synth import workloads


def test_hand_example_drops_the_fill():
    """A = [[4,-1,-1],[-1,4,0],[-1,0,4]]: IC(0) keeps L's pattern in A's lower
    triangle, so the (2,1) fill of the exact factor is dropped."""
    A = sp.csr_matrix(np.array([[4.0, -1, -1], [-1, 4, 0], [-1, 0, 4]]))
    L = ic0.ic0(A).toarray()
    want = np.array([[2.0, 0, 0], [-0.5, math.sqrt(15) / 2, 0], [-0.5, 0, math.sqrt(15) / 2]])
    np.testing.assert_allclose(L, want, rtol=1e-15, atol=0)
    exact = np.linalg.cholesky(A.toarray())
    assert exact[2, 1] != 0 and L[2, 1] == 0


def test_tridiagonal_is_exact_cholesky():
    """No fill in a tridiagonal matrix: IC(0) is the Cholesky factor."""
    n = 40
    A = sp.diags([-np.ones(n - 1), 2.5 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1], format="csr")
    np.testing.assert_allclose(ic0.ic0(A).toarray(), np.linalg.cholesky(A.toarray()), rtol=1e-13,
                               atol=1e-15)


def small_cp2():
    w = workloads.square_inclusion(npts=12, seed=2)
    m = w["mesh"]
    geo = geometry.build(m["xy"], m["tri"], w["side_tag"])
    perm = ordering.rcm(geo["nbr"])
    A = asm.assemble(geo, perm, asm.CP2, w["params"], w["nu"], w["dt"])["A"]
    return A, w["rhs"]["cp2"][perm]


def test_product_matches_a_on_its_pattern():
    A, _ = small_cp2()
    L = ic0.ic0(A)
    Lc = sp.coo_matrix(L)
    assert np.all(Lc.row >= Lc.col)
    lowA = sp.tril(A)
    assert (abs(sp.csr_matrix((np.ones(Lc.nnz), (Lc.row, Lc.col)), shape=A.shape)) -
            abs(sp.csr_matrix((np.ones(lowA.nnz), (lowA.row, lowA.col)), shape=A.shape))).nnz == 0
    P = (L @ L.T).tocsr()
    Ad = A.toarray()
    Pd = P.toarray()
    mask = Ad != 0
    np.testing.assert_allclose(Pd[mask], Ad[mask], rtol=1e-12, atol=1e-12 * np.abs(Ad).max())
    assert np.abs(Pd[~mask]).max() > 0  # the dropped fill shows off the pattern


def test_ic_pcg_converges_in_fewer_iterations():
    A, b = small_cp2()
    x_j, ij = opcg.pcg(A, b, tol=1e-10, replace_every=10)
    x_i, ii = opcg.pcg(A, b, tol=1e-10, replace_every=10, precond=opcg.IC0)
    assert ij["status"] == 0 and ii["status"] == 0
    assert ii["iters"] < ij["iters"]
    xd = opcg.dense_solve(A, b)
    assert np.linalg.norm(x_i - xd) <= 1e-8 * np.linalg.norm(xd)
