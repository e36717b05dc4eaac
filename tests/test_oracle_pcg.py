"""Pins for the oracle's PCG (dense Cholesky, statuses, stopping rule)."""
import numpy as np
import scipy.sparse as sp

from oracle import assemble as asm
from oracle import geometry, ordering, pcg
from synth import workloads


def system(npts=24, kind=asm.CP2, rhs="cp2"):
    w = workloads.square_inclusion(npts=npts, seed=3)
    m = w["mesh"]
    geo = geometry.build(m["xy"], m["tri"], w["side_tag"])
    perm = ordering.rcm(geo["nbr"])
    A = asm.assemble(geo, perm, kind, w["params"], w["nu"], w["dt"])["A"]
    return A, w["rhs"][rhs][perm]


def test_pcg_matches_dense_cholesky():
    A, b = system()
    assert A.shape[0] <= 2000
    x, info = pcg.pcg(A, b, tol=1e-10)
    assert info["status"] == pcg.OK and info["rel_res_true"] <= 1e-10
    assert info["iters"] % 50 == 0
    xd = pcg.dense_solve(A, b)
    assert np.linalg.norm(x - xd) <= 1e-9 * np.linalg.norm(xd)
    # the dense solution itself is a residual check on true_residual
    assert pcg.rel_residual(A, b, xd) < 1e-11


def test_pcg_cp1_matches_dense_cholesky():
    A, b = system(kind=asm.CP1X, rhs="cp1x")
    x, info = pcg.pcg(A, b, tol=1e-12)
    xd = pcg.dense_solve(A, b)
    assert info["status"] == pcg.OK
    assert np.linalg.norm(x - xd) <= 1e-11 * np.linalg.norm(xd)


def test_full_size_square_inclusion_reaches_tolerance():
    A, b = system(npts=64)
    x, info = pcg.pcg(A, b, tol=1e-10)
    assert info["status"] == pcg.OK and info["rel_res_true"] <= 1e-10


def test_true_residual_is_exact_on_integer_data():
    A = sp.csr_matrix(np.array([[4.0, -1.0, 0.0], [-1.0, 4.0, -1.0], [0.0, -1.0, 4.0]]))
    x = np.array([1.0, 2.0, 3.0])
    b = np.array([2.0 + 2 ** -40, 4.0, 10.0])
    np.testing.assert_array_equal(pcg.true_residual(A, b, x), [2 ** -40, 0.0, 0.0])


def test_statuses():
    A, b = system()
    x, info = pcg.pcg(A, b, tol=1e-10, max_it=5)
    assert info["status"] == pcg.MAXIT and info["iters"] == 5 and info["rel_res_true"] > 1e-10
    x, info = pcg.pcg(A, np.zeros(A.shape[0]))
    assert info["iters"] == 0 and not np.any(x)
    xs, _ = pcg.pcg(A, b, tol=1e-10)
    x, info = pcg.pcg(A, b, tol=1e-9, x0=xs)
    assert info["iters"] == 0 and info["status"] == pcg.OK
    # p.q = 0 at the first step, far from the solution: a breakdown
    indef = sp.csr_matrix(np.diag([1.0, -1.0]))
    x, info = pcg.pcg(indef, np.array([1.0, 1.0]))
    assert info["status"] == pcg.BREAKDOWN and info["iters"] == 0
    # three rows, indefinite: CG ends within three steps, then p.q reaches 0
    # on an iterate that solves the system, which is convergence
    indef = sp.csr_matrix(np.diag([1.0, -1.0, 2.0]))
    x, info = pcg.pcg(indef, np.array([1.0, 1.0, 1.0]))
    assert info["status"] == pcg.OK and np.allclose(x, [1.0, -1.0, 0.5], rtol=0, atol=1e-15)


def test_systems_of_one_and_two_rows_converge():
    """CG solves an n-row system within n iterations.  On one and two rows the
    recursion then reaches p.q = 0 before the first convergence test; the
    iterate, which meets the tolerance, is a converged solve (pinned against
    the direct solution), and a breakdown far from the solution stays one."""
    for A in (sp.csr_matrix([[4.0]]), sp.csr_matrix([[5.0, -1.0], [-1.0, 3.0]])):
        b = np.arange(1.0, A.shape[0] + 1.0)
        x, info = pcg.pcg(A, b, tol=1e-10)
        assert info["status"] == pcg.OK and 1 <= info["iters"] < 50
        xd = np.linalg.solve(A.toarray(), b)
        assert np.linalg.norm(x - xd) <= 1e-13 * np.linalg.norm(xd)
        assert info["rel_res_true"] <= 1e-15


def test_two_sum_is_error_free():
    from fractions import Fraction

    rng = np.random.default_rng(0)
    a = rng.standard_normal(200) * 10.0 ** rng.integers(-8, 8, 200)
    b = rng.standard_normal(200) * 10.0 ** rng.integers(-8, 8, 200)
    s, e = pcg.two_sum(a, b)
    for ai, bi, si, ei in zip(a, b, s, e):
        assert Fraction(si) + Fraction(ei) == Fraction(ai) + Fraction(bi)
        assert abs(ei) <= abs(np.spacing(si))


def test_unreachable_tolerance_reports_stagnation():
    A, b = system(npts=12)
    x, info = pcg.pcg(A, b, tol=1e-19, max_it=50000, stag_checks=10)
    assert info["status"] == pcg.STAGNATED and info["iters"] < 50000
    assert info["rel_res_true"] < 1e-12


def test_chebyshev_preconditioner_closed_form_on_eigenvectors():
    # for A v = lam D v the steps from z = 0 on A z = A v leave the error
    # R_k(lam) v with R_k(t) = T_k((theta - t)/delta) / T_k(theta/delta), so
    # z = (1 - R_k(lam)) v; T_k evaluated by numpy's Chebyshev series
    import scipy.linalg as sla
    from numpy.polynomial import chebyshev as C

    A, _ = system(npts=8)
    M = A.toarray()
    d = np.diag(M)
    lam, V = sla.eigh(M, np.diag(d))
    assert lam.max() <= 2.0 + 1e-12 and lam.min() > 0  # the Gershgorin bound used
    a, bnd = pcg.chebyshev_interval()
    theta, delta = 0.5 * (bnd + a), 0.5 * (bnd - a)
    for k in (2, 3, 5, 8):
        Tk = C.Chebyshev.basis(k)
        for i in (0, 1, len(lam) // 2, len(lam) - 1):
            v = V[:, i]
            z = pcg.chebyshev_apply(A, 1.0 / d, M @ v, k)
            R = Tk((theta - lam[i]) / delta) / Tk(theta / delta)
            np.testing.assert_allclose(z, (1.0 - R) * v, rtol=0, atol=1e-10 * np.abs(v).max())


def test_chebyshev_preconditioner_is_spd_and_cg_converges_faster():
    A, b = system(npts=10)
    n = A.shape[0]
    dinv = 1.0 / A.diagonal()
    Minv = np.column_stack([pcg.chebyshev_apply(A, dinv, e, 4) for e in np.eye(n)])
    assert np.abs(Minv - Minv.T).max() <= 1e-12 * np.abs(Minv).max()
    assert np.linalg.eigvalsh(0.5 * (Minv + Minv.T)).min() > 0
    A, b = system()
    xd = pcg.dense_solve(A, b)
    x1, i1 = pcg.pcg(A, b, tol=1e-10, replace_every=1)
    for k in (2, 4, 6):
        xk, ik = pcg.pcg(A, b, tol=1e-10, precond=pcg.CHEBYSHEV, degree=k, replace_every=1)
        assert ik["status"] == pcg.OK and ik["rel_res_true"] <= 1e-10
        assert np.linalg.norm(xk - xd) <= 1e-9 * np.linalg.norm(xd)
        assert ik["iters"] < i1["iters"]
