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
    indef = sp.csr_matrix(np.diag([1.0, -1.0, 2.0]))
    x, info = pcg.pcg(indef, np.array([1.0, 1.0, 1.0]))
    assert info["status"] == pcg.BREAKDOWN


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
