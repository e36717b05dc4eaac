"""Pins for the oracle's cell tensors and corrector matrices."""
import math

import numpy as np
import pytest

from oracle import assemble as asm
from oracle import geometry, ordering
from oracle import pcg
from synth import fields, meshes, workloads

NU, DT = 1.5e-5, 19.0


def test_cell_tensor_closed_forms():
    eps = np.array([1.0, 0.4, 0.35])
    logk = np.log(np.array([1e-3, 1e-3, 1e-4]))
    chi = np.array([0.0, 1.0, 0.5])
    one, zero = np.ones(3), np.zeros(3)
    ct = asm.cell_tensors(eps, logk, chi, one, zero, one, NU, DT)
    # fluid cell (chi = 0): Kfrak = 0, M = I/dt, Xi = eps dt I
    assert ct["K11"][0] == 0 and ct["M11"][0] == 1 / DT and ct["X11"][0] == eps[0] * DT
    # isotropic: Xi = eps dt / (1 + nu eps dt k) I with k = chi / K
    k = chi * np.exp(-logk)
    np.testing.assert_allclose(ct["X11"], eps * DT / (1 + NU * eps * DT * k), rtol=1e-15)
    np.testing.assert_allclose(ct["X22"], ct["X11"], rtol=0)
    assert np.all(ct["X12"] == 0)
    np.testing.assert_allclose(ct["M11"], 1 / DT + NU * eps * k, rtol=1e-15)


def test_anisotropic_tensor_matches_eq_aniso():
    beta, alpha, kk = 100.0, math.radians(30.0), 1e-4
    R = np.array([[math.cos(alpha), -math.sin(alpha)], [math.sin(alpha), math.cos(alpha)]])
    K = R @ np.diag([kk / beta, kk]) @ np.linalg.inv(R)
    g11, g12, g22 = fields.aniso_shape(beta, alpha)
    np.testing.assert_allclose(np.linalg.inv(K) * kk, [[g11, g12], [g12, g22]], rtol=1e-12)
    eps = np.array([0.35])
    ct = asm.cell_tensors(eps, np.log([kk]), np.ones(1), [g11], [g12], [g22], NU, DT)
    S = np.array([[ct["S11"][0], ct["S12"][0]], [ct["S12"][0], ct["S22"][0]]])
    X = np.array([[ct["X11"][0], ct["X12"][0]], [ct["X12"][0], ct["X22"][0]]])
    np.testing.assert_allclose(S @ X, eps[0] * DT * np.eye(2), atol=1e-12 * eps[0] * DT)
    # Xi = eps M^{-1} with M = I/dt + nu eps K^{-1}
    M = np.eye(2) / DT + NU * eps[0] * np.linalg.inv(K)
    np.testing.assert_allclose(X, eps[0] * np.linalg.inv(M), rtol=1e-12)


def small_case(aniso):
    m = meshes.square_jittered_grid(9, 0.3, 4)
    c = meshes.centroids(m)
    n = m["tri"].shape[0]
    rng = np.random.default_rng(0)
    prm = {
        "eps": rng.uniform(0.3, 1.0, n), "logk": np.log(rng.uniform(1e-5, 1e-3, n)),
        "chi": rng.uniform(0.0, 1.0, n), "g11": np.ones(n), "g12": np.zeros(n), "g22": np.ones(n),
    }
    if aniso:
        g11, g12, g22 = fields.aniso_shape(100.0, math.radians(30.0))
        prm.update(g11=np.full(n, g11), g12=np.full(n, g12), g22=np.full(n, g22))
    tag = workloads.side_tags(m["group"], [meshes.G_LEFT, meshes.G_TOP], [meshes.G_RIGHT])
    geo = geometry.build(m["xy"], m["tri"], tag)
    perm = ordering.rcm(geo["nbr"])
    return geo, perm, prm


@pytest.mark.parametrize("aniso", [False, True])
@pytest.mark.parametrize("kind", [asm.CP1X, asm.CP1Y, asm.CP2])
def test_matrix_invariants(kind, aniso):
    geo, perm, prm = small_case(aniso)
    out = asm.assemble(geo, perm, kind, prm, NU, DT)
    A = out["A"]
    n = geo["n"]
    row_ptr, col = ordering.csr_pattern(geo["nbr"], perm)
    assert np.array_equal(A.indptr, row_ptr) and np.array_equal(A.indices, col)
    assert (A != A.T).nnz == 0  # bitwise symmetric: one weight per side
    D = A.toarray()
    off = D - np.diag(np.diag(D))
    assert np.all(np.diag(D) > 0)
    assert np.all(off[A.toarray() != 0] < 0) or True
    rows = np.repeat(np.arange(n), np.diff(A.indptr))
    offd = A.data[rows != A.indices]
    assert np.all(offd < 0)  # M-matrix sign pattern
    # row excess = mass term (CP1) or Dirichlet weights (CP2)
    sw = out["weights"]
    inv = np.empty(n, np.int64)
    inv[perm] = np.arange(n)
    excess = np.diag(D) + off.sum(axis=1)
    want = (sw["mass"] + np.where(sw["dirichlet"], sw["w"], 0.0).sum(axis=1))[perm]
    assert np.all(np.abs(excess - want) <= 8 * np.finfo(float).eps * np.diag(D))
    assert np.linalg.eigvalsh(D).min() > 0


def test_cp1_x_and_y_agree_only_when_isotropic():
    geo, perm, prm = small_case(False)
    Ax = asm.assemble(geo, perm, asm.CP1X, prm, NU, DT)["A"]
    Ay = asm.assemble(geo, perm, asm.CP1Y, prm, NU, DT)["A"]
    assert (Ax != Ay).nnz == 0
    geo, perm, prm = small_case(True)
    Ax = asm.assemble(geo, perm, asm.CP1X, prm, NU, DT)["A"]
    Ay = asm.assemble(geo, perm, asm.CP1Y, prm, NU, DT)["A"]
    assert (Ax != Ay).nnz > 0


def _linear_field_case(kind, mass_on):
    """Constant isotropic coefficient, linear field eta = a + g.x: the two-point
    flux is exact, so the solve reproduces eta at the circumcenters."""
    m = meshes.square_jittered_grid(16, 0.3, 8)
    n = m["tri"].shape[0]
    tag = workloads.side_tags(m["group"], [meshes.G_RIGHT, meshes.G_TOP], [meshes.G_RIGHT, meshes.G_TOP])
    geo = geometry.build(m["xy"], m["tri"], tag)
    perm = ordering.rcm(geo["nbr"])
    eps = 0.7
    prm = asm.default_params(n, eps=np.full(n, eps), chi=np.zeros(n))  # fluid: Xi = eps dt I
    a, gx, gy = 0.3, -1.7, 0.9
    cc = geometry.circumcenters(m["xy"], m["tri"])
    exact = a + gx * cc[:, 0] + gy * cc[:, 1]
    P = m["xy"][m["tri"]]
    mid = np.stack([0.5 * (P[:, (j + 1) % 3] + P[:, (j + 2) % 3]) for j in range(3)], axis=1)
    g_dir = a + gx * mid[..., 0] + gy * mid[..., 1]
    out = asm.assemble(geo, perm, kind, prm, NU, DT, g_dirichlet=g_dir)
    coef = NU if kind != asm.CP2 else eps * DT
    t = geo["t"]
    l = np.hypot(t[..., 0], t[..., 1])
    gn = (gx * t[..., 1] - gy * t[..., 0]) / l  # g . n_j
    bit = 2 if kind == asm.CP2 else 1
    neumann = (~geo["interior"]) & ((geo["tag"] & bit) == 0)
    b = out["b_lift"] + np.where(neumann, coef * gn * l, 0.0).sum(axis=1)
    if mass_on:
        ct = asm.cell_tensors(prm["eps"], prm["logk"], prm["chi"], prm["g11"], prm["g12"], prm["g22"], NU, DT)
        b = b + ct["M11"] * geo["area"] * exact
    x = pcg.dense_solve(out["A"], b[perm])
    return x, exact[perm]


def test_cp2_reproduces_linear_field():
    x, exact = _linear_field_case(asm.CP2, False)
    assert np.max(np.abs(x - exact)) <= 1e-11 * np.max(np.abs(exact))


def test_cp1_reproduces_linear_field():
    x, exact = _linear_field_case(asm.CP1X, True)
    assert np.max(np.abs(x - exact)) <= 1e-11 * np.max(np.abs(exact))


def test_normal_quadratic_special_directions():
    # n is the outward normal of a CCW side vector t: n = rot(-90 deg) t / |t|
    a11, a12, a22 = 3.0, 0.7, 2.0
    t = np.array([[1.0, 0.0], [0.0, 2.0], [1.0, 1.0], [-1.0, 1.0]])
    got = asm.normal_quadratic(t, a11, a12, a22)
    # t along +x -> n = (0,-1); t along +y -> n = (1,0); t = (1,1) -> n = (1,-1)/sqrt2;
    # t = (-1,1) -> n = (1,1)/sqrt2
    want = [a22, a11, (a11 - 2 * a12 + a22) / 2, (a11 + 2 * a12 + a22) / 2]
    np.testing.assert_allclose(got, want, rtol=1e-15)
