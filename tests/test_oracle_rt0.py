"""Pins for the oracle's averaged fluxes and RT0 velocity (Sec. 3.2.2,
eq. flux_k_+_2/3; Sec. 3.2.3, eq. eta_flux; App. A, eq. RT0)."""
import math

import numpy as np
import pytest

from oracle import assemble as asm
from oracle import crossflux as cf
from oracle import geometry, rt0
from synth import fields, meshes, workloads

NU, DT = 1.5e-5, 19.0


def square(npts=12, seed=3, cp1=(1, 3, 4), cp2=(2,)):
    m = meshes.square_jittered_grid(npts, 0.3, seed)
    tag = workloads.side_tags(m["group"], list(cp1), list(cp2))
    return geometry.build(m["xy"], m["tri"], tag)


def test_two_cell_area_weighting_by_hand():
    """Two triangles sharing the side (1,0)-(0.4,0.9): the shared flux is the
    mean of the two normal fluxes weighted by the other cell's area."""
    xy = np.array([[0.0, 0.0], [1.0, 0.0], [0.4, 0.9], [1.3, 1.1]])
    tri = np.array([[0, 1, 2], [1, 3, 2]])
    geo = geometry.build(xy, tri, np.zeros((2, 3), np.int8))
    u, v = np.array([2.0, -1.0]), np.array([0.5, 3.0])
    F = rt0.flux_average(geo, u, v)
    # side 0 of cell 0 (opposite node 0) is the shared one, from (1,0) to (0.4,0.9)
    assert geo["nbr"][0, 0] == 1
    A0 = 0.5 * abs(1.0 * 0.9 - 0.0 * 0.4)
    A1 = 0.5 * abs((1.3 - 1.0) * (0.9 - 0.0) - (1.1 - 0.0) * (0.4 - 1.0))
    tx, ty = 0.4 - 1.0, 0.9 - 0.0
    l = math.hypot(tx, ty)
    nx, ny = ty / l, -tx / l
    want = ((u[0] * nx + v[0] * ny) * A1 + (u[1] * nx + v[1] * ny) * A0) / (A0 + A1) * l
    assert abs(F[0, 0] - want) <= 1e-15 * abs(want)
    jp = geo["nbr_side"][0, 0]
    assert F[1, jp] == -F[0, 0]


def test_flux_average_continuity_and_uniform_field():
    geo = square()
    rng = np.random.default_rng(0)
    n = geo["n"]
    F = rt0.flux_average(geo, rng.standard_normal(n), rng.standard_normal(n))
    e, j = np.nonzero(geo["interior"])
    assert np.array_equal(F[e, j], -F[geo["nbr"][e, j], geo["nbr_side"][e, j]])
    # a uniform field (also prescribed on the CP1 Dirichlet sides): the normal
    # fluxes exactly, and B_1 = sum_j Fbar_j = u0 . sum_j l_j n_j = 0
    u0 = (0.7, -0.3)
    g = np.ones((n, 3))
    F = rt0.flux_average(geo, np.full(n, u0[0]), np.full(n, u0[1]), u0[0] * g, u0[1] * g)
    nrm, l = rt0.normals(geo)
    exact = (u0[0] * nrm[..., 0] + u0[1] * nrm[..., 1]) * l
    np.testing.assert_allclose(F, exact, rtol=1e-14, atol=1e-16)
    assert np.abs(F.sum(axis=1)).max() <= 1e-15 * l.max()


def test_boundary_sides_prescribed_or_own_flux():
    geo = square()
    n = geo["n"]
    rng = np.random.default_rng(1)
    u, v = rng.standard_normal(n), rng.standard_normal(n)
    gx, gy = rng.standard_normal((n, 3)), rng.standard_normal((n, 3))
    F = rt0.flux_average(geo, u, v, gx, gy)
    nrm, l = rt0.normals(geo)
    bnd = ~geo["interior"]
    pres = bnd & ((geo["tag"] & 1) != 0)
    free = bnd & ((geo["tag"] & 1) == 0)
    assert pres.any() and free.any()
    np.testing.assert_allclose(F[pres], ((gx * nrm[..., 0] + gy * nrm[..., 1]) * l)[pres], rtol=1e-15)
    ue = (u[:, None] * nrm[..., 0] + v[:, None] * nrm[..., 1]) * l
    np.testing.assert_allclose(F[free], ue[free], rtol=1e-15)


def test_rt0_basis_fluxes():
    """Q = e_j gives flux 1 through side j and 0 through the two others
    (the field is linear, so its side flux is its midpoint value times l)."""
    geo = square(npts=6)
    n = geo["n"]
    P = geo["xy"][geo["tri"]]
    nrm, l = rt0.normals(geo)
    for j in range(3):
        Q = np.zeros((n, 3))
        Q[:, j] = 1.0
        for k in range(3):
            mid = 0.5 * (P[:, (k + 1) % 3] + P[:, (k + 2) % 3])
            uk = rt0.rt0_velocity(geo, Q, at=mid)
            flux = (uk * nrm[:, k]).sum(axis=1) * l[:, k]
            np.testing.assert_allclose(flux, float(j == k), atol=1e-12)


def test_rt0_reproduces_constant_fields():
    geo = square()
    u0 = np.array([0.3, 1.7])
    nrm, l = rt0.normals(geo)
    Q = (nrm @ u0) * l
    got = rt0.rt0_velocity(geo, Q)
    np.testing.assert_allclose(got, np.broadcast_to(u0, got.shape), rtol=1e-12, atol=1e-14)


def test_linear_eta_gives_xi_grad_eta():
    """Constant anisotropic Xi, linear eta, B_1 = 0: the step's fluxes are
    the exact normal fluxes of Xi grad(eta) and the RT0 velocity is that
    constant vector in every cell."""
    geo = square(cp1=(), cp2=(1, 2, 3, 4))
    n = geo["n"]
    g11, g12, g22 = fields.aniso_shape(100.0, math.radians(30.0))
    prm = {"eps": np.full(n, 0.35), "logk": np.full(n, math.log(1e-4)), "chi": np.ones(n),
           "g11": np.full(n, g11), "g12": np.full(n, g12), "g22": np.full(n, g22)}
    cc = geometry.circumcenters(geo["xy"], geo["tri"])
    P = geo["xy"][geo["tri"]]
    mid = np.stack([0.5 * (P[:, (j + 1) % 3] + P[:, (j + 2) % 3]) for j in range(3)], axis=1)
    G = np.array([0.7, -1.3])
    eta, gmid = cc @ G + 0.25, mid @ G + 0.25
    Q = rt0.step_fluxes(geo, prm, NU, DT, np.zeros((n, 3)), eta, eta, gmid)
    ct = asm.cell_tensors(prm["eps"], prm["logk"], prm["chi"], prm["g11"], prm["g12"], prm["g22"], NU, DT)
    X = np.array([[ct["X11"][0], ct["X12"][0]], [ct["X12"][0], ct["X22"][0]]])
    want = X @ G
    got = rt0.rt0_velocity(geo, Q)
    assert np.abs(got - want).max() <= 1e-8 * np.abs(want).max()
    assert np.abs(Q.sum(axis=1)).max() <= 1e-8 * np.abs(Q).max()


def test_cell_sums_are_the_second_solve_residual():
    """sum_j Q_j = (B_1 + lift + cross(eta~) - A eta)_e for any eta, eta~:
    the step's fluxes balance exactly when the second CP2 system is solved,
    and the two-solve sequence with direct solves gives balanced cells."""
    m = workloads.channel(24, 2, aniso=True)
    geo = geometry.build(m["mesh"]["xy"], m["mesh"]["tri"], m["side_tag"])
    n = geo["n"]
    prm, nu, dt = m["params"], m["nu"], m["dt"]
    rng = np.random.default_rng(4)
    u, v = rng.standard_normal(n), rng.standard_normal(n)
    gx, gy = rng.standard_normal((n, 3)), rng.standard_normal((n, 3))
    g2 = rng.standard_normal((n, 3))
    fbar = rt0.flux_average(geo, u, v, gx, gy)
    b1 = fbar.sum(axis=1)
    o = asm.assemble(geo, np.arange(n), asm.CP2, prm, nu, dt, g_dirichlet=g2)
    A, lift = o["A"], o["b_lift"]
    eta_t, eta = rng.standard_normal(n), rng.standard_normal(n)
    Q = rt0.step_fluxes(geo, prm, nu, dt, fbar, eta, eta_t, g2)
    cross = cf.cross_terms(geo, prm, nu, dt, eta_t, g2)["cross"]
    want = b1 + lift + cross - A @ eta
    scale = np.abs(fbar).sum(axis=1) + np.abs(A) @ np.abs(eta) + np.abs(lift) + cf.cross_terms(
        geo, prm, nu, dt, eta_t, g2)["scale"]
    assert np.all(np.abs(Q.sum(axis=1) - want) <= 1e-13 * scale)
    et, e2, _ = cf.two_step_dense(geo, A, prm, nu, dt, b1 + lift, g2)
    Q = rt0.step_fluxes(geo, prm, nu, dt, fbar, e2, et, g2)
    assert np.abs(Q.sum(axis=1)).max() <= 1e-10 * np.abs(Q).max()
