"""Pins for the oracle's coupled CP1 (Sec. 3.2.2, eq. cs1_sys2,
eq. CS1_sys_coeff; App. B, eq. A1)."""
import math

import numpy as np
import pytest

from oracle import assemble as asm
from oracle import cp1coupled as cc
from oracle import geometry, ordering
from synth import fields, meshes, workloads

NU = 1.5e-5


def case(npts=14, seed=3, beta=100.0, alpha_deg=30.0, K=1e-4, eps0=0.35, random_dir=False):
    m = meshes.square_jittered_grid(npts, 0.3, seed)
    tag = workloads.side_tags(m["group"], [meshes.G_LEFT, meshes.G_BOTTOM, meshes.G_TOP],
                              [meshes.G_RIGHT])
    geo = geometry.build(m["xy"], m["tri"], tag)
    n = geo["n"]
    rng = np.random.default_rng(seed)
    if random_dir:
        s = np.array([fields.aniso_shape(b, a) for b, a in
                      zip(rng.uniform(1, beta, n), rng.uniform(0, math.pi, n))])
        g11, g12, g22 = s[:, 0], s[:, 1], s[:, 2]
    else:
        a, b, d = fields.aniso_shape(beta, math.radians(alpha_deg))
        g11, g12, g22 = np.full(n, a), np.full(n, b), np.full(n, d)
    prm = {"eps": np.full(n, eps0), "logk": np.full(n, math.log(K)), "chi": rng.uniform(0.5, 1, n),
           "g11": g11, "g12": g12, "g22": g22}
    # coarse cells: the mass term M A_e must not be negligible against nu T
    dt = 0.05 * K / (NU * eps0)
    perm = ordering.rcm(geo["nbr"])
    Ax = asm.assemble(geo, perm, asm.CP1X, prm, NU, dt)["A"]
    Ay = asm.assemble(geo, perm, asm.CP1Y, prm, NU, dt)["A"]
    m_cell = cc.coupling_weights(geo, prm, NU, dt)
    return geo, perm, prm, dt, Ax, Ay, m_cell


def test_m12_is_the_mass_tensor_offdiagonal():
    """M12 of the cell tensors equals the off-diagonal of I/dt + nu eps K^-1
    with K built from eq. aniso directly."""
    beta, alpha, kk, eps, dt = 100.0, math.radians(30.0), 1e-4, 0.35, 3.0
    R = np.array([[math.cos(alpha), -math.sin(alpha)], [math.sin(alpha), math.cos(alpha)]])
    K = R @ np.diag([kk / beta, kk]) @ R.T
    M = np.eye(2) / dt + NU * eps * np.linalg.inv(K)
    g11, g12, g22 = fields.aniso_shape(beta, alpha)
    ct = asm.cell_tensors(np.array([eps]), np.log([kk]), np.ones(1), [g11], [g12], [g22], NU, dt)
    assert abs(ct["M12"][0] - M[0, 1]) <= 1e-12 * abs(M[0, 1])
    assert abs(ct["M11"][0] - M[0, 0]) <= 1e-12 * M[0, 0]
    assert abs(ct["M22"][0] - M[1, 1]) <= 1e-12 * M[1, 1]


def test_coupled_matrix_is_spd_and_the_cell_blocks_are_the_mass_tensors():
    geo, perm, prm, dt, Ax, Ay, m_cell = case(npts=8)
    n = geo["n"]
    C = cc.coupled_matrix(Ax, Ay, m_cell[perm]).toarray()
    assert np.array_equal(C, C.T)
    assert np.linalg.eigvalsh(C).min() > 0
    # subtracting nu L (x) I and the Dirichlet terms leaves M_e A_e per cell
    ct = asm.cell_tensors(prm["eps"], prm["logk"], prm["chi"], prm["g11"], prm["g12"], prm["g22"],
                          NU, dt)
    i = 5
    e = perm[i]
    blk = C[np.ix_([i, n + i], [i, n + i])]
    lap = Ax[i, i] - ct["M11"][e] * geo["area"][e]
    np.testing.assert_allclose(blk - lap * np.eye(2),
                               geo["area"][e] * np.array([[ct["M11"][e], ct["M12"][e]],
                                                          [ct["M12"][e], ct["M22"][e]]]),
                               rtol=1e-12)


@pytest.mark.parametrize("random_dir", [False, True])
def test_block_iteration_converges_to_the_coupled_solution(random_dir):
    """A manufactured pair (u*, v*): with direct inner solves the loop of
    App. B reaches the solution of the coupled system."""
    geo, perm, prm, dt, Ax, Ay, m_cell = case(random_dir=random_dir)
    n = geo["n"]
    rng = np.random.default_rng(1)
    us, vs = rng.standard_normal(n), rng.standard_normal(n)
    C = cc.coupled_matrix(Ax, Ay, m_cell[perm])
    b = C @ np.concatenate([us, vs])
    sx, sy = cc.dense_solvers(Ax, Ay)
    out = cc.block_iteration(sx, sy, m_cell[perm], b[:n], b[n:], toll=1e-7, max_outer=200)
    assert out["converged"]
    assert out["outer"] >= 2  # the coupling is not negligible here
    # err <= toll bounds the relative change of one component by toll^2
    assert np.linalg.norm(out["u"] - us) <= 1e-9 * np.linalg.norm(us)
    assert np.linalg.norm(out["v"] - vs) <= 1e-9 * np.linalg.norm(vs)
    # block Jacobi: the errors fall by orders of magnitude over the loop
    e = np.array(out["errs"])
    assert e[-1] < 1e-5 * e[0]


def test_isotropic_case_decouples():
    """M12 = 0 (isotropic K): the first coupled pass repeats the first solves,
    the loop stops after one pass and each component is its scalar solve."""
    geo, perm, prm, dt, Ax, Ay, m_cell = case(beta=1.0)
    assert np.all(m_cell == 0)
    n = geo["n"]
    rng = np.random.default_rng(2)
    bx, by = rng.standard_normal(n), rng.standard_normal(n)
    sx, sy = cc.dense_solvers(Ax, Ay)
    out = cc.block_iteration(sx, sy, m_cell[perm], bx, by)
    assert out["outer"] == 1 and out["errs"] == [0.0]
    assert np.array_equal(out["u"], sx(bx, None)) and np.array_equal(out["v"], sy(by, None))


def test_err_definition():
    """App. B test: square roots of the two norms."""
    old = np.array([3.0, 4.0])
    new = old + np.array([0.0, 2.0 ** -11])  # exact in float64
    assert math.isclose(cc.err_app_b(new, old), math.sqrt(2.0 ** -11) / math.sqrt(5.0),
                        rel_tol=1e-15)
    assert cc.err_app_b(np.zeros(2), np.zeros(2)) == 0.0
    assert cc.err_app_b(np.ones(2), np.zeros(2)) == np.inf


def test_pcg_inner_solves_match_direct():
    geo, perm, prm, dt, Ax, Ay, m_cell = case()
    n = geo["n"]
    rng = np.random.default_rng(4)
    bx, by = rng.standard_normal(n), rng.standard_normal(n)
    d = cc.block_iteration(*cc.dense_solvers(Ax, Ay), m_cell[perm], bx, by, toll=1e-5)
    p = cc.block_iteration(*cc.pcg_solvers(Ax, Ay), m_cell[perm], bx, by, toll=1e-5)
    assert d["outer"] == p["outer"]
    assert np.linalg.norm(p["u"] - d["u"]) <= 1e-8 * np.linalg.norm(d["u"])
    assert np.linalg.norm(p["v"] - d["v"]) <= 1e-8 * np.linalg.norm(d["v"])


def test_both_components_use_the_previous_iterate():
    """eq. A1 updates u and v from iterate i (block Jacobi, not Gauss-Seidel):
    one coupled pass gives u1 = A_x^-1 (b_x - m v0), v1 = A_y^-1 (b_y - m u0)
    with u0, v0 the uncoupled solves."""
    geo, perm, prm, dt, Ax, Ay, m_cell = case(npts=10)
    n = geo["n"]
    rng = np.random.default_rng(6)
    bx, by = rng.standard_normal(n), rng.standard_normal(n)
    m = m_cell[perm]
    Dx, Dy = Ax.toarray(), Ay.toarray()
    u0, v0 = np.linalg.solve(Dx, bx), np.linalg.solve(Dy, by)
    out = cc.block_iteration(*cc.dense_solvers(Ax, Ay), m, bx, by, toll=np.inf)
    assert out["outer"] == 1
    np.testing.assert_allclose(out["u"], np.linalg.solve(Dx, bx - m * v0), rtol=1e-10, atol=1e-14)
    np.testing.assert_allclose(out["v"], np.linalg.solve(Dy, by - m * u0), rtol=1e-10, atol=1e-14)
    # a Gauss-Seidel pass (v from the new u) differs measurably here
    u1 = out["u"]
    assert np.linalg.norm(np.linalg.solve(Dy, by - m * u1) - out["v"]) > 1e-6 * np.linalg.norm(out["v"])


def test_loop_stops_when_either_component_settles():
    """err = min(err_x, err_y): a settled x component ends the loop even while
    y still changes (stub solvers)."""
    calls = {"y": 0}

    def sx(r, x0):
        return np.ones(4)

    def sy(r, x0):
        calls["y"] += 1
        return np.full(4, float(calls["y"]))

    out = cc.block_iteration(sx, sy, np.zeros(4), np.zeros(4), np.zeros(4), toll=1e-4)
    assert out["outer"] == 1 and out["errs"] == [0.0] and out["converged"]


def test_block_inverses_invert_the_cell_blocks():
    geo, perm, prm, dt, Ax, Ay, m_cell = case(npts=8, random_dir=True)
    m = m_cell[perm]
    i11, i12, i22 = cc.block_inverses(Ax, Ay, m)
    dx, dy = Ax.diagonal(), Ay.diagonal()
    for e in range(0, geo["n"], 7):
        Pe = np.array([[dx[e], m[e]], [m[e], dy[e]]])
        np.testing.assert_allclose(Pe @ np.array([[i11[e], i12[e]], [i12[e], i22[e]]]), np.eye(2),
                                   atol=1e-13)


@pytest.mark.parametrize("random_dir", [False, True])
def test_coupled_pcg_reaches_the_direct_solution(random_dir):
    """Block-Jacobi CG on the coupled system against a sparse direct solve of
    it, for a manufactured pair and a smooth right-hand side."""
    import scipy.sparse.linalg as spl

    geo, perm, prm, dt, Ax, Ay, m_cell = case(random_dir=random_dir)
    n = geo["n"]
    m = m_cell[perm]
    C = cc.coupled_matrix(Ax, Ay, m)
    rng = np.random.default_rng(9)
    xs = np.concatenate([rng.standard_normal(n), rng.standard_normal(n)])
    b = C @ xs
    (u, v), info = cc.coupled_pcg(Ax, Ay, m, b[:n], b[n:])
    assert info["status"] == 0 and info["rel_res_true"] <= 1e-10 and info["iters"] % 50 == 0
    x = np.concatenate([u, v])
    assert np.linalg.norm(x - xs) <= 1e-8 * np.linalg.norm(xs)
    xd = spl.spsolve(C.tocsc(), b)
    assert np.linalg.norm(x - xd) <= 1e-8 * np.linalg.norm(xd)


def test_coupled_pcg_on_the_channel_and_the_loop_limit():
    """On a small anisotropic channel (eq. aniso block, 11,840 cells) the
    coupled CG reaches the direct solution, and the loop of App. B converges
    towards the same solution (slowly: the block's cell tensors are strongly
    coupled)."""
    import scipy.sparse.linalg as spl

    w = workloads.channel(30, 3, aniso=True)
    m_ = w["mesh"]
    geo = geometry.build(m_["xy"], m_["tri"], w["side_tag"])
    perm = ordering.rcm(geo["nbr"])
    Ax = asm.assemble(geo, perm, asm.CP1X, w["params"], w["nu"], w["dt"])["A"]
    Ay = asm.assemble(geo, perm, asm.CP1Y, w["params"], w["nu"], w["dt"])["A"]
    m = cc.coupling_weights(geo, w["params"], w["nu"], w["dt"])[perm]
    n = geo["n"]
    bx, by = w["rhs"]["cp1x"][perm], w["rhs"]["cp1y"][perm]
    (u, v), info = cc.coupled_pcg(Ax, Ay, m, bx, by)
    assert info["status"] == 0
    xd = spl.spsolve(cc.coupled_matrix(Ax, Ay, m).tocsc(), np.concatenate([bx, by]))
    assert np.linalg.norm(np.concatenate([u, v]) - xd) <= 1e-9 * np.linalg.norm(xd)
    fx, fy = spl.factorized(Ax.tocsc()), spl.factorized(Ay.tocsc())
    lp = cc.block_iteration(lambda r, x0: fx(r), lambda r, x0: fy(r), m, bx, by, toll=1e-3,
                            max_outer=400)
    assert lp["converged"] and lp["outer"] > 50
    e_loop = np.linalg.norm(np.concatenate([lp["u"], lp["v"]]) - xd) / np.linalg.norm(xd)
    assert e_loop < 1e-3
