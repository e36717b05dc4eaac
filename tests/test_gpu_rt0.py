"""GPU parity of the averaged side fluxes (flux_average) and the RT0 velocity
update (rt0_update) against the oracle (Sec. 3.2.2, eq. flux_k_+_2/3;
Sec. 3.2.3, eq. eta_flux; App. A, eq. RT0), and the whole step on the GPU.

Tolerances (u = 2^-53), per side or cell, from the magnitudes each value is
built from:
  * fbar: 16 u (|u_e| + |v_e| + |u_ep| + |v_ep| + |g|) l; b1: their sum.
  * Q: 32 u (|fbar| + |w| (|eta_e| + |eta_ep|) + l S), w the CP2 weight and
    S the oracle's magnitude sum of the tangential term.
  * velocity: sum_j [(8 u |Q_j| + tol(Q_j)) |c - x_j| + 4 u |Q_j| (|x_j| + |c|)]
    / (2 A): the oracle takes differences of node coordinates.
Fluxes from the two cells of a side are compared bitwise (continuity).  The
whole step (coupled CP1, averaged fluxes, the two CP2 solves, RT0) checks that
the cell sums of Q equal the second CP2 system's residual under the oracle's
matrix, which the solve brings below 1e-10 relative; per cell to 1e-13 of
the magnitudes involved, |A||eta| included (the GPU's weights match the
oracle's matrix entries to 1e-13 relative).
"""
import functools
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import assemble as oasm  # noqa: E402
from oracle import crossflux as ocf  # noqa: E402
from oracle import geometry, ordering, rt0  # noqa: E402
from oracle import pcg as opcg  # noqa: E402
from synth import fields, meshes, workloads  # noqa: E402

pytestmark = pytest.mark.gpu
U = 2.0 ** -53


def B():
    from paper_2309_03543_amd import binding

    return binding


@functools.lru_cache(maxsize=None)
def case(name):
    if name == "square":
        w = workloads.square_inclusion(npts=20, seed=3)
        rng = np.random.default_rng(5)
        n = w["mesh"]["tri"].shape[0]
        s = np.array([fields.aniso_shape(b, a) for b, a in
                      zip(rng.uniform(1, 50, n), rng.uniform(0, math.pi, n))])
        w["params"] = dict(w["params"], g11=s[:, 0], g12=s[:, 1], g22=s[:, 2])
    else:
        w = workloads.channel(30, 3, aniso=True)
    m = w["mesh"]
    geo = geometry.build(m["xy"], m["tri"], w["side_tag"])
    perm = ordering.rcm(geo["nbr"])
    mesh = B().Mesh(m["xy"], m["tri"], w["side_tag"])
    dev = torch.device("cuda:0")
    tprm = {k: torch.tensor(v, device=dev) for k, v in w["params"].items()}
    return {"w": w, "geo": geo, "perm": perm, "mesh": mesh, "tprm": tprm, "dev": dev,
            "n": geo["n"]}


def T(c, a):
    return torch.tensor(np.ascontiguousarray(a), device=c["dev"])


def fbar_tol(c, u, v, gx, gy):
    geo = c["geo"]
    _, l = rt0.normals(geo)
    o = np.maximum(geo["nbr"], 0)
    mag = (np.abs(u) + np.abs(v))[:, None] + np.where(geo["interior"], (np.abs(u) + np.abs(v))[o], 0.0)
    return 16 * U * (mag + np.abs(gx) + np.abs(gy)) * l


@pytest.mark.parametrize("name", ["square", "channel"])
def test_flux_average_matches_oracle(name):
    c = case(name)
    rng = np.random.default_rng(1)
    n = c["n"]
    u, v = rng.standard_normal(n), rng.standard_normal(n)
    gx, gy = rng.standard_normal((n, 3)), rng.standard_normal((n, 3))
    fbar, b1 = B().flux_average(c["mesh"], T(c, u), T(c, v), T(c, gx), T(c, gy))
    fbar, b1 = fbar.cpu().numpy(), b1.cpu().numpy()
    want = rt0.flux_average(c["geo"], u, v, gx, gy)
    tol = fbar_tol(c, u, v, gx, gy)
    assert np.all(np.abs(fbar - want) <= tol)
    assert np.all(np.abs(b1 - want.sum(axis=1)) <= tol.sum(axis=1) + 4 * U * np.abs(want).sum(axis=1))
    geo = c["geo"]
    e, j = np.nonzero(geo["interior"])
    assert np.array_equal(fbar[e, j], -fbar[geo["nbr"][e, j], geo["nbr_side"][e, j]])
    # null Dirichlet velocities are zeros; b1 may be omitted
    f0, _ = B().flux_average(c["mesh"], T(c, u), T(c, v))
    want0 = rt0.flux_average(c["geo"], u, v)
    assert np.all(np.abs(f0.cpu().numpy() - want0) <= fbar_tol(c, u, v, 0 * gx, 0 * gy))


def q_tol(c, fbar, eta, eta_t, g):
    w = c["w"]
    geo = c["geo"]
    sw = oasm.side_weights(geo, oasm.CP2, w["params"], w["nu"], w["dt"])["w"]
    o = np.maximum(geo["nbr"], 0)
    other = np.where(geo["interior"], np.abs(eta)[o], np.abs(g))
    split = ocf.conormal_split(geo, ocf.side_tensors(geo, w["params"], w["nu"], w["dt"]))
    est = ocf.tangential_estimates(geo, split, eta_t, g)
    _, S = ocf.tangential_terms(geo, est)
    return 32 * U * (np.abs(fbar) + np.abs(sw) * (np.abs(eta)[:, None] + other) + split["l"] * S)


@pytest.mark.parametrize("name", ["square", "channel"])
def test_rt0_update_matches_oracle(name):
    c = case(name)
    w = c["w"]
    n = c["n"]
    rng = np.random.default_rng(2)
    fbar = rng.standard_normal((n, 3))
    eta, eta_t = rng.standard_normal(n) + 1.0, rng.standard_normal(n) + 1.0
    g = rng.standard_normal((n, 3))
    u, v, q = B().rt0_update(c["mesh"], c["tprm"], w["nu"], w["dt"], T(c, eta_t), T(c, eta),
                             T(c, fbar), g_dirichlet=T(c, g))
    q = q.cpu().numpy()
    Qo = rt0.step_fluxes(c["geo"], w["params"], w["nu"], w["dt"], fbar, eta, eta_t, g)
    tq = q_tol(c, fbar, eta, eta_t, g)
    assert np.all(np.abs(q - Qo) <= tq)
    uo = rt0.rt0_velocity(c["geo"], Qo)
    P = c["geo"]["xy"][c["geo"]["tri"]]
    cen = P.mean(axis=1)
    A2 = 2 * c["geo"]["area"][:, None]
    arm = np.linalg.norm(cen[:, None, :] - P, axis=-1) / A2
    # the oracle forms x - x_j from node coordinates: its rounding is relative
    # to |x|, not to the cell size
    coord = 4 * U * (np.abs(P).sum(axis=-1) + np.abs(cen).sum(axis=-1)[:, None]) / A2
    tu = ((8 * U * np.abs(Qo) + tq) * arm + np.abs(Qo) * coord).sum(axis=1)
    assert np.all(np.abs(u.cpu().numpy() - uo[:, 0]) <= tu)
    assert np.all(np.abs(v.cpu().numpy() - uo[:, 1]) <= tu)


def test_rt0_update_errors():
    c = case("square")
    w = c["w"]
    n = c["n"]
    z = np.zeros(n)
    bad = z.copy()
    bad[3] = np.inf
    with pytest.raises(B().PMError) as ei:
        B().rt0_update(c["mesh"], c["tprm"], w["nu"], w["dt"], T(c, z), T(c, bad),
                       T(c, np.zeros((n, 3))))
    assert ei.value.status == B().PM_NONFINITE
    with pytest.raises(B().PMError) as ei:
        B().rt0_update(c["mesh"], c["tprm"], w["nu"], w["dt"], T(c, bad), T(c, z),
                       T(c, np.zeros((n, 3))))
    assert ei.value.status == B().PM_NONFINITE


def inflow_velocity(mesh_dict, n):
    """Prescribed velocity (1, 0) on the inflow sides x = 0, 0 elsewhere."""
    gx = np.where(mesh_dict["group"] == meshes.G_LEFT, 1.0, 0.0)
    return gx, np.zeros((n, 3))


def whole_step(c):
    """Coupled CP1 (block-Jacobi CG) -> averaged fluxes -> two CP2 solves ->
    RT0 velocity, every step on the GPU; returns what the checks need."""
    w = c["w"]
    nu, dt = w["nu"], w["dt"]
    n = c["n"]
    vx = B().assemble_corrector(c["mesh"], B().PM_CP1X, c["tprm"], nu, dt)["val64"]
    vy = B().assemble_corrector(c["mesh"], B().PM_CP1Y, c["tprm"], nu, dt)["val64"]
    u1, v1, i1 = B().cp1_solve_coupled_pcg(c["mesh"], c["tprm"], nu, dt, vx, vy,
                                           T(c, w["rhs"]["cp1x"]), T(c, w["rhs"]["cp1y"]))
    assert i1["status"] == 0
    gx, gy = inflow_velocity(w["mesh"], n)
    fbar, b1 = B().flux_average(c["mesh"], u1, v1, T(c, gx), T(c, gy))
    cp2 = B().assemble_corrector(c["mesh"], B().PM_CP2, c["tprm"], nu, dt, b_lift=True)
    b = b1 + cp2["b_lift"]
    eta, eta_t, infos = B().cp2_solve_two_step(c["mesh"], cp2["val64"], c["tprm"], nu, dt, b)
    assert [i["status"] for i in infos] == [0, 0]
    b2 = B().cp2_cross_rhs(c["mesh"], c["tprm"], nu, dt, eta_t, b)
    u2, v2, q = B().rt0_update(c["mesh"], c["tprm"], nu, dt, eta_t, eta, fbar)
    return {k: x.cpu().numpy() for k, x in
            dict(fbar=fbar, b1=b1, b2=b2, eta=eta, u2=u2, v2=v2, q=q).items()}


def check_step(c, out, A):
    geo = c["geo"]
    perm = c["perm"]
    q = out["q"]
    e, j = np.nonzero(geo["interior"])
    assert np.array_equal(q[e, j], -q[geo["nbr"][e, j], geo["nbr_side"][e, j]])
    res_vec = np.empty(c["n"])
    res_vec[perm] = opcg.true_residual(A, out["b2"][perm], out["eta"][perm])
    # rounding of the flux sums and of b2, and the oracle's matrix entries,
    # which match the GPU's weights to 1e-13 relative (assembly parity bound)
    aeta = np.empty(c["n"])
    aeta[perm] = abs(A) @ np.abs(out["eta"][perm])
    scale = (np.abs(out["fbar"]).sum(axis=1) + np.abs(q - out["fbar"]).sum(axis=1)
             + np.abs(out["b2"]) + aeta)
    assert np.all(np.abs(q.sum(axis=1) - res_vec) <= 1e-13 * scale)
    rel = np.linalg.norm(q.sum(axis=1)) / np.linalg.norm(out["b2"])
    assert rel <= 1.01e-10
    return rel


def test_whole_step_on_the_channel():
    c = case("channel")
    w = c["w"]
    A = oasm.assemble(c["geo"], c["perm"], oasm.CP2, w["params"], w["nu"], w["dt"])["A"]
    out = whole_step(c)
    check_step(c, out, A)
