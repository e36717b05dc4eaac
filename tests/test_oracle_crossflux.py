"""Pins for the oracle's CP2 cross terms (co-normal tangential fluxes) and the
right-hand side B_2 of the second CP2 solve (Sec. 3.2.3, eq. Cs2_7,
eq. eta_flux; App. C, eq. A3.1-A3.2)."""
import math

import numpy as np
import pytest

from oracle import assemble as asm
from oracle import crossflux as cf
from oracle import geometry, ordering, pcg
from synth import fields, meshes, workloads

NU, DT = 1.5e-5, 19.0


def aniso_params(n, beta=100.0, alpha_deg=30.0, eps=0.35, K=1e-4, rng=None):
    """Constant anisotropic cell data (rng: per-cell random data instead)."""
    g11, g12, g22 = fields.aniso_shape(beta, math.radians(alpha_deg))
    if rng is None:
        return {"eps": np.full(n, eps), "logk": np.full(n, math.log(K)), "chi": np.ones(n),
                "g11": np.full(n, g11), "g12": np.full(n, g12), "g22": np.full(n, g22)}
    ang = rng.uniform(0.0, math.pi, n)
    shp = [fields.aniso_shape(b, a) for b, a in zip(rng.uniform(1.0, 100.0, n), ang)]
    s = np.array(shp)
    return {"eps": rng.uniform(0.3, 1.0, n), "logk": np.log(rng.uniform(3e-5, 3e-4, n)),
            "chi": rng.uniform(0.0, 1.0, n), "g11": s[:, 0], "g12": s[:, 1], "g22": s[:, 2]}


def square(npts=12, seed=3, dirichlet_all=True):
    m = meshes.square_jittered_grid(npts, 0.3, seed)
    if dirichlet_all:
        cp2 = [meshes.G_LEFT, meshes.G_RIGHT, meshes.G_BOTTOM, meshes.G_TOP]
    else:
        cp2 = [meshes.G_RIGHT]
    tag = workloads.side_tags(m["group"], [], cp2)
    return m, geometry.build(m["xy"], m["tri"], tag)


def linear_field(geo, grad=(0.7, -1.3), c0=0.25):
    """eta = c0 + grad . x at circumcenters and at side midpoints."""
    cc = geometry.circumcenters(geo["xy"], geo["tri"])
    P = geo["xy"][geo["tri"]]
    mid = np.stack([0.5 * (P[:, (j + 1) % 3] + P[:, (j + 2) % 3]) for j in range(3)], axis=1)
    gx, gy = grad
    return c0 + gx * cc[:, 0] + gy * cc[:, 1], c0 + gx * mid[..., 0] + gy * mid[..., 1]


def test_conormal_split_identities():
    """d_j = d_{j,n} n_j + d_{j,tau}, d_{j,tau} is tangential, and the
    co-normal coefficients rebuild it from the other two sides' normals."""
    _, geo = square()
    prm = aniso_params(geo["n"], rng=np.random.default_rng(1))
    Xs = cf.side_tensors(geo, prm, NU, DT)
    sp = cf.conormal_split(geo, Xs)
    nrm = sp["n"]
    assert np.abs(np.einsum("eja,eja->ej", sp["dtau"], nrm)).max() < 1e-15 * np.abs(sp["d"]).max()
    rebuilt = np.einsum("eja,eaz->ejz", sp["c"], nrm)
    np.testing.assert_allclose(rebuilt, sp["dtau"], atol=1e-13 * np.abs(sp["d"]).max())
    assert np.all(sp["c"][:, [0, 1, 2], [0, 1, 2]] == 0)
    # normal part is the matrix's n.Xi.n (the quadratic form of the assembly)
    np.testing.assert_allclose(sp["dn"], np.einsum("eja,ejab,ejb->ej", nrm, Xs, nrm), rtol=1e-14)


def test_conormal_orthogonal_normals_reduce_to_projection():
    """Right angle at node 0: the normals of sides 1 and 2 are orthogonal, so
    the co-normal coefficients of side 0 are the plain projections."""
    xy = np.array([[0.0, 0.0], [2.0, 0.0], [0.0, 1.0]])
    tri = np.array([[0, 1, 2]])
    geo = geometry.build(xy, tri, np.zeros((1, 3), np.int8))
    prm = {"eps": np.array([0.5]), "logk": np.array([math.log(1e-4)]), "chi": np.array([1.0]),
           "g11": np.array([3.0]), "g12": np.array([0.8]), "g22": np.array([1.0])}
    sp = cf.conormal_split(geo, cf.side_tensors(geo, prm, NU, DT))
    for a in (1, 2):
        proj = sp["dtau"][0, 0] @ sp["n"][0, a]
        assert abs(sp["c"][0, 0, a] - proj) <= 1e-14 * abs(proj) + 1e-300
    assert abs(sp["c"][0, 0, 1]) > 0 and abs(sp["c"][0, 0, 2]) > 0


@pytest.mark.parametrize("grad", [(0.7, -1.3), (1.0, 0.0), (0.0, 1.0), (-2.0, 0.5)])
def test_side_flux_exact_for_linear_eta(grad):
    """With constant anisotropic Xi and linear eta, the discrete flux of every
    side (normal two-point part plus the tangential terms) equals
    l_j (Xi grad eta) . n_j; on an all-Dirichlet square every estimate exists.
    The reference value is computed from the gradient directly, without the
    co-normal decomposition."""
    _, geo = square()
    prm = aniso_params(geo["n"])
    eta, gmid = linear_field(geo, grad)
    Fl = cf.side_flux(geo, prm, NU, DT, eta, eta, gmid)
    ct = asm.cell_tensors(prm["eps"], prm["logk"], prm["chi"], prm["g11"], prm["g12"], prm["g22"], NU, DT)
    X = np.array([[ct["X11"][0], ct["X12"][0]], [ct["X12"][0], ct["X22"][0]]])
    t = geo["t"]
    N = np.stack([t[..., 1], -t[..., 0]], axis=-1)  # l_j n_j
    exact = N @ (X @ np.asarray(grad))
    scale = np.abs(N).sum(axis=-1) * np.abs(X @ np.asarray(grad)).max()
    assert np.all(cf.tangential_estimates(geo, cf.conormal_split(geo, cf.side_tensors(geo, prm, NU, DT)), eta, gmid)["avail"])
    err = np.abs(Fl - exact) / scale
    assert err.max() < 1e-8, err.max()
    # without the tangential terms the flux is wrong by O(1): the pin has teeth
    sp = cf.conormal_split(geo, cf.side_tensors(geo, prm, NU, DT))
    q, _, _ = cf.normal_derivatives(geo, eta, gmid)
    assert (np.abs(sp["l"] * sp["dn"] * q - exact) / scale).max() > 1e-2


def test_flux_continuity_and_boundary_rules():
    """T_j(e) = -T_{j'}(ep) bitwise on every interior side (eq. eta_flux gives
    a continuous flux); no tangential term on Neumann sides; estimates that
    need a Neumann side are unavailable."""
    _, geo = square(npts=14, dirichlet_all=False)
    rng = np.random.default_rng(7)
    prm = aniso_params(geo["n"], rng=rng)
    eta = rng.standard_normal(geo["n"])
    g = rng.standard_normal((geo["n"], 3))
    out = cf.cross_terms(geo, prm, NU, DT, eta, g)
    T = out["T"]
    e, j = np.nonzero(geo["interior"])
    ep, jp = geo["nbr"][e, j], geo["nbr_side"][e, j]
    assert np.array_equal(T[e, j], -T[ep, jp])
    neumann = (~geo["interior"]) & ((geo["tag"] & 2) == 0)
    assert np.all(T[neumann] == 0)
    avail = out["est"]["avail"]
    for c in range(geo["n"]):
        for k in range(3):
            others = [(k + 1) % 3, (k + 2) % 3]
            assert avail[c, k] == (not any(neumann[c, a] for a in others))
    # every availability branch occurs on this mesh
    a_e, a_p = avail[e, j], avail[ep, jp]
    for x, y in [(True, True), (True, False), (False, True)]:
        assert np.any((a_e == x) & (a_p == y))
    # interior sides sum to zero over the mesh; only Dirichlet sides remain
    l = out["split"]["l"]
    dirichlet = (~geo["interior"]) & ((geo["tag"] & 2) != 0)
    np.testing.assert_allclose(out["cross"].sum(), (l * T)[dirichlet].sum(),
                               atol=1e-12 * out["scale"].sum())


def test_isotropic_xi_gives_b2_equal_b1():
    """Isotropic (even heterogeneous) Xi has no tangential part: B_2 = B_1."""
    _, geo = square()
    rng = np.random.default_rng(2)
    n = geo["n"]
    prm = {"eps": rng.uniform(0.3, 1.0, n), "logk": np.log(rng.uniform(1e-5, 1e-3, n)),
           "chi": rng.uniform(0, 1, n), "g11": np.ones(n), "g12": np.zeros(n), "g22": np.ones(n)}
    eta = rng.standard_normal(n)
    out = cf.cross_terms(geo, prm, NU, DT, eta)
    # what an O(|d_j|) tangential part would give
    sp = out["split"]
    _, _, qabs = cf.normal_derivatives(geo, eta)
    ref = (sp["l"] * np.linalg.norm(sp["d"], axis=-1)).sum(axis=1) * qabs.sum(axis=1)
    assert np.abs(out["cross"]).max() <= 1e-14 * ref.max()


def test_linear_eta_solves_the_full_system():
    """eq. Cs2_6 / A3.3 with B_1 = 0 (div(Xi grad eta) = 0 for linear eta and
    constant Xi) and Dirichlet data g = eta on every boundary side: the linear
    field satisfies A eta - lift = sum_j l_j T_j(eta) at strong anisotropy
    (Xi eigenvalue ratio about 50)."""
    _, geo = square(npts=16, seed=5)
    n = geo["n"]
    prm = aniso_params(n)
    eta, gmid = linear_field(geo)
    out = asm.assemble(geo, np.arange(n), asm.CP2, prm, NU, DT, g_dirichlet=gmid)
    A, lift = out["A"], out["b_lift"]
    cr = cf.cross_terms(geo, prm, NU, DT, eta, gmid)
    res = A @ eta - lift - cr["cross"]
    assert np.abs(res).max() < 1e-8 * (np.abs(A) @ np.abs(eta)).max()
    # the two-point part alone is off by O(1) relative to the cross terms
    assert np.abs(A @ eta - lift).max() > 1e-2 * np.abs(cr["cross"]).max()


def test_two_solve_sequence_mild_anisotropy():
    """The sequence of eq. Cs2_7 is the first step of the fixed-point
    iteration eta <- A^{-1}(b + C eta); with mild anisotropy (Xi eigenvalue
    ratio 2) its contraction factor is below 1: the second solve moves eta~
    towards the linear solution and repeating it converges there."""
    _, geo = square(npts=16, seed=5)
    n = geo["n"]
    prm = aniso_params(n, beta=3.0)
    eta, gmid = linear_field(geo)
    out = asm.assemble(geo, np.arange(n), asm.CP2, prm, NU, DT, g_dirichlet=gmid)
    A, lift = out["A"], out["b_lift"]
    eta_t, eta2, _ = cf.two_step_dense(geo, A, prm, NU, DT, lift, gmid)
    e1 = np.abs(eta_t - eta).max()
    e2 = np.abs(eta2 - eta).max()
    assert e1 > 1e-3 * np.abs(eta).max()
    assert e2 < 0.3 * e1
    x = eta2
    for _ in range(40):
        x = pcg.dense_solve(A, cf.rhs_b2(geo, prm, NU, DT, x, lift, gmid))
    assert np.abs(x - eta).max() < 1e-10 * np.abs(eta).max()


def test_channel_aniso_cross_terms_nonzero_only_in_block():
    """On the channel workload the tangential terms vanish in the isotropic
    fluid and are nonzero inside the anisotropic block."""
    w = workloads.channel(n_rows=24, seed=2, aniso=True)
    m = w["mesh"]
    geo = geometry.build(m["xy"], m["tri"], w["side_tag"])
    rng = np.random.default_rng(0)
    eta = rng.standard_normal(geo["n"])
    out = cf.cross_terms(geo, w["params"], w["nu"], w["dt"], eta)
    aniso = w["params"]["chi"] > 0  # Kfrak = 0 where chi = 0: Xi = eps dt I
    touched = aniso | np.any(aniso[np.maximum(geo["nbr"], 0)] & geo["interior"], axis=1)
    assert np.abs(out["cross"][~touched]).max() <= 1e-14 * out["scale"].max()
    assert np.abs(out["cross"][aniso]).max() > 1e-6 * out["scale"].max()
