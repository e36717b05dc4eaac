"""Pins for the oracle's adjoint gradients (derivative closed forms, identity, FD)."""
import math

import numpy as np
import pytest

from oracle import adjoint as adj
from oracle import assemble as asm
from oracle import geometry, ordering, pcg
from synth import fields, meshes, workloads

NU, DT = 1.5e-5, 19.0


def params(n, seed, aniso):
    rng = np.random.default_rng(seed)
    p = {
        "eps": rng.uniform(0.3, 1.0, n), "logk": np.log(rng.uniform(1e-5, 1e-3, n)),
        "chi": np.where(rng.uniform(size=n) < 0.25, 0.0, rng.uniform(0.2, 1.0, n)),
        "g11": np.ones(n), "g12": np.zeros(n), "g22": np.ones(n),
    }
    if aniso:
        a, b, c = fields.aniso_shape(100.0, math.radians(30.0))
        p.update(g11=np.full(n, a), g12=np.full(n, b), g22=np.full(n, c))
    return p


@pytest.mark.parametrize("aniso", [False, True])
def test_tensor_derivatives_match_finite_differences(aniso):
    n = 50
    p = params(n, 1, aniso)
    td = adj.tensor_derivatives(p, NU, DT)
    for key, dname, mname in (("logk", "dXi_ds", "dM11_ds"), ("eps", "dXi_de", "dM11_de")):
        h = 1e-6 * np.maximum(1.0, np.abs(p[key]))
        pp, pm = dict(p), dict(p)
        pp[key] = p[key] + h
        pm[key] = p[key] - h
        a = asm.cell_tensors(**{k: pp[k] for k in ("eps", "logk", "chi", "g11", "g12", "g22")}, nu=NU, dt=DT)
        b = asm.cell_tensors(**{k: pm[k] for k in ("eps", "logk", "chi", "g11", "g12", "g22")}, nu=NU, dt=DT)
        for (i, j), comp in (((0, 0), "X11"), ((0, 1), "X12"), ((1, 1), "X22")):
            fd = (a[comp] - b[comp]) / (2 * h)
            scale = np.abs(a["X11"]) + np.abs(a["X22"])
            assert np.all(np.abs(td[dname][:, i, j] - fd) <= 1e-6 * scale)
        fd = (a["M11"] - b["M11"]) / (2 * h)
        assert np.all(np.abs(td[mname] - fd) <= 1e-6 * (np.abs(a["M11"])))


def setup(kind, aniso, npts=10):
    m = meshes.square_jittered_grid(npts, 0.3, 6)
    n = m["tri"].shape[0]
    tag = workloads.side_tags(m["group"], [meshes.G_LEFT, meshes.G_TOP], [meshes.G_RIGHT])
    geo = geometry.build(m["xy"], m["tri"], tag)
    perm = ordering.rcm(geo["nbr"])
    p = params(n, 2, aniso)
    b = np.random.default_rng(3).standard_normal(n)
    return geo, perm, p, b


def solve(geo, perm, kind, p, b, g=None):
    out = asm.assemble(geo, perm, kind, p, NU, DT, g)
    x = pcg.dense_solve(out["A"], (b + out["b_lift"])[perm])
    y = np.empty_like(x)
    y[perm] = x
    return y


@pytest.mark.parametrize("kind", [asm.CP1X, asm.CP2])
@pytest.mark.parametrize("aniso", [False, True])
def test_gradient_matches_central_differences(kind, aniso):
    geo, perm, p, b = setup(kind, aniso)
    n = geo["n"]
    rng = np.random.default_rng(9)
    probes = rng.choice(n, 12, replace=False)
    target = rng.standard_normal(12)
    g = np.zeros((n, 3))
    g[geo["tag"] != 0] = 0.5  # non-zero Dirichlet data exercises the lift term

    base = asm.assemble(geo, perm, kind, p, NU, DT, g)
    eta = solve(geo, perm, kind, p, b, g)
    gL = np.zeros(n)
    gL[probes] = 2 * (eta[probes] - target)
    out = adj.adjoint(geo, perm, kind, p, NU, DT, eta, gL, g_dirichlet=g, tol=1e-13)

    def delta_loss(pp):
        # difference form: A(p') d = (lift(p') - lift(p)) - (A(p') - A(p)) eta, no cancellation in L
        o = asm.assemble(geo, perm, kind, pp, NU, DT, g)
        rhs = (o["b_lift"] - base["b_lift"])[perm] - (o["A"] - base["A"]) @ eta[perm]
        dp = pcg.dense_solve(o["A"], rhs)
        d = np.empty_like(dp)
        d[perm] = dp
        return float(np.sum(d[probes] * (2 * (eta[probes] - target) + d[probes])))

    cells = rng.choice(n, 8, replace=False)
    for key, gname in (("logk", "grad_logk"), ("eps", "grad_eps")):
        for c in cells:
            # step 1e-5: truncation O(h^2) stays far below the round-off of the solves
            h = 1e-5 * max(1.0, abs(p[key][c]))
            pp, pm = {k: v.copy() for k, v in p.items()}, {k: v.copy() for k, v in p.items()}
            pp[key][c] += h
            pm[key][c] -= h
            fd = (delta_loss(pp) - delta_loss(pm)) / (2 * h)
            an = out[gname][c]
            assert abs(an - fd) <= 1e-6 * abs(fd) + 1e-8 * np.abs(out[gname]).max(), (key, c, an, fd)


def test_adjoint_identity_and_zero_fluid_gradient():
    geo, perm, p, b = setup(asm.CP2, False, npts=14)
    eta = solve(geo, perm, asm.CP2, p, b)
    gL = np.random.default_rng(4).standard_normal(geo["n"])
    out = adj.adjoint(geo, perm, asm.CP2, p, NU, DT, eta, gL, tol=1e-12)
    # A symmetric: lambda . b = g . eta
    lhs, rhs = float(out["lambda"] @ b), float(gL @ eta)
    assert abs(lhs - rhs) <= 1e-9 * (abs(lhs) + abs(rhs))
    # log-permeability does not act where chi = 0
    assert np.all(out["grad_logk"][p["chi"] == 0] == 0)
