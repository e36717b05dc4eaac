"""GPU adjoint: pcg_adjoint against the CPU FP64 adjoint and against central
finite differences taken with GPU solves; the autograd wrapper reproduces it."""
import functools

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spl

torch = pytest.importorskip("torch")

from oracle import adjoint as oadj  # noqa: E402
from oracle import assemble as oasm  # noqa: E402
from oracle import geometry, ordering  # noqa: E402
from oracle import pcg as opcg  # noqa: E402
from synth import workloads  # noqa: E402

pytestmark = pytest.mark.gpu
TOL = 1e-11


def B():
    from paper_2309_03543_amd import binding

    return binding


@functools.lru_cache(maxsize=None)
def case(name):
    w = workloads.channel(30, 3, aniso=(name == "aniso"))
    m = w["mesh"]
    geo = geometry.build(m["xy"], m["tri"], w["side_tag"])
    perm = ordering.rcm(geo["nbr"])
    mesh = B().Mesh(m["xy"], m["tri"], w["side_tag"])
    dev = torch.device("cuda:0")
    n = geo["n"]
    rng = np.random.default_rng(5)
    probes = rng.choice(n, 64, replace=False)
    return {"w": w, "geo": geo, "perm": perm, "mesh": mesh, "dev": dev, "probes": probes,
            "target": rng.standard_normal(64) * 1e-3}


def forward(c, kind, params_np, g=None):
    w = c["w"]
    prm = {k: torch.tensor(v, device=c["dev"]) for k, v in params_np.items()}
    gd = None if g is None else torch.tensor(g, device=c["dev"])
    out = B().assemble_corrector(c["mesh"], kind, prm, w["nu"], w["dt"], g_dirichlet=gd, b_lift=True)
    rhs = torch.tensor(w["rhs"]["cp2" if kind == 2 else "cp1x"], device=c["dev"]) + out["b_lift"]
    x, info = B().pcg_solve(c["mesh"], out["val64"], rhs, tol=TOL)
    assert info["status"] == 0
    return prm, gd, out, rhs, x


@pytest.mark.parametrize("name,kind", [("iso", 2), ("aniso", 2), ("iso", 0), ("aniso", 1)])
def test_adjoint_matches_cpu_adjoint_and_finite_differences(name, kind):
    c = case(name)
    w = c["w"]
    n = c["geo"]["n"]
    g = np.zeros((n, 3))
    g[c["geo"]["tag"] != 0] = 0.01
    prm, gd, out, rhs, x = forward(c, kind, w["params"], g)
    eta = x.cpu().numpy()
    pr, tg = c["probes"], c["target"]
    gL = np.zeros(n)
    gL[pr] = 2 * (eta[pr] - tg)
    lam, gs, ge, info = B().pcg_adjoint(c["mesh"], kind, prm, w["nu"], w["dt"], out["val64"], x,
                                        torch.tensor(gL, device=c["dev"]), g_dirichlet=gd, tol=TOL)
    assert info["status"] == 0
    # CPU FP64 adjoint from the oracle's own forward solve (same inputs, no
    # GPU value enters the oracle)
    perm = c["perm"]
    ao = oasm.assemble(c["geo"], perm, kind, w["params"], w["nu"], w["dt"], g)
    rhs_o = w["rhs"]["cp2" if kind == 2 else "cp1x"] + ao["b_lift"]
    xp, io = opcg.pcg(ao["A"], rhs_o[perm], tol=TOL)
    assert io["status"] == opcg.OK
    eta_o = np.empty(n)
    eta_o[perm] = xp
    gL_o = np.zeros(n)
    gL_o[pr] = 2 * (eta_o[pr] - tg)
    o = oadj.adjoint(c["geo"], perm, kind, w["params"], w["nu"], w["dt"], eta_o, gL_o,
                     g_dirichlet=g, tol=TOL)
    # both sides solve forward and adjoint systems to a 1e-11 relative
    # residual; the solutions agree to ~1e-10 and the bilinear gradients to
    # a few 1e-9 on this mesh
    lam_g = lam.cpu().numpy()
    assert np.linalg.norm(lam_g - o["lambda"]) <= 1e-8 * np.linalg.norm(o["lambda"])
    for got, key in ((gs, "grad_logk"), (ge, "grad_eps")):
        ref = o[key]
        got = got.cpu().numpy()
        print(f"{name} kind {kind} {key}: relative difference {np.linalg.norm(got - ref) / np.linalg.norm(ref):.2e}")
        assert np.linalg.norm(got - ref) <= 1e-8 * np.linalg.norm(ref)
    if kind == 2:
        chi = w["params"]["chi"]
        assert np.all(gs.cpu().numpy()[chi == 0] == 0)

    # central differences (step 1e-6) in difference form on the GPU-assembled
    # matrices: A(p') d = (lift(p') - lift(p)) - (A(p') - A(p)) eta,
    # dL = sum d (2(eta - t) + d).  The small systems for d are solved by a
    # sparse direct solve, whose error (~u*cond) is far below the 1e-11
    # tolerance an iterative solve would need here.
    rp, colx = c["mesh"].export()[1:]
    A0 = sp.csr_matrix((out["val64"].cpu().numpy(), colx, rp), shape=(n, n))
    lift0 = out["b_lift"].cpu().numpy()

    def dloss(pp):
        prm2 = {k: torch.tensor(v, device=c["dev"]) for k, v in pp.items()}
        o2 = B().assemble_corrector(c["mesh"], kind, prm2, w["nu"], w["dt"], g_dirichlet=gd, b_lift=True)
        A1 = sp.csr_matrix((o2["val64"].cpu().numpy(), colx, rp), shape=(n, n))
        r_perm = -((A1 - A0) @ eta[perm])
        r = np.empty(n)
        r[perm] = r_perm
        r += o2["b_lift"].cpu().numpy() - lift0
        dp = spl.spsolve(A1.tocsc(), r[perm])
        d = np.empty(n)
        d[perm] = dp
        return float(np.sum(d[pr] * (2 * (eta[pr] - tg) + d[pr])))

    rng = np.random.default_rng(8)
    chi = w["params"]["chi"]
    cand = np.flatnonzero(chi > 0)
    cells = np.concatenate([rng.choice(cand, 10, replace=False), rng.choice(n, 10, replace=False)])
    gsn, gen = gs.cpu().numpy(), ge.cpu().numpy()
    for key, gv in (("logk", gsn), ("eps", gen)):
        scale = np.abs(gv).max()
        for cidx in cells[:10] if key == "eps" else cells:
            h = 1e-6
            pp = {k: v.copy() for k, v in w["params"].items()}
            pm = {k: v.copy() for k, v in w["params"].items()}
            pp[key][cidx] += h
            pm[key][cidx] -= h
            fd = (dloss(pp) - dloss(pm)) / (2 * h)
            # forward and adjoint solves stop at a 1e-11 relative residual, so both
            # the gradient and the difference quotient around eta carry errors of
            # order cond(A) * 1e-11 relative to the largest gradient: the same
            # check with the CPU oracle in place of every GPU step shows up to
            # 4e-6 * max|g| for CP2 and 1e-10 for CP1 on this mesh
            assert abs(fd - gv[cidx]) <= 1e-3 * abs(gv[cidx]) + 2e-5 * scale, (key, cidx, fd, gv[cidx])


def test_autograd_function_uses_the_adjoint():
    from paper_2309_03543_amd.autograd import SolveSpec, corrector_solve

    c = case("iso")
    w = c["w"]
    dev = c["dev"]
    logk = torch.tensor(w["params"]["logk"], device=dev, requires_grad=True)
    eps = torch.tensor(w["params"]["eps"], device=dev, requires_grad=True)
    b = torch.tensor(w["rhs"]["cp2"], device=dev, requires_grad=True)
    spec = SolveSpec(c["mesh"], 2, w["nu"], w["dt"], chi=torch.tensor(w["params"]["chi"], device=dev),
                     opts={"tol": TOL})
    eta = corrector_solve(logk, eps, b, spec)
    pr = torch.tensor(c["probes"], device=dev)
    loss = torch.sum((eta[pr] - torch.tensor(c["target"], device=dev)) ** 2)
    loss.backward()
    gL = torch.zeros_like(eta)
    gL[pr] = 2 * (eta.detach()[pr] - torch.tensor(c["target"], device=dev))
    prm = {"eps": eps.detach(), "logk": logk.detach(), "chi": spec.chi}
    val = B().assemble_corrector(c["mesh"], 2, prm, w["nu"], w["dt"])["val64"]
    lam, gs, ge, _ = B().pcg_adjoint(c["mesh"], 2, prm, w["nu"], w["dt"], val, eta.detach(), gL, tol=TOL)
    assert torch.equal(logk.grad, gs) and torch.equal(eps.grad, ge) and torch.equal(b.grad, lam)
