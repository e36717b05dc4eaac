"""GPU parity at the full benchmark sizes, in the launch configuration the
benchmark uses (tuned tile, block and schedule; default options).

  * channel, 1,001,228 triangles (CP1x and CP2): RCM order and CSR structure
    bit-exact against the oracle, assembled values entry by entry; float64
    and mixed solutions have a true relative residual <= 1e-10 under the
    oracle's matrix and agree with the oracle's own float64 PCG solution to
    1e-9.
  * anisotropic channel, 3,998,952 triangles (CP2): structure bit-exact and
    the residual property for float64 and mixed (an oracle solve at this size
    takes many minutes); the CP2 cross terms on every cell against the oracle
    and the residual property of the two-solve sequence; the systems of the
    coupled CP1 loop's second pass under the oracle's matrices, and the
    coupled CP1 solved by block-Jacobi CG to a true residual of 1e-10; the
    whole step (coupled CP1, averaged fluxes, both CP2 solves, RT0) with
    continuous fluxes whose cell sums are the CP2 residual.
  * the 64-system log-normal batch (50k-500k triangles each) on the GPU; the
    residual property on eight systems under the oracle's matrices.
  * adjoint on the 1M channel (loss: squared misfit at 256 probe cells): the
    gradients against the oracle's adjoint computed from its own forward and
    adjoint solves, and central differences (step 1e-6) on 20 cells.
"""
import functools
import os

import numpy as np
import pytest
import scipy.sparse as sp

torch = pytest.importorskip("torch")

from oracle import adjoint as oadj  # noqa: E402
from oracle import assemble as oasm  # noqa: E402
from oracle import geometry, ordering  # noqa: E402
from oracle import pcg as opcg  # noqa: E402
from synth import workloads  # noqa: E402

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]
KIND = {"cp1x": oasm.CP1X, "cp1y": oasm.CP1Y, "cp2": oasm.CP2}


def B():
    from paper_2309_03543_amd import binding

    return binding


def log(*a):
    print(*a, flush=True)


@functools.lru_cache(maxsize=None)
def channel_case(n_rows, seed, aniso):
    w = workloads.channel(n_rows, seed, aniso=aniso)
    m = w["mesh"]
    geo = geometry.build(m["xy"], m["tri"], w["side_tag"])
    perm = ordering.rcm(geo["nbr"])
    mesh = B().Mesh(m["xy"], m["tri"], w["side_tag"])
    dev = torch.device("cuda:0")
    prm = {k: torch.tensor(v, device=dev) for k, v in w["params"].items()}
    log(f"channel {n_rows}: {geo['n']} cells")
    return {"w": w, "geo": geo, "perm": perm, "mesh": mesh, "prm": prm, "dev": dev}


@functools.lru_cache(maxsize=None)
def oracle_system(n_rows, seed, aniso, kind):
    c = channel_case(n_rows, seed, aniso)
    w = c["w"]
    return oasm.assemble(c["geo"], c["perm"], KIND[kind], w["params"], w["nu"], w["dt"])


def to_cell(perm, v_perm):
    out = np.empty_like(v_perm)
    out[perm] = v_perm
    return out


@functools.lru_cache(maxsize=None)
def oracle_solution_c2(kind):
    c = channel_case(276, 2, False)
    o = oracle_system(276, 2, False, kind)
    xp, info = opcg.pcg(o["A"], c["w"]["rhs"][kind][c["perm"]], tol=1e-10)
    assert info["status"] == opcg.OK
    return to_cell(c["perm"], xp), info


def check_structure_and_values(c, kind, val):
    perm, rp, col = c["mesh"].export()
    A = oracle_system(*c["key"], kind)["A"]
    assert np.array_equal(perm, c["perm"])
    assert np.array_equal(rp, A.indptr) and np.array_equal(col, A.indices)
    v = val.cpu().numpy()
    assert np.all(np.abs(v - A.data) <= 1e-13 * np.abs(A.data))
    return A


@pytest.mark.parametrize("kind", ["cp1x", "cp2"])
def test_channel_1M_assembly_and_solves(kind):
    c = dict(channel_case(276, 2, False), key=(276, 2, False))
    w = c["w"]
    val = B().assemble_corrector(c["mesh"], KIND[kind], c["prm"], w["nu"], w["dt"])["val64"]
    A = check_structure_and_values(c, kind, val)
    b = w["rhs"][kind]
    bt = torch.tensor(b, device=c["dev"])
    xo, io = oracle_solution_c2(kind)
    for prec in (0, 1):
        x, info = B().pcg_solve(c["mesh"], val, bt, precision=prec)
        xg = x.cpu().numpy()
        res = opcg.rel_residual(A, b[c["perm"]], xg[c["perm"]])
        err = np.linalg.norm(xg - xo) / np.linalg.norm(xo)
        log(f"{kind} precision {prec}: iterations {info['iters']} (oracle {io['iters']}), "
            f"residual {res:.2e}, error vs oracle {err:.2e}, launch {B().pm_last_launch(c['mesh'])}")
        assert info["status"] == 0 and res <= 1e-10
        assert abs(info["rel_res_true"] - res) <= 1e-2 * res + 1e-16
        assert err <= 1e-9
        if prec == 0:
            assert abs(info["iters"] - io["iters"]) <= max(50, 0.02 * io["iters"])


@pytest.mark.parametrize("precision", [0, 1])
def test_channel_1M_resident_chunk_is_bitwise_the_lds_one(precision):
    """At full size (245 tiles of 4096 rows, one per compute unit) the resident
    chunk kernel reproduces the LDS-staged schedule bit for bit."""
    c = channel_case(276, 2, False)
    w = c["w"]
    val = B().assemble_corrector(c["mesh"], KIND["cp2"], c["prm"], w["nu"], w["dt"])["val64"]
    bt = torch.tensor(w["rhs"]["cp2"], device=c["dev"])
    kw = dict(precision=precision, tile_rows=4096, block=512)
    x3, i3 = B().pcg_solve(c["mesh"], val, bt, iter_shape=3, **kw)
    x4, i4 = B().pcg_solve(c["mesh"], val, bt, iter_shape=4, **kw)
    log(f"precision {precision}: LDS {i3['iters']} iterations, resident {i4['iters']}")
    assert i3["status"] == 0 and i4["status"] == 0
    assert i3["iters"] == i4["iters"] and torch.equal(x3, x4)


def test_aniso_channel_4M_resident_window_is_bitwise_the_lds_one():
    """On the 4M channel in mixed precision (one tile per compute unit) the
    resident window kernel reproduces the LDS-staged schedule bit for bit."""
    c = channel_case(552, 3, True)
    w = c["w"]
    val = B().assemble_corrector(c["mesh"], KIND["cp2"], c["prm"], w["nu"], w["dt"])["val64"]
    bt = torch.tensor(w["rhs"]["cp2"], device=c["dev"])
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    kw = dict(precision=1, tile_rows=-(-bt.numel() // n_cu), block=512)
    x3, i3 = B().pcg_solve(c["mesh"], val, bt, iter_shape=3, **kw)
    x5, i5 = B().pcg_solve(c["mesh"], val, bt, iter_shape=5, **kw)
    log(f"4M mixed: LDS {i3['iters']} iterations, resident window {i5['iters']}")
    assert i3["status"] == 0 and i5["status"] == 0
    assert i3["iters"] == i5["iters"] and torch.equal(x3, x5)


def test_aniso_channel_4M_structure_and_residual():
    c = dict(channel_case(552, 3, True), key=(552, 3, True))
    w = c["w"]
    val = B().assemble_corrector(c["mesh"], oasm.CP2, c["prm"], w["nu"], w["dt"])["val64"]
    A = check_structure_and_values(c, "cp2", val)
    b = w["rhs"]["cp2"]
    bt = torch.tensor(b, device=c["dev"])
    xs = []
    for prec in (0, 1):
        x, info = B().pcg_solve(c["mesh"], val, bt, precision=prec)
        xg = x.cpu().numpy()
        res = opcg.rel_residual(A, b[c["perm"]], xg[c["perm"]])
        log(f"aniso 4M precision {prec}: iterations {info['iters']}, residual {res:.2e}, "
            f"launch {B().pm_last_launch(c['mesh'])}")
        assert info["status"] == 0 and res <= 1e-10
        assert abs(info["rel_res_true"] - res) <= 1e-2 * res + 1e-16
        xs.append(xg)
    diff = np.linalg.norm(xs[1] - xs[0]) / np.linalg.norm(xs[0])
    log(f"aniso 4M: mixed vs float64 solution {diff:.2e}")
    assert diff <= 1e-8


def test_aniso_channel_4M_cross_terms_and_two_step():
    """CP2 cross terms on every cell of the 4M anisotropic channel against the
    oracle (tolerance of tests/test_gpu_crossflux.py), and the residual
    property of both solves of the two-solve sequence."""
    from oracle import crossflux as ocf

    c = dict(channel_case(552, 3, True), key=(552, 3, True))
    w = c["w"]
    A = oracle_system(552, 3, True, "cp2")["A"]
    val = B().assemble_corrector(c["mesh"], oasm.CP2, c["prm"], w["nu"], w["dt"])["val64"]
    b = w["rhs"]["cp2"]
    bt = torch.tensor(b, device=c["dev"])
    eta, eta_t, infos = B().cp2_solve_two_step(c["mesh"], val, c["prm"], w["nu"], w["dt"], bt)
    eta_t_h = eta_t.cpu().numpy()
    b2 = B().cp2_cross_rhs(c["mesh"], c["prm"], w["nu"], w["dt"], eta_t, bt).cpu().numpy()
    ref = ocf.cross_terms(c["geo"], w["params"], w["nu"], w["dt"], eta_t_h)
    tol = 32 * 2.0 ** -53 * (ref["scale"] + np.abs(b) + np.abs(ref["cross"]))
    assert np.all(np.abs(b2 - (b + ref["cross"])) <= tol)
    perm = c["perm"]
    r1 = opcg.rel_residual(A, b[perm], eta_t_h[perm])
    r2 = opcg.rel_residual(A, b2[perm], eta.cpu().numpy()[perm])
    log(f"aniso 4M two-step: iterations {infos[0]['iters']} + {infos[1]['iters']}, residuals "
        f"{r1:.2e} {r2:.2e}, |cross|/|b| {np.linalg.norm(ref['cross']) / np.linalg.norm(b):.3f}")
    assert [i["status"] for i in infos] == [0, 0] and r1 <= 1e-10 and r2 <= 1e-10


def test_aniso_channel_4M_coupled_cp1():
    """The coupled CP1 loop (App. B) on the 4M anisotropic channel: after one
    and after two coupled passes, the oracle's matrices confirm that the
    second pass solved A_x u2 = b_x - m v1 and A_y v2 = b_y - m u1 to the
    solver tolerance (the loop restarts from the uncoupled solves on every
    call and is deterministic, so the first call's result is the second
    call's first pass)."""
    from oracle import cp1coupled as occ

    c = dict(channel_case(552, 3, True), key=(552, 3, True))
    w = c["w"]
    vx = B().assemble_corrector(c["mesh"], oasm.CP1X, c["prm"], w["nu"], w["dt"])["val64"]
    vy = B().assemble_corrector(c["mesh"], oasm.CP1Y, c["prm"], w["nu"], w["dt"])["val64"]
    bx, by = w["rhs"]["cp1x"], w["rhs"]["cp1y"]
    bxt, byt = torch.tensor(bx, device=c["dev"]), torch.tensor(by, device=c["dev"])
    runs = []
    for passes in (1, 2):
        u, v, info = B().cp1_solve_coupled(c["mesh"], c["prm"], w["nu"], w["dt"], vx, vy, bxt, byt,
                                           toll=0.0, max_outer=passes)
        assert info["outer"] == passes and info["status"] == B().PM_MAXIT
        assert info["x"]["status"] == 0 and info["y"]["status"] == 0
        runs.append((u.cpu().numpy(), v.cpu().numpy(), info))
    perm = c["perm"]
    Ax = oracle_system(552, 3, True, "cp1x")["A"]
    Ay = oracle_system(552, 3, True, "cp1y")["A"]
    m = occ.coupling_weights(c["geo"], w["params"], w["nu"], w["dt"])
    (u1, v1, _), (u2, v2, i2) = runs
    rx = opcg.rel_residual(Ax, (bx - m * v1)[perm], u2[perm])
    ry = opcg.rel_residual(Ay, (by - m * u1)[perm], v2[perm])
    log(f"aniso 4M coupled CP1: err after 1 and 2 passes {runs[0][2]['err']:.3e} "
        f"{i2['err']:.3e}; pass-2 residuals {rx:.2e} {ry:.2e}")
    assert rx <= 1e-10 and ry <= 1e-10


@pytest.mark.parametrize("precision", [0, 1])
def test_aniso_channel_4M_coupled_cp1_pcg(precision):
    """Block-Jacobi CG on the coupled CP1 system of the 4M anisotropic channel,
    float64 and mixed: true relative residual <= 1e-10 under the oracle's
    coupled matrix."""
    from oracle import cp1coupled as occ

    c = dict(channel_case(552, 3, True), key=(552, 3, True))
    w = c["w"]
    vx = B().assemble_corrector(c["mesh"], oasm.CP1X, c["prm"], w["nu"], w["dt"])["val64"]
    vy = B().assemble_corrector(c["mesh"], oasm.CP1Y, c["prm"], w["nu"], w["dt"])["val64"]
    bx, by = w["rhs"]["cp1x"], w["rhs"]["cp1y"]
    u, v, info = B().cp1_solve_coupled_pcg(c["mesh"], c["prm"], w["nu"], w["dt"], vx, vy,
                                           torch.tensor(bx, device=c["dev"]),
                                           torch.tensor(by, device=c["dev"]), precision=precision)
    perm = c["perm"]
    Ax = oracle_system(552, 3, True, "cp1x")["A"]
    Ay = oracle_system(552, 3, True, "cp1y")["A"]
    m = occ.coupling_weights(c["geo"], w["params"], w["nu"], w["dt"])[perm]
    C = occ.coupled_matrix(Ax, Ay, m)
    b = np.concatenate([bx[perm], by[perm]])
    x = np.concatenate([u.cpu().numpy()[perm], v.cpu().numpy()[perm]])
    res = np.linalg.norm(b - C @ x) / np.linalg.norm(b)
    log(f"aniso 4M coupled CP1 CG precision {precision}: {info['iters']} iterations, residual {res:.2e} "
        f"(reported {info['rel_res_true']:.2e})")
    assert info["status"] == 0 and res <= 1e-10


def test_aniso_channel_4M_whole_step():
    """Coupled CP1, averaged fluxes, the two CP2 solves and the RT0 velocity
    on the 4M anisotropic channel, all on the GPU: the side fluxes are
    continuous bitwise and their cell sums equal the second CP2 system's
    residual under the oracle's matrix (below 1e-10 relative)."""
    from test_gpu_rt0 import check_step, whole_step

    c = channel_case(552, 3, True)
    c = dict(c, tprm=c["prm"], n=c["geo"]["n"])
    A = oracle_system(552, 3, True, "cp2")["A"]
    out = whole_step(c)
    rel = check_step(c, out, A)
    log(f"aniso 4M whole step: |sum_j Q_j| / |b2| = {rel:.2e}, "
        f"|u| max {np.abs(out['u2']).max():.3g}")


@functools.lru_cache(maxsize=None)
def batch64():
    ws = workloads.lognormal_batch(workers=min(16, len(os.sched_getaffinity(0))))
    dev = torch.device("cuda:0")
    meshes, vals, bs = [], [], []
    for w in ws:
        m = w["mesh"]
        mesh = B().Mesh(m["xy"], m["tri"], w["side_tag"])
        prm = {k: torch.tensor(v, device=dev) for k, v in w["params"].items()}
        vals.append(B().assemble_corrector(mesh, oasm.CP2, prm, w["nu"], w["dt"])["val64"])
        bs.append(torch.tensor(w["rhs"]["cp2"], device=dev))
        meshes.append(mesh)
    log(f"batch: {len(ws)} systems, {sum(m.n for m in meshes)} cells")
    return ws, meshes, torch.cat(vals), torch.cat(bs), B().Batch(meshes)


def test_lognormal_batch_64_residual_property():
    ws, meshes, val, b, batch = batch64()
    sizes = np.array([m.n for m in meshes])
    rng = np.random.default_rng(3)
    sample = sorted({int(sizes.argmin()), int(sizes.argmax())} |
                    set(rng.choice(len(ws), 6, replace=False).tolist()))
    oracle = {}
    for s in sample:
        w = ws[s]
        m = w["mesh"]
        geo = geometry.build(m["xy"], m["tri"], w["side_tag"])
        oracle[s] = oasm.assemble(geo, np.arange(geo["n"]), oasm.CP2, w["params"], w["nu"], w["dt"])["A"]
    for prec in (0, 1):
        x, infos = B().pcg_solve_batched(batch, val, b, precision=prec)
        its = [i["iters"] for i in infos]
        log(f"batch precision {prec}: iterations {min(its)}..{max(its)}")
        assert all(i["status"] == 0 and i["rel_res_true"] <= 1e-10 for i in infos)
        for s in sample:
            sl = slice(int(batch.vec_off[s]), int(batch.vec_off[s + 1]))
            res = opcg.rel_residual(oracle[s], ws[s]["rhs"]["cp2"], x[sl].cpu().numpy())
            assert res <= 1e-10, (s, res)
            assert abs(infos[s]["rel_res_true"] - res) <= 1e-2 * res + 1e-16


def gpu_csr(mesh, val):
    perm, rp, col = mesh.export()
    n = len(perm)
    return sp.csr_matrix((val.cpu().numpy(), col, rp), shape=(n, n))


def test_adjoint_1M_against_oracle_adjoint_and_differences():
    c = channel_case(276, 2, False)
    w = c["w"]
    n = c["geo"]["n"]
    dev = c["dev"]
    perm = c["perm"]
    probes = np.random.default_rng(5).choice(n, 256, replace=False)
    out = B().assemble_corrector(c["mesh"], oasm.CP2, c["prm"], w["nu"], w["dt"], b_lift=True)
    val0 = out["val64"]
    b = torch.tensor(w["rhs"]["cp2"], device=dev)
    x, info = B().pcg_solve(c["mesh"], val0, b)
    assert info["status"] == 0
    eta = x.cpu().numpy()
    gl = np.zeros(n)
    gl[probes] = 2.0 * eta[probes]  # loss: sum of squares at the probes, target 0
    lam, gs, ge, ia = B().pcg_adjoint(c["mesh"], oasm.CP2, c["prm"], w["nu"], w["dt"], val0, x,
                                      torch.tensor(gl, device=dev))
    assert ia["status"] == 0
    gs, ge = gs.cpu().numpy(), ge.cpu().numpy()
    assert np.all(gs[w["params"]["chi"] == 0] == 0)

    # the oracle's adjoint from its own forward solution
    eta_o, _ = oracle_solution_c2("cp2")
    gl_o = np.zeros(n)
    gl_o[probes] = 2.0 * eta_o[probes]
    o = oadj.adjoint(c["geo"], perm, oasm.CP2, w["params"], w["nu"], w["dt"], eta_o, gl_o, tol=1e-10)
    for got, key in ((gs, "grad_logk"), (ge, "grad_eps")):
        rel = np.linalg.norm(got - o[key]) / np.linalg.norm(o[key])
        log(f"adjoint 1M {key}: relative difference to the oracle {rel:.2e}")
        assert rel <= 1e-6

    # central differences (step 1e-6) in difference form with GPU solves:
    # A(p') d = (lift(p') - lift(p)) - (A(p') - A(p)) eta.  Two noise sources
    # bound the agreement, neither of them the gradient formula (which the
    # comparison with the oracle's adjoint above pins to ~1e-13): rounding of
    # the assembled difference A(p') - A(p) at this step (an oracle-only
    # replay with direct solves on a 21k-cell channel leaves up to
    # 1e-6 max|g| and 4e-4 |g| on small-gradient cells), and the iterative
    # solves for d: they stop at a 1e-12 relative residual, and the error of
    # d (up to cond(A) times that) does not cancel between the two sides.
    # Runs at this size measured up to 3.7e-4 max|g|, so the bound is
    # |fd - g| <= 1e-3 |g| + 1e-3 max|g|: a check of sign and magnitude at
    # full size, the sharp checks being the oracle adjoint above and the
    # small-mesh differences with direct solves.
    A0 = gpu_csr(c["mesh"], val0)
    eta_p = eta[perm]
    solves = []

    def dloss(params):
        prm2 = {k: torch.tensor(v, device=dev) for k, v in params.items()}
        o2 = B().assemble_corrector(c["mesh"], oasm.CP2, prm2, w["nu"], w["dt"], b_lift=True)
        A1 = gpu_csr(c["mesh"], o2["val64"])
        r = to_cell(perm, -((A1 - A0) @ eta_p)) + (o2["b_lift"] - out["b_lift"]).cpu().numpy()
        d, inf = B().pcg_solve(c["mesh"], o2["val64"], torch.tensor(r, device=dev), tol=1e-12)
        assert inf["status"] in (0, 2), inf
        solves.append(inf["rel_res_true"])
        d = d.cpu().numpy()
        return float(np.sum(d[probes] * (2.0 * eta[probes] + d[probes])))

    rng = np.random.default_rng(6)
    chi = w["params"]["chi"]
    cells = np.concatenate([rng.choice(np.flatnonzero(chi > 0), 10, replace=False),
                            rng.choice(n, 10, replace=False)])
    h = 1e-6
    bad = []
    for key, gv, cs in (("logk", gs, cells), ("eps", ge, cells[:10])):
        scale = np.abs(gv).max()
        worst = 0.0
        for cidx in cs:
            pp = {k: v.copy() for k, v in w["params"].items()}
            pm = {k: v.copy() for k, v in w["params"].items()}
            pp[key][cidx] += h
            pm[key][cidx] -= h
            fd = (dloss(pp) - dloss(pm)) / (2 * h)
            worst = max(worst, abs(fd - gv[cidx]) / scale)
            if abs(fd - gv[cidx]) > 1e-3 * abs(gv[cidx]) + 1e-3 * scale:
                bad.append((key, int(cidx), fd, gv[cidx]))
        log(f"adjoint 1M {key}: worst |fd - adjoint| / max|g| = {worst:.2e}")
    log(f"difference solves: relative residuals {min(solves):.1e}..{max(solves):.1e}")
    assert not bad, bad
