"""GPU batched solve: each system against the single-system solve and the oracle."""
import functools

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import assemble as oasm  # noqa: E402
from oracle import geometry, ordering  # noqa: E402
from oracle import pcg as opcg  # noqa: E402
from synth import workloads  # noqa: E402

pytestmark = pytest.mark.gpu


def B():
    from paper_2309_03543_amd import binding

    return binding


@functools.lru_cache(maxsize=None)
def batch_case(n_sys=5, lo=2000, hi=12000, seed=11):
    ws = workloads.lognormal_batch(n_sys=n_sys, seed=seed, lo=lo, hi=hi)
    dev = torch.device("cuda:0")
    meshes, vals, bs, oracle = [], [], [], []
    for w in ws:
        m = w["mesh"]
        mesh = B().Mesh(m["xy"], m["tri"], w["side_tag"])
        prm = {k: torch.tensor(v, device=dev) for k, v in w["params"].items()}
        vals.append(B().assemble_corrector(mesh, B().PM_CP2, prm, w["nu"], w["dt"])["val64"])
        bs.append(torch.tensor(w["rhs"]["cp2"], device=dev))
        meshes.append(mesh)
        geo = geometry.build(m["xy"], m["tri"], w["side_tag"])
        perm = ordering.rcm(geo["nbr"])
        A = oasm.assemble(geo, perm, oasm.CP2, w["params"], w["nu"], w["dt"])["A"]
        oracle.append((perm, A, w["rhs"]["cp2"][perm]))
    batch = B().Batch(meshes)
    return {"ws": ws, "meshes": meshes, "vals": vals, "bs": bs, "batch": batch, "oracle": oracle}


def packed(c):
    return torch.cat(c["vals"]), torch.cat(c["bs"])


@pytest.mark.parametrize("precision", [0, 1])
def test_batched_matches_single_and_oracle(precision):
    c = batch_case()
    batch = c["batch"]
    assert batch.vec_off[-1] == sum(m.n for m in c["meshes"])
    val, b = packed(c)
    x, infos = B().pcg_solve_batched(batch, val, b, precision=precision)
    torch.cuda.synchronize()
    for s, (mesh, info) in enumerate(zip(c["meshes"], infos)):
        xs = x[batch.vec_off[s]: batch.vec_off[s + 1]]
        x1, i1 = B().pcg_solve(mesh, c["vals"][s], c["bs"][s], precision=precision)
        assert info["status"] == 0 and i1["status"] == 0
        assert abs(info["iters"] - i1["iters"]) <= 50
        perm, A, bo = c["oracle"][s]
        xg = xs.cpu().numpy()[perm]
        assert opcg.rel_residual(A, bo, xg) <= 1e-10
        assert abs(info["rel_res_true"] - opcg.rel_residual(A, bo, xg)) <= 1e-2 * info["rel_res_true"] + 1e-16
        ref = x1.cpu().numpy()[perm]
        assert np.linalg.norm(xg - ref) <= 1e-9 * np.linalg.norm(ref)
        if precision == 0:
            xo, io = opcg.pcg(A, bo, tol=1e-10)
            assert np.linalg.norm(xg - xo) <= 1e-9 * np.linalg.norm(xo)


def test_batched_replays_are_identical_and_masks_a_bad_system():
    c = batch_case()
    batch = c["batch"]
    val, b = packed(c)
    x1, i1 = B().pcg_solve_batched(batch, val, b)
    x2, i2 = B().pcg_solve_batched(batch, val, b)
    assert torch.equal(x1, x2) and [i["iters"] for i in i1] == [i["iters"] for i in i2]
    bad = b.clone()
    bad[int(batch.vec_off[2]) + 3] = float("nan")
    x3, i3 = B().pcg_solve_batched(batch, val, bad)
    for s in range(len(c["meshes"])):
        sl = slice(int(batch.vec_off[s]), int(batch.vec_off[s + 1]))
        if s == 2:
            assert i3[s]["status"] == B().PM_NONFINITE
        else:
            assert i3[s]["status"] == 0 and torch.equal(x3[sl], x1[sl])


def test_batched_iteration_limit():
    c = batch_case()
    val, b = packed(c)
    x, infos = B().pcg_solve_batched(c["batch"], val, b, max_it=20)
    assert all(i["status"] == B().PM_MAXIT and i["iters"] == 20 for i in infos)


@pytest.mark.parametrize("shape", [-1, 1, 2, 3])
def test_batched_schedules_agree(shape):
    # split schedule and fused kernels of several shapes, tiles straddling no
    # system: every system converges to the same solution
    c = batch_case()
    batch = c["batch"]
    val, b = packed(c)
    x1, i1 = B().pcg_solve_batched(batch, val, b)
    for tile, block in ((256, 64), (1024, 256), (2048, 512)):
        x2, i2 = B().pcg_solve_batched(batch, val, b, tile_rows=tile, block=block, iter_shape=shape)
        for s in range(len(c["meshes"])):
            sl = slice(int(batch.vec_off[s]), int(batch.vec_off[s + 1]))
            assert i2[s]["status"] == 0 and i2[s]["rel_res_true"] <= 1e-10
            assert torch.linalg.norm(x2[sl] - x1[sl]) <= 1e-9 * torch.linalg.norm(x1[sl])
            assert abs(i2[s]["iters"] - i1[s]["iters"]) <= 100


def test_batched_chebyshev_matches_single_solves():
    c = batch_case()
    batch = c["batch"]
    val, b = packed(c)
    cheb = dict(precond=B().PM_PREC_CHEBYSHEV, cheb_degree=4)
    for precision in (0, 1):
        x, infos = B().pcg_solve_batched(batch, val, b, precision=precision, **cheb)
        for s, mesh in enumerate(c["meshes"]):
            sl = slice(int(batch.vec_off[s]), int(batch.vec_off[s + 1]))
            x1, i1 = B().pcg_solve(mesh, c["vals"][s], c["bs"][s], precision=precision, **cheb)
            assert infos[s]["status"] == 0 and i1["status"] == 0
            assert abs(infos[s]["iters"] - i1["iters"]) <= 50
            perm, A, bo = c["oracle"][s]
            xg = x[sl].cpu().numpy()[perm]
            assert opcg.rel_residual(A, bo, xg) <= 1e-10
            ref = x1.cpu().numpy()[perm]
            assert np.linalg.norm(xg - ref) <= 1e-9 * np.linalg.norm(ref)


def few_cell_system(n_cells, dev):
    """One equilateral triangle, or two forming a rhombus, with every boundary
    side a Dirichlet side; per-cell parameters of the small inclusion
    workload.  Returns the mesh, matrix, right-hand side and oracle data."""
    import math

    h = math.sqrt(3.0) / 2
    xy = np.array([[0.0, 0.0], [1.0, 0.0], [0.5, h], [1.5, h]])[: n_cells + 2]
    tri = np.array([[0, 1, 2], [1, 3, 2]])[:n_cells]
    interior = geometry.build(xy, tri, np.zeros((n_cells, 3), np.int8))["interior"]
    tag = np.where(interior, 0, 3).astype(np.int8)
    geo = geometry.build(xy, tri, tag)
    perm = ordering.rcm(geo["nbr"])
    w = workloads.square_inclusion(npts=5, seed=2)
    params = {k: np.ascontiguousarray(v[:n_cells]) for k, v in w["params"].items()}
    mesh = B().Mesh(xy, tri, tag)
    prm = {k: torch.tensor(v, device=dev) for k, v in params.items()}
    val = B().assemble_corrector(mesh, B().PM_CP2, prm, w["nu"], w["dt"])["val64"]
    b = np.random.default_rng(7 + n_cells).standard_normal(n_cells)
    A = oasm.assemble(geo, perm, oasm.CP2, params, w["nu"], w["dt"])["A"]
    return mesh, val, torch.tensor(b, device=dev), (perm, A, b[perm])


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_with_one_and_two_cell_systems(precision):
    """A 1-cell, a larger and a 2-cell system in one batch.  The small systems
    end their recursion before the first convergence test (a zero residual or
    p.q = 0), and in float32 storage are solved on from their iterate; the
    larger one is unaffected.  Each matches its single solve and the oracle."""
    dev = torch.device("cuda:0")
    big = batch_case()
    parts = [few_cell_system(1, dev),
             (big["meshes"][0], big["vals"][0], big["bs"][0], big["oracle"][0]),
             few_cell_system(2, dev)]
    batch = B().Batch([p[0] for p in parts])
    val = torch.cat([p[1] for p in parts])
    b = torch.cat([p[2] for p in parts])
    x, infos = B().pcg_solve_batched(batch, val, b, precision=precision)
    torch.cuda.synchronize()
    for s, (mesh, v, bs, (perm, A, bo)) in enumerate(parts):
        info = infos[s]
        xg = x[batch.vec_off[s]: batch.vec_off[s + 1]].cpu().numpy()[perm]
        assert info["status"] == 0
        assert opcg.rel_residual(A, bo, xg) <= 1e-10
        x1, i1 = B().pcg_solve(mesh, v, bs, precision=precision)
        assert i1["status"] == 0
        ref = x1.cpu().numpy()[perm]
        assert np.linalg.norm(xg - ref) <= 1e-9 * np.linalg.norm(ref)
        if precision == 0:
            xo, io = opcg.pcg(A, bo, tol=1e-10)
            assert io["status"] == opcg.OK
            assert np.linalg.norm(xg - xo) <= 1e-9 * np.linalg.norm(xo)
