"""GPU parity: the HIP library against the CPU oracle on the same seeded inputs.

Tolerances
  * CSR structure and ordering: bit-exact (integer work).
  * Assembled values: |gpu - oracle| <= 1e-13 |oracle| per entry (the two
    differ only in the rounding of exp and the order of a few products).
  * FP64 and mixed solves: true relative residual <= 1e-10 (evaluated by the
    oracle on the GPU solution) and relative error <= 1e-9 against the oracle's
    float64 solution; iteration counts within one replacement period.
"""
import functools
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import assemble as oasm  # noqa: E402
from oracle import geometry, ordering  # noqa: E402
from oracle import pcg as opcg  # noqa: E402
from synth import meshes, workloads  # noqa: E402

pytestmark = pytest.mark.gpu

KIND = {"cp1x": oasm.CP1X, "cp1y": oasm.CP1Y, "cp2": oasm.CP2}


def B():
    from paper_2309_03543_amd import binding

    return binding


@functools.lru_cache(maxsize=None)
def case(name):
    if name == "c1":
        w = workloads.square_inclusion()
    elif name == "chan":
        w = workloads.channel(30, 2)
    elif name == "aniso":
        w = workloads.channel(30, 3, aniso=True)
    elif name == "tiny":
        w = workloads.square_inclusion(npts=5, seed=2)
    else:
        raise KeyError(name)
    m = w["mesh"]
    geo = geometry.build(m["xy"], m["tri"], w["side_tag"])
    perm = ordering.rcm(geo["nbr"])
    mesh = B().Mesh(m["xy"], m["tri"], w["side_tag"])
    dev = torch.device("cuda:0")
    prm = {k: torch.tensor(v, device=dev) for k, v in w["params"].items()}
    return {"w": w, "geo": geo, "perm": perm, "mesh": mesh, "prm": prm, "dev": dev}


def oracle_matrix(c, kind, g=None):
    w = c["w"]
    return oasm.assemble(c["geo"], c["perm"], KIND[kind], w["params"], w["nu"], w["dt"], g)


def to_perm(c, v):
    return np.asarray(v)[c["perm"]]


@pytest.mark.parametrize("name", ["c1", "chan", "aniso", "tiny"])
def test_structure_export_matches_oracle(name):
    c = case(name)
    perm, rp, col = c["mesh"].export()
    rp2, col2 = ordering.csr_pattern(c["geo"]["nbr"], c["perm"])
    assert np.array_equal(perm, c["perm"]) and np.array_equal(rp, rp2) and np.array_equal(col, col2)


@pytest.mark.parametrize("name", ["c1", "chan", "aniso"])
@pytest.mark.parametrize("kind", ["cp1x", "cp1y", "cp2"])
def test_assembly_matches_oracle(name, kind):
    c = case(name)
    w = c["w"]
    n = c["geo"]["n"]
    g = np.random.default_rng(5).standard_normal((n, 3))
    o = oracle_matrix(c, kind, g)
    gd = torch.tensor(g, device=c["dev"])
    out = B().assemble_corrector(c["mesh"], KIND[kind], c["prm"], w["nu"], w["dt"], g_dirichlet=gd,
                                 val32=True, dinv=True, b_lift=True)
    v = out["val64"].cpu().numpy()
    ref = o["A"].data
    assert np.all(np.abs(v - ref) <= 1e-13 * np.abs(ref))
    # one weight per side: the GPU matrix is bitwise symmetric
    import scipy.sparse as sp

    A = sp.csr_matrix((v, o["A"].indices, o["A"].indptr), shape=o["A"].shape)
    assert (A != A.T).nnz == 0
    assert np.array_equal(out["val32"].cpu().numpy(), v.astype(np.float32))
    np.testing.assert_array_equal(out["dinv"].cpu().numpy(), 1.0 / A.diagonal())
    bl = out["b_lift"].cpu().numpy()
    assert np.all(np.abs(bl - o["b_lift"]) <= 1e-13 * np.abs(o["b_lift"]) + 1e-300)


def solve_both(name, kind, precision, rhs=None, **kw):
    c = case(name)
    w = c["w"]
    A = oracle_matrix(c, kind)["A"]
    b = w["rhs"][rhs or ("cp1x" if kind.startswith("cp1") else "cp2")]
    val = B().assemble_corrector(c["mesh"], KIND[kind], c["prm"], w["nu"], w["dt"])["val64"]
    bt = torch.tensor(b, device=c["dev"])
    x, info = B().pcg_solve(c["mesh"], val, bt, precision=precision, **kw)
    torch.cuda.synchronize()
    xo, io = opcg.pcg(A, to_perm(c, b), tol=kw.get("tol", 1e-10), max_it=kw.get("max_it", 100000),
                      replace_every=kw.get("replace_every", 50), stag_checks=kw.get("stag_checks", 40),
                      precond=kw.get("precond", 0), degree=kw.get("cheb_degree", 4))
    return c, A, to_perm(c, b), to_perm(c, x.cpu().numpy()), info, xo, io


@pytest.mark.parametrize("name,kind", [("c1", "cp2"), ("chan", "cp2"), ("chan", "cp1x"),
                                       ("aniso", "cp2"), ("aniso", "cp1y"), ("tiny", "cp2")])
def test_fp64_solve_matches_oracle(name, kind):
    c, A, b, xg, info, xo, io = solve_both(name, kind, 0)
    assert info["status"] == 0 and io["status"] == 0
    res = opcg.rel_residual(A, b, xg)
    assert res <= 1e-10
    assert abs(info["rel_res_true"] - res) <= 1e-2 * res + 1e-16
    assert np.linalg.norm(xg - xo) <= 1e-9 * np.linalg.norm(xo)
    assert abs(info["iters"] - io["iters"]) <= max(50, 0.02 * io["iters"])


@pytest.mark.parametrize("name,kind", [("c1", "cp2"), ("chan", "cp2"), ("aniso", "cp2"), ("chan", "cp1x")])
def test_mixed_solve_reaches_fp64_accuracy(name, kind):
    c, A, b, xg, info, xo, io = solve_both(name, kind, 1)
    assert info["status"] == 0
    res = opcg.rel_residual(A, b, xg)
    assert res <= 1e-10
    err = np.linalg.norm(xg - xo) / np.linalg.norm(xo)
    print(f"mixed {name} {kind}: iters {info['iters']} vs fp64 oracle {io['iters']}, err {err:.2e}")
    assert err <= 1e-9


@pytest.mark.parametrize("m", [1, 2, 7, 50])
def test_replacement_period_odd_and_even(m):
    # each chunk alternates the iteration buffers m - 1 times; odd and even m
    # end the chunk in different buffers
    for prec in (0, 1):
        c, A, b, xg, info, xo, io = solve_both("chan", "cp2", prec, replace_every=m)
        assert info["status"] == 0 and io["status"] == 0
        assert opcg.rel_residual(A, b, xg) <= 1e-10
        assert np.linalg.norm(xg - xo) <= 1e-9 * np.linalg.norm(xo)
        if prec == 0:
            assert abs(info["iters"] - io["iters"]) <= max(2 * m, 0.02 * io["iters"])


@pytest.mark.parametrize("name,kind,degree", [("c1", "cp2", 4), ("chan", "cp2", 2), ("chan", "cp2", 8),
                                              ("chan", "cp1x", 4), ("aniso", "cp2", 5), ("tiny", "cp2", 3)])
def test_chebyshev_solve_matches_oracle(name, kind, degree):
    cheb = dict(precond=B().PM_PREC_CHEBYSHEV, cheb_degree=degree)
    c, A, b, xg, info, xo, io = solve_both(name, kind, 0, **cheb)
    assert info["status"] == 0 and io["status"] == 0
    res = opcg.rel_residual(A, b, xg)
    assert res <= 1e-10 and abs(info["rel_res_true"] - res) <= 1e-2 * res + 1e-16
    assert np.linalg.norm(xg - xo) <= 1e-9 * np.linalg.norm(xo)
    assert abs(info["iters"] - io["iters"]) <= max(50, 0.02 * io["iters"])
    # mixed precision with the same preconditioner reaches the same accuracy
    c, A, b, xm, im, _, _ = solve_both(name, kind, 1, **cheb)
    assert im["status"] == 0 and opcg.rel_residual(A, b, xm) <= 1e-10
    assert np.linalg.norm(xm - xo) <= 1e-9 * np.linalg.norm(xo)
    print(f"chebyshev {degree} {name} {kind}: iters {info['iters']} (oracle {io['iters']}), mixed {im['iters']}")


@pytest.mark.parametrize("m", [1, 7])
def test_chebyshev_odd_replacement_periods_and_limit(m):
    cheb = dict(precond=B().PM_PREC_CHEBYSHEV, cheb_degree=3, replace_every=m)
    c, A, b, xg, info, xo, io = solve_both("chan", "cp2", 0, **cheb)
    assert info["status"] == 0 and opcg.rel_residual(A, b, xg) <= 1e-10
    assert np.linalg.norm(xg - xo) <= 1e-9 * np.linalg.norm(xo)
    c, A, b, xg, info, xo, io = solve_both("c1", "cp2", 0, max_it=11, **cheb)
    assert info["status"] == B().PM_MAXIT and info["iters"] == 11 and io["iters"] == 11
    assert np.linalg.norm(xg - xo) <= 1e-10 * np.linalg.norm(xo)


def test_iteration_limit_and_partial_iterate():
    c, A, b, xg, info, xo, io = solve_both("c1", "cp2", 0, max_it=7)
    assert info["status"] == B().PM_MAXIT and info["iters"] == 7
    assert io["status"] == opcg.MAXIT and io["iters"] == 7
    assert np.linalg.norm(xg - xo) <= 1e-10 * np.linalg.norm(xo)


def test_warm_start_and_zero_rhs():
    c = case("c1")
    w = c["w"]
    val = B().assemble_corrector(c["mesh"], B().PM_CP2, c["prm"], w["nu"], w["dt"])["val64"]
    b = torch.tensor(w["rhs"]["cp2"], device=c["dev"])
    x, info = B().pcg_solve(c["mesh"], val, b)
    x2, info2 = B().pcg_solve(c["mesh"], val, b, x=x.clone(), x0_is_zero=False)
    assert info2["iters"] == 0 and info2["status"] == 0
    z = torch.zeros_like(b)
    x3, info3 = B().pcg_solve(c["mesh"], val, z, x=torch.ones_like(b), x0_is_zero=False)
    assert info3["status"] == 0 and info3["iters"] == 0 and not torch.any(x3)


def test_solves_are_deterministic_and_launch_shape_independent():
    c = case("chan")
    w = c["w"]
    val = B().assemble_corrector(c["mesh"], B().PM_CP2, c["prm"], w["nu"], w["dt"])["val64"]
    b = torch.tensor(w["rhs"]["cp2"], device=c["dev"])
    x1, i1 = B().pcg_solve(c["mesh"], val, b)
    x2, i2 = B().pcg_solve(c["mesh"], val, b)
    assert torch.equal(x1, x2) and i1["iters"] == i2["iters"]
    for prec in (0, 1):
        xr, ir = B().pcg_solve(c["mesh"], val, b, precision=prec)
        for tile, block, shape in ((256, 256, 1), (768, 64, 2), (4096, 512, 1), (1024, 256, -1),
                                   (512, 128, -1), (2048, 256, 2), (1024, 192, 1), (1024, 256, 3),
                                   (2048, 512, 3), (300, 64, 3), (1024, 256, 4), (2048, 256, 4),
                                   (300, 64, 4)):
            x3, i3 = B().pcg_solve(c["mesh"], val, b, precision=prec, tile_rows=tile, block=block,
                                   iter_shape=shape)
            assert i3["status"] == 0
            assert torch.linalg.norm(x3 - xr) <= 1e-9 * torch.linalg.norm(xr)
            assert B().pm_last_launch(c["mesh"]) == {"tile_rows": tile, "block": block,
                                                      "iter_shape": shape}
            x4, i4 = B().pcg_solve(c["mesh"], val, b, precision=prec, tile_rows=tile, block=block,
                                   iter_shape=shape)
            assert torch.equal(x3, x4) and i3["iters"] == i4["iters"]


def test_lds_staged_iteration_is_bitwise_the_gather_one():
    c = case("chan")
    w = c["w"]
    val = B().assemble_corrector(c["mesh"], B().PM_CP2, c["prm"], w["nu"], w["dt"])["val64"]
    b = torch.tensor(w["rhs"]["cp2"], device=c["dev"])
    for prec in (0, 1):
        for tile, block in ((1024, 256), (2048, 512)):
            x1, i1 = B().pcg_solve(c["mesh"], val, b, precision=prec, tile_rows=tile, block=block,
                                   iter_shape=1)
            x3, i3 = B().pcg_solve(c["mesh"], val, b, precision=prec, tile_rows=tile, block=block,
                                   iter_shape=3)
            assert i1["status"] == 0 and torch.equal(x1, x3) and i1["iters"] == i3["iters"]


def test_resident_chunk_is_bitwise_the_lds_one():
    """The resident chunk kernel (iter_shape 4: a chunk's m - 1 iterations in
    one launch, the tiles' rows held on chip, a grid barrier between
    iterations) and the resident window kernel (iter_shape 5: only the
    windows' p and z on chip) give bitwise the solutions and iteration
    counts of the LDS-staged kernel at the same tiles: both precisions,
    tiles of 4, 8 and (shape 5) 10 rows per thread, chunks of 50, 7, 2 and 1
    iterations, and an iteration limit that stops inside a chunk."""
    for name in ("chan", "aniso"):
        c = case(name)
        w = c["w"]
        val = B().assemble_corrector(c["mesh"], B().PM_CP2, c["prm"], w["nu"], w["dt"])["val64"]
        b = torch.tensor(w["rhs"]["cp2"], device=c["dev"])
        for prec in (0, 1):
            for tile, block in ((1024, 256), (2048, 256), (2048, 512), (512, 128), (5000, 512)):
                for m in (50, 7, 2, 1):
                    kw = dict(precision=prec, tile_rows=tile, block=block, replace_every=m)
                    x3, i3 = B().pcg_solve(c["mesh"], val, b, iter_shape=3, **kw)
                    assert i3["status"] == 0
                    # shape 4 holds at most 8 rows per thread; shape 5 any tile
                    for shape in ((4, 5) if tile <= 8 * block else (5,)):
                        x4, i4 = B().pcg_solve(c["mesh"], val, b, iter_shape=shape, **kw)
                        assert i4["status"] == 0
                        assert i3["iters"] == i4["iters"] and torch.equal(x3, x4), (
                            name, prec, tile, block, m, shape)
            kw = dict(precision=prec, tile_rows=2048, block=256, max_it=73)
            x3, i3 = B().pcg_solve(c["mesh"], val, b, iter_shape=3, **kw)
            for shape in (4, 5):
                x4, i4 = B().pcg_solve(c["mesh"], val, b, iter_shape=shape, **kw)
                assert i3["status"] == i4["status"] == B().PM_MAXIT
                assert i3["iters"] == i4["iters"] and torch.equal(x3, x4)
    # more than eight rows per thread is not a resident shape
    c = case("chan")
    w = c["w"]
    val = B().assemble_corrector(c["mesh"], B().PM_CP2, c["prm"], w["nu"], w["dt"])["val64"]
    b = torch.tensor(w["rhs"]["cp2"], device=c["dev"])
    with pytest.raises(B().PMError) as e:
        B().pcg_solve(c["mesh"], val, b, tile_rows=4096, block=256, iter_shape=4)
    assert e.value.status == B().PM_INVALID_ARG and "resident" in str(e.value)
    x, info = B().pcg_solve(c["mesh"], val, b, tile_rows=2048, block=256, iter_shape=4)
    assert info["status"] == 0


def test_resident_barrier_that_gives_up_falls_back_to_streaming(monkeypatch):
    """With the barrier's wait bound set to zero polls every wait of a
    resident kernel (schedules 4 and 5) gives up, each block then exiting
    normally; the solve is redone on the LDS schedule with the same tiles and
    matches it bitwise."""
    c = case("chan")
    w = c["w"]
    val = B().assemble_corrector(c["mesh"], B().PM_CP2, c["prm"], w["nu"], w["dt"])["val64"]
    b = torch.tensor(w["rhs"]["cp2"], device=c["dev"])
    kw = dict(tile_rows=2048, block=256)
    x3, i3 = B().pcg_solve(c["mesh"], val, b, iter_shape=3, **kw)
    for shape in (4, 5):
        monkeypatch.setenv("PMCORR_RESIDENT_SPINS", "0")
        x4, i4 = B().pcg_solve(c["mesh"], val, b, iter_shape=shape, **kw)
        assert i4["status"] == 0 and i4["iters"] == i3["iters"] and torch.equal(x3, x4)
        assert B().pm_last_launch(c["mesh"])["iter_shape"] == 3
        monkeypatch.delenv("PMCORR_RESIDENT_SPINS")
        x5, i5 = B().pcg_solve(c["mesh"], val, b, iter_shape=shape, **kw)
        assert B().pm_last_launch(c["mesh"])["iter_shape"] == shape
        assert i5["iters"] == i3["iters"] and torch.equal(x3, x5)


def test_kernel_timing_hook_on_every_schedule():
    """pm_time_kernel times the last solve's kernels and returns the bytes its
    header documents; on the resident schedule it times chunk-length launches
    and returns the time per iteration.  Solves after the timing give the
    same answer as before it."""
    c = case("chan")
    w = c["w"]
    val = B().assemble_corrector(c["mesh"], B().PM_CP2, c["prm"], w["nu"], w["dt"])["val64"]
    b = torch.tensor(w["rhs"]["cp2"], device=c["dev"])
    n = c["geo"]["n"]
    for prec, sv in ((0, 8), (1, 4)):
        for shape in (-1, 1, 3, 4, 5):
            kw = dict(precision=prec, tile_rows=2048, block=256, iter_shape=shape)
            x1, i1 = B().pcg_solve(c["mesh"], val, b, **kw)
            for which, reps in ((0, 20), (1, 4), (2, 5)):
                ms, by = B().pm_time_kernel(c["mesh"], which, reps)
                assert math.isfinite(ms) and 0.0 < ms < 50.0
                if which == 0:
                    assert by == n * (4 * sv + 3 * 2 + 3 * sv)
                elif which == 1:
                    assert by == n * (4 * sv + 3 * 2 + (10 if shape == -1 else 8) * sv)
            x2, i2 = B().pcg_solve(c["mesh"], val, b, **kw)
            assert torch.equal(x1, x2) and i1["iters"] == i2["iters"]


@functools.lru_cache(maxsize=None)
def few_cells(n_cells):
    """One equilateral triangle, or two forming a rhombus; every boundary side
    is a Dirichlet side of both problems; per-cell parameters of the small
    inclusion workload."""
    h = math.sqrt(3.0) / 2
    xy = np.array([[0.0, 0.0], [1.0, 0.0], [0.5, h], [1.5, h]])[: n_cells + 2]
    tri = np.array([[0, 1, 2], [1, 3, 2]])[:n_cells]
    interior = geometry.build(xy, tri, np.zeros((n_cells, 3), np.int8))["interior"]
    tag = np.where(interior, 0, 3).astype(np.int8)
    geo = geometry.build(xy, tri, tag)
    w = workloads.square_inclusion(npts=5, seed=2)
    params = {k: np.ascontiguousarray(v[:n_cells]) for k, v in w["params"].items()}
    dev = torch.device("cuda:0")
    return {"geo": geo, "perm": ordering.rcm(geo["nbr"]), "mesh": B().Mesh(xy, tri, tag),
            "params": params, "prm": {k: torch.tensor(v, device=dev) for k, v in params.items()},
            "nu": w["nu"], "dt": w["dt"], "dev": dev}


@pytest.mark.parametrize("n_cells", [1, 2])
@pytest.mark.parametrize("kind", ["cp1x", "cp2"])
def test_one_and_two_cell_systems(n_cells, kind):
    """The smallest meshes: assembly to the oracle's values, and every schedule
    in both precisions converges (CG ends within n iterations, before the
    first convergence test) to the oracle's solution."""
    c = few_cells(n_cells)
    A = oasm.assemble(c["geo"], c["perm"], KIND[kind], c["params"], c["nu"], c["dt"])["A"]
    val = B().assemble_corrector(c["mesh"], KIND[kind], c["prm"], c["nu"], c["dt"])["val64"]
    assert np.all(np.abs(val.cpu().numpy() - A.data) <= 1e-13 * np.abs(A.data))
    b = np.random.default_rng(n_cells).standard_normal(n_cells)
    bp = b[c["perm"]]
    xo, io = opcg.pcg(A, bp, tol=1e-10)
    assert io["status"] == opcg.OK
    bt = torch.tensor(b, device=c["dev"])
    shapes = [{}] + [dict(tile_rows=256, block=256, iter_shape=s) for s in (-1, 0, 1, 2, 3, 4, 5)]
    for prec in (0, 1):
        for shape in shapes:
            print(f"== cells {n_cells} {kind} precision {prec} {shape}", flush=True)
            x, info = B().pcg_solve(c["mesh"], val, bt, precision=prec, **shape)
            xg = x.cpu().numpy()[c["perm"]]
            assert info["status"] == 0
            assert opcg.rel_residual(A, bp, xg) <= 1e-10
            assert np.linalg.norm(xg - xo) <= 1e-9 * np.linalg.norm(xo)


def test_error_statuses():
    Bm = B()
    c = case("tiny")
    w = c["w"]
    bad = dict(c["prm"])
    bad["eps"] = c["prm"]["eps"].clone()
    bad["eps"][0] = float("nan")
    with pytest.raises(Bm.PMError) as e:
        Bm.assemble_corrector(c["mesh"], Bm.PM_CP2, bad, w["nu"], w["dt"])
    assert e.value.status == Bm.PM_NONFINITE
    val = Bm.assemble_corrector(c["mesh"], Bm.PM_CP2, c["prm"], w["nu"], w["dt"])["val64"]
    b = torch.tensor(w["rhs"]["cp2"], device=c["dev"])
    b[1] = float("inf")
    with pytest.raises(Bm.PMError) as e:
        Bm.pcg_solve(c["mesh"], val, b)
    assert e.value.status == Bm.PM_NONFINITE
    # CP2 on a mesh without a CP2 Dirichlet side is singular
    m = w["mesh"]
    tag = np.where(w["side_tag"] & 2, 1, w["side_tag"]).astype(np.int8)
    mesh2 = Bm.Mesh(m["xy"], m["tri"], tag)
    with pytest.raises(Bm.PMError) as e:
        Bm.assemble_corrector(mesh2, Bm.PM_CP2, c["prm"], w["nu"], w["dt"])
    assert e.value.status == Bm.PM_SINGULAR


def test_chebyshev_options_are_checked():
    c = case("tiny")
    w = c["w"]
    val = B().assemble_corrector(c["mesh"], B().PM_CP2, c["prm"], w["nu"], w["dt"])["val64"]
    b = torch.tensor(w["rhs"]["cp2"], device=c["dev"])
    for deg in (1, 17):
        with pytest.raises(B().PMError) as e:
            B().pcg_solve(c["mesh"], val, b, precond=B().PM_PREC_CHEBYSHEV, cheb_degree=deg)
        assert e.value.status == -1
    with pytest.raises(B().PMError):
        B().pcg_solve(c["mesh"], val, b, precond=2)


def test_unreachable_tolerance_stagnates_like_the_oracle():
    c, A, b, xg, info, xo, io = solve_both("tiny", "cp2", 0, tol=1e-19, stag_checks=10)
    assert info["status"] == B().PM_STAGNATED and io["status"] == opcg.STAGNATED
    assert opcg.rel_residual(A, b, xg) < 1e-12


def test_wide_column_offsets_match_narrow_bitwise():
    """32-bit column indices (the path of meshes whose RCM bandwidth exceeds
    32767) give bitwise the same solutions as the 16-bit offsets, for every
    schedule, both precisions and both preconditioners, at fixed launch
    shapes; 16 bits are restored afterwards."""
    c = case("chan")
    w = c["w"]
    mesh = c["mesh"]
    val = B().assemble_corrector(mesh, B().PM_CP2, c["prm"], w["nu"], w["dt"])["val64"]
    b = torch.tensor(w["rhs"]["cp2"], device=c["dev"])
    shapes = [dict(tile_rows=1024, block=256, iter_shape=1), dict(tile_rows=2048, block=256, iter_shape=2),
              dict(tile_rows=2048, block=512, iter_shape=3), dict(tile_rows=1024, block=256, iter_shape=-1),
              dict(tile_rows=2048, block=256, iter_shape=4), dict(tile_rows=1024, block=256, iter_shape=4),
              dict(tile_rows=3000, block=512, iter_shape=5)]
    runs = []
    try:
        for bits in (16, 32):
            mesh.set_index_bits(bits)
            assert mesh.stats["index_bits"] == bits
            out = []
            for prec in (0, 1):
                for sh in shapes:
                    x, info = B().pcg_solve(mesh, val, b, precision=prec, **sh)
                    out.append((x.cpu().numpy(), info["iters"], info["status"]))
                x, info = B().pcg_solve(mesh, val, b, precision=prec, precond=1, cheb_degree=4,
                                        tile_rows=2048, block=256)
                out.append((x.cpu().numpy(), info["iters"], info["status"]))
            runs.append(out)
    finally:
        mesh.set_index_bits(16)
    for (x16, it16, st16), (x32, it32, st32) in zip(*runs):
        assert st16 == 0 and st32 == 0 and it16 == it32
        assert np.array_equal(x16, x32)
    with pytest.raises(B().PMError):
        mesh.set_index_bits(8)
