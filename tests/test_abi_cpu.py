"""CPU-side checks of the C ABI: the library loads, exports every declared
symbol, and its host structure builder matches the oracle bit for bit."""
import os
import re

import numpy as np
import pytest

from conftest import ROOT
from oracle import geometry, ordering
from paper_2309_03543_amd import binding as B
from synth import meshes, workloads


def declared_symbols():
    names = []
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names += re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b([a-z_][a-z0-9_]*)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    lib = B.lib()
    names = declared_symbols()
    assert "pcg_solve" in names and "assemble_corrector" in names and len(names) >= 15
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(B.EXPORTED) == names


def declared_arity():
    """Parameter count of every function the headers declare."""
    out = {}
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b([a-z_][a-z0-9_]*)\s*\(([^)]*)\)\s*;",
                                 src, flags=re.M):
                args = m.group(2).strip()
                out[m.group(1)] = 0 if args in ("", "void") else args.count(",") + 1
    return out


def test_binding_signatures_match_the_header():
    """The binding declares as many ctypes arguments as the header has
    parameters, for every function (a mismatch would shift arguments)."""
    B.lib()
    ar = declared_arity()
    assert set(ar) == set(declared_symbols())
    lib = B.lib()
    for name, n in ar.items():
        f = getattr(lib, name)
        assert f.argtypes is not None, name
        assert len(f.argtypes) == n, (name, len(f.argtypes), n)


def test_status_strings():
    assert B.status_string(0) == "ok"
    assert B.status_string(B.PM_NOT_DELAUNAY) == "mesh not Delaunay"


@pytest.mark.parametrize("case", ["square", "channel", "aniso", "lattice"])
def test_structure_matches_oracle_bitwise(case):
    if case == "square":
        w = workloads.square_inclusion()
    elif case == "channel":
        w = workloads.channel(24, 2)
    elif case == "aniso":
        w = workloads.channel(18, 3, aniso=True)
    else:
        w = workloads.lognormal_batch(n_sys=1, seed=7, lo=3000, hi=3000)[0]
    m = w["mesh"]
    perm, rp, col, T, st = B.pm_structure_host(m["xy"], m["tri"], w["side_tag"])
    geo = geometry.build(m["xy"], m["tri"], w["side_tag"])
    p2 = ordering.rcm(geo["nbr"])
    rp2, col2 = ordering.csr_pattern(geo["nbr"], p2)
    assert np.array_equal(perm, p2)
    assert np.array_equal(rp, rp2) and np.array_equal(col, col2)
    assert np.array_equal(T, geo["T"])  # same operations in the same order
    assert st["nnz"] == rp2[-1] and st["bandwidth"] == ordering.bandwidth(rp2, col2)
    assert st["n_boundary_sides"] == int((~geo["interior"]).sum())


def test_hand_graph_orders_through_a_mesh():
    # a strip of triangles is a path graph: RCM starts at the lower-index end
    xy = np.array([[0.0, 0.0], [1.0, 0.0], [2.0, 0.0], [0.5, 0.9], [1.5, 0.9], [2.5, 0.9]])
    tri = np.array([[0, 1, 3], [1, 4, 3], [1, 2, 4], [2, 5, 4]])
    perm, rp, col, T, st = B.pm_structure_host(xy, tri, np.zeros((4, 3), np.int8))
    geo = geometry.build(xy, tri, np.zeros((4, 3), np.int8))
    assert perm.tolist() == ordering.rcm(geo["nbr"]).tolist() == [3, 2, 1, 0]


@pytest.mark.parametrize(
    "xy,tri,status",
    [
        (np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]]), np.array([[0, 2, 1]]), B.PM_BAD_MESH),
        (np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]]), np.array([[0, 1, 1]]), B.PM_BAD_MESH),
        (np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]]), np.array([[0, 1, 3]]), B.PM_INVALID_ARG),
        (np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]]), np.zeros((0, 3), np.int64), B.PM_INVALID_ARG),
        (np.array([[0.0, 0.0], [1.0, np.inf], [0.0, 1.0]]), np.array([[0, 1, 2]]), B.PM_NONFINITE),
        (np.array([[0.0, 0.0], [1.0, 0.0], [1.0, 1.0], [0.0, 1.0]]), np.array([[0, 1, 2], [0, 2, 3]]),
         B.PM_NOT_DELAUNAY),
        (np.array([[0.0, 0.0], [1.0, 0.0], [0.5, 1.0], [0.5, -1.0], [0.5, 2.0]]),
         np.array([[0, 1, 2], [1, 0, 3], [0, 1, 4]]), B.PM_BAD_MESH),
    ],
)
def test_structure_errors_match_oracle(xy, tri, status):
    with pytest.raises(B.PMError) as e:
        B.pm_structure_host(xy, tri, np.zeros(tri.shape, np.int8))
    assert e.value.status == status
    with pytest.raises(geometry.MeshError) as e2:
        geometry.build(xy, tri, np.zeros(tri.shape, np.int8))
    assert e2.value.status == status


def test_dirichlet_obtuse_side_rejected_only_when_tagged():
    xy = np.array([[0.0, 0.0], [2.0, 0.0], [1.0, 0.3]])
    tri = np.array([[0, 1, 2]])
    B.pm_structure_host(xy, tri, np.zeros((1, 3), np.int8))
    tag = np.zeros((1, 3), np.int8)
    tag[0, 2] = 2
    with pytest.raises(B.PMError) as e:
        B.pm_structure_host(xy, tri, tag)
    assert e.value.status == B.PM_NOT_DELAUNAY
