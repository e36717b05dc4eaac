"""Pins for the oracle's geometry (closed forms, special cases, invariants)."""
import math

import numpy as np
import pytest

from oracle import geometry
from synth import meshes, workloads


def equilateral_pair():
    s = math.sqrt(3.0) / 2.0
    xy = np.array([[0.0, 0.0], [1.0, 0.0], [0.5, s], [0.5, -s]])
    tri = np.array([[0, 1, 2], [1, 0, 3]])
    return xy, tri


def test_equilateral_transmissibility_closed_form():
    xy, tri = equilateral_pair()
    tag = np.zeros((2, 3), np.int8)
    tag[0, 0] = 2  # one Dirichlet side (length 1)
    geo = geometry.build(xy, tri, tag)
    # shared side: opposite node 2 in both cells; cot 60 deg = 1/sqrt(3) on both sides
    assert geo["nbr"][0, 2] == 1 and geo["nbr"][1, 2] == 0
    assert abs(geo["T"][0, 2] - math.sqrt(3.0)) <= 4 * np.spacing(math.sqrt(3.0))
    assert geo["T"][0, 2] == geo["T"][1, 2]
    # boundary side: l / (circumcenter-to-midpoint distance) = 1 / (1/(2 sqrt 3))
    assert abs(geo["T"][0, 0] - 2.0 * math.sqrt(3.0)) <= 8 * np.spacing(2 * math.sqrt(3.0))
    cc = geometry.circumcenter_distances(geo)
    assert abs(cc["d"][0, 2] - 1.0 / math.sqrt(3.0)) < 1e-15
    assert abs(cc["d"][0, 0] - 0.5 / math.sqrt(3.0)) < 1e-15


def test_right_isosceles_pair_is_cocircular():
    xy = np.array([[0.0, 0.0], [1.0, 0.0], [1.0, 1.0], [0.0, 1.0]])
    tri = np.array([[0, 1, 2], [0, 2, 3]])
    with pytest.raises(geometry.MeshError) as e:
        geometry.build(xy, tri, np.zeros((2, 3), np.int8))
    assert e.value.status == geometry.NOT_DELAUNAY


def test_flipped_diagonal_is_not_delaunay_and_good_one_is():
    xy = np.array([[0.0, 0.0], [1.0, -0.2], [2.0, 0.0], [1.0, 0.2]])
    good = np.array([[0, 1, 3], [1, 2, 3]])
    bad = np.array([[0, 1, 2], [0, 2, 3]])
    geometry.build(xy, good, np.zeros((2, 3), np.int8))
    with pytest.raises(geometry.MeshError) as e:
        geometry.build(xy, bad, np.zeros((2, 3), np.int8))
    assert e.value.status == geometry.NOT_DELAUNAY


def test_obtuse_boundary_side_only_matters_when_dirichlet():
    # one triangle whose angle at node 2 is obtuse: side 2 (nodes 0-1) sees >90 deg
    xy = np.array([[0.0, 0.0], [2.0, 0.0], [1.0, 0.3]])
    tri = np.array([[0, 1, 2]])
    geometry.build(xy, tri, np.zeros((1, 3), np.int8))  # Neumann: fine
    tag = np.zeros((1, 3), np.int8)
    tag[0, 2] = 1
    with pytest.raises(geometry.MeshError) as e:
        geometry.build(xy, tri, tag)
    assert e.value.status == geometry.NOT_DELAUNAY


@pytest.mark.parametrize(
    "xy,tri,status",
    [
        (np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]]), np.array([[0, 2, 1]]), geometry.BAD_MESH),  # clockwise
        (np.array([[0.0, 0.0], [1.0, 0.0], [2.0, 0.0]]), np.array([[0, 1, 2]]), geometry.BAD_MESH),  # zero area
        (np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]]), np.array([[0, 1, 1]]), geometry.BAD_MESH),  # repeated node
        (np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]]), np.array([[0, 1, 3]]), geometry.INVALID_ARG),
        (np.array([[0.0, 0.0], [1.0, np.nan], [0.0, 1.0]]), np.array([[0, 1, 2]]), geometry.NONFINITE),
    ],
)
def test_invalid_meshes(xy, tri, status):
    with pytest.raises(geometry.MeshError) as e:
        geometry.build(xy, tri, np.zeros(tri.shape, np.int8))
    assert e.value.status == status


def test_non_manifold_side():
    xy = np.array([[0.0, 0.0], [1.0, 0.0], [0.5, 1.0], [0.5, -1.0], [0.5, 2.0]])
    tri = np.array([[0, 1, 2], [1, 0, 3], [0, 1, 4]])
    with pytest.raises(geometry.MeshError) as e:
        geometry.build(xy, tri, np.zeros((3, 3), np.int8))
    assert e.value.status == geometry.BAD_MESH


def test_cot_form_matches_circumcenter_form_on_jittered_mesh():
    w = workloads.square_inclusion()
    m = w["mesh"]
    geo = geometry.build(m["xy"], m["tri"], w["side_tag"])
    cc = geometry.circumcenter_distances(geo)
    interior = geo["interior"]
    T_cc = cc["l"] / cc["d"]
    cot = geo["cot"]
    o = np.maximum(geo["nbr"], 0)
    co = cot[o, np.maximum(geo["nbr_side"], 0)]
    cond = (np.abs(cot) + np.abs(co)) / np.abs(cot + co)
    rel = np.abs(T_cc - geo["T"]) / geo["T"]
    # the circumcenter form loses accuracy like the cot sum's conditioning
    assert np.all(rel[interior] <= 1e-11 * (1 + cond[interior]))
    dirichlet = (~interior) & (geo["tag"] != 0)
    assert np.all(rel[dirichlet] <= 1e-11)
    assert np.all(cc["d"][interior] > 0)


def test_euler_counts_and_pairing():
    for m in (meshes.square_jittered_grid(20, 0.3, 5), meshes.channel_mesh(12, 2)):
        geo = geometry.build(m["xy"], m["tri"], np.zeros(m["tri"].shape, np.int8))
        n, N = geo["n"], m["xy"].shape[0]
        nb = int((~geo["interior"]).sum())
        assert n == 2 * N - nb - 2  # Euler for a triangulated disc
        e, j = np.nonzero(geo["interior"])
        ep, jp = geo["nbr"][e, j], geo["nbr_side"][e, j]
        assert np.all(geo["nbr"][ep, jp] == e) and np.all(geo["nbr_side"][ep, jp] == j)
        # the shared side holds the same two nodes, traversed in opposite directions
        tri = m["tri"]
        assert np.all(tri[e, (j + 1) % 3] == tri[ep, (jp + 2) % 3])
        assert np.all(tri[e, (j + 2) % 3] == tri[ep, (jp + 1) % 3])
        # boundary sides of the rectangle are exactly the sides with no neighbour
        assert np.array_equal(~geo["interior"], m["group"] != 0)
