"""Named synthetic workloads shaped like the paper's test cases.

Each builder returns a dict with
  mesh      xy, tri, group (synth.meshes)
  side_tag  int8 [n,3] bit mask: bit 0 = Dirichlet side of CP1,
            bit 1 = Dirichlet side of CP2 (Neumann otherwise)
  params    eps, logk, chi, g11, g12, g22 per cell (float64)
  nu, dt    kinematic viscosity and time step
  rhs       right-hand sides per corrector kind ("cp1x", "cp1y", "cp2")
  name, recipe

Recipes
  square_inclusion   unit square, 64x64 jittered grid (0.3h, seed 1); porous
                     square [0.3,0.7]^2 (eps0 0.4, K 1e-3) with a tanh
                     transition of width 0.02; CP2 Dirichlet on x = 1,
                     unit inflow on x = 0, walls y = 0, 1
  channel            [0,4]x[0,1] with a porous block [1.5,2.5]x[0,0.5]; jittered
                     triangular lattice (0.15h) refined 2x and 4x near the
                     block's exposed sides; eps 1 -> 0.35 and chi 0 -> 1 ramp
                     linearly over 0.01 inside the block; K 1e-4 (optionally
                     anisotropic, ratio 100 rotated 30 deg); CP2: inflow x = 0,
                     Dirichlet x = 4; CP1: Dirichlet on walls and inflow
  lognormal_batch    unit squares with triangular-lattice meshes of seeded
                     sizes, log-normal K (mean ln K -6, sigma 1, Gaussian
                     covariance length 0.05), eps 0.4; BCs as square_inclusion
Common: nu = 1.5e-5 (the paper's value); dt chosen so that nu*eps0*dt/K = 1.
"""
from __future__ import annotations

import math

import numpy as np

from . import fields, meshes

NU = 1.5e-5
CP1_DIRICHLET, CP2_DIRICHLET = 1, 2


def side_tags(group, cp1_groups, cp2_groups):
    tag = np.zeros(group.shape, np.int8)
    for gid in cp1_groups:
        tag[group == gid] |= CP1_DIRICHLET
    for gid in cp2_groups:
        tag[group == gid] |= CP2_DIRICHLET
    return tag


def square_inclusion(npts=64, jitter=0.3, seed=1):
    mesh = meshes.square_jittered_grid(npts, jitter, seed)
    c = meshes.centroids(mesh)
    K, eps0 = 1e-3, 0.4
    prm = fields.tanh_inclusion(c, eps0=eps0, K=K)
    n = mesh["tri"].shape[0]
    return {
        "name": f"square_inclusion_{npts}x{npts}",
        "mesh": mesh,
        "side_tag": side_tags(mesh["group"], [meshes.G_LEFT, meshes.G_BOTTOM, meshes.G_TOP], [meshes.G_RIGHT]),
        "params": prm,
        "nu": NU,
        "dt": K / (NU * eps0),
        "rhs": {
            "cp2": fields.boundary_flux_rhs(mesh, meshes.G_LEFT, -1.0),
            "cp1x": 1e-6 * fields.smooth_field(c, seed + 10),
            "cp1y": 1e-6 * fields.smooth_field(c, seed + 11),
            "random": fields.random_rhs(n, seed + 20),
        },
        "recipe": f"unit square {npts}x{npts} grid jitter {jitter}h seed {seed}",
    }


def channel(n_rows=276, seed=2, aniso=False):
    mesh = meshes.channel_mesh(n_rows, seed)
    c = meshes.centroids(mesh)
    K, eps0 = 1e-4, 0.35
    prm = fields.channel_block(c, eps0=eps0, K=K,
                               beta=100.0 if aniso else None, alpha_deg=30.0 if aniso else None)
    n = mesh["tri"].shape[0]
    return {
        "name": f"channel_{'aniso_' if aniso else ''}{n_rows}rows",
        "mesh": mesh,
        "side_tag": side_tags(mesh["group"], [meshes.G_LEFT, meshes.G_BOTTOM, meshes.G_TOP], [meshes.G_RIGHT]),
        "params": prm,
        "nu": NU,
        "dt": K / (NU * eps0),
        "rhs": {
            "cp2": fields.boundary_flux_rhs(mesh, meshes.G_LEFT, -1.0),
            "cp1x": 1e-6 * fields.smooth_field(c, seed + 10),
            "cp1y": 1e-6 * fields.smooth_field(c, seed + 11),
            "random": fields.random_rhs(n, seed + 20),
        },
        "recipe": f"4x1 channel, {n_rows} coarse rows, refined 4x at the block, seed {seed}",
    }


def _lognormal_system(args):
    s, target, seed, mean_logk, eps0, dt = args
    mesh = meshes.unit_square_lattice(int(target), seed * 1000 + s)
    c = meshes.centroids(mesh)
    prm = fields.lognormal_square(c, seed * 1000 + 500 + s, mean_logk=mean_logk, eps=eps0)
    return {
        "name": f"lognormal_{s}",
        "mesh": mesh,
        "side_tag": side_tags(mesh["group"], [meshes.G_LEFT, meshes.G_BOTTOM, meshes.G_TOP], [meshes.G_RIGHT]),
        "params": prm,
        "nu": NU,
        "dt": dt,
        "rhs": {"cp2": fields.boundary_flux_rhs(mesh, meshes.G_LEFT, -1.0)},
        "recipe": f"unit square lattice ~{target} cells seed {seed * 1000 + s}",
    }


def lognormal_batch(n_sys=64, seed=4, lo=50_000, hi=500_000, workers=1):
    """Systems are generated independently (each from its own seeds), so
    `workers` > 1 spreads them over a process pool with identical results."""
    sizes = np.random.default_rng(seed).integers(lo, hi + 1, n_sys)
    eps0, mean_logk = 0.4, -6.0
    dt = math.exp(mean_logk) / (NU * eps0)
    jobs = [(s, t, seed, mean_logk, eps0, dt) for s, t in enumerate(sizes.tolist())]
    if workers > 1 and n_sys > 1:
        import multiprocessing as mp

        with mp.get_context("spawn").Pool(min(workers, n_sys)) as pool:
            return pool.map(_lognormal_system, jobs, chunksize=1)
    return [_lognormal_system(j) for j in jobs]
