"""Seeded per-cell input fields and right-hand sides.

Porosity eps, log-permeability s = ln K, the transition factor chi in [0,1]
and the normalised inverse-shape tensor G of every cell are sampled at cell
centroids.  Profiles follow the paper's test descriptions: the tanh
transition layer of eq. 3 (Test 1), the linear ramp of eq. permb_test2
(Test 2) and the rotated anisotropy of eq. aniso.  Right-hand sides are
synthetic fluxes or smooth seeded fields.  No corrector arithmetic here.
"""
from __future__ import annotations

import math

import numpy as np

from . import meshes


def box_signed_distance(c, box):
    """Signed distance to the axis-aligned box (x0, x1, y0, y1); > 0 outside."""
    x0, x1, y0, y1 = box
    x, y = c[:, 0], c[:, 1]
    dx = np.maximum(np.maximum(x0 - x, 0.0), x - x1)
    dy = np.maximum(np.maximum(y0 - y, 0.0), y - y1)
    outside = np.sqrt(dx * dx + dy * dy)
    inside = -np.minimum(np.minimum(x - x0, x1 - x), np.minimum(y - y0, y1 - y))
    return np.where((dx > 0) | (dy > 0), outside, inside)


def tanh_inclusion(c, box=(0.3, 0.7, 0.3, 0.7), eps0=0.4, width=0.02, K=1e-3):
    """Square porous inclusion with the tanh transition of eq. 3: the layer's
    centreline lies width/2 inside the box, slope theta = 8/width, d > 0 on the
    fluid side (eps -> 1, chi -> 0)."""
    d = box_signed_distance(c, box) + 0.5 * width
    th = 8.0 / width
    tt = np.tanh(th * d)
    n = c.shape[0]
    return {
        "eps": 0.5 * (1.0 - eps0) * tt + 0.5 * (1.0 + eps0),
        "logk": np.full(n, math.log(K)),
        "chi": 0.5 * (1.0 - tt),
        "g11": np.ones(n), "g12": np.zeros(n), "g22": np.ones(n),
    }


def aniso_shape(beta: float, alpha_rad: float):
    """G = R diag(beta, 1) R^T: K = R diag(k/beta, k) R^{-1} (eq. aniso) inverted
    and divided by 1/k."""
    ca, sa = math.cos(alpha_rad), math.sin(alpha_rad)
    g11 = beta * ca * ca + sa * sa
    g12 = (beta - 1.0) * ca * sa
    g22 = beta * sa * sa + ca * ca
    return g11, g12, g22


def channel_block(c, eps0=0.35, ramp=0.01, K=1e-4, beta=None, alpha_deg=None):
    """Porous block [1.5,2.5]x[0,0.5]: eps and chi ramp linearly from the
    block's exposed sides inwards over `ramp` (eq. permb_test2 style)."""
    x0, x1, yt = meshes.BLOCK
    inb = (c[:, 0] > x0) & (c[:, 0] < x1) & (c[:, 1] < yt)
    dist = meshes.block_interface_distance(c[:, 0], c[:, 1])
    t = np.where(inb, np.minimum(dist / ramp, 1.0), 0.0)
    n = c.shape[0]
    if beta is None:
        g11, g12, g22 = np.ones(n), np.zeros(n), np.ones(n)
    else:
        a, b, d = aniso_shape(beta, math.radians(alpha_deg))
        g11, g12, g22 = np.full(n, a), np.full(n, b), np.full(n, d)
    return {
        "eps": 1.0 - (1.0 - eps0) * t,
        "logk": np.full(n, math.log(K)),
        "chi": t,
        "g11": g11, "g12": g12, "g22": g22,
    }


def gaussian_random_field(c, seed, sigma=1.0, ell=0.05, grid=1024, span=2.0):
    """Stationary Gaussian field with covariance sigma^2 exp(-r^2 / (2 ell^2)),
    synthesised spectrally on a periodic [0, span)^2 grid and bilinearly
    interpolated at the points c (which must lie in [0, span/2]^2 so the
    periodic wrap is many correlation lengths away)."""
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((grid, grid))
    k = np.fft.fftfreq(grid, d=span / grid)
    kx, ky = np.meshgrid(k, k, indexing="ij")
    S = np.exp(-2.0 * math.pi ** 2 * ell ** 2 * (kx * kx + ky * ky))
    a = np.sqrt(S) * (sigma / math.sqrt(S.mean()))
    f = np.real(np.fft.ifft2(np.fft.fft2(w) * a))
    h = span / grid
    gx = c[:, 0] / h
    gy = c[:, 1] / h
    i0 = np.floor(gx).astype(np.int64)
    j0 = np.floor(gy).astype(np.int64)
    fx = gx - i0
    fy = gy - j0
    i0 %= grid
    j0 %= grid
    i1 = (i0 + 1) % grid
    j1 = (j0 + 1) % grid
    return ((1 - fx) * (1 - fy) * f[i0, j0] + fx * (1 - fy) * f[i1, j0]
            + (1 - fx) * fy * f[i0, j1] + fx * fy * f[i1, j1])


def lognormal_square(c, seed, mean_logk=-6.0, sigma=1.0, ell=0.05, eps=0.4):
    n = c.shape[0]
    s = mean_logk + gaussian_random_field(c, seed, sigma=sigma, ell=ell)
    return {
        "eps": np.full(n, eps), "logk": s, "chi": np.ones(n),
        "g11": np.ones(n), "g12": np.zeros(n), "g22": np.ones(n),
    }


def boundary_flux_rhs(mesh, group_id, u_normal):
    """Right-hand side sum_j Fl_j of a start-from-rest step: zero interior
    fluxes, and the prescribed outward flux u_normal * l_j on the sides of one
    boundary group (u_normal < 0 for inflow)."""
    xy, tri, group = mesh["xy"], mesh["tri"], mesh["group"]
    b = np.zeros(tri.shape[0])
    for j in range(3):
        a = xy[tri[:, (j + 1) % 3]]
        e = xy[tri[:, (j + 2) % 3]]
        l = np.hypot(e[:, 0] - a[:, 0], e[:, 1] - a[:, 1])
        b += np.where(group[:, j] == group_id, u_normal * l, 0.0)
    return b


def smooth_field(c, seed, modes=8, scale=1.0):
    """Sum of `modes` seeded sinusoids with wavenumbers up to 4 per unit."""
    rng = np.random.default_rng(seed)
    out = np.zeros(c.shape[0])
    for _ in range(modes):
        kx, ky = rng.uniform(-4.0, 4.0, 2)
        ph = rng.uniform(0.0, 2 * math.pi)
        a = rng.standard_normal()
        out += a * np.sin(2 * math.pi * (kx * c[:, 0] + ky * c[:, 1]) + ph)
    return scale * out


def random_rhs(n, seed):
    return np.random.default_rng(seed).standard_normal(n)
