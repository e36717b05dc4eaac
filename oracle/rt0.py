"""Oracle: averaged side fluxes after CP1, the CP2 source B_1 they give, and
the RT0 velocity at the end of the step.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Paper passages followed
  * Sec. 3.2.2, eq. flux_k_+_2/3: the flux through an interior side j of e is
    the mean of the two cells' normal fluxes weighted by the other cell's
    area, (u_e . n_j A_ep - u_ep . n_jp A_e) / (A_e + A_ep) l_j, with n_jp
    the same side's outward normal seen from ep (= -n_j); it is continuous
    but does not balance within a cell.
  * eq. CS2_sys_coeff: B_1 of cell e is the sum of its three fluxes.
  * eq. eta_flux and the text after it: the side flux of Xi grad(eta) is
    added, Q_j = Fbar_j + Fl_j^eta; the three Q of a cell then sum to zero.
  * App. A, eq. RT0: u(x) = sum_j Q_j (x - x_j) / (2 A_e), x_j the node
    opposite side j, Q_j the outward flux through side j; with zero sum it is
    constant in the cell (eq. RT0_prop), and u_e^{k+1} is that constant.

Readings (listed in the design notes)
  * Boundary sides (the paper defers its boundary conditions to its
    ref. [29]): a side with a prescribed velocity (a CP1 Dirichlet side)
    carries (g . n_j) l_j with g the prescribed velocity; any other boundary
    side carries the cell's own normal flux (u_e . n_j) l_j.
  * u_e is evaluated at the centroid of e: the cell mean of the linear RT0
    field, equal to its constant value when the fluxes balance.
"""
from __future__ import annotations

import numpy as np

from . import crossflux

CP1_BIT = 1


def normals(geo: dict) -> tuple:
    """Outward unit normals n[e, j] and side lengths l[e, j]."""
    t = geo["t"]
    l = np.sqrt(t[..., 0] ** 2 + t[..., 1] ** 2)
    return np.stack([t[..., 1] / l, -t[..., 0] / l], axis=-1), l


def flux_average(geo: dict, u, v, gx=None, gy=None) -> np.ndarray:
    """Fbar[e, j] for cell velocities (u, v) (eq. flux_k_+_2/3); gx, gy
    [n, 3] the prescribed velocity on CP1 Dirichlet sides (None = 0)."""
    u = np.asarray(u, np.float64)
    v = np.asarray(v, np.float64)
    n = geo["n"]
    gx = np.zeros((n, 3)) if gx is None else np.asarray(gx, np.float64).reshape(n, 3)
    gy = np.zeros((n, 3)) if gy is None else np.asarray(gy, np.float64).reshape(n, 3)
    nrm, l = normals(geo)
    nx, ny = nrm[..., 0], nrm[..., 1]
    A = geo["area"]
    o = np.maximum(geo["nbr"], 0)
    un_e = u[:, None] * nx + v[:, None] * ny     # u_e . n_j
    un_p = u[o] * nx + v[o] * ny                 # u_ep . n_j = -(u_ep . n_jp)
    A_e = np.repeat(A[:, None], 3, axis=1)
    A_p = A[o]
    interior = (un_e * A_p + un_p * A_e) / (A_e + A_p) * l
    prescribed = (gx * nx + gy * ny) * l
    own = un_e * l
    bnd = np.where((geo["tag"] & CP1_BIT) != 0, prescribed, own)
    return np.where(geo["interior"], interior, bnd)


def rt0_velocity(geo: dict, Q, at=None) -> np.ndarray:
    """The RT0 field of the side fluxes Q[e, j] (eq. RT0) evaluated at the
    points at[e] (default: the centroids); returns [n, 2]."""
    Q = np.asarray(Q, np.float64)
    P = geo["xy"][geo["tri"]]  # [n, 3 nodes, 2]
    x = P.mean(axis=1) if at is None else np.asarray(at, np.float64)
    A = geo["area"]
    out = np.zeros((geo["n"], 2))
    for j in range(3):
        out += Q[:, j, None] * (x - P[:, j]) / (2.0 * A[:, None])
    return out


def step_fluxes(geo: dict, params: dict, nu: float, dt: float, fbar, eta, eta_tilde,
                g_cp2=None) -> np.ndarray:
    """Q[e, j] = Fbar_j + Fl_j^eta (eq. eta_flux: two-point part in eta,
    tangential part in eta~)."""
    return np.asarray(fbar, np.float64) + crossflux.side_flux(geo, params, nu, dt, eta, eta_tilde,
                                                              g_cp2)
