"""Oracle: cell tensors and the CP1 / CP2 corrector matrices.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Paper passages followed
  * Sec. 3.1 (after eq. discr_form_FTS): m = nu*eps*Kfrak, M0 = I + m*dt, and
    Sec. 3.2.2: M = M0/dt, so M = I/dt + nu*eps*Kfrak, with Kfrak = K^{-1}
    the inverse permeability (Sec. 2).
  * Sec. 3.2.3, eq. Cs2_4: Xi = eps * M^{-1}.
  * Sec. 3.2.2, eq. CS1_sys_coeff: CP1 diagonal M11*A_e (x system) or
    M22*A_e (y system) plus nu*sum_j l_j/d_{e,ep}; off-diagonal -nu*l_j/d_{e,ep}.
  * Sec. 3.2.3, eq. CS2_sys_coeff with d_{j,n} = (Xi_j n_j).n_j (text before
    eq. Cs2_6): CP2 diagonal sum_j (l_j/d) d_{j,n}; off-diagonal -(l_j/d) d_{j,n}.

Readings where the paper is silent or garbled (listed in the design notes)
  * per-cell inputs: Kfrak_c = chi_c * exp(-s_c) * G_c with s = ln K and G the
    normalised inverse-shape tensor (identity when isotropic; for the
    anisotropy of eq. aniso, G = R diag(beta, 1) R^T); the side average of Xi
    is the arithmetic mean of the two cells' tensors, and a boundary side
    uses its own cell's tensor;
  * Dirichlet boundary sides add w_b = T_b * (CP1: nu, CP2: n.Xi_e.n) to the
    diagonal and w_b * g_b to the right-hand side; Neumann sides add nothing;
  * the CP1 matrix takes the signs of eq. CS1_sys_coeff (the only SPD choice).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

CP1X, CP1Y, CP2 = 0, 1, 2


def cell_tensors(eps, logk, chi, g11, g12, g22, nu: float, dt: float) -> dict:
    """Kfrak, M = I/dt + nu*eps*Kfrak and Xi = eps*dt*(I + nu*eps*dt*Kfrak)^{-1}."""
    eps = np.asarray(eps, np.float64)
    k = np.asarray(chi, np.float64) * np.exp(-np.asarray(logk, np.float64))
    K11, K12, K22 = k * g11, k * g12, k * g22
    M11 = 1.0 / dt + nu * eps * K11
    M12 = nu * eps * K12
    M22 = 1.0 / dt + nu * eps * K22
    c = nu * eps * dt
    S11, S12, S22 = 1.0 + c * K11, c * K12, 1.0 + c * K22
    det = S11 * S22 - S12 * S12
    f = eps * dt / det
    return {
        "K11": K11, "K12": K12, "K22": K22,
        "M11": M11, "M12": M12, "M22": M22,
        "S11": S11, "S12": S12, "S22": S22, "det": det,
        "X11": f * S22, "X12": -f * S12, "X22": f * S11,
    }


def normal_quadratic(t, a11, a12, a22):
    """n^T A n for the unit normal n = (t_y, -t_x)/|t| of the side vector t."""
    tx, ty = t[..., 0], t[..., 1]
    return (ty * ty * a11 - 2.0 * tx * ty * a12 + tx * tx * a22) / (tx * tx + ty * ty)


def default_params(n, eps=None, logk=None, chi=None, g11=None, g12=None, g22=None):
    one = np.ones(n)
    return {
        "eps": one if eps is None else np.asarray(eps, np.float64),
        "logk": np.zeros(n) if logk is None else np.asarray(logk, np.float64),
        "chi": one if chi is None else np.asarray(chi, np.float64),
        "g11": one if g11 is None else np.asarray(g11, np.float64),
        "g12": np.zeros(n) if g12 is None else np.asarray(g12, np.float64),
        "g22": one if g22 is None else np.asarray(g22, np.float64),
    }


def side_weights(geo: dict, kind: int, params: dict, nu: float, dt: float) -> dict:
    """Per (cell, side) matrix weights in the original cell order.

    w[e, j]  weight of interior side j (the same value from both cells) or of a
             Dirichlet boundary side; 0 for Neumann sides
    mass[e]  the CP1 mass term (0 for CP2)
    """
    ct = cell_tensors(params["eps"], params["logk"], params["chi"], params["g11"],
                      params["g12"], params["g22"], nu, dt)
    T, t, nbr, interior, tag = geo["T"], geo["t"], geo["nbr"], geo["interior"], geo["tag"]
    bit = 1 if kind in (CP1X, CP1Y) else 2
    dirichlet = (~interior) & ((tag & bit) != 0)
    o = np.maximum(nbr, 0)
    if kind in (CP1X, CP1Y):
        w_int = nu * T
        w_bnd = nu * T
        mass = (ct["M11"] if kind == CP1X else ct["M22"]) * geo["area"]
    else:
        X11, X12, X22 = ct["X11"], ct["X12"], ct["X22"]
        a11 = 0.5 * (X11[:, None] + X11[o])
        a12 = 0.5 * (X12[:, None] + X12[o])
        a22 = 0.5 * (X22[:, None] + X22[o])
        w_int = T * normal_quadratic(t, a11, a12, a22)
        w_bnd = T * normal_quadratic(t, X11[:, None], X12[:, None], X22[:, None])
        mass = np.zeros(geo["n"])
    w = np.where(interior, w_int, np.where(dirichlet, w_bnd, 0.0))
    return {"w": w, "mass": mass, "dirichlet": dirichlet, "tensors": ct}


def assemble(geo: dict, perm: np.ndarray, kind: int, params: dict, nu: float, dt: float,
             g_dirichlet=None) -> dict:
    """CSR matrix of the corrector system in the renumbered (perm) order.

    Returns csr (scipy, rows/cols in new order, canonical pattern), diag,
    and b_lift = sum over Dirichlet sides of w_b * g_b in the ORIGINAL cell
    order.
    """
    n = geo["n"]
    sw = side_weights(geo, kind, params, nu, dt)
    w, interior = sw["w"], geo["interior"]
    diag = sw["mass"] + w.sum(axis=1)
    e = geo["cell"][interior]
    o = geo["nbr"][interior]
    rows = np.concatenate([np.arange(n), e])
    cols = np.concatenate([np.arange(n), o])
    vals = np.concatenate([diag, -w[interior]])
    perm = np.asarray(perm, np.int64)
    inv = np.empty(n, np.int64)
    inv[perm] = np.arange(n)
    A = sp.csr_matrix((vals, (inv[rows], inv[cols])), shape=(n, n))
    A.sort_indices()
    if g_dirichlet is None:
        b_lift = np.zeros(n)
    else:
        g = np.asarray(g_dirichlet, np.float64).reshape(n, 3)
        b_lift = np.where(sw["dirichlet"], w * g, 0.0).sum(axis=1)
    return {"A": A, "diag_cell": diag, "b_lift": b_lift, "weights": sw}


def to_cell_order(A_perm: sp.csr_matrix, perm: np.ndarray) -> sp.csr_matrix:
    """The same matrix with rows/columns in the original cell order."""
    P = sp.csr_matrix((np.ones(len(perm)), (np.arange(len(perm)), np.asarray(perm))),
                      shape=(len(perm), len(perm)))
    return (P.T @ A_perm @ P).tocsr()
