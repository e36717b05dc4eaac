"""Oracle: the tangential (cross) flux terms of the CP2 and the right-hand side
B_2 of its second solve.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Paper passages followed
  * Sec. 3.2.3, eq. Cs2_5 and the text after it: the flux of Xi grad(eta)
    through side j of cell e is l_j d_j . grad(eta) with d_j = Xi_j n_j (n_j
    the outward unit normal); d_j splits into its normal part d_{j,n} n_j,
    d_{j,n} = d_j . n_j, and its tangential part d_{j,tau}.
  * App. C, eq. A3.1: d_{j,tau} is decomposed along the outward unit normals
    n_a, n_b of the two other sides of e (co-normal decomposition),
    d_{j,tau} = c_a n_a + c_b n_b.
  * App. C, eq. A3.2: a normal derivative n_a . grad(eta) is the difference
    quotient of eta between the two circumcenters across side a, divided by
    their signed distance d; the tangential term of side j is the mean of the
    estimate built in e and the one built in the neighbour ep.
  * eq. Cs2_7 and eq. eta_flux: the first solve A eta~ = B_1 gives eta~;
    the tangential terms, evaluated with eta~, move to the right-hand side of
    the second solve A eta = B_2 (B_2 as printed after eq. CS2_sys_coeff, with
    the sign reading below).

Readings (the paper's printed forms disagree with each other; each is listed
in the design notes)
  * "d_{tau n_l} alpha_l" is the signed coefficient c_l of the co-normal
    decomposition.  The printed definition as the dot product d_{j,tau} . n_l
    with alpha_l its sign would make the product non-negative and would not
    reconstruct d_{j,tau} unless n_a and n_b were orthogonal.
  * Signs and the factor 1/2: cell c estimates, for its own side k and its
    own outward normal, E_{c,k} = sum_a c_a (eta_nb(a) - eta_c) / d_a.
    The tangential term of side j seen from e is
        T_j(e) = (E_{e,j} - E_{ep,j'}) / 2,
    j' the same side seen from ep (whose outward normal is -n_j), so that
    T_j(e) = -T_{j'}(ep) (the flux is continuous) and the flux
        Fl_j(e) = l_j d_{j,n} (eta_ep - eta_e) / d_{e,ep} + l_j T_j(e)
    equals l_j (Xi grad eta) . n_j exactly for linear eta and constant Xi.
    The cell balance of eq. Cs2_5 then reads
        A eta = B_1 + sum_j l_j T_j(eta~) = B_2.
  * Distances are the ones the matrix uses: d = l / T with T the
    transmissibility of the side (interior: circumcenter to circumcenter;
    Dirichlet boundary: circumcenter to side midpoint).
  * Boundary sides (the paper defers its CP2 boundary conditions to its
    ref. [29]): a CP2 Dirichlet side a enters an estimate with its side value
    g_a in place of eta_nb(a); an estimate that needs a Neumann side is
    unavailable.  An interior side with one estimate unavailable takes the
    other one alone (still continuous); with none, no tangential term.  A
    Dirichlet side j of e takes E_{e,j} alone; a Neumann side carries no
    tangential term (its flux is the prescribed one).
  * The side tensor is the one of the matrix: the mean of the two cells'
    Xi on an interior side, the cell's own Xi on a boundary side.
"""
from __future__ import annotations

import numpy as np

from . import assemble as asm

CP2_BIT = 2


def side_tensors(geo: dict, params: dict, nu: float, dt: float) -> np.ndarray:
    """Xi_j per (cell, side) as [n, 3, 2, 2]: the cells' mean on interior
    sides, the cell's own tensor on boundary sides (eq. Cs2_4)."""
    ct = asm.cell_tensors(params["eps"], params["logk"], params["chi"], params["g11"],
                          params["g12"], params["g22"], nu, dt)
    X = np.empty((geo["n"], 2, 2))
    X[:, 0, 0], X[:, 0, 1], X[:, 1, 0], X[:, 1, 1] = ct["X11"], ct["X12"], ct["X12"], ct["X22"]
    o = np.maximum(geo["nbr"], 0)
    own = np.repeat(X[:, None], 3, axis=1)
    mean = 0.5 * (own + X[o])
    return np.where(geo["interior"][..., None, None], mean, own)


def unit_normals(geo: dict) -> tuple:
    """Outward unit normal n_j and length l_j of every side: the side vector
    rotated clockwise (cells are counter-clockwise)."""
    t = geo["t"]
    l = np.sqrt(t[..., 0] ** 2 + t[..., 1] ** 2)
    nrm = np.stack([t[..., 1] / l, -t[..., 0] / l], axis=-1)
    return nrm, l


def conormal_split(geo: dict, Xs: np.ndarray) -> dict:
    """Per (cell e, side j): d_j = Xi_j n_j, d_{j,n} = d_j . n_j,
    d_{j,tau} = d_j - d_{j,n} n_j, and the coefficients c[e, j, a] of
    d_{j,tau} on the outward normals of the other two sides a of e (c is 0
    for a = j), from the 2x2 system [n_a n_b] (c_a, c_b)^T = d_{j,tau}.
    cbound[e, j] = |d_j| ||[n_a n_b]^{-1}||_F bounds |c| for any tangential
    part up to |d_j|: the size against which rounding in c is measured (c
    itself cancels to 0 when Xi is isotropic)."""
    nrm, l = unit_normals(geo)
    n = geo["n"]
    d = np.einsum("ejab,ejb->eja", Xs, nrm)
    dn = np.einsum("eja,eja->ej", d, nrm)
    dtau = d - dn[..., None] * nrm
    c = np.zeros((n, 3, 3))
    cbound = np.zeros((n, 3))
    for j in range(3):
        a, b = (j + 1) % 3, (j + 2) % 3
        Mab = np.stack([nrm[:, a], nrm[:, b]], axis=-1)  # columns n_a, n_b
        cab = np.linalg.solve(Mab, dtau[:, j][..., None])[..., 0]
        c[:, j, a] = cab[:, 0]
        c[:, j, b] = cab[:, 1]
        cbound[:, j] = np.linalg.norm(d[:, j], axis=-1) * np.linalg.norm(np.linalg.inv(Mab), axis=(1, 2))
    return {"d": d, "dn": dn, "dtau": dtau, "c": c, "cbound": cbound, "n": nrm, "l": l}


def normal_derivatives(geo: dict, eta, g=None) -> tuple:
    """Per (cell e, side a): the difference quotient estimating n_a . grad(eta),
    (eta_nb - eta_e) / d on interior sides and (g_a - eta_e) / d on CP2
    Dirichlet sides, with d = l / T; and whether it exists (False on Neumann
    sides).  Also the bound (|eta_nb| + |eta_e|) / d used for tolerances."""
    eta = np.asarray(eta, np.float64)
    n = geo["n"]
    g = np.zeros((n, 3)) if g is None else np.asarray(g, np.float64).reshape(n, 3)
    _, l = unit_normals(geo)
    interior = geo["interior"]
    dirichlet = (~interior) & ((geo["tag"] & CP2_BIT) != 0)
    other = np.where(interior, eta[np.maximum(geo["nbr"], 0)], np.where(dirichlet, g, 0.0))
    T = geo["T"]
    have = interior | dirichlet
    dist = np.where(have, l / np.where(have, T, 1.0), 1.0)
    q = np.where(have, (other - eta[:, None]) / dist, 0.0)
    qabs = np.where(have, (np.abs(other) + np.abs(eta)[:, None]) / dist, 0.0)
    return q, have, qabs


def tangential_estimates(geo: dict, split: dict, eta, g=None) -> dict:
    """E[e, j] = sum over the other sides a of e of c[e, j, a] times the
    normal-derivative estimate of side a: cell e's estimate of
    d_{j,tau} . grad(eta) (App. C, eq. A3.2); avail[e, j] is False when a
    Neumann side would be needed."""
    q, have, qabs = normal_derivatives(geo, eta, g)
    c, cb = split["c"], split["cbound"]
    E = np.zeros((geo["n"], 3))
    Eabs = np.zeros((geo["n"], 3))
    avail = np.ones((geo["n"], 3), bool)
    for j in range(3):
        for a in ((j + 1) % 3, (j + 2) % 3):
            E[:, j] += c[:, j, a] * q[:, a]
            Eabs[:, j] += cb[:, j] * qabs[:, a]
            avail[:, j] &= have[:, a]
    E = np.where(avail, E, 0.0)
    Eabs = np.where(avail, Eabs, 0.0)
    return {"E": E, "avail": avail, "Eabs": Eabs}


def tangential_terms(geo: dict, est: dict) -> tuple:
    """T[e, j] per the reading above (continuous across interior sides), and
    the matching bound built from |E|."""
    E, avail, Eabs = est["E"], est["avail"], est["Eabs"]
    nbr, nbs = geo["nbr"], geo["nbr_side"]
    interior = geo["interior"]
    o, os_ = np.maximum(nbr, 0), np.maximum(nbs, 0)
    Ep, ap, Epabs = E[o, os_], avail[o, os_], Eabs[o, os_]
    both = avail & ap
    T_int = np.where(both, 0.5 * (E - Ep), np.where(avail, E, np.where(ap, -Ep, 0.0)))
    S_int = np.where(both, 0.5 * (Eabs + Epabs), np.where(avail, Eabs, np.where(ap, Epabs, 0.0)))
    dirichlet = (~interior) & ((geo["tag"] & CP2_BIT) != 0)
    T_bnd = np.where(dirichlet & avail, E, 0.0)
    S_bnd = np.where(dirichlet & avail, Eabs, 0.0)
    return np.where(interior, T_int, T_bnd), np.where(interior, S_int, S_bnd)


def cross_terms(geo: dict, params: dict, nu: float, dt: float, eta_tilde, g=None) -> dict:
    """sum_j l_j T_j(e) for every cell (original order), evaluated at eta~.

    Returns cross[n], scale[n] (the same sum with every product and
    difference replaced by magnitudes: a rounding error bound of the
    evaluation is a small multiple of 2^-53 * scale), T[n, 3] and the
    co-normal split."""
    split = conormal_split(geo, side_tensors(geo, params, nu, dt))
    est = tangential_estimates(geo, split, eta_tilde, g)
    T, S = tangential_terms(geo, est)
    l = split["l"]
    return {"cross": (l * T).sum(axis=1), "scale": (l * S).sum(axis=1), "T": T,
            "split": split, "est": est}


def rhs_b2(geo: dict, params: dict, nu: float, dt: float, eta_tilde, b, g=None) -> np.ndarray:
    """B_2 = b + sum_j l_j T_j(eta~) with b the right-hand side of the first
    solve (B_1 plus the Dirichlet lift)."""
    return np.asarray(b, np.float64) + cross_terms(geo, params, nu, dt, eta_tilde, g)["cross"]


def side_flux(geo: dict, params: dict, nu: float, dt: float, eta, eta_tilde, g=None) -> np.ndarray:
    """Fl[e, j]: the flux of Xi grad(eta) out of e through side j
    (eq. eta_flux): the two-point normal part in eta plus l_j T_j(eta~).
    Neumann sides carry 0."""
    eta = np.asarray(eta, np.float64)
    split = conormal_split(geo, side_tensors(geo, params, nu, dt))
    q, have, _ = normal_derivatives(geo, eta, g)
    T, _ = tangential_terms(geo, tangential_estimates(geo, split, eta_tilde, g))
    l = split["l"]
    return np.where(have, l * split["dn"] * q, 0.0) + l * T


def two_step_dense(geo: dict, A_cell, params: dict, nu: float, dt: float, b, g=None) -> tuple:
    """The sequence of eq. Cs2_7 with direct solves (small meshes): eta~ from
    A eta~ = b, then eta from A eta = b + sum_j l_j T_j(eta~).  A_cell is
    the CP2 matrix in the original cell order."""
    from . import pcg
    eta_t = pcg.dense_solve(A_cell, b)
    b2 = rhs_b2(geo, params, nu, dt, eta_t, b, g)
    return eta_t, pcg.dense_solve(A_cell, b2), b2
