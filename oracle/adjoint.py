"""Oracle: adjoint of the corrector solve and parameter gradients.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper does not differentiate its solver; this follows from the corrector
systems it defines (eq. CS1_sys_coeff, eq. CS2_sys_coeff) by the chain rule.
With A(theta) eta = b + b_lift(theta) and a loss L(eta), and because A is
symmetric, the adjoint lambda solves A lambda = dL/deta and

  dL/dtheta_c = lambda . (d b_lift/dtheta_c - (dA/dtheta_c) eta).

A = sum_f w_f (e_e - e_ep)(e_e - e_ep)^T + sum_{Dirichlet b} w_b e_c e_c^T
    + diag(mass), so, cell by cell,

  CP2:  dL/dtheta_c = - sum_{interior f of c} dw_f/dtheta_c (lam_c - lam_o)(eta_c - eta_o)
                      - sum_{Dirichlet b of c} dw_b/dtheta_c lam_c (eta_c - g_b)
        with w_f = T_f n.(Xi_e + Xi_ep)/2.n, so dw_f/dtheta_c = T_f n.(dXi_c/dtheta_c).n / 2,
        and w_b = T_b n.Xi_c.n;
  CP1x: dL/dtheta_c = - lam_c eta_c A_c dM11_c/dtheta_c (the face weights nu*T
        do not depend on the parameters); CP1y likewise with M22.

Cell-tensor derivatives, with S = I + nu eps dt Kfrak, Xi = eps dt S^{-1} and
Kfrak = chi exp(-s) G:
  dKfrak/ds = -Kfrak,  dXi/ds  = eps dt S^{-1} (nu eps dt Kfrak) S^{-1},
  dXi/deps = dt S^{-1} - eps dt S^{-1} (nu dt Kfrak) S^{-1},
  dM/ds = -nu eps Kfrak,  dM/deps = nu Kfrak.
"""
from __future__ import annotations

import numpy as np

from . import assemble as asm
from . import pcg as pcg_mod


def _mat2(a11, a12, a22):
    return np.stack([np.stack([a11, a12], -1), np.stack([a12, a22], -1)], -2)


def tensor_derivatives(params: dict, nu: float, dt: float) -> dict:
    """dXi/ds, dXi/deps, dM11/ds, dM11/deps, dM22/ds, dM22/deps per cell."""
    ct = asm.cell_tensors(params["eps"], params["logk"], params["chi"], params["g11"],
                          params["g12"], params["g22"], nu, dt)
    eps = np.asarray(params["eps"], np.float64)
    Kf = _mat2(ct["K11"], ct["K12"], ct["K22"])
    Sinv = np.linalg.inv(_mat2(ct["S11"], ct["S12"], ct["S22"]))
    c = (nu * eps * dt)[:, None, None]
    dXi_ds = (eps * dt)[:, None, None] * (Sinv @ (c * Kf) @ Sinv)
    dXi_de = dt * Sinv - (eps * dt)[:, None, None] * (Sinv @ ((nu * dt) * Kf) @ Sinv)
    return {
        "dXi_ds": dXi_ds, "dXi_de": dXi_de,
        "dM11_ds": -nu * eps * ct["K11"], "dM11_de": nu * ct["K11"],
        "dM22_ds": -nu * eps * ct["K22"], "dM22_de": nu * ct["K22"],
    }


def gradients(geo: dict, kind: int, params: dict, nu: float, dt: float, eta, lam,
              g_dirichlet=None) -> dict:
    """dL/ds and dL/deps per cell (original cell order) from eta and lambda."""
    n = geo["n"]
    eta = np.asarray(eta, np.float64)
    lam = np.asarray(lam, np.float64)
    td = tensor_derivatives(params, nu, dt)
    if kind in (asm.CP1X, asm.CP1Y):
        key = "11" if kind == asm.CP1X else "22"
        base = -lam * eta * geo["area"]
        return {"grad_logk": base * td["dM" + key + "_ds"], "grad_eps": base * td["dM" + key + "_de"]}
    T, t, nbr, interior, tag = geo["T"], geo["t"], geo["nbr"], geo["interior"], geo["tag"]
    dirichlet = (~interior) & ((tag & 2) != 0)
    o = np.maximum(nbr, 0)
    g = np.zeros((n, 3)) if g_dirichlet is None else np.asarray(g_dirichlet, np.float64).reshape(n, 3)
    out = {}
    for name, D in (("grad_logk", td["dXi_ds"]), ("grad_eps", td["dXi_de"])):
        qn = asm.normal_quadratic(t, D[:, None, 0, 0], D[:, None, 0, 1], D[:, None, 1, 1])
        f_int = -0.5 * T * qn * (lam[:, None] - lam[o]) * (eta[:, None] - eta[o])
        f_bnd = -T * qn * lam[:, None] * (eta[:, None] - g)
        out[name] = np.where(interior, f_int, np.where(dirichlet, f_bnd, 0.0)).sum(axis=1)
    return out


def adjoint(geo, perm, kind, params, nu, dt, eta, grad_eta, g_dirichlet=None, tol=1e-12,
            replace_every=50):
    """Solve A lambda = grad_eta (cell order in and out) and return gradients."""
    perm = np.asarray(perm, np.int64)
    A = asm.assemble(geo, perm, kind, params, nu, dt, g_dirichlet)["A"]
    gp = np.asarray(grad_eta, np.float64)[perm]
    lam_p, info = pcg_mod.pcg(A, gp, tol=tol, replace_every=replace_every)
    lam = np.empty_like(lam_p)
    lam[perm] = lam_p
    gr = gradients(geo, kind, params, nu, dt, eta, lam, g_dirichlet)
    gr["lambda"] = lam
    gr["info"] = info
    return gr
