"""Oracle: the coupled CP1 velocity correction for anisotropic permeability.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Paper passages followed
  * Sec. 3.2.2, eq. cs1_sys2: with anisotropic permeability the mass tensor M
    of a cell has an off-diagonal M12 = M21 = nu eps Kfrak_12 (Sec. 3.1:
    M = I/dt + nu eps Kfrak), so the x and y corrections are coupled
    through the cell term M12 A_e.
  * eq. CS1_sys_coeff: the x system has the CP1x matrix (diagonal
    M11 A_e + nu sum l/d) and the right-hand side B_x - M12 A_e v; the y
    system the CP1y matrix and B_y - M21 A_e u.
  * App. B, eq. A1: the two systems are solved in turn: first without the
    coupling term, then repeatedly with the coupling evaluated at the
    previous iterate of the other component (both updates use iterate i),
    until err = min(err_x, err_y) <= toll with
    err_x = sqrt(||u^{i+1} - u^i||) / sqrt(||u^i||) (likewise y).

Readings (listed in the design notes)
  * Norms are Euclidean norms over all cells.  The printed test takes square
    roots of the norms, so err <= toll means a relative change of at most
    toll^2; it takes the smaller of the two components' changes, so the loop
    ends once either component has settled.  Both are kept as printed.  A
    component whose previous iterate is exactly zero counts as settled when
    its new iterate is zero too, and as unsettled otherwise.
  * The coupled system itself,
        [ A_x        diag(m) ] [u]   [B_x]
        [ diag(m)    A_y     ] [v] = [B_y],   m_e = M12_e A_e,
    is symmetric positive definite: it is nu L (x) I plus the block diagonal
    of the cell tensors M_e A_e (SPD per cell) plus the Dirichlet terms.
    The loop is block Jacobi on it, which converges for any SPD two-block
    matrix; its limit is the coupled solution.
  * coupled_pcg solves the coupled system directly with conjugate gradients
    and the cells' 2x2 diagonal blocks as preconditioner (block Jacobi; the
    blocks are SPD).  This is not in the paper; it reaches the limit of the
    paper's loop in one solve.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import assemble as asm
from . import pcg as opcg


def coupling_weights(geo: dict, params: dict, nu: float, dt: float) -> np.ndarray:
    """m_e = M12_e A_e per cell (original order)."""
    ct = asm.cell_tensors(params["eps"], params["logk"], params["chi"], params["g11"],
                          params["g12"], params["g22"], nu, dt)
    return ct["M12"] * geo["area"]


def coupled_matrix(A_x, A_y, m_perm) -> sp.csr_matrix:
    """The 2n x 2n matrix of both components, blocks in the order (x, y);
    A_x, A_y and m in the same (renumbered) order."""
    D = sp.diags(np.asarray(m_perm, np.float64))
    return sp.bmat([[A_x, D], [D, A_y]], format="csr")


def err_app_b(new, old) -> float:
    """One component's change in the loop test of App. B, eq. A1."""
    d = float(np.linalg.norm(np.asarray(new) - np.asarray(old)))
    o = float(np.linalg.norm(old))
    if o == 0.0:
        return 0.0 if d == 0.0 else np.inf
    return np.sqrt(d) / np.sqrt(o)


def block_iteration(solve_x, solve_y, m, b_x, b_y, toll=1e-4, max_outer=50) -> dict:
    """App. B, eq. A1.  solve_x(rhs, x0) / solve_y(rhs, x0) return the solution
    of the x / y system (x0: previous iterate or None).  m, b_x, b_y and the
    results share one ordering.  Returns u, v, the number of coupled
    iterations after the first pair of solves, the errors and whether the
    test was met."""
    m = np.asarray(m, np.float64)
    b_x = np.asarray(b_x, np.float64)
    b_y = np.asarray(b_y, np.float64)
    u = solve_x(b_x, None)
    v = solve_y(b_y, None)
    errs = []
    converged = False
    i = 0
    while i < max_outer:
        u_new = solve_x(b_x - m * v, u)
        v_new = solve_y(b_y - m * u, v)
        err = min(err_app_b(u_new, u), err_app_b(v_new, v))
        errs.append(err)
        u, v = u_new, v_new
        i += 1
        if err <= toll:
            converged = True
            break
    return {"u": u, "v": v, "outer": i, "errs": errs, "converged": converged}


def dense_solvers(A_x, A_y):
    """Direct solvers for block_iteration (small systems)."""
    return (lambda r, x0: opcg.dense_solve(A_x, r)), (lambda r, x0: opcg.dense_solve(A_y, r))


def pcg_solvers(A_x, A_y, tol=1e-10):
    """The oracle's PCG for block_iteration, warm-started at the previous
    iterate from the second solve on."""
    def mk(A):
        def solve(r, x0):
            x, info = opcg.pcg(A, r, tol=tol, x0=x0)
            if info["status"] != opcg.OK:
                raise RuntimeError(f"inner PCG failed: {info}")
            return x
        return solve
    return mk(A_x), mk(A_y)


def block_inverses(A_x, A_y, m_perm) -> tuple:
    """Inverse of each cell's 2x2 diagonal block [[A_x,ee, m_e], [m_e, A_y,ee]]
    of the coupled matrix, as (i11, i12, i22); the blocks are SPD (the cell's
    mass tensor times A_e plus the same positive Laplacian and Dirichlet terms
    on both diagonal entries)."""
    dx, dy = A_x.diagonal(), A_y.diagonal()
    m = np.asarray(m_perm, np.float64)
    det = dx * dy - m * m
    return dy / det, -m / det, dx / det


def coupled_pcg(A_x, A_y, m_perm, b_x, b_y, tol=1e-10, max_it=100000, check_every=50) -> tuple:
    """Conjugate gradients on the coupled system with the 2x2 block-Jacobi
    preconditioner (the cells' diagonal blocks), x0 = 0, written out
    plainly: q = C p, alpha = rho / p.q, x += alpha p, r -= alpha q,
    z = P^{-1} r, rho' = r.z, p = z + (rho'/rho) p.  Every check_every
    iterations the true residual ||b - C x|| is evaluated and the solve stops
    once it is <= tol ||b||.  The recursive residual is not replaced.
    Returns ((u, v), info) in the order of the inputs."""
    n = A_x.shape[0]
    C = coupled_matrix(A_x, A_y, m_perm)
    i11, i12, i22 = block_inverses(A_x, A_y, m_perm)

    def prec(r):
        rx, ry = r[:n], r[n:]
        return np.concatenate([i11 * rx + i12 * ry, i12 * rx + i22 * ry])

    b = np.concatenate([np.asarray(b_x, np.float64), np.asarray(b_y, np.float64)])
    bnorm = float(np.linalg.norm(b))
    x = np.zeros(2 * n)
    info = {"iters": 0, "status": opcg.OK, "rel_res_true": 0.0}
    if bnorm == 0.0:
        return (x[:n], x[n:]), info
    r = b.copy()
    z = prec(r)
    p = z.copy()
    rho = float(r @ z)
    k = 0
    while k < max_it:
        q = C @ p
        pq = float(p @ q)
        if not (pq > 0.0) or not np.isfinite(pq):
            info["status"] = opcg.BREAKDOWN
            break
        alpha = rho / pq
        x += alpha * p
        r -= alpha * q
        z = prec(r)
        rho_new = float(r @ z)
        p = z + (rho_new / rho) * p
        rho = rho_new
        k += 1
        if k % check_every == 0:
            res = float(np.linalg.norm(b - C @ x)) / bnorm
            if res <= tol:
                info.update(iters=k, rel_res_true=res)
                return (x[:n], x[n:]), info
    info["iters"] = k
    info["rel_res_true"] = float(np.linalg.norm(b - C @ x)) / bnorm
    if info["status"] == opcg.OK:
        info["status"] = opcg.MAXIT
    elif info["status"] == opcg.BREAKDOWN and info["rel_res_true"] <= tol:
        info["status"] = opcg.OK  # converged before p.q reached zero, as in pcg()
    return (x[:n], x[n:]), info
