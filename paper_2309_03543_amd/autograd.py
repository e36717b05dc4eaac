"""torch.autograd wrapper of a corrector solve.

CorrectorSolve.apply(logk, eps, b, ctx_args) returns eta = A(logk, eps)^{-1}
(b + b_lift).  Its backward is the library's hand-written adjoint
(pcg_adjoint): one more PCG solve with the same symmetric matrix, then a
cell-wise gather kernel for dL/dlogk and dL/deps; dL/db = lambda.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import torch

from . import binding as B


@dataclass
class SolveSpec:
    mesh: B.Mesh
    kind: int
    nu: float
    dt: float
    chi: torch.Tensor | None = None
    g11: torch.Tensor | None = None
    g12: torch.Tensor | None = None
    g22: torch.Tensor | None = None
    g_dirichlet: torch.Tensor | None = None
    opts: dict = field(default_factory=dict)


class CorrectorSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, logk, eps, b, spec: SolveSpec):
        params = {"eps": eps.detach().contiguous(), "logk": logk.detach().contiguous(),
                  "chi": spec.chi, "g11": spec.g11, "g12": spec.g12, "g22": spec.g22}
        lift = spec.g_dirichlet is not None
        out = B.assemble_corrector(spec.mesh, spec.kind, params, spec.nu, spec.dt,
                                   g_dirichlet=spec.g_dirichlet, b_lift=lift)
        rhs = b.detach().contiguous()
        if lift:
            rhs = rhs + out["b_lift"]
        eta, info = B.pcg_solve(spec.mesh, out["val64"], rhs, **spec.opts)
        if info["status"] != 0:
            raise B.PMError(info["status"], "forward corrector solve did not converge")
        ctx.spec = spec
        ctx.params = params
        ctx.save_for_backward(out["val64"], eta)
        return eta

    @staticmethod
    def backward(ctx, grad_eta):
        val64, eta = ctx.saved_tensors
        spec = ctx.spec
        lam, gs, ge, info = B.pcg_adjoint(spec.mesh, spec.kind, ctx.params, spec.nu, spec.dt, val64,
                                          eta, grad_eta.contiguous(), g_dirichlet=spec.g_dirichlet,
                                          **spec.opts)
        if info["status"] != 0:
            raise B.PMError(info["status"], "adjoint corrector solve did not converge")
        return gs, ge, lam, None


def corrector_solve(logk, eps, b, spec: SolveSpec):
    return CorrectorSolve.apply(logk, eps, b, spec)
