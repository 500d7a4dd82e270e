"""``torch.autograd.Function`` around the converged scattering solve: chi, eps -> emergent intensities.

Forward: set the medium, solve to convergence, formal solution at the converged J, emergent top
intensities of the upward directions ([n_theta/2 * n_phi, ny, nx]).  Backward: the library's adjoint
(``rt3d_adjoint_emergent``) gives dL/dchi and dL/deps through the fixed point.  Both run in the HIP
library; this module only passes device tensors.  B is a constant (no gradient).
"""
from __future__ import annotations

import torch

from . import rt3d


class EmergentIntensity(torch.autograd.Function):
    """I_em = EmergentIntensity.apply(chi, eps, B, solver, tol, max_iter, inner_sweeps, adj_tol).

    chi, eps, B: contiguous float64 CUDA tensors (nz, ny, nx); solver: an ``rt3d.Solver`` of that
    grid (its state is overwritten).  The backward pass restores the medium and the converged J if the
    solver was used in between."""

    @staticmethod
    def forward(ctx, chi, eps, B, solver, tol=1e-12, max_iter=2000, inner_sweeps=30, adj_tol=1e-12):
        chi, eps, B = (t.detach().contiguous() for t in (chi, eps, B))
        solver.set_medium(chi, eps, B)
        st, it, c = solver.solve(tol, max_iter, inner_sweeps)
        if st != rt3d.RT3D_OK:
            raise rt3d.Rt3dError(st, f"forward solve did not converge ({it} steps, c = {c:.3e})")
        J = torch.empty_like(chi)
        solver.get_J(J)
        n_up = solver.n_dir // 2
        nz, ny, nx = solver.shape
        Jfs = torch.empty_like(chi)
        solver.formal_solution(None, Jfs)
        I_em = torch.empty((n_up, ny, nx), dtype=torch.float64, device=chi.device)
        solver.emergent_top(I_em)
        torch.cuda.current_stream().synchronize()
        ctx.solver = solver
        ctx.args = (adj_tol, max_iter, inner_sweeps)
        ctx.token = solver._token
        ctx.save_for_backward(chi, eps, B, J)
        return I_em

    @staticmethod
    def backward(ctx, grad_I):
        chi, eps, B, J = ctx.saved_tensors
        solver = ctx.solver
        if solver._token != ctx.token:
            solver.set_medium(chi, eps, B)
        solver.set_J(J)
        adj_tol, max_iter, inner_sweeps = ctx.args
        dchi = torch.empty_like(chi)
        deps = torch.empty_like(chi)
        solver.adjoint(grad_I.detach().contiguous(), adj_tol, max_iter, inner_sweeps, dchi=dchi, deps=deps)
        torch.cuda.current_stream().synchronize()
        return dchi, deps, None, None, None, None, None, None


def emergent_intensity(chi, eps, B, solver, tol=1e-12, max_iter=2000, inner_sweeps=30, adj_tol=1e-12):
    """Differentiable emergent top intensities of the converged solution (see EmergentIntensity)."""
    return EmergentIntensity.apply(chi, eps, B, solver, tol, max_iter, inner_sweeps, adj_tol)
