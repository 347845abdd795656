"""torch.autograd wrapper of the Stokes solve (adjoint through the C ABI).

Forward: u, p = K(nu)^-1 f~(f) with the Dirichlet data of the problem.
Backward: hhg_adjoint_rhs forms the adjoint right-hand side (dL/du on free
velocity rows, Pi^T dL/dp, with Pi the mean-zero projection of the pressure
when it has a null space), the adjoint system K lambda = that right-hand side
reuses the same symmetric saddle-point multigrid (hhg_solve), and hhg_grad
evaluates dL/df = R^T lambda and dL/dnu_e = lambda^T (df~/dnu_e - dK/dnu_e x)
in a kernel.  Everything past the argument marshalling runs in the library.
The backward pass re-installs the viscosity of its own forward call, so
solves at other viscosities in between do not change the gradient.
"""
from __future__ import annotations

import numpy as np
import torch

from . import HHG_OK, HHGError, Solver


class StokesProblem:
    """A solver plus the nodal data that stay fixed across forward calls."""

    def __init__(self, solver: Solver, dirichlet_nodal=None, rtol=1e-8, max_cycles=100):
        self.s = solver
        self.rtol = rtol
        self.max_cycles = max_cycles
        N = solver.num_nodes()
        ijk, dmask = solver.node_info()
        self.dirichlet = torch.tensor(dmask, device=solver.device)
        x0 = torch.zeros(4, N, dtype=torch.float64, device=solver.device)
        if dirichlet_nodal is not None:
            bc = torch.as_tensor(dirichlet_nodal, dtype=torch.float64, device=solver.device)
            x0[:3] = torch.where(self.dirichlet[None, :], bc, torch.zeros_like(bc))
        self.x0 = x0
        self._nu = None
        self.last_info = None

    def set_viscosity(self, nu):
        nu_np = nu.detach().double().cpu().numpy()
        if self._nu is None or not np.array_equal(nu_np, self._nu):
            self.s.set_viscosity(nu_np)
            self._nu = nu_np.copy()

    def solve(self, rhs_internal, x0_nodal):
        x = self.s.scatter(x0_nodal)
        info = self.s.solve(x, rhs_internal, rtol=self.rtol, max_cycles=self.max_cycles)
        self.last_info = info
        if info["status"] != HHG_OK:
            raise HHGError(info["status"], f"solve did not converge: {info}")
        return x


class StokesSolve(torch.autograd.Function):
    """(f [3,N], nu [nt]) -> (u [3,N], p [N]) for a StokesProblem."""

    @staticmethod
    def forward(ctx, f, nu, prob: StokesProblem):
        prob.set_viscosity(nu)
        s = prob.s
        f_int = s.scatter(f.detach().contiguous())
        b = s.rhs(f_int)
        x = prob.solve(b, prob.x0)
        out = s.gather(x)
        ctx.prob = prob
        ctx.x = x
        ctx.f_int = f_int
        ctx.nu = nu.detach().clone()
        return out[:3].clone(), out[3].clone()

    @staticmethod
    def backward(ctx, gu, gp):
        prob = ctx.prob
        s = prob.s
        prob.set_viscosity(ctx.nu)
        N = s.num_nodes()
        g = torch.zeros(4, N, dtype=torch.float64, device=s.device)
        if gu is not None:
            g[:3] = gu
        if gp is not None:
            g[3] = gp
        lam = prob.solve(s.adjoint_rhs(s.scatter(g)),
                         torch.zeros(4, N, dtype=torch.float64, device=s.device))
        dnu, df_int = s.grad(ctx.x, lam, ctx.f_int)
        df = s.gather(df_int)
        return df, dnu, None
