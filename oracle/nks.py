"""Newton-Krylov-Schwarz comparator, FP64 oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The classical method the paper compares against (Section 3, the beam test):
Newton's method on F(u) = 0 itself, each step DF(u_k) du = F(u_k) solved by
GMRES preconditioned with a *linear* two-level Schwarz operator built at u_k.

Readings (the paper names the method and the coarse space, not the form):
  * right preconditioning, so GMRES minimises the true linear residual and
    stops at ||F(u_k) - DF(u_k) du|| <= gmres_rtol ||F(u_k)||;
  * M^{-1} = sum_i P~_i (R_i DF(u_k) P_i)^{-1} R_i + Phi (Phi^T DF(u_k) Phi)^{-1}
    Phi^T: restricted additive Schwarz on the same overlapping subdomains,
    restricted prolongations and coarse basis as the nonlinear method
    (without a coarse basis: the one-level operator);
  * u_{k+1} = u_k - du, stop when ||F(u_k)|| <= rtol ||F(u_0)||.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .schwarz import Schwarz, gmres_mgs


class NKS:
    """Newton with right-preconditioned GMRES; S supplies the subdomains
    (and, if built, the coarse basis) of a Schwarz object."""

    def __init__(self, S: Schwarz):
        self.S = S
        self.P = S.P

    def factor(self, u):
        """Local factorisations of R_i DF(u) P_i (rows and columns V_i) and
        of the Galerkin matrix Phi^T DF(u) Phi."""
        J = self.P.jacobian(u).tocsr()
        loc = []
        for s in self.S.subs:
            Vd = s["Vd"]
            loc.append(sla.lu_factor(J[Vd][:, Vd].toarray(), check_finite=False))
        co = None
        if self.S.Phi is not None:
            A0 = (self.S.PhiT @ (J @ self.S.Phi)).toarray()
            co = sla.lu_factor(A0, check_finite=False)
        return J, loc, co

    def precond(self, fac, r):
        """M^{-1} r."""
        _, loc, co = fac
        y = np.zeros_like(r)
        for s, lu in zip(self.S.subs, loc):
            z = sla.lu_solve(lu, r[s["Vd"]])
            y[s["owned"]] += z[s["owned_loc"]]
        if co is not None:
            y += self.S.Phi @ sla.lu_solve(co, self.S.PhiT @ r)
        return y

    def solve(self, u0=None, rtol=1e-8, maxit=50, gmres_rtol=1e-6,
              gmres_restart=50, gmres_maxit=1000):
        P = self.P
        u = np.zeros(P.ndof) if u0 is None else np.array(u0, dtype=np.float64)
        F = P.residual(u)
        r0 = float(np.linalg.norm(F))
        stats = {"outer": 0, "gmres": [], "res": [r0], "converged": False}
        for _ in range(maxit):
            if float(np.linalg.norm(F)) <= rtol * r0:
                stats["converged"] = True
                break
            fac = self.factor(u)
            J = fac[0]
            y, its = gmres_mgs(lambda x: J @ self.precond(fac, x), F, rtol=gmres_rtol,
                               restart=gmres_restart, maxit=gmres_maxit)
            stats["gmres"].append(its)
            u = u - self.precond(fac, y)
            F = P.residual(u)
            stats["outer"] += 1
            stats["res"].append(float(np.linalg.norm(F)))
            if not np.all(np.isfinite(F)):
                break
        else:
            stats["converged"] = float(np.linalg.norm(F)) <= rtol * r0
        return u, stats
