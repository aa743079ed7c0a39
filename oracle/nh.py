"""Q1 finite elements for 2-D compressible Neo-Hooke elasticity, FP64 oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Problem (eq. 2 of the paper, Section 1): -div P(F) = 0 with the first
Piola-Kirchhoff stress of a compressible Neo-Hooke material,

    P(F) = mu (F - F^{-T}) + lambda ln(det F) F^{-T},   F = I + grad u,

with mu = E/(2(1+nu)) and lambda = E nu/((1+nu)(1-2nu)) (the paper prints
the first factor as E/(1(1+nu)) and the logarithm next to det F F^{-T}; the
reading taken is the standard form above, the gradient of the stored energy
psi = mu/2 (tr F^T F - 2) - mu ln J + lambda/2 (ln J)^2).  Dirichlet dofs
carry identity rows, the load enters as nodal forces (F(u) = f_int(u) -
f_ext), and dofs are node-major, interleaved (u_x, u_y).

Discretisation (reading): bilinear quadrilaterals, 2 x 2 Gauss quadrature,
counter-clockwise nodes; tangent modulus
    A_iJkL = mu d_ik d_JL + lambda Finv_Ji Finv_Lk - (lambda ln J - mu) Finv_Jk Finv_Li.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

_XI = np.array([[-1.0, -1.0], [1.0, -1.0], [1.0, 1.0], [-1.0, 1.0]])
_G = 1.0 / np.sqrt(3.0)
GAUSS = np.array([[-_G, -_G], [_G, -_G], [_G, _G], [-_G, _G]])


class DetFError(RuntimeError):
    """A quadrature point has det F <= 0 (the deformation is not admissible)."""


def q1_shape_grads(xi, eta):
    """dN_a/dxi, dN_a/deta (4 x 2) of N_a = (1 + xi_a xi)(1 + eta_a eta)/4."""
    return 0.25 * np.stack([_XI[:, 0] * (1 + _XI[:, 1] * eta),
                            _XI[:, 1] * (1 + _XI[:, 0] * xi)], axis=1)


def _kinematics(X, ue):
    """Per Gauss point: weights w det(J_map), material gradients of N (E,4,2),
    deformation gradients F (E,2,2)."""
    out = []
    for xi, eta in GAUSS:
        dN = q1_shape_grads(xi, eta)                      # (4, 2)
        Jm = np.einsum("eai,aj->eij", X, dN)              # dX_i/dxi_j
        det = Jm[:, 0, 0] * Jm[:, 1, 1] - Jm[:, 0, 1] * Jm[:, 1, 0]
        if np.any(det <= 0):
            raise ValueError("elements must be counter-clockwise and non-degenerate")
        Jinv = np.linalg.inv(Jm)
        grads = np.einsum("aj,eji->eai", dN, Jinv)        # dN_a/dX_i
        F = np.eye(2)[None] + np.einsum("eai,eaJ->eiJ", ue, grads)
        out.append((det, grads, F))
    return out


def stress(F, mu, lam):
    """P(F), Finv, ln J for a batch of deformation gradients."""
    J = F[:, 0, 0] * F[:, 1, 1] - F[:, 0, 1] * F[:, 1, 0]
    if np.any(J <= 0):
        raise DetFError("det F <= 0")
    Finv = np.linalg.inv(F)
    FinvT = np.transpose(Finv, (0, 2, 1))
    lnJ = np.log(J)
    P = mu * (F - FinvT) + (lam * lnJ)[:, None, None] * FinvT
    return P, Finv, lnJ


def modulus(Finv, lnJ, mu, lam):
    """A_iJkL = dP_iJ / dF_kL (E,2,2,2,2)."""
    d = np.eye(2)
    A = mu * np.einsum("ik,JL->iJkL", d, d)[None]
    A = A + lam * np.einsum("eJi,eLk->eiJkL", Finv, Finv)
    A = A - (lam * lnJ - mu)[:, None, None, None, None] * np.einsum("eJk,eLi->eiJkL", Finv, Finv)
    return A


def energy_density(F, mu, lam):
    J = F[:, 0, 0] * F[:, 1, 1] - F[:, 0, 1] * F[:, 1, 0]
    lnJ = np.log(J)
    return 0.5 * mu * (np.einsum("eij,eij->e", F, F) - 2.0) - mu * lnJ + 0.5 * lam * lnJ ** 2


def nh_element(X, ue, mu, lam):
    """Internal-force vectors r (E,8) and stiffness matrices K (E,8,8) of Q1
    elements with nodes X (E,4,2) and displacements ue (E,4,2); element dof
    2a + i is component i of node a."""
    E = X.shape[0]
    r = np.zeros((E, 4, 2))
    K = np.zeros((E, 4, 2, 4, 2))
    for det, grads, F in _kinematics(X, ue):
        P, Finv, lnJ = stress(F, mu, lam)
        A = modulus(Finv, lnJ, mu, lam)
        r += det[:, None, None] * np.einsum("eiJ,eaJ->eai", P, grads)
        K += det[:, None, None, None, None] * np.einsum("eaJ,eiJkL,ebL->eaibk", grads, A, grads)
    return r.reshape(E, 8), K.reshape(E, 8, 8)


def nh_energy(X, ue, mu, lam):
    """Stored energy of each element (E,)."""
    e = np.zeros(X.shape[0])
    for det, _, F in _kinematics(X, ue):
        e += det * energy_density(F, mu, lam)
    return e


class NHProblem:
    """The discrete Neo-Hooke problem F(u) = f_int(u) - f_ext = 0 (eq. 3)."""

    d = 2

    def __init__(self, case: dict, load_scale: float = 1.0):
        self.case = case
        self.xy = np.asarray(case["xy"], dtype=np.float64)
        self.conn = np.asarray(case["conn"], dtype=np.int64)
        self.N = len(self.xy)
        self.E = len(self.conn)
        self.ndof = 2 * self.N
        self.mu = float(case["mu"])
        self.lam = float(case["lam"])
        self.X = self.xy[self.conn]
        self.edofs = (2 * self.conn[:, :, None] + np.arange(2)).reshape(self.E, 8)
        self.dir_dofs = np.asarray(case["dirichlet"], dtype=np.int64)
        self.is_dir = np.zeros(self.ndof, dtype=bool)
        self.is_dir[self.dir_dofs] = True
        self.dir_value = np.zeros(self.ndof)
        self.dir_value[self.dir_dofs] = np.asarray(case["dirichlet_vals"], dtype=np.float64)
        self.f_full = np.asarray(case["nodal_force"], dtype=np.float64)
        self.set_load_scale(load_scale)

    def set_load_scale(self, s):
        """External forces s * f (load stepping)."""
        self.load_scale = float(s)
        f = s * self.f_full
        f[self.is_dir] = 0.0
        self.ext_load = f
        self.b = f.copy()

    def element_local(self, elems, ve):
        """Element internal forces and stiffnesses for local dof values ve."""
        E = len(elems)
        return nh_element(self.X[elems], np.asarray(ve).reshape(E, 4, 2), self.mu, self.lam)

    def residual(self, u):
        r, _ = nh_element(self.X, u[self.edofs].reshape(self.E, 4, 2), self.mu, self.lam)
        F = np.zeros(self.ndof)
        np.add.at(F, self.edofs, r)
        F -= self.ext_load
        d = self.is_dir
        F[d] = u[d] - self.dir_value[d]
        return F

    def jacobian(self, u):
        _, K = nh_element(self.X, u[self.edofs].reshape(self.E, 4, 2), self.mu, self.lam)
        rows = np.repeat(self.edofs, 8, axis=1).ravel()
        cols = np.tile(self.edofs, (1, 8)).ravel()
        keep = ~self.is_dir[rows]
        A = sp.coo_matrix((K.ravel()[keep], (rows[keep], cols[keep])),
                          shape=(self.ndof, self.ndof)).tocsr()
        dd = self.dir_dofs
        A = A + sp.coo_matrix((np.ones(len(dd)), (dd, dd)), shape=A.shape).tocsr()
        A.sum_duplicates()
        return A

    def energy(self, u):
        """Total potential energy (free dofs): stored energy - f_ext . u."""
        e = nh_energy(self.X, u[self.edofs].reshape(self.E, 4, 2), self.mu, self.lam)
        return float(e.sum() - self.ext_load @ u)

    def nullspace(self, nodes):
        """Interface values of the GDSW functions of one component (rows:
        node-major dofs of `nodes`): the two translations, and the
        infinitesimal rotation (-(y - y_c), x - x_c) about the component's
        centroid when it has at least two nodes."""
        n = len(nodes)
        tx = np.zeros(2 * n)
        ty = np.zeros(2 * n)
        tx[0::2] = 1.0
        ty[1::2] = 1.0
        out = [tx, ty]
        if n >= 2:
            p = self.xy[nodes]
            c = p.mean(axis=0)
            rot = np.zeros(2 * n)
            rot[0::2] = -(p[:, 1] - c[1])
            rot[1::2] = p[:, 0] - c[0]
            out.append(rot)
        return out
