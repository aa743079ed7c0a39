"""P1 finite-element residual and Jacobian of the nonlinear diffusion problem.

Problem (eq. 1 of the paper, Section 1):  -div((u^2+1) grad u) = 1 in the
unit square, u = 0 on the boundary.  Generalised, as the workloads need, to

    -div( kappa(x) (1 + beta u^2) grad u ) = f,   u = g on the Dirichlet set,

with kappa constant per element and beta in {0, 1} (beta = 0 is the linear
problem used to check the reduction to linear Schwarz).

Discretisation (the paper only says "regular square mesh"; reading taken):
P1 triangles; the nonlinear stiffness term is integrated exactly; the load is
integrated with the edge-midpoint rule from the samples of f the input holds
(f = 1 when none are given).  Dirichlet nodes carry identity rows
F_g(u) = u_g - g_g, so F has one entry per mesh node (the abstract discrete
problem F(u) = 0, eq. 3).

FP64 throughout.  Test infrastructure only (see the package docstring).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def p1_geometry(xy: np.ndarray, conn: np.ndarray):
    """Per-element stiffness G_ab = |T| grad(phi_a).grad(phi_b) and area |T|.

    With b_a = y_{a+1} - y_{a+2}, c_a = x_{a+2} - x_{a+1} (indices mod 3),
    grad(phi_a) = (b_a, c_a) / (2|T|), so G_ab = (b_a b_b + c_a c_b) / (4|T|).
    """
    p = xy[conn]
    x = p[..., 0]
    y = p[..., 1]
    b = np.stack([y[:, 1] - y[:, 2], y[:, 2] - y[:, 0], y[:, 0] - y[:, 1]], 1)
    c = np.stack([x[:, 2] - x[:, 1], x[:, 0] - x[:, 2], x[:, 1] - x[:, 0]], 1)
    area2 = b[:, 0] * c[:, 1] - b[:, 1] * c[:, 0]
    if np.any(area2 <= 0):
        raise ValueError("elements must be counter-clockwise and non-degenerate")
    G = (b[:, :, None] * b[:, None, :] + c[:, :, None] * c[:, None, :]) \
        / (2.0 * area2)[:, None, None]
    return G, 0.5 * area2


def p1_load(area: np.ndarray, elem_load) -> np.ndarray:
    """Element load vectors l_a = int_T f phi_a, edge-midpoint quadrature.

    The rule puts weight |T|/3 on each edge midpoint, where phi_a is 1/2 on the
    two edges through vertex a and 0 on the opposite one, hence
    l_a = |T|/6 (f(m_{a,a+1}) + f(m_{a-1,a})).  elem_load holds f at the
    midpoints of edges (v0,v1), (v1,v2), (v2,v0); None means f = 1.
    """
    if elem_load is None:
        return np.repeat((area / 3.0)[:, None], 3, axis=1)
    fm = np.asarray(elem_load, dtype=np.float64)
    w = area / 6.0
    return np.stack([w * (fm[:, 0] + fm[:, 2]),
                     w * (fm[:, 0] + fm[:, 1]),
                     w * (fm[:, 1] + fm[:, 2])], axis=1)


def p1_element(ue, G, kappa, beta, load):
    """Element residual r and Jacobian K at element nodal values ue (E,3).

    Weak form of eq. (1): r_a = int_T kappa (1 + beta u^2) grad u . grad phi_a
    - l_a.  For P1, grad u is constant on T and int_T u^2 = |T| m_T with
    m_T = (U^2 + sum_a u_a^2) / 12, U = sum_a u_a (from int phi_a phi_b =
    |T| (1 + delta_ab) / 12), so r_a = kappa (1 + beta m_T) s_a - l_a with
    s_a = sum_b G_ab u_b.  Differentiating, dm_T/du_c = (U + u_c) / 6 and
    K_ac = kappa [ (1 + beta m_T) G_ac + beta s_a (U + u_c) / 6 ].
    """
    U = ue.sum(axis=1)
    m = (U * U + (ue * ue).sum(axis=1)) / 12.0
    s = np.einsum("eab,eb->ea", G, ue)
    coef = kappa * (1.0 + beta * m)
    r = coef[:, None] * s - load
    K = coef[:, None, None] * G \
        + (beta * kappa / 6.0)[:, None, None] * s[:, :, None] \
        * (ue + U[:, None])[:, None, :]
    return r, K


class P1Problem:
    """The discrete nonlinear problem F(u) = 0 (eq. 3) of one input case."""

    d = 1  # dofs per node

    def __init__(self, case: dict):
        self.case = case
        self.xy = np.asarray(case["xy"], dtype=np.float64)
        self.conn = np.asarray(case["conn"], dtype=np.int64)
        self.N = len(self.xy)
        self.E = len(self.conn)
        self.G, self.area = p1_geometry(self.xy, self.conn)
        coef = case.get("elem_coef")
        self.kappa = np.ones(self.E) if coef is None else np.asarray(coef, np.float64)
        self.beta = float(case.get("beta", 1.0))
        self.load = p1_load(self.area, case.get("elem_load"))
        self.dir_nodes = np.asarray(case["dirichlet"], dtype=np.int64)
        self.dir_vals = np.asarray(case["dirichlet_vals"], dtype=np.float64)
        self.is_dir = np.zeros(self.N, dtype=bool)
        self.is_dir[self.dir_nodes] = True
        self.dir_value = np.zeros(self.N)
        self.dir_value[self.dir_nodes] = self.dir_vals
        # assembled load vector b (zero on Dirichlet rows): F(u) = A(u)u - b
        b = np.zeros(self.N)
        np.add.at(b, self.conn, self.load)
        b[self.is_dir] = 0.0
        self.b = b
        self.ndof = self.N
        # the load is part of the element residuals; no nodal forces
        self.ext_load = np.zeros(self.N)

    def element_local(self, elems, ve):
        """Element residuals (load included) and Jacobians for local values."""
        return p1_element(ve, self.G[elems], self.kappa[elems], self.beta,
                          self.load[elems])

    def nullspace(self, nodes):
        """Interface values of the GDSW function of one component: 1."""
        return [np.ones(len(nodes))]

    def element(self, u, elems=None):
        """Element residuals and Jacobians at the global vector u."""
        if elems is None:
            elems = slice(None)
        conn = self.conn[elems]
        return p1_element(u[conn], self.G[elems], self.kappa[elems],
                          self.beta, self.load[elems])

    def residual(self, u: np.ndarray) -> np.ndarray:
        """F(u): assembled element residuals, identity rows u_g - g_g on
        Dirichlet nodes."""
        r, _ = self.element(u)
        F = np.zeros(self.N)
        np.add.at(F, self.conn, r)
        F[self.is_dir] = u[self.is_dir] - self.dir_value[self.is_dir]
        return F

    def jacobian(self, u: np.ndarray) -> sp.csr_matrix:
        """DF(u) as CSR: assembled element Jacobians, identity Dirichlet rows."""
        _, K = self.element(u)
        rows = np.repeat(self.conn, 3, axis=1).ravel()
        cols = np.tile(self.conn, (1, 3)).ravel()
        keep = ~self.is_dir[rows]
        A = sp.coo_matrix((K.ravel()[keep], (rows[keep], cols[keep])),
                          shape=(self.N, self.N)).tocsr()
        d = self.dir_nodes
        A = A + sp.coo_matrix((np.ones(len(d)), (d, d)),
                              shape=(self.N, self.N)).tocsr()
        A.sum_duplicates()
        return A
