"""Pins of the oracle's P1 discretisation against mathematics.

Each test checks the oracle against something other than its own formulas:
quadrature of the weak form with independently computed gradients, finite
differences, the linear patch test, an exact load integral, and the
convergence order for a manufactured solution of eq. (1).
"""
import numpy as np
import pytest

import synth
from oracle.p1 import P1Problem, p1_element, p1_geometry, p1_load
from oracle.schwarz import global_newton

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


def _random_triangles(rng, n):
    p = rng.uniform(-1.0, 1.0, size=(n, 3, 2))
    # make counter-clockwise
    v1 = p[:, 1] - p[:, 0]
    v2 = p[:, 2] - p[:, 0]
    cw = v1[:, 0] * v2[:, 1] - v1[:, 1] * v2[:, 0] < 0
    p[cw, 1], p[cw, 2] = p[cw, 2].copy(), p[cw, 1].copy()
    return p


def test_element_residual_matches_quadrature_of_weak_form():
    """r_a + l_a = int_T kappa (1 + beta u^2) grad u . grad phi_a, evaluated
    with gradients from the inverse affine map and the 3-point edge-midpoint
    rule (exact for the quadratic 1 + u^2)."""
    rng = np.random.default_rng(11)
    n = 200
    p = _random_triangles(rng, n)
    xy = p.reshape(-1, 2)
    conn = np.arange(3 * n).reshape(n, 3)
    G, area = p1_geometry(xy, conn)
    ue = rng.normal(size=(n, 3))
    kappa = rng.uniform(0.5, 2.0, size=n)
    zero = np.zeros((n, 3))
    for beta in (0.0, 1.0):
        r, _ = p1_element(ue, G, kappa, beta, zero)
        for e in range(n):
            Jm = np.stack([p[e, 1] - p[e, 0], p[e, 2] - p[e, 0]], axis=1)
            ref_grads = np.array([[-1.0, -1.0], [1.0, 0.0], [0.0, 1.0]])
            grads = ref_grads @ np.linalg.inv(Jm)  # rows: grad phi_a
            gu = ue[e] @ grads
            A = 0.5 * abs(np.linalg.det(Jm))
            mids = [(0, 1), (1, 2), (2, 0)]
            quad = sum((1.0 + beta * (0.5 * (ue[e, a] + ue[e, b])) ** 2)
                       for a, b in mids) * A / 3.0
            ref = kappa[e] * quad * (grads @ gu)
            np.testing.assert_allclose(r[e], ref, rtol=1e-12, atol=1e-12)


def test_load_exact_for_linear_f():
    """For linear f the edge-midpoint rule is exact: int_T f phi_a =
    |T|/12 (2 f_a + f_b + f_c) (from int phi_a phi_b = |T|(1+delta)/12)."""
    rng = np.random.default_rng(3)
    n = 50
    p = _random_triangles(rng, n)
    xy = p.reshape(-1, 2)
    conn = np.arange(3 * n).reshape(n, 3)
    _, area = p1_geometry(xy, conn)
    f = lambda q: 1.0 + 2.0 * q[..., 0] - 3.0 * q[..., 1]  # noqa: E731
    load = p1_load(area, f(synth.edge_midpoints(xy, conn)))
    fv = f(p)
    ref = area[:, None] / 12.0 * (fv + fv.sum(axis=1, keepdims=True))
    np.testing.assert_allclose(load, ref, rtol=1e-13, atol=1e-15)


def test_load_integrates_domain():
    """sum_g b_g = int_Omega f (partition of unity of the hat functions):
    area 1 for f = 1; 4/pi^2 for sin(pi x) sin(pi y) up to O(h^2)."""
    case = synth.diffusion_case(16, 16, synth.even_cuts(16, 2),
                                synth.even_cuts(16, 2), 1)
    P = P1Problem(case)
    assert abs(P.load.sum() - 1.0) < 1e-14
    f = lambda q: np.sin(np.pi * q[..., 0]) * np.sin(np.pi * q[..., 1])  # noqa
    case2 = synth.diffusion_case(64, 64, synth.even_cuts(64, 2),
                                 synth.even_cuts(64, 2), 1, forcing=f)
    P2 = P1Problem(case2)
    assert abs(P2.load.sum() - 4.0 / np.pi ** 2) < 2e-4


def test_jacobian_matches_central_differences():
    case = synth.small_case(n=6, boxes=2, overlap=1, coef_seed=5,
                            forcing_seed=7)
    P = P1Problem(case)
    rng = np.random.default_rng(0)
    u = rng.normal(scale=0.7, size=P.N)
    A = P.jacobian(u).toarray()
    eps = 1e-6
    Afd = np.zeros_like(A)
    for j in range(P.N):
        e = np.zeros(P.N)
        e[j] = eps
        Afd[:, j] = (P.residual(u + e) - P.residual(u - e)) / (2 * eps)
    np.testing.assert_allclose(A, Afd, rtol=1e-7, atol=1e-8)
    # the nonlinear term makes DF nonsymmetric (rank-1 element updates)
    assert np.abs(A - A.T).max() > 1e-3


def test_patch_test_linear_solution():
    """beta = 0, kappa = 1, u linear: grad u is constant, so the stiffness
    part vanishes at every interior node and F_g = -b_g."""
    case = synth.small_case(n=10, boxes=2, overlap=1, beta=0.0)
    P = P1Problem(case)
    u = 1.0 + 2.0 * P.xy[:, 0] - 3.0 * P.xy[:, 1]
    F = P.residual(u)
    inner = ~P.is_dir
    np.testing.assert_allclose(F[inner], -P.b[inner], rtol=0, atol=1e-14)


def _manufactured_case(n):
    def f(q):
        x = q[..., 0]
        y = q[..., 1]
        um = np.sin(np.pi * x) * np.sin(np.pi * y)
        grad2 = (np.cos(np.pi * x) * np.sin(np.pi * y)) ** 2 \
            + (np.sin(np.pi * x) * np.cos(np.pi * y)) ** 2
        return 2 * np.pi ** 2 * um * (1 + um ** 2) - 2 * np.pi ** 2 * um * grad2
    return synth.diffusion_case(n, n, synth.even_cuts(n, 2),
                                synth.even_cuts(n, 2), 1, forcing=f)


def test_manufactured_solution_second_order():
    """u_m = sin(pi x) sin(pi y) solves -div((1+u^2) grad u) = f for the f
    above (since -div((1+u^2) grad u) = -(1+u^2) lap u - 2u |grad u|^2);
    the P1 nodal error must decay as h^2."""
    errs = []
    for n in (16, 32, 64):
        P = P1Problem(_manufactured_case(n))
        u, _ = global_newton(P)
        um = np.sin(np.pi * P.xy[:, 0]) * np.sin(np.pi * P.xy[:, 1])
        errs.append(np.abs(u - um).max())
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(orders > 1.9) and np.all(orders < 2.1), (errs, orders)


def test_global_newton_dense_sparse_agree_and_quadratic():
    P = P1Problem(synth.small_case(n=10, boxes=2, overlap=1, forcing_seed=2))
    u1, _ = global_newton(P, dense=True)
    u2, _ = global_newton(P, dense=False)
    assert np.abs(u1 - u2).max() <= 1e-14 * np.abs(u1).max()
    assert np.linalg.norm(P.residual(u1)) < 1e-15
    # quadratic convergence: e_{k+1} <= C e_k^2 along the Newton sequence
    u = np.zeros(P.N)
    errs = []
    for _ in range(4):
        u = u - np.linalg.solve(P.jacobian(u).toarray(), P.residual(u))
        errs.append(np.abs(u - u1).max())
    assert errs[2] <= 10 * errs[1] ** 2 + 1e-15


def test_random_field_separable_form():
    """The generator's separable evaluation of the random-feature field on
    grid centroids equals the direct sum, and has unit variance."""
    f = synth.rff_field(11)
    xy, conn = synth.p1_grid(48, 48)
    cen = xy[conn].mean(axis=1)
    omega, phase = f
    direct = np.sqrt(2.0 / len(phase)) * np.cos(cen @ omega.T + phase).sum(axis=-1)
    np.testing.assert_allclose(synth.rff_eval(cen, f), direct, rtol=0, atol=1e-12)
