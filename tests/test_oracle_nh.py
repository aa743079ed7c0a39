"""Pins of the oracle's Neo-Hooke elasticity (Q1) and of the dof-generic
Schwarz oracle on it, against mathematics.

Element: zero stress in the reference state, objectivity, the residual as
the gradient of the stored energy, the tangent as the derivative of the
residual (and symmetric), the reduction to isotropic linear elasticity at
F = I against an independently written B^T D B element, rigid-body modes in
the kernel of the unconstrained stiffness, and the small-load limit.
Method: the fixed point of the preconditioned system equals brute-force
global Newton, the GDSW space reproduces rigid-body modes on subdomains away
from the clamp, the exact tangent matches its literal form and finite
differences, and load stepping reaches the continuation solution.
"""
import numpy as np
import pytest

import synth
from oracle import NHProblem, Schwarz, global_newton
from oracle.nh import DetFError, modulus, nh_element, nh_energy, stress

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")
MU, LAM = 80.76923076923077, 121.15384615384616


def _quads(rng, n):
    """Random convex counter-clockwise quadrilaterals (perturbed squares)."""
    base = np.array([[0.0, 0.0], [1.0, 0.0], [1.0, 1.0], [0.0, 1.0]])
    X = base[None] * rng.uniform(0.5, 2.0, size=(n, 1, 2)) \
        + rng.uniform(-0.1, 0.1, size=(n, 4, 2)) + rng.normal(size=(n, 1, 2))
    return X


def test_reference_state_is_stress_free():
    rng = np.random.default_rng(0)
    X = _quads(rng, 20)
    r, K = nh_element(X, np.zeros((20, 4, 2)), MU, LAM)
    assert np.abs(r).max() <= 1e-12
    P, _, _ = stress(np.repeat(np.eye(2)[None], 3, axis=0), MU, LAM)
    assert np.abs(P).max() == 0.0


def test_objectivity():
    """Rotating the deformed configuration rotates the nodal forces."""
    rng = np.random.default_rng(1)
    X = _quads(rng, 10)
    u = 0.05 * rng.normal(size=(10, 4, 2))
    th = 0.7
    Q = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    x = X + u
    u_rot = np.einsum("ij,eaj->eai", Q, x) - X
    r, _ = nh_element(X, u, MU, LAM)
    r2, _ = nh_element(X, u_rot, MU, LAM)
    ref = np.einsum("ij,eaj->eai", Q, r.reshape(10, 4, 2)).reshape(10, 8)
    np.testing.assert_allclose(r2, ref, rtol=1e-10, atol=1e-10)


def test_residual_is_energy_gradient_and_tangent_is_its_derivative():
    rng = np.random.default_rng(2)
    X = _quads(rng, 4)
    u = 0.05 * rng.normal(size=(4, 4, 2))
    r, K = nh_element(X, u, MU, LAM)
    eps = 1e-6
    g = np.zeros((4, 8))
    Kfd = np.zeros((4, 8, 8))
    for k in range(8):
        du = np.zeros((4, 8))
        du[:, k] = eps
        up = u + du.reshape(4, 4, 2)
        um = u - du.reshape(4, 4, 2)
        g[:, k] = (nh_energy(X, up, MU, LAM) - nh_energy(X, um, MU, LAM)) / (2 * eps)
        Kfd[:, :, k] = (nh_element(X, up, MU, LAM)[0] - nh_element(X, um, MU, LAM)[0]) / (2 * eps)
    np.testing.assert_allclose(r, g, rtol=1e-7, atol=1e-7)
    np.testing.assert_allclose(K, Kfd, rtol=1e-7, atol=1e-6)
    np.testing.assert_allclose(K, np.transpose(K, (0, 2, 1)), rtol=1e-12, atol=1e-10)


def test_linear_elasticity_at_identity():
    """A(I) = lambda d_iJ d_kL + mu (d_ik d_JL + d_iL d_Jk), and the element
    stiffness at u = 0 equals int B^T D B with the plane-strain D in Voigt
    notation (e_xx, e_yy, 2 e_xy), 2 x 2 Gauss points."""
    d = np.eye(2)
    A = modulus(np.repeat(np.eye(2)[None], 1, axis=0), np.zeros(1), MU, LAM)[0]
    ref = LAM * np.einsum("iJ,kL->iJkL", d, d) + MU * (
        np.einsum("ik,JL->iJkL", d, d) + np.einsum("iL,Jk->iJkL", d, d))
    np.testing.assert_allclose(A, ref, rtol=1e-14, atol=1e-12)
    rng = np.random.default_rng(3)
    X = _quads(rng, 3)
    _, K = nh_element(X, np.zeros((3, 4, 2)), MU, LAM)
    D = np.array([[LAM + 2 * MU, LAM, 0.0], [LAM, LAM + 2 * MU, 0.0], [0.0, 0.0, MU]])
    g = 1.0 / np.sqrt(3.0)
    xi_a = np.array([-1.0, 1.0, 1.0, -1.0])
    eta_a = np.array([-1.0, -1.0, 1.0, 1.0])
    for e in range(3):
        Ke = np.zeros((8, 8))
        for xi in (-g, g):
            for eta in (-g, g):
                dxi = 0.25 * xi_a * (1 + eta_a * eta)
                deta = 0.25 * eta_a * (1 + xi_a * xi)
                Jm = np.array([[dxi @ X[e, :, 0], deta @ X[e, :, 0]],
                               [dxi @ X[e, :, 1], deta @ X[e, :, 1]]])
                gx, gy = np.linalg.solve(Jm.T, np.stack([dxi, deta]))
                B = np.zeros((3, 8))
                B[0, 0::2] = gx
                B[1, 1::2] = gy
                B[2, 0::2] = gy
                B[2, 1::2] = gx
                Ke += np.linalg.det(Jm) * B.T @ D @ B
        np.testing.assert_allclose(K[e], Ke, rtol=1e-12, atol=1e-9)


def test_rigid_modes_in_kernel_of_unconstrained_stiffness():
    case = synth.small_elasticity_case(nx=6, ny=4, boxes=(2, 2))
    case = dict(case, dirichlet=np.zeros(0, np.int64), dirichlet_vals=np.zeros(0))
    P = NHProblem(case)
    K = P.jacobian(np.zeros(P.ndof))
    x, y = P.xy[:, 0], P.xy[:, 1]
    modes = [np.ravel(np.stack([np.ones_like(x), 0 * x], 1)),
             np.ravel(np.stack([0 * x, np.ones_like(x)], 1)),
             np.ravel(np.stack([-y, x], 1))]
    for m in modes:
        assert np.abs(K @ m).max() <= 1e-10 * np.abs(K).max()


def test_det_f_guard():
    X = _quads(np.random.default_rng(4), 1)
    u = np.zeros((1, 4, 2))
    u[0, 2] = -5.0 * (X[0, 2] - X[0, 0])   # folds the element
    with pytest.raises(DetFError):
        nh_element(X, u, MU, LAM)


def test_small_load_matches_linear_elasticity():
    case = synth.small_elasticity_case(nx=8, ny=4, boxes=(2, 2), traction=(0.0, -1e-3))
    P = NHProblem(case)
    u, _ = global_newton(P)
    K = P.jacobian(np.zeros(P.ndof))
    ulin = np.linalg.solve(K.toarray(), P.ext_load)
    rel = np.linalg.norm(u - ulin) / np.linalg.norm(ulin)
    assert rel <= 1e-3, rel
    assert np.linalg.norm(u) > 0


@pytest.mark.parametrize("coupling", ["one_level", "additive"])
def test_fixed_point_equals_global_newton(coupling):
    case = synth.small_elasticity_case(nx=8, ny=4, boxes=(2, 2), overlap=1,
                                       traction=(0.0, -2.0), two_level=True)
    P = NHProblem(case)
    ug, _ = global_newton(P)
    S = Schwarz(P, coupling)
    u, st = S.solve(rtol=1e-12, gmres_rtol=1e-12)
    assert st["converged"]
    assert np.linalg.norm(u - ug) <= 1e-10 * np.linalg.norm(ug)
    assert np.abs(S.evaluate(ug)).max() <= 1e-11 * np.abs(ug).max()


def test_zero_load_is_solved_by_zero():
    case = synth.small_elasticity_case(nx=6, ny=4, boxes=(2, 2), traction=(0.0, 0.0))
    S = Schwarz(NHProblem(case), "additive")
    u, st = S.solve()
    assert st["converged"] and st["outer"] == 0 and not np.any(u)


def test_gdsw_reproduces_rigid_modes_away_from_clamp():
    case = synth.small_elasticity_case(nx=12, ny=6, boxes=(3, 2), overlap=1)
    P = NHProblem(case)
    S = Schwarz(P, "additive")
    x, y = P.xy[:, 0], P.xy[:, 1]
    modes = {"tx": np.ravel(np.stack([np.ones_like(x), 0 * x], 1)),
             "ty": np.ravel(np.stack([0 * x, np.ones_like(x)], 1)),
             "rot": np.ravel(np.stack([-y, x], 1))}
    # coefficients: per component, translations by the mode's value at the
    # centroid and the rotation coefficient 1 (rotation mode only)
    for name, m in modes.items():
        c = []
        for nodes, _ in S.components:
            cx, cy = P.xy[nodes].mean(axis=0)
            vals = {"tx": (1.0, 0.0, 0.0), "ty": (0.0, 1.0, 0.0),
                    "rot": (-cy, cx, 1.0)}[name]
            c.extend(vals[:3] if len(nodes) >= 2 else vals[:2])
        c = np.array(c)
        assert len(c) == S.n0
        phi = S.Phi @ c
        floating = 0
        for i in range(S.n_sub):
            el = np.nonzero(S.part == i)[0]
            nodes = np.unique(P.conn[el])
            if S.node_dir[nodes].any():
                continue
            floating += 1
            dofs = (2 * nodes[:, None] + np.arange(2)).ravel()
            np.testing.assert_allclose(phi[dofs], m[dofs], rtol=0, atol=1e-12)
        assert floating >= 2


def test_tangent_identity_literal_and_finite_differences():
    case = synth.small_elasticity_case(nx=8, ny=4, boxes=(2, 2), overlap=1,
                                       traction=(0.0, -2.0))
    P = NHProblem(case)
    S = Schwarz(P, "additive")
    ug, _ = global_newton(P)
    rng = np.random.default_rng(5)
    u = 0.5 * ug + 0.01 * rng.normal(size=P.ndof)
    u[P.is_dir] = 0.0
    Fx = S.evaluate(u)
    v = rng.normal(size=P.ndof)
    t1 = S.tangent(v)
    t2 = S.tangent_literal(v)
    np.testing.assert_allclose(t1, t2, rtol=0, atol=1e-12 * np.abs(t1).max())
    eps = 1e-6 * np.linalg.norm(u) / np.linalg.norm(v)
    fd = (S.evaluate(u + eps * v) - S.evaluate(u - eps * v)) / (2 * eps)
    assert np.abs(fd - t1).max() <= 1e-6 * np.abs(t1).max()
    del Fx


def test_load_stepping_reaches_continuation_solution():
    case = synth.small_elasticity_case(nx=8, ny=4, boxes=(2, 2), overlap=1,
                                       traction=(0.0, -6.0))
    P = NHProblem(case)
    S = Schwarz(P, "additive")
    u, steps = S.solve_load_steps(4, rtol=1e-12, gmres_rtol=1e-12)
    assert len(steps) == 4 and all(st["converged"] for st in steps)
    ug, _ = global_newton(P, u0=u)
    assert np.linalg.norm(u - ug) <= 1e-10 * np.linalg.norm(ug)
    tip = u[2 * (len(P.xy) - 1) + 1]
    assert tip < -0.01                      # the free end moves down


def test_rgdsw_elasticity_reproduces_rigid_modes_away_from_clamp():
    case = synth.small_elasticity_case(nx=16, ny=12, boxes=(4, 3), overlap=1)
    P = NHProblem(case)
    S = Schwarz(P, "additive", coarse="rgdsw")
    assert S.n0 == 6 * 3          # six interior crosspoints, 3 functions each
    checked = 0
    x, y = P.xy[:, 0], P.xy[:, 1]
    modes = {"tx": np.ravel(np.stack([np.ones_like(x), 0 * x], 1)),
             "ty": np.ravel(np.stack([0 * x, np.ones_like(x)], 1)),
             "rot": np.ravel(np.stack([-y, x], 1))}
    for name, m in modes.items():
        c = []
        for k in S.coarse_nodes:
            cx, cy = P.xy[S.components[k][0]].mean(axis=0)
            c.extend({"tx": (1.0, 0.0, 0.0), "ty": (0.0, 1.0, 0.0), "rot": (-cy, cx, 1.0)}[name])
        phi = S.Phi @ np.array(c)
        for i in range(S.n_sub):
            el = np.nonzero(S.part == i)[0]
            nodes = np.unique(P.conn[el])
            # subdomains whose closure touches no boundary edge of an interface
            if np.any(np.isclose(P.xy[nodes, 0], 0.0)) or np.any(np.isclose(P.xy[nodes, 0], 2.0)) \
                    or np.any(np.isclose(P.xy[nodes, 1], 0.0)) or np.any(np.isclose(P.xy[nodes, 1], 1.0)):
                continue
            dofs = (2 * nodes[:, None] + np.arange(2)).ravel()
            np.testing.assert_allclose(phi[dofs], m[dofs], atol=1e-12)
            checked += 1
    assert checked >= 2 * 3


def test_traction_and_body_loads_are_consistent():
    """The nodal forces of the elasticity inputs against the exact integrals
    they stand for.  For any v in the Q1 space, sum_a f_a v(x_a) =
    int t v ds (traction on x = lx) and int b v dA (volume force), because
    f_a = int t phi_a ds and f_a = int b phi_a dA.  On the edge the traces
    1 and y, in the body 1, x, y and xy, are all in that space; their exact
    integrals are closed forms.  A lumping that put the load at the wrong
    nodes, double-counted a segment or dropped an end would fail the first
    moments even where the totals agree."""
    lx, ly, t = 2.0, 1.0, (0.7, -3.0)
    case = synth.elasticity_case(10, 6, lx, ly, [0, 5, 10], [0, 3, 6], 1, traction=t)
    f, xy = case["nodal_force"], case["xy"]
    fx, fy = f[0::2], f[1::2]
    x, y = xy[:, 0], xy[:, 1]
    assert np.all(f.reshape(-1, 2)[~np.isclose(x, lx)] == 0.0)
    assert abs(fx.sum() - t[0] * ly) <= 1e-14
    assert abs(fy.sum() - t[1] * ly) <= 1e-14
    assert abs((fx * y).sum() - t[0] * ly ** 2 / 2) <= 1e-14
    assert abs((fy * y).sum() - t[1] * ly ** 2 / 2) <= 1e-14
    # every interior edge node carries t h, the two ends t h / 2
    right = np.isclose(x, lx)
    h = ly / 6
    ends = right & (np.isclose(y, 0.0) | np.isclose(y, ly))
    np.testing.assert_allclose(fy[right & ~ends], t[1] * h, rtol=1e-14)
    np.testing.assert_allclose(fy[ends], t[1] * h / 2, rtol=1e-14)
    b = (0.4, -2.5)
    beam = synth.elasticity_case(10, 4, 5.0, 1.0, [0, 10], [0, 4], 1, traction=(0.0, 0.0),
                                 body=b, clamp_right=True)
    f, xy = beam["nodal_force"], beam["xy"]
    x, y = xy[:, 0], xy[:, 1]
    L, H = 5.0, 1.0
    for c in (0, 1):
        fc = f[c::2]
        assert abs(fc.sum() - b[c] * L * H) <= 1e-13
        assert abs((fc * x).sum() - b[c] * L ** 2 * H / 2) <= 1e-12
        assert abs((fc * y).sum() - b[c] * L * H ** 2 / 2) <= 1e-13
        assert abs((fc * x * y).sum() - b[c] * L ** 2 * H ** 2 / 4) <= 1e-12
