"""Pins of the oracle's nonlinear Schwarz method against mathematics.

  * partition of unity and owned-in-V_i invariants (eq. 8);
  * reduction to linear restricted additive Schwarz for beta = 0, checked
    against explicit matrices cut from the globally assembled operator;
  * the fixed point of the preconditioned system equals the brute-force
    global Newton solution (one-level and additive);
  * GDSW: reproduction of constants on floating subdomains, discrete
    harmonicity of the interior extension, number of coarse functions;
  * coarse correction of a linear problem in one Newton step;
  * exact tangent against its literal definition and central differences;
  * GMRES against a dense solve of the assembled tangent;
  * quadratic convergence of the local Newton iteration.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle.p1 import P1Problem
from oracle.schwarz import Schwarz, global_newton, gmres_mgs


def _schwarz(coupling="one_level", inner_eta=1e-10, **kw):
    case = synth.small_case(**kw)
    P = P1Problem(case)
    return P, Schwarz(P, coupling, inner_eta=inner_eta)


@pytest.mark.parametrize("overlap", [1, 2])
@pytest.mark.parametrize("uneven", [False, True])
def test_partition_of_unity(overlap, uneven):
    P, S = _schwarz(n=13, boxes=3, overlap=overlap, uneven=uneven)
    counts = np.zeros(P.N, dtype=int)
    for s in S.subs:
        counts[s["owned"]] += 1
        # owned(i) subset of V_i
        assert np.all(np.isin(s["owned"], s["V"]))
        # V_i and Gamma_i are disjoint and every element touching V_i is in the patch
        assert not np.intersect1d(s["V"], s["Gam"]).size
        touching = np.nonzero(np.isin(P.conn, s["V"]).any(axis=1))[0]
        assert np.all(np.isin(touching, s["elems"]))
    assert np.all(counts == 1)
    # sum_i P~_i R_i v = v
    v = np.random.default_rng(1).normal(size=P.N)
    acc = np.zeros(P.N)
    for s in S.subs:
        x = v[s["V"]]
        acc[s["owned"]] += x[s["owned_loc"]]
    np.testing.assert_array_equal(acc, v)


def _ras_matrix(A, S, coupling):
    """M^-1 of linear restricted Schwarz from the globally assembled A
    (independent of the local assembly), with M_1 = sum_i P~_i (R_i A R_i^T)^-1
    R_i and C_0 = Phi (Phi^T A Phi)^-1 Phi^T:
      one_level M_1;  additive M_1 + C_0;  hybrid M_1 (I - A C_0) + C_0
    (coarse correction first, then the local solves on the corrected
    residual)."""
    N = A.shape[0]
    Ad = A.toarray()
    M = np.zeros((N, N))
    for s in S.subs:
        V = s["V"]
        Ainv = np.linalg.inv(Ad[np.ix_(V, V)])
        Pt = np.zeros((N, len(V)))
        Pt[s["owned"], s["owned_loc"]] = 1.0
        Rm = np.zeros((len(V), N))
        Rm[np.arange(len(V)), V] = 1.0
        M += Pt @ Ainv @ Rm
    if coupling != "one_level":
        Phi = S.Phi.toarray()
        C0 = Phi @ np.linalg.inv(Phi.T @ Ad @ Phi) @ Phi.T
        if coupling == "hybrid":
            M = M @ (np.eye(N) - Ad @ C0)
        M += C0
    return M


@pytest.mark.parametrize("coupling", ["one_level", "additive", "hybrid"])
def test_linear_reduction_to_ras(coupling):
    """beta = 0: T_i(u) = J_ii^-1 R_i (A u - b) and F_x(u) = M^-1 (A u - b)
    with M^-1 the (two-level additive) RAS preconditioner; the outer Newton
    iteration converges in one step."""
    P, S = _schwarz(coupling, n=12, boxes=3, overlap=1, beta=0.0,
                    forcing_seed=4, coef_seed=9)
    rng = np.random.default_rng(5)
    u = rng.normal(size=P.N)
    u[P.is_dir] = 0.0
    A = P.jacobian(np.zeros(P.N))
    res = A @ u - P.b
    Fx = S.evaluate(u)
    M = _ras_matrix(A, S, coupling)
    np.testing.assert_allclose(Fx, M @ res, rtol=0, atol=1e-13 * np.abs(M @ res).max())
    for sol in S.state["sols"]:
        assert sol["its"] <= 2
    # tangent is M^-1 A
    v = rng.normal(size=P.N)
    np.testing.assert_allclose(S.tangent(v), M @ (A @ v), rtol=0,
                               atol=1e-12 * np.abs(M @ (A @ v)).max())
    usol, st = S.solve(rtol=1e-10, gmres_rtol=1e-13)
    assert st["outer"] == 1
    uex = np.linalg.solve(A.toarray(), P.b)
    assert np.abs(usol - uex).max() <= 1e-11 * np.abs(uex).max()


@pytest.mark.parametrize("coupling", ["one_level", "additive", "hybrid"])
@pytest.mark.parametrize("n,boxes,overlap", [(8, 2, 1), (12, 3, 1), (12, 3, 2), (13, 3, 2)])
def test_fixed_point_is_global_solution(coupling, n, boxes, overlap):
    """If F(u*) = 0 then every T_i(u*) = 0 and T_0(u*) = 0 (eqs. 4, 9), so
    the nonlinear Schwarz solution equals the global Newton solution."""
    P, S = _schwarz(coupling, n=n, boxes=boxes, overlap=overlap,
                    forcing_seed=3, uneven=(n == 13), inner_eta=1e-14)
    ug, _ = global_newton(P, dense=True)
    Fx0 = np.linalg.norm(S.evaluate(np.zeros(P.N)))
    assert np.linalg.norm(S.evaluate(ug)) <= 1e-13 * Fx0
    u, st = S.solve(rtol=1e-14, gmres_rtol=1e-12)
    assert st["converged"]
    assert np.linalg.norm(u - ug) <= 1e-12 * np.linalg.norm(ug)


def test_gdsw_invariants():
    """Sum of the scalar GDSW functions is 1 on every node of subdomains
    away from the Dirichlet boundary; interior rows are discrete harmonic;
    the count is (bx-1)(by-1) vertices + bx(by-1) + by(bx-1) edges."""
    P, S = _schwarz("additive", n=16, boxes=4, overlap=1)
    assert S.n0 == 3 * 3 + 4 * 3 + 4 * 3
    Phi = S.Phi.toarray()
    rowsum = Phi.sum(axis=1)
    A = P.jacobian(np.zeros(P.N)).toarray()
    for i in range(S.n_sub):
        el = np.nonzero(S.part == i)[0]
        nodes = np.unique(P.conn[el])
        if not P.is_dir[nodes].any():
            np.testing.assert_allclose(rowsum[nodes], 1.0, atol=1e-13)
    for (i, I, bnd) in S.interior_blocks:
        np.testing.assert_allclose(A[I] @ Phi, 0.0, atol=1e-13)
    # Dirichlet rows vanish; interface rows are indicator functions
    assert np.all(Phi[P.is_dir] == 0.0)
    for k, (nodes, _) in enumerate(S.components):
        np.testing.assert_array_equal(Phi[nodes, k], 1.0)


def test_gdsw_extension_at_a_linearisation_point():
    """The energy-minimising extension with DF(u_lin) in place of DF(0):
    interior rows are discrete harmonic for the assembled DF(u_lin) (not for
    DF(0)), interface rows are the same indicator functions."""
    case = synth.small_case(n=16, boxes=4, overlap=1, two_level=True, forcing_seed=3)
    P = P1Problem(case)
    u_lin = 2.0 * np.sin(np.pi * P.xy[:, 0]) * np.sin(np.pi * P.xy[:, 1])
    S0 = Schwarz(P, "additive")
    S = Schwarz(P, "additive", coarse_lin=u_lin)
    Phi, Phi0 = S.Phi.toarray(), S0.Phi.toarray()
    A = P.jacobian(u_lin).toarray()
    A0 = P.jacobian(np.zeros(P.N)).toarray()
    for (i, I, bnd) in S.interior_blocks:
        np.testing.assert_allclose(A[I] @ Phi, 0.0, atol=1e-13)
        assert np.abs(A0[I] @ Phi).max() > 1e-3
    iface = np.zeros(P.N, dtype=bool)
    for nodes, _ in S.components:
        iface[nodes] = True
    np.testing.assert_array_equal(Phi[iface], Phi0[iface])
    assert np.abs(Phi - Phi0).max() > 1e-3


def test_coarse_linear_one_step():
    """beta = 0: T_0(u) = (Phi^T A Phi)^-1 Phi^T (A u - b)."""
    P, S = _schwarz("additive", n=12, boxes=3, overlap=1, beta=0.0,
                    forcing_seed=8)
    u = np.random.default_rng(2).normal(size=P.N)
    A = P.jacobian(np.zeros(P.N)).toarray()
    Phi = S.Phi.toarray()
    ref = np.linalg.solve(Phi.T @ A @ Phi, Phi.T @ (A @ u - P.b))
    co = S.coarse_solve(u)
    assert co["its"] <= 2
    np.testing.assert_allclose(co["c"], ref, rtol=0, atol=1e-13 * np.abs(ref).max())


@pytest.mark.parametrize("coupling", ["one_level", "additive", "hybrid"])
def test_tangent_identity_literal_and_fd(coupling):
    P, S = _schwarz(coupling, n=10, boxes=2, overlap=1, forcing_seed=6,
                    coef_seed=1)
    rng = np.random.default_rng(7)
    ug, _ = global_newton(P)
    u = ug + 0.3 * rng.normal(size=P.N) * np.abs(ug).max()
    u[P.is_dir] = 0.0
    S.evaluate(u)
    v = rng.normal(size=P.N)
    v[P.is_dir] = 0.0
    y = S.tangent(v)
    yl = S.tangent_literal(v)
    np.testing.assert_allclose(y, yl, rtol=0, atol=1e-13 * np.abs(y).max())
    eps = 1e-6 * np.linalg.norm(u) / np.linalg.norm(v)
    S2 = Schwarz(P, coupling)
    S2.inner_eta = 1e-14
    S2.inner_rtol = 1e-15
    fd = (S2.evaluate(u + eps * v) - S2.evaluate(u - eps * v)) / (2 * eps)
    np.testing.assert_allclose(y, fd, rtol=0, atol=1e-6 * np.abs(y).max())


def test_gmres_matches_dense_solve():
    P, S = _schwarz("additive", n=10, boxes=2, overlap=1, forcing_seed=1)
    S.evaluate(np.zeros(P.N))
    N = P.N
    T = np.stack([S.tangent(e) for e in np.eye(N)], axis=1)
    b = S.evaluate(np.zeros(N))
    x, its = gmres_mgs(S.tangent, b, rtol=1e-12, restart=7, maxit=500)
    xd = np.linalg.solve(T, b)
    assert its > 7  # restarts exercised
    np.testing.assert_allclose(x, xd, rtol=0, atol=1e-10 * np.abs(xd).max())


def test_band_lu_matches_lapack_dense_solve():
    """The oracle's band LU (gbtrf/gbtrs) against numpy.linalg.solve (dense
    LAPACK gesv): on a random banded matrix that needs row interchanges and
    on a real local Jacobian J_ii (several right-hand sides)."""
    from oracle.schwarz import band_lu_factor, band_lu_solve
    rng = np.random.default_rng(7)
    n, kl, ku = 60, 4, 3
    A = np.zeros((n, n))
    for k in range(-kl, ku + 1):
        A += np.diag(rng.normal(size=n - abs(k)), k)
    A[np.arange(n), np.arange(n)] *= 1e-3   # small diagonal: pivoting needed
    b = rng.normal(size=(n, 3))
    fac = band_lu_factor(A)
    assert fac[2] == kl and fac[3] == ku
    np.testing.assert_allclose(band_lu_solve(fac, b), np.linalg.solve(A, b),
                               rtol=0, atol=1e-12 * np.abs(np.linalg.solve(A, b)).max())
    P, S = _schwarz("one_level", n=20, boxes=2, overlap=2, forcing_seed=2)
    ug, _ = global_newton(P)
    s = S.subs[0]
    J, B = S.local_jacobian(0, 3.0 * ug[s["Vd"]], ug[s["Gd"]])
    rhs = B @ rng.normal(size=(B.shape[1], 2))
    x = band_lu_solve(band_lu_factor(J), rhs)
    ref = np.linalg.solve(J, rhs)
    np.testing.assert_allclose(x, ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    np.testing.assert_allclose(band_lu_solve(band_lu_factor(J), rhs[:, 0]), ref[:, 0],
                               rtol=0, atol=1e-12 * np.abs(ref).max())


def test_local_newton_quadratic():
    P, S = _schwarz("one_level", n=16, boxes=2, overlap=2, forcing_seed=2)
    ug, _ = global_newton(P)
    sol = S.local_solve(0, 40.0 * ug)
    h = sol["hist"]
    assert sol["its"] >= 3
    for a, b in zip(h[:-1], h[1:]):
        if b > 1e-13 and a > 1e-13:
            assert b <= 10.0 * a * a / max(h[0], 1e-300) * 1e3 or b < 1e-3 * a
    # terminal iterations contract at least quadratically-fast
    assert h[-1] <= 1e-12 * h[0] + 1e-14


# ------------------------------------------------------------------ RGDSW
def test_rgdsw_size_weights_and_constants():
    """RGDSW option 2.2: one function per interior crosspoint on box
    partitions; on an edge between two ancestor vertices the inverse-distance
    weights are the linear interpolants (they sum to one); the basis
    reproduces constants on subdomains away from the boundary."""
    case = synth.small_case(n=24, boxes=4, overlap=2, two_level=True)
    P = P1Problem(case)
    S = Schwarz(P, "additive", coarse="rgdsw")
    assert S.n0 == 9
    Phi = S.Phi.toarray()
    tot = Phi.sum(axis=1)
    # interface node halfway between two crosspoints (x = 0.25, y = 0.375)
    xy = P.xy
    g = int(np.nonzero(np.isclose(xy[:, 0], 0.25) & np.isclose(xy[:, 1], 0.375))[0][0])
    w = Phi[g][Phi[g] != 0]
    assert len(w) == 2 and np.allclose(w, 0.5, atol=1e-14)
    g2 = int(np.nonzero(np.isclose(xy[:, 0], 0.25) & np.isclose(xy[:, 1], 0.25 + 1 / 24))[0][0])
    w2 = np.sort(Phi[g2][Phi[g2] != 0])
    np.testing.assert_allclose(w2, [1 / 6, 5 / 6], atol=1e-14)
    # floating subdomains: the closure of interior boxes
    for i in (5, 6, 9, 10):
        el = np.nonzero(S.part == i)[0]
        nodes = np.unique(P.conn[el])
        np.testing.assert_allclose(tot[nodes], 1.0, atol=1e-12)
    # an edge ending at the Dirichlet boundary: the Dirichlet end (0.25, 0)
    # enters the inverse-distance sum as a zero-valued ancestor, so at
    # (0.25, 1/24), with the crosspoint (0.25, 0.25) at distance 5/24 and the
    # Dirichlet node at 1/24, the only function has the weight
    # (24/5) / (24/5 + 24) = 1/6
    g3 = int(np.nonzero(np.isclose(xy[:, 0], 0.25) & np.isclose(xy[:, 1], 1 / 24))[0][0])
    w3 = Phi[g3][Phi[g3] != 0]
    assert len(w3) == 1
    assert abs(w3[0] - 1.0 / 6.0) <= 1e-14
    # one node further up, distances 4/24 (crosspoint) and 2/24 (Dirichlet):
    # d_D / (d_D + d_v) = (2/24) / (6/24) = 1/3
    g4 = int(np.nonzero(np.isclose(xy[:, 0], 0.25) & np.isclose(xy[:, 1], 2 / 24))[0][0])
    assert abs(tot[g4] - 1.0 / 3.0) <= 1e-14


def test_rgdsw_fixed_point_and_linear_coarse():
    case = synth.small_case(n=12, boxes=3, overlap=1, two_level=True, forcing_seed=4)
    P = P1Problem(case)
    ug, _ = global_newton(P)
    S = Schwarz(P, "additive", coarse="rgdsw")
    u, st = S.solve(rtol=1e-12, gmres_rtol=1e-12)
    assert st["converged"]
    assert np.linalg.norm(u - ug) <= 1e-10 * np.linalg.norm(ug)
    lin = synth.small_case(n=12, boxes=3, overlap=1, two_level=True, beta=0.0, forcing_seed=4)
    PL = P1Problem(lin)
    SL = Schwarz(PL, "additive", coarse="rgdsw")
    uu = np.random.default_rng(1).normal(size=PL.N)
    A = PL.jacobian(uu)
    co = SL.coarse_solve(uu)
    A0 = (SL.PhiT @ (A @ SL.Phi)).toarray()
    ref = np.linalg.solve(A0, SL.PhiT @ PL.residual(uu))
    np.testing.assert_allclose(co["c"], ref, rtol=1e-12, atol=1e-13)
