"""Pins of the Newton-Krylov-Schwarz comparator (oracle/nks.py).

  * the preconditioner is the linear (two-level) restricted additive
    Schwarz matrix cut from the globally assembled Jacobian, built here
    independently with dense matrices;
  * with a tight GMRES tolerance NKS is Newton's method: after k steps its
    iterate equals the k-th iterate of Newton with direct solves;
  * Neo-Hooke: same solution as global Newton, one- and two-level.
"""
import numpy as np
import pytest

import synth
from oracle import NKS, NHProblem, P1Problem, Schwarz, global_newton


def _ras_dense(J, S, with_coarse):
    N = J.shape[0]
    Jd = J.toarray()
    M = np.zeros((N, N))
    for s in S.subs:
        V = s["Vd"]
        Pt = np.zeros((N, len(V)))
        Pt[s["owned"], s["owned_loc"]] = 1.0
        Rm = np.zeros((len(V), N))
        Rm[np.arange(len(V)), V] = 1.0
        M += Pt @ np.linalg.inv(Jd[np.ix_(V, V)]) @ Rm
    if with_coarse:
        Phi = S.Phi.toarray()
        M += Phi @ np.linalg.inv(Phi.T @ Jd @ Phi) @ Phi.T
    return M


@pytest.mark.parametrize("coupling", ["one_level", "additive"])
def test_preconditioner_is_ras(coupling):
    case = synth.small_case(n=12, boxes=3, overlap=1, forcing_seed=5, coef_seed=2,
                            two_level=(coupling == "additive"))
    P = P1Problem(case)
    N = NKS(Schwarz(P, coupling))
    rng = np.random.default_rng(3)
    u = 0.3 * rng.normal(size=P.N)
    u[P.is_dir] = 0.0
    fac = N.factor(u)
    M = _ras_dense(fac[0], N.S, coupling == "additive")
    r = rng.normal(size=P.N)
    np.testing.assert_allclose(N.precond(fac, r), M @ r, rtol=0, atol=1e-12 * np.abs(M @ r).max())


@pytest.mark.parametrize("coupling", ["one_level", "additive"])
def test_tight_gmres_is_global_newton(coupling):
    case = synth.small_case(n=16, boxes=4, overlap=2, forcing_seed=3,
                            two_level=(coupling == "additive"))
    P = P1Problem(case)
    u, st = NKS(Schwarz(P, coupling)).solve(rtol=1e-12, gmres_rtol=1e-14)
    assert st["converged"] and st["outer"] >= 2
    # Newton's k-th iterate with direct solves, k = the NKS step count
    uk, its = global_newton(P, maxit=st["outer"], dense=True)
    assert its == st["outer"]
    assert np.linalg.norm(u - uk) <= 1e-12 * np.linalg.norm(uk)
    # and one step fewer is a different (unconverged) iterate
    uk1, _ = global_newton(P, maxit=st["outer"] - 1, dense=True)
    assert np.linalg.norm(P.residual(uk1)) > 1e-12 * st["res"][0]


@pytest.mark.parametrize("coupling", ["one_level", "additive"])
def test_neohooke_solution(coupling):
    case = synth.small_elasticity_case(nx=12, ny=6, boxes=(3, 2), overlap=1,
                                       traction=(0.0, -3.0), two_level=(coupling == "additive"))
    P = NHProblem(case)
    u, st = NKS(Schwarz(P, coupling)).solve(rtol=1e-10)
    ug, _ = global_newton(P)
    assert st["converged"]
    assert np.linalg.norm(u - ug) <= 1e-8 * np.linalg.norm(ug)


def test_beam_symmetry_and_methods_agree():
    """The paper's beam set-up (both ends clamped, volume force) on a small
    mesh: the consistent load sums to -force * area; the discrete solution
    is mirror-symmetric about x = 2.5 (u_x odd, u_y even); NKS, additive and
    hybrid nonlinear Schwarz (RGDSW) reach it."""
    f = 4.0
    case = synth.beam_case(f, nx=20, ny=4, boxes=(5, 1), overlap=1)
    assert abs(case["nodal_force"][1::2].sum() + f * 5.0) <= 1e-12
    P = NHProblem(case)
    ug, _ = global_newton(P)
    xy = P.xy
    mirror = np.lexsort((xy[:, 1], np.round(5.0 - xy[:, 0], 9)))
    order = np.lexsort((xy[:, 1], np.round(xy[:, 0], 9)))
    ux, uy = ug[0::2], ug[1::2]
    np.testing.assert_allclose(ux[order], -ux[mirror], atol=1e-10 * np.abs(uy).max())
    np.testing.assert_allclose(uy[order], uy[mirror], atol=1e-10 * np.abs(uy).max())
    assert uy.min() < -0.05  # it does deform
    for coupling in ("additive", "hybrid"):
        S = Schwarz(P, coupling, coarse="rgdsw")
        u, st = S.solve(rtol=1e-10)
        assert st["converged"] and np.linalg.norm(u - ug) <= 1e-8 * np.linalg.norm(ug)
    u, st = NKS(Schwarz(P, "additive", coarse="rgdsw")).solve(rtol=1e-10)
    assert st["converged"] and np.linalg.norm(u - ug) <= 1e-8 * np.linalg.norm(ug)
