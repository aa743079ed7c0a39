"""Compressible Neo-Hooke elasticity (Q1, two dofs per node): HIP path
through the C ABI against the FP64 oracle.

Tolerances as for diffusion: F(u) 1e-12 of its largest entry (same formula,
different summation order); F_x and the tangent 1e-10 of their largest
entries (band LU vs dense LU on stiffer local problems); the solution of the
outer iteration 1e-10 relative with equal outer iteration counts.
"""
import numpy as np
import pytest

import synth
from oracle import NHProblem, Schwarz, global_newton
from tests._lib import ensure_built

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    ensure_built()
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _solver(case, **kw):
    from paper_2410_24138_amd import Solver
    return Solver(case, **kw)


def _np(t):
    return t.detach().cpu().numpy()


def _close(a, b, rel):
    scale = max(np.abs(b).max(), 1e-300)
    err = np.abs(a - b).max() / scale
    assert err <= rel, f"max err {err:.3e} > {rel:.1e}"


CASES = [
    dict(nx=8, ny=4, boxes=(2, 2), overlap=1, traction=(0.0, -2.0)),
    dict(nx=12, ny=6, boxes=(3, 2), overlap=2, traction=(0.5, -3.0)),
    dict(nx=10, ny=5, boxes=(2, 2), overlap=1, traction=(0.0, -4.0)),
]


def _probe(P, seed=1):
    ug, _ = global_newton(P)
    rng = np.random.default_rng(seed)
    u = 0.5 * ug + 0.02 * np.abs(ug).max() * rng.normal(size=P.ndof)
    u[P.is_dir] = 0.0
    return u


@pytest.mark.parametrize("kw", CASES)
def test_global_residual(kw):
    case = synth.small_elasticity_case(two_level=False, **kw)
    P = NHProblem(case)
    s = _solver(case, coupling="one_level")
    u = _probe(P)
    _close(_np(s.residual(u)), P.residual(u), 1e-12)


@pytest.mark.parametrize("kw", CASES)
def test_precond_residual_and_tangent_one_level(kw):
    case = synth.small_elasticity_case(two_level=False, **kw)
    P = NHProblem(case)
    S = Schwarz(P, "one_level")
    s = _solver(case, coupling="one_level")
    u = _probe(P, 2)
    _close(_np(s.precond_residual(u)), S.evaluate(u), 1e-10)
    np.testing.assert_array_equal(s.inner_iterations(), [sol["its"] for sol in S.state["sols"]])
    rng = np.random.default_rng(3)
    for _ in range(2):
        v = rng.normal(size=P.ndof)
        _close(_np(s.tangent(v)), S.tangent(v), 1e-10)


@pytest.mark.parametrize("kw", CASES[:2])
def test_solve_one_level(kw):
    case = synth.small_elasticity_case(two_level=False, **kw)
    P = NHProblem(case)
    S = Schwarz(P, "one_level")
    u_ref, st_ref = S.solve()
    uu, st, rc = _solver(case, coupling="one_level").solve()
    assert rc == 0 and st["converged"] and st["outer_its"] == st_ref["outer"]
    assert np.linalg.norm(_np(uu) - u_ref) <= 1e-10 * np.linalg.norm(u_ref)


@pytest.mark.parametrize("kw", CASES[:2])
def test_coarse_basis_rigid_modes(kw):
    """GDSW basis with translations and rotations: equal to the oracle's."""
    case = synth.small_elasticity_case(two_level=True, **kw)
    S = Schwarz(NHProblem(case), "additive")
    s = _solver(case, coupling="additive")
    _close(s.coarse_basis().toarray(), S.Phi.toarray(), 1e-12)


@pytest.mark.parametrize("kw", CASES)
def test_precond_residual_and_tangent_additive(kw):
    case = synth.small_elasticity_case(two_level=True, **kw)
    P = NHProblem(case)
    S = Schwarz(P, "additive")
    s = _solver(case, coupling="additive")
    u = _probe(P, 4)
    _close(_np(s.precond_residual(u)), S.evaluate(u), 1e-10)
    rng = np.random.default_rng(5)
    for _ in range(2):
        v = rng.normal(size=P.ndof)
        _close(_np(s.tangent(v)), S.tangent(v), 1e-10)


@pytest.mark.parametrize("kw", CASES[:2])
def test_solve_additive(kw):
    case = synth.small_elasticity_case(two_level=True, **kw)
    P = NHProblem(case)
    S = Schwarz(P, "additive")
    u_ref, st_ref = S.solve()
    uu, st, rc = _solver(case, coupling="additive").solve()
    assert rc == 0 and st["converged"] and st["outer_its"] == st_ref["outer"]
    assert np.linalg.norm(_np(uu) - u_ref) <= 1e-10 * np.linalg.norm(u_ref)


def test_rgdsw_elasticity():
    case = synth.small_elasticity_case(nx=16, ny=12, boxes=(4, 3), overlap=1,
                                       traction=(0.0, -2.0), two_level=True)
    P = NHProblem(case)
    S = Schwarz(P, "additive", coarse="rgdsw")
    s = _solver(case, coupling="additive", coarse="rgdsw")
    _close(s.coarse_basis().toarray(), S.Phi.toarray(), 1e-12)
    u = _probe(P, 6)
    _close(_np(s.precond_residual(u)), S.evaluate(u), 1e-10)
    v = np.random.default_rng(7).normal(size=P.ndof)
    _close(_np(s.tangent(v)), S.tangent(v), 1e-10)
    u_ref, st_ref = S.solve()
    uu, st, rc = _solver(case, coupling="additive", coarse="rgdsw").solve()
    assert rc == 0 and st["outer_its"] == st_ref["outer"]
    assert np.linalg.norm(_np(uu) - u_ref) <= 1e-10 * np.linalg.norm(u_ref)


@pytest.mark.parametrize("variant", [1, 2, 3])
def test_lu_variants_elasticity(variant):
    """Each band LU form on Neo-Hooke Jacobians under load, whose pivoting
    interchanges rows (unlike the diagonally dominant diffusion Jacobians):
    F_x, inner iteration counts and the tangent as in the oracle."""
    case = synth.small_elasticity_case(nx=16, ny=8, boxes=(2, 2), overlap=2,
                                       traction=(1.0, -4.0), two_level=True)
    P = NHProblem(case)
    S = Schwarz(P, "additive")
    s = _solver(case, coupling="additive", lu_variant=variant)
    u = _probe(P, 9)
    _close(_np(s.precond_residual(u)), S.evaluate(u), 1e-10)
    np.testing.assert_array_equal(s.inner_iterations(), [sol["its"] for sol in S.state["sols"]])
    v = np.random.default_rng(10).normal(size=P.ndof)
    _close(_np(s.tangent(v)), S.tangent(v), 1e-10)


@pytest.mark.parametrize("coarse", ["gdsw", "rgdsw"])
def test_hybrid_elasticity(coarse):
    """Hybrid coupling (eq. 11) on Neo-Hooke: F_h, the tangent (eq. 12) and
    the outer iteration as in the oracle."""
    case = synth.small_elasticity_case(nx=16, ny=8, boxes=(4, 2), overlap=1,
                                       traction=(0.5, -3.0), two_level=True)
    P = NHProblem(case)
    S = Schwarz(P, "hybrid", coarse=coarse)
    s = _solver(case, coupling="hybrid", coarse=coarse)
    u = _probe(P, 11)
    _close(_np(s.precond_residual(u)), S.evaluate(u), 1e-10)
    np.testing.assert_array_equal(s.inner_iterations(), [sol["its"] for sol in S.state["sols"]])
    v = np.random.default_rng(12).normal(size=P.ndof)
    _close(_np(s.tangent(v)), S.tangent(v), 1e-10)
    u_ref, st_ref = S.solve()
    uu, st, rc = _solver(case, coupling="hybrid", coarse=coarse).solve()
    assert rc == 0 and st["outer_its"] == st_ref["outer"]
    assert np.linalg.norm(_np(uu) - u_ref) <= 1e-10 * np.linalg.norm(u_ref)


@pytest.mark.parametrize("coupling", ["additive", "hybrid"])
def test_tuned_streams_elasticity(coupling):
    """Neo-Hooke with every stream option on (graphs, chord coarse steps,
    the second stream, the autotuner): the outer iteration, F_x and the
    tangent as in the oracle."""
    from paper_2410_24138_amd import nls
    f = nls.FLAG_GRAPH | nls.FLAG_COARSE_CHORD | nls.FLAG_OVERLAP | nls.FLAG_AUTOTUNE
    case = synth.small_elasticity_case(nx=18, ny=9, boxes=(3, 2), overlap=2,
                                       traction=(0.5, -3.0), two_level=True)
    P = NHProblem(case)
    S = Schwarz(P, coupling)
    u_ref, st_ref = S.solve()
    s = _solver(case, coupling=coupling, flags=f)
    uu, st, rc = s.solve()
    assert rc == 0 and st["outer_its"] == st_ref["outer"]
    assert np.linalg.norm(_np(uu) - u_ref) <= 1e-10 * np.linalg.norm(u_ref)
    u = 0.7 * u_ref  # an admissible point off the solution (det F > 0)
    ref = S.evaluate(u)
    assert np.all(np.isfinite(ref))
    _close(_np(s.precond_residual(u)), ref, 1e-10)
    v = np.random.default_rng(14).normal(size=P.ndof)
    _close(_np(s.tangent(v)), S.tangent(v), 1e-10)


def test_det_f_error_code():
    """A state that inverts elements (u_x = -2x: F_11 = -1, det F < 0) makes
    the local residuals undefined: the solver reports NLS_EDETF (the kernel
    finishes normally and flags the subdomain)."""
    from paper_2410_24138_amd import NLSError
    import paper_2410_24138_amd.nls as nls
    case = synth.small_elasticity_case(nx=12, ny=6, boxes=(3, 2), overlap=1,
                                       traction=(0.0, -1.0), two_level=False)
    P = NHProblem(case)
    u = np.zeros(P.ndof)
    u[0::2] = -2.0 * P.xy[:, 0]
    u[P.is_dir] = 0.0
    s = _solver(case, coupling="one_level")
    with pytest.raises(NLSError) as e:
        s.precond_residual(u)
    assert e.value.code == nls.NLS_EDETF


def test_structured_q1_mesh_and_load_factor():
    """nls_set_mesh_structured on Q1 gives the case's mesh (identical F and
    solve); a solve at load_factor 0.5 equals the oracle on the half load."""
    case = synth.small_elasticity_case(nx=16, ny=8, boxes=(4, 2), overlap=1,
                                       traction=(0.0, -3.0), two_level=True)
    a = _solver(case, coupling="additive")
    b = _solver(case, coupling="additive", structured=(16, 8, 2.0, 1.0))
    P = NHProblem(case)
    u = _probe(P, 5)
    np.testing.assert_array_equal(_np(a.residual(u)), _np(b.residual(u)))
    half = dict(case)
    half["nodal_force"] = 0.5 * case["nodal_force"]
    S = Schwarz(NHProblem(half), "additive")
    u_ref, st_ref = S.solve()
    uu, st, rc = b.solve(load_factor=0.5)
    assert rc == 0 and st["outer_its"] == st_ref["outer"]
    assert np.linalg.norm(_np(uu) - u_ref) <= 1e-10 * np.linalg.norm(u_ref)


def test_standalone_local_assembly_elasticity():
    """nls_eval_local on Neo-Hooke (2 dofs per node, 2x2 Gauss): residual
    and [J_ii | B_i] rows against the oracle, by global dof."""
    from tests.test_gpu_parity import _local_parts
    case = synth.small_elasticity_case(nx=12, ny=8, boxes=(3, 2), overlap=2,
                                       traction=(0.5, -2.0), two_level=False)
    P = NHProblem(case)
    S = Schwarz(P, "one_level")
    u = _probe(P, 4)
    s = _solver(case, coupling="one_level")
    for i, (vd, r, J) in enumerate(_local_parts(s, u)):
        sub = S.subs[i]
        ro = S.local_residual(i, u[sub["Vd"]], u[sub["Gd"]])
        Jo, Bo = S.local_jacobian(i, u[sub["Vd"]], u[sub["Gd"]])
        pos = {int(g): k for k, g in enumerate(sub["Vd"])}
        order = np.array([pos[int(g)] for g in vd])
        assert np.abs(r - ro[order]).max() <= 1e-12 * np.abs(ro).max()
        cols = np.concatenate([sub["Vd"], sub["Gd"]])
        Jfull = np.concatenate([Jo, Bo], axis=1)
        jscale = np.abs(Jfull).max()
        for a in range(len(sub["Vd"])):
            for c in np.nonzero(Jfull[a])[0]:
                key = (int(sub["Vd"][a]), int(cols[c]))
                assert abs(J.get(key, 0.0) - Jfull[a, c]) <= 1e-12 * jscale, key
        assert len(J) >= np.count_nonzero(Jfull)
