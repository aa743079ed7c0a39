"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Tolerances (FP64 mode):
  * F(u): element-wise 1e-13 of max|F| (same formula, different summation
    order: a few ulps of the largest term);
  * F_x(u), tangent: element-wise 1e-11 of the max (local solves stop at the
    same Newton step on both sides; the rest is rounding of band LU vs
    dense LU, bounded by cond(J_ii) * eps ~ 1e3 * 1e-16 per solve);
  * solution of the outer iteration: relative 2-norm error 1e-10 against the
    oracle run with the same settings, and equal outer iteration counts.
Mixed mode (FP32 LU + FP64 refinement): relative error 1e-8 against FP64.
"""
import os

import numpy as np
import pytest

import synth
from oracle import P1Problem, Schwarz, global_newton
from tests._lib import ensure_built

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


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


SMALL = [
    dict(n=12, boxes=3, overlap=1),
    dict(n=13, boxes=3, overlap=2, uneven=True, forcing_seed=3),
    dict(n=20, boxes=4, overlap=2, coef_seed=7, forcing_seed=5),
    dict(n=17, boxes=2, overlap=1, forcing_seed=1, uneven=True),
]


@pytest.mark.parametrize("kw", SMALL)
def test_global_residual(kw):
    case = synth.small_case(**kw)
    P = P1Problem(case)
    s = _solver(case)
    rng = np.random.default_rng(0)
    u = rng.normal(size=P.N)
    _close(_np(s.residual(u)), P.residual(u), 1e-13)


def _probe_point(P, case, scale=0.5, seed=1):
    ug, _ = global_newton(P)
    rng = np.random.default_rng(seed)
    u = scale * ug + 0.1 * np.abs(ug).max() * rng.normal(size=P.N)
    u[P.is_dir] = P.dir_value[P.is_dir]
    return u


@pytest.mark.parametrize("coupling", ["one_level", "additive", "hybrid"])
@pytest.mark.parametrize("kw", SMALL)
def test_precond_residual_and_tangent(kw, coupling):
    case = synth.small_case(two_level=(coupling != "one_level"), **kw)
    P = P1Problem(case)
    S = Schwarz(P, coupling)
    s = _solver(case, coupling=coupling)
    u = _probe_point(P, case)
    Fx_ref = S.evaluate(u)
    Fx = _np(s.precond_residual(u))
    _close(Fx, Fx_ref, 1e-11)
    its = s.inner_iterations()
    np.testing.assert_array_equal(its, [sol["its"] for sol in S.state["sols"]])
    rng = np.random.default_rng(3)
    for _ in range(2):
        v = rng.normal(size=P.N)
        _close(_np(s.tangent(v)), S.tangent(v), 1e-11)


@pytest.mark.parametrize("coupling", ["one_level", "additive", "hybrid"])
def test_tangent_with_subdomains_under_one_block(coupling):
    """Subdomains of 9 rows (fewer than one 16-row block of the blocked
    tangent solve, kl = ku = 4): F_x and the tangent against the oracle."""
    kw = dict(n=6, boxes=3, overlap=1, forcing_seed=2)
    case = synth.small_case(two_level=(coupling != "one_level"), **kw)
    P = P1Problem(case)
    S = Schwarz(P, coupling)
    s = _solver(case, coupling=coupling)
    u = _probe_point(P, case)
    _close(_np(s.precond_residual(u)), S.evaluate(u), 1e-11)
    rng = np.random.default_rng(4)
    for _ in range(2):
        v = rng.normal(size=P.N)
        _close(_np(s.tangent(v)), S.tangent(v), 1e-11)


@pytest.mark.parametrize("kw", [dict(n=16, boxes=4, overlap=1),
                                dict(n=13, boxes=3, overlap=2, uneven=True, coef_seed=2),
                                dict(n=24, boxes=3, overlap=2, forcing_seed=9)])
def test_coarse_basis(kw):
    case = synth.small_case(two_level=True, **kw)
    S = Schwarz(P1Problem(case), "additive")
    s = _solver(case, coupling="additive")
    Phi = s.coarse_basis().toarray()
    _close(Phi, S.Phi.toarray(), 1e-12)


@pytest.mark.parametrize("coupling", ["one_level", "additive", "hybrid"])
@pytest.mark.parametrize("kw", [dict(n=12, boxes=3, overlap=1),
                                dict(n=24, boxes=4, overlap=2, forcing_seed=2),
                                dict(n=21, boxes=3, overlap=1, uneven=True, coef_seed=3)])
def test_solve_matches_oracle(kw, coupling):
    case = synth.small_case(two_level=(coupling != "one_level"), **kw)
    P = P1Problem(case)
    S = Schwarz(P, coupling)
    u_ref, st_ref = S.solve()
    s = _solver(case, coupling=coupling)
    u, st, rc = s.solve()
    u = _np(u)
    assert rc == 0 and st["converged"]
    assert st["outer_its"] == st_ref["outer"]
    assert np.linalg.norm(u - u_ref) <= 1e-10 * np.linalg.norm(u_ref)
    assert st["inner_its_total"] == sum(st_ref["inner"])
    for a, b in zip(st["gmres_its"], st_ref["gmres"]):
        assert abs(a - b) <= 1


@pytest.mark.parametrize("precision", ["fp32_ir", "bf16_ir"])
@pytest.mark.parametrize("two_level", [False, True])
def test_mixed_precision_matches_fp64(two_level, precision):
    """binary32 local LU (and the trial with bfloat16 operands in its
    trailing updates), FP64 residuals and refinement: the oracle's solution
    to 1e-8, the same outer and inner iteration counts as binary64."""
    case = synth.small_case(n=32, boxes=4, overlap=2, forcing_seed=4,
                            two_level=two_level)
    u64, st64, _ = _solver(case).solve()
    u32, st32, rc = _solver(case, precision=precision).solve()
    assert rc == 0 and st32["converged"]
    assert st32["outer_its"] == st64["outer_its"]
    assert st32["inner_its_total"] == st64["inner_its_total"]
    u64, u32 = _np(u64), _np(u32)
    assert np.linalg.norm(u32 - u64) <= 1e-8 * np.linalg.norm(u64)
    S = Schwarz(P1Problem(case), "additive" if two_level else "one_level")
    u_ref, st_ref = S.solve()
    assert np.linalg.norm(u32 - u_ref) <= 1e-8 * np.linalg.norm(u_ref)


def test_bf16_trial_elasticity():
    """The bfloat16 trial on Neo-Hooke Jacobians under load (row
    interchanges in the LU): F_x against the oracle to the mixed-mode bar."""
    from oracle import NHProblem
    case = synth.small_elasticity_case(nx=16, ny=8, boxes=(2, 2), overlap=2,
                                       traction=(1.0, -4.0), two_level=True)
    P = NHProblem(case)
    S = Schwarz(P, "additive")
    u_ref, st_ref = S.solve()
    uu, st, rc = _solver(case, coupling="additive", precision="bf16_ir").solve()
    assert rc == 0 and st["outer_its"] == st_ref["outer"]
    assert np.linalg.norm(_np(uu) - u_ref) <= 1e-8 * np.linalg.norm(u_ref)


def test_deterministic():
    case = synth.small_case(n=20, boxes=4, overlap=2, forcing_seed=6, two_level=True)
    s = _solver(case)
    u = np.random.default_rng(4).normal(size=len(case["xy"])) * 0.01
    a = _np(s.precond_residual(u))
    b = _np(s.precond_residual(u))
    np.testing.assert_array_equal(a, b)


def test_error_paths():
    from paper_2410_24138_amd import NLSError
    import paper_2410_24138_amd.nls as nls
    case = synth.small_case(n=12, boxes=3, overlap=1, forcing_seed=1)
    bad = dict(case)
    fl = case["elem_load"].copy()
    fl[5, 1] = np.nan
    bad["elem_load"] = fl
    with pytest.raises(NLSError) as e:
        _solver(bad).solve()
    assert e.value.code == nls.NLS_ENAN
    with pytest.raises(NLSError) as e:
        _solver(case, inner_maxit=1).solve(np.full(len(case["xy"]), 0.0))
    assert e.value.code == nls.NLS_ELOCAL
    s = _solver(case, gmres_maxit=1, outer_maxit=2)
    u, st, rc = s.solve()
    assert rc == nls.NLS_ENOCONV and not st["converged"] and st["outer_its"] == 2
    with pytest.raises(NLSError) as e:
        s.tangent(np.zeros(len(case["xy"]))) if False else _solver(case).tangent(
            np.zeros(len(case["xy"])))
    assert e.value.code == nls.NLS_ESTATE


def _batch_case():
    cs = [synth.small_case(n=12, boxes=3, overlap=2, forcing_seed=1, two_level=True),
          synth.small_case(n=17, boxes=2, overlap=2, coef_seed=3, two_level=True, uneven=True),
          synth.small_case(n=24, boxes=4, overlap=2, forcing_seed=5, two_level=True)]
    return synth.concat_cases(cs)


def test_batch_of_instances():
    """Independent problems joined into one disconnected mesh: one launch per
    size bucket over all their subdomains and a block-diagonal coarse level;
    F_x, the tangent and the solve match the oracle on the joined problem."""
    case = _batch_case()
    P = P1Problem(case)
    S = Schwarz(P, "additive")
    s = _solver(case, coupling="additive")
    u = _probe_point(P, case)
    _close(_np(s.precond_residual(u)), S.evaluate(u), 1e-11)
    v = np.random.default_rng(9).normal(size=P.N)
    _close(_np(s.tangent(v)), S.tangent(v), 1e-11)
    u_ref, st_ref = S.solve()
    uu, st, rc = _solver(case, coupling="additive").solve()
    uu = _np(uu)
    assert rc == 0 and st["outer_its"] == st_ref["outer"]
    assert np.linalg.norm(uu - u_ref) <= 1e-10 * np.linalg.norm(u_ref)


@pytest.mark.parametrize("coupling", ["one_level", "additive", "hybrid"])
def test_graph_gmres_matches_step_by_step(coupling):
    """GMRES with device-side rotations and graph-replayed Arnoldi blocks:
    same outer and GMRES counts and the same solution as the step-by-step
    driver; the captured graphs are replayed across outer iterations and
    solves, with eager work in between, and give identical results."""
    from paper_2410_24138_amd import nls
    case = synth.small_case(n=32, boxes=4, overlap=2, forcing_seed=7, coef_seed=2,
                            two_level=(coupling != "one_level"))
    ue, ste, _ = _solver(case, coupling=coupling).solve()
    sg = _solver(case, coupling=coupling, flags=nls.FLAG_GRAPH)
    ug1, stg1, rc = sg.solve()
    assert rc == 0 and stg1["outer_its"] == ste["outer_its"]
    for a, b in zip(stg1["gmres_its"], ste["gmres_its"]):
        assert abs(a - b) <= 1
    ue, ug1 = _np(ue), _np(ug1)
    assert np.linalg.norm(ug1 - ue) <= 1e-10 * np.linalg.norm(ue)
    F = _np(sg.residual(ug1))
    assert np.all(np.isfinite(F))
    for _ in range(2):
        ug2, stg2, _ = sg.solve()
        np.testing.assert_array_equal(_np(ug2), ug1)
        assert stg2["gmres_its"] == stg1["gmres_its"]


@pytest.mark.parametrize("flags", ["chord", "lu_apply", "chord+lu_apply+graph", "overlap",
                                   "chord+graph+overlap"])
def test_coarse_variants_match_oracle(flags):
    """Chord steps for T_0, band LU solves in place of the explicit coarse
    inverse, the coarse solve beside the local solves: F_x, the tangent and
    the solve match the oracle."""
    from paper_2410_24138_amd import nls
    f = 0
    f |= nls.FLAG_COARSE_CHORD if "chord" in flags else 0
    f |= nls.FLAG_COARSE_LU_APPLY if "lu_apply" in flags else 0
    f |= nls.FLAG_GRAPH if "graph" in flags else 0
    f |= nls.FLAG_OVERLAP if "overlap" in flags else 0
    case = synth.small_case(n=24, boxes=4, overlap=2, forcing_seed=2, two_level=True)
    P = P1Problem(case)
    S = Schwarz(P, "additive")
    u = _probe_point(P, case)
    s = _solver(case, coupling="additive", flags=f)
    _close(_np(s.precond_residual(u)), S.evaluate(u), 1e-10)
    v = np.random.default_rng(5).normal(size=P.N)
    _close(_np(s.tangent(v)), S.tangent(v), 1e-10)
    u_ref, st_ref = S.solve()
    uu, st, rc = _solver(case, coupling="additive", flags=f).solve()
    assert rc == 0 and st["outer_its"] == st_ref["outer"]
    assert np.linalg.norm(_np(uu) - u_ref) <= 1e-10 * np.linalg.norm(u_ref)


@pytest.mark.parametrize("variant", [1, 2, 3])
def test_lu_variants_match_oracle(variant):
    """Each band LU form (blocked NB=16, NB=8, unblocked) in the fused local
    solve: same F_x, tangent and inner iteration counts as the oracle."""
    kw = dict(n=21, boxes=3, overlap=2, uneven=True, coef_seed=4, forcing_seed=8)
    for coupling in ("one_level", "additive"):
        case = synth.small_case(two_level=(coupling == "additive"), **kw)
        P = P1Problem(case)
        S = Schwarz(P, coupling)
        s = _solver(case, coupling=coupling, lu_variant=variant)
        u = _probe_point(P, case)
        _close(_np(s.precond_residual(u)), S.evaluate(u), 1e-11)
        np.testing.assert_array_equal(s.inner_iterations(),
                                      [sol["its"] for sol in S.state["sols"]])
        v = np.random.default_rng(2).normal(size=P.N)
        _close(_np(s.tangent(v)), S.tangent(v), 1e-11)


def test_autotuned_solve_matches_oracle():
    from paper_2410_24138_amd import nls
    case = _batch_case()
    S = Schwarz(P1Problem(case), "additive")
    u_ref, st_ref = S.solve()
    f = nls.FLAG_AUTOTUNE | nls.FLAG_GRAPH | nls.FLAG_COARSE_CHORD
    s = _solver(case, coupling="additive", flags=f)
    before = s.tuning()
    uu, st, rc = s.solve()
    after = s.tuning()
    assert rc == 0 and st["outer_its"] == st_ref["outer"]
    assert np.linalg.norm(_np(uu) - u_ref) <= 1e-10 * np.linalg.norm(u_ref)
    assert before["lu_variant"] == [0] * len(before["lu_variant"])
    assert all(v in (1, 2, 3) for v in after["lu_variant"])
    assert all(0 < b <= 160 * 1024 for b in after["lds_bytes"])
    assert sum(after["n_sub"]) == int(case["n_sub"])
    assert min(after["coarse_ms"]) > 0.0
    uu2, st2, _ = s.solve()
    np.testing.assert_array_equal(_np(uu2), _np(uu))


def test_autotuned_precision_choice():
    """A mixed-precision handle with the autotuner runs its local solves in
    the faster of binary32-LU-with-refinement and binary64 LU; either way
    the solution is the oracle's to the mixed-precision tolerance and the
    outer iteration count is the same."""
    from paper_2410_24138_amd import nls
    case = _batch_case()
    S = Schwarz(P1Problem(case), "additive")
    u_ref, st_ref = S.solve()
    f = nls.FLAG_AUTOTUNE | nls.FLAG_GRAPH | nls.FLAG_COARSE_CHORD
    s = _solver(case, coupling="additive", precision="fp32_ir", flags=f)
    assert s.tuning()["local_precision"] == "fp32_ir"
    uu, st, rc = s.solve()
    assert rc == 0 and st["outer_its"] == st_ref["outer"]
    assert s.tuning()["local_precision"] in ("fp32_ir", "fp64")
    assert np.linalg.norm(_np(uu) - u_ref) <= 1e-8 * np.linalg.norm(u_ref)
    uu2, st2, _ = s.solve()
    assert np.linalg.norm(_np(uu2) - u_ref) <= 1e-8 * np.linalg.norm(u_ref)


@pytest.mark.parametrize("kw", [dict(n=24, boxes=4, overlap=2, forcing_seed=2),
                                dict(n=21, boxes=3, overlap=1, uneven=True, coef_seed=3)])
def test_rgdsw_matches_oracle(kw):
    """RGDSW option 2.2 coarse space (the paper's): basis, F_x, tangent and
    the solve match the oracle."""
    case = synth.small_case(two_level=True, **kw)
    P = P1Problem(case)
    S = Schwarz(P, "additive", coarse="rgdsw")
    s = _solver(case, coupling="additive", coarse="rgdsw")
    _close(s.coarse_basis().toarray(), S.Phi.toarray(), 1e-12)
    u = _probe_point(P, case)
    _close(_np(s.precond_residual(u)), S.evaluate(u), 1e-11)
    v = np.random.default_rng(8).normal(size=P.N)
    _close(_np(s.tangent(v)), S.tangent(v), 1e-11)
    u_ref, st_ref = S.solve()
    uu, st, rc = _solver(case, coupling="additive", coarse="rgdsw").solve()
    assert rc == 0 and st["outer_its"] == st_ref["outer"]
    assert np.linalg.norm(_np(uu) - u_ref) <= 1e-10 * np.linalg.norm(u_ref)


@pytest.mark.parametrize("flags", ["overlap", "chord+graph+overlap", "lu_apply+overlap"])
def test_hybrid_with_second_stream_matches_oracle(flags):
    """Hybrid coupling (eqs. 11, 12) with the second stream on: the tangent's
    coarse factorisations run beside the local ones (the coarse term of the
    hybrid tangent stays in series, it feeds the local term).  Uneven boxes,
    so that the local kernels run in several size buckets at once."""
    from paper_2410_24138_amd import nls
    f = nls.FLAG_OVERLAP
    f |= nls.FLAG_COARSE_CHORD if "chord" in flags else 0
    f |= nls.FLAG_COARSE_LU_APPLY if "lu_apply" in flags else 0
    f |= nls.FLAG_GRAPH if "graph" in flags else 0
    case = synth.small_case(n=48, boxes=3, overlap=2, uneven=True, coef_seed=5, forcing_seed=3,
                            two_level=True)
    P = P1Problem(case)
    S = Schwarz(P, "hybrid")
    s = _solver(case, coupling="hybrid", flags=f)
    assert len(s.tuning()["n_sub"]) >= 2  # several size buckets, one stream each
    u = _probe_point(P, case)
    _close(_np(s.precond_residual(u)), S.evaluate(u), 1e-10)
    np.testing.assert_array_equal(s.inner_iterations(), [sol["its"] for sol in S.state["sols"]])
    for seed in (3, 4):
        v = np.random.default_rng(seed).normal(size=P.N)
        _close(_np(s.tangent(v)), S.tangent(v), 1e-10)
    u_ref, st_ref = S.solve()
    uu, st, rc = _solver(case, coupling="hybrid", flags=f).solve()
    assert rc == 0 and st["outer_its"] == st_ref["outer"]
    assert np.linalg.norm(_np(uu) - u_ref) <= 1e-10 * np.linalg.norm(u_ref)


def test_structured_mesh_entry_point():
    """nls_set_mesh_structured generates the same P1 grid as the explicit
    mesh of the case: F(u) and the solve are identical."""
    case = synth.small_case(n=20, boxes=4, overlap=2, forcing_seed=2, two_level=True)
    a = _solver(case)
    b = _solver(case, structured=(20, 20, 1.0, 1.0))
    u = np.random.default_rng(3).normal(size=len(case["xy"]))
    np.testing.assert_array_equal(_np(a.residual(u)), _np(b.residual(u)))
    ua, sa, _ = a.solve()
    ub, sb, _ = b.solve()
    np.testing.assert_array_equal(_np(ua), _np(ub))
    assert sa["outer_its"] == sb["outer_its"]


def test_load_factor_matches_scaled_problem():
    """nls_solve with load_factor s solves the problem with the load samples
    scaled by s (oracle on the scaled case), and leaves the set load in
    place for the next solve."""
    case = synth.small_case(n=24, boxes=4, overlap=2, forcing_seed=5, two_level=True)
    scaled = dict(case)
    scaled["elem_load"] = 0.4 * case["elem_load"]
    S = Schwarz(P1Problem(scaled), "additive")
    u_ref, st_ref = S.solve()
    s = _solver(case)
    u, st, rc = s.solve(load_factor=0.4)
    assert rc == 0 and st["outer_its"] == st_ref["outer"]
    assert np.linalg.norm(_np(u) - u_ref) <= 1e-10 * np.linalg.norm(u_ref)
    u_full, _ = Schwarz(P1Problem(case), "additive").solve()
    u2, _, _ = s.solve()
    assert np.linalg.norm(_np(u2) - u_full) <= 1e-10 * np.linalg.norm(u_full)


def test_coarse_basis_at_linearisation_point():
    """nls_build_coarse with u_lin: the extension uses DF(u_lin); basis, F_x
    and the solve match the oracle built at the same point."""
    case = synth.small_case(n=24, boxes=4, overlap=2, forcing_seed=2, two_level=True)
    P = P1Problem(case)
    u_lin = 2.0 * np.sin(np.pi * P.xy[:, 0]) * np.sin(np.pi * P.xy[:, 1])
    S = Schwarz(P, "additive", coarse_lin=u_lin)
    s = _solver(case, coupling="additive", coarse_lin=u_lin)
    _close(s.coarse_basis().toarray(), S.Phi.toarray(), 1e-12)
    u = _probe_point(P, case)
    _close(_np(s.precond_residual(u)), S.evaluate(u), 1e-11)
    u_ref, st_ref = S.solve()
    uu, st, rc = _solver(case, coupling="additive", coarse_lin=u_lin).solve()
    assert rc == 0 and st["outer_its"] == st_ref["outer"]
    assert np.linalg.norm(_np(uu) - u_ref) <= 1e-10 * np.linalg.norm(u_ref)


def _local_parts(s, u):
    """GPU standalone assembly mapped to global dof ids: per subdomain the
    residual rows and the Jacobian rows as {(row dof, col dof): value}."""
    pat = s.local_pattern()
    r, jv = s.eval_local(u)
    r, jv = _np(r), _np(jv)
    out = []
    for i in range(len(pat["off_v"]) - 1):
        a0, a1 = pat["off_v"][i], pat["off_v"][i + 1]
        vd = pat["row_dof"][a0:a1]
        gd = pat["gamma_dof"][pat["off_g"][i]:pat["off_g"][i + 1]]
        colmap = np.concatenate([vd, gd])
        J = {}
        for a in range(a1 - a0):
            for t in range(pat["rowptr"][a0 + a], pat["rowptr"][a0 + a + 1]):
                J[(int(vd[a]), int(colmap[pat["col"][t]]))] = jv[t]
        out.append((vd, r[a0:a1], J))
    return out


@pytest.mark.parametrize("kw", [dict(n=16, boxes=4, overlap=2, forcing_seed=3, coef_seed=2),
                                dict(n=13, boxes=3, overlap=1, uneven=True)])
def test_standalone_local_assembly(kw):
    """nls_eval_local (A1-A3 on their own): the local residual R_i F(u) and
    the rows [J_ii | B_i] of every subdomain at x = R_i u against the
    oracle's local residual and Jacobian (patch elements only), mapped by
    global dof."""
    case = synth.small_case(**kw)
    P = P1Problem(case)
    S = Schwarz(P, "one_level")
    u = _probe_point(P, case)
    s = _solver(case)
    for i, (vd, r, J) in enumerate(_local_parts(s, u)):
        sub = S.subs[i]
        ro = S.local_residual(i, u[sub["Vd"]], u[sub["Gd"]])
        Jo, Bo = S.local_jacobian(i, u[sub["Vd"]], u[sub["Gd"]])
        pos = {int(g): k for k, g in enumerate(sub["Vd"])}
        order = np.array([pos[int(g)] for g in vd])
        scale = max(np.abs(ro).max(), 1e-300)
        assert np.abs(r - ro[order]).max() <= 1e-13 * scale
        cols = np.concatenate([sub["Vd"], sub["Gd"]])
        Jfull = np.concatenate([Jo, Bo], axis=1)
        jscale = np.abs(Jfull).max()
        dense = {}
        for a in range(len(sub["Vd"])):
            for c in np.nonzero(Jfull[a])[0]:
                dense[(int(sub["Vd"][a]), int(cols[c]))] = Jfull[a, c]
        for key, v in dense.items():
            assert abs(J.get(key, 0.0) - v) <= 1e-13 * jscale, key
        for key, v in J.items():
            assert abs(dense.get(key, 0.0) - v) <= 1e-13 * jscale, key
