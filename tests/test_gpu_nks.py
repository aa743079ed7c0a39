"""Newton-Krylov-Schwarz comparator on the GPU (nls_solve_nks through the C
ABI) against the oracle's NKS: equal outer iteration counts, GMRES counts
within one per step (classical Gram-Schmidt with reorthogonalisation vs
modified Gram-Schmidt), solutions within 1e-10 relative."""
import numpy as np
import pytest

import synth
from oracle import NKS, NHProblem, P1Problem, Schwarz, global_newton
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


def _check(P, case, coupling, coarse="gdsw"):
    S = Schwarz(P, coupling, coarse=coarse)
    u_ref, st_ref = NKS(S).solve()
    assert st_ref["converged"]
    s = _solver(case, coupling=coupling, coarse=coarse)
    u, st, rc = s.solve_nks()
    assert rc == 0 and st["converged"]
    assert st["outer_its"] == st_ref["outer"]
    for a, b in zip(st["gmres_its"], st_ref["gmres"]):
        assert abs(a - b) <= 1
    u = _np(u)
    assert np.linalg.norm(u - u_ref) <= 1e-10 * np.linalg.norm(u_ref)
    return s, st


@pytest.mark.parametrize("coupling,coarse", [("one_level", "gdsw"), ("additive", "gdsw"),
                                             ("additive", "rgdsw")])
@pytest.mark.parametrize("kw", [dict(n=24, boxes=4, overlap=2, forcing_seed=2),
                                dict(n=21, boxes=3, overlap=1, uneven=True, coef_seed=3)])
def test_nks_diffusion(kw, coupling, coarse):
    case = synth.small_case(two_level=(coupling != "one_level"), **kw)
    _check(P1Problem(case), case, coupling, coarse)


@pytest.mark.parametrize("coupling", ["one_level", "additive"])
def test_nks_elasticity(coupling):
    case = synth.small_elasticity_case(nx=16, ny=8, boxes=(4, 2), overlap=1,
                                       traction=(0.5, -3.0), two_level=(coupling != "one_level"))
    P = NHProblem(case)
    s, st = _check(P, case, coupling)
    # the NKS solution is the discrete solution
    ug, _ = global_newton(P)
    u, _, _ = s.solve_nks()
    assert np.linalg.norm(_np(u) - ug) <= 1e-7 * np.linalg.norm(ug)


def test_nks_then_schwarz_state():
    """nls_solve_nks overwrites the local factors; a following nonlinear
    Schwarz solve on the same handle evaluates afresh and matches."""
    case = synth.small_case(n=16, boxes=4, overlap=1, forcing_seed=4, two_level=True)
    P = P1Problem(case)
    S = Schwarz(P, "additive")
    u_ref, st_ref = S.solve()
    s = _solver(case, coupling="additive")
    s.solve_nks()
    u, st, rc = s.solve()
    assert rc == 0 and st["outer_its"] == st_ref["outer"]
    assert np.linalg.norm(_np(u) - u_ref) <= 1e-10 * np.linalg.norm(u_ref)


@pytest.mark.parametrize("method", ["nks", "additive", "hybrid"])
def test_beam_matches_oracle(method):
    """The paper's beam set-up (both ends clamped, volume force 6) with RGDSW
    on a small mesh: each method as in the oracle."""
    case = synth.beam_case(6.0, nx=40, ny=8, boxes=(5, 2), overlap=1)
    P = NHProblem(case)
    coupling = "additive" if method == "nks" else method
    S = Schwarz(P, coupling, coarse="rgdsw")
    if method == "nks":
        u_ref, st_ref = NKS(S).solve()
    else:
        u_ref, st_ref = S.solve()
    s = _solver(case, coupling=coupling, coarse="rgdsw")
    u, st, rc = s.solve_nks() if method == "nks" else s.solve()
    assert rc == 0 and st["converged"] and st["outer_its"] == st_ref["outer"]
    assert np.linalg.norm(_np(u) - u_ref) <= 1e-10 * np.linalg.norm(u_ref)
