"""Independent solves in one call (nls_solve_batch): four instances of the
batched diffusion workload (grids 139..161, 8x8 to 14x14 subdomains, overlap
2, GDSW, coefficient exp(g) of a unit-variance random field), each on a
stream of its own.  Per instance: its own outer Newton iteration and status;
the solution equals the oracle's for that instance alone (element-wise
1e-10, equal outer count) and is identical to the instance solved alone on
the GPU."""
import numpy as np
import pytest

import synth
from oracle import P1Problem, Schwarz
from tests._lib import ensure_built

pytestmark = pytest.mark.gpu

INSTANCES = (14, 24, 31, 3)


@pytest.fixture(scope="module", autouse=True)
def _lib():
    ensure_built()
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_solve_batch_matches_oracle_per_instance():
    import torch
    from paper_2410_24138_amd import Solver
    from paper_2410_24138_amd.nls import solve_batch
    cases = [synth.config4_instance(b) for b in INSTANCES]
    streams = [torch.cuda.Stream() for _ in cases]
    solvers = [Solver(c, stream=st.cuda_stream) for c, st in zip(cases, streams)]
    us, sts, codes, rc = solve_batch(solvers)
    assert rc == 0 and codes == [0] * len(cases)
    for case, s, u, st in zip(cases, solvers, us, sts):
        S = Schwarz(P1Problem(case), "additive")
        u_ref, st_ref = S.solve()
        un = u.cpu().numpy()
        assert st["converged"] and st["outer_its"] == st_ref["outer"], case["name"]
        err = np.abs(un - u_ref).max() / np.abs(u_ref).max()
        assert err <= 1e-10, (case["name"], err)
        alone, st1, _ = s.solve()
        np.testing.assert_array_equal(alone.cpu().numpy(), un)
        assert st1["outer_its"] == st["outer_its"]
    # a repeated handle is refused
    from paper_2410_24138_amd import NLSError
    with pytest.raises(NLSError):
        solve_batch([solvers[0], solvers[0]])
    for s in solvers:
        s.close()


def test_solve_batch_reports_each_instance():
    """One instance that cannot converge in its outer iteration limit (a
    single outer step) beside one that can: per-instance codes, and the
    batch returns NLS_ENOCONV."""
    import torch
    from paper_2410_24138_amd import Solver
    from paper_2410_24138_amd.nls import NLS_ENOCONV, solve_batch
    c0 = synth.config4_instance(14)
    c1 = synth.config4_instance(24)
    st0, st1 = torch.cuda.Stream(), torch.cuda.Stream()
    s0 = Solver(c0, stream=st0.cuda_stream)
    s1 = Solver(c1, stream=st1.cuda_stream, outer_maxit=1)
    us, sts, codes, rc = solve_batch([s0, s1])
    assert codes[0] == 0 and sts[0]["converged"]
    assert codes[1] == NLS_ENOCONV and not sts[1]["converged"] and sts[1]["outer_its"] == 1
    assert rc == NLS_ENOCONV
