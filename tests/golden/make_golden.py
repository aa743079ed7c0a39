"""Write the stored oracle traces used by the GPU parity tests.

Calls only the FP64 CPU oracle and the seeded input generator.  Output:
tests/golden/<workload>.json with the outer Newton trace (outer, GMRES and
inner iteration counts, residual norms) and the solution at a fixed sample
of nodes, plus the brute-force global Newton solution at the same nodes.

    python tests/golden/make_golden.py diffusion_512x512_16x16_ov2_gdsw
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import P1Problem, Schwarz, global_newton  # noqa: E402

CASES = {
    "diffusion_64x64_4x4_ov1": synth.config1,
    "diffusion_512x512_16x16_ov2_gdsw": synth.config2,
}


def main(name):
    case = CASES[name]()
    P = P1Problem(case)
    coupling = "additive" if case["two_level"] else "one_level"
    t0 = time.time()
    S = Schwarz(P, coupling)
    t_setup = time.time() - t0
    t0 = time.time()
    u, st = S.solve(rtol=1e-8, gmres_rtol=1e-6, gmres_restart=50,
                    gmres_maxit=1000)
    t_solve = time.time() - t0
    ug, gits = global_newton(P)
    rng = np.random.default_rng(123)
    sample = np.sort(rng.choice(P.N, size=256, replace=False))
    out = {
        "workload": name,
        "coupling": coupling,
        "settings": {"outer_rtol": 1e-8, "gmres_rtol": 1e-6,
                     "gmres_restart": 50, "gmres_maxit": 1000,
                     "inner_rtol": 1e-12, "inner_eta": 1e-10,
                     "inner_maxit": 30},
        "outer": st["outer"], "gmres": st["gmres"], "inner": st["inner"],
        "coarse": st["coarse"], "res": st["res"],
        "converged": bool(st["converged"]),
        "n0": int(getattr(S, "n0", 0)),
        "u_norm": float(np.linalg.norm(u)),
        "sample_nodes": sample.tolist(),
        "u_sample": u[sample].tolist(),
        "u_global_newton_norm": float(np.linalg.norm(ug)),
        "u_global_newton_sample": ug[sample].tolist(),
        "rel_err_vs_global_newton": float(np.linalg.norm(u - ug) / np.linalg.norm(ug)),
        "oracle_seconds": {"setup": t_setup, "solve": t_solve},
    }
    with open(os.path.join(HERE, name + ".json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps({k: out[k] for k in ("outer", "gmres", "inner", "coarse",
                                          "res", "rel_err_vs_global_newton",
                                          "oracle_seconds")}))


if __name__ == "__main__":
    for n in sys.argv[1:] or list(CASES):
        main(n)
