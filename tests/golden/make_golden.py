"""Write the stored oracle traces used by the GPU parity tests.

Calls only the FP64 CPU oracle and the seeded input generator.  Output:
tests/golden/<workload>.json with the outer Newton trace (outer, GMRES and
inner iteration counts, residual norms) and the solution at a fixed sample
of nodes, plus the brute-force global Newton solution at the same nodes;
tests/golden/<workload>.npz with the full vectors: "u", the oracle's
solution at the benchmark settings (outer rtol 1e-8, GMRES rtol 1e-6), and
"u_global_newton", the brute-force global Newton solution.

    python tests/golden/make_golden.py diffusion_512x512_16x16_ov2_gdsw

The RGDSW workload is the 512x512 problem with the RGDSW coarse space (its
u_global_newton is the same discrete solution and is not stored again).
The elasticity workload (10 load steps) stores the global Newton
continuation solution of every step (plain definition of the result) and,
with --schwarz, the oracle's outer Newton trace of every step; the .npz
holds the vectors of the last step.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import NHProblem, P1Problem, Schwarz, global_newton  # noqa: E402

CASES = {
    "diffusion_64x64_4x4_ov1": (synth.config1, "gdsw"),
    "diffusion_512x512_16x16_ov2_gdsw": (synth.config2, "gdsw"),
    "diffusion_512x512_16x16_ov2_rgdsw": (synth.config2, "rgdsw"),
}
ELASTIC = {"neohooke_256x128_8x8_ov2_gdsw": synth.config3}
N_STEPS = 10


def main_elastic(name, schwarz):
    case = ELASTIC[name]()
    P = NHProblem(case)
    rng = np.random.default_rng(321)
    sample = np.sort(rng.choice(P.ndof, size=256, replace=False))
    tip = 2 * (len(P.xy) - 1) + 1          # vertical dof of the top-right corner
    out = {"workload": name, "n_steps": N_STEPS, "sample_dofs": sample.tolist(),
           "tip_dof": int(tip), "steps": []}
    t0 = time.time()
    ug = np.zeros(P.ndof)
    for k in range(1, N_STEPS + 1):
        P.set_load_scale(k / N_STEPS)
        ug, its = global_newton(P, u0=ug)
        out["steps"].append({"scale": k / N_STEPS, "newton_its": its,
                             "u_global_newton_norm": float(np.linalg.norm(ug)),
                             "tip": float(ug[tip]),
                             "u_global_newton_sample": ug[sample].tolist()})
        print(k, its, float(ug[tip]), flush=True)
    out["global_newton_seconds"] = time.time() - t0
    if schwarz:
        P.set_load_scale(0.0)
        t0 = time.time()
        S = Schwarz(P, "additive")
        out["n0"] = int(S.n0)
        u, steps = S.solve_load_steps(N_STEPS, rtol=1e-8, gmres_rtol=1e-6,
                                      gmres_restart=50, gmres_maxit=1000)
        out["oracle_seconds"] = time.time() - t0
        out["settings"] = {"outer_rtol": 1e-8, "gmres_rtol": 1e-6, "gmres_restart": 50,
                           "gmres_maxit": 1000, "inner_rtol": 1e-12, "inner_eta": 1e-10,
                           "inner_maxit": 30}
        for rec, st in zip(out["steps"], steps):
            rec.update({"outer": st["outer"], "gmres": st["gmres"], "inner": st["inner"],
                        "coarse": st["coarse"], "converged": bool(st["converged"])})
        out["u_sample"] = u[sample].tolist()
        out["u_norm"] = float(np.linalg.norm(u))
        np.savez(os.path.join(HERE, name + ".npz"), u=u, u_global_newton=ug)
    with open(os.path.join(HERE, name + ".json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps({k: out[k] for k in out if k not in ("steps", "sample_dofs", "u_sample")}))


def main(name):
    make, coarse = CASES[name]
    case = make()
    P = P1Problem(case)
    coupling = "additive" if case["two_level"] else "one_level"
    t0 = time.time()
    S = Schwarz(P, coupling, coarse=coarse)
    t_setup = time.time() - t0
    t0 = time.time()
    u, st = S.solve(rtol=1e-8, gmres_rtol=1e-6, gmres_restart=50,
                    gmres_maxit=1000)
    t_solve = time.time() - t0
    ug, gits = global_newton(P)
    if coarse == "gdsw":
        np.savez(os.path.join(HERE, name + ".npz"), u=u, u_global_newton=ug)
    else:
        np.savez(os.path.join(HERE, name + ".npz"), u=u)
    rng = np.random.default_rng(123)
    sample = np.sort(rng.choice(P.N, size=256, replace=False))
    out = {
        "workload": name,
        "coupling": coupling,
        "coarse_space": coarse if case["two_level"] else "none",
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
    args = [a for a in sys.argv[1:] if not a.startswith("--")]
    for n in args or list(CASES) + list(ELASTIC):
        if n in ELASTIC:
            main_elastic(n, "--schwarz" in sys.argv)
        else:
            main(n)
