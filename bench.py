#!/usr/bin/env python3
"""Benchmark of the two-level nonlinear Schwarz hot path on one MI355X.

Workload: nonlinear diffusion -div((1+u^2) grad u) = f on a 512x512 P1 grid
of the unit square (263,169 nodes), 16x16 box subdomains with a 2-element
overlap, additive two-level coupling with the GDSW coarse space, f a seeded
sum of 8 Fourier modes with amplitudes U(0,10), u_0 = 0, outer tolerance
1e-8.  One step = one complete outer Newton solve from u = 0 (all local
nonlinear solves, coarse corrections, GMRES on the exact tangent).

Forms: "plain" (FP64 everywhere, Newton for the coarse correction, GMRES
driven step by step from the host); "fp64_tuned" (FP64, GMRES rotations on
the device with blocks of Arnoldi steps replayed as HIP graphs, chord steps
for the coarse correction, autotuned LU variant per size bucket and coarse
apply strategy); "chosen" (as fp64_tuned with FP32 local LU and FP64
iterative refinement).  The JSON value is the fastest form whose solution
meets 1e-8 against the stored global Newton solution.  Every timed solve is checked
against the stored FP64 oracle trace (sampled solution, norm, outer count).

Prints one JSON line.  Metric: subdomain Newton solves per second
(local nonlinear solves T_i completed / wall time of the solves), with
time-to-1e-8 as ms_per_step.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "subdomain Newton solves/s; time-to-1e-8 per global solve, plain vs chosen"
# form -> (local LU precision, driver features)
FORMS = {
    "plain": ("fp64", ()),                 # FP64, GMRES step by step from the host
    "fp64_graph": ("fp64", ("graph",)),    # FP64, graph-replayed GMRES blocks
    # graphs, the coarse Newton solve beside the local solves, autotuned
    # LU variants and coarse apply
    "fp64_tuned": ("fp64", ("graph", "autotune", "overlap")),
    # as fp64_tuned with chord steps for the coarse correction (eq. 9): T_0
    # agrees with Newton's to the coarse stopping tolerance only
    "fp64_tuned_chord": ("fp64", ("graph", "chord", "autotune", "overlap")),
    # as fp64_tuned with the RGDSW coarse space (the paper's choice)
    "fp64_tuned_rgdsw": ("fp64", ("graph", "autotune", "overlap", "rgdsw")),
    # every pattern on a mixed-precision handle: the autotuner chooses the
    # local precision (FP32 LU with FP64 refinement, or FP64) by measured time
    "chosen": ("fp32_ir", ("graph", "autotune", "overlap")),
    # FP32 local LU + FP64 refinement kept throughout
    "fp32_ir": ("fp32_ir", ("graph", "overlap")),
    # trial: as fp32_ir with bfloat16 operands in the LU's trailing updates
    "bf16_ir": ("bf16_ir", ("graph", "overlap")),
}
HBM_PEAK_GBS = 8000.0
# HBM bytes per dispatch measured with rocprofv3 FETCH_SIZE/WRITE_SIZE (two
# passes, calibrated against a 256 MiB copy; profiles/hbm_traffic_*.md), valid
# only for the kernel source they were taken with.
MEASURED_TRAFFIC = {"kernels_sha1": "1b8d4f8c1ba10a1092991d3e2d9452176e14f1b7",
                    "bytes": {"k_local_newton": 1729753495, "k_local_factor": 397416786, "k_tangent_blocks": 359828439, "k_tangent_mfma": 3106679445, "k_tangent_gemv": 280765810, "k_coarse_galerkin": 84064600, "k_coarse_galerkin_sum": 97875451, "k_coarse_lu": 1517538, "k_coarse_inv_blocks": 1150762, "k_coarse_inv_mfma": 20875817, "k_coarse_apply_inverse": 4101910, "k_mdot_partial": 23556716, "k_maxpy_mdot_totals": 31341962, "k_prolong": 27326741, "k_coarse_ty": 20663292, "k_coarse_q": 80454912}}


def unit_work(case, elem_bytes=8):
    """Algorithmic work of one unit (one local Newton iteration of one
    subdomain) per subdomain, as the hot-path table counts it: residual
    bytes 8 (3 n_i + |Gamma_i|) (x, trace and load in, r out); Jacobian
    bytes 8 x 7 n_i (the sparse nonzeros out, 7 per row for P1); band factor
    bytes n_i (2 kl_i + ku_i + 1) x elem_bytes (the 3w + 1 stored diagonals);
    band LU flops 2 n_i kl_i^2 (w = kl)."""
    from paper_2410_24138_amd import nls
    m = nls.inspect_partition(case)
    n = (m["off_v"][1:] - m["off_v"][:-1]).astype(float)
    ng = (m["off_g"][1:] - m["off_g"][:-1]).astype(float)
    kl, ku = m["kl"].astype(float), m["ku"].astype(float)
    return {"residual": 8.0 * (3 * n + ng), "jacobian": 8.0 * 7 * n,
            "factor": n * (2 * kl + ku + 1) * elem_bytes, "lu_flops": 2.0 * n * kl * kl,
            "n": n, "ng": ng, "kl": kl, "ku": ku}


def _cpu_model():
    """CPU model name, sockets, physical cores and hardware threads of this
    host (from lscpu, else /proc/cpuinfo)."""
    import subprocess
    info = {"model": None, "sockets": None, "physical_cores": None, "threads": os.cpu_count()}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        kv = {}
        for line in out.splitlines():
            if ":" in line:
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
        info["model"] = kv.get("Model name")
        sockets = int(kv.get("Socket(s)", "0") or 0)
        cps = int(kv.get("Core(s) per socket", "0") or 0)
        info["sockets"] = sockets or None
        info["physical_cores"] = sockets * cps or None
        info["threads"] = int(kv.get("CPU(s)", info["threads"] or 0) or 0) or info["threads"]
    except Exception:
        pass
    if info["model"] is None:
        try:
            for line in open("/proc/cpuinfo"):
                if line.startswith("model name"):
                    info["model"] = line.split(":", 1)[1].strip()
                    break
        except OSError:
            pass
    return info


def cpu_baseline(case):
    """The oracle's full solve of the workload (outer Newton to 1e-8, the
    benchmark's settings) on the host, timed from u = 0 to the converged
    iterate with the set-up (maps, GDSW basis) timed apart; one BLAS thread
    (the oracle's loops are serial Python, its local LU a LAPACK band
    factorisation per subdomain).  Value: local nonlinear solves per second
    of solve time, the GPU line's unit."""
    import contextlib
    from oracle import P1Problem, Schwarz
    try:
        from threadpoolctl import threadpool_limits
        one_thread = threadpool_limits(limits=1)
    except Exception:
        one_thread = contextlib.nullcontext()
    with one_thread:
        t0 = time.perf_counter()
        S = Schwarz(P1Problem(case), "additive" if case.get("two_level") else "one_level")
        t_setup = time.perf_counter() - t0
        t0 = time.perf_counter()
        u, st = S.solve(rtol=1e-8, gmres_rtol=1e-6, gmres_restart=50, gmres_maxit=1000)
        t_solve = time.perf_counter() - t0
    solves = S.n_sub * (st["outer"] + 1)
    cpu = _cpu_model()
    return {"value": round(solves / t_solve, 2), "unit": "subdomain Newton solves/s",
            "cores": 1, "kind": "oracle",
            "time_to_1e-8_ms": round(1e3 * t_solve, 1), "setup_ms": round(1e3 * t_setup, 1),
            "outer_its": st["outer"], "gmres_its": st["gmres"], "inner_its": st["inner"],
            "converged": bool(st["converged"]),
            "host": cpu,
            "sample": f"the oracle's whole solve of {case['name']} from u = 0 to outer rtol "
                      f"1e-8 ({solves} local nonlinear solves in {st['outer'] + 1} "
                      f"evaluations, {sum(st['inner'])} local Newton steps, band LAPACK LU), "
                      f"one thread on {cpu.get('model')}"}


def make_solver(case, form, device_index=0, **kw):
    """The solver handle of a benchmark form (the flag sets of FORMS)."""
    from paper_2410_24138_amd import Solver, nls
    prec, extra = FORMS[form]
    return Solver(case, precision=prec, device=device_index,
                  coarse="rgdsw" if "rgdsw" in extra else "gdsw",
                  flags=nls.FLAG_PROFILE | (nls.FLAG_GRAPH if "graph" in extra else 0)
                  | (nls.FLAG_COARSE_CHORD if "chord" in extra else 0)
                  | (nls.FLAG_COARSE_LU_APPLY if "luapply" in extra else 0)
                  | (nls.FLAG_AUTOTUNE if "autotune" in extra else 0)
                  | (nls.FLAG_OVERLAP if "overlap" in extra else 0), **kw)


def golden_for(form, name="diffusion_512x512_16x16_ov2_gdsw"):
    """The stored oracle trace (json) and full vectors (npz: the oracle's
    solution at the same settings and coarse space, and the brute-force
    global Newton solution u*) that a form is checked against."""
    import numpy as np
    gname = name.replace("_gdsw", "_rgdsw") if "rgdsw" in FORMS[form][1] else name
    gdir = os.path.join(ROOT, "tests", "golden")
    golden = json.load(open(os.path.join(gdir, gname + ".json")))
    with np.load(os.path.join(gdir, gname + ".npz")) as z:
        u_ref = z["u"].copy()
    with np.load(os.path.join(gdir, name + ".npz")) as z:
        u_star = z["u_global_newton"].copy()
    return golden, u_ref, u_star


def parity_bar(res, form):
    """Relative error bar against the same-settings oracle: 1e-10 when the
    local solves ran in binary64 (all-FP64 mode), 1e-8 after refinement of
    binary32 local solves.  A chord coarse iteration is all-FP64 but agrees
    with the oracle's Newton T_0 to the coarse stopping tolerance only, so
    it does not meet the 1e-10 bar and is reported beside the headline."""
    return 1e-10 if _local_fp64(res, form) else 1e-8


def run_form(case, form, steps, warmup, device):
    import numpy as np
    import torch
    golden, u_ref, u_star = golden_for(form, case["name"])
    s = make_solver(case, form, device.index or 0)
    N = s.N
    for _ in range(warmup):
        u = torch.zeros(N, dtype=torch.float64, device=device)
        s.solve_(u)
    us = [torch.zeros(N, dtype=torch.float64, device=device) for _ in range(steps)]
    torch.cuda.synchronize(device)
    t0 = time.perf_counter()
    stats = [s.solve_(u) for u in us]
    torch.cuda.synchronize(device)
    wall = time.perf_counter() - t0
    errs, errs_or = [], []
    for u in us:
        un = u.cpu().numpy()
        errs.append(float(np.linalg.norm(un - u_star) / np.linalg.norm(u_star)))
        errs_or.append(float(np.abs(un - u_ref).max() / np.abs(u_ref).max()))
    solves = sum(st["local_solves"] for st in stats)
    out = {
        "ms_per_solve": 1e3 * wall / steps,
        "solves_per_s": solves / wall,
        "local_solves_per_step": solves / steps,
        "outer_its": stats[-1]["outer_its"],
        "gmres_its": stats[-1]["gmres_its"],
        "inner_its_total": stats[-1]["inner_its_total"],
        "coarse_its_total": stats[-1]["coarse_its_total"],
        "phase_ms": {k: round(sum(st[k] for st in stats) / steps, 3)
                     for k in ("ms_inner", "ms_coarse", "ms_gmres", "ms_other", "ms_overlap")},
        # ||u - u*||_2 / ||u*||_2 against the global Newton solution
        "rel_err_vs_global_newton": max(errs),
        # max_g |u_g - u_ref,g| / max |u_ref| against the oracle's solution
        # at the same settings and coarse space (full vectors)
        "rel_err_vs_oracle_same_settings": max(errs_or),
        "oracle_trace": golden["workload"],
        "outer_its_match_oracle": all(st["outer_its"] == golden["outer"] for st in stats),
        "converged": all(st["converged"] for st in stats),
        "kernels": {
            "local_newton": {"launches": sum(st["n_local_launches"] for st in stats),
                             "ms": sum(st["ms_local_kernel"] for st in stats)},
            "tangent_local": {"launches": sum(st["n_tangent_launches"] for st in stats),
                              "ms": sum(st["ms_tangent_kernel"] for st in stats)},
        },
        "inner_its_steps": sum(st["inner_its_total"] for st in stats),
        "tuning": s.tuning(),
    }
    out["parity_bar"] = parity_bar(out, form)
    # distance to u*: 1e-8, or the oracle's own distance at outer rtol 1e-8
    # where that is larger (64x64 one-level: 1.2e-8)
    star_bar = max(1e-8, golden.get("rel_err_vs_global_newton", 0.0) + 1e-10)
    out["meets_parity"] = bool(out["converged"] and out["outer_its_match_oracle"]
                               and out["rel_err_vs_oracle_same_settings"] <= out["parity_bar"]
                               and out["rel_err_vs_global_newton"] <= star_bar)
    s.close()
    return out


def run_batch(steps, warmup, device, n_inst=32):
    """Batch of independent diffusion solves (grids 128..384, 8..16 boxes per
    side, overlap 2, GDSW, kappa = exp(g) with a unit-variance random field),
    three ways: nls_solve_batch (one handle and stream per instance, every
    instance with its own outer Newton iteration and status, the handles
    driven concurrently); the instances one after another; and one handle
    over the joined disconnected mesh (every local solve of every instance
    in the same launches, but one stopping rule for the whole batch)."""
    import numpy as np
    import torch
    import synth
    from paper_2410_24138_amd import Solver
    from paper_2410_24138_amd.nls import solve_batch
    cases = [synth.config4_instance(b) for b in range(n_inst)]
    streams = [torch.cuda.Stream(device) for _ in cases]
    hs = [Solver(c, stream=st.cuda_stream) for c, st in zip(cases, streams)]
    for _ in range(warmup):
        solve_batch(hs)
    torch.cuda.synchronize(device)
    t0 = time.perf_counter()
    outs = [solve_batch(hs) for _ in range(steps)]
    torch.cuda.synchronize(device)
    t_batch = (time.perf_counter() - t0) / steps
    ub, st_b, codes, rc = outs[-1]
    # the same handles one after another
    for _ in range(warmup):
        for h in hs:
            h.solve()
    torch.cuda.synchronize(device)
    t0 = time.perf_counter()
    seq = [[h.solve() for h in hs] for _ in range(steps)]
    torch.cuda.synchronize(device)
    t_seq = (time.perf_counter() - t0) / steps
    diffs = [float((u1.cpu() - u2.cpu()).abs().max() / u2.cpu().abs().max())
             for u1, (u2, _, _) in zip(ub, seq[-1])]
    for h in hs:
        h.close()
    joined = synth.concat_cases(cases, name=f"diffusion_batch_{n_inst}_grf")
    sj = Solver(joined)
    N = sj.N
    for _ in range(warmup):
        sj.solve_(torch.zeros(N, dtype=torch.float64, device=device))
    us = [torch.zeros(N, dtype=torch.float64, device=device) for _ in range(steps)]
    torch.cuda.synchronize(device)
    t0 = time.perf_counter()
    st_j = [sj.solve_(u) for u in us]
    torch.cuda.synchronize(device)
    t_joined = (time.perf_counter() - t0) / steps
    uj = us[0].cpu().numpy()
    off, jdiff = 0, []
    for c, u2 in zip(cases, ub):
        ui = u2.cpu().numpy()
        jdiff.append(float(np.abs(uj[off:off + len(ui)] - ui).max() / np.abs(ui).max()))
        off += len(ui)
    sj.close()
    solves_b = sum(s["local_solves"] for s in st_b)
    return {
        "metric": "subdomain Newton solves/s (batch of independent solves)",
        "workload": joined["name"], "instances": n_inst, "nodes": N,
        "subdomains": int(joined["n_sub"]),
        "nls_solve_batch": {"ms_per_batch": round(1e3 * t_batch, 2),
                            "solves_per_s": round(solves_b / t_batch, 1),
                            "codes": codes, "all_converged": all(s["converged"] for s in st_b),
                            "outer_its": [s["outer_its"] for s in st_b],
                            "max_rel_diff_vs_alone": max(diffs)},
        "one_instance_after_another": {"ms_per_batch": round(1e3 * t_seq, 2),
                                       "solves_per_s": round(solves_b / t_seq, 1)},
        "joined_mesh_one_stopping_rule": {"ms_per_batch": round(1e3 * t_joined, 2),
                                          "outer_its": st_j[-1]["outer_its"],
                                          "converged": all(s["converged"] for s in st_j),
                                          "max_rel_diff_vs_per_instance": max(jdiff)},
        "speedup_batch_vs_sequential": round(t_seq / t_batch, 3),
    }


def run_learned(device, amp, train_seeds, eval_seeds, epochs, batch=256, capacity=100_000):
    """Learned initial guess on the 512x512 / 16x16 / overlap-2 / GDSW shape:
    capture (features, target) pairs from the solver's own local solves on
    training forcings (8 Fourier modes, amplitudes U(0, amp)), train the
    network on the GPU, then solve held-out forcings with and without it.
    Every held-out solve is timed from u = 0 to 1e-8; the solutions with and
    without the network are compared."""
    import numpy as np
    import torch
    import synth
    from paper_2410_24138_amd import Solver
    base = synth.config2()
    mid = synth.edge_midpoints(base["xy"], base["conn"])

    def load(seed):
        return synth.fourier_eval(mid, synth.fourier_modes(seed, amp=amp))

    s = Solver(base)
    N = s.N
    s.guess_capture(capacity)
    t0 = time.perf_counter()
    n_solves = 0
    for sd in train_seeds:
        s.set_load(load(sd))
        s.solve_(torch.zeros(N, dtype=torch.float64, device=device))
        n_solves += 1
        if s.guess_count() >= capacity:
            break
    torch.cuda.synchronize(device)
    t_capture = time.perf_counter() - t0
    X, T = s.guess_captured()
    n = X.shape[0]
    s.guess_capture(0)
    s.guess_set_model(synth.mlp_init(1))
    order = synth.epoch_orders(2, n, epochs)
    tr = s.guess_train(X, T, epochs=epochs, batch=batch, lr=1e-3, order=order, cosine=True)
    del X, T
    rows = []
    for sd in eval_seeds:
        s.set_load(load(sd))
        out = {}
        for mode in ("plain", "learned"):
            s.guess_enable(mode == "learned")
            s.solve_(torch.zeros(N, dtype=torch.float64, device=device))  # warm-up
            u = torch.zeros(N, dtype=torch.float64, device=device)
            torch.cuda.synchronize(device)
            t1 = time.perf_counter()
            st = s.solve_(u)
            torch.cuda.synchronize(device)
            out[mode] = {"ms": 1e3 * (time.perf_counter() - t1), "u": u, "st": st}
        diff = float(torch.linalg.norm(out["learned"]["u"] - out["plain"]["u"])
                     / torch.linalg.norm(out["plain"]["u"]))
        rows.append({"seed": sd,
                     "ms_plain": out["plain"]["ms"], "ms_learned": out["learned"]["ms"],
                     "inner_plain": out["plain"]["st"]["inner_its_total"],
                     "inner_learned": out["learned"]["st"]["inner_its_total"],
                     "outer_plain": out["plain"]["st"]["outer_its"],
                     "outer_learned": out["learned"]["st"]["outer_its"],
                     "used": out["learned"]["st"]["guess_used"],
                     "fallback": out["learned"]["st"]["guess_fallback"],
                     "solves": out["learned"]["st"]["local_solves"],
                     "converged": bool(out["plain"]["st"]["converged"]
                                       and out["learned"]["st"]["converged"]),
                     "rel_diff": diff})
    s.close()
    med = lambda k: float(np.median([r[k] for r in rows]))  # noqa: E731
    ip = sum(r["inner_plain"] for r in rows)
    il = sum(r["inner_learned"] for r in rows)
    return {
        "metric": "time-to-1e-8 per global solve with and without the learned initial guess",
        "workload": f"diffusion_512x512_16x16_ov2_gdsw_amp{amp:g}",
        "forcing": f"8 Fourier modes, amplitudes U(0,{amp:g}), k,l in 1..8",
        "train": {"seeds": f"{train_seeds[0]}..{train_seeds[0] + n_solves - 1}",
                  "samples": int(n), "capture_s": round(t_capture, 2), "epochs": epochs,
                  "batch": batch, "steps": tr["steps"], "train_ms": round(tr["ms"], 1),
                  "loss_first_epoch": tr["epoch_loss"][0], "loss_last_epoch": tr["final_loss"]},
        "eval_seeds": f"{eval_seeds[0]}..{eval_seeds[-1]}",
        "median_ms_plain": round(med("ms_plain"), 3),
        "median_ms_learned": round(med("ms_learned"), 3),
        "speedup": round(med("ms_plain") / med("ms_learned"), 4),
        "inner_its_plain": ip, "inner_its_learned": il,
        "inner_its_saved_frac": round(1 - il / ip, 4) if ip else None,
        "guess_used": sum(r["used"] for r in rows),
        "guess_fallback": sum(r["fallback"] for r in rows),
        "local_solves": sum(r["solves"] for r in rows),
        "outer_its_equal": all(r["outer_plain"] == r["outer_learned"] for r in rows),
        "all_converged": all(r["converged"] for r in rows),
        "max_rel_diff_learned_vs_plain": max(r["rel_diff"] for r in rows),
        "per_seed": [{k: (round(v, 3) if isinstance(v, float) and k != "rel_diff" else v)
                      for k, v in r.items()} for r in rows],
    }


def run_learned_nh(device, train_runs=40, epochs=30, batch=256, capacity=100_000,
                   n_load_steps=10, held_out=(6000, 6001, 6002)):
    """Learned initial guess on the 256x128 Q1 Neo-Hooke cantilever (8x8
    seeded cuts, overlap 2, GDSW, 10 load steps): (features, target) pairs
    captured from the solver's own converged local solves on training runs
    with cut seeds 5400.. and right-edge traction tau_max ~ U(2, 6), the
    network trained on the GPU, then the continuation solved with and
    without it: the 256x128 workload itself (cut seed 3, tau_max = 4) and
    held-out cut seeds with tau_max ~ U(2, 6).  Every continuation is timed
    from u = 0; solutions with and without the network are compared."""
    import torch
    import synth
    from paper_2410_24138_amd import Solver

    def case_for(seed, tau):
        cx, cy = synth.seeded_cuts(seed, 256, 128)
        return synth.elasticity_case(256, 128, 2.0, 1.0, cx, cy, 2, traction=(0.0, -tau),
                                     name=f"neohooke_256x128_cuts{seed}_tau{tau:.2f}")

    rng = np.random.default_rng(5400)
    Xs, Ts = [], []
    n = 0
    t0 = time.perf_counter()
    runs = 0
    for k in range(train_runs):
        tau = float(rng.uniform(2.0, 6.0))
        s = Solver(case_for(5400 + k, tau))
        s.guess_capture(capacity - n)
        s.solve_load_steps(n_load_steps)
        X, T = s.guess_captured()
        Xs.append(X.cpu())
        Ts.append(T.cpu())
        n += X.shape[0]
        runs += 1
        s.close()
        if n >= capacity:
            break
    t_capture = time.perf_counter() - t0
    X = torch.cat(Xs).to(device)
    T = torch.cat(Ts).to(device)
    del Xs, Ts
    trainer = Solver(synth.config3())
    trainer.guess_set_model(synth.mlp_init(1))
    order = synth.epoch_orders(2, n, epochs)
    tr = trainer.guess_train(X, T, epochs=epochs, batch=batch, lr=1e-3, order=order, cosine=True)
    params, norm = trainer.guess_get_model()
    trainer.close()
    del X, T
    evals = [("neohooke_256x128_8x8_ov2_gdsw", synth.config3())]
    for sd in held_out:
        evals.append((f"cuts{sd}", case_for(sd, float(np.random.default_rng(sd).uniform(2, 6)))))
    rows = []
    for name, case in evals:
        s = Solver(case)
        s.guess_set_model(params, norm)
        out = {}
        for mode in ("plain", "learned"):
            s.guess_enable(mode == "learned")
            s.solve_load_steps(n_load_steps)  # warm-up
            torch.cuda.synchronize(device)
            t1 = time.perf_counter()
            u, sts, rc = s.solve_load_steps(n_load_steps)
            torch.cuda.synchronize(device)
            out[mode] = {"ms": 1e3 * (time.perf_counter() - t1), "u": u, "sts": sts, "rc": rc}
        s.close()
        up, ul = out["plain"]["u"], out["learned"]["u"]
        sp, sl = out["plain"]["sts"], out["learned"]["sts"]
        rows.append({
            "case": name,
            "ms_plain": round(out["plain"]["ms"], 2), "ms_learned": round(out["learned"]["ms"], 2),
            "inner_plain": sum(st["inner_its_total"] for st in sp),
            "inner_learned": sum(st["inner_its_total"] for st in sl),
            "outer_plain": [st["outer_its"] for st in sp],
            "outer_learned": [st["outer_its"] for st in sl],
            "used": sum(st["guess_used"] for st in sl),
            "fallback": sum(st["guess_fallback"] for st in sl),
            "solves": sum(st["local_solves"] for st in sl),
            "converged": out["plain"]["rc"] == 0 and out["learned"]["rc"] == 0,
            "rel_diff": float(torch.linalg.norm(ul - up) / torch.linalg.norm(up))})
    ip = sum(r["inner_plain"] for r in rows)
    il = sum(r["inner_learned"] for r in rows)
    return {
        "metric": "time per 10-step continuation with and without the learned initial guess",
        "workload": "neohooke_256x128_8x8_ov2_gdsw (+ held-out cuts)",
        "train": {"runs": runs, "cut_seeds": f"5400..{5400 + runs - 1}", "tau_max": "U(2,6)",
                  "samples": int(n), "capture_s": round(t_capture, 2), "epochs": epochs,
                  "batch": batch, "steps": tr["steps"], "train_ms": round(tr["ms"], 1),
                  "loss_first_epoch": tr["epoch_loss"][0], "loss_last_epoch": tr["final_loss"]},
        "inner_its_plain": ip, "inner_its_learned": il,
        "inner_its_saved_frac": round(1 - il / ip, 4) if ip else None,
        "outer_its_equal": all(r["outer_plain"] == r["outer_learned"] for r in rows),
        "all_converged": all(r["converged"] for r in rows),
        "max_rel_diff_learned_vs_plain": max(r["rel_diff"] for r in rows),
        "speedup_config3": round(rows[0]["ms_plain"] / rows[0]["ms_learned"], 4),
        "per_case": rows,
    }


def run_elasticity(forms, steps, warmup, device, n_load_steps=10):
    """Compressible Neo-Hooke cantilever, 256x128 Q1 cells on [0,2]x[0,1]
    (66,306 dofs), 8x8 subdomains at seeded cuts, overlap 2, GDSW with
    translations and rotations, clamped at x = 0, right-edge traction
    ramped to (0,-4) in 10 load steps, each warm-started from the last.
    One step of this workload = the whole 10-step continuation from u = 0.
    Checked against the stored global Newton continuation solution."""
    import numpy as np
    import torch
    import synth
    from paper_2410_24138_amd import Solver, nls
    case = synth.config3()
    golden = json.load(open(os.path.join(ROOT, "tests", "golden", case["name"] + ".json")))
    idx = np.array(golden["sample_dofs"])
    ref = np.array(golden["steps"][-1]["u_global_newton_sample"])
    res = {}
    for f in forms:
        prec, extra = FORMS[f]
        s = Solver(case, precision=prec, device=device.index or 0,
                   coarse="rgdsw" if "rgdsw" in extra else "gdsw",
                   flags=nls.FLAG_PROFILE | (nls.FLAG_GRAPH if "graph" in extra else 0)
                   | (nls.FLAG_COARSE_CHORD if "chord" in extra else 0)
                   | (nls.FLAG_AUTOTUNE if "autotune" in extra else 0)
                   | (nls.FLAG_OVERLAP if "overlap" in extra else 0))
        from paper_2410_24138_amd import NLSError
        try:
            for _ in range(warmup):
                s.solve_load_steps(n_load_steps)
            torch.cuda.synchronize(device)
            t0 = time.perf_counter()
            outs = [s.solve_load_steps(n_load_steps) for _ in range(steps)]
            torch.cuda.synchronize(device)
            wall = (time.perf_counter() - t0) / steps
        except NLSError as e:
            # reported, not hidden: the form does not reach the solution
            res[f] = {"converged": False, "error": str(e), "code": int(e.code),
                      "rel_err_vs_global_newton": None, "ms_per_continuation": None}
            s.close()
            print(json.dumps({"form": f, **res[f]}), file=sys.stderr, flush=True)
            continue
        u, sts, rc = outs[-1]
        un = u.cpu().numpy()
        solves = sum(st["local_solves"] for st in sts)
        res[f] = {
            "ms_per_continuation": round(1e3 * wall, 3),
            "solves_per_s": round(solves / wall, 1),
            "outer_its": [st["outer_its"] for st in sts],
            "gmres_its": [st["gmres_its"] for st in sts],
            "inner_its_total": sum(st["inner_its_total"] for st in sts),
            "local_solves": solves,
            "converged": rc == 0 and all(st["converged"] for st in sts),
            "rel_err_vs_global_newton": float(np.abs(un[idx] - ref).max() / np.abs(ref).max()),
            "tip_deflection": float(un[golden["tip_dof"]]),
            "phase_ms": {k: round(sum(st[k] for st in sts), 3)
                         for k in ("ms_inner", "ms_coarse", "ms_gmres", "ms_other")},
            "tuning": s.tuning(),
        }
        if "steps" in golden and "outer" in golden["steps"][0]:
            res[f]["outer_its_oracle"] = [st["outer"] for st in golden["steps"]]
        s.close()
        print(json.dumps({"form": f, **res[f]}), file=sys.stderr, flush=True)
    ok = {f: r for f, r in res.items() if r["converged"] and r["rel_err_vs_global_newton"] <= 1e-8
          and "rgdsw" not in FORMS[f][1]}
    best = min(ok, key=lambda f: ok[f]["ms_per_continuation"]) if ok else forms[0]
    return {
        "metric": "time-to-1e-8 per 10-step load continuation; subdomain Newton solves/s",
        "workload": case["name"], "dofs": 2 * len(case["xy"]), "subdomains": case["n_sub"],
        "load_steps": n_load_steps, "best_form": best,
        "time_to_1e-8_ms": {f: r["ms_per_continuation"] for f, r in res.items()},
        "forms": res,
    }


# the paper's forces, then larger ones until the methods fail
BEAM_FORCES = (4.0, 4.5, 5.0, 6.0, 7.0, 7.5, 9.0, 10.0, 11.0, 12.0, 13.0, 14.0, 15.0)


def run_beam(device, forces=BEAM_FORCES, nx=320, ny=64, boxes=(20, 4)):
    """Robustness sweep on the paper's beam (both ends clamped, volume force
    (0, -f)): Newton-Krylov-Schwarz and the additive and hybrid nonlinear
    Schwarz methods, all with the RGDSW coarse space, each force solved from
    u = 0 with the paper's settings for this test (outer rtol 1e-4, inner
    rtol 1e-5, at most 100 GMRES iterations per outer step)."""
    import numpy as np
    import torch
    import synth
    from paper_2410_24138_amd import Solver
    from paper_2410_24138_amd.nls import NLSError
    opts = dict(outer_rtol=1e-4, inner_rtol=1e-5, gmres_maxit=100, outer_maxit=30)
    rows = []
    for f in forces:
        case = synth.beam_case(f, nx=nx, ny=ny, boxes=boxes, overlap=2)
        sols = {}
        for method in ("nks", "additive", "hybrid"):
            coupling = "additive" if method == "nks" else method
            s = Solver(case, coupling=coupling, coarse="rgdsw", device=device.index or 0, **opts)
            rec = {"force": f, "method": method}
            t0 = time.perf_counter()
            try:
                u, st, rc = s.solve_nks() if method == "nks" else s.solve()
                torch.cuda.synchronize(device)
                rec.update(ok=bool(rc == 0 and st["converged"]), rc=int(rc),
                           outer_its=st["outer_its"], gmres_total=st["gmres_its_total"],
                           res_ratio=st["res_final"] / max(st["res0"], 1e-300))
                if rec["ok"]:
                    sols[method] = u.detach().cpu().numpy()
            except NLSError as e:
                rec.update(ok=False, rc=int(e.code), error=str(e))
            rec["ms"] = round((time.perf_counter() - t0) * 1e3, 2)
            s.close()
            rows.append(rec)
            print(json.dumps(rec), file=sys.stderr, flush=True)
        if len(sols) > 1:
            ref = next(iter(sols.values()))
            spread = max(float(np.abs(v - ref).max()) for v in sols.values())
            for r in rows:
                if r["force"] == f:
                    r["max_diff_between_methods"] = spread
                    r["tip_scale"] = float(np.abs(ref).max())
    return {"workload": f"beam_{nx}x{ny}_{boxes[0]}x{boxes[1]}_ov2_rgdsw",
            "metric": "converged (yes/no), outer and GMRES iterations, time per force",
            "settings": opts, "runs": rows}


def run_assembly(device, reps=50):
    """The assembly step on its own at the 512x512 workload: nls_eval_local
    (local residual and Jacobian rows of all 256 subdomains at x = R_i u)
    called reps times; the kernel's duration comes from the kernel trace of
    this run (each call synchronises, so the wall time per call includes
    the launch).  Prints the bytes a launch moves."""
    import numpy as np
    import torch
    import synth
    from paper_2410_24138_amd import Solver
    case = synth.config2()
    with np.load(os.path.join(ROOT, "tests", "golden", case["name"] + ".npz")) as z:
        u = torch.from_numpy(z["u"]).to(device)
    s = Solver(case)
    pat = s.local_pattern()
    rows = len(pat["row_dof"])
    nnz = len(pat["col"])
    ng = len(pat["gamma_dof"])
    r = torch.empty(rows, dtype=torch.float64, device=device)
    jv = torch.empty(nnz, dtype=torch.float64, device=device)
    for _ in range(3):
        s.eval_local(u, r=r, jval=jv)
    torch.cuda.synchronize(device)
    t0 = time.perf_counter()
    for _ in range(reps):
        s.eval_local(u, r=r, jval=jv)
    torch.cuda.synchronize(device)
    wall_us = 1e6 * (time.perf_counter() - t0) / reps
    for _ in range(reps):
        s.eval_local(u, r=r, jacobian=False)
    torch.cuda.synchronize(device)
    s.close()
    alg = 8.0 * (3 * rows + ng) + 8.0 * nnz
    alg_res = 8.0 * (3 * rows + ng)
    return {"workload": case["name"], "kernel": "k_local_assemble",
            "rows": rows, "nnz": nnz, "gamma": ng, "reps": reps,
            "algorithmic_bytes_per_launch": alg,
            "algorithmic_bytes_residual_only": alg_res,
            "wall_us_per_call_incl_launch_and_sync": round(wall_us, 2)}


def measured_traffic(kernel):
    """Counter-measured HBM bytes of a kernel, or None if the source changed."""
    import hashlib
    src = os.path.join(ROOT, "paper_2410_24138_amd", "csrc", "kernels.hip")
    sha = hashlib.sha1(open(src, "rb").read()).hexdigest()
    if sha != MEASURED_TRAFFIC["kernels_sha1"]:
        return None
    return MEASURED_TRAFFIC["bytes"].get(kernel)


def _local_fp64(res, form):
    """Whether the local solves ran in FP64 (FP64 form, or the autotuner of
    a mixed form chose FP64)."""
    return FORMS[form][0] == "fp64" or res.get("tuning", {}).get("local_precision") == "fp64"


def roofline(case, res, form):
    """Roofline of the dominant kernel (the fused local Newton kernel, by
    event-timed share of the solve): achieved = algorithmic bytes per launch
    / average launch duration, the bytes being the per-unit figure (residual
    + Jacobian + band factor, unit_work) times the units one launch
    processes (the local Newton iterations of that evaluation, from the
    measured counts).  Also reported: the band-LU flop rate against the
    FP64 peak, the implementation's own bytes per launch (factors written
    and read back, Jacobian written and read), and the counter-measured
    HBM traffic where it was taken for this kernel source."""
    elem = 8 if _local_fp64(res, form) else 4
    w = unit_work(case, elem)
    k = res["kernels"]["local_newton"]
    launches = max(k["launches"], 1)
    units_per_launch = res["inner_its_steps"] / launches
    per_unit = float(np.mean(w["residual"] + w["jacobian"] + w["factor"]))
    per_launch = units_per_launch * per_unit
    flops = units_per_launch * float(np.mean(w["lu_flops"]))
    avg_s = k["ms"] / launches / 1e3
    achieved = per_launch / avg_s / 1e9
    # implementation: per step L and U written, U read by the backward
    # solve, J written and read, vectors
    n, ng, kl, ku = w["n"], w["ng"], w["kl"], w["ku"]
    fac = n * (2 * kl + ku + 1) * elem
    facu = n * (kl + ku + 1) * elem
    impl = units_per_launch * float(np.mean(fac + facu + 8 * 2 * 7 * n + 8 * 2 * n))
    traffic = measured_traffic("k_local_newton") if _local_fp64(res, form) else None
    return {"kernel": "k_local_newton", "bound": "hbm", "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "algorithmic_bytes_per_launch": round(per_launch),
            "bytes_per_unit": round(per_unit), "units_per_launch": round(units_per_launch, 2),
            "implementation_bytes_per_launch": round(impl),
            "traffic_over_algorithmic": round(traffic / per_launch, 3) if traffic else None,
            "lu_flops_per_launch": round(flops), "lu_tflops": round(flops / avg_s / 1e12, 3),
            "lu_flop_frac_fp64": round(flops / avg_s / 78.6e12, 5),
            "avg_launch_us": round(avg_s * 1e6, 2), "launches": k["launches"]}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--forms",
                    default="plain,fp64_tuned,chosen,fp32_ir,bf16_ir,fp64_tuned_chord,"
                            "fp64_tuned_rgdsw")
    ap.add_argument("--workload", default="diffusion512",
                    choices=["diffusion512", "diffusion64", "batch", "learned", "learned_nh",
                             "elasticity", "beam", "assembly"])
    ap.add_argument("--amp", type=float, default=10.0,
                    help="forcing amplitude of the learned workload")
    ap.add_argument("--train-seeds", type=int, default=130)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 256 MiB device copy (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the solver runs on a single MI355X; "
              "sharding the subdomains over several GPUs is not implemented", file=sys.stderr)
        sys.exit(2)
    import torch
    import synth
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    from paper_2410_24138_amd import nls
    if not os.path.exists(nls.LIB_PATH):
        from paper_2410_24138_amd.build import build
        build()
    device = torch.device("cuda", 0)
    if args.copy_calibration:
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device=device)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize(device)
        del src, dst
    if args.workload == "learned_nh":
        print(json.dumps(run_learned_nh(device, epochs=args.epochs)), flush=True)
        return
    if args.workload == "assembly":
        print(json.dumps(run_assembly(device)), flush=True)
        return
    if args.workload == "batch":
        print(json.dumps(run_batch(args.steps, args.warmup, device)), flush=True)
        return
    if args.workload == "beam":
        print(json.dumps(run_beam(device)), flush=True)
        return
    if args.workload == "elasticity":
        forms = [f for f in args.forms.split(",") if f]
        print(json.dumps(run_elasticity(forms, args.steps, args.warmup, device)), flush=True)
        return
    if args.workload == "learned":
        res = run_learned(device, args.amp, list(range(5000, 5000 + args.train_seeds)),
                          list(range(6000, 6010)), args.epochs)
        print(json.dumps(res), flush=True)
        return
    small = args.workload == "diffusion64"
    case = synth.config1() if small else synth.config2()
    forms = [f for f in args.forms.split(",") if f]
    if small:  # one level: no coarse space, so no chord or RGDSW forms
        forms = [f for f in forms if "chord" not in f and "rgdsw" not in f]
    res = {}
    for f in forms:
        res[f] = run_form(case, f, args.steps, args.warmup, device)
        print(json.dumps({"form": f, **{k: v for k, v in res[f].items()
                                        if k not in ("kernels",)}}), file=sys.stderr, flush=True)
    # the headline is the workload as named (GDSW vertex+edge coarse space),
    # among the forms that meet the parity bar (same outer iteration count as
    # the oracle, its solution to 1e-10 in binary64 or 1e-8 in mixed mode,
    # u* to 1e-8); RGDSW forms are reported beside it
    ok = {f: r for f, r in res.items() if r["meets_parity"] and "rgdsw" not in FORMS[f][1]}
    best = min(ok, key=lambda f: ok[f]["ms_per_solve"]) if ok else forms[0]
    r = res[best]
    line = {
        "metric": METRIC,
        "value": round(r["solves_per_s"], 1),
        "unit": "subdomain Newton solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["ms_per_solve"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if _local_fp64(r, best) else "f32+f64",
        "data": "synthetic",
        "config": {"workload": case["name"],
                   "grid": "64x64 P1" if small else "512x512 P1", "nodes": len(case["xy"]),
                   "subdomains": int(case["n_sub"]), "overlap": int(case["overlap"]),
                   "coarse": "none (one level)" if small else "GDSW vertex+edge",
                   "form": best, "outer_rtol": 1e-8, "parallelism": "1 GPU"},
        "time_to_1e-8_ms": {f: round(res[f]["ms_per_solve"], 3) for f in res},
        "forms": {f: {k: v for k, v in res[f].items()} for f in res},
        "roofline": roofline(case, r, best),
    }
    if "plain" in res and "chosen" in res:
        line["speedup_chosen_vs_plain"] = round(res["plain"]["ms_per_solve"]
                                                / res["chosen"]["ms_per_solve"], 3)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(case)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
