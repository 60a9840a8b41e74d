#!/usr/bin/env python3
"""IsoMP seconds/step on one MI355X, with the roofline of the dominant kernel and the oracle
timed on the host beside it.

A step is one isospectral-midpoint step (eq. (isomp)): fixed-point evaluations (stream solve,
A = P W~, lower Q = A P with the fused update and residual) until the change of W~ is below
1e-12 in the infinity norm.  The workload is synthetic: W_0 = sum_lm i omega_lm T_lm with seeded
random omega_lm (workloads/), assembled on the GPU by the library's basis kernel.

Prints ONE compact JSON line last on stdout (rank 0 of 1; the full record of every leg goes to
the --detail-out file, progress to stderr):
  value = seconds per step (lower is better), with inputs resident in HBM;
  roofline = the product A = P W~ (8 N^3 flops per launch) against the FP64 MFMA peak, its
  average launch time taken from HIP events recorded on the library's stream during the timed
  steps;
  cpu_baseline = the FP64 oracle (numpy/scipy, all host BLAS threads) on a bounded sample.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6  # MI355X dense FP64 (matrix and vector)

# Memory bytes per launch of zgemm_f64_kernel (A = P W~) at N = 4096, from two rocprofv3 --pmc
# passes (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each scaled by what the same counter
# reads for a plain copy of known size in the same runs (torch's clone of the 256 MiB W_0:
# 1.00 both ways).  Valid only for the kernel sources the counters were taken on.
MEASURED_TRAFFIC = {"N": 4096,
                    "sources": ["paper_2206_05466_amd/csrc/gemm_f64.hip",
                                "paper_2206_05466_amd/csrc/tile_f64.h"],
                    "sha256_16": "5c6a83e41b505c1f",
                    "bytes": (2532654.7 * 1.00 + 262144.0 * 1.00) * 1024}


def sources_hash(paths):
    import hashlib

    h = hashlib.sha256()
    for rel in paths:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(N):
    if N == MEASURED_TRAFFIC["N"] and MEASURED_TRAFFIC["bytes"] is not None and \
            sources_hash(MEASURED_TRAFFIC["sources"]) == MEASURED_TRAFFIC["sha256_16"]:
        return MEASURED_TRAFFIC["bytes"]
    return None



PAPER_S_PER_STEP_N4096 = 0.55  # Sec. 3.4: ~2500 CPU cores, ScaLAPACK, N = 4096, 3 iterations


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def blas_threads():
    try:
        from threadpoolctl import threadpool_info

        n = [d.get("num_threads", 0) for d in threadpool_info() if d.get("user_api") == "blas"]
        return max(n) if n else os.cpu_count()
    except Exception:
        return os.cpu_count()


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def ensemble_cpu_baseline(sizes, law, seed0, h, evals):
    """The oracle over the ensemble, one simulation after the other: one oracle step with
    `evals` evaluations (tol = 0) timed for the first simulation of each size, weighted by how
    many simulations have that size.  Returns oracle steps/s over the whole ensemble."""
    import oracle
    from workloads import omega_coeffs

    total = 0.0
    for n in sorted(set(sizes)):
        j = sizes.index(n)
        W0 = oracle.assemble(n, omega_coeffs(n, seed0 + j, law))
        t0 = time.perf_counter()
        oracle.isomp_step(W0, h, 0.0, evals)
        total += (time.perf_counter() - t0) * sizes.count(n)
    return {"value": len(sizes) / total, "unit": "steps/s", "cores": blas_threads(),
            "cpu_model": cpu_model(), "kind": "oracle",
            "sample": f"one oracle step with {evals} evaluation(s) per size class, weighted by the "
                      f"class counts {[sizes.count(n) for n in sorted(set(sizes))]}"}


def cpu_baseline(N, om_seed, law, h, mean_evals, lmax=32):
    """Oracle IsoMP step at the same N, scaled to the GPU run's mean number of evaluations.

    The oracle's per-step cost does not depend on the values of W, so its input is assembled
    (by the oracle) from the same seeded coefficients truncated to degree <= lmax, which keeps
    the O(N^3) full-spectrum basis computation out of the run.  One step with K evaluations
    (tol = 0 fixes the count) is timed, K the nearest whole number to the GPU's mean, and the
    time is scaled by mean / K (an evaluation is all but the whole cost of a step).
    """
    import numpy as np

    import oracle
    from workloads import omega_coeffs

    K = max(1, int(round(mean_evals)))
    om = omega_coeffs(N, om_seed, law, lmax=lmax)
    W0 = oracle.assemble(N, om, lmax=lmax)
    t0 = time.perf_counter()
    _, k, _ = oracle.isomp_step(W0, h, 0.0, K)
    dt = time.perf_counter() - t0
    assert k == K
    return {
        "value": dt * mean_evals / K,
        "unit": "s/step",
        "cores": blas_threads(),
        "cpu_model": cpu_model(),
        "kind": "oracle",
        "sample_short": f"1 oracle step, N={N}, {K} evaluations, scaled to {mean_evals:.2f}",
        "sample": (f"1 oracle IsoMP step at N={N} with K={K} evaluations ({dt:.2f} s), scaled by "
                   f"{mean_evals:.3f}/{K} to the GPU run's mean evaluations per step; input "
                   f"assembled by the oracle from the same seeded coefficients truncated to "
                   f"l<={lmax}; numpy/scipy FP64, OpenBLAS ZGEMM + LAPACK pttrs"),
    }


def _ens_split_slices():
    from workloads import WORKLOADS

    return WORKLOADS["ensemble64"]["split_slices"]


def ensemble_leg(nsteps, prec, ref=None, with_cpu=False):
    """64 independent simulations, N uniform over {128, 256, 384, 512}: one graph launch per step.
    Returns the record and the final states; with `ref` (the FP64 leg's final states, same
    initial states and step count) the record carries the largest relative Frobenius distance
    of a member to its FP64 counterpart."""
    import torch

    from paper_2206_05466_amd import PREC_SPLIT, Ensemble, Zeuler
    from workloads import WORKLOADS, ensemble_sizes, omega_coeffs

    cfg = WORKLOADS["ensemble64"]
    sizes = ensemble_sizes(cfg["nsim"], cfg["size_seed"], cfg["sizes"])
    # evaluation cap of the captured step: one above the most any step of this workload needs
    # (4, the first, from W_n, whose residual then just meets tol); start_step_* report that
    # step.  Split precision: the slices the parity tests check at this run's length (the
    # lower product takes one fewer)
    h, K, tol, slices = cfg["h"], cfg["K"], cfg["tol"], cfg["split_slices"]
    split = prec == PREC_SPLIT
    ctxs = {n: Zeuler(n) for n in sorted(set(sizes))}
    Ws = [ctxs[n].basis_assemble(omega_coeffs(n, cfg["seed0"] + j, cfg["law"])) for j, n in enumerate(sizes)]
    Wseq = [W.clone() for W in Ws]
    ens = Ensemble(sizes)
    ens.set_initial_guess(3)  # polynomial start, steps 1-3 with the run's states (reading 9)
    ens.set_update_form(1)    # W_{n+1} = W_n + h (A - A^H) (reading 12)
    ens.set_steady_cap(cfg["steady_cap"], cfg["steady_from"])
    if split:
        ens.set_split_slices(slices)
        for z in ctxs.values():
            z.set_split_slices(slices)
    ens.run(Ws, h, 1, tol, K, prec=prec)  # first run: autotuning + capture
    its0, res0 = ens.stats()  # a step from W_n: the most evaluations a step of the run needs
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ens.run(Ws, h, nsteps, tol, K, prec=prec)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    its, res = ens.stats()
    choice, tune_ms = ens.tuning(prec)
    dist = None
    if ref is not None:
        dist = max(float((torch.linalg.norm(W - R) / torch.linalg.norm(R)).item()) for W, R in zip(Ws, ref))
    # sequential reference: the single-simulation entry point, one simulation after the other
    seq_steps = max(1, min(5, nsteps))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for j, n in enumerate(sizes):
        ctxs[n].set_initial_guess(3)
        ctxs[n].set_update_form(1)
        ctxs[n].isomp_run(Wseq[j], h, seq_steps, tol, K, prec=prec)
    torch.cuda.synchronize()
    dts = time.perf_counter() - t1
    ens.close()
    for z in ctxs.values():
        z.close()
    n3 = sum(n ** 3 for n in sizes) / len(sizes)
    cands = (["work order: largest first", "work order: interleaved"] if split else
             ["128x64 tiles, largest first", "128x64 tiles, interleaved",
              "64x64 tiles, largest first", "64x64 tiles, interleaved"])
    rec = {
        "workload": f"ensemble64: {len(sizes)} simulations, N drawn from {cfg['sizes']} (seed "
                    f"{cfg['size_seed']}), simulation j seeded {cfg['seed0']}+j, sigma_l law "
                    f"{cfg['law']}, h={h}, tol={tol}, maxit={K}, polynomial start, "
                    + (f"split-precision products (INT8 MFMA, {slices} slices)" if split else "FP64 products"),
        "sizes_histogram": {str(n): sizes.count(n) for n in sorted(set(sizes))},
        "steps": nsteps,
        "s_per_ensemble_step": dt / nsteps,
        "aggregate_steps_per_s": len(sizes) * nsteps / dt,
        "last_step_iters": {"min": min(its), "max": max(its)},
        "last_step_max_resid": max(res),
        "start_step_iters": {"min": min(its0), "max": max(its0)},
        "start_step_max_resid": max(res0),
        "evaluation_cap": K,
        "steady_cap": {"cap": cfg["steady_cap"], "from_step": cfg["steady_from"]},
        "fp64_equiv_tflops": 12.0 * n3 * len(sizes) * sum(its) / len(its) / (dt / nsteps) / 1e12,
        "autotune": {"choice": choice, "ms_per_step": tune_ms, "candidates": cands},
        "sequential_single_context_steps_per_s": len(sizes) * seq_steps / dts,
        "speedup_vs_sequential": (len(sizes) * nsteps / dt) / (len(sizes) * seq_steps / dts),
    }
    if dist is not None:
        rec["max_member_rel_frobenius_vs_fp64_ensemble"] = dist
    if with_cpu:
        ev = max(1, int(round(sum(its) / len(its))))
        rec["cpu_baseline"] = ensemble_cpu_baseline(sizes, cfg["law"], cfg["seed0"], h, ev)
    return rec, Ws


def small_leg(steps):
    """Workload n512 (one simulation, N = 512, 100 steps): the single-simulation entry point
    (one host check of the residual per evaluation) and the same simulation as an ensemble of
    one (graph-captured step, on-device stopping)."""
    import torch

    from paper_2206_05466_amd import PREC_FP64, Ensemble, Zeuler
    from workloads import WORKLOADS, omega_coeffs

    cfg = WORKLOADS["n512"]
    N, h, tol = cfg["N"], cfg["h"], cfg["tol"]
    z = Zeuler(N)
    W0 = z.basis_assemble(omega_coeffs(N, cfg["seeds"][0], cfg["law"]))
    z.set_initial_guess(3)
    z.set_update_form(1)
    W = W0.clone()
    z.isomp_run(W, h, 2, tol, cfg["maxit"])
    W = W0.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its, res = z.isomp_run(W, h, steps, tol, cfg["maxit"])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # the stopping rule on the device (every evaluation up to the cap enqueued, skipped once the
    # step has converged): eagerly, and the whole run captured into one graph and replayed
    cap = 5
    z.set_stopping(1)
    Wd = W0.clone()
    z.isomp_run(Wd, h, 2, tol, cap)
    Wd = W0.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its_d, _ = z.isomp_run(Wd, h, steps, tol, cap)
    torch.cuda.synchronize()
    dt_dev = time.perf_counter() - t0
    sg = torch.cuda.Stream()
    zg = Zeuler(N, stream=sg)
    zg.set_stopping(1)
    zg.set_initial_guess(3)
    zg.set_update_form(1)
    zg.set_steady_cap(2, 4)  # from the fifth step: one skipped evaluation per step, not four
    Wgr = W0.clone()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=sg):
        zg.isomp_run_async(Wgr, h, steps, tol, cap)
    graph.replay()  # warm-up replay from W0
    torch.cuda.synchronize()
    Wgr.copy_(W0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    graph.replay()
    torch.cuda.synchronize()
    dt_graph = time.perf_counter() - t0
    its_g, _, _ = zg.run_stats(steps)
    dev_diff = float(torch.linalg.norm(Wgr - W).item() + torch.linalg.norm(Wd - W).item())
    del graph
    zg.close()
    Wg = W0.clone()
    with Ensemble([N]) as ens:  # the 64-simulation ensemble's settings
        ens.set_initial_guess(3)
        ens.set_update_form(1)
        ens.set_steady_cap(2, 4)
        ens.run([Wg.clone()], h, 2, tol, cap, prec=PREC_FP64)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ens.run([Wg], h, steps, tol, cap, prec=PREC_FP64)
        torch.cuda.synchronize()
        dtg = time.perf_counter() - t0
    diff = float((torch.linalg.norm(Wg - W) / torch.linalg.norm(W)).item())
    z.close()
    return {
        "workload": f"n512: one simulation, N={N}, sigma_l law {cfg['law']}, h={h}, tol={tol}, {steps} steps",
        "single_context_s_per_step": dt / steps,
        "iters_per_step": {"min": min(its), "max": max(its), "mean": sum(its) / len(its)},
        "device_stopping_s_per_step": dt_dev / steps,
        "device_stopping_graph_s_per_step": dt_graph / steps,
        "device_stopping_evaluation_cap": cap,
        "device_stopping_same_counts_and_result": its_d == list(its) and its_g == list(its) and dev_diff == 0.0,
        "graph_ensemble_of_one_s_per_step": dtg / steps,
        "rel_frobenius_between_the_two": diff,
        "note": "every form starts the steps after the first from the polynomial extrapolation "
                "of the run's midpoints and states (guess mode 3) and forms W_{n+1} = W_n + "
                "h (A - A^H); the captured run and the ensemble of one cap the evaluations at 5, "
                "and at 2 from the fifth step",
    }


def long_leg(steps):
    """Workload long512: the paper's long-run initial condition (random degrees 2..20, unit
    spectral norm, Sec. 4) at N = 512, `steps` steps with the polynomial start.  Every
    `sample` steps: the Casimirs C_2..C_5 and the kinetic energy (sum of E_l from the basis
    extraction); at the end the energy spectrum's share above degree 20 and its log-log
    slope over 21 <= l <= 200."""
    import numpy as np
    import torch

    from paper_2206_05466_amd import Zeuler
    from workloads import WORKLOADS, omega_coeffs

    cfg = WORKLOADS["long512"]
    N, h, tol, sample = cfg["N"], cfg["h"], cfg["tol"], cfg["sample"]
    z = Zeuler(N)
    W = z.basis_assemble(omega_coeffs(N, cfg["seed"], cfg["law"]))
    W /= float(np.linalg.norm(W.cpu().numpy(), 2))  # input recipe: unit spectral norm
    z.set_initial_guess(3)
    z.set_update_form(1)
    z.set_continuation(True)  # one trajectory: each call continues the last one's history
    nf0 = float(torch.linalg.norm(W).item())

    def diag():
        c = z.casimirs(W, 5)
        E = z.energy_spectrum(z.basis_extract(W)).cpu().numpy()
        return c, E

    c0, E0 = diag()
    rows, t_run, it_max, res_max, it_sum = [], 0.0, 0, 0.0, 0
    done = 0
    while done < steps:
        k = min(sample, steps - done)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        its, res = z.isomp_run(W, h, k, tol, cfg["maxit"])
        torch.cuda.synchronize()
        t_run += time.perf_counter() - t0
        it_max = max(it_max, max(its))
        it_sum += sum(its)
        res_max = max(res_max, max(res))
        done += k
        c, E = diag()
        if done % (100 * sample) == 0:
            log(f"long512: {done} steps, C2 drift {abs(c[1] - c0[1]) / abs(c0[1]):.2e}")
        rows.append({"step": done,
                     "C2_rel": abs(c[1] - c0[1]) / abs(c0[1]),
                     "C3_over_normF3": abs(c[2] - c0[2]) / nf0 ** 3,
                     "C4_rel": abs(c[3] - c0[3]) / abs(c0[3]),
                     "C5_over_normF5": abs(c[4] - c0[4]) / nf0 ** 5,
                     "energy_rel": abs(E.sum() - E0.sum()) / E0.sum()})
    l = np.arange(N)
    sel = (l >= 21) & (l <= 200) & (E > 0)
    slope = float(np.polyfit(np.log(l[sel]), np.log(E[sel]), 1)[0]) if sel.sum() > 2 else None
    z.set_continuation(False)
    # the same run from W_n at every step and from the linear start, drift at the end only
    # (at most 10^4 steps each)
    csteps = min(steps, 10000)
    other = {}
    for name, mode, form in (("start_from_Wn_every_step", 0, 0), ("linear_start", 1, 0),
                             ("polynomial_start_second_line_form", 2, 0),
                             ("linear_start_difference_form", 1, 1)):
        W = z.basis_assemble(omega_coeffs(N, cfg["seed"], cfg["law"]))
        W /= float(np.linalg.norm(W.cpu().numpy(), 2))
        z.set_initial_guess(mode)
        z.set_update_form(form)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        its0, res0 = z.isomp_run(W, h, csteps, tol, cfg["maxit"])
        torch.cuda.synchronize()
        t_o = time.perf_counter() - t0
        c, _ = diag()
        other[name] = {"steps": csteps, "s_per_step": t_o / csteps,
                       "mean_iters_per_step": sum(its0) / len(its0),
                       "max_resid": max(res0), "C2_rel": abs(c[1] - c0[1]) / abs(c0[1]),
                       "C4_rel": abs(c[3] - c0[3]) / abs(c0[3])}
    z.close()
    return {
        "workload": f"long512: N={N}, sigma_l law paper (degrees 2..20, seed {cfg['seed']}), "
                    f"unit spectral norm, h={h}, tol={tol}, {steps} steps, polynomial start "
                    f"(one trajectory: the calls between the samples every {sample} steps "
                    f"continue each other, ze_set_continuation)",
        "s_per_step": t_run / steps,
        "max_iters_per_step": it_max,
        "max_resid": res_max,
        "drift": rows,
        "energy_share_above_l20": {"start": float(E0[21:].sum() / E0.sum()),
                                   "end": float(E[21:].sum() / E.sum())},
        "end_spectrum_loglog_slope_l21_200": slope,
        "mean_iters_per_step": it_sum / steps,
        "start_from_Wn_every_step": other["start_from_Wn_every_step"],
        "linear_start": other["linear_start"],
        "polynomial_start_second_line_form": other["polynomial_start_second_line_form"],
        "linear_start_difference_form": other["linear_start_difference_form"],
        "update_forms": "main run: W_{n+1} = W_n + h (A - A^H); the comparison runs name theirs "
                        "(second line: the default, the second line of eq. (isomp))",
        "note": "Casimirs by ze_casimirs, energy by ze_basis_extract + ze_energy_spectrum, "
                "sampled between timed chunks (not in s_per_step)",
    }


def orders_leg():
    """Workload orders512: the long-run initial condition at N = 512 stepped to t = 2 at
    orders 2, 4 and 6 (ze_set_order) for several h, each compared with an order-6 run at a
    much smaller step: error, evaluations and time per unit of simulated time."""
    import numpy as np
    import torch

    from paper_2206_05466_amd import Zeuler
    from workloads import WORKLOADS, omega_coeffs

    cfg = WORKLOADS["orders512"]
    N, T, tol = cfg["N"], cfg["T"], cfg["tol"]
    z = Zeuler(N)
    W0 = z.basis_assemble(omega_coeffs(N, cfg["seed"], cfg["law"]))
    W0 /= float(np.linalg.norm(W0.cpu().numpy(), 2))
    z.set_initial_guess(2)
    z.set_update_form(1)

    def run(order, h):
        n = int(round(T / h))
        z.set_order(order)
        W = W0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        its, res = z.isomp_run(W, h, n, tol, cfg["maxit"])
        torch.cuda.synchronize()
        return W, time.perf_counter() - t0, sum(its), max(res)

    run(4, cfg["hs"][0])  # warm-up
    Wref, t_ref, e_ref, r_ref = run(6, cfg["h_ref"])
    nref = float(torch.linalg.norm(Wref).item())
    rows = []
    for order in (2, 4, 6):
        for h in cfg["hs"]:
            W, dt, ev, rmax = run(order, h)
            rows.append({"order": order, "h": h, "steps": int(round(T / h)), "evaluations": ev,
                         "s_per_unit_time": dt / T, "max_resid": rmax, "converged": rmax < tol,
                         "rel_frobenius_error": float(torch.linalg.norm(W - Wref).item()) / nref})
    z.close()
    return {
        "workload": f"orders512: N={N}, sigma_l law paper (seed {cfg['seed']}), unit spectral "
                    f"norm, t = 0 .. {T}, tol={tol}, polynomial substep starts, W_{{n+1}} = W_n + h C",
        "reference": {"order": 6, "h": cfg["h_ref"], "evaluations": e_ref, "max_resid": r_ref},
        "runs": rows,
        "note": "error is against the order-6 reference run (self-convergence), not an exact solution",
    }


def casimir_drift(c0, c1, W):
    """Relative drift of C_2, C_4; C_3 relative to ||W||_F^3 (C_3 can be tiny)."""
    import torch

    nf = float(torch.linalg.norm(W).item())
    return {f"C{k+1}": float(abs(c1[k] - c0[k]) / (abs(c0[k]) if k != 2 else nf ** 3)) for k in (1, 2, 3)}


def measure_single(wname, steps, warmup, slist, copy_probe_mib=0, with_mixed=True, with_crt=True):
    """One simulation of workload wname: FP64 (start from W_n, the linear start, then the
    polynomial start of the headline) and the split-precision runs (polynomial start), each over
    `steps` timed steps of one ze_isomp_run call from the same W0."""
    import torch

    from paper_2206_05466_amd import PREC_FP64, PREC_SPLIT, Zeuler
    from workloads import WORKLOADS, omega_coeffs

    cfg = WORKLOADS[wname]
    N, h, tol, maxit, law = cfg["N"], cfg["h"], cfg["tol"], cfg["maxit"], cfg["law"]
    seed = cfg["seeds"][0]
    z = Zeuler(N)
    log(f"workload {wname}: N={N} law={law} h={h} tol={tol}")
    t0 = time.perf_counter()
    W = z.basis_assemble(omega_coeffs(N, seed, law))
    torch.cuda.synchronize()
    log(f"W0 assembled on GPU in {time.perf_counter() - t0:.2f} s")
    c0 = z.casimirs(W, 4)
    W0 = W.clone()

    def timed_run(Wx, prec, guess, form=1, events=True):
        """Warm-up run, then one timed ze_isomp_run of `steps` steps on Wx (in place); events:
        the per-phase HIP events on (the kernels' live durations) or off."""
        z.set_update_form(form)
        z.set_initial_guess(guess)
        Ww = Wx.clone()
        z.isomp_run(Ww, h, max(warmup, 1), tol, maxit, prec)
        del Ww
        z.profile(events)
        z.profile_read(reset=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        its, res = z.isomp_run(Wx, h, steps, tol, maxit, prec)
        torch.cuda.synchronize()
        dtx = time.perf_counter() - t0
        prof = z.profile_read() if events else None
        z.profile(False)
        return dtx, its, res, prof

    # the default readings: W~ starts from W_n, W_{n+1} from the second line of eq. (isomp)
    Wp = W0.clone()
    dt_plain, iters_plain, _, _ = timed_run(Wp, PREC_FP64, 0, 0)
    log(f"{wname} fp64, start W_n: {dt_plain / steps * 1e3:.2f} ms/step, iters={iters_plain}")
    # steps after the first start from 2 W_n - F_prev
    Wl = W0.clone()
    dt_lin, iters_lin, _, _ = timed_run(Wl, PREC_FP64, 1, 0)
    log(f"{wname} fp64, linear start: {dt_lin / steps * 1e3:.2f} ms/step, iters={iters_lin}")
    # polynomial start with the second-line form of W_{n+1}
    Ws2 = W0.clone()
    dt_p0, iters_p0, _, _ = timed_run(Ws2, PREC_FP64, 2, 0)
    log(f"{wname} fp64, polynomial start, second-line form: {dt_p0 / steps * 1e3:.2f} ms/step, "
        f"iters={iters_p0}")
    # the polynomial start from the midpoints alone, W_{n+1} = W_n + h C
    Wm2 = W0.clone()
    dt_m2, iters_m2, _, _ = timed_run(Wm2, PREC_FP64, 2, 1)
    log(f"{wname} fp64, polynomial start (midpoints only): {dt_m2 / steps * 1e3:.2f} ms/step, "
        f"iters={iters_m2}")
    # headline: polynomial extrapolation of the run's previous midpoints, the third and fourth
    # steps with the run's states as well, W_{n+1} = W_n + h C
    dt, iters, resids, prof = timed_run(W, PREC_FP64, 3, 1)
    log(f"{wname} fp64, polynomial start: {dt / steps * 1e3:.2f} ms/step, iters={iters}")
    # the same run without the per-phase events: what they cost
    Wq = W0.clone()
    dt_q, iters_q, _, _ = timed_run(Wq, PREC_FP64, 3, 1, events=False)
    quiet_same = bool(torch.equal(Wq, W)) and list(iters_q) == list(iters)
    del Wq
    log(f"{wname} fp64, polynomial start, no phase events: {dt_q / steps * 1e3:.2f} ms/step "
        f"(same result: {quiet_same})")
    c1 = z.casimirs(W, 4)
    plain_vs_extrap = float(torch.linalg.norm(Wp - W).item() / torch.linalg.norm(W).item())
    lin_vs_extrap = float(torch.linalg.norm(Wl - W).item() / torch.linalg.norm(W).item())
    p0_vs_extrap = float(torch.linalg.norm(Ws2 - W).item() / torch.linalg.norm(W).item())
    m2_vs_extrap = float(torch.linalg.norm(Wm2 - W).item() / torch.linalg.norm(W).item())
    del Wl, Ws2, Wm2
    if copy_probe_mib > 0:
        n = copy_probe_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # mixed: A = P W~ in FP64, the lower product (h^2/4 weight) on INT8 with 4 slices
    mixed = crt = None
    if with_mixed:
        mixed = mixed_run(z, timed_run, W0, W, c0, dt, steps, wname)
    if with_crt:
        crt = crt_run(z, timed_run, W0, W, c0, dt, steps, wname)

    split = None
    if slist:
        runs = []
        for ns in slist:
            z.set_split_slices(ns)
            Ws = W0.clone()
            dts, its_s, _, profs = timed_run(Ws, PREC_SPLIT, 3)
            cs = z.casimirs(Ws, 4)
            diff = float(torch.linalg.norm(Ws - W).item() / torch.linalg.norm(W).item())
            sps = dts / steps
            p1 = profs["product_PW"][0] / max(profs["product_PW"][1], 1)
            drift_s = casimir_drift(c0, cs, Ws)
            runs.append({
                "slices": ns,
                "s_per_step": sps,
                "speedup_vs_fp64": (dt / steps) / sps,
                "iters_per_step": list(its_s),
                "rel_frobenius_vs_fp64_run": diff,
                "casimir_drift_rel": drift_s,
                "meets_stated_accuracy": diff <= 1e-10 and max(drift_s.values()) <= 1e-11,
                "phases": {k: {"avg_ms": v[0] / max(v[1], 1), "launches": v[1]} for k, v in profs.items()},
                "product_PW_fp64_equiv_tflops": 8.0 * N ** 3 / (p1 * 1e-3) / 1e12,
                "product_PW_int8_tops": 8.0 * N ** 3 * ns * (ns + 1) / 2 / (p1 * 1e-3) / 1e12,
            })
            log(f"{wname} split s={ns}: {sps*1e3:.2f} ms/step, rel diff vs fp64 {diff:.2e}")
        ok = [r for r in runs if r["meets_stated_accuracy"]]
        best = min(ok, key=lambda r: r["s_per_step"]) if ok else None
        split = {
            "stated_accuracy": "after the timed steps, rel. Frobenius distance to the FP64 run <= 1e-10 "
                               "and Casimir drift <= 1e-11 (the FP64 path's parity bar)",
            "best_at_stated_accuracy": None if best is None else {
                "slices": best["slices"], "s_per_step": best["s_per_step"],
                "speedup_vs_fp64": best["speedup_vs_fp64"],
                "rel_frobenius_vs_fp64_run": best["rel_frobenius_vs_fp64_run"]},
            "runs": runs,
            "note": "same W0 and step count as the FP64 run; product_PW includes the slicing kernels",
        }
    z.close()
    return {
        "N": N, "h": h, "tol": tol, "maxit": maxit, "law": law, "seed": seed, "steps": steps,
        "s_per_step": dt / steps, "iters_per_step": list(iters), "max_resid": max(resids),
        "prof": prof, "casimir_drift_rel": casimir_drift(c0, c1, W),
        "without_phase_events": {"s_per_step": dt_q / steps, "same_result": quiet_same},
        "fp64_start_from_Wn": {"s_per_step": dt_plain / steps, "iters_per_step": list(iters_plain),
                               "rel_frobenius_vs_headline_run": plain_vs_extrap},
        "fp64_linear_start": {"s_per_step": dt_lin / steps, "iters_per_step": list(iters_lin),
                              "rel_frobenius_vs_headline_run": lin_vs_extrap},
        "fp64_polynomial_start_second_line_form": {
            "s_per_step": dt_p0 / steps, "iters_per_step": list(iters_p0),
            "rel_frobenius_vs_headline_run": p0_vs_extrap},
        "fp64_polynomial_start_midpoints_only": {
            "s_per_step": dt_m2 / steps, "iters_per_step": list(iters_m2),
            "rel_frobenius_vs_headline_run": m2_vs_extrap},
        "split_precision": split,
        "mixed_precision": mixed,
        "crt_precision": crt,
    }


def crt_run(z, timed_run, W0, W, c0, dt, steps, wname):
    """The same run with ZE_PREC_CRT (A = P W~ in the modular INT8 form, the lower product on
    INT8 with 4 slices), compared with the FP64 headline run W; plus the product alone."""
    import torch

    from paper_2206_05466_amd import PREC_CRT, PREC_FP64

    z.set_split_slices(5)
    Wc = W0.clone()
    dtc, its_c, res_c, prof_c = timed_run(Wc, PREC_CRT, 3)
    N = W.shape[0]
    Xa, Xb = W0.clone(), Wc.clone()
    out = torch.empty_like(Xa)
    gemm = {}
    for name, prec in (("fp64", PREC_FP64), ("crt", PREC_CRT)):
        z.zgemm(Xa, Xb, out, prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            z.zgemm(Xa, Xb, out, prec)
        torch.cuda.synchronize()
        gemm[name] = (time.perf_counter() - t0) / 3
        gemm[name + "_result"] = out.clone()
    rel_gemm = float((torch.linalg.norm(gemm["crt_result"] - gemm["fp64_result"]) /
                      torch.linalg.norm(gemm["fp64_result"])).item())
    rec = {
        "s_per_step": dtc / steps, "speedup_vs_fp64": dt / dtc,
        "iters_per_step": list(its_c), "max_resid": max(res_c), "moduli": 16,
        "rel_frobenius_vs_fp64_run": float(torch.linalg.norm(Wc - W).item() / torch.linalg.norm(W).item()),
        "casimir_drift_rel": casimir_drift(c0, z.casimirs(Wc, 4), Wc),
        "phases": {k: {"avg_ms": v[0] / max(v[1], 1), "launches": v[1]} for k, v in prof_c.items()},
        "zgemm_ms": {"fp64": gemm["fp64"] * 1e3, "crt": gemm["crt"] * 1e3},
        "zgemm_crt_fp64_equiv_tflops": 8.0 * N ** 3 / gemm["crt"] / 1e12,
        "zgemm_rel_frobenius_crt_vs_fp64": rel_gemm,
    }
    log(f"{wname} crt (modular INT8 A, 4-slice Q): {dtc / steps * 1e3:.2f} ms/step, rel diff vs fp64 "
        f"{rec['rel_frobenius_vs_fp64_run']:.2e}; zgemm {gemm['crt'] * 1e3:.2f} vs fp64 {gemm['fp64'] * 1e3:.2f} ms")
    return rec


def mixed_run(z, timed_run, W0, W, c0, dt, steps, wname):
    """The same run with ZE_PREC_MIXED (FP64 A = P W~, the lower product on INT8 with 4
    slices), compared with the FP64 headline run W."""
    import torch

    from paper_2206_05466_amd import PREC_MIXED

    z.set_split_slices(5)
    Wm = W0.clone()
    dtm, its_m, res_m, prof_m = timed_run(Wm, PREC_MIXED, 3)
    mixed = {
        "s_per_step": dtm / steps, "speedup_vs_fp64": dt / dtm,
        "iters_per_step": list(its_m), "max_resid": max(res_m), "lower_product_slices": 4,
        "rel_frobenius_vs_fp64_run": float(torch.linalg.norm(Wm - W).item() / torch.linalg.norm(W).item()),
        "casimir_drift_rel": casimir_drift(c0, z.casimirs(Wm, 4), Wm),
        "phases": {k: {"avg_ms": v[0] / max(v[1], 1), "launches": v[1]} for k, v in prof_m.items()},
    }
    log(f"{wname} mixed (FP64 A, 4-slice Q): {dtm / steps * 1e3:.2f} ms/step, rel diff vs fp64 "
        f"{mixed['rel_frobenius_vs_fp64_run']:.2e}")
    return mixed


def phases_of(prof):
    return {k: {"avg_ms": v[0] / max(v[1], 1), "launches": v[1]} for k, v in prof.items()}


def _sig(x, digits=4):
    """x rounded to `digits` significant digits (None and non-floats pass through)."""
    if isinstance(x, float) and x == x and x not in (float("inf"), float("-inf")) and x != 0.0:
        return float(f"{x:.{digits - 1}e}")
    return x


def _pick(rec, *keys):
    for k in keys:
        if rec is None:
            return None
        rec = rec.get(k) if isinstance(rec, dict) else None
    return rec


def compact_record(out, detail_path=None):
    """The one JSON line bench.py prints last: the headline, the roofline and the CPU baseline
    of the full record, and one or two figures from each leg (the whole record goes to the
    detail file).  Stays well under 2 KB."""
    def leg_split(rec):
        best = _pick(rec, "split_precision", "best_at_stated_accuracy")
        if not best:
            return None
        return {"slices": best["slices"], "s_per_step": _sig(best["s_per_step"]),
                "speedup_vs_fp64": _sig(best["speedup_vs_fp64"], 3),
                "rel_vs_fp64_run": _sig(best["rel_frobenius_vs_fp64_run"], 2)}

    def leg_alt(rec):
        if not rec:
            return None
        return {"s_per_step": _sig(rec["s_per_step"]), "speedup_vs_fp64": _sig(rec["speedup_vs_fp64"], 3),
                "rel_vs_fp64_run": _sig(rec["rel_frobenius_vs_fp64_run"], 2)}

    iters = out["iters_per_step"]
    ph = out["phases"]
    roof = dict(out["roofline"])
    roof.pop("context_library_zgemm", None)
    roof = {k: _sig(v) for k, v in roof.items()}
    wn = out["fp64_start_from_Wn"]
    rec = {k: out[k] for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
                               "steps_per_s", "higher_is_better", "scaling", "vs_baseline", "dtype",
                               "data")}
    for k in ("ms_per_step", "steps_per_s", "vs_baseline"):
        rec[k] = _sig(rec[k])
    cfg = out["config"]
    rec["config"] = {"workload": cfg["workload"].split(":")[0], "N": cfg["N"], "h": cfg["h"],
                     "tol": cfg["tol"], "law": cfg["law"], "seed": cfg["seed"],
                     "start": "polynomial", "update": "W_n + h C"}
    rec["iters_per_step"] = iters
    rec["evals_per_step"] = _sig(sum(iters) / len(iters))
    rec["eval_ms"] = {k: _sig(v["avg_ms"]) for k, v in ph.items()}
    rec["fp64_start_from_Wn"] = {"s_per_step": _sig(wn["s_per_step"]),
                                 "evals_per_step": _sig(sum(wn["iters_per_step"]) / len(wn["iters_per_step"])),
                                 "vs_paper_0.55s": _sig(wn["s_per_step"] / PAPER_S_PER_STEP_N4096)}
    rec["roofline"] = roof
    lib = out["roofline"].get("context_library_zgemm")
    if lib:
        rec["vendor_zgemm_ms"] = _sig(lib["ms"])
    rec["solve_hbm_GBps"] = _sig(out["solve_hbm"]["achieved_GBps"])
    rec["split"] = leg_split(out)
    rec["crt"] = leg_alt(out.get("crt_precision"))
    rec["mixed"] = leg_alt(out.get("mixed_precision"))
    n2 = out.get("n2048")
    if n2:
        rec["n2048"] = {"fp64_s_per_step": _sig(n2["fp64_s_per_step"]), "split": leg_split(n2),
                        "crt_s_per_step": _sig(_pick(n2, "crt_precision", "s_per_step"))}
    ens = out.get("ensemble")
    if ens:
        rec["ensemble64_steps_per_s"] = {
            "fp64": _sig(ens["fp64"]["aggregate_steps_per_s"]),
            "split": _sig(ens["split"]["aggregate_steps_per_s"]),
            "split_slices": ens.get("split_slices"),
            "split_rel_vs_fp64": _sig(ens["split"].get("max_member_rel_frobenius_vs_fp64_ensemble"), 2)}
    n512 = out.get("n512")
    if n512:
        rec["n512_s_per_step"] = _sig(n512["single_context_s_per_step"])
        rec["n512_device_stop_graph_s_per_step"] = _sig(n512.get("device_stopping_graph_s_per_step"))
    cb = out.get("cpu_baseline")
    if cb:
        rec["cpu_baseline"] = {"value": _sig(cb["value"]), "unit": cb["unit"], "cores": cb["cores"],
                               "kind": cb["kind"], "sample": cb["sample_short"],
                               "cpu_model": cb.get("cpu_model")}
    else:
        rec["cpu_baseline"] = None
    rec["detail"] = detail_path
    return rec


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="n4096")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--split-slices", default="3,4,5",
                    help="comma-separated slice counts of the split-precision runs ('' or 0: skip)")
    ap.add_argument("--n2048-steps", type=int, default=20,
                    help="timed steps of the N=2048 leg, FP64 and split (0: skip it)")
    ap.add_argument("--n512-steps", type=int, default=100,
                    help="timed steps of the N=512 leg (0: skip it)")
    ap.add_argument("--long-steps", type=int, default=10000,
                    help="steps of the long-run drift leg (N=512, paper initial condition; 0: skip)")
    ap.add_argument("--mixed", type=int, default=1,
                    help="1: also time the mixed-precision run (FP64 A, INT8 lower product), 0: skip")
    ap.add_argument("--crt", type=int, default=1,
                    help="1: also time the modular-INT8 run (ZE_PREC_CRT A, INT8 lower product), 0: skip")
    ap.add_argument("--orders", type=int, default=1,
                    help="1: run the orders512 leg (orders 2/4/6 accuracy against cost), 0: skip")
    ap.add_argument("--ensemble-steps", type=int, default=50,
                    help="steps of the 64-simulation ensemble legs, FP64 and split (0: skip them)")
    ap.add_argument("--detail-out", default="bench_detail.json",
                    help="file that receives the full record of every leg ('' : none); the last "
                         "stdout line is a compact summary of it")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="after the timed steps, run 3 plain device-to-device copies of this many "
                         "MiB (a known-size reference for hardware traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the multi-GPU decomposition of the step is a "
              "design note, not built; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2206_05466_amd import PREC_FP64, PREC_SPLIT

    torch.cuda.set_device(0)
    slist = [int(x) for x in str(args.split_slices).split(",") if x.strip() and int(x) > 0]
    m = measure_single(args.workload, args.steps, args.warmup, slist, args.copy_probe_mib,
                       args.mixed > 0, args.crt > 0)
    N, prof = m["N"], m["prof"]

    n2048 = None
    if args.n2048_steps > 0 and args.workload != "n2048":
        m2 = measure_single("n2048", args.n2048_steps, args.warmup, slist, 0, args.mixed > 0,
                            args.crt > 0)
        p2 = m2["prof"]["product_PW"]
        n2048 = {
            "workload": f"n2048: one simulation, N=2048, sigma_l law {m2['law']}, h={m2['h']}, "
                        f"tol={m2['tol']}, {m2['steps']} steps, polynomial start",
            "fp64_s_per_step": m2["s_per_step"],
            "fp64_iters_per_step": m2["iters_per_step"],
            "fp64_casimir_drift_rel": m2["casimir_drift_rel"],
            "fp64_start_from_Wn_s_per_step": m2["fp64_start_from_Wn"]["s_per_step"],
            "product_PW_tflops": 8.0 * 2048 ** 3 / (p2[0] / max(p2[1], 1) * 1e-3) / 1e12,
            "phases": phases_of(m2["prof"]),
            "split_precision": m2["split_precision"],
            "mixed_precision": m2["mixed_precision"],
            "crt_precision": m2["crt_precision"],
        }

    n512 = small_leg(args.n512_steps) if args.n512_steps > 0 else None
    long512 = long_leg(args.long_steps) if args.long_steps > 0 else None
    orders512 = orders_leg() if args.orders > 0 else None

    ens = None
    if args.ensemble_steps > 0:
        rec64, ref = ensemble_leg(args.ensemble_steps, PREC_FP64, with_cpu=not args.no_cpu_baseline)
        ens = {"fp64": rec64,
               "split": ensemble_leg(args.ensemble_steps, PREC_SPLIT, ref=ref)[0],
               "split_slices": _ens_split_slices()}
        del ref
        ens["split_speedup_vs_fp64"] = (ens["split"]["aggregate_steps_per_s"] /
                                        ens["fp64"]["aggregate_steps_per_s"])
        log(f"ensemble: fp64 {ens['fp64']['aggregate_steps_per_s']:.0f} steps/s, split "
            f"{ens['split']['aggregate_steps_per_s']:.0f} steps/s")

    # context: the vendor library's complex GEMM (torch.matmul on complex128) at the same size
    Xa = torch.randn(N, N, dtype=torch.complex128, device="cuda")
    Xb = torch.randn(N, N, dtype=torch.complex128, device="cuda")
    torch.matmul(Xa, Xb)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        Xc = torch.matmul(Xa, Xb)
    torch.cuda.synchronize()
    lib_ms = (time.perf_counter() - t0) / 3 * 1e3
    del Xa, Xb, Xc

    s_per_step = m["s_per_step"]
    iters = m["iters_per_step"]
    gemm_ms, gemm_n = prof["product_PW"]
    gemm_avg_s = gemm_ms / gemm_n * 1e-3
    achieved = 8.0 * N ** 3 / gemm_avg_s / 1e12
    solve_avg_s = prof["stream_solve"][0] / max(prof["stream_solve"][1], 1) * 1e-3
    solve_bytes = 24.0 * N * N  # read lower W~ (8 N^2 B), write P (16 N^2 B)
    low_ms = prof["lower_product_epilogue"][0] / max(prof["lower_product_epilogue"][1], 1)

    out = {
        "metric": "IsoMP seconds/step (FP64)",
        "value": s_per_step,
        "unit": "s/step",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": s_per_step * 1e3,
        "steps_per_s": 1.0 / s_per_step,
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": s_per_step / PAPER_S_PER_STEP_N4096 if N == 4096 else None,
        "vs_baseline_note": ("value / 0.55 s (paper, N=4096 on ~2500 CPU cores, 3 iterations); "
                             "context, other hardware") if N == 4096 else None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: one simulation, N={N}, W0 = sum i omega_lm T_lm with "
                        f"seeded omega_lm, sigma_l law {m['law']}, h={m['h']}, tol={m['tol']}, "
                        f"maxit={m['maxit']}",
            "N": N, "h": m["h"], "tol": m["tol"], "law": m["law"], "seed": m["seed"], "prec": "fp64",
        },
        "iters_per_step": iters,
        "max_resid": m["max_resid"],
        "initial_guess": "the second step starts from 2 W_n - F_prev, later ones from the polynomial "
                         "(degree <= 3) through the run's previous midpoints, the third and fourth "
                         "with the n-th backward difference of the run's states added "
                         "(ze_set_initial_guess 3); every step still iterates until the change "
                         "is below tol",
        "fp64_polynomial_start_midpoints_only": m["fp64_polynomial_start_midpoints_only"],
        "fp64_without_phase_events": m["without_phase_events"],
        "fp64_start_from_Wn": m["fp64_start_from_Wn"],
        "fp64_linear_start": m["fp64_linear_start"],
        "fp64_polynomial_start_second_line_form": m["fp64_polynomial_start_second_line_form"],
        "update_form": "W_{n+1} = W_n + h (A - A^H) (ze_set_update_form 1; the two lines of "
                       "eq. (isomp) differ by exactly h [P~, W~]); the W_n, linear and "
                       "second-line-form runs use the default form, the second line of eq. (isomp)",
        "casimir_drift_rel": m["casimir_drift_rel"],
        "phases": phases_of(prof),
        "gemm_flops_per_step": sum(iters) / len(iters) * 12.0 * N ** 3,
        "achieved_step_tflops": sum(iters) / len(iters) * 12.0 * N ** 3 / s_per_step / 1e12,
        "roofline": {
            "kernel": "zgemm_f64_kernel (A = P W~)",
            "bound": "mfma",
            "achieved": achieved,
            "peak": PEAK_FP64_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP64_TFLOPS,
            "traffic": measured_traffic(N),
            "context_library_zgemm": {"ms": lib_ms, "tflops": 8.0 * N ** 3 / (lib_ms * 1e-3) / 1e12,
                                      "what": "torch.matmul on complex128 N x N (the vendor BLAS), "
                                              "same size, same run"},
        },
        "solve_hbm": {
            "achieved_GBps": solve_bytes / solve_avg_s / 1e9,
            "peak_GBps": 8000.0,
            "bytes_per_launch": solve_bytes,
            "note": "stream solve: algorithmic bytes 24 N^2 (read lower W~, write full P)",
        },
        "lower_product_tflops": 4.0 * N ** 3 / (low_ms * 1e-3) / 1e12,
        "cpu_baseline": None,
        "split_precision": m["split_precision"],
        "mixed_precision": m["mixed_precision"],
        "crt_precision": m["crt_precision"],
        "n2048": n2048,
        "n512": n512,
        "long512": long512,
        "orders512": orders512,
        "ensemble": ens,
    }
    if not args.no_cpu_baseline:
        mean_evals = sum(iters) / len(iters)
        log(f"cpu baseline: oracle step at N={N}, {mean_evals:.3f} evaluations per step ...")
        out["cpu_baseline"] = cpu_baseline(N, m["seed"], m["law"], m["h"], mean_evals)
        log(f"cpu baseline {out['cpu_baseline']['value']:.2f} s/step")
    detail = args.detail_out or None
    if detail:
        d = os.path.dirname(detail)
        if d:
            os.makedirs(d, exist_ok=True)
        with open(detail, "w") as f:
            json.dump(out, f, indent=1)
        log(f"full record written to {detail}")
    print(json.dumps(compact_record(out, detail)), flush=True)


if __name__ == "__main__":
    main()
