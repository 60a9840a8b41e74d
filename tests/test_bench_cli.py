"""bench.py's host-side contract (CPU): more than one GPU is refused with a message and exit
status 2 before anything touches a GPU; the workload table names every configuration the
legs read, with the sizes and step counts the measurement is quoted on."""

import os
import subprocess
import sys

from workloads import WORKLOADS

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, cwd=ROOT, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_workload_table():
    for name in ("n64", "n512", "n2048", "n4096", "ensemble64", "long512", "orders512"):
        assert name in WORKLOADS, name
    assert WORKLOADS["n4096"]["N"] == 4096 and WORKLOADS["n2048"]["N"] == 2048
    assert WORKLOADS["ensemble64"]["nsim"] == 64
    assert WORKLOADS["long512"]["steps"] >= 10000
    assert all(WORKLOADS[k]["tol"] == 1e-12 for k in ("n512", "n2048", "n4096", "long512"))


def _canned_record():
    """A full bench record with every leg present, shaped as bench.py's main() builds it."""
    phases = {k: {"avg_ms": 1.23456789, "launches": 24} for k in
              ("stream_solve", "product_PW", "lower_product_epilogue", "residual")}
    run = {"slices": 4, "s_per_step": 0.00623456, "speedup_vs_fp64": 2.5876543,
           "iters_per_step": [3, 2, 2] + [1] * 17, "rel_frobenius_vs_fp64_run": 3.2345e-11,
           "casimir_drift_rel": {"C2": 1e-14, "C3": 2e-17, "C4": 3e-14},
           "meets_stated_accuracy": True, "phases": phases,
           "product_PW_fp64_equiv_tflops": 201.2345, "product_PW_int8_tops": 2012.345}
    split = {"stated_accuracy": "x" * 200, "runs": [dict(run, slices=s) for s in (3, 4, 5)],
             "best_at_stated_accuracy": {k: run[k] for k in ("slices", "s_per_step", "speedup_vs_fp64",
                                                             "rel_frobenius_vs_fp64_run")},
             "note": "y" * 100}
    alt = {"s_per_step": 0.0102345678, "speedup_vs_fp64": 1.5712345, "iters_per_step": run["iters_per_step"],
           "max_resid": 9.9e-13, "rel_frobenius_vs_fp64_run": 7.8123e-18, "casimir_drift_rel": {},
           "phases": phases}
    ens = {"aggregate_steps_per_s": 43012.3456789, "max_member_rel_frobenius_vs_fp64_ensemble": 6.4123e-10,
           "workload": "z" * 300}
    wn = {"s_per_step": 0.0396123456, "iters_per_step": [3] * 20, "rel_frobenius_vs_headline_run": 8.9e-16}
    return {
        "metric": "IsoMP seconds/step (FP64)", "value": 0.0161234567, "unit": "s/step", "n_gpus": 1,
        "steps": 20, "warmup": 5, "ms_per_step": 16.1234567, "steps_per_s": 62.0123456,
        "higher_is_better": False, "scaling": "strong", "vs_baseline": 0.029312345,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "n4096: one simulation, N=4096, W0 = sum i omega_lm T_lm with seeded "
                               "omega_lm, sigma_l law inv1.5, h=0.005, tol=1e-12, maxit=50",
                   "N": 4096, "h": 0.005, "tol": 1e-12, "law": "inv1.5", "seed": 0, "prec": "fp64"},
        "iters_per_step": [3, 2, 2] + [1] * 17, "max_resid": 9.1e-13, "phases": phases,
        "fp64_start_from_Wn": wn, "fp64_linear_start": wn, "fp64_polynomial_start_second_line_form": wn,
        "roofline": {"kernel": "zgemm_f64_kernel (A = P W~)", "bound": "mfma", "achieved": 66.3123456,
                     "peak": 78.6, "unit": "TFLOP/s", "frac": 0.84367891, "traffic": 3845123456.789,
                     "context_library_zgemm": {"ms": 7.91234, "tflops": 69.5, "what": "w" * 100}},
        "solve_hbm": {"achieved_GBps": 2060.123456, "peak_GBps": 8000.0, "bytes_per_launch": 4.0e8},
        "cpu_baseline": {"value": 4.3412345, "unit": "s/step", "cores": 16,
                         "cpu_model": "AMD EPYC 9575F 64-Core Processor", "kind": "oracle",
                         "sample_short": "1 oracle step, N=4096, 1 evaluations, scaled to 1.20",
                         "sample": "s" * 400},
        "split_precision": split, "mixed_precision": alt, "crt_precision": alt,
        "n2048": {"fp64_s_per_step": 0.00250123456, "split_precision": split, "crt_precision": alt},
        "n512": {"single_context_s_per_step": 0.000131234567},
        "long512": {"drift": [{"step": k} for k in range(10)]}, "orders512": {"runs": []},
        "ensemble": {"fp64": ens, "split": ens, "split_slices": 4},
    }


def test_compact_line_parses_and_stays_small():
    """The driver reads the last stdout line: it must be one JSON object of a few hundred
    bytes with the contract's keys, the roofline and the CPU baseline, whatever the legs hold."""
    import json

    sys.path.insert(0, ROOT)
    import bench

    rec = bench.compact_record(_canned_record(), "bench_detail.json")
    line = json.dumps(rec)
    assert "\n" not in line and len(line) < 2048, len(line)
    back = json.loads(line)
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in back, k
    assert back["config"]["workload"] == "n4096" and back["dtype"] == "f64"
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in back["roofline"], k
    assert abs(back["roofline"]["frac"] - 0.8437) < 1e-4
    for k in ("value", "unit", "cores", "kind", "sample"):
        assert k in back["cpu_baseline"], k
    assert back["fp64_start_from_Wn"]["evals_per_step"] == 3.0
    # legs that were skipped leave their keys out or null, never break the line
    bare = _canned_record()
    for k in ("n2048", "n512", "ensemble", "mixed_precision", "crt_precision", "cpu_baseline"):
        bare[k] = None
    bare["split_precision"] = None
    line = json.dumps(bench.compact_record(bare, None))
    assert len(line) < 2048 and json.loads(line)["cpu_baseline"] is None
