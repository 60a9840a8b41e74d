"""Oracle parity in exactly the configurations bench.py times (eqs. (isomp), (isomp_iter)).

Full sizes (N = 4096 and 2048): the workloads' full-spectrum fields (every degree l <= N - 1),
W_0 assembled by the library's basis kernel as in the bench; polynomial starting iterate from
the run's midpoints, the third and fourth steps with the run's states as well (guess mode 3,
the oracle's solution_differences), W_{n+1} = W_n + h (A - A^H), tol 1e-12; FP64, the split form at the
bench's slice count (4; the lower product 3), the modular INT8 form and the mixed form.  The
oracle's trajectories come from tests/golden/fullsize_n*.npz (written by
make_fullsize_reference.py there, which calls only the oracle): every entry of three rows and
2048 seeded random entries of W_0 and of the state after 10 and 20 steps (N = 4096) or 20
steps (N = 2048), with the evaluation counts and Casimirs.  Bars: relative Frobenius distance
over the stored entries 1e-12 for the FP64-accurate forms and 1e-10 for the split form, the
oracle's evaluation counts for the FP64 form, and Casimir drift <= 1e-11 (C_2, C_4 relative,
C_3 against ||W_0||_F^3).

The 64-simulation ensemble: the bench's run (one step, then 50, each a run call of its own;
guess mode 3; evaluation cap 5, and 2 from the fifth step of a call; FP64 and the split form at
the workload's slice count), one member of each size class against the oracle's run of the same
two calls.
"""

import os

import numpy as np
import pytest

import oracle as O
from workloads import WORKLOADS, ensemble_sizes, omega_coeffs

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
SPLIT_SLICES = 4  # bench.py's headline split runs at N = 2048 and 4096


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2206_05466_amd import load_library

    load_library()
    return torch.device("cuda", 0)


def reference(N):
    with np.load(os.path.join(GOLDEN, f"fullsize_n{N}.npz")) as f:
        return {k: f[k] for k in f.files}


def sampled(Wd, ref):
    rows = torch.as_tensor(ref["rows"], device=Wd.device)
    r = torch.as_tensor(ref["sample_r"], device=Wd.device)
    c = torch.as_tensor(ref["sample_c"], device=Wd.device)
    return np.concatenate([Wd[rows].cpu().numpy().ravel(), Wd[r, c].cpu().numpy()])


def sampled_rel(Wd, ref, tag):
    got = sampled(Wd, ref)
    exp = np.concatenate([ref[f"{tag}_rows"].ravel(), ref[f"{tag}_sample"]])
    return float(np.linalg.norm(got - exp) / np.linalg.norm(exp))


def casimir_drift(z, Wd, c0, nf0):
    c = z.casimirs(Wd, 4)
    return max(abs(c[1] - c0[1]) / abs(c0[1]), abs(c[3] - c0[3]) / abs(c0[3]),
               abs(c[2] - c0[2]) / nf0 ** 3)


def run_timed(z, W0d, ref, steps, prec, slices=None):
    cfg_h, tol, maxit = float(ref["h"]), float(ref["tol"]), int(ref["maxit"])
    assert bool(ref["solution_differences"])  # the stored run's start: guess mode 3
    z.set_initial_guess(3)
    z.set_update_form(1)
    if slices is not None:
        z.set_split_slices(slices)
    Wd = W0d.clone()
    its, res = z.isomp_run(Wd, cfg_h, steps, tol, maxit, prec)
    torch.cuda.synchronize()
    return Wd, list(its), list(res)


@pytest.mark.parametrize("N", [4096, 2048])
def test_fullsize_timed_configurations_against_oracle(dev, N):
    from paper_2206_05466_amd import PREC_CRT, PREC_FP64, PREC_MIXED, PREC_SPLIT, Zeuler

    ref = reference(N)
    wname = f"n{N}"
    cfg = WORKLOADS[wname]
    assert int(ref["N"]) == N and float(ref["h"]) == cfg["h"] and int(ref["seed"]) == cfg["seeds"][0]
    z = Zeuler(N)
    W0d = z.basis_assemble(omega_coeffs(N, cfg["seeds"][0], cfg["law"]))
    torch.cuda.synchronize()
    e0 = sampled_rel(W0d, ref, "W0")
    assert e0 < 1e-12, e0  # the GPU basis against LAPACK's eigenvectors, whole spectrum
    c0, nf0 = ref["W0_casimirs"], float(ref["W0_fro"])
    iters_ref = [int(k) for k in ref["iters"]]
    tol = float(ref["tol"])
    report = {}
    for steps in [int(s) for s in ref["steps"]]:
        tag = f"W{steps}"
        Wd, its, res = run_timed(z, W0d, ref, steps, PREC_FP64)
        assert its == iters_ref[:steps] and max(res) < tol, (steps, its, iters_ref)
        e = sampled_rel(Wd, ref, tag)
        report[f"fp64_{steps}"] = e
        assert e < 1e-12, (steps, e)
        assert casimir_drift(z, Wd, c0, nf0) < 1e-11
    steps = int(ref["steps"][-1])
    tag = f"W{steps}"
    for name, prec, slices, bar in (("split4", PREC_SPLIT, SPLIT_SLICES, 1e-10),
                                    ("crt", PREC_CRT, 5, 1e-12),
                                    ("mixed", PREC_MIXED, 5, 1e-12)):
        Wd, its, res = run_timed(z, W0d, ref, steps, prec, slices)
        e = sampled_rel(Wd, ref, tag)
        report[name] = e
        assert max(res) < tol, (name, res)
        assert e < bar, (name, e)
        assert casimir_drift(z, Wd, c0, nf0) < 1e-11, name
        if prec != PREC_SPLIT:
            assert its == iters_ref[:steps], (name, its)
    z.close()
    print(f"N={N}: W0 {e0:.1e}, " + ", ".join(f"{k} {v:.1e}" for k, v in report.items()))


@pytest.mark.parametrize("prec_name", ["fp64", "split"])
def test_ensemble64_timed_configuration(dev, prec_name):
    from paper_2206_05466_amd import PREC_FP64, PREC_SPLIT, Ensemble, Zeuler

    cfg = WORKLOADS["ensemble64"]
    sizes = ensemble_sizes(cfg["nsim"], cfg["size_seed"], cfg["sizes"])
    h, tol, K, steps = cfg["h"], cfg["tol"], cfg["K"], cfg["steps"]
    split = prec_name == "split"
    picks = [sizes.index(n) for n in sorted(set(sizes))]
    W0s = {j: O.assemble(sizes[j], omega_coeffs(sizes[j], cfg["seed0"] + j, cfg["law"])) for j in picks}
    ctxs = {n: Zeuler(n) for n in sorted(set(sizes))}
    Ws = [torch.from_numpy(W0s[j]).cuda() if j in W0s else
          ctxs[n].basis_assemble(omega_coeffs(n, cfg["seed0"] + j, cfg["law"]))
          for j, n in enumerate(sizes)]
    for z in ctxs.values():
        z.close()
    prec = PREC_SPLIT if split else PREC_FP64
    with Ensemble(sizes) as ens:
        ens.set_initial_guess(3)
        ens.set_update_form(1)
        ens.set_steady_cap(cfg["steady_cap"], cfg["steady_from"])
        if split:
            ens.set_split_slices(cfg["split_slices"])
        ens.run(Ws, h, 1, tol, K, prec=prec)   # the bench's first call (tuning, capture)
        ens.run(Ws, h, steps, tol, K, prec=prec)
        its, res = ens.stats()
    torch.cuda.synchronize()
    assert max(res) < tol
    bar = 1e-10 if split else 1e-12
    worst = 0.0
    for j in picks:
        W1, _, _ = O.isomp_run(W0s[j], h, 1, tol, K, extrapolate=True, degree=3, update="difference",
                               solution_differences=True)
        Wr, it_ref, _ = O.isomp_run(W1, h, steps, tol, K, extrapolate=True, degree=3,
                                    update="difference", solution_differences=True)
        W = Ws[j].cpu().numpy()
        e = np.linalg.norm(W - Wr) / np.linalg.norm(Wr)
        worst = max(worst, e)
        if not split:
            assert its[j] == it_ref[-1], (j, its[j], it_ref[-1])
        assert e < bar, (j, sizes[j], e)
        c0, c1 = O.casimirs(W0s[j], 4), O.casimirs(W, 4)
        assert abs(c1[1] - c0[1]) / abs(c0[1]) < 1e-11 and abs(c1[3] - c0[3]) / abs(c0[3]) < 1e-11
    print(f"ensemble {prec_name}: largest member distance to the oracle {worst:.1e}")
