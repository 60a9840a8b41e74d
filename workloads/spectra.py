"""Random spherical-harmonic vorticity spectra (seeded; no method arithmetic).

A workload draws omega_lm for l = lmin..lmax with E|omega_lm|^2 = sigma_l^2 and the reality
condition omega_{l,-m} = (-1)^m conj(omega_lm) of a real vorticity field:

* omega_l0 = sigma_l z            (z standard normal, real);
* omega_lm = sigma_l (z1 + i z2)/sqrt(2),  m = 1..l   (so E|omega_lm|^2 = sigma_l^2);

with the normals drawn from ``numpy.random.default_rng(seed)`` in this fixed order: for
each l ascending, one block of 2l+1 normals z[0..2l], z[0] for m = 0 and
(z[2m-1], z[2m]) for m >= 1.  omega_00 = 0 (zero mean vorticity, W traceless).
Coefficients are stored flat at index l*l + l + m, length N*N.

Spectral laws (sigma_l):

* ``inv1``   -- (l+1)^-1 over l = 1..N-1;
* ``inv1.5`` -- (l+1)^-1.5 over l = 1..N-1;
* ``paper``  -- 1 over 2 <= l <= 20, 0 elsewhere: the random large-scale initial condition
  of the paper's long simulation (Sec. 4), random coefficients of comparable size on the
  degrees 2 to 20 only.
"""

import numpy as np


def sigma_law(law: str, l: np.ndarray) -> np.ndarray:
    l = np.asarray(l, dtype=np.float64)
    if law == "inv1":
        return np.where(l >= 1, 1.0 / (l + 1.0), 0.0)
    if law == "inv1.5":
        return np.where(l >= 1, (l + 1.0) ** -1.5, 0.0)
    if law == "paper":
        return np.where((l >= 2) & (l <= 20), 1.0, 0.0)
    raise ValueError(f"unknown spectral law {law!r}")


def omega_coeffs(N: int, seed: int, law: str = "inv1", lmax: int | None = None) -> np.ndarray:
    """Flat complex128 coefficients omega[l*l+l+m] for a real random vorticity field."""
    if N < 1:
        raise ValueError("N must be >= 1")
    lmax = N - 1 if lmax is None else min(lmax, N - 1)
    if law == "paper":
        lmax = min(lmax, 20)
    rng = np.random.default_rng(seed)
    omega = np.zeros(N * N, dtype=np.complex128)
    r2 = 1.0 / np.sqrt(2.0)
    for l in range(1, lmax + 1):
        z = rng.standard_normal(2 * l + 1)
        sig = float(sigma_law(law, np.array([l]))[0])
        base = l * l + l
        omega[base] = sig * z[0]
        m = np.arange(1, l + 1)
        c = sig * (z[2 * m - 1] + 1j * z[2 * m]) * r2
        omega[base + m] = c
        omega[base - m] = np.where(m % 2 == 0, 1.0, -1.0) * np.conj(c)
    return omega


def ensemble_sizes(nsim: int = 64, seed: int = 0, choices=(128, 256, 384, 512)) -> list:
    """Matrix sizes of an ensemble of independent simulations, N_j uniform over ``choices``."""
    rng = np.random.default_rng(seed)
    return [int(x) for x in rng.choice(np.asarray(choices), size=nsim)]


# The workloads (sizes, spectra, time steps, step counts) the tests and the benchmark use.
WORKLOADS = {
    "n64":   dict(N=64,   law="inv1",   h=0.01,  steps=10,  tol=1e-12, maxit=50, seeds=(0, 1, 2)),
    "n512":  dict(N=512,  law="inv1",   h=0.005, steps=100, tol=1e-12, maxit=50, seeds=(0,)),
    "n2048": dict(N=2048, law="inv1.5", h=0.005, steps=20,  tol=1e-12, maxit=50, seeds=(0,)),
    "n4096": dict(N=4096, law="inv1.5", h=0.005, steps=10,  tol=1e-12, maxit=50, seeds=(0,)),
    # K: the evaluation cap of the graph-captured ensemble step (one above the 4 that the
    # first step, from W_n, needs); steady_cap from steady_from: the cap of the later steps of
    # a run (one above the single evaluation they need once the polynomial start has reached
    # degree 3); split_slices: the slices of its split-precision products
    "ensemble64": dict(nsim=64, sizes=(128, 256, 384, 512), law="inv1", h=0.005, steps=50,
                       K=5, steady_cap=2, steady_from=4, tol=1e-12, split_slices=5, size_seed=0,
                       seed0=1000),
    # the paper's long-run initial condition (degrees 2..20, unit spectral norm, Sec. 4)
    "long512": dict(N=512, law="paper", h=0.005, steps=10000, tol=1e-12, maxit=50, seed=0,
                    sample=1000),
    # the same initial condition to t = 2 at orders 2, 4, 6 over several step sizes, against
    # an order-6 run at a smaller step (accuracy against cost)
    "orders512": dict(N=512, law="paper", seed=0, T=2.0, hs=(0.4, 0.2, 0.1, 0.05),
                      h_ref=0.025, tol=1e-13, maxit=50),
}
