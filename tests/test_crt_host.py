"""The modular (CRT) form's integer arithmetic, built for the host from the same header the
kernels use and checked against Python's exact integers (no GPU): the reconstruction of X from
int32 values congruent to X modulo the 16 moduli, over |X| up to 0.49 M (the bit count keeps
the products below 0.99^2 M / 2), and the balanced residues of integers held exactly in a
double (up to 53 significant bits, below 2^61 in magnitude), which the residue kernels form in
FP64."""

import os
import random
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
MODULI = [256, 255, 253, 251, 247, 241, 239, 233, 229, 227, 223, 211, 199, 197, 193, 191]


@pytest.fixture(scope="module")
def prog(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("crt") / "crt_host_check")
    cmd = [hipcc, "--offload-arch=gfx950", "-O2", "-std=c++17",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "paper_2206_05466_amd", "csrc"), "-I", os.path.join(ROOT, "include"),
           os.path.join(HERE, "host", "crt_host_check.hip"), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    return out


def balanced(y, p):
    r = y % p
    return r - p if r > (p - 1) // 2 else r


def test_moduli_coprime_and_range():
    from math import gcd, log2, prod
    for i, a in enumerate(MODULI):
        assert a <= 256
        for b in MODULI[i + 1:]:
            assert gcd(a, b) == 1
    assert 125 < log2(prod(MODULI)) < 125.2


def test_reconstruct_and_residues_exact(prog):
    from math import prod
    M = prod(MODULI)
    rng = random.Random(2206)
    cases = [0, 1, -1, 2 ** 53, -(2 ** 53) - 1, 2 ** 64 + 1, (M * 49) // 100, -((M * 49) // 100)]
    cases += [rng.choice([-1, 1]) * rng.getrandbits(rng.randint(1, 124)) for _ in range(3000)]
    lines, ys = [], []
    for X in cases:
        g = []
        for p in MODULI:
            # some int32 congruent to X mod p, as the INT8 products give (|g| < 2^31)
            g.append(X % p + p * rng.randint(-(2 ** 30) // p, (2 ** 30) // p))
        # an integer as the residue kernels hold it: exact in a double, |y| < 2^62
        y = rng.choice([-1, 1]) * (rng.getrandbits(rng.randint(0, 53)) << rng.randint(0, 8))
        ys.append(y)
        lines.append(" ".join([str(X)] + [str(v) for v in g] + [str(y)]))
    r = subprocess.run([prog], input="\n".join(lines) + "\n", capture_output=True, text=True,
                       timeout=60)
    assert r.returncode == 0, r.stderr
    out = r.stdout.split("\n")
    for X, y, line in zip(cases, ys, out):
        f = line.split()
        got = float.fromhex(f[0])
        want = float(X)  # correctly rounded
        # exact when X is representable, else within one ulp (two conversions of 64-bit halves)
        if abs(X) < 2 ** 53:
            assert got == want, (X, got)
        else:
            assert abs(got - want) <= abs(want) * 2.0 ** -52, (X, got, want)
        assert [int(v) for v in f[1:]] == [balanced(y, p) for p in MODULI], y
