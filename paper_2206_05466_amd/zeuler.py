"""ctypes binding of libzeuler.so (include/zeuler.h): argument marshalling only.

Every computation runs in the HIP library; this module checks tensor arguments (device,
dtype, shape, contiguity), passes their device pointers and raises on error codes.  Torch is
used for device memory and streams only.  There is no fallback: without the built library
(``python -m paper_2206_05466_amd.build``) every call raises.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libzeuler.so")

ZE_OK, ZE_EINVAL, ZE_ENOMEM, ZE_ENOTCONV, ZE_ENONFINITE, ZE_EHIP = range(6)
PREC_FP64, PREC_SPLIT, PREC_MIXED, PREC_CRT = 0, 1, 2, 3

# Exported names and signatures, as declared in include/zeuler.h.
_c_int, _c_double, _vp = ctypes.c_int, ctypes.c_double, ctypes.c_void_p
_P_int, _P_double = ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)
SIGNATURES = {
    "ze_strerror": (ctypes.c_char_p, [_c_int]),
    "ze_last_error": (ctypes.c_char_p, []),
    "ze_create": (_c_int, [_c_int, _vp, ctypes.POINTER(_vp)]),
    "ze_destroy": (_c_int, [_vp]),
    "ze_size": (_c_int, [_vp]),
    "ze_stream_solve": (_c_int, [_vp, _vp, _vp]),
    "ze_isomp_step": (_c_int, [_vp, _vp, _c_double, _c_double, _c_int, _c_int, _P_int, _P_double]),
    "ze_isomp_run": (_c_int, [_vp, _vp, _c_double, _c_double, _c_int, _c_int, _c_int, _P_int, _P_double]),
    "ze_casimirs": (_c_int, [_vp, _vp, _c_int, _P_double]),
    "ze_basis_assemble": (_c_int, [_vp, _vp, _vp]),
    "ze_basis_extract": (_c_int, [_vp, _vp, _vp]),
    "ze_energy_spectrum": (_c_int, [_vp, _vp, _vp]),
    "ze_zgemm": (_c_int, [_vp, _vp, _vp, _vp, _c_int]),
    "ze_zgemm_noalloc": (_c_int, [_c_int, _vp, _vp, _vp, _vp]),
    "ze_set_split_slices": (_c_int, [_vp, _c_int]),
    "ze_set_initial_guess": (_c_int, [_vp, _c_int]),
    "ze_set_split_slices_lower": (_c_int, [_vp, _c_int]),
    "ze_set_update_form": (_c_int, [_vp, _c_int]),
    "ze_set_validation": (_c_int, [_vp, _c_int]),
    "ze_set_order": (_c_int, [_vp, _c_int]),
    "ze_set_stopping": (_c_int, [_vp, _c_int]),
    "ze_set_steady_cap": (_c_int, [_vp, _c_int, _c_int]),
    "ze_set_continuation": (_c_int, [_vp, _c_int]),
    "ze_run_stats": (_c_int, [_vp, _c_int, _P_int, _P_double]),
    "ze_profile": (_c_int, [_vp, _c_int]),
    "ze_profile_read": (_c_int, [_vp, _P_double, ctypes.POINTER(ctypes.c_longlong), _c_int]),
    "ze_ensemble_create": (_c_int, [_c_int, _P_int, _vp, ctypes.POINTER(_vp)]),
    "ze_ensemble_destroy": (_c_int, [_vp]),
    "ze_ensemble_run": (_c_int, [_vp, ctypes.POINTER(_vp), _c_double, _c_double, _c_int, _c_int, _c_int]),
    "ze_ensemble_step": (_c_int, [_vp, ctypes.POINTER(_vp), _c_double, _c_double, _c_int, _c_int]),
    "ze_ensemble_stats": (_c_int, [_vp, _P_int, _P_double]),
    "ze_ensemble_tuning": (_c_int, [_vp, _c_int, _P_int, _P_double]),
    "ze_ensemble_set_split_slices": (_c_int, [_vp, _c_int]),
    "ze_ensemble_set_initial_guess": (_c_int, [_vp, _c_int]),
    "ze_ensemble_set_split_slices_lower": (_c_int, [_vp, _c_int]),
    "ze_ensemble_set_update_form": (_c_int, [_vp, _c_int]),
    "ze_ensemble_set_steady_cap": (_c_int, [_vp, _c_int, _c_int]),
    "ze_ensemble_set_continuation": (_c_int, [_vp, _c_int]),
}

PHASES = ("stream_solve", "product_PW", "lower_product_epilogue", "residual_reduce")

_lib = None


def load_library():
    """Load libzeuler.so and declare its signatures (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2206_05466_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


class ZeulerError(RuntimeError):
    def __init__(self, status: int, where: str, detail: bool = False):
        lib = load_library()
        msg = lib.ze_strerror(status).decode()
        extra = lib.ze_last_error().decode() if (status == ZE_EHIP or detail) else ""
        super().__init__(f"{where}: {msg}" + (f" ({extra})" if extra else ""))
        self.status = status


def _check(status: int, where: str, detail: bool = False):
    if status != ZE_OK:
        raise ZeulerError(status, where, detail)


def zgemm_noalloc(A, B, out, stream=None):
    """C = A B (FP64) through ze_zgemm_noalloc: no context, no device allocation in the
    library.  A, B, out: contiguous N x N complex128 tensors on the current device; `out` is
    caller-allocated (this function allocates nothing either)."""
    import torch

    lib = load_library()
    N = A.shape[0] if A.dim() == 2 else -1
    dev = torch.device("cuda", torch.cuda.current_device())
    for name, X in (("A", A), ("B", B), ("out", out)):
        if (not isinstance(X, torch.Tensor) or X.dtype != torch.complex128 or X.device != dev
                or tuple(X.shape) != (N, N) or not X.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous {N}x{N} complex128 tensor on {dev}")
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    _check(lib.ze_zgemm_noalloc(N, _vp(A.data_ptr()), _vp(B.data_ptr()), _vp(out.data_ptr()),
                                _vp(st.cuda_stream)), "ze_zgemm_noalloc", detail=True)
    return out


@dataclass
class StepInfo:
    iters: int
    resid: float
    converged: bool


class Zeuler:
    """One context of libzeuler for matrix size N on the current torch device and stream."""

    def __init__(self, N: int, stream=None):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("libzeuler needs a GPU (torch.cuda.is_available() is False)")
        self.lib = load_library()
        self.N = int(N)
        self.device = torch.device("cuda", torch.cuda.current_device())
        st = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.stream = st
        self._ctx = ctypes.c_void_p()
        _check(self.lib.ze_create(self.N, ctypes.c_void_p(st.cuda_stream), ctypes.byref(self._ctx)),
               "ze_create")

    def close(self):
        if getattr(self, "_ctx", None) is not None and self._ctx.value:
            self.lib.ze_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- argument checks ------------------------------------------------------------
    def _mat(self, X, name):
        import torch

        if not isinstance(X, torch.Tensor) or X.dtype != torch.complex128:
            raise TypeError(f"{name} must be a torch.complex128 tensor")
        if X.device != self.device or not X.is_contiguous() or tuple(X.shape) != (self.N, self.N):
            raise ValueError(f"{name} must be a contiguous ({self.N}, {self.N}) tensor on {self.device}")
        return ctypes.c_void_p(X.data_ptr())

    def empty(self):
        import torch

        return torch.empty((self.N, self.N), dtype=torch.complex128, device=self.device)

    # -- calls ------------------------------------------------------------------------
    def stream_solve(self, W, out=None):
        """P = Delta_N^+ W (device tensors)."""
        P = self.empty() if out is None else out
        _check(self.lib.ze_stream_solve(self._ctx, self._mat(W, "W"), self._mat(P, "P")),
               "ze_stream_solve")
        return P

    def zgemm(self, A, B, out=None, prec: int = PREC_FP64):
        C = self.empty() if out is None else out
        _check(self.lib.ze_zgemm(self._ctx, self._mat(A, "A"), self._mat(B, "B"), self._mat(C, "C"),
                                 int(prec)), "ze_zgemm")
        return C

    def isomp_step(self, W, h: float, tol: float = 1e-12, maxit: int = 50,
                   prec: int = PREC_FP64, allow_notconv: bool = True) -> StepInfo:
        """One IsoMP step, W updated in place (W_n -> W_{n+1})."""
        k = ctypes.c_int(0)
        r = ctypes.c_double(0.0)
        st = self.lib.ze_isomp_step(self._ctx, self._mat(W, "W"), float(h), float(tol), int(maxit),
                                    int(prec), ctypes.byref(k), ctypes.byref(r))
        if st == ZE_ENOTCONV and allow_notconv:
            return StepInfo(k.value, r.value, False)
        _check(st, "ze_isomp_step", detail=True)
        return StepInfo(k.value, r.value, True)

    def isomp_run(self, W, h: float, nsteps: int, tol: float = 1e-12, maxit: int = 50,
                  prec: int = PREC_FP64):
        """nsteps IsoMP steps in place.  Returns (iterations, residuals) per step."""
        its = (ctypes.c_int * max(nsteps, 1))()
        res = (ctypes.c_double * max(nsteps, 1))()
        st = self.lib.ze_isomp_run(self._ctx, self._mat(W, "W"), float(h), float(tol), int(maxit),
                                   int(nsteps), int(prec), its, res)
        if st not in (ZE_OK, ZE_ENOTCONV):
            _check(st, "ze_isomp_run", detail=True)
        return list(its)[:nsteps], list(res)[:nsteps]

    def isomp_run_async(self, W, h: float, nsteps: int, tol: float = 1e-12, maxit: int = 50,
                        prec: int = PREC_FP64):
        """nsteps steps with no per-step results and (with set_stopping(1)) no synchronisation:
        the form that can be captured into a graph; run_stats() reads the counts afterwards."""
        _check(self.lib.ze_isomp_run(self._ctx, self._mat(W, "W"), float(h), float(tol), int(maxit),
                                     int(nsteps), int(prec), None, None), "ze_isomp_run", detail=True)

    def set_stopping(self, mode: int):
        """0: tolerance test on the host after each evaluation; 1: on the device (no
        synchronisation per evaluation; every precision)."""
        _check(self.lib.ze_set_stopping(self._ctx, int(mode)), "ze_set_stopping")

    def set_steady_cap(self, cap: int, from_step: int = 4):
        """Evaluation cap min(maxit, cap) for the steps from index from_step on of each run (with
        the polynomial starts); 0 restores maxit for every step."""
        _check(self.lib.ze_set_steady_cap(self._ctx, int(cap), int(from_step)), "ze_set_steady_cap")

    def set_continuation(self, on: bool = True):
        """With it on, an isomp_run on the same W (unchanged since) with the same h, precision
        and step options as the last one continues its trajectory (step index and midpoint
        history) instead of starting at step 0."""
        _check(self.lib.ze_set_continuation(self._ctx, int(bool(on))), "ze_set_continuation")

    def run_stats(self, nsteps: int):
        """(iterations, residuals, status) of the last nsteps steps of the last run (on-device
        stopping); synchronises the context's stream."""
        its = (ctypes.c_int * max(nsteps, 1))()
        res = (ctypes.c_double * max(nsteps, 1))()
        st = self.lib.ze_run_stats(self._ctx, int(nsteps), its, res)
        if st not in (ZE_OK, ZE_ENOTCONV, ZE_ENONFINITE):
            _check(st, "ze_run_stats", detail=True)
        return list(its)[:nsteps], list(res)[:nsteps], st

    def casimirs(self, W, kmax: int) -> np.ndarray:
        """[Tr W, Tr W^2, ..., Tr W^kmax] (complex128 numpy array)."""
        out = (ctypes.c_double * (2 * kmax))()
        _check(self.lib.ze_casimirs(self._ctx, self._mat(W, "W"), int(kmax), out), "ze_casimirs")
        a = np.frombuffer(out, dtype=np.float64).copy()
        return a[0::2] + 1j * a[1::2]

    def basis_assemble(self, omega, out=None):
        """W = sum_lm i omega_lm T_lm from flat coefficients omega[l*l+l+m] (length N*N)."""
        import torch

        om = torch.as_tensor(omega, dtype=torch.complex128).to(self.device).contiguous()
        if om.numel() != self.N * self.N:
            raise ValueError("omega must hold N*N coefficients")
        W = self.empty() if out is None else out
        _check(self.lib.ze_basis_assemble(self._ctx, ctypes.c_void_p(om.data_ptr()), self._mat(W, "W")),
               "ze_basis_assemble")
        return W

    def basis_extract(self, W, out=None):
        """omega_lm = -i <T_lm, W>_F for all (l, m), flat at index l*l+l+m (device tensor)."""
        import torch

        om = torch.empty(self.N * self.N, dtype=torch.complex128, device=self.device) if out is None else out
        if om.numel() != self.N * self.N or om.dtype != torch.complex128 or not om.is_contiguous() \
                or om.device != self.device:
            raise ValueError("out must be a contiguous complex128 tensor of N*N on the context's device")
        _check(self.lib.ze_basis_extract(self._ctx, self._mat(W, "W"), ctypes.c_void_p(om.data_ptr())),
               "ze_basis_extract")
        return om

    def energy_spectrum(self, omega):
        """E_l = sum_m |omega_lm|^2 / (l(l+1)), l = 0..N-1 (device tensor of N doubles)."""
        import torch

        om = torch.as_tensor(omega, dtype=torch.complex128).to(self.device).contiguous()
        if om.numel() != self.N * self.N:
            raise ValueError("omega must hold N*N coefficients")
        E = torch.empty(self.N, dtype=torch.float64, device=self.device)
        _check(self.lib.ze_energy_spectrum(self._ctx, ctypes.c_void_p(om.data_ptr()),
                                           ctypes.c_void_p(E.data_ptr())), "ze_energy_spectrum")
        return E

    def set_initial_guess(self, mode: int):
        """0: each step starts from W_n; 1: steps after the first in isomp_run start from the
        extrapolation 2 W_n - F_prev of the previous converged midpoint; 2 (order 2 only):
        from the polynomial extrapolation (degree up to 3) of the run's previous midpoints,
        after which a step usually takes one evaluation; 3: as 2, with the run's states added
        to the starts of its third and fourth steps (order 2) and, with update form 1, the
        slope at W_0 to the second step's, which saves their second evaluations."""
        _check(self.lib.ze_set_initial_guess(self._ctx, int(mode)), "ze_set_initial_guess")

    def set_order(self, order: int):
        """Order of isomp_step / isomp_run: 2 (the midpoint map), 4 or 6 (its symmetric
        compositions, 3 and 9 midpoint substeps per step); iteration counts are then summed
        and residuals maximised over the substeps of a step."""
        _check(self.lib.ze_set_order(self._ctx, int(order)), "ze_set_order")

    def set_split_slices(self, slices: int):
        """Slices per operand of the PREC_SPLIT products (2 .. s_max(N): 8 up to N = 4096, 7 at
        8192, 3 at 16384; the int32 exactness bound)."""
        _check(self.lib.ze_set_split_slices(self._ctx, int(slices)), "ze_set_split_slices")

    def set_validation(self, on: bool = True):
        """Check the input W of isomp_step / isomp_run for skew-Hermitian and traceless to 1e-12
        (relative to max |W_rc|) before stepping; a failing W raises ZeulerError."""
        _check(self.lib.ze_set_validation(self._ctx, 1 if on else 0), "ze_set_validation")

    def set_update_form(self, form: int):
        """How W_{n+1} is formed: 0 (default) the second line of eq. (isomp) at the last
        iterate; 1 W_n + h (A - A^H), which conserves the spectrum to O(h ||P|| r) at a stopped
        iterate and lets the polynomial start take one evaluation per step."""
        _check(self.lib.ze_set_update_form(self._ctx, int(form)), "ze_set_update_form")

    def set_split_slices_lower(self, slices: int):
        """Slices of the lower product Q = A P (2 .. the product's slices; default one fewer,
        since Q's term enters the map with h^2/4 against h/2)."""
        _check(self.lib.ze_set_split_slices_lower(self._ctx, int(slices)), "ze_set_split_slices_lower")

    def profile(self, on: bool = True):
        """Turn per-phase event timing of isomp_step on or off."""
        _check(self.lib.ze_profile(self._ctx, int(bool(on))), "ze_profile")

    def profile_read(self, reset: bool = False) -> dict:
        """{phase: (total ms, launches)} accumulated since the last reset."""
        ms = (ctypes.c_double * 4)()
        n = (ctypes.c_longlong * 4)()
        _check(self.lib.ze_profile_read(self._ctx, ms, n, int(bool(reset))), "ze_profile_read")
        return {PHASES[i]: (ms[i], n[i]) for i in range(4)}


class Ensemble:
    """nsim independent simulations of sizes N_j stepped together (ze_ensemble_*)."""

    def __init__(self, sizes, stream=None):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("libzeuler needs a GPU (torch.cuda.is_available() is False)")
        self.lib = load_library()
        self.sizes = [int(n) for n in sizes]
        self.device = torch.device("cuda", torch.cuda.current_device())
        st = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.stream = st
        arr = (ctypes.c_int * len(self.sizes))(*self.sizes)
        self._ens = ctypes.c_void_p()
        _check(self.lib.ze_ensemble_create(len(self.sizes), arr, ctypes.c_void_p(st.cuda_stream),
                                           ctypes.byref(self._ens)), "ze_ensemble_create")

    def close(self):
        if getattr(self, "_ens", None) is not None and self._ens.value:
            self.lib.ze_ensemble_destroy(self._ens)
            self._ens = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _ptrs(self, Ws):
        import torch

        if len(Ws) != len(self.sizes):
            raise ValueError("one matrix per simulation")
        for W, n in zip(Ws, self.sizes):
            if (not isinstance(W, torch.Tensor) or W.dtype != torch.complex128 or W.device != self.device
                    or not W.is_contiguous() or tuple(W.shape) != (n, n)):
                raise ValueError(f"each W must be a contiguous ({n}, {n}) complex128 tensor on {self.device}")
        return (ctypes.c_void_p * len(Ws))(*[W.data_ptr() for W in Ws])

    def run(self, Ws, h: float, nsteps: int = 1, tol: float = 1e-12, K: int = 8,
            prec: int = PREC_FP64):
        """nsteps steps of every simulation, each W updated in place."""
        _check(self.lib.ze_ensemble_run(self._ens, self._ptrs(Ws), float(h), float(tol), int(K),
                                        int(nsteps), int(prec)), "ze_ensemble_run")

    def stats(self):
        """(evaluations, residual) per simulation for the last step."""
        n = len(self.sizes)
        its = (ctypes.c_int * n)()
        res = (ctypes.c_double * n)()
        _check(self.lib.ze_ensemble_stats(self._ens, its, res), "ze_ensemble_stats")
        return list(its), list(res)

    def set_split_slices(self, slices: int):
        """Slices per operand of the ensemble's PREC_SPLIT products (2 .. s_max of the largest N)."""
        _check(self.lib.ze_ensemble_set_split_slices(self._ens, int(slices)),
               "ze_ensemble_set_split_slices")

    def set_update_form(self, form: int):
        """Form of W_{n+1} for the ensemble's steps (as Zeuler.set_update_form)."""
        _check(self.lib.ze_ensemble_set_update_form(self._ens, int(form)),
               "ze_ensemble_set_update_form")

    def set_split_slices_lower(self, slices: int):
        """Slices of the ensemble's lower products (2 .. the product's slices)."""
        _check(self.lib.ze_ensemble_set_split_slices_lower(self._ens, int(slices)),
               "ze_ensemble_set_split_slices_lower")

    def set_continuation(self, on: bool = True):
        """With it on, a run on the same matrices (unchanged since) with the same h, precision
        and step options continues the last run's trajectories instead of starting at step 0."""
        _check(self.lib.ze_ensemble_set_continuation(self._ens, int(bool(on))),
               "ze_ensemble_set_continuation")

    def set_initial_guess(self, mode: int):
        """0: every step starts from W_n; 1: steps after the first of a run start each simulation
        from 2 W_n - F_prev; 2, 3: the polynomial starts (as Zeuler.set_initial_guess)."""
        _check(self.lib.ze_ensemble_set_initial_guess(self._ens, int(mode)),
               "ze_ensemble_set_initial_guess")

    def set_steady_cap(self, cap: int, from_step: int = 4):
        """Evaluation cap min(K, cap) for the steps from index from_step on of each run (with the
        polynomial start); 0 restores K for every step."""
        _check(self.lib.ze_ensemble_set_steady_cap(self._ens, int(cap), int(from_step)),
               "ze_ensemble_set_steady_cap")

    def tuning(self, prec: int = PREC_FP64):
        """(choice, [ms per step of the candidates]) of the autotuner for precision prec:
        FP64 has 4 candidates (2 * tile shape + work order), PREC_SPLIT 2 (work order)."""
        ch = ctypes.c_int(0)
        ms = (ctypes.c_double * 4)()
        _check(self.lib.ze_ensemble_tuning(self._ens, int(prec), ctypes.byref(ch), ms),
               "ze_ensemble_tuning")
        return ch.value, list(ms)[: (2 if prec == PREC_SPLIT else 4)]

