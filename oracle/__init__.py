"""Plain FP64 CPU oracle for the isospectral-midpoint Zeitlin--Euler step on the sphere.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or execute this
package: only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` use it.  It shares no code with the HIP path (``paper_2206_05466_amd``) and
does not import it; the only code both sides share is the seeded input generator in
``workloads/``, which holds random draws and no arithmetic of the method.

What it computes, with the passage of Cifani, Viviani & Modin (arXiv 2206.05466) each part
follows:

* ``laplacian``  -- the quantised Laplacian Delta_N: the tridiagonal blocks Delta^m of
  eq. (delta_tria) (Sec. 3.2) and, for tiny N, the dense N^2 x N^2 operator built from the
  spin-s representation, whose spectrum -l(l+1) is eq. (lap_prop).
* ``stream``     -- the stream solve P = Delta_N^+ W, one tridiagonal system per diagonal,
  eq. (sub_tria_W) (Sec. 3.3), with LAPACK's positive-definite tridiagonal routines.
* ``isomp``      -- the isospectral midpoint step, eq. (isomp) (Sec. 2), reached by the
  fixed-point iteration eq. (isomp_iter) with the infinity-norm stopping rule (Sec. 2);
  and the order-4 and order-6 symmetric compositions of that step (the higher-order members
  of the family Sec. 2 names).
* ``casimirs``   -- C_k(W) = Tr(W^k), eq. (W_pow).
* ``basis``      -- the quantised basis T_lm as eigenvectors of Delta^m (Sec. 3.2) and the
  assembly W = sum_lm i omega_lm T_lm, eq. (W0); plus the inverse projection and the
  kinetic energy spectrum of the coefficients (Sec. 4).

Every function is pinned by ``tests/test_oracle_*.py`` against closed forms, brute force
on tiny N and invariants that the paper and the mathematics fix (see the docstrings).
"""

from .laplacian import delta_tridiag, spin_matrices, brute_laplacian, apply_laplacian
from .stream import stream_solve
from .isomp import (isomp_step, isomp_run, extrapolate_midpoints, start_from_history,
                    start_second_step, composition_weights, isomp_composed_run)
from .casimirs import casimirs, casimirs_eig
from .basis import eigvecs, assemble, extract, energy_spectrum

__all__ = [
    "delta_tridiag", "spin_matrices", "brute_laplacian", "apply_laplacian",
    "stream_solve", "isomp_step", "isomp_run", "extrapolate_midpoints", "start_from_history",
    "start_second_step",
    "composition_weights", "isomp_composed_run", "casimirs", "casimirs_eig",
    "eigvecs", "assemble", "extract", "energy_spectrum",
]
