"""Discrete Casimirs C_k(W) = Tr(W^k), eq. (W_pow) (oracle).

``casimirs`` is the definition written out (repeated products, then the trace).
``casimirs_eig`` is an independent route through the spectrum: iW is Hermitian, so
W = -i U diag(lambda) U^H and Tr(W^k) = sum_j (-i lambda_j)^k (LAPACK ``zheevd`` via
``numpy.linalg.eigvalsh``).
"""

import numpy as np


def casimirs(W: np.ndarray, kmax: int) -> np.ndarray:
    """[C_1, ..., C_kmax] with C_k = Tr(W^k) (complex128)."""
    W = np.asarray(W, dtype=np.complex128)
    out = np.zeros(kmax, dtype=np.complex128)
    Wk = np.eye(W.shape[0], dtype=np.complex128)
    for k in range(1, kmax + 1):
        Wk = Wk @ W
        out[k - 1] = np.trace(Wk)
    return out


def casimirs_eig(W: np.ndarray, kmax: int) -> np.ndarray:
    """Tr(W^k) from the eigenvalues of the Hermitian matrix iW."""
    lam = np.linalg.eigvalsh(1j * np.asarray(W, dtype=np.complex128))
    mu = -1j * lam
    return np.array([np.sum(mu ** k) for k in range(1, kmax + 1)], dtype=np.complex128)
