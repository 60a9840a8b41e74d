"""The allocation-free product ze_zgemm_noalloc against the context product ze_zgemm (FP64).

Both run the same FP64 MFMA kernel; the allocation-free one keeps its split-K partial sums
in the library's fixed device array, whose size can give a different K split, so the two
agree to the rounding of a length-2N real dot product: elementwise within
2 * (2N) * 2^-53 * (|A| |B|)_ij of each other and of the exact product (numpy's FP64 product
stands in for it at the same bound).  Two calls in a row, the second with a smaller N, show
that what the first call left in the array does not leak into the second.
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _rand(rng, N):
    return rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))


def test_noalloc_product_matches_context_product_twice():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2206_05466_amd import PREC_FP64, Zeuler, zgemm_noalloc

    rng = np.random.default_rng(77)
    # N = 1000: 128 tiles of 128 x 64, a partial round split along K into partial sums in the
    # array; N = 600: 50 such tiles, split again (fewer partial sums over the last call's);
    # N = 200: the small kernel (49 tiles of 32 x 32, no partial sums); N = 2048: whole rounds
    # only, no partial sums
    for N in (1000, 600, 200, 2048):
        A, B = _rand(rng, N), _rand(rng, N)
        Ad, Bd = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
        out = torch.full((N, N), complex(np.nan, np.nan), dtype=torch.complex128, device="cuda")
        zgemm_noalloc(Ad, Bd, out)
        with Zeuler(N) as z:
            ref = z.zgemm(Ad, Bd, prec=PREC_FP64)
        torch.cuda.synchronize()
        got, ctx = out.cpu().numpy(), ref.cpu().numpy()
        bound = 2 * (2 * N) * 2.0 ** -53 * (np.abs(A.real) + np.abs(A.imag)) @ (np.abs(B.real) + np.abs(B.imag))
        assert np.all(np.isfinite(got)), N
        assert np.all(np.abs(got - ctx) <= bound), N
        assert np.all(np.abs(got - A @ B) <= bound), N
