"""Host-side input generators (no GPU): the banded test matrices of the norm
comparison and the sparse-to-BSR conversion used to feed them to the library."""
import numpy as np
import pytest

from fockgen import banded_sym, bsr_to_dense, dense_to_bsr, sparse_to_bsr
from oracle import sp2_oracle as O


@pytest.mark.parametrize("permute", [False, True])
@pytest.mark.parametrize("n,bw", [(130, 10), (700, 100)])
def test_sparse_to_bsr_matches_dense(n, bw, permute):
    A = banded_sym(n, half_bw=bw, seed=3, permute=permute)
    Ad = A.toarray()
    assert np.array_equal(Ad, Ad.T)
    M, R = sparse_to_bsr(A), dense_to_bsr(Ad)
    assert np.array_equal(M.row_ptr, R.row_ptr) and np.array_equal(M.col_idx, R.col_idx)
    assert np.array_equal(M.val, R.val)
    assert np.array_equal(bsr_to_dense(M), Ad)


def test_banded_structure_and_norms():
    """Band of half width bw with entries in [0, 1e-3); the permutation keeps
    the spectrum and the Frobenius norm, and the Frob-Inf norm bounds the
    spectral norm in both orderings."""
    n, bw = 600, 40
    A = banded_sym(n, half_bw=bw, seed=0).toarray()
    i, j = np.nonzero(A)
    assert np.max(np.abs(i - j)) <= bw and A.min() >= 0.0 and A.max() < 1e-3
    P = banded_sym(n, half_bw=bw, seed=0, permute=True).toarray()
    assert np.allclose(np.linalg.eigvalsh(A), np.linalg.eigvalsh(P), atol=1e-14)
    assert O.frobenius_norm(A) == pytest.approx(O.frobenius_norm(P), rel=1e-14)
    for M in (A, P):
        s = O.spectral_norm_sym(M)
        for cbs in (64, 128):
            assert s <= O.frob_inf_norm(M, cbs) * (1 + 1e-12)
