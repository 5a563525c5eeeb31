"""Pins of the oracle's norms and truncation.

* ||A||_2 <= ||A||_m <= ||A||_M for symmetric A (section "Upper bounds for the
  spectral norm"), with the spectral norm from LAPACK, on random and banded
  matrices like those of Figure 1, and closed forms on the identity.
* The truncation removes a part E with ||E||_F <= tau or ||E||_M <= tau, as
  measured directly on X - X~, never removes a diagonal block, and removes the
  longest ascending prefix (brute force over prefixes on tiny inputs).
"""
import itertools
import math

import numpy as np
import pytest

from oracle import sp2_oracle as O


def _rand_sym(n, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n))
    return A + A.T


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("sub", [7, 16, 50])
def test_norm_inequalities(seed, sub):
    A = _rand_sym(120, seed)
    s2 = O.spectral_norm_sym(A)
    m = O.frob_spectral_norm(A, sub)
    M = O.frob_inf_norm(A, sub)
    assert s2 <= m * (1 + 1e-12)
    assert m <= M * (1 + 1e-12)
    assert M <= O.frobenius_norm(A) * math.sqrt((120 + sub - 1) // sub) + 1e-12


def test_norm_inequalities_banded():
    """Symmetric banded matrix with entries U(0, 1e-3) and half-width 300, as in
    Figure 1 (smaller n)."""
    rng = np.random.default_rng(0)
    n, hw = 900, 300
    A = rng.uniform(0.0, 1e-3, size=(n, n))
    A = np.triu(A) + np.triu(A, 1).T
    i, j = np.indices((n, n))
    A[np.abs(i - j) > hw] = 0.0
    s2 = O.spectral_norm_sym(A)
    for sub in (100, 500):
        assert s2 <= O.frob_spectral_norm(A, sub) <= O.frob_inf_norm(A, sub) * (1 + 1e-12)


def test_frobinf_scales_like_spectral_norm_banded():
    """Figure 1 text: for banded matrices the Frob-Inf norm levels off with the
    matrix size, like the spectral norm, while the Frobenius norm keeps growing
    (as the square root of the size)."""
    def band(n):
        rng = np.random.default_rng(0)
        A = rng.uniform(0.0, 1e-3, size=(n, n))
        A = np.triu(A) + np.triu(A, 1).T
        i, j = np.indices((n, n))
        A[np.abs(i - j) > 300] = 0.0
        return A
    a, b = band(1500), band(3000)
    assert O.frobenius_norm(b) / O.frobenius_norm(a) > 1.35
    assert O.frob_inf_norm(b, 100) / O.frob_inf_norm(a, 100) < 1.05
    assert O.frob_inf_norm(b, 500) / O.frob_inf_norm(a, 500) < 1.05


def test_norm_closed_forms():
    n, s = 96, 32
    I = np.eye(n)
    assert O.spectral_norm_sym(I) == pytest.approx(1.0)
    assert O.frobenius_norm(I) == pytest.approx(math.sqrt(n))
    assert O.frob_inf_norm(I, s) == pytest.approx(math.sqrt(s))
    assert O.frob_spectral_norm(I, s) == pytest.approx(math.sqrt(s))
    assert O.inf_norm(np.ones((5, 5))) == 5.0


def _block_sym(nbr, bs, seed, scale_spread=4.0):
    rng = np.random.default_rng(seed)
    n = nbr * bs
    X = np.zeros((n, n))
    for I in range(nbr):
        for J in range(I, nbr):
            b = rng.standard_normal((bs, bs)) * 10 ** rng.uniform(-scale_spread, 0)
            if I == J:
                b = b + b.T
            X[I * bs:(I + 1) * bs, J * bs:(J + 1) * bs] = b
            X[J * bs:(J + 1) * bs, I * bs:(I + 1) * bs] = b.T
    return X


@pytest.mark.parametrize("seed", range(6))
def test_frobenius_truncation_bound_and_prefix(seed):
    bs, nbr = 2, 5
    X = _block_sym(nbr, bs, seed)
    M = np.ones((nbr, nbr), dtype=bool)
    n2 = O.block_norms2(X, bs)
    cand = sorted(((n2[I, J], I * nbr + J, I, J) for I in range(nbr) for J in range(I + 1, nbr)))
    for tau in (1e-3, 1e-2, 0.1, 1.0):
        Xt, Mt, info = O.truncate(X, M, tau, O.TRUNC_FROB, bs)
        E = X - Xt
        assert O.frobenius_norm(E) <= tau * (1 + 1e-12)
        assert info.err_frob == pytest.approx(O.frobenius_norm(E), rel=1e-12, abs=1e-300)
        assert all(Mt[i, i] for i in range(nbr))
        # brute force: the longest prefix whose full-matrix Frobenius norm fits
        best = 0
        for m in range(len(cand) + 1):
            Em = np.zeros_like(X)
            for _, _, I, J in cand[:m]:
                Em[I * bs:(I + 1) * bs, J * bs:(J + 1) * bs] = X[I * bs:(I + 1) * bs, J * bs:(J + 1) * bs]
                Em[J * bs:(J + 1) * bs, I * bs:(I + 1) * bs] = X[J * bs:(J + 1) * bs, I * bs:(I + 1) * bs]
            if O.frobenius_norm(Em) <= tau:
                best = m
            else:
                break
        removed = {(I, J) for _, _, I, J in cand[:best]}
        got = {(I, J) for I in range(nbr) for J in range(I + 1, nbr) if not Mt[I, J]}
        assert got == removed


@pytest.mark.parametrize("seed", range(6))
def test_frobinf_truncation_bound(seed):
    bs, nbr, cbs = 2, 9, 6  # coarse blocks of 3 fine blocks, last one ragged
    X = _block_sym(nbr, bs, seed)
    rng = np.random.default_rng(100 + seed)
    M = np.triu(rng.random((nbr, nbr)) < 0.7)
    M = M | M.T
    M[np.arange(nbr), np.arange(nbr)] = True
    X = X * O.expand_mask(M, X.shape[0], bs)
    for tau in (1e-3, 1e-2, 0.1, 1.0):
        Xt, Mt, info = O.truncate(X, M, tau, O.TRUNC_FROBINF, bs, cbs)
        E = X - Xt
        assert O.frob_inf_norm(E, cbs) <= tau * (1 + 1e-12)
        assert info.err_mixed == pytest.approx(O.frob_inf_norm(E, cbs), rel=1e-12, abs=1e-300)
        assert info.err_frob == pytest.approx(O.frobenius_norm(E), rel=1e-12, abs=1e-300)
        assert all(Mt[i, i] for i in range(nbr))
        assert not np.any(Mt & ~M)


def test_frobinf_equals_frobenius_single_coarse_block():
    bs, nbr = 2, 6
    X = _block_sym(nbr, bs, 7)
    M = np.ones((nbr, nbr), dtype=bool)
    for tau in (1e-2, 0.3):
        a = O.truncate(X, M, tau, O.TRUNC_FROB, bs)[1]
        b = O.truncate(X, M, tau, O.TRUNC_FROBINF, bs, coarse_bs=bs * nbr)[1]
        assert np.array_equal(a, b)


def test_frobinf_tie_order_by_index():
    """Equal block norms are taken in (I, J) order."""
    bs, nbr = 1, 4
    X = np.eye(nbr) + 0.1 * (np.ones((nbr, nbr)) - np.eye(nbr))
    M = np.ones((nbr, nbr), dtype=bool)
    # each off-diagonal pair weighs 2 * 0.01; budget fits exactly two of them
    Xt, Mt, info = O.truncate(X, M, math.sqrt(0.04), O.TRUNC_FROB, bs)
    removed = [(I, J) for I, J in itertools.combinations(range(nbr), 2) if not Mt[I, J]]
    assert removed == [(0, 1), (0, 2)]
