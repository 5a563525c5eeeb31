"""Pins of the oracle's general (full-pattern) product, ``general_product``:
explicit block loops on tiny inputs, the transpose identity (A B)^T =
B^T A^T, and the symmetric special case, in which it must reproduce the
oracle's own polynomial step of Algorithm 2 (a different formula: Y Y or
2 Z - Z Z) and the symmetric square's pattern and work count."""
import numpy as np
import pytest

from fockgen import bsr_to_dense, lattice_fock
from oracle import sp2_oracle as O


def random_general(nbr, bs, density, seed, diag=True):
    rng = np.random.default_rng(seed)
    M = rng.random((nbr, nbr)) < density
    if diag:
        M[np.arange(nbr), np.arange(nbr)] = True
    A = rng.standard_normal((nbr * bs, nbr * bs)) * O.expand_mask(M, nbr * bs, bs)
    return A, M


def loops_product(A, MA, B, MB, G, MG, a, b, c, bs, n):
    """The same quantity block by block with explicit loops."""
    nbr = MA.shape[0]
    out = np.zeros((n, n))
    P = np.zeros((nbr, nbr), dtype=bool)
    triples = 0
    blk = lambda X, I, J: X[I * bs:(I + 1) * bs, J * bs:(J + 1) * bs]
    for I in range(nbr):
        for J in range(nbr):
            acc = np.zeros((bs, bs))
            hit = False
            for K in range(nbr):
                if MA[I, K] and MB[K, J]:
                    hit = True
                    triples += 1
                    for r in range(bs):
                        for s in range(bs):
                            acc[r, s] += sum(blk(A, I, K)[r, k] * blk(B, K, J)[k, s] for k in range(bs))
            o = c * acc
            if G is not None and MG[I, J]:
                o = o + b * blk(G, I, J)
                hit = True
            if a != 0.0 and I == J:
                o = o + a * np.eye(bs)
                hit = True
            if hit:
                P[I, J] = True
                out[I * bs:(I + 1) * bs, J * bs:(J + 1) * bs] = o
    return out, P, triples


@pytest.mark.parametrize("seed,a,b,c,with_g", [(0, 0.0, 0.0, 1.0, False), (1, 0.25, -0.5, 2.0, True),
                                               (2, 1.0, 2.0, -1.0, True), (3, 0.0, 1.0, 1.0, True)])
def test_general_product_by_block_loops(seed, a, b, c, with_g):
    bs, nbr = 3, 5
    A, MA = random_general(nbr, bs, 0.4, seed, diag=False)
    B, MB = random_general(nbr, bs, 0.4, seed + 10, diag=False)
    G, MG = random_general(nbr, bs, 0.3, seed + 20, diag=False) if with_g else (None, None)
    n = nbr * bs
    out, P, sums = O.general_product(A, MA, B, MB, G, MG, a, b, c, bs=bs)
    ref, Pref, triples = loops_product(A, MA, B, MB, G, MG, a, b, c, bs, n)
    assert np.array_equal(P, Pref)
    assert np.allclose(out, ref, rtol=1e-13, atol=1e-13)
    Gd = G if with_g else np.zeros((n, n))
    S = loops_product(A, MA, B, MB, None, None, 0.0, 0.0, 1.0, bs, n)[0]
    assert sums[0] == pytest.approx(float(np.sum((Gd - S) ** 2)), rel=1e-12)
    assert sums[1] == pytest.approx(float(sum(Gd[i, i] for i in range(n))), abs=1e-12)
    assert sums[2] == pytest.approx(float(sum(S[i, i] for i in range(n))), abs=1e-12)
    assert sums[3] == 2.0 * bs ** 3 * triples


def test_general_product_transpose_identity():
    bs, nbr = 4, 7
    A, MA = random_general(nbr, bs, 0.35, 5)
    B, MB = random_general(nbr, bs, 0.35, 6)
    out, P, _ = O.general_product(A, MA, B, MB, bs=bs)
    outT, PT, _ = O.general_product(B.T, MB.T, A.T, MA.T, bs=bs)
    assert np.array_equal(PT, P.T)
    assert np.allclose(outT, out.T, rtol=1e-13, atol=1e-13)
    # non-symmetric operands give a non-symmetric result
    assert not np.allclose(out, out.T)


def test_general_square_is_the_polynomial_step():
    """X_1 = f_1(X~_0) of the oracle's expansion (no truncation), formed as the
    general product a I + b X + c X X of the symmetric X~_0 in full storage."""
    Fh, info = lattice_fock(4, seed=0)
    F = bsr_to_dense(Fh)
    lmin, lmax = O.gershgorin_bounds(F)
    ref = O.sp2(F, info["n_occ"], lmin, lmax, -0.5, 0.5, trunc_norm=O.TRUNC_NONE, keep_tape=True, n_max_cap=3)
    for i in (1, 2, 3):
        p, al = ref.p[i], ref.alpha[i]
        if p == 1:
            a, b, c = (1 - al) ** 2, 2 * al * (1 - al), al * al
        else:
            a, b, c = 0.0, 2 * al, -al * al
        X, M = ref.X[i - 1], ref.masks[i - 1]
        out, P, sums = O.general_product(X, M, X, M, X, M, a, b, c)
        assert np.array_equal(P, O.pattern_square(M))
        assert np.allclose(out, ref.X[i], rtol=0, atol=1e-12 * np.abs(ref.X[i]).max())
        assert np.array_equal(out, out.T) or np.allclose(out, out.T, rtol=0, atol=1e-14)
        # the general product does every block product of both triangles: twice
        # the symmetric square's work less the diagonal output blocks' share
        Mi = M.astype(np.int64)
        assert sums[3] == 2.0 * O.BS ** 3 * (2 * O._triples_upper(M) - int(np.trace(Mi @ Mi)))
        assert sums[0] == pytest.approx(ref.e[i - 1] ** 2, rel=1e-10)
