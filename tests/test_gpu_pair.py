"""GPU parity of the two-operand tiled product (sp2_pair_product) against
dense NumPy products of the same seeded operands: anticommutator (the
derivative of the square used by the adjoint), commutator with an
antisymmetric result, and the product with an antisymmetric operand (both
used by the subspace correction)."""
import numpy as np
import pytest

from fockgen import BSR, bsr_to_dense, random_sym_bsr

from gpu_helpers import rel, to_dense, upper_mask

pytestmark = pytest.mark.gpu

CASES = [(200, 1.0, 1), (1000, 0.35, 2), (1500, 0.12, 3)]


def _mask(M):
    m = np.zeros((M.nbr, M.nbr), dtype=bool)
    m[M.rows(), M.col_idx] = True
    return m | m.T


def _pair_pattern(Mx, My):
    a, b = Mx.astype(np.int64), My.astype(np.int64)
    return ((a @ b) > 0) | ((b @ a) > 0)


def _expand(M, n):
    return np.kron(M, np.ones((64, 64), dtype=bool))[:n, :n]


def _antisym_bsr(n, density, seed):
    """Antisymmetric matrix held by its upper blocks (lower = -transpose)."""
    S = random_sym_bsr(n, density, seed=seed)
    val = S.val.copy()
    I = S.rows()
    d = I == S.col_idx
    val[d] = val[d] - val[d].transpose(0, 2, 1)
    # zero the padding rows / columns of the last block row
    pad = S.nbr * 64 - n
    if pad:
        last = S.nbr - 1
        val[I == last, 64 - pad:, :] = 0.0
        val[S.col_idx == last, :, 64 - pad:] = 0.0
    return S.with_values(val)


def _anti_dense(M):
    """Dense antisymmetric matrix of upper blocks (lower blocks = -transpose)."""
    P = np.zeros((M.nbr, M.nbr, 64, 64))
    I, J = M.rows(), M.col_idx.astype(np.int64)
    P[I, J] = M.val
    off = I != J
    P[J[off], I[off]] = -M.val[off].transpose(0, 2, 1)
    return P.transpose(0, 2, 1, 3).reshape(M.nbr * 64, M.nbr * 64)[: M.n, : M.n]


def _anti_to_dense_dev(M):
    n, rp, ci, v = M.to_host()
    return _anti_dense(BSR(n, rp, ci, v))


@pytest.mark.parametrize("n,dens,seed", CASES)
def test_anticommutator_fp64(gpu_lib, n, dens, seed):
    sp2 = gpu_lib
    Xh, Yh = random_sym_bsr(n, dens, seed=seed, std=0.1), random_sym_bsr(n, dens * 0.6, seed=seed + 10, std=0.1)
    Gh = random_sym_bsr(n, dens * 0.5, seed=seed + 20)
    X, Y, G = (sp2.BsrMatrix.from_host(m) for m in (Xh, Yh, Gh))
    out, sums = sp2.pair_product(X, Y, G, sign=1, a=0.3, b=-0.5, c=1.7)
    Xd, Yd, Gd = bsr_to_dense(Xh), bsr_to_dense(Yh), bsr_to_dense(Gh)
    MP = _pair_pattern(_mask(Xh), _mask(Yh))
    assert np.array_equal(upper_mask(out), np.triu(MP))
    E = _expand(MP, n)
    ref = (0.3 * np.eye(n) - 0.5 * Gd + 1.7 * (Xd @ Yd + Yd @ Xd)) * E
    got = to_dense(out)
    assert rel(got, ref) <= 1e-13
    assert sums[0] == pytest.approx(float(np.sum(ref ** 2)), rel=1e-12)


@pytest.mark.parametrize("n,dens,seed", CASES[:2])
def test_commutator_antisymmetric_result(gpu_lib, n, dens, seed):
    sp2 = gpu_lib
    Xh, Yh = random_sym_bsr(n, dens, seed=seed), random_sym_bsr(n, dens * 0.5, seed=seed + 3)
    out, sums = sp2.pair_product(sp2.BsrMatrix.from_host(Xh), sp2.BsrMatrix.from_host(Yh), sign=-1)
    Xd, Yd = bsr_to_dense(Xh), bsr_to_dense(Yh)
    ref = Xd @ Yd - Yd @ Xd
    got = _anti_to_dense_dev(out)
    assert rel(got, ref) <= 1e-13
    # lower blocks mirror the stored ones exactly; diagonal blocks are
    # antisymmetric up to rounding
    assert np.linalg.norm(got + got.T) <= 1e-13 * np.linalg.norm(got)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("n,dens,seed", CASES[:2])
def test_commutator_with_antisymmetric_operand(gpu_lib, prec, n, dens, seed):
    """[X, C] = X C - C X with C antisymmetric is symmetric."""
    sp2 = gpu_lib
    Xh = random_sym_bsr(n, dens, seed=seed, std=0.1)
    Ch = _antisym_bsr(n, dens * 0.6, seed + 5)
    out, _ = sp2.pair_product(sp2.BsrMatrix.from_host(Xh), sp2.BsrMatrix.from_host(Ch), sign=-1, y_antisym=True,
                              c=-0.25, precision=prec)
    Xd, Cd = bsr_to_dense(Xh), _anti_dense(Ch)
    ref = -0.25 * (Xd @ Cd - Cd @ Xd)
    got = to_dense(out)
    Xa, Ca = np.abs(Xd), np.abs(Cd)
    mag = 0.25 * (Xa @ Ca + Ca @ Xa)
    if prec == "fp64":
        assert rel(got, ref) <= 1e-13
    else:
        # FP32 rounding of the operands and of the accumulation (plus, for
        # BF16x3, 3 * 2^-16 per product from the split)
        u = 2.0 ** -24
        split = 3 * 2.0 ** -16 if prec == "bf16x3" else 0.0
        bound = (split + 4 * u * (n + 4)) * mag + 1e-30
        assert np.all(np.abs(got - ref) <= bound)


def test_pair_fp32_anticommutator_bound(gpu_lib):
    sp2 = gpu_lib
    n = 1000
    Xh, Yh = random_sym_bsr(n, 0.35, seed=7, std=0.1), random_sym_bsr(n, 0.2, seed=8, std=0.1)
    out, _ = sp2.pair_product(sp2.BsrMatrix.from_host(Xh), sp2.BsrMatrix.from_host(Yh), G=sp2.BsrMatrix.from_host(Yh),
                              sign=1, b=2.0, c=-1.0, precision="fp32")
    Xd, Yd = bsr_to_dense(Xh), bsr_to_dense(Yh)
    MP = _pair_pattern(_mask(Xh), _mask(Yh))
    ref = (2.0 * Yd - (Xd @ Yd + Yd @ Xd)) * _expand(MP, n)
    Xa, Ya = np.abs(Xd), np.abs(Yd)
    bound = 4 * 2.0 ** -24 * (2 * Ya + (n + 4) * (Xa @ Ya + Ya @ Xa)) + 1e-30
    assert np.all(np.abs(to_dense(out) - ref) <= bound)
