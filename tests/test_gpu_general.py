"""GPU parity of the general (full-pattern) storage path against the oracle:
sp2_general_from_upper and sp2_general_product (FP64 and BF16x3, both tile
edges), non-symmetric operands with different patterns, a ragged last block
row, the symmetric special case against the symmetric square, and the
degenerate and invalid inputs."""
import numpy as np
import pytest

from fockgen import (bsr_to_dense, general_block_mask, general_bsr_to_dense, lattice_fock, random_general_bsr,
                     random_sym_bsr)
from oracle import sp2_oracle as O

from gpu_helpers import general_mask, to_dense, to_dense_general, upper_mask

pytestmark = pytest.mark.gpu

# n (ragged unless a multiple of 64), density of A / B / G, seed
CASES = [(64, 1.0, 0), (200, 0.7, 1), (1000, 0.35, 2), (1150, 0.8, 3), (1500, 0.12, 4)]


def _oracle(Ah, Bh, Gh, a, b, c):
    A, B = general_bsr_to_dense(Ah), general_bsr_to_dense(Bh)
    G = general_bsr_to_dense(Gh) if Gh is not None else None
    MG = general_block_mask(Gh) if Gh is not None else None
    return O.general_product(A, general_block_mask(Ah), B, general_block_mask(Bh), G, MG, a, b, c)


@pytest.mark.parametrize("n,dens,seed", CASES)
@pytest.mark.parametrize("coef", [(0.0, 0.0, 1.0), (0.3, -0.7, 1.9)])
def test_general_product_fp64_matches_oracle(gpu_lib, n, dens, seed, coef):
    sp2 = gpu_lib
    a, b, c = coef
    Ah = random_general_bsr(n, dens, seed=seed, std=0.1)
    Bh = random_general_bsr(n, dens, seed=seed + 100, std=0.1)
    Gh = random_general_bsr(n, dens / 2, seed=seed + 200) if b != 0.0 else None
    G = sp2.BsrMatrix.from_host(Gh) if Gh is not None else None
    out, sums = sp2.general_product(sp2.BsrMatrix.from_host(Ah), sp2.BsrMatrix.from_host(Bh), G, a, b, c, "fp64")
    ref, P, rsums = _oracle(Ah, Bh, Gh, a, b, c)
    assert np.array_equal(general_mask(out), P)
    D = to_dense_general(out)
    # both sides within the worst-case FP64 bound (n + 2) u of the exact value
    scale = abs(c) * (np.abs(general_bsr_to_dense(Ah)) @ np.abs(general_bsr_to_dense(Bh))) + abs(a)
    if Gh is not None:
        scale = scale + abs(b) * np.abs(general_bsr_to_dense(Gh))
    assert np.all(np.abs(D - ref) <= 2 * (n + 2) * 2.0 ** -53 * scale + 1e-300)
    assert sums[0] == pytest.approx(rsums[0], rel=1e-12)
    assert sums[1] == pytest.approx(rsums[1], rel=1e-12, abs=1e-12)
    assert sums[2] == pytest.approx(rsums[2], rel=1e-12, abs=1e-12)
    assert sums[3] == rsums[3]


@pytest.mark.parametrize("n,dens,seed", CASES[1:4])
def test_general_product_bf16x3_bound(gpu_lib, monkeypatch, n, dens, seed):
    """BF16x3 (hi*hi + hi*lo + lo*hi, FP32 accumulation): each product term is
    off by at most 3 * 2^-16 |x||y|, plus FP32 rounding of the inputs, the
    accumulation and the output; the 2 x 2 and 4 x 4 tile kernels give the
    same bits."""
    sp2 = gpu_lib
    a, b, c = 0.25, 0.5, -1.5
    Ah = random_general_bsr(n, dens, seed=seed, std=0.1)
    Bh = random_general_bsr(n, dens, seed=seed + 100, std=0.1)
    Gh = random_general_bsr(n, dens / 2, seed=seed + 200, std=0.1)
    A, B, G = (sp2.BsrMatrix.from_host(M) for M in (Ah, Bh, Gh))
    res = {}
    for tb in ("2", "4"):
        monkeypatch.setenv("SP2_BF16X3_TILE", tb)
        res[tb] = sp2.general_product(A, B, G, a, b, c, "bf16x3")
    out, sums = res["4"]
    ref, P, rsums = _oracle(Ah, Bh, Gh, a, b, c)
    assert np.array_equal(general_mask(out), P)
    Aa, Ba = np.abs(general_bsr_to_dense(Ah)), np.abs(general_bsr_to_dense(Bh))
    Ga = np.abs(general_bsr_to_dense(Gh))
    u = 2.0 ** -24
    AB = Aa @ Ba
    bound = abs(c) * (3 * 2.0 ** -16 * AB + 4 * u * (n + 2) * AB) + 4 * u * (abs(b) * Ga + abs(a)) + 1e-30
    err = np.abs(to_dense_general(out) - ref)
    assert np.all(err <= bound)
    assert sums[3] == rsums[3]
    assert np.array_equal(res["2"][0].val.cpu().numpy(), out.val.cpu().numpy())
    assert res["2"][1] == sums


@pytest.mark.parametrize("n,dens,seed", [(64, 1.0, 0), (1000, 0.35, 2), (1500, 0.12, 4)])
def test_general_from_upper(gpu_lib, n, dens, seed):
    """The general storage of a symmetric upper-BSR matrix holds both
    triangles: the same dense matrix, bit for bit, on the mirrored pattern."""
    sp2 = gpu_lib
    Uh = random_sym_bsr(n, dens, seed=seed)
    G = sp2.general_from_upper(sp2.BsrMatrix.from_host(Uh))
    from fockgen import block_mask_of_bsr

    assert np.array_equal(general_mask(G), block_mask_of_bsr(Uh))
    assert np.array_equal(to_dense_general(G), bsr_to_dense(Uh))


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_general_square_equals_symmetric_square(gpu_lib, prec):
    """A symmetric X in general storage squared by the general product gives,
    on the upper blocks, the symmetric square's result bit for bit (same
    block products in the same order), and the lower blocks are their
    transposes: exactly in FP64; in BF16x3 to the FP32 accumulation rounding,
    since the transposed entry takes the lo*hi and hi*lo terms in the other
    order (as the two triangles of a diagonal block of the symmetric square
    do).  The general product does the block products of both triangles (the
    oracle's count)."""
    sp2 = gpu_lib
    Fh, info = lattice_fock(6, seed=0)
    X = sp2.BsrMatrix.from_host(Fh.with_values(Fh.val * 0.05))
    a, b, c = 0.1, 0.4, -0.6
    S, ssum = sp2.square_step(X, a, b, c, prec)
    Xg = sp2.general_from_upper(X)
    Gm, gsum = sp2.general_product(Xg, Xg, Xg, a, b, c, prec)
    Dg, Ds = to_dense_general(Gm), to_dense(S)
    assert np.array_equal(np.triu(general_mask(Gm)), upper_mask(S))
    assert np.array_equal(np.triu(Dg), np.triu(Ds))
    if prec == "fp64":
        assert np.array_equal(Dg, Dg.T)
    else:
        Xa = np.abs(to_dense(X))
        n = Xa.shape[0]
        bound = 2 * (n + 2) * 2.0 ** -24 * abs(c) * (Xa @ Xa) + 2.0 ** -23 * np.abs(Dg) + 1e-30
        assert np.all(np.abs(Dg - Dg.T) <= bound)
        assert not np.array_equal(Dg, Dg.T)  # the order effect is real
    # ||X - S||^2: the lower blocks of a BF16x3 square differ from the
    # mirrored upper ones by the FP32 accumulation rounding
    assert gsum[0] == pytest.approx(ssum[0], rel=1e-12 if prec == "fp64" else 1e-9)
    assert gsum[1] == pytest.approx(ssum[1], rel=1e-13) and gsum[2] == pytest.approx(ssum[2], rel=1e-13)
    M = upper_mask(X) | upper_mask(X).T
    Mi = M.astype(np.int64)
    assert gsum[3] == 2.0 * 64 ** 3 * int((Mi @ Mi).sum())
    assert gsum[3] == 2 * ssum[3] - 2.0 * 64 ** 3 * int(np.trace(Mi @ Mi))


def test_general_product_degenerate(gpu_lib):
    """Disjoint K sets (an empty product), a product into one ragged block,
    the identity as right operand, and invalid inputs."""
    sp2 = gpu_lib
    n = 300
    nbr = (n + 63) // 64
    # A only in block column 0, B only in block rows 1..: no K matches
    Ah = random_general_bsr(n, 1.0, seed=1)
    keep = Ah.col_idx == 0
    rp = np.concatenate([[0], np.cumsum(np.bincount(Ah.rows()[keep], minlength=nbr))])
    Ah0 = type(Ah)(n, rp, Ah.col_idx[keep], Ah.val[keep])
    Bh = random_general_bsr(n, 1.0, seed=2)
    keepb = Bh.rows() != 0
    rpb = np.concatenate([[0], np.cumsum(np.bincount(Bh.rows()[keepb], minlength=nbr))])
    Bh1 = type(Bh)(n, rpb, Bh.col_idx[keepb], Bh.val[keepb])
    out, sums = sp2.general_product(sp2.BsrMatrix.from_host(Ah0), sp2.BsrMatrix.from_host(Bh1))
    assert out.nnzb == 0 and sums[3] == 0.0
    # with a != 0 the diagonal is present: out = a I
    out, sums = sp2.general_product(sp2.BsrMatrix.from_host(Ah0), sp2.BsrMatrix.from_host(Bh1), a=2.0)
    assert np.array_equal(to_dense_general(out), 2.0 * np.eye(n))
    # one ragged block (n < 64)
    Ah = random_general_bsr(40, 1.0, seed=3)
    Bh = random_general_bsr(40, 1.0, seed=4)
    out, _ = sp2.general_product(sp2.BsrMatrix.from_host(Ah), sp2.BsrMatrix.from_host(Bh))
    ref = general_bsr_to_dense(Ah) @ general_bsr_to_dense(Bh)
    assert np.allclose(to_dense_general(out), ref, rtol=0, atol=1e-13 * np.abs(ref).max())
    # A times the identity (in general storage) is A on A's pattern
    Ah = random_general_bsr(n, 0.5, seed=5)
    Ih = random_general_bsr(n, 0.0, seed=0, keep_diag=True)
    iv = np.broadcast_to(np.eye(64), Ih.val.shape).copy()
    iv[-1, n - 64 * (nbr - 1):, :] = 0.0  # zero rows and columns past n
    Ih = Ih.with_values(iv)
    out, _ = sp2.general_product(sp2.BsrMatrix.from_host(Ah), sp2.BsrMatrix.from_host(Ih))
    assert np.array_equal(general_mask(out), general_block_mask(Ah))
    assert np.array_equal(to_dense_general(out), general_bsr_to_dense(Ah))
    # invalid: FP32 arithmetic, sizes that differ, a lower block given to the
    # symmetric square
    A = sp2.BsrMatrix.from_host(Ah)
    with pytest.raises(RuntimeError, match="precision"):
        sp2.general_product(A, A, precision="fp32")
    with pytest.raises(RuntimeError, match="differ"):
        sp2.general_product(A, sp2.BsrMatrix.from_host(random_general_bsr(n + 64, 0.5, seed=6)))
    with pytest.raises(RuntimeError, match="row <= col"):
        sp2.square_step(A, 0.0, 0.0, 1.0)
