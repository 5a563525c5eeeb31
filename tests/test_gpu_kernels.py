"""GPU parity of the single steps of the hot path against the oracle, through
the C ABI: symbolic + numeric square with the fused update and reductions,
truncation, Gershgorin bounds."""
import math

import numpy as np
import pytest

from fockgen import BSR, bsr_to_dense, lattice_fock, random_sym_bsr
from oracle import sp2_oracle as O

from gpu_helpers import rel, to_dense, upper_mask

pytestmark = pytest.mark.gpu

CASES = [  # (n, density, seed)
    (64, 1.0, 0),
    (200, 1.0, 1),      # ragged: 4 block rows, last one 8 rows
    (1000, 0.35, 2),    # 16 block rows, ragged, sparse pattern
    (1500, 0.12, 3),    # very sparse
]


def _oracle_square(X, n, a, b, c):
    """a I + b X + c X^2 restricted to the block pattern of X^2 (plain dense)."""
    Xd = bsr_to_dense(X)
    S = Xd @ Xd
    M = O.structural_mask(Xd, 64) | np.eye(X.nbr, dtype=bool)
    # the stored pattern, including exactly-zero stored blocks
    Mst = np.zeros((X.nbr, X.nbr), dtype=bool)
    Mst[X.rows(), X.col_idx] = True
    Mst = Mst | Mst.T
    MS = O.pattern_square(Mst)
    out = a * np.eye(n) + b * Xd + c * S
    out = out * O.expand_mask(MS, n, 64)
    return Xd, S, out, MS, Mst


@pytest.mark.parametrize("n,dens,seed", CASES)
def test_square_step_fp64(gpu_lib, n, dens, seed):
    sp2 = gpu_lib
    Xh = random_sym_bsr(n, dens, seed=seed, std=0.1)
    a, b, c = 0.3, -0.7, 1.3
    X = sp2.BsrMatrix.from_host(Xh)
    Y, sums = sp2.square_step(X, a, b, c, "fp64")
    Xd, S, ref, MS, Mst = _oracle_square(Xh, n, a, b, c)
    # output pattern is exactly the block pattern of X^2 (upper)
    assert np.array_equal(upper_mask(Y), np.triu(MS))
    Yd = to_dense(Y)
    assert rel(Yd, ref) <= 1e-13
    e2 = float(np.sum((Xd - S) ** 2))
    assert sums[0] == pytest.approx(e2, rel=1e-12)
    assert sums[1] == pytest.approx(np.trace(Xd), rel=1e-12, abs=1e-12)
    assert sums[2] == pytest.approx(np.trace(S), rel=1e-12)
    assert sums[3] == 2.0 * 64 ** 3 * O._triples_upper(Mst)


@pytest.mark.parametrize("n,dens,seed", CASES[1:3])
def test_square_step_fp32(gpu_lib, n, dens, seed):
    sp2 = gpu_lib
    Xh = random_sym_bsr(n, dens, seed=seed, std=0.1)
    X = sp2.BsrMatrix.from_host(Xh)
    Y, sums = sp2.square_step(X, 0.0, 2.0, -1.0, "fp32")
    Xd, S, ref, MS, Mst = _oracle_square(Xh, n, 0.0, 2.0, -1.0)
    assert np.array_equal(upper_mask(Y), np.triu(MS))
    # FP32 inputs and products (unit roundoff 2^-24), accumulated over <= n terms
    Xa = np.abs(Xd)
    bound = 4 * 2.0 ** -24 * (2 * Xa + (n + 2) * (Xa @ Xa)) + 1e-30
    assert np.all(np.abs(to_dense(Y) - ref) <= bound)


def _spread_bsr(n, seed, dens=0.8):
    """Random symmetric BSR whose block norms span many decades."""
    M = random_sym_bsr(n, dens, seed=seed)
    rng = np.random.default_rng(seed + 50)
    scale = 10.0 ** rng.uniform(-7, 0, size=M.nnzb)
    I = M.rows()
    scale[I == M.col_idx] = 1.0
    return M.with_values(M.val * scale[:, None, None])


@pytest.mark.parametrize("norm,cbs", [("frob", 4096), ("frobinf", 256), ("frobinf", 128), ("frobinf", 4096)])
@pytest.mark.parametrize("tau", [1e-6, 1e-4, 1e-2])
def test_truncate_matches_oracle(gpu_lib, norm, cbs, tau):
    sp2 = gpu_lib
    Mh = _spread_bsr(1100, seed=7)
    Md = bsr_to_dense(Mh)
    mask = np.zeros((Mh.nbr, Mh.nbr), dtype=bool)
    mask[Mh.rows(), Mh.col_idx] = True
    mask = mask | mask.T
    Xt_ref, Mt_ref, info = O.truncate(Md, mask, tau, norm, 64, cbs)
    Xt, err = sp2.truncate(sp2.BsrMatrix.from_host(Mh), tau, norm, cbs)
    got = upper_mask(Xt)
    assert np.array_equal(got, np.triu(Mt_ref)), "removed block sets differ"
    assert info.removed > 0 or tau == 1e-6
    assert err[0] == pytest.approx(info.err_frob, rel=1e-12, abs=1e-300)
    assert err[1] == pytest.approx(info.err_mixed, rel=1e-12, abs=1e-300)
    assert np.array_equal(to_dense(Xt), Xt_ref)


@pytest.mark.parametrize("norm,cbs", [("frob", 4096), ("frobinf", 4096)])
@pytest.mark.parametrize("tau", [1e-2, 1e-1])
def test_truncate_long_segments_match_oracle(gpu_lib, norm, cbs, tau):
    """Segments with more candidates than one gather round of the selection
    (256): over a thousand upper blocks in one segment, the budget running
    out after the first round; same removed set, error and values as the
    oracle."""
    sp2 = gpu_lib
    Mh = _spread_bsr(3300, seed=11)
    Md = bsr_to_dense(Mh)
    mask = np.zeros((Mh.nbr, Mh.nbr), dtype=bool)
    mask[Mh.rows(), Mh.col_idx] = True
    mask = mask | mask.T
    Xt_ref, Mt_ref, info = O.truncate(Md, mask, tau, norm, 64, cbs)
    assert Mh.nnzb > 1000 and info.removed > 256
    Xt, err = sp2.truncate(sp2.BsrMatrix.from_host(Mh), tau, norm, cbs)
    assert np.array_equal(upper_mask(Xt), np.triu(Mt_ref)), "removed block sets differ"
    assert err[0] == pytest.approx(info.err_frob, rel=1e-12, abs=1e-300)
    assert err[1] == pytest.approx(info.err_mixed, rel=1e-12, abs=1e-300)
    assert np.array_equal(to_dense(Xt), Xt_ref)


def test_truncate_ties_in_block_order(gpu_lib):
    """Equal block norms are removed in (I, J) order."""
    sp2 = gpu_lib
    n, nbr = 256, 4
    vals, rows, cols = [], [], []
    for I in range(nbr):
        for J in range(I, nbr):
            blk = np.full((64, 64), 1e-3) if I != J else np.eye(64)
            rows.append(I)
            cols.append(J)
            vals.append(blk)
    rp = np.zeros(nbr + 1, dtype=np.int64)
    np.add.at(rp, np.array(rows) + 1, 1)
    Mh = BSR(n, np.cumsum(rp), np.array(cols, dtype=np.int32), np.array(vals))
    # each off-diagonal block: weight 2 * 4096 * 1e-6; budget fits exactly 2 of 6
    tau = math.sqrt(2 * 2 * 4096 * 1e-6) * (1 + 1e-12)
    Xt, err = sp2.truncate(sp2.BsrMatrix.from_host(Mh), tau, "frob")
    m = upper_mask(Xt)
    removed = [(I, J) for I in range(nbr) for J in range(I + 1, nbr) if not m[I, J]]
    assert removed == [(0, 1), (0, 2)]


@pytest.mark.parametrize("L", [4, 6, 8])
def test_gershgorin(gpu_lib, L):
    sp2 = gpu_lib
    Fh, _ = lattice_fock(L, seed=L)
    lo, hi = sp2.gershgorin(sp2.BsrMatrix.from_host(Fh))
    rlo, rhi = O.gershgorin_bounds(bsr_to_dense(Fh))
    assert lo == pytest.approx(rlo, rel=1e-13)
    assert hi == pytest.approx(rhi, rel=1e-13)


def test_deterministic_square(gpu_lib):
    sp2 = gpu_lib
    X = sp2.BsrMatrix.from_host(random_sym_bsr(1000, 0.5, seed=11))
    Y1, s1 = sp2.square_step(X, 0.1, 0.2, 0.3)
    Y2, s2 = sp2.square_step(X, 0.1, 0.2, 0.3)
    assert s1 == s2
    assert bool((Y1.val == Y2.val).all())


@pytest.mark.parametrize("n,dens,seed", CASES[1:3])
def test_square_step_bf16x3(gpu_lib, n, dens, seed):
    """hi*hi + hi*lo + lo*hi with x = hi + lo + d, |lo| <= 2^-8 |x|,
    |d| <= 2^-16 |x|: each product is off by at most 3 * 2^-16 |x||y|, plus FP32
    rounding of the inputs and of the accumulation."""
    sp2 = gpu_lib
    Xh = random_sym_bsr(n, dens, seed=seed, std=0.1)
    X = sp2.BsrMatrix.from_host(Xh)
    Y, sums = sp2.square_step(X, 0.0, 2.0, -1.0, "bf16x3")
    Xd, S, ref, MS, Mst = _oracle_square(Xh, n, 0.0, 2.0, -1.0)
    assert np.array_equal(upper_mask(Y), np.triu(MS))
    Xa = np.abs(Xd)
    u = 2.0 ** -24
    bound = 3 * 2.0 ** -16 * (Xa @ Xa) + 4 * u * (2 * Xa + (n + 2) * (Xa @ Xa)) + 1e-30
    err = np.abs(to_dense(Y) - ref)
    assert np.all(err <= bound)
    # and it is genuinely better than a plain bf16 product (error ~2^-8)
    assert np.max(err / (Xa @ Xa + 1e-30)) < 2.0 ** -12


@pytest.mark.parametrize("cbs", [64, 128, 256, 4096])
@pytest.mark.parametrize("n,dens,seed", [(64, 1.0, 0), (1000, 0.35, 2), (1500, 0.12, 3)])
def test_matrix_norms(gpu_lib, n, dens, seed, cbs):
    """Frobenius and Frob-Inf norms of the full symmetric matrix against the
    oracle's definitions (ragged last coarse submatrix included), and the
    Frob-Inf norm bounds the spectral norm."""
    sp2 = gpu_lib
    Mh = _spread_bsr(n, seed=seed, dens=dens)
    Md = bsr_to_dense(Mh)
    f, m = sp2.matrix_norms(sp2.BsrMatrix.from_host(Mh), cbs)
    assert f == pytest.approx(O.frobenius_norm(Md), rel=1e-12)
    assert m == pytest.approx(O.frob_inf_norm(Md, cbs), rel=1e-12)
    assert O.spectral_norm_sym(Md) <= m * (1 + 1e-12)


@pytest.mark.parametrize("permute", [False, True])
def test_matrix_norms_banded(gpu_lib, permute):
    """The banded test matrices of the norm comparison, plain and permuted."""
    from fockgen import banded_sym, sparse_to_bsr

    sp2 = gpu_lib
    A = banded_sym(1500, half_bw=150, seed=4, permute=permute)
    Ad = A.toarray()
    for cbs in (128, 512):
        f, m = sp2.matrix_norms(sp2.BsrMatrix.from_host(sparse_to_bsr(A)), cbs)
        assert f == pytest.approx(O.frobenius_norm(Ad), rel=1e-12)
        assert m == pytest.approx(O.frob_inf_norm(Ad, cbs), rel=1e-12)


@pytest.mark.parametrize("n,dens,seed", [(200, 1.0, 1), (1100, 0.8, 5), (1000, 0.35, 2)])
def test_bf16x3_tile_edges_bitwise(gpu_lib, monkeypatch, n, dens, seed):
    """The 4 x 4-tile BF16x3 square (operands loaded straight to LDS) and the
    2 x 2-tile one accumulate in the same order: bit-identical results, on a
    ragged block count (18 block rows) and on a sparse pattern too."""
    sp2 = gpu_lib
    X = sp2.BsrMatrix.from_host(random_sym_bsr(n, dens, seed=seed, std=0.1))
    out = {}
    for tb in ("2", "4"):
        monkeypatch.setenv("SP2_BF16X3_TILE", tb)
        Y, sums = sp2.square_step(X, 0.1, 0.2, -0.3, "bf16x3")
        out[tb] = (to_dense(Y), sums)
    assert np.array_equal(out["2"][0], out["4"][0])
    assert out["2"][1] == out["4"][1]


@pytest.mark.parametrize("sign,anti", [(1, False), (-1, False), (-1, True)])
def test_bf16x3_tile_edges_bitwise_pair(gpu_lib, monkeypatch, sign, anti):
    """Two-operand mode (anticommutator, commutator, antisymmetric right
    operand): both tile edges give bit-identical results."""
    sp2 = gpu_lib
    n = 1100
    Xh = random_sym_bsr(n, 0.7, seed=8, std=0.1)
    Yh = random_sym_bsr(n, 0.6, seed=9, std=0.1)
    if anti:
        I = Yh.rows()
        v = Yh.val.copy()
        d = I == Yh.col_idx
        v[d] = v[d] - v[d].transpose(0, 2, 1)
        Yh = Yh.with_values(v)
    X, Y = sp2.BsrMatrix.from_host(Xh), sp2.BsrMatrix.from_host(Yh)
    out = {}
    for tb in ("2", "4"):
        monkeypatch.setenv("SP2_BF16X3_TILE", tb)
        P, sums = sp2.pair_product(X, Y, sign=sign, y_antisym=anti, precision="bf16x3")
        out[tb] = (P.val.cpu().numpy(), P.col_idx.cpu().numpy(), sums)
    assert np.array_equal(out["2"][1], out["4"][1])
    assert np.array_equal(out["2"][0], out["4"][0])
    assert out["2"][2] == out["4"][2]


@pytest.mark.parametrize("n,dens,seed", [(30, 1.0, 7), (64, 1.0, 8), (100, 1.0, 9), (130, 1.0, 10),
                                         (200, 1.0, 1), (1050, 1.0, 4), (1150, 0.3, 5), (2000, 0.08, 6)])
def test_f64_lds_kernel_bitwise(gpu_lib, monkeypatch, n, dens, seed):
    """The FP64 square with operands loaded straight to LDS and the
    register-staged one accumulate in the same order: bit-identical squares and
    sums, from one partial block up (1, 1, 2, 3 block rows), on ragged block
    counts (4, 17, 18, 32 block rows; 17 leaves tiles
    with an absent second row / column) and on sparse patterns."""
    sp2 = gpu_lib
    X = sp2.BsrMatrix.from_host(random_sym_bsr(n, dens, seed=seed, std=0.1))
    out = {}
    for k in ("tile", "lds"):
        if k == "tile":
            monkeypatch.setenv("SP2_F64_KERNEL", "tile")
        else:
            monkeypatch.delenv("SP2_F64_KERNEL", raising=False)
        Y, sums = sp2.square_step(X, 0.1, 0.2, -0.3, "fp64")
        out[k] = (Y.val.cpu().numpy(), Y.col_idx.cpu().numpy(), sums)
    assert np.array_equal(out["tile"][1], out["lds"][1])
    assert np.array_equal(out["tile"][0].view(np.uint64), out["lds"][0].view(np.uint64))
    assert out["tile"][2] == out["lds"][2]


@pytest.mark.parametrize("sign,anti,with_g", [(1, False, False), (-1, False, False), (-1, True, False),
                                              (1, False, True), (-1, True, True)])
def test_f64_lds_kernel_bitwise_pair(gpu_lib, monkeypatch, sign, anti, with_g):
    """Two-operand mode of the FP64 LDS-loaded kernel (anticommutator,
    commutator, antisymmetric right operand, a I + b G term): bit-identical to
    the register-staged kernel, on a ragged block count (18 block rows) with
    two sparse patterns."""
    sp2 = gpu_lib
    n = 1100
    Xh = random_sym_bsr(n, 0.7, seed=8, std=0.1)
    Yh = random_sym_bsr(n, 0.6, seed=9, std=0.1)
    if anti:
        I = Yh.rows()
        v = Yh.val.copy()
        d = I == Yh.col_idx
        v[d] = v[d] - v[d].transpose(0, 2, 1)
        Yh = Yh.with_values(v)
    X, Y = sp2.BsrMatrix.from_host(Xh), sp2.BsrMatrix.from_host(Yh)
    G = X if with_g else None
    coef = dict(a=0.3, b=-0.7, c=1.1) if with_g else {}
    out = {}
    for k in ("tile", "lds"):
        if k == "tile":
            monkeypatch.setenv("SP2_F64_KERNEL", "tile")
        else:
            monkeypatch.delenv("SP2_F64_KERNEL", raising=False)
        P, sums = sp2.pair_product(X, Y, G=G, sign=sign, y_antisym=anti, precision="fp64", **coef)
        out[k] = (P.val.cpu().numpy(), P.col_idx.cpu().numpy(), sums)
    assert np.array_equal(out["tile"][1], out["lds"][1])
    assert np.array_equal(out["tile"][0].view(np.uint64), out["lds"][0].view(np.uint64))
    assert out["tile"][2] == out["lds"][2]
