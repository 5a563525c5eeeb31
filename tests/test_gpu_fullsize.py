"""Parity at the full size of the 20 x 20 x 20 x 4 lattice workload (N = 32,000,
500 block rows), in the launch configuration bench.py times:

* one square of a dense-ish random symmetric matrix of that size: sampled
  output blocks recomputed one by one on the CPU (sum over K of X_IK X_KJ,
  written out here), plus e^2 and the traces against the whole matrix;
* the FP64 expansion on the lattice Fock matrix: properties that hold at any
  size -- trace n_occ, idempotency of sampled blocks within the reported
  ||D - D^2||_F, commutation with F on sampled blocks, the stopping criterion,
  the reported error bound.
"""
import numpy as np
import pytest

from fockgen import BSR, lattice_fock, random_sym_bsr

from gpu_helpers import upper_mask

pytestmark = pytest.mark.gpu


def _blocks(M):
    """dict (I, J) -> block (upper) of a host BSR."""
    n, rp, ci, v = M
    rows = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
    return {(int(i), int(j)): v[k] for k, (i, j) in enumerate(zip(rows, ci))}


def _get(blk, I, J):
    if I <= J:
        return blk.get((I, J))
    b = blk.get((J, I))
    return None if b is None else b.T


@pytest.fixture(scope="module")
def big_random():
    n = 32000
    Xh = random_sym_bsr(n, 0.25, seed=21, std=0.05)
    return n, Xh


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_square_full_size_sampled_blocks(gpu_lib, big_random, prec):
    sp2 = gpu_lib
    n, Xh = big_random
    nbr = Xh.nbr
    X = sp2.BsrMatrix.from_host(Xh)
    a, b, c = 0.0, 2.0, -1.0
    Y, sums = sp2.square_step(X, a, b, c, prec)
    xb = _blocks((Xh.n, Xh.row_ptr, Xh.col_idx, Xh.val))
    yb = _blocks(Y.to_host())
    rng = np.random.default_rng(3)
    samples = [(0, 0), (nbr - 1, nbr - 1), (0, nbr - 1)]
    samples += [tuple(sorted(rng.integers(0, nbr, 2))) for _ in range(12)]
    u = 2.0 ** -24
    for I, J in samples:
        S = np.zeros((64, 64))
        A = np.zeros((64, 64))
        for K in range(nbr):
            x1, x2 = _get(xb, I, K), _get(xb, K, J)
            if x1 is not None and x2 is not None:
                S += x1 @ x2
                A += np.abs(x1) @ np.abs(x2)
        xij = _get(xb, I, J)
        ref = b * (xij if xij is not None else 0.0) + c * S
        got = yb.get((I, J))
        if got is None:
            assert not A.any()
            continue
        if prec == "fp64":
            assert np.max(np.abs(got - ref)) <= 1e-12 * max(np.max(np.abs(ref)), 1e-300) + 1e-13 * np.max(A)
        else:
            xa = np.abs(xij) if xij is not None else 0.0
            bound = 3 * 2.0 ** -16 * A + 4 * u * (2 * xa + (nbr * 64 + 2) * A) + 1e-30
            assert np.all(np.abs(got - ref) <= bound)
    if prec == "fp64":
        # whole-matrix traces: tr X and tr X^2 = ||X||_F^2 (X symmetric)
        trX = sum(np.trace(v) for (i, j), v in xb.items() if i == j)
        fro2 = sum((1.0 if i == j else 2.0) * np.sum(v * v) for (i, j), v in xb.items())
        assert sums[1] == pytest.approx(trX, rel=1e-12, abs=1e-9)
        assert sums[2] == pytest.approx(fro2, rel=1e-12)


def test_lattice20_fp64_expansion_properties(gpu_lib):
    sp2 = gpu_lib
    Fh, info = lattice_fock(20, seed=0)
    no = info["n_occ"]
    F = sp2.BsrMatrix.from_host(Fh)
    lmin, lmax = sp2.gershgorin(F)
    r = sp2.density(F, no, lmin, lmax, -0.22567309855547694, 0.2265131434679548, trunc_norm="frobinf",
                    tau_fixed=1e-6, coarse_bs=4096)
    assert r.status == 0 and r.stop_reason == "criterion"
    assert r.iters["e"][-1] <= 1e-5
    n, rp, ci, v = r.D.to_host()
    db = _blocks((n, rp, ci, v))
    fb = _blocks((Fh.n, Fh.row_ptr, Fh.col_idx, Fh.val))
    nbr = Fh.nbr
    tr = sum(np.trace(b) for (i, j), b in db.items() if i == j)
    assert abs(tr - no) <= 1e-6
    # sampled blocks (I, J): (D^2 - D)_IJ is bounded by the whole-matrix
    # ||D - D^2||_F = e_n the library reports; [F, D]_IJ at the level of the
    # truncation tolerance
    nbrs = {}
    for (i, j) in db:
        nbrs.setdefault(i, set()).add(j)
        nbrs.setdefault(j, set()).add(i)
    fn = {}
    for (i, j) in fb:
        fn.setdefault(i, set()).add(j)
        fn.setdefault(j, set()).add(i)
    rng = np.random.default_rng(5)
    rows = [0, nbr // 2, nbr - 1] + [int(x) for x in rng.integers(0, nbr, 3)]
    e_n = float(r.iters["e"][-1])
    worst_idem = worst_comm = 0.0
    for I in rows:
        cols = sorted(set([I, max(I - 1, 0), min(I + 1, nbr - 1)] + [int(x) for x in rng.integers(0, nbr, 17)]))
        for J in cols:
            D2 = np.zeros((64, 64))
            for K in nbrs.get(I, ()):
                dkj = _get(db, K, J)
                if dkj is not None:
                    D2 += _get(db, I, K) @ dkj
            dij = _get(db, I, J)
            worst_idem = max(worst_idem, np.linalg.norm(D2 - (dij if dij is not None else 0.0)))
            FD = np.zeros((64, 64))
            DF = np.zeros((64, 64))
            for K in fn.get(I, ()):
                dkj = _get(db, K, J)
                if dkj is not None:
                    FD += _get(fb, I, K) @ dkj
            for K in nbrs.get(I, ()):
                fkj = _get(fb, K, J)
                if fkj is not None:
                    DF += _get(db, I, K) @ fkj
            worst_comm = max(worst_comm, np.linalg.norm(FD - DF))
    print(f"e_n = {e_n:.3e}, sampled max ||(D^2 - D)_IJ|| = {worst_idem:.3e}, ||[F, D]_IJ|| = {worst_comm:.3e}")
    assert worst_idem <= e_n * (1 + 1e-6) + 1e-12
    assert worst_comm <= 1e-4
    assert np.isfinite(r.subspace_err_bound) and r.subspace_err_bound > 0
