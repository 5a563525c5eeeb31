"""Pins of the oracle's occupied-subspace correction (``subspace_correction``)
against what the mathematics fixes:

* the exact projector is a fixed point (Delta = [D, [D, F]] = 0);
* the derivative of the polynomial sequence applied to Delta equals the
  closed-form first-order perturbation of the spectral projector
  (Daleckii-Krein: the occupied-virtual part divided by lambda_o - lambda_v,
  the rest zero), written out here from the eigendecomposition;
* for a projector rotated by a small angle theta away from the exact one the
  corrected result is O(theta^2) accurate: halving theta divides the error by
  at least about four (for this symmetric perturbation the measured order is
  three), while the input error is O(theta).
"""
import numpy as np
import pytest

from fockgen import dense_spectrum
from oracle import sp2_oracle as O


def _exact(F, no):
    lam, Y = np.linalg.eigh(F)
    return lam, Y, Y[:, :no] @ Y[:, :no].T


@pytest.fixture(scope="module")
def case():
    n, no = 192, 96
    F, lam, _ = dense_spectrum(n, seed=5)
    r = O.sp2(F, no, -1.0, 1.0, -0.1, 0.1, accel=True, trunc_norm=O.TRUNC_NONE, idem_stop=1e-14, keep_tape=True)
    return F, no, r


def _rotated(Dst, theta, seed):
    """U Dst U^T with the orthogonal Cayley transform U of theta * A, A antisymmetric."""
    n = Dst.shape[0]
    A = np.random.default_rng(seed).normal(size=(n, n))
    A = (A - A.T) / np.linalg.norm(A - A.T, 2)
    I = np.eye(n)
    U = np.linalg.solve(I - 0.5 * theta * A, I + 0.5 * theta * A)
    return U @ Dst @ U.T


def test_exact_projector_is_fixed_point(case):
    F, no, r = case
    _, _, Dst = _exact(F, no)
    D, info = O.subspace_correction(F, Dst, r.X[: r.n], r.p, r.alpha, r.lmin, r.lmax)
    assert info["delta_norm"] <= 1e-12
    assert np.linalg.norm(D - Dst) <= 1e-12


def test_derivative_step_is_daleckii_krein(case):
    F, no, r = case
    lam, Y, Dst = _exact(F, no)
    D1 = _rotated(Dst, 1e-4, seed=1)
    D2, info = O.subspace_correction(F, D1, r.X[: r.n], r.p, r.alpha, r.lmin, r.lmax, purify=0)
    dD = D2 - D1
    Delta = D1 @ (D1 @ F - F @ D1) - (D1 @ F - F @ D1) @ D1
    # closed form: (Y^T Delta Y)_ov / (lam_o - lam_v) on the occupied-virtual blocks
    G = Y.T @ Delta @ Y
    K = np.zeros_like(G)
    K[:no, no:] = G[:no, no:] / (lam[:no, None] - lam[None, no:])
    K[no:, :no] = K[:no, no:].T
    ref = Y @ K @ Y.T
    assert np.linalg.norm(dD - ref) <= 1e-9 * np.linalg.norm(ref)
    assert info["step_norm"] == pytest.approx(np.linalg.norm(ref), rel=1e-9)


def test_rotated_projector_second_order(case):
    F, no, r = case
    _, _, Dst = _exact(F, no)
    errs, ins = [], []
    for theta in (2e-3, 1e-3, 5e-4):
        D1 = _rotated(Dst, theta, seed=3)
        D, _ = O.subspace_correction(F, D1, r.X[: r.n], r.p, r.alpha, r.lmin, r.lmax)
        ins.append(np.linalg.norm(D1 - Dst))
        errs.append(np.linalg.norm(D - Dst))
    for k in range(2):
        assert 1.8 <= ins[k] / ins[k + 1] <= 2.2          # input error O(theta)
        assert errs[k] / errs[k + 1] >= 3.0               # corrected error O(theta^2) (or better)
    assert errs[0] <= 1e-2 * ins[0]
    # idempotency and trace restored by the purification
    assert np.linalg.norm(D @ D - D) <= 1e-10
    assert abs(np.trace(D) - no) <= 1e-10


def test_block_dropping_budget(case):
    """With a drop budget the correction is still close to the exact projector."""
    F, no, r = case
    _, _, Dst = _exact(F, no)
    D1 = _rotated(Dst, 1e-3, seed=4)
    D, _ = O.subspace_correction(F, D1, r.X[: r.n], r.p, r.alpha, r.lmin, r.lmax, beta=1e-8)
    assert np.linalg.norm(D - Dst) <= 1e-2 * np.linalg.norm(D1 - Dst)


def test_mcweeny_purification_closed_form():
    """One McWeeny purification step maps every eigenvalue x of a symmetric P
    to 3x^2 - 2x^3 and keeps the eigenvectors: with Delta = 0 (P commutes with
    F) the correction reduces to that step, checked against the spectral
    formula on P = Q diag(x) Q^T."""
    n = 128
    rng = np.random.default_rng(11)
    Q, R = np.linalg.qr(rng.standard_normal((n, n)))
    Q = Q * np.sign(np.diag(R))
    x = np.concatenate([1.0 - rng.uniform(0, 0.05, n // 2), rng.uniform(0, 0.05, n - n // 2)])
    lam = np.where(x > 0.5, -1.0, 1.0) * np.linspace(0.2, 1.0, n)
    F = (Q * lam) @ Q.T
    F = 0.5 * (F + F.T)
    P = (Q * x) @ Q.T
    P = 0.5 * (P + P.T)
    D, _ = O.subspace_correction(F, P, [], [-1], [1.0], -1.0, 1.0, purify=1, purify_form="mcweeny")
    want = (Q * (3 * x ** 2 - 2 * x ** 3)) @ Q.T
    assert np.linalg.norm(D - want) <= 1e-13 * np.sqrt(n)
    # the SP2 pair x^2 then 2x - x^2 is a different polynomial (x^2 (2 - x^2))
    D2, _ = O.subspace_correction(F, P, [], [-1], [1.0], -1.0, 1.0, purify=2)
    assert np.linalg.norm(D2 - (Q * (x ** 2 * (2 - x ** 2))) @ Q.T) <= 1e-13 * np.sqrt(n)
