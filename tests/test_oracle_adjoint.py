"""Pins of the oracle's adjoint of the discrete recursion.

* Daleckii-Krein closed form of the gradient of tr(W D) for the exact
  spectral projector (untruncated runs converge to it).
* Dot-product test <W, J dF> = <J^T W, dF>.
* Central finite differences (h = 1e-5) of the frozen forward map.
"""
import numpy as np
import pytest

from fockgen import bsr_to_dense, dense_spectrum, lattice_fock, random_sym_on_pattern
from oracle import sp2_oracle as O


def _sym(n, seed, std=1.0):
    rng = np.random.default_rng(seed)
    A = rng.normal(0, std, (n, n))
    return np.triu(A) + np.triu(A, 1).T


@pytest.fixture(scope="module")
def c0_run():
    F, lam, Y = dense_spectrum(256, seed=2)
    r = O.sp2(F, 128, -1.0, 1.0, -0.1, 0.1, accel=True, trunc_norm=O.TRUNC_NONE,
              idem_stop=1e-12, keep_tape=True)
    return F, r


def test_vjp_daleckii_krein(c0_run):
    F, r = c0_run
    W = _sym(F.shape[0], 11)
    g = O.vjp(r, F, W)
    g_dk = O.daleckii_krein_gradient(F, 128, W)
    assert O.frobenius_norm(g - g_dk) <= 1e-8 * O.frobenius_norm(g_dk)


def test_jvp_daleckii_krein(c0_run):
    F, r = c0_run
    dF = _sym(F.shape[0], 12, 1e-3)
    dD = O.jvp(r, F, dF)
    # first-order perturbation of the projector: D'(F)[dF] in the eigenbasis
    lam, Y = np.linalg.eigh(F)
    Yo, Yv = Y[:, :128], Y[:, 128:]
    C = (Yo.T @ dF @ Yv) / (lam[:128, None] - lam[None, 128:])
    ref = Yo @ C @ Yv.T
    ref = ref + ref.T
    assert O.frobenius_norm(dD - ref) <= 1e-8 * O.frobenius_norm(ref)


def test_dot_product_truncated_lattice():
    Fb, info = lattice_fock(6, seed=0)
    F = bsr_to_dense(Fb)
    no = info["n_occ"]
    lmin, lmax = O.gershgorin_bounds(F)
    r = O.sp2(F, no, lmin, lmax, -0.37, 0.34, accel=True, trunc_norm=O.TRUNC_FROBINF,
              tau_fixed=1e-2, coarse_bs=128, keep_tape=True)
    assert sum(t.removed for t in r.trunc) > 0
    W = bsr_to_dense(random_sym_on_pattern(Fb, 1.0, seed=2))
    dF = bsr_to_dense(random_sym_on_pattern(Fb, 1e-3, seed=1))
    lhs = float(np.sum(W * O.jvp(r, F, dF)))
    rhs = float(np.sum(O.vjp(r, F, W) * dF))
    assert lhs == pytest.approx(rhs, rel=1e-10)


def test_finite_differences_truncated_lattice():
    Fb, info = lattice_fock(6, seed=0)
    F = bsr_to_dense(Fb)
    no = info["n_occ"]
    lmin, lmax = O.gershgorin_bounds(F)
    r = O.sp2(F, no, lmin, lmax, -0.37, 0.34, accel=True, trunc_norm=O.TRUNC_FROBINF,
              tau_fixed=1e-2, coarse_bs=128, keep_tape=True)
    dF = bsr_to_dense(random_sym_on_pattern(Fb, 1e-3, seed=1))
    W = bsr_to_dense(random_sym_on_pattern(Fb, 1.0, seed=2))
    h = 1e-5
    Dp = O.replay(r, F + h * dF)
    Dm = O.replay(r, F - h * dF)
    fd = (Dp - Dm) / (2 * h)
    jv = O.jvp(r, F, dF)
    assert O.frobenius_norm(fd - jv) <= 1e-6 * O.frobenius_norm(jv)
    fd_l = float(np.sum(W * fd))
    assert fd_l == pytest.approx(float(np.sum(O.vjp(r, F, W) * dF)), rel=1e-6)
    # the replay at F itself reproduces the recorded forward result exactly
    assert np.array_equal(O.replay(r, F), r.D)
