"""Pins of the oracle against the definition of D and the paper's guarantees.

* D equals sum_{i<=n_occ} y_i y_i^T (section "Introduction") on untruncated
  inputs, computed by LAPACK diagonalisation (a textbook routine).
* Invariants of a spectral projector: idempotency, trace, [F, D] = 0.
* The error-control guarantee ||D - P_Xn||_2 <= gamma when the thresholds of
  eq. (tau_trunc) are used (section "Error control").
* The per-iteration e_i and t_i equal the values obtained from the eigenvalues
  of X~_i (closed form for symmetric matrices).
"""
import numpy as np
import pytest

from fockgen import bsr_to_dense, dense_spectrum, lattice_fock
from oracle import sp2_oracle as O


@pytest.fixture(scope="module")
def c0():
    F, lam, Y = dense_spectrum(512, seed=0)
    return F, lam, Y


@pytest.mark.parametrize("accel", [False, True])
def test_dense_c0_matches_diagonalization(c0, accel):
    F, lam, Y = c0
    r = O.sp2(F, 256, -1.0, 1.0, -0.1, 0.1, accel=accel, trunc_norm=O.TRUNC_NONE, idem_stop=1e-12)
    D_eig = Y[:, :256] @ Y[:, :256].T
    assert O.frobenius_norm(r.D - D_eig) <= 1e-10
    d = O.diagnostics(r.D, F, 256)
    assert d["idempotency"] <= 1e-12
    assert d["trace_err"] <= 1e-10
    assert d["commutator"] <= 1e-10 * O.frobenius_norm(F)
    # also against LAPACK on F itself (not the generator's eigenvectors)
    D2, _ = O.density_by_diagonalization(F, 256)
    assert O.frobenius_norm(r.D - D2) <= 1e-10


def test_sp2acc_needs_fewer_iterations(c0):
    F, _, _ = c0
    r0 = O.sp2(F, 256, -1.0, 1.0, -0.1, 0.1, accel=False, trunc_norm=O.TRUNC_NONE, idem_stop=1e-12)
    r1 = O.sp2(F, 256, -1.0, 1.0, -0.1, 0.1, accel=True, trunc_norm=O.TRUNC_NONE, idem_stop=1e-12)
    assert r1.n < r0.n
    # SP2 is SP2ACC with alpha_i = 1 and n_min = 1 (section "Density matrix construction")
    assert all(a == 1.0 for a in r0.alpha[1:]) and r0.sched.n_min == 1


def test_e_and_t_from_eigenvalues(c0):
    """e_i = ||X~ - X~^2||_F and t_i = tr(X~ - X~^2) equal sqrt(sum (x - x^2)^2)
    and sum (x - x^2) over the eigenvalues x of X~_i."""
    F, _, _ = c0
    r = O.sp2(F, 256, -1.0, 1.0, -0.1, 0.1, accel=True, trunc_norm=O.TRUNC_NONE,
              idem_stop=1e-12, keep_tape=True)
    for i in range(0, r.n + 1, 3):
        x = np.linalg.eigvalsh(r.X[i])
        y = x - x * x
        assert r.e[i] == pytest.approx(np.sqrt(np.sum(y * y)), rel=1e-9, abs=1e-13)
        assert r.t[i] == pytest.approx(np.sum(y), rel=1e-9, abs=1e-11)


def test_ragged_lattice_matches_diagonalization():
    """L = 6 lattice: N = 864 is not a multiple of the 64 block size."""
    Fb, info = lattice_fock(6, seed=0)
    F = bsr_to_dense(Fb)
    no = info["n_occ"]
    lmin, lmax = O.gershgorin_bounds(F)
    lam = np.linalg.eigvalsh(F)
    h = lam[no - 1] + 0.02
    lu = lam[no] - 0.02
    r = O.sp2(F, no, lmin, lmax, h, lu, accel=True, trunc_norm=O.TRUNC_NONE)
    D, _ = O.density_by_diagonalization(F, no)
    assert O.frobenius_norm(r.D - D) <= 1e-10
    assert abs(np.trace(r.D) - no) <= 1e-10


@pytest.mark.parametrize("norm,cbs", [(O.TRUNC_FROBINF, 256), (O.TRUNC_FROB, 4096)])
def test_error_control_guarantee(norm, cbs):
    """With tau_i from eq. (tau_trunc) the occupied-subspace error is at most
    gamma, and at most the bound sum ||E_i|| / (xi_i - ||E_i||)."""
    Fb, info = lattice_fock(8, seed=0)
    F = bsr_to_dense(Fb)
    no = info["n_occ"]
    lmin, lmax = O.gershgorin_bounds(F)
    lam = np.linalg.eigvalsh(F)
    gamma = 0.05
    r = O.sp2(F, no, lmin, lmax, lam[no - 1] + 0.01, lam[no] - 0.01, accel=True,
              trunc_norm=norm, gamma=gamma, coarse_bs=cbs)
    assert sum(t.removed for t in r.trunc) > 0  # truncation really acted
    D, _ = O.density_by_diagonalization(F, no)
    w, V = np.linalg.eigh(r.D)
    P = V[:, -no:] @ V[:, -no:].T
    err = O.spectral_norm_sym(D - P)
    assert err <= gamma
    assert err <= r.subspace_err_bound
    assert r.subspace_err_bound <= gamma


def test_gershgorin_contains_spectrum():
    Fb, _ = lattice_fock(6, seed=3)
    F = bsr_to_dense(Fb)
    lmin, lmax = O.gershgorin_bounds(F)
    lam = np.linalg.eigvalsh(F)
    assert lmin <= lam[0] and lam[-1] <= lmax
    # closed form: a diagonal matrix has radius 0
    d = np.array([3.0, -2.0, 0.5])
    assert O.gershgorin_bounds(np.diag(d)) == (-2.0, 3.0)
    # closed form: [[a, b], [b, a]] gives [a - |b|, a + |b|], which are the eigenvalues
    assert O.gershgorin_bounds(np.array([[1.0, -2.0], [-2.0, 1.0]])) == (-1.0, 3.0)


def test_input_validation():
    F, _, _ = dense_spectrum(64, seed=1)
    with pytest.raises(O.OracleError):
        O.sp2(F, 0, -1, 1)
    with pytest.raises(O.OracleError):
        O.sp2(F, 64, -1, 1)
    with pytest.raises(O.OracleError):
        O.sp2(F, 32, 1, -1)
    with pytest.raises(O.OracleError):
        O.sp2(F, 32, -1, 1, 0.2, 0.1)  # homo_ub >= lumo_lb
    G = F.copy()
    G[0, 1] = np.nan
    with pytest.raises(O.OracleError):
        O.sp2(G, 32, -1, 1)
