"""GPU checks of the occupied-subspace correction (sp2_options.correct):

* FP64 expansion + correction equals the oracle's FP64 expansion followed by
  the oracle's ``subspace_correction`` with the same drop budget, block for
  block;
* low-precision expansions (FP32, BF16x3) with the correction reach the exact
  projector from diagonalisation far more closely than without it, and the
  truncated low-precision run lands within 1e-5 of the truncated FP64 run.
"""
import numpy as np
import pytest

from fockgen import bsr_to_dense, dense_spectrum, dense_to_bsr, lattice_fock
from oracle import sp2_oracle as O

from gpu_helpers import rel, to_dense, upper_mask

pytestmark = pytest.mark.gpu


def _exact(F, no):
    lam, Y = np.linalg.eigh(F)
    return lam, Y[:, :no] @ Y[:, :no].T


def test_fp64_correction_matches_oracle(gpu_lib):
    sp2 = gpu_lib
    Fh, info = lattice_fock(6, seed=0)
    Fd = bsr_to_dense(Fh)
    no = info["n_occ"]
    lmin, lmax = O.gershgorin_bounds(Fd)
    kw = dict(accel=True, trunc_norm="frobinf", tau_fixed=1e-4, coarse_bs=128)
    ref = O.sp2(Fd, no, lmin, lmax, -0.37, 0.34, keep_tape=True, **kw)
    Dref, inf = O.subspace_correction(Fd, ref.D, ref.X[: ref.n], ref.p, ref.alpha, lmin, lmax, beta=1e-9,
                                      tau_purify=ref.tau[ref.n], trunc_norm="frobinf", coarse_bs=128)
    # corr_deriv_tol 1e-300: every derivative step, as the oracle takes them
    r = sp2.density(sp2.BsrMatrix.from_host(Fh), no, lmin, lmax, -0.37, 0.34, correct=1, corr_tol=1e-9,
                    corr_deriv_tol=1e-300, **kw)
    assert r.n_iter == ref.n
    assert r.correction["corr_rounds"] == 1
    D = to_dense(r.D)
    assert np.array_equal(upper_mask(r.D), np.triu(O.structural_mask(Dref, 64) | np.eye(Fh.nbr, dtype=bool)))
    assert np.max(np.abs(D - Dref)) <= 1e-10
    assert r.correction["corr_delta_norm"] == pytest.approx(inf["delta_norm"], rel=1e-8)
    assert r.correction["corr_step_norm"] == pytest.approx(inf["step_norm"], rel=1e-8)


@pytest.mark.parametrize("prec,rounds,tol", [("fp32", 1, 1e-8), ("bf16x3", 2, 2e-6)])
def test_low_precision_dense_corrected(gpu_lib, prec, rounds, tol):
    """Dense N = 512 (Haar eigenvectors, gap 0.2), no truncation.  The
    derivative is taken along the low-precision iterates, so one round leaves
    a relative error of the order of their noise (~1e-2 for BF16x3, whose
    iterates end at e ~ 1e-3); a second round removes most of the rest."""
    sp2 = gpu_lib
    Fd, lam, _ = dense_spectrum(512, seed=0)
    _, Dst = _exact(Fd, 256)
    F = sp2.BsrMatrix.from_host(dense_to_bsr(Fd))
    kw = dict(trunc_norm="none", precision=prec, switch_tol=0.0)
    plain = sp2.density(F, 256, -1.0, 1.0, -0.1, 0.1, precision=prec, trunc_norm="none")
    r = sp2.density(F, 256, -1.0, 1.0, -0.1, 0.1, correct=rounds, **kw)
    e_plain = np.linalg.norm(to_dense(plain.D) - Dst)
    D = to_dense(r.D)
    e_corr = np.linalg.norm(D - Dst)
    print(f"{prec}: ||D - D*||_F without correction {e_plain:.3e}, with {e_corr:.3e}; "
          f"n = {r.n_iter}, switch {r.switch_iter}, {r.correction}")
    assert r.switch_iter == -1  # the expansion stayed in the low precision
    assert set(r.iters["precision"]) == {1 if prec == "fp32" else 2}
    assert e_corr <= tol
    assert e_corr <= 1e-2 * e_plain
    assert np.linalg.norm(D @ D - D) <= 1e-6
    assert abs(np.trace(D) - 256) <= 1e-6


@pytest.mark.parametrize("prec,rounds", [("fp32", 1), ("bf16x3", 2)])
def test_low_precision_lattice_target(gpu_lib, prec, rounds):
    """Lattice 8 x 8 x 8 x 4 (N = 2048), tau = 1e-6 Frob-Inf: the corrected
    low-precision result is within 1e-5 of the FP64 expansion's result (same
    truncation), and at least as close to the exact projector."""
    sp2 = gpu_lib
    Fh, info = lattice_fock(8, seed=0)
    Fd = bsr_to_dense(Fh)
    no = info["n_occ"]
    lam, Dst = _exact(Fd, no)
    lmin, lmax = O.gershgorin_bounds(Fd)
    gap = lam[no] - lam[no - 1]
    h, lu = lam[no - 1] + 0.01 * gap, lam[no] - 0.01 * gap
    F = sp2.BsrMatrix.from_host(Fh)
    kw = dict(trunc_norm="frobinf", tau_fixed=1e-6, coarse_bs=512)
    r64 = sp2.density(F, no, lmin, lmax, h, lu, **kw)
    r = sp2.density(F, no, lmin, lmax, h, lu, precision=prec, switch_tol=0.0, correct=rounds, **kw)
    D64, D = to_dense(r64.D), to_dense(r.D)
    e_ref = np.linalg.norm(D - D64)
    e_st, e64_st = np.linalg.norm(D - Dst), np.linalg.norm(D64 - Dst)
    print(f"{prec}: ||D - D_fp64||_F = {e_ref:.3e}, ||D - D*|| = {e_st:.3e}, ||D_fp64 - D*|| = {e64_st:.3e}")
    assert e_ref <= 1e-5
    assert e_st <= e64_st + 1e-6
    assert abs(np.trace(D) - no) <= 1e-6


def test_stored_and_recomputed_iterates_give_identical_result(gpu_lib):
    """The correction's X~_1 .. X~_{n-1} kept on the device, copied to pinned
    host memory and back on the copy stream (corr_mem = 1 byte), or recomputed
    from the recorded masks and polynomials (no host memory either): the same
    D bit for bit."""
    sp2 = gpu_lib
    Fh, info = lattice_fock(6, seed=0)
    Fd = bsr_to_dense(Fh)
    no = info["n_occ"]
    lmin, lmax = O.gershgorin_bounds(Fd)
    F = sp2.BsrMatrix.from_host(Fh)
    kw = dict(trunc_norm="frobinf", tau_fixed=1e-5, coarse_bs=128, precision="bf16x3", switch_tol=0.0, correct=1)
    r1 = sp2.density(F, no, lmin, lmax, -0.37, 0.34, **kw)
    r2 = sp2.density(F, no, lmin, lmax, -0.37, 0.34, corr_mem=1, **kw)
    r3 = sp2.density(F, no, lmin, lmax, -0.37, 0.34, corr_mem=1, corr_host_mem=-1, **kw)
    c1, c2, c3 = r1.correction, r2.correction, r3.correction
    print(c1, c2, c3, sep="\n")
    assert c1["seq_host_bytes"] == 0 and c1["corr_recomputed"] == 0
    assert c2["seq_bytes"] < c1["seq_bytes"] and c2["seq_host_bytes"] > 0 and c2["corr_recomputed"] == 0
    assert c3["seq_host_bytes"] == 0 and c3["corr_recomputed"] > 0
    for r in (r2, r3):
        assert np.array_equal(upper_mask(r1.D), upper_mask(r.D))
        assert np.array_equal(to_dense(r1.D), to_dense(r.D))


def test_fp64_mcweeny_correction_matches_oracle(gpu_lib):
    """FP64 expansion + correction with one McWeeny purification
    (P' = P + R - (P R + R P), R = P^2 - P) equals the oracle's expansion +
    ``subspace_correction(purify_form="mcweeny")`` block for block."""
    sp2 = gpu_lib
    Fh, info = lattice_fock(6, seed=0)
    Fd = bsr_to_dense(Fh)
    no = info["n_occ"]
    lmin, lmax = O.gershgorin_bounds(Fd)
    kw = dict(accel=True, trunc_norm="frobinf", tau_fixed=1e-4, coarse_bs=128)
    ref = O.sp2(Fd, no, lmin, lmax, -0.37, 0.34, keep_tape=True, **kw)
    Dref, inf = O.subspace_correction(Fd, ref.D, ref.X[: ref.n], ref.p, ref.alpha, lmin, lmax, beta=1e-9,
                                      purify=1, purify_form="mcweeny", tau_purify=ref.tau[ref.n],
                                      trunc_norm="frobinf", coarse_bs=128)
    r = sp2.density(sp2.BsrMatrix.from_host(Fh), no, lmin, lmax, -0.37, 0.34, correct=1, corr_tol=1e-9,
                    corr_mcweeny=1, corr_purify=1, corr_deriv_tol=1e-300, **kw)
    D = to_dense(r.D)
    print(f"max |D - D_oracle| = {np.max(np.abs(D - Dref)):.3e}")
    assert r.n_iter == ref.n
    assert np.array_equal(upper_mask(r.D), np.triu(O.structural_mask(Dref, 64) | np.eye(Fh.nbr, dtype=bool)))
    assert np.max(np.abs(D - Dref)) <= 1e-10
    assert r.correction["corr_step_norm"] == pytest.approx(inf["step_norm"], rel=1e-8)


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_mcweeny_low_precision_lattice_target(gpu_lib, prec):
    """Lattice 8 x 8 x 8 x 4, tau = 1e-6: the low-precision expansion with the
    correction and one McWeeny purification (its cubic term in the low
    arithmetic) lands within 1e-5 of the FP64 expansion, as the two-square
    purification does."""
    sp2 = gpu_lib
    Fh, info = lattice_fock(8, seed=0)
    Fd = bsr_to_dense(Fh)
    no = info["n_occ"]
    lam, Dst = _exact(Fd, no)
    lmin, lmax = O.gershgorin_bounds(Fd)
    gap = lam[no] - lam[no - 1]
    h, lu = lam[no - 1] + 0.01 * gap, lam[no] - 0.01 * gap
    F = sp2.BsrMatrix.from_host(Fh)
    kw = dict(trunc_norm="frobinf", tau_fixed=1e-6, coarse_bs=512)
    r64 = sp2.density(F, no, lmin, lmax, h, lu, **kw)
    r = sp2.density(F, no, lmin, lmax, h, lu, precision=prec, switch_tol=0.0, correct=1, corr_mcweeny=1,
                    corr_purify=1, **kw)
    D64, D = to_dense(r64.D), to_dense(r.D)
    e_ref = np.linalg.norm(D - D64)
    print(f"{prec} + McWeeny: ||D - D_fp64||_F = {e_ref:.3e}, ||D^2 - D|| = {np.linalg.norm(D @ D - D):.3e}")
    assert e_ref <= 1e-5
    assert np.linalg.norm(D @ D - D) <= 1e-6
    assert abs(np.trace(D) - no) <= 1e-6
