"""End-to-end parity against the oracle on the 12 x 12 x 12 x 4 lattice
(N = 6912) with the benchmark's options: SP2ACC, tau = 1e-6, Frob-Inf
truncation with 4096-row submatrices, Gershgorin bounds.  This size reaches
the paths the smaller parity cases do not: 108 block rows (the K scan over
four bitmap words), two coarse block rows of the Frob-Inf budget, and output
patterns dense enough for the 4 x 4-tile BF16x3 kernel.

* FP64 meets the FP64 parity bar (same n, p_i, alpha_i, masks; e_i and t_i to
  1e-10; D to 1e-9 relative; homo/lumo to 1e-9).
* The low-precision expansions with the subspace correction land within
  1e-5 of the oracle's D.
* Without the correction (FP64 tail from e_i < 1e-3) the error is held to a
  bound twice the measured one.
"""
import numpy as np
import pytest

from fockgen import bsr_to_dense, lattice_fock
from oracle import sp2_oracle as O

from gpu_helpers import rel, to_dense, upper_mask

pytestmark = pytest.mark.gpu

KW = dict(accel=True, trunc_norm="frobinf", tau_fixed=1e-6, coarse_bs=4096)


@pytest.fixture(scope="module")
def l12():
    Fh, info = lattice_fock(12, seed=0)
    Fd = bsr_to_dense(Fh)
    no = info["n_occ"]
    lam = np.linalg.eigvalsh(Fd)
    gap = lam[no] - lam[no - 1]
    h, lu = lam[no - 1] + 0.01 * gap, lam[no] - 0.01 * gap
    lmin, lmax = O.gershgorin_bounds(Fd)
    ref = O.sp2(Fd, no, lmin, lmax, h, lu, **KW)
    print(f"oracle: n={ref.n} ({ref.stop_reason}) nnzb {ref.nnzb[0]} .. {max(ref.nnzb)} of "
          f"{Fh.nbr * (Fh.nbr + 1) // 2}")
    return Fh, no, lmin, lmax, h, lu, ref


def test_l12_reaches_the_large_paths(l12):
    Fh, no, lmin, lmax, h, lu, ref = l12
    assert Fh.nbr == 108 and (Fh.nbr + 31) // 32 == 4  # four bitmap words per block row
    assert (Fh.nbr * 64 + 4095) // 4096 == 2            # two coarse block rows
    assert max(ref.nnzb) >= 0.35 * Fh.nbr * (Fh.nbr + 1) / 2  # 4 x 4 BF16x3 tiles
    assert sum(t.removed for t in ref.trunc) > 0


def test_fp64_matches_oracle_l12(gpu_lib, l12):
    sp2 = gpu_lib
    Fh, no, lmin, lmax, h, lu, ref = l12
    r = sp2.density(sp2.BsrMatrix.from_host(Fh), no, lmin, lmax, h, lu, **KW)
    N = ref.D.shape[0]
    e_gpu, e_ref = r.iters["e"], np.array(ref.e)
    print(f"n={r.n_iter}/{ref.n}, max|de|={np.max(np.abs(e_gpu - e_ref)):.3e}, "
          f"||D - D_or||/||D_or|| = {rel(to_dense(r.D), ref.D):.3e}")
    assert r.n_iter == ref.n and r.stop_reason == ref.stop_reason and r.status == ref.status
    assert list(r.iters["p"][1:]) == list(ref.p[1:])
    assert np.array_equal(r.iters["alpha"], np.array(ref.alpha))
    assert np.allclose(e_gpu, e_ref, rtol=1e-10, atol=1e-12 * np.sqrt(N))
    assert np.allclose(r.iters["t"], ref.t, rtol=1e-10, atol=1e-12 * np.sqrt(N))
    assert list(r.iters["nnzb"]) == list(ref.nnzb)
    assert np.allclose(r.iters["trunc_err_mixed"], [t.err_mixed for t in ref.trunc], rtol=1e-9, atol=1e-300)
    assert np.array_equal(upper_mask(r.D), np.triu(ref.mask))
    assert rel(to_dense(r.D), ref.D) <= 1e-9
    assert r.homo_est == pytest.approx(ref.homo_ub_est, abs=1e-9)
    assert r.lumo_est == pytest.approx(ref.lumo_lb_est, abs=1e-9)


@pytest.mark.parametrize("prec,mcweeny,fast", [("bf16x3", 1, False), ("bf16x3", 0, False), ("fp32", 1, False),
                                               ("bf16x3", 1, True)])
def test_corrected_low_precision_matches_oracle_l12(gpu_lib, l12, prec, mcweeny, fast):
    """fast: the benchmark's settings (the expansion stops at its noise floor,
    derivative steps stop at e_k < 0.2, the correction's intermediates are
    truncated within a Frobenius budget of 3e-7 each)."""
    sp2 = gpu_lib
    Fh, no, lmin, lmax, h, lu, ref = l12
    extra = dict(low_floor_stop=1, corr_deriv_tol=0.2, corr_tol=3e-7) if fast else {}
    r = sp2.density(sp2.BsrMatrix.from_host(Fh), no, lmin, lmax, h, lu, precision=prec, switch_tol=0.0,
                    correct=1, corr_mcweeny=mcweeny, corr_purify=1 if mcweeny else 2, **extra, **KW)
    D = to_dense(r.D)
    err = np.linalg.norm(D - ref.D)
    print(f"{prec} + correction (mcweeny={mcweeny}, fast={fast}): ||D - D_oracle||_F = {err:.3e}, status "
          f"{r.status} ({r.stop_reason}), n={r.n_iter}, {r.correction}")
    assert r.status == 0
    if fast:  # the first e_i below ten times the BF16x3 rounding noise ends the expansion
        assert r.stop_reason == "noise_floor"
        nu = 1.6e-5 * np.sqrt(r.iters["trace"][-1])
        assert r.iters["e"][-1] < 10 * nu and all(r.iters["e"][2:-1] >= 10 * 1.6e-5 * np.sqrt(
            np.maximum(r.iters["trace"][2:-1], 1.0)))
    assert err <= 1e-5
    if fast:
        # one McWeeny step maps an eigenvalue's distance d from {0, 1} to
        # 3 d^2 - 2 d^3, and sum d^2 ~ e^2 with e = ||P - P^2||_F of its input:
        # |tr D - n_occ| <= 3 e^2 (the expansion stopped earlier, e is larger)
        e = r.correction["corr_e_last"]
        assert abs(np.trace(D) - no) <= 3.3 * e * e + 1e-9
    else:
        assert abs(np.trace(D) - no) <= 1e-6


# measured ||D - D_oracle||_F of the FP64-tail runs (the bound is twice that)
TAIL_ERR = {"fp32": 1.6e-4, "bf16x3": 1.2e-3}


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_fp64_tail_error_bound_l12(gpu_lib, l12, prec):
    sp2 = gpu_lib
    Fh, no, lmin, lmax, h, lu, ref = l12
    r = sp2.density(sp2.BsrMatrix.from_host(Fh), no, lmin, lmax, h, lu, precision=prec, switch_tol=1e-3, **KW)
    D = to_dense(r.D)
    err = np.linalg.norm(D - ref.D)
    print(f"{prec} + FP64 tail: ||D - D_oracle||_F = {err:.3e}, switch {r.switch_iter}, n={r.n_iter}, "
          f"status {r.status} ({r.stop_reason})")
    assert r.switch_iter >= 1
    assert err <= 2 * TAIL_ERR[prec]
    assert abs(np.trace(D) - no) <= 1e-6
