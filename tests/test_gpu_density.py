"""End-to-end GPU parity of sp2_density against the oracle through the C ABI:
same iteration count, polynomial sequence and scale-and-fold parameters,
e_i and t_i, block masks, D and homo/lumo estimates."""
import numpy as np
import pytest

from fockgen import bsr_to_dense, dense_spectrum, dense_to_bsr, lattice_fock
from oracle import sp2_oracle as O

from gpu_helpers import rel, to_dense, upper_mask

pytestmark = pytest.mark.gpu


def _compare_runs(r, ref, d_tol=1e-9):
    """FP64 parity bar: e_i and t_i agree to 1e-10 relative plus an absolute
    floor of 1e-12 sqrt(N) (round-off of X - X^2 when X is nearly idempotent);
    p_i, alpha_i, n and the masks agree exactly."""
    N = ref.D.shape[0]
    e_gpu, e_ref = r.iters["e"], np.array(ref.e)
    de = np.abs(e_gpu[: len(e_ref)] - e_ref) if len(e_gpu) == len(e_ref) else None
    print(f"n={r.n_iter}/{ref.n} max|de|={None if de is None else de.max():.3e}")
    assert r.n_iter == ref.n
    assert list(r.iters["p"][1:]) == list(ref.p[1:])
    assert np.array_equal(r.iters["alpha"], np.array(ref.alpha))
    atol = 1e-12 * np.sqrt(N)
    assert np.allclose(e_gpu, e_ref, rtol=1e-10, atol=atol)
    assert np.allclose(r.iters["t"], ref.t, rtol=1e-10, atol=atol)
    assert list(r.iters["nnzb"]) == list(ref.nnzb)
    assert np.array_equal(upper_mask(r.D), np.triu(ref.mask))
    assert rel(to_dense(r.D), ref.D) <= d_tol
    for a, b in ((r.homo_est, ref.homo_ub_est), (r.lumo_est, ref.lumo_lb_est)):
        if np.isnan(b):
            assert np.isnan(a)
        else:
            assert a == pytest.approx(b, abs=1e-9)


@pytest.mark.parametrize("accel", [False, True])
def test_dense_c0(gpu_lib, accel):
    sp2 = gpu_lib
    Fd, lam, Y = dense_spectrum(512, seed=0)
    ref = O.sp2(Fd, 256, -1.0, 1.0, -0.1, 0.1, accel=accel, trunc_norm=O.TRUNC_NONE, idem_stop=1e-12)
    F = sp2.BsrMatrix.from_host(dense_to_bsr(Fd))
    r = sp2.density(F, 256, -1.0, 1.0, -0.1, 0.1, accel=accel, trunc_norm="none", idem_stop=1e-12)
    _compare_runs(r, ref)
    D_eig = Y[:, :256] @ Y[:, :256].T
    assert np.linalg.norm(to_dense(r.D) - D_eig) <= 1e-10
    assert r.stop_reason == ref.stop_reason


@pytest.mark.parametrize("accel,hb,lb", [(False, -0.05, 0.05), (False, -0.02, 0.02), (True, -0.02, 0.02)])
def test_stop_by_criterion_before_n_max(gpu_lib, accel, hb, lb):
    """Algorithm 2's stopping test on the GPU: with loose homo/lumo bounds the
    untruncated dense run converges before n_max and the criterion, not n_max,
    ends it at the oracle's index (pinned on the CPU by the scalar eigenvalue
    iteration)."""
    sp2 = gpu_lib
    Fd, lam, Y = dense_spectrum(512, seed=0)
    ref = O.sp2(Fd, 256, -1.0, 1.0, hb, lb, accel=accel, trunc_norm=O.TRUNC_NONE)
    assert ref.stop_reason == "criterion"
    F = sp2.BsrMatrix.from_host(dense_to_bsr(Fd))
    r = sp2.density(F, 256, -1.0, 1.0, hb, lb, accel=accel, trunc_norm="none")
    print(f"accel={accel} bounds={hb},{lb}: gpu n={r.n_iter} ({r.stop_reason}) oracle n={ref.n} n_max={r.n_max}")
    assert r.stop_reason == "criterion"
    assert r.n_iter == ref.n
    if not accel:
        assert r.n_iter < r.n_max
    assert r.status == 0
    _compare_runs(r, ref)


@pytest.mark.parametrize("L,norm,tau,cbs", [
    (6, "frobinf", 1e-3, 256),
    (6, "frob", 3e-3, 4096),
    (8, "frobinf", 1e-3, 512),
    (8, "frobinf", 1e-2, 256),
])
def test_lattice_truncated(gpu_lib, L, norm, tau, cbs):
    sp2 = gpu_lib
    Fh, info = lattice_fock(L, seed=0)
    Fd = bsr_to_dense(Fh)
    no = info["n_occ"]
    lmin, lmax = O.gershgorin_bounds(Fd)
    lam = np.linalg.eigvalsh(Fd)
    h, lu = lam[no - 1] + 0.01, lam[no] - 0.01
    ref = O.sp2(Fd, no, lmin, lmax, h, lu, accel=True, trunc_norm=norm, tau_fixed=tau, coarse_bs=cbs)
    r = sp2.density(sp2.BsrMatrix.from_host(Fh), no, lmin, lmax, h, lu, accel=True, trunc_norm=norm,
                    tau_fixed=tau, coarse_bs=cbs)
    assert sum(t.removed for t in ref.trunc) > 0
    _compare_runs(r, ref)
    assert np.allclose(r.iters["trunc_err_mixed"], [t.err_mixed for t in ref.trunc], rtol=1e-9, atol=1e-300)


def test_gamma_schedule_and_bound(gpu_lib):
    sp2 = gpu_lib
    Fh, info = lattice_fock(8, seed=0)
    Fd = bsr_to_dense(Fh)
    no = info["n_occ"]
    lmin, lmax = O.gershgorin_bounds(Fd)
    ref = O.sp2(Fd, no, lmin, lmax, -0.31, 0.33, accel=True, trunc_norm="frobinf", gamma=0.05, coarse_bs=256)
    r = sp2.density(sp2.BsrMatrix.from_host(Fh), no, lmin, lmax, -0.31, 0.33, accel=True, trunc_norm="frobinf",
                    gamma=0.05, coarse_bs=256)
    _compare_runs(r, ref)
    assert np.allclose(r.iters["tau"], ref.tau, rtol=1e-15, atol=0)
    assert r.subspace_err_bound == pytest.approx(ref.subspace_err_bound, rel=1e-9)


def test_trace_correcting_two_run_protocol(gpu_lib):
    sp2 = gpu_lib
    Fh, info = lattice_fock(6, seed=0)
    Fd = bsr_to_dense(Fh)
    no = info["n_occ"]
    lmin, lmax = O.gershgorin_bounds(Fd)
    ref1 = O.sp2(Fd, no, lmin, lmax, trunc_norm="frobinf", tau_fixed=1e-3, coarse_bs=256)
    F = sp2.BsrMatrix.from_host(Fh)
    r1 = sp2.density(F, no, lmin, lmax, trunc_norm="frobinf", tau_fixed=1e-3, coarse_bs=256)
    _compare_runs(r1, ref1)
    ref2 = O.sp2(Fd, no, lmin, lmax, ref1.homo_ub_est, ref1.lumo_lb_est, trunc_norm="frobinf", tau_fixed=1e-3,
                 coarse_bs=256)
    r2 = sp2.density(F, no, lmin, lmax, ref1.homo_ub_est, ref1.lumo_lb_est, trunc_norm="frobinf", tau_fixed=1e-3,
                     coarse_bs=256)
    _compare_runs(r2, ref2)


def test_error_codes(gpu_lib):
    sp2 = gpu_lib
    Fd, lam, Y = dense_spectrum(128, seed=3)
    F = sp2.BsrMatrix.from_host(dense_to_bsr(Fd))
    with pytest.raises(sp2.Sp2Error) as e:
        sp2.density(F, 64, -1.0, 1.0, 0.2, 0.1)
    assert e.value.code == -2
    with pytest.raises(sp2.Sp2Error) as e:
        sp2.density(F, 0, -1.0, 1.0)
    assert e.value.code == -1
    with pytest.raises(sp2.Sp2Error) as e:
        sp2.density(F, 64, 1.0, -1.0)
    assert e.value.code == -1
    bad = dense_to_bsr(Fd)
    bad.val[0, 3, 5] = np.nan
    with pytest.raises(sp2.Sp2Error) as e:
        sp2.density(sp2.BsrMatrix.from_host(bad), 64, -1.0, 1.0)
    assert e.value.code == -3
    # wrong bounds: the true homo lies above the given homo_ub -> trace warning or non-convergence
    r = sp2.density(F, 64, -1.0, 1.0, lam[63] - 0.3, lam[63] - 0.25, trunc_norm="none")
    assert r.status in (1, 2)


def test_mixed_fp32_reports_error(gpu_lib):
    sp2 = gpu_lib
    Fh, info = lattice_fock(8, seed=0)
    Fd = bsr_to_dense(Fh)
    no = info["n_occ"]
    lmin, lmax = O.gershgorin_bounds(Fd)
    F = sp2.BsrMatrix.from_host(Fh)
    r64 = sp2.density(F, no, lmin, lmax, -0.31, 0.33, trunc_norm="frobinf", tau_fixed=1e-6, coarse_bs=512)
    r32 = sp2.density(F, no, lmin, lmax, -0.31, 0.33, trunc_norm="frobinf", tau_fixed=1e-6, coarse_bs=512,
                      precision="fp32")
    assert r32.switch_iter >= 1
    assert set(r32.iters["precision"][: r32.switch_iter]) == {1}
    assert set(r32.iters["precision"][r32.switch_iter:]) == {0}
    D64, D32 = to_dense(r64.D), to_dense(r32.D)
    err = np.linalg.norm(D32 - D64)
    print(f"mixed fp32 vs fp64: ||dD||_F = {err:.3e}, n = {r32.n_iter} vs {r64.n_iter}")
    assert err <= 1e-3
    assert abs(np.trace(D32) - no) <= 1e-6


def test_mixed_bf16x3_reports_error(gpu_lib):
    sp2 = gpu_lib
    Fh, info = lattice_fock(8, seed=0)
    Fd = bsr_to_dense(Fh)
    no = info["n_occ"]
    lmin, lmax = O.gershgorin_bounds(Fd)
    F = sp2.BsrMatrix.from_host(Fh)
    r64 = sp2.density(F, no, lmin, lmax, -0.31, 0.33, trunc_norm="frobinf", tau_fixed=1e-6, coarse_bs=512)
    rb = sp2.density(F, no, lmin, lmax, -0.31, 0.33, trunc_norm="frobinf", tau_fixed=1e-6, coarse_bs=512,
                     precision="bf16x3")
    assert rb.switch_iter >= 1
    assert set(rb.iters["precision"][: rb.switch_iter]) == {2}
    err = np.linalg.norm(to_dense(rb.D) - to_dense(r64.D))
    print(f"mixed bf16x3 vs fp64: ||dD||_F = {err:.3e}, n = {rb.n_iter} vs {r64.n_iter}, switch {rb.switch_iter}")
    assert err <= 5e-2
    assert abs(np.trace(to_dense(rb.D)) - no) <= 1e-6


def test_low_precision_to_the_end(gpu_lib):
    """switch_tol < 0: every square in FP32, the stopping criterion evaluated on
    the FP32 e_i; the result is symmetric, has the right trace, is idempotent to
    FP32 level and close to the FP64 run; homo/lumo bounds, from the FP32 e_i
    above the FP32 floor only, still bound the true homo and lumo."""
    sp2 = gpu_lib
    Fh, info = lattice_fock(8, seed=0)
    Fd = bsr_to_dense(Fh)
    no = info["n_occ"]
    lmin, lmax = O.gershgorin_bounds(Fd)
    F = sp2.BsrMatrix.from_host(Fh)
    kw = dict(trunc_norm="frobinf", tau_fixed=1e-6, coarse_bs=512)
    r64 = sp2.density(F, no, lmin, lmax, -0.31, 0.33, **kw)
    r = sp2.density(F, no, lmin, lmax, -0.31, 0.33, precision="fp32", switch_tol=-1.0, **kw)
    assert r.status == 0 and r.stop_reason == "criterion"
    assert r.switch_iter == -1
    assert set(r.iters["precision"]) == {1}
    D = to_dense(r.D)
    assert np.array_equal(D, D.T)
    assert abs(np.trace(D) - no) <= 1e-2  # FP32 rounding of every iterate's trace
    assert np.linalg.norm(D @ D - D) <= 5e-3
    assert np.linalg.norm(D - to_dense(r64.D)) <= 5e-3
    lam = np.linalg.eigvalsh(Fd)
    homo, lumo = lam[no - 1], lam[no]
    assert not np.isnan(r.homo_est) and not np.isnan(r.lumo_est)
    assert homo <= r.homo_est + 1e-9 and r.lumo_est - 1e-9 <= lumo
    assert r.homo_est < r.lumo_est


@pytest.mark.parametrize("prec,correct", [("fp64", 0), ("bf16x3", 0), ("bf16x3", 1)])
def test_stepped_solver_equals_density(gpu_lib, prec, correct):
    """sp2_density_begin / _step / _end do the work of sp2_density: bit-identical
    D, the same statistics, one step per iteration of Algorithm 2 plus one per
    product of the correction, and step flops summing to the run's."""
    import torch

    sp2 = gpu_lib
    Fh, info = lattice_fock(8, seed=0)
    Fd = bsr_to_dense(Fh)
    no = info["n_occ"]
    lmin, lmax = O.gershgorin_bounds(Fd)
    opts = dict(accel=True, trunc_norm="frobinf", tau_fixed=1e-5, coarse_bs=512, precision=prec, correct=correct,
                switch_tol=0.0 if correct else 1e-3)
    F = sp2.BsrMatrix.from_host(Fh)
    ref = sp2.density(F, no, lmin, lmax, -0.31, 0.33, **opts)
    s = sp2.Solver(F, no, lmin, lmax, -0.31, 0.33, **opts)
    steps, flops = 0, 0.0
    done = False
    kinds = []
    while not done:
        st = s.step()
        done = st["done"]
        steps += 1
        flops += st["flops"]
        kinds.append(st["kind"])
        assert st["wall_s"] > 0.0
        if st["kind"] == "iteration":
            assert st["iteration"] == steps - 1
            k = {"fp64": 0, "fp32": 1, "bf16x3": 2}[st["precision"]]
            assert st["kernel_flops"][k] == pytest.approx(st["flops"], rel=1e-12)
            assert st["kernel_s"][k] > 0.0
    r = s.end()
    with pytest.raises(sp2.Sp2Error):
        s2 = sp2.Solver(F, no, lmin, lmax, -0.31, 0.33, **opts)
        s2.end()  # before the expansion finished
    print(f"{prec} correct={correct}: {steps} steps, n={r.n_iter}, flops {flops:.4e} vs {ref.alg_flops:.4e}")
    assert torch.equal(r.D.row_ptr, ref.D.row_ptr) and torch.equal(r.D.col_idx, ref.D.col_idx)
    assert torch.equal(r.D.val, ref.D.val)
    assert r.n_iter == ref.n_iter and r.stop_reason == ref.stop_reason and r.status == ref.status
    assert np.array_equal(r.iters["e"], ref.iters["e"])
    assert flops == pytest.approx(ref.alg_flops, rel=1e-12)
    assert r.alg_flops == ref.alg_flops
    n_corr = 0
    if correct:
        assert r.correction["corr_rounds"] == 1
        n_corr = steps - (r.n_iter + 1)
        assert n_corr >= 3  # commutator, Delta, purification (and the derivative steps)
    assert steps == r.n_iter + 1 + n_corr
    assert kinds == ["iteration"] * (r.n_iter + 1) + ["correction"] * n_corr
