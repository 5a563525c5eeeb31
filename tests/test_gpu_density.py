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


@pytest.fixture(scope="module")
def l8_oracle():
    """The 8 x 8 x 8 x 4 lattice (N = 2048), tau = 1e-6 Frob-Inf(512), and the
    oracle's FP64 expansion of it."""
    Fh, info = lattice_fock(8, seed=0)
    Fd = bsr_to_dense(Fh)
    no = info["n_occ"]
    lmin, lmax = O.gershgorin_bounds(Fd)
    lam = np.linalg.eigvalsh(Fd)
    ref = O.sp2(Fd, no, lmin, lmax, -0.31, 0.33, trunc_norm="frobinf", tau_fixed=1e-6, coarse_bs=512)
    return Fh, Fd, no, lmin, lmax, lam, ref


# ||D - D_oracle||_F measured for the FP64-tail runs on the 8^3 lattice; the
# tests allow twice that
MIXED_L8_ERR = {"fp32": 8.5e-5, "bf16x3": 6.0e-4}


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_mixed_fp64_tail_error(gpu_lib, l8_oracle, prec):
    """Low-precision squares with an FP64 tail: the subspace error of the
    low-precision iterations stays (section "Error control"), held here to
    twice its measured size against the oracle's D; idempotency and trace are
    restored by the tail."""
    sp2 = gpu_lib
    Fh, Fd, no, lmin, lmax, lam, ref = l8_oracle
    F = sp2.BsrMatrix.from_host(Fh)
    kw = dict(trunc_norm="frobinf", tau_fixed=1e-6, coarse_bs=512)
    r64 = sp2.density(F, no, lmin, lmax, -0.31, 0.33, **kw)
    r = sp2.density(F, no, lmin, lmax, -0.31, 0.33, precision=prec, **kw)
    code = {"fp32": 1, "bf16x3": 2}[prec]
    assert r.switch_iter >= 1
    assert set(r.iters["precision"][: r.switch_iter]) == {code}
    assert set(r.iters["precision"][r.switch_iter:]) == {0}
    D = to_dense(r.D)
    err, err64 = np.linalg.norm(D - ref.D), np.linalg.norm(D - to_dense(r64.D))
    print(f"mixed {prec}: ||D - D_oracle||_F = {err:.3e}, ||D - D_fp64||_F = {err64:.3e}, n = {r.n_iter} vs "
          f"{r64.n_iter}, switch {r.switch_iter}, status {r.status} ({r.stop_reason})")
    assert err <= 2 * MIXED_L8_ERR[prec]
    assert abs(np.trace(D) - no) <= 1e-6
    assert np.linalg.norm(D @ D - D) <= 1e-9


# ||D - D_FP64-stored tail||_F measured for the FP32-stored tail on the 8^3
# lattice; the test allows twice that
TAIL32_L8_DIFF = {"fp32": 1.3e-6, "bf16x3": 9.4e-6}


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_fp32_stored_fp64_tail(gpu_lib, l8_oracle, prec):
    """tail_storage = 1: the FP64 tail multiplies FP32-stored iterates in FP64
    arithmetic.  Same low-precision phase and switch as the FP64-stored tail;
    the tail squares are FP64 (precision code 0); idempotency reaches the FP32
    storage floor (the rounding E of an iterate to FP32 has ||E||_F <=
    2^-24 ||X||_F, and X - X^2 picks up E's occupied-occupied and
    virtual-virtual parts), the trace error stays within sqrt(N) ||D^2 - D||_F
    (the eigenvalue bound of the trace error model), the result is within
    twice its measured distance of the FP64-stored tail's, and the recorded
    map replays bit for bit."""
    sp2 = gpu_lib
    Fh, Fd, no, lmin, lmax, lam, ref = l8_oracle
    F = sp2.BsrMatrix.from_host(Fh)
    kw = dict(trunc_norm="frobinf", tau_fixed=1e-6, coarse_bs=512, precision=prec)
    r64 = sp2.density(F, no, lmin, lmax, -0.31, 0.33, **kw)
    r = sp2.density(F, no, lmin, lmax, -0.31, 0.33, tail_storage=1, record_tape=True, **kw)
    code = {"fp32": 1, "bf16x3": 2}[prec]
    assert r.switch_iter == r64.switch_iter >= 1
    assert set(r.iters["precision"][: r.switch_iter]) == {code}
    assert set(r.iters["precision"][r.switch_iter:]) == {0}
    assert np.array_equal(r.iters["e"][: r.switch_iter], r64.iters["e"][: r64.switch_iter])
    D, D64 = to_dense(r.D), to_dense(r64.D)
    N = D.shape[0]
    idem = np.linalg.norm(D @ D - D)
    floor = 2.0 ** -24 * np.sqrt(no)
    diff = np.linalg.norm(D - D64)
    print(f"{prec} FP32-stored tail: n = {r.n_iter} ({r.stop_reason}), e_n = {r.iters['e'][-1]:.3e}, "
          f"||D^2 - D||_F = {idem:.3e} (storage floor {floor:.2e}), |tr D - n_occ| = {abs(np.trace(D) - no):.3e}, "
          f"||D - D_tail64||_F = {diff:.3e}, ||D - D_oracle||_F = {np.linalg.norm(D - ref.D):.3e}")
    assert r.status == 0
    assert idem <= r.iters["e"][-1] + 4 * floor
    assert r.iters["e"][-1] <= r64.iters["e"][-1] + 4 * floor
    assert abs(np.trace(D) - no) <= np.sqrt(N) * idem + 1e-9
    assert diff <= 2 * TAIL32_L8_DIFF[prec]
    assert np.array_equal(to_dense(r.tape.replay(F)), D)
    # Step 3 with the FP32-storage noise of the tail's e_i: valid bounds
    homo, lumo = lam[no - 1], lam[no]
    print(f"homo/lumo estimates {r.homo_est:.5f} / {r.lumo_est:.5f} (exact {homo:.5f} / {lumo:.5f}; "
          f"FP64-stored tail {r64.homo_est:.5f} / {r64.lumo_est:.5f})")
    assert not np.isnan(r.homo_est) and not np.isnan(r.lumo_est)
    assert homo <= r.homo_est + 1e-9 and r.lumo_est - 1e-9 <= lumo


def test_fp32_stored_tail_lds_kernel_bitwise(gpu_lib, monkeypatch, l8_oracle):
    """The FP64 squares of FP32-stored iterates in the LDS-loaded kernel
    (FP32 quarter slices widened to FP64 at the fragment reads) and in the
    register-staged one give the same expansion bit for bit."""
    sp2 = gpu_lib
    Fh, Fd, no, lmin, lmax, lam, ref = l8_oracle
    F = sp2.BsrMatrix.from_host(Fh)
    kw = dict(trunc_norm="frobinf", tau_fixed=1e-6, coarse_bs=512, precision="fp32", tail_storage=1)
    out = {}
    for k in ("tile", "lds"):
        if k == "tile":
            monkeypatch.setenv("SP2_F64_KERNEL", "tile")
        else:
            monkeypatch.delenv("SP2_F64_KERNEL", raising=False)
        r = sp2.density(F, no, lmin, lmax, -0.31, 0.33, **kw)
        out[k] = (r.D.val.cpu().numpy(), r.iters["e"].copy(), r.n_iter, r.switch_iter)
    assert out["tile"][2:] == out["lds"][2:] and out["lds"][3] >= 1
    assert np.array_equal(out["tile"][1], out["lds"][1])
    assert np.array_equal(out["tile"][0].view(np.uint64), out["lds"][0].view(np.uint64))


def test_tail_storage_invalid(gpu_lib, l8_oracle):
    sp2 = gpu_lib
    Fh, Fd, no, lmin, lmax, lam, ref = l8_oracle
    F = sp2.BsrMatrix.from_host(Fh)
    with pytest.raises(RuntimeError, match="tail_storage"):
        sp2.density(F, no, lmin, lmax, -0.31, 0.33, precision="fp32", tail_storage=2)
    with pytest.raises(RuntimeError, match="tail_storage"):
        sp2.density(F, no, lmin, lmax, -0.31, 0.33, precision="fp32", tail_storage=1, correct=1)


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_mixed_homo_lumo_valid_and_tight(gpu_lib, l8_oracle, prec):
    """Step 3 on a mixed run: low-precision e_i enter above ten times their
    rounding noise (as e_i + noise), the FP64 tail's e_i as in an FP64 run.
    The estimates bound the true homo and lumo and the estimated gap is at
    least 0.8 of the FP64 run's; a run that stays in low precision to the end
    still gives valid (looser) bounds."""
    sp2 = gpu_lib
    Fh, Fd, no, lmin, lmax, lam, ref = l8_oracle
    homo, lumo = lam[no - 1], lam[no]
    F = sp2.BsrMatrix.from_host(Fh)
    kw = dict(trunc_norm="frobinf", tau_fixed=1e-6, coarse_bs=512)
    r64 = sp2.density(F, no, lmin, lmax, -0.31, 0.33, **kw)
    r = sp2.density(F, no, lmin, lmax, -0.31, 0.33, precision=prec, **kw)
    low = sp2.density(F, no, lmin, lmax, -0.31, 0.33, precision=prec, switch_tol=-1.0, **kw)
    print(f"{prec}: exact {homo:.5f} / {lumo:.5f}; fp64 {r64.homo_est:.5f} / {r64.lumo_est:.5f}; tail "
          f"{r.homo_est:.5f} / {r.lumo_est:.5f}; low to the end {low.homo_est:.5f} / {low.lumo_est:.5f}")
    for x in (r, low):
        assert not np.isnan(x.homo_est) and not np.isnan(x.lumo_est)
        assert homo <= x.homo_est + 1e-9 and x.lumo_est - 1e-9 <= lumo
    assert r.lumo_est - r.homo_est >= 0.8 * (r64.lumo_est - r64.homo_est)


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
    # error model: every eigenvalue x of D lies within |x (1 - x)| of 0 or 1, so
    # |tr D - n_occ| <= sum_j |x_j (1 - x_j)| <= sqrt(N) ||D - D^2||_F; the
    # expansion stops with ||D - D^2||_F at its FP32 e_n plus the rounding noise
    # of that FP32 e, kappa sqrt(tr D) with kappa = 4e-6
    N = Fd.shape[0]
    e_n = r.iters["e"][-1]
    nu = 4e-6 * np.sqrt(np.trace(D))
    print(f"FP32 to the end: |tr D - n_occ| = {abs(np.trace(D) - no):.3e}, ||D^2 - D||_F = "
          f"{np.linalg.norm(D @ D - D):.3e}, e_n = {e_n:.3e}, noise {nu:.3e}, bound {np.sqrt(N) * (e_n + nu):.3e}")
    assert np.linalg.norm(D @ D - D) <= e_n + nu
    assert abs(np.trace(D) - no) <= np.sqrt(N) * (e_n + nu)
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
