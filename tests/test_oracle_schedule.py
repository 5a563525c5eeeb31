"""Pins of the oracle's Step 1 schedule, stopping test and homo/lumo estimates.

* The bound images l_i, q_i must contain the actual eigenvalue images of
  X~_i (eigenvalues by LAPACK), and when the bounds are exact eigenvalues the
  scale-and-fold images are attained (the fold maps both ends of the interval
  onto the same value), which fixes alpha_i.
* The stopping constant C of Algorithm 2 is the paper's printed value and the
  criterion does not fire above the round-off floor on exact runs.
* Iteration estimates are plausible against the counts printed in section
  "Numerical experiments" (plausibility only, not parity).
* Homo/lumo estimates (Step 3) are valid one-sided bounds of the exact homo
  and lumo eigenvalues, with slack below 5% of the gap.
"""
import json
import os

import numpy as np
import pytest

from fockgen import bsr_to_dense, dense_spectrum, lattice_fock
from oracle import sp2_oracle as O

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def _spectrum_with_endpoints(n=256, seed=5):
    """Symmetric matrix whose eigenvalues include -1, 1 (the spectral bounds)
    and the homo/lumo values -0.2 / 0.15 exactly."""
    rng = np.random.default_rng(seed)
    no = n // 2
    lam = np.concatenate([[-1.0], rng.uniform(-0.95, -0.25, no - 2), [-0.2],
                          [0.15], rng.uniform(0.2, 0.95, n - no - 2), [1.0]])
    Q, R = np.linalg.qr(rng.standard_normal((n, n)))
    Q = Q * np.sign(np.diag(R))
    F = (Q * lam) @ Q.T
    return 0.5 * (F + F.T), np.sort(lam), no


@pytest.mark.parametrize("accel", [False, True])
def test_bounds_contain_and_attain_images(accel):
    F, lam, no = _spectrum_with_endpoints()
    r = O.sp2(F, no, -1.0, 1.0, -0.2, 0.15, accel=accel, trunc_norm=O.TRUNC_NONE,
              keep_tape=True, idem_stop=1e-13)
    s = r.sched
    for i in range(0, min(r.n, s.n_max) + 1):
        x = np.linalg.eigvalsh(r.X[i])  # ascending: unoccupied images first
        unocc_max = x[: len(x) - no].max()
        occ_min = x[len(x) - no:].min()
        tol = 1e-12 * (i + 1)
        assert unocc_max <= s.l[i] + tol
        assert occ_min >= 1.0 - s.q[i] - tol
        if s.l[i] > 1e-6:
            assert unocc_max == pytest.approx(s.l[i], rel=1e-8)
        if s.q[i] > 1e-6:
            assert 1.0 - occ_min == pytest.approx(s.q[i], rel=1e-8)


def test_acceleration_switch_off():
    s = O.schedule(-1.0, 1.0, -0.2, 0.15, accel=True)
    for i in range(1, s.n_max + 1):
        if i >= s.n_min:
            assert s.alpha[i] == 1.0
        else:
            assert s.alpha[i] > 1.0
    assert s.xi[0] == pytest.approx((0.15 + 0.2) / 2.0)


def test_tau_schedule_eq():
    """eq. (tau_trunc): tau_i (1 + g) = g xi_i with g = gamma / (n_max + 1)."""
    gamma = 1e-3
    s = O.schedule(-1.0, 1.0, -0.1, 0.1, accel=True, gamma=gamma)
    g = gamma / (s.n_max + 1)
    for i in range(s.n_max + 1):
        assert s.tau[i] * (1 + g) == pytest.approx(g * s.xi[i], rel=1e-14)
    # summing the per-iteration budget over n_max + 1 iterations gives gamma
    assert sum(s.tau[i] / (s.xi[i] - s.tau[i]) for i in range(s.n_max + 1)) == pytest.approx(gamma, rel=1e-12)


def test_stop_constant_is_paper_value():
    assert O.C_STOP == GOLD["stop_constant_C"]["value"]


def test_criterion_does_not_fire_above_roundoff():
    """On exact (untruncated) runs the convergence order of e_i cannot drop
    before round-off dominates: the criterion fires only when e_i is tiny."""
    F, lam, Y = dense_spectrum(512, seed=0)
    for accel in (False, True):
        r = O.sp2(F, 256, -1.0, 1.0, -0.1, 0.1, accel=accel, trunc_norm=O.TRUNC_NONE)
        if r.stop_reason == "criterion":
            assert r.e[r.n] < 1e-10


def test_iteration_estimates_plausible():
    """Plausibility against the printed estimates for water clusters
    (SP2 35-37, SP2ACC 22-23): some symmetric gap gives both at once."""
    sp2_lo, sp2_hi = GOLD["water_sp2_iterations"]["estimated"]
    acc_lo, acc_hi = GOLD["water_sp2acc_iterations"]["estimated"]
    hits = []
    for xgap in np.geomspace(1e-3, 2e-2, 60):
        h = -xgap  # spectrum [-1, 1] mapped to [0, 1]: x-gap = (lumo - homo) / 2
        s0 = O.schedule(-1.0, 1.0, h, h + 2 * xgap, accel=False)
        s1 = O.schedule(-1.0, 1.0, h, h + 2 * xgap, accel=True)
        if sp2_lo <= s0.n_max <= sp2_hi and acc_lo <= s1.n_max <= acc_hi:
            hits.append(xgap)
    assert hits, "no gap reproduces both printed estimates"
    # SP2ACC always needs fewer iterations than SP2
    for xgap in (1e-4, 1e-3, 1e-2, 0.1):
        s0 = O.schedule(-1.0, 1.0, -xgap, xgap, accel=False)
        s1 = O.schedule(-1.0, 1.0, -xgap, xgap, accel=True)
        assert s1.n_max < s0.n_max


@pytest.mark.parametrize("accel", [False, True])
def test_homo_lumo_estimates_valid_c0(accel):
    F, lam, Y = dense_spectrum(512, seed=0)
    r = O.sp2(F, 256, -1.0, 1.0, -0.1, 0.1, accel=accel, trunc_norm=O.TRUNC_NONE, idem_stop=1e-12)
    homo, lumo = lam[255], lam[256]
    gap = lumo - homo
    assert r.homo_ub_est >= homo - 1e-10
    assert r.lumo_lb_est <= lumo + 1e-10
    assert r.homo_ub_est - homo <= 0.05 * gap
    assert lumo - r.lumo_lb_est <= 0.05 * gap


def test_homo_lumo_two_run_protocol_lattice():
    """Run 1: trace-correcting expansion without bounds; its estimates feed
    run 2 (SP2ACC) as in section "Numerical experiments"."""
    Fb, info = lattice_fock(6, seed=0)
    F = bsr_to_dense(Fb)
    no = info["n_occ"]
    lam = np.linalg.eigvalsh(F)
    lmin, lmax = O.gershgorin_bounds(F)
    r1 = O.sp2(F, no, lmin, lmax, trunc_norm=O.TRUNC_NONE)
    assert r1.sched.mode == "tc2"
    assert r1.homo_ub_est >= lam[no - 1] - 1e-10
    assert r1.lumo_lb_est <= lam[no] + 1e-10
    r2 = O.sp2(F, no, lmin, lmax, r1.homo_ub_est, r1.lumo_lb_est, trunc_norm=O.TRUNC_NONE)
    D, _ = O.density_by_diagonalization(F, no)
    assert O.frobenius_norm(r2.D - D) <= 1e-10
    assert r2.n < r1.n
    gap = lam[no] - lam[no - 1]
    assert lam[no - 1] <= r2.homo_ub_est <= lam[no - 1] + 0.05 * gap
    assert lam[no] - 0.05 * gap <= r2.lumo_lb_est <= lam[no]
