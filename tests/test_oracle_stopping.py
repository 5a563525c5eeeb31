"""Pin of the oracle's e_i, t_i sequences and of the stopping index of
Algorithm 2 by the scalar eigenvalue iteration (closed form of an untruncated
run).

For F = Q diag(lam) Q^T and no truncation, every iterate is
X_i = Q diag(x_i) Q^T with x_0 = (lmax - lam) / w and x_i = f_i(x_{i-1}) per
eigenvalue, f_i(x) = ((1 - a) + a x)^2 (p_i = 1) or 2 a x - (a x)^2 (p_i = 0),
a = alpha_i (Algorithm 2).  So e_i = ||x_i - x_i^2||_2 and
t_i = sum(x_i - x_i^2) are known without any matrix product; the scalar
iteration resolves e_i far below the round-off floor of the matrix iteration.

Stopping index.  Algorithm 2 stops at the first i >= max(n_min, 2) with
p_i != p_{i-1} and e_i > C e_{i-2}^2.  In exact arithmetic two SP2 steps
contract e at most by the factor 4.41 < C (the supremum of
y(f(g(x))) / y(x)^2 for the pair (x^2, 2x - x^2), y(x) = x - x^2), so the
criterion fires only once the computed e_i sits on the round-off floor phi of
the matrix iteration.  Modelling the computed e_i as max(s_i, phi) with the
exact s_i from the scalar iteration predicts the stopping index; the
prediction is the same for every phi in [2^-53 sqrt(N), 2^-52 N] on the cases
below, so the pin does not depend on the precise floor.  A criterion that
fires early (before s_i reaches the floor), late (an admissible step after
it) or never (the run ends at n_max) fails it; the loose-bound SP2 cases
converge several iterations before n_max, where a stop by n_max and a stop by
the criterion differ.
"""
import math

import numpy as np
import pytest

from fockgen import dense_spectrum
from oracle import sp2_oracle as O

# (accel, homo_ub, lumo_lb): exact bounds of the dense N = 512 spectrum are
# -0.1 / 0.1; the looser ones leave n_max beyond the convergence point.
CASES = [
    (False, -0.1, 0.1),
    (True, -0.1, 0.1),
    (False, -0.05, 0.05),
    (True, -0.05, 0.05),
    (False, -0.02, 0.02),
    (True, -0.02, 0.02),
]


def scalar_iteration(lam, lmin, lmax, p, alpha, n):
    """e_i and t_i of the untruncated expansion from the eigenvalues alone."""
    x = (lmax - np.asarray(lam, dtype=np.float64)) / (lmax - lmin)
    s, t = [], []
    for i in range(n + 1):
        if i > 0:
            a = alpha[i]
            x = ((1.0 - a) + a * x) ** 2 if p[i] == 1 else 2.0 * a * x - (a * x) ** 2
        y = x - x * x
        s.append(float(np.sqrt(np.sum(y * y))))
        t.append(float(np.sum(y)))
    return s, t


def predicted_stop(s, p, n_min, n_max, phi, C=6.8872):
    """First admissible i at which max(s_i, phi) > C max(s_{i-2}, phi)^2, else
    n_max (the stopping test of Algorithm 2 on the floor model)."""
    for i in range(2, n_max + 1):
        if i >= max(n_min, 2) and p[i] != p[i - 1]:
            ei, em = max(s[i], phi), max(s[i - 2], phi)
            if ei > C * em * em:
                return i
    return n_max


def _floors(N):
    return np.geomspace(2.0 ** -53 * math.sqrt(N), 2.0 ** -52 * N, 25)


@pytest.fixture(scope="module")
def c0():
    F, lam, _ = dense_spectrum(512, seed=0)
    return F, lam


def stop_window(F, lam, accel, hb, lb):
    sch = O.schedule(-1.0, 1.0, hb, lb, accel=accel)
    s, t = scalar_iteration(lam, -1.0, 1.0, sch.p, sch.alpha, sch.n_max)
    preds = {predicted_stop(s, sch.p, sch.n_min, sch.n_max, phi) for phi in _floors(F.shape[0])}
    return sch, s, t, preds


def test_two_step_contraction_below_C():
    """The exact two-step supremum 4.41 of y(f(g(x))) / y(x)^2 lies below the
    paper's C = 6.8872, so exact runs never trigger the criterion: the
    supremum over a fine grid, for both orders of the pair."""
    x = np.linspace(1e-6, 1.0 - 1e-6, 2_000_001)
    y = x - x * x
    sq = lambda v: v * v
    fl = lambda v: 2 * v - v * v
    r1 = (lambda z: z - z * z)(fl(sq(x))) / (y * y)
    r2 = (lambda z: z - z * z)(sq(fl(x))) / (y * y)
    sup = max(r1.max(), r2.max())
    assert sup == pytest.approx(4.4092, abs=1e-3)
    assert sup < O.C_STOP


@pytest.mark.parametrize("accel,hb,lb", CASES)
def test_e_t_sequences_match_scalar_iteration(c0, accel, hb, lb):
    F, lam = c0
    N = F.shape[0]
    r = O.sp2(F, N // 2, -1.0, 1.0, hb, lb, accel=accel, trunc_norm=O.TRUNC_NONE)
    sch, s, t, _ = stop_window(F, lam, accel, hb, lb)
    assert list(r.p[1:]) == list(sch.p[1: r.n + 1])
    floor = 2.0 ** -52 * N
    for i in range(r.n + 1):
        assert abs(r.e[i] - s[i]) <= 1e-12 * s[i] + floor, (i, r.e[i], s[i])
        assert abs(r.t[i] - t[i]) <= 1e-12 * abs(t[i]) + floor, (i, r.t[i], t[i])


@pytest.mark.parametrize("accel,hb,lb", CASES)
def test_stopping_index_from_scalar_iteration(c0, accel, hb, lb):
    F, lam = c0
    N = F.shape[0]
    sch, s, _, preds = stop_window(F, lam, accel, hb, lb)
    assert len(preds) == 1, f"prediction depends on the floor: {preds}"
    n_pred = preds.pop()
    r = O.sp2(F, N // 2, -1.0, 1.0, hb, lb, accel=accel, trunc_norm=O.TRUNC_NONE)
    assert r.stop_reason == "criterion"
    assert r.n == n_pred
    # the stop comes once the exact e has dropped below the floor
    assert s[r.n] < 2.0 ** -52 * N


def test_loose_bounds_stop_before_n_max(c0):
    """The cases that separate a stop by the criterion from a stop by n_max."""
    F, lam = c0
    for accel, hb, lb in ((False, -0.05, 0.05), (False, -0.02, 0.02)):
        sch, _, _, preds = stop_window(F, lam, accel, hb, lb)
        assert max(preds) < sch.n_max


def test_homo_lumo_from_scalar_sequence(c0):
    """Step 3 estimates of the oracle equal those computed from the scalar
    e-sequence.  The estimates use e_i down to 1e3 * 2^-52 * sqrt(N) = 5e-12,
    where the matrix e_i carries a relative round-off of up to ~1e-4; pulled
    back through the inverse polynomials that moves a bound by ~1e-8."""
    F, lam = c0
    for accel, hb, lb in CASES:
        r = O.sp2(F, 256, -1.0, 1.0, hb, lb, accel=accel, trunc_norm=O.TRUNC_NONE)
        sch, s, _, _ = stop_window(F, lam, accel, hb, lb)
        r2 = O.Result(D=None, mask=None, n=r.n, stop_reason=r.stop_reason, status=r.status, sched=r.sched,
                      p=r.p, alpha=r.alpha, tau=r.tau, e=s[: r.n + 1], t=r.t, nnzb=r.nnzb, trunc=r.trunc,
                      masks=[], X=[], trX=r.trX, lmin=-1.0, lmax=1.0, n_occ=256)
        h, lu = O.homo_lumo_estimates(r2, 512)
        assert h == pytest.approx(r.homo_ub_est, abs=1e-7)
        assert lu == pytest.approx(r.lumo_lb_est, abs=1e-7)
        assert r.homo_ub_est >= lam[255] - 1e-10 and r.lumo_lb_est <= lam[256] + 1e-10


@pytest.mark.parametrize("planted_C,kind", [(1e300, "never"), (1e15, "late"), (1e-30, "early"), (1e-12, "early")])
def test_pin_catches_planted_criterion(c0, monkeypatch, planted_C, kind):
    """A wrong stopping constant planted in the oracle makes the pin fail: one
    that never fires ends at n_max, one that fires too early stops while the
    exact e_i is still resolvable."""
    F, lam = c0
    monkeypatch.setattr(O, "C_STOP", planted_C)
    caught = False
    for accel, hb, lb in ((False, -0.05, 0.05), (False, -0.02, 0.02), (True, -0.02, 0.02)):
        sch, s, _, preds = stop_window(F, lam, accel, hb, lb)
        r = O.sp2(F, 256, -1.0, 1.0, hb, lb, accel=accel, trunc_norm=O.TRUNC_NONE)
        if r.stop_reason != "criterion" or r.n not in preds:
            caught = True
    assert caught, kind
