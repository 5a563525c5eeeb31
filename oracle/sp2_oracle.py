"""Plain, slow CPU FP64 oracle of the SP2 / SP2ACC density-matrix expansion.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or call this module.  It shares
no code with the HIP implementation in ``paper_1909_12533_amd`` and does not
import it.

Follows A. Kruchinina, E. Rudberg, E. H. Rubensson, "Efficient computation of
the density matrix with error control on distributed computer systems"
(arXiv:1909.12533):

* the density matrix D = theta(mu I - F) (section "Introduction");
* the SP2 / SP2ACC recursive expansion, Algorithms 1 and 2 and Steps 1-3 of
  section "Density matrix construction";
* the truncation threshold schedule, eq. (tau_trunc), and the error-control
  bound on the occupied subspace (section "Error control");
* the Frobenius and Frob-Inf truncation norms (section "Upper bounds for the
  spectral norm");
* beyond the paper, for low-precision expansions: the first-order correction
  of the occupied subspace, ``subspace_correction``;
* the product of matrices in general (full-pattern) storage, the format of the
  paper's general matrix wrapper (section "Implementation details"),
  ``general_product``.

Matrices are stored dense in float64, with a symmetric boolean block mask
(nbr x nbr, block size ``bs``) that records which blocks are structurally
present.  Dense products of masked matrices are exact zeros outside the block
pattern, so every result equals the block-sparse result up to summation order.

Parts of the method that the paper delegates to other papers are implemented
as the readings listed here; each one is a "reading", not a quotation:

* Step 1 (the polynomial sequence p_i, scale-and-fold parameters alpha_i,
  n_max and n_min) -- ``schedule``;
* Step 3 (homo/lumo estimates from e_i and t_i) -- ``homo_lumo_estimates``;
* the truncation procedure that realises ||E_i|| <= tau_i -- ``truncate``.

Pins (tests that hold this oracle to something other than itself) live in
``tests/test_oracle_*.py``.  Functions without a pin say "parity unpinned".
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

BS = 64
# Constant of the parameterless stopping criterion (Algorithm 2).
C_STOP = 6.8872
# n_max: first iteration at which both bound images are within 2^-52 of 0 / 1.
DELTA_N = 2.0 ** -52
# Acceleration is used only while max(l, q) >= DELTA_ACC (reading of Step 1).
DELTA_ACC = 1e-2

TRUNC_NONE = "none"
TRUNC_FROB = "frob"
TRUNC_FROBINF = "frobinf"


class OracleError(ValueError):
    pass


# ==========================================================================
# norms (section "Upper bounds for the spectral norm")
# ==========================================================================

def frobenius_norm(A):
    """||A||_F, the square root of the sum of squared entries."""
    return math.sqrt(float(np.sum(np.asarray(A, dtype=np.float64) ** 2)))


def spectral_norm_sym(A):
    """||A||_2 = spectral radius rho(A) for a symmetric A (eigenvalues by
    LAPACK); test-only, the paper notes it is expensive for large systems."""
    w = np.linalg.eigvalsh(A)
    return float(np.max(np.abs(w)))


def inf_norm(A):
    """||A||_inf, the largest row sum of absolute values."""
    return float(np.max(np.sum(np.abs(A), axis=1)))


def submatrix_frobenius(A, sub):
    """Matrix of Frobenius norms of the sub x sub submatrices of A (the last
    submatrix row/column may be smaller)."""
    n = A.shape[0]
    nb = (n + sub - 1) // sub
    P = np.zeros((nb * sub, nb * sub))
    P[:n, :n] = A
    B = P.reshape(nb, sub, nb, sub)
    return np.sqrt(np.sum(B * B, axis=(1, 3)))


def frob_spectral_norm(A, sub):
    """Frobenius-spectral mixed norm ||A||_m: the spectral norm of the matrix
    of submatrix Frobenius norms (section "Upper bounds for the spectral
    norm")."""
    N = submatrix_frobenius(A, sub)
    return float(np.max(np.linalg.svd(N, compute_uv=False)))


def frob_inf_norm(A, sub):
    """Frob-Inf mixed norm ||A||_M: the infinity norm of the matrix of
    submatrix Frobenius norms (section "Upper bounds for the spectral
    norm")."""
    return inf_norm(submatrix_frobenius(A, sub))


# ==========================================================================
# helpers on block masks
# ==========================================================================

def nblocks(n, bs):
    return (n + bs - 1) // bs


def block_norms2(X, bs):
    """Squared Frobenius norm of every bs x bs block (nbr x nbr)."""
    return submatrix_frobenius(X, bs) ** 2


def structural_mask(X, bs):
    """Blocks holding at least one non-zero entry."""
    return block_norms2(X, bs) > 0.0


def expand_mask(M, n, bs):
    """Element mask (n x n) of a block mask."""
    return np.repeat(np.repeat(M, bs, axis=0), bs, axis=1)[:n, :n]


def pattern_square(M):
    """Block pattern of X^2 for a symmetric X with block pattern M: (I, J) is
    present when some K has (I, K) and (K, J) present."""
    Mi = M.astype(np.int64)
    return (Mi @ Mi) > 0


def upper_count(M):
    return int(np.count_nonzero(np.triu(M)))


# ==========================================================================
# Gershgorin bounds (Step 1: lambda_min <= lambda_1, lambda_max >= lambda_N)
# ==========================================================================

def gershgorin_bounds(F):
    """Interval [lmin, lmax] containing all eigenvalues of F, from the
    Gershgorin circle theorem: every eigenvalue lies in some disc centred at
    F_ii with radius sum_{j != i} |F_ij|."""
    F = np.asarray(F, dtype=np.float64)
    d = np.diag(F)
    r = np.sum(np.abs(F), axis=1) - np.abs(d)
    return float(np.min(d - r)), float(np.max(d + r))


# ==========================================================================
# Step 1: schedule
# ==========================================================================

@dataclass
class Schedule:
    """Polynomial sequence and truncation thresholds (Step 1).  Index 0 of
    p/alpha is unused; l[i], q[i], xi[i], tau[i] refer to X_i."""

    mode: str  # "bounds" or "tc2"
    w: float
    p: list = field(default_factory=list)
    alpha: list = field(default_factory=list)
    l: list = field(default_factory=list)
    q: list = field(default_factory=list)
    xi: list = field(default_factory=list)
    tau: list = field(default_factory=list)
    n_max: int = 0
    n_min: int = 1


def schedule(lmin, lmax, homo_ub, lumo_lb, accel=True, gamma=0.0, tau_fixed=0.0, n_max_cap=100):
    """Step 1 of section "Density matrix construction" from homo/lumo bounds.

    Reading (the paper defers to Algorithm 4 of its stopping-criterion
    reference): the images of the spectrum in X_i are tracked by two
    complement bounds: every unoccupied eigenvalue image lies in [0, l_i] and
    every occupied image in [1 - q_i, 1].  With w = lmax - lmin, X_0 gives
    l_0 = (lmax - lumo_lb)/w and q_0 = (homo_ub - lmin)/w.  Each iteration
    picks the polynomial that attacks the larger bound: p_i = 1 (x^2 family)
    when l_{i-1} > q_{i-1}, else p_i = 0 (2x - x^2 family); a tie gives 0.
    Scale-and-fold takes alpha_i = 2/(2 - l) (p = 1) or 2/(2 - q) (p = 0), the
    value for which both ends of the interval being folded land on the same
    image; acceleration stops (alpha_i = 1) once max(l, q) < DELTA_ACC.
    n_max is the first i with max(l_i, q_i) <= 2^-52 (capped), n_min the first
    i with alpha_i = 1.  The gap lower bound is xi_i = 1 - q_i - l_i and the
    thresholds follow eq. (tau_trunc) unless a fixed tau is given."""
    if not (lmin < lmax):
        raise OracleError("lmin must be < lmax")
    w = lmax - lmin
    l = (lmax - lumo_lb) / w
    q = (homo_ub - lmin) / w
    s = Schedule(mode="bounds", w=w)
    s.p.append(-1)
    s.alpha.append(1.0)
    s.l.append(l)
    s.q.append(q)
    n_max = n_max_cap
    for i in range(1, n_max_cap + 1):
        p = 1 if l > q else 0
        if accel and max(l, q) >= DELTA_ACC:
            a = 2.0 / (2.0 - l) if p == 1 else 2.0 / (2.0 - q)
        else:
            a = 1.0
        if p == 1:
            # f(x) = ((1 - a) + a x)^2
            lo = (1.0 - a) * (1.0 - a)
            hi = (1.0 - a + a * l) * (1.0 - a + a * l)
            l_new = max(lo, hi)
            q_new = a * q * (2.0 - a * q)
        else:
            # f(x) = 2 a x - (a x)^2
            l_new = a * l * (2.0 - a * l)
            lo = (1.0 - a + a * q) * (1.0 - a + a * q)
            hi = (1.0 - a) * (1.0 - a)
            q_new = max(lo, hi)
        l, q = l_new, q_new
        s.p.append(p)
        s.alpha.append(a)
        s.l.append(l)
        s.q.append(q)
        if max(l, q) <= DELTA_N:
            n_max = i
            break
    s.n_max = n_max
    s.n_min = n_max + 1
    for i in range(1, n_max + 1):
        if s.alpha[i] == 1.0:
            s.n_min = i
            break
    s.xi = [1.0 - s.q[i] - s.l[i] for i in range(n_max + 1)]
    if tau_fixed > 0.0:
        s.tau = [tau_fixed] * (n_max + 1)
    elif gamma > 0.0:
        g = gamma / (n_max + 1)
        s.tau = [g * s.xi[i] / (1.0 + g) for i in range(n_max + 1)]
    else:
        s.tau = [0.0] * (n_max + 1)
    return s


def schedule_tc2(lmin, lmax, tau_fixed=0.0, n_max_cap=100):
    """Schedule of the trace-correcting expansion used when no homo/lumo
    bounds are known (the first of the two runs in section "Numerical
    experiments"): p_i is chosen during the run from traces, alpha_i = 1,
    n_max is the cap and thresholds are the fixed ad-hoc tau."""
    if not (lmin < lmax):
        raise OracleError("lmin must be < lmax")
    s = Schedule(mode="tc2", w=lmax - lmin)
    s.n_max = n_max_cap
    s.n_min = 1
    s.p = [-1]
    s.alpha = [1.0] * (n_max_cap + 1)
    s.tau = [tau_fixed] * (n_max_cap + 1)
    return s


# ==========================================================================
# truncation  (X~_i = X_i + E_i with ||E_i|| <= tau_i)
# ==========================================================================

@dataclass
class TruncInfo:
    removed: int = 0
    err_frob: float = 0.0  # ||E||_F of the full symmetric E
    err_mixed: float = 0.0  # ||E||_M with the coarse partition


def _coarse_error_norms(n2_removed_upper, nbr, cb):
    """Frob-Inf norm of the removed part E: coarse-block Frobenius norms of the
    full symmetric E, then the largest coarse row sum."""
    nc = (nbr + cb - 1) // cb
    E2 = np.zeros((nc, nc))
    I, J = np.nonzero(n2_removed_upper)
    for a, b in zip(I, J):
        v = n2_removed_upper[a, b]
        R, S = a // cb, b // cb
        if R == S:
            E2[R, R] += 2.0 * v
        else:
            E2[R, S] += v
            E2[S, R] += v
    return float(np.max(np.sum(np.sqrt(E2), axis=1))) if nc > 0 else 0.0


def truncate(X, M, tau, norm=TRUNC_FROBINF, bs=BS, coarse_bs=4096):
    """Remove small blocks of the symmetric matrix X (block pattern M) so that
    the removed part E satisfies ||E|| <= tau (section "Error control",
    inequality (error_tau_trunc)), in the Frobenius norm or in the Frob-Inf
    norm of section "Upper bounds for the spectral norm".

    Reading of the procedure (the paper only states the bound): diagonal
    blocks are never removed.  Candidates are the present upper off-diagonal
    blocks, visited in ascending order of squared block norm, ties broken by
    (I, J); the longest prefix is removed whose weighted sum of squared norms
    stays within the budget.
      * Frobenius: one budget tau^2 for the whole matrix, weight 2 (a block
        and its mirror).
      * Frob-Inf with coarse blocks of ``coarse_bs`` rows: m_R is the number
        of coarse blocks of coarse row R (full symmetric matrix) holding a
        present block; coarse block (R, S), R <= S, gets the budget
        (tau / max(m_R, m_S))^2; a fine block weighs 2 inside a diagonal
        coarse block (it appears twice in E_RR) and 1 elsewhere.  Then every
        coarse row sum of ||E_RS||_F is at most tau.
    Returns (X~, M~, TruncInfo)."""
    n = X.shape[0]
    nbr = nblocks(n, bs)
    info = TruncInfo()
    if norm == TRUNC_NONE or tau <= 0.0:
        return X, M, info
    n2 = block_norms2(X, bs)
    I, J = np.nonzero(np.triu(M, 1))
    if I.size == 0:
        return X, M, info
    vals = n2[I, J]
    if norm == TRUNC_FROB:
        seg = np.zeros(I.size, dtype=np.int64)
        weight = np.full(I.size, 2.0)
        budget = {0: tau * tau}
    elif norm == TRUNC_FROBINF:
        if coarse_bs % bs != 0:
            raise OracleError("coarse_bs must be a multiple of bs")
        cb = coarse_bs // bs
        nc = (nbr + cb - 1) // cb
        occ = np.zeros((nc, nc), dtype=bool)
        MI, MJ = np.nonzero(M)
        occ[MI // cb, MJ // cb] = True
        m = occ.sum(axis=1)
        R = I // cb
        S = J // cb
        seg = R * nc + S
        weight = np.where(R == S, 2.0, 1.0)
        budget = {}
        for s in np.unique(seg):
            r, c = divmod(int(s), nc)
            beta = tau / max(m[r], m[c])
            budget[int(s)] = beta * beta
    else:
        raise OracleError(f"unknown truncation norm {norm!r}")

    remove = np.zeros(I.size, dtype=bool)
    lin = I * nbr + J
    for s in np.unique(seg):
        idx = np.nonzero(seg == s)[0]
        order = idx[np.lexsort((lin[idx], vals[idx]))]
        acc = 0.0
        b = budget[int(s)]
        for k in order:
            nxt = acc + weight[k] * vals[k]
            if nxt <= b:
                acc = nxt
                remove[k] = True
            else:
                break
    Mt = M.copy()
    rI, rJ = I[remove], J[remove]
    Mt[rI, rJ] = False
    Mt[rJ, rI] = False
    Xt = X * expand_mask(Mt, n, bs)
    info.removed = int(remove.sum())
    info.err_frob = math.sqrt(float(np.sum(2.0 * vals[remove])))
    n2r = np.zeros((nbr, nbr))
    n2r[rI, rJ] = vals[remove]
    cbs = (coarse_bs // bs) if norm == TRUNC_FROBINF else nbr
    info.err_mixed = _coarse_error_norms(n2r, nbr, cbs)
    return Xt, Mt, info


# ==========================================================================
# Steps 1-2: Algorithms 1 and 2
# ==========================================================================

@dataclass
class Result:
    D: np.ndarray
    mask: np.ndarray
    n: int
    stop_reason: str
    status: int
    sched: Schedule
    p: list
    alpha: list
    tau: list
    e: list
    t: list
    nnzb: list
    trunc: list
    masks: list
    X: list  # X~_i (kept only when keep_tape)
    trX: list = field(default_factory=list)  # tr X~_i
    homo_ub_est: float = float("nan")
    lumo_lb_est: float = float("nan")
    subspace_err_bound: float = float("nan")
    alg_flops: float = 0.0
    lmin: float = 0.0
    lmax: float = 0.0
    n_occ: int = 0


STATUS_OK = 0
WARN_NOT_CONVERGED = 1
WARN_TRACE = 2


def _validate(F, n_occ, lmin, lmax, homo_ub, lumo_lb):
    if F.ndim != 2 or F.shape[0] != F.shape[1]:
        raise OracleError("F must be square")
    if not np.all(np.isfinite(F)):
        raise OracleError("F has non-finite entries")
    if not np.array_equal(F, F.T):
        raise OracleError("F must be symmetric")
    N = F.shape[0]
    if not (0 < n_occ < N):
        raise OracleError("n_occ must lie in (0, N)")
    if not (lmin < lmax):
        raise OracleError("lmin must be < lmax")
    if (homo_ub is None) != (lumo_lb is None):
        raise OracleError("give both homo/lumo bounds or neither")
    if homo_ub is not None and not (lmin <= homo_ub < lumo_lb <= lmax):
        raise OracleError("bounds must satisfy lmin <= homo_ub < lumo_lb <= lmax")


def sp2(F, n_occ, lmin, lmax, homo_ub=None, lumo_lb=None, *, accel=True,
        trunc_norm=TRUNC_FROBINF, gamma=0.0, tau_fixed=0.0, coarse_bs=4096,
        idem_stop=0.0, n_max_cap=100, bs=BS, keep_tape=False):
    """Density matrix by the SP2 / SP2ACC recursive expansion.

    Step 1 (schedule, thresholds), Algorithm 1 (X_0, first truncation,
    e_0, t_0), Algorithm 2 (polynomial steps, truncation, e_i, t_i and the
    parameterless stopping test), Step 3 (homo/lumo estimates), all of
    section "Density matrix construction".  SP2 is the special case
    alpha_i = 1, n_min = 1 (``accel=False``).  Without bounds the
    trace-correcting choice of p_i is used (reading: p_i = 1 when the trace of
    X~^2 is closer to n_occ than that of 2X~ - X~^2; a tie gives 0).

    Stopping (reading): stop at i when i >= max(n_min, 2), p_i != p_{i-1} and
    e_i > C e_{i-2}^2, or when ``idem_stop`` > 0 and e_i <= idem_stop; when
    neither fires by n_max the run ends at n_max with a warning.  The output
    is the stored (truncated) X~_n."""
    F = np.asarray(F, dtype=np.float64)
    _validate(F, n_occ, lmin, lmax, homo_ub, lumo_lb)
    N = F.shape[0]
    nbr = nblocks(N, bs)
    if homo_ub is not None:
        sch = schedule(lmin, lmax, homo_ub, lumo_lb, accel, gamma, tau_fixed, n_max_cap)
    else:
        sch = schedule_tc2(lmin, lmax, tau_fixed, n_max_cap)
    w = lmax - lmin
    I_N = np.eye(N)

    # ---- Algorithm 1 -----------------------------------------------------
    X0 = (lmax * I_N - F) / w
    M0 = structural_mask(F, bs)
    M0[np.arange(nbr), np.arange(nbr)] = True
    Xt, M, tinfo = truncate(X0, M0, sch.tau[0], trunc_norm, bs, coarse_bs)
    S = Xt @ Xt
    MS = pattern_square(M)

    res = Result(D=None, mask=None, n=0, stop_reason="", status=STATUS_OK, sched=sch,
                 p=[-1], alpha=[1.0], tau=[sch.tau[0]], e=[], t=[], nnzb=[upper_count(M)],
                 trunc=[tinfo], masks=[M.copy()], X=[Xt.copy()] if keep_tape else [],
                 lmin=lmin, lmax=lmax, n_occ=n_occ)
    res.e.append(frobenius_norm(Xt - S))
    res.t.append(float(np.trace(Xt) - np.trace(S)))
    res.trX.append(float(np.trace(Xt)))
    res.alg_flops += 2.0 * bs ** 3 * _triples_upper(M)

    # ---- Algorithm 2 -----------------------------------------------------
    n = None
    for i in range(1, sch.n_max + 1):
        if sch.mode == "bounds":
            p, a = sch.p[i], sch.alpha[i]
        else:
            trS = float(np.trace(S))
            trX = float(np.trace(Xt))
            p = 1 if abs(trS - n_occ) < abs(2.0 * trX - trS - n_occ) else 0
            a = 1.0
        if p == 1:
            Y = (1.0 - a) * I_N + a * Xt
            X = Y @ Y
        else:
            Z = a * Xt
            X = 2.0 * Z - Z @ Z
        tau_i = sch.tau[i]
        Xt, M, tinfo = truncate(X, MS, tau_i, trunc_norm, bs, coarse_bs)
        S = Xt @ Xt
        MS = pattern_square(M)
        res.p.append(p)
        res.alpha.append(a)
        res.tau.append(tau_i)
        res.nnzb.append(upper_count(M))
        res.trunc.append(tinfo)
        res.masks.append(M.copy())
        if keep_tape:
            res.X.append(Xt.copy())
        res.e.append(frobenius_norm(Xt - S))
        res.t.append(float(np.trace(Xt) - np.trace(S)))
        res.trX.append(float(np.trace(Xt)))
        res.alg_flops += 2.0 * bs ** 3 * _triples_upper(M)
        e = res.e
        if i >= max(sch.n_min, 2) and res.p[i] != res.p[i - 1] and e[i] > C_STOP * e[i - 2] ** 2:
            n = i
            res.stop_reason = "criterion"
            break
        if idem_stop > 0.0 and e[i] <= idem_stop:
            n = i
            res.stop_reason = "idempotency"
            break
    if n is None:
        n = sch.n_max
        res.stop_reason = "n_max"
        res.status = WARN_NOT_CONVERGED
    res.n = n
    res.D = Xt
    res.mask = M
    if sch.mode == "tc2":
        sch.n_max = n
    # ---- Step 3 ----------------------------------------------------------
    res.homo_ub_est, res.lumo_lb_est = homo_lumo_estimates(res, N)
    res.subspace_err_bound = subspace_error_bound(res)
    if abs(float(np.trace(Xt)) - n_occ) > 0.5 and res.status == STATUS_OK:
        res.status = WARN_TRACE
    return res


def _triples_upper(M):
    """Number of block products (I, K, J), I <= J, in the square of a matrix
    with block pattern M (the algorithmic work of one symmetric square)."""
    Mi = M.astype(np.int64)
    C = Mi @ Mi
    return int(np.sum(np.triu(C)))


# ==========================================================================
# Step 3: homo/lumo estimates
# ==========================================================================

def homo_lumo_estimates(res: Result, N):
    """Homo/lumo estimates from e_i and t_i (Step 3; the paper defers the
    algorithm to its interior-eigenvalue reference).

    Reading: since ||X - X^2||_2 <= ||X - X^2||_F = e_i, every eigenvalue x of
    X~_i has x(1 - x) <= e_i, so with u = 2 e_i / (1 + sqrt(1 - 4 e_i)) it lies
    in [0, u] or [1 - u, 1].  Iteration i is used when these two clusters are
    known to separate occupied from unoccupied images: with bounds, when the
    forward bounds satisfy l_i < 1 - u and q_i < 1 - u; without bounds, when
    |tr X~_i - n_occ| < 1/2 - N u.  Then the lumo image is <= u and the homo
    image >= 1 - u, and these are pulled back through f_i, ..., f_1 on the
    branch that faces the gap:
        p = 1:  u <- (sqrt(u) + a - 1)/a,      q <- q / ((1 + sqrt(1 - q)) a)
        p = 0:  u <- u / ((1 + sqrt(1 - u)) a), q <- (a - 1 + sqrt(q))/a
    giving homo <= lmin + q w and lumo >= lmax - u w.  Only e_i in
    [e_floor, 1/4) with e_floor = 1e3 * 2^-52 * sqrt(N) are used (below it the
    images of occupied eigenvalues round to 1 in float64).  The tightest
    bounds over all usable i are returned (nan when none is usable)."""
    sch = res.sched
    w = res.lmax - res.lmin
    e_floor = 1e3 * DELTA_N * math.sqrt(N)
    best_h = math.inf
    best_l = -math.inf
    for i in range(0, res.n + 1):
        e = res.e[i]
        if not (e_floor <= e < 0.25):
            continue
        u = 2.0 * e / (1.0 + math.sqrt(1.0 - 4.0 * e))
        if sch.mode == "bounds":
            ok = sch.l[i] < 1.0 - u and sch.q[i] < 1.0 - u
        else:
            ok = abs(res.trX[i] - res.n_occ) < 0.5 - N * u
        if not ok:
            continue
        uu, qq = u, u
        for j in range(i, 0, -1):
            p, a = res.p[j], res.alpha[j]
            if p == 1:
                uu = (math.sqrt(uu) + a - 1.0) / a
                qq = qq / ((1.0 + math.sqrt(1.0 - qq)) * a)
            else:
                uu = uu / ((1.0 + math.sqrt(1.0 - uu)) * a)
                qq = (a - 1.0 + math.sqrt(qq)) / a
        best_h = min(best_h, res.lmin + qq * w)
        best_l = max(best_l, res.lmax - uu * w)
    h = best_h if math.isfinite(best_h) else float("nan")
    lo = best_l if math.isfinite(best_l) else float("nan")
    return h, lo


def subspace_error_bound(res: Result):
    """Bound on ||D - P_Xn|| from section "Error control":
    sum_i ||E_i|| / (xi_i - ||E_i||), with the Frob-Inf norm of E_i as the
    upper bound of its spectral norm (section "Upper bounds for the spectral
    norm").  nan without gap bounds (trace-correcting run)."""
    sch = res.sched
    if sch.mode != "bounds":
        return float("nan")
    tot = 0.0
    for i in range(res.n + 1):
        E = res.trunc[i].err_mixed
        if E == 0.0:
            continue
        tot += E / (sch.xi[i] - E)
    return tot


# ==========================================================================
# reference density matrix by diagonalisation (section "Introduction")
# ==========================================================================

def density_by_diagonalization(F, n_occ):
    """D = sum_{i <= n_occ} y_i y_i^T over the eigenvectors of the n_occ
    lowest eigenvalues (eq. (eig_problem_D)).  Returns (D, eigenvalues)."""
    lam, Y = np.linalg.eigh(np.asarray(F, dtype=np.float64))
    Yo = Y[:, :n_occ]
    return Yo @ Yo.T, lam


# ==========================================================================
# adjoint of the discrete recursion (frozen schedule and masks)
# ==========================================================================

def _apply_mask(X, M, bs):
    return X * expand_mask(M, X.shape[0], bs)


def replay(res: Result, F, bs=BS):
    """Forward map with the schedule (p_i, alpha_i, n) and the block masks of
    a recorded run frozen: X~_0 = M_0 o (lmax I - F)/w,
    X~_i = M_i o f_i(X~_{i-1}).  Used for finite differences."""
    F = np.asarray(F, dtype=np.float64)
    N = F.shape[0]
    w = res.lmax - res.lmin
    I_N = np.eye(N)
    Xt = _apply_mask((res.lmax * I_N - F) / w, res.masks[0], bs)
    for i in range(1, res.n + 1):
        p, a = res.p[i], res.alpha[i]
        if p == 1:
            Y = (1.0 - a) * I_N + a * Xt
            X = Y @ Y
        else:
            Z = a * Xt
            X = 2.0 * Z - Z @ Z
        Xt = _apply_mask(X, res.masks[i], bs)
    return Xt


def _tape(res: Result, F, bs):
    """X~_0 .. X~_{n-1} of the frozen forward map (recomputed when the run did
    not keep them)."""
    if res.X and len(res.X) >= res.n:
        return res.X
    F = np.asarray(F, dtype=np.float64)
    N = F.shape[0]
    w = res.lmax - res.lmin
    I_N = np.eye(N)
    out = [_apply_mask((res.lmax * I_N - F) / w, res.masks[0], bs)]
    for i in range(1, res.n):
        p, a = res.p[i], res.alpha[i]
        Xt = out[-1]
        if p == 1:
            Y = (1.0 - a) * I_N + a * Xt
            X = Y @ Y
        else:
            Z = a * Xt
            X = 2.0 * Z - Z @ Z
        out.append(_apply_mask(X, res.masks[i], bs))
    return out


def jvp(res: Result, F, dF, bs=BS):
    """Directional derivative dD = J dF of the frozen discrete map (reading:
    schedule, n and masks are held fixed; lmin and lmax are constants).
    dX~_0 = -M_0 o dF / w, then the derivative of each polynomial:
        p = 1: dX_i = a (Y dX~ + dX~ Y),  Y = (1 - a) I + a X~_{i-1}
        p = 0: dX_i = 2 a dX~ - a^2 (X~_{i-1} dX~ + dX~ X~_{i-1})
    followed by the mask M_i."""
    tape = _tape(res, F, bs)
    N = F.shape[0]
    w = res.lmax - res.lmin
    I_N = np.eye(N)
    dX = _apply_mask(-np.asarray(dF, dtype=np.float64) / w, res.masks[0], bs)
    for i in range(1, res.n + 1):
        p, a = res.p[i], res.alpha[i]
        Xt = tape[i - 1]
        if p == 1:
            Y = (1.0 - a) * I_N + a * Xt
            dX = a * (Y @ dX + dX @ Y)
        else:
            dX = 2.0 * a * dX - a * a * (Xt @ dX + dX @ Xt)
        dX = _apply_mask(dX, res.masks[i], bs)
    return dX


def vjp(res: Result, F, W, bs=BS):
    """Gradient of L = tr(W D) with respect to F for the frozen discrete map:
    Xbar_n = W, then for i = n..1: G = M_i o Xbar and
        p = 1: Xbar = a (Y G + G Y),  Y = (1 - a) I + a X~_{i-1}
        p = 0: Xbar = 2 a G - a^2 (X~_{i-1} G + G X~_{i-1})
    and finally Fbar = -(M_0 o Xbar) / w."""
    tape = _tape(res, F, bs)
    N = F.shape[0]
    w = res.lmax - res.lmin
    I_N = np.eye(N)
    Xbar = np.asarray(W, dtype=np.float64).copy()
    for i in range(res.n, 0, -1):
        G = _apply_mask(Xbar, res.masks[i], bs)
        p, a = res.p[i], res.alpha[i]
        Xt = tape[i - 1]
        if p == 1:
            Y = (1.0 - a) * I_N + a * Xt
            Xbar = a * (Y @ G + G @ Y)
        else:
            Xbar = 2.0 * a * G - a * a * (Xt @ G + G @ Xt)
    return -_apply_mask(Xbar, res.masks[0], bs) / w


def daleckii_krein_gradient(F, n_occ, W):
    """Closed-form gradient of tr(W D) for the exact spectral projector D of a
    symmetric F with a gap: sum over occupied o and virtual v of
    (y_o^T W y_v)/(lam_o - lam_v) (y_o y_v^T + y_v y_o^T)."""
    lam, Y = np.linalg.eigh(np.asarray(F, dtype=np.float64))
    Yo, Yv = Y[:, :n_occ], Y[:, n_occ:]
    C = (Yo.T @ W @ Yv) / (lam[:n_occ, None] - lam[None, n_occ:])
    G = Yo @ C @ Yv.T
    return G + G.T


# ==========================================================================
# occupied-subspace correction (extension for low-precision expansions)
# ==========================================================================

def _drop_small_blocks(X, beta, bs):
    """Frobenius truncation of X with budget beta over its present blocks
    (``truncate`` with the Frobenius norm); X may be antisymmetric."""
    if beta <= 0.0:
        return X
    M = structural_mask(X, bs)
    Xt, _, _ = truncate(X, M, beta, TRUNC_FROB, bs)
    return Xt


def subspace_correction(F, D, X_seq, p, alpha, lmin, lmax, *, rounds=1, purify=2, beta=0.0, tau_purify=0.0,
                        trunc_norm=TRUNC_FROBINF, coarse_bs=4096, bs=BS, purify_form="sp2"):
    """First-order correction of the occupied subspace of a near-projector D,
    for expansions whose squares ran in low precision: the paper notes (section
    "Error control") that an error in the occupied subspace made by one
    iteration is not removed by later ones, so finishing in FP64 restores
    idempotency and trace but keeps the subspace error.

    With D = theta + E, E occupied-virtual, Delta = [D, [D, F]] =
    D F (I - D) + (I - D) F D has occupied-virtual part (lambda_v - lambda_o)
    E_ov in the eigenbasis of F; the derivative J of the map F -> theta(mu I - F)
    divides that part by (lambda_o - lambda_v) (first-order perturbation of a
    spectral projector), so D + J Delta = theta + O(||E||^2).  J is applied as
    the derivative of the run's own polynomial steps along its iterates
    X_seq = [X~_0, ..., X~_{n-1}] with polynomials p[1..n], alpha[1..n]:
        dX~_0 = -Delta / (lmax - lmin),
        p = 1: dX_i = a (Y dX~ + dX~ Y), Y = (1 - a) I + a X~_{i-1},
        p = 0: dX_i = 2 a dX~ - a^2 (X~_{i-1} dX~ + dX~ X~_{i-1}),
    without the run's masks.  C = [D, F], Delta and every dX_i lose their
    smallest blocks within the Frobenius budget ``beta`` (0 = keep all).  Then
    ``purify`` FP64 steps restore idempotency, each truncated with tau_purify
    in ``trunc_norm``: X^2, 2X - X^2, ... (``purify_form="sp2"``) or McWeeny's
    3X^2 - 2X^3 (``"mcweeny"``), which maps every eigenvalue x to
    3x^2 - 2x^3 and so moves both clusters toward 0 and 1 quadratically in one
    step.  Returns (D, info) with the norms of Delta and of the correction of
    the last round."""
    F = np.asarray(F, dtype=np.float64)
    D = np.asarray(D, dtype=np.float64)
    w = lmax - lmin
    n = len(X_seq)
    info = {}
    for _ in range(rounds):
        C = _drop_small_blocks(D @ F - F @ D, beta, bs)
        Delta = D @ C - C @ D
        dX = _drop_small_blocks(-Delta / w, beta, bs)
        for i in range(n):
            a = alpha[i + 1]
            Xt = X_seq[i]
            if p[i + 1] == 1:
                Y = (1.0 - a) * np.eye(D.shape[0]) + a * Xt
                dX = a * (Y @ dX + dX @ Y)
            else:
                dX = 2.0 * a * dX - a * a * (Xt @ dX + dX @ Xt)
            dX = _drop_small_blocks(dX, beta, bs)
        info = {"delta_norm": frobenius_norm(Delta), "step_norm": frobenius_norm(dX)}
        P = D + dX
        M = structural_mask(P, bs)
        M[np.arange(M.shape[0]), np.arange(M.shape[0])] = True
        for k in range(purify):
            if purify_form == "mcweeny":
                S = P @ P
                X = 3.0 * S - 2.0 * (P @ S)
                M2 = pattern_square(M)
                MX = (M.astype(np.int64) @ M2.astype(np.int64)) > 0
            elif purify_form == "sp2":
                X = P @ P if k % 2 == 0 else 2.0 * P - P @ P
                MX = pattern_square(M)
            else:
                raise OracleError(f"unknown purification {purify_form!r}")
            P, M, _ = truncate(X, MX, tau_purify, trunc_norm, bs, coarse_bs)
        D = P
    return D, info


# ==========================================================================
# general (full-pattern) storage
# ==========================================================================

def general_pattern(MA, MB, MG=None, diag=False):
    """Block pattern of a product A B of general (not necessarily symmetric)
    matrices: (I, J) is present when some K has A's block (I, K) and B's block
    (K, J) present.  The pattern MG of an added matrix and, with ``diag``, the
    diagonal blocks are joined to it."""
    P = (np.asarray(MA, dtype=np.int64) @ np.asarray(MB, dtype=np.int64)) > 0
    if MG is not None:
        P = P | np.asarray(MG, dtype=bool)
    if diag:
        P = P | np.eye(P.shape[0], dtype=bool)
    return P


def general_product(A, MA, B, MB, G=None, MG=None, a=0.0, b=0.0, c=1.0, bs=BS):
    """out = a I + b G + c A B on the block pattern of ``general_pattern``
    (the diagonal joined when a != 0), for matrices in general storage (every
    present block of both triangles stored; the general matrix wrapper of
    section "Implementation details", which section "Numerical experiments"
    compares with the symmetric one).  A, B, G are dense; MA, MB, MG their
    block masks (blocks outside a mask are taken as zero).  Returns
    (out, P, sums) with sums = [||G - A B||_F^2, tr G, tr(A B), flops], where
    flops = 2 bs^3 per block triple (I, K, J) with (I, K) in MA and (K, J) in
    MB."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    Am = A * expand_mask(MA, n, bs)
    Bm = np.asarray(B, dtype=np.float64) * expand_mask(MB, n, bs)
    if G is None:
        Gm = np.zeros((n, n))
    else:
        Gm = np.asarray(G, dtype=np.float64) * expand_mask(MG, n, bs)
    P = general_pattern(MA, MB, MG if G is not None else None, diag=(a != 0.0))
    S = Am @ Bm
    out = (a * np.eye(n) + b * Gm + c * S) * expand_mask(P, n, bs)
    triples = int((np.asarray(MA, dtype=np.int64) @ np.asarray(MB, dtype=np.int64)).sum())
    sums = [frobenius_norm(Gm - S) ** 2, float(np.trace(Gm)), float(np.trace(S)), 2.0 * bs ** 3 * triples]
    return out, P, sums


# ==========================================================================
# diagnostics
# ==========================================================================

def diagnostics(D, F, n_occ):
    """||D^2 - D||_F, |tr D - n_occ| and ||F D - D F||_F."""
    return {
        "idempotency": frobenius_norm(D @ D - D),
        "trace_err": abs(float(np.trace(D)) - n_occ),
        "commutator": frobenius_norm(F @ D - D @ F),
    }
