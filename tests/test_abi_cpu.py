"""CPU checks of the C ABI library (no GPU, no compute calls on a device):

* the shared library loads and exports every function that include/sp2dm.h
  declares, and the Python binding declares the same set;
* the library's host scalar control (Step 1 schedule, Step 3 homo/lumo
  estimates) equals the oracle's independent implementation bit for bit on a
  sweep of bounds, and rejects inconsistent bounds.
"""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

from fockgen import bsr_to_dense, dense_spectrum, lattice_fock
from oracle import sp2_oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_1909_12533_amd import _lib

    if not os.path.exists(_lib.LIB_PATH):  # build only when nothing is built
        from paper_1909_12533_amd import build

        build.build(verbose=False)
    return _lib.load()


def _header_functions():
    text = open(os.path.join(ROOT, "include", "sp2dm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sp2_[a-z_0-9]+)\s*\(", text)) - {"sp2_alloc_fn", "sp2_free_fn"})


def test_exports_match_header(lib):
    from paper_1909_12533_amd import _lib

    declared = _header_functions()
    assert len(declared) >= 20
    for name in declared:
        assert hasattr(lib, name), f"{name} declared in sp2dm.h but not exported"
    assert sorted(_lib.EXPORTS) == declared
    assert lib.sp2_version().startswith(b"sp2dm")


def _c_schedule(lib, lmin, lmax, h, lu, accel, gamma=0.0, tau=0.0, cap=100):
    n = cap + 1
    nmax, nmin = C.c_int32(), C.c_int32()
    p = (C.c_int32 * n)()
    arrs = [(C.c_double * n)() for _ in range(5)]
    rc = lib.sp2_schedule(lmin, lmax, h, lu, int(accel), gamma, tau, cap, C.byref(nmax), C.byref(nmin), p, *arrs)
    if rc != 0:
        return rc, None
    k = nmax.value + 1
    return rc, dict(n_max=nmax.value, n_min=nmin.value, p=list(p[:k]),
                    alpha=list(arrs[0][:k]), l=list(arrs[1][:k]), q=list(arrs[2][:k]),
                    xi=list(arrs[3][:k]), tau=list(arrs[4][:k]))


@pytest.mark.parametrize("accel", [False, True])
def test_schedule_bitwise_vs_oracle(lib, accel):
    rng = np.random.default_rng(0)
    cases = [(-1.0, 1.0, -0.1, 0.1), (-1.0, 1.0, -0.2, 0.15), (-12.4, 12.3, -0.22, 0.23)]
    for _ in range(60):
        lmin, lmax = -rng.uniform(0.5, 20), rng.uniform(0.5, 20)
        a, b = np.sort(rng.uniform(lmin, lmax, 2))
        if b - a < 1e-4:
            continue
        cases.append((lmin, lmax, a, b))
    for lmin, lmax, h, lu in cases:
        for gamma, tau in ((1e-3, 0.0), (0.0, 1e-6)):
            rc, c = _c_schedule(lib, lmin, lmax, h, lu, accel, gamma, tau)
            assert rc == 0
            s = O.schedule(lmin, lmax, h, lu, accel=accel, gamma=gamma, tau_fixed=tau)
            assert c["n_max"] == s.n_max and c["n_min"] == s.n_min
            assert c["p"] == s.p and c["alpha"] == s.alpha
            assert c["l"] == s.l and c["q"] == s.q and c["xi"] == s.xi and c["tau"] == s.tau


def test_schedule_rejects_bad_bounds(lib):
    assert _c_schedule(lib, -1.0, 1.0, 0.2, 0.1, True)[0] == -2
    assert _c_schedule(lib, -1.0, 1.0, -1.5, 0.1, True)[0] == -2
    assert _c_schedule(lib, 1.0, -1.0, -0.1, 0.1, True)[0] == -1
    assert _c_schedule(lib, -1.0, 1.0, -0.1, 0.1, True, cap=0)[0] == -1


def _c_homo_lumo(lib, res, N):
    n = res.n
    dp = lambda v: (C.c_double * len(v))(*v)  # noqa: E731
    s = res.sched
    bounds = s.mode == "bounds"
    h, lu = C.c_double(), C.c_double()
    rc = lib.sp2_homo_lumo(int(bounds), n, dp(res.e[: n + 1]), dp(res.trX[: n + 1]),
                           (C.c_int32 * (n + 1))(*res.p[: n + 1]), dp(res.alpha[: n + 1]),
                           dp(s.l[: n + 1]) if bounds else None, dp(s.q[: n + 1]) if bounds else None,
                           res.lmin, res.lmax, N, res.n_occ, C.byref(h), C.byref(lu))
    assert rc == 0
    return h.value, lu.value


def _same(a, b):
    return (math.isnan(a) and math.isnan(b)) or a == b


@pytest.mark.parametrize("accel", [False, True])
def test_homo_lumo_bitwise_vs_oracle_dense(lib, accel):
    F, lam, _ = dense_spectrum(256, seed=4)
    r = O.sp2(F, 128, -1.0, 1.0, -0.1, 0.1, accel=accel, trunc_norm=O.TRUNC_NONE, idem_stop=1e-12)
    h, lu = _c_homo_lumo(lib, r, 256)
    assert _same(h, r.homo_ub_est) and _same(lu, r.lumo_lb_est)
    assert not math.isnan(h)


def test_homo_lumo_bitwise_vs_oracle_trace_correcting(lib):
    Fh, info = lattice_fock(4, seed=1)
    F = bsr_to_dense(Fh)
    lmin, lmax = O.gershgorin_bounds(F)
    r = O.sp2(F, info["n_occ"], lmin, lmax, trunc_norm=O.TRUNC_NONE)
    h, lu = _c_homo_lumo(lib, r, F.shape[0])
    assert _same(h, r.homo_ub_est) and _same(lu, r.lumo_lb_est)
