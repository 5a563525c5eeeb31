"""Python binding of ``libsp2dm.so``: argument marshalling only.

Every step of the density-matrix expansion runs inside the HIP library; this
module moves pointers and sizes across the C ABI (``include/sp2dm.h``).
PyTorch supplies device memory (its caching allocator is installed as the
library's allocator) and the stream.  There is no CPU fallback: every call
raises when the library or a GPU is missing.
"""
from __future__ import annotations

import ctypes as C
import math
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _lib as L

_PREC = {"fp64": L.PREC_FP64, "fp32": L.PREC_FP32, "bf16x3": L.PREC_BF16X3}
_PREC_NAME = {v: k for k, v in _PREC.items()}
_NORM = {"none": L.TRUNC_NONE, "frob": L.TRUNC_FROB, "frobinf": L.TRUNC_FROBINF}
_STOP = {L.STOP_CRITERION: "criterion", L.STOP_IDEMPOTENCY: "idempotency", L.STOP_NMAX: "n_max",
         L.STOP_NOISE_FLOOR: "noise_floor", 0: ""}


class Sp2Error(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"sp2 error {code}: {msg}")
        self.code = code


def load_library():
    lib = L.load()
    if not torch.cuda.is_available():
        raise RuntimeError("libsp2dm needs a ROCm GPU; none is visible")
    return lib


# --------------------------------------------------------------------------
# matrices
# --------------------------------------------------------------------------

class BsrMatrix:
    """Upper-BSR matrix in device memory (64 x 64 blocks, see sp2dm.h)."""

    def __init__(self, n, row_ptr, col_idx, val):
        self.n = int(n)
        self.nbr = (self.n + 63) // 64
        self.row_ptr = row_ptr
        self.col_idx = col_idx
        self.val = val
        assert row_ptr.dtype == torch.int64 and col_idx.dtype == torch.int32 and val.dtype == torch.float64
        assert row_ptr.is_contiguous() and col_idx.is_contiguous() and val.is_contiguous()
        assert row_ptr.numel() == self.nbr + 1 and val.shape == (col_idx.numel(), 64, 64)

    @property
    def nnzb(self):
        return int(self.col_idx.numel())

    @property
    def device(self):
        return self.val.device

    @classmethod
    def from_host(cls, M, device="cuda"):
        """From any object with numpy fields n, row_ptr, col_idx, val."""
        return cls(M.n,
                   torch.as_tensor(np.ascontiguousarray(M.row_ptr, dtype=np.int64)).to(device),
                   torch.as_tensor(np.ascontiguousarray(M.col_idx, dtype=np.int32)).to(device),
                   torch.as_tensor(np.ascontiguousarray(M.val, dtype=np.float64)).to(device))

    def to_host(self):
        """(n, row_ptr, col_idx, val) as numpy arrays."""
        return (self.n, self.row_ptr.cpu().numpy(), self.col_idx.cpu().numpy(), self.val.cpu().numpy())

    def _struct(self):
        s = L.sp2_bsr()
        s.n = self.n
        s.bs = 64
        s.owned = 0
        s.nbr = self.nbr
        s.nnzb = self.nnzb
        s.row_ptr = self.row_ptr.data_ptr()
        s.col_idx = self.col_idx.data_ptr() if self.nnzb else None
        s.val = self.val.data_ptr() if self.nnzb else None
        return s


# --------------------------------------------------------------------------
# context
# --------------------------------------------------------------------------

class Context:
    """An sp2 context on one device and stream; device memory comes from
    PyTorch's caching allocator."""

    def __init__(self, device=None, stream=None, torch_allocator=True):
        self.lib = load_library()
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        rc = self.lib.sp2_create(C.byref(h), self.device.index, C.c_void_p(self.stream.cuda_stream))
        if rc != 0:
            raise Sp2Error(rc, "sp2_create failed")
        self.h = h
        self._cb = None
        if torch_allocator:
            dev, stream = self.device.index, self.stream
            hip = _hip_runtime()
            big = set()  # pointers from hipMalloc

            def _hip_malloc(nbytes):
                p = C.c_void_p()
                hip.hipSetDevice(dev)
                if hip.hipMalloc(C.byref(p), C.c_size_t(int(nbytes))) != 0 or not p.value:
                    return None
                big.add(p.value)
                return p.value

            def _alloc(nbytes, user):
                # matrix pools (hundreds of MB to tens of GB) bypass the caching
                # allocator, whose split segments could not serve the next large
                # request; small buffers reuse PyTorch's cache
                if nbytes >= _BIG_ALLOC:
                    p = _hip_malloc(nbytes)
                    if p is None:
                        torch.cuda.synchronize(dev)
                        torch.cuda.empty_cache()
                        p = _hip_malloc(nbytes)
                    return p
                try:
                    return torch.cuda.caching_allocator_alloc(int(nbytes), device=dev, stream=stream)
                except Exception:
                    pass
                try:
                    torch.cuda.synchronize(dev)
                    torch.cuda.empty_cache()
                    return torch.cuda.caching_allocator_alloc(int(nbytes), device=dev, stream=stream)
                except Exception:
                    return None

            def _free(ptr, user):
                if ptr in big:
                    big.discard(ptr)
                    hip.hipFree(C.c_void_p(ptr))  # waits for the device work that may use it
                else:
                    torch.cuda.caching_allocator_delete(ptr)

            self._cb = (L.ALLOC_FN(_alloc), L.FREE_FN(_free))
            self._check(self.lib.sp2_set_allocator(self.h, self._cb[0], self._cb[1], None))

    def _check(self, rc, allow_warn=True):
        if rc < 0 or (rc > 0 and not allow_warn):
            msg = self.lib.sp2_last_error(self.h).decode()
            raise Sp2Error(rc, msg)
        return rc

    def trim(self):
        self.lib.sp2_trim(self.h)

    def close(self):
        if getattr(self, "h", None):
            self.lib.sp2_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def take(self, ptr):
        """Copy a library-owned matrix into torch tensors and free it (the
        library's cached buffers are released first, to make room)."""
        self.lib.sp2_trim(self.h)
        m = ptr.contents
        n, nbr, nnzb = int(m.n), int(m.nbr), int(m.nnzb)
        row_ptr = torch.empty(nbr + 1, dtype=torch.int64, device=self.device)
        col_idx = torch.empty(nnzb, dtype=torch.int32, device=self.device)
        val = torch.empty((nnzb, 64, 64), dtype=torch.float64, device=self.device)
        try:
            self._check(self.lib.sp2_bsr_copy(self.h, ptr, row_ptr.data_ptr(),
                                              col_idx.data_ptr() if nnzb else None,
                                              val.data_ptr() if nnzb else None))
        finally:
            self.lib.sp2_bsr_free(self.h, ptr)
        return BsrMatrix(n, row_ptr, col_idx, val)


_CTX = {}

_BIG_ALLOC = 256 << 20
_HIP = None


def _hip_runtime():
    """The HIP runtime PyTorch already loaded (hipMalloc / hipFree for large
    library buffers)."""
    global _HIP
    if _HIP is None:
        for name in ("libamdhip64.so", "libamdhip64.so.7", "/opt/rocm/lib/libamdhip64.so"):
            try:
                lib = C.CDLL(name)
                break
            except OSError:
                lib = None
        if lib is None:
            raise RuntimeError("HIP runtime library not found")
        lib.hipMalloc.restype = C.c_int
        lib.hipMalloc.argtypes = [C.POINTER(C.c_void_p), C.c_size_t]
        lib.hipFree.restype = C.c_int
        lib.hipFree.argtypes = [C.c_void_p]
        lib.hipSetDevice.restype = C.c_int
        lib.hipSetDevice.argtypes = [C.c_int]
        _HIP = lib
    return _HIP


def context(device=None) -> Context:
    dev = torch.cuda.current_device() if device is None else int(device)
    stream = torch.cuda.current_stream(dev)
    key = (dev, stream.cuda_stream)
    if key not in _CTX:
        _CTX[key] = Context(dev, stream)
    return _CTX[key]


# --------------------------------------------------------------------------
# entry points
# --------------------------------------------------------------------------

def gershgorin(F: BsrMatrix, ctx: Context | None = None):
    """Gershgorin bounds (lmin, lmax) of F."""
    ctx = ctx or context(F.device.index)
    lo, hi = C.c_double(), C.c_double()
    s = F._struct()
    ctx._check(ctx.lib.sp2_gershgorin(ctx.h, C.byref(s), C.byref(lo), C.byref(hi)))
    return lo.value, hi.value


def options(**kw):
    o = L.sp2_options()
    L.load().sp2_options_default(C.byref(o))
    for k, v in kw.items():
        if k in ("precision", "adjoint_precision"):
            v = _PREC[v] if isinstance(v, str) else int(v)
        elif k == "trunc_norm":
            v = _NORM[v] if isinstance(v, str) else int(v)
        elif k == "accel":
            v = int(bool(v))
        elif k == "record_tape":
            v = int(bool(v))
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


@dataclass
class DensityResult:
    D: BsrMatrix
    status: int
    homo_est: float
    lumo_est: float
    n_iter: int
    n_max: int
    n_min: int
    stop_reason: str
    switch_iter: int
    subspace_err_bound: float
    time_s: float
    alg_flops: float
    max_nnzb: int
    square_time_s: float = 0.0
    correction: dict = field(default_factory=dict)
    iters: dict = field(default_factory=dict)
    tape: "Tape | None" = None


class Tape:
    """Recorded forward run (schedule, masks, checkpoints) for the adjoint."""

    def __init__(self, ctx: Context, h):
        self.ctx = ctx
        self.h = h

    def info(self):
        n, k, b = C.c_int32(), C.c_int32(), C.c_int64()
        self.ctx._check(self.ctx.lib.sp2_tape_info(self.h, C.byref(n), C.byref(k), C.byref(b)))
        return {"n_iter": n.value, "n_checkpoints": k.value, "device_bytes": b.value}

    def _call(self, fn, M: BsrMatrix):
        out = C.POINTER(L.sp2_bsr)()
        s = M._struct()
        self.ctx._check(fn(self.ctx.h, self.h, C.byref(s), C.byref(out)))
        r = self.ctx.take(out)
        self.ctx.trim()
        return r

    def vjp(self, W: BsrMatrix) -> BsrMatrix:
        """dL/dF for L = tr(W D) (W symmetric)."""
        return self._call(self.ctx.lib.sp2_vjp, W)

    def jvp(self, dF: BsrMatrix) -> BsrMatrix:
        return self._call(self.ctx.lib.sp2_jvp, dF)

    def replay(self, F: BsrMatrix) -> BsrMatrix:
        return self._call(self.ctx.lib.sp2_replay, F)

    def free(self):
        if self.h:
            self.ctx.lib.sp2_tape_free(self.ctx.h, self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class _Stats:
    """Host arrays of an sp2_stats record and the DensityResult built from it."""

    _DOUBLE = ("e", "t", "trace", "alpha", "tau", "trunc_err_frob", "trunc_err_mixed", "iter_time_s", "iter_flops",
               "square_time_s")

    def __init__(self, n_max_cap):
        cap = int(n_max_cap) + 1
        self.arr = {k: np.zeros(cap) for k in self._DOUBLE}
        self.arr_p = np.zeros(cap, dtype=np.int32)
        self.arr_prec = np.zeros(cap, dtype=np.int32)
        self.arr_nnzb = np.zeros(cap, dtype=np.int64)
        st = L.sp2_stats()
        st.capacity = cap
        for k, a in self.arr.items():
            setattr(st, k, a.ctypes.data_as(C.POINTER(C.c_double)))
        st.p = self.arr_p.ctypes.data_as(C.POINTER(C.c_int32))
        st.precision = self.arr_prec.ctypes.data_as(C.POINTER(C.c_int32))
        st.nnzb = self.arr_nnzb.ctypes.data_as(C.POINTER(C.c_int64))
        self.st = st

    def result(self, ctx, rc, D, he, le, tape_h, record_tape):
        st = self.st
        n = int(st.n_iter)
        iters = {k: a[: n + 1].copy() for k, a in self.arr.items()}
        iters["p"] = self.arr_p[: n + 1].copy()
        iters["precision"] = self.arr_prec[: n + 1].copy()
        iters["nnzb"] = self.arr_nnzb[: n + 1].copy()
        return DensityResult(D=D, status=rc, homo_est=he, lumo_est=le, n_iter=n, n_max=int(st.n_max),
                             n_min=int(st.n_min), stop_reason=_STOP.get(int(st.stop_reason), "?"),
                             switch_iter=int(st.switch_iter), subspace_err_bound=float(st.subspace_err_bound),
                             time_s=float(st.time_s), alg_flops=float(st.alg_flops), max_nnzb=int(st.max_nnzb),
                             square_time_s=float(st.square_time_total_s),
                             correction={k: getattr(st, k) for k in ("corr_rounds", "corr_time_s", "corr_flops",
                                                                     "corr_delta_norm", "corr_step_norm",
                                                                     "corr_e_last", "corr_max_nnzb", "seq_bytes",
                                                                     "seq_host_bytes", "corr_recomputed",
                                                                     "device_peak_bytes")},
                             iters=iters, tape=Tape(ctx, tape_h) if record_tape else None)


def _bounds(homo_ub, lumo_lb):
    hub = C.byref(C.c_double(homo_ub)) if homo_ub is not None else None
    llb = C.byref(C.c_double(lumo_lb)) if lumo_lb is not None else None
    return hub, llb


def density(F: BsrMatrix, n_occ: int, lmin: float, lmax: float, homo_ub=None, lumo_lb=None,
            ctx: Context | None = None, **opts) -> DensityResult:
    """D = theta(mu I - F) by SP2 / SP2ACC; see sp2_density in sp2dm.h."""
    ctx = ctx or context(F.device.index)
    o = options(**opts)
    sts = _Stats(o.n_max_cap)
    hub, llb = _bounds(homo_ub, lumo_lb)
    out = C.POINTER(L.sp2_bsr)()
    he, le = C.c_double(), C.c_double()
    tape_h = C.c_void_p()
    s = F._struct()
    rc = ctx.lib.sp2_density(ctx.h, C.byref(s), int(n_occ), float(lmin), float(lmax), hub, llb, C.byref(o),
                             C.byref(out), C.byref(he), C.byref(le), C.byref(sts.st),
                             C.byref(tape_h) if o.record_tape else None)
    ctx._check(rc)
    D = ctx.take(out)
    ctx.trim()
    return sts.result(ctx, rc, D, he.value, le.value, tape_h, o.record_tape)


class Solver:
    """The expansion one unit of work at a time (sp2_density_begin / _step /
    _end in sp2dm.h): ``step()`` runs one iteration of Algorithm 2, or one
    product of the subspace correction."""

    def __init__(self, F: BsrMatrix, n_occ: int, lmin: float, lmax: float, homo_ub=None, lumo_lb=None,
                 ctx: Context | None = None, **opts):
        self.ctx = ctx or context(F.device.index)
        self.F = F  # borrowed by the library until end()
        self.o = options(**opts)
        self._s = F._struct()
        hub, llb = _bounds(homo_ub, lumo_lb)
        self.h = C.c_void_p()
        self.ctx._check(self.ctx.lib.sp2_density_begin(self.ctx.h, C.byref(self._s), int(n_occ), float(lmin),
                                                       float(lmax), hub, llb, C.byref(self.o), C.byref(self.h)))
        self.done = False

    def step(self) -> dict:
        """One step; returns its sp2_step_info as a dict (done, kind, iteration,
        precision, flops, wall_s, kernel_s[3], kernel_flops[3])."""
        info = L.sp2_step_info()
        self.ctx._check(self.ctx.lib.sp2_density_step(self.ctx.h, self.h, C.byref(info)))
        self.done = bool(info.done)
        return {"done": self.done, "kind": {L.STEP_ITERATION: "iteration", L.STEP_CORRECTION: "correction"}[info.kind],
                "iteration": int(info.iteration), "precision": _PREC_NAME[int(info.precision)],
                "flops": float(info.flops), "wall_s": float(info.wall_s), "kernel_s": list(info.kernel_s),
                "kernel_flops": list(info.kernel_flops), "kernel_launches": list(info.kernel_launches)}

    def end(self) -> DensityResult:
        sts = _Stats(self.o.n_max_cap)
        out = C.POINTER(L.sp2_bsr)()
        he, le = C.c_double(), C.c_double()
        tape_h = C.c_void_p()
        rc = self.ctx.lib.sp2_density_end(self.ctx.h, self.h, C.byref(out), C.byref(he), C.byref(le),
                                          C.byref(sts.st), C.byref(tape_h) if self.o.record_tape else None)
        self.ctx._check(rc)
        D = self.ctx.take(out)
        self.free()
        self.ctx.trim()
        return sts.result(self.ctx, rc, D, he.value, le.value, tape_h, self.o.record_tape)

    def free(self):
        if self.h:
            self.ctx.lib.sp2_solver_free(self.ctx.h, self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def square_step(X: BsrMatrix, a: float, b: float, c: float, precision="fp64", ctx: Context | None = None):
    """One square of Algorithm 2: returns (a I + b X + c X^2 on the pattern of
    X^2, [||X - X^2||_F^2, tr X, tr X^2, flops])."""
    ctx = ctx or context(X.device.index)
    out = C.POINTER(L.sp2_bsr)()
    sums = (C.c_double * 4)()
    s = X._struct()
    p = _PREC[precision] if isinstance(precision, str) else int(precision)
    ctx._check(ctx.lib.sp2_square_step(ctx.h, C.byref(s), float(a), float(b), float(c), p, C.byref(out), sums))
    r = ctx.take(out)
    ctx.trim()
    return r, list(sums)


def pair_product(X: BsrMatrix, Y: BsrMatrix, G: BsrMatrix | None = None, sign=1, y_antisym=False, a=0.0, b=0.0,
                 c=1.0, precision="fp64", ctx: Context | None = None):
    """a I + b G + c (X Y + sign Y X) on the block pattern of X Y + Y X;
    returns (out, [||out||_F^2, flops]); see sp2_pair_product in sp2dm.h."""
    ctx = ctx or context(X.device.index)
    out = C.POINTER(L.sp2_bsr)()
    sums = (C.c_double * 2)()
    sx, sy = X._struct(), Y._struct()
    sg = G._struct() if G is not None else None
    p = _PREC[precision] if isinstance(precision, str) else int(precision)
    ctx._check(ctx.lib.sp2_pair_product(ctx.h, C.byref(sx), C.byref(sy), C.byref(sg) if sg is not None else None,
                                        int(sign), int(bool(y_antisym)), float(a), float(b), float(c), p,
                                        C.byref(out), sums))
    r = ctx.take(out)
    ctx.trim()
    return r, list(sums)


def general_from_upper(U: BsrMatrix, ctx: Context | None = None):
    """General (full-pattern) storage of the symmetric matrix held by the
    upper-BSR U; see sp2_general_from_upper in sp2dm.h."""
    ctx = ctx or context(U.device.index)
    out = C.POINTER(L.sp2_bsr)()
    s = U._struct()
    ctx._check(ctx.lib.sp2_general_from_upper(ctx.h, C.byref(s), C.byref(out)))
    r = ctx.take(out)
    ctx.trim()
    return r


def general_product(A: BsrMatrix, B: BsrMatrix, G: BsrMatrix | None = None, a=0.0, b=0.0, c=1.0, precision="fp64",
                    ctx: Context | None = None):
    """a I + b G + c A B for matrices in general storage, on the block
    pattern of A B (joined with G's, and the diagonal when a != 0); returns
    (out, [||G - A B||_F^2, tr G, tr A B, flops]); see sp2_general_product in
    sp2dm.h."""
    ctx = ctx or context(A.device.index)
    out = C.POINTER(L.sp2_bsr)()
    sums = (C.c_double * 4)()
    sa, sb = A._struct(), B._struct()
    sg = G._struct() if G is not None else None
    p = _PREC[precision] if isinstance(precision, str) else int(precision)
    ctx._check(ctx.lib.sp2_general_product(ctx.h, C.byref(sa), C.byref(sb), C.byref(sg) if sg is not None else None,
                                           float(a), float(b), float(c), p, C.byref(out), sums))
    r = ctx.take(out)
    ctx.trim()
    return r, list(sums)


def matrix_norms(A: BsrMatrix, coarse_bs=4096, ctx: Context | None = None):
    """(||A||_F, ||A||_M) of the symmetric matrix held by A's upper blocks;
    ||A||_M is the Frob-Inf norm with coarse_bs x coarse_bs submatrices."""
    ctx = ctx or context(A.device.index)
    f, m = C.c_double(), C.c_double()
    s = A._struct()
    ctx._check(ctx.lib.sp2_matrix_norms(ctx.h, C.byref(s), int(coarse_bs), C.byref(f), C.byref(m)))
    ctx.trim()
    return f.value, m.value


def matrix_norms_noalloc(A: BsrMatrix, coarse_bs=4096, ctx: Context | None = None):
    """matrix_norms through sp2_matrix_norms_noalloc: no device allocation,
    the library's fixed device scratch array instead."""
    ctx = ctx or context(A.device.index)
    f, m = C.c_double(), C.c_double()
    s = A._struct()
    ctx._check(ctx.lib.sp2_matrix_norms_noalloc(ctx.h, C.byref(s), int(coarse_bs), C.byref(f), C.byref(m)))
    return f.value, m.value


def truncate(X: BsrMatrix, tau: float, norm="frobinf", coarse_bs=4096, ctx: Context | None = None):
    """Truncation with ||E|| <= tau; returns (X~, (||E||_F, ||E||_M))."""
    ctx = ctx or context(X.device.index)
    out = C.POINTER(L.sp2_bsr)()
    err = (C.c_double * 2)()
    s = X._struct()
    nm = _NORM[norm] if isinstance(norm, str) else int(norm)
    ctx._check(ctx.lib.sp2_truncate(ctx.h, C.byref(s), float(tau), nm, int(coarse_bs), C.byref(out), err))
    r = ctx.take(out)
    ctx.trim()
    return r, (err[0], err[1])
