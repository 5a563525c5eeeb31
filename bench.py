"""Benchmark of the SP2 / SP2ACC density-matrix hot path on one MI355X.

Workload (default): the tight-binding Fock matrix on a 30 x 30 x 30 lattice
with 4 basis functions per atom (N = 108,000), SP2ACC with 64 x 64 leaf
blocks, tau = 1e-6 (Frob-Inf truncation, 4096 submatrices), Gershgorin
spectral bounds, homo/lumo bounds from the trace-correcting first run of the
two-run protocol of the paper's "Numerical experiments" section (its result
is recorded in bench_run1.json).  The timed path is the mixed-precision one:
BF16x3 squares to the expansion's own stopping criterion, then the FP64
occupied-subspace correction; the plain FP64 expansion of the same input is
run once beside it as the reference (time to D and ||D - D_FP64||_F).

One step = one unit of the stepped C ABI (sp2_density_step): one iteration
of Algorithm 2 (planning, MFMA square with the fused update, e_i and t_i,
the stopping test, truncation) or one block product of the correction; the
first step of a solve also runs Step 1 and Algorithm 1, its last Step 3 and
the export of D.  Solves run back to back; W untimed steps, then K timed
steps; every step is synchronized and timed on its own, so the time to D of
a solve is the sum of its steps.  Inputs are resident in HBM before timing.

Prints one JSON line: value = block-sparse TFLOP/s of a solve (the
expansion's algorithmic flops 2 * 64^3 * #{(I,K,J): I <= J, X~_IK != 0 !=
X~_KJ} over its time to D), the time to D, the roofline of the dominant MFMA
kernel over the timed steps (device time from HIP events on the stream it
runs on), the FP64 reference and the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0 / 3.0}  # dense MFMA TFLOP/s (algorithmic for bf16x3)

CONFIGS = {
    "c1": dict(L=20, tau=1e-6),
    "c2": dict(L=30, tau=1e-6),
    "c4": dict(L=40, tau=1e-5),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(L=12, tau=1e-6):
    """The CPU oracle (dense FP64 NumPy, unchanged) on a bounded sample: one
    SP2ACC run on the 12 x 12 x 12 lattice (N = 6912) of the same generator
    and options, with homo/lumo bounds from diagonalisation widened by 1% of
    the gap."""
    import numpy as np
    from threadpoolctl import threadpool_info

    from fockgen import bsr_to_dense, lattice_fock
    from oracle import sp2_oracle as O

    Fh, info = lattice_fock(L, seed=0)
    Fd = bsr_to_dense(Fh)
    no = info["n_occ"]
    lam = np.linalg.eigvalsh(Fd)
    gap = lam[no] - lam[no - 1]
    h, lu = lam[no - 1] + 0.01 * gap, lam[no] - 0.01 * gap
    lmin, lmax = O.gershgorin_bounds(Fd)
    t0 = time.perf_counter()
    r = O.sp2(Fd, no, lmin, lmax, h, lu, accel=True, trunc_norm=O.TRUNC_FROBINF, tau_fixed=tau, coarse_bs=4096)
    dt = time.perf_counter() - t0
    blas = [p for p in threadpool_info() if p.get("user_api") == "blas"]
    threads = max([p.get("num_threads", 1) for p in blas] or [1])
    return {
        "value": r.alg_flops / dt / 1e12,
        "unit": "TFLOP/s",
        "cores": int(threads),
        "kind": "oracle",
        "sample": f"one SP2ACC run (tau={tau}, Frob-Inf) of the {L}x{L}x{L}x4 lattice, N={info['n']}, "
                  f"n={r.n} iterations, {dt:.1f} s, algorithmic block-sparse flops / wall time",
        "host_cpu_count": os.cpu_count(),
        "blas": [f"{p.get('internal_api')} {p.get('version')} ({p.get('num_threads')} threads)" for p in blas],
    }


# dominant kernel of a run in each bulk precision, and the sources it is built from
KERNELS = {
    "fp64": ("k_square_f64_lds", ["paper_1909_12533_amd/csrc/kernels_f64.hip", "paper_1909_12533_amd/csrc/mfma.h"]),
    "fp32": ("k_square_tile", ["paper_1909_12533_amd/csrc/kernels_tile.hip", "paper_1909_12533_amd/csrc/mfma.h"]),
    "bf16x3": ("k_square_tile4_bf16x3", ["paper_1909_12533_amd/csrc/kernels_bf16x3.hip",
                                          "paper_1909_12533_amd/csrc/mfma.h"]),
}


def kernel_source_hash(prec="fp64"):
    import hashlib

    h = hashlib.sha256()
    root = os.path.dirname(os.path.abspath(__file__))
    for f in KERNELS[prec][1]:
        with open(os.path.join(root, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic_per_launch(prec, L):
    """HBM bytes per launch of the run's dominant square kernel from the
    committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary of this workload, each
    counter scaled by what it read for a 1 GiB device copy in the same run;
    None when there is no summary for this kernel and workload or the kernel
    sources changed since the counters were taken."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                        f"{KERNELS[prec][0]}_{prec}_lattice{L}_pmc.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            parts = line.split()
            if len(parts) == 2 and not line.startswith("#"):
                kv[parts[0]] = parts[1]
    if kv.get("source_sha256") != kernel_source_hash(prec):
        return None
    kib = float(kv["fetch_kib_per_launch"]) * float(kv["fetch_factor"]) + \
        float(kv["write_kib_per_launch"]) * float(kv["write_factor"])
    return round(kib * 1024.0)


def bsr_diff_frobenius(A, B):
    """||A - B||_F of two symmetric upper-BSR device matrices (blocks matched
    by (I, J); off-diagonal blocks count twice for their mirrors)."""
    import torch

    def keys(M):
        rows = torch.repeat_interleave(torch.arange(M.nbr, device=M.device), torch.diff(M.row_ptr))
        return rows, M.col_idx.long(), rows * M.nbr + M.col_idx.long()

    ra, ca, ka = keys(A)
    rb, cb, kb = keys(B)
    pos = torch.searchsorted(kb, ka).clamp(max=max(kb.numel() - 1, 0))
    hit = kb[pos] == ka
    wa = torch.where(ra == ca, 1.0, 2.0).double()
    wb = torch.where(rb == cb, 1.0, 2.0).double()
    tot = torch.zeros((), dtype=torch.float64, device=A.val.device)
    chunk = 1 << 16  # blocks per pass (2 GB of FP64 differences)
    for a in range(0, ka.numel(), chunk):
        sl = slice(a, a + chunk)
        d = A.val[sl].clone()
        h = hit[sl]
        d[h] -= B.val[pos[sl][h]]
        tot += (wa[sl] * (d * d).sum(dim=(1, 2))).sum()
        del d
    used = torch.zeros(kb.numel(), dtype=torch.bool, device=kb.device)
    used[pos[hit]] = True
    rest = torch.nonzero(~used).flatten()
    for a in range(0, rest.numel(), chunk):
        idx = rest[a:a + chunk]
        tot += (wb[idx] * (B.val[idx] ** 2).sum(dim=(1, 2))).sum()
    return float(tot.sqrt())


def bsr_inner(A, B):
    """Frobenius inner product of two symmetric upper-BSR device matrices (whole
    matrices: off-diagonal blocks count twice)."""
    import torch

    def keys(M):
        rows = torch.repeat_interleave(torch.arange(M.nbr, device=M.device), torch.diff(M.row_ptr))
        return rows, rows * M.nbr + M.col_idx.long()

    ra, ka = keys(A)
    rb, kb = keys(B)
    if kb.numel() == 0 or ka.numel() == 0:
        return 0.0
    pos = torch.searchsorted(kb, ka).clamp(max=kb.numel() - 1)
    hit = kb[pos] == ka
    w = torch.where(ra[hit] == A.col_idx.long()[hit], 1.0, 2.0).double()
    return float((w * (A.val[hit] * B.val[pos[hit]]).sum(dim=(1, 2))).sum())


def adjoint_bench(sp2, F, Fh, no, lmin, lmax, hub, llb, opts, precisions):
    """Response dD = J dF and gradient of L = tr(W D) through the hand-written
    adjoint on the workload's F: dF and W random symmetric on F's block pattern
    (entries N(0, 1e-3) and N(0, 1)), sqrt(n) checkpoints of X~_i.  FP64:
    central finite differences of the recorded map (h = 1e-5) and the
    dot-product test; low precision: relative error of J dF and of the gradient
    against the FP64 ones.  Labels "forward/adjoint" run the adjoint steps of
    the low-precision iterations in another arithmetic."""
    import torch

    from fockgen import random_sym_on_pattern

    dFh = random_sym_on_pattern(Fh, 1e-3, seed=1)
    Wh = random_sym_on_pattern(Fh, 1.0, seed=2)
    dF = sp2.BsrMatrix.from_host(dFh, "cuda:0")
    W = sp2.BsrMatrix.from_host(Wh, "cuda:0")
    out = {}
    ref = {}
    for label in precisions:
        head, *extra = label.split("@")
        prec, _, adj = head.partition("/")
        mo = dict(precision=prec, switch_tol=1e-3) if prec != "fp64" else {}
        if adj:
            mo["adjoint_precision"] = adj
        for kv in extra:  # "@low_start_xi=0.3", "@switch_tol=1e-2"
            k, _, v = kv.partition("=")
            mo[k] = float(v)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = sp2.density(F, no, lmin, lmax, hub, llb, record_tape=True, **mo, **opts)
        torch.cuda.synchronize()
        t_fwd = time.perf_counter() - t0
        info = r.tape.info()
        t0 = time.perf_counter()
        g = r.tape.vjp(W)
        torch.cuda.synchronize()
        t_vjp = time.perf_counter() - t0
        t0 = time.perf_counter()
        jv = r.tape.jvp(dF)
        torch.cuda.synchronize()
        t_jvp = time.perf_counter() - t0
        rec = {"n_iter": r.n_iter, "forward_s": round(t_fwd, 4), "vjp_s": round(t_vjp, 4), "jvp_s": round(t_jvp, 4),
               "n_checkpoints": info["n_checkpoints"], "tape_device_bytes": info["device_bytes"],
               "forward_device_peak_bytes": r.correction["device_peak_bytes"],
               "square_precisions": "".join("dsb"[int(k)] for k in r.iters["precision"]),
               "flops_low_frac": float(sum(f for f, k in zip(r.iters["iter_flops"], r.iters["precision"]) if k != 0)
                                       / max(sum(r.iters["iter_flops"]), 1.0))}
        lhs, rhs = bsr_inner(W, jv), bsr_inner(g, dF)
        rec["dot_test_rel"] = abs(lhs - rhs) / max(abs(lhs), 1e-300)
        if prec == "fp64":
            h = 1e-5
            Fp = sp2.BsrMatrix(F.n, F.row_ptr, F.col_idx, (F.val + h * dF.val).contiguous())
            Fm = sp2.BsrMatrix(F.n, F.row_ptr, F.col_idx, (F.val - h * dF.val).contiguous())
            Dp, Dm = r.tape.replay(Fp), r.tape.replay(Fm)
            if not (torch.equal(Dp.row_ptr, jv.row_ptr) and torch.equal(Dp.col_idx, jv.col_idx)):
                raise RuntimeError("replay and JVP patterns differ")
            fd = (Dp.val - Dm.val) / (2 * h)
            num = bsr_diff_frobenius(sp2.BsrMatrix(F.n, Dp.row_ptr, Dp.col_idx, fd.contiguous()), jv)
            rec["fd_rel_err_jvp"] = num / math.sqrt(bsr_inner(jv, jv))
            ref = {"g": g, "jv": jv}
            del Dp, Dm, Fp, Fm, fd
        elif ref:
            rec["grad_rel_err_vs_fp64"] = bsr_diff_frobenius(g, ref["g"]) / math.sqrt(bsr_inner(ref["g"], ref["g"]))
            rec["jvp_rel_err_vs_fp64"] = bsr_diff_frobenius(jv, ref["jv"]) / math.sqrt(bsr_inner(ref["jv"], ref["jv"]))
        log(f"adjoint {label}: {rec}")
        out[label] = rec
        r.tape.free()
        del r
        torch.cuda.empty_cache()
    return out


def storage_bench(sp2, F, no, lmin, lmax, hub, llb, opts, prec):
    """Symmetric vs general storage (the paper's comparison of its symmetric
    and general matrix wrappers, section "Numerical experiments"): the
    workload's expansion is run square by square (the FP64 run's polynomials
    and thresholds); every X~_i is squared both by the symmetric square
    (upper blocks stored and computed) and, after conversion to general
    storage, by the general product a I + b X + c X X (every block of both
    triangles stored and computed).  Reports per-iteration wall time of each
    call (synchronized, planning and allocation included), stored blocks and
    block products, and the totals over the run."""
    import numpy as np
    import torch

    ref = sp2.density(F, no, lmin, lmax, hub, llb, **opts)
    it = ref.iters
    n = ref.n_iter
    w = lmax - lmin
    # X~_0 = (lmax I - F) / w on F's pattern, truncated with tau_0
    val = (-F.val / w).contiguous()
    rp = F.row_ptr.cpu().numpy()
    ci = F.col_idx.cpu().numpy()
    diag = np.nonzero(ci == np.repeat(np.arange(len(rp) - 1), np.diff(rp)))[0]
    nreal = F.n
    for k, I in zip(diag, range(len(diag))):
        m = min(64, nreal - 64 * I)
        idx = torch.arange(m, device=val.device)
        val[int(k), idx, idx] += lmax / w
    X = sp2.BsrMatrix(F.n, F.row_ptr, F.col_idx, val)
    X, _ = sp2.truncate(X, float(it["tau"][0]), opts["trunc_norm"], opts["coarse_bs"])
    rows = []
    tot = {"symmetric_s": 0.0, "general_s": 0.0, "convert_s": 0.0, "symmetric_flop": 0.0, "general_flop": 0.0}
    for i in range(1, n + 1):
        p, al = int(it["p"][i]), float(it["alpha"][i])
        a, b, c = ((1 - al) ** 2, 2 * al * (1 - al), al * al) if p == 1 else (0.0, 2 * al, -al * al)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Y, ss = sp2.square_step(X, a, b, c, prec)
        torch.cuda.synchronize()
        t_sym = time.perf_counter() - t0
        t0 = time.perf_counter()
        Xg = sp2.general_from_upper(X)
        torch.cuda.synchronize()
        t_conv = time.perf_counter() - t0
        t0 = time.perf_counter()
        Yg, gs = sp2.general_product(Xg, Xg, Xg, a, b, c, prec)
        torch.cuda.synchronize()
        t_gen = time.perf_counter() - t0
        row = {"i": i - 1, "nnzb_sym": X.nnzb, "nnzb_general": Xg.nnzb, "out_nnzb_sym": Y.nnzb,
               "out_nnzb_general": Yg.nnzb, "symmetric_s": round(t_sym, 4), "general_s": round(t_gen, 4),
               "convert_s": round(t_conv, 4), "symmetric_tflop": ss[3] / 1e12, "general_tflop": gs[3] / 1e12,
               "e_rel_diff": abs(math.sqrt(max(gs[0], 0.0)) - math.sqrt(max(ss[0], 0.0))) / max(math.sqrt(ss[0]),
                                                                                                  1e-300)}
        rows.append(row)
        tot["symmetric_s"] += t_sym
        tot["general_s"] += t_gen
        tot["convert_s"] += t_conv
        tot["symmetric_flop"] += ss[3]
        tot["general_flop"] += gs[3]
        log(f"storage iter {i - 1}: {row}")
        del Xg, Yg
        X, _ = sp2.truncate(Y, float(it["tau"][i]), opts["trunc_norm"], opts["coarse_bs"])
        del Y
    out = {"precision": prec, "n_iter": n, "iterations": rows, **{k: round(v, 4) if k.endswith("_s") else v
                                                                   for k, v in tot.items()}}
    out["time_ratio"] = tot["general_s"] / tot["symmetric_s"]
    out["flop_ratio"] = tot["general_flop"] / tot["symmetric_flop"]
    out["stored_ratio_last"] = rows[-1]["nnzb_general"] / rows[-1]["nnzb_sym"]
    log(f"storage: symmetric {tot['symmetric_s']:.3f} s, general {tot['general_s']:.3f} s "
        f"(ratio {out['time_ratio']:.2f}, flops ratio {out['flop_ratio']:.2f}), conversion {tot['convert_s']:.3f} s")
    return out


def norm_study(sp2, sizes, half_bw=300, coarse=(128, 512)):
    """The paper's norm comparison (section "Upper bounds for the spectral
    norm"): symmetric banded matrices with entries U(0, 1e-3) and bandwidth
    2 x 300 + 1, plain and randomly permuted; Frobenius and Frob-Inf norms
    (coarse submatrices of 128 and 512 rows, the multiples of 64 nearest the
    paper's 100 and 500) by the library's norm kernels, the spectral norm by a
    CPU Lanczos solve (invariant under the permutation)."""
    import scipy.sparse.linalg as spla
    import torch

    from fockgen import banded_sym, sparse_to_bsr

    out = []
    for n in sizes:
        A = banded_sym(n, half_bw=half_bw, seed=0)
        spec = float(abs(spla.eigsh(A, k=1, which="LM", return_eigenvectors=False)[0]))
        for perm in (False, True):
            M = sparse_to_bsr(banded_sym(n, half_bw=half_bw, seed=0, permute=perm) if perm else A)
            D = sp2.BsrMatrix.from_host(M, "cuda:0")
            row = {"n": n, "permuted": perm, "nnzb": M.nnzb, "spectral": spec}
            for cbs in coarse:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                f, m = sp2.matrix_norms(D, cbs)
                torch.cuda.synchronize()
                row["frobenius"] = f
                row[f"frobinf_{cbs}"] = m
                row[f"gpu_ms_{cbs}"] = round(1e3 * (time.perf_counter() - t0), 3)
            log(f"norms n={n} permuted={perm}: spectral {spec:.4g} Frobenius {row['frobenius']:.4g} "
                + " ".join(f"FrobInf({c}) {row[f'frobinf_{c}']:.4g}" for c in coarse))
            out.append(row)
            del D
    return out


def stepped_run(sp2, F, no, lmin, lmax, hub, llb, opts, warmup, steps):
    """Solves of the workload, one after the other, run step by step through
    the stepped C ABI (one step = one iteration of Algorithm 2 or one product
    of the subspace correction; the first step of a solve includes Step 1 and
    Algorithm 1, its last Step 3 and the export of D).  ``warmup`` untimed
    steps, then exactly ``steps`` timed ones between two synchronizations;
    the first solve is then run to its end if it has not finished.  Every step
    is timed on its own (synchronized before and after), so the time to D of
    the first solve is the sum of its steps."""
    import torch

    recs, first = [], None
    st = {"solver": None, "solve": -1}

    def one(phase):
        nonlocal first
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if st["solver"] is None:
            st["solver"] = sp2.Solver(F, no, lmin, lmax, hub, llb, **opts)
            st["solve"] += 1
        info = st["solver"].step()
        res = None
        if info["done"]:
            res = st["solver"].end()
            st["solver"] = None
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        info.update(solve=st["solve"], wall=dt, phase=phase)
        recs.append(info)
        if res is not None and first is None:
            first = res
        bf = info["kernel_flops"][2] / max(info["kernel_s"][2], 1e-30) / 1e12 if info["kernel_s"][2] > 0 else 0.0
        log(f"{phase} step {len(recs) - 1:3d}: solve {info['solve']} {info['kind']:10s} it {info['iteration']:3d} "
            f"{info['precision']:6s} {dt:8.3f} s  {info['flops'] / 1e12:9.2f} TF"
            + (f"  bf16x3 kernels {bf:6.1f} TF/s" if bf else "") + ("  [solve done]" if info["done"] else ""))

    for _ in range(warmup):
        one("warmup")
    torch.cuda.synchronize()
    t_a = time.perf_counter()
    for _ in range(steps):
        one("timed")
    torch.cuda.synchronize()
    t_b = time.perf_counter()
    while first is None:
        one("finish")
    if st["solver"] is not None:
        st["solver"].free()
        st["solver"] = None
    return recs, first, t_b - t_a


def trace_of(D):
    """tr D from the diagonal blocks (the first block of each block row when
    present), on the device."""
    import torch

    first = D.row_ptr[:-1]
    has = first < D.row_ptr[1:]
    rows = torch.arange(D.nbr, device=D.device)[has]
    dpos = first[has]
    dpos = dpos[D.col_idx[dpos].to(torch.int64) == rows]
    return float(torch.diagonal(D.val[dpos], dim1=1, dim2=2).sum())


def run1_bounds(config, L, tau):
    """Committed run-1 estimates of this workload (None when absent)."""
    path = os.path.join(ROOT, "bench_run1.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    r = d.get(config)
    if not r or r.get("L") != L or r.get("tau") != tau:
        return None
    return r["homo_ub"], r["lumo_lb"], r.get("bounds_from")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed steps (one step: an iteration of Algorithm 2 or a "
                                                          "product of the subspace correction)")
    ap.add_argument("--warmup", type=int, default=5, help="untimed steps before the timed ones")
    ap.add_argument("--config", default="c2", choices=sorted(CONFIGS))
    ap.add_argument("--precision", default="bf16x3", choices=["fp64", "fp32", "bf16x3"],
                    help="arithmetic of the bulk squares of the timed path (default: BF16x3 with the correction)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="copy a buffer of this size once before timing (reference for HBM traffic counters)")
    ap.add_argument("--correct", type=int, default=None,
                    help="subspace-correction rounds (default: 0 for fp64, 1 for fp32 / bf16x3)")
    ap.add_argument("--corr-tol", type=float, default=3e-7,
                    help="Frobenius budget for dropping blocks of each of the correction's intermediates (default "
                         "3e-7: at N = 108,000 ||D - D_FP64||_F stays at 5.5e-6 for 1e-9 to 3e-7 and reaches 1.7e-5 "
                         "at 1e-6; 0 = the library default 1e-9)")
    ap.add_argument("--corr-purify", type=int, default=None, help="purification steps per correction round")
    ap.add_argument("--corr-mcweeny", type=int, default=1,
                    help="1 (default): purify with one McWeeny step (an FP64 square and a low-precision product); "
                         "0: FP64 squares X^2, 2X - X^2")
    ap.add_argument("--corr-deriv-tol", type=float, default=0.2,
                    help="the correction's derivative steps stop at the first X~_k with e_k below this (default 0.2: "
                         "at N = 108,000 the last four steps, two of them at e_k = 0.12-0.17, change "
                         "||D - D_FP64||_F by under 1e-6; the McWeeny purification projects the rest)")
    ap.add_argument("--corr-low-floor-stop", type=int, default=1,
                    help="with the correction: the low-precision expansion stops at the first e_i below ten times "
                         "its rounding noise (1, default) or by the criterion of Algorithm 2 (0)")
    ap.add_argument("--tail-storage", type=int, default=0,
                    help="1: the FP64 tail multiplies FP32-stored iterates in FP64 (expansions whose FP64 iterates "
                         "do not fit in device memory)")
    ap.add_argument("--low-start-xi", type=float, default=0.0,
                    help="FP64 squares until the gap image xi_i reaches this value, then --precision")
    ap.add_argument("--no-reference", action="store_true",
                    help="with a low --precision: skip the FP64 reference run (largest workloads)")
    ap.add_argument("--adjoint", action="store_true",
                    help="instead of the expansion benchmark: JVP and VJP of tr(W D) in FP64 and mixed precision")
    ap.add_argument("--adjoint-runs", default="fp64,fp32,bf16x3,bf16x3/fp32",
                    help="forward[/adjoint][@option=value...] arithmetics and options of the adjoint benchmark "
                         "(errors need fp64 first)")
    ap.add_argument("--switch-tol", type=float, default=None,
                    help="FP64 tail once ||X - X^2||_F < this (default: 0 with the correction, else 1e-3; "
                         "< 0: no FP64 tail)")
    ap.add_argument("--norms", default=None,
                    help="instead of the expansion benchmark: the norm comparison (spectral vs Frobenius vs "
                         "Frob-Inf) on banded and permuted matrices of these sizes, e.g. 1024,2048,4096")
    ap.add_argument("--storage", action="store_true",
                    help="instead of the expansion benchmark: every square of the expansion done in symmetric storage "
                         "and in general (full-pattern) storage, in --precision (fp64 or bf16x3)")
    ap.add_argument("--n-max-cap", type=int, default=None,
                    help="stop after this many iterations (a capped run of a workload too long for one call)")
    ap.add_argument("--bounds", default=None,
                    help="homo_ub,lumo_lb known in advance (e.g. from a previous SCF cycle): skips the first run")
    ap.add_argument("--run1-precision", default="fp64", choices=["fp64", "fp32"],
                    help="arithmetic of the trace-correcting first run (fp32: FP32 squares and an FP64 tail on "
                         "FP32-stored iterates, for workloads whose FP64 iterates do not fit)")
    ap.add_argument("--run1-only", action="store_true", help="stop after the trace-correcting first run")
    ap.add_argument("--run1", action="store_true",
                    help="run the trace-correcting first run even when bench_run1.json holds its result")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (the method runs on one GPU with no sharding); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np  # noqa: F401
    import torch

    from fockgen import lattice_fock
    from paper_1909_12533_amd import sp2

    if args.norms:
        res = norm_study(sp2, [int(x) for x in args.norms.split(",")])
        print(json.dumps({"norm_study": res}), flush=True)
        return

    cfg = dict(CONFIGS[args.config])
    L, tau, prec = cfg["L"], cfg["tau"], args.precision
    torch.cuda.set_device(0)
    t = time.perf_counter()
    Fh, info = lattice_fock(L, seed=0)
    log(f"generated lattice L={L} N={info['n']} nnzb={Fh.nnzb} in {time.perf_counter() - t:.1f} s")
    F = sp2.BsrMatrix.from_host(Fh, "cuda:0")
    no = info["n_occ"]
    lmin, lmax = sp2.gershgorin(F)
    opts = dict(accel=True, trunc_norm="frobinf", tau_fixed=tau, coarse_bs=4096)
    run1 = None
    if args.bounds:
        hub, llb = (float(x) for x in args.bounds.split(","))
        bounds_from = "given"
    elif not args.run1 and run1_bounds(args.config, L, tau):
        hub, llb, note = run1_bounds(args.config, L, tau)
        bounds_from = note or "run 1 (trace-correcting FP64 run) recorded in bench_run1.json"
    else:
        t = time.perf_counter()
        r1o = dict(opts)
        if args.run1_precision != "fp64":  # FP32 squares, FP64 tail on FP32-stored iterates
            r1o.update(precision=args.run1_precision, switch_tol=1e-3, tail_storage=1)
        r1 = sp2.density(F, no, lmin, lmax, **r1o)
        run1 = {"L": L, "n": info["n"], "tau": tau, "homo_ub": r1.homo_est, "lumo_lb": r1.lumo_est,
                "n_iter": r1.n_iter, "time_s": round(time.perf_counter() - t, 2), "status": r1.status,
                "precision": args.run1_precision, "trace_err": abs(trace_of(r1.D) - no)}
        log(f"run 1 (trace-correcting): {json.dumps(run1)}")
        hub, llb = r1.homo_est, r1.lumo_est
        bounds_from = f"run 1 (trace-correcting {args.run1_precision.upper()} run) in this job"
        del r1
        if args.run1_only:
            print(json.dumps({"run1": run1, "config": args.config}), flush=True)
            return

    if args.calibrate_copy_mib > 0:
        nb = args.calibrate_copy_mib << 20
        src = torch.ones(nb, dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: {nb} bytes read, {nb} bytes written")
        del src, dst

    if args.storage:
        res = storage_bench(sp2, F, no, lmin, lmax, hub, llb, opts, prec if prec != "fp32" else "fp64")
        print(json.dumps({"storage": res, "workload": f"lattice {L}^3 x 4, N={info['n']}, tau={tau}"}), flush=True)
        return

    if args.adjoint:
        res = adjoint_bench(sp2, F, Fh, no, lmin, lmax, hub, llb, opts, args.adjoint_runs.split(","))
        print(json.dumps({"adjoint": res, "workload": f"lattice {L}^3 x 4, N={info['n']}, tau={tau}"}), flush=True)
        return

    correct = args.correct if args.correct is not None else (0 if prec == "fp64" else 1)
    switch_tol = args.switch_tol if args.switch_tol is not None else (0.0 if correct else 1e-3)
    mopts = dict(precision=prec, correct=correct)
    if prec != "fp64":
        mopts["switch_tol"] = switch_tol
    if correct and args.corr_tol:
        mopts["corr_tol"] = args.corr_tol
    if correct and args.corr_mcweeny:
        mopts["corr_mcweeny"] = 1
        mopts["corr_purify"] = 1
    if args.corr_purify is not None:
        mopts["corr_purify"] = args.corr_purify
    if args.corr_deriv_tol is not None:
        mopts["corr_deriv_tol"] = args.corr_deriv_tol
    if correct and args.corr_low_floor_stop:
        mopts["low_floor_stop"] = 1
    if args.n_max_cap is not None:
        mopts["n_max_cap"] = args.n_max_cap
    if args.tail_storage:
        mopts["tail_storage"] = args.tail_storage
    if args.low_start_xi > 0.0:
        mopts["low_start_xi"] = args.low_start_xi

    # ---- the timed path, step by step
    recs, res, t_timed = stepped_run(sp2, F, no, lmin, lmax, hub, llb, {**mopts, **opts}, args.warmup, args.steps)
    first = [r for r in recs if r["solve"] == 0]
    time_to_d = sum(r["wall"] for r in first)
    exp_flops = sum(r["flops"] for r in first if r["kind"] == "iteration")
    timed = [r for r in recs if r["phase"] == "timed"]
    # roofline of the dominant kernel over the timed steps: the MFMA block-product
    # kernels of the run's bulk arithmetic (HIP events on the library's stream)
    code = {"fp64": 0, "fp32": 1, "bf16x3": 2}[prec]
    k_fl = sum(r["kernel_flops"][code] for r in timed)
    k_s = sum(r["kernel_s"][code] for r in timed)
    k_n = sum(r["kernel_launches"][code] for r in timed)
    achieved = k_fl / k_s / 1e12 if k_s > 0 else 0.0
    # the same kernels over the whole first solve (the launches a kernel trace of
    # this command lists for the timed path), by arithmetic
    solve_kernels = {name: {"launches": sum(r["kernel_launches"][c] for r in first),
                            "device_s": round(sum(r["kernel_s"][c] for r in first), 4),
                            "alg_tflop": round(sum(r["kernel_flops"][c] for r in first) / 1e12, 3)}
                     for c, name in enumerate(("fp64", "fp32", "bf16x3"))}
    D = res.D
    checks = {"status": res.status, "stop": res.stop_reason, "n_iter": res.n_iter,
              "trace_err": abs(trace_of(D) - no), "e_n": float(res.iters["e"][-1]),
              "homo_est": None if math.isnan(res.homo_est) else res.homo_est,
              "lumo_est": None if math.isnan(res.lumo_est) else res.lumo_est,
              "steps_per_solve": len(first), "expansion_s": round(sum(r["wall"] for r in first
                                                                     if r["kind"] == "iteration"), 3),
              "correction": res.correction}
    log(f"solve 0: {len(first)} steps, time to D {time_to_d:.3f} s, expansion {checks['expansion_s']:.3f} s, "
        f"status {res.status} ({res.stop_reason}), n={res.n_iter}, e_n={checks['e_n']:.3e}, "
        f"trace error {checks['trace_err']:.3e}")
    del recs
    if prec != "fp64" and not args.no_reference:
        ctx = sp2.context(0)
        ctx.trim()
        torch.cuda.empty_cache()
        t = time.perf_counter()
        ref = sp2.density(F, no, lmin, lmax, hub, llb, precision="fp64", **opts)
        torch.cuda.synchronize()
        t_ref = time.perf_counter() - t
        err = bsr_diff_frobenius(D, ref.D)
        checks.update({"err_vs_fp64_D": err, "fp64_time_to_D_s": round(t_ref, 3),
                       "speedup_vs_fp64": round(t_ref / time_to_d, 4), "fp64_status": ref.status,
                       "fp64_stop": ref.stop_reason, "fp64_n_iter": ref.n_iter,
                       "fp64_trace_err": abs(trace_of(ref.D) - no)})
        log(f"FP64 reference: {t_ref:.3f} s, status {ref.status} ({ref.stop_reason}), n={ref.n_iter}; "
            f"||D - D_fp64||_F = {err:.3e}, speedup {t_ref / time_to_d:.3f}x")
        del ref
    dtype = {"fp64": "f64", "fp32": "f32+f64", "bf16x3": "bf16x3+f64"}[prec]
    line = {
        "metric": "time-to-D (s), block-sparse TFLOP/s; mixed vs FP64 at ||D-D_ref||_F<=1e-5",
        "value": round(exp_flops / time_to_d / 1e12, 4),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * t_timed / args.steps, 3),
        "time_to_D_s": round(time_to_d, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {
            "workload": f"tight-binding Fock {L}x{L}x{L} lattice x 4 basis fns (N={info['n']}), "
                        f"{'FP64 SP2ACC' if prec == 'fp64' else prec.upper() + ' SP2ACC'}"
                        f"{' + FP64 subspace correction' if correct else ''}, 64x64 blocks, "
                        f"tau={tau} Frob-Inf(4096), Gershgorin bounds, homo/lumo from the trace-correcting run 1",
            "n": info["n"], "n_occ": no, "tau": tau, "precision": prec, "bounds": [hub, llb],
            "bounds_from": bounds_from,
            "step": "one iteration of Algorithm 2 or one product of the subspace correction; value = the "
                    "expansion's block-sparse flops / time to D of one solve (sum of its steps)",
            "alg_tflop_expansion": round(exp_flops / 1e12, 3),
            "device_peak_gb": round(res.correction["device_peak_bytes"] / 1e9, 2),
            # the library options of the timed solve (beyond the Frob-Inf truncation above)
            "options": {k: v for k, v in mopts.items() if k != "precision"},
        },
        "checks": checks,
        "roofline": {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK[prec], "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK[prec], 4), "traffic": traffic_per_launch(prec, L),
                     "kernel": f"{KERNELS[prec][0]} ({prec.upper()} MFMA block products, timed steps)",
                     "timed_launches": k_n, "avg_launch_ms": round(1e3 * k_s / max(k_n, 1), 3),
                     "solve_kernels": solve_kernels},
    }
    if run1:
        line["config"]["run1"] = run1
    del D, res
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)...")
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
