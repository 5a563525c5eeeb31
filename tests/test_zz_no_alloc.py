"""sp2_matrix_norms_noalloc (no device allocation, fixed device scratch)
against sp2_matrix_norms through the C ABI: bit-identical norms on two calls
in a row, the second with a smaller matrix (the scratch keeps the last call's
contents, so whatever must start at zero is cleared by each call), and the
size limit rejected before any device work."""
import ctypes as C

import numpy as np
import pytest

from fockgen import lattice_fock, random_sym_on_pattern

pytestmark = pytest.mark.gpu


def test_noalloc_norms_equal_allocating_entry_point(gpu_lib):
    sp2 = gpu_lib
    big, _ = lattice_fock(8, seed=0)          # N = 2048, 32 block rows
    small, _ = lattice_fock(5, seed=3)        # N = 500, ragged last block
    W = random_sym_on_pattern(big, 1.0, seed=4)
    for M, cbs in ((big, 256), (W, 128), (small, 128), (small, 64)):
        A = sp2.BsrMatrix.from_host(M, "cuda:0")
        f0, m0 = sp2.matrix_norms(A, cbs)
        f1, m1 = sp2.matrix_norms_noalloc(A, cbs)
        print(f"n={M.n} nnzb={M.nnzb} coarse={cbs}: frob {f0!r} / {f1!r}, frobinf {m0!r} / {m1!r}")
        assert f1 == f0 and m1 == m0
        assert f0 > 0 and m0 >= f0 / np.sqrt((M.n + cbs - 1) // cbs) - 1e-12


def test_noalloc_norms_reject_oversize(gpu_lib):
    import torch

    sp2 = gpu_lib
    ctx = sp2.context(0)
    rp = torch.zeros(2, dtype=torch.int64, device="cuda:0")
    # claims 6 million blocks: more scratch than the library holds; rejected
    # before any device access
    from paper_1909_12533_amd import _lib

    s = _lib.sp2_bsr(n=64, bs=64, owned=0, nbr=1, nnzb=6_000_000, row_ptr=rp.data_ptr(),
                         col_idx=rp.data_ptr(), val=rp.data_ptr())
    f, m = C.c_double(), C.c_double()
    rc = ctx.lib.sp2_matrix_norms_noalloc(ctx.h, C.byref(s), 4096, C.byref(f), C.byref(m))
    assert rc == -1
    assert b"too large" in ctx.lib.sp2_last_error(ctx.h)
