"""Shared helpers of the GPU tests: conversions between the device matrices of
the HIP binding and the dense arrays of the oracle (format only)."""
import numpy as np

from fockgen import BSR, bsr_to_dense


def to_dense(M):
    n, rp, ci, v = M.to_host()
    return bsr_to_dense(BSR(n, rp, ci, v))


def upper_mask(M):
    """Upper-triangle block mask of a device matrix (nbr x nbr bool)."""
    n, rp, ci, v = M.to_host()
    nbr = (n + 63) // 64
    m = np.zeros((nbr, nbr), dtype=bool)
    rows = np.repeat(np.arange(nbr), np.diff(rp))
    m[rows, ci] = True
    return m


def rel(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def to_dense_general(M):
    """Dense matrix of a device matrix in general (full-pattern) storage."""
    from fockgen import general_bsr_to_dense

    n, rp, ci, v = M.to_host()
    return general_bsr_to_dense(BSR(n, rp, ci, v))


def general_mask(M):
    """Block mask (nbr x nbr bool) of a device matrix in general storage."""
    n, rp, ci, v = M.to_host()
    nbr = (n + 63) // 64
    m = np.zeros((nbr, nbr), dtype=bool)
    rows = np.repeat(np.arange(nbr), np.diff(rp))
    m[rows, ci] = True
    return m
