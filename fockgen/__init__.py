"""Seeded synthetic Fock-like inputs and block-sparse format helpers.

This module is shared by the oracle, the tests and the benchmark.  It holds no
arithmetic of the density-matrix method itself: it only draws random matrices
and moves numbers between dense and block-sparse (BSR) layouts.

Workloads (the paper's own Fock matrices, from HF/3-21G calculations on a
Glu-Ala helix and on water clusters, section "Numerical experiments", are not
available; these synthetic matrices stand in for them.  Like the paper's
matrices they have a bounded number of non-zeros per row and a homo-lumo gap
that does not shrink with system size):

* ``dense_spectrum``: F = Q diag(lam) Q^T with Q Haar-random orthogonal and a
  prescribed spectrum with a gap.  Exact eigenpairs are returned, so the
  definition D = sum_{i<=n_occ} y_i y_i^T (section "Introduction") is known.
* ``lattice_fock``: a tight-binding Fock matrix on an L x L x L cubic lattice
  with 4 basis functions per atom, onsite energies -1/+1 on the two
  sublattices plus N(0, 0.05) noise, and hoppings
  0.3 exp(-r/1.5) U(-1, 1) between atoms at Manhattan distance 1 <= r <= 4
  (open boundaries).  Atoms are numbered in 3-D Morton order and the 4 basis
  functions of an atom are contiguous, so that 64 x 64 blocks cover compact
  groups of 16 atoms.

BSR convention used everywhere in this repository ("upper BSR"):
``row_ptr`` int64[nbr+1], ``col_idx`` int32[nnzb] (col >= row, strictly
increasing inside a block row), ``val`` float64[nnzb, bs, bs] (each block
row-major).  Only blocks on or above the block diagonal are stored; a block
below the diagonal is the transpose of its mirror.  When n is not a multiple of
bs the last block row/column is padded with exact zeros.
"""
from __future__ import annotations

import numpy as np

BS = 64

__all__ = [
    "BS",
    "BSR",
    "dense_spectrum",
    "lattice_fock",
    "lattice_positions_morton",
    "random_sym_on_pattern",
    "random_sym_bsr",
    "dense_to_bsr",
    "bsr_to_dense",
    "block_mask_of_bsr",
]


class BSR:
    """Host-side upper BSR matrix (numpy arrays)."""

    def __init__(self, n, row_ptr, col_idx, val, bs=BS):
        self.n = int(n)
        self.bs = int(bs)
        self.nbr = (self.n + self.bs - 1) // self.bs
        self.row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
        self.col_idx = np.ascontiguousarray(col_idx, dtype=np.int32)
        self.val = np.ascontiguousarray(val, dtype=np.float64)
        assert self.row_ptr.shape == (self.nbr + 1,)
        assert self.val.shape == (self.col_idx.shape[0], self.bs, self.bs)

    @property
    def nnzb(self):
        return int(self.col_idx.shape[0])

    def rows(self):
        """Block-row index of every stored block."""
        return np.repeat(np.arange(self.nbr, dtype=np.int64), np.diff(self.row_ptr))

    def with_values(self, val):
        return BSR(self.n, self.row_ptr, self.col_idx, val, self.bs)


# --------------------------------------------------------------------------
# format helpers
# --------------------------------------------------------------------------

def dense_to_bsr(A, bs=BS, keep_diag=True):
    """Upper BSR of a symmetric dense matrix.  A block is stored when it has
    any non-zero entry; diagonal blocks are always stored when ``keep_diag``."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    nbr = (n + bs - 1) // bs
    P = np.zeros((nbr * bs, nbr * bs))
    P[:n, :n] = A
    B = P.reshape(nbr, bs, nbr, bs).transpose(0, 2, 1, 3)
    nz = np.any(B != 0.0, axis=(2, 3))
    if keep_diag:
        nz[np.arange(nbr), np.arange(nbr)] = True
    nz = np.triu(nz)
    I, J = np.nonzero(nz)  # row-major order: sorted by (I, J)
    row_ptr = np.zeros(nbr + 1, dtype=np.int64)
    np.add.at(row_ptr, I + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    val = np.ascontiguousarray(B[I, J])
    return BSR(n, row_ptr, J.astype(np.int32), val, bs)


def bsr_to_dense(M: BSR):
    """Symmetric dense matrix of an upper BSR (lower blocks mirrored)."""
    bs, nbr = M.bs, M.nbr
    P = np.zeros((nbr, nbr, bs, bs))
    I = M.rows()
    J = M.col_idx.astype(np.int64)
    P[I, J] = M.val
    off = I != J
    P[J[off], I[off]] = M.val[off].transpose(0, 2, 1)
    return P.transpose(0, 2, 1, 3).reshape(nbr * bs, nbr * bs)[: M.n, : M.n].copy()


def block_mask_of_bsr(M: BSR):
    """Symmetric boolean nbr x nbr mask of stored blocks."""
    mask = np.zeros((M.nbr, M.nbr), dtype=bool)
    I = M.rows()
    J = M.col_idx.astype(np.int64)
    mask[I, J] = True
    mask[J, I] = True
    return mask


# --------------------------------------------------------------------------
# dense test matrix with known spectrum
# --------------------------------------------------------------------------

def dense_spectrum(n=512, n_occ=None, occ_range=(-1.0, -0.1), virt_range=(0.1, 1.0), seed=0):
    """F = Q diag(lam) Q^T with Q Haar-random (QR of a Gaussian matrix with the
    signs of diag(R) folded into Q) and n_occ eigenvalues drawn uniformly in
    ``occ_range`` and n - n_occ in ``virt_range``.

    Returns (F, lam_sorted, Y) with Y[:, i] the eigenvector of lam_sorted[i]."""
    if n_occ is None:
        n_occ = n // 2
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((n, n))
    Q, R = np.linalg.qr(G)
    Q = Q * np.sign(np.diag(R))[None, :]
    lam_o = rng.uniform(occ_range[0], occ_range[1], size=n_occ)
    lam_v = rng.uniform(virt_range[0], virt_range[1], size=n - n_occ)
    lam = np.concatenate([lam_o, lam_v])
    order = np.argsort(lam, kind="stable")
    lam = lam[order]
    Y = Q[:, order]
    F = (Y * lam[None, :]) @ Y.T
    F = 0.5 * (F + F.T)
    return F, lam, Y


# --------------------------------------------------------------------------
# tight-binding lattice Fock matrix
# --------------------------------------------------------------------------

def _morton3(x, y, z, bits=11):
    code = np.zeros_like(x, dtype=np.int64)
    for b in range(bits):
        code |= ((x >> b) & 1) << (3 * b + 2)
        code |= ((y >> b) & 1) << (3 * b + 1)
        code |= ((z >> b) & 1) << (3 * b)
    return code


def lattice_positions_morton(L):
    """Integer coordinates (n_atoms, 3) of the L^3 lattice in Morton order."""
    g = np.arange(L, dtype=np.int64)
    x, y, z = np.meshgrid(g, g, g, indexing="ij")
    x, y, z = x.ravel(), y.ravel(), z.ravel()
    order = np.argsort(_morton3(x, y, z), kind="stable")
    return np.stack([x[order], y[order], z[order]], axis=1)


def _half_space_displacements(rmax):
    """Displacements d with 1 <= |d|_1 <= rmax and d > 0 lexicographically
    (each unordered atom pair once), in a fixed order."""
    out = []
    for dx in range(-rmax, rmax + 1):
        for dy in range(-rmax, rmax + 1):
            for dz in range(-rmax, rmax + 1):
                r = abs(dx) + abs(dy) + abs(dz)
                if r < 1 or r > rmax:
                    continue
                if (dx, dy, dz) > (0, 0, 0):
                    out.append((dx, dy, dz, r))
    return out


def lattice_fock(L, nbf=4, onsite=1.0, noise_std=0.05, hop=0.3, decay=1.5, rmax=4, seed=0, bs=BS):
    """Upper BSR of the tight-binding Fock matrix described in the module
    docstring.  Returns (F_bsr, info) where info holds n, n_occ, n_atoms.

    Random draws (numpy PCG64, ``seed``): first the onsite noise, shape
    (n_atoms, nbf) in Morton atom order; then, for every displacement of
    ``_half_space_displacements`` in order, an array (n_pairs, nbf, nbf) of
    U(-1, 1) for the atom pairs (a, a + d) inside the lattice, taken in Morton
    order of a."""
    rng = np.random.default_rng(seed)
    pos = lattice_positions_morton(L)
    na = pos.shape[0]
    n = na * nbf
    nbr = (n + bs - 1) // bs
    apb = bs // nbf  # atoms per block (bs must be a multiple of nbf)
    assert apb * nbf == bs
    # position -> Morton rank lookup
    rank_of = np.empty((L, L, L), dtype=np.int64)
    rank_of[pos[:, 0], pos[:, 1], pos[:, 2]] = np.arange(na)

    parity = (pos.sum(axis=1) & 1)
    eps = np.where(parity == 0, -onsite, onsite)
    noise = rng.normal(0.0, noise_std, size=(na, nbf))
    diag_vals = (eps[:, None] + noise)  # (na, nbf)

    # collect atom-pair sub-blocks (a < b in Morton rank, oriented upper)
    pa_list, pb_list, blk_list = [], [], []
    for dx, dy, dz, r in _half_space_displacements(rmax):
        tgt = pos + np.array([dx, dy, dz])
        ok = np.all((tgt >= 0) & (tgt < L), axis=1)
        a = np.nonzero(ok)[0]
        b = rank_of[tgt[ok, 0], tgt[ok, 1], tgt[ok, 2]]
        h = rng.uniform(-1.0, 1.0, size=(a.shape[0], nbf, nbf)) * (hop * np.exp(-r / decay))
        # H[a, b] = h ; H[b, a] = h^T.  Store oriented so that row atom < col atom.
        swap = a > b
        ra = np.where(swap, b, a)
        rb = np.where(swap, a, b)
        h = np.where(swap[:, None, None], h.transpose(0, 2, 1), h)
        pa_list.append(ra)
        pb_list.append(rb)
        blk_list.append(h)
    pa = np.concatenate(pa_list)
    pb = np.concatenate(pb_list)
    hb = np.concatenate(blk_list)

    # block pattern
    BI = pa // apb
    BJ = pb // apb
    key = BI * nbr + BJ
    diag_keys = np.arange(nbr, dtype=np.int64) * (nbr + 1)
    ukeys = np.unique(np.concatenate([key, diag_keys]))
    I = ukeys // nbr
    J = ukeys % nbr
    row_ptr = np.zeros(nbr + 1, dtype=np.int64)
    np.add.at(row_ptr, I + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    val = np.zeros((ukeys.shape[0], bs, bs))
    slot = np.searchsorted(ukeys, key)
    ro = (pa % apb) * nbf
    co = (pb % apb) * nbf
    same = BI == BJ  # pair inside a diagonal block: store its mirror too
    for i in range(nbf):
        for j in range(nbf):
            val[slot, ro + i, co + j] = hb[:, i, j]
            val[slot[same], co[same] + j, ro[same] + i] = hb[same, i, j]
    # onsite terms (diagonal entries only)
    dslot = np.searchsorted(ukeys, (np.arange(na) // apb) * (nbr + 1))
    do = (np.arange(na) % apb) * nbf
    for i in range(nbf):
        val[dslot, do + i, do + i] = diag_vals[:, i]
    F = BSR(n, row_ptr, J.astype(np.int32), val, bs)
    info = {"n": n, "n_occ": int((parity == 0).sum()) * nbf, "n_atoms": na, "L": L}
    return F, info


# --------------------------------------------------------------------------
# random symmetric matrices on a block pattern
# --------------------------------------------------------------------------

def random_sym_on_pattern(M: BSR, std=1.0, seed=0):
    """Symmetric matrix with the block pattern of ``M``: N(0, std^2) entries
    on stored blocks, mirrored inside diagonal blocks, zero in padding."""
    rng = np.random.default_rng(seed)
    val = rng.normal(0.0, std, size=M.val.shape)
    I = M.rows()
    diag = I == M.col_idx
    val[diag] = np.triu(val[diag]) + np.triu(val[diag], 1).transpose(0, 2, 1)
    _zero_padding(M.n, M.nbr, M.bs, I, M.col_idx, val)
    return M.with_values(val)


def random_sym_bsr(n, density, seed=0, bs=BS, std=1.0, keep_diag=True):
    """Random symmetric upper BSR: each off-diagonal upper block is present
    with probability ``density``; entries N(0, std^2)."""
    rng = np.random.default_rng(seed)
    nbr = (n + bs - 1) // bs
    present = rng.random((nbr, nbr)) < density
    present = np.triu(present, 1)
    if keep_diag:
        present[np.arange(nbr), np.arange(nbr)] = True
    I, J = np.nonzero(present)
    row_ptr = np.zeros(nbr + 1, dtype=np.int64)
    np.add.at(row_ptr, I + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    val = rng.normal(0.0, std, size=(I.shape[0], bs, bs))
    diag = I == J
    val[diag] = np.triu(val[diag]) + np.triu(val[diag], 1).transpose(0, 2, 1)
    _zero_padding(n, nbr, bs, I, J, val)
    return BSR(n, row_ptr, J.astype(np.int32), val, bs)


def banded_sym(n, half_bw=300, hi=1e-3, seed=0, permute=False):
    """Symmetric banded matrix (scipy CSR) with entries U(0, hi) on
    |i - j| <= half_bw (bandwidth 2 half_bw + 1), the test matrices of the
    paper's norm comparison (section "Upper bounds for the spectral norm");
    with ``permute`` the rows and columns are permuted by one seeded random
    permutation (P A P^T)."""
    import scipy.sparse as sps

    rng = np.random.default_rng(seed)
    i = np.repeat(np.arange(n), half_bw + 1)
    j = i + np.tile(np.arange(half_bw + 1), n)
    keep = j < n
    i, j = i[keep], j[keep]
    v = rng.uniform(0.0, hi, size=i.shape[0])
    off = i != j
    A = sps.coo_matrix((np.concatenate([v, v[off]]), (np.concatenate([i, j[off]]), np.concatenate([j, i[off]]))),
                       shape=(n, n)).tocsr()
    if permute:
        p = np.random.default_rng(seed + 1).permutation(n)
        A = A[p][:, p].tocsr()
    return A


def sparse_to_bsr(A, bs=BS):
    """Upper BSR of a symmetric scipy sparse matrix, without a dense copy;
    diagonal blocks are always stored."""
    A = A.tocoo()
    A.sum_duplicates()  # every entry then has its own position in its block
    n = A.shape[0]
    nbr = (n + bs - 1) // bs
    bi, bj = A.row // bs, A.col // bs
    up = bj >= bi
    r, c, v, bi, bj = A.row[up], A.col[up], A.data[up], bi[up], bj[up]
    ids = np.unique(np.concatenate([bi.astype(np.int64) * nbr + bj, np.arange(nbr, dtype=np.int64) * (nbr + 1)]))
    I, J = ids // nbr, ids % nbr
    pos = np.searchsorted(ids, bi.astype(np.int64) * nbr + bj)
    flat = (pos * bs + (r % bs)) * bs + (c % bs)
    order = np.argsort(flat, kind="stable")  # write in memory order
    val = np.zeros(ids.shape[0] * bs * bs)
    val[flat[order]] = v[order]
    val = val.reshape(ids.shape[0], bs, bs)
    row_ptr = np.zeros(nbr + 1, dtype=np.int64)
    np.add.at(row_ptr, I + 1, 1)
    return BSR(n, np.cumsum(row_ptr), J.astype(np.int32), val, bs)


def _zero_padding(n, nbr, bs, I, J, val):
    pad = nbr * bs - n
    if pad == 0:
        return
    last = nbr - 1
    val[I == last, bs - pad:, :] = 0.0
    val[J == last, :, bs - pad:] = 0.0


# --------------------------------------------------------------------------
# general (full-pattern) storage: every present block of both triangles
# --------------------------------------------------------------------------

def random_general_bsr(n, density, seed=0, bs=BS, std=1.0, keep_diag=False):
    """Random matrix in general block storage (no symmetry): each block of
    either triangle is present with probability ``density``; entries
    N(0, std^2); rows and columns past n are zero."""
    rng = np.random.default_rng(seed)
    nbr = (n + bs - 1) // bs
    present = rng.random((nbr, nbr)) < density
    if keep_diag:
        present[np.arange(nbr), np.arange(nbr)] = True
    I, J = np.nonzero(present)  # row-major order: sorted by (I, J)
    row_ptr = np.zeros(nbr + 1, dtype=np.int64)
    np.add.at(row_ptr, I + 1, 1)
    val = rng.normal(0.0, std, size=(I.shape[0], bs, bs))
    _zero_padding(n, nbr, bs, I, J, val)
    return BSR(n, np.cumsum(row_ptr), J.astype(np.int32), val, bs)


def general_bsr_to_dense(M: BSR):
    """Dense matrix of a BSR in general storage (blocks as stored)."""
    bs, nbr = M.bs, M.nbr
    P = np.zeros((nbr, nbr, bs, bs))
    P[M.rows(), M.col_idx.astype(np.int64)] = M.val
    return P.transpose(0, 2, 1, 3).reshape(nbr * bs, nbr * bs)[: M.n, : M.n].copy()


def general_block_mask(M: BSR):
    """nbr x nbr boolean mask of the blocks stored in general storage."""
    mask = np.zeros((M.nbr, M.nbr), dtype=bool)
    mask[M.rows(), M.col_idx.astype(np.int64)] = True
    return mask
