"""torch.autograd wrapper of the density-matrix expansion and its hand-written
adjoint.

`density_matrix(F_val, F_rows, n, n_occ, lmin, lmax, ...)` returns the values
of D (upper BSR blocks, pattern returned alongside) as a differentiable
function of the stored upper blocks of F.  The backward pass calls the
library's VJP of the recorded recursion (schedule, iteration count and block
masks frozen; sqrt(n) checkpoints), i.e. the derivative of the discrete map
that produced D.

Stored-block convention: an off-diagonal stored block stands for itself and
its mirror, so for a loss L(D_val) the full symmetric W with tr(W dD) = dL has
W_IJ = W_JI^T = g_IJ / 2 off the diagonal and W_II = (g_II + g_II^T) / 2; the
gradient with respect to a stored off-diagonal block of F is twice the
corresponding block of dL/dF (both mirrors move), a diagonal block takes it
once.
"""
from __future__ import annotations

import torch

from . import sp2


def _block_keys(row_ptr, col_idx, nbr):
    rows = torch.repeat_interleave(torch.arange(nbr, device=row_ptr.device), torch.diff(row_ptr))
    return rows, col_idx.long(), rows * nbr + col_idx.long()


def _gather_on_pattern(src: sp2.BsrMatrix, row_ptr, col_idx, nbr):
    """Values of `src` on the block pattern (row_ptr, col_idx); missing blocks 0."""
    _, _, k_dst = _block_keys(row_ptr, col_idx, nbr)
    _, _, k_src = _block_keys(src.row_ptr, src.col_idx, nbr)
    out = torch.zeros((k_dst.numel(), 64, 64), dtype=torch.float64, device=src.val.device)
    if k_src.numel() == 0 or k_dst.numel() == 0:
        return out
    pos = torch.searchsorted(k_src, k_dst).clamp(max=k_src.numel() - 1)
    hit = k_src[pos] == k_dst
    out[hit] = src.val[pos[hit]]
    return out


class _DensityFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, F_val, row_ptr, col_idx, n, n_occ, lmin, lmax, homo_ub, lumo_lb, opts):
        F = sp2.BsrMatrix(n, row_ptr, col_idx, F_val.detach().contiguous())
        r = sp2.density(F, n_occ, lmin, lmax, homo_ub, lumo_lb, record_tape=True, **opts)
        ctx.tape = r.tape
        ctx.F_pattern = (row_ptr, col_idx, n)
        ctx.D_pattern = (r.D.row_ptr, r.D.col_idx)
        ctx.result = r
        ctx.mark_non_differentiable(r.D.row_ptr, r.D.col_idx)
        return r.D.val, r.D.row_ptr, r.D.col_idx

    @staticmethod
    def backward(ctx, g, _g_rows=None, _g_cols=None):
        row_ptr, col_idx, n = ctx.F_pattern
        nbr = (n + 63) // 64
        d_rows, d_cols = ctx.D_pattern
        rows, cols, _ = _block_keys(d_rows, d_cols, nbr)
        off = (rows != cols)
        W = g.detach().clone()
        W[off] *= 0.5
        W[~off] = 0.5 * (W[~off] + W[~off].transpose(1, 2))
        Fbar = ctx.tape.vjp(sp2.BsrMatrix(n, d_rows, d_cols, W.contiguous()))
        grad = _gather_on_pattern(Fbar, row_ptr, col_idx, nbr)
        frows, fcols, _ = _block_keys(row_ptr, col_idx, nbr)
        grad[frows != fcols] *= 2.0
        return grad, None, None, None, None, None, None, None, None, None


def density_matrix(F_val, row_ptr, col_idx, n, n_occ, lmin, lmax, homo_ub=None, lumo_lb=None, **opts):
    """Differentiable D = theta(mu I - F) for F given by its stored upper
    blocks F_val (nnzb, 64, 64) on the pattern (row_ptr, col_idx).  Returns
    (D_val, D_row_ptr, D_col_idx); gradients flow to F_val through the
    library's VJP.  Options are those of `sp2.density`."""
    return _DensityFn.apply(F_val, row_ptr, col_idx, int(n), int(n_occ), float(lmin), float(lmax),
                            homo_ub, lumo_lb, dict(opts))
