"""Truncated RQRCP without trailing update (test infrastructure only).

Follows Algorithm 5 of Duersch & Gu in the paper's order.  The input A is never
modified.  State carried between blocks: the reflectors Y (m x K), the
connection matrix T (K x K), the reflector inner products W^T (K x n) and the
finished rows of R (K x n), all with columns in the current pivoted order.

Formulas used (Section 4.1):
* block-reflector composition T = [[T1, -T1 Y1^T Y2 T2], [0, T2]];
* inner products W2^T = T2^T (Y2^T A - (Y2^T Y1) W1^T);
* any part of the transformed matrix is A - Y W^T: the selected columns are built
  from it before their panel QR, and the new rows of R after the W update;
* the sample update of eq. (update1).

Readings where the text is ambiguous:
* the sample used in block J is the one produced at the end of block J-1 (the
  caption writes B^[J] where Algorithm 4 writes B^[J-1]);
* "A^[J]" in the permutation line means the original matrix with its columns
  permuted, not an updated trailing matrix;
* W^T is formed for every column position (the oracle does not skip finished
  columns), R rows are written only on and right of the diagonal block.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .householder import form_t, householder_qr, unit_lower
from .qrcp import PivotTrace, apply_transpositions, partial_qrcp
from .rqrcp import sample_update


@dataclass
class TRQRCPResult:
    y: np.ndarray       # m x k reflectors, unit diagonal explicit, zeros above
    t: np.ndarray       # k x k upper triangular, Q = I - Y T Y^T
    r: np.ndarray       # k x n, columns in pivoted order: A P ~ Q[:, :k] R
    jpvt: np.ndarray    # n
    tau: np.ndarray     # k (diagonal of T)
    wt: np.ndarray      # k x n reflector inner products (pivoted order)
    trace: PivotTrace
    sample_scale: float
    blocks: list


def trqrcp(a, omega, b, p, k, keep_blocks=False):
    a0 = np.asarray(a, dtype=np.float64)
    m, n = a0.shape
    k = int(k)
    ell = b + p
    if np.shape(omega) != (ell, m):
        raise ValueError("omega must be (b+p) x m")
    jpvt = np.arange(n, dtype=np.int64)
    y = np.zeros((m, 0))
    t = np.zeros((0, 0))
    wt = np.zeros((0, n))
    r = np.zeros((k, n))
    trace = PivotTrace()
    blocks = []
    bmat = np.asarray(omega, dtype=np.float64) @ a0            # B^[0] = Omega A
    scale = float(np.max(np.sqrt(np.sum(bmat * bmat, axis=0)))) if bmat.size else 0.0
    col0 = 0
    while col0 < k:
        bj = min(b, k - col0)
        sq = partial_qrcp(bmat, bj)
        trace.best += sq.trace.best
        trace.second += sq.trace.second
        # permute the column order of A (index map), W^T and the finished R rows
        apply_transpositions(jpvt, sq.pivots, offset=col0, axis=0)
        apply_transpositions(wt, sq.pivots, offset=col0)
        apply_transpositions(r, sq.pivots, offset=col0)
        ap = a0[:, jpvt]                                         # A^[J] (permuted original)
        sel = slice(col0, col0 + bj)
        a_hat = ap[:, sel] - y @ wt[:, sel]                     # selected columns of A - Y W^T
        panel, tau2 = householder_qr(a_hat[col0:, :])
        v2 = unit_lower(panel, bj)
        y2 = np.zeros((m, bj))
        y2[col0:, :] = v2
        t2 = form_t(v2, tau2)
        w2t = t2.T @ (y2.T @ ap - (y2.T @ y) @ wt)              # new inner products
        t = np.block([[t, -t @ (y.T @ y2) @ t2],
                      [np.zeros((bj, t.shape[0])), t2]])
        y = np.hstack([y, y2])
        wt = np.vstack([wt, w2t])
        rows = (ap - y @ wt)[col0:col0 + bj, :]                 # new rows of R
        r11 = np.triu(panel[:bj, :bj])
        r[col0:col0 + bj, col0:col0 + bj] = r11
        r[col0:col0 + bj, col0 + bj:] = rows[:, col0 + bj:]
        if keep_blocks:
            blocks.append(dict(col0=col0, bj=bj, a_hat=a_hat, rows=rows, r11=r11))
        col0 += bj
        if col0 < k:
            bmat = sample_update(sq, r11, r[col0 - bj:col0, col0:], bj)
    return TRQRCPResult(y, t, r, jpvt, np.diag(t).copy(), wt, trace, scale, blocks)
