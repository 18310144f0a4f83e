"""Randomized QRCP (test infrastructure only).

* ``rqrcp``: Algorithm 4 (RQRCP) with the sample update formula, eq. (update1):
  B1 = S12 - S11 R11^{-1} R12, B2 = S22.
* ``rsrqrcp``: the repeated-sampling variant named in Section 3.4 (replace the
  sample update by a fresh projection B = Omega_J A_J of the trailing matrix).
* ``single_sample_rqrcp``: Algorithm 3 (one sketch, k pivots, QR, R12 = Q^T A).

All steps in the paper's order, float64 numpy, one library primitive per step
(matrix product, triangular solve).  Random matrices are inputs, never drawn
here.

Readings where the paper is silent:
* the last block takes b_J = k - (J-1) b columns while ell stays b + p;
* eq. (update1) needs R11 nonsingular (Section 3.2).  When a block's R11 has a
  diagonal entry with |R_ii| <= eps max(m, n) |R_00| (numerically singular),
  ``info`` records that column (1-based) and from then on every next sample is
  a fresh projection of the updated trailing matrix (repeated sampling,
  Section 3.4), B = Omega[:, :M'] A^[J], with the leading M' columns of the
  given Omega (no new random matrix is drawn here);
* R11^{-1} R12 is a triangular solve, then multiplied by S11;
* the block transformation is applied as A <- A - Y (T^T (Y^T A)), i.e. Q^T A
  with Q = I - Y T Y^T built by the forward recurrence.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla

from .householder import form_t, householder_qr, unit_lower
from .qrcp import PivotTrace, apply_transpositions, partial_qrcp


@dataclass
class RQRCPResult:
    qr: np.ndarray          # m x n in-place form (R on/above diag, reflectors below)
    tau: np.ndarray         # k
    jpvt: np.ndarray        # n
    t_blocks: list          # list of b_J x b_J T matrices, one per block
    trace: PivotTrace       # sample norms per step (best / runner-up)
    sample_scale: float     # largest initial sample column norm
    blocks: list = field(default_factory=list)   # optional per-block records
    info: int = 0           # 0, or the 1-based column where R11 was numerically singular


def _block_loop(a, k, b, first_sample, next_sample, keep_blocks=False):
    w = np.array(a, dtype=np.float64, order="F", copy=True)
    m, n = w.shape
    jpvt = np.arange(n, dtype=np.int64)
    tau = np.zeros(k)
    t_blocks = []
    trace = PivotTrace()
    blocks = []
    bmat = first_sample(w)
    scale = float(np.max(np.sqrt(np.sum(bmat * bmat, axis=0)))) if bmat.size else 0.0
    col0 = 0
    while col0 < k:
        bj = min(b, k - col0)
        sq = partial_qrcp(bmat, bj)                          # sample pivots
        trace.best += sq.trace.best
        trace.second += sq.trace.second
        a_before = w[col0:, col0:].copy() if keep_blocks else None
        apply_transpositions(w, sq.pivots, offset=col0)      # A and finished R rows
        apply_transpositions(jpvt, sq.pivots, offset=col0, axis=0)
        panel, tj = householder_qr(w[col0:, col0:col0 + bj])  # b reflectors, R11
        w[col0:, col0:col0 + bj] = panel
        y = unit_lower(panel, bj)
        t = form_t(y, tj)
        tau[col0:col0 + bj] = tj
        t_blocks.append(t)
        if col0 + bj < n:
            c = w[col0:, col0 + bj:]
            c -= y @ (t.T @ (y.T @ c))                     # R12 rows and A^[J]
            w[col0:, col0 + bj:] = c
        r11 = np.triu(panel[:bj, :bj])
        r12 = w[col0:col0 + bj, col0 + bj:]
        if keep_blocks:
            blocks.append(dict(col0=col0, bj=bj, b_in=bmat.copy(), sample=sq,
                               a_before=a_before, y=y, t=t, r11=r11.copy(),
                               r12=r12.copy(), a_after=w[col0 + bj:, col0 + bj:].copy()))
        col0 += bj
        if col0 < k:
            bmat = next_sample(sq, r11, r12, w, col0, bj)
            if keep_blocks:
                blocks[-1]["b_out"] = bmat.copy()
    return w, tau, jpvt, t_blocks, trace, scale, blocks


def sample_update(sq, r11, r12, bj):
    """Equation (update1): B1 = S12 - S11 R11^{-1} R12, B2 = S22."""
    s = sq.s
    s11 = s[:bj, :bj]
    s12 = s[:bj, bj:]
    s22 = s[bj:, bj:]
    x = sla.solve_triangular(r11, r12, lower=False)
    b1 = s12 - s11 @ x
    return np.vstack([b1, s22])


def rqrcp(a, omega, b, p, k=None, keep_blocks=False):
    """Algorithm 4.  ``omega`` is the ell x m Gaussian matrix, ell = b + p."""
    m, n = np.shape(a)
    k = min(m, n) if k is None else int(k)
    ell = b + p
    if np.shape(omega) != (ell, m):
        raise ValueError("omega must be (b+p) x m")
    om = np.asarray(omega, dtype=np.float64)
    eps = np.finfo(np.float64).eps
    state = {"fallback": False, "info": 0}

    def first(w):
        return om @ w                                       # B^[0] = Omega A

    def nxt(sq, r11, r12, w, col0, bj):
        # col0 is the next block's first column; w[0, 0] is R_00
        if not state["fallback"]:
            small = np.flatnonzero(np.abs(np.diag(r11)) <= eps * max(m, n) * abs(w[0, 0]))
            if small.size:                                  # R11 numerically singular
                state["fallback"] = True
                state["info"] = col0 - bj + int(small[0]) + 1
        if state["fallback"]:
            trailing = w[col0:, col0:]                      # A^[J], already updated
            return om[:, :trailing.shape[0]] @ trailing     # a fresh projection
        return sample_update(sq, r11, r12, bj)

    w, tau, jpvt, tb, trace, scale, blocks = _block_loop(a, k, b, first, nxt, keep_blocks)
    return RQRCPResult(w, tau, jpvt, tb, trace, scale, blocks, state["info"])


def rsrqrcp(a, omegas, b, p, k=None):
    """Repeated-sampling RQRCP: B^[J] = Omega^[J] A^[J] with a fresh Omega per block.

    ``omegas(J, rows)`` returns the ell x rows Gaussian matrix of block J
    (J = 0 for the first sample over all m rows).
    """
    m, n = np.shape(a)
    k = min(m, n) if k is None else int(k)

    def first(w):
        return np.asarray(omegas(0, m), dtype=np.float64) @ w

    counter = {"J": 0}

    def nxt(sq, r11, r12, w, col0, bj):
        counter["J"] += 1
        trailing = w[col0:, col0:]
        return np.asarray(omegas(counter["J"], trailing.shape[0]), dtype=np.float64) @ trailing

    w, tau, jpvt, tb, trace, scale, _ = _block_loop(a, k, b, first, nxt)
    return RQRCPResult(w, tau, jpvt, tb, trace, scale)


def single_sample_rqrcp(a, omega, k):
    """Algorithm 3: ell = k + p rows of Omega, k pivots from one sample.

    Returns (qr, tau, jpvt, trace) with qr's first k rows holding R (k x n).
    """
    a = np.asarray(a, dtype=np.float64)
    m, n = a.shape
    bmat = np.asarray(omega, dtype=np.float64) @ a
    sq = partial_qrcp(bmat, k)
    w = np.array(a, order="F", copy=True)
    jpvt = np.arange(n, dtype=np.int64)
    apply_transpositions(w, sq.pivots)
    apply_transpositions(jpvt, sq.pivots, axis=0)
    panel, tau = householder_qr(w[:, :k])
    w[:, :k] = panel
    y = unit_lower(panel, k)
    t = form_t(y, tau)
    if k < n:
        w[:, k:] -= y @ (t.T @ (y.T @ w[:, k:]))           # R12 = Q^T A(:, k+1:)
    return w, tau, jpvt, sq.trace
