"""QR with column pivoting, Businger-Golub form (test infrastructure only).

Follows Algorithm 1 of Duersch & Gu (QRCP with BLAS-2 Householder reflections):
at each step j choose the column with maximal trailing 2-norm, swap it into
position j, form its reflector and apply it to the trailing columns.  The paper
removes row j's contribution from the stored norms; the oracle instead recomputes
every trailing norm exactly at every step, which is the plain definition of
"maximum trailing 2-norm" (the downdate is only a faster route to it).

Reading of unstated details:
* ties: the lowest current position wins (first maximum in position order);
* the permutation is the ordered product of transpositions (j <-> p_j);
* reflectors follow ``oracle.householder.reflector``.

The per-step best and runner-up norms are recorded so tests can tell which pivot
decisions are well separated ("certified") and which are near-ties, where any
choice is acceptable (Section 3.3, sample bias discussion).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .householder import reflector


@dataclass
class PivotTrace:
    """Per-step pivot evidence: best and runner-up trailing norms."""
    best: list = field(default_factory=list)
    second: list = field(default_factory=list)

    def certified(self, nu_scale, rel=1e-10, abs_=1e-13):
        """Boolean per step: gap between best and runner-up exceeds the noise floor."""
        b = np.asarray(self.best)
        s = np.asarray(self.second)
        return (b - s) > rel * b + abs_ * nu_scale

    def prefix(self, nu_scale, rel=1e-10, abs_=1e-13):
        """Length of the leading run of certified steps."""
        c = self.certified(nu_scale, rel, abs_)
        bad = np.flatnonzero(~c)
        return int(bad[0]) if bad.size else int(c.size)


def _trailing_norms(r, j):
    return np.sqrt(np.sum(r[j:, j:] * r[j:, j:], axis=0))


def qrcp_inplace(r, steps, perm=None, trace=None):
    """Run ``steps`` Businger-Golub steps on the float64 array ``r`` in place.

    Every column, including those never chosen, receives every reflection.  On
    return the first ``steps`` rows hold R, reflector tails sit below the
    diagonal of the first ``steps`` columns, and ``r[steps:, steps:]`` holds the
    transformed trailing block.  Returns (tau, pivots) where pivots[j] is the
    position swapped with j at step j.
    """
    m, n = r.shape
    tau = np.zeros(steps)
    pivots = np.zeros(steps, dtype=np.int64)
    for j in range(steps):
        nu = _trailing_norms(r, j)
        q = int(np.argmax(nu))           # first maximum = lowest current position
        if trace is not None:
            trace.best.append(float(nu[q]))
            rest = np.delete(nu, q)
            trace.second.append(float(rest.max()) if rest.size else 0.0)
        p = j + q
        pivots[j] = p
        if p != j:
            r[:, [j, p]] = r[:, [p, j]]
            if perm is not None:
                perm[[j, p]] = perm[[p, j]]
        v, t, beta = reflector(r[j:, j])
        if j + 1 < n:
            w = v @ r[j:, j + 1:]
            r[j:, j + 1:] -= t * np.outer(v, w)
        r[j, j] = beta
        r[j + 1:, j] = v[1:]
        tau[j] = t
    return tau, pivots


@dataclass
class QRCPResult:
    qr: np.ndarray        # m x n: R on/above diagonal, reflector tails below
    tau: np.ndarray       # k reflector coefficients
    jpvt: np.ndarray      # (A P)[:, j] = A[:, jpvt[j]]
    trace: PivotTrace
    nu0_max: float        # largest initial column norm


def qrcp(a, k=None):
    """Algorithm 1 on A (m x n) for k = min(m, n) steps unless given."""
    r = np.array(a, dtype=np.float64, order="F", copy=True)
    m, n = r.shape
    k = min(m, n) if k is None else int(k)
    jpvt = np.arange(n, dtype=np.int64)
    trace = PivotTrace()
    nu0 = float(np.max(np.sqrt(np.sum(r * r, axis=0)))) if n else 0.0
    tau, _ = qrcp_inplace(r, k, jpvt, trace)
    return QRCPResult(r, tau, jpvt, trace, nu0)


@dataclass
class SampleQRCP:
    """Partial QRCP of a sample B (ell x N) for b steps (the sample pivot block).

    ``s`` is the transformed sample [[S11, S12], [0, S22]] in pivoted column
    order with the sub-diagonal of the first b columns zeroed, ``u_qr``/``u_tau``
    keep the sample reflectors (U = H_1 ... H_b), ``pivots`` the transpositions.
    """
    s: np.ndarray
    u_qr: np.ndarray
    u_tau: np.ndarray
    pivots: np.ndarray
    trace: PivotTrace


def partial_qrcp(bmat, steps):
    """QRCP(B, b) of Algorithm 4: only ``steps`` pivots, all columns transformed."""
    r = np.array(bmat, dtype=np.float64, order="F", copy=True)
    trace = PivotTrace()
    tau, piv = qrcp_inplace(r, steps, None, trace)
    s = r.copy()
    for j in range(steps):
        s[j + 1:, j] = 0.0
    return SampleQRCP(s, r, tau, piv, trace)


def apply_transpositions(x, pivots, offset=0, axis=1):
    """Apply transpositions (offset + j <-> offset + pivots[j]) in order along ``axis``."""
    for j, p in enumerate(pivots):
        a, b = offset + j, offset + int(p)
        if a != b:
            if axis == 1:
                x[:, [a, b]] = x[:, [b, a]]
            else:
                x[[a, b]] = x[[b, a]]
    return x
