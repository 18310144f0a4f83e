"""Householder building blocks of the FP64 oracle (test infrastructure only).

Plain numpy float64, no blocking beyond what the paper's formulas state.

Paper passages followed (Duersch & Gu, arXiv:2008.04447):
* Section 2 (Related Work), reflector definition: y = x - (-sign(x_1) ||x|| e_1),
  tau = 2 / y^T y, H = I - y tau y^T.  The oracle stores the same reflector
  rescaled so its leading entry is 1 (the in-place storage of Section 2.2, where
  reflectors occupy the strict lower triangle).
* Section 2.1, compact WY form: Q = I - Y T Y^T with T upper triangular.
"""
from __future__ import annotations

import numpy as np


def reflector(x):
    """Reflector of column x: returns (v, tau, beta) with (I - tau v v^T) x = beta e_1.

    beta = -sign(x_0) ||x|| with sign(0) = +1, v = (x - beta e_1)/(x_0 - beta)
    (so v_0 = 1) and tau = (beta - x_0)/beta, which equals the paper's
    2/(y^T y) after the rescaling y = (x_0 - beta) v.  A column whose tail is zero
    but x_0 != 0 is still reflected (tau = 2, beta = -x_0), as the paper's formula
    gives.  An all-zero column has no reflection: tau = 0, beta = 0, v = e_1.
    """
    x = np.array(x, dtype=np.float64, copy=True)
    alpha = x[0]
    s = float(np.sqrt(np.dot(x, x)))
    v = np.zeros_like(x)
    v[0] = 1.0
    if s == 0.0:
        return v, 0.0, 0.0
    sgn = 1.0 if alpha >= 0.0 else -1.0
    beta = -sgn * s
    v[1:] = x[1:] / (alpha - beta)
    tau = (beta - alpha) / beta
    return v, tau, beta


def householder_qr(a):
    """Unpivoted Householder QR of an M x c block (Section 2 reflections, no pivoting).

    Returns (qr, tau) with R on/above the diagonal of ``qr`` and the reflector
    tails below it (unit diagonal implicit).
    """
    r = np.array(a, dtype=np.float64, order="F", copy=True)
    m, c = r.shape
    steps = min(m, c)
    tau = np.zeros(steps)
    for j in range(steps):
        v, t, beta = reflector(r[j:, j])
        if j + 1 < c:
            w = v @ r[j:, j + 1:]
            r[j:, j + 1:] -= t * np.outer(v, w)
        r[j, j] = beta
        r[j + 1:, j] = v[1:]
        tau[j] = t
    return r, tau


def unit_lower(qr, c=None):
    """Explicit reflector matrix Y (M x c): unit diagonal, zeros above, tails below."""
    m = qr.shape[0]
    c = qr.shape[1] if c is None else c
    y = np.tril(np.asarray(qr[:, :c], dtype=np.float64), -1)
    y[np.arange(min(m, c)), np.arange(min(m, c))] = 1.0
    return y


def form_t(y, tau):
    """Compact-WY connection matrix T with H_1 ... H_c = I - Y T Y^T (Section 2.1).

    Forward recurrence: T[j, j] = tau_j and
    T[:j, j] = -tau_j T[:j, :j] (Y[:, :j]^T y_j).
    """
    c = y.shape[1]
    t = np.zeros((c, c))
    for j in range(c):
        t[j, j] = tau[j]
        if j:
            t[:j, j] = -tau[j] * (t[:j, :j] @ (y[:, :j].T @ y[:, j]))
    return t


def form_q(y, tau, ncols=None):
    """Explicit Q[:, :ncols] = H_1 ... H_c [I; 0], applying reflectors right to left."""
    m, c = y.shape
    ncols = c if ncols is None else ncols
    q = np.zeros((m, ncols))
    q[np.arange(min(m, ncols)), np.arange(min(m, ncols))] = 1.0
    for j in reversed(range(c)):
        v = y[:, j]
        q -= tau[j] * np.outer(v, v @ q)
    return q
