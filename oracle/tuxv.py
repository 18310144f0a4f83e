"""TUXV approximation of the truncated SVD (test infrastructure only).

Follows Algorithm 6 of Duersch & Gu: TRQRCP gives (U0, R, P); Z0 = R P^T
restores the original column order; an LQ factorization of Z0 (the QR of Z0^T)
gives V1; Z1 = A V1; the QR of Z1 gives U1 and the k x k connection matrix X1,
so A ~ U1 X1 V1^T (eq. TUXV).  Further iterations alternate LQ and QR until
j_max.  The parameter tau of the paper's signature is unused there and dropped.
The optional SVD of X (Section 4.2) is returned as ``sigma``.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .householder import form_q, householder_qr, unit_lower
from .trqrcp import trqrcp


@dataclass
class TUXVResult:
    u: np.ndarray      # m x k orthonormal columns
    x: np.ndarray      # k x k (upper for odd j_max)
    v: np.ndarray      # n x k orthonormal columns
    sigma: np.ndarray  # singular values of X, descending
    trq: object        # the TRQRCP result of the first step


def _thin_qr(z):
    """Householder QR of a tall block: explicit Q[:, :c] and c x c upper R."""
    qr, tau = householder_qr(z)
    c = z.shape[1]
    y = unit_lower(qr, c)
    return form_q(y, tau, c), np.triu(qr[:c, :c])


def tuxv(a, omega, b, p, k, jmax=1):
    a = np.asarray(a, dtype=np.float64)
    m, n = a.shape
    trq = trqrcp(a, omega, b, p, k)
    z0 = np.zeros((k, n))
    z0[:, trq.jpvt] = trq.r                         # Z0 = R P^T
    v, xt = _thin_qr(z0.T)                          # LQ of Z0: Z0 = X0 V1^T
    x = xt.T
    u = None
    j = 1
    while True:
        z = a @ v                                   # Z_j = A V_j
        u, x = _thin_qr(z)                          # X_j upper
        if j == jmax:
            break
        z = u.T @ a                                 # Z_{j+1} = U^T A
        v, xt = _thin_qr(z.T)
        x = xt.T                                    # X_{j+1} lower
        if j + 1 == jmax:
            break
        j += 2
    sigma = np.linalg.svd(x, compute_uv=False)
    return TUXVResult(u, x, v, sigma, trq)
