"""Test-side helpers that rebuild factors from stored reflectors one explicit
Householder matrix at a time (an arithmetic route independent of the oracle's
compact-WY code)."""
import numpy as np


def explicit_h(v, tau):
    v = np.asarray(v, dtype=np.float64)
    return np.eye(v.size) - tau * np.outer(v, v)


def q_from_inplace(qr, tau, m=None):
    """Full m x m Q = H_1 ... H_k from an in-place array (tails below the diagonal)."""
    qr = np.asarray(qr, dtype=np.float64)
    m = qr.shape[0] if m is None else m
    q = np.eye(m)
    for j in range(len(tau)):
        v = np.zeros(m)
        v[j] = 1.0
        v[j + 1:] = qr[j + 1:, j]
        q = q @ explicit_h(v, tau[j])
    return q


def q_from_y(y, tau):
    m = y.shape[0]
    q = np.eye(m)
    for j in range(y.shape[1]):
        q = q @ explicit_h(y[:, j], tau[j])
    return q


def spectral_norm(x):
    return float(np.linalg.norm(x, 2))
