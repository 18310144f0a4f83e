"""Pins of the oracle's Householder reflector and Businger-Golub QRCP.

Every check here compares the oracle against something other than itself:
explicit reflection matrices, brute force over all column orders, Gram
determinants, LAPACK's dgeqp3 (through scipy), closed-form inputs and theorems
bounding QRCP's diagonal.
"""
import itertools

import numpy as np
import pytest
import scipy.linalg as sla

import oracle
import synth
from tests.helpers import explicit_h, q_from_inplace, spectral_norm


# ---------------------------------------------------------------- reflector
@pytest.mark.parametrize("seed", range(5))
def test_reflector_maps_to_axis_and_matches_paper_form(seed):
    x = synth.gaussian((7,), 100 + seed)
    v, tau, beta = oracle.reflector(x)
    h = explicit_h(v, tau)
    e1 = np.zeros(7)
    e1[0] = 1.0
    np.testing.assert_allclose(h @ x, beta * e1, atol=1e-14 * np.linalg.norm(x))
    np.testing.assert_allclose(h @ h.T, np.eye(7), atol=1e-14)
    assert v[0] == 1.0
    assert abs(abs(beta) - np.linalg.norm(x)) <= 1e-14 * np.linalg.norm(x)
    assert np.sign(beta) == -np.sign(x[0])                 # -sign(a_1) ||a|| e_1
    # the paper's unscaled form: y = a + sign(a_1)||a|| e_1, tau = 2/(y^T y)
    y = x.copy()
    y[0] += np.sign(x[0]) * np.linalg.norm(x)
    h_paper = np.eye(7) - np.outer(y, y) * (2.0 / (y @ y))
    np.testing.assert_allclose(h, h_paper, atol=1e-14)
    assert np.linalg.norm(y) >= np.linalg.norm(x)           # stability remark


def test_reflector_special_cases():
    v, tau, beta = oracle.reflector(np.array([0.0, 3.0, 4.0]))     # sign(0) = +1
    assert beta == -5.0
    np.testing.assert_allclose(explicit_h(v, tau) @ [0.0, 3.0, 4.0], [-5.0, 0, 0], atol=1e-15)
    v, tau, beta = oracle.reflector(np.array([2.0, 0.0, 0.0]))     # zero tail: reflect
    assert (tau, beta) == (2.0, -2.0)
    v, tau, beta = oracle.reflector(np.zeros(3))                    # zero column: identity
    assert (tau, beta) == (0.0, 0.0)


def test_unpivoted_qr_matches_lapack_up_to_signs():
    a = synth.gaussian((30, 12), 7)
    qr, tau = oracle.householder_qr(a)
    r_or = np.triu(qr[:12])
    q_la, r_la = np.linalg.qr(a)
    np.testing.assert_allclose(np.abs(r_or), np.abs(r_la), rtol=1e-12, atol=1e-13)
    q = q_from_inplace(qr, tau)[:, :12]
    d = np.sign(np.diag(r_or)) * np.sign(np.diag(r_la))
    np.testing.assert_allclose(q, q_la * d[None, :], atol=1e-13)


def test_form_t_equals_product_of_reflections():
    a = synth.gaussian((20, 6), 8)
    qr, tau = oracle.householder_qr(a)
    y = oracle.unit_lower(qr, 6)
    t = oracle.form_t(y, tau)
    prod = np.eye(20)
    for j in range(6):
        prod = prod @ explicit_h(y[:, j], tau[j])
    np.testing.assert_allclose(np.eye(20) - y @ t @ y.T, prod, atol=1e-14)
    assert np.allclose(t, np.triu(t))


# ---------------------------------------------------------------- QRCP
def _greedy_certificate(a, perm):
    """|R_jj| >= ||R(j:, c)|| for every later column c (the QRCP choice rule)."""
    r = np.linalg.qr(a[:, perm], mode="r")
    n = a.shape[1]
    for j in range(n):
        tail = np.linalg.norm(r[j:, j:], axis=0)
        if np.any(tail[1:] > abs(r[j, j]) * (1 + 1e-12)):
            return False
    return True


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_qrcp_brute_force_6x6(seed):
    a = synth.gaussian((6, 6), seed) * (1.0 + np.arange(6))[None, :] ** 0.5
    winners = [p for p in itertools.permutations(range(6)) if _greedy_certificate(a, list(p))]
    assert len(winners) == 1
    res = oracle.qrcp(a)
    assert list(res.jpvt) == list(winners[0])


@pytest.mark.parametrize("seed", [4, 5])
def test_qrcp_greedy_volume_from_gram_determinants(seed):
    """Each pivot maximizes sqrt(det(A_S^T A_S)) over S + {c} (Section 2)."""
    a = synth.gaussian((8, 6), seed)
    res = oracle.qrcp(a)
    chosen = []
    for j in range(6):
        best, arg = -1.0, None
        for c in range(6):
            if c in chosen:
                continue
            s = chosen + [c]
            vol = np.linalg.det(a[:, s].T @ a[:, s])
            if vol > best:
                best, arg = vol, c
        assert res.jpvt[j] == arg
        chosen.append(arg)


def test_qrcp_known_pivots_and_lapack_dgeqp3():
    a, perm = synth.graded_known_pivots(60, 40, 21, decay=4.0, eta=1e-3)
    res = oracle.qrcp(a)
    np.testing.assert_array_equal(res.jpvt, perm)
    d = 10.0 ** (-4.0 * np.arange(40) / 40)
    np.testing.assert_allclose(np.abs(np.diag(res.qr)[:40]), d, rtol=2e-2)
    r_la, piv_la = sla.qr(a, mode="r", pivoting=True)
    np.testing.assert_array_equal(res.jpvt, piv_la)
    np.testing.assert_allclose(np.abs(np.triu(res.qr[:40])), np.abs(r_la[:40]),
                               rtol=1e-12, atol=1e-12 * np.abs(r_la).max())


def test_qrcp_theorems_and_invariants():
    m, n = 50, 40
    sig = synth.spectrum("pow10", n, scale=8.0)
    a = synth.low_rank(m, n, sig, 31, 32)
    res = oracle.qrcp(a)
    rdiag = np.abs(np.diag(res.qr)[:n])
    assert rdiag[0] == pytest.approx(np.linalg.norm(a, axis=0).max(), rel=1e-14)
    assert np.all(rdiag[1:] <= rdiag[:-1] * (1 + 1e-12))            # non-increasing
    sv = np.linalg.svd(a, compute_uv=False)
    assert np.all(rdiag >= sv[:n] / np.sqrt(n - np.arange(n)) * (1 - 1e-10))
    assert np.all(np.cumsum(np.log(rdiag)) <= np.cumsum(np.log(sv[:n])) + 1e-10)
    q = q_from_inplace(res.qr, res.tau)
    r = np.triu(res.qr)
    ap = a[:, res.jpvt]
    assert np.linalg.norm(ap - q @ r) / np.linalg.norm(a) <= 1e-13
    assert spectral_norm(q.T @ q - np.eye(m)) <= 1e-13


def test_partial_qrcp_trailing_frobenius_equals_trailing_norms():
    a = synth.gaussian((30, 25), 41)
    r = np.array(a, copy=True)
    tau, piv = oracle.qrcp_inplace(r, 7)
    # orthogonal invariance: ||A||_F^2 = ||R(0:7, :)||_F^2 + ||trailing block||_F^2
    top = np.triu(r[:7])
    assert np.linalg.norm(a) ** 2 == pytest.approx(
        np.linalg.norm(top) ** 2 + np.linalg.norm(r[7:, 7:]) ** 2, rel=1e-13)
    # and the leading 7 rows + trailing block reproduce A P up to the 7 reflections
    perm = np.arange(25)
    oracle.apply_transpositions(perm, piv, axis=0)
    q = q_from_inplace(r, tau)
    full = np.triu(r)
    full[7:, 7:] = r[7:, 7:]
    np.testing.assert_allclose(q @ full, a[:, perm], atol=1e-13 * np.abs(a).max())
