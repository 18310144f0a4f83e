"""Pins of the oracle's RQRCP (Algorithm 4), RSRQRCP and single-sample RQRCP.

* Omega = I with ell = m reduces RQRCP to textbook QRCP (pivots identical), and
  identity samples of every trailing matrix do the same for RSRQRCP.
* The sample update formula equals an explicit re-projection of the trailing
  matrix with Omega^[J] = (U^T Omega^[J-1] Q)(:, b+1:), and the lower-left block of
  U^T Omega Q vanishes (Sections 3.2 and 3.4, eq. sample / sampleR).
* Invariants of any column-pivoted Householder QR.
* The Gaussian sketch moments E||Omega a||^2 = ell ||a||^2, Var = 2 ell ||a||^4
  (Section 3) and the posterior CDF values printed with Figure 1.
"""
import os

import numpy as np
import pytest
import scipy.special as sps

import oracle
import synth
from tests.helpers import explicit_h, q_from_inplace, q_from_y, spectral_norm

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_identity_compression_reduces_to_qrcp():
    m, n, b, p = 40, 60, 8, 32
    sig = synth.spectrum("pow10", 40, scale=10.0)
    a = synth.low_rank(m, n, sig, 51, 52)
    res = oracle.rqrcp(a, np.eye(m), b, p, k=32)
    ref = oracle.qrcp(a, k=32)
    np.testing.assert_array_equal(res.jpvt, ref.jpvt)
    np.testing.assert_allclose(np.abs(np.triu(res.qr[:32])), np.abs(np.triu(ref.qr[:32])),
                               rtol=1e-10, atol=1e-12)


def test_first_block_pivots_are_qrcp_of_the_sample():
    a = synth.gaussian((80, 70), 61)
    om = synth.omega(12, 80, 62)
    res = oracle.rqrcp(a, om, 8, 4, k=8)
    ref = oracle.qrcp(om @ a, k=8)
    np.testing.assert_array_equal(res.jpvt[:8], ref.jpvt[:8])


def _explicit_u(sq, ell):
    u = np.eye(ell)
    for j in range(len(sq.u_tau)):
        v = np.zeros(ell)
        v[j] = 1.0
        v[j + 1:] = sq.u_qr[j + 1:, j]
        u = u @ explicit_h(v, sq.u_tau[j])
    return u


def test_sample_update_equals_explicit_reprojection():
    m, n, b, p = 60, 50, 6, 4
    ell = b + p
    sig = synth.spectrum("pow10", 50, scale=12.0)
    a = synth.low_rank(m, n, sig, 71, 72)
    om = synth.omega(ell, m, 73)
    res = oracle.rqrcp(a, om, b, p, k=30, keep_blocks=True)
    om_j = om.copy()
    for blk in res.blocks:
        bj = blk["bj"]
        sq = blk["sample"]
        u = _explicit_u(sq, ell)
        q = q_from_y(blk["y"], res.tau[blk["col0"]:blk["col0"] + bj])
        om_hat = u.T @ om_j @ q
        # lower-left block of U^T Omega Q vanishes: Omega_hat_21 = 0
        scale = np.abs(om_hat).max()
        assert np.abs(om_hat[bj:, :bj]).max() <= 1e-12 * scale
        # S11 = Omega_hat_11 R11 (upper triangular Omega_hat_11)
        np.testing.assert_allclose(om_hat[:bj, :bj] @ blk["r11"], sq.s[:bj, :bj],
                                   atol=1e-11 * np.abs(sq.s).max())
        om_j = om_hat[:, bj:]
        if "b_out" in blk:
            explicit = om_j @ blk["a_after"]
            np.testing.assert_allclose(blk["b_out"], explicit,
                                       atol=1e-11 * np.abs(explicit).max())


def test_rqrcp_invariants_and_t_blocks():
    m, n, b, p = 120, 90, 16, 8
    sig = synth.spectrum("pow10", 90, scale=20.0)
    a = synth.low_rank(m, n, sig, 81, 82)
    om = synth.omega(b + p, m, 83)
    res = oracle.rqrcp(a, om, b, p)
    q = q_from_inplace(res.qr, res.tau)
    r = np.triu(res.qr)
    assert np.linalg.norm(a[:, res.jpvt] - q @ r) / np.linalg.norm(a) <= 1e-13
    assert spectral_norm(q.T @ q - np.eye(m)) <= 1e-13
    assert sorted(res.jpvt) == list(range(n))
    col0 = 0
    for t in res.t_blocks:
        bj = t.shape[0]
        y = oracle.unit_lower(res.qr[col0:, col0:col0 + bj], bj)
        prod = np.eye(m - col0)
        for j in range(bj):
            prod = prod @ explicit_h(y[:, j], res.tau[col0 + j])
        np.testing.assert_allclose(np.eye(m - col0) - y @ t @ y.T, prod, atol=1e-13)
        col0 += bj


def test_rqrcp_pivot_quality_tracks_qrcp():
    """|R_jj| follows the known spectrum like QRCP does (Section 5.3 claim)."""
    m = n = 300
    sig = synth.spectrum("pow10", n, scale=30.0)
    a = synth.low_rank(m, n, sig, 91, 92)
    res = oracle.rqrcp(a, synth.omega(40, m, 93), 32, 8)
    ref = oracle.qrcp(a)
    rd = np.abs(np.diag(res.qr))
    qd = np.abs(np.diag(ref.qr))
    ratio = rd / sig
    assert ratio.min() > 1e-2 and ratio.max() < 1e2
    for kk in (30, 100, 200):
        err = np.linalg.norm(np.triu(res.qr)[kk:, kk:])
        err_ref = np.linalg.norm(np.triu(ref.qr)[kk:, kk:])
        assert err <= 4.0 * err_ref
    # the chosen column always carries a sizable fraction of the largest trailing norm
    w = np.array(a, copy=True)[:, res.jpvt]
    q = q_from_inplace(res.qr, res.tau)
    full = q.T @ w
    for j in range(0, 280, 7):
        tail = np.linalg.norm(full[j:, j:], axis=0)
        assert tail[0] >= tail.max() / 8.0


def test_rsrqrcp_first_block_and_invariants():
    m, n, b, p = 70, 60, 8, 6
    a = synth.gaussian((m, n), 101)

    def omegas(j, rows):
        return synth.omega(b + p, rows, 200 + j)

    res = oracle.rsrqrcp(a, omegas, b, p)
    one = oracle.rqrcp(a, omegas(0, m), b, p, k=b)
    np.testing.assert_array_equal(res.jpvt[:b], one.jpvt[:b])
    q = q_from_inplace(res.qr, res.tau)
    assert np.linalg.norm(a[:, res.jpvt] - q @ np.triu(res.qr)) / np.linalg.norm(a) <= 1e-13


def test_rsrqrcp_identity_samples_reduce_to_qrcp():
    """With ell >= m and every Omega^[J] the first rows of the identity, each
    block's fresh sample is the trailing matrix itself padded with zero rows, so
    every block (not only the first) picks textbook QRCP's pivots."""
    m, n, b, p = 24, 40, 4, 20
    sig = synth.spectrum("pow10", 24, scale=8.0)
    a = synth.low_rank(m, n, sig, 121, 122)

    def omegas(j, rows):
        return np.eye(b + p, rows)

    res = oracle.rsrqrcp(a, omegas, b, p, k=20)
    ref = oracle.qrcp(a, k=20)
    np.testing.assert_array_equal(res.jpvt[:20], ref.jpvt[:20])
    np.testing.assert_allclose(np.abs(np.triu(res.qr[:20])), np.abs(np.triu(ref.qr[:20])),
                               rtol=1e-10, atol=1e-12)


def test_single_sample_equals_one_block_rqrcp():
    m, n, k, p = 90, 70, 10, 8
    a = synth.gaussian((m, n), 111)
    om = synth.omega(k + p, m, 112)
    w, tau, jpvt, _ = oracle.single_sample_rqrcp(a, om, k)
    res = oracle.rqrcp(a, om, k, p, k=k)
    np.testing.assert_array_equal(jpvt, res.jpvt)
    np.testing.assert_allclose(np.triu(w[:k]), np.triu(res.qr[:k]), atol=1e-13)


def test_sketch_moments():
    """E||Omega a||^2 = ell ||a||^2 and Var = 2 ell ||a||^4 for Gaussian Omega."""
    ell, m, trials = 8, 5, 200000
    a = np.array([1.0, -2.0, 0.5, 0.0, 3.0])
    om = synth.gaussian((trials, ell, m), 121)
    s = np.sum((om @ a) ** 2, axis=1)
    na2 = a @ a
    assert s.mean() == pytest.approx(ell * na2, rel=0.01)
    assert s.var() == pytest.approx(2 * ell * na2 ** 2, rel=0.03)


def test_latent_cdf_matches_figure1_caption():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "latent_cdf.txt"))
            if l.strip() and not l.startswith("#")]
    for ell_s, tau_s, pct_s in rows:
        ell, tau, pct = int(ell_s), float(tau_s), float(pct_s)
        exact = sps.gammaincc(ell / 2.0, (ell - 2.0) / (2.0 * tau))
        # the caption quotes two significant figures (0.1947% is printed as 0.20%)
        assert abs(100 * exact - pct) <= 0.03 * pct
        trials = 400000
        om = synth.gaussian((trials, ell), 130 + ell)                   # Omega a, ||a|| = 1
        phi = (ell - 2.0) / np.sum(om * om, axis=1)
        freq = np.mean(phi < tau)
        sd = np.sqrt(exact * (1 - exact) / trials)
        assert abs(freq - exact) <= 5 * sd


# ----------------------------------------------------------------------------- rank fallback
def _zero_columns(m, n, r, seed):
    """m x n with r Gaussian columns and n - r exactly zero columns at seeded positions."""
    a = synth.gaussian((m, n), seed)
    zero = synth.rng(seed + 1).permutation(n)[:n - r]
    a[:, zero] = 0.0
    return a, np.sort(zero)


def test_rank_fallback_info_on_zero_columns():
    """Eq. (update1) divides by R11 (Section 3.2).  With r nonzero columns, R_jj = 0
    exactly from j = r on, so the block holding column r reports info = r + 1 and
    the later samples are fresh projections: the result stays finite and is still a
    valid pivoted QR, with an exactly zero trailing block."""
    m, n, r, b, p = 120, 90, 50, 16, 8
    a, zero = _zero_columns(m, n, r, 81)
    res = oracle.rqrcp(a, synth.omega(b + p, m, 82), b, p)
    assert res.info == r + 1
    assert np.isfinite(res.qr).all() and np.isfinite(res.tau).all()
    assert set(res.jpvt[r:]) == set(zero)
    assert np.all(np.triu(res.qr)[r:] == 0.0)
    q = q_from_inplace(res.qr, res.tau)
    assert np.linalg.norm(a[:, res.jpvt] - q @ np.triu(res.qr)) <= 1e-13 * np.linalg.norm(a)
    assert spectral_norm(q.T @ q - np.eye(m)) <= 1e-13
    # the same matrix through plain eq. (update1) would divide by zero
    with np.errstate(all="ignore"):
        blk = oracle.rqrcp(a, synth.omega(b + p, m, 82), b, p, k=64, keep_blocks=True).blocks[3]
    assert np.min(np.abs(np.diag(blk["r11"]))) == 0.0


def test_rank_fallback_identity_compression_reduces_to_qrcp():
    """With Omega = I (ell = m) every sample, updated or re-projected, carries the
    exact trailing norms, so RQRCP with the fallback picks QRCP's pivots at every
    step, past the rank too (zero columns tie and go by position on both sides).
    A fallback that projected the matrix before its block update, or the wrong
    rows of it, would change the pivots after the fallback."""
    m, n, b, p = 48, 40, 8, 40
    a, _ = synth.graded_known_pivots(m, n, 83, ratio=0.8)
    a[:, synth.rng(84).permutation(n)[:12]] = 0.0
    res = oracle.rqrcp(a, np.eye(m), b, p)
    ref = oracle.qrcp(a)
    assert res.info == 29
    np.testing.assert_array_equal(res.jpvt, ref.jpvt)
    np.testing.assert_allclose(np.abs(np.triu(res.qr)[:n]), np.abs(np.triu(ref.qr)[:n]),
                               rtol=1e-10, atol=1e-13)


def test_rank_fallback_quiet_on_full_rank():
    m, n, b, p = 300, 240, 32, 8
    sig = synth.spectrum("pow10", 240, scale=40.0)
    a = synth.low_rank(m, n, sig, 85, 86)
    assert oracle.rqrcp(a, synth.omega(b + p, m, 87), b, p).info == 0


def test_exact_tie_goes_to_lowest_position():
    """Duplicated columns give bitwise-equal sample norms: the first step is an
    exact tie, which the lowest current position wins (reading c2)."""
    a = synth.gaussian((300, 240), 11)
    a[:, 3] *= 10.0
    a[:, 7] = a[:, 3]
    res = oracle.rqrcp(a, synth.omega(40, 300, 12), 32, 8)
    assert res.trace.best[0] == res.trace.second[0]
    assert res.jpvt[0] == 3
