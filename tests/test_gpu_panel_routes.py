"""The two panel routes of the RQRCP block loop against the FP64 oracle.

Panels whose first Cholesky factor is well conditioned are factored by two
passes of Cholesky QR followed by Householder reconstruction; the others by the
column-by-column Householder loop.  Both must reproduce the oracle's pivots,
R, tau and T (Section 2 reflections, Algorithm 4).  Which route a panel takes
is fixed by the inputs: the tests check the conditioning of the oracle's panels
on the CPU so that each route is known to be exercised.
"""
import numpy as np
import pytest

import oracle
import synth
from test_gpu_rqrcp import ABS, REL, _check_against_oracle, _rqrcp_case, api  # noqa: F401  (fixture)
from tests.helpers import q_from_inplace

pytestmark = pytest.mark.gpu

GATE = 16384.0          # largest/smallest diagonal of the first Cholesky factor


def _panel_diag_ratios(a, om, b, p, k):
    """max/min |R_jj| of each block of the oracle's factorization (pivoted)."""
    ref = oracle.rqrcp(a, om, b, p, k=k)
    d = np.abs(np.diag(ref.qr[:k, :k]))
    return [d[c:c + b].max() / d[c:c + b].min() for c in range(0, k, b)]


def _apply_q(qr, tau, x):
    """H_1 ... H_k x for the reflectors stored below the diagonal of qr."""
    x = np.array(x, dtype=np.float64, copy=True)
    for j in reversed(range(len(tau))):
        v = np.concatenate(([1.0], qr[j + 1:, j]))
        x[j:] -= tau[j] * np.outer(v, v @ x[j:])
    return x


def _check_tall(a, om, b, p, k, qr, jpvt, tau, T):
    """Oracle comparison for tall panels without forming the m x m Q."""
    m, n = a.shape
    ref = oracle.rqrcp(a, om, b, p, k=k)
    pre = ref.trace.prefix(ref.sample_scale, REL, ABS)
    assert sorted(jpvt) == list(range(n))
    np.testing.assert_array_equal(jpvt[:pre], ref.jpvt[:pre])
    rows = min(pre, k)
    d = np.linalg.norm(np.triu(qr[:k])[:rows] - np.triu(ref.qr[:k])[:rows], axis=1)
    nrm = np.linalg.norm(np.triu(ref.qr[:k])[:rows], axis=1)
    assert np.all(d <= 1e-10 * nrm + 1e-12 * np.linalg.norm(a))
    if pre >= k:
        np.testing.assert_allclose(tau, ref.tau, atol=1e-10)
    r_full = np.triu(qr)
    r_full[k:, k:] = qr[k:, k:]
    qk = _apply_q(qr, tau, np.eye(m, k))
    assert np.linalg.norm(qk.T @ qk - np.eye(k), 2) <= 1e-13
    ap = a[:, jpvt]
    assert np.linalg.norm(ap - _apply_q(qr, tau, r_full)) / np.linalg.norm(a) <= 1e-13
    col0 = 0
    while col0 < k:
        bj = min(b, k - col0)
        y = oracle.unit_lower(qr[col0:, col0:col0 + bj], bj)
        np.testing.assert_allclose(T[:bj, col0:col0 + bj], oracle.form_t(y, tau[col0:col0 + bj]),
                                   atol=1e-12)
        col0 += bj


def test_routes_mixed_in_one_factorization(api):
    """Block 1: 64 large Gaussian columns (Cholesky QR); later blocks: steeply
    graded columns (column-by-column route)."""
    m, b, p = 600, 64, 8
    g = synth.gaussian((m, 64), 5100) * 1e3
    h, _ = synth.graded_known_pivots(m, 128, 5101, ratio=0.8, eta=1e-3)
    a = np.asfortranarray(np.hstack([g, h]))
    n = a.shape[1]
    om = synth.omega(b + p, m, 5102)
    ratios = _panel_diag_ratios(a, om, b, p, n)
    assert ratios[0] <= GATE / 10 and min(ratios[1:]) >= GATE * 10, ratios
    qr, jpvt, tau, T = _rqrcp_case(api, m, n, b, p, n, a, om)
    _check_against_oracle(a, om, b, p, n, qr, jpvt, tau, T, min_prefix=64)


@pytest.mark.parametrize("m,n,b", [
    (51200, 96, 64),     # 200 workgroups: some reduce-scatter slices are empty
    (700, 130, 64),      # 3 workgroups: a slice larger than the workgroup
    (90, 90, 48),        # one workgroup, ragged last block
])
def test_cholqr_route_shapes(api, m, n, b):
    p = 8
    a = synth.gaussian((m, n), 5200 + m)
    om = synth.omega(b + p, m, 5201 + n)
    ratios = _panel_diag_ratios(a, om, b, p, min(m, n))
    assert max(ratios[:-1] or [0.0]) <= GATE / 10, ratios
    k = min(m, n)
    qr, jpvt, tau, T = _rqrcp_case(api, m, n, b, p, k, a, om)
    if m > 4000:
        _check_tall(a, om, b, p, k, qr, jpvt, tau, T)
    else:
        _check_against_oracle(a, om, b, p, k, qr, jpvt, tau, T, min_prefix=1)


def _second_pass_offset(a, jpvt, b):
    """max |Q1^T Q1 - I| after one Cholesky-QR pass over the first panel (the
    quantity that selects the closed form of the second pass), in numpy FP64."""
    x = a[:, jpvt[:b]]
    r1 = np.linalg.cholesky(x.T @ x).T
    q1 = np.linalg.solve(r1.T, x.T).T
    return float(np.abs(q1.T @ q1 - np.eye(b)).max())


@pytest.mark.parametrize("kappa", [1.0, 300.0, 3e4])
def test_second_pass_routes(api, kappa):
    """The second Cholesky-QR pass of a tall panel takes one of three routes by
    the offset max|Q1^T Q1 - I| of the first pass: within 64 eps (kappa ~ 1,
    offset ~2 eps) Q1 is kept as it is; up to 1e-10 (kappa = 300, ~1e-12) the
    closed form R2 = I + F is used; beyond (kappa = 3e4, ~6e-9) the Cholesky
    sweep runs, while the first factor's diagonal ratio (~4.4e3) keeps the
    Cholesky-QR route.  All three against the oracle."""
    m, b, p = 3000, 64, 8
    n = k = b
    sig = np.geomspace(1.0, 1.0 / kappa, n)
    a = np.asfortranarray(synth.low_rank(m, n, sig, 5200, 5201))
    om = synth.omega(b + p, m, 5202)
    ref = oracle.rqrcp(a, om, b, p, k=k)
    off = _second_pass_offset(a, ref.jpvt, b)
    eps = np.finfo(np.float64).eps
    if kappa == 1.0:
        assert off <= 8 * eps, off
    elif kappa == 300.0:
        assert 640 * eps <= off <= 1e-11, off
    else:
        assert off >= 1e-9, off
    ratios = _panel_diag_ratios(a, om, b, p, k)
    assert ratios[0] <= GATE / 2, ratios            # the Cholesky-QR route in every case
    qr, jpvt, tau, T = _rqrcp_case(api, m, n, b, p, k, a, om)
    _check_tall(a, om, b, p, k, qr, jpvt, tau, T)


def _kahan(n, theta, pert):
    """Kahan's matrix diag(s^j (1 - pert j)) (I - c striu(ones)), c = cos theta,
    s = sin theta: QRCP keeps its column order, the diagonal of R decays only
    geometrically, yet kappa grows like (1 + c)^n."""
    c, s = np.cos(theta), np.sin(theta)
    k = np.eye(n) - c * np.triu(np.ones((n, n)), 1)
    return np.diag(s ** np.arange(n) * (1.0 - pert * np.arange(n))) @ k


@pytest.mark.parametrize("theta", [1.3, 1.2, 1.15])
def test_kahan_panel_falls_back(api, theta):
    """Kahan-like panels (kappa 1e8 .. 3e12) whose first Cholesky factor has a
    small diagonal ratio (10 .. 3000), so the diagonal gate lets them into the
    Cholesky-QR route: the first pass's offset max|Q1^T Q1 - I| (1e-2 .. 1,
    beyond the 1e-4 limit) sends them to the column-by-column route (a failed
    second Cholesky would too).  With Omega = I (ell = m) the sample QRCP is
    QRCP itself.  Checked is what a backward-stable route guarantees whatever
    kappa: the GPU's own residual and orthogonality, and T.  R and the late
    pivots of such a panel are only determined to about kappa eps (its forward
    condition): the pivots must agree over the first half, and while they
    agree the R rows, matched by column, within 1e-10 ||R_i|| + 64 kappa eps ||A||."""
    m, b, p = 96, 64, 32
    a = np.asfortranarray(synth.haar(m, 64, 5300) @ _kahan(64, theta, 1e-7))
    om = np.eye(m)
    ratios = _panel_diag_ratios(a, om, b, p, 64)
    assert ratios[0] <= GATE / 4, ratios          # the diagonal gate admits the panel
    qr, jpvt, tau, T = _rqrcp_case(api, m, 64, b, p, 64, a, om)
    ref = oracle.rqrcp(a, om, b, p)
    np.testing.assert_array_equal(jpvt[:32], ref.jpvt[:32])
    q = q_from_inplace(qr, tau)
    r = np.triu(qr)
    assert np.linalg.norm(a[:, jpvt] - q @ r) / np.linalg.norm(a) <= 1e-13
    assert np.linalg.norm(q.T @ q - np.eye(m), 2) <= 1e-13
    diff = np.flatnonzero(jpvt != ref.jpvt)
    rows = int(diff[0]) if diff.size else 64
    where = np.empty(64, dtype=np.int64)
    where[ref.jpvt] = np.arange(64)
    r_ref = np.triu(ref.qr)[:64]
    kappa = np.linalg.cond(r_ref)
    d = np.linalg.norm(r[:rows] - r_ref[:rows, where[jpvt]], axis=1)
    assert np.all(d <= 1e-10 * np.linalg.norm(r_ref[:rows], axis=1)
                  + 64 * kappa * np.finfo(float).eps * np.linalg.norm(a))
    np.testing.assert_allclose(T[:64, :64], oracle.form_t(oracle.unit_lower(qr, 64), tau),
                               atol=1e-12)
