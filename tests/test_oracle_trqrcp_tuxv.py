"""Pins of the oracle's TRQRCP (Algorithm 5) and TUXV (Algorithm 6).

* TRQRCP gives the same pivots, reflectors and R rows as RQRCP stopped at rank k
  with the same Omega (Section 4.1: it only avoids the trailing update).
* I - Y T Y^T equals the product of the explicit reflections; W^T = T^T Y^T A P.
* The selected columns rebuilt from A - Y W^T agree with the R rows already
  finished; rows of A - Y W^T for a block vanish left of the block.
* TUXV: U X V^T = A V V^T, Eckart-Young / projection error sandwich, singular
  value interlacing, exact recovery on rank-k input, and equality with QLP from
  a full RQRCP truncated to rank k (Section 4.2).
"""
import numpy as np
import pytest

import oracle
import synth
from tests.helpers import explicit_h, q_from_inplace


def _case(m=90, n=70, b=8, p=6, k=24, seed=300):
    sig = synth.spectrum("pow10", min(m, n), scale=15.0)
    a = synth.low_rank(m, n, sig, seed, seed + 1)
    om = synth.omega(b + p, m, seed + 2)
    return a, om, b, p, k


def test_trqrcp_equals_truncated_rqrcp():
    a, om, b, p, k = _case()
    tr = oracle.trqrcp(a, om, b, p, k)
    rq = oracle.rqrcp(a, om, b, p, k=k)
    np.testing.assert_array_equal(tr.jpvt, rq.jpvt)
    y_rq = oracle.unit_lower(rq.qr, k)
    np.testing.assert_allclose(tr.y, y_rq, atol=1e-12)
    np.testing.assert_allclose(tr.r, np.triu(rq.qr[:k]), atol=1e-12 * np.abs(tr.r).max())
    np.testing.assert_allclose(tr.tau, rq.tau, atol=1e-13)


def test_trqrcp_t_and_inner_products():
    a, om, b, p, k = _case(seed=310)
    tr = oracle.trqrcp(a, om, b, p, k, keep_blocks=True)
    m = a.shape[0]
    prod = np.eye(m)
    for j in range(k):
        prod = prod @ explicit_h(tr.y[:, j], tr.tau[j])
    np.testing.assert_allclose(np.eye(m) - tr.y @ tr.t @ tr.y.T, prod, atol=1e-13)
    ap = a[:, tr.jpvt]
    np.testing.assert_allclose(tr.wt, tr.t.T @ tr.y.T @ ap, atol=1e-12 * np.abs(ap).max())
    for blk in tr.blocks:
        c0, bj = blk["col0"], blk["bj"]
        if c0:
            np.testing.assert_allclose(blk["a_hat"][:c0], tr.r[:c0, c0:c0 + bj],
                                       atol=1e-12 * np.abs(a).max())
            assert np.abs(blk["rows"][:, :c0]).max() <= 1e-12 * np.abs(a).max()


def test_tuxv_closed_form_and_error_sandwich():
    a, om, b, p, k = _case(m=120, n=100, b=8, p=8, k=24, seed=320)
    res = oracle.tuxv(a, om, b, p, k)
    u, x, v = res.u, res.x, res.v
    np.testing.assert_allclose(u.T @ u, np.eye(k), atol=1e-13)
    np.testing.assert_allclose(v.T @ v, np.eye(k), atol=1e-13)
    assert np.allclose(x, np.triu(x))
    np.testing.assert_allclose(u @ x @ v.T, a @ v @ v.T, atol=1e-13 * np.abs(a).max())
    sv = np.linalg.svd(a, compute_uv=False)
    e_svd = np.sqrt(np.sum(sv[k:] ** 2))
    e_tuxv = np.linalg.norm(a - u @ x @ v.T)
    q = q_from_inplace(np.pad(res.trq.y, ((0, 0), (0, 0))), res.trq.tau)[:, :k]
    z0 = np.zeros((k, a.shape[1]))
    z0[:, res.trq.jpvt] = res.trq.r
    e_qr = np.linalg.norm(a - q @ z0)
    assert e_svd * (1 - 1e-12) <= e_tuxv <= e_qr * (1 + 1e-12)
    assert np.all(res.sigma <= sv[:k] * (1 + 1e-12))


def test_tuxv_exact_rank_k_recovers_singular_values():
    m, n, k = 80, 60, 12
    sig = synth.spectrum("pow10", k, scale=6.0)
    a = synth.low_rank(m, n, sig, 330, 331)
    res = oracle.tuxv(a, synth.omega(12, m, 332), 4, 8, k)
    np.testing.assert_allclose(res.sigma, sig, rtol=1e-12)
    assert np.linalg.norm(a - res.u @ res.x @ res.v.T) <= 1e-13 * np.linalg.norm(a)


def test_tuxv_equals_truncated_full_qlp():
    """Section 4.2: TUXV (j_max=1) equals QLP via full RQRCP, truncated to rank k."""
    m, n, b, p, k = 100, 80, 8, 6, 16
    a, om, *_ = _case(m=m, n=n, b=b, p=p, k=k, seed=340)
    res = oracle.tuxv(a, om, b, p, k)
    full = oracle.rqrcp(a, om, b, p)
    r = np.triu(full.qr[:min(m, n)])
    z = np.zeros_like(r)
    z[:, full.jpvt] = r                                # R P^T
    # LQ of R P^T via QR of its transpose; leading k columns of L
    qt, lt = np.linalg.qr(z.T)
    vk = qt[:, :k]
    approx_full = a @ vk @ vk.T                          # Q0 L(:, :k) V(:, :k)^T
    np.testing.assert_allclose(res.u @ res.x @ res.v.T, approx_full,
                               atol=1e-11 * np.abs(a).max())


def test_tuxv_second_iteration_runs_and_is_lower_triangular():
    a, om, b, p, k = _case(m=70, n=60, b=8, p=6, k=16, seed=350)
    r1 = oracle.tuxv(a, om, b, p, k, jmax=1)
    r2 = oracle.tuxv(a, om, b, p, k, jmax=2)
    assert np.allclose(r2.x, np.tril(r2.x))
    e1 = np.linalg.norm(a - r1.u @ r1.x @ r1.v.T)
    e2 = np.linalg.norm(a - r2.u @ r2.x @ r2.v.T)
    assert e2 <= e1 * (1 + 1e-10)


def test_tuxv_alternations_converge_to_the_truncated_svd():
    """Each alternation of Algorithm 6 is one step of subspace iteration.
    After an odd number of steps U X V^T = A V V^T, and after an even number it
    is U U^T A.  Each is the best approximation in a subspace that contains the
    previous one, so the error never grows.  With a gap sigma_{k+1} / sigma_k = 0.1
    it reaches the Eckart-Young optimum geometrically."""
    m, n, k, b, p = 90, 70, 12, 8, 6
    sig = np.concatenate([np.linspace(1.0, 0.5, k), 0.05 * np.linspace(1.0, 0.1, min(m, n) - k)])
    a = synth.low_rank(m, n, sig, 410, 411)
    om = synth.omega(b + p, m, 412)
    opt = np.sqrt(np.sum(sig[k:] ** 2))
    excess = []
    for jmax in range(1, 7):
        r = oracle.tuxv(a, om, b, p, k, jmax=jmax)
        approx = r.u @ r.x @ r.v.T
        closed = a @ r.v @ r.v.T if jmax % 2 else r.u @ (r.u.T @ a)
        np.testing.assert_allclose(approx, closed, atol=1e-13)
        tri = np.triu(r.x) if jmax % 2 else np.tril(r.x)
        np.testing.assert_array_equal(r.x, tri)
        excess.append(np.linalg.norm(a - approx) / opt - 1.0)
    assert excess[0] > 1e-4                        # one pass is visibly short of optimal
    assert all(e2 <= e1 + 1e-14 for e1, e2 in zip(excess, excess[1:]))
    assert excess[-1] <= 1e-9
