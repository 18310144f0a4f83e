"""The zero-allocation sample QRCP (rq_sample_qrcp_noalloc) against the
workspace-backed rq_sample_qrcp: same kernels, so the results must agree bit
for bit, on two calls in a row (the second smaller, so stale scratch contents
from the first call must not leak into it)."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    from paper_2008_04447_amd import api as _api
    return _api


def _dev(api, x):
    return api.colmajor(x, device=torch.device("cuda", 0))


def test_noalloc_matches_workspace_entry_point(api):
    h = api.Handle(0)
    cases = [(72, 16384, 64, 9100), (72, 8000, 64, 9101), (40, 1000, 32, 9102)]
    for ell, n, steps, seed in cases:
        print(f"noalloc case ell={ell} n={n} steps={steps} seed={seed}", flush=True)
        b = synth.gaussian((ell, n), seed) * (1.0 + np.arange(n) % 5)[None, :]
        B_ref = _dev(api, b)
        perm_ref = api.sample_qrcp(B_ref, steps, handle=h)
        h.sync()
        B = _dev(api, b)
        perm = torch.full((n,), -7, dtype=torch.int64, device=B.device)
        api.sample_qrcp_noalloc(B, steps, perm, handle=h)
        h.sync()
        assert torch.equal(perm, perm_ref)
        assert torch.equal(B, B_ref)
        assert sorted(perm.cpu().numpy()) == list(range(n))
    h.close()


def test_noalloc_rejects_beyond_scratch(api):
    from paper_2008_04447_amd import _lib
    h = api.Handle(0)
    n = 16385
    B = api.empty_colmajor(8, n, torch.float64, torch.device("cuda", 0))
    perm = torch.empty(n, dtype=torch.int64, device=B.device)
    with pytest.raises(api.RQError) as e:
        api.sample_qrcp_noalloc(B, 4, perm, handle=h)
    assert e.value.code == _lib.RQ_E_UNSUPPORTED
    h.close()
