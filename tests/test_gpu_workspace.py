"""GPU check of the workspace query: after rq_workspace_reserve of what
rq_workspace_query reports, running the entry point does not grow the handle's
workspace (the query covers everything the call carves), and the query is not
far above what a call actually needs to have reserved."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    from paper_2008_04447_amd import api as _api
    return _api


def _run(api, op, h, m, n, k, b, p, f32):
    from paper_2008_04447_amd import _lib
    dev = torch.device("cuda", 0)
    a = synth.gaussian((m, n), 4700)
    om = api.colmajor(synth.omega(b + p, m, 4701), device=dev)
    A = api.colmajor(a, dtype=torch.float32 if f32 else torch.float64, device=dev)
    if op == _lib.RQ_OP_RQRCP:
        api.rqrcp_factor(A, om, b, p, k, handle=h)
    elif op == _lib.RQ_OP_RSRQRCP:
        nblk = (k + b - 1) // b
        oms = torch.from_numpy(np.ascontiguousarray(synth.gaussian((nblk, m, b + p), 4702))).to(dev)
        api.rsrqrcp_factor(A, oms, b, p, k, handle=h)
    elif op == _lib.RQ_OP_QRCP:
        api.qrcp_factor(A, k, nb=b, handle=h)
    elif op == _lib.RQ_OP_TRQRCP:
        api.trqrcp_truncate(A, om, b, p, k, handle=h)
    elif op == _lib.RQ_OP_TUXV:
        api.tuxv_svd(A, om, b, p, k, handle=h)
    elif op == _lib.RQ_OP_SKETCH:
        api.sketch(om, A, handle=h)
    else:
        api.sample_qrcp(api.colmajor(synth.gaussian((b + p, n), 4703), device=dev), k, handle=h)
    h.sync()


@pytest.mark.parametrize("opname,f32", [("RQRCP", False), ("RSRQRCP", False), ("QRCP", False),
                                        ("TRQRCP", False), ("TRQRCP", True), ("TUXV", False),
                                        ("TUXV", True), ("SKETCH", True), ("SAMPLE_QRCP", False)])
def test_reserved_workspace_is_enough(api, opname, f32):
    from paper_2008_04447_amd import _lib
    op = getattr(_lib, "RQ_OP_" + opname)
    m, n, k, b, p = 700, 530, 96, 32, 8
    if opname == "SAMPLE_QRCP":
        k = 32
    prec = _lib.RQ_MIXED_BF16 if f32 else _lib.RQ_FP64
    # a call on a fresh handle reserves exactly the query (plus its growth margin)
    h0 = api.Handle(0)
    q = h0.workspace_query(op, m, n, k, b, p, prec)
    assert q > 0
    _run(api, op, h0, m, n, k, b, p, f32)
    grown = h0.workspace_size()
    assert q <= grown <= q + q // 8 + 1, (q, grown)
    # after reserving the query the call allocates nothing more
    h1 = api.Handle(0)
    h1.workspace_reserve(q)
    before = h1.workspace_size()
    _run(api, op, h1, m, n, k, b, p, f32)
    assert h1.workspace_size() == before
    h0.close()
    h1.close()
