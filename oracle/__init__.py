"""FP64 CPU oracle for the RQRCP family (Duersch & Gu, arXiv:2008.04447).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import or call anything here; the library in
``paper_2008_04447_amd`` never does, and shares no code with it.

Plain, slow, float64 numpy that follows the paper's algorithms step by step:
* ``qrcp``              Algorithm 1 (Businger-Golub QRCP, exact trailing norms);
* ``partial_qrcp``      QRCP(B, b) on a sample, all columns transformed;
* ``rqrcp``             Algorithm 4 with the sample update eq. (update1);
* ``rsrqrcp``           Algorithm 4 with repeated sampling (Section 3.4);
* ``single_sample_rqrcp`` Algorithm 3;
* ``trqrcp``            Algorithm 5 (truncated, no trailing update);
* ``tuxv``              Algorithm 6 (TUXV, j_max iterations).

Every function is pinned by ``tests/test_oracle_*.py`` against brute force,
closed forms, identities stated in the paper, LAPACK (scipy) on well-separated
inputs and theorems that bound QRCP's diagonal.  The per-step pivot evidence is
reported through ``PivotTrace`` so parity tests can restrict exact pivot
comparison to well-separated decisions.
"""
from .householder import form_q, form_t, householder_qr, reflector, unit_lower
from .qrcp import (PivotTrace, QRCPResult, SampleQRCP, apply_transpositions,
                   partial_qrcp, qrcp, qrcp_inplace)
from .rqrcp import RQRCPResult, rqrcp, rsrqrcp, sample_update, single_sample_rqrcp
from .trqrcp import TRQRCPResult, trqrcp
from .tuxv import TUXVResult, tuxv

__all__ = [
    "form_q", "form_t", "householder_qr", "reflector", "unit_lower",
    "PivotTrace", "QRCPResult", "SampleQRCP", "apply_transpositions", "partial_qrcp",
    "qrcp", "qrcp_inplace", "RQRCPResult", "rqrcp", "rsrqrcp", "sample_update",
    "single_sample_rqrcp", "TRQRCPResult", "trqrcp", "TUXVResult", "tuxv",
]
