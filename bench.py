#!/usr/bin/env python3
"""Benchmark of the RQRCP hot path on one MI355X.

Default workload: FP64 RQRCP full factorization of an 8000 x 8000 i.i.d. N(0,1)
matrix with b = 64, p = 8 (Omega 72 x 8000).  One step = the whole hot path on
one resident copy of A: sketch, then per block the sample QRCP, permutation,
panel + T, inner products, trailing update and sample update.  Every step
factors its own pre-staged copy of A, so nothing but the factorization runs in
the timed region.  The throughput counts the nominal 4n^3/3 flops of a full
Householder QR (the same count used for plain QRCP and unpivoted QR).

Prints progress on stderr and one JSON line on stdout.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp64_tflops": 78.6, "hbm_gbs": 8000.0}
MFMA_CLASSES = {"sketch", "inner_products", "trailing_update", "sample_update", "qp3_gemv"}


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def nominal_qr_flops(m, n, k):
    """Householder QR flops for k columns of an m x n matrix: sum_j 4 (m-j)(n-j)."""
    return float(sum(4.0 * (m - j) * (n - j) for j in range(k)))


def profile_table(h):
    from paper_2008_04447_amd import _lib
    import ctypes
    lib = _lib.load()
    out = {}
    for i in range(lib.rq_profile_count(h.ptr)):
        name = ctypes.c_char_p()
        launches = ctypes.c_int64()
        ms, fl, by = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        lib.rq_profile_get(h.ptr, i, ctypes.byref(name), ctypes.byref(launches), ctypes.byref(ms),
                           ctypes.byref(fl), ctypes.byref(by))
        if launches.value:
            out[name.value.decode()] = dict(launches=launches.value, ms=ms.value, flops=fl.value,
                                            bytes=by.value)
    return out


def roofline(prof, steps):
    """Roofline entry of the kernel class with the largest total time."""
    name, rec = max(prof.items(), key=lambda kv: kv[1]["ms"])
    sec = rec["ms"] * 1e-3
    if name in MFMA_CLASSES:
        achieved = rec["flops"] / sec / 1e12
        peak = PEAK["fp64_tflops"]
        bound, unit = "mfma", "TFLOP/s"
    else:
        achieved = rec["bytes"] / sec / 1e9
        peak = PEAK["hbm_gbs"]
        bound, unit = "hbm", "GB/s"
    return {"kernel": name, "bound": bound, "achieved": round(achieved, 4), "peak": peak,
            "unit": unit, "frac": round(achieved / peak, 5), "traffic": None,
            "launches_per_step": rec["launches"] / steps,
            "avg_launch_us": round(rec["ms"] * 1e3 / rec["launches"], 3),
            "share_of_step": None}


def cpu_baseline(a, om, b, p, kc):
    """The FP64 oracle on a bounded sample: the first kc pivots of the same matrix."""
    import numpy as np  # noqa: F401
    import oracle
    cores = len(os.sched_getaffinity(0))
    t = time.perf_counter()
    oracle.rqrcp(a, om, b, p, k=kc)
    dt = time.perf_counter() - t
    m, n = a.shape
    fl = nominal_qr_flops(m, n, kc)
    return {"value": round(fl / dt / 1e12, 6), "unit": "TFLOP/s", "cores": cores, "kind": "oracle",
            "seconds": round(dt, 3),
            "sample": f"oracle RQRCP (numpy FP64) of the first {kc} pivots ({kc // b} blocks) of "
                      f"the same {m}x{n} matrix; flops = sum_j<{kc} 4(m-j)(n-j)"}


def bench_rqrcp(args):
    import numpy as np
    import torch

    import synth
    from paper_2008_04447_amd import _lib, api

    m = n = args.n
    b, p = 64, 8
    ell = b + p
    dev = torch.device("cuda", 0)
    log(f"generating A {m}x{n} N(0,1) and Omega {ell}x{m}")
    a = synth.gaussian((m, n), synth.seed_for(1, "U"))
    om = synth.omega(ell, m, synth.seed_for(1, "Omega"))
    A0 = api.colmajor(a, device=dev)
    Om = api.colmajor(om, device=dev)
    copies = [A0.clone(memory_format=torch.preserve_format) for _ in range(args.warmup + args.steps)]
    for c in copies:
        assert c.stride(0) == 1
    h = api.default_handle(0)
    torch.cuda.synchronize()
    log(f"warmup {args.warmup} step(s)")
    for i in range(args.warmup):
        api.rqrcp_factor(copies[i], Om, b, p, handle=h)
        h.sync()
    lib = _lib.load()
    lib.rq_profile_start(h.ptr)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outs = []
    for i in range(args.steps):
        outs.append(api.rqrcp_factor(copies[args.warmup + i], Om, b, p, handle=h))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lib.rq_profile_stop(h.ptr)
    h.sync()
    ms = (t1 - t0) * 1e3 / args.steps
    prof = profile_table(h)
    flops = nominal_qr_flops(m, n, n)
    value = flops / (ms * 1e-3) / 1e12
    log(f"timed {args.steps} step(s): {ms:.2f} ms/step, {value:.3f} TFLOP/s")

    # quick correctness guard: first block of pivots equals the oracle's sample QRCP
    jpvt = outs[-1][0].cpu().numpy()
    import oracle
    sq = oracle.partial_qrcp(om @ a, b)
    first = np.arange(n)
    oracle.apply_transpositions(first, sq.pivots, axis=0)
    pre = sq.trace.prefix(float(np.linalg.norm(om @ a, axis=0).max()), 1e-10, 1e-13)
    ok = bool(np.array_equal(jpvt[:pre], first[:pre]))
    log(f"first-block pivots vs oracle: certified prefix {pre}, equal={ok}")

    plain = None
    if not args.no_plain:
        # plain QRCP (Algorithm 2) on the same matrix, same device: the comparator
        qsteps = max(1, min(args.steps, 2))
        qcopies = [A0.clone(memory_format=torch.preserve_format) for _ in range(qsteps + 1)]
        log(f"plain QRCP: 1 warmup + {qsteps} timed step(s)")
        api.qrcp_factor(qcopies[0], nb=32, handle=h)
        h.sync()
        lib.rq_profile_start(h.ptr)
        torch.cuda.synchronize()
        tq0 = time.perf_counter()
        for i in range(qsteps):
            qj, _ = api.qrcp_factor(qcopies[1 + i], nb=32, handle=h)
        torch.cuda.synchronize()
        tq1 = time.perf_counter()
        lib.rq_profile_stop(h.ptr)
        h.sync()
        qms = (tq1 - tq0) * 1e3 / qsteps
        qprof = profile_table(h)
        plain = {"ms_per_step": round(qms, 3), "value": round(flops / (qms * 1e-3) / 1e12, 4),
                 "unit": "TFLOP/s", "nb": 32, "steps": qsteps,
                 "rqrcp_speedup": round(qms / ms, 3),
                 "kernels_ms_per_step": {k: round(v["ms"] / qsteps, 3) for k, v in qprof.items()}}
        log(f"plain QRCP {qms:.2f} ms/step -> RQRCP speedup {qms / ms:.2f}x")
        del qcopies

    roof = roofline(prof, args.steps)
    roof["share_of_step"] = round(prof[roof["kernel"]]["ms"] / args.steps / ms, 4)
    res = {
        "metric": "RQRCP FP64 TFLOP/s (nominal 4n^3/3) on one MI355X",
        "value": round(value, 4),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"rqrcp_fp64_{m}x{n}_gauss", "m": m, "n": n, "k": n, "b": b,
                   "p": p},
        "roofline": roof,
        "first_block_pivots_match_oracle": ok,
        "kernels_ms_per_step": {k: round(v["ms"] / args.steps, 3) for k, v in prof.items()},
        "plain_qrcp": plain,
    }
    if not args.no_cpu:
        log("timing the CPU oracle on a bounded sample")
        res["cpu_baseline"] = cpu_baseline(a, om, b, p, args.cpu_k)
        log(f"cpu baseline {res['cpu_baseline']['value']} TFLOP/s "
            f"({res['cpu_baseline']['seconds']} s, {res['cpu_baseline']['cores']} cores)")
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=8000)
    ap.add_argument("--cpu-k", type=int, default=512, help="pivots of the CPU oracle sample")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain-QRCP comparison")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); this build has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)
    res = bench_rqrcp(args)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
