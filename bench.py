#!/usr/bin/env python3
"""Benchmark of the RQRCP hot path on one MI355X.

Default workload: FP64 RQRCP full factorization of an 8000 x 8000 i.i.d. N(0,1)
matrix with b = 64, p = 8 (Omega 72 x 8000).  One step = the whole hot path on
one resident copy of A: sketch, then per block the sample QRCP, permutation,
panel + T, inner products, trailing update and sample update.  Every step
factors its own pre-staged copy of A, so nothing but the factorization runs in
the timed region.  The throughput counts the nominal 4n^3/3 flops of a full
Householder QR (the same count used for plain QRCP and unpivoted QR).

Before the timed steps, one step runs with every kernel bracketed by HIP events:
its per-kernel times are the reported breakdown (`kernels_ms_per_step`, with the
wall time of that step as `profiled_ms_per_step`) and its longest kernel class
is the one the roofline covers.  The timed steps bracket only that class with
events (two per launch), since events around every launch add device time of
their own; the plain QRCP comparator and the repeated-sampling RQRCP
(Section 3.4: a fresh sketch of each trailing matrix instead of the sample
update) are timed with no events at all.

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

PEAK = {"fp64_tflops": 78.6, "bf16_tflops": 2500.0, "hbm_gbs": 8000.0}
MFMA_CLASSES = {"sketch", "inner_products", "trailing_update", "sample_update", "qp3_gemv",
                "sketch_bf16", "inner_products_bf16"}


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


ALL_CLASSES = 0xFFFFFFFF


def class_mask(h, names):
    """Bit mask of the library's kernel classes with the given names."""
    from paper_2008_04447_amd import _lib
    import ctypes
    lib = _lib.load()
    mask = 0
    for i in range(lib.rq_profile_count(h.ptr)):
        name = ctypes.c_char_p()
        launches = ctypes.c_int64()
        ms, fl, by = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        lib.rq_profile_get(h.ptr, i, ctypes.byref(name), ctypes.byref(launches), ctypes.byref(ms),
                           ctypes.byref(fl), ctypes.byref(by))
        if name.value.decode() in names:
            mask |= 1 << i
    return mask


def profiled_step(fn, h):
    """One call of fn with every kernel bracketed by HIP events: the per-kernel
    breakdown and the call's wall time in ms (the events add device time of
    their own, so this time is not the throughput measurement)."""
    import torch
    from paper_2008_04447_amd import _lib
    lib = _lib.load()
    lib.rq_profile_classes(h.ptr, ALL_CLASSES)
    lib.rq_profile_start(h.ptr)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = fn()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lib.rq_profile_stop(h.ptr)
    h.sync()
    return (t1 - t0) * 1e3, profile_table(h), out


def dominant(breakdown):
    return max(breakdown.items(), key=lambda kv: kv[1]["ms"])[0] if breakdown else None


PROFILE = os.path.join(ROOT, "profiles", "rqrcp_fp64_8000_kernels.txt")
KERNEL_SOURCES = {"sample_qrcp": ["sample_qrcp.hip"], "panel": ["panel.hip"],
                  "inner_products": ["blas.hip"], "trailing_update": ["blas.hip"]}


def source_hash(cls):
    """Hash of the sources a kernel class is built from (as recorded in the profile)."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_2008_04447_amd", "csrc")
    h = hashlib.sha256()
    for fn in KERNEL_SOURCES[cls] + ["device_common.hpp", "kernels.hpp"]:
        with open(os.path.join(csrc, fn), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, cls):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated) from the committed
    rocprofv3 summary, or None when absent or measured on other kernel sources."""
    if cls not in KERNEL_SOURCES or not os.path.exists(PROFILE):
        return None
    with open(PROFILE) as f:
        for line in f:
            if not line.startswith("TRAFFIC "):
                continue
            kv = dict(item.split("=", 1) for item in line.split()[1:])
            if kv.get("workload") == workload and kv.get("class") == cls:
                if kv.get("source") != source_hash(cls):
                    return None
                return float(kv["fetch_bytes"]) + float(kv["write_bytes"])
    return None


def roofline(prof, steps, workload=None):
    """Roofline entry of the kernel class with the largest total time.  A
    contraction class is MFMA-bound when its algorithmic flops per byte reach
    the ridge of its dtype (peak flops / HBM bandwidth), else HBM-bound."""
    name, rec = max(prof.items(), key=lambda kv: kv[1]["ms"])
    sec = rec["ms"] * 1e-3
    fpeak = PEAK["bf16_tflops" if name.endswith("_bf16") else "fp64_tflops"]
    mfma = name in MFMA_CLASSES and (rec["bytes"] <= 0 or
                                     rec["flops"] / rec["bytes"] * PEAK["hbm_gbs"] * 1e-3 >= fpeak)
    if mfma:
        achieved = rec["flops"] / sec / 1e12
        peak = fpeak
        bound, unit = "mfma", "TFLOP/s"
    else:
        achieved = rec["bytes"] / sec / 1e9
        peak = PEAK["hbm_gbs"]
        bound, unit = "hbm", "GB/s"
    return {"kernel": name, "bound": bound, "achieved": round(achieved, 4), "peak": peak,
            "unit": unit, "frac": round(achieved / peak, 5),
            "traffic": measured_traffic(workload, name) if workload else None,
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
    copies = [A0.clone(memory_format=torch.preserve_format)
              for _ in range(args.warmup + 1 + args.steps)]
    for c in copies:
        assert c.stride(0) == 1
    h = api.default_handle(0)
    torch.cuda.synchronize()
    log(f"warmup {args.warmup} step(s)")
    for i in range(args.warmup):
        api.rqrcp_factor(copies[i], Om, b, p, handle=h)
        h.sync()
    lib = _lib.load()
    # one step with every kernel timed: the per-kernel breakdown and the dominant kernel
    pms, breakdown, _ = profiled_step(lambda: api.rqrcp_factor(copies[args.warmup], Om, b, p,
                                                               handle=h), h)
    dom = dominant(breakdown)
    log(f"profiled step {pms:.2f} ms (every kernel bracketed by events); dominant kernel {dom}")
    # the timed steps: events only around the dominant kernel (its launch durations
    # give the roofline), none around the others
    lib.rq_profile_classes(h.ptr, class_mask(h, [dom]))
    lib.rq_profile_start(h.ptr)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outs = []
    for i in range(args.steps):
        outs.append(api.rqrcp_factor(copies[args.warmup + 1 + i], Om, b, p, handle=h))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lib.rq_profile_stop(h.ptr)
    lib.rq_profile_classes(h.ptr, ALL_CLASSES)
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
        qcopies = [A0.clone(memory_format=torch.preserve_format) for _ in range(qsteps + 2)]
        log(f"plain QRCP: 1 warmup + 1 profiled + {qsteps} timed step(s)")
        api.qrcp_factor(qcopies[0], nb=32, handle=h)
        h.sync()
        qpms, qprof, _ = profiled_step(lambda: api.qrcp_factor(qcopies[1], nb=32, handle=h), h)
        lib.rq_profile_classes(h.ptr, 0)
        torch.cuda.synchronize()
        tq0 = time.perf_counter()
        for i in range(qsteps):
            qj, _ = api.qrcp_factor(qcopies[2 + i], nb=32, handle=h)
        torch.cuda.synchronize()
        tq1 = time.perf_counter()
        lib.rq_profile_classes(h.ptr, ALL_CLASSES)
        h.sync()
        qms = (tq1 - tq0) * 1e3 / qsteps
        plain = {"ms_per_step": round(qms, 3), "value": round(flops / (qms * 1e-3) / 1e12, 4),
                 "unit": "TFLOP/s", "nb": 32, "steps": qsteps,
                 "rqrcp_speedup": round(qms / ms, 3),
                 "profiled_ms_per_step": round(qpms, 3),
                 "kernels_ms_per_step": {k: round(v["ms"], 3) for k, v in qprof.items()}}
        log(f"plain QRCP {qms:.2f} ms/step -> RQRCP speedup {qms / ms:.2f}x")
        del qcopies

    resampled = None
    if not args.no_resample:
        # RQRCP with repeated sampling (Section 3.4) on the same matrix: each block
        # sketches its updated trailing matrix with a fresh Omega instead of the
        # sample update (slice 0 is the Omega above, so block 0 is the same)
        nblk = (n + b - 1) // b
        oms = torch.empty((nblk, m, ell), dtype=torch.float64, device=dev)
        oms[0] = torch.from_numpy(np.ascontiguousarray(om.T)).to(dev)
        for j in range(1, nblk):
            oms[j] = torch.from_numpy(np.ascontiguousarray(
                synth.omega(ell, m, synth.seed_for(1, "Omega") + 100 + j).T)).to(dev)
        rsteps = max(1, min(args.steps, 2))
        rcopies = [A0.clone(memory_format=torch.preserve_format) for _ in range(rsteps + 2)]
        log(f"repeated sampling: 1 warmup + 1 profiled + {rsteps} timed step(s)")
        api.rsrqrcp_factor(rcopies[0], oms, b, p, handle=h)
        h.sync()
        rpms, rprof, _ = profiled_step(lambda: api.rsrqrcp_factor(rcopies[1], oms, b, p, handle=h), h)
        lib.rq_profile_classes(h.ptr, 0)
        torch.cuda.synchronize()
        tr0 = time.perf_counter()
        for i in range(rsteps):
            api.rsrqrcp_factor(rcopies[2 + i], oms, b, p, handle=h)
        torch.cuda.synchronize()
        tr1 = time.perf_counter()
        lib.rq_profile_classes(h.ptr, ALL_CLASSES)
        h.sync()
        rms = (tr1 - tr0) * 1e3 / rsteps
        resampled = {"ms_per_step": round(rms, 3), "value": round(flops / (rms * 1e-3) / 1e12, 4),
                     "unit": "TFLOP/s", "steps": rsteps,
                     "sample_update_saving": round(1.0 - ms / rms, 4),
                     "profiled_ms_per_step": round(rpms, 3),
                     "kernels_ms_per_step": {k: round(v["ms"], 3) for k, v in rprof.items()}}
        log(f"repeated sampling {rms:.2f} ms/step: the sample update saves {1.0 - ms / rms:.1%}")
        del rcopies, oms

    roof = roofline(prof, args.steps, f"rqrcp_fp64_{m}x{n}_gauss")
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
        "profiled_ms_per_step": round(pms, 3),
        "kernels_ms_per_step": {k: round(v["ms"], 3) for k, v in breakdown.items()},
        "plain_qrcp": plain,
        "repeated_sampling": resampled,
    }
    if not args.no_cpu:
        log("timing the CPU oracle on a bounded sample")
        res["cpu_baseline"] = cpu_baseline(a, om, b, p, args.cpu_k)
        log(f"cpu baseline {res['cpu_baseline']['value']} TFLOP/s "
            f"({res['cpu_baseline']['seconds']} s, {res['cpu_baseline']['cores']} cores)")
    return res


def trqrcp_flops(m, n, k, b, p):
    """Algorithmic flops of TRQRCP: sketch, per block Y2^T A, R rows, selected
    columns, panel, small products, sample update."""
    ell = b + p
    f = 2.0 * ell * m * n
    c0 = 0
    while c0 < k:
        bj = min(b, k - c0)
        M, N = m - c0, n - c0
        Nt = N - bj
        f += 2.0 * bj * M * Nt + 2.0 * bj * (c0 + bj) * Nt + 2.0 * M * bj * c0 + 2.0 * M * bj * bj
        f += 2.0 * bj * M * c0 + 2.0 * bj * c0 * Nt + 2.0 * bj * bj * Nt
        c0 += bj
    return f


def _gpu_mem_clear():
    import gc
    import torch
    gc.collect()
    torch.cuda.empty_cache()


def _timed(fn, steps, warmup, h):
    """Warm-up calls, one profiled call (per-kernel breakdown), then `steps`
    timed calls with events only around the dominant kernel.  Returns ms per
    timed call, the last output, the dominant kernel's timings and the
    breakdown."""
    import torch
    from paper_2008_04447_amd import _lib
    lib = _lib.load()
    for _ in range(warmup):
        fn()
        h.sync()
    _, breakdown, _ = profiled_step(fn, h)
    lib.rq_profile_classes(h.ptr, class_mask(h, [dominant(breakdown)]))
    lib.rq_profile_start(h.ptr)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = None
    for _ in range(steps):
        out = fn()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lib.rq_profile_stop(h.ptr)
    lib.rq_profile_classes(h.ptr, ALL_CLASSES)
    h.sync()
    return (t1 - t0) * 1e3 / steps, out, profile_table(h), breakdown


def bench_trqrcp_c3(args):
    """Mixed-precision TRQRCP, rank 512, on a 20000 x 20000 FP32 matrix with
    sigma_i = exp(-i/200) (only sigma_i > 1e-9, i < 4145, is drawn: the rest is
    below FP32 resolution).  Error vs the library's own FP64 TRQRCP on the same
    matrix (which the parity tests pin to the FP64 oracle)."""
    import numpy as np
    import torch
    import synth
    from paper_2008_04447_amd import api
    m = n = 20000
    k, b, p = 512, 64, 8
    dev = torch.device("cuda", 0)
    sig = synth.spectrum("exp", 4145, scale=200.0)
    log("C3: drawing A 20000x20000 (exp(-i/200)) on the GPU")
    A64 = synth.low_rank_device(m, n, sig, synth.seed_for(2, "U"), dev)
    A32 = torch.empty((n, m), dtype=torch.float32, device=dev).t()
    A32.copy_(A64)
    A64.copy_(A32)                              # the FP64 run sees the same FP32 values
    om = api.colmajor(synth.omega(b + p, m, synth.seed_for(2, "Omega")), device=dev)
    h = api.default_handle(0)
    ms, out, prof, brk = _timed(lambda: api.trqrcp_truncate(A32, om, b, p, k, handle=h),
                                args.c3_steps, 1, h)
    ms64, out64, _, _ = _timed(lambda: api.trqrcp_truncate(A64, om, b, p, k, handle=h), 1, 1, h)

    def err(o):
        jp, Y, T, R = o
        ap = A64[:, jp]
        qk = -(Y @ (T @ Y[:k, :].T))            # Q[:, :k] = I[:, :k] - Y T Y_1^T
        qk[:k, :] += torch.eye(k, dtype=torch.float64, device=dev)
        return float(torch.linalg.norm(ap - qk @ R) / torch.linalg.norm(A64))
    e32, e64 = err(out), err(out64)
    opt = float(np.sqrt(np.sum(sig[k:] ** 2) / np.sum(sig ** 2)))
    fl = trqrcp_flops(m, n, k, b, p)
    roof = roofline(prof, args.c3_steps)
    res = {"ms_per_step": round(ms, 3), "value": round(fl / (ms * 1e-3) / 1e12, 4), "unit": "TFLOP/s",
           "dtype": "bf16-mfma/fp32-acc, fp64 panel", "fp64_ms_per_step": round(ms64, 3),
           "trunc_error": e32, "trunc_error_fp64": e64, "error_ratio": round(e32 / e64, 5),
           "optimal_svd_error": opt, "flops_per_step": fl, "roofline": roof,
           "kernels_ms_per_step": {kk: round(v["ms"], 3) for kk, v in brk.items()},
           "config": {"workload": "trqrcp_mixed_20000x20000_exp200", "m": m, "n": n, "k": k, "b": b,
                      "p": p}}
    log(f"C3: {ms:.2f} ms/step ({res['value']} TFLOP/s), error {e32:.5e} vs fp64 {e64:.5e} "
        f"ratio {e32 / e64:.4f}")
    del A64, A32, out, out64
    _gpu_mem_clear()
    return res


def bench_tuxv_c4(args):
    """Mixed-precision TUXV, rank 256, on 50000 x 8000 FP32:
    U diag((i+1)^-1.5) V^T + N(0, 1e-12) noise (std 1e-6)."""
    import numpy as np
    import torch
    import synth
    from paper_2008_04447_amd import api
    m, n, k, b, p = 50000, 8000, 256, 64, 8
    dev = torch.device("cuda", 0)
    sig = synth.spectrum("poly", n, power=1.5)
    log("C4: drawing A 50000x8000 ((i+1)^-1.5 + noise) on the GPU")
    A64 = synth.low_rank_device(m, n, sig, synth.seed_for(3, "U"), dev)
    A64 += synth.gaussian_device(m, n, synth.seed_for(3, "noise"), dev, std=1e-6)
    A32 = torch.empty((n, m), dtype=torch.float32, device=dev).t()
    A32.copy_(A64)
    A64.copy_(A32)
    om = api.colmajor(synth.omega(b + p, m, synth.seed_for(3, "Omega")), device=dev)
    h = api.default_handle(0)
    ms, out, prof, brk = _timed(lambda: api.tuxv_svd(A32, om, b, p, k, handle=h), args.c4_steps,
                                1, h)
    ms64, out64, _, _ = _timed(lambda: api.tuxv_svd(A64, om, b, p, k, handle=h), 1, 1, h)

    def err(o):
        U, X, V, _ = o
        return float(torch.linalg.norm(A64 - U @ (X @ V.T)) / torch.linalg.norm(A64))
    e32, e64 = err(out), err(out64)
    # a second alternation (jmax = 2: the LQ of U^T A after the QR of A V)
    ms2, out2, _, _ = _timed(lambda: api.tuxv_svd(A32, om, b, p, k, handle=h, jmax=2), 1, 1, h)
    e2 = err(out2)
    del out2
    s32 = torch.linalg.svdvals(out[1]).cpu().numpy()
    s64 = torch.linalg.svdvals(out64[1]).cpu().numpy()
    rel = np.abs(s32 - s64) / s64
    fl = trqrcp_flops(m, n, k, b, p) + 2.0 * m * n * k + 8.0 * (m + n) * k * k
    roof = roofline(prof, args.c4_steps)
    res = {"ms_per_step": round(ms, 3), "value": round(fl / (ms * 1e-3) / 1e12, 4), "unit": "TFLOP/s",
           "dtype": "bf16-mfma/fp32-acc, fp64 panel", "fp64_ms_per_step": round(ms64, 3),
           "approx_error": e32, "approx_error_fp64": e64, "error_ratio": round(e32 / e64, 5),
           "sigma_rel_err_median": float(np.median(rel)), "sigma_rel_err_max": float(rel.max()),
           "sigma_rel_err_median_top64": float(np.median(rel[:64])),
           "jmax2": {"ms_per_step": round(ms2, 3), "approx_error": e2},
           "flops_per_step": fl, "roofline": roof,
           "kernels_ms_per_step": {kk: round(v["ms"], 3) for kk, v in brk.items()},
           "config": {"workload": "tuxv_mixed_50000x8000_poly1.5_noise1e-6", "m": m, "n": n, "k": k,
                      "b": b, "p": p}}
    log(f"C4: {ms:.2f} ms/step ({res['value']} TFLOP/s), error ratio {e32 / e64:.4f}, "
        f"sigma rel err median {np.median(rel):.2e}")
    del A64, A32, out, out64
    _gpu_mem_clear()
    return res


def bench_serve_c5(args):
    """Serving: Poisson arrivals (mean 200/s) of TRQRCP / TUXV requests (50/50),
    m, n ~ U[256, 4096], k ~ U{16,32,64,128,256}, b = min(64, k), p = 8, FP32
    A = U diag(10^(-i/50)) V^T (only sigma_i >= 1e-9, i < 450, is drawn), Omega
    seeded per request.  A pool of distinct matrices is drawn up front into
    page-locked host memory and requests cycle through it."""
    import numpy as np
    import torch
    import synth
    from paper_2008_04447_amd import api
    rng = synth.rng(synth.seed_for(4, "perm"))
    dev = torch.device("cuda", 0)
    n_warm, n_req, rate = args.serve_warmup, args.serve_requests, args.serve_rate
    pool = []
    log(f"C5: drawing {args.serve_pool} request matrices")
    for i in range(args.serve_pool):
        m = int(rng.integers(256, 4097))
        n = int(rng.integers(256, 4097))
        r = min(m, n, 450)
        sig = synth.spectrum("pow10", r, scale=50.0)
        a = synth.low_rank_device(m, n, sig, synth.seed_for(4, "U") + 17 * i, dev, torch.float32)
        host = api.pinned_empty((m, n), np.float32)
        host[:] = a.cpu().numpy()
        pool.append(host)
        del a
    _gpu_mem_clear()
    total = n_warm + n_req
    ks = rng.choice([16, 32, 64, 128, 256], size=total)
    ops = rng.integers(0, 2, size=total)
    gaps = rng.exponential(1.0 / rate, size=total)
    log(f"C5: drawing {total} per-request Omega into page-locked memory")
    oms = []
    for i in range(total):
        m = pool[i % len(pool)].shape[0]
        b = min(64, int(min(ks[i], m, pool[i % len(pool)].shape[1])))
        om = api.pinned_empty((b + 8, m), np.float64)
        om[:] = synth.omega(b + 8, m, synth.seed_for(4, "Omega") + i)
        oms.append(om)
    srv = api.Server(args.serve_budget_gb * (1 << 30), slots=args.serve_slots, max_m=4096, max_n=4096,
                     max_k=256, max_ell=72)
    flops = 0.0
    lat, ids = [], []
    try:
        t_next = time.perf_counter()
        t_first = None
        for i in range(total):
            a = pool[i % len(pool)]
            m, n = a.shape
            k = int(min(ks[i], m, n))
            b = min(64, k)
            om = oms[i]
            t_next += gaps[i]
            while time.perf_counter() < t_next:
                time.sleep(min(5e-4, max(0.0, t_next - time.perf_counter())))
            if i == n_warm:
                t_first = time.perf_counter()
            ids.append(srv.submit(int(ops[i]), a, om, b, 8, k, outputs=False))
            if i % 500 == 0:
                log(f"C5: submitted {i}/{total}")
        res_all = [srv.wait(x) for x in ids]
        t_last = time.perf_counter()
        st = srv.stats()
    finally:
        srv.stop()
    timed = res_all[n_warm:]
    bad = [r for r in timed if r["state"] != 2 or r["status"] != 0]
    lat = np.array([r["latency_ms"] for r in timed])
    q = np.array([r["queue_ms"] for r in timed])
    flops = float(sum(r["flops"] for r in timed))
    span = t_last - t_first
    res = {"p50_ms": round(float(np.percentile(lat, 50)), 3),
           "p99_ms": round(float(np.percentile(lat, 99)), 3),
           "mean_ms": round(float(lat.mean()), 3), "queue_p99_ms": round(float(np.percentile(q, 99)), 3),
           "requests": n_req, "warmup_requests": n_warm, "rate_per_s": rate,
           "achieved_rate_per_s": round(n_req / span, 2), "aggregate_tflops": round(flops / span / 1e12, 5),
           "failed": len(bad), "slots": args.serve_slots, "budget_gb": args.serve_budget_gb,
           "peak_running": st["peak_running"], "peak_bytes": st["peak_bytes"],
           "config": {"workload": "serve_trqrcp_tuxv_poisson200_m256-4096_fp32",
                      "pool_matrices": len(pool)}}
    log(f"C5: p50 {res['p50_ms']} ms, p99 {res['p99_ms']} ms, {res['aggregate_tflops']} TFLOP/s, "
        f"peak running {st['peak_running']}")
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
    ap.add_argument("--no-resample", action="store_true",
                    help="skip the repeated-sampling RQRCP comparison")
    ap.add_argument("--skip", default="", help="comma list of secondary workloads to skip: "
                    "trqrcp,tuxv,serving")
    ap.add_argument("--c3-steps", type=int, default=3)
    ap.add_argument("--c4-steps", type=int, default=3)
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-warmup", type=int, default=200)
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-pool", type=int, default=48)
    ap.add_argument("--serve-slots", type=int, default=8)
    ap.add_argument("--serve-budget-gb", type=int, default=8)
    ap.add_argument("--only", default="", choices=["", "trqrcp", "tuxv", "serving"],
                    help="run only this secondary workload and print its result (for profiling)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device-to-device copy 3 times (HBM counter calibration)")
    args = ap.parse_args()
    args.skip = [x for x in args.skip.split(",") if x]
    if args.copy_calibration:
        import torch
        x = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
        y = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        for _ in range(3):
            x.copy_(y)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_call": 8 << 27, "calls": 3}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the library has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)
    workloads = (("trqrcp_mixed_20000", bench_trqrcp_c3), ("tuxv_mixed_50000x8000", bench_tuxv_c4),
                 ("serving", bench_serve_c5))
    if args.only:
        name, fn = next(w for w in workloads if w[0].split("_")[0] == args.only)
        print(json.dumps({name: fn(args)}), flush=True)
        return
    res = bench_rqrcp(args)
    secondary = {}
    for name, fn in workloads:
        if name.split("_")[0] in args.skip:
            continue
        try:
            secondary[name] = fn(args)
        except Exception as e:          # report, keep the headline line intact
            log(f"{name} failed: {type(e).__name__}: {e}")
            secondary[name] = {"error": f"{type(e).__name__}: {e}"}
    res["secondary"] = secondary
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
