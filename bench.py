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


def cpu_info():
    """Host cores this process may use and the CPU model (lscpu, else /proc/cpuinfo)."""
    import subprocess
    cores = len(os.sched_getaffinity(0))
    model = None
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
                break
    except Exception:
        pass
    if model is None:
        try:
            with open("/proc/cpuinfo") as f:
                for line in f:
                    if line.startswith("model name"):
                        model = line.split(":", 1)[1].strip()
                        break
        except OSError:
            pass
    return cores, model


def cpu_baseline(a, om, b, p, kc):
    """The FP64 oracle on a bounded sample: the first kc pivots of the same matrix.
    Returns the baseline entry and the oracle's result (for the pivot/R check)."""
    import oracle
    cores, model = cpu_info()
    t = time.perf_counter()
    ref = oracle.rqrcp(a, om, b, p, k=kc)
    dt = time.perf_counter() - t
    m, n = a.shape
    fl = nominal_qr_flops(m, n, kc)
    entry = {"value": round(fl / dt / 1e12, 6), "unit": "TFLOP/s", "cores": cores, "kind": "oracle",
             "cpu_model": model, "seconds": round(dt, 3),
             "sample": f"oracle RQRCP (numpy FP64) of the first {kc} pivots ({kc // b} blocks) of "
                       f"the same {m}x{n} matrix; flops = sum_j<{kc} 4(m-j)(n-j)"}
    return entry, ref


def oracle_block_check(a, jp, r_top, tau, ref, b):
    """GPU pivots and R rows against the oracle's first kc pivots (Algorithm 4 with
    eq. update1 on the same Omega): pivots on the certified prefix, R rows compared
    column by column through both permutations."""
    import numpy as np
    n = a.shape[1]
    pre = ref.trace.prefix(ref.sample_scale, 1e-10, 1e-13)
    kc = ref.tau.size
    pre = min(pre, kc)
    equal = bool(np.array_equal(jp[:pre], ref.jpvt[:pre]))
    where = np.empty(n, dtype=np.int64)
    where[ref.jpvt] = np.arange(n)
    r_ref = np.triu(ref.qr[:pre])[:, where[jp]]
    d = np.linalg.norm(np.triu(r_top[:pre]) - r_ref, axis=1)
    nrm = np.linalg.norm(r_ref, axis=1)
    floor = 1e-12 * np.linalg.norm(a)
    ok_rows = bool(np.all(d <= 1e-10 * nrm + floor))
    return {"pivots_compared": int(pre), "of": int(kc), "pivots_equal": equal,
            "r_rows_within_tol": ok_rows,
            "r_rows_max_rel_diff": float(np.max(d / np.maximum(nrm, 1e-300))) if pre else None,
            "tau_max_rel_diff": float(np.max(np.abs(tau[:pre] - ref.tau[:pre]) /
                                             np.maximum(np.abs(ref.tau[:pre]), 1e-300))) if pre else None}


def _block_t(y, tau):
    """T of a block of reflectors by the forward recurrence (Q_J = I - Y T Y^T)."""
    import torch
    bj = y.shape[1]
    t = torch.zeros((bj, bj), dtype=torch.float64, device=y.device)
    g = y.t().contiguous() @ y
    for j in range(bj):
        t[j, j] = tau[j]
        if j:
            t[:j, j] = -tau[j] * (t[:j, :j] @ g[:j, j])
    return t


def apply_q(qr, tau, T, b, x, transpose=False):
    """x <- Q x (or Q^T x) for Q = H_0 ... H_{k-1} held in the in-place array qr
    (reflector tails below the diagonal) with block T (b x k, or None: formed by
    the forward recurrence), in FP64 on the device."""
    import torch
    k = tau.numel()
    blocks = list(range(0, k, b))
    for c0 in (blocks if transpose else reversed(blocks)):
        bj = min(b, k - c0)
        y = torch.tril(qr[c0:, c0:c0 + bj], -1)
        y.diagonal().fill_(1.0)
        t = T[:bj, c0:c0 + bj] if T is not None else _block_t(y, tau[c0:c0 + bj])
        if transpose:
            t = t.t()
        x[c0:] -= y @ (t.contiguous() @ (y.t().contiguous() @ x[c0:]))
    return x


def qr_residual(A0, qr, tau, jpvt, T, b):
    """||A P - Q R||_F / ||A||_F and ||Q^T Q g - g|| / ||g|| on 16 Gaussian vectors,
    computed on the device in FP64 from a factorization's outputs."""
    import torch
    import synth
    m, n = qr.shape
    x = apply_q(qr, tau, T, b, torch.triu(qr).clone())
    rel = float(torch.linalg.norm(A0[:, jpvt] - x) / torch.linalg.norm(A0))
    del x
    g = torch.from_numpy(synth.gaussian((m, 16), 4400)).to(qr.device)
    back = apply_q(qr, tau, T, b, apply_q(qr, tau, T, b, g.clone(), transpose=True))
    orth = float(torch.linalg.norm(back - g) / torch.linalg.norm(g))
    return rel, orth


def headline_matrix(variant, m, n, dev):
    """The two 8000 x 8000 inputs of the FP64 RQRCP-vs-QRCP workload: i.i.d. N(0,1),
    and Haar U, V with sigma_i = 10^(-6 i / n) (drawn on the device)."""
    import numpy as np
    import synth
    if variant == "gauss":
        return synth.gaussian((m, n), synth.seed_for(1, "U"))
    sig = synth.spectrum("pow10x", n, decades=6.0, span=float(n))
    return np.asfortranarray(synth.low_rank_device(m, n, sig, synth.seed_for(1, "V"), dev).cpu().numpy())


def run_plain_qrcp(A0, steps, h, flops, rq_ms=None):
    """Plain QRCP (Algorithm 2) on the same matrix: 1 warm-up, 1 profiled and
    `steps` timed calls (no events), plus the residual of the last one."""
    import torch
    from paper_2008_04447_amd import _lib, api
    lib = _lib.load()
    m, n = A0.shape
    qcopies = [A0.clone(memory_format=torch.preserve_format) for _ in range(steps + 2)]
    log(f"plain QRCP: 1 warmup + 1 profiled + {steps} timed step(s)")
    api.qrcp_factor(qcopies[0], nb=32, handle=h)
    h.sync()
    qpms, qprof, _ = profiled_step(lambda: api.qrcp_factor(qcopies[1], nb=32, handle=h), h)
    lib.rq_profile_classes(h.ptr, 0)
    torch.cuda.synchronize()
    tq0 = time.perf_counter()
    for i in range(steps):
        qj, qt = api.qrcp_factor(qcopies[2 + i], nb=32, handle=h)
    torch.cuda.synchronize()
    tq1 = time.perf_counter()
    lib.rq_profile_classes(h.ptr, ALL_CLASSES)
    h.sync()
    qms = (tq1 - tq0) * 1e3 / steps
    rel, orth = qr_residual(A0, qcopies[1 + steps], qt, qj, None, 64)
    # the HBM floor of Algorithm 2: the trailing matrix read once per column
    floor_bytes = float(sum(8.0 * (m - j) * (n - j) for j in range(min(m, n))))
    floor_ms = floor_bytes / (PEAK["hbm_gbs"] * 1e9) * 1e3
    out = {"ms_per_step": round(qms, 3), "value": round(flops / (qms * 1e-3) / 1e12, 4),
           "unit": "TFLOP/s", "nb": 32, "steps": steps,
           "residual": rel, "orthogonality": orth,
           "hbm_floor_ms": round(floor_ms, 3), "frac_of_hbm_floor": round(floor_ms / qms, 4),
           "profiled_ms_per_step": round(qpms, 3),
           "kernels_ms_per_step": {k: round(v["ms"], 3) for k, v in qprof.items()}}
    if rq_ms:
        out["rqrcp_speedup"] = round(qms / rq_ms, 3)
    log(f"plain QRCP {qms:.2f} ms/step ({floor_ms / qms:.1%} of its HBM floor), residual {rel:.2e}")
    del qcopies
    return out


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
    a = headline_matrix("gauss", m, n, dev)
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
    # the error at which the throughput is quoted: the last timed factorization
    last = copies[args.warmup + args.steps]
    jpvt_t, tau_t, T_t, info_t = outs[-1]
    resid, orth = qr_residual(A0, last, tau_t, jpvt_t, T_t, b)
    log(f"residual ||AP - QR||/||A|| = {resid:.2e}, orthogonality {orth:.2e}, "
        f"info {int(info_t.item())}")
    jp = jpvt_t.cpu().numpy()
    r_top = last[:args.cpu_k].cpu().numpy()
    tau_h = tau_t.cpu().numpy()
    del copies[:-1]

    plain = None
    if not args.no_plain:
        plain = run_plain_qrcp(A0, max(1, min(args.steps, 2)), h, flops, ms)

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
    sq_ms = breakdown.get("sample_qrcp", {}).get("ms", 0.0)
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
        "fp64_frac_whole_step": round(value / PEAK["fp64_tflops"], 4),
        "residual": resid,
        "orthogonality": orth,
        "info": int(info_t.item()),
        "sample_qrcp_us_per_pivot": round(sq_ms * 1e3 / n, 3),
        "profiled_ms_per_step": round(pms, 3),
        "kernels_ms_per_step": {k: round(v["ms"], 3) for k, v in breakdown.items()},
        "plain_qrcp": plain,
        "repeated_sampling": resampled,
    }
    if not args.no_cpu:
        log("timing the CPU oracle on a bounded sample")
        res["cpu_baseline"], ref = cpu_baseline(a, om, b, p, args.cpu_k)
        res["oracle_check"] = oracle_block_check(a, jp, r_top, tau_h, ref, b)
        log(f"cpu baseline {res['cpu_baseline']['value']} TFLOP/s "
            f"({res['cpu_baseline']['seconds']} s, {res['cpu_baseline']['cores']} cores); "
            f"oracle check {res['oracle_check']}")
        del ref
    del copies, A0
    _gpu_mem_clear()
    if "c2graded" not in args.skip:
        res["c2_graded"] = bench_c2_graded(args, om, Om, h)
    return res


def bench_c2_graded(args, om, Om, h):
    """The second matrix of the FP64 RQRCP-vs-QRCP workload: Haar U, V with
    sigma_i = 10^(-6 i / n), b = 64, p = 8, the same Omega: RQRCP timed with no
    events, its residual and the oracle check of its first blocks, and plain QRCP
    on the same matrix."""
    import torch
    from paper_2008_04447_amd import _lib, api
    m = n = args.n
    b, p = 64, 8
    dev = torch.device("cuda", 0)
    log("C2 graded: drawing Haar U, V with sigma_i = 10^(-6 i / n)")
    a = headline_matrix("graded", m, n, dev)
    A0 = api.colmajor(a, device=dev)
    steps = max(1, min(args.steps, 3))
    copies = [A0.clone(memory_format=torch.preserve_format) for _ in range(steps + 1)]
    lib = _lib.load()
    api.rqrcp_factor(copies[0], Om, b, p, handle=h)
    h.sync()
    lib.rq_profile_classes(h.ptr, 0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        out = api.rqrcp_factor(copies[1 + i], Om, b, p, handle=h)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lib.rq_profile_classes(h.ptr, ALL_CLASSES)
    h.sync()
    ms = (t1 - t0) * 1e3 / steps
    flops = nominal_qr_flops(m, n, n)
    jpvt_t, tau_t, T_t, info_t = out
    resid, orth = qr_residual(A0, copies[steps], tau_t, jpvt_t, T_t, b)
    res = {"ms_per_step": round(ms, 3), "value": round(flops / (ms * 1e-3) / 1e12, 4),
           "unit": "TFLOP/s", "steps": steps, "residual": resid, "orthogonality": orth,
           "info": int(info_t.item()),
           "config": {"workload": f"rqrcp_fp64_{m}x{n}_graded_1e-6", "m": m, "n": n, "k": n,
                      "b": b, "p": p}}
    log(f"C2 graded: {ms:.2f} ms/step, residual {resid:.2e}")
    if not args.no_cpu:
        import oracle
        ref = oracle.rqrcp(a, om, b, p, k=args.cpu_k)
        res["oracle_check"] = oracle_block_check(a, jpvt_t.cpu().numpy(),
                                                 copies[steps][:args.cpu_k].cpu().numpy(),
                                                 tau_t.cpu().numpy(), ref, b)
        log(f"C2 graded oracle check {res['oracle_check']}")
        del ref
    del copies
    if not args.no_plain:
        res["plain_qrcp"] = run_plain_qrcp(A0, 1, h, flops, ms)
    del A0
    _gpu_mem_clear()
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
    below FP32 resolution).  Its truncation error is compared with the FP64
    oracle's (Algorithm 5 in numpy on the host, same FP32 values and Omega), and
    with the library's own FP64 path; the oracle's time is the CPU timing of the
    truncated routine at this size."""
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
    om_h = synth.omega(b + p, m, synth.seed_for(2, "Omega"))
    om = api.colmajor(om_h, device=dev)
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
           "trunc_error": e32, "trunc_error_fp64_gpu": e64, "error_ratio_vs_fp64_gpu": round(e32 / e64, 5),
           "optimal_svd_error": opt, "flops_per_step": fl, "roofline": roof,
           # FP32 A read by the sketch and by the Y2^T A pass of every block
           "hbm_frac_whole_step": round(4.0 * m * n * (1 + (k + b - 1) // b) / (ms * 1e-3)
                                        / (PEAK["hbm_gbs"] * 1e9), 4),
           "kernels_ms_per_step": {kk: round(v["ms"], 3) for kk, v in brk.items()},
           "config": {"workload": "trqrcp_mixed_20000x20000_exp200", "m": m, "n": n, "k": k, "b": b,
                      "p": p}}
    log(f"C3: {ms:.2f} ms/step ({res['value']} TFLOP/s), error {e32:.5e} vs fp64 gpu {e64:.5e}")
    del out, out64
    if not args.no_oracle_ref:
        import oracle
        log("C3: FP64 oracle (Algorithm 5, numpy) on the host, full size")
        a_h = A64.cpu().numpy()
        cores, model = cpu_info()
        t = time.perf_counter()
        ref = oracle.trqrcp(a_h, om_h, b, p, k)
        dt = time.perf_counter() - t
        del a_h
        e_or = err((torch.from_numpy(ref.jpvt).to(dev), torch.from_numpy(ref.y).to(dev),
                    torch.from_numpy(ref.t).to(dev), torch.from_numpy(ref.r).to(dev)))
        del ref
        res.update({"trunc_error_oracle": e_or, "error_ratio": round(e32 / e_or, 5),
                    "fp64_error_ratio": round(e64 / e_or, 6),
                    "cpu_oracle": {"seconds": round(dt, 2), "value": round(fl / dt / 1e12, 5),
                                   "unit": "TFLOP/s", "cores": cores, "cpu_model": model,
                                   "kind": "oracle", "sample": "the whole workload"}})
        log(f"C3: oracle error {e_or:.5e} ({dt:.1f} s on {cores} cores): mixed ratio "
            f"{e32 / e_or:.4f}, fp64 ratio {e64 / e_or:.6f}")
    del A64, A32
    _gpu_mem_clear()
    return res


def bench_tuxv_c4(args):
    """Mixed-precision TUXV, rank 256, on 50000 x 8000 FP32:
    U diag((i+1)^-1.5) V^T + N(0, 1e-12) noise (std 1e-6).  The error and the
    singular values of X (computed on the device) are compared with the FP64
    oracle's (Algorithm 6 in numpy on the host, same FP32 values and Omega), and
    the oracle's sigma(X) with the spectrum that generated A."""
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
    om_h = synth.omega(b + p, m, synth.seed_for(3, "Omega"))
    om = api.colmajor(om_h, device=dev)
    h = api.default_handle(0)
    ms, out, prof, brk = _timed(lambda: api.tuxv_svd(A32, om, b, p, k, handle=h), args.c4_steps,
                                1, h)
    ms64, out64, _, _ = _timed(lambda: api.tuxv_svd(A64, om, b, p, k, handle=h), 1, 1, h)
    # with the singular values of X on the device
    mss, outs, _, brks = _timed(lambda: api.tuxv_svd(A32, om, b, p, k, handle=h, sigma=True), 2, 1, h)

    def err(U, X, V):
        return float(torch.linalg.norm(A64 - U @ (X @ V.T)) / torch.linalg.norm(A64))
    e32, e64 = err(*out[:3]), err(*out64[:3])
    # a second alternation (jmax = 2: the LQ of U^T A after the QR of A V)
    ms2, out2, _, _ = _timed(lambda: api.tuxv_svd(A32, om, b, p, k, handle=h, jmax=2), 1, 1, h)
    e2 = err(*out2[:3])
    del out2
    s32 = outs[4].cpu().numpy()
    fl = trqrcp_flops(m, n, k, b, p) + 2.0 * m * n * k + 8.0 * (m + n) * k * k
    roof = roofline(prof, args.c4_steps)
    res = {"ms_per_step": round(ms, 3), "value": round(fl / (ms * 1e-3) / 1e12, 4), "unit": "TFLOP/s",
           "dtype": "bf16-mfma/fp32-acc, fp64 panel", "fp64_ms_per_step": round(ms64, 3),
           "approx_error": e32, "approx_error_fp64_gpu": e64,
           "error_ratio_vs_fp64_gpu": round(e32 / e64, 5),
           "with_sigma_ms_per_step": round(mss, 3),
           "svd_of_x_ms": round(brks.get("svd", {}).get("ms", 0.0), 3),
           "jmax2": {"ms_per_step": round(ms2, 3), "approx_error": e2},
           "flops_per_step": fl, "roofline": roof,
           "kernels_ms_per_step": {kk: round(v["ms"], 3) for kk, v in brk.items()},
           "config": {"workload": "tuxv_mixed_50000x8000_poly1.5_noise1e-6", "m": m, "n": n, "k": k,
                      "b": b, "p": p}}
    log(f"C4: {ms:.2f} ms/step ({res['value']} TFLOP/s), with sigma {mss:.2f} ms")
    del out, out64, outs
    if not args.no_oracle_ref:
        import oracle
        log("C4: FP64 oracle (Algorithm 6, numpy) on the host, full size")
        a_h = A64.cpu().numpy()
        cores, model = cpu_info()
        t = time.perf_counter()
        ref = oracle.tuxv(a_h, om_h, b, p, k)
        dt = time.perf_counter() - t
        del a_h
        e_or = err(torch.from_numpy(ref.u).to(dev), torch.from_numpy(ref.x).to(dev),
                   torch.from_numpy(ref.v).to(dev))
        rel = np.abs(s32 - ref.sigma) / ref.sigma
        rel_spec = np.abs(ref.sigma - sig[:k]) / sig[:k]
        res.update({"approx_error_oracle": e_or, "error_ratio": round(e32 / e_or, 5),
                    "fp64_error_ratio": round(e64 / e_or, 6),
                    "sigma_rel_err_vs_oracle_median": float(np.median(rel)),
                    "sigma_rel_err_vs_oracle_max": float(rel.max()),
                    "sigma_rel_err_vs_oracle_median_top64": float(np.median(rel[:64])),
                    "oracle_sigma_rel_err_vs_spectrum_median": float(np.median(rel_spec)),
                    "oracle_sigma_rel_err_vs_spectrum_max": float(rel_spec.max()),
                    "cpu_oracle": {"seconds": round(dt, 2), "value": round(fl / dt / 1e12, 5),
                                   "unit": "TFLOP/s", "cores": cores, "cpu_model": model,
                                   "kind": "oracle", "sample": "the whole workload"}})
        log(f"C4: oracle error {e_or:.5e} ({dt:.1f} s): mixed ratio {e32 / e_or:.4f}; sigma vs "
            f"oracle median {np.median(rel):.2e}, oracle vs spectrum median {np.median(rel_spec):.2e}")
        del ref
    del A64, A32
    _gpu_mem_clear()
    return res


def _serve_once(pool, oms, ks, ops, tols, gaps, n_warm, n_req, budget, slots, sample=()):
    """One serving run: submit warm-up + timed requests at the given arrival gaps,
    wait for all, and return latency statistics (timed requests only) plus the
    results of the sampled requests (whose outputs are copied back)."""
    import numpy as np
    from paper_2008_04447_amd import api
    srv = api.Server(budget, slots=slots, max_m=4096, max_n=4096, max_k=256, max_ell=72)
    total = n_warm + n_req
    ids = []
    try:
        t_next = time.perf_counter()
        t_first = None
        for i in range(total):
            a = pool[i % len(pool)]
            m, n = a.shape
            k = int(min(ks[i], m, n))
            t_next += gaps[i]
            while time.perf_counter() < t_next:
                time.sleep(min(5e-4, max(0.0, t_next - time.perf_counter())))
            if i == n_warm:
                t_first = time.perf_counter()
            ids.append(srv.submit(int(ops[i]), a, oms[i], min(64, k), 8, k, outputs=i in sample,
                                  tol=tols[i], sigma=i in sample))
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
    out = {"p50_ms": round(float(np.percentile(lat, 50)), 3),
           "p99_ms": round(float(np.percentile(lat, 99)), 3),
           "mean_ms": round(float(lat.mean()), 3),
           "queue_p99_ms": round(float(np.percentile(q, 99)), 3),
           "requests": n_req, "warmup_requests": n_warm,
           "achieved_rate_per_s": round(n_req / span, 2),
           "aggregate_tflops": round(flops / span / 1e12, 5), "failed": len(bad),
           "budget_gb": round(budget / (1 << 30), 3), "peak_running": st["peak_running"],
           "peak_bytes": st["peak_bytes"],
           "fp64_routed": int(sum(1 for r in timed if r["prec_used"] == 0)),
           "mixed_routed": int(sum(1 for r in timed if r["prec_used"] == 1))}
    return out, {i: res_all[i] for i in sample}


def bench_serve_c5(args):
    """Serving: Poisson arrivals (mean 200/s) of TRQRCP / TUXV requests (50/50),
    m, n ~ U[256, 4096], k ~ U{16,32,64,128,256}, b = min(64, k), p = 8, FP32
    A = U diag(10^(-i/50)) V^T (only sigma_i >= 1e-9, i < 450, is drawn), Omega
    seeded per request.  A pool of distinct matrices is drawn up front into
    page-locked host memory and requests cycle through it.  Each request asks
    for the accuracy of its rank (the optimal rank-k error of the spectrum) and
    the server picks BF16 or FP64 arithmetic for it (RQ_AUTO).

    Runs: the whole free HBM as the budget at 200/s (the reported latencies),
    then a binding 2 GB budget at 200, 400 and 800 requests/s.  A sample of
    requests (one per operation and rank) returns its outputs, whose errors are
    compared with the FP64 oracle's outside the latency clock."""
    import numpy as np
    import torch
    import oracle
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
    oms, tols = [], []
    for i in range(total):
        m, n = pool[i % len(pool)].shape
        k = int(min(ks[i], m, n))
        b = min(64, k)
        om = api.pinned_empty((b + 8, m), np.float64)
        om[:] = synth.omega(b + 8, m, synth.seed_for(4, "Omega") + i)
        oms.append(om)
        sg = synth.spectrum("pow10", min(m, n, 450), scale=50.0)
        tols.append(float(np.sqrt(np.sum(sg[k:] ** 2) / np.sum(sg ** 2))))
    # one sampled request per (operation, rank) among the timed ones
    sample, seen = [], set()
    for i in range(n_warm, total):
        key = (int(ops[i]), int(ks[i]))
        if key not in seen:
            seen.add(key)
            sample.append(i)
    free, _ = torch.cuda.mem_get_info()
    full = int(min(free - (4 << 30), 64 << 30))
    log(f"C5: {n_req} requests at {rate}/s, budget {full / 2**30:.1f} GB (free HBM)")
    main, outs = _serve_once(pool, oms, ks, ops, tols, gaps, n_warm, n_req, full, args.serve_slots,
                             set(sample))
    log(f"C5: p50 {main['p50_ms']} ms, p99 {main['p99_ms']} ms, {main['aggregate_tflops']} TFLOP/s, "
        f"peak running {main['peak_running']}, fp64/mixed {main['fp64_routed']}/{main['mixed_routed']}")
    # errors of the sampled requests against the FP64 oracle (outside the clock)
    ratios = []
    for i in sample:
        a = pool[i % len(pool)].astype(np.float64)
        m, n = a.shape
        k = int(min(ks[i], m, n))
        b = min(64, k)
        res = outs[i]
        jp, o0, o1, o2 = res["outputs"]
        if ops[i] == 0:
            ref = oracle.trqrcp(a, oms[i], b, 8, k)
            qk = -(o0 @ (o1 @ o0[:k].T))
            qk[:k] += np.eye(k)
            e = np.linalg.norm(a[:, jp] - qk @ o2) / np.linalg.norm(a)
            qr = -(ref.y @ (ref.t @ ref.y[:k].T))
            qr[:k] += np.eye(k)
            e_ref = np.linalg.norm(a[:, ref.jpvt] - qr @ ref.r) / np.linalg.norm(a)
        else:
            ref = oracle.tuxv(a, oms[i], b, 8, k)
            e = np.linalg.norm(a - o0 @ o1 @ o2.T) / np.linalg.norm(a)
            e_ref = np.linalg.norm(a - ref.u @ ref.x @ ref.v.T) / np.linalg.norm(a)
        ratios.append({"op": "trqrcp" if ops[i] == 0 else "tuxv", "m": m, "n": n, "k": k,
                       "prec": "fp64" if res["prec_used"] == 0 else "bf16",
                       "error": float(e), "oracle_error": float(e_ref),
                       "ratio": round(float(e / e_ref), 5)})
    worst = max(r["ratio"] for r in ratios) if ratios else None
    log(f"C5: sampled errors vs the FP64 oracle: worst ratio {worst}")
    sweep = []
    for r2 in args.serve_sweep:
        nq = min(n_req, args.serve_sweep_requests)
        g2 = gaps * (rate / r2)
        out, _ = _serve_once(pool, oms, ks, ops, tols, g2, n_warm // 2, nq, 2 << 30,
                             args.serve_slots)
        out["rate_per_s"] = r2
        sweep.append(out)
        log(f"C5: 2 GB budget at {r2}/s: p50 {out['p50_ms']} ms, p99 {out['p99_ms']} ms, "
            f"{out['aggregate_tflops']} TFLOP/s, peak running {out['peak_running']}, "
            f"achieved {out['achieved_rate_per_s']}/s")
    res = dict(main)
    res.update({"rate_per_s": rate, "slots": args.serve_slots,
                "sampled_errors": ratios, "worst_error_ratio_vs_oracle": worst,
                "budget_2gb_sweep": sweep,
                "config": {"workload": "serve_trqrcp_tuxv_poisson200_m256-4096_fp32",
                           "pool_matrices": len(pool), "precision": "auto (tol = optimal rank-k error)"}})
    return res


# name, m, n, spectrum (kind, parameter, floor)
QUALITY_MATRICES = (
    ("smooth_1733x1733_pow10", 1733, 1733, ("pow10", 3.0 / 1733.0, 0.0)),
    ("smooth_2232x2232_poly1", 2232, 2232, ("poly", 1.0, 0.0)),
    ("smooth_2442x3888_poly1.5", 2442, 3888, ("poly", 1.5, 1e-3)),
    ("smooth_2658x2525_exp100", 2658, 2525, ("exp", 100.0, 1e-6)),
)


def quality_spectrum(kind, c, floor, r):
    import numpy as np
    i = np.arange(r, dtype=np.float64)
    if kind == "pow10":
        sig = 10.0 ** (-c * i)
    elif kind == "poly":
        sig = (i + 1.0) ** (-c)
    else:
        sig = np.exp(-i / c)
    return sig + floor


def quality_matrix(idx, dev):
    """Synthetic stand-in for one of the matrices of the decomposition-quality
    experiment (Section 5.3, Figure 4), at its shape: strongly correlated
    neighbouring columns (synth.smooth_columns) with a prescribed spectrum
    (10^(-c i), (i+1)^(-c) or exp(-i/c), plus a floor)."""
    import synth
    name, m, n, (kind, c, floor) = QUALITY_MATRICES[idx]
    sig = quality_spectrum(kind, c, floor, min(m, n))
    return name, synth.smooth_columns(m, n, sig, synth.seed_for(5, "U") + 31 * idx, dev)


def trailing_errors(qr, kmax, ranks, norm_a):
    """Relative truncation errors ||A P - Q(:, :k) R(:k, :)||_F / ||A||_F of a
    pivoted QR held in place (first kmax columns factored): the norm of rows k..
    of R and of the trailing block."""
    import torch
    rf = torch.triu(qr)
    rf[kmax:, kmax:] = qr[kmax:, kmax:]
    rows = (rf * rf).sum(dim=1)
    tail = torch.flip(torch.cumsum(torch.flip(rows, [0]), 0), [0])
    return [float(torch.sqrt(tail[k]) / norm_a) for k in ranks]


def quality_curves(a, ranks, seeds, b=32, p=8, h=None, with_qr=True):
    """Error against rank for presorted unpivoted QR, QRCP (Algorithm 2 on the
    GPU), RQRCP (Algorithm 4; TRQRCP gives the same factor at every rank) and
    TUXV (Algorithm 6) over `seeds` Gaussian Omega, and the truncated SVD."""
    import numpy as np
    import torch
    import synth
    from paper_2008_04447_amd import api
    dev = a.device
    m, n = a.shape
    kmax = max(ranks)
    na = float(torch.linalg.norm(a))
    sv = torch.linalg.svdvals(a)
    tail = torch.flip(torch.cumsum(torch.flip(sv * sv, [0]), 0), [0])
    out = {"ranks": list(ranks), "svd": [float(torch.sqrt(tail[k]) / na) for k in ranks]}
    if with_qr:
        order = torch.argsort(torch.linalg.norm(a, dim=0), descending=True)
        q, _ = torch.linalg.qr(a[:, order[:kmax]].contiguous())
        errs = []
        for k in ranks:
            qk = q[:, :k]
            errs.append(float(torch.linalg.norm(a - qk @ (qk.t().contiguous() @ a)) / na))
        out["qr_presorted"] = errs
    x = api.colmajor(a, device=dev)
    api.qrcp_factor(x, kmax, nb=32, handle=h)
    out["qrcp"] = trailing_errors(x, kmax, ranks, na)
    rq, tx = [], []
    for s in range(seeds):
        om = api.colmajor(synth.omega(b + p, m, synth.seed_for(5, "Omega") + s), device=dev)
        x.copy_(a)
        api.rqrcp_factor(x, om, b, p, kmax, handle=h)
        rq.append(trailing_errors(x, kmax, ranks, na))
        row = []
        for k in ranks:
            U, X, V, _ = api.tuxv_svd(a, om, b, p, k, handle=h)
            row.append(float(torch.linalg.norm(a - U @ (X @ V.t().contiguous())) / na))
        tx.append(row)
    rq, tx = np.array(rq), np.array(tx)
    for key, arr in (("rqrcp", rq), ("tuxv", tx)):
        out[key] = {"median": np.median(arr, 0).tolist(), "min": arr.min(0).tolist(),
                    "max": arr.max(0).tolist()}
    return out, rq, tx


def bench_quality(args):
    """Synthetic analogue of the decomposition-quality experiment (Section 5.3,
    Figure 4): error against rank, median / min / max over `quality_seeds`
    Gaussian Omega, b = 32, p = 8, for presorted QR, QRCP, RQRCP (= TRQRCP
    truncated), TUXV and the SVD, on matrices at the four shapes of the paper's
    test set (their data are not available; see quality_matrix)."""
    import numpy as np
    import torch
    from paper_2008_04447_amd import api
    dev = torch.device("cuda", 0)
    h = api.default_handle(0)
    ranks = list(range(32, 321, 32))
    res = {"seeds": args.quality_seeds, "b": 32, "p": 8, "matrices": {}}
    t0 = time.perf_counter()
    for idx in range(len(QUALITY_MATRICES)):
        name, a = quality_matrix(idx, dev)
        curves, rq, tx = quality_curves(a, ranks, args.quality_seeds, h=h)
        h.sync()
        svd, qrcp = np.array(curves["svd"]), np.array(curves["qrcp"])
        med_rq, med_tx = np.median(rq, 0), np.median(tx, 0)
        curves["summary"] = {
            "rqrcp_median_over_qrcp_max": float(np.max(med_rq / qrcp)),
            "rqrcp_median_over_qrcp_min": float(np.min(med_rq / qrcp)),
            "tuxv_median_over_svd_max": float(np.max(med_tx / svd)),
            "tuxv_below_rqrcp_every_run": bool(np.all(tx <= rq * (1 + 1e-12))),
            "tuxv_above_svd_every_run": bool(np.all(tx >= svd * (1 - 1e-12))),
            "rqrcp_spread_max": float(np.max(rq.max(0) / rq.min(0))),
            "tuxv_spread_max": float(np.max(tx.max(0) / tx.min(0))),
            "qr_presorted_over_qrcp_min": float(np.min(np.array(curves["qr_presorted"]) / qrcp)),
        }
        res["matrices"][name] = curves
        log(f"quality {name}: {curves['summary']}")
        del a
        _gpu_mem_clear()
    res["seconds"] = round(time.perf_counter() - t0, 1)
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
                    "c2graded,trqrcp,tuxv,serving")
    ap.add_argument("--c3-steps", type=int, default=3)
    ap.add_argument("--c4-steps", type=int, default=3)
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-warmup", type=int, default=200)
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-pool", type=int, default=48)
    ap.add_argument("--serve-slots", type=int, default=8)
    ap.add_argument("--serve-sweep", default="200,400,800",
                    help="arrival rates (per s) of the 2 GB-budget sweep")
    ap.add_argument("--serve-sweep-requests", type=int, default=1000)
    ap.add_argument("--quality-seeds", type=int, default=100,
                    help="Omega seeds per matrix of the quality experiment (--only quality)")
    ap.add_argument("--no-oracle-ref", action="store_true",
                    help="skip the full-size FP64 oracle references of the truncated workloads")
    ap.add_argument("--only", default="", choices=["", "trqrcp", "tuxv", "serving", "quality"],
                    help="run only this secondary workload and print its result (for profiling)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device-to-device copy 3 times (HBM counter calibration)")
    args = ap.parse_args()
    args.skip = [x for x in args.skip.split(",") if x]
    args.serve_sweep = [float(x) for x in args.serve_sweep.split(",") if x]
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
    if args.only == "quality":
        print(json.dumps({"quality": bench_quality(args)}), flush=True)
        return
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
