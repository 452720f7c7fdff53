#!/usr/bin/env python3
"""Throughput benchmark of the FTLM hot path on one MI355X.

Workload (default): 24 spins s=1/2 on a ring, J = 1 K nearest neighbour plus
all-pairs dipolar coupling at seeded positions on a 1 nm sphere, g = 2,
B = 0.5 T along a seeded direction; Hilbert dimension 2^24; complex128;
R = 10 Gaussian random vectors, N_L = 150 Lanczos steps, 200 temperatures.
One step = one complete FTLM curve: start vectors, O v_1, 150 Lanczos steps
(H*v + update), Krylov eigenpairs, Boltzmann sums for ln Z, E, C, M.

Prints one JSON line.  value = FTLM curves per second (inputs resident in HBM).
roofline = the dominant kernel (the Lanczos H*v launch): algorithmic flops
8 * nnz/row * dim * columns per launch over its mean duration measured with HIP
events around each launch in one extra profiled run.
cpu_baseline = the CPU oracle (plain C, OpenMP) timed on a bounded sample: a few
of its H*v products on one column of the same workload, extrapolated to curves/s
as R * N_L products per curve (vector updates, tridiagonal and sums ignored).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK = {"f64": 78.6, "f32": 157.3}  # TFLOP/s, MI355X published vector peaks
HBM_PEAK_GBPS = 8000.0


def _kernel_sha():
    """Hash of the sources that define the H*v kernels (kernels, their shared
    device helpers and internal header)."""
    h = hashlib.sha256()
    for name in ("kernels.hip", "stream.hip", "hv_common.hpp", "device_reduce.hpp", "ftlm_internal.hpp"):
        h.update(open(os.path.join(ROOT, "paper_2607_25585_amd", "csrc", name), "rb").read())
    return h.hexdigest()[:16]


def _traffic(workload, precision):
    """HBM bytes per H*v launch from the committed rocprofv3 counter summary,
    or None when the kernel source changed since the counters were taken."""
    p = os.path.join(ROOT, "profiles", "hv_traffic.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
        e = d.get("%s_%s" % (workload, precision))
        if not e or e.get("kernel_sha") != _kernel_sha():
            return None
        return float(e["bytes_per_launch"])
    except Exception:
        return None


def cpu_baseline(sysm, spec, budget_s=12.0):
    import numpy as np
    from oracle import ftlm as of
    ham = of.Ham(sysm)
    rng = np.random.default_rng(0)
    v = rng.standard_normal(ham.dim) + 1j * rng.standard_normal(ham.dim)
    times = []
    t_start = time.perf_counter()
    while True:
        t0 = time.perf_counter()
        v = ham.apply(v)
        v /= np.linalg.norm(v)
        times.append(time.perf_counter() - t0)
        if len(times) >= 2 and time.perf_counter() - t_start > budget_s:
            break
        if len(times) >= 20:
            break
    t_hv = float(np.median(times))
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": 1.0 / (spec.R * spec.n_lanczos * t_hv), "unit": "curves/s",
            "cores": threads, "kind": "oracle", "cpu_model": _cpu_model(),
            "cpus_visible": os.cpu_count(),
            "sample": "%d oracle H*v products on one column (%.2f s each, median), "
                      "extrapolated x R*N_L = %d per curve" % (len(times), t_hv,
                                                               spec.R * spec.n_lanczos)}


def cpu_oracle_report(cfg4=True):
    """The oracle (CPU, FP64, OpenMP) timed on this host for every workload:
    H*v per workload (median of five products for cfg1 and cfg2_hb, two for
    cfg2, one for the 5^12-row cfg4 and cfg4_hb); one whole cfg1 curve
    (R=20, N_L=100) and one whole surrogate-ring run; curves/s of cfg2 and cfg4
    extrapolated from their H*v products (x R*N_L), and of the stratified
    batched subset (one instance per spin count x 4 directions) from one H*v
    per instance (x directions*R*N_L).  Each entry says what it extrapolates."""
    import numpy as np

    import ftlm_workloads as W
    from oracle import ftlm as of
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    out = {"cpu_model": _cpu_model(), "threads": threads, "cpus_visible": os.cpu_count(), "workloads": {}}
    res = out["workloads"]

    def hv_s(sysm, n=2):
        ham = of.Ham(sysm)
        rng = np.random.default_rng(0)
        v = rng.standard_normal(ham.dim) + 1j * rng.standard_normal(ham.dim)
        ts = []
        for _ in range(n):
            t0 = time.perf_counter()
            v = ham.apply(v)
            ts.append(time.perf_counter() - t0)
            v /= np.linalg.norm(v)
            print("cpu oracle H*v dim %d: %.3f s" % (ham.dim, ts[-1]), file=sys.stderr, flush=True)
        del ham
        return float(np.median(ts)), len(ts)

    for name in ("cfg1", "cfg2", "cfg2_hb", "cfg4_hb") + (("cfg4",) if cfg4 else ()):
        sysm, spec = W.WORKLOADS[name]()
        t, n = hv_s(sysm, 5 if name in ("cfg1", "cfg2_hb") else 1 if name.startswith("cfg4") else 2)
        res[name] = {"dim": W.dimension(sysm.two_s), "oracle_hv_s": round(t, 5), "hv_samples": n,
                     "curves_per_s_extrapolated": 1.0 / (spec.R * spec.n_lanczos * t),
                     "extrapolation": "x R*N_L = %d H*v per curve" % (spec.R * spec.n_lanczos)}
        print("cpu oracle %s done" % name, file=sys.stderr, flush=True)
    s1, spec1 = W.cfg1()
    t0 = time.perf_counter()
    of.ftlm(s1, spec1.R, spec1.n_lanczos, spec1.T, seed=spec1.seed)
    res["cfg1"]["whole_curve_s"] = round(time.perf_counter() - t0, 4)
    res["cfg1"]["curves_per_s_measured"] = 1.0 / res["cfg1"]["whole_curve_s"]
    s5 = W.cfg5_system(W.cfg5_params(1)[0])
    sp5 = W.cfg5_runspec()
    t0 = time.perf_counter()
    of.ftlm(s5, sp5.R, sp5.n_lanczos, sp5.T, seed=1)
    t5 = time.perf_counter() - t0
    res["surrogate_ring"] = {"dim": W.dimension(s5.two_s), "whole_run_s": round(t5, 4),
                             "curves_per_s_measured": 1.0 / t5,
                             "run": "R=%d, N_L=%d, %d temperatures" % (sp5.R, sp5.n_lanczos, len(sp5.T))}
    print("cpu oracle surrogate ring done", file=sys.stderr, flush=True)
    systems, spec3, _fields = W.cfg3()
    pick = stratified_cfg3(systems)
    n_dirs = 4
    total = 0.0
    per = []
    for k in pick:
        t, _n = hv_s(systems[k], 1)
        per.append({"instance": k, "N": systems[k].n_sites, "oracle_hv_s": round(t, 5)})
        total += n_dirs * spec3.R * spec3.n_lanczos * t
    res["cfg3_stratified"] = {"curves": len(pick) * n_dirs, "instances": per,
                              "curves_per_s_extrapolated": len(pick) * n_dirs / total,
                              "extrapolation": "one H*v per instance x %d directions x R*N_L = %d" % (
                                  n_dirs, spec3.R * spec3.n_lanczos)}
    print("cpu oracle cfg3 subset done", file=sys.stderr, flush=True)
    return out


def _cpu_model():
    """The host CPU's model name (Linux /proc/cpuinfo), or None."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def curve_err(x, ref):
    import numpy as np
    ref = np.asarray(ref)
    floor = 1e-3 * np.max(np.abs(ref))
    return float(np.max(np.abs(np.asarray(x) - ref) / np.maximum(np.abs(ref), max(floor, 1e-300))))


def stratified_cfg3(systems):
    """Indices of the first instance of each spin count 14..22 of the batched
    workload (one instance per size, as the batched protocol's subset asks)."""
    pick = []
    for n in range(14, 23):
        ks = [k for k, s in enumerate(systems) if s.n_sites == n]
        if ks:
            pick.append(ks[0])
    return pick


def batched_vs_plain(n_dirs=4, tune=True, tune_cache=None):
    """Batched FP32-storage FTLM against plain FP64 FTLM on the same curves: a
    stratified subset of the 64-instance batched workload (the first instance
    of every spin count 14..22), n_dirs of its 50 field directions each, R = 16,
    N_L = 120, same seeded random vectors.  The batched launch (columns per
    item, grid, unit rows, unit order) comes from the batched autotuner, timed
    outside the measured region."""
    import numpy as np
    import torch

    import ftlm_workloads as W
    import paper_2607_25585_amd as F
    systems, spec, fields = W.cfg3()
    pick = stratified_cfg3(systems)
    systems = [systems[k] for k in pick]
    n_inst = len(systems)
    fl = [fields[k][:n_dirs] for k in pick]
    hams = [F.Hamiltonian(s) for s in systems]
    btune = None
    if tune:
        from paper_2607_25585_amd import autotune
        if tune_cache:
            os.environ["FTLM_TUNE_CACHE"] = tune_cache
        btune = autotune.tune_batched(hams, spec.R, spec.T, fl, seed=spec.seed, precision=F.FTLM_C64,
                                      use_cache=bool(tune_cache))
        print("batched autotune done", btune, file=sys.stderr, flush=True)
    # warm-up on a tiny run (kernel loading), outside the timed region
    F.run_batched(hams[:1], spec.R, 4, spec.T, [fl[0][:1]], seed=spec.seed, precision=F.FTLM_C64)
    F.run(hams[0], spec.R, 4, spec.T, seed=spec.seed, fields=fl[0][:1])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bat = F.run_batched(hams, spec.R, spec.n_lanczos, spec.T, fl, seed=spec.seed, precision=F.FTLM_C64,
                        columns=btune["columns"] if btune else 0)
    torch.cuda.synchronize()
    t_b = time.perf_counter() - t0
    print("batched fp32 subset done", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    plain = [F.run(h, spec.R, spec.n_lanczos, spec.T, seed=spec.seed, fields=fl[k], instance=k)
             for k, h in enumerate(hams)]
    F.batched_set_tuning(0, 0, 0)
    torch.cuda.synchronize()
    t_p = time.perf_counter() - t0
    print("plain fp64 subset done", file=sys.stderr, flush=True)
    n_curves = n_inst * n_dirs
    err_c = max(curve_err(bat[k]["C"][f], plain[k]["C"][f]) for k in range(n_inst) for f in range(n_dirs))
    err_m = max(curve_err(bat[k]["M"][f], plain[k]["M"][f]) for k in range(n_inst) for f in range(n_dirs))
    return {"curves": n_curves, "subset": "instances %s (N=%s, one per spin count) x field directions "
            "0..%d, R=%d, N_L=%d" % (pick, [s.n_sites for s in systems], n_dirs - 1, spec.R, spec.n_lanczos),
            "batched_tuning": btune,
            "batched_fp32_curves_per_s": round(n_curves / t_b, 4),
            "plain_fp64_curves_per_s": round(n_curves / t_p, 4),
            "speedup": round(t_p / t_b, 3), "max_C_err_vs_plain_fp64": err_c,
            "max_M_err_vs_plain_fp64": err_m, "C_within_1e-3": bool(err_c <= 1e-3)}


def cfg3_full(mode, first, last, save, group=8, tune_cache=None):
    """The whole 64-instance batched workload (50 field directions, R = 16,
    N_L = 120, 200 temperatures) or instances [first, last) of it: batched
    FP32 storage (one run_batched call per group of instances, each instance
    drawing its own random vectors, so the groups give the curves of one run)
    or plain FP64 (one run per instance, all its directions), timed from the
    first call to the last with the Hamiltonians compiled beforehand.  The
    batched launch is the batched autotuner's choice on the stratified subset
    (one instance per spin count, 4 directions), tuned outside the timed
    region.  Saves every curve (ln Z, E, C, M) to `save` (npz) for
    cfg3_compare."""
    import numpy as np
    import torch

    import ftlm_workloads as W
    import paper_2607_25585_amd as F
    systems, spec, fields = W.cfg3()
    idx = list(range(first, last))
    hams = [F.Hamiltonian(systems[k]) for k in idx]
    btune = None
    if mode == "batched":
        from paper_2607_25585_amd import autotune
        if tune_cache:
            os.environ["FTLM_TUNE_CACHE"] = tune_cache
        pick = stratified_cfg3(systems)
        th = [F.Hamiltonian(systems[k]) for k in pick]
        btune = autotune.tune_batched(th, spec.R, spec.T, [fields[k][:4] for k in pick], seed=spec.seed,
                                      precision=F.FTLM_C64, use_cache=bool(tune_cache))
        for h in th:
            h.close()
        print("batched autotune done", btune, file=sys.stderr, flush=True)
        F.run_batched(hams[:1], spec.R, 4, spec.T, [fields[idx[0]][:1]], seed=spec.seed, precision=F.FTLM_C64)
    else:
        F.run(hams[0], spec.R, 4, spec.T, seed=spec.seed, fields=fields[idx[0]][:1])
    torch.cuda.synchronize()
    out = {kk: np.zeros((len(idx), fields.shape[1], len(spec.T))) for kk in ("lnZ", "E", "C", "M")}
    t0 = time.perf_counter()
    if mode == "batched":
        for g0 in range(0, len(idx), group):
            res = F.run_batched(hams[g0:g0 + group], spec.R, spec.n_lanczos, spec.T,
                                [fields[k] for k in idx[g0:g0 + group]], seed=spec.seed, precision=F.FTLM_C64,
                                columns=btune["columns"], instance0=idx[g0])
            for j, r in enumerate(res):
                for kk in out:
                    out[kk][g0 + j] = r[kk]
            print("batched instances %d..%d done (%.1f s)" % (idx[g0], idx[min(g0 + group, len(idx)) - 1],
                                                              time.perf_counter() - t0), file=sys.stderr, flush=True)
        F.batched_set_tuning(0, 0, 0)
    else:
        for j, k in enumerate(idx):
            r = F.run(hams[j], spec.R, spec.n_lanczos, spec.T, seed=spec.seed, fields=fields[k], instance=k)
            for kk in out:
                out[kk][j] = r[kk]
            print("plain instance %d done (%.1f s)" % (k, time.perf_counter() - t0), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    np.savez(save, instances=np.array(idx), **out)
    n_curves = len(idx) * fields.shape[1]
    return {"mode": mode, "instances": [first, last], "curves": n_curves, "seconds": round(dt, 2),
            "curves_per_s": round(n_curves / dt, 4), "batched_tuning": btune,
            "spins": [systems[k].n_sites for k in idx]}


def cfg3_compare(batched_file, plain_files):
    """Accuracy gate of the whole batched workload: every batched FP32 curve
    against the plain FP64 curve of the same instance, direction and random
    vectors; max over T of the relative C and M error (floor 1e-3 of the
    curve's maximum)."""
    import numpy as np
    b = np.load(batched_file)
    bi = {int(k): j for j, k in enumerate(b["instances"])}
    ec, em = [], []
    for f in plain_files:
        p = np.load(f)
        for j, k in enumerate(p["instances"]):
            jb = bi[int(k)]
            for d in range(p["C"].shape[1]):
                ec.append(curve_err(b["C"][jb, d], p["C"][j, d]))
                em.append(curve_err(b["M"][jb, d], p["M"][j, d]))
    ec, em = np.array(ec), np.array(em)
    return {"curves_compared": int(len(ec)), "max_C_err": float(ec.max()), "p99_C_err": float(np.quantile(ec, 0.99)),
            "max_M_err": float(em.max()), "curves_C_err_above_1e-3": int((ec > 1e-3).sum()),
            "C_within_1e-3": bool(ec.max() <= 1e-3)}


def hv_rate(ham, dt, reps):
    """Median of reps H*v launches, each bracketed by HIP events on the current
    stream (the one ham.apply launches on)."""
    import torch
    g = torch.Generator(device="cuda")
    g.manual_seed(0)
    v = torch.randn((ham.dim,), dtype=dt, device="cuda", generator=g)
    w = torch.empty_like(v)
    ham.apply(v, w)
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        ham.apply(v, w)
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    del v, w
    torch.cuda.empty_cache()
    return float(sorted(times)[len(times) // 2]), float(min(times))


def hv_hbm(cases=(("cfg4", "c128"), ("cfg4", "c64"), ("cfg4_hb", "c128"), ("cfg2_hb", "c128")), reps=20):
    """H*v alone at full size, one column, tuned launch, for the large single
    system (12 spins 2, all-pairs dipolar) in complex128 and complex64 storage,
    and for the short-range variants where the HBM roofline binds (nearest and
    next-nearest Heisenberg exchange, field along z).  algorithmic bytes = read v
    + write w once (32 B per row at complex128, 16 at complex64); flops = 8 per
    stored nonzero; traffic = calibrated rocprofv3 FETCH_SIZE + WRITE_SIZE per
    product from profiles/hv_traffic.json (null when the kernel sources changed
    since the counters were taken, or when no counters were taken)."""
    import torch

    import ftlm_workloads as W
    import paper_2607_25585_amd as F
    from paper_2607_25585_amd import autotune
    out = {}
    for wl, pr in cases:
        sysm = W.WORKLOADS[wl]()[0]
        ham = F.Hamiltonian(sysm)
        prec, dt, es = (F.FTLM_C128, torch.complex128, 16) if pr == "c128" else (F.FTLM_C64, torch.complex64, 8)
        tuning = autotune.tune(ham, prec, 1, use_cache=False)
        ms, ms_min = hv_rate(ham, dt, reps)
        alg = 2.0 * es * ham.dim
        gbps = alg / (ms * 1e-3) / 1e9
        tf = 8.0 * ham.nnz_per_row * ham.dim / (ms * 1e-3) / 1e12
        vpeak = PEAK["f64"] if pr == "c128" else PEAK["f32"]
        out["%s_%s" % (wl, pr)] = {
            "dim": ham.dim, "nnz_per_row": round(ham.nnz_per_row, 3), "precision": pr,
            "hv_ms_median": round(ms, 4), "hv_ms_min": round(ms_min, 4),
            "algorithmic_bytes": alg, "achieved_GBps": round(gbps, 1), "peak_GBps": HBM_PEAK_GBPS,
            "frac": round(gbps / HBM_PEAK_GBPS, 4), "TFLOPs": round(tf, 3),
            "valu_frac": round(tf / vpeak, 4), "valu_peak_TFLOPs": vpeak,
            "traffic": _traffic(wl, pr), "tuning": tuning}
        print("hv_hbm %s %s done" % (wl, pr), file=sys.stderr, flush=True)
        ham.close()
        del ham
        torch.cuda.empty_cache()
    return out


def stream_bw(sizes_mib=(48, 96, 4096)):
    """Streaming rates of plain device kernels (torch's copy and sum) by buffer
    size, each timed with HIP events on the current stream: the ceiling the
    H*v traffic rates compare with.  Buffers of 48 and 96 MiB stay in the
    last-level cache once touched; 4 GiB streams from HBM."""
    import torch
    out = []
    for mb in sizes_mib:
        n = mb * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
            a.sum()
        torch.cuda.synchronize()
        reps = max(10, 8000 // mb)

        def ms_per(fn):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                fn()
            e1.record()
            e1.synchronize()
            return e0.elapsed_time(e1) / reps

        nbytes = mb * (1 << 20)
        tc = ms_per(lambda: b.copy_(a))
        ts = ms_per(lambda: a.sum())
        out.append({"MiB": mb, "copy_GBps_read_plus_write": round(2 * nbytes / (tc * 1e-3) / 1e9, 1),
                    "sum_GBps_read": round(nbytes / (ts * 1e-3) / 1e9, 1), "reps": reps})
        print("stream_bw %d MiB done" % mb, file=sys.stderr, flush=True)
        del a, b
        torch.cuda.empty_cache()
    return out


def hv_only(args, sysm, spec, ham, prec, K):
    """H*v throughput alone: a plain device copy of 1 GiB (the calibration
    kernel for HBM byte counters), then args.hv_reps applications of the tuned
    H*v, each bracketed by HIP events on the launching stream."""
    import torch
    src = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    src.fill_(1)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    dt = torch.complex128 if args.precision == "c128" else torch.complex64
    g = torch.Generator(device="cuda")
    g.manual_seed(0)
    shape = (ham.dim,) if K == 1 else (ham.dim, K)
    v = torch.randn(shape, dtype=dt, device="cuda", generator=g)
    w = torch.empty_like(v)
    ham.apply(v, w)
    torch.cuda.synchronize()
    times = []
    for _ in range(args.hv_reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        ham.apply(v, w)
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    ms = float(sorted(times)[len(times) // 2])
    es = 16 if args.precision == "c128" else 8
    nnz = ham.nnz_per_row
    gbps = 2.0 * es * ham.dim * K / (ms * 1e-3) / 1e9
    tflops = 8.0 * nnz * ham.dim * K / (ms * 1e-3) / 1e12
    return {"metric": "H*v algorithmic GB/s (read v + write w)", "value": round(gbps, 2),
            "unit": "GB/s", "n_gpus": 1, "hv_reps": args.hv_reps, "hv_ms_median": round(ms, 4),
            "hv_ms_min": round(min(times), 4), "tflops": round(tflops, 3),
            "hbm_frac_algorithmic": round(gbps / HBM_PEAK_GBPS, 4),
            "f64_or_f32_valu_frac": round(tflops / PEAK["f64" if es == 16 else "f32"], 4),
            "dtype": "f64" if es == 16 else "f32", "data": "synthetic",
            "config": {"workload": "%s: N=%d spins, dim %d, %s, %d columns" % (
                args.workload, sysm.n_sites, ham.dim, args.precision, K),
                "nnz_per_row": round(nnz, 3)}}


def surrogate_report(n_train, n_test, train_s, n_val=500, tol=0.10, t_min=2.0, n_powder_sets=8, n_dirs=50,
                     r_truth=160, tols=(0.05, 0.10, 0.15, 0.20), save=None, n_members=4):
    """The learned surrogate on the 8-spin s=3/2 ring data: FTLM training curves
    (batched FP32 path, R=20, N_L=100, 200 temperatures), an ensemble of n_members
    MLPs trained by the library's BF16/FP32 kernels, and its errors against a reference
    that is itself FTLM: FP64 curves with r_truth random vectors (statistical error
    sqrt(20 / r_truth) of the R=20 recipe's).  The gate is calibrated on a
    validation split so that the accepted curves have their 90th percentile of C
    error above t_min at most tol (also reported for each of `tols`); next to the
    surrogate's errors stand those of an FP64 FTLM run with the recipe's R=20 on the
    same held-out sets, the alternative the surrogate replaces.  Then the
    powder-average protocol: n_dirs field directions x 200 T per set, surrogate
    against batched FTLM, curves/s and the error of the powder average."""
    import numpy as np
    import torch

    import ftlm_workloads as W
    from paper_2607_25585_amd import surrogate as S
    T = W.t_grid()
    spec = W.cfg5_runspec()
    ptrain = W.cfg5_params(n_train, seed=5000)
    ptest = W.cfg5_params(n_test, seed=5001)
    pval = W.cfg5_params(n_val, seed=5002)
    t0 = time.perf_counter()
    parts = []
    for a in range(0, n_train, 1024):  # chunk seeds depend only on the row offset
        parts.append(S.generate_dataset(ptrain[a:a + 1024], T, spec.R, spec.n_lanczos, seed=spec.seed + a,
                                        chunk=256))
        print("surrogate: %d training curves" % min(n_train, a + 1024), file=sys.stderr, flush=True)
    lz, mm, cc = (np.concatenate([p[i] for p in parts]) for i in range(3))
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t0
    print("surrogate: %d training curves in %.1f s" % (n_train, t_gen), file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    lzr, mmr, ccr = S.generate_dataset(ptest, T, spec.R, spec.n_lanczos, seed=spec.seed + 999, chunk=256,
                                       precision=0)
    torch.cuda.synchronize()
    t_ftlm64 = time.perf_counter() - t0
    print("surrogate: %d held-out FP64 curves (R=%d) in %.1f s" % (n_test, spec.R, t_ftlm64), file=sys.stderr,
          flush=True)
    # reference curves: FP64 FTLM with r_truth vectors (chunks sized for r_truth columns per set)
    chunk_t = max(8, (256 * spec.R) // r_truth)
    lzt, mmt, cct = S.generate_dataset(ptest, T, r_truth, spec.n_lanczos, seed=spec.seed + 1499, chunk=chunk_t,
                                       precision=0)
    print("surrogate: %d held-out reference curves (R=%d)" % (n_test, r_truth), file=sys.stderr, flush=True)
    _lv, _mv, ccv = S.generate_dataset(pval, T, r_truth, spec.n_lanczos, seed=spec.seed + 1999, chunk=chunk_t,
                                       precision=0)
    print("surrogate: %d validation reference curves (R=%d)" % (n_val, r_truth), file=sys.stderr, flush=True)
    x = S.encode_inputs(ptrain, T)
    y = S.encode_targets(lz, mm, cc, T)
    models, losses = [], []
    t0 = time.perf_counter()
    for seed in range(n_members):
        m = S.MLP(seed=seed)
        last = [time.perf_counter()]

        def progress(ep, loss, last=last, seed=seed):
            if time.perf_counter() - last[0] > 20.0:
                print("surrogate: member %d epoch %d loss %.3g" % (seed, ep, loss), file=sys.stderr, flush=True)
                last[0] = time.perf_counter()
        losses.append(S.train(m, x, y, epochs=400, batch=4096, lr=2e-3, seed=seed, time_budget_s=train_s,
                              progress=progress)[-1])
        models.append(m)
        print("surrogate: member %d trained" % seed, file=sys.stderr, flush=True)
    t_train = time.perf_counter() - t0
    print("surrogate: trained in %.1f s" % t_train, file=sys.stderr, flush=True)
    ens = S.Surrogate(models, t_min=t_min)
    if save:
        # every member's decoded curves on the validation and held-out sets, with the
        # reference curves, for studies of the gate score
        mv = [S.decode_outputs(y, T) for y in ens._members(pval, T)]
        mt = [S.decode_outputs(y, T) for y in ens._members(ptest, T)]
        np.savez(save, T=T, pval=pval, ptest=ptest, C_val_ref=ccv, C_test_ref=cct, M_test_ref=mmt,
                 C_test_r20=ccr, C_val_members=np.array([m[2] for m in mv]),
                 C_test_members=np.array([m[2] for m in mt]), M_test_members=np.array([m[1] for m in mt]))
    plz, pm, pc, score = ens.predict(ptest, T)
    dom = ens.in_domain(ptest, T)
    eC1_all = S.c_relerr(pc, cct, T, t_min)
    q = lambda a: {"median": float(np.median(a)), "p90": float(np.quantile(a, 0.9)), "max": float(np.max(a))} if len(a) else None  # noqa: E731
    gate_scan = []
    for tl in tols:
        a_val = ens.calibrate(pval, ccv, T, tol=tl, quantile=0.9)
        acc_t = dom & (score <= ens.threshold)
        gate_scan.append({"tol_p90": tl, "threshold": ens.threshold, "validation_acceptance": a_val,
                          "heldout_acceptance": float(np.mean(acc_t)),
                          "heldout_accepted_C_relerr_A12_T_ge_tmin": q(eC1_all[acc_t])})
    acc_val = ens.calibrate(pval, ccv, T, tol=tol, quantile=0.9)
    ftlm_r20 = S.c_relerr(ccr, cct, T, t_min)
    torch.cuda.synchronize()
    reps = 20
    t0 = time.perf_counter()
    for _ in range(reps):
        ens.predict(ptest, T)
    torch.cuda.synchronize()
    t_sur = (time.perf_counter() - t0) / reps

    def rel(a, b, cols=slice(None)):
        a, b = a[:, cols], b[:, cols]
        floor = 1e-3 * np.max(np.abs(b), axis=1, keepdims=True)
        return np.max(np.abs(a - b) / np.maximum(np.abs(b), np.maximum(floor, 1e-12)), axis=1)
    eC, eM = rel(pc, cct), np.max(np.abs(pm - mmt), axis=1)
    eZ = np.max(np.abs(plz - lzt), axis=1)
    hi = T >= t_min
    eC1, eM1 = rel(pc, cct, hi), rel(pm, mmt, hi)
    acc = dom & (score <= ens.threshold)
    rms = lambda a, b: float(np.sqrt(np.mean((a - b) ** 2)))  # noqa: E731

    # powder average: every held-out set's |B| over n_dirs directions uniform on the sphere
    rng = np.random.default_rng(5003)
    dirs = W.unit_vectors(rng, n_dirs)
    theta, phi = np.arccos(np.clip(dirs[:, 2], -1, 1)), np.mod(np.arctan2(dirs[:, 1], dirs[:, 0]), 2 * np.pi)
    pp = np.repeat(ptest, n_dirs, axis=0)
    pp[:, 4] = np.tile(theta, n_test)
    pp[:, 5] = np.tile(phi, n_test)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _l, pm_p, pc_p, sc_p = ens.predict(pp, T)
    torch.cuda.synchronize()
    t_sur_p = time.perf_counter() - t0
    acc_p = (sc_p <= ens.threshold).reshape(n_test, n_dirs)
    sub = pp[: n_powder_sets * n_dirs]
    t0 = time.perf_counter()
    _l, pm_f, pc_f = S.generate_dataset(sub, T, spec.R, spec.n_lanczos, seed=spec.seed + 2999, chunk=200,
                                        precision=1)
    torch.cuda.synchronize()
    t_ftlm_p = time.perf_counter() - t0
    print("surrogate: powder protocol done", file=sys.stderr, flush=True)
    cs = pc_p[: n_powder_sets * n_dirs].reshape(n_powder_sets, n_dirs, -1).mean(1)
    cf = pc_f.reshape(n_powder_sets, n_dirs, -1).mean(1)
    ms_ = pm_p[: n_powder_sets * n_dirs].reshape(n_powder_sets, n_dirs, -1).mean(1)
    mf = pm_f.reshape(n_powder_sets, n_dirs, -1).mean(1)
    return {"train_sets": n_train, "validation_sets": n_val, "test_sets": n_test, "T_points": len(T),
            "rmse_all_T": {"lnZ": rms(plz, lzt), "M_muB": rms(pm, mmt), "C_kB": rms(pc, cct)},
            "t_min_K": t_min,
            "heldout_C_relerr_A12_T_ge_tmin": q(eC1), "heldout_M_relerr_A12_T_ge_tmin": q(eM1),
            "reference": "FP64 FTLM, R=%d, N_L=%d" % (r_truth, spec.n_lanczos),
            "ftlm_R%d_fp64_C_relerr_A12_T_ge_tmin" % spec.R: q(ftlm_r20),
            "ftlm_R%d_fp64_M_relerr_A12_T_ge_tmin" % spec.R: q(rel(mmr, mmt, hi)),
            "gate_scan": gate_scan,
            "members": n_members,
            "gate": {"score": "ensemble spread on C above t_min (std over members / |mean|, floor 1e-3 max)",
                     "tolerance": "p90 of C relative error above %g K <= %g" % (t_min, tol),
                     "threshold": ens.threshold, "validation_acceptance": acc_val,
                     "heldout_acceptance": float(np.mean(acc)),
                     "heldout_accepted_C_relerr_A12_T_ge_tmin": q(eC1[acc]),
                     "heldout_accepted_M_relerr_A12_T_ge_tmin": q(eM1[acc]),
                     "powder_directions_accepted": float(np.mean(acc_p))},
            "ftlm_fp32_batched_curves_per_s": round(n_train / t_gen, 3),
            "ftlm_fp64_batched_curves_per_s": round(n_test / t_ftlm64, 3),
            "surrogate_curves_per_s": round(n_test / t_sur, 1),
            "speedup_vs_fp64_ftlm": round((n_test / t_sur) / (n_test / t_ftlm64), 1),
            "powder": {"directions": n_dirs, "T_points": len(T),
                       "surrogate_curves_per_s": round(len(pp) / t_sur_p, 1),
                       "ftlm_fp32_curves_per_s": round(len(sub) / t_ftlm_p, 2),
                       "surrogate_powder_sets_per_s": round(n_test / t_sur_p, 2),
                       "ftlm_powder_sets_per_s": round(n_powder_sets / t_ftlm_p, 4),
                       "powder_C_relerr_A12_T_ge_tmin": q(rel(cs, cf, hi)),
                       "powder_M_relerr_A12_T_ge_tmin": q(rel(ms_, mf, hi)),
                       "ftlm_sets": n_powder_sets},
            "train_s": round(t_train, 1), "final_losses": [float(v) for v in losses],
            "heldout_C_relerr_A12": q(eC), "heldout_M_abserr_muB": q(eM), "heldout_lnZ_abserr": q(eZ)}


def extras_report():
    """Throughput of the forms beyond the plain method, each on its own workload:
    sFTLM with time-reversed pairs on the N=6, s=5/2 ring (both printed fields),
    the Chebyshev expansion next to FTLM on the same random vectors (s=1 ring),
    and the powder-averaged FTLM of the Mn9 cube (10 dodecahedron directions)."""
    import numpy as np
    import torch

    import ftlm_workloads as W
    import paper_2607_25585_amd as F
    out = {}
    sysm, spec = W.ring6()
    ham = F.Hamiltonian(sysm)
    fields = [[0.0, 0.0, 0.1], [0.0, 0.0, 1.0]]
    F.run_sftlm(ham, 2, 8, spec.T, seed=spec.seed, fields=fields[:1])  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = F.run_sftlm(ham, spec.R, spec.n_lanczos, spec.T, seed=spec.seed, fields=fields)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out["sftlm_ring6"] = {"curves": 2, "R": spec.R, "N_L": spec.n_lanczos, "dim": ham.dim,
                          "curves_per_s": round(2 / dt, 4), "s_per_curve": round(dt / 2, 3),
                          "M_at_T_min": [float(r["M"][f][0]) for f in range(2)]}
    print("extras: sFTLM done", file=sys.stderr, flush=True)
    ham.close()
    sysm, spec = W.cfg1()
    ham = F.Hamiltonian(sysm)
    T = spec.T
    F.run(ham, 2, 8, T, seed=spec.seed)
    F.run_kpm(ham, 2, 16, T, seed=spec.seed)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lz = F.run(ham, spec.R, spec.n_lanczos, T, seed=spec.seed)
    torch.cuda.synchronize()
    t_l = time.perf_counter() - t0
    t0 = time.perf_counter()
    kp = F.run_kpm(ham, spec.R, 2000, T, seed=spec.seed, n_bound_steps=60)
    torch.cuda.synchronize()
    t_k = time.perf_counter() - t0
    lz32 = F.run(ham, spec.R, spec.n_lanczos, T, seed=spec.seed, precision=F.FTLM_C64)
    out["fp32_vs_fp64_cfg1"] = {"R": spec.R, "N_L": spec.n_lanczos,
                                "lnZ_abs": float(np.max(np.abs(lz32["lnZ"][0] - lz["lnZ"][0]))),
                                "E_rel": curve_err(lz32["E"][0], lz["E"][0]),
                                "C_rel": curve_err(lz32["C"][0], lz["C"][0]),
                                "M_rel": curve_err(lz32["M"][0], lz["M"][0]),
                                "E0_abs": float(abs(lz32["E_min"][0] - lz["E_min"][0]))}
    hiT = T >= 1.0
    out["kpm_cfg1"] = {"R": spec.R, "N_moments": 2000, "lanczos_N_L": spec.n_lanczos,
                       "kpm_curves_per_s": round(1 / t_k, 3), "lanczos_curves_per_s": round(1 / t_l, 3),
                       "max_C_rel_diff_T_ge_1K": curve_err(kp["C"][0][hiT], lz["C"][0][hiT]),
                       "E_lo": float(kp["E_lo"][0]), "E_hi": float(kp["E_hi"][0])}
    print("extras: KPM done", file=sys.stderr, flush=True)
    ham.close()
    sysm, spec = W.mn9()
    ham = F.Hamiltonian(sysm)
    F.run(ham, 1, 4, spec.T, seed=spec.seed)
    torch.cuda.synchronize()
    R, NL = 4, 100
    t0 = time.perf_counter()
    res = F.run(ham, R, NL, spec.T, seed=spec.seed, fields=spec.fields)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    powder = res["M"].mean(axis=0)
    out["mn9_powder"] = {"dim": ham.dim, "directions": len(spec.fields), "R": R, "N_L": NL,
                         "curves_per_s": round(len(spec.fields) / dt, 4),
                         "powder_M_T_over_B_at_T_max": float(powder[-1] * spec.T[-1] / 1.0),
                         "T_max": float(spec.T[-1]), "B_T": 1.0}
    print("extras: Mn9 done", file=sys.stderr, flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cfg2", choices=["cfg1", "cfg2", "cfg2_hb", "cfg4", "cfg4_hb", "ring6", "mn9"])
    ap.add_argument("--precision", default="c128", choices=["c128", "c64"])
    ap.add_argument("--columns", type=int, default=0,
                    help="random vectors iterated together (0 = library default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-hbm", action="store_true",
                    help="skip the short-range H*v GB/s object (cfg4_hb, cfg2_hb)")
    ap.add_argument("--batched-only", action="store_true",
                    help="only the batched-FP32 vs plain-FP64 comparison on the cfg3 subset")
    ap.add_argument("--cfg3-full", choices=["batched", "plain"], default=None,
                    help="the whole 64-instance batched workload (or --instances) on one path; "
                    "saves every curve to --save")
    ap.add_argument("--instances", default="0:64", help="instance range first:last for --cfg3-full")
    ap.add_argument("--save", default="cfg3_curves.npz")
    ap.add_argument("--cfg3-compare", nargs="+", default=None,
                    help="BATCHED.npz PLAIN.npz [PLAIN.npz ...]: accuracy gate of --cfg3-full runs (CPU only)")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--tune-cache", default=None,
                    help="JSON tuning cache: reuse a stored choice instead of timing the candidates")
    ap.add_argument("--hv-only", action="store_true",
                    help="time the H*v product alone (GB/s line) instead of whole curves")
    ap.add_argument("--hv-reps", type=int, default=20)
    ap.add_argument("--cpu-oracle", action="store_true",
                    help="time the CPU oracle on every workload (no GPU used)")
    ap.add_argument("--stream-bw", action="store_true",
                    help="streaming rates of plain device copy and sum kernels by buffer size")
    ap.add_argument("--extras", action="store_true",
                    help="sFTLM (ring6), Chebyshev vs Lanczos (cfg1) and Mn9 powder throughput")
    ap.add_argument("--surrogate", action="store_true",
                    help="surrogate report on the s=3/2 ring data instead of the FTLM curve bench")
    ap.add_argument("--surrogate-train", type=int, default=20000)
    ap.add_argument("--surrogate-test", type=int, default=1000)
    ap.add_argument("--surrogate-train-s", type=float, default=120.0, help="training seconds per member")
    ap.add_argument("--surrogate-tol", type=float, default=0.10,
                    help="gate contract: p90 of the C relative error above --surrogate-tmin")
    ap.add_argument("--surrogate-tmin", type=float, default=2.0)
    ap.add_argument("--surrogate-rtruth", type=int, default=160,
                    help="random vectors of the FP64 FTLM reference curves (held-out and validation sets)")
    ap.add_argument("--surrogate-members", type=int, default=4, help="ensemble members")
    ap.add_argument("--surrogate-save", default=None,
                    help="npz file for the members' curves and the reference curves (gate studies)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    if args.cpu_oracle:
        out = {"metric": "CPU oracle timings by workload (FP64, OpenMP)", "data": "synthetic",
               "config": {"workload": "cfg1, cfg2, cfg2_hb, cfg4_hb, cfg4, surrogate ring, cfg3 stratified subset"}}
        out.update(cpu_oracle_report())
        print(json.dumps(out), flush=True)
        return

    if args.cfg3_compare:
        out = {"metric": "max relative C, M error of batched FP32 against plain FP64, whole cfg3",
               "config": {"workload": "cfg3: 64 instances x 50 field directions, R=16, N_L=120"}}
        out.update(cfg3_compare(args.cfg3_compare[0], args.cfg3_compare[1:]))
        print(json.dumps(out), flush=True)
        return

    import numpy as np
    import torch

    import ftlm_workloads as W
    import paper_2607_25585_amd as F

    torch.cuda.set_device(0)
    if args.cfg3_full:
        a, b = (int(x) for x in args.instances.split(":"))
        out = {"metric": "FTLM curves/s, whole cfg3 (%s path)" % args.cfg3_full, "unit": "curves/s", "n_gpus": 1,
               "dtype": "c64 storage, f64 recurrence" if args.cfg3_full == "batched" else "f64",
               "data": "synthetic", "config": {"workload": "cfg3: instances %d..%d x 50 field directions, "
                                                           "R=16, N_L=120, 200 temperatures" % (a, b - 1)}}
        out.update(cfg3_full(args.cfg3_full, a, b, args.save, tune_cache=args.tune_cache))
        print(json.dumps(out), flush=True)
        return
    if args.stream_bw:
        out = {"metric": "device streaming GB/s by buffer size (torch copy and sum)", "n_gpus": 1,
               "peak_GBps": HBM_PEAK_GBPS, "data": "synthetic", "config": {"workload": "float64 buffers"}}
        out["sizes"] = stream_bw()
        print(json.dumps(out), flush=True)
        return
    if args.extras:
        out = {"metric": "curves/s of sFTLM, Chebyshev and powder-averaged FTLM", "n_gpus": 1,
               "data": "synthetic", "config": {"workload": "ring6 / cfg1 / mn9"}}
        out.update(extras_report())
        print(json.dumps(out), flush=True)
        return
    if args.batched_only:
        out = {"metric": "FTLM curves/s batched-FP32 vs plain FP64 at C(T) <=1e-3 rel", "n_gpus": 1,
               "data": "synthetic",
               "config": {"workload": "cfg3 stratified subset: one instance per N=14..22 x 4 field directions"}}
        out["batched_fp32_vs_plain_fp64"] = batched_vs_plain(tune_cache=args.tune_cache)
        print(json.dumps(out), flush=True)
        return
    if args.surrogate:
        out = {"metric": "surrogate curves/s vs FTLM at held-out accuracy", "n_gpus": 1, "data": "synthetic",
               "config": {"workload": "8-spin s=3/2 ring, MLP 7-256-256-256-3 (bf16 weights, fp32 accumulate)"}}
        out.update(surrogate_report(args.surrogate_train, args.surrogate_test, args.surrogate_train_s,
                                    tol=args.surrogate_tol, t_min=args.surrogate_tmin,
                                    r_truth=args.surrogate_rtruth, save=args.surrogate_save,
                                    n_members=args.surrogate_members))
        print(json.dumps(out), flush=True)
        return
    sysm, spec = W.WORKLOADS[args.workload]()
    prec = F.FTLM_C128 if args.precision == "c128" else F.FTLM_C64
    ham = F.Hamiltonian(sysm)
    # the library's default column count (ftlm_run_params.columns = 0)
    K = args.columns if args.columns > 0 else (
        1 if ham.dim >= (1 << 20) else min(spec.R, 4) if ham.dim >= (1 << 17)
        else min(spec.R, 16) if ham.dim >= (1 << 14) else min(spec.R, 64))
    ws = None

    def step(time_hv=False):
        return F.run(ham, spec.R, spec.n_lanczos, spec.T, seed=spec.seed, precision=prec,
                     columns=K, workspace=ws, time_hv=time_hv)

    # size the workspace once, outside the timed region
    import ctypes
    from paper_2607_25585_amd import _ffi
    if not args.hv_only:
        p, keep = F._params(spec.R, spec.n_lanczos, spec.T, spec.seed, None, prec, K, None, 0)
        nb = ctypes.c_size_t()
        _ffi.check(_ffi.lib().ftlm_run_workspace_size(ham.handle, ctypes.byref(p), ctypes.byref(nb)))
        ws = torch.empty(int(nb.value), dtype=torch.uint8, device="cuda")
    tuning = None
    if not args.no_tune:
        from paper_2607_25585_amd import autotune
        if args.tune_cache:
            os.environ["FTLM_TUNE_CACHE"] = args.tune_cache
        tuning = autotune.tune(ham, prec, K, use_cache=bool(args.tune_cache))
        print("autotune done", tuning, file=sys.stderr, flush=True)

    if args.hv_only:
        out = hv_only(args, sysm, spec, ham, prec, K)
        out["hv_tuning"] = tuning
        print(json.dumps(out), flush=True)
        return

    for _ in range(args.warmup):
        step()
        print("warmup step done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        res = step()
        print("timed step %d done" % i, file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    value = args.steps / elapsed

    prof = step(time_hv=True)
    hv_ms = float(prof["hv_ms"][0] / max(int(prof["hv_launches"][0]), 1))
    nnz = ham.nnz_per_row
    flops = 8.0 * nnz * ham.dim * K
    dt = "f64" if prec == F.FTLM_C128 else "f32"
    achieved = flops / (hv_ms * 1e-3) / 1e12
    es = 16 if prec == F.FTLM_C128 else 8
    hv_gbps = 2.0 * es * ham.dim * K / (hv_ms * 1e-3) / 1e9
    traffic = _traffic(args.workload, args.precision)
    roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK[dt], "unit": "TFLOP/s",
            "frac": round(achieved / PEAK[dt], 4), "traffic": traffic}

    out = {
        "metric": "H·v HBM GB/s; FTLM curves/s batched-FP32 vs plain FP64 at C(T) ≤1e-3 rel",
        "value": round(value, 5),
        "unit": "curves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == F.FTLM_C128 else "f32-storage/f64-recurrence",
        "data": "synthetic",
        "config": {"workload": "%s: N=%d spins, dim %d, %s, R=%d, N_L=%d, %d temperatures, "
                               "%d columns per wave" % (args.workload, sysm.n_sites, ham.dim,
                                                        args.precision, spec.R, spec.n_lanczos,
                                                        len(spec.T), K),
                   "nnz_per_row": round(nnz, 3)},
        "hv_ms_per_launch": round(hv_ms, 4),
        "hv_algorithmic_GBps": round(hv_gbps, 1),
        "hv_hbm_frac_algorithmic": round(hv_gbps / HBM_PEAK_GBPS, 4),
        "roofline": roof,
        "E_min": float(res["E_min"][0]),
        "hv_tuning": tuning,
    }
    if not args.no_batched:
        out["batched_fp32_vs_plain_fp64"] = batched_vs_plain(tune_cache=args.tune_cache)
    if not args.no_hbm:
        out["hv_hbm"] = hv_hbm()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(sysm, spec)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
