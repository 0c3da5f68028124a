#!/usr/bin/env python3
"""Benchmark of the online solve f^ ~ K^{-1} u on one MI355X.

Workload (the headline configuration): 1D FIO, N = 2^18, Phi = x xi + c(x)|xi|,
c(x) = (2 + sin 2 pi x)/16, q = 9 Chebyshev points, HSS tolerance 1e-3 with
p = 10 oversampling, 64 right-hand sides u = K~ f with f complex Gaussian (seed 1).
One step solves all 64 right-hand sides by iterative refinement with a step count
fixed beforehand by the residual-checked solve (relative residual 5e-9) of a held-out
block (seed 2); the residual-checked solve of the timed block is timed and reported
too.  The relative error of every column of f^ against f is checked after the timed
region and must be below 1e-8 (`accuracy_ok`; a path that misses it is not chosen
as the headline, and the run exits with status 3 if the headline misses it):
  fp64  : K~^* and K~ applied in FP64;
  mixed : K~^* applied in FP32 (FP32 factors and coefficients), residual K~ f and
          the ULV solve in FP64;
  split16: as mixed, with the transfer factors of K~^* applied on the matrix cores
          in split FP16 (hi + lo halves, FP32 accumulation).
`value` is the faster mixed path's RHS/s (64 / seconds per step; `config.mixed_variant`
names it); the FP64 path and the other mixed path are reported beside it.  Offline work
(BF, HSS and ULV construction) happens before the timed region; inputs are resident in
HBM when it starts.  Also reported: `roofline` (explicit-form work of the dominant
kernel against the published peaks, spill and counter traffic beside it), the serving
workload in split-FP16 and FP64 at 200 requests/s and at a saturating rate, the N = 2^16
direct FP64 solve (with c = 0), the 2D and variable-amplitude workloads, and the oracle
timed on the host (`cpu_baseline`).

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline] [--no-serve] ...
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP16_MFMA_PEAK_TFLOPS = 2500.0 # MI355X dense FP16 matrix (no sparsity)
FP64_PEAK_TFLOPS = 78.6        # MI355X FP64 vector
# MI355X FP32 vector, published (it counts packed FP32: 2 lanes per instruction).  Every kernel here
# is compiled without packed FP32, which caps what they can reach at half of it:
# 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz = 78.6 TFLOP/s.
FP32_PEAK_TFLOPS = 157.3
FP32_NONPACKED_TFLOPS = 78.6
METRIC = "RHS solved/s at N=2^18, rel err 1e-8: FP64 vs mixed; p50/p99 latency"


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_source_hash():
    """Hash of the butterfly apply kernels' source; stored counter traffic is valid only for it."""
    import hashlib
    h = hashlib.sha256()
    for f in ("bf_apply.h", "bf_apply_f64.hip", "bf_apply_f32.hip", "bf_lowprec.hip"):
        with open(os.path.join(ROOT, "paper_2609_11520_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_traffic(kernel):
    """HBM bytes per launch measured with rocprofv3 (FETCH_SIZE + WRITE_SIZE, scaled by a copy kernel),
    from profiles/traffic.json, or None when the kernel source changed since the counters were taken."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    with open(p) as fh:
        d = json.load(fh)
    if d.get("source_hash") != kernel_source_hash():
        return None
    v = d.get("kernels", {}).get(kernel)
    return None if v is None else v.get("hbm_bytes_per_launch")


def copy_calibration(torch, nbytes=1 << 30):
    """A plain device copy of known size; its FETCH_SIZE / WRITE_SIZE readings scale the counters."""
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    src.fill_(1)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def traffic_from(fetch_dir, write_dir, n=1 << 18, k=64, q=9, out_path=None):
    """Writes profiles/traffic.json from two rocprofv3 counter runs of this benchmark (--pmc
    FETCH_SIZE, then --pmc WRITE_SIZE, csv output) and prints a markdown summary.  The counters
    (KiB per dispatch) are scaled by what they read for the 1 GiB device copy of
    copy_calibration; per kernel label, the average over the run's dispatches at N = n with k
    columns (one column tile)."""
    import csv
    import glob

    def load(d, counter):
        f = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
        if not f:
            raise SystemExit("no counter_collection.csv under " + d)
        per = {}
        for r in csv.DictReader(open(f[0])):
            if r["Counter_Name"] != counter:
                continue
            key = int(r["Dispatch_Id"])
            name, grid, v = r["Kernel_Name"], int(r["Grid_Size"]), float(r["Counter_Value"])
            old = per.get(key)
            per[key] = (name, grid, v + (old[2] if old else 0.0))
        return per

    fetch, write = load(fetch_dir, "FETCH_SIZE"), load(write_dir, "WRITE_SIZE")
    one_gib_kib = float(1 << 20)
    cf = [v for (_, _, v) in write.values() if abs(v - one_gib_kib) < 0.01 * one_gib_kib]
    copies = [fetch[d][2] for d, (_, _, v) in write.items()
              if abs(v - one_gib_kib) < 0.01 * one_gib_kib and d in fetch and fetch[d][2] > 0.25 * one_gib_kib]
    if not copies or not cf:
        raise SystemExit("the 1 GiB calibration copy was not found in the counter runs")
    fs, ws = one_gib_kib / max(copies), one_gib_kib / max(cf)
    tiles = n >> 3
    labels = {
        "bf_split16": (lambda nm: nm.startswith("void fio::(anonymous namespace)::k_split_fused<3,")
                       or "k_split_fused<3," in nm, tiles * 512),
        "bf_struct_f64": (lambda nm: "k_struct_fused<double, 9, 3," in nm and nm.split(">")[0].endswith("false"), tiles * 512),
        "bf_struct_f32": (lambda nm: "k_struct_fused<float, 9, 3," in nm and nm.split(">")[0].endswith("false"), tiles * 512),
        "bf_struct_leaf_f64": (lambda nm: "k_struct_fused<double, 9, 3," in nm and nm.split(">")[0].endswith("true"), tiles * 512),
        "bf_struct_leaf_f32": (lambda nm: "k_struct_fused<float, 9, 3," in nm and nm.split(">")[0].endswith("true"), tiles * 512),
        "bf_leaf_out_f64": (lambda nm: "k_leaf_io<double, 9, false," in nm, (n >> 3) // 4 * 256),
        "bf_leaf_out_f32": (lambda nm: "k_leaf_io<float, 9, false," in nm, (n >> 3) // 4 * 256),
    }
    out = {"source_hash": kernel_source_hash(), "fetch_scale": fs, "write_scale": ws, "kernels": {},
           "note": "hbm_bytes_per_launch: FETCH_SIZE x fetch_scale + WRITE_SIZE x write_scale per launch "
                   "(KiB -> bytes), N=2^%d, %d RHS; algorithmic and spill bytes per launch by the explicit-form "
                   "model of bench.kernel_model" % (int(np.log2(n)), k)}
    rows = []
    for lab, (match, grid) in labels.items():
        ds = [d for d, (nm, g, _) in write.items() if match(nm) and g == grid and d in fetch]
        if not ds:
            continue
        b = [(fetch[d][2] * fs + write[d][2] * ws) * 1024.0 for d in ds]
        avg = sum(b) / len(b)
        rec = {"hbm_bytes_per_launch": avg, "dispatches": len(ds),
               "fetch_kib_per_launch": sum(fetch[d][2] for d in ds) / len(ds),
               "write_kib_per_launch": sum(write[d][2] for d in ds) / len(ds)}
        m = kernel_model(lab, n, q, k)
        if m is not None:
            rec["algorithmic_bytes_per_launch"] = m[0]
            rec["spill_bytes_per_launch"] = m[2]
        out["kernels"][lab] = rec
        rows.append((lab, len(ds), rec["fetch_kib_per_launch"], rec["write_kib_per_launch"], avg,
                     rec.get("algorithmic_bytes_per_launch"), rec.get("spill_bytes_per_launch")))
    with open(out_path or os.path.join(ROOT, "profiles", "traffic.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print("calibration: FETCH_SIZE x %.4f, WRITE_SIZE x %.4f (1 GiB copy)" % (fs, ws))
    print()
    print("| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | HBM bytes | explicit-form bytes | ratio | spill bytes |")
    print("|---|---|---|---|---|---|---|---|")
    for lab, nd, fk, wk, hb, ab, sb in rows:
        print("| %s | %d | %.0f | %.0f | %.3e | %s | %s | %s |" % (
            lab, nd, fk, wk, hb, "-" if ab is None else "%.3e" % ab, "-" if ab is None else "%.2f" % (hb / ab),
            "-" if sb is None else "%.3e" % sb))


def pass_plan(n, kmax=3):
    """Structured butterfly passes of one apply: (levels, applies M) per launch."""
    L = int(np.log2(n))
    nl = max(L - 3, L // 2) - L // 2
    plan = []
    hi = nl
    while hi > 0:                       # C side (or B* side) from the top, M on the last pass
        lo = max(hi - kmax, 0)
        plan.append((hi - lo, lo == 0))
        hi = lo
    lo = 0
    while lo < nl:
        hi = min(lo + kmax, nl)
        plan.append((hi - lo, False))
        lo = hi
    return plan


def kernel_model(name, n, q, k):
    """Algorithmic work per launch of the butterfly kernels, by the explicit-factor count:
    (bytes, flops, spill_bytes, peak_tflops).

    The method's work is the product with the explicit factors of eq. bf: every entry read once
    per apply (16 B in FP64, 8 B in FP32 or as split-FP16 hi + lo halves) and a complex
    multiply-add (8 flops) per entry and column; the three split products count 3 x 8.  A
    structured pass (3 transfer levels of (N/2) 4q^2 entries each, plus M's N q^2 on the pass that
    applies it) is charged those entries whatever form the kernel reads them in.  The N x k
    vectors read and written by an apply (2 N k 16 B) belong to its leaf kernels; the per-pass
    round trip of the coefficient block (2 N q k e) is an implementation cost, reported apart as
    spill_bytes."""
    e = 16 if name.endswith("f64") else 8
    plan = pass_plan(n)
    transfer = (n // 2) * 4 * q * q              # entries of one transfer level
    mid = n * q * q
    if name == "bf_split16" or name.startswith("bf_struct"):
        ent = sum(kl * transfer + (mid if epi else 0) for kl, epi in plan) / len(plan)
        mult = 3 if name == "bf_split16" else 1
        peak = FP16_MFMA_PEAK_TFLOPS if name == "bf_split16" else (
            FP64_PEAK_TFLOPS if e == 16 else FP32_PEAK_TFLOPS)
        return ent * e, mult * 8.0 * ent * k, 2.0 * n * q * k * (8 if name == "bf_split16" else e), peak
    if name.startswith("bf_transfer"):
        return transfer * e, 8.0 * transfer * k, 2.0 * n * q * k * e, FP64_PEAK_TFLOPS if e == 16 else FP32_PEAK_TFLOPS
    return None


def roofline_of(name, n, q, k, avg_ms, traffic):
    """The roofline record of one kernel: bound = the larger of the explicit-factor byte and flop
    times at the published peaks; frac = bound time / measured time."""
    m = kernel_model(name, n, q, k)
    if m is None:
        return None
    byts, flops, spill, peak = m
    t_mem, t_alu = byts / (HBM_PEAK_GBS * 1e9), flops / (peak * 1e12)
    if t_mem >= t_alu:
        ach = byts / (avg_ms * 1e-3) / 1e9
        r = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
             "frac": round(ach / HBM_PEAK_GBS, 4)}
    else:
        ach = flops / (avg_ms * 1e-3) / 1e12
        r = {"bound": "mfma" if name == "bf_split16" else "alu", "achieved": round(ach, 2), "peak": peak,
             "unit": "TFLOP/s", "frac": round(ach / peak, 4)}
    r.update({"traffic": traffic, "kernel": name, "avg_launch_ms": round(avg_ms, 4),
              "algorithmic_bytes_per_launch": int(byts), "algorithmic_flops_per_launch": float(flops),
              "spill_bytes_per_launch": int(spill),
              "achieved_with_spill_gbs": round((byts + spill) / (avg_ms * 1e-3) / 1e9, 1),
              "traffic_over_algorithmic": None if traffic is None else round(traffic / byts, 3)})
    if name.endswith("f32"):
        r["fp32_nonpacked_peak"] = FP32_NONPACKED_TFLOPS
    return r


def host_info():
    """Host CPU model and thread count (what lscpu and nproc report)."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:
        nproc = os.cpu_count()
    return {"cpu_model": model, "nproc": nproc, "logical_cpus": os.cpu_count()}


def cpu_baseline(n, q, nrhs_gpu, ir_steps, ranks, repeats=3):
    """The oracle as it stands timed on the host: its FP64 refinement solve (oracle.solve.refine:
    f = F K~^* u, then `ir_steps` steps of f += F K~^*(u - K~ f)) of one of the benchmark's
    right-hand sides (column 0 of the same seeded f, u = K~ f with the oracle's own factors of the
    same operator), the median of `repeats` runs after one warm-up, on all host cores and on one.
    The ULV factors come from HSS generators with the tree and per-node ranks of the GPU
    construction and seeded entries (the oracle's own HSS construction of this operator takes
    hours on the host); a ULV solve's cost depends only on those shapes."""
    from threadpoolctl import threadpool_limits
    from oracle import bf as obf, fio as ofio, ulv as oulv, solve as osolve
    import fio_inputs as fi
    log("cpu baseline: building the oracle factors (untimed)")
    B = obf.BF1D(n, q, ofio.PHASE_SIN16)
    f = fi.rhs(1, n, 1)
    u = B.apply(f)
    fac = oulv.factor(synthetic_hss(n, 64, ranks))
    res = {}
    for label, threads in (("all_cores", None), ("one_core", 1)):
        with threadpool_limits(limits=threads):
            osolve.refine(B, fac, u, ir_steps)
            walls, cpus = [], []
            for _ in range(repeats):
                t0, c0 = time.perf_counter(), time.process_time()
                osolve.refine(B, fac, u, ir_steps)
                walls.append(time.perf_counter() - t0)
                cpus.append(time.process_time() - c0)
        i = int(np.argsort(walls)[len(walls) // 2])
        res[label] = {"s_per_rhs": round(walls[i], 3), "rhs_per_s": round(1.0 / walls[i], 4),
                      "threads_used": round(cpus[i] / walls[i], 2), "runs_s": [round(w, 3) for w in walls]}
    host = host_info()
    return {"value": res["all_cores"]["rhs_per_s"], "unit": "RHS/s",
            "cores": max(1, int(round(res["all_cores"]["threads_used"]))), "kind": "oracle",
            "sample": "oracle FP64 refinement solve (oracle.solve.refine, %d steps: %d K~* and %d K~ applies "
                      "and %d ULV solves, plus the final residual) of 1 of the %d RHS at N=%d: column 0 of the "
                      "same seeded f, u = K~ f from the oracle's own factors; ULV factors of seeded HSS "
                      "generators with the GPU construction's tree and per-node ranks; median of %d runs after "
                      "1 warm-up" % (ir_steps, ir_steps + 1, ir_steps + 1, ir_steps + 1, nrhs_gpu, n, repeats,),
            "host": host, "all_cores": res["all_cores"], "one_core": res["one_core"]}


def synthetic_hss(n, leaf, ranks):
    """Hermitian positive definite HSS generators (timing only) on the tree of N / leaf leaves
    with the given per-node ranks {level: [rank of node j]}: orthonormal bases, small coupling
    blocks and N I leaf blocks, all seeded."""
    from oracle import hss as ohss
    import fio_inputs as fi
    h = ohss.HSS(n, leaf)
    Lh = h.Lh
    for l in range(1, Lh + 1):
        h.rank[l] = [int(r) for r in ranks[l]]
    for l in range(1, Lh + 1):
        h.U[l] = []
        for j in range(2 ** l):
            m, r = h.m_of(l, j), h.rank[l][j]
            Q, _ = np.linalg.qr(fi.complex_gaussian(j, fi.PURPOSE_DATA, m, max(r, 1), level=l))
            h.U[l].append(Q[:, :r])
    for l in range(Lh):
        h.B[l] = [0.01 * fi.complex_gaussian(j, fi.PURPOSE_DATA, h.rank[l + 1][2 * j + 1], h.rank[l + 1][2 * j],
                                             level=100 + l) for j in range(2 ** l)]
    h.D = [n * np.eye(leaf, dtype=np.complex128) for _ in range(2 ** Lh)]
    return h


def serving_operators(F, torch, fi, rel_res=5e-9):
    """The serving workload's three resident operators N = 2^14, 2^16, 2^18 (phase (2 + sin 2 pi x)/16,
    q = 9, HSS tolerance 1e-3), each with its refinement step count per low precision calibrated on
    a seeded calibration block (seed 100 + e) that no served request uses."""
    dev = torch.device("cuda")
    ops = []
    for e in (14, 16, 18):
        n = 1 << e
        B = F.BF(n, 9, 2.0 / 16, 1.0 / 16, precs=(F.FIO_PREC_FP64, F.FIO_PREC_SPLIT_FP16))
        U = F.ULV(F.HSS.from_bf(B, tol=1e-3, p=10, seed=1003))
        fcal = torch.from_numpy(np.ascontiguousarray(fi.rhs(100 + e, n, 32).T)).to(dev).t()
        ucal = B.apply(fcal)
        nir = {}
        for name, prec in (("split16", F.FIO_PREC_SPLIT_FP16), ("fp64", F.FIO_PREC_FP64)):
            _, info = F.approx_solve(B, U, ucal, mode=F.FIO_SOLVE_IR, prec=prec, rel_res_tol=rel_res, max_ir=6)
            nir[name] = max(1, info.ir_steps)
        fpool = fi.rhs(4 + e, n, 32)
        fd = torch.from_numpy(np.ascontiguousarray(fpool.T)).to(dev).t()
        ops.append({"n": n, "B": B, "U": U, "u": B.apply(fd), "f": fpool, "nir": nir})
    torch.cuda.synchronize()
    return ops


def serving(F, torch, fi, ops, variant, duration, rate, seed=4, mem_budget=0, streams=2):
    """Serving workload: Poisson arrivals at `rate` requests/s for `duration` s, each request 1..32
    right-hand sides (uniform) for an operator drawn uniformly from `ops`; `variant` "split16"
    (refinement with the split-FP16 K~^*) or "fp64" (the same refinement in FP64), step counts
    calibrated per operator on held-out columns; batches of up to 64 columns on `streams` slots
    whose arenas share `mem_budget` bytes, replayed from captured hipGraphs.  Latency = completion
    - submission (host clock); sustained RHS/s = RHS served / (last completion - first submission).
    Every served column is checked against its known f (u = K~ f)."""
    prec = F.FIO_PREC_SPLIT_FP16 if variant == "split16" else F.FIO_PREC_FP64
    arr = fi.poisson_arrivals(seed, rate, duration)
    ks = fi.integers(seed, fi.PURPOSE_DATA, 1, 32, len(arr))
    which = fi.integers(seed + 1, fi.PURPOSE_DATA, 0, len(ops) - 1, len(arr))
    # every request gets its own output block; inputs are column slices of the operator's pool
    outs = [F.empty(ops[w]["n"], int(k)) for w, k in zip(which, ks)]
    warm = [F.empty(o["n"], 1) for o in ops]
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    srv = F.Server(max_batch_rhs=64, streams=streams, mem_budget=mem_budget, use_graphs=True, width_bucket=16)
    ids = [srv.add_operator(o["B"], o["U"], mode=F.FIO_SOLVE_IR, prec=prec, max_ir=o["nir"][variant])
           for o in ops]
    # warm-up request per operator (the server allocates its arenas and captures its graphs here)
    for i, o in enumerate(ops):
        srv.submit(ids[i], o["u"][:, :1], warm[i])
    srv.wait_all()
    torch.cuda.synchronize()
    held = free0 - torch.cuda.mem_get_info()[0]
    nwarm = len(ops)
    t0 = srv.now()
    rids = []
    for t, w, k, out in zip(arr, which, ks, outs):
        while srv.now() - t0 < t:
            time.sleep(min(2e-4, max(0.0, t - (srv.now() - t0))))
        rids.append(srv.submit(ids[w], ops[w]["u"][:, :int(k)], out))
    srv.wait_all()
    lat, first, last = [], None, 0.0
    for r in rids:
        i = srv.info(r)
        lat.append((i["t_done"] - i["t_submit"]) * 1e3)
        first = i["t_submit"] if first is None else min(first, i["t_submit"])
        last = max(last, i["t_done"])
    err = 0.0
    for w, k, out in zip(which, ks, outs):
        fh = out.cpu().numpy()
        f = ops[w]["f"][:, :int(k)]
        err = max(err, float((np.linalg.norm(fh - f, axis=0) / np.linalg.norm(f, axis=0)).max()))
    st = srv.stats()
    srv.close()
    lat = np.array(lat)
    rhs = int(np.sum(ks))
    return {"variant": variant, "rate_req_per_s": rate, "duration_s": duration, "seed": seed,
            "requests": len(rids), "rhs": rhs, "offered_rhs_per_s": round(rhs / duration, 1),
            "rhs_per_s": round(rhs / (last - first), 1),
            "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                           "mean": float(lat.mean()), "max": float(lat.max())},
            "batches": st["batches"] - nwarm, "max_queue": st["max_queue"],
            "mem_budget_bytes": mem_budget, "device_bytes_held": int(held), "peak_batch_bytes": st["peak_bytes"],
            "max_col_rel_err": err, "accuracy_ok": bool(err <= 1e-8),
            "ir_steps": [o["nir"][variant] for o in ops]}


def graph_replay(F, torch, fn, out, f_host, k, steps, warmup):
    """Capture fn (one solve into out, no host synchronisation, no allocation) into a graph and
    time its replays; the error of the replayed result is checked against f_host afterwards."""
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fn()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    out.zero_()
    for _ in range(warmup):
        g.replay()
    torch.cuda.synchronize()
    lat = []
    t0 = time.perf_counter()
    for _ in range(steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        g.replay()
        e1.record()
        lat.append((e0, e1))
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    lat_ms = np.array([x.elapsed_time(y) for x, y in lat])
    err = np.linalg.norm(out.cpu().numpy() - f_host, axis=0) / np.linalg.norm(f_host, axis=0)
    del g
    return {"value": k / (ms / 1e3), "ms_per_step": ms, "max_col_rel_err": float(err.max()),
            "latency_ms": {"p50": float(np.percentile(lat_ms, 50)), "p99": float(np.percentile(lat_ms, 99))}}


def chosen(report):
    """The choices of a fio_bf_autotune report."""
    return [x.strip()[len("chosen "):] for x in report.split(";") if x.strip().startswith("chosen")]


def workload_2d(F, torch, fi, steps, warmup, rel_res=5e-9, solve=True, var_amp=False):
    """2D workload (Section 5.2 phase, a = 1; with var_amp, Section 5.3's isotropic phase
    c(x)||xi||, c = (3 + sin 2 pi x1 sin 2 pi x2)/8, and amplitude H0^(1)(2 pi rho) exp(-2 pi i rho)):
    n = 128 per dimension (N = 16384, odd L), q = 9 (r = 81), 8 right-hand sides.  Times the BF
    applies (FP64 and FP32, forward and adjoint) with per-kernel events, and, after the offline
    HSS (tolerance 1e-3, p = 10) and ULV construction, the direct FP64 solve, the refinement to a
    relative residual of 5e-9 (FP64 and mixed) and the preconditioned CG to 1e-12."""
    n, k, q = 128, 8, 9
    N = n * n
    dev = torch.device("cuda")
    t = time.perf_counter()
    if var_amp:
        B = F.BF(n, q, 3.0 / 8, 1.0 / 8, precs=(F.FIO_PREC_FP64, F.FIO_PREC_FP32), dim=2,
                 phase_kind=F.FIO_PHASE2_ISO, amp="hankel")
    else:
        B = F.BF(n, q, 2.0 / 16, 1.0 / 16, precs=(F.FIO_PREC_FP64, F.FIO_PREC_FP32), dim=2)
    torch.cuda.synchronize()
    t_bf = time.perf_counter() - t
    f_host = fi.rhs(1, N, k)
    f = torch.from_numpy(np.ascontiguousarray(f_host.T)).to(dev).t()
    out = F.empty(N, k)
    ws = torch.empty(B.workspace_size(k, F.FIO_PREC_FP64), dtype=torch.uint8, device=dev)
    # tile autotuner: the 8-column applies in both precisions, and the wide blocks (64+ columns)
    # of the HSS sampling in FP64
    tuned = {}
    for prec, pn in ((F.FIO_PREC_FP64, "fp64_k8"), (F.FIO_PREC_FP32, "fp32_k8")):
        tuned[pn] = chosen(B.autotune(f, prec=prec, reps=5, ws=ws))
    wide = torch.randn((64, N), dtype=torch.complex128, device=dev).t()
    tuned["fp64_k64"] = chosen(B.autotune(wide, prec=F.FIO_PREC_FP64, reps=2))
    del wide
    applies, kstats = {}, {}
    for prec, pn in ((F.FIO_PREC_FP64, "fp64"), (F.FIO_PREC_FP32, "fp32")):
        for adj in (False, True):
            fn = B.apply_adj if adj else B.apply
            for _ in range(warmup):
                fn(f, prec=prec, out=out, ws=ws)
            torch.cuda.synchronize()
            F.timing_reset()
            F.timing_enable(True)
            t0 = time.perf_counter()
            for _ in range(steps):
                fn(f, prec=prec, out=out, ws=ws)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / steps
            F.timing_enable(False)
            key = "%s_%s" % (pn, "adj" if adj else "fwd")
            applies[key] = {"ms": round(ms, 4), "rhs_per_s": k / (ms / 1e3)}
            kstats[key] = {kn: F.timing_query(kn) for kn in F.timing_names()}
    # roofline of the dominant 2D kernel: the FP64 middle factor, explicit q^2 x q^2 blocks streamed once
    # per 8-column chunk, plus the coefficients in and out
    L = 7
    h = (L + 1) // 2
    S = 4 ** h
    nM = S * S * q ** 4
    chunks = (k + 7) // 8
    byts = nM * 16 * chunks + 2 * N * q * q * k * 16
    flops = 8.0 * nM * k
    cnt, tot = kstats["fp64_fwd"]["bf2_M_f64"]
    avg = tot / cnt
    roof = {"kernel": "bf2_M_f64", "bound": "hbm", "achieved": round(byts / (avg * 1e-3) / 1e9, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(byts / (avg * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "avg_launch_ms": round(avg, 4), "algorithmic_bytes_per_launch": int(byts),
            "algorithmic_flops_per_launch": flops}
    wl = ("2D FIO n=128 (N=16384), Phi = x.xi + c(x)||xi||, c = (3 + sin sin)/8, amplitude "
          "H0(1)(2 pi rho) exp(-2 pi i rho) of Section 5.3" if var_amp else
          "2D FIO n=128 (N=16384), Phi = x.xi + sqrt(c1^2 xi1^2 + c2^2 xi2^2) of Section 5.2")
    res = {"workload": wl + ", q=9, 8 RHS (seed 1)",
           "bf_build_s": round(t_bf, 3), "autotuned_tiles": tuned, "apply": applies, "roofline_middle": roof,
           "kernels_ms": {kk: {kn: [c, round(m, 3)] for kn, (c, m) in v.items()} for kk, v in kstats.items()}}
    if solve:
        t = time.perf_counter()
        H = F.HSS.from_bf(B, tol=1e-3, p=10, seed=1003)
        torch.cuda.synchronize()
        t_hss = time.perf_counter() - t
        t = time.perf_counter()
        U = F.ULV(H)
        torch.cuda.synchronize()
        t_ulv = time.perf_counter() - t
        u = B.apply(f)
        sol = {}
        fd = F.empty(N, k)
        for _ in range(warmup):
            F.approx_solve(B, U, u, out=fd)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            F.approx_solve(B, U, u, out=fd)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        err = np.linalg.norm(fd.cpu().numpy() - f_host, axis=0) / np.linalg.norm(f_host, axis=0)
        sol["direct_fp64"] = {"ms": round(ms, 3), "rhs_per_s": k / (ms / 1e3), "max_col_rel_err": float(err.max())}
        for name, prec in (("fp64", F.FIO_PREC_FP64), ("mixed", F.FIO_PREC_FP32)):
            _, info = F.approx_solve(B, U, u, mode=F.FIO_SOLVE_IR, prec=prec, rel_res_tol=rel_res, max_ir=10, out=fd)
            nir = max(1, info.ir_steps)
            kw = dict(mode=F.FIO_SOLVE_IR, prec=prec, rel_res_tol=0.0, max_ir=nir, out=fd)
            for _ in range(warmup):
                F.approx_solve(B, U, u, **kw)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                F.approx_solve(B, U, u, **kw)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / steps
            err = np.linalg.norm(fd.cpu().numpy() - f_host, axis=0) / np.linalg.norm(f_host, axis=0)
            sol[name] = {"ms": round(ms, 3), "rhs_per_s": k / (ms / 1e3), "ir_steps": nir,
                         "max_col_rel_err": float(err.max())}
        # the paper's iterative solver: PCG preconditioned by F to a relative residual of 1e-12
        _, info = F.approx_solve(B, U, u, mode=F.FIO_SOLVE_PCG, rel_res_tol=1e-12, max_ir=30, out=fd)
        nit = info.ir_steps
        kw = dict(mode=F.FIO_SOLVE_PCG, rel_res_tol=0.0, max_ir=nit, out=fd)
        for _ in range(warmup):
            F.approx_solve(B, U, u, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            F.approx_solve(B, U, u, **kw)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        err = np.linalg.norm(fd.cpu().numpy() - f_host, axis=0) / np.linalg.norm(f_host, axis=0)
        sol["pcg_fp64"] = {"ms": round(ms, 3), "rhs_per_s": k / (ms / 1e3), "iterations": nit,
                           "max_col_rel_err": float(err.max())}
        # the same construction with the K~^* K~ samples applied in FP32 (hss_opts.sample_prec)
        torch.cuda.synchronize()
        t = time.perf_counter()
        H32 = F.HSS.from_bf(B, tol=1e-3, p=10, seed=1003, sample_prec=F.FIO_PREC_FP32)
        torch.cuda.synchronize()
        t_hss32 = time.perf_counter() - t
        U32 = F.ULV(H32)
        _, info32 = F.approx_solve(B, U32, u, mode=F.FIO_SOLVE_IR, prec=F.FIO_PREC_FP32, rel_res_tol=rel_res,
                                   max_ir=10, out=fd)
        err32 = np.linalg.norm(fd.cpu().numpy() - f_host, axis=0) / np.linalg.norm(f_host, axis=0)
        sol["mixed_on_fp32_sampled_hss"] = {"ir_steps": int(info32.ir_steps), "max_col_rel_err": float(err32.max())}
        del H32, U32
        # Section 3.1's sample count s_l = m_l + r_l + p with the rank guessed from the level below
        # (hss_opts.adaptive); the test-matrix columns drawn are counted through the callback
        drawn = {"adaptive": 0, "default": 0}

        def counting(key):
            inner = F.omega_torch(1003)

            def cb(ctx, level, rows, cols, out, stream):
                drawn[key] += int(cols)
                return inner(ctx, level, rows, cols, out, stream)
            return F._lib.OMEGA_FN(cb), inner
        cb_def = counting("default")
        F.HSS.from_bf(B, tol=1e-3, p=10, omega=cb_def[0])
        torch.cuda.synchronize()
        cb_ad = counting("adaptive")
        t = time.perf_counter()
        Had = F.HSS.from_bf(B, tol=1e-3, p=10, omega=cb_ad[0], adaptive=True)
        torch.cuda.synchronize()
        t_hss_ad = time.perf_counter() - t
        Uad = F.ULV(Had)
        _, info_ad = F.approx_solve(B, Uad, u, mode=F.FIO_SOLVE_IR, prec=F.FIO_PREC_FP32, rel_res_tol=rel_res,
                                    max_ir=10, out=fd)
        err_ad = np.linalg.norm(fd.cpu().numpy() - f_host, axis=0) / np.linalg.norm(f_host, axis=0)
        sol["mixed_on_adaptive_hss"] = {"ir_steps": int(info_ad.ir_steps), "max_col_rel_err": float(err_ad.max())}
        del Had, Uad
        res.update({"offline_s": {"hss": round(t_hss, 2), "ulv": round(t_ulv, 2),
                                  "hss_fp32_samples": round(t_hss32, 2), "hss_adaptive_samples": round(t_hss_ad, 2)},
                    "hss_sample_columns": drawn,
                    "hss_max_rank_per_level": {str(l): int(max(v)) for l, v in H.ranks().items()},
                    "solve": sol})
    return res


def workload_var_amp(F, torch, fi, steps, warmup, n=1 << 18, k=64, rel_res=1e-9):
    """Section 5.1's variable-amplitude operator at N = 2^18: a Gaussian sum of m = 10 terms
    (sigma^2 = 0.1, seeded centers) and the phase (2 + sin 2 pi x)/8 |xi|, q = 9, 64 right-hand
    sides.  Times the offline build (BF, HSS at tolerance 1e-3 with p = 10, ULV), the split-FP16
    refinement to a relative residual of 1e-9 (step count calibrated, then fixed; the amplitude
    makes K~ worse conditioned than the unit-amplitude operator, so a residual of 5e-9 leaves
    errors near 2e-8) and the
    preconditioned CG to 1e-12 (its iteration count is the figure Section 5.1 reports)."""
    dev = torch.device("cuda")
    cx, cxi = fi.amplitude_centers(1, n)
    t = time.perf_counter()
    B = F.BF(n, 9, 2.0 / 8, 1.0 / 8, precs=(F.FIO_PREC_FP64, F.FIO_PREC_FP32, F.FIO_PREC_SPLIT_FP16),
             amp=(cx, cxi, 0.1))
    torch.cuda.synchronize()
    t_bf = time.perf_counter() - t
    t = time.perf_counter()
    H = F.HSS.from_bf(B, tol=1e-3, p=10, seed=1005)
    torch.cuda.synchronize()
    t_hss = time.perf_counter() - t
    ranks = H.ranks()
    t = time.perf_counter()
    U = F.ULV(H)
    torch.cuda.synchronize()
    t_ulv = time.perf_counter() - t
    f_host = fi.rhs(1, n, k)
    f = torch.from_numpy(np.ascontiguousarray(f_host.T)).to(dev).t()
    u = B.apply(f)
    B.autotune(u, prec=F.FIO_PREC_SPLIT_FP16, reps=3)
    out = F.empty(n, k)

    def err():
        return float((np.linalg.norm(out.cpu().numpy() - f_host, axis=0) / np.linalg.norm(f_host, axis=0)).max())

    def timed(kw):
        for _ in range(warmup):
            _, info = F.approx_solve(B, U, u, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            _, info = F.approx_solve(B, U, u, **kw)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / steps, info

    res = {}
    ws = torch.empty(F.solve_workspace_size(B, U, k, F.FIO_SOLVE_IR, F.FIO_PREC_SPLIT_FP16, rel_res, 8),
                     dtype=torch.uint8, device=dev)
    _, info = timed(dict(mode=F.FIO_SOLVE_IR, prec=F.FIO_PREC_SPLIT_FP16, rel_res_tol=rel_res, max_ir=8,
                         out=out, ws=ws))
    nir, rr = info.ir_steps, info.rel_res
    ms, _ = timed(dict(mode=F.FIO_SOLVE_IR, prec=F.FIO_PREC_SPLIT_FP16, rel_res_tol=0.0, max_ir=nir, out=out, ws=ws))
    res["split16_ir"] = {"value": k / (ms / 1e3), "ms_per_step": round(ms, 3), "ir_steps": int(nir),
                         "rel_res": rr, "max_col_rel_err": err()}
    wsp = torch.empty(F.solve_workspace_size(B, U, k, F.FIO_SOLVE_PCG, F.FIO_PREC_FP64, 1e-12, 30),
                      dtype=torch.uint8, device=dev)
    ms, info = timed(dict(mode=F.FIO_SOLVE_PCG, prec=F.FIO_PREC_FP64, rel_res_tol=1e-12, max_ir=30, out=out, ws=wsp))
    res["pcg_fp64"] = {"value": k / (ms / 1e3), "ms_per_step": round(ms, 3), "iterations": int(info.ir_steps),
                       "rel_res": info.rel_res, "max_col_rel_err": err()}
    ms, _ = timed(dict(out=out))
    res["direct_fp64"] = {"value": k / (ms / 1e3), "ms_per_step": round(ms, 3), "max_col_rel_err": err()}
    res.update({"workload": "1D FIO N=2^%d, Gaussian-sum amplitude m=10 sigma^2=0.1, c(x)=(2+sin 2pi x)/8, q=9, "
                            "HSS tol 1e-3, p=10, %d RHS, refinement to rel residual %g" % (int(np.log2(n)), k,
                                                                               rel_res),
                "offline_s": {"bf": round(t_bf, 3), "hss": round(t_hss, 3), "ulv": round(t_ulv, 3)},
                "hss_max_rank_per_level": {str(l): int(max(v)) for l, v in ranks.items()}})
    del B, H, U
    return res


def workload_2e16(F, torch, fi, steps, warmup, n=1 << 16, k=16):
    """The N = 2^16 configuration: phase (2 + sin 2 pi x)/16 (and c = 0, the DFT), q = 9, HSS
    tolerance 1e-3 with p = 10 oversampling, 16 complex Gaussian right-hand sides (seed 1),
    u = K~ f; times the GPU build (BF, HSS, ULV) and the direct FP64 solve f^ = F K~^* u
    (RHS/s, per-column error against f)."""
    dev = torch.device("cuda")
    res = {"workload": "1D FIO N=2^16, q=9, HSS tol 1e-3, p=10, 16 RHS (seed 1), direct FP64 solve"}
    for label, (c0, c1) in (("c_sin16", (2.0 / 16, 1.0 / 16)), ("c_zero_dft", (0.0, 0.0))):
        t = time.perf_counter()
        B = F.BF(n, 9, c0, c1)
        torch.cuda.synchronize()
        t_bf = time.perf_counter() - t
        t = time.perf_counter()
        H = F.HSS.from_bf(B, tol=1e-3, p=10, seed=1001)
        torch.cuda.synchronize()
        t_hss = time.perf_counter() - t
        t = time.perf_counter()
        U = F.ULV(H)
        torch.cuda.synchronize()
        t_ulv = time.perf_counter() - t
        f_host = fi.rhs(1, n, k)
        u = B.apply(torch.from_numpy(np.ascontiguousarray(f_host.T)).to(dev).t())
        out = F.empty(n, k)
        ws = torch.empty(F.solve_workspace_size(B, U, k), dtype=torch.uint8, device=dev)
        for _ in range(warmup):
            F.approx_solve(B, U, u, out=out, ws=ws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            F.approx_solve(B, U, u, out=out, ws=ws)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        err = np.linalg.norm(out.cpu().numpy() - f_host, axis=0) / np.linalg.norm(f_host, axis=0)
        res[label] = {"direct_fp64_rhs_per_s": round(k / (ms / 1e3), 1), "ms_per_solve": round(ms, 4),
                      "max_col_rel_err": float(err.max()),
                      "offline_s": {"bf": round(t_bf, 3), "hss": round(t_hss, 3), "ulv": round(t_ulv, 3)},
                      "hss_max_rank": int(max(max(v) for v in H.ranks().values()))}
        del B, H, U
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=1 << 18)
    ap.add_argument("--nrhs", type=int, default=64)
    ap.add_argument("--q", type=int, default=9)
    ap.add_argument("--hss-tol", type=float, default=1e-3)
    ap.add_argument("--rel-res", type=float, default=5e-9)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--saturate-rate", type=float, default=1500.0,
                    help="offered request rate of the saturation runs (above the server's capacity)")
    ap.add_argument("--saturate-seconds", type=float, default=1.5)
    ap.add_argument("--serve-budget-gib", type=float, default=24.0,
                    help="device memory budget of the server's batch arenas")
    ap.add_argument("--no-cfg-2e16", action="store_true", help="skip the N=2^16, 16-RHS direct-solve workload")
    ap.add_argument("--no-2d", action="store_true", help="skip the 2D workload")
    ap.add_argument("--only-2d", action="store_true", help="run the 2D workload alone (for profiling)")
    ap.add_argument("--no-2d-solve", action="store_true", help="2D: time the applies only")
    ap.add_argument("--no-amp", action="store_true", help="skip the variable-amplitude workload")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"), default=None,
                    help="write profiles/traffic.json from two rocprofv3 counter runs of this benchmark and exit")
    ap.add_argument("--tune-file", default=None,
                    help="tile table of the headline operator: loaded when the file exists, else tuned and written")
    a = ap.parse_args()
    if a.traffic_from:
        traffic_from(*a.traffic_from, n=a.n, k=a.nrhs, q=a.q)
        return
    if a.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path; run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import fio_inputs as fi
    import paper_2609_11520_amd as F
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    F.lib()
    n, k, q = a.n, a.nrhs, a.q
    dev = torch.device("cuda")

    def sync():
        torch.cuda.synchronize()

    log("device", torch.cuda.get_device_name(0))
    copy_calibration(torch)
    if a.only_2d:
        w2d = workload_2d(F, torch, fi, a.steps, a.warmup, solve=not a.no_2d_solve)
        print(json.dumps({"workload_2d": w2d}), flush=True)
        return
    t = time.perf_counter()
    B = F.BF(n, q, 2.0 / 16, 1.0 / 16, precs=(F.FIO_PREC_FP64, F.FIO_PREC_FP32, F.FIO_PREC_SPLIT_FP16))
    sync()
    t_bf = time.perf_counter() - t
    t = time.perf_counter()
    H = F.HSS.from_bf(B, tol=a.hss_tol, p=10, seed=1003)
    sync()
    t_hss = time.perf_counter() - t
    ranks = H.ranks()
    t = time.perf_counter()
    U = F.ULV(H)
    sync()
    t_ulv = time.perf_counter() - t
    log("offline: BF %.2fs, HSS %.2fs, ULV %.2fs; max ranks per level %s" %
        (t_bf, t_hss, t_ulv, {l: int(max(v)) for l, v in ranks.items()}))
    # the same construction with Section 3.1's adaptive sample count (leaf rank guess 16, then the
    # largest rank of the level below); timed for the offline figures only
    t = time.perf_counter()
    Had = F.HSS.from_bf(B, tol=a.hss_tol, p=10, seed=1003, rhat=16, adaptive=True)
    sync()
    t_hss_ad = time.perf_counter() - t
    ranks_ad = {str(l): int(max(v)) for l, v in Had.ranks().items()}
    del Had

    f_host = fi.rhs(1, n, k)
    f = torch.from_numpy(np.ascontiguousarray(f_host.T)).to(dev).t()
    u = B.apply(f)
    # calibration block: other seeded columns (seed 2), never timed or checked
    fcal = torch.from_numpy(np.ascontiguousarray(fi.rhs(2, n, k).T)).to(dev).t()
    ucal = B.apply(fcal)
    del fcal
    sync()
    # tile autotuner: levels per fused pass, leaf fold and (split precision) engine for the
    # 64-column applies of each precision; --tune-file reuses a table written by an earlier run
    tuned = {}
    tune_source = "tuned in this run"
    if a.tune_file and os.path.exists(a.tune_file):
        with open(a.tune_file) as fh:
            B.tune_import(fh.read())
        tune_source = "loaded from " + a.tune_file
        for prec, pn in ((F.FIO_PREC_FP64, "fp64"), (F.FIO_PREC_FP32, "fp32"), (F.FIO_PREC_SPLIT_FP16, "split16")):
            tuned[pn] = [("%s " % d) + " ".join("%s=%d" % kv for kv in B.get_tile(k, prec=prec, adj=d == "adj").items())
                         for d in ("fwd", "adj")]
    else:
        for prec, pn in ((F.FIO_PREC_FP64, "fp64"), (F.FIO_PREC_FP32, "fp32"), (F.FIO_PREC_SPLIT_FP16, "split16")):
            tuned[pn] = chosen(B.autotune(u, prec=prec, reps=3))
        if a.tune_file:
            with open(a.tune_file, "w") as fh:
                fh.write(B.tune_export())
    log("autotuned tiles (%s)" % tune_source, json.dumps(tuned))
    # the split-precision K~^* apply with each engine pinned (matrix cores: split-FP16 passes;
    # vector units: FP32 structured passes), whatever the tuner chose, so that both engines are
    # measured on every run; the tuned configuration is restored afterwards
    split_engines = {}
    tuned_adj = B.get_tile(k, prec=F.FIO_PREC_SPLIT_FP16, adj=True)
    wsa = torch.empty(B.workspace_size(k, F.FIO_PREC_SPLIT_FP16), dtype=torch.uint8, device=dev)
    ya = F.empty(n, k)
    for eng, valu in (("mfma", 0), ("valu", 1)):
        cfg = dict(tuned_adj)
        cfg.update(kmax=3, valu=valu)
        B.set_tile(k, F.FIO_PREC_SPLIT_FP16, True, **cfg)
        for _ in range(2):
            B.apply_adj(u, prec=F.FIO_PREC_SPLIT_FP16, out=ya, ws=wsa)
        sync()
        F.timing_reset()
        F.timing_enable(True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            B.apply_adj(u, prec=F.FIO_PREC_SPLIT_FP16, out=ya, ws=wsa)
        e1.record()
        sync()
        F.timing_enable(False)
        rec = {"apply_ms": round(e0.elapsed_time(e1) / 10, 4)}
        pk = "bf_split16" if valu == 0 else "bf_struct_f32"
        cnt, ms = F.timing_query(pk)
        if cnt:
            rec["pass_kernel"] = pk
            rec["roofline"] = roofline_of(pk, n, q, k, ms / cnt, stored_traffic(pk))
        split_engines[eng] = rec
    B.set_tile(k, F.FIO_PREC_SPLIT_FP16, True, **tuned_adj)
    split_engines["tuned_adjoint_engine"] = "valu" if tuned_adj["valu"] else "mfma"
    del ya, wsa
    log("split-precision K~^* engines", json.dumps(split_engines))

    results = {}
    kernel_stats = {}
    checked = {}
    for name, prec in (("fp64", F.FIO_PREC_FP64), ("mixed", F.FIO_PREC_FP32),
                       ("split16", F.FIO_PREC_SPLIT_FP16)):
        out = F.empty(n, k)
        ws = torch.empty(F.solve_workspace_size(B, U, k, F.FIO_SOLVE_IR, prec, a.rel_res, 6), dtype=torch.uint8,
                         device=dev)
        # calibration on the held-out block: the residual-checked solve (one FP64 residual per step,
        # read back) fixes the number of refinement steps this operator needs
        kwc = dict(mode=F.FIO_SOLVE_IR, prec=prec, rel_res_tol=a.rel_res, max_ir=6, out=out, ws=ws)
        _, info = F.approx_solve(B, U, ucal, **kwc)
        nir = info.ir_steps
        # the residual-checked solve on the timed block, timed and reported too
        for _ in range(a.warmup):
            _, info = F.approx_solve(B, U, u, **kwc)
        sync()
        t0 = time.perf_counter()
        for _ in range(a.steps):
            _, info = F.approx_solve(B, U, u, **kwc)
        sync()
        ms_c = (time.perf_counter() - t0) * 1e3 / a.steps
        errc = np.linalg.norm(out.cpu().numpy() - f_host, axis=0) / np.linalg.norm(f_host, axis=0)
        checked[name] = {"value": k / (ms_c / 1e3), "ms_per_step": ms_c, "ir_steps": info.ir_steps,
                         "rel_res": info.rel_res, "max_col_rel_err": float(errc.max()),
                         "accuracy_ok": bool(errc.max() <= 1e-8)}
        # timed: the same refinement with the calibrated step count and no host synchronisation
        kw = dict(mode=F.FIO_SOLVE_IR, prec=prec, rel_res_tol=0.0, max_ir=nir, out=out, ws=ws)
        for _ in range(a.warmup):
            F.approx_solve(B, U, u, **kw)
        sync()
        F.timing_reset()
        F.timing_enable(True)
        lat = []
        steps_taken = []
        sync()
        t0 = time.perf_counter()
        for _ in range(a.steps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            _, info = F.approx_solve(B, U, u, **kw)
            e1.record()
            steps_taken.append(info.ir_steps)
            lat.append((e0, e1))
        sync()
        wall = time.perf_counter() - t0
        F.timing_enable(False)
        lat_ms = np.array([x.elapsed_time(y) for x, y in lat])
        for kn in F.timing_names():
            cnt, ms = F.timing_query(kn)
            kernel_stats.setdefault(name, {})[kn] = (cnt, ms)
        fh = out.detach().cpu().numpy()
        err = np.linalg.norm(fh - f_host, axis=0) / np.linalg.norm(f_host, axis=0)
        ms_step = wall * 1e3 / a.steps
        results[name] = {"value": k / (ms_step / 1e3), "ms_per_step": ms_step, "max_col_rel_err": float(err.max()),
                         "accuracy_ok": bool(err.max() <= 1e-8), "calibrated_on": "seed 2 (held out)",
                         "ir_steps": int(max(steps_taken)), "residual_checked": checked[name],
                         "latency_ms": {"p50": float(np.percentile(lat_ms, 50)), "p99": float(np.percentile(lat_ms, 99))}}
        # the same solve captured once into a hipGraph and replayed: the same kernels, without the
        # per-launch host overhead between them
        out.zero_()
        results[name]["graph"] = graph_replay(F, torch, lambda: F.approx_solve(B, U, u, **kw), out, f_host, k,
                                              a.steps, a.warmup)
        log(name, json.dumps(results[name]))

    # the headline launch mode: eager or graph replay, whichever is faster for the head variant
    out = F.empty(n, k)
    for _ in range(a.warmup):
        F.approx_solve(B, U, u, out=out)
    sync()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        F.approx_solve(B, U, u, out=out)
    sync()
    ms_direct = (time.perf_counter() - t0) * 1e3 / a.steps
    err_d = float((np.linalg.norm(out.cpu().numpy() - f_host, axis=0) / np.linalg.norm(f_host, axis=0)).max())
    # the same direct solve with K~^* in split FP16: its error is the HSS approximation's either way
    for _ in range(a.warmup):
        F.approx_solve(B, U, u, prec=F.FIO_PREC_SPLIT_FP16, out=out)
    sync()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        F.approx_solve(B, U, u, prec=F.FIO_PREC_SPLIT_FP16, out=out)
    sync()
    ms_direct16 = (time.perf_counter() - t0) * 1e3 / a.steps
    err_d16 = float((np.linalg.norm(out.cpu().numpy() - f_host, axis=0) / np.linalg.norm(f_host, axis=0)).max())

    # the paper's iterative solver (Sec. 4.1, Sec. 5): CG on the normal equation preconditioned by F,
    # to a relative residual of 1e-12; residual-checked, then with the iteration count fixed
    pcg = {}
    wsp = torch.empty(F.solve_workspace_size(B, U, k, F.FIO_SOLVE_PCG, F.FIO_PREC_FP64, 1e-12, 30),
                      dtype=torch.uint8, device=dev)
    for label, tol in (("residual_checked", 1e-12), ("fixed_iterations", 0.0)):
        kwp = dict(mode=F.FIO_SOLVE_PCG, prec=F.FIO_PREC_FP64, rel_res_tol=tol,
                   max_ir=30 if tol > 0 else pcg["residual_checked"]["iterations"], out=out, ws=wsp)
        for _ in range(a.warmup):
            _, info = F.approx_solve(B, U, u, **kwp)
        sync()
        t0 = time.perf_counter()
        for _ in range(a.steps):
            _, info = F.approx_solve(B, U, u, **kwp)
        sync()
        ms = (time.perf_counter() - t0) * 1e3 / a.steps
        e = float((np.linalg.norm(out.cpu().numpy() - f_host, axis=0) / np.linalg.norm(f_host, axis=0)).max())
        pcg[label] = {"value": k / (ms / 1e3), "ms_per_step": round(ms, 3), "iterations": int(info.ir_steps),
                      "rel_res": info.rel_res, "max_col_rel_err": e}
    # the fixed-iteration PCG (no host synchronisation) replayed from a captured hipGraph
    kwg = dict(mode=F.FIO_SOLVE_PCG, prec=F.FIO_PREC_FP64, rel_res_tol=0.0,
               max_ir=pcg["residual_checked"]["iterations"], out=out, ws=wsp)
    out.zero_()
    pcg["fixed_iterations"]["graph"] = graph_replay(F, torch, lambda: F.approx_solve(B, U, u, **kwg), out, f_host,
                                                    k, a.steps, a.warmup)
    log("pcg", json.dumps(pcg))

    for nm, r in results.items():
        r["graph"]["accuracy_ok"] = bool(r["graph"]["max_col_rel_err"] <= 1e-8)
    # the headline mixed path: the faster of the two low-precision variants among those whose every
    # column reached rel err 1e-8 (eager and replayed)
    ok = [v for v in ("split16", "mixed") if results[v]["accuracy_ok"] and results[v]["graph"]["accuracy_ok"]]
    cands = ok or ["split16", "mixed"]
    head = max(cands, key=lambda v: max(results[v]["value"], results[v]["graph"]["value"]))
    launch = "hipGraph replay" if results[head]["graph"]["value"] > results[head]["value"] else "eager"
    # roofline of the dominant kernel of the headline path (most time per step), and of the
    # kernel furthest below its bound
    ks = kernel_stats[head]
    dom = max(ks, key=lambda kn: ks[kn][1])
    roof = roofline_of(dom, n, q, k, ks[dom][1] / ks[dom][0], stored_traffic(dom))
    if roof:
        roof["launches"] = ks[dom][0]
    others = {}
    for kn, (cnt, tot) in ks.items():
        r = roofline_of(kn, n, q, k, tot / cnt, stored_traffic(kn))
        if r:
            r["launches"] = cnt
            others[kn] = r

    serve = None
    if not a.no_serve:
        del B, H, U
        torch.cuda.empty_cache()
        log("serving workload")
        sops = serving_operators(F, torch, fi)
        budget = int(a.serve_budget_gib * (1 << 30))
        serve = {"budget_gib": a.serve_budget_gib}
        for variant in ("split16", "fp64"):
            serve[variant] = serving(F, torch, fi, sops, variant, a.serve_seconds, a.serve_rate, mem_budget=budget)
            log("serving", variant, json.dumps(serve[variant]))
        for variant in ("split16", "fp64"):
            serve["saturated_" + variant] = serving(F, torch, fi, sops, variant, a.saturate_seconds,
                                                    a.saturate_rate, seed=5, mem_budget=budget)
            log("serving saturated", variant, json.dumps(serve["saturated_" + variant]))
        del sops
        torch.cuda.empty_cache()

    w16 = None
    if not a.no_cfg_2e16:
        torch.cuda.empty_cache()
        log("N=2^16 direct-solve workload")
        w16 = workload_2e16(F, torch, fi, a.steps, a.warmup)
        log("2e16", json.dumps(w16))

    w2d = None
    if not a.no_2d:
        torch.cuda.empty_cache()
        log("2D workload")
        w2d = workload_2d(F, torch, fi, a.steps, a.warmup, solve=not a.no_2d_solve)
        log("2d", json.dumps(w2d))
    w2a = None
    if not a.no_2d and not a.no_amp:
        torch.cuda.empty_cache()
        log("2D variable-amplitude workload")
        w2a = workload_2d(F, torch, fi, a.steps, a.warmup, solve=not a.no_2d_solve, var_amp=True)
        log("2d_var_amp", json.dumps(w2a))

    wamp = None
    if not a.no_amp:
        torch.cuda.empty_cache()
        log("variable-amplitude workload")
        wamp = workload_var_amp(F, torch, fi, a.steps, a.warmup)
        log("var_amp", json.dumps(wamp))
        if wamp["split16_ir"]["max_col_rel_err"] > 1e-8:
            log("ERROR: variable-amplitude refinement missed rel err 1e-8: %g" % wamp["split16_ir"]["max_col_rel_err"])

    cpu = None
    if not a.no_cpu_baseline:
        cpu = cpu_baseline(n, q, k, results["fp64"]["ir_steps"], ranks)

    mixed = dict(results[head])
    if launch != "eager":
        mixed.update({kk: results[head]["graph"][kk] for kk in ("value", "ms_per_step", "max_col_rel_err",
                                                                "latency_ms")})
    for nm, r in results.items():
        for lm, rr in (("eager", r), ("graph", r["graph"])):
            if rr["max_col_rel_err"] > 1e-8:
                log("ERROR: %s path (%s) missed rel err 1e-8: %g" % (nm, lm, rr["max_col_rel_err"]))
    accuracy_ok = bool(mixed["max_col_rel_err"] <= 1e-8 and head in ok)
    line = {
        "metric": METRIC, "value": round(mixed["value"], 2), "unit": "RHS/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": round(mixed["ms_per_step"], 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": ("fp16x2+fp32+fp64" if head == "split16" and split_engines["tuned_adjoint_engine"] == "mfma"
                  else "fp32+fp64"),
        "data": "synthetic",
        "config": {"workload": "1D FIO N=2^%d, c(x)=(2+sin 2pi x)/16, q=%d, HSS tol %g, p=10, %d RHS, "
                               "refinement steps calibrated to rel residual %g" % (int(np.log2(n)), q, a.hss_tol, k,
                                                                                    a.rel_res),
                   "n": n, "nrhs": k, "q": q, "hss_tol": a.hss_tol, "mixed_variant": head, "launch": launch,
                   "calibration": "refinement step count from the residual-checked solve of a held-out block "
                                  "(seed 2); the timed block (seed 1) is checked against its f",
                   "autotuned_tiles": tuned, "tune_source": tune_source,
                   "hss_max_rank_per_level": {str(l): int(max(v)) for l, v in ranks.items()}},
        "mixed": results["mixed"], "split16": results["split16"], "fp64": results["fp64"],
        "direct_fp64": {"ms_per_step": round(ms_direct, 3), "value": k / (ms_direct / 1e3),
                        "max_col_rel_err": err_d},
        "direct_split16": {"ms_per_step": round(ms_direct16, 3), "value": k / (ms_direct16 / 1e3),
                           "max_col_rel_err": err_d16},
        "pcg_fp64": pcg,
        "latency_ms": mixed["latency_ms"],
        "offline_s": {"bf": round(t_bf, 3), "hss": round(t_hss, 3), "ulv": round(t_ulv, 3),
                      "hss_adaptive_rhat16": round(t_hss_ad, 3), "hss_adaptive_max_rank_per_level": ranks_ad},
        "kernels_ms": {p: {kn: [c, round(m, 3)] for kn, (c, m) in d.items()} for p, d in kernel_stats.items()},
        "serving": serve, "workload_2d": w2d, "workload_var_amp": wamp, "workload_2d_var_amp": w2a,
        "workload_2e16": w16, "split_precision_engines": split_engines, "accuracy_ok": accuracy_ok,
        "roofline": roof, "roofline_by_kernel": others, "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    if not accuracy_ok:
        log("ERROR: the headline path missed rel err 1e-8 on some column")
        sys.exit(3)


if __name__ == "__main__":
    main()
