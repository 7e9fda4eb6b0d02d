"""Benchmark of the R-STHOSVD hot path on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--precision f32]

A step is one whole decomposition (every mode: sketch, power step, QR,
projection + Gram, FP64 symmetric EVD, factor, truncation) of a tensor
already resident in HBM.  Prints one JSON line with the tensor throughput
(GB/s of input per second), the roofline of the dominant kernel measured live
with HIP events, the whole path's fraction of its HBM roofline, and the FP64
oracle timed on the host over a bounded sample; beside them the batched
(512 small tensors) and served (Poisson arrivals) workloads.
"""
import argparse
import ctypes
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0          # MI355X HBM3E, GB/s
PEAKS_TFLOPS = {"f32": 157.3, "f64": 78.6, "bf16": 2500.0}
# HBM bytes of the dominant kernel from two rocprofv3 counter runs (FETCH_SIZE,
# WRITE_SIZE), calibrated on a plain copy of known size; valid only while the
# kernel's source is the one the counters were taken on
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pmc_traffic.json")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def algorithmic_counts(dims, ranks, p, q, elem, order=None):
    """Per-mode algorithmic bytes / flops of the minimal pass structure:
    (2 + q) reads of the current tensor, B written and read once, the
    truncated tensor written once."""
    d = list(dims)
    order = list(range(len(dims))) if order is None else list(order)
    modes = []
    for n in order:
        M = int(np.prod(d))
        I = d[n]
        J = M // I
        K = min(ranks[n] + p, I, J)
        R = ranks[n]
        byts = elem * ((2 + q) * M + 2 * K * J + R * J)
        flops = (4 + 4 * q) * K * M + 2 * K * K * J + 2 * R * K * J
        modes.append(dict(mode=n, M=M, I=I, J=J, K=K, R=R, bytes=byts, flops=flops,
                          power_bytes=elem * M, power_flops=4 * K * M,
                          sketch_bytes=elem * M, sketch_flops=2 * K * M))
        d[n] = R
    return modes


GOLDEN = {"r_sthosvd_200x4_r25": os.path.join(ROOT, "tests", "golden", "r_sthosvd_200x4_r25_oracle.npz")}


def oracle_rel_error(workload):
    """E of the FP64 oracle on the full workload, from the stored oracle run
    (tests/golden), or None when there is none for this workload."""
    path = GOLDEN.get(workload)
    if not path or not os.path.exists(path):
        return None
    return float(np.load(path, allow_pickle=False)["rel_error"])


def bench_batched(dev, steps, prec, seed=1, count=512):
    """512 order-3 FP32 tensors (extents 32..256, exact ranks 4..32, noise
    1e-4; R-STHOSVD at the true ranks, p = 5, q = 1) on the given precision
    path: one graph launch per batch, against the same tensors decomposed by
    512 sequential calls."""
    import torch
    from paper_2001_07124_amd import api
    from paper_2001_07124_amd.inputs import batch_specs, batch_tensors
    specs = batch_specs(count=count, seed=seed)
    t0 = time.perf_counter()
    xs = batch_tensors(specs, seed=seed, noise=1e-4, dtype=np.float32)
    xds = [api.to_device(x, dev) for x in xs]
    torch.cuda.synchronize()
    nbytes = float(sum(x.nbytes for x in xs))
    log(f"[bench] batch: {count} tensors, {nbytes / 1e9:.2f} GB, generated in {time.perf_counter() - t0:.1f}s")
    items = [(xd, r, 5, 1, i, prec) for i, (xd, (d, r)) in enumerate(zip(xds, specs))]
    s = torch.cuda.Stream(dev)
    t0 = time.perf_counter()
    b = api.Batch(items, autotune=True, stream=s)
    t_plan = time.perf_counter() - t0
    with torch.cuda.stream(s):
        b.run(stream=s)                      # captures the graph
        b.run(stream=s)
    s.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(s):
        e0.record(s)
        for _ in range(steps):
            b.run(stream=s)
        e1.record(s)
    s.synchronize()
    ms = e0.elapsed_time(e1) / steps
    errs = [r.rel_error for r in b.results]
    # the same work as independent single decompositions, one after another
    decs = [api.Decomposer(d, r, p=5, q=1, seed=i, dtype=torch.float32, precision=prec, device=dev)
            for i, (d, r) in enumerate(specs)]
    for dec, xd in zip(decs, xds):
        dec.run(xd, stream=s)
    s.synchronize()
    e0.record(s)
    for dec, xd in zip(decs, xds):
        dec.run(xd, stream=s)
    e1.record(s)
    s.synchronize()
    ms_seq = e0.elapsed_time(e1)
    log(f"[bench] batch ({prec}): {ms:.3f} ms per batch ({b.launches} launches, one graph), "
        f"sequential {ms_seq:.3f} ms")
    # the same per-item algorithmic bytes as the headline's path roofline
    alg = sum(sum(m["bytes"] for m in algorithmic_counts(d, r, 5, 1, 4)) for d, r in specs)
    out = {"workload": f"batch_{count}_order3_32to256_r4to32", "precision": prec, "tensors": count,
           "tensor_GB": round(nbytes / 1e9, 3), "ms_per_batch": round(ms, 3),
           "value": round(nbytes / (ms * 1e-3) / 1e9, 2), "unit": "GB/s",
           "launches_per_batch": b.launches, "graph": True,
           "sequential_ms": round(ms_seq, 3), "speedup_vs_sequential": round(ms_seq / ms, 2),
           "algorithmic_bytes": alg, "hbm_roofline_ms": round(alg / (HBM_PEAK_GBPS * 1e9) * 1e3, 4),
           "hbm_roofline_frac": round(alg / (HBM_PEAK_GBPS * 1e9) * 1e3 / ms, 4),
           "rel_error_median": float(np.median(errs)), "rel_error_max": float(np.max(errs)),
           "plan_and_tune_s": round(t_plan, 2)}
    b.close()
    return out


# The streaming kernels keep a mode's I x K accumulators in registers: modes
# of up to 256 rows take K <= 64, up to 512 rows K <= 32.  The serving mix is
# drawn within those limits (extents up to 512 instead of 1024).
MAX_SERVE_EXTENT = 512


def serve_rank_cap(extent, p=10):
    return (64 if extent <= 256 else 32) - p


def serve_requests(count, seed=3, pool_tensors=24):
    """Request mix of the serving workload: order 3 or 4, total size
    log-uniform in [64^3, 1024 x 1024 x 256], extents around size^(1/N) with
    a seeded jitter, clamped to [16, 512]; ranks uniform in 8..64 capped at
    the extent and at 54 (so that K = R + 10 stays within the 64-column
    limit, and by serve_rank_cap for taller modes); p = 10, q in {0, 1},
    FP32 or BF16 path.  The tensors themselves
    come from a pool of `pool_tensors` shapes drawn the same way."""
    rng = np.random.default_rng([seed, 3])
    shapes = []
    for _ in range(pool_tensors):
        N = int(rng.integers(3, 5))
        size = float(np.exp(rng.uniform(np.log(64.0 ** 3), np.log(1024.0 * 1024 * 256))))
        base = size ** (1.0 / N)
        dims = [int(np.clip(round(base * np.exp(rng.uniform(-0.3, 0.3))), 16, MAX_SERVE_EXTENT))
                for _ in range(N)]
        shapes.append(tuple(dims))
    reqs = []
    for i in range(count):
        k = int(rng.integers(0, pool_tensors))
        dims = shapes[k]
        ranks = tuple(int(min(rng.integers(8, 65), d, serve_rank_cap(d))) for d in dims)
        reqs.append(dict(tensor=k, ranks=ranks, q=int(rng.integers(0, 2)),
                         prec=("bf16" if rng.integers(0, 2) else "f32"), seed=i,
                         gap=float(rng.exponential(1.0))))
    return shapes, reqs


def bench_serving(dev, rate=200.0, duration_s=2.0, slots=8, pool_gb=24.0):
    """Poisson arrivals at `rate` requests/s for `duration_s`, every request a
    decomposition of a tensor already in HBM; p50/p99 latency (completion -
    arrival) and completed requests/s; then the same requests all at once
    (saturation throughput)."""
    import torch
    from paper_2001_07124_amd import api
    from paper_2001_07124_amd.inputs import tucker_tensor
    count = int(rate * duration_s)
    shapes, reqs = serve_requests(count)
    t0 = time.perf_counter()
    xds = []
    for k, dims in enumerate(shapes):
        r0 = tuple(min(16, d) for d in dims)
        xds.append(api.to_device(tucker_tensor(dims, r0, seed=500 + k, noise=1e-3,
                                               dtype=np.float32)[0], dev))
    torch.cuda.synchronize()
    log(f"[bench] serving: {len(shapes)} tensors ({sum(x.numel() for x in xds) * 4 / 1e9:.2f} GB) "
        f"in {time.perf_counter() - t0:.1f}s, {count} requests at {rate:.0f}/s")
    srv = api.Server(pool_bytes=int(pool_gb * (1 << 30)), slots=slots, device=dev)

    def run(gap_scale):
        tickets = []
        t_start = time.perf_counter()
        t_next = t_start
        for r in reqs:
            t_next += r["gap"] * gap_scale
            while time.perf_counter() < t_next:
                pass
            tickets.append(srv.submit(xds[r["tensor"]], r["ranks"], p=10, q=r["q"], seed=r["seed"],
                                      precision=r["prec"])[0])
        srv.drain()
        wall = time.perf_counter() - t_start
        lat = []
        for t in tickets:
            st, (ts, tb, te) = srv.poll(t)
            lat.append(te - ts)
            srv.release(t)
        return np.array(lat), wall

    run(0.0)                                   # warm-up: every shape once
    lat, wall = run(1.0 / rate)
    lat_sat, wall_sat = run(0.0)
    srv.close()
    log(f"[bench] serving: p50 {np.percentile(lat, 50):.2f} ms, p99 {np.percentile(lat, 99):.2f} ms, "
        f"{count / wall:.1f} req/s; saturation {count / wall_sat:.1f} req/s")
    return {"workload": "serve_order3_4_64cubed_to_1024x1024x256", "rate_req_s": rate,
            "requests": count, "slots": slots,
            "p50_ms": round(float(np.percentile(lat, 50)), 3),
            "p99_ms": round(float(np.percentile(lat, 99)), 3),
            "req_per_s": round(count / wall, 1),
            "saturation_req_per_s": round(count / wall_sat, 1),
            "saturation_p50_ms": round(float(np.percentile(lat_sat, 50)), 3)}


def cpu_baseline(x, w):
    """Time the FP64 oracle on a bounded sample: the leading slabs of the
    last mode, same ranks / p / q / seed."""
    from oracle.tucker import r_sthosvd as oracle_r_sthosvd
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:  # pragma: no cover
        threads = os.cpu_count() or 1
    dims = x.shape
    slab = int(np.prod(dims[:-1]))
    # the smallest valid sample: R_N + 1 leading slabs of the last mode
    s = min(int(w["target"][-1]) + 1, dims[-1])
    sub = x[..., :s].astype(np.float64)
    t0 = time.perf_counter()
    oracle_r_sthosvd(sub, w["target"], w["p"], w["q"], w["seed"])
    t = time.perf_counter() - t0
    nbytes = slab * s * x.dtype.itemsize
    return {"value": nbytes / t / 1e9, "unit": "GB/s", "cores": int(threads), "kind": "oracle",
            "sample": f"R-STHOSVD of the leading {s} of {dims[-1]} last-mode slabs "
                      f"({'x'.join(str(v) for v in dims[:-1])}x{s}, {nbytes / 1e9:.2f} GB as "
                      f"{x.dtype.name}), oracle incl. its explicit-residual E, {t:.1f} s, "
                      f"host cpu_count={os.cpu_count()}"}


def measured_traffic(kernel, workload, prec):
    """HBM bytes per launch of `kernel` from the committed counter runs, or
    None when there are none for this kernel/workload/precision or the
    kernel's source changed since they were taken."""
    import hashlib
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
        with open(os.path.join(ROOT, t["source"]), "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
    except (OSError, ValueError, KeyError):
        return None
    if (sha != t.get("source_sha256") or t.get("kernel") != kernel
            or t.get("workload") != workload or t.get("precision") != prec):
        return None
    return int(t["traffic_bytes_per_launch"])


def copy_probe(dev, nbytes=1 << 30):
    """A plain device copy of known size, for calibrating the HBM counters."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device=dev).fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    log(f"[bench] copy probe: {nbytes} bytes copied")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="r_sthosvd_200x4_r25")
    ap.add_argument("--precision", default=None,
                    help="bf16 (default for FP32 tensors: bf16 sketch/projection, split-bf16 power step) or f32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel-reps", type=int, default=5)
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the FP32 comparison path")
    ap.add_argument("--no-batch", action="store_true", help="skip the 512-tensor batched line")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving measurement")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also copy 1 GiB device to device (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on exactly one GPU; --gpus must be 1"}))
        sys.exit(2)

    import torch
    from paper_2001_07124_amd import api
    from paper_2001_07124_amd.inputs import WORKLOADS, tucker_tensor

    w = dict(WORKLOADS[args.workload])
    prec = args.precision or ("bf16" if w["dtype"] == np.float32 else w["prec"])
    dims, ranks = w["dims"], w["target"]
    log(f"[bench] generating {args.workload} dims={dims}")
    t0 = time.perf_counter()
    x, core, _ = tucker_tensor(dims, w["ranks"], seed=w["data_seed"], factors=w["factors"],
                               decay=w["decay"], noise=w["noise"], dtype=w["dtype"])
    log(f"[bench] generated in {time.perf_counter() - t0:.1f}s; uploading")
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    xd = api.to_device(x, dev)
    torch.cuda.synchronize()
    tt = torch.float64 if w["dtype"] == np.float64 else torch.float32
    stream = torch.cuda.current_stream(dev)

    def time_path(p_name, steps, warmup):
        dec = api.Decomposer(dims, ranks, algo=w["algo"], p=w["p"], q=w["q"], seed=w["seed"],
                             dtype=tt, precision=p_name, device=dev)
        for _ in range(warmup):
            dec.run(xd)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t_w = time.perf_counter()
        ev0.record(stream)
        for _ in range(steps):
            dec.run(xd)
        ev1.record(stream)
        torch.cuda.synchronize()
        t_w = time.perf_counter() - t_w
        res = dec.result()
        return ev0.elapsed_time(ev1) / steps, res.rel_error, dec.ws_bytes, t_w

    log(f"[bench] {prec} path: warmup {args.warmup}, timing {args.steps} steps")
    ms, e_gpu, ws_bytes, t_wall = time_path(prec, args.steps, args.warmup)
    log(f"[bench] {prec}: {ms:.3f} ms/step, E={e_gpu:.6f}")
    compare = None
    if prec != w["prec"] and not args.no_compare:
        ms_ref, e_ref, _, _ = time_path(w["prec"], max(2, args.steps // 2), 1)
        log(f"[bench] {w['prec']}: {ms_ref:.3f} ms/step, E={e_ref:.6f}")
        compare = {"precision": w["prec"], "ms_per_step": round(ms_ref, 4),
                   "value": round(float(np.prod(dims)) * np.dtype(w["dtype"]).itemsize / (ms_ref * 1e-3) / 1e9, 2),
                   "rel_error": e_ref, "abs_rel_error_diff_vs_headline": abs(e_ref - e_gpu)}
    elem = np.dtype(w["dtype"]).itemsize
    tensor_bytes = float(np.prod(dims)) * elem
    value = tensor_bytes / (ms * 1e-3) / 1e9
    modes = algorithmic_counts(dims, ranks, w["p"], w["q"], elem)
    alg_bytes = sum(m["bytes"] for m in modes)
    alg_flops = sum(m["flops"] for m in modes)
    path_roof_ms = alg_bytes / (HBM_PEAK_GBPS * 1e9) * 1e3

    # mode-1 streaming kernels, each timed live with HIP events on the stream
    # it is launched on, through its step-level entry point (kernel plus a
    # small fixed-order reduction of the per-workgroup partials)
    m0 = modes[0]
    view = (1, dims[0], int(np.prod(dims[1:])))
    flat = xd.as_strided((xd.numel(),), (1,))
    qmat = torch.linalg.qr(torch.randn(dims[0], m0["K"], dtype=torch.float64))[0].to(dev, tt)
    kernels = {
        "sketch": (lambda: api.sketch(flat, view, m0["K"], 0, 0, 2, precision=prec),
                   m0["sketch_bytes"], m0["sketch_flops"]),
        "project": (lambda: api.ttm(flat, view, m0["K"], qmat, want_gram=True, precision=prec),
                    m0["sketch_bytes"] + elem * m0["K"] * m0["J"], 2 * m0["K"] * m0["M"]),
    }
    if w["q"] > 0:
        kernels["power"] = (lambda: api.power(flat, view, qmat, precision=prec),
                            m0["power_bytes"], m0["power_flops"])
    ktimes = {}
    for name, (fn, kb, kf) in kernels.items():
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.kernel_reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        kms = e0.elapsed_time(e1) / args.kernel_reps
        ktimes[name] = {"ms": round(kms, 4), "GBps": round(kb / (kms * 1e-3) / 1e9, 1),
                        "TFLOPs": round(kf / (kms * 1e-3) / 1e12, 2), "bytes": kb, "flops": kf}
    dom = max(ktimes, key=lambda k: ktimes[k]["ms"])
    kd = ktimes[dom]
    peak_tf = PEAKS_TFLOPS["f64" if elem == 8 else ("bf16" if prec == "bf16" else "f32")]
    mfma_frac = kd["TFLOPs"] / peak_tf
    hbm_frac = kd["GBps"] / HBM_PEAK_GBPS
    if mfma_frac > hbm_frac:
        roofline = {"bound": "mfma", "achieved": kd["TFLOPs"], "peak": peak_tf, "unit": "TFLOP/s",
                    "frac": round(mfma_frac, 4), "traffic": None}
    else:
        roofline = {"bound": "hbm", "achieved": kd["GBps"], "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                    "frac": round(hbm_frac, 4), "traffic": None}
    roofline["traffic"] = measured_traffic(dom, args.workload, prec)
    roofline.update({"kernel": f"mode-1 {dom} pass ({prec})", "kernel_ms": kd["ms"],
                     "algorithmic_bytes": kd["bytes"], "algorithmic_flops": kd["flops"],
                     "mode1_kernels": ktimes})

    out = {
        "metric": "R-STHOSVD tensor GB/s (% HBM roofline) at 1e-3 rel err",
        "value": round(value, 2), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": prec, "data": "synthetic",
        "config": {"workload": args.workload, "dims": list(dims), "ranks": list(ranks),
                   "p": w["p"], "q": w["q"], "precision": prec, "algo": w["algo"]},
        "rel_error": e_gpu,
        "rel_error_oracle": oracle_rel_error(args.workload),
        "path": {"algorithmic_bytes": alg_bytes, "algorithmic_flops": alg_flops,
                 "algorithmic_GBps": round(alg_bytes / (ms * 1e-3) / 1e9, 1),
                 "hbm_roofline_ms": round(path_roof_ms, 4),
                 "hbm_roofline_frac": round(path_roof_ms / ms, 4),
                 "workspace_bytes": ws_bytes},
        "roofline": roofline,
        "compare_path": compare,
        "wall_s_timed": round(t_wall, 3),
    }
    if not args.no_batch:
        log("[bench] batched workload")
        out["batched"] = bench_batched(dev, max(3, args.steps // 2), prec if elem == 4 else "f32")
    if not args.no_serve:
        log("[bench] serving workload")
        out["serving"] = bench_serving(dev)
    if args.copy_probe:
        copy_probe(dev)
    if not args.no_cpu_baseline:
        log("[bench] timing the oracle on a bounded host sample")
        out["cpu_baseline"] = cpu_baseline(x, w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
