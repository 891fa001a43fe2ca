#!/usr/bin/env python3
"""Benchmark of the DtN build and apply on one MI355X.

Workload (default): 1024 x 1024 grid, Helmholtz d = -(40 pi)^2 (20 wavelengths
across the unit square), b = c = 0, leaf boxes of side 32, 1024 Dirichlet
vectors with U[-1, 1] entries (seed 3001).  One step = one build of the DtN
operator from device-resident coefficients plus one apply to the 1024
device-resident vectors.  The headline value is the build time in seconds
(median over the timed steps); the apply rate and latency are reported beside
it.

Also reported:
  roofline      - the dominant kernel of the timed steps (largest summed HIP-event
                  time), its algorithmic work per launch over its average launch
                  duration, against the MI355X peak of its bound;
  cpu_baseline  - the CPU oracle timed on this host on a bounded sample (one
                  level-1 quadrant of the same build), scaled to a full build by
                  the algorithmic flop model; the same leg measures the relative
                  error of the GPU operator against the oracle's closed form.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DtN build s @n=1024; apply solves/s + p99 latency vs plain FP64, rel err≤1e-6"
ROLES = ("gemm_inv", "gemm_x", "gemm_schur", "gemm_update", "gemm_comp")
# kernel instantiation -> (profiler families it runs, bound, MI355X peak of that bound)
KERNELS = {
    "k_gemm_batched<0,double>": (ROLES, "mfma", 78.6),
    "k_gemm_batched<3,double>": (tuple(r + "_t32" for r in ROLES), "mfma", 78.6),
    "k_gemm_batched<4,double>": (tuple(r + "_t32k64" for r in ROLES), "mfma", 78.6),
    "k_gemm_batched<1|2,double>": (tuple(r + "_t128" for r in ROLES), "mfma", 78.6),
    "k_gemm_batched<0,float>": (tuple(r + "_f32" for r in ROLES), "mfma", 157.3),
    "k_gemm_single<2>": (("apply_gemm",), "mfma", 78.6),
    "k_small_wave/k_small_fast": (("small_schur",), "latency", 78.6),
    # latency-bound (a chain of dependent pivot steps per block); work counted as the blocks'
    # LU factorisation, 2/3 bs^3 flops each, against the FP64 peak
    "k_base_inv2": (("base_inv",), "latency", 78.6),
    "k_couple": (("couple",), "hbm", 8000.0),
    "k_large_gather": (("large_gather",), "hbm", 8000.0),
    "k_apply_splitk+k_apply_reduce": (("apply_splitk",), "hbm", 8000.0),
    "k_scale_copy": (("scale_copy",), "hbm", 8000.0),
    "k_pchol": (("pchol",), "latency", 78.6),
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="cfg3")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--apply-reps", type=int, default=50)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-compression", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=10000)
    ap.add_argument("--serve-max-cols", type=int, default=256)
    return ap.parse_args()


def compression_leg(dtn, W, sptr):
    """n = 2048, leaf 32, convection-diffusion: dense FP64 build against the build with the top
    merges compressed at tol 1e-10 (default levels); error of the compressed operator against
    the dense one, ranks per level."""
    import numpy as np
    import torch
    P = W.config("cfg4", "convdiff")
    dev = torch.device("cuda:0")
    to_dev = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    b, c, d = to_dev(P.b), to_dev(P.c), to_dev(P.d)
    out = {"workload": P.name, "n": P.n, "leaf": P.leaf, "tol": P.tol}
    ops = {}
    for name, tol in (("dense", 0.0), ("compressed", P.tol)):
        dtn.build(P.n, b, c, d, leaf=P.leaf, tol=tol, stream=sptr).free()
        ts = []
        for q in range(3):
            t0 = time.perf_counter()
            op = dtn.build(P.n, b, c, d, leaf=P.leaf, tol=tol, stream=sptr)
            ts.append(time.perf_counter() - t0)
            if q < 2:
                op.free()
        ops[name] = op
        out[name + "_build_ms"] = round(statistics.median(ts) * 1e3, 3)
    st = ops["compressed"].stats()
    out["max_rank_per_level"] = st["max_rank"][: st["levels"] + 1]
    out["speedup"] = round(out["dense_build_ms"] / out["compressed_build_ms"], 3)
    Td, Tc = ops["dense"].dense(), ops["compressed"].dense()
    out["rel_err_vs_dense"] = float(np.linalg.norm(Tc - Td) / np.linalg.norm(Td))
    for op in ops.values():
        op.free()
    return out


def serving_leg(dtn, W, count, max_cols):
    """The serving workload: 8 resident operators, `count` apply requests (k ~ U{1..64}).
    Saturation = all requests offered at t = 0; then Poisson arrivals at 0.8 x saturation.
    Plain comparator: the same requests applied one by one (dtn_apply, no batching)."""
    import numpy as np
    import torch
    probs = W.serving_operators()
    specs = [dict(n=P.n, b=P.b, c=P.c, d=P.d, leaf=P.leaf) for P in probs]
    for o in dtn.build_many(specs):                      # warm the fused plan
        o.free()
    t0 = time.perf_counter()
    ops = dtn.build_many(specs)                          # all eight problems in one plan
    build_s = time.perf_counter() - t0
    for sp in specs:                                     # warm the eight single-problem plans
        dtn.build(**sp).free()
    t0 = time.perf_counter()
    for o in [dtn.build(**sp) for sp in specs]:          # one problem per build
        o.free()
    build_seq_s = time.perf_counter() - t0
    free, _ = torch.cuda.mem_get_info()
    budget = max(int(free) - (16 << 30), 1 << 30)
    srv = dtn.Server(budget_bytes=budget, max_batch_cols=max_cols)
    try:
        ids = [srv.add_op(op) for op in ops]
        gaps, which, ks = W.serving_requests(count)
        rng = np.random.default_rng(5102)
        pools = [np.asfortranarray(rng.uniform(-1, 1, (op.nb, 128))) for op in ops]
        outs = [np.zeros((op.nb, 128), order="F") for op in ops]
        offs = rng.integers(0, 65, count)
        reqs = [(int(which[q]), int(ks[q]), int(offs[q])) for q in range(count)]

        def schedule(times):
            return [(times[q], ids[o], pools[o][:, f:f + k], outs[o][:, f:f + k])
                    for q, (o, k, f) in enumerate(reqs[:len(times)])]

        def run(times):
            srv.reset_stats()
            tickets = srv.replay(schedule(times))
            for t in tickets:
                srv.wait(t)
            return srv.stats()

        run(np.zeros(min(count, 500)))                       # warm-up
        sat = run(np.zeros(count))
        sat_rate = sat["applies_done"] / sat["span_s"]
        lam = 0.8 * sat_rate
        st = run(np.cumsum(gaps) / lam)
        # plain FP64 comparator: one synchronous apply per request
        nplain = min(count, 2000)
        tp = time.perf_counter()
        solves = 0
        for o, k, f in reqs[:nplain]:
            ops[o].apply(pools[o][:, f:f + k])
            solves += k
        plain = solves / (time.perf_counter() - tp)
        return {
            "operators": [P.name for P in probs], "requests": count, "max_batch_cols": max_cols,
            "budget_gb": round(budget / 2**30, 1), "operator_build_fused_s": round(build_s, 4),
            "operator_build_one_by_one_s": round(build_seq_s, 4),
            "saturation_requests_per_s": round(sat_rate, 1), "saturation_solves_per_s": round(sat["solves_per_s"], 1),
            "lambda_requests_per_s": round(lam, 1), "solves_per_s": round(st["solves_per_s"], 1),
            "p50_ms": round(st["p50_ms"], 4), "p99_ms": round(st["p99_ms"], 4),
            "mean_batch_cols": round(st["mean_batch_cols"], 2), "batches": st["batches"],
            "plain_solves_per_s": round(plain, 1), "plain_sample_requests": nplain,
            "vs_plain": round(st["solves_per_s"] / plain, 3) if plain > 0 else None,
        }
    finally:
        srv.close()
        for op in ops:
            op.free()


def roofline_of(prof: dict) -> dict:
    """The dominant kernel (largest summed HIP-event time over the timed steps): algorithmic work
    per launch over its average launch duration, against the MI355X peak of its bound."""
    best = None
    for kern, (fams, bound, peak) in KERNELS.items():
        ents = [prof[f] for f in fams if f in prof]
        if not ents:
            continue
        ms = sum(e["total_ms"] for e in ents)
        if best is None or ms > best[1]:
            best = (kern, ms, ents, bound, peak)
    kern, ms, ents, bound, peak = best
    launches = sum(e["launches"] for e in ents)
    avg_ms = ms / max(launches, 1)
    if bound == "hbm":
        achieved = sum(e["bytes"] for e in ents) / launches / (avg_ms * 1e-3) / 1e9
        unit = "GB/s"
    else:
        achieved = sum(e["flops"] for e in ents) / launches / (avg_ms * 1e-3) / 1e12
        unit = "TFLOP/s"
    return {"kernel": kern, "bound": bound, "achieved": round(achieved, 3), "peak": peak, "unit": unit,
            "frac": round(achieved / peak, 4), "traffic": None, "launches": launches,
            "avg_launch_ms": round(avg_ms, 5),
            "algorithmic_bytes_per_launch": round(sum(e["bytes"] for e in ents) / launches, 1),
            "algorithmic_flops_per_launch": round(sum(e["flops"] for e in ents) / launches, 1)}


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in ("kernels.hip", "kernels.h", "common.h", "plan.cpp", "plan.h"):
        with open(os.path.join(ROOT, "paper_1302_5995_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def committed_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` from the committed counter summary (two rocprofv3 --pmc
    runs, FETCH_SIZE and WRITE_SIZE, each scaled by the copy kernel's reading), or None when the
    summary is missing, covers another kernel/workload, or the kernel sources changed since."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as fh:
            tr = json.load(fh)
    except (OSError, ValueError):
        return None, None
    ent = tr.get(workload, {}).get(kernel)
    if not ent or ent.get("source_hash") != kernel_source_hash():
        return None, None
    return ent["bytes_per_launch"], "profiles/traffic.json"


def closed_form_error(P, T_gpu):
    import numpy as np
    from oracle import dst_dtn
    Tref = dst_dtn(P.n, float(P.d[0]))
    return float(np.linalg.norm(T_gpu - Tref) / np.linalg.norm(Tref))


def cpu_baseline(P, T_gpu, level_flops):
    """Oracle on this host: one level-1 quadrant of the same build, scaled by the flop model."""
    import numpy as np
    from threadpoolctl import threadpool_info
    from oracle import assemble, dst_dtn
    from oracle.grid import build_tree
    from oracle.nd import box_schur
    pools = threadpool_info()
    threads = max([t.get("num_threads", 1) for t in pools] + [1])
    blas = sorted({f"{t.get('internal_api', '?')} {t.get('version', '')}".strip() for t in pools
                   if t.get("user_api") == "blas"})
    cpu = "?"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    cpu = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    M = assemble(P.n, P.b, P.c, P.d).tocsr()
    root = build_tree(P.n, P.leaf)
    quad = root.children[0]
    t0 = time.perf_counter()
    box_schur(M, P.n, quad)
    dt = time.perf_counter() - t0
    total = sum(level_flops)
    quad_share = sum(level_flops[1:]) / 4.0
    est = dt * total / quad_share
    out = {"value": round(est, 3), "unit": "s", "cores": threads, "kind": "oracle", "cpu": cpu,
           "blas": ", ".join(blas) or "?",
           "sample": f"oracle nested-dissection build of the SW level-1 quadrant ({quad.sx}x{quad.sy} nodes, "
                     f"{dt:.2f} s), scaled by the flop model share {quad_share / total:.4f} of the full build"}
    err = None
    if P.b is None and P.c is None and P.d is not None and np.all(P.d == P.d[0]):
        Tref = dst_dtn(P.n, float(P.d[0]))
        err = float(np.linalg.norm(T_gpu - Tref) / np.linalg.norm(Tref))
    return out, err


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the build runs on a single MI355X and --gpus {args.gpus} is not "
              f"supported (how the build would shard is described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import paper_1302_5995_amd as dtn
    import workloads as W

    P = W.config(args.workload)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    to_dev = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    b, c, d = to_dev(P.b), to_dev(P.c), to_dev(P.d)
    nb, k = P.nb, P.k
    G = torch.from_numpy(np.ascontiguousarray(P.G().T)).to(dev).t()      # column-major nb x k
    Y = torch.empty((k, nb), dtype=torch.float64, device=dev).t()
    # a dedicated stream (default priority): the library launches on it and the events below
    # bracket exactly the library's work (torch's default stream is the null stream)
    stream = torch.cuda.Stream(device=dev)
    torch.cuda.set_stream(stream)
    sptr = stream.cuda_stream

    def step():
        op = dtn.build(P.n, b, c, d, leaf=P.leaf, stream=sptr)
        op.apply_device(G, Y, stream=sptr)
        return op

    for _ in range(args.warmup):
        step().free()
    torch.cuda.synchronize()

    # one untimed step with every launch between HIP events: the per-family breakdown and the
    # dominant kernel; in the timed steps only that kernel's launches carry events (events around
    # all ~250 launches of a build would add ~2 ms to it)
    dtn.profile_reset()
    dtn.profile_select(None)
    dtn.profile_enable(True)
    step().free()
    torch.cuda.synchronize()
    dtn.profile_enable(False)
    prof_all = dtn.profile_read()
    dominant = roofline_of(prof_all)["kernel"]
    dtn.profile_reset()
    dtn.profile_select(list(KERNELS[dominant][0]))
    dtn.profile_enable(True)
    build_s, apply_ms = [], []
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    op = None
    for _ in range(args.steps):
        if op is not None:
            op.free()
        tb = time.perf_counter()
        op = dtn.build(P.n, b, c, d, leaf=P.leaf, stream=sptr)
        build_s.append(time.perf_counter() - tb)
        ev0.record(stream)
        op.apply_device(G, Y, stream=sptr)
        ev1.record(stream)
        ev1.synchronize()
        apply_ms.append(ev0.elapsed_time(ev1))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dtn.profile_enable(False)
    dtn.profile_select(None)
    T_after_build = op.dense() if os.environ.get("DTN_BENCH_DEBUG") else None
    prof = dtn.profile_read()
    stats = op.stats()

    # apply latency distribution (no profiling events): k = P.k and k = 1
    lat = {}
    for kk in (k, 1):
        Gk, Yk = G[:, :kk], Y[:, :kk]
        for _ in range(3):
            op.apply_device(Gk, Yk, stream=sptr)
        torch.cuda.synchronize()
        ts = []
        for _ in range(args.apply_reps):
            ev0.record(stream)
            op.apply_device(Gk, Yk, stream=sptr)
            ev1.record(stream)
            ev1.synchronize()
            ts.append(ev0.elapsed_time(ev1))
        ts.sort()
        lat[kk] = {"p50_ms": ts[len(ts) // 2], "p99_ms": ts[min(len(ts) - 1, int(math.ceil(0.99 * len(ts))) - 1)],
                   "solves_per_s": kk / (ts[len(ts) // 2] * 1e-3)}

    # plain copy kernel of known size (256 MiB read + 256 MiB written): the reference point that
    # scales the FETCH_SIZE / WRITE_SIZE counters of a --pmc run of this same command
    src = torch.ones(32 << 20, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    del src, dst

    roof = roofline_of(prof)
    roof["launches_per_step"] = roof.pop("launches") / args.steps
    roof["traffic"], roof["traffic_source"] = committed_traffic(roof["kernel"], P.name)
    value = statistics.median(build_s)
    result = {
        "metric": METRIC,
        "value": round(value, 6),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round((t1 - t0) / args.steps * 1e3, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": P.name, "n": P.n, "leaf": P.leaf, "k": k, "nb": nb,
                   "precision": "fp64", "batching": "fused"},
        "build_ms": {"median": round(value * 1e3, 3), "min": round(min(build_s) * 1e3, 3)},
        "build_model_tflops": round(stats["flops"] / value / 1e12, 3),
        "apply": {"k": k, "solves_per_s": round(lat[k]["solves_per_s"], 1), "p50_ms": round(lat[k]["p50_ms"], 4),
                  "p99_ms": round(lat[k]["p99_ms"], 4), "k1_p50_ms": round(lat[1]["p50_ms"], 4),
                  "k1_p99_ms": round(lat[1]["p99_ms"], 4)},
        "roofline": roof,
        # every family, from the untimed fully profiled step
        "kernels": {f: {"launches_per_step": v["launches"], "ms_per_step": round(v["total_ms"], 4)}
                    for f, v in sorted(prof_all.items())},
    }
    # mixed precision (FP32-MFMA products below the top two levels): time and error.  A mixed
    # request on a problem with d < 0 runs FP64 (reported); the n = 1024 Laplace operator shows the
    # FP32 products themselves
    T_mixed = None
    laplace_T = None
    if not args.no_mixed:
        def timed(bb, cc, dd, prec, reps=3):
            for _ in range(2):
                dtn.build(P.n, bb, cc, dd, leaf=P.leaf, stream=sptr, precision=prec).free()
            ts = []
            for q in range(reps):
                tb = time.perf_counter()
                o = dtn.build(P.n, bb, cc, dd, leaf=P.leaf, stream=sptr, precision=prec)
                ts.append(time.perf_counter() - tb)
                if q < reps - 1:
                    o.free()
            return statistics.median(ts), o
        ms, opm = timed(b, c, d, dtn.MIXED)
        ran = opm.stats()["precision"]
        result["mixed"] = {"build_ms": round(ms * 1e3, 3), "speedup_vs_fp64": round(value / ms, 3),
                           "precision_used": "mixed" if ran == dtn.MIXED else "fp64"}
        T_mixed = opm.dense()
        opm.free()
        if P.n == 1024:
            l64, o64 = timed(None, None, None, dtn.FP64)
            lmx, omx = timed(None, None, None, dtn.MIXED)
            result["mixed_laplace_n1024"] = {
                "fp64_build_ms": round(l64 * 1e3, 3), "mixed_build_ms": round(lmx * 1e3, 3),
                "speedup": round(l64 / lmx, 3),
                "precision_used": "mixed" if omx.stats()["precision"] == dtn.MIXED else "fp64"}
            laplace_T = (o64.dense(), omx.dense())       # errors in the oracle leg below
            o64.free()
            omx.free()
    if not args.no_plain:
        # comparator: the same FP64 kernels with one box, merge or product per launch
        plain_s = []
        for _ in range(2):
            tb = time.perf_counter()
            opp = dtn.build(P.n, b, c, d, leaf=P.leaf, stream=sptr, batching=dtn.PLAIN)
            plain_s.append(time.perf_counter() - tb)
            opp.free()
        result["plain_build_ms"] = round(plain_s[-1] * 1e3, 3)
        result["vs_plain_build"] = round(plain_s[-1] / value, 3)
    if not args.no_compression:
        result["compression"] = compression_leg(dtn, W, sptr)
    if not args.no_serving:
        result["serving"] = serving_leg(dtn, W, args.serve_requests, args.serve_max_cols)
    if not args.no_cpu_baseline:
        torch.cuda.synchronize()
        T = op.dense()
        if T_after_build is not None:
            print("debug: T changed by applies:", float(np.abs(T - T_after_build).max()), file=sys.stderr)
        cb, err = cpu_baseline(P, T, stats["level_flops"])
        result["cpu_baseline"] = cb
        result["rel_err_vs_oracle"] = err
        if err is not None and T_mixed is not None:
            result["mixed"]["rel_err_vs_oracle"] = closed_form_error(P, T_mixed)
        if laplace_T is not None:
            from oracle import dst_dtn
            Tl = dst_dtn(P.n, 0.0)
            for key, Tx in zip(("fp64_rel_err_vs_closed_form", "rel_err_vs_closed_form"), laplace_T):
                result["mixed_laplace_n1024"][key] = float(np.linalg.norm(Tx - Tl) / np.linalg.norm(Tl))
    else:
        result["cpu_baseline"] = None
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
