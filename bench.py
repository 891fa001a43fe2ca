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
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--no-suite", action="store_true")
    ap.add_argument("--no-structured", action="store_true")
    ap.add_argument("--no-cold", action="store_true")
    ap.add_argument("--no-body", action="store_true")
    ap.add_argument("--suite-n", type=int, default=1024)
    ap.add_argument("--e12-n", type=int, default=512)
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


def structured_leg(dtn, P, b, c, d, sptr, T_dense, dense_ms, kii_tol=1e-12):
    """The bench workload built with the structured merges of Section 6, Step 1 (K_ii of the merges
    whose children's rings reach 1000 inverted in HBS form by Algorithm 1 at local tolerance kii_tol,
    X by Algorithm 2): build time against the dense build, merges taken, error against the dense T.
    The Helmholtz interface blocks are indefinite and amplify the local tolerance about a thousandfold,
    hence 1e-12."""
    import numpy as np
    dtn.build(P.n, b, c, d, leaf=P.leaf, stream=sptr, kii_tol=kii_tol).free()
    ts = []
    for q in range(3):
        t0 = time.perf_counter()
        op = dtn.build(P.n, b, c, d, leaf=P.leaf, stream=sptr, kii_tol=kii_tol)
        ts.append(time.perf_counter() - t0)
        if q < 2:
            op.free()
    st = op.stats()
    T = op.dense()
    op.free()
    ms = statistics.median(ts) * 1e3
    return {"kii_tol": kii_tol, "structured_merges": st["structured_merges"], "build_ms": round(ms, 3),
            "dense_build_ms": round(dense_ms, 3), "speedup": round(dense_ms / ms, 3),
            "rel_err_vs_dense": float(np.linalg.norm(T - T_dense) / np.linalg.norm(T_dense))}


def body_leg(dtn, W, sptr, sizes=(512, 1024), counts=(10, 100, 1000)):
    """Section 7.3's experiment (Table 5): the random Laplacian I problem with N_body loads at random nodes
    of a localized square; build time of T and F together against T alone, the apply of both, and at
    n = 512 the error of F against the oracle's sparse-solve definition (ten loads, every column)."""
    import numpy as np
    import torch
    dev = torch.device("cuda:0")
    rows = []
    F512, nodes512 = None, None
    for n in sizes:
        P = W.paper_problem("randlap1", n)
        to_dev = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(dev)
        b, c, d = to_dev(P.b), to_dev(P.c), to_dev(P.d)
        kw = dict(leaf=32, coef_form=dtn.COEF_NETWORK, stream=sptr)
        dtn.build(n, b, c, d, **kw).free()
        ts = []
        for _ in range(3):
            t0 = time.perf_counter()
            dtn.build(n, b, c, d, **kw).free()
            ts.append(time.perf_counter() - t0)
        base_ms = statistics.median(ts) * 1e3
        rng = np.random.default_rng(7000 + n)
        lo, hi = 3 * n // 8, 5 * n // 8
        for cnt in counts:
            pts = set()
            while len(pts) < cnt:
                pts.add((int(rng.integers(lo, hi)), int(rng.integers(lo, hi))))
            nodes = sorted(pts)
            dtn.build(n, b, c, d, body_nodes=nodes, **kw).free()
            ts = []
            for q in range(3):
                t0 = time.perf_counter()
                op = dtn.build(n, b, c, d, body_nodes=nodes, **kw)
                ts.append(time.perf_counter() - t0)
                if q < 2:
                    op.free()
            G = torch.rand((1, op.nb), dtype=torch.float64, device=dev).t()
            Q = torch.rand((1, cnt), dtype=torch.float64, device=dev).t()
            for _ in range(3):
                op.apply_body_device(G, Q, stream=sptr)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(20):
                op.apply_body_device(G, Q, stream=sptr)
            torch.cuda.synchronize()
            solve_ms = (time.perf_counter() - t0) / 20 * 1e3
            if n == 512 and cnt == counts[0]:
                F512, nodes512 = op.body(), nodes
            op.free()
            rows.append({"n": n, "n_body": cnt, "build_ms": round(statistics.median(ts) * 1e3, 3),
                         "build_without_loads_ms": round(base_ms, 3), "solve_k1_ms": round(solve_ms, 4)})
    return rows, (F512, nodes512)


def cold_build(cfg):
    """First build of the workload in a fresh process (HIP module load, device set-up, plan creation and
    upload, then the build), against the later builds of the timed loop; measured in a child process."""
    import subprocess
    code = ("import sys, time; sys.path.insert(0, %r); import numpy as np; import workloads as W; "
            "import paper_1302_5995_amd as dtn; P = W.config(%r); t0 = time.perf_counter(); "
            "op = dtn.build(P.n, P.b, P.c, P.d, leaf=P.leaf); t1 = time.perf_counter(); "
            "op2 = dtn.build(P.n, P.b, P.c, P.d, leaf=P.leaf); t2 = time.perf_counter(); "
            "print('%%.3f %%.3f' %% ((t1 - t0) * 1e3, (t2 - t1) * 1e3))") % (ROOT, cfg)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    if r.returncode != 0:
        return {"error": r.stderr.strip().splitlines()[-1] if r.stderr.strip() else "failed"}
    first, second = (float(x) for x in r.stdout.split())
    return {"first_build_ms": first, "second_build_ms": second}


def paper_suite_leg(dtn, W, n, sptr):
    """The eleven problems of the paper's Section 7.1 at n x n (leaf 32): build time (median of 3), the
    operator's HBS form at the paper's local tolerance 1e-7 (memory in MB and per ring node, largest rank
    per level; cf. the paper's Tables 2 and 4), and one-vector apply times through the dense operator and
    through the HBS factors; for the PDE problems also the solution operator G (R2 ring rows) in inverse
    HBS form by Algorithm 1 at the same tolerance: inversion time, memory (the quantity of Table 2) and
    apply time by Algorithm 2.  Returns the table and the dense operators of the constant-coefficient
    problems (their closed-form errors are taken in the oracle leg)."""
    import numpy as np
    import torch
    dev = torch.device("cuda:0")
    rows, keep = [], {}
    for name in W.PAPER_PROBLEMS:
        P = W.paper_problem(name, n, leaf=32)
        form = dtn.COEF_NETWORK if P.form == "network" else dtn.COEF_PDE
        to_dev = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(dev)
        b, c, d = to_dev(P.b), to_dev(P.c), to_dev(P.d)
        ts = []
        for q in range(4):
            t0 = time.perf_counter()
            op = dtn.build(n, b, c, d, leaf=32, coef_form=form, stream=sptr)
            ts.append(time.perf_counter() - t0)
            if q < 3:
                op.free()
        row = {"problem": name, "build_ms": round(statistics.median(ts[1:]) * 1e3, 3),
               "pivoting": "partial" if op.stats()["pivoting_used"] == dtn.PIVOT_PARTIAL else "none"}
        if name in ("laplace", "helmholtz1", "helmholtz2", "helmholtz3", "helmholtz4"):
            keep[name] = (float(P.d[0]) if P.d is not None else 0.0, op.dense())
        g = torch.from_numpy(np.random.default_rng(7).uniform(-1, 1, (1, op.nb))).to(dev).t()
        y = torch.empty_like(g)
        def lat(fn, reps=30):
            for _ in range(3):
                fn()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            ms = []
            for _ in range(reps):
                e0.record(); fn(); e1.record(); e1.synchronize()
                ms.append(e0.elapsed_time(e1))
            return round(sorted(ms)[len(ms) // 2], 4)
        row["apply_dense_k1_ms"] = lat(lambda: op.apply_device(g, y))
        try:
            t0 = time.perf_counter()
            info = op.hbs_compress(1e-7, 64)
            row["hbs_compress_ms"] = round((time.perf_counter() - t0) * 1e3, 2)
            row["hbs_mb"] = round(info["bytes"] / 1e6, 3)
            row["hbs_mb_per_n"] = round(info["bytes"] / 1e6 / n, 5)
            row["hbs_max_rank"] = info["max_rank"]
            row["apply_hbs_k1_ms"] = lat(lambda: op.apply_hbs_device(g, y))
        except dtn.DtnError as e:
            row["hbs_error"] = str(e)
        op.free()
        if P.form != "network":
            # the solution operator G = S'^{-1} (R2 ring rows; T^{-1} = h G) in inverse HBS form at the
            # paper's local tolerance: its memory (the paper's Table 2 quantity) and its apply
            opr = dtn.build(n, b, c, d, leaf=32, ring_rows=dtn.RING_R2, stream=sptr)
            try:
                t0 = time.perf_counter()
                info = opr.hbs_invert(1e-7, 64)
                row["G_invert_ms"] = round((time.perf_counter() - t0) * 1e3, 2)
                row["G_hbs_mb"] = round(info["bytes"] / 1e6, 3)
                row["G_hbs_mb_per_n"] = round(info["bytes"] / 1e6 / n, 5)
                row["G_max_rank"] = info["max_rank"]
                row["apply_G_k1_ms"] = lat(lambda: opr.apply_hbs_inverse_device(g, y))
            except dtn.DtnError as e:
                row["G_error"] = str(e)
            opr.free()
        rows.append(row)
    return rows, keep


def error_leg(dtn, W, n, sptr, tol=1e-7):
    """Section 7.1's e1 / e2 inputs: for every PDE problem of the suite at n x n, G r through the inverse
    HBS factors (R2 ring rows, local tolerance tol) for a random unit r and a smooth r.  The exact G r
    (a sparse solve of the full system) and the errors are taken in the oracle leg."""
    import numpy as np
    import torch
    dev = torch.device("cuda:0")
    R = W.error_vectors(n)
    Rd = torch.from_numpy(np.ascontiguousarray(R.T)).to(dev).t()
    out = {}
    for name in W.PAPER_PROBLEMS:
        P = W.paper_problem(name, n, leaf=32)
        if P.form == "network":
            continue
        to_dev = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(dev)
        op = dtn.build(n, to_dev(P.b), to_dev(P.c), to_dev(P.d), leaf=32, ring_rows=dtn.RING_R2, stream=sptr)
        try:
            op.hbs_invert(tol, 64)
            Y = op.apply_hbs_inverse_device(Rd).cpu().numpy()
            out[name] = (P, Y * (n - 1))          # G R = h^{-1} T^{-1} R
        except dtn.DtnError as e:
            out[name] = (P, str(e))
        op.free()
    return R, out


def serving_bounds(reqs, nbs, results, span_s, solves):
    """Ceilings of the served rate from the requests as they were batched: HBM (8 nb^2 bytes of T per
    batch, shared by its requests in proportion to their columns, plus 16 nb k bytes of G and Y per
    request, at 8 TB/s) and the host link (G in and Y out, 8 nb k bytes each way, PCIe 5 x16 at 64 GB/s
    per direction)."""
    hbm = pcie = 0.0
    for (o, k, _), res in zip(reqs, results):
        nb = nbs[o]
        hbm += 8.0 * nb * nb * k / max(res["batch_cols"], k) + 16.0 * nb * k
        pcie += 8.0 * nb * k
    hbm_s, pcie_s = hbm / 8.0e12, pcie / 64.0e9
    achieved = solves / span_s
    return {"hbm_roofline_solves_per_s": round(solves / hbm_s, 1), "pcie_roofline_solves_per_s": round(solves / pcie_s, 1),
            "bound": "pcie" if pcie_s > hbm_s else "hbm",
            "frac_of_bound": round(achieved / (solves / max(hbm_s, pcie_s)), 4),
            "frac_of_hbm_roofline": round(achieved / (solves / hbm_s), 4)}


def serving_leg(dtn, W, count, max_cols):
    """The serving workload: 8 resident operators, `count` apply requests (k ~ U{1..64}), each arrival a
    build request with probability 0.002 (n in {128, 256}, admitted by HBM footprint).  Saturation = all
    applies offered at t = 0; then Poisson arrivals at 0.5, 0.8 (headline) and 0.95 x saturation.
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

        builds = W.serving_builds(count)
        nbs = {q: op.nb for q, op in enumerate(ops)}

        def run(times, with_builds=False):
            srv.reset_stats()
            sched = schedule(times)
            if with_builds:
                for q, P in builds.items():
                    if q < len(times):
                        sched.append((times[q], "build", dict(n=P.n, b=P.b, c=P.c, d=P.d, leaf=P.leaf)))
            order = sorted(range(len(sched)), key=lambda q: sched[q][0])
            tickets = srv.replay([sched[q] for q in order])
            res = [None] * len(sched)
            for q, t in zip(order, tickets):
                res[q] = srv.wait(t)[1]
            for r in res[len(times):]:                      # operators built by requests leave again
                if r["op_id"] >= 0:
                    srv.remove_op(r["op_id"])
            return srv.stats(), res[:len(times)]

        for P in builds.values():                            # warm the build plans
            dtn.build(P.n, P.b, P.c, P.d, leaf=P.leaf).free()
        run(np.zeros(min(count, 500)))                       # warm-up
        sat, _ = run(np.zeros(count))
        sat_rate = sat["applies_done"] / sat["span_s"]
        sweep = {}
        for f in (0.5, 0.8, 0.95):
            stf, resf = run(np.cumsum(gaps) / (f * sat_rate), with_builds=True)
            sweep[str(f)] = {"lambda_requests_per_s": round(f * sat_rate, 1),
                             "solves_per_s": round(stf["solves_per_s"], 1), "p50_ms": round(stf["p50_ms"], 4),
                             "p99_ms": round(stf["p99_ms"], 4), "mean_batch_cols": round(stf["mean_batch_cols"], 2),
                             "builds_done": stf["builds_done"], "build_p50_ms": round(stf["build_p50_ms"], 3),
                             "build_p99_ms": round(stf["build_p99_ms"], 3),
                             **serving_bounds(reqs, nbs, resf, stf["span_s"], stf["solves_done"])}
            if f == 0.8:
                st = stf
        lam = 0.8 * sat_rate
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
            "builds_in_stream": len(builds), "load_sweep": sweep,
            "plain_solves_per_s": round(plain, 1), "plain_sample_requests": nplain,
            "vs_plain": round(st["solves_per_s"] / plain, 3) if plain > 0 else None,
        }
    finally:
        srv.close()
        for op in ops:
            op.free()


def roofline_of(prof: dict, rank: int = 0) -> dict:
    """The dominant kernel (largest summed HIP-event time over the timed steps; rank 1: the next one):
    algorithmic work per launch over its average launch duration, against the MI355X peak of its bound."""
    cands = []
    for kern, (fams, bound, peak) in KERNELS.items():
        ents = [prof[f] for f in fams if f in prof]
        if not ents:
            continue
        cands.append((kern, sum(e["total_ms"] for e in ents), ents, bound, peak))
    cands.sort(key=lambda t: -t[1])
    if rank >= len(cands):
        return None
    kern, ms, ents, bound, peak = cands[rank]
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
    # one BLAS thread: the SW level-2 box timed with one thread and with all, the build estimate above
    # scaled by that ratio
    from threadpoolctl import threadpool_limits
    box2 = quad.children[0]
    t0 = time.perf_counter()
    box_schur(M, P.n, box2)
    dtn_all = time.perf_counter() - t0
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        box_schur(M, P.n, box2)
        dt1 = time.perf_counter() - t0
        out["one_thread"] = {"value": round(est * dt1 / dtn_all, 3), "unit": "s",
                             "sample": f"SW level-2 box ({box2.sx}x{box2.sy} nodes) {dt1:.2f} s on one thread "
                                       f"against {dtn_all:.2f} s on {threads}, applied to the estimate above"}
        # the oracle's apply (numpy matmul with the GPU's operator) at a few widths, one thread and all
        rng = np.random.default_rng(5)
        app = {}
        for kk in (1, 16, 64):
            G = rng.uniform(-1, 1, (T_gpu.shape[0], kk))
            reps = max(3, int(64 // kk))
            t0 = time.perf_counter()
            for _ in range(reps):
                T_gpu @ G
            app[str(kk)] = round(kk * reps / (time.perf_counter() - t0), 1)
        out["apply_solves_per_s_one_thread"] = app
    app = {}
    for kk in (1, 16, 64):
        G = np.random.default_rng(6).uniform(-1, 1, (T_gpu.shape[0], kk))
        reps = max(3, int(256 // kk))
        t0 = time.perf_counter()
        for _ in range(reps):
            T_gpu @ G
        app[str(kk)] = round(kk * reps / (time.perf_counter() - t0), 1)
    out["apply_solves_per_s"] = app
    err = None
    if P.b is None and P.c is None and P.d is not None and np.all(P.d == P.d[0]):
        Tref = dst_dtn(P.n, float(P.d[0]))
        err = float(np.linalg.norm(T_gpu - Tref) / np.linalg.norm(Tref))
    return out, err


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the build runs on a single MI355X and --gpus {args.gpus} is not "
              f"supported (several GPUs would each build and serve their own operators)", file=sys.stderr)
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
    # autotuner (untimed): the product tiles of this workload's launch shapes, timed per tile; the timed
    # builds below take their tiles from it, and a leg at the end times the fixed thresholds
    tune_rep = None
    if not args.no_tune:
        dtn.tune_clear()
        tune_rep = dtn.tune(P.n, b, c, d, leaf=P.leaf, reps=3, stream=sptr)
        for _ in range(2):
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
    runner_up = roofline_of(prof_all, 1)
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

    # apply latency distribution (no profiling events): k = P.k (MFMA GEMM), 64 and 1 (split-K)
    lat = {}
    for kk in (k, 64, 1):
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

    if tune_rep is not None:
        # the same builds with the planner's fixed tile thresholds, with the same events around the
        # dominant kernel's launches as the timed builds
        dtn.tune_enable(False)
        for _ in range(2):
            dtn.build(P.n, b, c, d, leaf=P.leaf, stream=sptr).free()
        dtn.profile_reset()
        dtn.profile_select(list(KERNELS[dominant][0]))
        dtn.profile_enable(True)
        dflt = []
        for _ in range(args.steps):
            tb = time.perf_counter()
            dtn.build(P.n, b, c, d, leaf=P.leaf, stream=sptr).free()
            dflt.append(time.perf_counter() - tb)
        torch.cuda.synchronize()
        dtn.profile_enable(False)
        dtn.profile_select(None)
        dtn.profile_reset()
        dtn.tune_enable(True)
        tuned_ms = statistics.median(build_s) * 1e3
        default_ms = statistics.median(dflt) * 1e3
        autotune = {"launch_shapes": len(tune_rep),
                    "changed_from_thresholds": sum(1 for v in tune_rep.values() if v["tile"] != v["default"]),
                    "tuned_build_ms": round(tuned_ms, 3), "default_build_ms": round(default_ms, 3),
                    "speedup": round(default_ms / tuned_ms, 3)}
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
        "pivoting": {"used": "partial" if stats["pivoting_used"] == dtn.PIVOT_PARTIAL else "none",
                     "min_pivot_ratio": stats["min_pivot_ratio"], "max_growth": stats["max_growth"]},
        "apply": {"k": k, "solves_per_s": round(lat[k]["solves_per_s"], 1), "p50_ms": round(lat[k]["p50_ms"], 4),
                  "p99_ms": round(lat[k]["p99_ms"], 4), "k1_p50_ms": round(lat[1]["p50_ms"], 4),
                  "k1_p99_ms": round(lat[1]["p99_ms"], 4), "k64_p50_ms": round(lat[64]["p50_ms"], 4),
                  "k64_solves_per_s": round(lat[64]["solves_per_s"], 1),
                  # split-K at its widest against streaming T once at 8 TB/s
                  "k64_frac_of_hbm": round(8.0 * nb * nb / (lat[64]["p50_ms"] * 1e-3) / 8e12, 4)},
        "roofline": roof,
        "autotune": autotune if tune_rep is not None else None,
        # the next kernel by time, from the fully profiled step (events around every launch)
        "roofline_runner_up": runner_up,
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
        # the same comparison on the n = 256 convection-diffusion configuration (leaf 16)
        P2 = W.config("cfg2")
        t2 = {}
        for mode in (dtn.FUSED, dtn.PLAIN):
            ts = []
            for _ in range(3):
                tb = time.perf_counter()
                o2 = dtn.build(P2.n, P2.b, P2.c, P2.d, leaf=P2.leaf, stream=sptr, batching=mode)
                ts.append(time.perf_counter() - tb)
                o2.free()
            t2[mode] = sorted(ts[1:])[0]
        result["plain_vs_fused_" + P2.name] = {"fused_ms": round(t2[dtn.FUSED] * 1e3, 3),
                                               "plain_ms": round(t2[dtn.PLAIN] * 1e3, 3),
                                               "speedup": round(t2[dtn.PLAIN] / t2[dtn.FUSED], 2)}
    if not args.no_cold:
        result["cold_build_ms"] = cold_build(args.workload)
    if not args.no_structured:
        result["structured"] = structured_leg(dtn, P, b, c, d, sptr, op.dense(), value * 1e3)
    body_F = None
    if not args.no_body:
        result["body_loads"], body_F = body_leg(dtn, W, sptr)
    if not args.no_compression:
        result["compression"] = compression_leg(dtn, W, sptr)
    if not args.no_serving:
        result["serving"] = serving_leg(dtn, W, args.serve_requests, args.serve_max_cols)
    suite_T = e12 = None
    if not args.no_suite:
        result["paper_suite"], suite_T = paper_suite_leg(dtn, W, args.suite_n, sptr)
        e12 = error_leg(dtn, W, args.e12_n, sptr)
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
        if suite_T:
            from oracle import dst_dtn
            errs = {}
            for name, (dval, Tx) in suite_T.items():
                Tr = dst_dtn(args.suite_n, dval)
                errs[name] = float(np.linalg.norm(Tx - Tr) / np.linalg.norm(Tr))
            for row in result["paper_suite"]:
                if row["problem"] in errs:
                    row["rel_err_vs_closed_form"] = errs[row["problem"]]
        if e12 is not None:
            from oracle import solution_apply
            R, got = e12
            table = {}
            for name, (Pq, Y) in got.items():
                if isinstance(Y, str):
                    table[name] = {"error": Y}
                    continue
                X = solution_apply(Pq.n, R, Pq.b, Pq.c, Pq.d)
                e = np.linalg.norm(Y - X, axis=0) / np.linalg.norm(X, axis=0)
                table[name] = {"e1": float(e[0]), "e2": float(e[1])}
            result["paper_errors"] = {"n": args.e12_n, "tol": 1e-7, "ring_rows": "R2", "problems": table}
        if body_F is not None and body_F[0] is not None:
            from oracle import body_operator
            Pb = W.paper_problem("randlap1", 512)
            Fr = body_operator(512, body_F[1], Pb.b, Pb.c, Pb.d, form="network")
            err_b = float(np.linalg.norm(body_F[0] - Fr) / np.linalg.norm(Fr))
            for row in result["body_loads"]:
                if row["n"] == 512 and row["n_body"] == len(body_F[1]):
                    row["rel_err_vs_oracle"] = err_b
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
