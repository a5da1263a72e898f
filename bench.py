#!/usr/bin/env python
"""Benchmark: batched ALB generation on one MI355X.

One step = the whole hot path on one batch: seeded cold start -> LOBPCG to a
residual of 1e-8 Ha on every element -> ALBs (restriction + orthonormalisation),
for the 4x4 graphene-like slab (16 extended elements of 48x48x64, 40 states
each, FP64).  The mixed-precision path (FP32 stage, FP64 refinement) is timed
on the same batch and reported beside it, and so is a pass with all elements in
one stream (kernel durations without overlap).

Prints one JSON line.  Inputs are resident in HBM before the timed region.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FP64_PEAK_TFLOPS = 78.6        # MI355X FP64 (vector and matrix)
CLASSES = ("plane", "zcol", "nonlocal", "teter", "gram", "rotate", "rayleigh_ritz", "other")
# kernel symbol of each timing class's main kernel (rocprofv3 names)
CLASS_KERNEL = {"plane": "k_plane", "zcol": "k_zcol", "nonlocal": "k_nl_", "teter": "k_plane",
                "gram": "k_gram", "rotate": "k_rotate", "rayleigh_ritz": "k_rr_lds", "other": "k_residual"}

# HBM bytes per launch from `rocprofv3 --pmc FETCH_SIZE` and `--pmc WRITE_SIZE` runs of
# `bench.py --steps 1 --warmup 0 --no-mixed --no-isolated --no-cpu-baseline --copy-probe-mib 1024`
# on the C2 batch, scaled by what the counters read for the 1 GiB device copy of the same
# run (profiles/c2_fp64_hbm_traffic.md).  Valid only for the kernel source they were taken
# on: `traffic` is reported null once the file's SHA-256 differs.
PMC_TRAFFIC = {
    "rayleigh_ritz": {"config": "c2", "source": "paper_2003_00407_amd/csrc/k_dense.hip",
                      "sha256": "19f84bf8edb687395f94fa0caae0bbab454419c92fba272ecc90d225115659fa",
                      "bytes_per_launch": 3987692},
    "rotate": {"config": "c2", "source": "paper_2003_00407_amd/csrc/k_dense.hip",
               "sha256": "19f84bf8edb687395f94fa0caae0bbab454419c92fba272ecc90d225115659fa",
               "bytes_per_launch": 792666642},
    "gram": {"config": "c2", "source": "paper_2003_00407_amd/csrc/k_dense.hip",
             "sha256": "19f84bf8edb687395f94fa0caae0bbab454419c92fba272ecc90d225115659fa",
             "bytes_per_launch": 1005228684},
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c2")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-isolated", action="store_true", help="skip the one-stream pass")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=8, help="oracle LOBPCG iterations in the CPU sample")
    ap.add_argument("--method", default="lobpcg", choices=["lobpcg", "chfsi"])
    ap.add_argument("--cheb-degree", type=int, default=16)
    ap.add_argument("--graph-iters", type=int, default=0,
                    help="LOBPCG steps captured per HIP graph replay (0: launch per kernel)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="copy a buffer of this size once before timing (reference for PMC byte counters)")
    return ap.parse_args()


def run_path(E, x0, precision, steps, warmup, tol, torch, graph_iters=0, method=0, degree=16):
    """Warm up, then time `steps` full solves + ALBs; returns timing and kernel stats."""
    kw = dict(precision=precision, tol=tol, graph_iters=graph_iters, method=method, cheb_degree=degree)
    for _ in range(warmup):
        E.solve(x0, **kw)
        E.make_alb()
    torch.cuda.synchronize()
    E.timing(enable=True, reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = None
    res = None
    for _ in range(steps):
        eig, res, iters, st = E.solve(x0, **kw)
        E.make_alb()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms, launches, work = E.timing(enable=False, reset=True)
    return {"seconds": t1 - t0, "iters": iters, "ms": ms, "launches": launches,
            "work": work, "max_resid": float(res.max().item())}


def kernel_table(r):
    """Per kernel class: total ms, launches, average launch, achieved algorithmic rate."""
    tab = {}
    for i, name in enumerate(CLASSES):
        if r["launches"][i]:
            row = {"ms_total": round(r["ms"][i], 3), "launches": int(r["launches"][i]),
                   "avg_us": round(1000.0 * r["ms"][i] / r["launches"][i], 2)}
            if r["work"][i] > 0 and r["ms"][i] > 0:
                rate = r["work"][i] / (r["ms"][i] / 1000.0)
                if i <= 3:
                    row["GBs"] = round(rate / 1e9, 1)
                else:
                    row["TFLOPs"] = round(rate / 1e12, 2)
            tab[name] = row
    return tab


def source_sha(path):
    with open(os.path.join(HERE, path), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def roofline_for(r, config, with_traffic=True):
    """Roofline of the dominant kernel class (most GPU time) over a run's kernels."""
    i = int(np.argmax(r["ms"]))
    name = CLASSES[i]
    ms, n, w = r["ms"][i], max(1, r["launches"][i]), r["work"][i]
    avg_s = ms / 1000.0 / n
    if i <= 3:       # HBM-bound passes: algorithmic bytes per launch / duration
        achieved = (w / n) / avg_s / 1e9
        peak, unit, bound = HBM_PEAK_GBS, "GB/s", "hbm"
    elif i <= 5:     # subspace GEMMs on FP64 MFMA: algorithmic flops per launch / duration
        achieved = (w / n) / avg_s / 1e12
        peak, unit, bound = FP64_PEAK_TFLOPS, "TFLOP/s", "mfma"
    else:            # small dense FP64, one workgroup per element: vector ALU
        achieved = (w / n) / avg_s / 1e12
        peak, unit, bound = FP64_PEAK_TFLOPS, "TFLOP/s", "alu"
    traffic = None
    t = PMC_TRAFFIC.get(name) if with_traffic else None
    if t and t["config"] == config and source_sha(t["source"]) == t["sha256"]:
        traffic = t["bytes_per_launch"]
    return {"kernel": name, "symbol": CLASS_KERNEL[name], "bound": bound, "achieved": round(achieved, 4),
            "peak": peak, "unit": unit, "frac": round(achieved / peak, 5), "traffic": traffic,
            "avg_launch_us": round(avg_s * 1e6, 2), "launches": int(n),
            "work_per_launch": w / n}


def hpsi_rate(r):
    """H*psi GB/s: algorithmic bytes of the H*psi passes over their summed time."""
    ms = r["ms"][0] + r["ms"][1] + r["ms"][2]
    by = r["work"][0] + r["work"][1] + r["work"][2]
    return round(by / (ms / 1000.0) / 1e9, 2) if ms > 0 else None


def cpu_baseline(cfg, n_iters_scale, cpu_iters):
    """The oracle (plain NumPy/SciPy FP64) on a bounded sample: one element, a few LOBPCG iterations."""
    import workloads as W
    from oracle import lobpcg as olob
    from oracle.planewave import n_workers
    el = cfg.elements[5]
    J = el.n_states
    x0 = W.initial_block(el.npts, J + W.guard_count(J), cfg.x0_seed_base + 5).T
    t0 = time.perf_counter()
    r = olob.lobpcg(el, x0, J, tol=1e-30, max_iter=cpu_iters)
    dt = time.perf_counter() - t0
    per_iter = dt / max(1, r.iters)
    est = per_iter * n_iters_scale
    return {"value": round(1.0 / est, 5), "unit": "element-solves/s", "cores": n_workers(),
            "kind": "oracle",
            "sample": (f"element 5 of {cfg.n_elem}: {r.iters} oracle LOBPCG iterations in {dt:.1f} s "
                       f"({per_iter:.2f} s/iteration), scaled to the {n_iters_scale} iterations the "
                       f"GPU needed for that element to reach 1e-8 (ALB SVD time negligible)")}


def make_x0(cfg, E, D, torch):
    if cfg.name == "c4":
        # 2.3e9 starting values: drawn on the device from a seeded generator
        gen = torch.Generator(device="cuda").manual_seed(cfg.x0_seed_base)
        return torch.randn(int(E.offsets(D.DG_OFF_X0)[-1]), dtype=torch.float64, device="cuda", generator=gen)
    return torch.tensor(D.pack_initial(cfg.elements, cfg.x0_seed_base), dtype=torch.float64, device="cuda")


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU only (--gpus {args.gpus} requested); "
              "the element batch would shard across GPUs by whole elements with no communication, "
              "which is not measured here.", file=sys.stderr)
        sys.exit(2)
    import torch
    import workloads as W
    from paper_2003_00407_amd import dgalb as D
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    cfg = W.make_config(args.config)
    els = cfg.elements
    E = D.Elements(els)
    x0 = make_x0(cfg, E, D, torch)
    if args.copy_probe_mib > 0:
        buf = torch.empty(args.copy_probe_mib << 20, dtype=torch.uint8, device="cuda")
        buf2 = torch.empty_like(buf)
        buf2.copy_(buf)
        del buf, buf2
    torch.cuda.synchronize()
    print(f"[bench] config={cfg.name} elements={len(els)} grid={els[0].n} J={els[0].n_states}",
          file=sys.stderr, flush=True)
    meth = D.DG_LOBPCG if args.method == "lobpcg" else D.DG_CHFSI
    r64 = run_path(E, x0, D.DG_FP64, args.steps, args.warmup, args.tol, torch, args.graph_iters, meth,
                   args.cheb_degree)
    print(f"[bench] fp64: {r64['seconds']:.3f}s for {args.steps} steps, iters {[int(i) for i in r64['iters']]}",
          file=sys.stderr, flush=True)
    n = len(els)
    value = n * args.steps / r64["seconds"]
    out = {
        "metric": "ALB element-solves/s + Hψ GB/s, mixed vs FP64 on one GPU at 1e-8 Ha eigen error",
        "value": round(value, 4),
        "unit": "element-solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1000.0 * r64["seconds"] / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": cfg.name + ": " + cfg.description, "n_elem": n,
                   "grid": list(els[0].n), "states": els[0].n_states,
                   "tol": args.tol, "method": args.method, "precision": "fp64", "graph_iters": args.graph_iters,
                   "element_groups": int(os.environ.get("DG_STREAMS", "0")) or max(1, min(4, n // 4))},
        "hpsi_GBs_fp64": hpsi_rate(r64),
        "iters_fp64": [int(i) for i in r64["iters"]],
        "max_resid_fp64": r64["max_resid"],
        "kernels_fp64": kernel_table(r64),
        "roofline": roofline_for(r64, cfg.name),
    }
    if not args.no_mixed:
        rmx = run_path(E, x0, D.DG_MIXED, args.steps, args.warmup, args.tol, torch, args.graph_iters, meth,
                       args.cheb_degree)
        print(f"[bench] mixed: {rmx['seconds']:.3f}s", file=sys.stderr, flush=True)
        out["mixed"] = {"value": round(n * args.steps / rmx["seconds"], 4),
                        "ms_per_step": round(1000.0 * rmx["seconds"] / args.steps, 3),
                        "speedup_vs_fp64": round(r64["seconds"] / rmx["seconds"], 3),
                        "iters": [int(i) for i in rmx["iters"]], "max_resid": rmx["max_resid"],
                        "kernels": kernel_table(rmx)}
    if not args.no_isolated:
        # all elements in one stream: kernel durations without overlap between element groups
        del E
        E1 = D.Elements(els, n_streams=1)
        r1 = run_path(E1, x0, D.DG_FP64, 1, 0, args.tol, torch)
        print(f"[bench] one stream: {r1['seconds']:.3f}s", file=sys.stderr, flush=True)
        # kernels without overlap between groups: the dominant class's roofline here is
        # the per-kernel figure (in the timed region launches of four groups share the GPU)
        out["one_stream_fp64"] = {"value": round(n / r1["seconds"], 4), "hpsi_GBs": hpsi_rate(r1),
                                  "kernels": kernel_table(r1),
                                  "roofline": roofline_for(r1, cfg.name, with_traffic=False)}
    if not args.no_cpu_baseline:
        print("[bench] timing the oracle sample on the host", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(cfg, int(r64["iters"][5]), args.cpu_iters)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
