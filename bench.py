"""Benchmark of the low-rank covariance-inverse hot path on one MI355X.

Default workload (the headline configuration): n = 262144 points uniform in
[0,1]^2, Matern-3/2 (s = 1, ell = 0.1), nugget sigma2 = 1e-3, Gaussian Omega
N(0, 1/d) rounded to bf16, d = 512, A = n x 16 N(0,1), leaves of 4096 rows.
One step = sketch (bf16 matrix cores, K tiles on the fly) -> blocked QR (FP32
leaves, FP64 tree) -> Woodbury solve (FP64 core), inputs resident in HBM.

Prints one JSON line: TFLOP/s on algorithmic flops, ms per step, a roofline
object for the sketch kernel (HIP events on the launch stream), the plain
FP64 GPU path timed beside it with the error between the two, and the FP64
CPU oracle timed on a bounded row sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAKS = {  # MI355X published dense peaks
    "bf16_tflops": 2500.0,
    "fp32_tflops": 157.3,
    "fp64_tflops": 78.6,
    "hbm_gbs": 8000.0,
}
METRIC = "K⁻¹A low-rank solve s & TFLOP/s, FP32/BF16 vs FP64 GPU, n=262144 d=512"


def algorithmic_flops(n: int, d: int, m: int, leaf_rows: int, omega: str) -> dict:
    """Flops the method itself needs per forward pass (not what the kernels waste)."""
    nleaf = -(-n // leaf_rows)
    rows = [leaf_rows] * (nleaf - 1) + [n - (nleaf - 1) * leaf_rows]
    geqrf = lambda mm, k: 2.0 * mm * k * k - 2.0 / 3.0 * k ** 3  # Householder QR of mm x k
    if omega == "gauss":
        sketch = 2.0 * n * n * d
    else:  # SRHT: n^2 kernel values plus n (log2 d + 1) adds per row (Sec. 1, Sec. 3.2)
        sketch = n * n * (math.log2(d) + 1.0)
    leaf = sum(geqrf(r, d) for r in rows)
    tree = (nleaf - 1) * geqrf(2 * d, d)
    f = {
        "sketch": sketch,
        "leaf_qr": leaf,
        "tree_qr": tree,
        "q_formation": leaf + tree,
        "omega_t_q": 2.0 * n * d * d,
        "core": 3.0 * d ** 3,
        "apply": 4.0 * n * d * m,
    }
    f["total"] = sum(f.values())
    return f


def source_hash(*files) -> str:
    h = hashlib.sha256()
    for fn in files:
        with open(os.path.join(ROOT, fn), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(kernel_key: str, src_hash: str):
    """HBM bytes per launch from the committed counter summary, if it still
    describes the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", "counters_sketch_bf16_c3_n262144_d512.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("kernel") != kernel_key or kv.get("source_hash") != src_hash:
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(w, x, om_np, sketch_flops: float, budget_s: float = 12.0) -> dict:
    """The FP64 oracle's sketch on a bounded sample of rows (the stage that holds
    >99% of the algorithmic flops), rate scaled to TFLOP/s with the same
    algorithmic count per row as the GPU figure."""
    from threadpoolctl import threadpool_info

    from oracle import sketch as osk

    threads = max([t.get("num_threads", 1) for t in threadpool_info()] + [1])
    rows_done, t0 = 0, time.perf_counter()
    rng = np.random.default_rng(11)
    block = 64
    while time.perf_counter() - t0 < budget_s and rows_done < w.n:
        rows = rng.choice(w.n, block, replace=False)
        osk.sketch_rows(x, rows, w.kernel, w.ell, w.s, om_np, k_round=None)
        rows_done += block
    el = time.perf_counter() - t0
    flops = sketch_flops / w.n * rows_done
    per_row = "2 n d" if w.omega == "gauss" else "n (log2 d + 1)"
    return {"value": flops / el / 1e12, "unit": "TFLOP/s", "cores": int(threads), "kind": "oracle",
            "sample": f"FP64 oracle sketch Y[rows,:] = K_f[rows,:] Omega for {rows_done} random rows of the "
                      f"n={w.n}, d={w.d} workload ({el:.1f} s; {per_row} flops per row)"}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="C3")
    ap.add_argument("--fp64-steps", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="only copy a buffer of this many MiB device to device (reference kernel for the HBM "
                         "byte counters), then exit")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (see DESIGN.md for how it "
              "would shard)", file=sys.stderr)
        return 2

    import torch

    import workloads as W
    from paper_1312_1869_amd import api

    dev = torch.device("cuda:0")
    if args.calib_copy_mib > 0:
        src = torch.ones(args.calib_copy_mib << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calib_copy_bytes": src.numel() * 4}), flush=True)
        return 0
    w = W.WORKLOADS[args.workload]
    prec = w.prec
    rp = "f32" if prec == "bf16" else prec
    rdt = torch.float64 if rp == "f64" else torch.float32

    # ---- inputs (host generation, then resident in HBM before timing)
    x = W.points(w)
    A = W.rhs(w)
    if w.omega == "srht":
        signs, cols = W.srht_draw(w)
        om_np = {"kind": "srht", "signs": signs, "cols": cols}
        om = api.Omega.srht(signs, cols, dev)
        om64 = om
    else:
        om_t = W.gauss_omega(w)
        om_np = {"kind": "gauss", "omega_t": om_t}
        om = api.Omega.gauss(om_t, prec, dev)
        om64 = None if args.no_fp64 else api.Omega.gauss(om_t, "f64", dev)
    X = torch.from_numpy(x).to(dev)
    Ad = torch.from_numpy(A).to(dev, rdt)
    hyp = api.Hyper(w.kernel, w.ell, w.s)
    torch.cuda.synchronize()

    def step(prec_, om_, A_, want_yprime=False):
        return api.forward(X, hyp, om_, prec_, w.sigma2, A_, w.leaf_rows, want_yprime=want_yprime)

    # ---- warmup and timed steps
    for _ in range(args.warmup):
        step(prec, om, Ad)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = step(prec, om, Ad)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms = el / args.steps * 1e3
    info = int(out.sol.info.item())

    flops = algorithmic_flops(w.n, w.d, w.m, w.leaf_rows, w.omega)
    tflops = flops["total"] / (ms / 1e3) / 1e12

    # ---- per-stage breakdown and sketch-kernel duration (events on the launch stream)
    stream = torch.cuda.current_stream(dev)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    sk_ms = []
    stages = {"sketch": [], "tsqr": [], "solve": []}
    for _ in range(max(3, min(args.steps, 10))):
        ev[0].record(stream)
        Y, _ = api.sketch(X, hyp, om, prec)
        ev[1].record(stream)
        Q, R = api.tsqr(Y, w.leaf_rows, rp)
        ev[2].record(stream)
        api.lowrank_solve(Q, R, om, prec, w.sigma2, Ad)
        ev[3].record(stream)
        torch.cuda.synchronize()
        stages["sketch"].append(ev[0].elapsed_time(ev[1]))
        stages["tsqr"].append(ev[1].elapsed_time(ev[2]))
        stages["solve"].append(ev[2].elapsed_time(ev[3]))
    stage_ms = {k: float(np.mean(v)) for k, v in stages.items()}
    sk = stage_ms["sketch"]

    src = source_hash("paper_1312_1869_amd/csrc/sketch_dense.hip", "paper_1312_1869_amd/csrc/common.hpp")
    if w.omega == "gauss":
        kernel_key = {"bf16": "sketch_bf16_kernel", "f32": "sketch_dense_kernel<1",
                      "f64": "sketch_dense_kernel<0"}[prec]
        peak, unit, bound = (PEAKS["bf16_tflops"] if prec == "bf16" else
                             PEAKS["fp32_tflops"] if prec == "f32" else PEAKS["fp64_tflops"]), "TFLOP/s", "mfma"
        achieved = flops["sketch"] / (sk / 1e3) / 1e12
    else:
        kernel_key = "sketch_srht_kernel"
        # plain ALU bound: lane operations of the transform (adds) against the FP32 vector peak
        peak, unit, bound = PEAKS["fp32_tflops"] / 2.0, "Tops/s", "alu"
        achieved = flops["sketch"] / (sk / 1e3) / 1e12
    traffic = read_traffic(kernel_key, src)
    roofline = {"bound": bound, "achieved": achieved, "peak": peak, "unit": unit, "frac": achieved / peak,
                "traffic": traffic, "kernel": kernel_key, "ms_per_launch": sk, "algorithmic_per_launch":
                flops["sketch"]}

    result = {
        "metric": METRIC, "value": tflops, "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": prec, "data": "synthetic",
        "config": {"workload": f"{w.name}: n={w.n} D={w.D} {w.kernel} ell={w.ell} s={w.s} sigma2={w.sigma2} "
                               f"{w.omega} d={w.d} m={w.m} leaf_rows={w.leaf_rows}",
                   "global_batch": w.n, "seq_len": w.d, "parallelism": "single-gpu"},
        "seconds_per_solve": ms / 1e3, "stages_ms": stage_ms, "algorithmic_flops": flops, "info": info,
        "roofline": roofline,
    }

    # ---- plain FP64 GPU path beside it, and the error between the two
    if not args.no_fp64 and prec != "f64":
        A64 = Ad.double()
        step("f64", om64, A64)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.fp64_steps):
            out64 = step("f64", om64, A64)
        torch.cuda.synchronize()
        ms64 = (time.perf_counter() - t0) / args.fp64_steps * 1e3
        xa, xb = out.sol.X.double(), out64.sol.X
        rel = ((xa - xb).abs().max() / xb.abs().max()).item()
        ld_rel = abs(out.sol.logdet.item() - out64.sol.logdet.item()) / abs(out64.sol.logdet.item())
        result["fp64_path"] = {"ms_per_step": ms64, "tflops": flops["total"] / (ms64 / 1e3) / 1e12,
                               "speedup_of_mixed": ms64 / ms, "x_rel_diff_vs_fp64": rel,
                               "logdet_rel_diff_vs_fp64": ld_rel}

    if not args.no_cpu_baseline:
        cb = cpu_baseline(w, x, om_np, flops["sketch"])
        result["cpu_baseline"] = cb

    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
