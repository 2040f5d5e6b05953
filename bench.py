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
    # plain FP32 vector adds without packed math (the build disables packed
    # FP32): 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
    "fp32_add_tops": 256 * 4 * 16 * 2.4e9 / 1e12,
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
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
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
            "nproc": os.cpu_count(), "cpu_model": model,
            "sample": f"FP64 oracle sketch Y[rows,:] = K_f[rows,:] Omega for {rows_done} random rows of the "
                      f"n={w.n}, d={w.d} workload ({el:.1f} s; {per_row} flops per row)"}


def _event_ms(fn, reps: int, torch, stream) -> float:
    """Mean duration of fn() over reps, HIP events on the launch stream."""
    fn()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def srht_sketch_rates(name: str, reps: int, torch, api, W, dev) -> dict:
    """SRHT sketch at a workload: time per launch, kernel evaluations/s and
    transform adds/s against the plain FP32 add rate."""
    w = W.WORKLOADS[name]
    x = torch.from_numpy(W.points(w)).to(dev)
    signs, cols = W.srht_draw(w)
    om = api.Omega.srht(signs, cols, dev)
    hyp = api.Hyper(w.kernel, w.ell, w.s)
    stream = torch.cuda.current_stream(dev)
    ms = _event_ms(lambda: api.sketch(x, hyp, om, w.prec), reps, torch, stream)
    ms_fused = _event_ms(lambda: api.sketch(x, hyp, om, w.prec, want_yprime=True), reps, torch, stream)
    adds = w.n * w.n * (math.log2(w.d) + 1.0)
    return {"workload": f"{name}: n={w.n} D={w.D} {w.kernel} SRHT d={w.d} {w.prec}", "ms": ms,
            "ms_fused_with_dlogell": ms_fused, "kernel_evals_per_s": w.n * w.n / (ms / 1e3),
            "adds_per_s": adds / (ms / 1e3), "alu_peak_adds_per_s": PEAKS["fp32_add_tops"] * 1e12,
            "alu_frac": adds / (ms / 1e3) / (PEAKS["fp32_add_tops"] * 1e12)}


def structured_rates(torch, api, W, dev) -> dict:
    """Cosine / Hartley Omega (any n): the C2 shape with n = 60000 (not a power
    of two, so Walsh-Hadamard does not apply): writing Omega out, the FP32 and
    bf16 dense sketches of it, and the FP32 forward (sketch, TSQR, solve)."""
    w = W.small(W.WORKLOADS["C2"], 60000)
    xnp = W.points(w)
    x = torch.from_numpy(xnp).to(dev)
    A = torch.from_numpy(W.rhs(w)).to(dev, torch.float32)
    signs, cols = W.srht_draw(w)
    hyp = api.Hyper(w.kernel, w.ell, w.s)
    stream = torch.cuda.current_stream(dev)
    out = {"workload": f"n={w.n} D={w.D} {w.kernel} ell={w.ell} d={w.d} m={w.m} leaf_rows={w.leaf_rows}"}
    for t in ("dct", "dht"):
        gen_ms = _event_ms(lambda: api.Omega.structured(t, signs, cols, "f32", dev), 3, torch, stream)
        om32 = api.Omega.structured(t, signs, cols, "f32", dev)
        omb = api.Omega.structured(t, signs, cols, "bf16", dev)
        sk32 = _event_ms(lambda: api.sketch(x, hyp, om32, "f32"), 3, torch, stream)
        skb = _event_ms(lambda: api.sketch(x, hyp, omb, "bf16"), 3, torch, stream)
        fw = _event_ms(lambda: api.forward(x, hyp, om32, "f32", w.sigma2, A, w.leaf_rows), 3, torch, stream)
        out[t] = {"omega_write_ms": gen_ms, "sketch_f32_ms": sk32, "sketch_bf16_ms": skb, "forward_f32_ms": fw,
                  "sketch_f32_frac_of_fp32_mfma_peak": 2.0 * w.n * w.n * w.d / (sk32 / 1e3) / 1e12
                  / PEAKS["fp32_tflops"]}
    return out


def grid_rates(torch, api, W, dev, g: int = 16) -> dict:
    """A grid of g range parameters at the log-likelihood workload (FP32, SRHT
    d = 256, the stabilising shift sigma2 / 10): one lr_sketch_grid call against
    g single sketches, and the whole log-likelihood grid."""
    w = W.WORKLOADS["C4"]
    xnp = W.points(w)
    x = torch.from_numpy(xnp).to(dev)
    yv = torch.from_numpy(W.gp_targets(w, xnp)).to(dev)
    signs, cols = W.srht_draw(w)
    om = api.Omega.srht(signs, cols, dev)
    hyps = [api.Hyper(w.kernel, float(e), w.s) for e in np.linspace(0.5 * w.ell, 2.0 * w.ell, g)]
    nu = 0.1 * w.sigma2
    stream = torch.cuda.current_stream(dev)
    grid_ms = _event_ms(lambda: api.sketch_grid(x, hyps, om, "f32", nu=nu), 3, torch, stream)
    single_ms = _event_ms(lambda: [api.sketch(x, h, om, "f32", nu=nu) for h in hyps], 3, torch, stream)
    ll_ms = _event_ms(lambda: api.loglik_grid(x, hyps, [w.sigma2] * g, om, "f32", yv, w.leaf_rows, nu=nu), 2,
                      torch, stream)
    return {"workload": f"C4 shape, FP32, {g} values of ell in [{0.5 * w.ell}, {2.0 * w.ell}], nu = sigma2/10",
            "sketch_grid_ms": grid_ms, "single_sketches_ms": single_ms, "loglik_grid_ms": ll_ms}


def c5_forward_backward(torch, api, W, dev) -> dict:
    """The largest workload (n = 2^20, d = 1024, FP32, A 2^20 x 16): the forward
    with the fused derivative sketch, and the backward of <A, K~^{-1} A>."""
    w = W.WORKLOADS["C5"]
    x = torch.from_numpy(W.points(w)).to(dev)
    A = torch.from_numpy(W.rhs(w)).to(dev)
    signs, cols = W.srht_draw(w)
    om = api.Omega.srht(signs, cols, dev)
    hyp = api.Hyper(w.kernel, w.ell, w.s)
    stream = torch.cuda.current_stream(dev)
    state = {}

    def fwd():
        state["fw"] = api.forward(x, hyp, om, "f32", w.sigma2, A, w.leaf_rows, want_yprime=True)

    def bwd():
        fw = state["fw"]
        api.backward(x, hyp, om, "f32", fw.sol, fw.Q, w.sigma2, 1, A, V=A, Yprime=fw.Yprime, R=fw.R)

    f_ms = _event_ms(fwd, 1, torch, stream)
    b_ms = _event_ms(bwd, 1, torch, stream)
    out = {"workload": f"C5: n={w.n} SE SRHT d={w.d} m={w.m}, FP32", "forward_fused_ms": f_ms, "backward_ms": b_ms}
    del state
    return out


def _exact_c4():
    """Exact dense log-likelihood and gradient at the log-likelihood workload,
    as stored by tests/golden/make_exact_reference.py (None if absent)."""
    path = os.path.join(ROOT, "tests", "golden", "exact_dense_reference.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                k, v = line.split()
                vals[k] = float(v)
    return vals


def c1_error_vs_exact(torch, api, W, dev) -> dict:
    """The plain FP64 workload (n = 2048, SE, SRHT d = 64): the GPU's X~ against
    the exact K^-1 A, from a dense float64 Cholesky of K_f + sigma2 I on the
    host (torch CPU), and log|K~| against log|K|."""
    w = W.WORKLOADS["C1"]
    xnp = W.points(w)
    A = W.rhs(w)
    signs, cols = W.srht_draw(w)
    om = api.Omega.srht(signs, cols, dev)
    fw = api.forward(torch.from_numpy(xnp).to(dev), api.Hyper(w.kernel, w.ell, w.s), om, "f64", w.sigma2,
                     torch.from_numpy(A).to(dev, torch.float64), w.leaf_rows)
    xt = torch.from_numpy(xnp).double()
    r2 = torch.cdist(xt, xt).square()
    k = w.s ** 2 * torch.exp(-r2 / (2.0 * w.ell ** 2)) + w.sigma2 * torch.eye(w.n, dtype=torch.float64)
    lo = torch.linalg.cholesky(k)
    xe = torch.cholesky_solve(torch.from_numpy(A).double(), lo)
    xg = fw.sol.X.cpu()
    return {"workload": f"C1: n={w.n} {w.kernel} ell={w.ell} sigma2={w.sigma2} SRHT d={w.d}, FP64 path",
            "x_rel_err_vs_exact": float((xg - xe).norm() / xe.norm()),
            "logdet": fw.sol.logdet.item(), "logdet_exact": float(2.0 * torch.log(torch.diagonal(lo)).sum())}


def loglik_timing(torch, api, W, dev) -> dict:
    """The log-likelihood workload (n = 32768, d = 256): forward + log-likelihood
    and the hyperparameter backward, FP64 (nu = 0) and FP32 with a stabilising
    shift (at nu = 0 its float32 core is indefinite): nu = sigma2 / 10 and
    sigma2 / 300. Each path's log-likelihood and gradient are compared with the
    exact dense values (the shift is a change of method, so its error against
    them grows with nu)."""
    w = W.WORKLOADS["C4"]
    xnp = W.points(w)
    x = torch.from_numpy(xnp).to(dev)
    yv = W.gp_targets(w, xnp)
    signs, cols = W.srht_draw(w)
    om = api.Omega.srht(signs, cols, dev)
    hyp = api.Hyper(w.kernel, w.ell, w.s)
    stream = torch.cuda.current_stream(dev)
    exact = _exact_c4()
    out = {"workload": f"C4: n={w.n} D={w.D} {w.kernel} SRHT d={w.d} (targets: random-Fourier-feature GP draw)"}
    for key, prec, nu in (("f64", "f64", 0.0), ("f32", "f32", 0.1 * w.sigma2),
                          ("f32_small_shift", "f32", w.sigma2 / 300.0)):
        dt = torch.float64 if prec == "f64" else torch.float32
        y = torch.from_numpy(yv).to(dev, dt).reshape(-1, 1)
        state = {}

        def fwd():
            fw = api.forward(x, hyp, om, prec, w.sigma2, y, w.leaf_rows, nu=nu, want_yprime=True)
            state["ll"] = api.loglik(y, fw.sol.X, fw.sol.logdet, fw.sol.info, prec)
            state["fw"] = fw

        def bwd():
            fw = state["fw"]
            state["g"], _ = api.backward(x, hyp, om, prec, fw.sol, fw.Q, w.sigma2, 0, y, Yprime=fw.Yprime, R=fw.R,
                                         nu=nu)

        f_ms = _event_ms(fwd, 3, torch, stream)
        b_ms = _event_ms(bwd, 3, torch, stream)
        info = int(state["fw"].sol.info.item())
        row = {"nu": nu, "forward_loglik_ms": f_ms, "backward_ms": b_ms, "info": info}
        if info == 0:
            ll = float(state["ll"].item())
            g = [float(v) for v in state["g"].cpu()]
            row.update({"loglik": ll, "grad": g})
            if exact is not None:
                row["loglik_err_vs_exact"] = ll - exact["c4_loglik_exact"]
                row["grad_err_vs_exact"] = [g[i] - exact[k] for i, k in enumerate(
                    ("c4_grad_logell_exact", "c4_grad_logs_exact", "c4_grad_logsigma2_exact"))]
        out[key] = row
    # the projection variant in FP32 with no shift (its core stays positive definite)
    y = torch.from_numpy(yv).to(dev, torch.float32).reshape(-1, 1)
    state = {}

    def fwd_proj():
        Y, _ = api.sketch(x, hyp, om, "f32")
        Q, _ = api.tsqr(Y, w.leaf_rows, "f32")
        r = api.projection_solve(x, hyp, Q, "f32", w.sigma2, y, clip=True)
        state["ll"] = api.loglik(y, r.X, r.logdet, r.info, "f32")
        state["info"] = r.info

    row = {"nu": 0.0, "forward_loglik_ms": _event_ms(fwd_proj, 3, torch, stream),
           "info": int(state["info"].item()), "loglik": float(state["ll"].item())}
    if exact is not None:
        row["loglik_err_vs_exact"] = row["loglik"] - exact["c4_loglik_exact"]
    out["f32_projection"] = row
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="C3")
    ap.add_argument("--fp64-steps", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--with-backward", action="store_true",
                    help="time forward (with the fused derivative sketch) + hyperparameter backward per step "
                         "(log-likelihood for one right-hand side, else the adjoint of <A, K~^-1 A>)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the FP32 path, SRHT, apply and log-likelihood measurements")
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
    rp = "f32" if prec in ("bf16", "bf16x2") else prec
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
    if args.with_backward:
        # the float32 log-likelihood at d near the kernel's numerical rank needs
        # the stabilising shift (its core is indefinite without it)
        bw_nu = 0.1 * w.sigma2 if (w.m == 1 and prec != "f64") else 0.0
        bw_mode = 0 if w.m == 1 else 1

        def step(prec_, om_, A_, want_yprime=False):  # noqa: F811
            fw = api.forward(X, hyp, om_, prec_, w.sigma2, A_, w.leaf_rows, nu=bw_nu, want_yprime=True)
            api.backward(X, hyp, om_, prec_, fw.sol, fw.Q, w.sigma2, bw_mode, A_, V=None if bw_mode == 0 else A_,
                         Yprime=fw.Yprime, R=fw.R, nu=bw_nu)
            return fw

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
        # plain ALU bound: the transform's adds against the non-packed FP32 add rate
        peak, unit, bound = PEAKS["fp32_add_tops"], "Tops/s", "alu"
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
                   "global_batch": w.n, "seq_len": w.d, "parallelism": "single-gpu",
                   "step": "forward + backward" if args.with_backward else "forward"},
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

    if not args.no_extras and w.name == "C3":
        # the FP32 path on the same workload: float32 kernel tiles on FP32 matrix cores
        om32 = api.Omega.gauss(om_np["omega_t"], "f32", dev)
        sk32 = _event_ms(lambda: api.sketch(X, hyp, om32, "f32"), 1, torch, stream)
        out32 = step("f32", om32, Ad)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(2):
            out32 = step("f32", om32, Ad)
        torch.cuda.synchronize()
        ms32 = (time.perf_counter() - t0) / 2 * 1e3
        f32 = {"ms_per_step": ms32, "tflops": flops["total"] / (ms32 / 1e3) / 1e12, "sketch_ms": sk32,
               "sketch_frac_of_fp32_mfma_peak": flops["sketch"] / (sk32 / 1e3) / 1e12 / PEAKS["fp32_tflops"]}
        if "fp64_path" in result:
            xb = out64.sol.X
            f32["x_rel_diff_vs_fp64"] = ((out32.sol.X.double() - xb).abs().max() / xb.abs().max()).item()
            f32["logdet_rel_diff_vs_fp64"] = abs(out32.sol.logdet.item() - out64.sol.logdet.item()) / abs(
                out64.sol.logdet.item())
        result["fp32_path"] = f32
        del om32, out32
        # the two-term bf16 sketch (K to 16 bits, two bf16 products per tile)
        omx2 = api.Omega.gauss(om_np["omega_t"], "bf16x2", dev)
        skx2 = _event_ms(lambda: api.sketch(X, hyp, omx2, "bf16x2"), 3, torch, stream)
        outx2 = step("bf16x2", omx2, Ad)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            outx2 = step("bf16x2", omx2, Ad)
        torch.cuda.synchronize()
        msx2 = (time.perf_counter() - t0) / 3 * 1e3
        x2 = {"ms_per_step": msx2, "tflops": flops["total"] / (msx2 / 1e3) / 1e12, "sketch_ms": skx2,
              "sketch_bf16_products_per_s": 2.0 * flops["sketch"] / (skx2 / 1e3) / 1e12,
              "sketch_frac_of_bf16_mfma_peak": 2.0 * flops["sketch"] / (skx2 / 1e3) / 1e12 / PEAKS["bf16_tflops"]}
        if "fp64_path" in result:
            xb = out64.sol.X
            x2["x_rel_diff_vs_fp64"] = ((outx2.sol.X.double() - xb).abs().max() / xb.abs().max()).item()
            x2["logdet_rel_diff_vs_fp64"] = abs(outx2.sol.logdet.item() - out64.sol.logdet.item()) / abs(
                out64.sol.logdet.item())
            x2["speedup_vs_fp64"] = result["fp64_path"]["ms_per_step"] / msx2
        result["bf16x2_path"] = x2
        del omx2, outx2
        # Woodbury apply: lowrank_solve with the m right-hand sides minus without
        Q, R = out.Q, out.R
        ms_m = _event_ms(lambda: api.lowrank_solve(Q, R, om, prec, w.sigma2, Ad), 5, torch, stream)
        ms_0 = _event_ms(lambda: api.lowrank_solve(Q, R, om, prec, w.sigma2, None), 5, torch, stream)
        app_ms = max(ms_m - ms_0, 1e-6)
        app_bytes = 2.0 * w.n * w.d * 4 + 3.0 * w.n * w.m * 4  # Q twice, A twice, X once
        result["apply"] = {"ms": app_ms, "algorithmic_bytes": app_bytes, "gbs": app_bytes / (app_ms / 1e3) / 1e9,
                           "frac_of_hbm_peak": app_bytes / (app_ms / 1e3) / 1e9 / PEAKS["hbm_gbs"]}
        result["srht"] = [srht_sketch_rates("C2", 3, torch, api, W, dev),
                          srht_sketch_rates("C5", 1, torch, api, W, dev)]
        result["loglik"] = loglik_timing(torch, api, W, dev)
        result["c1_exact"] = c1_error_vs_exact(torch, api, W, dev)
        result["structured_omega"] = structured_rates(torch, api, W, dev)
        result["hyperparameter_grid"] = grid_rates(torch, api, W, dev)
        result["c5_forward_backward"] = c5_forward_backward(torch, api, W, dev)
        # blocked-QR shapes on this workload's sketch: the binary tree with and
        # without forming Q, and groups of 2 and 4 blocks run in sequence (Eq. 5)
        Ys, _ = api.sketch(X, hyp, om, prec)
        shapes = {}
        for g, want_q in ((1, True), (1, False), (2, True), (4, True)):
            key = f"group{g}" + ("" if want_q else "_r_only")
            shapes[key] = _event_ms(lambda: api.tsqr_tree(Ys, w.leaf_rows, rp, group=g, want_q=want_q), 3, torch,
                                    stream)
        result["tsqr_shapes_ms"] = shapes
        del Ys

    if not args.no_cpu_baseline:
        cb = cpu_baseline(w, x, om_np, flops["sketch"])
        result["cpu_baseline"] = cb

    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
