"""Benchmark: SR steps/s of the warm-started SR step on one MI355X.

Workload (default): the FP32 form, N=8192 samples, M=100000 parameters, rank
r=256, q=2 passes, lambda=1e-3, synthetic O with a k^-1.2 spectrum rotating by
0.01 per step (workloads.CONFIGS["f32_n8192_m100k_r256"]).  Inputs are generated on the GPU and
resident in HBM before timing.  A step is one whole call of wssr_step: centring,
gradient, q passes (two products, CholeskyQR2 of both sides), Rayleigh-Ritz,
signs and the Woodbury apply.

Prints one JSON line.  `--gpus` above 1 is not supported (single-GPU build).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SR steps/s at N×M×r vs plain FP32; HBM GB/s; rel err of δ vs FP64 oracle"
PEAK_FP32_TFLOPS = 157.3
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "hbm_traffic_wssr_step_f32_n8192_m100k_r256.md")


def recorded_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary, or
    None when there is none or the kernel source changed since it was taken
    (the summary records the SHA-256 of the source file it measured)."""
    import hashlib
    import re
    try:
        text = open(TRAFFIC_RECORD).read()
    except OSError:
        return None
    for mt in re.finditer(r"traffic-record: kernel=(\S+) bytes_per_launch=(\d+) source=(\S+) sha256=([0-9a-f]+)", text):
        if mt.group(1) != kernel:
            continue
        try:
            src = open(os.path.join(ROOT, mt.group(3)), "rb").read()
        except OSError:
            return None
        return int(mt.group(2)) if hashlib.sha256(src).hexdigest() == mt.group(4) else None
    return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="f32_n8192_m100k_r256", help="workload name (workloads.CONFIGS)")
    ap.add_argument("--ring", type=int, default=4, help="distinct O_t held in HBM and cycled")
    ap.add_argument("--cpu-baseline", type=int, default=1)
    ap.add_argument("--cpu-cols", type=int, default=0, help="columns of the oracle sample (0: auto)")
    ap.add_argument("--plain-inputs", type=int, default=0,
                    help="draw O, E_L and V_0 i.i.d. Gaussian (no QR factorisation in the generator); "
                         "for hardware-counter runs, whose byte counts do not depend on the values")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="run one elementwise copy of this many MiB before timing, as the reference "
                         "point that scales the HBM byte counters of a counter-collection run")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU; --gpus above 1 is not supported", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2512_05749_amd import Wssr
    from workloads import CONFIGS, Workload

    cfg = CONFIGS[args.config]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t0 = time.time()
    if args.plain_inputs:
        gen = torch.Generator(device=dev).manual_seed(cfg.seed)
        os_ = [torch.randn(cfg.n, cfg.m, generator=gen, device=dev) for _ in range(args.ring)]
        es = [cfg.el_mean + cfg.el_std * torch.randn(cfg.n, generator=gen, device=dev, dtype=torch.float64)
              for _ in range(args.ring)]
        v = torch.randn(cfg.m, cfg.r, generator=gen, device=dev) / math.sqrt(cfg.m)
    else:
        wl = Workload(cfg, device=dev, gen_dtype=torch.float32)
        os_ = [wl.o(t) for t in range(1, args.ring + 1)]
        es = [wl.e_l(t) for t in range(1, args.ring + 1)]
        v = wl.v0()
        del wl.w0, wl.u0
    torch.cuda.synchronize()
    log(f"generated {args.ring} x O ({cfg.n}x{cfg.m}) in {time.time() - t0:.1f}s")
    if args.copy_calibration:
        # one elementwise kernel reading and writing exactly copy_calibration MiB
        src = torch.ones(args.copy_calibration << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        log(f"copy calibration: {args.copy_calibration} MiB read + written by one neg kernel")
        del src, dst

    n, m, r, q, lam = cfg.n, cfg.m, cfg.r, cfg.q, cfg.lam
    h = Wssr(n_max=n, m_max=m, r_max=r, q_max=8, device=dev)
    delta = torch.empty(m, dtype=torch.float64, device=dev)
    sigma = torch.empty(r, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev)

    # step 1: cold start (8 passes from V_0), reported separately
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    h.step(os_[0], es[0], v, lam, q=8, delta=delta, sigma=sigma)
    e1.record(stream)
    code, diag = h.status()
    cold_ms = e0.elapsed_time(e1)
    log(f"cold step (q=8): {cold_ms:.2f} ms, status {code}, diag {diag}")
    if code < 0:
        raise SystemExit(f"cold step failed with status {code}")

    t = 1
    for _ in range(args.warmup):
        h.step(os_[t % args.ring], es[t % args.ring], v, lam, q=q, delta=delta, sigma=sigma)
        t += 1
    torch.cuda.synchronize()
    log("warmup done")

    h.profile(True)
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    for k in range(args.steps):
        starts[k].record(stream)
        h.step(os_[t % args.ring], es[t % args.ring], v, lam, q=q, delta=delta, sigma=sigma)
        ends[k].record(stream)
        t += 1
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    prof = h.profile_read()
    h.profile(False)
    code, diag = h.status()
    per_step = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    ms_per_step = wall * 1e3 / args.steps
    log(f"timed {args.steps} steps: {ms_per_step:.3f} ms/step (wall), median event {np.median(per_step):.3f} ms, "
        f"status {code}, diag {diag}")
    if code < 0:
        raise SystemExit(f"timed steps failed with status {code}")

    flops_gemm = 2.0 * n * m * r            # one product launch (2 N M r)
    kern = {}
    for name, (ms, cnt) in prof.items():
        avg = ms / max(cnt, 1)
        kern[name] = dict(avg_ms=avg, launches=cnt, tflops=flops_gemm / (avg * 1e-3) / 1e12)
    log(f"kernels: {kern}")
    dom = max(kern, key=lambda k: kern[k]["avg_ms"])
    achieved = kern[dom]["tflops"]
    roofline = {"bound": "mfma", "achieved": round(achieved, 2), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP32_TFLOPS, 4), "traffic": recorded_traffic("k_gemm_" + dom),
                "kernel": "k_gemm_" + dom, "avg_ms": round(kern[dom]["avg_ms"], 4),
                "flops_per_launch": flops_gemm,
                "other": {k: {"avg_ms": round(v_["avg_ms"], 4), "tflops": round(v_["tflops"], 2)}
                          for k, v_ in kern.items() if k != dom}}

    out = {
        "metric": METRIC,
        "value": round(1e3 / ms_per_step, 3),
        "unit": "SR steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic, i.i.d. Gaussian O (counter run)" if args.plain_inputs else "synthetic",
        "config": {"workload": f"{cfg.name}: FP32 WSSR step, N={n} M={m} r={r} q={q} lambda={lam}, "
                               f"spectrum k^-{cfg.alpha}, rotation {cfg.theta}/step",
                   "n": n, "m": m, "r": r, "q": q, "lambda": lam},
        "cold_step_ms": round(cold_ms, 3),
        "step_ms_median_events": round(float(np.median(per_step)), 4),
        "roofline": roofline,
    }

    if args.cpu_baseline:
        out["cpu_baseline"], acc = cpu_baseline(args, cfg, os_[1], es[1], v, h)
        out["accuracy_vs_oracle"] = acc
    h.close()
    print(json.dumps(out), flush=True)


def cpu_baseline(args, cfg, o_dev, e_dev, v_dev, h):
    """Time the FP64 oracle on a column sample of the same workload (the first
    `cols` parameters of one step's O, same E_L, the matching rows of V as the
    warm start) and scale the per-step time by M / cols to a full step.  Every
    stage of the step is linear in M except the N x r and r x r ones, which the
    scaling counts M / cols times over, so the reported rate is a slight
    underestimate of the oracle's full-size rate.  The GPU path is run on the
    same sample instance to report its delta error against the oracle."""
    import numpy as np
    import torch

    from oracle import wssr_oracle as orc
    from tests.metrics import rel, sigma_rel_gated

    n, m, r, q, lam = cfg.n, cfg.m, cfg.r, cfg.q, cfg.lam
    cols = args.cpu_cols or max(4 * r, m // 8)
    o_s = o_dev[:, :cols].contiguous()
    v_s = v_dev[:cols].contiguous()
    o_np = o_s.double().cpu().numpy()
    e_np = e_dev.cpu().numpy()
    v_np = v_s.double().cpu().numpy()
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    try:
        from threadpoolctl import threadpool_info
        info = threadpool_info()
        if info:
            threads = max(int(i.get("num_threads", threads)) for i in info)
    except Exception:
        pass
    log(f"oracle on a {n}x{cols} column sample, {threads} threads ...")
    t0 = time.perf_counter()
    ref = orc.wssr_step(o_np, e_np, v_np, lam, r, q)
    dt = time.perf_counter() - t0
    full_s = dt * m / cols
    log(f"oracle sample step {dt:.1f}s -> {full_s:.1f}s per full step")

    # GPU on the same sample instance
    from paper_2512_05749_amd import Wssr
    hs = Wssr(n_max=n, m_max=cols, r_max=r, q_max=q)
    vv = v_s.clone()
    d, s = hs.step(o_s, e_dev, vv, lam, q=q)
    code, _ = hs.status()
    hs.close()
    acc = {"sample": f"N={n}, first {cols} of M={m} columns, warm start = matching rows of V",
           "status": code,
           "delta_rel_err": rel(d.cpu().numpy(), ref["delta"]),
           "sigma_rel_err_gated": sigma_rel_gated(s.cpu().numpy(), ref["sigma"], lam),
           "v_orth_err": float(np.abs(vv.double().cpu().numpy().T @ vv.double().cpu().numpy()
                                      - np.eye(r)).max())}
    log(f"accuracy on the sample: {acc}")
    base = {"value": round(1.0 / full_s, 6), "unit": "SR steps/s", "cores": threads, "kind": "oracle",
            "sample": f"one step of the FP64 oracle on N={n} x {cols} columns (of M={m}), r={r}, q={q}: "
                      f"{dt:.2f}s, scaled by M/{cols} to a full step"}
    return base, acc


if __name__ == "__main__":
    main()
