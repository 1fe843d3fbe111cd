"""Benchmark: SR steps/s of the warm-started SR step on one MI355X.

Default workload: the largest single-GPU instance, N=16384 samples,
M=4,000,000 parameters, rank r=512, q=3 passes, lambda=1e-3, synthetic O with
a k^-1.3 spectrum rotating by 0.005 per step (workloads.CONFIGS
["bf16_n16384_m4m_r512_q3"]), stored in BF16 (131 GB) and run in the BF16
form with the split correction of the skinny operand (two products).  The
FP32 row blocks of O are generated on the GPU and stored through the
library's ingest, which also forms the gradient from the unrounded values; O
is resident in HBM before timing.  A step is one whole call of wssr_step_g:
q passes (two products, CholeskyQR2 of both sides), Rayleigh-Ritz, signs and
the Woodbury apply.  Beside it, in the same JSON line: the FP32 form on the
same recipe at M=2e6 (its FP32 O is 131 GB), the FP32 benchmark workload
f32_n8192_m100k_r256 as a secondary record, the FP64 oracle on a column
sample (CPU baseline and the accuracy of the form against it), and the
ingest time.

--config picks another workload (f32_n8192_m100k_r256, bf16_n16384_m1m_r512,
or batch16_mixed for the batched form beside the same problems one after
another); --form another precision form.  --sweep 1 times the two product
kernels alone on N=16384, M=1e6 over a range of ranks, FP32 and BF16, against
both rooflines (HBM and MFMA): the small ranks are memory-bound.

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
# committed counter summaries per (workload, M, form)
TRAFFIC_RECORDS = {
    ("f32_n8192_m100k_r256", 100_000, "f32"): "hbm_traffic_wssr_step_f32_n8192_m100k_r256.md",
    ("bf16_n16384_m4m_r512_q3", 4_000_000, "bf16_split"): "hbm_traffic_wssr_step_bf16split_n16384_m4m_r512_q3.md",
}


def recorded_traffic(kernel, record):
    """Bytes per launch of `kernel` moved between the L2 and the memory side
    (FETCH_SIZE + WRITE_SIZE) from the committed counter summary `record`, or
    None when there is none or the kernel source changed since it was taken
    (the summary records the SHA-256 of the source file it measured)."""
    import hashlib
    import re
    try:
        text = open(os.path.join(ROOT, "profiles", record)).read()
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
    ap.add_argument("--steps", type=int, default=0, help="timed steps (0: the workload's own count, 10 for the "
                                                                 "largest instance, 20 otherwise)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="bf16_n16384_m4m_r512_q3",
                    help="workload name (workloads.CONFIGS), or batch16_mixed for the batched form")
    ap.add_argument("--ring", type=int, default=0,
                    help="distinct O_t held in HBM and cycled (0: 4, or 1 above 2^30 elements)")
    ap.add_argument("--form", default=None, choices=["f32", "bf16", "bf16_split", "bf16x2"],
                    help="storage and product precision of O (default: the workload's own form)")
    ap.add_argument("--lanes", type=int, default=4, help="batched workload: concurrent lanes of the handle")
    ap.add_argument("--compare-f32", type=int, default=-1,
                    help="BF16 forms: also time the FP32 form (1: the same instance; -1: the workload's own "
                         "comparison, FP32 at M=2e6 for the largest instance; 0: none)")
    ap.add_argument("--secondary", type=int, default=1,
                    help="also time the FP32 benchmark workload f32_n8192_m100k_r256 as a secondary record")
    ap.add_argument("--averaged", type=float, default=0.95,
                    help="also time the averaged-state step with this weight on the same data (0: skip)")
    ap.add_argument("--sketch", default="16,0;16,1",
                    help="randomized-sketch cold steps to time on the headline data: 'p,q;p,q' (oversampling "
                         "capped so that r + p <= 512; empty: skip)")
    ap.add_argument("--spring", type=int, default=1,
                    help="time MinSR/SPRING in sample space on the same data (workloads with N <= 8192)")
    ap.add_argument("--cpu-baseline", type=int, default=1)
    ap.add_argument("--cpu-cols", type=int, default=0, help="columns of the oracle sample (0: auto)")
    ap.add_argument("--plain-inputs", type=int, default=0,
                    help="draw O, E_L and V_0 i.i.d. Gaussian (no QR factorisation in the generator); "
                         "for hardware-counter runs, whose byte counts do not depend on the values")
    ap.add_argument("--m", type=int, default=0,
                    help="override the workload's M (number of parameters), e.g. the FP32 comparison of the "
                         "largest instance at M=2e6")
    ap.add_argument("--sweep", type=int, default=0,
                    help="time the product kernels alone over a range of ranks (roofline sweep)")
    ap.add_argument("--sweep-n", type=int, default=16384)
    ap.add_argument("--sweep-m", type=int, default=1_000_000)
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="run one elementwise copy of this many MiB before timing, as the reference "
                         "point that scales the HBM byte counters of a counter-collection run")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


PEAK_BF16_TFLOPS = 2516.6
PRODUCTS = {"f32": 1, "bf16": 1, "bf16_split": 2, "bf16x2": 3}


def time_form(h, form, o_ring, e_ring, g_ring, v_start, cfg, args, dev, avg=None):
    """Cold step, warm-up and timed steps of one precision form on handle h;
    returns the timings, the product-kernel profile and the last status.  The
    BF16 forms use the gradient their ingest formed from the unrounded O
    (g_ring); the FP32 form forms it inside the step.  avg: the averaged-state
    step with that weight, from the zero state."""
    import numpy as np
    import torch

    m, r, q, lam = cfg.m, cfg.r, cfg.q, cfg.lam
    ring = len(o_ring)
    v = v_start.clone()
    delta = torch.empty(m, dtype=torch.float64, device=dev)
    sigma = torch.zeros(r, dtype=torch.float64, device=dev)
    l_state = torch.zeros(r, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev)
    tag = form if avg is None else f"{form}, averaged {avg}"

    def one(t, qq):
        k = t % ring
        g = None if g_ring is None else g_ring[k]
        if avg is not None:
            h.step_avg(o_ring[k], e_ring[k], v, lam, avg, sigma, l_state, q=qq, delta=delta, g=g)
        elif g is None:
            h.step(o_ring[k], e_ring[k], v, lam, q=qq, delta=delta, sigma=sigma)
        else:
            h.step(o_ring[k], None, v, lam, q=qq, delta=delta, sigma=sigma, g=g)

    # step 1: cold start (8 passes from V_0), reported separately
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    one(0, 8)
    e1.record(stream)
    code, diag = h.status()
    cold_ms = e0.elapsed_time(e1)
    cold_delta = delta.clone() if avg is None else None
    log(f"[{tag}] cold step (q=8): {cold_ms:.2f} ms, status {code}, diag {diag}")
    if code < 0:
        raise SystemExit(f"cold step failed with status {code}")

    t = 1
    for _ in range(args.warmup):
        one(t, q)
        t += 1
    torch.cuda.synchronize()
    log(f"[{tag}] warmup done")

    h.profile(True)
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    for k in range(args.steps):
        starts[k].record(stream)
        one(t, q)
        ends[k].record(stream)
        t += 1
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    prof = h.profile_read()
    h.profile(False)
    code, diag = h.status()
    per_step = [s_.elapsed_time(e_) for s_, e_ in zip(starts, ends)]
    ms_per_step = wall * 1e3 / args.steps
    log(f"[{tag}] timed {args.steps} steps: {ms_per_step:.3f} ms/step (wall), median event "
        f"{np.median(per_step):.3f} ms, status {code}, diag {diag}")
    if code < 0:
        raise SystemExit(f"timed steps failed with status {code}")
    return dict(ms_per_step=ms_per_step, median_ms=float(np.median(per_step)),
                p10_ms=float(np.percentile(per_step, 10)), p90_ms=float(np.percentile(per_step, 90)),
                cold_ms=cold_ms, prof=prof, diag=diag, v=v, cold_delta=cold_delta)


def time_spring(h, form, o_ring, e_ring, cfg, dev, momentum, steps):
    """MinSR / SPRING in sample space (the paper's comparison system) on the
    same data: one untimed call, then `steps` timed calls with the momentum
    state carried; the FP64 product T = O O^T and the Cholesky reported
    against the FP64 MFMA peak."""
    import numpy as np
    import torch

    n, m = cfg.n, cfg.m
    dth = torch.zeros(m, dtype=torch.float64, device=dev)
    delta = torch.empty(m, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev)
    h.spring(o_ring[0], e_ring[0], cfg.lam, momentum=momentum, eta=0.05, dtheta=dth, delta=delta)
    torch.cuda.synchronize()
    h.profile(True)
    ms = []
    for k in range(steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        h.spring(o_ring[(k + 1) % len(o_ring)], e_ring[(k + 1) % len(e_ring)], cfg.lam, momentum=momentum,
                 eta=0.05, dtheta=dth, delta=delta)
        e1.record(stream)
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    prof = h.profile_read()
    h.profile(False)
    code, diag = h.status()
    pm, pc = prof.get("spring_product", (0.0, 0))
    cm, cc = prof.get("spring_cholesky", (0.0, 0))
    t_ms = pm / max(pc, 1)
    flops = float(n) * (n + 1) * m                  # the N(N+1)/2 distinct entries of T, 2M flops each
    rec = {"momentum": momentum, "ms_per_step": round(float(np.median(ms)), 3),
           "value": round(1e3 / float(np.median(ms)), 3), "status": code,
           "product_T": {"ms": round(t_ms, 3), "TFLOP/s": round(flops / (t_ms * 1e-3) / 1e12, 2),
                         "peak_TFLOP/s": 78.6, "frac": round(flops / (t_ms * 1e-3) / 1e12 / 78.6, 4)},
           "cholesky_ms": round(cm / max(cc, 1), 3)}
    log(f"[{form}] SPRING (momentum {momentum}): {rec}")
    return rec


def time_sketch(h, form, o_ring, e_ring, g_ring, cfg, dev, p, q, cold_delta):
    """One randomized-sketch step (oversampling p, q power passes) on the
    first O, as the cold start, against the q = 8 cold step on the same O:
    its time and the relative difference of the two directions."""
    import torch

    m, r, n = cfg.m, cfg.r, cfg.n
    gen = torch.Generator(device=dev).manual_seed(cfg.seed + 101)
    omega = torch.randn(n, r + p, generator=gen, device=dev, dtype=torch.float32)
    v = torch.empty(m, r, dtype=torch.float32, device=dev)
    delta = torch.empty(m, dtype=torch.float64, device=dev)
    g = None if g_ring is None else g_ring[0]
    stream = torch.cuda.current_stream(dev)
    ms = []
    for _ in range(2):          # the first call warms the code paths
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        h.step_sketch(o_ring[0], e_ring[0] if g is None else None, omega, v, cfg.lam, q=q, delta=delta, g=g)
        e1.record(stream)
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    code, diag = h.status()
    diff = float((delta - cold_delta).norm() / cold_delta.norm())
    log(f"[{form}] sketch cold step (p={p}, q={q}): {ms[-1]:.2f} ms, status {code}, "
        f"delta vs the 8-pass cold step {diff:.2e}")
    return {"p": p, "q": q, "ms": round(ms[-1], 3), "status": code, "delta_rel_diff_vs_8_pass_cold": diff}


def product_kernel(form, side, cfg):
    """Name of the product kernel the library launches for this form and
    side: the FP32 products take their direct-to-LDS form when the rows of O
    and of the skinny operand are 16-byte aligned (the inputs here are
    contiguous torch tensors, so that is r % 4 == 0, plus M % 4 == 0 on the
    sample side)."""
    if form != "f32":
        # BF16: O's rows are whole 16-byte chunks (8 elements); one O plane and
        # r > 256: the skinny operand streamed into registers
        if cfg.m % 8 != 0:
            return "k_gemm16_" + side
        if form != "bf16x2" and cfg.r > 256:
            return "k_gemm16_" + side + "_rs"
        return "k_gemm16_" + side + "_dma"
    aligned = cfg.r % 4 == 0 and (cfg.m % 4 == 0 or side == "param_side")
    if aligned and side == "param_side" and cfg.r <= 32:
        return "k_gemm_param_side_narrow"      # 32-column tile, O staged through registers
    return "k_gemm_" + side + ("_dma" if aligned else "")


def column_tile(form, r, side):
    """Column-tile width of the product kernels for rank r (aligned inputs;
    BF16 with one plane of each operand)."""
    if form == "f32":
        return 32 if r <= 32 else 64 if r <= 64 else 128 if r <= 128 else 256
    return 64 if r <= 64 else 128 if r <= 128 else 256 if r <= 256 else 512


def roofline_of(form, prof, cfg):
    n, m, r = cfg.n, cfg.m, cfg.r
    flops_gemm = 2.0 * n * m * r * PRODUCTS[form]     # MFMA flops of one product launch
    peak = PEAK_FP32_TFLOPS if form == "f32" else PEAK_BF16_TFLOPS
    kern = {}
    for name, (ms, cnt) in prof.items():
        avg = ms / max(cnt, 1)
        kern[name] = dict(avg_ms=avg, launches=cnt, tflops=flops_gemm / (avg * 1e-3) / 1e12)
    log(f"[{form}] kernels: {kern}")
    dom = max(kern, key=lambda k: kern[k]["avg_ms"])
    achieved = kern[dom]["tflops"]
    return {"bound": "mfma", "achieved": round(achieved, 2), "peak": peak, "unit": "TFLOP/s",
            "frac": round(achieved / peak, 4),
            "traffic": (recorded_traffic(product_kernel(form, dom, cfg), TRAFFIC_RECORDS[(cfg.name, cfg.m, form)])
                        if (cfg.name, cfg.m, form) in TRAFFIC_RECORDS else None),
            "kernel": product_kernel(form, dom, cfg), "avg_ms": round(kern[dom]["avg_ms"], 4),
            "flops_per_launch": flops_gemm, "products": PRODUCTS[form],
            "other": {k: {"avg_ms": round(v_["avg_ms"], 4), "tflops": round(v_["tflops"], 2)}
                      for k, v_ in kern.items() if k != dom}}


PEAK_HBM_GBS = 8000.0
SWEEP_RANKS = {"f32": [8, 16, 32, 64, 128, 256], "bf16": [16, 32, 64, 128, 256, 512]}


def run_sweep(args):
    """The two products alone on an N x M O (i.i.d. Gaussian values; the
    kernels' work does not depend on them), for each rank of SWEEP_RANKS:
    the kernel time (HIP events around each product launch, read back from
    the library), its algorithmic bytes and flops, and the fraction of the
    roofline it reaches, roofline time = max(bytes / HBM peak, flops / MFMA
    peak).  Algorithmic bytes of a product: one read of O, one of the skinny
    operand, one write of the output (FP32)."""
    import torch

    from paper_2512_05749_amd import Wssr

    n, m = args.sweep_n, args.sweep_m
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    gen = torch.Generator(device=dev).manual_seed(11)
    rows = []
    for form in ("f32", "bf16"):
        dt = torch.float32 if form == "f32" else torch.bfloat16
        o = torch.randn(n, m, device=dev, dtype=dt, generator=gen)
        b_o = 4 if form == "f32" else 2
        peak = PEAK_FP32_TFLOPS if form == "f32" else PEAK_BF16_TFLOPS
        for r in SWEEP_RANKS[form]:
            h = Wssr(n_max=n, m_max=m, r_max=r, q_max=2, device=dev, dtype=form)
            v = torch.randn(m, r, device=dev, dtype=torch.float32, generator=gen)
            x = torch.randn(n, r, device=dev, dtype=torch.float32, generator=gen)
            h.sample_side(o, v)
            h.param_side(o, x)
            torch.cuda.synchronize()
            h.profile(True)
            for _ in range(3):
                h.sample_side(o, v)
                h.param_side(o, x)
            torch.cuda.synchronize()
            prof = h.profile_read()
            h.profile(False)
            h.close()
            del v, x
            flops = 2.0 * n * m * r
            for side in ("sample_side", "param_side"):
                ms_, cnt = prof[side]
                avg = ms_ / max(cnt, 1)
                nbytes = n * m * b_o + 4.0 * (m * r + n * r)
                t_hbm, t_mfma = nbytes / (PEAK_HBM_GBS * 1e9), flops / (peak * 1e12)
                bound = "hbm" if t_hbm >= t_mfma else "mfma"
                row = {"form": form, "r": r, "side": side, "kernel": product_kernel(form, side, type("C", (), {"m": m, "r": r})),
                       "tile_cols": column_tile(form, r, side),
                       "ms": round(avg, 4), "GB/s": round(nbytes / (avg * 1e-3) / 1e9, 1),
                       "TFLOP/s": round(flops / (avg * 1e-3) / 1e12, 1), "bound": bound,
                       "frac_of_bound": round(max(t_hbm, t_mfma) / (avg * 1e-3), 4)}
                rows.append(row)
                log(f"[sweep] {row}")
        del o
        torch.cuda.empty_cache()
    print(json.dumps({"sweep": "product kernels alone", "n": n, "m": m, "peaks": {"hbm_GBs": PEAK_HBM_GBS,
                      "fp32_TFs": PEAK_FP32_TFLOPS, "bf16_TFs": PEAK_BF16_TFLOPS}, "rows": rows}))


def run_batched(args):
    """The batched form: 16 uneven problems (workloads.batch_configs) in one
    wssr_step_batched call per step, lanes picked by the autotuner; beside it,
    the same problems one after another on a single stream."""
    import numpy as np
    import torch

    from paper_2512_05749_amd import Wssr
    from workloads import Workload, batch_configs

    cfgs = batch_configs()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t0 = time.time()
    probs = []
    for c in cfgs:
        wl = Workload(c, device=dev, gen_dtype=torch.float32)
        probs.append(dict(O=wl.o(1), e_l=wl.e_l(1), V=wl.v0(), lam=c.lam, q=8))
        del wl
        torch.cuda.empty_cache()
    torch.cuda.synchronize()
    count = len(probs)
    log(f"generated {count} problems ({sum(c.n * c.m for c in cfgs) * 4 / 1e9:.1f} GB of O) in "
        f"{time.time() - t0:.1f}s")
    nmax, mmax, rmax = max(c.n for c in cfgs), max(c.m for c in cfgs), max(c.r for c in cfgs)
    stream = torch.cuda.current_stream(dev)

    def timed_batches(h, k):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        e0.record(stream)
        for _ in range(k):
            h.step_batched(probs)
        e1.record(stream)
        torch.cuda.synchronize()
        codes = h.batched_status(count)
        if any(c < 0 for c in codes):
            raise SystemExit(f"batched step failed: {codes}")
        return (time.perf_counter() - w0) * 1e3 / k, e0.elapsed_time(e1) / k

    h = Wssr(n_max=nmax, m_max=mmax, r_max=rmax, q_max=8, device=dev, lanes=args.lanes)
    c0 = time.perf_counter()
    h.step_batched(probs)                    # step 1: cold start, 8 passes
    torch.cuda.synchronize()
    cold_ms = (time.perf_counter() - c0) * 1e3
    log(f"cold batched step (q=8): {cold_ms:.1f} ms, status {h.batched_status(count)}")
    for p in probs:
        p["q"] = 2
    tl, td, tms = h.tune_batched(probs, reps=1)
    log(f"autotuner: {tl} lanes, split sized for slots/{td}, {tms:.1f} ms per batch")
    for _ in range(args.warmup):
        h.step_batched(probs)
    ms_wall, ms_ev = timed_batches(h, args.steps)
    log(f"batched: {ms_wall:.2f} ms per batched step (wall), {ms_ev:.2f} ms (events)")
    h.close()
    hs = Wssr(n_max=nmax, m_max=mmax, r_max=rmax, q_max=8, device=dev, lanes=0)
    hs.step_batched(probs)
    seq_wall, seq_ev = timed_batches(hs, args.steps)
    hs.close()
    log(f"one after another: {seq_wall:.2f} ms per batched step")
    flops = sum(4.0 * c.q * c.n * c.m * c.r for c in cfgs)      # the products of one batched step
    achieved = flops / (ms_wall * 1e-3) / 1e12
    out = {
        "metric": METRIC,
        "value": round(count * 1e3 / ms_wall, 3),
        "unit": "SR steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_wall, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"batch16_mixed: {count} independent FP32 WSSR problems per batched step, "
                               f"N in {{2048..16384}}, M in [2e4, 4e5], r in {{64, 128, 256}}, q=2, "
                               f"lambda log-uniform [1e-4, 1e-2]",
                   "problems": [dict(n=c.n, m=c.m, r=c.r, lam=round(c.lam, 6), a=round(c.alpha, 3)) for c in cfgs],
                   "lanes": args.lanes},
        "value_note": "problem steps per second (problems x batched steps / s); ms_per_step is per batched step",
        "cold_step_ms": round(cold_ms, 3),
        "autotuner": {"lanes": tl, "split_divisor": td, "ms": round(tms, 3)},
        "one_after_another": {"ms_per_step": round(seq_wall, 4), "value": round(count * 1e3 / seq_wall, 3)},
        "vs_one_after_another": round(seq_wall / ms_wall, 3),
        "roofline": {"bound": "mfma", "achieved": round(achieved, 2), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_FP32_TFLOPS, 4), "traffic": None,
                     "kernel": "all product kernels of the batch over the whole batched step",
                     "flops_per_launch": flops},
    }
    print(json.dumps(out), flush=True)


def env_info(dev):
    """ROCm version, gfx target and current clocks (best effort)."""
    import subprocess

    import torch
    info = {"gfx": torch.cuda.get_device_properties(dev).gcnArchName, "torch": torch.__version__}
    try:
        info["rocm"] = open("/opt/rocm/.info/version").read().strip()
    except OSError:
        info["rocm"] = None
    if any(k.startswith("ROCPROF") for k in os.environ):
        # under the profiler the query's own interpreter start is refused
        info["clocks"] = None
        return info
    try:
        res = subprocess.run(["rocm-smi", "--showclocks", "--json"], capture_output=True, text=True, timeout=20)
        js = json.loads(res.stdout) if res.returncode == 0 else {}
        card = next(iter(js.values()), {}) if js else {}
        info["clocks"] = {k: v for k, v in card.items() if "clock" in k.lower() and ("sclk" in k or "mclk" in k
                                                                                   or "fclk" in k)}
    except Exception:
        info["clocks"] = None
    return info


# form and FP32 comparison of each workload: the precision-form instance runs
# its single-product BF16 form beside FP32 on the same instance; the largest
# instance runs BF16 with the split correction, beside FP32 at M = 2e6 (its
# FP32 O at the full M would be 262 GB)
DEFAULT_FORM = {"bf16_n16384_m1m_r512": "bf16", "bf16_n16384_m4m_r512_q3": "bf16_split"}
COMPARE_F32_M = {"bf16_n16384_m1m_r512": 0, "bf16_n16384_m4m_r512_q3": 2_000_000}


def oracle_cols(args, cfg):
    """Columns of the oracle's sample: about 10-30 s of oracle work on the
    box's cores."""
    n, m, r, q = cfg.n, cfg.m, cfg.r, cfg.q
    return args.cpu_cols or min(m, max(4 * r, m // 8, 1), max(4 * r, int(1.3e12 / (8.0 * n * r * q))))


def generate(h, cfg, form, ring, dev, args, sample_cols=0):
    """Draw `ring` steps' inputs of cfg into HBM.  FP32: O itself.  BF16
    forms: the library's ingest stores each FP32 row block in the form and
    forms g from the unrounded values (the FP32 matrix is never held whole).
    Returns O list, E_L list, g list (None for FP32), V_0, the first columns
    of step 1's unrounded O (for the oracle's sample), and the ingest time."""
    import torch

    from workloads import Workload
    t0 = time.time()
    os_, es, gs = [], [], []
    sample = None
    ingest_ms = 0.0
    stream = torch.cuda.current_stream(dev)
    if args.plain_inputs:
        gen = torch.Generator(device=dev).manual_seed(cfg.seed)

        def blocks(t):
            rows = max(64, min(cfg.n, (1 << 30) // cfg.m))
            for i in range(0, cfg.n, rows):
                yield i, torch.randn(min(rows, cfg.n - i), cfg.m, generator=gen, device=dev)
        el = lambda t: cfg.el_mean + cfg.el_std * torch.randn(cfg.n, generator=gen, device=dev,  # noqa: E731
                                                              dtype=torch.float64)
        v0 = lambda: torch.randn(cfg.m, cfg.r, generator=gen, device=dev) / math.sqrt(cfg.m)  # noqa: E731
        wl = None
    else:
        wl = Workload(cfg, device=dev, gen_dtype=torch.float32)
        blocks, el, v0 = wl.o_blocks, wl.e_l, wl.v0
    for t in range(1, ring + 1):
        e = el(t)
        es.append(e)
        if form == "f32":
            o = torch.empty(cfg.n, cfg.m, dtype=torch.float32, device=dev)
            for i, blk in blocks(t):
                o[i:i + blk.shape[0]] = blk
            os_.append(o)
            if t == 1 and sample_cols:
                sample = o[:, :sample_cols].clone()
            gs = None
            continue
        st = h.storage_like(cfg.n, cfg.m)
        g = torch.empty(cfg.m, dtype=torch.float64, device=dev)
        if t == 1 and sample_cols:
            sample = torch.empty(cfg.n, sample_cols, dtype=torch.float32, device=dev)
        for i, blk in blocks(t):
            a_, b_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a_.record(stream)
            h.ingest(blk, e, i, out=st, g=g)
            b_.record(stream)
            b_.synchronize()
            ingest_ms += a_.elapsed_time(b_)
            if sample is not None and t == 1:
                sample[i:i + blk.shape[0]] = blk[:, :sample_cols]
            del blk
        code, _ = h.status()
        if code != 0:
            raise SystemExit(f"ingest of step {t} failed with status {code}")
        os_.append(st)
        gs.append(g)
    v = v0()
    del wl
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    log(f"generated {ring} x O ({cfg.n}x{cfg.m}, form {form}) in {time.time() - t0:.1f}s"
        + (f", ingest {ingest_ms / ring:.1f} ms per O" if form != "f32" else ""))
    return os_, es, gs, v, sample, ingest_ms / ring


def hbm_of(form, prof, cfg, res):
    """Achieved HBM rates: the dominant product kernel (its algorithmic bytes:
    one read of O, one of the skinny operand, one write of its FP32 output),
    and the whole step (2q reads of O plus the skinny traffic of about 24 q M r
    bytes; the BF16 forms make no gradient pass, the FP32 form one)."""
    n, m, r, q = cfg.n, cfg.m, cfg.r, cfg.q
    b_o = 4 if form == "f32" else (4 if form == "bf16x2" else 2)
    per = {}
    for side, (ms, cnt) in prof.items():
        avg = ms / max(cnt, 1)
        nbytes = n * m * b_o + 4.0 * (m * r + n * r) + (4.0 * m * r if side == "param_side" else 8.0 * n * r)
        per[side] = {"GB/s": round(nbytes / (avg * 1e-3) / 1e9, 1), "bytes_per_launch": nbytes}
    step_bytes = 2.0 * q * n * m * b_o + 24.0 * q * m * r + (n * m * b_o if form == "f32" else 0.0)
    return {"kernels": per, "step_GB/s": round(step_bytes / (res["ms_per_step"] * 1e-3) / 1e9, 1),
            "step_bytes": step_bytes, "peak_GB/s": PEAK_HBM_GBS}


def run_single(args, cfg, form, dev, sample_cols=0, ring=0, averaged=0.0, sketch=(), spring=False):
    """Generate, time and release one workload in one form; returns the
    result record, the step-1 sample columns and V (for the accuracy leg)."""
    import torch

    from paper_2512_05749_amd import Wssr
    ring = ring or args.ring or (4 if cfg.n * cfg.m <= (1 << 30) else 1)
    p_max = max([p_ for p_, _ in sketch], default=0)
    h = Wssr(n_max=cfg.n, m_max=cfg.m, r_max=min(512, cfg.r + p_max), q_max=8, device=dev, dtype=form,
             sample_space=spring)
    os_, es, gs, v, sample, ingest_ms = generate(h, cfg, form, ring, dev, args, sample_cols)
    if args.copy_calibration:
        # one elementwise kernel reading and writing exactly copy_calibration MiB
        src = torch.ones(args.copy_calibration << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        log(f"copy calibration: {args.copy_calibration} MiB read + written by one neg kernel")
        del src, dst
    res = time_form(h, form, os_, es, gs, v, cfg, args, dev)
    sk = None
    if sketch:
        sk = [time_sketch(h, form, os_, es, gs, cfg, dev, p_, q_, res["cold_delta"]) for p_, q_ in sketch]
    sp = time_spring(h, form, os_, es, cfg, dev, 0.9, 3) if spring else None
    res_avg = None
    if averaged > 0:
        # the averaged-state step on the same data and handle
        res_avg = time_form(h, form, os_, es, gs, v, cfg, args, dev, avg=averaged)
    h.close()
    e1 = es[0]
    del os_, gs
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    rec = {"value": round(1e3 / res["ms_per_step"], 3), "ms_per_step": round(res["ms_per_step"], 4),
           "step_ms_events": {"median": round(res["median_ms"], 4), "p10": round(res["p10_ms"], 4),
                              "p90": round(res["p90_ms"], 4)},
           "cold_step_ms": round(res["cold_ms"], 3),
           "roofline": roofline_of(form, res["prof"], cfg),
           "hbm": hbm_of(form, res["prof"], cfg, res),
           "diag": res["diag"]}
    if form != "f32":
        rec["ingest_ms_per_O"] = round(ingest_ms, 3)
    if sk:
        rec["sketch_cold_start"] = sk
    if sp:
        rec["spring"] = sp
    if res_avg is not None:
        rec["averaged"] = {"weight": averaged, "value": round(1e3 / res_avg["ms_per_step"], 3),
                           "ms_per_step": round(res_avg["ms_per_step"], 4),
                           "step_ms_events": {"median": round(res_avg["median_ms"], 4),
                                              "p10": round(res_avg["p10_ms"], 4),
                                              "p90": round(res_avg["p90_ms"], 4)},
                           "cold_step_ms": round(res_avg["cold_ms"], 3),
                           "time_vs_plain_step": round(res_avg["ms_per_step"] / res["ms_per_step"], 4),
                           "diag": res_avg["diag"]}
    return rec, sample, e1, res["v"]


def describe(cfg, form):
    return (f"{cfg.name}: WSSR step, O {form}, N={cfg.n} M={cfg.m} r={cfg.r} q={cfg.q} lambda={cfg.lam}, "
            f"spectrum k^-{cfg.alpha}, rotation {cfg.theta}/step")


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU; --gpus above 1 is not supported", file=sys.stderr)
        sys.exit(2)
    if args.sweep:
        return run_sweep(args)
    if args.config == "batch16_mixed":
        args.steps = args.steps or 20
        # the lanes and their second streams need their own hardware queues to
        # run side by side (HIP maps streams onto this many queues; set before
        # the runtime starts)
        os.environ.setdefault("GPU_MAX_HW_QUEUES", str(min(32, 2 * args.lanes + 2)))
        return run_batched(args)
    import dataclasses

    import torch

    from workloads import CONFIGS

    cfg = CONFIGS[args.config]
    if args.m:
        cfg = dataclasses.replace(cfg, m=args.m)
    form = args.form or DEFAULT_FORM.get(cfg.name, "f32")
    steps_default = cfg.steps if cfg.name in DEFAULT_FORM else 20
    if args.steps <= 0:
        args.steps = steps_default
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    cols = oracle_cols(args, cfg) if args.cpu_baseline else 0
    sketch = []
    for item in filter(None, args.sketch.split(";")):
        p_, q_ = (int(x) for x in item.split(","))
        sketch.append((min(p_, 512 - cfg.r), q_))
    rec, sample, e1, v_end = run_single(args, cfg, form, dev, sample_cols=cols, averaged=args.averaged,
                                        sketch=sketch, spring=bool(args.spring) and cfg.n <= 8192)
    out = {
        "metric": METRIC,
        "value": rec["value"],
        "unit": "SR steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": rec["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if form == "f32" else "bf16",
        "data": "synthetic, i.i.d. Gaussian O (counter run)" if args.plain_inputs else "synthetic",
        "config": {"workload": describe(cfg, form), "n": cfg.n, "m": cfg.m, "r": cfg.r, "q": cfg.q,
                   "lambda": cfg.lam, "form": form},
        "cold_step_ms": rec["cold_step_ms"],
        "step_ms_events": rec["step_ms_events"],
        "roofline": rec["roofline"],
        "hbm": rec["hbm"],
    }
    if form != "f32":
        out["ingest_ms_per_O"] = rec["ingest_ms_per_O"]
    if "averaged" in rec:
        out["averaged_state_step"] = rec["averaged"]
    if "sketch_cold_start" in rec:
        out["sketch_cold_start"] = rec["sketch_cold_start"]
    if "spring" in rec:
        out["spring_same_data"] = rec["spring"]
        out["wssr_vs_spring_time"] = round(rec["spring"]["ms_per_step"] / rec["ms_per_step"], 3)
    oracle = OracleSample(args, cfg, sample, e1, v_end[:cols], form, cols) if args.cpu_baseline else None
    del sample, v_end
    torch.cuda.empty_cache()
    # the FP32 form beside it: the same instance, or the same recipe at the M
    # whose FP32 O fits
    if args.compare_f32 == 1:
        cmp_m = cfg.m
    elif args.compare_f32 < 0:
        cmp_m = COMPARE_F32_M.get(cfg.name) or cfg.m
    else:
        cmp_m = 0
    if form != "f32" and cmp_m:
        cfg32 = dataclasses.replace(cfg, m=cmp_m)
        r32, _, _, _ = run_single(args, cfg32, "f32", dev)
        key = "fp32_same_instance" if cmp_m == cfg.m else f"fp32_same_recipe_m{cmp_m}"
        out[key] = {"workload": describe(cfg32, "f32"), **{k: r32[k] for k in
                    ("value", "ms_per_step", "step_ms_events", "cold_step_ms", "roofline", "hbm")}}
        out["vs_fp32"] = {"steps_per_s_ratio": round(rec["value"] / r32["value"], 3),
                          "parameters_per_s_ratio": round(rec["value"] * cfg.m / (r32["value"] * cmp_m), 3)}
    if args.secondary and cfg.name != "f32_n8192_m100k_r256":
        c2 = CONFIGS["f32_n8192_m100k_r256"]
        steps = args.steps
        args.steps = 20
        r2, _, _, _ = run_single(args, c2, "f32", dev, spring=bool(args.spring))
        args.steps = steps
        out["secondary"] = {"f32_n8192_m100k_r256": {"workload": describe(c2, "f32"), "steps": 20,
                                                     **{k: r2[k] for k in ("value", "ms_per_step", "step_ms_events",
                                                                           "roofline", "hbm")}}}
        if "spring" in r2:
            out["secondary"]["f32_n8192_m100k_r256"]["spring_same_data"] = r2["spring"]
            out["secondary"]["f32_n8192_m100k_r256"]["wssr_vs_spring_time"] = round(
                r2["spring"]["ms_per_step"] / r2["ms_per_step"], 3)
    if oracle is not None:
        try:
            out["cpu_baseline"], out["accuracy_vs_oracle"] = oracle.finish()
        except (Exception, SystemExit) as exc:   # the line is printed without them
            log(f"oracle sample failed: {exc!r}")
            out["cpu_baseline"] = {"value": None, "unit": "SR steps/s", "cores": oracle.threads, "kind": "oracle",
                                   "sample": f"the oracle's run on the column sample failed: {exc!r}"}
            out["accuracy_vs_oracle"] = None
    out["env"] = env_info(dev)
    print(json.dumps(out), flush=True)


def _oracle_job(o32, e_np, v32, cols, lam, r, q, threads, queue, wide=1):
    """Child process (spawned, so that it shares nothing with the parent's
    GPU runtime): the FP64 oracle step on the first `cols` columns of the
    sample (the accuracy reference), timed, and when wide > 1 the same step on
    those columns tiled `wide` times (V's rows tiled and scaled by
    1/sqrt(wide), so that every r x r matrix of the step is the sample's up to
    a scale and the Rayleigh-Ritz SVD takes the same sweeps), timed: a second
    point of time against columns that differs from the first only in the
    work that grows with the column count."""
    sys.path.insert(0, ROOT)
    try:
        from threadpoolctl import threadpool_limits
        limiter = threadpool_limits(limits=threads)
    except Exception:
        limiter = None
    import numpy as np

    from oracle import wssr_oracle as orc
    # an untimed small step first: thread pools, first-touch allocations and
    # imports are paid there, not in the first timed point
    nw, mw = min(256, o32.shape[0]), min(2048, cols)
    rw = min(r, 16, nw - 1, mw)
    orc.wssr_step(np.asarray(o32[:nw, :mw], dtype=np.float64), e_np[:nw], np.asarray(v32[:mw, :rw], dtype=np.float64),
                  lam, rw, 1)
    o_np = np.asarray(o32[:, :cols], dtype=np.float64)
    v_np = np.asarray(v32[:cols], dtype=np.float64)
    t0 = time.perf_counter()
    ref = orc.wssr_step(o_np, e_np, v_np, lam, r, q)
    res = {"delta": ref["delta"], "sigma": ref["sigma"], "v": ref["v"], "g": ref["g"],
           "seconds": time.perf_counter() - t0}
    del o_np, v_np, ref
    if wide > 1:
        o2 = np.tile(np.asarray(o32[:, :cols], dtype=np.float64), (1, wide))
        v2 = np.tile(np.asarray(v32[:cols], dtype=np.float64), (wide, 1)) / np.sqrt(wide)
        t0 = time.perf_counter()
        orc.wssr_step(o2, e_np, v2, lam, r, q)
        res["seconds_wide"] = time.perf_counter() - t0
        del o2, v2
    queue.put(res)
    del limiter


class OracleSample:
    """The accuracy leg and the CPU baseline on a column sample of the
    workload: the first `cols` parameters of step 1's unrounded O, the same
    E_L, and the matching rows of the V the timed steps ended with as the warm
    start.  The GPU runs that sample instance in the benchmarked form, the
    way the benchmark feeds it (BF16 forms: the library's ingest of the FP32
    sample, then the step with the ingested g).  The FP64 oracle then runs in
    child processes on the host cores while the GPU goes on with other work:
    on the unrounded O (the end-to-end error of the form, where the BF16 bar
    applies) and, for the BF16 forms, on the values O holds in storage (the
    implementation error).  The CPU baseline times the oracle on the sample
    and on the sample tiled WIDE times along the columns: the step's time is
    linear in the column count (every stage but the N x r and r x r ones
    grows with M, those do not), and the tiled copy keeps the r x r work the
    same up to scale (the same Rayleigh-Ritz sweeps, whose count varies with
    the data and would otherwise swamp the difference), so the two points
    give the time of a full step, a + b M."""

    WIDE = 5

    def __init__(self, args, cfg, o_sample, e_dev, v_sample, form, cols):
        import multiprocessing as mp

        from paper_2512_05749_amd import Wssr
        from workloads import stored_values

        self.cfg, self.form = cfg, form
        n, r, q, lam = cfg.n, cfg.r, cfg.q, cfg.lam
        self.cols = cols
        self.cols_wide = self.WIDE * cols
        o32 = o_sample.cpu().numpy()
        e_np = e_dev.cpu().numpy()
        v32 = v_sample.cpu().numpy()
        o_acc = o_sample[:, :cols].contiguous()
        hs = Wssr(n_max=n, m_max=cols, r_max=r, q_max=q, dtype=form)
        vv = v_sample[:cols].clone().contiguous()
        stored = None
        if form == "f32":
            d, s_ = hs.step(o_acc, e_dev, vv, lam, q=q)
        else:
            st = hs.storage_like(n, cols)
            g, _ = hs.ingest(o_acc, e_dev, 0, out=st)
            d, s_ = hs.step(st, None, vv, lam, q=q, g=g)
            stored = stored_values(st).float().cpu().numpy()
        self.code, _ = hs.status()
        hs.close()
        del o_acc
        self.d, self.s, self.v = d.cpu().numpy(), s_.cpu().numpy(), vv.double().cpu().numpy()
        ncpu = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        # the timed run gets most of the cores; the second one little (its
        # time is not reported)
        self.threads = max(1, ncpu - 2) if stored is not None else ncpu
        ctx = mp.get_context("spawn")
        self.q_main, self.q_stored = ctx.Queue(), ctx.Queue()
        # daemon children: a run given up on ends with the benchmark
        self.p_main = ctx.Process(daemon=True, target=_oracle_job,
                                  args=(o32, e_np, v32, cols, lam, r, q, self.threads, self.q_main, self.WIDE))
        self.p_main.start()
        self.p_stored = None
        if stored is not None:
            # the stored values are exact in FP32 (BF16, or the sum of two
            # BF16 planes, which FP32 holds to the plane's 17 bits)
            self.p_stored = ctx.Process(daemon=True, target=_oracle_job,
                                        args=(stored, e_np, v32[:cols], cols, lam, r, q,
                                              max(1, ncpu - self.threads), self.q_stored))
            self.p_stored.start()
        log(f"oracle on {n}x{cols} and {n}x{self.cols_wide} column samples started ({self.threads} threads)")

    WAIT_LIMIT_S = 420.0   # after the GPU legs; a slower host gives no CPU baseline rather than no line

    @classmethod
    def _wait(cls, queue, proc):
        import queue as _q
        t0 = time.time()
        while True:
            try:
                res = queue.get(timeout=30)
                break
            except _q.Empty:
                if not proc.is_alive():
                    raise RuntimeError("oracle process ended without a result")
                if time.time() - t0 > cls.WAIT_LIMIT_S:
                    proc.terminate()
                    proc.join()
                    raise RuntimeError(f"oracle sample not done after {cls.WAIT_LIMIT_S:.0f}s")
                log(f"waiting for the oracle ({time.time() - t0:.0f}s)")
        proc.join()
        return res

    def finish(self):
        import numpy as np

        from tests.metrics import orth_err, rel, sigma_rel_gated
        cfg, form = self.cfg, self.form
        lam = cfg.lam
        ref = self._wait(self.q_main, self.p_main)
        dt = ref["seconds"]
        dt2 = ref.get("seconds_wide", dt)
        # time against columns through the two points; where they do not
        # separate the column-linear part from the run-to-run noise of the
        # r x r part (the wider sample no slower), the longer of the two
        # sample times is reported, a lower bound on the full step's time
        b = (dt2 - dt) / (self.cols_wide - self.cols) if self.cols_wide > self.cols else 0.0
        a = dt - b * self.cols
        fit = b > 0 and a >= 0
        full_s = a + b * cfg.m if fit else max(dt, dt2)
        log(f"oracle sample steps {dt:.1f}s ({self.cols} columns), {dt2:.1f}s ({self.cols_wide} columns) -> "
            f"{full_s:.1f}s per full step")
        err = {"delta_rel_err": rel(self.d, ref["delta"]),
               "delta_max_err_rel_to_max": float(np.abs(self.d - ref["delta"]).max() / np.abs(ref["delta"]).max()),
               "sigma_rel_err_gated": sigma_rel_gated(self.s, ref["sigma"], lam)}
        acc = {"sample": f"N={cfg.n}, first {self.cols} of M={cfg.m} columns, warm start = matching rows of the "
                         f"timed steps' V", "status": self.code, "form": form, "v_orth_err": orth_err(self.v)}
        if form == "f32":
            acc.update(err)
        else:
            acc["vs_unrounded_O"] = err
            try:
                ref_s = self._wait(self.q_stored, self.p_stored)
            except RuntimeError as exc:
                log(f"oracle on the stored values: {exc}")
                ref_s = None
            if ref_s is None:
                acc["vs_stored_O"] = None
            else:
                # the oracle's subspace and singular values on the stored
                # values, applied to the gradient of the unrounded O (the one
                # the library's ingest forms): the implementation error of the
                # BF16 path
                from oracle import wssr_oracle as orc
                d_s = orc.woodbury_apply(ref_s["v"], ref_s["sigma"], ref["g"], lam)
                acc["vs_stored_O"] = {"delta_rel_err": rel(self.d, d_s),
                                      "sigma_rel_err_gated": sigma_rel_gated(self.s, ref_s["sigma"], lam),
                                      "gradient": "of the unrounded O in both"}
        log(f"accuracy on the sample: {acc}")
        base = {"value": round(1.0 / full_s, 6), "unit": "SR steps/s", "cores": self.threads, "kind": "oracle",
                "sample": (f"one step of the FP64 oracle (r={cfg.r}, q={cfg.q}) on N={cfg.n} x {self.cols} columns "
                           f"of M={cfg.m}: {dt:.2f}s, and on those columns tiled {self.WIDE} times "
                           f"({self.cols_wide} columns): {dt2:.2f}s; "
                           + (f"a full step from the line through the two points, {a:.1f}s + {b * 1e3:.3f}ms "
                              f"per column" if fit else "the two points do not separate the per-column part from "
                              "the noise; the longer sample time is reported, a lower bound on a full step"))}
        return base, acc


if __name__ == "__main__":
    main()
