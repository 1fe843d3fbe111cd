"""Benchmark: SR steps/s of the warm-started SR step on one MI355X.

Default workload: the FP32 form, N=8192 samples, M=100000 parameters, rank
r=256, q=2 passes, lambda=1e-3, synthetic O with a k^-1.2 spectrum rotating by
0.01 per step (workloads.CONFIGS["f32_n8192_m100k_r256"]).  Inputs are
generated on the GPU and resident in HBM before timing.  A step is one whole
call of wssr_step: centring, gradient, q passes (two products, CholeskyQR2 of
both sides), Rayleigh-Ritz, signs and the Woodbury apply.

--form bf16 | bf16_split | bf16x2 times a BF16 precision form instead
(--config bf16_n16384_m1m_r512 for the precision-form instance), and
--compare-f32 1 times the FP32 form on the same instance beside it.
--config batch16_mixed times the batched form (16 uneven problems per
wssr_step_batched call) beside the same problems run one after another.
--sweep 1 times the two product kernels alone on the precision-form shape
(N=16384, M=1e6) over a range of ranks, FP32 and BF16, and reports each
against both rooflines (HBM and MFMA): the small ranks are memory-bound.

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
    ap.add_argument("--config", default="f32_n8192_m100k_r256",
                    help="workload name (workloads.CONFIGS), or batch16_mixed for the batched form")
    ap.add_argument("--ring", type=int, default=0,
                    help="distinct O_t held in HBM and cycled (0: 4, or 1 above 2^30 elements)")
    ap.add_argument("--form", default="f32", choices=["f32", "bf16", "bf16_split", "bf16x2"],
                    help="storage and product precision of O")
    ap.add_argument("--lanes", type=int, default=4, help="batched workload: concurrent lanes of the handle")
    ap.add_argument("--compare-f32", type=int, default=0,
                    help="also time the FP32 form on the same instance and report the ratio")
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


def time_form(form, o_ring, e_ring, v_start, cfg, args, dev):
    """Cold step, warm-up and timed steps of one precision form; returns the
    timings, the product-kernel profile and the last status."""
    import numpy as np
    import torch

    from paper_2512_05749_amd import Wssr

    n, m, r, q, lam = cfg.n, cfg.m, cfg.r, cfg.q, cfg.lam
    ring = len(o_ring)
    v = v_start.clone()
    h = Wssr(n_max=n, m_max=m, r_max=r, q_max=8, device=dev, dtype=form)
    delta = torch.empty(m, dtype=torch.float64, device=dev)
    sigma = torch.empty(r, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev)

    # step 1: cold start (8 passes from V_0), reported separately
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    h.step(o_ring[0], e_ring[0], v, lam, q=8, delta=delta, sigma=sigma)
    e1.record(stream)
    code, diag = h.status()
    cold_ms = e0.elapsed_time(e1)
    log(f"[{form}] cold step (q=8): {cold_ms:.2f} ms, status {code}, diag {diag}")
    if code < 0:
        raise SystemExit(f"cold step failed with status {code}")

    t = 1
    for _ in range(args.warmup):
        h.step(o_ring[t % ring], e_ring[t % ring], v, lam, q=q, delta=delta, sigma=sigma)
        t += 1
    torch.cuda.synchronize()
    log(f"[{form}] warmup done")

    h.profile(True)
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    for k in range(args.steps):
        starts[k].record(stream)
        h.step(o_ring[t % ring], e_ring[t % ring], v, lam, q=q, delta=delta, sigma=sigma)
        ends[k].record(stream)
        t += 1
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    prof = h.profile_read()
    h.profile(False)
    code, diag = h.status()
    h.close()
    per_step = [s_.elapsed_time(e_) for s_, e_ in zip(starts, ends)]
    ms_per_step = wall * 1e3 / args.steps
    log(f"[{form}] timed {args.steps} steps: {ms_per_step:.3f} ms/step (wall), median event "
        f"{np.median(per_step):.3f} ms, status {code}, diag {diag}")
    if code < 0:
        raise SystemExit(f"timed steps failed with status {code}")
    return dict(ms_per_step=ms_per_step, median_ms=float(np.median(per_step)), cold_ms=cold_ms, prof=prof,
                diag=diag, v=v)


def product_kernel(form, side, cfg):
    """Name of the product kernel the library launches for this form and
    side: the FP32 products take their direct-to-LDS form when the rows of O
    and of the skinny operand are 16-byte aligned (the inputs here are
    contiguous torch tensors, so that is r % 4 == 0, plus M % 4 == 0 on the
    sample side)."""
    if form != "f32":
        # BF16: O's rows are whole 16-byte chunks (8 elements)
        return "k_gemm16_" + side + ("_dma" if cfg.m % 8 == 0 else "")
    aligned = cfg.r % 4 == 0 and (cfg.m % 4 == 0 or side == "param_side")
    if aligned and side == "param_side" and cfg.r <= 32:
        return "k_gemm_param_side_narrow"      # 32-column tile, O staged through registers
    return "k_gemm_" + side + ("_dma" if aligned else "")


def column_tile(form, r, side):
    """Column-tile width of the product kernels for rank r (aligned inputs;
    BF16 with one plane of each operand)."""
    if form == "f32":
        return 32 if r <= 32 else 64 if r <= 64 else 128 if r <= 128 else 256
    if side == "param_side" and r > 256:
        return 256              # two 256-column tiles per row block
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
            "traffic": recorded_traffic(product_kernel(form, dom, cfg)) if form == "f32" else None,
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


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU; --gpus above 1 is not supported", file=sys.stderr)
        sys.exit(2)
    if args.sweep:
        return run_sweep(args)
    if args.config == "batch16_mixed":
        # the lanes and their second streams need their own hardware queues to
        # run side by side (HIP maps streams onto this many queues; set before
        # the runtime starts)
        os.environ.setdefault("GPU_MAX_HW_QUEUES", str(min(32, 2 * args.lanes + 2)))
        return run_batched(args)
    import torch

    from workloads import CONFIGS, Workload, to_storage

    cfg = CONFIGS[args.config]
    if args.m:
        import dataclasses
        cfg = dataclasses.replace(cfg, m=args.m)
    form = args.form
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    ring = args.ring or (4 if cfg.n * cfg.m <= (1 << 30) else 1)
    keep_f32 = form == "f32" or args.compare_f32 or args.cpu_baseline
    t0 = time.time()
    o32, ost, es = [], [], []
    if args.plain_inputs:
        gen = torch.Generator(device=dev).manual_seed(cfg.seed)
        for _ in range(ring):
            o = torch.randn(cfg.n, cfg.m, generator=gen, device=dev)
            es.append(cfg.el_mean + cfg.el_std * torch.randn(cfg.n, generator=gen, device=dev, dtype=torch.float64))
            if form != "f32":
                ost.append(to_storage(o, form))
            o32.append(o if keep_f32 else None)
            del o
        v = torch.randn(cfg.m, cfg.r, generator=gen, device=dev) / math.sqrt(cfg.m)
    else:
        wl = Workload(cfg, device=dev, gen_dtype=torch.float32)
        for t in range(1, ring + 1):
            es.append(wl.e_l(t))
            if form in ("bf16", "bf16_split") and not keep_f32:
                # straight to BF16, block by block (the same rounding as
                # to_storage, without the FP32 copy of O)
                ost.append(wl.o(t, dtype=torch.bfloat16))
                o32.append(None)
                continue
            o = wl.o(t)
            if form != "f32":
                ost.append(to_storage(o, form))
            o32.append(o if keep_f32 else None)
            del o
        v = wl.v0()
        del wl
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    log(f"generated {ring} x O ({cfg.n}x{cfg.m}, form {form}) in {time.time() - t0:.1f}s")
    if args.copy_calibration:
        # one elementwise kernel reading and writing exactly copy_calibration MiB
        src = torch.ones(args.copy_calibration << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        log(f"copy calibration: {args.copy_calibration} MiB read + written by one neg kernel")
        del src, dst

    n, m, r, q, lam = cfg.n, cfg.m, cfg.r, cfg.q, cfg.lam
    res = time_form(form, o32 if form == "f32" else ost, es, v, cfg, args, dev)
    out = {
        "metric": METRIC,
        "value": round(1e3 / res["ms_per_step"], 3),
        "unit": "SR steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(res["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if form == "f32" else "bf16",
        "data": "synthetic, i.i.d. Gaussian O (counter run)" if args.plain_inputs else "synthetic",
        "config": {"workload": f"{cfg.name}: WSSR step, O {form}, N={n} M={m} r={r} q={q} lambda={lam}, "
                               f"spectrum k^-{cfg.alpha}, rotation {cfg.theta}/step",
                   "n": n, "m": m, "r": r, "q": q, "lambda": lam, "form": form},
        "cold_step_ms": round(res["cold_ms"], 3),
        "step_ms_median_events": round(res["median_ms"], 4),
        "roofline": roofline_of(form, res["prof"], cfg),
    }
    if form != "f32" and args.compare_f32:
        ref = time_form("f32", o32, es, v, cfg, args, dev)
        out["fp32_same_instance"] = {"ms_per_step": round(ref["ms_per_step"], 4),
                                     "value": round(1e3 / ref["ms_per_step"], 3),
                                     "roofline": roofline_of("f32", ref["prof"], cfg)}
        out["vs_fp32_same_instance"] = round(ref["ms_per_step"] / res["ms_per_step"], 3)
    if args.cpu_baseline:
        out["cpu_baseline"], acc = cpu_baseline(args, cfg, o32[min(1, ring - 1)], es[min(1, ring - 1)], v, form)
        out["accuracy_vs_oracle"] = acc
    print(json.dumps(out), flush=True)


def cpu_baseline(args, cfg, o_dev, e_dev, v_dev, form="f32"):
    """Time the FP64 oracle on a column sample of the same workload (the first
    `cols` parameters of one step's O, same E_L, the matching rows of V as the
    warm start) and scale the per-step time by M / cols to a full step.  Every
    stage of the step is linear in M except the N x r and r x r ones, which the
    scaling counts M / cols times over, so the reported rate is a slight
    underestimate of the oracle's full-size rate.  The GPU path is run on the
    same sample instance, in the benchmarked precision form, to report its
    errors against the oracle: on the values O holds in storage (the
    implementation error) and, for the BF16 forms, also on the unrounded O
    (the end-to-end error of the form)."""
    import numpy as np
    import torch

    from oracle import wssr_oracle as orc
    from tests.metrics import rel, sigma_rel_gated

    n, m, r, q, lam = cfg.n, cfg.m, cfg.r, cfg.q, cfg.lam
    # about 10-30 s of oracle work on the machine's cores at the benchmark shape
    cols = args.cpu_cols or min(m, max(4 * r, m // 8, 1), max(4 * r, int(1.3e12 / (8.0 * n * r * q))))
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
    from workloads import stored_values, to_storage
    hs = Wssr(n_max=n, m_max=cols, r_max=r, q_max=q, dtype=form)
    o_in = to_storage(o_s, form)
    vv = v_s.clone()
    d, s = hs.step(o_in, e_dev, vv, lam, q=q)
    code, _ = hs.status()
    hs.close()
    acc = {"sample": f"N={n}, first {cols} of M={m} columns, warm start = matching rows of V",
           "status": code, "form": form,
           "delta_rel_err": rel(d.cpu().numpy(), ref["delta"]),
           "sigma_rel_err_gated": sigma_rel_gated(s.cpu().numpy(), ref["sigma"], lam),
           "v_orth_err": float(np.abs(vv.double().cpu().numpy().T @ vv.double().cpu().numpy()
                                      - np.eye(r)).max())}
    if form != "f32":
        # the oracle on the values O holds in storage
        ref_s = orc.wssr_step(stored_values(o_in).cpu().numpy(), e_np, v_np, lam, r, q)
        acc["vs_unrounded_O"] = {"delta_rel_err": acc.pop("delta_rel_err"),
                                 "sigma_rel_err_gated": acc.pop("sigma_rel_err_gated")}
        acc["vs_stored_O"] = {"delta_rel_err": rel(d.cpu().numpy(), ref_s["delta"]),
                              "sigma_rel_err_gated": sigma_rel_gated(s.cpu().numpy(), ref_s["sigma"], lam)}
    log(f"accuracy on the sample: {acc}")
    base = {"value": round(1.0 / full_s, 6), "unit": "SR steps/s", "cores": threads, "kind": "oracle",
            "sample": f"one step of the FP64 oracle on N={n} x {cols} columns (of M={m}), r={r}, q={q}: "
                      f"{dt:.2f}s, scaled by M/{cols} to a full step"}
    return base, acc


if __name__ == "__main__":
    main()
