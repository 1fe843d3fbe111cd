"""The benchmark workload at its full size (N=8192 samples, M=100000 parameters,
r=256, q=2, lambda=1e-3), in the launch configuration the benchmark times:
one warm-started step on the GPU against the FP64 oracle given the same inputs
(the whole step, not a sample of it; the oracle takes about half a minute)."""
import numpy as np
import pytest
import torch

from oracle import wssr_oracle as orc
from tests.metrics import orth_err, rel, sigma_rel_gated, weighted_projector_err
from workloads import CONFIGS, Workload

pytestmark = pytest.mark.gpu


def _np(t):
    return t.detach().double().cpu().numpy()


@pytest.mark.timeout(900)
def test_benchmark_workload_full_size():
    from paper_2512_05749_amd import Wssr
    cfg = CONFIGS["f32_n8192_m100k_r256"]
    wl = Workload(cfg, device="cuda", gen_dtype=torch.float32)
    h = Wssr(n_max=cfg.n, m_max=cfg.m, r_max=cfg.r, q_max=8)
    try:
        # step 1 (cold, 8 passes) gives the warm start of step 2
        v = wl.v0()
        h.step(wl.o(1), wl.e_l(1), v, cfg.lam, q=8)
        assert h.status()[0] == 0
        o, e = wl.o(2), wl.e_l(2)
        v_in = v.clone()
        delta, sigma = h.step(o, e, v, cfg.lam, q=cfg.q)
        code, diag = h.status()
        assert code == 0, diag
    finally:
        h.close()
    o_np, e_np, vin_np = _np(o), _np(e), _np(v_in)
    del o
    torch.cuda.empty_cache()
    ref = orc.wssr_step(o_np, e_np, vin_np, cfg.lam, cfg.r, cfg.q)
    d_err = rel(_np(delta), ref["delta"])
    s_err = sigma_rel_gated(_np(sigma), ref["sigma"], cfg.lam)
    w_g = orc.woodbury_weights(_np(sigma), cfg.lam)
    w_o = orc.woodbury_weights(ref["sigma"], cfg.lam)
    wp = weighted_projector_err(_np(v), w_g, ref["v"], w_o)
    print(f"full size: delta rel err {d_err:.2e}, sigma {s_err:.2e}, weighted projector {wp:.2e}", flush=True)
    assert d_err <= 1e-4
    assert s_err <= 1e-4
    assert orth_err(_np(v)) <= 1e-5
    assert wp <= 1e-4
    # signs follow the rule wherever the inner product with V_in is clear
    ip = np.sum(ref["v"] * vin_np, axis=0)
    clear = np.abs(ip) > 1e-3
    assert np.all(np.sum(_np(v) * ref["v"], axis=0)[clear] > 0)
