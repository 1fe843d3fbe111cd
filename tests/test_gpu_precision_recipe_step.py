"""Whole steps on the precision-form recipe (spectrum k^-1.0 plus 1e-4 noise,
rotation 0.01 per step, E_L ~ N(-10, 0.5^2), lambda = 1e-3, r = 512, q = 2)
with N = 16384 samples and M = 8192 parameters (the recipe with a column
count the oracle can run), against the FP64 oracle on the unrounded O: the
FP32 form, and the three BF16 forms fed the way the benchmark feeds them (the
library's ingest of the FP32 rows, then the step with the ingested
gradient).  The warm start is the FP32 form's 8-pass step on the previous
O."""
import numpy as np
import pytest
import torch

from oracle import wssr_oracle as orc
from tests.metrics import orth_err, rel, sigma_rel_gated
from workloads import Config, Workload

pytestmark = pytest.mark.gpu

N, M, R, Q, LAM = 16384, 8192, 512, 2, 1e-3
# FP32 at its bars; BF16 storage of O at the BF16 bar; the two-plane form
# holds O to about 2^-17
TOL = {"f32": 1e-4, "bf16": 1e-2, "bf16_split": 1e-2, "bf16x2": 1e-3}


def _np(t):
    return t.detach().double().cpu().numpy()


@pytest.mark.timeout(900)
def test_precision_recipe_step_all_forms():
    from paper_2512_05749_amd import Wssr
    cfg = Config("precision_recipe_m8192", n=N, m=M, r=R, q=Q, lam=LAM, steps=2, alpha=1.0, theta=0.01,
                 eta=1e-4, el_mean=-10.0, el_std=0.5, seed=3, k=4096)
    wl = Workload(cfg, device="cuda", gen_dtype=torch.float32)
    o0, e0, o1, e1 = wl.o(0), wl.e_l(0), wl.o(1), wl.e_l(1)
    v = wl.v0()
    h = Wssr(n_max=N, m_max=M, r_max=R, q_max=8)
    h.step(o0, e0, v, LAM, q=8)
    assert h.status()[0] == 0
    h.close()
    v_in = v.clone()
    print("warm start done; oracle ...", flush=True)
    ref = orc.wssr_step(_np(o1), _np(e1), _np(v_in), LAM, R, Q)
    print("oracle done", flush=True)
    for form in ("f32", "bf16", "bf16_split", "bf16x2"):
        h = Wssr(n_max=N, m_max=M, r_max=R, q_max=Q, dtype=form)
        try:
            vv = v_in.clone()
            if form == "f32":
                delta, sigma = h.step(o1, e1, vv, LAM, q=Q)
            else:
                stored = h.storage_like(N, M)
                g, _ = h.ingest(o1, e1, 0, out=stored)
                delta, sigma = h.step(stored, None, vv, LAM, q=Q, g=g)
            code, diag = h.status()
        finally:
            h.close()
        assert code == 0, (form, diag)
        d_err = rel(_np(delta), ref["delta"])
        d_max = float(np.abs(_np(delta) - ref["delta"]).max() / np.abs(ref["delta"]).max())
        s_err = sigma_rel_gated(_np(sigma), ref["sigma"], LAM)
        print(f"{form}: delta rel {d_err:.2e} (element-wise {d_max:.2e}), sigma {s_err:.2e}", flush=True)
        assert d_err <= TOL[form], form
        assert d_max <= TOL[form], form
        assert s_err <= TOL[form], form
        assert orth_err(_np(vv)) <= 1e-5, form
