"""The averaged-state step (wssr_step_avg through the C ABI) against the FP64
oracle's averaged_step (Sec. 4.1): chains of steps from the zero state over a
drifting subspace, each step teacher-forced (the oracle gets the GPU's input
state), on ragged shapes that span several tiles of every kernel; weight 0
against the plain step; the BF16 split form with the ingest gradient against
the oracle on the unrounded O."""
import numpy as np
import pytest
import torch

from oracle import wssr_oracle as orc
from tests.metrics import orth_err, rel, sigma_rel_gated, weighted_projector_err
from workloads import Config, Workload

pytestmark = pytest.mark.gpu

# FP32 form: the bars of the plain step (delta, gated sigma 1e-4, V
# orthonormal to 1e-5); the stored pair enters through Obar L = V (sigma o l),
# which does not depend on rotations inside clusters of equal singular values.
TOL = 1e-4


def _np(t):
    return t.detach().double().cpu().numpy()


def _max_rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.abs(a - b).max() / np.abs(b).max())


def _workload(n, m, r, seed, alpha=1.1, theta=0.01, steps=4):
    cfg = Config("avg", n=n, m=m, r=r, q=2, lam=1e-3, steps=steps, alpha=alpha, theta=theta, eta=1e-3,
                 el_mean=-1.0, el_std=0.1, seed=seed)
    return cfg, Workload(cfg, device="cuda")


def _check(res, o, e, v_in, state, lam, r, q, avg, delta, v_out, sig_out, l_out, g_bar, tol):
    ref = orc.averaged_step(_np(o), _np(e), _np(v_in), state, lam, r, q, avg)
    d_err, d_max = rel(_np(delta), ref["delta"]), _max_rel(_np(delta), ref["delta"])
    s_err = sigma_rel_gated(_np(sig_out), ref["sigma"], lam)
    w_g = orc.woodbury_weights(_np(sig_out), lam)
    w_o = orc.woodbury_weights(ref["sigma"], lam)
    wp = weighted_projector_err(_np(v_out), w_g, ref["v"], w_o)
    ol_g = _np(v_out) @ (_np(sig_out) * _np(l_out))
    ol_o = ref["v"] @ (ref["sigma"] * ref["l"])
    ol_err = rel(ol_g, ol_o)
    gb_err = rel(_np(g_bar), ref["gbar"])
    res.append((d_err, d_max, s_err, wp, ol_err, gb_err))
    assert d_err <= tol and d_max <= tol, (d_err, d_max, s_err, wp, ol_err)
    assert s_err <= tol, s_err
    assert wp <= tol, wp
    assert ol_err <= tol, ol_err
    assert gb_err <= 1e-10, gb_err
    assert orth_err(_np(v_out)) <= 1e-5


@pytest.mark.parametrize("n,m,r,q,avg", [(700, 3001, 24, 3, 0.5), (1000, 5003, 130, 2, 0.95),
                                         (257, 1001, 7, 2, 0.9), (2048, 4096, 192, 2, 0.8)])
def test_averaged_chain_against_oracle(n, m, r, q, avg):
    from paper_2512_05749_amd import Wssr
    cfg, wl = _workload(n, m, r, seed=n + r)
    lam = cfg.lam
    h = Wssr(n_max=n, m_max=m, r_max=r, q_max=8)
    try:
        v = wl.v0()
        sig = torch.zeros(r, dtype=torch.float64, device="cuda")
        l = torch.zeros(r, dtype=torch.float64, device="cuda")
        g_bar = torch.empty(m, dtype=torch.float64, device="cuda")
        res = []
        for t in range(1, cfg.steps + 1):
            o, e = wl.o(t), wl.e_l(t)
            qq = 8 if t == 1 else q
            v_in = v.clone()
            state = None if t == 1 else dict(v=_np(v_in), sigma=_np(sig), l=_np(l))
            delta = h.step_avg(o, e, v, lam, avg, sig, l, q=qq, g_bar=g_bar)
            code, diag = h.status()
            assert code == 0, (t, code, diag)
            _check(res, o, e, v_in, state, lam, r, qq, avg, delta, v, sig, l, g_bar, TOL)
        print(f"n={n} m={m} r={r} avg={avg}: " + "; ".join(
            f"d {a:.1e}/{b:.1e} s {c:.1e} wp {d:.1e} OL {f:.1e}" for a, b, c, d, f, _ in res))
    finally:
        h.close()


def test_averaged_weight_zero_is_the_plain_step():
    """avg = 0: the history rows are zero and the step is wssr_step's, to
    rounding: the sample-side block has r more rows, all zero, which change
    the row chunking of its Gram sums (both are within the FP32 bars of the
    oracle; here they agree to 1e-5)."""
    from paper_2512_05749_amd import Wssr
    n, m, r = 900, 3000, 40
    cfg, wl = _workload(n, m, r, seed=5)
    h = Wssr(n_max=n, m_max=m, r_max=r, q_max=8)
    try:
        o, e = wl.o(2), wl.e_l(2)
        v0 = wl.v0()
        va, vb = v0.clone(), v0.clone()
        sig = torch.rand(r, dtype=torch.float64, device="cuda")    # ignored at weight 0
        l = torch.rand(r, dtype=torch.float64, device="cuda")
        g_bar = torch.empty(m, dtype=torch.float64, device="cuda")
        da = h.step_avg(o, e, va, cfg.lam, 0.0, sig, l, q=3, g_bar=g_bar)
        assert h.status()[0] == 0
        db, sb = h.step(o, e, vb, cfg.lam, q=3)
        assert h.status()[0] == 0
        assert rel(_np(da), _np(db)) < 1e-5
        assert rel(_np(sig), _np(sb)) < 1e-5
        assert float((va - vb).abs().max()) < 1e-4
        g = orc.gradient(_np(o), _np(e))
        assert rel(_np(g_bar), g) < 1e-11
    finally:
        h.close()


def test_averaged_rejects_bad_arguments():
    from paper_2512_05749_amd import Wssr
    from paper_2512_05749_amd.wssr import WssrError
    n, m, r = 200, 500, 8
    _, wl = _workload(n, m, r, seed=9)
    h = Wssr(n_max=n, m_max=m, r_max=r, q_max=2)
    try:
        o, e, v = wl.o(1), wl.e_l(1), wl.v0()
        sig = torch.zeros(r, dtype=torch.float64, device="cuda")
        l = torch.zeros(r, dtype=torch.float64, device="cuda")
        for bad in (-0.1, 1.0, float("nan")):
            with pytest.raises(WssrError):
                h.step_avg(o, e, v, 1e-3, bad, sig, l, q=2)
    finally:
        h.close()


# Against the oracle on the unrounded O: BF16 storage with the gradient of
# the unrounded values (ingest); the recipe of the largest instance (spectrum
# k^-1.3, rotation 0.005, q = 3) at reduced size.
def test_averaged_bf16_split_against_unrounded_O():
    from paper_2512_05749_amd import Wssr
    n, m, r, q, avg = 2048, 8000, 64, 3, 0.9
    cfg, wl = _workload(n, m, r, seed=77, alpha=1.3, theta=0.005)
    h = Wssr(n_max=n, m_max=m, r_max=r, q_max=8, dtype="bf16_split")
    try:
        v = wl.v0()
        sig = torch.zeros(r, dtype=torch.float64, device="cuda")
        l = torch.zeros(r, dtype=torch.float64, device="cuda")
        g_bar = torch.empty(m, dtype=torch.float64, device="cuda")
        stored = h.storage_like(n, m)
        res = []
        for t in range(1, cfg.steps + 1):
            o, e = wl.o(t), wl.e_l(t)
            g, _ = h.ingest(o, e, 0, out=stored)
            qq = 8 if t == 1 else q
            v_in = v.clone()
            state = None if t == 1 else dict(v=_np(v_in), sigma=_np(sig), l=_np(l))
            delta = h.step_avg(stored, e, v, cfg.lam, avg, sig, l, q=qq, g=g, g_bar=g_bar)
            code, diag = h.status()
            assert code == 0, (t, code, diag)
            _check(res, o, e, v_in, state, cfg.lam, r, qq, avg, delta, v, sig, l, g_bar, 1e-2)
        print("bf16_split averaged: " + "; ".join(f"d {a:.1e}/{b:.1e} s {c:.1e} OL {f:.1e}"
                                                   for a, b, c, d, f, _ in res))
    finally:
        h.close()
