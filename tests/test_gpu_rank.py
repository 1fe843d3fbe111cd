"""Adaptive rank (Sec. 4.3, eq. ruler; wssr_set_rank_ratio / wssr_rank_info)
and Alg. 1's own diag(R) ending (WSSR_DIAGR_EXTRACT) through the C ABI,
against the FP64 oracle: the truncated direction in both preconditioner
forms, the reported rank and growth flag, a growth loop over steps with the
warm start padded, and the diag(R) ending at one and several passes."""
import numpy as np
import pytest
import torch

from oracle import wssr_oracle as orc
from tests.metrics import rel, sigma_rel_gated
from workloads import Config, Workload, random_problem

pytestmark = pytest.mark.gpu

TOL = 1e-4


def _np(t):
    return t.detach().double().cpu().numpy()


def _ratio_between(sigma, k):
    """A ratio halfway (geometrically) between sigma_k^2/sigma_1^2 and
    sigma_{k+1}^2/sigma_1^2 (1-based k), so that the ruler keeps exactly k."""
    s2 = np.asarray(sigma) ** 2 / sigma[0] ** 2
    return float(np.sqrt(s2[k - 1] * s2[k]))


@pytest.mark.parametrize("floor", [False, True])
@pytest.mark.parametrize("keep", [5, 20])
def test_rank_ratio_truncation(floor, keep):
    from paper_2512_05749_amd import Wssr
    n, m, r, q, lam = 800, 3001, 32, 3, 1e-3
    o, e, v = random_problem(n, m, r, seed=11 + keep, device="cuda", alpha=1.0)
    pre = "floor" if floor else "damped"
    ref0 = orc.wssr_step(_np(o), _np(e), _np(v), lam, r, q, precond=pre)
    r_reg = _ratio_between(ref0["sigma"], keep)
    ref = orc.wssr_step(_np(o), _np(e), _np(v), lam, r, q, precond=pre, r_reg=r_reg)
    assert ref["r_eff"] == keep
    h = Wssr(n_max=n, m_max=m, r_max=r, q_max=4, floor_precond=floor)
    try:
        h.set_rank_ratio(r_reg)
        delta, sigma = h.step(o, e, v, lam, q=q)
        assert h.status()[0] == 0
        r_eff, grow = h.rank_info()
        assert (r_eff, grow) == (keep, False)
        d_err = rel(_np(delta), ref["delta"])
        print(f"keep {keep} floor {floor}: delta {d_err:.2e}")
        assert d_err <= TOL
        assert sigma_rel_gated(_np(sigma), ref["sigma"], lam) <= TOL
        h.set_rank_ratio(0.0)
        h.step(o, e, torch.tensor(_np(v), dtype=torch.float32, device="cuda"), lam, q=q)
        assert h.rank_info() == (r, True)
    finally:
        h.close()


def test_rank_growth_loop():
    """Alg. 2's growth: r_max starts at 8 and grows by half while the last
    computed column passes r_reg; each step (warm start padded with new
    columns) matches the oracle given the same V_in and ratio."""
    from paper_2512_05749_amd import Wssr
    from paper_2512_05749_amd.wssr import AdaptiveRank
    cfg = Config("grow", n=1024, m=4000, r=8, q=2, lam=1e-3, steps=5, alpha=0.8, theta=0.01, eta=1e-3,
                 el_mean=-1.0, el_std=0.1, seed=21)
    wl = Workload(cfg, device="cuda")
    h = Wssr(n_max=cfg.n, m_max=cfg.m, r_max=64, q_max=8)
    try:
        ar = AdaptiveRank(h, 8, 2e-3, 0.5, 64)
        v = wl.v0(8)
        gen = torch.Generator(device="cuda").manual_seed(5)
        ranks = []
        for t in range(1, cfg.steps + 1):
            (v,) = ar.grow_basis(v, gen)
            o, e = wl.o(t), wl.e_l(t)
            v_in = v.clone()
            qq = 8 if t == 1 else cfg.q
            delta, sigma = h.step(o, e, v, cfg.lam, q=qq)
            assert h.status()[0] == 0
            r_now = v.shape[1]
            r_eff = ar.after_step()
            ref = orc.wssr_step(_np(o), _np(e), _np(v_in), cfg.lam, r_now, qq, r_reg=2e-3)
            assert r_eff == ref["r_eff"]
            assert rel(_np(delta), ref["delta"]) <= TOL
            ranks.append((r_now, r_eff))
        print("r_max, r_eff per step:", ranks)
        assert ranks[-1][0] > 8                       # r_max grew
    finally:
        h.close()


@pytest.mark.parametrize("q", [1, 3])
def test_diag_extraction(q):
    from paper_2512_05749_amd import Wssr
    n, m, r, lam = 700, 3001, 24, 1e-3
    o, e, v = random_problem(n, m, r, seed=31 + q, device="cuda", alpha=1.2)
    v_in = v.clone()
    h = Wssr(n_max=n, m_max=m, r_max=r, q_max=4, diag_extract=True)
    try:
        delta, sigma = h.step(o, e, v, lam, q=q)
        assert h.status()[0] == 0
        ref = orc.wssr_step(_np(o), _np(e), _np(v_in), lam, r, q, extract="diag")
        d_err = rel(_np(delta), ref["delta"])
        s_err = float(np.abs(_np(sigma) - ref["sigma"]).max() / ref["sigma"][0])
        v_err = float(np.abs(_np(v) - ref["v"]).max())
        print(f"q={q}: delta {d_err:.2e} sigma {s_err:.2e} V {v_err:.2e}")
        assert d_err <= TOL and s_err <= 1e-5 and v_err <= 1e-4
        assert np.all(np.diff(_np(sigma)) <= 0)
        # the averaged step needs the Rayleigh-Ritz ending
        from paper_2512_05749_amd.wssr import WssrError
        z = torch.zeros(r, dtype=torch.float64, device="cuda")
        with pytest.raises(WssrError):
            h.step_avg(o, e, v, lam, 0.5, z, z.clone(), q=q)
    finally:
        h.close()
