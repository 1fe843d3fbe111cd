"""The randomized-sketch step (wssr_step_sketch through the C ABI) against the
FP64 oracle's sketch_step (App. A) on the same random block: ragged shapes
that span several tiles, the BF16 split form with the ingest gradient against
the oracle on the unrounded O, a low-rank O where the sketch is exact, the
sketch as the cold start of warm-started steps, and argument errors."""
import numpy as np
import pytest
import torch

from oracle import wssr_oracle as orc
from tests.metrics import orth_err, rel, sigma_rel_gated, weighted_projector_err
from workloads import random_problem

pytestmark = pytest.mark.gpu

TOL = 1e-4      # the FP32 bars of the plain step


def _np(t):
    return t.detach().double().cpu().numpy()


def _max_rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.abs(a - b).max() / np.abs(b).max())


def _omega(n, k, seed):
    gen = torch.Generator(device="cuda").manual_seed(seed)
    return torch.randn(n, k, generator=gen, device="cuda", dtype=torch.float32)


def _check(o, e, omega, lam, r, delta, v, sigma, tol, q=0, o_ref=None, g=None):
    """GPU against the oracle's sketch_step on o_ref (default: o), the
    oracle's V and sigma applied to g when given."""
    ref = orc.sketch_step(_np(o if o_ref is None else o_ref), _np(e), _np(omega), lam, r, q=q)
    if g is not None:
        ref["delta"] = orc.woodbury_apply(ref["v"], ref["sigma"], _np(g), lam)
    d_err, d_max = rel(_np(delta), ref["delta"]), _max_rel(_np(delta), ref["delta"])
    s_err = sigma_rel_gated(_np(sigma), ref["sigma"], lam)
    wp = weighted_projector_err(_np(v), orc.woodbury_weights(_np(sigma), lam), ref["v"],
                                orc.woodbury_weights(ref["sigma"], lam))
    assert d_err <= tol and d_max <= tol, (d_err, d_max, s_err, wp)
    assert s_err <= tol, s_err
    assert wp <= tol, wp
    assert orth_err(_np(v)) <= 1e-5
    # signs: the largest entry of each column is positive, so columns with a
    # clear singular-value gap agree with the oracle's
    s = ref["sigma"]
    gap = np.ones(r, bool)
    gap[1:] &= (s[:-1] - s[1:]) > 1e-3 * s[0]
    gap[:-1] &= (s[:-1] - s[1:]) > 1e-3 * s[0]
    dots = np.sum(_np(v) * ref["v"], axis=0)
    assert np.all(dots[gap] > 0.9), dots[gap].min()
    return d_err, s_err, wp


@pytest.mark.parametrize("n,m,r,p,q", [(700, 3001, 24, 8, 0), (1000, 5003, 120, 10, 0), (257, 1001, 7, 3, 0),
                                       (2048, 4096, 180, 12, 0), (500, 2000, 30, 0, 0), (700, 3001, 24, 8, 2),
                                       (1000, 5003, 120, 10, 1)])
def test_sketch_against_oracle(n, m, r, p, q):
    from paper_2512_05749_amd import Wssr
    o, e, _ = random_problem(n, m, r, seed=3 * n + r, device="cuda", alpha=1.2)
    omega = _omega(n, r + p, seed=n + p)
    h = Wssr(n_max=n, m_max=m, r_max=r + p, q_max=2)
    try:
        v = torch.empty(m, r, dtype=torch.float32, device="cuda")
        delta, sigma = h.step_sketch(o, e, omega, v, 1e-3, q=q)
        code, diag = h.status()
        assert code == 0, (code, diag)
        print(f"n={n} m={m} r={r} p={p} q={q}: delta/sigma/projector",
              _check(o, e, omega, 1e-3, r, delta, v, sigma, TOL, q=q))
    finally:
        h.close()


def test_sketch_exact_for_low_rank_O():
    """O of rank 16 (plus small column means): with r + p = 16 the sketch spans the
    row space and the step equals the oracle's exact rank-r step."""
    from paper_2512_05749_amd import Wssr
    n, m, r, p, k = 600, 2500, 8, 8, 16
    gen = torch.Generator(device="cuda").manual_seed(5)
    u = torch.linalg.qr(torch.randn(n, k, generator=gen, device="cuda", dtype=torch.float64))[0]
    w = torch.linalg.qr(torch.randn(m, k, generator=gen, device="cuda", dtype=torch.float64))[0]
    s = torch.logspace(0, -1.5, k, device="cuda", dtype=torch.float64)
    # column means small against the spread: the implicit centring's FP32
    # cancellation (which grows with the means) stays out of this test
    o = ((u * s) @ w.T * n ** 0.5 + 0.002 * torch.randn(m, generator=gen, device="cuda", dtype=torch.float64)).float()
    e = torch.randn(n, generator=gen, device="cuda", dtype=torch.float64)
    omega = _omega(n, r + p, seed=6)
    h = Wssr(n_max=n, m_max=m, r_max=r + p, q_max=2)
    try:
        v = torch.empty(m, r, dtype=torch.float32, device="cuda")
        delta, sigma = h.step_sketch(o, e, omega, v, 1e-3)
        assert h.status()[0] == 0
        errs = _check(o, e, omega, 1e-3, r, delta, v, sigma, TOL)
        exact = orc.delta_exact_r(_np(o), _np(e), 1e-3, r)
        sk = orc.sketch_step(_np(o), _np(e), _np(omega), 1e-3, r)["delta"]
        print("low rank: GPU vs sketch oracle", errs, "GPU vs exact", rel(_np(delta), exact),
              "sketch oracle vs exact", rel(sk, exact))
        assert rel(sk, exact) <= 1e-6
        assert rel(_np(delta), exact) <= 2 * TOL
    finally:
        h.close()


@pytest.mark.parametrize("q", [0, 1])
def test_sketch_bf16_split(q):
    """BF16 split storage with the ingest gradient.  Against the oracle on the
    stored values (same gradient): the FP32 bars.  Against the oracle on the
    unrounded O: the BF16 bar 1e-2 with one power pass.  Without power passes
    the sketch of App. A passes the storage rounding on at about 1.3e-2 (2.5e-2
    element-wise), and the oracle alone predicts the same: its results on the
    stored and on the unrounded O differ by that much.  That case is held to
    the implementation bar only (against the stored values)."""
    from paper_2512_05749_amd import Wssr
    n, m, r, p = 2048, 8000, 64, 16
    o, e, _ = random_problem(n, m, r, seed=41, device="cuda", alpha=1.3, eta=1e-4, el_mean=-10.0, el_std=0.5)
    omega = _omega(n, r + p, seed=42)
    h = Wssr(n_max=n, m_max=m, r_max=r + p, q_max=2, dtype="bf16_split")
    try:
        stored = h.storage_like(n, m)
        g, _ = h.ingest(o, e, 0, out=stored)
        v = torch.empty(m, r, dtype=torch.float32, device="cuda")
        delta, sigma = h.step_sketch(stored, None, omega, v, 1e-3, q=q, g=g)
        assert h.status()[0] == 0
        print(f"q={q} bf16_split sketch vs the stored O:",
              _check(o, e, omega, 1e-3, r, delta, v, sigma, TOL, q=q, o_ref=stored.float(), g=g))
        ref = orc.sketch_step(_np(o), _np(e), _np(omega), 1e-3, r, q=q)
        print(f"q={q} bf16_split sketch vs the unrounded O: delta {rel(_np(delta), ref['delta']):.2e} "
              f"(element-wise {_max_rel(_np(delta), ref['delta']):.2e})")
        if q > 0:
            _check(o, e, omega, 1e-3, r, delta, v, sigma, 1e-2, q=q)
    finally:
        h.close()


def test_sketch_as_cold_start():
    """The sketch's V seeds warm-started steps: the next plain step matches
    the oracle given the same V_in."""
    from paper_2512_05749_amd import Wssr
    n, m, r, p = 1024, 3000, 32, 10
    o, e, _ = random_problem(n, m, r, seed=51, device="cuda", alpha=1.2)
    omega = _omega(n, r + p, seed=52)
    h = Wssr(n_max=n, m_max=m, r_max=r + p, q_max=4)
    try:
        v = torch.empty(m, r, dtype=torch.float32, device="cuda")
        h.step_sketch(o, e, omega, v, 1e-3)
        assert h.status()[0] == 0
        o2, e2, _ = random_problem(n, m, r, seed=51, device="cuda", alpha=1.2, t=2)
        v_in = v.clone()
        delta, sigma = h.step(o2, e2, v, 1e-3, q=2)
        assert h.status()[0] == 0
        ref = orc.wssr_step(_np(o2), _np(e2), _np(v_in), 1e-3, r, 2)
        assert rel(_np(delta), ref["delta"]) <= TOL
        assert sigma_rel_gated(_np(sigma), ref["sigma"], 1e-3) <= TOL
    finally:
        h.close()


def test_sketch_rejects_bad_arguments():
    from paper_2512_05749_amd import Wssr
    from paper_2512_05749_amd.wssr import WssrError
    n, m, r = 40, 100, 8
    o, e, _ = random_problem(n, m, r, seed=61, device="cuda")
    h = Wssr(n_max=n, m_max=m, r_max=64, q_max=2)
    try:
        v = torch.empty(m, r, dtype=torch.float32, device="cuda")
        with pytest.raises(WssrError):                       # r + p > n - 1
            h.step_sketch(o, e, _omega(n, n, 1), v, 1e-3)
        with pytest.raises(ValueError):                      # fewer columns than r
            h.step_sketch(o, e, _omega(n, r - 1, 1), v, 1e-3)
        with pytest.raises(WssrError):                       # lambda <= 0
            h.step_sketch(o, e, _omega(n, r + 2, 1), v, 0.0)
    finally:
        h.close()
