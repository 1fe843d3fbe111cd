"""Whole-step parity of the HIP path (wssr_step through the C ABI) with the FP64
oracle: the small workload over consecutive warm-started steps, ragged shapes,
edge cases and failure handling."""
import numpy as np
import pytest
import torch

from oracle import wssr_oracle as orc
from tests.metrics import orth_err, rel, sigma_rel_gated, sin_max_angle, weighted_projector_err
from workloads import CONFIGS, Workload, random_problem

pytestmark = pytest.mark.gpu

# FP32 form tolerances: delta and gated sigma relative error <= 1e-4,
# orthonormality of V <= 1e-5.
TOL_DELTA = 1e-4
TOL_SIGMA = 1e-4
TOL_ORTH = 1e-5


def _np(t):
    return t.detach().double().cpu().numpy()


def _check_against_oracle(o, e, v_in, v_out, delta, sigma, lam, q, precond="damped"):
    ref = orc.wssr_step(_np(o), _np(e), _np(v_in), lam, v_in.shape[1], q, precond=precond)
    d_err = rel(_np(delta), ref["delta"])
    # element by element too: the largest deviation against the largest entry
    d_max = float(np.abs(_np(delta) - ref["delta"]).max() / np.abs(ref["delta"]).max())
    assert d_max <= TOL_DELTA, d_max
    s_err = sigma_rel_gated(_np(sigma), ref["sigma"], lam)
    o_err = orth_err(_np(v_out))
    w_g = orc.woodbury_weights(_np(sigma), lam, precond)
    w_o = orc.woodbury_weights(ref["sigma"], lam, precond)
    wp = weighted_projector_err(_np(v_out), w_g, ref["v"], w_o)
    assert d_err <= TOL_DELTA, (d_err, s_err, wp)
    assert s_err <= TOL_SIGMA, (d_err, s_err, wp)
    assert o_err <= TOL_ORTH
    assert wp <= 1e-4
    # signs follow the documented rule: agree with the oracle where the
    # inner product with V_in is clearly nonzero
    ip = np.sum(ref["v"] * _np(v_in), axis=0)
    clear = np.abs(ip) > 1e-3
    dots = np.sum(_np(v_out) * ref["v"], axis=0)
    assert np.all(dots[clear] > 0)
    return d_err, s_err, wp


@pytest.fixture(scope="module")
def ws():
    from paper_2512_05749_amd import Wssr
    h = Wssr(n_max=2048, m_max=5000, r_max=192, q_max=8)
    yield h
    h.close()


def test_small_workload_ten_steps(ws):
    """N=1024, M=2000, r=32, q=2, lambda=1e-3, rotation 0.02/step: step 1 cold
    (8 passes from V_0), then warm-started steps, each against the oracle given
    the same V_in (teacher forcing)."""
    cfg = CONFIGS["f32_n1024_m2k_r32"]
    wl = Workload(cfg, device="cuda")
    v = wl.v0()
    for t in range(1, cfg.steps + 1):
        o, e = wl.o(t), wl.e_l(t)
        q = 8 if t == 1 else cfg.q
        v_in = v.clone()
        delta, sigma = ws.step(o, e, v, cfg.lam, q=q)
        code, diag = ws.status()
        assert code == 0, (t, code, diag)
        _check_against_oracle(o, e, v_in, v, delta, sigma, cfg.lam, q)


@pytest.mark.parametrize("n,m,r,q", [(257, 1001, 7, 2), (500, 3000, 65, 3), (130, 200, 129, 2),
                                     (64, 4999, 1, 1), (2048, 4096, 192, 2),
                                     # aligned rows and r <= 32: the 32-column product kernels
                                     (1000, 4000, 32, 2), (333, 4096, 12, 3)])
def test_ragged_shapes(ws, n, m, r, q):
    o, e, v = random_problem(n, m, r, seed=n * 7 + r, device="cuda", alpha=1.0)
    v_in = v.clone()
    delta, sigma = ws.step(o, e, v, 1e-3, q=q)
    code, _ = ws.status()
    assert code == 0
    _check_against_oracle(o, e, v_in, v, delta, sigma, 1e-3, q)


def test_rank_512():
    """The largest rank: 512 columns (8 Cholesky tiles, 16 Jacobi workgroups)."""
    from paper_2512_05749_amd import Wssr
    h = Wssr(n_max=1100, m_max=2600, r_max=512, q_max=4)
    o, e, v = random_problem(1100, 2600, 512, seed=512, device="cuda", alpha=1.0)
    v_in = v.clone()
    delta, sigma = h.step(o, e, v, 1e-3, q=1)
    code, diag = h.status()
    h.close()
    assert code == 0, diag
    _check_against_oracle(o, e, v_in, v, delta, sigma, 1e-3, 1)


def test_floor_preconditioner():
    from paper_2512_05749_amd import Wssr
    h = Wssr(n_max=600, m_max=1500, r_max=16, q_max=4, floor_precond=True)
    o, e, v = random_problem(600, 1500, 12, seed=3, device="cuda", alpha=1.0, eta=1e-4)
    v_in = v.clone()
    lam = 1e-4
    delta, sigma = h.step(o, e, v, lam, q=4)
    assert h.status()[0] == 0
    assert (sigma ** 2 > lam).all()   # floor form amplifies directions below the floor
    _check_against_oracle(o, e, v_in, v, delta, sigma, lam, 4, precond="floor")
    h.close()


def test_full_rank_equals_direct_solve(ws):
    """r = n - 1 = rank of the centred matrix: the step is exact (delta_full)."""
    n, m = 60, 400
    o, e, v = random_problem(n, m, n - 1, seed=5, device="cuda", alpha=0.5)
    delta, sigma = ws.step(o, e, v, 1e-2, q=1)
    assert ws.status()[0] == 0
    ref = orc.sr_pushthrough(_np(o), _np(e), 1e-2)
    assert rel(_np(delta), ref) < 1e-4


def test_fixed_point(ws):
    """V_in = the exact top-r singular vectors: V_out spans the same space, sigma exact."""
    n, m, r = 300, 900, 10
    o, e, _ = random_problem(n, m, r, seed=6, device="cuda", alpha=1.0)
    v_ex, s_ex = orc.exact_topr(_np(o), r)
    v = torch.tensor(np.ascontiguousarray(v_ex), dtype=torch.float32, device="cuda").contiguous()
    delta, sigma = ws.step(o, e, v, 1e-3, q=1)
    assert ws.status()[0] == 0
    assert sin_max_angle(_np(v), v_ex) < 1e-3
    np.testing.assert_allclose(_np(sigma), s_ex, rtol=1e-4)
    assert np.all(np.sum(_np(v) * v_ex, 0) > 0.999)


def test_deterministic(ws):
    o, e, v = random_problem(700, 2500, 48, seed=8, device="cuda")
    outs = []
    for _ in range(2):
        vv = v.clone()
        d, s = ws.step(o, e, vv, 1e-3, q=2)
        outs.append((d.clone(), s.clone(), vv))
    assert torch.equal(outs[0][0], outs[1][0])
    assert torch.equal(outs[0][1], outs[1][1])
    assert torch.equal(outs[0][2], outs[1][2])


def test_invariance_shift_of_O_and_E(ws):
    """O -> O + 1 c^T and E_L -> E_L + c leave delta unchanged (centring)."""
    o, e, v = random_problem(400, 1200, 16, seed=9, device="cuda")
    v1 = v.clone()
    d1, s1 = ws.step(o, e, v1, 1e-3, q=2)
    c = torch.randn(1200, device="cuda") * 0.05
    v2 = v.clone()
    d2, s2 = ws.step(o + c[None, :], e + 3.0, v2, 1e-3, q=2)
    assert rel(_np(d2), _np(d1)) < 1e-4
    assert rel(_np(s2), _np(s1)) < 1e-4


def test_nonfinite_energy_leaves_outputs_untouched(ws):
    o, e, v = random_problem(200, 500, 8, seed=10, device="cuda")
    e[17] = float("nan")
    v_before = v.clone()
    delta = torch.full((500,), 7.0, dtype=torch.float64, device="cuda")
    sigma = torch.full((8,), 7.0, dtype=torch.float64, device="cuda")
    ws.step(o, e, v, 1e-3, q=2, delta=delta, sigma=sigma)
    code, _ = ws.status()
    assert code == -5
    assert torch.equal(v, v_before)
    assert (delta == 7.0).all() and (sigma == 7.0).all()


def test_nonfinite_O_is_reported(ws):
    o, e, v = random_problem(200, 500, 8, seed=11, device="cuda")
    o[5, 9] = float("inf")
    v_before = v.clone()
    ws.step(o, e, v, 1e-3, q=2)
    code, _ = ws.status()
    assert code in (-5, -6)
    assert torch.equal(v, v_before)


def test_rank_deficient(ws):
    """O with only 5 distinct rows (4 after centring) but r = 6: the bases of
    the iteration lose rank.  The library completes them, reports
    WARN_RANK_DEFICIENT, and delta matches the oracle, whose Householder QR
    completes them too (the extra singular values are zero, their weights 0).

    lambda = 1 here: g lies entirely in the 4-dimensional span of the top
    singular vectors, so delta = (g - V w V^T g) / lambda cancels down to about
    g / sigma^2, and the FP32 rounding of V (about 1e-7) enters delta
    amplified by sigma^2 / lambda (60 here; 6e4 at lambda = 1e-3)."""
    lam = 1.0
    g = torch.Generator(device="cuda").manual_seed(17)
    base = torch.randn(5, 300, device="cuda", generator=g)
    o = base[torch.arange(40, device="cuda") % 5].contiguous()
    e = torch.randn(40, dtype=torch.float64, device="cuda", generator=g)
    v = torch.randn(300, 6, device="cuda", generator=g)
    v_in = v.clone()
    delta, sigma = ws.step(o, e, v, lam, q=2)
    code, diag = ws.status()
    assert code == 1, (code, diag)
    ref = orc.wssr_step(_np(o), _np(e), _np(v_in), lam, 6, 2)
    assert rel(_np(delta), ref["delta"]) <= TOL_DELTA
    assert float(np.abs(_np(delta) - ref["delta"]).max() / np.abs(ref["delta"]).max()) <= TOL_DELTA
    # the four nonzero singular values agree; the rest are at rounding level
    np.testing.assert_allclose(_np(sigma)[:4], ref["sigma"][:4], rtol=1e-4)
    assert np.all(_np(sigma)[4:] < 1e-5 * _np(sigma)[0])
    assert orth_err(_np(v)) <= TOL_ORTH


def test_zero_column_breakdown(ws):
    """A zero column in V_in gives a zero column in the first basis, which no
    QR completes from the data: WSSR_ERR_BREAKDOWN, V, delta and sigma left
    as they were."""
    o, e, v = random_problem(200, 500, 8, seed=13, device="cuda")
    v[:, 3] = 0.0
    v_before = v.clone()
    delta = torch.full((500,), 7.0, dtype=torch.float64, device="cuda")
    sigma = torch.full((8,), 7.0, dtype=torch.float64, device="cuda")
    ws.step(o, e, v, 1e-3, q=2, delta=delta, sigma=sigma)
    code, _ = ws.status()
    assert code == -6
    assert torch.equal(v, v_before)
    assert (delta == 7.0).all() and (sigma == 7.0).all()


def test_handle_recovers_after_error(ws):
    o, e, v = random_problem(200, 500, 8, seed=12, device="cuda")
    bad = e.clone()
    bad[0] = float("inf")
    ws.step(o, bad, v.clone(), 1e-3)
    assert ws.status()[0] == -5
    v_in = v.clone()
    d, s = ws.step(o, e, v, 1e-3, q=2)
    assert ws.status()[0] == 0
    _check_against_oracle(o, e, v_in, v, d, s, 1e-3, 2)
