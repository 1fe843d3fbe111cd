"""The BF16 forms of the step (O stored in BF16, products on the BF16 MFMA
with FP32 accumulation): stage and whole-step parity with the FP64 oracle run
on the values O holds in storage, and the end-to-end error against the oracle
on the unrounded O for the split form."""
import numpy as np
import pytest
import torch

from oracle import wssr_oracle as orc
from tests.metrics import orth_err, rel, sigma_rel_gated, weighted_projector_err
from workloads import random_problem, stored_values, to_storage

pytestmark = pytest.mark.gpu

FORMS = ["bf16", "bf16_split", "bf16x2"]
# Products: the oracle evaluates the same sum of products the kernels form,
# with the FP32 skinny operand S split as the kernels split it (S_hi =
# RNE_bf16(S), S_lo = RNE_bf16(S - S_hi), torch's round to nearest even).
# What is left is FP32 accumulation over K <= 4096 terms, about
# sqrt(K) * 2^-24 ~ 4e-6 relative.
TOL_PRODUCT = 2e-5


def _split(x):
    hi = x.to(torch.bfloat16)
    lo = (x - hi.float()).to(torch.bfloat16)
    return hi.double().cpu().numpy(), lo.double().cpu().numpy()


def _expected(f, planes, s, form):
    """Sum of the products the form computes (f: an oracle product)."""
    s_hi, s_lo = _split(s)
    out = f(planes[0], s_hi)
    if form in ("bf16_split", "bf16x2"):
        out = out + f(planes[0], s_lo)
    if form == "bf16x2":
        out = out + f(planes[1], s_hi)
    return out


# Whole step against the oracle on the stored O: the split forms meet the FP32
# bars; bf16 meets the 1e-2 bar of the BF16 form.
TOL_DELTA = {"bf16": 1e-2, "bf16_split": 1e-4, "bf16x2": 1e-4}
TOL_SIGMA = {"bf16": 1e-2, "bf16_split": 1e-4, "bf16x2": 1e-4}


def _np(t):
    return t.detach().double().cpu().numpy()


@pytest.fixture(scope="module")
def handles():
    from paper_2512_05749_amd import Wssr
    hs = {f: Wssr(n_max=1200, m_max=5000, r_max=512, q_max=8, dtype=f) for f in FORMS}
    yield hs
    for h in hs.values():
        h.close()


# ragged shapes (guarded loads) and shapes whose O rows are whole 16-byte
# chunks (the direct-to-LDS kernels), for each column-tile width
SHAPES = [(257, 777, 7), (300, 1001, 40), (1000, 2999, 130), (520, 4096, 256), (1100, 3001, 300), (700, 2048, 512),
          (333, 2048, 100), (1000, 3000, 64), (520, 4096, 24), (700, 2048, 8),
          # fewer samples than one K-step of the parameter side
          (8, 4096, 16), (20, 2048, 300)]


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("n,m,r", SHAPES)
def test_products(handles, form, n, m, r):
    h = handles[form]
    o, e, v = random_problem(n, m, r, seed=n + r, device="cuda")
    os_ = to_storage(o, form)
    planes = [p.double().cpu().numpy() for p in (os_ if os_.dim() == 3 else [os_])]
    y = h.sample_side(os_, v).cpu().numpy()
    assert rel(y, _expected(orc.gemm_sample_side, planes, v, form)) < TOL_PRODUCT
    # the parameter-side stage computes O^T X / sqrt(n) with O itself (equal to
    # A^T X only while the columns of X sum to zero, which the BF16 pieces of
    # X need not do), so its reference is the uncentred product
    x = torch.randn(n, r, device="cuda")
    x -= x.mean(0, keepdim=True)
    z = h.param_side(os_, x).cpu().numpy()
    assert rel(z, _expected(lambda o_, x_: o_.T @ x_ / np.sqrt(n), planes, x, form)) < TOL_PRODUCT
    g = h.gradient(os_, e).cpu().numpy()
    assert rel(g, orc.gradient(stored_values(os_).cpu().numpy(), _np(e))) < 1e-12


@pytest.mark.parametrize("form", FORMS)
def test_products_streamk_narrow(form):
    """64-column tiles with more parameter-side tiles than one round of
    resident workgroups holds (stream-K), ragged N."""
    from paper_2512_05749_amd import Wssr
    n, m, r = 77, 140_000, 40
    h = Wssr(n_max=n, m_max=m, r_max=r, q_max=2, dtype=form)
    try:
        o, _, v = random_problem(n, m, r, seed=5, device="cuda")
        os_ = to_storage(o, form)
        planes = [p.double().cpu().numpy() for p in (os_ if os_.dim() == 3 else [os_])]
        y = h.sample_side(os_, v).cpu().numpy()
        assert rel(y, _expected(orc.gemm_sample_side, planes, v, form)) < TOL_PRODUCT
        x = torch.randn(n, r, device="cuda")
        x -= x.mean(0, keepdim=True)
        z = h.param_side(os_, x).cpu().numpy()
        assert rel(z, _expected(lambda o_, x_: o_.T @ x_ / np.sqrt(n), planes, x, form)) < TOL_PRODUCT
    finally:
        h.close()


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("n,m,r,q", [(1024, 2000, 32, 2), (600, 3000, 130, 3), (1100, 4000, 300, 2)])
def test_step_against_stored_values(handles, form, n, m, r, q):
    h = handles[form]
    o, e, v = random_problem(n, m, r, seed=3 * n + r, device="cuda", alpha=1.2, eta=1e-3)
    os_ = to_storage(o, form)
    v_in = v.clone()
    delta, sigma = h.step(os_, e, v, 1e-3, q=q)
    code, diag = h.status()
    assert code == 0, diag
    ref = orc.wssr_step(stored_values(os_).cpu().numpy(), _np(e), _np(v_in), 1e-3, r, q)
    assert rel(_np(delta), ref["delta"]) <= TOL_DELTA[form]
    assert sigma_rel_gated(_np(sigma), ref["sigma"], 1e-3) <= TOL_SIGMA[form]
    assert orth_err(_np(v)) <= 1e-5
    if form != "bf16":
        w_g = orc.woodbury_weights(_np(sigma), 1e-3)
        w_o = orc.woodbury_weights(ref["sigma"], 1e-3)
        assert weighted_projector_err(_np(v), w_g, ref["v"], w_o) <= 1e-4


def test_split_form_end_to_end_against_unrounded_O(handles):
    """bf16x2 holds O to about 16 bits, so the step stays within 1e-3 of the
    oracle on the unrounded FP32 O."""
    h = handles["bf16x2"]
    o, e, v = random_problem(1024, 2000, 32, seed=77, device="cuda", alpha=1.5)
    v_in = v.clone()
    delta, sigma = h.step(to_storage(o, "bf16x2"), e, v, 1e-3, q=2)
    assert h.status()[0] == 0
    ref = orc.wssr_step(_np(o), _np(e), _np(v_in), 1e-3, 32, 2)
    assert rel(_np(delta), ref["delta"]) <= 1e-3
    assert sigma_rel_gated(_np(sigma), ref["sigma"], 1e-3) <= 1e-3


def test_storage_planes_reproduce_O():
    """hi + lo of the two-plane storage is O to about 2^-17 relative (input encoding check)."""
    o = torch.randn(64, 300, dtype=torch.float32)
    st = to_storage(o, "bf16x2")
    err = (stored_values(st) - o.double()).abs() / o.double().abs().clamp_min(1e-30)
    assert float(err.max()) < 2.0 ** -16
