"""Stage-by-stage parity of the HIP kernels (through the C ABI) with the FP64
oracle, on shapes with ragged tiles in every dimension."""
import numpy as np
import pytest
import torch

from oracle import wssr_oracle as orc
from tests.metrics import orth_err, rel
from workloads import random_problem

pytestmark = pytest.mark.gpu

SHAPES = [  # (n, m, r): ragged in N, M and r; r crossing one and two 64-column tiles
    (257, 777, 7),
    (300, 1001, 40),
    (1000, 2999, 65),
    (1024, 2000, 32),
    (200, 4096, 130),
]


@pytest.fixture(scope="module")
def ws():
    from paper_2512_05749_amd import Wssr
    h = Wssr(n_max=1024, m_max=4096, r_max=192, q_max=8)
    yield h
    h.close()


def _inputs(n, m, r, seed, ld_pad=0):
    o, e, v = random_problem(n, m, r, seed=seed, device="cuda")
    if ld_pad:
        big = torch.zeros(n, m + ld_pad, device="cuda", dtype=torch.float32)
        big[:, m:] = float("nan")   # padding must never be read
        big[:, :m] = o
        o = big[:, :m]
    return o, e, v


@pytest.mark.parametrize("n,m,r", SHAPES)
@pytest.mark.parametrize("ld_pad", [0, 3])
def test_gradient(ws, n, m, r, ld_pad):
    o, e, _ = _inputs(n, m, r, seed=n + m, ld_pad=ld_pad)
    g = ws.gradient(o, e).cpu().numpy()
    ref = orc.gradient(o.double().cpu().numpy(), e.cpu().numpy())
    assert rel(g, ref) < 1e-12


@pytest.mark.parametrize("n,m,r", SHAPES)
@pytest.mark.parametrize("ld_pad", [0, 4])
def test_sample_side(ws, n, m, r, ld_pad):
    o, _, v = _inputs(n, m, r, seed=2 * n + m, ld_pad=ld_pad)
    y = ws.sample_side(o, v).cpu().numpy()
    ref = orc.gemm_sample_side(o.double().cpu().numpy(), v.double().cpu().numpy())
    assert rel(y, ref) < 2e-6


@pytest.mark.parametrize("n,m,r", SHAPES)
def test_param_side(ws, n, m, r):
    o, _, _ = _inputs(n, m, r, seed=3 * n + m, ld_pad=0)
    x = torch.randn(n, r, device="cuda", dtype=torch.float32)
    x -= x.mean(0, keepdim=True)            # columns sum to zero -> O^T X = O_bar^T X
    z = ws.param_side(o, x).cpu().numpy()
    ref = orc.gemm_param_side(o.double().cpu().numpy(), x.double().cpu().numpy())
    assert rel(z, ref) < 2e-6


@pytest.fixture(scope="module")
def ws_wide():
    from paper_2512_05749_amd import Wssr
    h = Wssr(n_max=512, m_max=140_000, r_max=256, q_max=2)
    yield h
    h.close()


# Enough parameter tiles (128 parameters each) that they exceed one round of
# resident workgroups (512 on MI355X), so the leftover tiles are shared out
# stream-K style and summed by the fix-up kernel; the last shape fills its
# second round and runs whole tiles only.
@pytest.mark.parametrize("n,m,r", [(200, 70_001, 40), (300, 100_003, 130), (77, 99_999, 256), (64, 128_000, 64)])
def test_param_side_many_tiles(ws_wide, n, m, r):
    o, _, _ = _inputs(n, m, r, seed=5 * n + r, ld_pad=0)
    x = torch.randn(n, r, device="cuda", dtype=torch.float32)
    x -= x.mean(0, keepdim=True)
    z = ws_wide.param_side(o, x).cpu().numpy()
    ref = orc.gemm_param_side(o.double().cpu().numpy(), x.double().cpu().numpy())
    assert rel(z, ref) < 2e-6
    # every parameter row is checked, not only the norm
    row_err = np.abs(z - ref).max(1) / (np.abs(ref).max() + 1e-30)
    assert row_err.max() < 1e-5


# Shapes whose rows are 16-byte aligned (M and r multiples of 4), so both
# products take their direct-to-LDS form, for each column-tile width (64, 128,
# 256), with ragged N, a ragged last parameter tile, partial column tiles, and
# (parameter side) more tiles than one round of workgroups.
DMA_SHAPES = [(333, 2048, 32), (500, 3000, 100), (257, 4100, 128), (500, 70_000, 200), (96, 100_000, 256),
              (511, 6_000, 256),
              # r <= 32: the 32-column tile, ragged rows and columns, and a
              # parameter side with more tiles than one round (stream-K)
              (257, 4100, 4), (100, 6_000, 20), (512, 3000, 32), (500, 140_000, 8), (77, 140_000, 28),
              # fewer samples than one K-step of the parameter side
              (8, 4096, 8), (16, 5000, 24), (5, 2000, 64)]


@pytest.mark.parametrize("n,m,r", DMA_SHAPES)
def test_products_aligned(ws_wide, n, m, r):
    o, _, v = _inputs(n, m, r, seed=7 * n + r, ld_pad=0)
    y = ws_wide.sample_side(o, v).cpu().numpy()
    ref = orc.gemm_sample_side(o.double().cpu().numpy(), v.double().cpu().numpy())
    assert rel(y, ref) < 2e-6
    x = torch.randn(n, r, device="cuda", dtype=torch.float32)
    x -= x.mean(0, keepdim=True)
    z = ws_wide.param_side(o, x).cpu().numpy()
    ref = orc.gemm_param_side(o.double().cpu().numpy(), x.double().cpu().numpy())
    assert rel(z, ref) < 2e-6
    row_err = np.abs(z - ref).max(1) / (np.abs(ref).max() + 1e-30)
    assert row_err.max() < 1e-5


@pytest.mark.parametrize("rows,r", [(100, 1), (333, 7), (1000, 64), (4000, 65), (4096, 130), (2500, 192),
                                    (3000, 512)])
def test_cholqr2(ws, ws512, rows, r):
    ws = ws512 if r > 192 else ws
    gen = torch.Generator(device="cuda").manual_seed(rows + r)
    x = torch.randn(rows, r, device="cuda", generator=gen)
    x = x * torch.logspace(0, -3, r, device="cuda")[None, :]        # condition number ~1e3
    q, rr = ws.cholqr2(x)
    q, rr = q.double().cpu().numpy(), rr.cpu().numpy()
    xd = x.double().cpu().numpy()
    assert orth_err(q) < 1e-6
    assert rel(q @ rr, xd) < 1e-6
    assert np.allclose(np.tril(rr, -1), 0) and np.all(np.diag(rr) > 0)
    _, r_ref = orc.qr_positive(xd)
    assert rel(rr, r_ref) < 1e-6


@pytest.mark.parametrize("rows,r", [(4000, 40), (3000, 130)])
def test_cholqr_second_round(ws, rows, r):
    """Nearly dependent columns (condition ~1e6): one FP64 CholeskyQR round would
    leave an orthogonality error ~1e-4, so the device must run the second round."""
    gen = torch.Generator(device="cuda").manual_seed(rows)
    x = torch.randn(rows, r, device="cuda", generator=gen, dtype=torch.float64)
    x[:, 1] = x[:, 0] + 1e-6 * x[:, 1]
    x = x.float()
    q, rr = ws.cholqr2(x)
    code, diag = ws.status()
    assert code == 0
    assert diag["second_rounds"] >= 1 and diag["kappa_max"] > 1e4
    q, rr = q.double().cpu().numpy(), rr.cpu().numpy()
    assert orth_err(q) < 2e-6
    assert rel(q @ rr, x.double().cpu().numpy()) < 1e-6


@pytest.fixture(scope="module")
def ws512():
    from paper_2512_05749_amd import Wssr
    h = Wssr(n_max=1200, m_max=3000, r_max=512, q_max=4)
    yield h
    h.close()


# r = 512 (the largest rank) only for the near-diagonal kind: the oracle's
# Jacobi takes about half a minute per 512 x 512 matrix
@pytest.mark.parametrize("r,kind", [(r, k) for r in [1, 2, 7, 33, 64, 100, 128, 192]
                                    for k in ["random", "graded", "near_diag"]] + [(512, "near_diag")])
def test_small_svd(ws, ws512, r, kind):
    ws = ws512 if r > 192 else ws
    rng = np.random.default_rng(r)
    if kind == "random":
        c = rng.standard_normal((r, r))
    elif kind == "graded":
        qa = np.linalg.qr(rng.standard_normal((r, r)))[0]
        qb = np.linalg.qr(rng.standard_normal((r, r)))[0]
        c = (qa * np.logspace(0, -4, r)) @ qb.T
    else:   # what the warm-started Rayleigh-Ritz sees: diagonal plus a small perturbation
        c = np.diag(np.sort(rng.random(r))[::-1] + 0.1) + 1e-2 * rng.standard_normal((r, r))
    s, p = ws.small_svd(torch.tensor(c, device="cuda"))
    s, p = s.cpu().numpy(), p.cpu().numpy()
    _, s_ref, p_ref = orc.jacobi_svd(c)
    np.testing.assert_allclose(s, s_ref, rtol=1e-10, atol=1e-13 * s_ref[0])
    assert orth_err(p) < 1e-12
    # C P = U diag(s) with orthogonal U: columns of C P are orthogonal with norms
    # s; the Jacobi stops at column cosines <= 1e-8 (or Gram entries at the
    # rounding level 64 eps ||C||_F^2)
    cp = c @ p
    gram = cp.T @ cp
    off = np.abs(gram - np.diag(np.diag(gram)))
    scale = np.sqrt(np.outer(np.diag(gram), np.diag(gram))) * 2e-8 + 1e-13 * np.sum(c * c)
    assert np.all(off <= scale)
    np.testing.assert_allclose(np.sqrt(np.diag(gram)), s, rtol=1e-10, atol=1e-13 * s[0])
    code, diag = ws.status()
    assert code == 0, diag


def test_argument_errors(ws):
    from paper_2512_05749_amd import WssrError
    o, e, v = random_problem(100, 300, 8, seed=1, device="cuda")
    with pytest.raises(WssrError):
        ws.step(o, e, torch.zeros(300, 100, device="cuda"), 1e-3)          # r > n - 1
    with pytest.raises(WssrError):
        ws.step(o, e, v.clone(), 0.0)                                       # lambda <= 0
    with pytest.raises(WssrError):
        ws.step(o, e, v.clone(), 1e-3, q=0)
    with pytest.raises(WssrError):
        ws.step(o, e, v.clone(), float("inf"))
    big = torch.zeros(2000, 300, device="cuda")
    with pytest.raises(WssrError):
        ws.step(big, torch.zeros(2000, dtype=torch.float64, device="cuda"), v.clone(), 1e-3)   # n > n_max
