"""The fast Grams (FP32 MFMA; BF16 MFMA on the two-plane split) and the
basis an intermediate pass carries on (wssr_dbg_gram, wssr_dbg_span_basis):
the Grams against FP64 numpy, and the
three ways the basis is made, each chosen where it should be and spanning
the input."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def _np(t):
    return t.detach().double().cpu().numpy()


@pytest.mark.parametrize("rows,r", [(5000, 64), (20011, 130), (3001, 7), (40000, 512)])
def test_gram_fp32_and_fp64(rows, r):
    from paper_2512_05749_amd import Wssr
    gen = torch.Generator(device="cuda").manual_seed(rows + r)
    x = torch.randn(rows, r, generator=gen, device="cuda") * torch.logspace(0, -3, r, device="cuda")
    h = Wssr(n_max=64, m_max=rows, r_max=r, q_max=2)
    try:
        want = _np(x).T @ _np(x)
        scale = np.sqrt(np.outer(np.diag(want), np.diag(want)))
        g64 = _np(h.gram(x))
        g32 = _np(h.gram(x, "fp32"))
        g16 = _np(h.gram(x, "bf16_split"))
        assert h.status()[0] == 0
        e64 = float(np.abs(g64 - want).max() / np.abs(want).max())
        e32 = float(np.abs((g32 - want) / scale).max())
        e16 = float(np.abs((g16 - want) / scale).max())
        print(f"rows={rows} r={r}: FP64 {e64:.1e}, relative to sqrt(G_ii G_jj): FP32 {e32:.1e}, "
              f"BF16 split {e16:.1e}")
        assert e64 < 1e-13
        # FP32 sums of 256 rows flushed into FP64: a few FP32 roundings of
        # the largest partial sum; the split adds its residual (2^-16 per
        # element, about 2^-15 / sqrt(rows) for residuals of random sign)
        assert e32 < 1e-6
        assert e16 < 2e-6
    finally:
        h.close()


def _sin_angle(a, b):
    qa, qb = np.linalg.qr(a)[0], np.linalg.qr(b)[0]
    c = np.linalg.svd(qa.T @ qb, compute_uv=False)
    return float(np.sqrt(max(0.0, 1.0 - min(1.0, c.min()) ** 2)))


@pytest.mark.parametrize("kind,want_mode", [("orthogonal", 0), ("mixed", 1), ("ill", 2)])
def test_span_basis_modes(kind, want_mode):
    from paper_2512_05749_amd import Wssr
    rows, r = 20000, 48
    gen = torch.Generator(device="cuda").manual_seed(7)
    q = torch.linalg.qr(torch.randn(rows, r, generator=gen, device="cuda", dtype=torch.float64))[0]
    scales = torch.logspace(0, -4, r, device="cuda", dtype=torch.float64)
    if kind == "orthogonal":
        x = q * scales
    elif kind == "mixed":
        mix = torch.eye(r, device="cuda", dtype=torch.float64) + 0.3 * torch.randn(r, r, generator=gen, device="cuda",
                                                                                 dtype=torch.float64) / r ** 0.5
        x = (q @ mix) * scales
    else:
        x = q.clone()
        x[:, 1] = x[:, 0] + 1e-5 * x[:, 1]                 # two columns at cosine 1 - 5e-11
        x = x * scales
    x = x.float().contiguous()
    h = Wssr(n_max=64, m_max=rows, r_max=r, q_max=2)
    try:
        v, mode = h.span_basis(x)
        assert h.status()[0] == 0
        vn, xn = _np(v), _np(x)
        print(kind, "mode", mode, "angle", _sin_angle(vn, xn))
        assert mode == want_mode
        # same span as the input (up to the input's own conditioning)
        if kind != "ill":
            assert _sin_angle(vn, xn) < 1e-4
        gram = vn.T @ vn
        d = np.sqrt(np.diag(gram))
        assert np.abs(gram / np.outer(d, d) - np.eye(r)).max() < (1e-3 if mode == 1 else 1e-5)
    finally:
        h.close()
