"""The allocation-free SVD entry point (wssr_small_svd_noalloc) against the
handle-based one (wssr_dbg_small_svd) on the same inputs: two calls in a row,
the second with a smaller matrix, so that the shared device array is reused
with a different size."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def _case(r, seed):
    g = torch.Generator(device="cpu").manual_seed(seed)
    # a graded, nearly diagonal upper-triangular matrix like the Rayleigh-Ritz
    # input of a warm-started step (off-diagonal entries small against the
    # diagonal, so the matrix is well conditioned)
    d = torch.arange(1, r + 1, dtype=torch.float64) ** -1.1
    c = torch.triu(torch.randn(r, r, generator=g, dtype=torch.float64), 1) * 1e-4 * d[None, :]
    c += torch.diag(d)
    return c.cuda().contiguous()


def test_noalloc_matches_handle_entry_point():
    from paper_2512_05749_amd import Wssr
    from paper_2512_05749_amd.wssr import small_svd_noalloc
    h = Wssr(n_max=600, m_max=600, r_max=512, q_max=2)
    try:
        for r, seed in [(300, 1), (77, 2)]:
            c = _case(r, seed)
            s_ref, p_ref = h.small_svd(c)
            assert h.status()[0] == 0
            s, p, st = small_svd_noalloc(c)
            torch.cuda.synchronize()
            assert int(st.item()) == 0
            np.testing.assert_allclose(s.cpu().numpy(), s_ref.cpu().numpy(), rtol=1e-12, atol=0)
            np.testing.assert_allclose(p.cpu().numpy(), p_ref.cpu().numpy(), rtol=0, atol=1e-12)
            # and it is an SVD of c
            cn = c.cpu().numpy()
            np.testing.assert_allclose(s.cpu().numpy(), np.linalg.svd(cn, compute_uv=False), rtol=1e-9)
    finally:
        h.close()


def test_noalloc_rejects_oversize():
    from paper_2512_05749_amd.wssr import WssrError, small_svd_noalloc
    with pytest.raises(WssrError):
        small_svd_noalloc(torch.zeros(513, 513, dtype=torch.float64, device="cuda"))
