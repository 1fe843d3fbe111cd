"""The two BF16 split-form products at the shape of the largest single
instance (N=16384 samples, M=4e6 parameters, r=512), made ragged (N=16360,
M=3,999,976) so that the last row tile on each side and the last K-step of
the parameter side are partial, in the launch configuration the benchmark
times.  Checked against the FP64 oracle on sampled output rows: on the
sample side 20 random rows and the last four; on the parameter side 32 random
rows, two rows of each tile that the stream-K schedule shares between
workgroups, and the last four.

O is drawn in BF16 with rows in pairs of opposite sign, so its column means
are exactly zero and the centred sample-side product is O V / sqrt(N) itself;
the reference then needs only the sampled rows of O.  V and X are split into
BF16 hi and lo planes by round to nearest even (torch's conversion), as the
kernels split them, and the reference multiplies by hi + lo in FP64: the
definition of the products (the oracle's gemm_sample_side and
gemm_param_side restricted to the sampled rows, with zero column means),
summed over blocks of parameters on the host."""
import numpy as np
import pytest
import torch

from tests.metrics import rel

pytestmark = pytest.mark.gpu

# FP32 accumulation: the sample side sums K = M / 8 = 5e5 terms per split-K
# range, about sqrt(5e5) * 2^-24 ~ 4e-5 relative; the parameter side
# K = N = 16360 terms, about 8e-6.  Five times those.
TOL_SAMPLE = 2e-4
TOL_PARAM = 5e-5


def _hi_lo_sum(x):
    """(hi + lo) in FP64 for x split as the kernels split it."""
    hi = x.to(torch.bfloat16)
    lo = (x - hi.float()).to(torch.bfloat16)
    return hi.double() + lo.double()


@pytest.mark.timeout(900)
def test_split_products_largest_shape():
    from paper_2512_05749_amd import Wssr
    n, m, r = 16360, 3_999_976, 512
    gen = torch.Generator(device="cuda").manual_seed(41)
    o = torch.empty(n, m, dtype=torch.bfloat16, device="cuda")
    for i in range(0, n, 512):
        half = (min(i + 512, n) - i) // 2       # n is even: whole pairs
        blk = torch.randn(half, m, generator=gen, device="cuda", dtype=torch.bfloat16)
        o[i:i + 2 * half:2] = blk
        o[i + 1:i + 2 * half:2] = -blk
        del blk
    v = torch.randn(m, r, generator=gen, device="cuda") / np.sqrt(m)
    x = torch.randn(n, r, generator=gen, device="cuda")
    torch.cuda.synchronize()
    print("generated", flush=True)

    h = Wssr(n_max=n, m_max=m, r_max=r, q_max=2, dtype="bf16_split")
    try:
        y = h.sample_side(o, v)
        z = h.param_side(o, x)
        torch.cuda.synchronize()
    finally:
        h.close()
    print("products done", flush=True)

    rng = np.random.default_rng(11)
    rows_y = np.unique(np.concatenate([rng.choice(n - 4, 20, replace=False), np.arange(n - 4, n)]))
    tiles = (m + 127) // 128
    full = tiles - tiles % 256          # whole tiles of the 256 resident workgroups
    sk_rows = np.concatenate([t * 128 + rng.choice(min(128, m - t * 128), 2, replace=False)
                              for t in range(full, tiles)])
    rows_z = np.unique(np.concatenate([rng.choice(full * 128, 32, replace=False), sk_rows,
                                       np.arange(m - 4, m)]))
    y_s = y[torch.from_numpy(rows_y).cuda()].cpu().numpy()
    z_s = z[torch.from_numpy(rows_z).cuda()].double().cpu().numpy()
    o_rows = o[torch.from_numpy(rows_y).cuda()].cpu()
    o_cols = o[:, torch.from_numpy(rows_z).cuda()].cpu()
    del y, z, o
    torch.cuda.empty_cache()

    # sample side: rows O_i (V_hi + V_lo) / sqrt(N), V streamed from the
    # device in blocks of rows
    ref_y = np.zeros((len(rows_y), r))
    for k in range(0, m, 1 << 16):
        vb = _hi_lo_sum(v[k:k + (1 << 16)].cpu()).numpy()
        ref_y += o_rows[:, k:k + (1 << 16)].double().numpy() @ vb
    ref_y /= np.sqrt(n)
    # parameter side: rows O[:, j]^T (X_hi + X_lo) / sqrt(N)
    ref_z = o_cols.double().numpy().T @ _hi_lo_sum(x.cpu()).numpy() / np.sqrt(n)
    err_y, err_z = rel(y_s, ref_y), rel(z_s, ref_z)
    print(f"largest-shape split products: sample side rel err {err_y:.2e} ({len(rows_y)} rows), "
          f"parameter side {err_z:.2e} ({len(rows_z)} rows, {len(sk_rows)} in stream-K tiles)", flush=True)
    assert err_y < TOL_SAMPLE
    assert err_z < TOL_PARAM
    assert np.max(np.abs(y_s - ref_y).max(1) / np.abs(ref_y).max()) < 10 * TOL_SAMPLE
    assert np.max(np.abs(z_s - ref_z).max(1) / np.abs(ref_z).max()) < 10 * TOL_PARAM
