"""The precision-form instance at its full size (N=16384 samples, M=1e6
parameters, r=512, O stored in BF16), in the launch configuration the
benchmark times: both products on the GPU against the FP64 oracle on sampled
output rows, which the oracle computes one by one from the stored values of O.

The sample-side product centres its result, so its reference needs the column
means of O over all N rows; they are summed on the host in FP64 from a copy of
the stored O (32 GB), in row blocks."""
import numpy as np
import pytest
import torch

from oracle import wssr_oracle as orc
from tests.metrics import rel
from workloads import CONFIGS, Workload, to_storage

pytestmark = pytest.mark.gpu

# FP32 accumulation inside each product: the sample side sums K = M/2 = 5e5
# terms per split-K range (the ranges are added in FP64), about
# sqrt(5e5) * 2^-24 ~ 4e-5 relative; the parameter side K = N = 16384 terms,
# about 8e-6.  Five times those.
TOL_SAMPLE = 2e-4
TOL_PARAM = 5e-5


def _split_hi(x):
    return x.to(torch.bfloat16).double().cpu().numpy()


@pytest.mark.timeout(900)
def test_precision_instance_products_full_size():
    from paper_2512_05749_amd import Wssr
    cfg = CONFIGS["bf16_n16384_m1m_r512"]
    n, m, r = cfg.n, cfg.m, cfg.r
    wl = Workload(cfg, device="cuda", gen_dtype=torch.float32)
    o32 = wl.o(1)
    o = to_storage(o32, "bf16")
    del o32
    v = wl.v0()
    del wl
    torch.cuda.empty_cache()
    gen = torch.Generator(device="cuda").manual_seed(29)
    x = torch.randn(n, r, device="cuda", generator=gen)
    x -= x.mean(0, keepdim=True)
    print("generated the instance", flush=True)

    h = Wssr(n_max=n, m_max=m, r_max=r, q_max=2, dtype="bf16")
    try:
        y = h.sample_side(o, v)
        z = h.param_side(o, x)
        torch.cuda.synchronize()
    finally:
        h.close()
    print("products done", flush=True)

    rng = np.random.default_rng(7)
    rows_y = np.sort(rng.choice(n, 24, replace=False))
    rows_z = np.sort(rng.choice(m, 64, replace=False))
    y_s = y[torch.from_numpy(rows_y).cuda()].cpu().numpy()
    z_s = z[torch.from_numpy(rows_z).cuda()].double().cpu().numpy()
    del y, z

    # host copy of the stored O and its column means (FP64, row blocks)
    o_host = o.cpu()
    del o
    torch.cuda.empty_cache()
    mu = torch.zeros(m, dtype=torch.float64)
    for i in range(0, n, 512):
        mu += o_host[i:i + 512].double().sum(0)
    mu /= n
    print("column means done", flush=True)

    # sample side: rows (O_i - mu) V_hi / sqrt(N), V rounded to BF16 as the kernel rounds it
    v_hi = _split_hi(v)
    a_rows = (o_host[torch.from_numpy(rows_y)].double() - mu[None, :]).numpy() / np.sqrt(n)
    ref_y = a_rows @ v_hi
    err_y = rel(y_s, ref_y)
    # parameter side: rows O[:, j]^T X_hi / sqrt(N) (the uncentred contract)
    x_hi = _split_hi(x)
    cols = o_host[:, torch.from_numpy(rows_z)].double().numpy()
    ref_z = cols.T @ x_hi / np.sqrt(n)
    err_z = rel(z_s, ref_z)
    print(f"full-size BF16 products: sample side rel err {err_y:.2e} (24 rows), "
          f"parameter side {err_z:.2e} (64 rows)", flush=True)
    assert err_y < TOL_SAMPLE
    assert err_z < TOL_PARAM
    # every sampled row, not only the norm
    assert np.max(np.abs(y_s - ref_y).max(1) / np.abs(ref_y).max()) < 10 * TOL_SAMPLE
    assert np.max(np.abs(z_s - ref_z).max(1) / np.abs(ref_z).max()) < 10 * TOL_PARAM
