"""Host logic of the benchmark (no GPU): the CPU baseline's second timing
point and the recorded memory-side traffic the benchmark line reports."""
import numpy as np

import bench
from oracle import wssr_oracle as orc


def test_tiled_sample_keeps_the_small_matrices():
    """The CPU baseline's second point runs the oracle on the sample tiled w
    times along the columns, with V's rows tiled and scaled by 1/sqrt(w).
    Then A_tiled = [A, ..., A] has the singular values sqrt(w) sigma and the
    right singular vectors V / sqrt(w) stacked w times, so every r x r matrix
    of the step is the sample's up to a scale and only the column-linear work
    grows."""
    rng = np.random.default_rng(3)
    n, cols, r, w = 300, 200, 8, 5
    o = rng.standard_normal((n, cols))
    e = rng.standard_normal(n)
    v = rng.standard_normal((cols, r))
    a = orc.wssr_step(o, e, v, 1e-3, r, 2)
    b = orc.wssr_step(np.tile(o, (1, w)), e, np.tile(v, (w, 1)) / np.sqrt(w), 1e-3, r, 2)
    assert np.max(np.abs(b["sigma"] / np.sqrt(w) - a["sigma"]) / a["sigma"]) < 1e-12
    for k in range(w):
        assert np.max(np.abs(b["v"][k * cols:(k + 1) * cols] * np.sqrt(w) - a["v"])) < 1e-12


def test_oracle_job_times_both_points():
    class Sink:
        def put(self, x):
            self.x = x

    rng = np.random.default_rng(4)
    n, cols, r = 200, 150, 6
    o = rng.standard_normal((n, cols)).astype(np.float32)
    e = rng.standard_normal(n)
    v = np.linalg.qr(rng.standard_normal((cols, r)))[0].astype(np.float32)
    sink = Sink()
    bench._oracle_job(o, e, v, cols, 1e-3, r, 2, 1, sink, 3)
    res = sink.x
    assert res["seconds"] > 0 and res["seconds_wide"] > 0
    ref = orc.wssr_step(o.astype(np.float64), e, v.astype(np.float64), 1e-3, r, 2)
    assert np.array_equal(res["delta"], ref["delta"])


def test_recorded_traffic_of_the_largest_instance():
    rec = bench.TRAFFIC_RECORDS[("bf16_n16384_m4m_r512_q3", 4_000_000, "bf16_split")]
    for kernel in ("k_gemm16_param_side_rs", "k_gemm16_sample_side_rs"):
        b = bench.recorded_traffic(kernel, rec)
        assert b is not None and b > 1e11, (kernel, b)
    assert bench.recorded_traffic("k_no_such_kernel", rec) is None


def test_product_kernel_names_follow_the_dispatch():
    """The kernel the benchmark names in its roofline object is the one the
    library launches for the form, side and shape."""
    from workloads import CONFIGS
    big = CONFIGS["bf16_n16384_m4m_r512_q3"]
    assert bench.product_kernel("bf16_split", "sample_side", big) == "k_gemm16_sample_side_rs"
    assert bench.product_kernel("bf16_split", "param_side", big) == "k_gemm16_param_side_rs"
    assert bench.product_kernel("bf16x2", "param_side", big) == "k_gemm16_param_side_dma"
    c2 = CONFIGS["f32_n8192_m100k_r256"]
    assert bench.product_kernel("f32", "param_side", c2) == "k_gemm_param_side_dma"
    assert bench.column_tile("bf16", 512, "param_side") == 512
    assert bench.column_tile("f32", 16, "sample_side") == 32
