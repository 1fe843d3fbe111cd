"""MinSR / SPRING in sample space (wssr_spring through the C ABI) against the
FP64 oracle's spring_step (Sec. 3.2): ragged N (partial Cholesky panels and
update tiles) and M, with and without momentum, the BF16 storage forms
against the oracle on the stored values, the damped full-rank identity with
the plain step, and argument errors."""
import numpy as np
import pytest
import torch

from oracle import wssr_oracle as orc
from tests.metrics import rel
from workloads import random_problem

pytestmark = pytest.mark.gpu

# Everything is FP64 from exact products of the stored values: the error is
# rounding times the condition number of T + lambda I (about 1e3 here).
TOL = 1e-8


def _np(t):
    return t.detach().double().cpu().numpy()


def _max_rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.mark.parametrize("n,m", [(300, 1000), (700, 3001), (1030, 2500), (129, 5003), (64, 200)])
@pytest.mark.parametrize("mom", [0.0, 0.9])
def test_spring_against_oracle(n, m, mom):
    from paper_2512_05749_amd import Wssr
    o, e, _ = random_problem(n, m, 8, seed=n + m, device="cuda", alpha=1.1)
    gen = torch.Generator(device="cuda").manual_seed(n)
    prev = torch.randn(m, generator=gen, device="cuda", dtype=torch.float64) * 1e-2
    h = Wssr(n_max=n, m_max=m, r_max=8, q_max=2, sample_space=True)
    try:
        dth = prev.clone()
        delta = h.spring(o, e, 1e-3, momentum=mom, eta=0.05, dtheta=dth)
        code, diag = h.status()
        assert code == 0, (code, diag)
        ref = orc.spring_step(_np(o), _np(e), _np(prev), 1e-3, mom, 0.05)
        d_err, d_max = rel(_np(delta), ref["delta"]), _max_rel(_np(delta), ref["delta"])
        print(f"n={n} m={m} momentum={mom}: delta {d_err:.2e} (element-wise {d_max:.2e})")
        assert d_err <= TOL and d_max <= TOL
        assert rel(_np(dth), ref["dtheta"]) <= TOL
    finally:
        h.close()


@pytest.mark.parametrize("form", ["bf16", "bf16x2"])
def test_spring_bf16_forms_on_the_stored_values(form):
    from paper_2512_05749_amd import Wssr
    n, m = 600, 4000
    o, e, _ = random_problem(n, m, 8, seed=77, device="cuda", alpha=1.1)
    h = Wssr(n_max=n, m_max=m, r_max=8, q_max=2, dtype=form, sample_space=True)
    try:
        stored = h.storage_like(n, m)
        h.ingest(o, e, 0, out=stored)
        prev = torch.randn(m, device="cuda", dtype=torch.float64) * 1e-2
        dth = prev.clone()
        delta = h.spring(stored, e, 1e-3, momentum=0.5, eta=0.1, dtheta=dth)
        assert h.status()[0] == 0
        vals = stored.double() if form == "bf16" else stored[0].double() + stored[1].double()
        ref = orc.spring_step(_np(vals), _np(e), _np(prev), 1e-3, 0.5, 0.1)
        assert rel(_np(delta), ref["delta"]) <= TOL
        assert rel(_np(dth), ref["dtheta"]) <= TOL
        unr = orc.spring_step(_np(o), _np(e), _np(prev), 1e-3, 0.5, 0.1)
        print(f"{form}: against the unrounded O {rel(_np(delta), unr['delta']):.2e}")
    finally:
        h.close()


def test_minsr_is_the_full_rank_limit_of_the_step():
    """Momentum 0: delta is (S + lambda I)^{-1} g, which the plain step reaches
    at full rank (r = N - 1 = rank of the centred O)."""
    from paper_2512_05749_amd import Wssr
    n, m = 129, 700
    o, e, v = random_problem(n, m, n - 1, seed=5, device="cuda", alpha=1.0)
    h = Wssr(n_max=n, m_max=m, r_max=n - 1, q_max=8, sample_space=True)
    try:
        d_minsr = h.spring(o, e, 1e-2)
        d_step, _ = h.step(o, e, v, 1e-2, q=8)
        assert h.status()[0] == 0
        assert rel(_np(d_step), _np(d_minsr)) <= 1e-4
        assert rel(_np(d_minsr), orc.sr_direct(_np(o), _np(e), 1e-2)) <= TOL
    finally:
        h.close()


def test_spring_rejects_bad_arguments():
    from paper_2512_05749_amd import Wssr
    from paper_2512_05749_amd.wssr import WssrError
    n, m = 100, 300
    o, e, _ = random_problem(n, m, 8, seed=3, device="cuda")
    h = Wssr(n_max=n, m_max=m, r_max=8, q_max=2)
    try:
        with pytest.raises(WssrError):                  # no sample-space workspace
            h.spring(o, e, 1e-3)
    finally:
        h.close()
    h = Wssr(n_max=n, m_max=m, r_max=8, q_max=2, sample_space=True)
    try:
        for lam, mom in ((0.0, 0.0), (1e-3, 1.0), (1e-3, -0.1)):
            with pytest.raises(WssrError):
                h.spring(o, e, lam, momentum=mom, dtheta=torch.zeros(m, dtype=torch.float64, device="cuda"))
        with pytest.raises(WssrError):                  # momentum without dtheta
            h.spring(o, e, 1e-3, momentum=0.5)
    finally:
        h.close()
