"""The batched form: many independent steps of uneven N, M, r and lambda in one
call, spread over concurrent lanes (optionally one replayed HIP graph).  Every
problem is checked against the FP64 oracle and against the same step run on
its own (bit for bit)."""
import numpy as np
import pytest
import torch

from oracle import wssr_oracle as orc
from tests.metrics import orth_err, rel, sigma_rel_gated, weighted_projector_err
from workloads import random_problem

pytestmark = pytest.mark.gpu


def _np(t):
    return t.detach().double().cpu().numpy()


def _problems(count=16, seed=4000):
    """Uneven problems: N in {128, 256, 512, 1024}, M uniform in [500, 4000],
    r in {8, 16, 32}, lambda log-uniform in [1e-4, 1e-2], spectrum k^-a with
    a uniform in [1.0, 1.5] (the batched workload's recipe, scaled down)."""
    rng = np.random.default_rng(seed)
    out = []
    for j in range(count):
        n = int(rng.choice([128, 256, 512, 1024]))
        m = int(rng.integers(500, 4001))
        r = int(rng.choice([8, 16, 32]))
        lam = float(10 ** rng.uniform(-4, -2))
        a = float(rng.uniform(1.0, 1.5))
        o, e, v = random_problem(n, m, r, seed=seed + j, alpha=a, device="cuda")
        out.append(dict(O=o, e_l=e, V=v, lam=lam, q=2))
    return out


def _copy(problems):
    return [dict(p, V=p["V"].clone()) for p in problems]


@pytest.fixture(scope="module")
def batch():
    return _problems()


def _single_results(problems):
    from paper_2512_05749_amd import Wssr
    h = Wssr(n_max=1024, m_max=4000, r_max=32, q_max=4)
    res = []
    for p in _copy(problems):
        d, s = h.step(p["O"], p["e_l"], p["V"], p["lam"], q=p["q"])
        assert h.status()[0] == 0
        res.append((d.clone(), s.clone(), p["V"]))
    h.close()
    return res


@pytest.mark.parametrize("lanes", [0, 4])
def test_batch_matches_oracle_and_single_steps(batch, lanes):
    from paper_2512_05749_amd import Wssr
    h = Wssr(n_max=1024, m_max=4000, r_max=32, q_max=4, lanes=lanes)
    probs = _copy(batch)
    v_in = [p["V"].clone() for p in probs]
    outs = h.step_batched(probs)
    codes = h.batched_status(len(probs))
    h.close()
    assert codes == [0] * len(probs)
    single = _single_results(batch)
    for j, (p, (d, s)) in enumerate(zip(probs, outs)):
        # the same kernels in the same configuration: identical results
        assert torch.equal(d, single[j][0]) and torch.equal(s, single[j][1]) and torch.equal(p["V"], single[j][2])
        ref = orc.wssr_step(_np(p["O"]), _np(p["e_l"]), _np(v_in[j]), p["lam"], p["V"].shape[1], p["q"])
        assert rel(_np(d), ref["delta"]) <= 1e-4, j
        assert sigma_rel_gated(_np(s), ref["sigma"], p["lam"]) <= 1e-4, j
        assert orth_err(_np(p["V"])) <= 1e-5
        w_g = orc.woodbury_weights(_np(s), p["lam"])
        w_o = orc.woodbury_weights(ref["sigma"], p["lam"])
        assert weighted_projector_err(_np(p["V"]), w_g, ref["v"], w_o) <= 1e-4, j


@pytest.mark.skip(reason="graph capture of the batched step is switched off: its first device run ended in a "
                         "host segmentation fault whose cause is not found yet")
def test_graph_replays_match_eager(batch):
    """One captured graph replayed three times, with eager work (restoring the
    warm starts) between the replays; every replay equals the eager batch."""
    from paper_2512_05749_amd import Wssr
    eager = Wssr(n_max=1024, m_max=4000, r_max=32, q_max=4, lanes=4)
    ref_probs = _copy(batch)
    ref = [(d.clone(), s.clone()) for d, s in eager.step_batched(ref_probs)]
    assert eager.batched_status(len(batch)) == [0] * len(batch)
    eager.close()

    h = Wssr(n_max=1024, m_max=4000, r_max=32, q_max=4, lanes=4, graph=True)
    probs = _copy(batch)
    v0 = [p["V"].clone() for p in batch]
    deltas = [torch.empty(p["V"].shape[0], dtype=torch.float64, device="cuda") for p in probs]
    sigmas = [torch.empty(p["V"].shape[1], dtype=torch.float64, device="cuda") for p in probs]
    for p, d, s in zip(probs, deltas, sigmas):
        p["delta"], p["sigma"] = d, s
    for rep in range(3):
        for p, v in zip(probs, v0):
            p["V"].copy_(v)              # eager work between the replays
        deltas_before = [d.clone().fill_(float("nan")) for d in deltas]
        for d, db in zip(deltas, deltas_before):
            d.copy_(db)
        h.step_batched(probs)
        assert h.batched_status(len(probs)) == [0] * len(probs), rep
        torch.cuda.synchronize()
        for j, p in enumerate(probs):
            assert torch.equal(deltas[j], ref[j][0]), (rep, j)
            assert torch.equal(sigmas[j], ref[j][1]), (rep, j)
            assert torch.equal(p["V"], ref_probs[j]["V"]), (rep, j)
    from paper_2512_05749_amd.wssr import lib
    assert h.graph_active(), lib().wssr_last_error(h._h).decode()
    h.close()


def test_tuner_keeps_inputs_and_results(batch):
    """The autotuner times the batch on scratch copies (the problems' V stays
    as it was) and the tuned batch still meets the oracle tolerances."""
    from paper_2512_05749_amd import Wssr
    h = Wssr(n_max=1024, m_max=4000, r_max=32, q_max=4, lanes=4)
    probs = _copy(batch[:8])
    v_in = [p["V"].clone() for p in probs]
    lanes, div, ms = h.tune_batched(probs, reps=1)
    assert 1 <= lanes <= 4 and div in (1, lanes) and ms > 0
    assert all(torch.equal(p["V"], v) for p, v in zip(probs, v_in))
    outs = h.step_batched(probs)
    assert h.batched_status(len(probs)) == [0] * len(probs)
    for j, (p, (d, s)) in enumerate(zip(probs, outs)):
        ref = orc.wssr_step(_np(p["O"]), _np(p["e_l"]), _np(v_in[j]), p["lam"], p["V"].shape[1], p["q"])
        assert rel(_np(d), ref["delta"]) <= 1e-4, j
    h.close()


def test_graph_flag_is_rejected_while_switched_off():
    from paper_2512_05749_amd import Wssr, WssrError
    with pytest.raises(WssrError):
        Wssr(n_max=64, m_max=100, r_max=4, lanes=2, graph=True)


def test_batch_errors_stay_per_problem(batch):
    from paper_2512_05749_amd import Wssr, WssrError
    h = Wssr(n_max=1024, m_max=4000, r_max=32, q_max=4, lanes=3)
    probs = _copy(batch[:5])
    probs[2]["e_l"] = probs[2]["e_l"].clone()
    probs[2]["e_l"][3] = float("nan")
    v_before = probs[2]["V"].clone()
    h.step_batched(probs)
    codes = h.batched_status(5)
    assert codes[2] == -5 and all(c == 0 for i, c in enumerate(codes) if i != 2)
    assert torch.equal(probs[2]["V"], v_before)
    bad = _copy(batch[:2])
    bad[1]["V"] = torch.zeros(bad[1]["O"].shape[1], bad[1]["O"].shape[0], device="cuda")   # r > n - 1
    with pytest.raises(WssrError):
        h.step_batched(bad)
    h.close()


@pytest.mark.timeout(900)
def test_batch_at_the_batched_workload_ranks():
    """Lanes with problems at the batched workload's ranks and sample counts
    (r in {64, 128, 256}, N in {2048, 4096}), with M reduced so that the
    oracle runs in seconds: per-problem status, parity with the oracle at the
    FP32 bars, and bit-identity with single steps."""
    from paper_2512_05749_amd import Wssr
    shapes = [(2048, 5000, 64), (4096, 3000, 128), (2048, 6000, 256), (4096, 4500, 64), (2048, 2500, 128),
              (4096, 5000, 256)]
    rng = np.random.default_rng(77)
    probs = []
    for j, (n, m, r) in enumerate(shapes):
        a = float(rng.uniform(1.0, 1.5))
        lam = float(10 ** rng.uniform(-4, -2))
        o, e, v = random_problem(n, m, r, seed=900 + j, alpha=a, eta=1e-4, el_mean=-10.0, el_std=0.5,
                                 device="cuda")
        probs.append(dict(O=o, e_l=e, V=v, lam=lam, q=2))
    v_in = [p["V"].clone() for p in probs]
    h = Wssr(n_max=4096, m_max=6000, r_max=256, q_max=2, lanes=4)
    work = _copy(probs)
    outs = h.step_batched(work)
    codes = h.batched_status(len(work))
    h.close()
    assert codes == [0] * len(work)
    hs = Wssr(n_max=4096, m_max=6000, r_max=256, q_max=2)
    for j, (p, (d, s)) in enumerate(zip(work, outs)):
        vv = v_in[j].clone()
        d1, s1 = hs.step(p["O"], p["e_l"], vv, p["lam"], q=2)
        assert hs.status()[0] == 0
        assert torch.equal(d, d1) and torch.equal(s, s1) and torch.equal(p["V"], vv), j
        ref = orc.wssr_step(_np(p["O"]), _np(p["e_l"]), _np(v_in[j]), p["lam"], p["V"].shape[1], 2)
        assert rel(_np(d), ref["delta"]) <= 1e-4, j
        assert float(np.abs(_np(d) - ref["delta"]).max() / np.abs(ref["delta"]).max()) <= 1e-4, j
        assert sigma_rel_gated(_np(s), ref["sigma"], p["lam"]) <= 1e-4, j
        assert orth_err(_np(p["V"])) <= 1e-5, j
    hs.close()
