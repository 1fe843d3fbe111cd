"""Pins for the FP64 oracle: each test checks it against something other than
itself -- hand-derived closed forms, LAPACK through numpy, identities, invariances
and convergence theory.  CPU only."""
import json
import pathlib

import numpy as np
import pytest

from oracle import wssr_oracle as orc

GOLDEN = pathlib.Path(__file__).parent / "golden"
rng0 = np.random.default_rng


def _problem(n, m, seed, spectrum=None, noise=1e-3, mean_shift=0.3):
    """Small random problem with a decaying spectrum (plain numpy, test-local)."""
    rng = rng0(seed)
    k = min(n, m)
    u = np.linalg.qr(rng.standard_normal((n, k)))[0]
    w = np.linalg.qr(rng.standard_normal((m, k)))[0]
    s = spectrum if spectrum is not None else np.arange(1, k + 1) ** -1.2
    o = np.sqrt(n) * (u * s) @ w.T + noise * rng.standard_normal((n, m))
    o += mean_shift * rng.standard_normal(m)[None, :]
    e_l = -1.0 + 0.1 * rng.standard_normal(n)
    return o, e_l


def _rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b)


# --------------------------------------------------------------- golden examples

def test_golden_hand_examples():
    cases = json.loads((GOLDEN / "hand_examples.json").read_text())["cases"]
    c1, c2 = cases
    o, e = np.array(c1["O"], float), np.array(c1["E_L"], float)
    np.testing.assert_allclose(orc.gradient(o, e), c1["g"], atol=1e-15)
    np.testing.assert_allclose(orc.sr_direct(o, e, c1["lam"]), c1["delta_full"], atol=1e-14)
    res = orc.wssr_step(o, e, np.array(c1["V_in"]), c1["lam"], c1["r"], 1)
    np.testing.assert_allclose(res["delta"], c1["delta_damped"], atol=1e-14)
    np.testing.assert_allclose(res["sigma"], c1["sigma"], atol=1e-14)
    np.testing.assert_allclose(res["v"], c1["V"], atol=1e-14)

    o, e = np.array(c2["O"], float), np.array(c2["E_L"], float)
    lam = c2["lam"]
    np.testing.assert_allclose(orc.gradient(o, e), c2["g"], atol=1e-15)
    np.testing.assert_allclose(orc.sr_direct(o, e, lam), c2["delta_full"], atol=1e-14)
    np.testing.assert_allclose(orc.sr_pushthrough(o, e, lam), c2["delta_full"], atol=1e-14)
    for key, r, q in (("r1", 1, 80), ("r2", 2, 1)):
        sub = c2[key]
        vin = np.array(sub["V_in"], float)
        for pre in ("damped", "floor"):
            res = orc.wssr_step(o, e, vin, lam, r, q, precond=pre)
            np.testing.assert_allclose(res["delta"], sub["delta_" + pre], atol=1e-13)
        np.testing.assert_allclose(res["sigma"], c2["sigma"][:r], atol=1e-13)
        np.testing.assert_allclose(res["v"], sub["V"], atol=1e-12)


def test_s_matrix_hand_values_and_loop_sum():
    """S = O_bar^T O_bar / N (eq. SN with the 1/N of eq. Osrn): the hand-derived
    S of both golden cases, and an element-by-element loop over samples."""
    for c in json.loads((GOLDEN / "hand_examples.json").read_text())["cases"]:
        np.testing.assert_allclose(orc.s_matrix(np.array(c["O"], float)), c["S"], atol=1e-15)
    o, _ = _problem(7, 5, seed=21)
    n, m = o.shape
    mu = [sum(o[k, j] for k in range(n)) / n for j in range(m)]
    loop = np.array([[sum((o[k, i] - mu[i]) * (o[k, j] - mu[j]) for k in range(n)) / n for j in range(m)]
                     for i in range(m)])
    np.testing.assert_allclose(orc.s_matrix(o), loop, rtol=1e-13, atol=1e-15)


# --------------------------------------------------------------- building blocks

@pytest.mark.parametrize("n", [1, 2, 7, 30])
def test_cholesky_and_triangular_vs_lapack(n):
    rng = rng0(n)
    x = rng.standard_normal((n + 3, n))
    g = x.T @ x + 0.1 * np.eye(n)
    low = orc.cholesky_lower(g)
    np.testing.assert_allclose(low, np.linalg.cholesky(g), rtol=1e-12, atol=1e-13)
    b = rng.standard_normal((n, 3))
    np.testing.assert_allclose(orc.spd_solve(g, b), np.linalg.solve(g, b), rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(orc.solve_upper(low.T, b), np.linalg.solve(low.T, b), rtol=1e-10,
                               atol=1e-12)


def test_cholesky_rejects_indefinite():
    with pytest.raises(np.linalg.LinAlgError):
        orc.cholesky_lower(np.array([[1.0, 2.0], [2.0, 1.0]]))


@pytest.mark.parametrize("shape", [(12, 5), (40, 40), (9, 1), (64, 33)])
def test_qr_positive(shape):
    x = rng0(3).standard_normal(shape)
    q, r = orc.qr_positive(x)
    np.testing.assert_allclose(q @ r, x, atol=1e-13)
    np.testing.assert_allclose(q.T @ q, np.eye(shape[1]), atol=1e-13)
    assert np.all(np.diag(r) > 0) and np.allclose(np.tril(r, -1), 0)


@pytest.mark.parametrize("kind", ["random", "graded", "rank_deficient", "odd", "wide", "diag"])
def test_jacobi_svd_vs_lapack(kind):
    rng = rng0(11)
    if kind == "random":
        c = rng.standard_normal((24, 24))
    elif kind == "graded":   # singular values spanning 12 decades (Demmel-Veselic test class)
        qa = np.linalg.qr(rng.standard_normal((20, 20)))[0]
        qb = np.linalg.qr(rng.standard_normal((20, 20)))[0]
        c = (qa * np.logspace(0, -12, 20)) @ qb.T
    elif kind == "rank_deficient":
        c = rng.standard_normal((16, 5)) @ rng.standard_normal((5, 16))
    elif kind == "odd":
        c = rng.standard_normal((13, 13))
    elif kind == "wide":
        c = rng.standard_normal((6, 15))
    else:
        c = np.diag([3.0, -1.0, 2.0, 0.0, 5.0])
    u, s, p = orc.jacobi_svd(c)
    ref = np.linalg.svd(c, compute_uv=False)
    k = min(c.shape)
    np.testing.assert_allclose(s[:k], ref, rtol=1e-12, atol=1e-13 * ref[0])
    assert np.all(s[k:] <= 1e-13 * ref[0])
    np.testing.assert_allclose(p.T @ p, np.eye(c.shape[1]), atol=1e-13)
    np.testing.assert_allclose((u * s) @ p.T, c, atol=1e-13 * ref[0])
    assert np.all(np.diff(s) <= 0)
    # singular subspaces where the gap is clear: compare projectors with LAPACK
    _, _, vt = np.linalg.svd(c)
    for j in range(k - 1):
        if ref[j] - ref[j + 1] > 1e-3 * ref[0] and (j == 0 or ref[j - 1] - ref[j] > 1e-3 * ref[0]):
            assert abs(abs(p[:, j] @ vt[j]) - 1) < 1e-10


# --------------------------------------------------------------- P1, P2: direct solves

@pytest.mark.parametrize("n,m", [(8, 20), (40, 30), (64, 200)])
def test_p1_direct_solve_vs_numpy(n, m):
    o, e = _problem(n, m, seed=n + m)
    lam = 1e-3
    a = (o - o.mean(0)) / np.sqrt(n)
    g_ref = a.T @ (e - e.mean()) / np.sqrt(n)
    ref = np.linalg.solve(a.T @ a + lam * np.eye(m), g_ref)
    assert _rel(orc.sr_direct(o, e, lam), ref) < 1e-10


@pytest.mark.parametrize("n,m", [(8, 20), (40, 30), (64, 200), (100, 60)])
def test_p2_pushthrough_equals_direct(n, m):
    o, e = _problem(n, m, seed=3 * n + m)
    for lam in (1e-2, 1e-4):
        assert _rel(orc.sr_pushthrough(o, e, lam), orc.sr_direct(o, e, lam)) < 1e-9


def test_gradient_definition_by_loop():
    """g_m = (1/N) sum_n (O[n,m] - mu_m)(E_L[n] - mean E_L): per-entry brute force."""
    o, e = _problem(9, 5, seed=4)
    g = orc.gradient(o, e)
    for m in range(5):
        mu = sum(o[n, m] for n in range(9)) / 9
        el = sum(e) / 9
        ref = sum((o[n, m] - mu) * (e[n] - el) for n in range(9)) / 9
        assert abs(g[m] - ref) < 1e-14


# --------------------------------------------------------------- P3: exactness at full rank

@pytest.mark.parametrize("n,m,q", [(10, 30, 1), (24, 50, 2), (17, 17, 3)])
def test_p3_exact_at_full_rank(n, m, q):
    o, e = _problem(n, m, seed=n * m)
    r = n - 1            # rank of the centred matrix
    vin = rng0(1).standard_normal((m, r))
    lam = 1e-3
    res = orc.wssr_step(o, e, vin, lam, r, q)
    assert _rel(res["delta"], orc.sr_direct(o, e, lam)) < 1e-9
    ref_s = np.linalg.svd((o - o.mean(0)) / np.sqrt(n), compute_uv=False)[:r]
    np.testing.assert_allclose(res["sigma"], ref_s, rtol=1e-9)


# --------------------------------------------------------------- P4, P5: fixed point, orthonormality

@pytest.mark.parametrize("q", [1, 3])
def test_p4_fixed_point(q):
    n, m, r = 40, 70, 6
    o, e = _problem(n, m, seed=5)
    v_ex, s_ex = orc.exact_topr(o, r)
    res = orc.wssr_step(o, e, v_ex, 1e-3, r, q)
    np.testing.assert_allclose(res["v"], v_ex, atol=1e-11)
    np.testing.assert_allclose(res["sigma"], s_ex, rtol=1e-12)
    assert _rel(res["delta"], orc.delta_exact_r(o, e, 1e-3, r)) < 1e-11
    # the exact vectors themselves agree with LAPACK's SVD of A
    _, s_l, vt = np.linalg.svd((o - o.mean(0)) / np.sqrt(n))
    np.testing.assert_allclose(s_ex, s_l[:r], rtol=1e-12)
    np.testing.assert_allclose(np.abs(np.sum(v_ex * vt[:r].T, axis=0)), 1, atol=1e-10)


def test_p5_orthonormal_output():
    o, e = _problem(50, 120, seed=6)
    res = orc.wssr_step(o, e, rng0(2).standard_normal((120, 9)), 1e-3, 9, 2)
    assert np.abs(res["v"].T @ res["v"] - np.eye(9)).max() < 1e-13


# --------------------------------------------------------------- P7: convergence rate

def test_p7_convergence_rate():
    n, m, r = 60, 90, 5
    spec = np.concatenate([[1.0, 0.9, 0.8, 0.7, 0.6], 0.3 * 0.9 ** np.arange(n - 5)])
    o, e = _problem(n, m, seed=7, spectrum=spec, noise=0.0, mean_shift=0.0)
    lam = 1e-2
    ref = orc.delta_exact_r(o, e, lam, r)
    vin = rng0(3).standard_normal((m, r))
    errs = [_rel(orc.wssr_step(o, e, vin, lam, r, q)["delta"], ref) for q in range(1, 8)]
    assert all(b < a for a, b in zip(errs, errs[1:]))
    s = np.linalg.svd((o - o.mean(0)) / np.sqrt(n), compute_uv=False)
    rate = (s[r] / s[r - 1]) ** 2
    fitted = np.exp(np.polyfit(np.arange(3, 8), np.log(errs[2:]), 1)[0])
    assert 0.5 * rate < fitted < 1.5 * rate


# --------------------------------------------------------------- P8: closed form

def test_p8_closed_form_noise_free():
    n, m, k = 30, 50, 8
    rng = rng0(8)
    u = np.linalg.qr(np.concatenate([np.ones((n, 1)), rng.standard_normal((n, k))], 1))[0][:, 1:]
    w = np.linalg.qr(rng.standard_normal((m, k)))[0]
    s = np.array([2.0, 1.5, 1.0, 0.5, 0.2, 0.1, 0.05, 0.01])
    o = np.sqrt(n) * (u * s) @ w.T + rng.standard_normal(m)[None, :]   # constant row shift
    e = rng.standard_normal(n)
    lam = 1e-2
    g = orc.gradient(o, e)
    closed = w @ ((w.T @ g) / (s ** 2 + lam)) + (g - w @ (w.T @ g)) / lam
    assert _rel(orc.sr_direct(o, e, lam), closed) < 1e-10
    res = orc.wssr_step(o, e, rng.standard_normal((m, k)), lam, k, 2)
    np.testing.assert_allclose(res["sigma"], s, rtol=1e-10)
    np.testing.assert_allclose(np.abs(np.sum(res["v"] * w, 0)), 1, atol=1e-10)
    assert _rel(res["delta"], closed) < 1e-10


# --------------------------------------------------------------- P9: invariances

def test_p9_invariances():
    n, m, r, q, lam = 25, 40, 4, 2, 1e-3
    o, e = _problem(n, m, seed=9)
    rng = rng0(9)
    vin = rng.standard_normal((m, r))
    base = orc.wssr_step(o, e, vin, lam, r, q)
    perm = rng.permutation(n)
    r1 = orc.wssr_step(o[perm], e[perm], vin, lam, r, q)
    assert _rel(r1["delta"], base["delta"]) < 1e-11
    r2 = orc.wssr_step(o + rng.standard_normal(m)[None, :], e + 7.0, vin, lam, r, q)
    assert _rel(r2["delta"], base["delta"]) < 1e-10
    c = 3.0
    r3 = orc.wssr_step(c * o, e, vin, c * c * lam, r, q)
    assert _rel(r3["delta"], base["delta"] / c) < 1e-11
    np.testing.assert_allclose(r3["sigma"], c * base["sigma"], rtol=1e-12)
    pm = rng.permutation(m)
    dsg = np.where(rng.random(m) < 0.5, -1.0, 1.0)
    # O -> O Pi D  (column j of the new O is d_j * O[:, pm[j]])
    r4 = orc.wssr_step(o[:, pm] * dsg, e, vin[pm] * dsg[:, None], lam, r, q)
    assert _rel(r4["delta"], base["delta"][pm] * dsg) < 1e-11
    r5 = orc.wssr_step(o, np.full(n, -2.5), vin, lam, r, q)
    assert np.abs(r5["delta"]).max() == 0.0


# --------------------------------------------------------------- P10: limits

def test_p10_large_damping_limit():
    o, e = _problem(20, 30, seed=10)
    g = orc.gradient(o, e)
    for lam in (1e6, 1e9):
        res = orc.wssr_step(o, e, rng0(0).standard_normal((30, 3)), lam, 3, 2)
        s1 = res["sigma"][0] ** 2
        assert _rel(lam * res["delta"], g) < 2 * s1 / lam


# --------------------------------------------------------------- P11: the two forms of C

def test_p11_projection_identity():
    """Q_Y^T A Q_Z = (R_Z R_Y^{-1})^T when Z = A^T Y and Y has full rank."""
    o, e = _problem(30, 45, seed=11)
    a = (o - o.mean(0)) / np.sqrt(30)
    v = orc.qr_positive(rng0(4).standard_normal((45, 6)))[0]
    y = a @ v
    z = a.T @ y
    qy, ry = orc.qr_positive(y)
    qz, rz = orc.qr_positive(z)
    c1 = qy.T @ (a @ qz)
    c2 = (rz @ np.linalg.inv(ry)).T
    np.testing.assert_allclose(c1, c2, atol=1e-12 * np.abs(c1).max())


def test_stage_products_by_loops():
    """The stage helpers the GPU stage tests compare against, checked against
    element-by-element sums on a tiny input: Y = A V, Z = A^T X and G = X^T X with
    A = (O - 1 mu^T)/sqrt(N) (eqs. Osr, Osrn)."""
    rng = rng0(21)
    n, m, r = 5, 7, 3
    o = rng.standard_normal((n, m)) + 2.0
    v = rng.standard_normal((m, r))
    x = rng.standard_normal((n, r))
    mu = [sum(o[i, j] for i in range(n)) / n for j in range(m)]
    y = np.zeros((n, r))
    z = np.zeros((m, r))
    for i in range(n):
        for k in range(r):
            y[i, k] = sum((o[i, j] - mu[j]) * v[j, k] for j in range(m)) / np.sqrt(n)
    for j in range(m):
        for k in range(r):
            z[j, k] = sum((o[i, j] - mu[j]) * x[i, k] for i in range(n)) / np.sqrt(n)
    gx = np.array([[sum(x[i, a] * x[i, b] for i in range(n)) for b in range(r)] for a in range(r)])
    assert _rel(orc.gemm_sample_side(o, v), y) < 1e-14
    assert _rel(orc.gemm_param_side(o, x), z) < 1e-14
    assert _rel(orc.gram(x), gx) < 1e-14
    # the sample-side product of a centred matrix has zero column sums
    assert np.abs(orc.gemm_sample_side(o, v).sum(0)).max() < 1e-12


def test_subspace_distance_closed_form():
    """span(e1, e2) against span(e1, cos t e2 + sin t e3): largest principal angle t."""
    t = 0.3
    v1 = np.eye(4)[:, :2]
    v2 = np.stack([np.eye(4)[:, 0], np.cos(t) * np.eye(4)[:, 1] + np.sin(t) * np.eye(4)[:, 2]], 1)
    assert abs(orc.subspace_distance(v1, 3.0 * v2) - np.sin(t)) < 1e-14
    assert orc.subspace_distance(v1, v1 @ np.array([[0.0, 2.0], [1.0, 1.0]])) < 1e-7


def test_woodbury_general_core_equals_dense_inverse():
    """Woodbury apply for a non-orthonormal V equals the dense (V S^2 V^T + lam I)^{-1} g."""
    rng = rng0(12)
    v = rng.standard_normal((25, 4))
    s = np.array([1.0, 0.5, 0.1, 0.0])
    g = rng.standard_normal(25)
    lam = 0.05
    dense = np.linalg.solve((v * s**2) @ v.T + lam * np.eye(25), g)
    assert _rel(orc.woodbury_apply(v, s, g, lam), dense) < 1e-12


def test_sign_rule():
    v = np.array([[1.0, 0.0], [0.0, -1.0], [0.0, 0.0]])
    ref = np.array([[-1.0, 0.0], [0.0, 0.0], [0.0, 1.0]])
    out = orc.fix_signs(v, ref)
    np.testing.assert_allclose(out, [[-1.0, 0.0], [0.0, 1.0], [0.0, 0.0]])


def test_step_rejects_bad_arguments():
    o, e = _problem(10, 12, seed=13)
    vin = np.ones((12, 3))
    with pytest.raises(ValueError):
        orc.wssr_step(o, e, vin, 1e-3, 10, 1)      # r > N - 1
    with pytest.raises(ValueError):
        orc.wssr_step(o, e, vin, 0.0, 3, 1)
    with pytest.raises(ValueError):
        orc.wssr_step(o, e, vin, 1e-3, 3, 0)
    o2 = o.copy()
    o2[3, 4] = np.nan
    with pytest.raises(FloatingPointError):
        orc.wssr_step(o2, e, vin, 1e-3, 3, 1)


# --------------------------------------------------------------- planted mistakes

def test_planted_mistakes_are_caught(monkeypatch):
    """A plausible slip in the oracle (factor 2 in g, no centring of O, a transposed
    projection) must fail at least one pin; run the pins against each slip."""
    cases = json.loads((GOLDEN / "hand_examples.json").read_text())["cases"]
    c2 = cases[1]
    o, e = np.array(c2["O"], float), np.array(c2["E_L"], float)

    def pins_pass():
        try:
            np.testing.assert_allclose(orc.gradient(o, e), c2["g"], atol=1e-14)
            np.testing.assert_allclose(orc.sr_direct(o, e, 1.0), c2["delta_full"], atol=1e-13)
            res = orc.wssr_step(o, e, np.eye(2), 1.0, 2, 1)
            np.testing.assert_allclose(res["delta"], c2["r2"]["delta_damped"], atol=1e-13)
            test_p11_projection_identity()
            test_p3_exact_at_full_rank(10, 30, 1)
        except AssertionError:
            return False
        return True

    assert pins_pass()
    real_center = orc.center_columns
    real_grad = orc.gradient
    real_scaled = orc.scaled_centered
    monkeypatch.setattr(orc, "gradient", lambda o_, e_: 2 * real_grad(o_, e_))
    assert not pins_pass()
    monkeypatch.setattr(orc, "gradient", real_grad)
    monkeypatch.setattr(orc, "center_columns", lambda o_: np.asarray(o_, float))
    assert not pins_pass()
    monkeypatch.setattr(orc, "center_columns", real_center)
    monkeypatch.setattr(orc, "scaled_centered", lambda o_: real_scaled(o_) * np.sqrt(o_.shape[0]))
    assert not pins_pass()
    monkeypatch.setattr(orc, "scaled_centered", real_scaled)
    assert pins_pass()


# --------------------------------------------------------------- averaged state (Sec. 4.1)

def _avg_problem(n, m, seed):
    o, e = _problem(n, m, seed, spectrum=np.linspace(1.0, 0.3, min(n, m)), noise=0.05)
    return o, e


def _avg_chain(n, m, avg, ranks, seed, lam=0.3, q=2):
    """Run averaged steps with the given rank per step; yield each step's
    inputs and result."""
    rng = rng0(seed)
    state = None
    for k, r in enumerate(ranks):
        o, e = _avg_problem(n, m, seed + 1 + k)
        v_in = rng.standard_normal((m, r))
        res = orc.averaged_step(o, e, v_in, state, lam, r, q, avg)
        yield o, e, res
        state = dict(v=res["v"], sigma=res["sigma"], l=res["l"])


@pytest.mark.parametrize("avg", [0.3, 0.7, 0.95])
def test_averaged_exact_svd_is_the_running_average(avg):
    """The remark after eq. barS: with an SVD that truncates nothing (rank r
    equal to the rank of the stacked matrix), Sbar^(k) = avg Sbar^(k-1) +
    (1-avg) S_N and gbar^(k) = avg gbar^(k-1) + (1-avg) g_N, from zero.  The
    gradient recursion holds only if the stored vector L reproduces the old
    gradient through the stored matrix (Obar L = Ohat Lhat), so it pins eq.
    Lbar, the singular-vector signs and the stacking weights."""
    n, m, lam = 5, 9, 0.3
    ranks = [4, 8, 9, 9]            # rank of the stacked matrix: min(k (N-1), M)
    s_prev, g_prev = np.zeros((m, m)), np.zeros(m)
    for o, e, res in _avg_chain(n, m, avg, ranks, seed=700, lam=lam):
        s_bar = (res["v"] * res["sigma"] ** 2) @ res["v"].T
        s_want = avg * s_prev + (1 - avg) * orc.s_matrix(o)
        g_want = avg * g_prev + (1 - avg) * orc.gradient(o, e)
        assert _rel(s_bar, s_want) < 1e-11
        assert _rel(res["gbar"], g_want) < 1e-11
        # the stored pair reproduces the averaged gradient: Obar L = gbar
        assert _rel(res["v"] @ (res["sigma"] * res["l"]), g_want) < 1e-10
        # the step direction: a dense solve with the averaged matrices
        assert _rel(res["delta"], np.linalg.solve(s_want + lam * np.eye(m), g_want)) < 1e-10
        s_prev, g_prev = s_want, g_want


def test_averaged_weight_zero_is_the_plain_step():
    """avg = 0 discards the history rows: the step equals the plain step."""
    n, m, r = 12, 30, 5
    o0, e0 = _avg_problem(n, m, 801)
    st = orc.averaged_step(o0, e0, rng0(1).standard_normal((m, r)), None, 0.1, r, 3, 0.5)
    state = dict(v=st["v"], sigma=st["sigma"], l=st["l"])
    o, e = _avg_problem(n, m, 802)
    v_in = rng0(2).standard_normal((m, r))
    got = orc.averaged_step(o, e, v_in, state, 1e-2, r, 3, 0.0)
    want = orc.wssr_step(o, e, v_in, 1e-2, r, 3)
    assert _rel(got["delta"], want["delta"]) < 1e-10
    assert _rel(got["sigma"], want["sigma"]) < 1e-12
    assert np.abs(got["v"] - want["v"]).max() < 1e-10
    assert _rel(got["gbar"], want["g"]) < 1e-13


def test_averaged_truncated_against_the_averaged_gram():
    """Truncated (r below the stacked rank), converged: sigma^2 and the span of
    V are the top-r eigenpairs of the averaged Gram avg U_s diag(sigma_s^2) U_s^T
    + (1-avg) S_N, formed here directly and decomposed by LAPACK; L is the
    projection of gbar on V scaled by 1/sigma (a converged singular triplet
    has sample-side vector Ohat^T v / sigma)."""
    n, m, r, avg = 40, 60, 6, 0.8
    rng = rng0(901)
    # a gap after the sixth value, so that 60 passes converge
    spec = np.r_[np.linspace(1.0, 0.6, r), 0.2 * np.linspace(1.0, 0.3, n - r)]
    o0, e0 = _problem(n, m, 902, spectrum=spec, noise=0.01)
    st = orc.averaged_step(o0, e0, rng.standard_normal((m, r)), None, 0.1, r, 60, avg)
    o = o0 + 0.02 * rng.standard_normal((n, m))     # the next step's samples: a nearby state
    e = e0 + 0.01 * rng.standard_normal(n)
    state = dict(v=st["v"], sigma=st["sigma"], l=st["l"])
    res = orc.averaged_step(o, e, st["v"], state, 0.1, r, 60, avg)
    gram = avg * (st["v"] * st["sigma"] ** 2) @ st["v"].T + (1 - avg) * orc.s_matrix(o)
    w, u = np.linalg.eigh(gram)
    w, u = w[::-1][:r], u[:, ::-1][:, :r]
    assert _rel(res["sigma"] ** 2, w) < 1e-10
    assert orc.subspace_distance(res["v"], u) < 1e-7      # the distance is a sine: floor ~sqrt(eps)
    g_want = avg * st["v"] @ (st["sigma"] * st["l"]) + (1 - avg) * orc.gradient(o, e)
    assert _rel(res["gbar"], g_want) < 1e-12
    assert _rel(res["l"], (res["v"].T @ g_want) / res["sigma"]) < 1e-8


def test_averaged_one_pass_projection_identity():
    """At any pass count the stored pair satisfies Obar L = P_V Ohat P_Y Lhat:
    with C = Q_Y^T Ohat^T Q_Z = G diag(s) P^T the Rayleigh-Ritz matrix, V =
    Q_Z P and L = G^T Q_Y^T Lhat give V diag(s) L = Q_Z C^T Q_Y^T Lhat.  At
    q = 1 the sample-side space is span(Ohat^T orth(V_in)), built here with
    LAPACK's QR from the stacked matrix written out."""
    n, m, r, avg = 30, 50, 5, 0.6
    rng = rng0(951)
    o0, e0 = _avg_problem(n, m, 952)
    st = orc.averaged_step(o0, e0, rng.standard_normal((m, r)), None, 0.1, r, 1, avg)
    o, e = _avg_problem(n, m, 953)
    v_in = rng.standard_normal((m, r))
    state = dict(v=st["v"], sigma=st["sigma"], l=st["l"])
    res = orc.averaged_step(o, e, v_in, state, 0.1, r, 1, avg)
    a = (o - o.mean(axis=0)) / np.sqrt(n)
    eps = e - e.mean()
    ahat = np.vstack([np.sqrt(1 - avg) * a, np.sqrt(avg) * (st["sigma"][:, None] * st["v"].T)])
    lhat = np.concatenate([np.sqrt(1 - avg) * eps / np.sqrt(n), np.sqrt(avg) * st["l"]])
    qy = np.linalg.qr(ahat @ np.linalg.qr(v_in)[0])[0]
    v = res["v"]
    want = v @ (v.T @ (ahat.T @ (qy @ (qy.T @ lhat))))
    assert _rel(v @ (res["sigma"] * res["l"]), want) < 1e-12


def test_averaged_rejects_bad_arguments():
    o, e = _avg_problem(6, 10, 5)
    v = np.ones((10, 3))
    for bad in (-0.1, 1.0):
        with pytest.raises(ValueError):
            orc.averaged_step(o, e, v, None, 0.1, 3, 1, bad)
    with pytest.raises(ValueError):
        orc.averaged_step(o, e, np.ones((10, 6)), None, 0.1, 6, 1, 0.5)   # r > N - 1 without history


def test_averaged_planted_mistakes_are_caught(monkeypatch):
    """Swapped stacking weights, L taken from the parameter-side rotation, and
    L without the output signs each fail the averaged pins."""
    def pins_pass():
        try:
            for avg in (0.3, 0.7):
                test_averaged_exact_svd_is_the_running_average(avg)
            test_averaged_truncated_against_the_averaged_gram()
            test_averaged_one_pass_projection_identity()
        except AssertionError:
            return False
        return True

    assert pins_pass()
    real_stack, real_l = orc.stack_averaged, orc.state_l

    def swapped(a, lbar, state, avg):
        return real_stack(a, lbar, state, 1.0 - avg) if state is not None else real_stack(a, lbar, state, avg)

    def l_from_p(last, sgn, lhat):
        return sgn * ((last["qy"] @ last["p"]).T @ lhat)

    def l_unsigned(last, sgn, lhat):
        return real_l(last, np.ones_like(sgn), lhat)

    for name, fn in (("stack_averaged", swapped), ("state_l", l_from_p), ("state_l", l_unsigned)):
        monkeypatch.setattr(orc, name, fn)
        assert not pins_pass(), (name, fn.__name__)
        monkeypatch.undo()


# --------------------------------------------------------------- randomized sketch (App. A)

def _sketch_problem(n, m, rank, seed, noise=0.0):
    rng = rng0(seed)
    u = np.linalg.qr(rng.standard_normal((n, rank)))[0]
    w = np.linalg.qr(rng.standard_normal((m, rank)))[0]
    s = np.geomspace(1.0, 0.05, rank)
    o = np.sqrt(n) * (u * s) @ w.T + noise * rng.standard_normal((n, m)) + rng.standard_normal(m)[None, :]
    return o, -1.0 + 0.1 * rng.standard_normal(n)


@pytest.mark.parametrize("q", [0, 1])
def test_sketch_exact_when_the_rank_fits(q):
    """A of rank at most r + p: Q spans its row space, so the rank-r result
    is the exact truncated SVD (LAPACK) and delta the exact-subspace Woodbury
    (against a dense solve with the rank-r S), with or without power passes."""
    n, m, rank, r, p = 40, 70, 9, 6, 4
    o, e = _sketch_problem(n, m, rank, 11)
    omega = rng0(12).standard_normal((n, r + p))
    res = orc.sketch_step(o, e, omega, 1e-2, r, q=q)
    a = (o - o.mean(axis=0)) / np.sqrt(n)
    _, s_ref, wt = np.linalg.svd(a)
    assert _rel(res["sigma"], s_ref[:r]) < 1e-12
    assert orc.subspace_distance(res["v"], wt[:r].T) < 1e-7
    s_r = (wt[:r].T * s_ref[:r] ** 2) @ wt[:r]
    g = a.T @ (e - e.mean()) / np.sqrt(n)
    assert _rel(res["delta"], np.linalg.solve(s_r + 1e-2 * np.eye(m), g)) < 1e-10


def test_sketch_within_the_randomized_bound():
    """Halko, Martinsson and Tropp's bounds (the source App. A follows): for a
    Gaussian Omega with p >= 2, the sketch's span satisfies ||A (I - Q Q^T)||
    <= (1 + 9 sqrt(r + p) sqrt(min(N, M))) sigma_{r+1} except with probability
    at most 6 p^-p (p = 8 here), and truncating to rank r adds at most
    sigma_{r+1}.  Checked on the oracle's rank-r V: ||A - A V V^T||_2 within
    the sum, against LAPACK's singular values."""
    n, m, r, p = 60, 120, 5, 8
    o, e = _sketch_problem(n, m, 30, 21, noise=1e-3)
    omega = rng0(22).standard_normal((n, r + p))
    res = orc.sketch_step(o, e, omega, 1e-2, r)
    a = (o - o.mean(axis=0)) / np.sqrt(n)
    s_ref = np.linalg.svd(a, compute_uv=False)
    v = res["v"]
    resid = np.linalg.norm(a - (a @ v) @ v.T, 2)
    assert resid <= (2 + 9 * np.sqrt(r + p) * np.sqrt(min(n, m))) * s_ref[r]
    assert resid >= s_ref[r] * (1 - 1e-12)          # no rank-r approximation does better
    # sigma are the singular values of A V, which never exceed the exact ones
    assert _rel(res["sigma"], np.linalg.svd(a @ v, compute_uv=False)) < 1e-12
    assert np.all(res["sigma"] <= s_ref[:r] * (1 + 1e-12))
    # output signs: the entry of largest magnitude of each column is positive
    k = np.argmax(np.abs(v), axis=0)
    assert np.all(v[k, np.arange(r)] > 0)


def test_sketch_power_passes_converge():
    """The power scheme tightens the randomized bound to the 1/(2q+1) power of
    its factor (Halko et al.): with q = 20 at this decaying spectrum the
    rank-r result is the exact truncated SVD (LAPACK), and no power pass
    increases ||A - A V V^T||."""
    n, m, r, p = 60, 120, 5, 5
    o, e = _sketch_problem(n, m, 30, 41, noise=1e-3)
    omega = rng0(42).standard_normal((n, r + p))
    a = (o - o.mean(axis=0)) / np.sqrt(n)
    _, s_ref, wt = np.linalg.svd(a)
    prev = np.inf
    for q in range(0, 21):
        res = orc.sketch_step(o, e, omega, 1e-2, r, q=q)
        resid = np.linalg.norm(a - (a @ res["v"]) @ res["v"].T, 2)
        assert resid <= prev * (1 + 1e-12)
        prev = resid
    assert _rel(res["sigma"], s_ref[:r]) < 1e-10
    assert orc.subspace_distance(res["v"], wt[:r].T) < 1e-7


def test_sketch_rejects_bad_arguments():
    o, e = _sketch_problem(10, 20, 5, 31)
    with pytest.raises(ValueError):
        orc.sketch_step(o, e, np.ones((9, 6)), 0.1, 4)          # wrong row count
    with pytest.raises(ValueError):
        orc.sketch_step(o, e, np.ones((10, 3)), 0.1, 4)         # fewer columns than r
    with pytest.raises(ValueError):
        orc.sketch_step(o, e, np.ones((10, 10)), 0.1, 4)        # r + p > N - 1


def test_sketch_planted_mistakes_are_caught(monkeypatch):
    """Dropping Q from the parameter-side factor, or taking the singular
    vectors from the wrong side of A Q, fails the exactness pin."""
    def pin_passes():
        try:
            test_sketch_exact_when_the_rank_fits(0)
        except (AssertionError, ValueError):
            return False
        return True

    assert pin_passes()
    real_svd = orc.jacobi_svd

    def left_side(c, *a, **k):
        u, s, p = real_svd(c, *a, **k)
        return u, s, u[: p.shape[0], : p.shape[1]]

    def no_q(a, omega, r):
        q = orc.qr_positive(a.T @ np.asarray(omega, float))[0]
        _u, s, p = real_svd(a @ q)
        return np.vstack([p[:, :r], np.zeros((a.shape[1] - p.shape[0], r))]), s[:r].copy()

    monkeypatch.setattr(orc, "jacobi_svd", left_side)
    assert not pin_passes()
    monkeypatch.undo()
    monkeypatch.setattr(orc, "randomized_svd", no_q)
    assert not pin_passes()
    monkeypatch.undo()


# --------------------------------------------------------------- MinSR / SPRING (Sec. 3.2)

def test_spring_momentum_zero_is_the_direct_solve():
    """MinSR (mu = 0) in the damped form: the sample-space solve equals the
    parameter-space (S + lam I)^{-1} g by a LAPACK solve of the M x M system."""
    n, m = 30, 80
    o, e = _problem(n, m, 71)
    res = orc.spring_step(o, e, None, 0.05, 0.0, 0.1)
    a = (o - o.mean(axis=0)) / np.sqrt(n)
    g = a.T @ (e - e.mean()) / np.sqrt(n)
    assert _rel(res["delta"], np.linalg.solve(a.T @ a + 0.05 * np.eye(m), g)) < 1e-10
    assert _rel(res["dtheta"], -0.1 * res["delta"]) < 1e-15


def test_spring_with_momentum_against_parameter_space_solve():
    """SPRING: delta = (A^T A + lam I)^{-1} A^T (eps/sqrt(N) - mu A dtheta)
    (the damped push-through identity with the modified right-hand side),
    solved by LAPACK in parameter space; dtheta = -eta delta + mu dtheta_prev."""
    n, m, mu, eta, lam = 25, 60, 0.9, 0.02, 0.01
    o, e = _problem(n, m, 72)
    prev = rng0(73).standard_normal(m)
    res = orc.spring_step(o, e, prev, lam, mu, eta)
    a = (o - o.mean(axis=0)) / np.sqrt(n)
    b = (e - e.mean()) / np.sqrt(n) - mu * a @ prev
    want = np.linalg.solve(a.T @ a + lam * np.eye(m), a.T @ b)
    assert _rel(res["delta"], want) < 1e-10
    assert _rel(res["dtheta"], -eta * want + mu * prev) < 1e-12


def test_spring_small_damping_is_the_minimum_norm_projection():
    """As lam -> 0 the SPRING direction is the minimum-norm solution of the
    sample-space system A delta = Ltilde (the Kaczmarz-type projection the
    method is built on): LAPACK's least-squares solution."""
    n, m, mu = 20, 70, 0.5
    o, e = _problem(n, m, 74, noise=0.3)
    prev = rng0(75).standard_normal(m)
    res = orc.spring_step(o, e, prev, 1e-11, mu, 1.0)
    a = (o - o.mean(axis=0)) / np.sqrt(n)
    b = (e - e.mean()) / np.sqrt(n) - mu * a @ prev
    want = np.linalg.lstsq(a, b, rcond=None)[0]
    assert _rel(res["delta"], want) < 1e-6


def test_spring_rejects_bad_arguments():
    o, e = _problem(10, 20, 76)
    for lam, mu in ((0.0, 0.1), (0.1, 1.0), (0.1, -0.2)):
        with pytest.raises(ValueError):
            orc.spring_step(o, e, np.zeros(20), lam, mu, 0.1)


# --------------------------------------------------------------- adaptive rank, diag(R) ending

def test_rank_ruler_hand_cases():
    """Eq. ruler on the squares of sigma: sigma = (1, 0.5, 0.3, 0.1) has
    sigma^2 ratios (1, 0.25, 0.09, 0.01)."""
    s = [1.0, 0.5, 0.3, 0.1]
    assert orc.rank_ruler(s, 0.0) == (4, True)
    assert orc.rank_ruler(s, 0.25) == (2, False)
    assert orc.rank_ruler(s, 0.1) == (2, False)
    assert orc.rank_ruler(s, 0.09) == (3, False)
    assert orc.rank_ruler(s, 0.01) == (4, True)
    assert orc.rank_ruler(s, 0.5) == (1, False)


def test_truncated_woodbury_against_dense_inverse():
    """Only the kept columns enter: delta = (V_k diag(s_k^2) V_k^T + lam I)^{-1} g,
    and the floor form sends the dropped directions to 1/lam."""
    rng = rng0(81)
    m, r = 40, 6
    v = np.linalg.qr(rng.standard_normal((m, r)))[0]
    s = np.array([2.0, 1.5, 1.0, 0.4, 0.2, 0.05])
    g = rng.standard_normal(m)
    lam, r_reg = 0.03, 0.02                     # keeps s^2 >= 0.08: the first four
    assert orc.rank_ruler(s, r_reg)[0] == 4
    d = orc.truncated_woodbury(v, s, g, lam, "damped", r_reg)
    vk = v[:, :4]
    want = np.linalg.solve((vk * s[:4] ** 2) @ vk.T + lam * np.eye(m), g)
    assert _rel(d, want) < 1e-12
    df = orc.truncated_woodbury(v, s, g, lam, "floor", r_reg)
    pinv = (vk / s[:4] ** 2) @ vk.T + (np.eye(m) - vk @ vk.T) / lam
    assert _rel(df, pinv @ g) < 1e-12


def test_diag_extraction_converges_to_the_svd():
    """Alg. 1's diag(R) ending: with many passes sigma and span(V) are the
    exact top-r (LAPACK), column by column where the gaps are clear, and
    sigma comes out sorted."""
    n, m, r = 50, 80, 5
    o, e = _problem(n, m, 82, spectrum=np.r_[np.linspace(1, 0.5, r), 0.05 * np.ones(n - r)], noise=0.0)
    a = (o - o.mean(axis=0)) / np.sqrt(n)
    _, s_ref, wt = np.linalg.svd(a)
    # without a Rayleigh-Ritz rotation the columns separate at the rate of
    # the gaps inside the top r, (0.875)^2 per pass here
    v, s = orc.ssi_diag_extract(a, rng0(83).standard_normal((m, r)), 120)
    assert np.all(np.diff(s) <= 0)
    assert _rel(s, s_ref[:r]) < 1e-10
    assert np.all(np.abs(np.sum(v * wt[:r].T, axis=0)) > 1 - 1e-8)
    res = orc.wssr_step(o, e, rng0(83).standard_normal((m, r)), 1e-2, r, 120, extract="diag")
    rr = orc.wssr_step(o, e, rng0(83).standard_normal((m, r)), 1e-2, r, 120)
    assert _rel(res["delta"], rr["delta"]) < 1e-8


def test_diag_extraction_one_pass_by_hand():
    """q = 1: sigma = |diag R| of A orth(V_in), sorted, V = orth(V_in)
    reordered (LAPACK QR written out here)."""
    n, m, r = 30, 40, 4
    o, e = _problem(n, m, 84)
    a = (o - o.mean(axis=0)) / np.sqrt(n)
    vin = rng0(85).standard_normal((m, r))
    q0 = np.linalg.qr(vin)[0]
    q0 = q0 * np.sign(np.diag(np.linalg.qr(vin)[1]))
    rr = np.linalg.qr(a @ q0)[1]
    s = np.abs(np.diag(rr))
    order = np.argsort(-s)
    v, sig = orc.ssi_diag_extract(a, vin, 1)
    assert _rel(sig, s[order]) < 1e-13
    assert np.abs(np.abs(v) - np.abs(q0[:, order])).max() < 1e-13


def test_step_reports_the_ruler():
    n, m, r = 40, 60, 8
    o, e = _problem(n, m, 86)
    res = orc.wssr_step(o, e, rng0(87).standard_normal((m, r)), 1e-3, r, 3, r_reg=0.05)
    assert (res["r_eff"], res["grow"]) == orc.rank_ruler(res["sigma"], 0.05)
    assert res["r_eff"] < r
