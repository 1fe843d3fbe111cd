"""Readings of the paper that the GPU design rests on, checked against the
FP64 oracle on the CPU (no GPU): an intermediate pass of the subspace
iteration may carry any well-conditioned basis Z T of the parameter-side
block in place of its orthonormal factor Q_Z, because the next pass depends
on Z only through its span (Alg. 1 in exact arithmetic); and the
Rayleigh-Ritz SVD is needed on the last pass only."""
import numpy as np
import pytest

from oracle import wssr_oracle as orc


def _problem(seed, n=400, m=900, r=12, alpha=1.1):
    rng = np.random.default_rng(seed)
    k = np.arange(1, min(n, m) + 1, dtype=np.float64)
    u = np.linalg.qr(rng.standard_normal((n, n)))[0]
    w = np.linalg.qr(rng.standard_normal((m, min(n, m))))[0]
    a = (u[:, :len(k)] * k ** -alpha) @ w.T
    v_in = rng.standard_normal((m, r))
    return a, v_in


def _span_carrying(a, v_in, q, basis):
    """q passes as the GPU runs them: Y = A V, Q_Y from its QR, Z = A^T Q_Y;
    an intermediate pass carries V = basis(Z); the last pass factors
    Z = Q_Z R_Z and ends with the Rayleigh-Ritz SVD of C = Q_Y^T A Q_Z."""
    v = v_in
    for p in range(1, q + 1):
        qy = orc.qr_positive(a @ v)[0]
        z = a.T @ qy
        if p < q:
            v = basis(z)
            continue
        qz = orc.qr_positive(z)[0]
        _, s, pm = orc.jacobi_svd(qy.T @ (a @ qz))
        return qz @ pm, s


def _scale_columns(z):
    return z / np.linalg.norm(z, axis=0)


def _chol_inverse(z):
    # R from the Cholesky of a perturbed Gram (as a fast Gram's factor would
    # be), V = Z R^{-1}: well conditioned, not orthonormal
    g = z.T @ z
    g = g * (1.0 + 1e-7 * np.random.default_rng(0).standard_normal(g.shape))
    g = 0.5 * (g + g.T)
    r_ = np.linalg.cholesky(g).T
    return np.linalg.solve(r_.T, z.T).T


@pytest.mark.parametrize("basis", [_scale_columns, _chol_inverse], ids=["scaled", "perturbed-R"])
@pytest.mark.parametrize("q", [2, 3])
def test_intermediate_passes_carry_only_the_span(basis, q):
    a, v_in = _problem(seed=q)
    v_ref, s_ref, _ = orc.ssi_svd(a, v_in, q)
    v, s = _span_carrying(a, v_in, q, basis)
    assert np.max(np.abs(s - s_ref) / s_ref) < 1e-10
    # the subspaces agree (projectors), whatever the rotation within ties
    assert np.abs(v @ v.T - v_ref @ v_ref.T).max() < 1e-10


def test_a_rank_losing_basis_would_not_do():
    """The reading needs a well-conditioned T: a basis that drops a direction
    changes the result (the GPU takes the FP64 CholeskyQR2 there)."""
    a, v_in = _problem(seed=5)
    v_ref, s_ref, _ = orc.ssi_svd(a, v_in, 2)

    def drop_last(z):
        zz = z.copy()
        zz[:, -1] = zz[:, 0]
        return zz

    _, s = _span_carrying(a, v_in, 2, drop_last)
    assert np.max(np.abs(s - s_ref) / s_ref) > 1e-2


@pytest.mark.parametrize("q", [1, 3])
def test_rayleigh_ritz_on_the_last_pass_only(q):
    """Reading A8: the GPU closes only the last pass with the Rayleigh-Ritz
    SVD; the oracle closes every pass.  An intermediate Rayleigh-Ritz step
    rotates Q_Z within its span, so the last pass sees the same subspace."""
    a, v_in = _problem(seed=10 + q)
    v_ref, s_ref, _ = orc.ssi_svd(a, v_in, q)
    v, s = _span_carrying(a, v_in, q, lambda z: orc.qr_positive(z)[0])
    assert np.max(np.abs(s - s_ref) / s_ref) < 1e-10
    assert np.abs(v @ v.T - v_ref @ v_ref.T).max() < 1e-10


def test_warm_start_needs_only_its_span():
    """Reading A13: the GPU feeds V_in to the first product as it is, the
    oracle takes its QR first; V_in and V_in T (T well conditioned) span the
    same space and give the same step."""
    a, v_in = _problem(seed=21)
    t = np.eye(v_in.shape[1]) + 0.3 * np.random.default_rng(22).standard_normal((v_in.shape[1],) * 2)
    v_ref, s_ref, _ = orc.ssi_svd(a, v_in, 2)
    v, s = _span_carrying(a, v_in @ t, 2, _scale_columns)
    assert np.max(np.abs(s - s_ref) / s_ref) < 1e-10
    assert np.abs(v @ v.T - v_ref @ v_ref.T).max() < 1e-10
