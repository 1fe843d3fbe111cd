"""Comparison metrics for the parity tests (test code, no step arithmetic)."""
import numpy as np


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def orth_err(v):
    v = np.asarray(v, dtype=np.float64)
    return float(np.abs(v.T @ v - np.eye(v.shape[1])).max())


def sin_max_angle(v1, v2):
    """sin of the largest principal angle between the column spans."""
    q1 = np.linalg.qr(np.asarray(v1, np.float64))[0]
    q2 = np.linalg.qr(np.asarray(v2, np.float64))[0]
    c = np.linalg.svd(q1.T @ q2, compute_uv=False)
    return float(np.sqrt(max(0.0, 1.0 - min(1.0, c.min()) ** 2)))


def weighted_projector_err(v1, w1, v2, w2):
    """|| V1 diag(w1) V1^T - V2 diag(w2) V2^T ||_2 via the stacked basis."""
    v1 = np.asarray(v1, np.float64)
    v2 = np.asarray(v2, np.float64)
    basis, _ = np.linalg.qr(np.concatenate([v1, v2], axis=1))
    a = basis.T @ v1
    b = basis.T @ v2
    d = (a * w1) @ a.T - (b * w2) @ b.T
    return float(np.linalg.norm(d, 2))


def sigma_rel_gated(s_gpu, s_ref, lam, gate=0.01):
    """Largest relative singular-value error over j with s_ref_j^2 >= gate * lam."""
    s_gpu = np.asarray(s_gpu, np.float64)
    s_ref = np.asarray(s_ref, np.float64)
    m = s_ref ** 2 >= gate * lam
    if not m.any():
        return 0.0
    return float(np.max(np.abs(s_gpu[m] - s_ref[m]) / s_ref[m]))
