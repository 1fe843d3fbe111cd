"""FP64 reference ("oracle") for one warm-started stochastic-reconfiguration step.

TEST INFRASTRUCTURE ONLY.  This module is the plain, slow CPU statement of what
one WSSR step computes.  Only the test suite, the smoke check and the CPU-baseline
leg of the benchmark may import it; the product path (the HIP library and its
Python binding) never does, and this module imports nothing from the product.

Everything is float64 numpy.  Matrix products and the library QR factorisation
(LAPACK Householder, via ``numpy.linalg.qr``) are used as single steps; the
Cholesky factorisation, the triangular solves and the one-sided Jacobi SVD are
written out here.  No blocking, fusion or reordering beyond the definitions.

Notation (paper -> here).  The paper's centred, 1/sqrt(N)-scaled log-derivative
matrix (Sec. 3.1, eq. Osrn) is parameters x samples; here the per-sample rows
arrive as ``o`` (N x M) and ``a = (o - 1 mu^T)/sqrt(N)`` is its transpose, so the
singular values ``sigma`` returned are those of ``a`` and the S-matrix is
``a^T a`` (eq. SN with the 1/N of eq. Osrn).  The warm start ``v`` (M x r) is the
paper's parameter-side singular basis U^(k) (Sec. 4.1, eq. svd:det); the pass
count ``q`` is the paper's m (Alg. 1).

Readings taken where the paper is silent or inconsistent (numbered as in the
design notes):
  * the gradient carries no factor 2 (eq. barg at averaging weight 0);
  * sample means use 1/N (eqs. loss:vmc, Osr);
  * the energies are centred explicitly and so is O;
  * each pass ends with a two-sided Rayleigh-Ritz step on the sample-side and
    parameter-side bases (replacing the diag(R) extraction that closes Alg. 1);
  * the preconditioner is the damped one, (V diag(sigma^2) V^T + lam I)^{-1},
    applied by the Woodbury identity; the paper's floor form (eq. updated_sr_1
    with floor lam) is available as ``precond="floor"``;
  * output signs: column j of V_out has a non-negative inner product with
    column j of V_in; if that product is below 1e-8 in magnitude, the entry of
    largest magnitude (lowest index on ties) is made positive.
  * adaptive rank (Sec. 4.3): the ratio of eq. ruler is taken on the
    eigenvalues of S (sigma^2); the truncation enters only the preconditioned
    direction, and the stored state and the warm start keep every column;
  * Alg. 1's own ending (diag(R) of the last sample-side block, sorted) is
    offered beside the Rayleigh-Ritz one; its parameter-side output is the
    orthonormal basis the last block was formed from;
  * averaged state (Sec. 4.1): the stored matrix is kept as its factors, the
    orthonormal U of the previous step and sigma (Obar = U diag(sigma)); the
    initial state is zero as the paper sets it, so the first step's Sbar is
    (1 - avg) S_N rather than the S_N that the plain averaging scheme (eq.
    ave_s) starts from; the sample-side singular factor V of eq. svd:det is the
    last pass's Q_Y G, signed like its parameter-side partner;
  * randomized sketch (App. A): the random block multiplies the sample side, so
    it is N x (r + p) (the paper prints the parameter count as its row count),
    and it is an input; the rank-r result has no warm start to sign against,
    so each column's entry of largest magnitude is made positive.
"""
from __future__ import annotations

import numpy as np

SIGN_TIE = 1e-8


# ----------------------------------------------------------------------------
# Estimators (Sec. 2.2 eqs. loss:vmc / gradient:vmc; Sec. 3.1 eqs. Osr, Osrn, Lbarn)
# ----------------------------------------------------------------------------

def center_energies(e_l):
    """epsilon = E_L - (1/N) sum E_L   (eq. Lbarn: L(x) = E_L(x) - L_N, eq. loss:vmc)."""
    e = np.asarray(e_l, dtype=np.float64)
    return e - e.mean()


def center_columns(o):
    """O_bar = O - 1 mu^T with mu the per-parameter sample mean (eq. Osr)."""
    o = np.asarray(o, dtype=np.float64)
    return o - o.mean(axis=0, keepdims=True)


def scaled_centered(o):
    """A = O_bar / sqrt(N): the transpose of the paper's matrix of eq. Osrn."""
    n = o.shape[0]
    return center_columns(o) / np.sqrt(n)


def gradient(o, e_l):
    """g = O_bar^T eps / N  (eq. barg with averaging weight 0: g = O L, no factor 2)."""
    n = o.shape[0]
    return center_columns(o).T @ center_energies(e_l) / n


def s_matrix(o):
    """S = O_bar^T O_bar / N = A^T A  (eq. SN with the 1/N scaling of eq. Osrn)."""
    a = scaled_centered(o)
    return a.T @ a


# ----------------------------------------------------------------------------
# Dense kernels written out: Cholesky, triangular solves
# ----------------------------------------------------------------------------

def cholesky_lower(g):
    """Lower Cholesky factor L with L L^T = g (column by column, textbook order).

    Raises np.linalg.LinAlgError when a pivot is not positive."""
    g = np.array(g, dtype=np.float64)
    n = g.shape[0]
    low = np.zeros_like(g)
    for j in range(n):
        d = g[j, j] - low[j, :j] @ low[j, :j]
        if not d > 0.0:
            raise np.linalg.LinAlgError(f"non-positive pivot {d} at column {j}")
        low[j, j] = np.sqrt(d)
        low[j + 1:, j] = (g[j + 1:, j] - low[j + 1:, :j] @ low[j, :j]) / low[j, j]
    return low


def solve_lower(low, b):
    """Forward substitution: x with L x = b (b may be a matrix)."""
    b = np.array(b, dtype=np.float64)
    x = np.zeros_like(b)
    for i in range(low.shape[0]):
        x[i] = (b[i] - low[i, :i] @ x[:i]) / low[i, i]
    return x


def solve_upper(up, b):
    """Back substitution: x with U x = b (b may be a matrix)."""
    b = np.array(b, dtype=np.float64)
    x = np.zeros_like(b)
    n = up.shape[0]
    for i in range(n - 1, -1, -1):
        x[i] = (b[i] - up[i, i + 1:] @ x[i + 1:]) / up[i, i]
    return x


def spd_solve(mat, b):
    """x = mat^{-1} b for symmetric positive definite mat, via cholesky_lower."""
    low = cholesky_lower(mat)
    return solve_upper(low.T, solve_lower(low, b))


# ----------------------------------------------------------------------------
# QR with a positive diagonal (Alg. 1 "QR decomposition")
# ----------------------------------------------------------------------------

def qr_positive(x):
    """Thin QR, x = Q R, with diag(R) >= 0.

    The factorisation itself is LAPACK's Householder QR; the signs are then
    fixed so that the factor is the unique one with a positive diagonal when
    x has full column rank (a zero diagonal entry keeps its column as is)."""
    x = np.asarray(x, dtype=np.float64)
    q, r = np.linalg.qr(x, mode="reduced")
    d = np.sign(np.diag(r))
    d[d == 0] = 1.0
    return q * d[None, :], r * d[:, None]


# ----------------------------------------------------------------------------
# One-sided (Hestenes) Jacobi SVD
# ----------------------------------------------------------------------------

def _round_robin(n):
    """Pairings of a round-robin tournament on n (even) players: n-1 rounds of n/2
    disjoint pairs; every pair meets exactly once per sweep."""
    players = list(range(n))
    rounds = []
    for _ in range(n - 1):
        half = n // 2
        p = np.array(players[:half])
        q = np.array(players[half:][::-1])
        rounds.append((np.minimum(p, q), np.maximum(p, q)))
        players = [players[0]] + [players[-1]] + players[1:-1]
    return rounds


def jacobi_svd(c, tol=None, max_sweeps=80):
    """SVD c = U diag(s) P^T by one-sided Jacobi rotations on the columns of c.

    Rotations of disjoint column pairs are applied a round at a time (a
    round-robin ordering).  A pair is skipped when |x_p . x_q| <= tol *
    ||x_p|| ||x_q||, or when one of the columns has fallen below eps * ||c||_F
    (it is then numerically zero: a rank-deficient c); the sweep loop stops
    when a whole sweep skipped every pair.
    Returns U (m x n, zero columns where s = 0), s (descending), P (n x n,
    orthogonal).  Works on any m x n; the default tolerance is sqrt(m) * eps."""
    x = np.array(c, dtype=np.float64)
    m, n = x.shape
    if tol is None:
        tol = np.sqrt(m) * np.finfo(np.float64).eps
    npad = n + (n % 2)
    if npad != n:
        x = np.concatenate([x, np.zeros((m, 1))], axis=1)
    p_acc = np.eye(npad)
    floor = (np.finfo(np.float64).eps * np.linalg.norm(x)) ** 2
    rounds = _round_robin(npad) if npad > 1 else []
    for _sweep in range(max_sweeps):
        rotated = False
        for ip, iq in rounds:
            xp, xq = x[:, ip], x[:, iq]
            alpha = np.einsum("ij,ij->j", xp, xp)
            beta = np.einsum("ij,ij->j", xq, xq)
            gamma = np.einsum("ij,ij->j", xp, xq)
            act = (np.abs(gamma) > tol * np.sqrt(alpha * beta)) & (np.minimum(alpha, beta) > floor)
            if not act.any():
                continue
            rotated = True
            ip, iq = ip[act], iq[act]
            alpha, beta, gamma = alpha[act], beta[act], gamma[act]
            zeta = (beta - alpha) / (2.0 * gamma)
            t = np.where(zeta >= 0, 1.0, -1.0) / (np.abs(zeta) + np.hypot(1.0, zeta))
            cs = 1.0 / np.sqrt(1.0 + t * t)
            sn = cs * t
            xp, xq = x[:, ip].copy(), x[:, iq].copy()
            x[:, ip] = cs * xp - sn * xq
            x[:, iq] = sn * xp + cs * xq
            pp, pq = p_acc[:, ip].copy(), p_acc[:, iq].copy()
            p_acc[:, ip] = cs * pp - sn * pq
            p_acc[:, iq] = sn * pp + cs * pq
        if not rotated:
            break
    else:
        raise RuntimeError("jacobi_svd: no convergence")
    # a padding column stays zero and never rotates, so the real block is closed
    x, p_acc = x[:, :n], p_acc[:n, :n]
    s = np.sqrt(np.einsum("ij,ij->j", x, x))
    order = np.argsort(-s, kind="stable")
    s = s[order]
    x = x[:, order]
    p_acc = p_acc[:, order]
    u = np.zeros_like(x)
    nz = s > 0
    u[:, nz] = x[:, nz] / s[nz]
    return u, s, p_acc


# ----------------------------------------------------------------------------
# Warm-started subspace iteration (Sec. 4.2, Alg. 1) and the step (Alg. 2)
# ----------------------------------------------------------------------------

def fix_signs(v_out, v_ref):
    """Sign rule for output singular vectors (the paper is silent on signs)."""
    v_out = v_out.copy()
    for j in range(v_out.shape[1]):
        ip = v_out[:, j] @ v_ref[:, j] if j < v_ref.shape[1] else 0.0
        if abs(ip) >= SIGN_TIE:
            s = 1.0 if ip >= 0 else -1.0
        else:
            k = int(np.argmax(np.abs(v_out[:, j])))
            s = 1.0 if v_out[k, j] >= 0 else -1.0
        v_out[:, j] *= s
    return v_out


def ssi_svd(a, v_in, q):
    """q passes of warm-started subspace iteration on A^T A, each ending in a
    two-sided Rayleigh-Ritz step.

    Alg. 1 orthonormalises the parameter-side block and multiplies by the
    data matrix twice per pass (in the paper's orientation).  Per pass here,
    with A = O_bar/sqrt(N):
        Y = A V            (sample side, N x r)
        Z = A^T Y          (parameter side, M x r)
        Q_Y R_Y = Y,  Q_Z R_Z = Z   (QR, positive diagonal)
        C = Q_Y^T (A Q_Z)           (r x r projection)
        C = G diag(s) P^T           (Jacobi SVD)
        V = Q_Z P,  sigma = s
    Returns V_out (M x r), sigma (r,), and a dict of the last pass's factors."""
    v = qr_positive(v_in)[0]
    last = {}
    for _ in range(q):
        y = a @ v
        z = a.T @ y
        qy, ry = qr_positive(y)
        qz, rz = qr_positive(z)
        c = qy.T @ (a @ qz)
        gl, s, p = jacobi_svd(c)
        v = qz @ p
        last = dict(y=y, z=z, qy=qy, ry=ry, qz=qz, rz=rz, c=c, gl=gl, s=s, p=p)
    v = fix_signs(v, v_in)
    return v, last["s"].copy(), last


def woodbury_weights(sigma, lam, precond="damped"):
    """Diagonal weights w with delta = (g - V diag(w) V^T g) / lam for orthonormal V.

    damped: (V diag(sigma^2) V^T + lam I)^{-1}  ->  w = sigma^2/(sigma^2+lam).
    floor:  eq. updated_sr_1 with floor lam: V diag(sigma^-2) V^T + (I - V V^T)/lam
            ->  w = 1 - lam/sigma^2 (needs sigma > 0)."""
    s2 = np.asarray(sigma, dtype=np.float64) ** 2
    if precond == "damped":
        return s2 / (s2 + lam)
    if precond == "floor":
        return 1.0 - lam / s2
    raise ValueError(precond)


def woodbury_apply(v, sigma, g, lam, precond="damped"):
    """delta = (V Sigma^2 V^T + lam I)^{-1} g by the Woodbury identity, valid for
    any V (not only orthonormal):
        (lam I + W W^T)^{-1} = (I - W (lam I + W^T W)^{-1} W^T) / lam,  W = V Sigma.
    The r x r core lam I + Sigma (V^T V) Sigma is solved by Cholesky.
    For precond="floor" (eq. updated_sr_1), V must be orthonormal."""
    v = np.asarray(v, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    s = np.asarray(sigma, dtype=np.float64)
    if precond == "floor":
        w = woodbury_weights(s, lam, "floor")
        return (g - v @ (w * (v.T @ g))) / lam
    wmat = v * s[None, :]
    core = lam * np.eye(len(s)) + wmat.T @ wmat
    return (g - wmat @ spd_solve(core, wmat.T @ g)) / lam


def ssi_diag_extract(a, v_in, q):
    """Alg. 1 as printed, with its closing diag(R) extraction: Q^1 = orth(V_in);
    each iteration forms the sample-side block A Q^i and the parameter-side
    block A^T A Q^i, whose orthonormal factor is Q^(i+1); after q iterations
    the QR of the last sample-side block A Q^q gives sigma = |diag(R)|, sorted
    in descending order, and the parameter-side output is Q^q with its columns
    in the same order (the normalised form of the printed output).
    Returns V (M x r), sigma (r,)."""
    qm = qr_positive(v_in)[0]
    for i in range(q):
        y = a @ qm
        if i == q - 1:
            _qs, rs = qr_positive(y)
            s = np.abs(np.diag(rs))
            order = np.argsort(-s, kind="stable")
            return qm[:, order], s[order].copy()
        qm = qr_positive(a.T @ y)[0]
    raise ValueError("q must be >= 1")


def rank_ruler(sigma, r_reg):
    """The adaptive rank of Sec. 4.3 (eq. ruler) on the r computed values: the
    number of i with sigma_i^2 / sigma_1^2 >= r_reg (the ratio is taken on the
    eigenvalues of S, the squares of sigma), and whether the largest computed
    index is in that set, which is the paper's condition for growing r_max.
    r_reg = 0 keeps every value.  Returns (r_eff, grow)."""
    s2 = np.asarray(sigma, dtype=np.float64) ** 2
    if len(s2) == 0:
        return 0, False
    keep = s2 >= r_reg * s2[0]
    r_eff = int(np.sum(keep))
    return r_eff, bool(keep[-1])


def truncated_woodbury(v, sigma, g, lam, precond="damped", r_reg=0.0):
    """The preconditioned direction with the rank of eq. ruler: only the first
    r_eff columns enter (eq. updated_sr_1 with U of rank r_eff)."""
    r_eff, _grow = rank_ruler(sigma, r_reg)
    return woodbury_apply(np.asarray(v)[:, :r_eff], np.asarray(sigma)[:r_eff], g, lam, precond)


def wssr_step(o, e_l, v_in, lam, r, q, precond="damped", r_reg=0.0, extract="rr"):
    """One WSSR step at averaging weight 0 (Alg. 2 with Alg. 1 for the SVD).

    Inputs: o (N x M) raw per-sample log-derivatives, e_l (N,) local energies,
    v_in (M x r) warm start, damping lam > 0, rank r, passes q >= 1.
    r_reg: the truncation ratio of eq. ruler (0: none).  extract: "rr" for
    the two-sided Rayleigh-Ritz ending, "diag" for Alg. 1's diag(R) ending.
    Returns dict(delta (M,), v (M x r), sigma (r,), g (M,), eps (N,))."""
    o = np.asarray(o, dtype=np.float64)
    n, m = o.shape
    if not (1 <= r <= min(n - 1, m)):
        raise ValueError("rank out of range")
    if q < 1 or not lam > 0:
        raise ValueError("bad q or lambda")
    if not (np.isfinite(o).all() and np.isfinite(e_l).all() and np.isfinite(v_in).all()):
        raise FloatingPointError("non-finite input")
    eps = center_energies(e_l)
    a = scaled_centered(o)
    g = a.T @ eps / np.sqrt(n)
    v_in = np.asarray(v_in, dtype=np.float64)[:, :r]
    if extract == "diag":
        v, sigma = ssi_diag_extract(a, v_in, q)
        v, last = fix_signs(v, v_in), {}
    else:
        v, sigma, last = ssi_svd(a, v_in, q)
    delta = truncated_woodbury(v, sigma, g, lam, precond, r_reg)
    r_eff, grow = rank_ruler(sigma, r_reg)
    return dict(delta=delta, v=v, sigma=sigma, g=g, eps=eps, last=last, r_eff=r_eff, grow=grow)


def stack_averaged(a, lbar, state, avg):
    """The averaged matrix and vector of eqs. Ohat and Lhat, transposed into this
    module's orientation (rows are samples).

    The paper stacks the stored matrix Obar^(k-1) (M x r_s) beside the new
    centred, scaled samples; transposed, the new sample rows sqrt(1-avg) A come
    first and the r_s history rows sqrt(avg) diag(sigma_s) U_s^T last (the order
    of rows changes no singular value or parameter-side vector; Lhat is stacked
    in the same order).  With state None (k = 0: Obar and Lbar are zero) there
    are no history rows."""
    w_new, w_old = np.sqrt(1.0 - avg), np.sqrt(avg)
    if state is None:
        return w_new * a, w_new * lbar
    u_s = np.asarray(state["v"], dtype=np.float64)
    s_s = np.asarray(state["sigma"], dtype=np.float64)
    l_s = np.asarray(state["l"], dtype=np.float64)
    hist = w_old * (s_s[:, None] * u_s.T)
    return np.concatenate([w_new * a, hist], axis=0), np.concatenate([w_new * lbar, w_old * l_s])


def state_l(last, sgn, lhat):
    """L^(k) = (sample-side singular vectors)^T Lhat (eq. Lbar).

    The sample-side singular vectors of the last pass are Q_Y G, with G the
    left singular vectors of the Rayleigh-Ritz matrix C; each column carries
    the sign its parameter-side partner was given."""
    w = last["qy"] @ last["gl"]
    return sgn * (w.T @ lhat)


def averaged_step(o, e_l, v_in, state, lam, r, q, avg, precond="damped", r_reg=0.0):
    """One WSSR step with the averaged state (Sec. 4.1: eqs. Ohat, Lhat,
    svd:det, Obar, Lbar, barg, barS and updated_sr_1; Alg. 2).

    state: None for the initial state (Obar^(0) = 0, Lbar^(0) = 0), else a dict
    with v (M x r_s, the orthonormal parameter-side factor U of the previous
    step), sigma (r_s,) and l (r_s,): the stored matrix is Obar = U diag(sigma)
    (eq. Obar) and the stored vector is l (eq. Lbar).  avg is the averaging
    weight delta of eq. Ohat, 0 <= avg < 1.  v_in (M x r) is the warm start of
    the subspace iteration (Alg. 2 uses U of the previous step).

    Steps, in the paper's order: stack (eqs. Ohat, Lhat); rank-r truncated SVD
    of the stacked matrix by the subspace iteration (eq. svd:det, Alg. 1 with
    the two-sided Rayleigh-Ritz reading); new state Obar = U Sigma (eq. Obar),
    L = V Lhat (eq. Lbar); averaged gradient gbar = Ohat Lhat (eq. barg); the
    update direction with Sbar = Obar Obar^T (eq. barS) in place of S.
    Returns dict(delta, v, sigma, l, gbar, g, eps, last)."""
    o = np.asarray(o, dtype=np.float64)
    n, m = o.shape
    if not 0.0 <= avg < 1.0:
        raise ValueError("averaging weight out of range")
    r_s = 0 if state is None else np.asarray(state["sigma"]).shape[0]
    if not (1 <= r <= min(n - 1 + r_s, m)):
        raise ValueError("rank out of range")
    if q < 1 or not lam > 0:
        raise ValueError("bad q or lambda")
    if not (np.isfinite(o).all() and np.isfinite(e_l).all() and np.isfinite(v_in).all()):
        raise FloatingPointError("non-finite input")
    eps = center_energies(e_l)
    a = scaled_centered(o)
    lbar = eps / np.sqrt(n)                       # eq. Lbarn with the 1/sqrt(N) of eq. Osrn
    ahat, lhat = stack_averaged(a, lbar, state, avg)
    v_in = np.asarray(v_in, dtype=np.float64)[:, :r]
    v, sigma, last = ssi_svd(ahat, v_in, q)
    sgn = np.where(np.einsum("ij,ij->j", v, last["qz"] @ last["p"]) >= 0, 1.0, -1.0)
    l_new = state_l(last, sgn, lhat)
    gbar = ahat.T @ lhat                          # eq. barg
    delta = truncated_woodbury(v, sigma, gbar, lam, precond, r_reg)
    g = a.T @ lbar
    return dict(delta=delta, v=v, sigma=sigma, l=l_new, gbar=gbar, g=g, eps=eps, last=last)


def randomized_svd(a, omega, r):
    """Rank-r SVD of A by randomized sketching (App. A, eq. randsvd).

    In the paper's orientation the matrix is A^T (parameters x samples) and the
    sketch multiplies it by a random sample-side block: Y = A^T Omega (M x
    (r+p)), Q = orth(Y), B = Q^T A^T ((r+p) x N), B = U_B Sigma V_B, and the
    parameter-side factor is Q U_B.  Omega is N x (r+p), drawn by the caller
    (the paper prints it with the parameter count as its row count; the product
    needs the sample count).  The SVD of B is taken from its transpose A Q
    (N x (r+p)), whose right singular vectors are the left ones of B.
    Returns V (M x r), sigma (r,)."""
    omega = np.asarray(omega, dtype=np.float64)
    q = qr_positive(a.T @ omega)[0]
    _u, s, p = jacobi_svd(a @ q)
    return q @ p[:, :r], s[:r].copy()


def sketch_step(o, e_l, omega, lam, r, q=0, precond="damped"):
    """One SR step whose rank-r SVD comes from the randomized sketch (the RSSR
    variant of the remark on randomized sketching in Sec. 4.1; App. A): no
    warm start, the oversampling p = omega's column count minus r.  q > 0:
    the power scheme of the same randomized range finder (Halko et al.), that
    is q passes of the subspace iteration at rank r + p started from
    orth(A^T Omega), then truncation to r.  Signs: no reference basis, so the
    entry of largest magnitude of each column is positive (the tie rule of the
    plain step).
    Returns dict(delta, v, sigma, g, eps)."""
    o = np.asarray(o, dtype=np.float64)
    n, m = o.shape
    omega = np.asarray(omega, dtype=np.float64)
    if omega.shape[0] != n or omega.shape[1] < r:
        raise ValueError("omega must be N x (r + p), p >= 0")
    if not (1 <= omega.shape[1] <= min(n - 1, m)) or r < 1:
        raise ValueError("rank out of range")
    if not lam > 0 or q < 0:
        raise ValueError("bad lambda or q")
    if not (np.isfinite(o).all() and np.isfinite(e_l).all() and np.isfinite(omega).all()):
        raise FloatingPointError("non-finite input")
    eps = center_energies(e_l)
    a = scaled_centered(o)
    g = a.T @ eps / np.sqrt(n)
    if q == 0:
        v, sigma = randomized_svd(a, omega, r)
    else:
        v0 = qr_positive(a.T @ omega)[0]
        v, sigma, _last = ssi_svd(a, v0, q)
        v, sigma = v[:, :r], sigma[:r].copy()
    v = fix_signs(v, np.zeros((m, 0)))
    delta = woodbury_apply(v, sigma, g, lam, precond)
    return dict(delta=delta, v=v, sigma=sigma, g=g, eps=eps)


# ----------------------------------------------------------------------------
# Plain definitions the step is checked against
# ----------------------------------------------------------------------------

def sr_direct(o, e_l, lam):
    """delta_full = (S + lam I)^{-1} g with S = A^T A formed (M x M), Cholesky solve
    (eq. param:update2 with the diagonal shift of Sec. 3.2)."""
    s = s_matrix(o)
    return spd_solve(s + lam * np.eye(s.shape[0]), gradient(o, e_l))


def sr_pushthrough(o, e_l, lam):
    """delta_full = A^T (A A^T + lam I)^{-1} eps/sqrt(N): the damped form of the
    T-matrix identity (eq. mT), solved in sample space (N x N)."""
    a = scaled_centered(o)
    n = o.shape[0]
    t = a @ a.T
    return a.T @ spd_solve(t + lam * np.eye(n), center_energies(e_l) / np.sqrt(n))


def spring_step(o, e_l, dtheta_prev, lam, mu, eta):
    """The comparison system of Sec. 3.2 in its damped form: MinSR (eq. mT)
    with the SPRING momentum (eq. param:spring), solved in sample space.

        Ltilde = eps/sqrt(N) - mu A dtheta_prev            (dtheta_prev = theta_k - theta_{k-1})
        delta  = A^T (A A^T + lam I)^{-1} Ltilde            (T = A A^T, eq. mT; no factor 2, A3)
        dtheta = -eta delta + mu dtheta_prev               (theta_{k+1} - theta_k)

    mu = 0 is MinSR, whose delta is the damped full-rank SR direction
    (S + lam I)^{-1} g.  dtheta_prev may be None when mu = 0.
    Returns dict(delta, dtheta, t (the N x N T + lam I), rhs (Ltilde))."""
    o = np.asarray(o, dtype=np.float64)
    n, m = o.shape
    if not lam > 0 or not 0.0 <= mu < 1.0:
        raise ValueError("bad lambda or momentum")
    a = scaled_centered(o)
    rhs = center_energies(e_l) / np.sqrt(n)
    prev = np.zeros(m) if dtheta_prev is None else np.asarray(dtheta_prev, dtype=np.float64)
    if mu != 0.0:
        rhs = rhs - mu * (a @ prev)
    t = a @ a.T + lam * np.eye(n)
    delta = a.T @ spd_solve(t, rhs)
    return dict(delta=delta, dtheta=-eta * delta + mu * prev, t=t, rhs=rhs)


def exact_topr(o, r):
    """Exact top-r right singular vectors and values of A by Jacobi SVD of A^T
    (columns of A^T are the N samples)."""
    a = scaled_centered(o)
    u, s, _p = jacobi_svd(a.T)
    return u[:, :r], s[:r]


def delta_exact_r(o, e_l, lam, r, precond="damped"):
    """The Woodbury apply with the exact top-r SVD (the limit q -> infinity)."""
    v, s = exact_topr(o, r)
    return woodbury_apply(v, s, gradient(o, e_l), lam, precond)


# ----------------------------------------------------------------------------
# Single-kernel definitions (the pieces the HIP path computes one by one)
# ----------------------------------------------------------------------------

def gemm_sample_side(o, v):
    """Y = A V = (O - 1 mu^T) V / sqrt(N)."""
    return scaled_centered(o) @ np.asarray(v, dtype=np.float64)


def gemm_param_side(o, x):
    """Z = A^T X = (O - 1 mu^T)^T X / sqrt(N)."""
    return scaled_centered(o).T @ np.asarray(x, dtype=np.float64)


def gram(x):
    """G = X^T X."""
    x = np.asarray(x, dtype=np.float64)
    return x.T @ x


def subspace_distance(v1, v2):
    """sin of the largest principal angle between span(v1) and span(v2)
    (both orthonormalised first)."""
    q1 = qr_positive(v1)[0]
    q2 = qr_positive(v2)[0]
    cosines = np.linalg.svd(q1.T @ q2, compute_uv=False)
    return float(np.sqrt(max(0.0, 1.0 - min(1.0, cosines.min()) ** 2)))
