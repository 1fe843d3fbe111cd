"""Seeded synthetic inputs for one warm-started SR step.

This module draws the inputs only; it contains none of the step's arithmetic
and is shared by the oracle-side tests and by the HIP-side tests and benchmark.

Recipe (stand-in for the per-sample log-derivatives of the paper's atomic and
molecular wave functions, which are not available):

    O_t = sqrt(N) * U_t diag(s) W_t^T + eta * G_t          (N x M, rows = samples)
    s_k = k^(-alpha), k = 1..K
    U_0 (N x K), W_0 (M x K): orthonormal, Q factors (positive diagonal) of
        Gaussian matrices
    U_t = R(t*theta) U_0,  W_t = R(t*theta) W_0: R rotates disjoint pairs of
        ambient coordinates (pi(2i), pi(2i+1)) of a seeded permutation pi by
        the same angle, so consecutive top-r subspaces drift by about theta
        (the slow drift the warm start exploits, Sec. 4.2 Table 1)
    G_t: i.i.d. N(0,1), fresh for each step
    E_L,t: i.i.d. N(el_mean, el_std^2), fresh for each step
    V_0: Q factor of an M x r Gaussian (the cold-start basis)

``s_k`` are the singular values of the clean part of O/sqrt(N).  Every
component has its own generator seeded from (seed, component, step), so any
step can be drawn alone.  Generation runs in torch on the requested device;
values differ between devices but are deterministic on each.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import torch


@dataclasses.dataclass(frozen=True)
class Config:
    name: str
    n: int            # samples (walkers)
    m: int            # parameters
    r: int            # rank
    q: int            # subspace-iteration passes per step
    lam: float        # damping
    steps: int
    alpha: float      # spectrum exponent
    theta: float      # rotation per step
    eta: float        # noise level
    el_mean: float
    el_std: float
    seed: int
    k: int = 0        # number of spectral components (0 -> n)
    dtype: str = "f32"

    @property
    def ncomp(self):
        return self.k if self.k else self.n


# The workloads, named by dtype and size: a small one the oracle checks in
# seconds, the FP32 benchmark instance, the BF16 precision-form instance, and the
# largest single instance.
CONFIGS = {c.name: c for c in [
    Config("f32_n1024_m2k_r32", n=1024, m=2000, r=32, q=2, lam=1e-3, steps=10,
           alpha=1.5, theta=0.02, eta=1e-3, el_mean=-1.0, el_std=0.1, seed=1),
    Config("f32_n8192_m100k_r256", n=8192, m=100_000, r=256, q=2, lam=1e-3, steps=20,
           alpha=1.2, theta=0.01, eta=1e-3, el_mean=-10.0, el_std=0.5, seed=2),
    Config("bf16_n16384_m1m_r512", n=16384, m=1_000_000, r=512, q=2, lam=1e-3, steps=20,
           alpha=1.0, theta=0.01, eta=1e-4, el_mean=-10.0, el_std=0.5, seed=3, k=4096,
           dtype="bf16"),
    Config("bf16_n16384_m4m_r512_q3", n=16384, m=4_000_000, r=512, q=3, lam=1e-3, steps=10,
           alpha=1.3, theta=0.005, eta=1e-4, el_mean=-10.0, el_std=0.5, seed=5, k=4096,
           dtype="bf16"),
]}



def batch_configs(count=16, seed=4):
    """The batched workload: `count` independent problems with N in {2048,
    4096, 8192, 16384}, M uniform in [20000, 400000], r in {64, 128, 256},
    lambda log-uniform in [1e-4, 1e-2] and spectrum k^-a, a uniform in
    [1.0, 1.5]; rotation 0.01 per step, noise 1e-4, E_L ~ N(-10, 0.5^2),
    min(N, 4096) spectral components (the components beyond are below the
    noise floor).  Problem j is seeded with 4000 + j."""
    rng = np.random.default_rng(seed)
    out = []
    for j in range(count):
        n = int(rng.choice([2048, 4096, 8192, 16384]))
        m = int(rng.integers(20_000, 400_001))
        r = int(rng.choice([64, 128, 256]))
        lam = float(10 ** rng.uniform(-4, -2))
        a = float(rng.uniform(1.0, 1.5))
        out.append(Config(f"batch16_mixed[{j}]", n=n, m=m, r=r, q=2, lam=lam, steps=20, alpha=a, theta=0.01,
                          eta=1e-4, el_mean=-10.0, el_std=0.5, seed=4000 + j, k=min(n, 4096)))
    return out


_COMPONENT = {"u": 1, "w": 2, "perm_n": 3, "perm_m": 4, "v0": 5, "noise": 6, "el": 7}


def _gen(device, seed, component, step=0):
    g = torch.Generator(device=device)
    g.manual_seed((seed * 1_000_003 + _COMPONENT[component] * 10_007 + step) & 0x7FFF_FFFF_FFFF)
    return g


_BIG = 1 << 28   # elements above which the large-instance code paths are used


def _orthonormal(x):
    """Q factor with a positive diagonal of R (Haar-distributed for Gaussian x).
    Tall matrices of more than 2^28 elements go through two rounds of
    Cholesky QR in float64 (a Gaussian matrix that tall is well conditioned,
    so this reaches the same unique Q as Householder QR, to rounding)."""
    if x.numel() > _BIG:
        # Gram on the device (FP64, accumulated over row blocks, so that no
        # FP64 copy of x is held), its Cholesky factor and the inverse of that
        # (k x k) on the host, then the product applied block by block in place
        y = x.contiguous()
        rows = max(1, (1 << 26) // y.shape[1])
        for _ in range(2):
            gram = torch.zeros(y.shape[1], y.shape[1], dtype=torch.float64, device=y.device)
            for i in range(0, y.shape[0], rows):
                b = y[i:i + rows].double()
                gram += b.T @ b
                del b
            low = np.linalg.cholesky(gram.cpu().numpy())
            rinv = torch.from_numpy(np.ascontiguousarray(np.linalg.inv(low.T))).to(y.device)
            for i in range(0, y.shape[0], rows):
                y[i:i + rows] = (y[i:i + rows].double() @ rinv).to(y.dtype)
        return y
    q, r = torch.linalg.qr(x)
    d = torch.sign(torch.diagonal(r))
    d[d == 0] = 1
    return (q * d).contiguous()


def _rotate_pairs_inplace(x, perm, angle, chunk=1 << 16):
    """Rotate rows (perm[2i], perm[2i+1]) of x by angle, in place, a chunk of
    pairs at a time (for factors too large to copy)."""
    npair = perm.numel() // 2
    c, s = math.cos(angle), math.sin(angle)
    for i in range(0, npair, chunk):
        a = perm[2 * i:2 * min(npair, i + chunk):2]
        b = perm[2 * i + 1:2 * min(npair, i + chunk):2]
        xa, xb = x[a].clone(), x[b].clone()
        x[a] = c * xa - s * xb
        x[b] = s * xa + c * xb


def _rotate_pairs(x, perm, angle):
    """Rotate rows (perm[2i], perm[2i+1]) of x by angle."""
    npair = perm.numel() // 2
    a, b = perm[0:2 * npair:2], perm[1:2 * npair:2]
    c, s = math.cos(angle), math.sin(angle)
    xa, xb = x[a], x[b]
    y = x.clone()
    y[a] = c * xa - s * xb
    y[b] = s * xa + c * xb
    return y


class Workload:
    """Holds the fixed factors of one configuration and draws step inputs."""

    def __init__(self, cfg: Config, device="cpu", gen_dtype=torch.float64, n=None, m=None):
        self.cfg = cfg
        self.device = torch.device(device)
        self.n = n or cfg.n
        self.m = m or cfg.m
        k = min(cfg.ncomp, self.n, self.m)
        self.k = k
        dev, sd = self.device, cfg.seed
        self.gen_dtype = gen_dtype
        gu = torch.randn(self.n, k, generator=_gen(dev, sd, "u"), device=dev, dtype=gen_dtype)
        gw = torch.randn(self.m, k, generator=_gen(dev, sd, "w"), device=dev, dtype=gen_dtype)
        self.u0 = _orthonormal(gu)
        self.w0 = _orthonormal(gw)
        del gu, gw
        self.perm_n = torch.randperm(self.n, generator=_gen(dev, sd, "perm_n"), device=dev)
        self.perm_m = torch.randperm(self.m, generator=_gen(dev, sd, "perm_m"), device=dev)
        self.spectrum = torch.arange(1, k + 1, device=dev, dtype=gen_dtype) ** (-cfg.alpha)
        # W_t of the large instances is rotated in place (W_0 is not kept):
        # the angle it currently stands at
        self._w_angle = 0.0

    def o_blocks(self, t):
        """O_t as consecutive blocks of rows: yields (first row, float32 block).
        Instances of more than 2^28 elements come in blocks of at most 1024
        rows and 2^30 elements (noise drawn block by block from the step's
        generator), so that no full-size temporary is held; smaller ones come
        as one block.  The values are those of o(t)."""
        cfg, dev = self.cfg, self.device
        ut = _rotate_pairs(self.u0, self.perm_n, t * cfg.theta)
        if self.w0.numel() > _BIG:
            # pair rotations compose by adding angles
            _rotate_pairs_inplace(self.w0, self.perm_m, t * cfg.theta - self._w_angle)
            self._w_angle = t * cfg.theta
            wt = self.w0
        else:
            wt = _rotate_pairs(self.w0, self.perm_m, t * cfg.theta)
        left = math.sqrt(self.n) * ut * self.spectrum[None, :]
        del ut
        gen = _gen(dev, cfg.seed, "noise", t)
        if self.n * self.m <= _BIG:
            o = left @ wt.T
            noise = torch.randn(self.n, self.m, generator=gen, device=dev, dtype=self.gen_dtype)
            o.add_(noise, alpha=cfg.eta)
            del noise
            yield 0, o.float().contiguous()
            return
        rows = max(64, min(1024, (1 << 30) // self.m))
        for i in range(0, self.n, rows):
            blk = left[i:i + rows] @ wt.T
            blk.add_(torch.randn(blk.shape, generator=gen, device=dev, dtype=self.gen_dtype), alpha=cfg.eta)
            yield i, blk.float().contiguous()
            del blk

    def o(self, t, dtype=torch.float32):
        """O_t (N x M) in the given dtype (converted from float32 block by
        block for the large instances)."""
        if self.n * self.m <= _BIG:
            (_, o), = list(self.o_blocks(t))
            return o.to(dtype).contiguous()
        out = torch.empty(self.n, self.m, device=self.device, dtype=dtype)
        for i, blk in self.o_blocks(t):
            out[i:i + blk.shape[0]] = blk.to(dtype)
        return out

    def e_l(self, t):
        cfg = self.cfg
        z = torch.randn(self.n, generator=_gen(self.device, cfg.seed, "el", t),
                        device=self.device, dtype=torch.float64)
        return cfg.el_mean + cfg.el_std * z

    def v0(self, r=None, dtype=torch.float32):
        r = r or self.cfg.r
        g = torch.randn(self.m, r, generator=_gen(self.device, self.cfg.seed, "v0"),
                        device=self.device, dtype=self.gen_dtype)
        return _orthonormal(g).to(dtype).contiguous()


def to_storage(o, form):
    """O in the storage format of a precision form (input encoding, done once
    by whoever produces O): "f32" -> float32; "bf16" and "bf16_split" ->
    bfloat16 (round to nearest even); "bf16x2" -> (2, n, m) bfloat16 planes
    hi = RNE(O), lo = RNE(O - hi)."""
    o = o.float()
    if form == "f32":
        return o.contiguous()
    hi = o.to(torch.bfloat16)
    if form in ("bf16", "bf16_split"):
        return hi.contiguous()
    if form == "bf16x2":
        lo = (o - hi.float()).to(torch.bfloat16)
        return torch.stack([hi, lo]).contiguous()
    raise ValueError(form)


def stored_values(o_stored):
    """The values a stored O represents, in float64 (hi + lo for two planes)."""
    if o_stored.dim() == 3:
        return o_stored[0].double() + o_stored[1].double()
    return o_stored.double()


def random_problem(n, m, r, seed, alpha=1.2, eta=1e-3, el_mean=-1.0, el_std=0.1,
                   device="cpu", dtype=torch.float32, theta=0.01, t=1):
    """A single step's inputs (O, E_L, V_in) of arbitrary shape, drawn with the
    same recipe; V_in is the exact-start-free cold basis V_0."""
    cfg = Config("adhoc", n=n, m=m, r=r, q=2, lam=1e-3, steps=1, alpha=alpha, theta=theta,
                 eta=eta, el_mean=el_mean, el_std=el_std, seed=seed)
    wl = Workload(cfg, device=device)
    return wl.o(t, dtype), wl.e_l(t), wl.v0(r, dtype)
