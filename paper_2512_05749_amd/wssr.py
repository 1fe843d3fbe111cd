"""ctypes binding of libwssr (include/wssr.h): argument marshalling only.

Every computation runs in the HIP kernels of libwssr.so; this module checks
tensor shapes, dtypes and devices, passes device pointers and the current
stream, and turns negative status codes into exceptions.  It fails loudly when
the library has not been built.
"""
from __future__ import annotations

import ctypes
import math
import pathlib

import torch

_PKG = pathlib.Path(__file__).resolve().parent
LIB_PATH = _PKG / "libwssr.so"

OK = 0
WARN_RANK_DEFICIENT = 1
WARN_NOT_CONVERGED = 2
ERR_INVALID_ARG = -1
ERR_NO_DEVICE = -2
ERR_OOM = -3
ERR_HIP = -4
ERR_NONFINITE = -5
ERR_BREAKDOWN = -6
ERR_TIMEOUT = -7
STATUS_NAMES = {0: "OK", 1: "WARN_RANK_DEFICIENT", 2: "WARN_NOT_CONVERGED", -1: "ERR_INVALID_ARG", -2: "ERR_NO_DEVICE", -3: "ERR_OOM",
                -4: "ERR_HIP", -5: "ERR_NONFINITE", -6: "ERR_BREAKDOWN", -7: "ERR_TIMEOUT"}

F32 = 0
BF16 = 1
BF16X2 = 2
BF16_SPLIT = 3
DTYPES = {"f32": F32, "bf16": BF16, "bf16x2": BF16X2, "bf16_split": BF16_SPLIT}
FLOOR_PRECOND = 0x1
GRAPH = 0x2
SAMPLE_SPACE = 0x4
DIAGR_EXTRACT = 0x8


class WssrError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class Config(ctypes.Structure):
    _fields_ = [("n_max", ctypes.c_int64), ("m_max", ctypes.c_int64), ("r_max", ctypes.c_int32),
                ("q_max", ctypes.c_int32), ("o_dtype", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("stream", ctypes.c_void_p), ("lanes", ctypes.c_int32)]


class Problem(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("m", ctypes.c_int64), ("ld_o", ctypes.c_int64), ("O", ctypes.c_void_p),
                ("e_l", ctypes.c_void_p), ("V", ctypes.c_void_p), ("lam", ctypes.c_double), ("r", ctypes.c_int32),
                ("q", ctypes.c_int32), ("delta", ctypes.c_void_p), ("sigma", ctypes.c_void_p)]


_lib = None

_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32
_D = ctypes.c_double
_SIGS = {
    "wssr_create": ([ctypes.POINTER(Config), ctypes.POINTER(_P)], ctypes.c_int),
    "wssr_destroy": ([_P], ctypes.c_int),
    "wssr_step": ([_P, _I64, _I64, _P, _I64, _P, _P, _D, _I32, _I32, _P, _P], ctypes.c_int),
    "wssr_step_g": ([_P, _I64, _I64, _P, _I64, _P, _P, _D, _I32, _I32, _P, _P], ctypes.c_int),
    "wssr_step_avg": ([_P, _I64, _I64, _P, _I64, _P, _P, _P, _D, _I32, _I32, _D, _P, _P, _P, _P], ctypes.c_int),
    "wssr_step_sketch": ([_P, _I64, _I64, _P, _I64, _P, _P, _P, _I32, _I32, _P, _D, _I32, _P, _P], ctypes.c_int),
    "wssr_spring": ([_P, _I64, _I64, _P, _I64, _P, _D, _D, _D, _P, _P], ctypes.c_int),
    "wssr_set_rank_ratio": ([_P, _D], ctypes.c_int),
    "wssr_rank_info": ([_P, ctypes.POINTER(_I32), ctypes.POINTER(_I32)], ctypes.c_int),
    "wssr_dbg_gram": ([_P, _I64, _P, _I32, _I32, _P], ctypes.c_int),
    "wssr_dbg_span_basis": ([_P, _I64, _P, _I32, _P, _P], ctypes.c_int),
    "wssr_ingest": ([_P, _I64, _I64, _I64, _I64, _P, _I64, _P, _P, _P, _I64, _P, _P], ctypes.c_int),
    "wssr_status_sync": ([_P, ctypes.POINTER(_I32), ctypes.POINTER(_D)], ctypes.c_int),
    "wssr_step_batched": ([_P, _P, _I32], ctypes.c_int),
    "wssr_batched_status": ([_P, _I32, ctypes.POINTER(_I32)], ctypes.c_int),
    "wssr_graph_active": ([_P, ctypes.POINTER(_I32)], ctypes.c_int),
    "wssr_tune_batched": ([_P, _P, _I32, _I32, ctypes.POINTER(_I32), ctypes.POINTER(_I32), ctypes.POINTER(_D)],
                          ctypes.c_int),
    "wssr_last_error": ([_P], ctypes.c_char_p),
    "wssr_version": ([], ctypes.c_char_p),
    "wssr_profile": ([_P, _I32], ctypes.c_int),
    "wssr_profile_read": ([_P, ctypes.POINTER(_D), ctypes.POINTER(_I64), _I32], ctypes.c_int),
    "wssr_dbg_sample_side": ([_P, _I64, _I64, _P, _I64, _P, _I32, _P], ctypes.c_int),
    "wssr_dbg_param_side": ([_P, _I64, _I64, _P, _I64, _P, _I32, _P], ctypes.c_int),
    "wssr_dbg_gradient": ([_P, _I64, _I64, _P, _I64, _P, _P], ctypes.c_int),
    "wssr_dbg_cholqr2": ([_P, _I64, _P, _I32, _P, _P], ctypes.c_int),
    "wssr_dbg_small_svd": ([_P, _P, _I32, _P, _P], ctypes.c_int),
    "wssr_small_svd_noalloc": ([_P, _I32, _P, _P, _P, _P], ctypes.c_int),
}


def lib():
    """Load libwssr.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not LIB_PATH.exists():
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2512_05749_amd.build`")
        handle = ctypes.CDLL(str(LIB_PATH))
        for name, (args, res) in _SIGS.items():
            fn = getattr(handle, name)
            fn.argtypes = args
            fn.restype = res
        _lib = handle
    return _lib


def version():
    return lib().wssr_version().decode()


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _need(t, name, dtype, device, shape=None, contiguous=False):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if t.device != device:
        raise ValueError(f"{name} must be on {device}, got {t.device}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if contiguous and not t.is_contiguous():
        # the library reads and writes packed arrays at the tensor's data pointer
        raise ValueError(f"{name} must be contiguous")


class Wssr:
    """One libwssr handle bound to a device and a stream."""

    def __init__(self, n_max, m_max, r_max, q_max=8, floor_precond=False, device=None, stream=None, dtype="f32",
                 lanes=0, graph=False, sample_space=False, diag_extract=False):
        """dtype: storage and product precision of O -- "f32"; "bf16" (one BF16
        product); "bf16_split" (BF16 O, skinny operand split in two); "bf16x2"
        (O as BF16 hi and lo planes, shape (2, n, m), three products).
        lanes, graph: the batched form (step_batched) -- problems run on this
        many concurrent lanes; graph captures a batch once and replays it.
        sample_space: allocate the n_max x n_max workspace of spring().
        diag_extract: Alg. 1's diag(R) ending instead of Rayleigh-Ritz."""
        if dtype not in DTYPES:
            raise ValueError(f"dtype must be one of {sorted(DTYPES)}")
        self.dtype = dtype
        device = torch.device(device if device is not None else "cuda")
        if device.type != "cuda":
            raise ValueError("libwssr runs on a HIP device")
        self.device = torch.device("cuda", device.index if device.index is not None else torch.cuda.current_device())
        with torch.cuda.device(self.device):
            s = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.stream = s
        flags = (FLOOR_PRECOND if floor_precond else 0) | (GRAPH if graph else 0) | \
            (SAMPLE_SPACE if sample_space else 0) | (DIAGR_EXTRACT if diag_extract else 0)
        cfg = Config(int(n_max), int(m_max), int(r_max), int(q_max), DTYPES[dtype], flags,
                     ctypes.c_void_p(s.cuda_stream), int(lanes))
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            code = lib().wssr_create(ctypes.byref(cfg), ctypes.byref(h))
        if code != OK:
            raise WssrError(code, lib().wssr_last_error(None).decode())
        self._h = h
        self.cfg = cfg

    # ------------------------------------------------------------------ util
    def _check(self, code):
        if code != OK:
            raise WssrError(code, lib().wssr_last_error(self._h).decode())

    def _o(self, O):
        if self.dtype == "bf16x2":
            # (2, n, m): hi plane then lo plane, the lo plane n * ld elements on
            if O.dim() != 3 or O.shape[0] != 2 or O.stride(2) != 1 or O.stride(1) < O.shape[2] or \
                    O.stride(0) != O.shape[1] * O.stride(1):
                raise ValueError("O must be (2, n, m) BF16 planes, row-major, the lo plane right after the hi plane")
            _need(O, "O", torch.bfloat16, self.device)
            return O.shape[1], O.shape[2], O.stride(1)
        if O.dim() != 2 or O.stride(1) != 1 or O.stride(0) < O.shape[1]:
            raise ValueError("O must be 2-D, row-major with unit column stride")
        _need(O, "O", torch.float32 if self.dtype == "f32" else torch.bfloat16, self.device)
        return O.shape[0], O.shape[1], O.stride(0)

    def _operand(self, t):
        """t itself when contiguous; otherwise a packed copy whose memory the
        caching allocator keeps until the work queued on the handle's stream
        so far has finished (the library may still be reading it after this
        call returns, when that stream is not torch's current one)."""
        if t.is_contiguous():
            return t
        c = t.contiguous()
        cur = torch.cuda.current_stream(self.device)
        if cur != self.stream:
            # the copy was queued on torch's current stream
            self.stream.wait_stream(cur)
        c.record_stream(self.stream)
        return c

    def close(self):
        if getattr(self, "_h", None):
            lib().wssr_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ step
    def step(self, O, e_l, V, lam, q=2, delta=None, sigma=None, g=None):
        """One WSSR step.  V (m x r, float32) is updated in place; returns (delta, sigma).
        With g (float64 [m], e.g. from ingest) the step uses that gradient
        (wssr_step_g) and e_l may be None."""
        n, m, ld = self._o(O)
        if V.dim() != 2 or not V.is_contiguous():
            raise ValueError("V must be a contiguous m x r tensor")
        r = V.shape[1]
        _need(V, "V", torch.float32, self.device, (m, r))
        if g is None:
            _need(e_l, "e_l", torch.float64, self.device, (n,), contiguous=True)
        else:
            _need(g, "g", torch.float64, self.device, (m,), contiguous=True)
        if delta is None:
            delta = torch.empty(m, dtype=torch.float64, device=self.device)
        if sigma is None:
            sigma = torch.empty(r, dtype=torch.float64, device=self.device)
        _need(delta, "delta", torch.float64, self.device, (m,), contiguous=True)
        _need(sigma, "sigma", torch.float64, self.device, (r,), contiguous=True)
        if g is None:
            self._check(lib().wssr_step(self._h, n, m, _ptr(O), ld, _ptr(e_l), _ptr(V), float(lam), r, int(q),
                                        _ptr(delta), _ptr(sigma)))
        else:
            self._check(lib().wssr_step_g(self._h, n, m, _ptr(O), ld, _ptr(g), _ptr(V), float(lam), r, int(q),
                                          _ptr(delta), _ptr(sigma)))
        return delta, sigma

    def step_avg(self, O, e_l, V, lam, avg, sig_state, l_state, q=2, delta=None, g=None, g_bar=None):
        """One WSSR step with the averaged state (wssr_step_avg).  V (m x r,
        float32), sig_state and l_state (float64 [r]) are updated in place:
        the state in is V diag(sig_state) and l_state of the previous step
        (zeros for the first), out the new one.  g: a gradient from ingest
        (optional); g_bar: where to write the averaged gradient (optional).
        Returns delta."""
        n, m, ld = self._o(O)
        if V.dim() != 2 or not V.is_contiguous():
            raise ValueError("V must be a contiguous m x r tensor")
        r = V.shape[1]
        _need(V, "V", torch.float32, self.device, (m, r))
        _need(e_l, "e_l", torch.float64, self.device, (n,), contiguous=True)
        _need(sig_state, "sig_state", torch.float64, self.device, (r,), contiguous=True)
        _need(l_state, "l_state", torch.float64, self.device, (r,), contiguous=True)
        if g is not None:
            _need(g, "g", torch.float64, self.device, (m,), contiguous=True)
        if g_bar is not None:
            _need(g_bar, "g_bar", torch.float64, self.device, (m,), contiguous=True)
        if delta is None:
            delta = torch.empty(m, dtype=torch.float64, device=self.device)
        _need(delta, "delta", torch.float64, self.device, (m,), contiguous=True)
        nul = ctypes.c_void_p(None)
        self._check(lib().wssr_step_avg(self._h, n, m, _ptr(O), ld, _ptr(e_l), _ptr(g) if g is not None else nul,
                                        _ptr(V), float(lam), r, int(q), float(avg), _ptr(sig_state),
                                        _ptr(l_state), _ptr(delta), _ptr(g_bar) if g_bar is not None else nul))
        return delta

    def step_sketch(self, O, e_l, omega, V, lam, q=0, delta=None, sigma=None, g=None):
        """SR step with the rank-r SVD from a randomized sketch (wssr_step_sketch):
        omega (float32, n x (r + p), contiguous) is the random sample-side block,
        q the power passes, V (m x r, float32) is written.  Returns (delta, sigma)."""
        n, m, ld = self._o(O)
        if V.dim() != 2 or not V.is_contiguous():
            raise ValueError("V must be a contiguous m x r tensor")
        r = V.shape[1]
        _need(V, "V", torch.float32, self.device, (m, r))
        if omega.dim() != 2 or omega.shape[0] != n or omega.shape[1] < r:
            raise ValueError("omega must be n x (r + p)")
        _need(omega, "omega", torch.float32, self.device, contiguous=True)
        p = omega.shape[1] - r
        if g is None:
            _need(e_l, "e_l", torch.float64, self.device, (n,), contiguous=True)
        else:
            _need(g, "g", torch.float64, self.device, (m,), contiguous=True)
        if delta is None:
            delta = torch.empty(m, dtype=torch.float64, device=self.device)
        if sigma is None:
            sigma = torch.empty(r, dtype=torch.float64, device=self.device)
        _need(delta, "delta", torch.float64, self.device, (m,), contiguous=True)
        _need(sigma, "sigma", torch.float64, self.device, (r,), contiguous=True)
        nul = ctypes.c_void_p(None)
        self._check(lib().wssr_step_sketch(self._h, n, m, _ptr(O), ld, _ptr(e_l) if e_l is not None else nul,
                                           _ptr(g) if g is not None else nul, _ptr(omega), p, int(q), _ptr(V),
                                           float(lam), r,
                                           _ptr(delta), _ptr(sigma)))
        return delta, sigma

    def spring(self, O, e_l, lam, momentum=0.0, eta=0.0, dtheta=None, delta=None):
        """MinSR / SPRING in sample space (wssr_spring; the handle needs
        sample_space=True).  dtheta (float64 [m]) is updated in place to
        -eta delta + momentum dtheta; returns delta."""
        n, m, ld = self._o(O)
        _need(e_l, "e_l", torch.float64, self.device, (n,), contiguous=True)
        if dtheta is not None:
            _need(dtheta, "dtheta", torch.float64, self.device, (m,), contiguous=True)
        if delta is None:
            delta = torch.empty(m, dtype=torch.float64, device=self.device)
        _need(delta, "delta", torch.float64, self.device, (m,), contiguous=True)
        nul = ctypes.c_void_p(None)
        self._check(lib().wssr_spring(self._h, n, m, _ptr(O), ld, _ptr(e_l), float(lam), float(momentum), float(eta),
                                      _ptr(dtheta) if dtheta is not None else nul, _ptr(delta)))
        return delta

    def set_rank_ratio(self, r_reg):
        """Truncation ratio of eq. ruler for the steps that follow (0: none)."""
        self._check(lib().wssr_set_rank_ratio(self._h, float(r_reg)))

    def rank_info(self):
        """(r_eff, grow) of the last step (synchronises)."""
        r_eff, grow = _I32(), _I32()
        self._check(lib().wssr_rank_info(self._h, ctypes.byref(r_eff), ctypes.byref(grow)))
        return r_eff.value, bool(grow.value)

    def storage_like(self, n, m):
        """An empty O buffer in this handle's storage form: (n, m) float32 or
        bfloat16, or (2, n, m) bfloat16 planes for bf16x2."""
        if self.dtype == "f32":
            return torch.empty(n, m, dtype=torch.float32, device=self.device)
        if self.dtype == "bf16x2":
            return torch.empty(2, n, m, dtype=torch.bfloat16, device=self.device)
        return torch.empty(n, m, dtype=torch.bfloat16, device=self.device)

    def ingest(self, block, e_l, row0, out=None, g=None, colmean=None, mu=None, n=None):
        """wssr_ingest: write rows row0 .. row0 + block.shape[0] - 1 of the
        float32 block into `out` (this handle's storage form, see
        storage_like; None: statistics only) and form g = O_bar^T eps / n and
        the column means from the unrounded values.  Blocks follow each other
        from row 0; g and colmean are final after the last one.  mu (float64
        [m]) is subtracted before storing.  Returns (g, colmean)."""
        if block.dim() != 2 or block.stride(1) != 1 or block.stride(0) < block.shape[1]:
            raise ValueError("block must be 2-D, row-major with unit column stride")
        _need(block, "block", torch.float32, self.device)
        rows, m = block.shape
        if out is not None:
            on, om, ld = self._o(out)
            if om != m:
                raise ValueError("out has a different column count")
            n = on
        elif n is None:
            raise ValueError("n (total rows) is needed when out is None")
        else:
            ld = m
        _need(e_l, "e_l", torch.float64, self.device, (n,), contiguous=True)
        if g is None:
            g = torch.empty(m, dtype=torch.float64, device=self.device)
        _need(g, "g", torch.float64, self.device, (m,), contiguous=True)
        if colmean is not None:
            _need(colmean, "colmean", torch.float64, self.device, (m,), contiguous=True)
        if mu is not None:
            _need(mu, "mu", torch.float64, self.device, (m,), contiguous=True)
        self._check(lib().wssr_ingest(self._h, n, m, int(row0), rows, _ptr(block), block.stride(0), _ptr(e_l),
                                      _ptr(mu) if mu is not None else None,
                                      _ptr(out) if out is not None else None, ld, _ptr(g),
                                      _ptr(colmean) if colmean is not None else None))
        return g, colmean

    def step_batched(self, problems):
        """One batched step.  problems: list of dicts with keys O, e_l, V, lam and
        optional q (default 2), delta, sigma.  Each V is updated in place;
        returns [(delta, sigma), ...]."""
        arr, outs, keep = self._problem_array(problems)
        self._check(lib().wssr_step_batched(self._h, ctypes.cast(arr, ctypes.c_void_p), len(problems)))
        self._last_batch = (arr, keep)
        return outs

    def _problem_array(self, problems):
        arr = (Problem * len(problems))()
        outs, keep = [], []
        for i, pb in enumerate(problems):
            O, e_l, V = pb["O"], pb["e_l"], pb["V"]
            n, m, ld = self._o(O)
            if V.dim() != 2 or not V.is_contiguous():
                raise ValueError("V must be a contiguous m x r tensor")
            r = V.shape[1]
            _need(V, "V", torch.float32, self.device, (m, r))
            _need(e_l, "e_l", torch.float64, self.device, (n,))
            delta, sigma = pb.get("delta"), pb.get("sigma")
            if delta is None:
                delta = torch.empty(m, dtype=torch.float64, device=self.device)
            if sigma is None:
                sigma = torch.empty(r, dtype=torch.float64, device=self.device)
            _need(delta, "delta", torch.float64, self.device, (m,), contiguous=True)
            _need(sigma, "sigma", torch.float64, self.device, (r,), contiguous=True)
            e_c = self._operand(e_l)
            arr[i] = Problem(n, m, ld, O.data_ptr(), e_c.data_ptr(), V.data_ptr(), float(pb["lam"]),
                             r, int(pb.get("q", 2)), delta.data_ptr(), sigma.data_ptr())
            outs.append((delta, sigma))
            keep.append(e_c)
        return arr, outs, keep

    def tune_batched(self, problems, reps=2):
        """Pick the lane count and split sizing for this batch by timing it
        (on scratch copies; the problems' V is not written).  Returns
        (lanes, split divisor, ms per batch)."""
        arr, _, keep = self._problem_array(problems)
        bl, bd, bms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        self._check(lib().wssr_tune_batched(self._h, ctypes.cast(arr, ctypes.c_void_p), len(problems), int(reps),
                                            ctypes.byref(bl), ctypes.byref(bd), ctypes.byref(bms)))
        del keep
        return bl.value, bd.value, bms.value

    def batched_status(self, count):
        """Synchronise and return the status code of each problem of the last batch."""
        codes = (ctypes.c_int32 * count)()
        self._check(lib().wssr_batched_status(self._h, count, codes))
        return list(codes)

    def graph_active(self):
        a = ctypes.c_int32()
        self._check(lib().wssr_graph_active(self._h, ctypes.byref(a)))
        return bool(a.value)

    def status(self):
        """Synchronise and return (numeric status code, diagnostics dict)."""
        code = ctypes.c_int32()
        diag = (ctypes.c_double * 6)()
        self._check(lib().wssr_status_sync(self._h, ctypes.byref(code), diag))
        return code.value, dict(min_rel_pivot=diag[0], jacobi_sweeps=diag[1], jacobi_cosine=diag[2],
                                cholesky_count=diag[3], kappa_max=diag[4], second_rounds=diag[5])

    def profile(self, enable=True):
        """Start (clearing) or stop recording HIP events around the product kernels."""
        self._check(lib().wssr_profile(self._h, 1 if enable else 0))

    def profile_read(self):
        """{'sample_side': (ms, launches), 'param_side': (ms, launches)} since
        profile(True), plus 'spring_product' and 'spring_cholesky' when
        wssr_spring ran."""
        ms = (ctypes.c_double * 4)()
        cnt = (ctypes.c_int64 * 4)()
        self._check(lib().wssr_profile_read(self._h, ms, cnt, 4))
        out = {"sample_side": (ms[0], cnt[0]), "param_side": (ms[1], cnt[1])}
        for k, name in ((2, "spring_product"), (3, "spring_cholesky")):
            if cnt[k]:
                out[name] = (ms[k], cnt[k])
        return out

    # -------------------------------------------------------- single stages
    def sample_side(self, O, V):
        n, m, ld = self._o(O)
        r = V.shape[1]
        _need(V, "V", torch.float32, self.device, (m, r))
        y = torch.empty(n, r, dtype=torch.float64, device=self.device)
        self._check(lib().wssr_dbg_sample_side(self._h, n, m, _ptr(O), ld, _ptr(self._operand(V)), r, _ptr(y)))
        return y

    def param_side(self, O, X):
        n, m, ld = self._o(O)
        r = X.shape[1]
        _need(X, "X", torch.float32, self.device, (n, r))
        z = torch.empty(m, r, dtype=torch.float32, device=self.device)
        self._check(lib().wssr_dbg_param_side(self._h, n, m, _ptr(O), ld, _ptr(self._operand(X)), r, _ptr(z)))
        return z

    def gradient(self, O, e_l):
        n, m, ld = self._o(O)
        _need(e_l, "e_l", torch.float64, self.device, (n,))
        g = torch.empty(m, dtype=torch.float64, device=self.device)
        self._check(lib().wssr_dbg_gradient(self._h, n, m, _ptr(O), ld, _ptr(self._operand(e_l)), _ptr(g)))
        return g

    def cholqr2(self, X):
        rows, r = X.shape
        _need(X, "X", torch.float32, self.device)
        X = self._operand(X)
        Q = torch.empty(rows, r, dtype=torch.float32, device=self.device)
        R = torch.empty(r, r, dtype=torch.float64, device=self.device)
        self._check(lib().wssr_dbg_cholqr2(self._h, rows, _ptr(X), r, _ptr(Q), _ptr(R)))
        return Q, R

    GRAM_KINDS = {"fp64": 0, "fp32": 1, "bf16_split": 2}

    def gram(self, X, kind="fp64"):
        """G = X^T X as the step forms it: "fp64" (the CholeskyQR2's),
        "fp32" (the last pass's probe) or "bf16_split" (the intermediate
        passes' probe)."""
        rows, r = X.shape
        _need(X, "X", torch.float32, self.device, contiguous=True)
        if kind not in self.GRAM_KINDS:
            raise WssrError(f"gram kind {kind!r} is not one of {sorted(self.GRAM_KINDS)}")
        G = torch.empty(r, r, dtype=torch.float64, device=self.device)
        self._check(lib().wssr_dbg_gram(self._h, rows, _ptr(X), r, self.GRAM_KINDS[kind], _ptr(G)))
        return G

    def span_basis(self, X):
        """(V, mode) of an intermediate pass's basis from Z = X."""
        rows, r = X.shape
        _need(X, "X", torch.float32, self.device, contiguous=True)
        V = torch.empty_like(X)
        mode = torch.empty(1, dtype=torch.int32, device=self.device)
        self._check(lib().wssr_dbg_span_basis(self._h, rows, _ptr(X), r, _ptr(V), _ptr(mode)))
        return V, int(mode.item())

    def small_svd(self, C):
        r = C.shape[0]
        _need(C, "C", torch.float64, self.device, (r, r))
        C = self._operand(C)
        s = torch.empty(r, dtype=torch.float64, device=self.device)
        P = torch.empty(r, r, dtype=torch.float64, device=self.device)
        self._check(lib().wssr_dbg_small_svd(self._h, _ptr(C), r, _ptr(s), _ptr(P)))
        return s, P


def small_svd_noalloc(C, s=None, P=None, status=None, stream=None):
    """wssr_small_svd_noalloc: C = G diag(s) P^T for an r x r float64 matrix on
    the current device, with no handle and no allocation inside the library
    (the outputs are allocated here when not given).  Returns (s, P, status)."""
    if C.dim() != 2 or C.shape[0] != C.shape[1]:
        raise ValueError("C must be square")
    r = C.shape[0]
    dev = C.device
    _need(C, "C", torch.float64, dev, (r, r), contiguous=True)
    if s is None:
        s = torch.empty(r, dtype=torch.float64, device=dev)
    if P is None:
        P = torch.empty(r, r, dtype=torch.float64, device=dev)
    if status is None:
        status = torch.empty(1, dtype=torch.int32, device=dev)
    _need(s, "s", torch.float64, dev, (r,), contiguous=True)
    _need(P, "P", torch.float64, dev, (r, r), contiguous=True)
    _need(status, "status", torch.int32, dev, (1,), contiguous=True)
    with torch.cuda.device(dev):
        st = stream if stream is not None else torch.cuda.current_stream(dev)
        code = lib().wssr_small_svd_noalloc(_ptr(C), r, _ptr(s), _ptr(P), _ptr(status),
                                            ctypes.c_void_p(st.cuda_stream))
    if code != OK:
        raise WssrError(code, "wssr_small_svd_noalloc failed")
    return s, P, status


class AdaptiveRank:
    """Host side of the adaptive rank of Sec. 4.3 and Alg. 2: the handle keeps
    only the columns that pass the ratio r_reg (eq. ruler, on the device);
    after each step, when the last computed column passed too, r_max grows to
    ceil((1 + eps) r_max), at most r_cap.  grow_basis() pads the warm start
    (and the averaged state) to the new r_max: the new columns are drawn by
    the caller's generator (any full-rank basis is a valid warm start), the
    state's new entries are zero (its stored matrix gains zero columns)."""

    def __init__(self, handle, r0, r_reg, eps, r_cap):
        if not (0 < r0 <= r_cap) or not (0.0 <= r_reg < 1.0) or not eps > 0:
            raise ValueError("bad adaptive-rank parameters")
        self.h, self.r_max, self.r_reg, self.eps, self.r_cap = handle, int(r0), float(r_reg), float(eps), int(r_cap)
        if handle is not None:
            handle.set_rank_ratio(self.r_reg)

    def next_rank(self, grow):
        """r_max for the next step given the last step's grow flag."""
        if grow and self.r_max < self.r_cap:
            self.r_max = min(self.r_cap, int(math.ceil((1.0 + self.eps) * self.r_max)))
        return self.r_max

    def after_step(self):
        """Read the last step's (r_eff, grow) and update r_max; returns r_eff."""
        r_eff, grow = self.h.rank_info()
        self.next_rank(grow)
        return r_eff

    def grow_basis(self, V, generator=None, state=()):
        """V (m x r_old, float32) padded to m x r_max; state tensors ([r_old])
        padded with zeros.  Returns (V, *state)."""
        m, r_old = V.shape
        if r_old >= self.r_max:
            return (V, *state)
        extra = torch.randn(m, self.r_max - r_old, generator=generator, device=V.device, dtype=V.dtype)
        v = torch.cat([V, extra * (1.0 / math.sqrt(m))], dim=1).contiguous()
        padded = [torch.cat([t, torch.zeros(self.r_max - r_old, dtype=t.dtype, device=t.device)]) for t in state]
        return (v, *padded)
