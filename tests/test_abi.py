"""The C-ABI library loads and exports every symbol the header declares; host
argument checks work without a GPU.  CPU only (no compute call)."""
import ctypes
import pathlib
import re

import pytest

ROOT = pathlib.Path(__file__).resolve().parents[1]
HEADER = ROOT / "include" / "wssr.h"


def declared_symbols():
    text = HEADER.read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(wssr_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    syms = declared_symbols()
    for s in ("wssr_create", "wssr_step", "wssr_destroy", "wssr_status_sync", "wssr_last_error"):
        assert s in syms


def test_library_exports_every_declared_symbol():
    from paper_2512_05749_amd import wssr
    lib = wssr.lib()
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing
    assert "gfx950" in wssr.version()


def test_binding_signatures_cover_header():
    from paper_2512_05749_amd import wssr
    assert set(declared_symbols()) == set(wssr._SIGS)


def test_create_rejects_bad_config_and_missing_device():
    from paper_2512_05749_amd import wssr
    lib = wssr.lib()
    h = ctypes.c_void_p()
    bad = wssr.Config(1, 10, 4, 2, 0, 0, None)          # n_max < 2
    assert lib.wssr_create(ctypes.byref(bad), ctypes.byref(h)) == wssr.ERR_INVALID_ARG
    assert not h.value
    bad = wssr.Config(100, 10, 513, 2, 0, 0, None)      # r_max > 512
    assert lib.wssr_create(ctypes.byref(bad), ctypes.byref(h)) == wssr.ERR_INVALID_ARG
    import torch
    if not torch.cuda.is_available():
        good = wssr.Config(100, 10, 4, 2, 0, 0, None)
        assert lib.wssr_create(ctypes.byref(good), ctypes.byref(h)) == wssr.ERR_NO_DEVICE
        assert not h.value
        assert lib.wssr_last_error(None)


def test_null_handle_calls_are_rejected():
    from paper_2512_05749_amd import wssr
    lib = wssr.lib()
    assert lib.wssr_destroy(None) == wssr.ERR_INVALID_ARG
    assert lib.wssr_step(None, 10, 10, None, 10, None, None, 1.0, 1, 1, None, None) == wssr.ERR_INVALID_ARG
    assert lib.wssr_step_avg(None, 10, 10, None, 10, None, None, None, 1.0, 1, 1, 0.5, None, None, None,
                             None) == wssr.ERR_INVALID_ARG
    assert lib.wssr_step_sketch(None, 10, 10, None, 10, None, None, None, 2, 0, None, 1.0, 1, None,
                                None) == wssr.ERR_INVALID_ARG
    assert lib.wssr_spring(None, 10, 10, None, 10, None, 1.0, 0.0, 0.0, None, None) == wssr.ERR_INVALID_ARG
    assert lib.wssr_set_rank_ratio(None, 0.1) == wssr.ERR_INVALID_ARG
    assert lib.wssr_rank_info(None, None, None) == wssr.ERR_INVALID_ARG
    code = ctypes.c_int32()
    assert lib.wssr_status_sync(None, ctypes.byref(code), None) == wssr.ERR_INVALID_ARG


def test_adaptive_rank_growth_rule():
    """Host logic of the rank growth (Alg. 2): r_max <- ceil((1 + eps) r_max)
    while the last column passes, capped; no growth otherwise."""
    import torch

    from paper_2512_05749_amd.wssr import AdaptiveRank
    ar = AdaptiveRank(None, 100, 0.01, 0.2, 200)
    assert ar.next_rank(False) == 100
    assert ar.next_rank(True) == 120
    assert ar.next_rank(True) == 144
    assert ar.next_rank(True) == 173
    assert ar.next_rank(True) == 200
    assert ar.next_rank(True) == 200
    ar = AdaptiveRank(None, 8, 0.01, 0.5, 64)
    ar.next_rank(True)
    v = torch.ones(30, 8)
    s, l = torch.ones(8, dtype=torch.float64), torch.ones(8, dtype=torch.float64)
    v2, s2, l2 = ar.grow_basis(v, torch.Generator().manual_seed(0), (s, l))
    assert v2.shape == (30, 12) and torch.equal(v2[:, :8], v)
    assert torch.equal(s2[8:], torch.zeros(4, dtype=torch.float64)) and torch.equal(l2[:8], l)
    for bad in ((0, 0.1, 0.1, 10), (20, 0.1, 0.1, 10), (5, 1.0, 0.1, 10), (5, 0.1, 0.0, 10)):
        with pytest.raises(ValueError):
            AdaptiveRank(None, *bad)
