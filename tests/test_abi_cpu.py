"""CPU-side checks of the C ABI: the HIP library loads and exports every
function declared in include/*.h (no GPU work is launched)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1108_1310_amd", "libpaper_lamg.so")


def declared_functions():
    names = set()
    for h in ("lamg.h", "lamg_test.h"):
        txt = open(os.path.join(ROOT, "include", h)).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        for m in re.finditer(r"\b(lamg_\w+)\s*\(", txt):
            names.add(m.group(1))
    return sorted(names)


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    names = declared_functions()
    assert "lamg_setup" in names and "lamg_solve_batch" in names and "lamg_t_gs" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_host_only_entry_points():
    """Entry points that touch no device memory: defaults, status strings,
    argument validation before any launch."""
    from paper_1108_1310_amd import lamg
    o = lamg.options()
    assert o.struct_size == ctypes.sizeof(lamg.Options)
    assert (o.gamma, o.nu_pre, o.nu_post, o.tv_k_min, o.tv_k_max, o.tv_sweeps) == (1.5, 1, 2, 4, 10, 3)
    assert abs(o.mu - 4 / 3) < 1e-15 and o.q_max == 2.5 and o.hub_factor == 8 and o.coarsest_max_n == 150
    L = lamg.lib()
    assert L.lamg_status_str(0) == b"ok"
    assert b"connected" in L.lamg_status_str(3)
    h = ctypes.c_void_p()
    # n < 1 and a bad struct_size are refused on the host
    assert L.lamg_setup(0, 0, None, None, None, None, ctypes.byref(h)) == lamg.E_INVALID_ARG
    bad = lamg.options()
    bad.struct_size = 3
    assert L.lamg_setup(4, 0, None, None, None, ctypes.byref(bad), ctypes.byref(h)) == lamg.E_INVALID_ARG
    assert L.lamg_setup(4, 3, None, None, None, None, ctypes.byref(h)) == lamg.E_INVALID_ARG
    # allocator hooks: both or neither
    half = lamg.options()
    half.alloc = lamg.ALLOC_FN(lambda nbytes, ctx: None)
    assert L.lamg_setup(4, 0, None, None, None, ctypes.byref(half), ctypes.byref(h)) == lamg.E_INVALID_ARG
    half = lamg.options()
    half.dealloc = lamg.DEALLOC_FN(lambda ptr, ctx: None)
    assert L.lamg_setup(4, 0, None, None, None, ctypes.byref(half), ctypes.byref(h)) == lamg.E_INVALID_ARG
    # per-level statistics: host-only, NULL handle refused; struct layout of the header
    st = lamg.LevelStats()
    assert ctypes.sizeof(lamg.LevelStats) == 48
    assert L.lamg_level_info(None, 0, ctypes.byref(st)) == lamg.E_INVALID_ARG
    # lean geometric multigrid: side a power of two in [4, LAMG_LGM_MAX_SIDE]
    for side in (0, 2, 3, 6, 100, 32768, -4):
        assert L.lamg_setup_lgm(side, None, ctypes.byref(h)) == lamg.E_INVALID_ARG, side
    assert L.lamg_setup_lgm(8, ctypes.byref(bad), ctypes.byref(h)) == lamg.E_INVALID_ARG
    assert h.value is None
    L.lamg_free(None)  # no-op
    # batch launch configuration: only -1 (autotune) and 0..3
    assert L.lamg_t_batch_config(lamg.BATCH_CONFIGS) == lamg.E_INVALID_ARG
    assert L.lamg_t_batch_config(-2) == lamg.E_INVALID_ARG
    assert L.lamg_t_batch_config(lamg.BATCH_CONFIGS - 1) == 0
    assert L.lamg_t_batch_config(-1) == 0
