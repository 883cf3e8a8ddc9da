"""CPU checks of the C ABI: the library loads, exports every function
include/esbgk.h declares, and its pure host paths (sizes, validation, error
codes) behave as documented.  No compute call is made here."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "esbgk.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(esbgk_[a-z_0-9]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def E():
    from paper_2512_03586_amd import esbgk
    if not os.path.exists(esbgk.LIB_PATH):
        pytest.fail("libesbgk.so not built (run __graft_entry__.build())")
    return esbgk


def test_header_declares_the_entry_points():
    names = declared_functions()
    for must in ("esbgk_workspace_size", "esbgk_create", "esbgk_destroy", "esbgk_set_state",
                 "esbgk_set_mask", "esbgk_set_f", "esbgk_step", "esbgk_get_moments",
                 "esbgk_get_mask", "esbgk_get_f", "esbgk_get_stats", "esbgk_indicator",
                 "esbgk_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol(E):
    L = C.CDLL(E.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_config_struct_layout_matches_header(E):
    # 12 int32 fields then 9 doubles, no padding
    assert C.sizeof(E.esbgk_config) == 12 * 4 + 9 * 8
    assert C.sizeof(E.esbgk_stats) == 8 + 8 + 8 + 4 * 4 + 8


def test_workspace_size_is_pure_and_scales(E):
    a = E.esbgk_workspace_size(E.make_config(32, 32, 16, 8.0, precision=E.FP64))
    b = E.esbgk_workspace_size(E.make_config(32, 32, 16, 8.0, precision=E.FP32))
    c = E.esbgk_workspace_size(E.make_config(32, 32, 16, 8.0, precision=E.BF16))
    assert a > b > c > 3 * 32 * 32 * 256 * 2
    big = E.esbgk_workspace_size(E.make_config(1024, 1024, 64, 20.0, precision=E.FP32))
    assert big > 3 * 1024 * 1024 * 4096 * 4       # three f buffers of 17 GB


@pytest.mark.parametrize("kw,msg", [
    (dict(nv=10), "multiple of 4"),
    (dict(nv=68), "multiple of 4"),
    (dict(beta=1.0), "beta"),
    (dict(scheme=7), "scheme"),
    (dict(eta=0.0), "eta"),
    (dict(precision=3, scheme=0), "mixed storage form needs ARS"),
    (dict(precision=4), "precision"),
    (dict(indicator=2, learned_k=0), "learned_k"),
])
def test_bad_configs_are_rejected(E, kw, msg):
    base = dict(nx=8, ny=8, nv=16, vmax=8.0)
    base.update(kw)
    nx, ny, nv, vmax = base.pop("nx"), base.pop("ny"), base.pop("nv"), base.pop("vmax")
    cfg = E.make_config(nx, ny, nv, vmax, **base)
    with pytest.raises(E.EsbgkError) as ei:
        E.esbgk_workspace_size(cfg)
    assert ei.value.code == E.EINVAL and msg in str(ei.value)


def test_create_checks_workspace(E):
    cfg = E.make_config(8, 8, 16, 8.0)
    L = E.lib()
    ctx = C.c_void_p()
    assert L.esbgk_create(C.byref(cfg), None, 1 << 20, C.byref(ctx)) == E.EINVAL
    assert L.esbgk_create(C.byref(cfg), C.c_void_p(256 * 1000 + 8), 1 << 30, C.byref(ctx)) == E.EINVAL
    assert b"aligned" in L.esbgk_last_error()
    need = E.esbgk_workspace_size(cfg)
    assert L.esbgk_create(C.byref(cfg), C.c_void_p(1 << 20), need - 1, C.byref(ctx)) == E.ENOMEM
