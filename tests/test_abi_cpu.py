"""Host-side checks of the C ABI that need no GPU: the library loads and exports
every entry point include/pm.h declares, and error strings are defined."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pm.h")
LIB = os.path.join(ROOT, "paper_1808_10580_amd", "libpm.so")


def declared_symbols():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(pm_[a-z_0-9]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libpm.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_header_declares_the_entry_points():
    syms = declared_symbols()
    for s in ("pm_create", "pm_problem_create", "pm_observe_time", "pm_observe_dirichlet",
              "pm_observe_time_batch", "pm_step", "pm_sync"):
        assert s in syms


def test_library_exports_every_declared_symbol(lib):
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing


def test_strerror_is_defined_for_every_status(lib):
    lib.pm_strerror.restype = ctypes.c_char_p
    for st in range(0, -7, -1):
        msg = lib.pm_strerror(st).decode()
        assert msg and msg != "unknown status"
    assert lib.pm_strerror(-99).decode() == "unknown status"


def test_null_arguments_are_rejected_without_a_device(lib):
    # argument validation happens before any HIP call
    assert lib.pm_create(None, 0, None) == -1
    assert lib.pm_sync(None) == -1
    f = lib.pm_observe_time
    f.argtypes = [ctypes.c_void_p] * 4 + [ctypes.c_int] + [ctypes.c_double] * 3 + \
        [ctypes.c_int64, ctypes.c_uint64] + [ctypes.c_void_p] * 3
    assert f(None, None, None, None, 1, 0.1, 1.0, 0.1, 1, 0, None, None, None) == -1


def test_binding_fails_loudly_without_library(monkeypatch):
    import paper_1808_10580_amd as pm
    monkeypatch.setattr(pm, "LIB_PATH", os.path.join(ROOT, "nonexistent", "libpm.so"))
    monkeypatch.setattr(pm, "_LIBH", None)
    with pytest.raises(RuntimeError, match="not built"):
        pm.lib()


def test_noalloc_limit_matches_the_header_and_null_arguments_are_rejected(lib):
    import paper_1808_10580_amd as pm
    txt = open(HEADER).read()
    m = re.search(r"#define PM_NOALLOC_MAX_CHUNKS (\d+)", txt)
    assert m and int(m.group(1)) == pm.NOALLOC_MAX_CHUNKS
    f = lib.pm_observe_time_noalloc
    f.argtypes = [ctypes.c_void_p] * 4 + [ctypes.c_int] + [ctypes.c_double] * 3 + \
        [ctypes.c_int64, ctypes.c_uint64] + [ctypes.c_void_p] * 3
    assert f(None, None, None, None, 1, 0.1, 1.0, 0.1, 1, 0, None, None, None) == -1
