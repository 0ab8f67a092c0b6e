"""CPU checks of the C ABI boundary: the library loads and exports every
symbol include/abip.h declares (no compute calls: there may be no GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "abip.h")
LIB = os.path.join(ROOT, "paper_1805_12344_amd", "libabip.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(abip_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["abip_setup", "abip_solve", "abip_solve_batch", "abip_backward", "abip_free",
                     "abip_last_error", "abip_default_settings"]:
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libabip.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name
    lib.abip_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.abip_version()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libabip.so not built")
def test_binding_exports_match_header():
    import paper_1805_12344_amd as pkg
    assert sorted(pkg.EXPORTS) == declared_functions()
    for name in pkg.EXPORTS:
        assert callable(getattr(pkg, name))


@pytest.mark.skipif(not os.path.exists(LIB), reason="libabip.so not built")
def test_default_settings_and_argument_errors_without_gpu():
    """Host-only entry points: defaults and argument validation touch no device."""
    import paper_1805_12344_amd as pkg
    s = pkg.abip_default_settings()
    assert s.eps == 1e-6 and s.alpha == 1.8 and s.beta == 1.0 and s.gamma == 0.5
    assert s.max_admm_iters == 1_000_000
    lib = pkg.lib()
    assert lib.abip_default_settings(None) == pkg.ABIP_E_INVALID
    assert lib.abip_solve(None, None, None, None, None) == pkg.ABIP_E_INVALID
    assert b"null" in lib.abip_last_error()
    assert lib.abip_free(None) == pkg.ABIP_OK
