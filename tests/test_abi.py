"""C-ABI library: loads on the CPU host and exports every declared symbol
(no compute calls: those need a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pitdyn.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pd_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_binding_symbols():
    import paper_1902_00387_amd as pd
    assert declared_symbols() == sorted(pd.SYMBOLS)


def test_library_exports_every_declared_symbol():
    import paper_1902_00387_amd as pd
    lib = ctypes.CDLL(pd.LIB_PATH)
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing


def test_library_is_built_for_gfx950():
    import paper_1902_00387_amd as pd
    blob = open(pd.LIB_PATH, "rb").read()
    assert b"gfx950" in blob


def test_null_context_calls_fail_cleanly():
    import paper_1902_00387_amd as pd
    assert pd.lib.pd_set_problem(None, 1, 10.0, 1.0, 32) == pd.EINVAL
    assert pd.lib.pd_set_path(None, 0) == pd.EINVAL
    assert pd.lib.pd_last_error(None) == b"null context"
    assert pd.lib.pd_create(None, 0) == pd.EINVAL
