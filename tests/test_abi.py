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
    assert pd.lib.pd_set_fine_blocking(None, 2, 3) == pd.EINVAL
    assert pd.lib.pd_get_fine_blocking(None, None, None) == pd.EINVAL
    assert pd.lib.pd_parareal_continue(None, 1e-8, 4, None) == pd.EINVAL
    assert pd.lib.pd_last_error(None) == b"null context"
    assert pd.lib.pd_create(None, 0) == pd.EINVAL


def test_report_struct_matches_header():
    """The binding's pd_report mirror has the header's fields, in order, with
    the same types and array length."""
    import paper_1902_00387_amd as pd
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    body = re.search(r"typedef struct \{(.*?)\} pd_report;", text, flags=re.S).group(1)
    fields = re.findall(r"(int|double)\s+([A-Za-z_0-9]+)(\[PD_MAX_ITER\])?;", body)
    mirror = pd.Report._fields_
    assert [n for _, n, _ in fields] == [n for n, _ in mirror]
    ctype = {"int": ctypes.c_int, "double": ctypes.c_double}
    for (t, n, arr), (_, ct) in zip(fields, mirror):
        want = ctype[t] * pd.MAX_ITER if arr else ctype[t]
        assert ctypes.sizeof(ct) == ctypes.sizeof(want), n
    assert "#define PD_MAX_ITER %d" % pd.MAX_ITER in open(HEADER).read()
