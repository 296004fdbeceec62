"""The C ABI library: it loads without a GPU, exports every function that
include/spgemm.h declares, and the binding's structs match the C layout."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "spgemm.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(spgemm_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_1504_05022_amd import lib as L
    if not os.path.exists(L.LIB_PATH):
        from paper_1504_05022_amd import build
        build.build()
    return L.load()


def test_exports_every_declared_function(lib):
    from paper_1504_05022_amd import lib as L
    names = declared_functions()
    assert set(names) == set(L.EXPORTS)
    for n in names:
        assert hasattr(lib, n), n


def test_status_strings(lib):
    from paper_1504_05022_amd import lib as L
    for code in (0, -1, -2, -3, -4, -5):
        assert lib.spgemm_strerror(code)
    o = L.default_options()
    assert list(o.bin_edges) == [32, 64, 128, 256, 512]
    assert o.long_slot == 256
    assert o.timing == 0 and o.timing_mask == 0


def test_struct_layout_matches_c(tmp_path):
    """Compile a C probe against the header and compare sizes and offsets."""
    from paper_1504_05022_amd import lib as L
    probe = tmp_path / "probe.c"
    fields = {"spgemm_csr": L.CsrDesc, "spgemm_options": L.Options, "spgemm_info": L.Info,
              "spgemm_batch_stats": L.BatchStats}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "spgemm.h"', "int main(void){"]
    for cname, ct in fields.items():
        lines.append('printf("%s %%zu\\n", sizeof(%s));' % (cname, cname))
        for f, _ in ct._fields_:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (cname, f, cname, f))
    lines.append("return 0;}")
    probe.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(probe), "-o", str(exe)])
    out = dict(l.rsplit(" ", 1) for l in subprocess.check_output([str(exe)], text=True).split("\n") if l)
    for cname, ct in fields.items():
        assert int(out[cname]) == ctypes.sizeof(ct), cname
        for f, _ in ct._fields_:
            assert int(out["%s.%s" % (cname, f)]) == getattr(ct, f).offset, (cname, f)


def test_null_arguments_are_rejected(lib):
    """Host-side argument checks run before any device work."""
    from paper_1504_05022_amd import lib as L
    plan = ctypes.c_void_p()
    rc = lib.spgemm_analyze(None, None, None, L._ALLOC_T(0), L._FREE_T(0), None, None,
                            ctypes.byref(plan), None)
    assert rc == -1
    assert b"NULL" in lib.spgemm_last_error()
    A = L.CsrDesc(4, 5, 0, 1, 0, 0, 1)
    B = L.CsrDesc(6, 5, 0, 1, 0, 0, 1)
    rc = lib.spgemm_analyze(ctypes.byref(A), ctypes.byref(B), None, L._ALLOC_T(0), L._FREE_T(0),
                            None, None, ctypes.byref(plan), None)
    assert rc == -1 and b"inner" in lib.spgemm_last_error()
    B2 = L.CsrDesc(5, 5, 0, 1, 0, 0, 0)
    rc = lib.spgemm_analyze(ctypes.byref(A), ctypes.byref(B2), None, L._ALLOC_T(0), L._FREE_T(0),
                            None, None, ctypes.byref(plan), None)
    assert rc == -1 and b"dtype" in lib.spgemm_last_error()
    big = L.CsrDesc(1 << 31, 5, 0, 1, 0, 0, 1)
    rc = lib.spgemm_analyze(ctypes.byref(big), ctypes.byref(B2), None, L._ALLOC_T(0),
                            L._FREE_T(0), None, None, ctypes.byref(plan), None)
    assert rc == -3
    opts = L.default_options(bin_edges=(33, 64, 128, 256, 512))
    rc = lib.spgemm_analyze(ctypes.byref(A), ctypes.byref(L.CsrDesc(5, 5, 0, 1, 0, 0, 1)),
                            ctypes.byref(opts), L._ALLOC_T(0), L._FREE_T(0), None, None,
                            ctypes.byref(plan), None)
    assert rc == -1 and b"bin_edges" in lib.spgemm_last_error()
    assert lib.spgemm_compute(None, None, None, None, None, None) == -1
    assert lib.spgemm_plan_destroy(None) == 0
