"""Host-only checks of the C ABI: the library loads without a GPU, exports
every entry point that include/fms.h declares, and its struct layouts agree
with the Python binding.  Nothing here launches GPU work."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fms.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fms_[a-z_]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    from paper_2007_14283_amd import _binding as B
    assert _declared() == sorted(B.EXPORTS)


def test_library_exports_every_declared_symbol():
    from paper_2007_14283_amd import _binding as B
    lib = ctypes.CDLL(B.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", B.LIB_PATH], capture_output=True, text=True).stdout
    for name in _declared():
        assert re.search(rf"\bT {name}\b", out), name


def test_default_params_and_status_strings():
    import paper_2007_14283_amd as F
    p = F.default_params()
    assert (p.bandwidth, p.gamma, p.n_initial, p.big_l, p.big_h, p.p_target) == (0.1, 0.9, 128, 2.0, 8.0, 0.99)
    assert (p.max_iter, p.max_rounds, p.precision, p.refine_iters, p.conv_tol) == (100, 32, 0, 2, 0.0)
    lib = F.library()
    for code in (0, -1, -2, -3, -4, -5):
        assert lib.fms_status_string(code)
    assert lib.fms_status_string(42) == b"unknown status"


def test_struct_layouts_match_header(tmp_path):
    from paper_2007_14283_amd import _binding as B
    src = tmp_path / "layout.c"
    structs = [("fms_params", B.FmsParams), ("fms_stats", B.FmsStats), ("fms_frame", B.FmsFrame),
               ("fms_tune_entry", B.FmsTuneEntry), ("fms_tune_report", B.FmsTuneReport)]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "fms.h"', "int main(void) {"]
    want = []
    for cname, py in structs:
        lines.append(f'printf("%zu\\n", sizeof({cname}));')
        want.append(ctypes.sizeof(py))
        for f, _ in py._fields_:
            lines.append(f'printf("%zu\\n", offsetof({cname}, {f}));')
            want.append(getattr(py, f).offset)
    lines += ["return 0; }"]
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    vals = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    assert vals == want


def test_missing_library_fails_loudly(tmp_path):
    from paper_2007_14283_amd import _binding as B
    with pytest.raises(RuntimeError):
        B.load.__wrapped__(str(tmp_path / "nope.so")) if hasattr(B.load, "__wrapped__") else \
            _fresh_load(B, str(tmp_path / "nope.so"))


def _fresh_load(B, path):
    saved = B._lib
    B._lib = None
    try:
        return B.load(path)
    finally:
        B._lib = saved


def test_null_handle_and_bad_counts_are_rejected_on_the_host():
    # Argument checks run before any HIP call, so they need no GPU.
    import paper_2007_14283_amd as F
    from paper_2007_14283_amd import _binding as B
    lib = F.library()
    p = B.FmsParams()
    lib.fms_default_params(ctypes.byref(p))
    nm = ctypes.c_int32(0)
    st = B.FmsStats()
    bad = B.FMS_ERR_INVALID_ARG
    assert lib.fms_destroy(None) == B.FMS_OK
    assert lib.fms_clear_tuning(None) == bad
    assert lib.fms_cluster(None, None, None, 32, 1, None, 4, 4, 32, ctypes.byref(p), None, None, 0,
                           ctypes.byref(nm), None, ctypes.byref(st)) == bad
    frames = (B.FmsFrame * 2)()
    offs = (ctypes.c_int32 * 3)()
    stats = (B.FmsStats * 2)()
    assert lib.fms_cluster_batch(None, None, 2, frames, 32, ctypes.byref(p), None, None, 0, offs, stats) == bad
    assert lib.fms_seed_order(None, None, 10, 0, None) == bad
    n_ent = ctypes.c_int32(0)
    rep = B.FmsTuneReport()
    assert lib.fms_autotune(None, None, frames, 32, ctypes.byref(p), None, 0, ctypes.byref(n_ent),
                            ctypes.byref(rep)) == bad
    # A batch tuner needs at least two frames (checked before the handle).
    assert lib.fms_autotune_batch(None, None, 1, frames, 32, ctypes.byref(p), None, 0, ctypes.byref(n_ent),
                                  ctypes.byref(rep)) == bad
