"""The C-ABI library loads and exports every entry point include/lqt.h declares.

CPU-only: loads the shared object and resolves symbols; makes no compute call.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lqt.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lqt_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("lqt_plan", "lqt_solve", "lqt_submit", "lqt_poll", "lqt_destroy", "lqt_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2104_03186_amd import _lib

    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("liblqt.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(_lib.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(_lib.EXPORTED) == set(declared_functions())


def test_last_error_without_plan_is_host_only():
    from paper_2104_03186_amd import _lib

    lib = _lib.load()
    s = lib.lqt_last_error(None)
    assert isinstance(s, bytes)


def test_product_path_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_2104_03186_amd import _lib

    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        _lib.load()


STRUCTS = {
    "lqt_problem": ("Problem", ["nx", "nu", "ny", "nyT", "T", "per_step", "F", "c", "L", "H", "X", "U", "r", "HT",
                                "XT", "rT", "x0", "M", "s"]),
    "lqt_outputs": ("Outputs", ["S", "v", "K", "d", "x", "u", "status"]),
    "lqt_nl_problem": ("NLProblem", ["model", "ny", "nyT", "T", "per_step", "dt", "H", "X", "U", "r", "HT", "XT",
                                     "rT", "x0"]),
    "lqt_fs_problem": ("FSProblem", ["nstates", "ncontrols", "T", "per_step", "next", "cost", "cost_T", "x0"]),
    "lqt_fs_outputs": ("FSOutputs", ["V", "u", "x", "ux", "status"]),
    "lqt_plan_desc": ("PlanDesc", ["device", "max_nx", "max_nu", "prec", "hbm_budget_bytes", "max_steps",
                                   "max_inflight", "trajectory"]),
    "lqt_routing": ("Routing", ["path", "block", "lane_chunk", "wave_chunk", "tree"]),
    "lqt_serve_stats": ("ServeStats", ["submitted", "completed", "batches", "queued", "running_batches",
                                       "max_running_batches", "max_batch", "pool_bytes", "pool_in_use",
                                       "pool_peak"]),
}


def test_binding_structs_match_the_header(tmp_path):
    """The ctypes mirrors in _lib.py have the header's sizes and field offsets
    (compiled with the host C compiler; no GPU)."""
    import shutil
    import subprocess

    from paper_2104_03186_amd import _lib

    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "lqt.h"', "int main(void) {"]
    for cname, (_, fields) in STRUCTS.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f in fields:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = {}
    for line in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines():
        cname, key, val = line.split()
        got[(cname, key)] = int(val)
    for cname, (pyname, fields) in STRUCTS.items():
        cls = getattr(_lib, pyname)
        assert ctypes.sizeof(cls) == got[(cname, "size")], cname
        for f in fields:
            assert getattr(cls, f).offset == got[(cname, f)], (cname, f)


def test_plan_rejects_unknown_trajectory_before_device_use():
    from paper_2104_03186_amd import _lib

    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("library not built")
    lib = _lib.load()
    d = _lib.PlanDesc(device=0, max_nx=4, max_nu=2, prec=_lib.PREC_FP64, trajectory=7)
    h = ctypes.c_void_p()
    assert lib.lqt_plan(ctypes.byref(d), ctypes.byref(h)) == _lib.EINVAL
    assert b"trajectory" in lib.lqt_last_error(None)
