"""CPU checks of the C ABI: the library loads, exports every declared symbol, the
ctypes structures match the C layout, and argument checks that precede any device
work reject bad input."""

import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2305_19013_amd import ecg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in sorted(os.listdir(os.path.join(ROOT, "include")))
           if h.endswith(".h")]


def declared_functions():
    names = set()
    for h in HEADERS:
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"\b(ecg_\w+)\s*\(", src):
            names.add(m.group(1))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    L = ecg.lib()
    names = declared_functions()
    assert "ecg_solve" in names and len(names) >= 18
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", ecg.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (ecg_\w+)", out))
    assert set(names) <= exported


def test_struct_layout_matches_c(tmp_path):
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "ecg.h"\n'
                   'int main(){printf("%zu %zu %zu %zu %zu %zu %zu\\n", sizeof(ecg_options), sizeof(ecg_report),'
                   ' offsetof(ecg_options, M), offsetof(ecg_report, vectors_stored), offsetof(ecg_report, status),'
                   ' offsetof(ecg_options, restart_tol), offsetof(ecg_report, vectors_peak));'
                   'return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    vals = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    assert vals == [C.sizeof(ecg.Options), C.sizeof(ecg.Report), ecg.Options.M.offset,
                    ecg.Report.vectors_stored.offset, ecg.Report.status.offset, ecg.Options.restart_tol.offset,
                    ecg.Report.vectors_peak.offset]


def test_options_default_values():
    o = ecg.options()
    assert o.tol == 1e-8 and o.kmax == 20000 and o.reduce == ecg.REDUCE_NONE
    assert o.switch_tol == 1e-5 and o.deflate_tol == 1e-14 and o.precision == ecg.FP64


def test_invalid_operator_rejected_before_device_work():
    L = ecg.lib()
    h = C.c_void_p()
    rp = np.array([0, 1, 2], dtype=np.int64)
    ci = np.array([0, 5], dtype=np.int32)  # column out of range
    v = np.ones(2)
    st = L.ecg_operator_create_csr(2, 2, rp.ctypes.data, ci.ctypes.data, v.ctypes.data, 0, None, C.byref(h))
    assert st == ecg.ECG_EINVAL
    assert b"column" in L.ecg_last_error()
    st = L.ecg_operator_create_csr(0, 0, rp.ctypes.data, ci.ctypes.data, v.ctypes.data, 0, None, C.byref(h))
    assert st == ecg.ECG_EINVAL


@pytest.mark.parametrize("part,t,msg", [([0, 1, 3], 3, b"outside"), ([0, 0, 2], 3, b"empty"),
                                        ([0, 1, 2], 65, b"t must")])
def test_invalid_partition_rejected(part, t, msg):
    L = ecg.lib()
    h = C.c_void_p()
    p = np.array(part, dtype=np.int32)
    st = L.ecg_partition_create(3, t, p.ctypes.data, 0, None, C.byref(h))
    assert st == ecg.ECG_EINVAL
    assert msg in L.ecg_last_error()


def test_c_example_builds_against_the_header_alone():
    """The C++ example uses only include/ecg.h and libecg.so (built by build())."""
    exe = os.path.join(ROOT, "paper_2305_19013_amd", "examples", "poisson_solve")
    src = exe + ".cpp"
    text = open(src).read()
    includes = [ln for ln in text.splitlines() if ln.startswith("#include")]
    assert includes and all(("hip/" in ln or '"ecg.h"' in ln or "<c" in ln or "<vector>" in ln) for ln in includes)
    assert os.path.exists(exe), "run __graft_entry__.build() first"
    out = subprocess.run(["readelf", "-d", exe], capture_output=True, text=True).stdout
    assert "libecg.so" in out
