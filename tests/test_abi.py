"""C-ABI surface checks that need no GPU: the library loads, exports every
function include/chaosvid.h declares, and rejects invalid keys before any
device work."""
import ctypes as ct
import os
import re

import numpy as np
import pytest

from paper_2302_07411_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "chaosvid.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cv_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_binding_exports():
    assert declared_functions() == sorted(binding.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = binding.load()
    for name in declared_functions():
        assert hasattr(lib, name), name


STRUCTS = {  # header typedef -> binding class
    "cv_geom": "CvGeom", "cv_launch": "CvLaunch", "cv_profile": "CvProfile",
    "cv_batch_item": "CvBatchItem", "cv_batch_shape": "CvBatchShape", "cv_batch_info": "CvBatchInfo",
    "cv_server_stats": "CvServerStats",
}


def test_struct_layouts_match_the_binding(tmp_path):
    """Every struct the binding marshals has the header's size and field
    offsets (a C program built with gcc against include/chaosvid.h prints
    them)."""
    import subprocess
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "chaosvid.h"', "int main(void) {"]
    for c_name, py_name in STRUCTS.items():
        cls = getattr(binding, py_name)
        lines.append(f'  printf("{c_name} size %zu\\n", sizeof({c_name}));')
        for field, _ in cls._fields_:
            c_field = "in" if field == "in_" else field
            lines.append(f'  printf("{c_name}.{field} %zu\\n", offsetof({c_name}, {c_field}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = dict(line.rsplit(" ", 1) for line in out if line)
    for c_name, py_name in STRUCTS.items():
        cls = getattr(binding, py_name)
        assert int(got[f"{c_name} size"]) == ct.sizeof(cls), c_name
        for field, _ in cls._fields_:
            assert int(got[f"{c_name}.{field}"]) == getattr(cls, field).offset, f"{c_name}.{field}"


def test_spec_version():
    assert binding.load().cv_spec_version() == 1


def _keysetup(H, W, C, n, r, pm):
    L = binding.load()
    g = binding.CvGeom(H, W, C, n, r)
    pm = np.ascontiguousarray(np.asarray(pm, np.float64).reshape(-1))
    h = ct.c_void_p()
    st = L.cv_keysetup(ct.byref(g), binding.CV_MAP_PLCM,
                       pm.ctypes.data_as(ct.POINTER(ct.c_double)), pm.size, 0, ct.byref(h))
    return st, h


GOOD = [0.3, 0.2, 0.6, 0.4]


@pytest.mark.parametrize("geom,pm,why", [
    ((8, 8, 1, 0, 5), [], "zero in geometry"),
    ((8, 8, 1, 9, 5), GOOD * 9, "more subframes than rows"),
    ((8, 8, 1, 2, 0), GOOD * 2, "zero in geometry"),
    ((8, 1, 1, 8, 5), GOOD * 8, "at least 2 bytes"),
    ((8, 8, 1, 2, 5), GOOD, "4 doubles per subframe"),
    ((8, 8, 1, 1, 5), [0.0, 0.2, 0.6, 0.4], "x0"),
    ((8, 8, 1, 1, 5), [1.0, 0.2, 0.6, 0.4], "x0"),
    ((8, 8, 1, 1, 5), [0.3, 0.5, 0.6, 0.4], "p must"),
    ((8, 8, 1, 1, 5), [0.3, 0.2, 0.6, 0.0], "p must"),
    ((8, 8, 1, 1, 5), [0.3, float("nan"), 0.6, 0.4], "p must"),
    ((10923, 16384, 3, 16, 5), GOOD * 16, "frame too large"),  # one row past the largest
])
def test_keysetup_rejects(geom, pm, why):
    st, h = _keysetup(*geom, pm)
    assert st == binding.CV_E_INVAL and not h.value
    assert why in binding.load().cv_last_error().decode()


def test_null_key_calls_are_rejected():
    L = binding.load()
    assert L.cv_encrypt_frames(None, None, None, None, 1, None) == binding.CV_E_INVAL
    assert L.cv_key_set_path(None, 0) == binding.CV_E_INVAL
    assert L.cv_keystream_frames(None, None, 1, None) == binding.CV_E_INVAL
    L.cv_key_free(None)
