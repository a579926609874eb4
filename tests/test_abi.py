"""The C ABI library loads and exports every symbol include/evis.h declares
(CPU only: no compute call is made)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "evis.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|void|const char \*)\s*(evis_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("evis_interpolate", "evis_generate_events", "evis_step_batch", "evis_create",
                 "evis_destroy", "evis_log_luminance", "evis_substep_count", "evis_autotune"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2607_08098_amd import evis
    lib = evis.load_library()
    names = declared_functions()
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # the binding knows the signature of each of them, and of nothing else
    assert sorted(evis.SIGNATURES) == names


def test_struct_layouts_match_the_header():
    from paper_2607_08098_amd import evis
    # evis_pair: 2 int32, 6 pointers, 2 int64
    assert ctypes.sizeof(evis.EvisPair) == 8 + 6 * 8 + 16
    assert ctypes.sizeof(evis.EvisSensor) == 8 + 16 + 16
    assert ctypes.sizeof(evis.EvisState) == 16
    assert ctypes.sizeof(evis.EvisEnv) == ctypes.sizeof(evis.EvisPair) + 40 + 16 + 8 + 8
    assert ctypes.sizeof(evis.EvisNoise) == 6 * 4 + 8 + 8
    assert ctypes.sizeof(evis.EvisTuning) == 24
    assert ctypes.sizeof(evis.EvisSoftEnv) == ctypes.sizeof(evis.EvisPair) + 7 * 8


def test_struct_layouts_match_a_c_compiler(tmp_path):
    """Sizes and field offsets of every ctypes mirror equal what gcc makes
    of include/evis.h."""
    import shutil
    import subprocess
    from paper_2607_08098_amd import evis
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    mirrors = {"evis_pair": evis.EvisPair, "evis_sensor": evis.EvisSensor,
               "evis_state": evis.EvisState, "evis_env": evis.EvisEnv, "evis_noise": evis.EvisNoise,
               "evis_tuning": evis.EvisTuning, "evis_soft_env": evis.EvisSoftEnv,
               "evis_image": evis.EvisImage}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "evis.h"', "int main(void) {"]
    for cname, cls in mirrors.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = {}
    for line in subprocess.check_output([str(exe)]).decode().splitlines():
        cname, field, val = line.split()
        got[(cname, field)] = int(val)
    for cname, cls in mirrors.items():
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert got[(cname, f)] == getattr(cls, f).offset, (cname, f)


def test_null_context_is_rejected_without_touching_a_gpu():
    from paper_2607_08098_amd import evis
    lib = evis.load_library()
    assert lib.evis_abi_version() == 2
    assert lib.evis_step_batch(None, None, 0, None, 0, None, None, 0, None) == evis.EVIS_ERR_INVALID
    assert lib.evis_interpolate(None, None, 1, 0, 1, 0, None, None, None) == evis.EVIS_ERR_INVALID
    assert lib.evis_generate_events(None, None, 1, 1, 1, 0, 1, None, None, 0, None, 0, None, 0,
                                    None) == evis.EVIS_ERR_INVALID
    assert lib.evis_last_error(None) == b"no context"


def test_binding_constants_match_the_header():
    """Every EVIS_* constant the binding defines equals the header's."""
    from paper_2607_08098_amd import evis
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    vals = {}
    for name, val in re.findall(r"#define\s+(EVIS_\w+)\s+\(?(-?\w+)\)?", text):
        vals[name] = val
    for name, val in re.findall(r"(EVIS_\w+)\s*=\s*(-?\w+)", text):
        vals[name] = val
    checked = 0
    for name in dir(evis):
        if name.startswith("EVIS_") and name in vals and isinstance(getattr(evis, name), int):
            v = vals[name]
            want = int(v, 16) if v.lower().startswith(("0x", "-0x")) else int(v.rstrip("f"))
            assert getattr(evis, name) == want, name
            checked += 1
    assert checked >= 12
