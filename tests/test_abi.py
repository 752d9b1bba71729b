"""C-ABI contract checks that need no GPU: the library loads, exports every
entry point include/nctrace.h declares, and fails cleanly without a device."""
import ctypes as C
import os
import re

import pytest

from paper_1902_01137_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "nctrace.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:nc_status|void|uint32_t|const char \*)\s*\**\s*(nc_\w+)\s*\(", text,
                                 flags=re.M)))


def test_every_declared_symbol_is_exported():
    L = _lib.load()
    names = declared_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(_lib.EXPORTED)


def test_abi_version():
    assert _lib.load().nc_abi_version() == 1


def test_struct_layouts_match_header():
    assert C.sizeof(_lib.FieldDesc) == 16 + 6 * 8
    assert C.sizeof(_lib.GridParams) == 24
    assert C.sizeof(_lib.Optics) == 7 * 8 + 8 + 8 + 8 + 8
    assert C.sizeof(_lib.KDist) == 8 + 2 * 16 * 8
    assert C.sizeof(_lib.Camera) == 16 + 12 * 8
    assert C.sizeof(_lib.Sampling) == 40
    assert C.sizeof(_lib.Launch) == 16
    assert C.sizeof(_lib.Progressive) == 24
    assert C.sizeof(_lib.ProgressReport) == 32


# ctypes mirror of each header struct
_STRUCTS = {
    "nc_field_desc": "FieldDesc", "nc_grid_params": "GridParams", "nc_optics": "Optics", "nc_camera": "Camera",
    "nc_sampling": "Sampling", "nc_launch": "Launch", "nc_progressive": "Progressive", "nc_kdist": "KDist",
    "nc_progress_report": "ProgressReport",
}


def test_struct_offsets_match_compiled_header(tmp_path):
    """Compile a C probe against the header and compare every field offset
    and struct size with the ctypes mirrors of the binding."""
    import json
    import subprocess
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "nctrace.h"', 'int main(void) {', 'printf("{");']
    first = True
    for cname, pname in _STRUCTS.items():
        py = getattr(_lib, pname)
        for f in py._fields_:
            lines.append('printf("%s\\"%s.%s\\": %%zu", offsetof(%s, %s));' % ("" if first else ",", cname, f[0],
                                                                               cname, f[0]))
            first = False
        lines.append('printf(",\\"%s\\": %%zu", sizeof(%s));' % (cname, cname))
    lines.append('printf(",\\"nc_counters\\": %zu", sizeof(nc_counters));')
    lines += ['printf("}\\n");', "return 0; }"]
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = json.loads(subprocess.check_output([str(exe)]).decode())
    assert got["nc_counters"] == 8 * _lib.N_COUNTER_WORDS == 8 * len(_lib.COUNTER_NAMES)
    for cname, pname in _STRUCTS.items():
        py = getattr(_lib, pname)
        assert got[cname] == C.sizeof(py), cname
        for f in py._fields_:
            assert got["%s.%s" % (cname, f[0])] == getattr(py, f[0]).offset, (cname, f[0])


def test_null_context_errors():
    L = _lib.load()
    assert L.nc_render(None, None, None, None, None, None, None, None, None) == _lib.NC_ERR_INVALID_ARG
    assert L.nc_grid_build(None, None, None, None, None) == _lib.NC_ERR_INVALID_ARG
    assert L.nc_ctx_create(0, None, None) == _lib.NC_ERR_INVALID_ARG
    assert b"NULL" in L.nc_last_error(None)


def test_no_device_is_reported():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    L = _lib.load()
    h = C.c_void_p()
    st = L.nc_ctx_create(0, None, C.byref(h))
    assert st == _lib.NC_ERR_DEVICE and not h.value
    assert L.nc_last_error(None)
