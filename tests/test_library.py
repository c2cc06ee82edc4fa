"""Host-side checks of the C-ABI library: it loads, exports every symbol that
include/seasd.h declares, and the binding's structures match the header.
No GPU is touched."""
import ctypes
import os
import re

import pytest

from paper_1506_08481_amd import seasd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    src = open(os.path.join(ROOT, "include", "seasd.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|int64_t|const char\*)\s+(seasd_\w+)\s*\(", src, re.M)))


def test_library_exports_header_symbols():
    if not os.path.exists(seasd.LIB_PATH):
        pytest.skip("libseasd.so not built")
    lib = ctypes.CDLL(seasd.LIB_PATH)
    declared = _header_functions()
    assert declared, "no declarations parsed"
    for name in declared:
        assert hasattr(lib, name), name
    assert set(declared) == set(seasd.SYMBOLS)


def _header_struct_fields(name):
    src = open(os.path.join(ROOT, "include", "seasd.h")).read()
    body = re.search(r"typedef struct %s \{(.*?)\} %s;" % (name, name), src, re.S).group(1)
    fields = []
    for line in body.splitlines():
        line = line.split("/*")[0].strip()
        if not line:
            continue
        if line.startswith("const "):
            line = line[len("const "):]
        typ, rest = line.split(None, 1)
        for f in rest.rstrip(";").split(","):
            f = f.strip()
            if f.startswith("*"):   # pointer field
                typ, f = typ + "*", f.lstrip("* ")
            fields.append((typ, f))
    return fields


@pytest.mark.parametrize("cname,pyclass", [("seasd_config", seasd.seasd_config),
                                           ("seasd_solve_stats", seasd.seasd_solve_stats),
                                           ("seasd_brownian_stats", seasd.seasd_brownian_stats),
                                           ("seasd_bsr6", seasd.seasd_bsr6)])
def test_binding_struct_layout_matches_header(cname, pyclass):
    cmap = {"int32_t": ctypes.c_int32, "int64_t": ctypes.c_int64, "double": ctypes.c_double,
            "int32_t*": ctypes.c_void_p, "double*": ctypes.c_void_p}
    hdr = _header_struct_fields(cname)
    names = [re.sub(r"\[\d+\]$", "", f) for _, f in hdr]
    assert names == [f for f, _ in pyclass._fields_]
    for (typ, f), (pf, pt) in zip(hdr, pyclass._fields_):
        m = re.search(r"\[(\d+)\]$", f)
        if m:   # fixed-size array field
            assert issubclass(pt, ctypes.Array) and pt._length_ == int(m.group(1)) and pt._type_ is cmap[typ], f
        else:
            assert cmap[typ] is pt, f


def test_default_config_and_validation_on_host():
    # seasd_default_config and the error strings touch no device state
    if not os.path.exists(seasd.LIB_PATH):
        pytest.skip("libseasd.so not built")
    c = seasd.default_config()
    assert tuple(c.grid) == (64, 64, 64) and c.P == 16 and c.rc_factor == 4.0 and c.precision == seasd.SEASD_FP64
    assert seasd.lib().seasd_error_string(seasd.SEASD_E_OVERLAP).decode().startswith("overlapping")


def test_bench_refuses_more_than_one_gpu():
    """The benchmark runs on one GPU; asking for more exits with a message
    before anything touches a device."""
    import json
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_binding_constants_match_header():
    """Every SEASD_* integer constant the binding defines has the header's value."""
    src = open(os.path.join(ROOT, "include", "seasd.h")).read()
    defs = {m.group(1): int(m.group(2)) for m in re.finditer(r"^#define\s+(SEASD_\w+)\s+(-?\d+)\b", src, re.M)}
    assert {"SEASD_FP64", "SEASD_FP32", "SEASD_MIXED"} <= set(defs)
    checked = 0
    for name, value in defs.items():
        if hasattr(seasd, name):
            assert getattr(seasd, name) == value, name
            checked += 1
    assert checked >= 10


def test_binding_rejects_bad_tensors_before_the_library():
    """The binding's argument checks run on the host: host memory, a
    non-tensor or an FP32 tensor is refused with TypeError before any pointer
    reaches the library (the GPU tests cover short tensors)."""
    import torch
    pos = torch.zeros((8, 3), dtype=torch.float64)
    with pytest.raises(TypeError):
        seasd._require(pos, (None, 3), "pos")                  # host memory
    with pytest.raises(TypeError):
        seasd._require([0.0] * 24, (None, 3), "pos")           # not a tensor
    with pytest.raises(TypeError):
        seasd._require_sphere_arrays(pos.float(), torch.ones(8), None)
