"""The C-ABI library on the CPU: it loads, exports every declared entry
point, and its host-only calls behave (no kernel launches here)."""
import ctypes
import os
import re
import subprocess

import pytest

import paper_1609_08114_amd as blp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "blp.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(blp_[a-z_]+)\s*\(", text)))


def test_header_matches_binding():
    assert declared_functions() == sorted(blp.EXPORTS)


def test_library_exports_every_declared_symbol():
    assert os.path.exists(blp.LIB_PATH), "libblp.so not built"
    out = subprocess.run(["nm", "-D", "--defined-only", blp.LIB_PATH], capture_output=True, text=True).stdout
    syms = set(ln.split()[-1] for ln in out.splitlines() if ln.strip())
    missing = [f for f in declared_functions() if f not in syms]
    assert not missing, missing
    lib = blp.lib()
    for f in declared_functions():
        assert getattr(lib, f) is not None


def test_host_only_calls():
    assert blp.blp_abi_version() == 5
    o = blp.blp_options_default()
    assert o.device == 0 and o.mode == 0 and o.variant == -1 and o.max_iter == 0
    vs = blp.variants()
    assert len(vs) >= 4
    for name, rows, cols in vs:
        assert rows >= 4 and cols >= 2 and name
    # rows x cols grows along the table's small end
    assert vs[0][1] * vs[0][2] <= vs[-1][1] * vs[-1][2]
    assert blp.blp_variant_info(len(vs)) is None
    assert blp.lib().blp_options_default(None) == blp.BLP_ERR_ARG
    assert blp.lib().blp_create(None, None) == blp.BLP_ERR_ARG


def test_null_handle_calls_fail_cleanly():
    L = blp.lib()
    assert L.blp_solve_batch(None, None, None, None) == blp.BLP_ERR_ARG
    assert L.blp_get_solution(None, 0, None, None, None, None, None) == blp.BLP_ERR_ARG
    assert L.blp_backward(None, None, None, None, None, None, None, None) == blp.BLP_ERR_ARG
    assert L.blp_last_error(None) == b"null handle"
    L.blp_destroy(None)


def test_create_without_gpu_reports_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    rc = blp.lib().blp_create(ctypes.byref(h), None)
    assert rc in (blp.BLP_ERR_HIP, blp.BLP_ERR_ARG) and not h.value


def test_struct_layouts_match_header(tmp_path):
    """The ctypes structures of the binding have the C header's field
    offsets and sizes (compiled and printed by gcc)."""
    src = tmp_path / "layout.c"
    fields = {"blp_options": [f for f, _ in blp.blp_options._fields_],
              "blp_batch": [f for f, _ in blp.blp_batch._fields_],
              "blp_outputs": [f for f, _ in blp.blp_outputs._fields_]}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "blp.h"', "int main(void) {"]
    for st, fs in fields.items():
        lines.append(f'printf("{st} %zu\\n", sizeof({st}));')
        for f in fs:
            lines.append(f'printf("{st}.{f} %zu\\n", offsetof({st}, {f}));')
    lines += ["return 0;", "}"]
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    got = dict(ln.split() for ln in subprocess.run([str(exe)], capture_output=True, text=True).stdout.splitlines())
    for st, cls in (("blp_options", blp.blp_options), ("blp_batch", blp.blp_batch), ("blp_outputs", blp.blp_outputs)):
        assert int(got[st]) == ctypes.sizeof(cls), st
        for f in fields[st]:
            assert int(got[f"{st}.{f}"]) == getattr(cls, f).offset, (st, f)
