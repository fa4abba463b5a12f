"""Host-side checks of the C ABI (no GPU needed): the library loads, exports every
function include/dg.h declares, and rejects bad arguments before touching the
device."""
import ctypes
import os
import re
import subprocess

import pytest

import paper_2507_11094_amd as dg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "dg.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dg_[a-z_]+)\s*\(", text)))


def test_header_declares_the_binding_list():
    assert declared_functions() == sorted(dg.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = dg.load_library()
    out = subprocess.run(["nm", "-D", "--defined-only", dg.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (dg_[a-z_]+)$", out, flags=re.M))
    for name in declared_functions():
        assert name in exported, name
        assert hasattr(lib, name)


def test_bad_arguments_are_rejected_on_the_host():
    lib = dg.load_library()
    out = ctypes.c_void_p()
    assert lib.dg_graph_create(0, 0, None, None, None, 0, None, ctypes.byref(out)) == dg.DG_EINVAL
    assert lib.dg_graph_create(4, -1, None, None, None, 0, None, ctypes.byref(out)) == dg.DG_EINVAL
    assert lib.dg_graph_create(4, 3, None, None, None, 0, None, ctypes.byref(out)) == dg.DG_EINVAL
    assert lib.dg_graph_create(4, 0, None, None, None, 0x80, None, ctypes.byref(out)) == dg.DG_EINVAL
    assert lib.dg_graph_create(4, 0, None, None, None, 0, None, None) == dg.DG_EINVAL
    assert lib.dg_apply_batch(None, 1, None, None, None, None, 0, 0, None) == dg.DG_EINVAL
    assert lib.dg_sssp_read(None, None, None, 0) == dg.DG_EINVAL
    assert lib.dg_pr_read(None, None, None, None, 0) == dg.DG_EINVAL
    assert lib.dg_tc_read(None, None) == dg.DG_EINVAL
    assert lib.dg_query_detach(None) == dg.DG_EINVAL
    assert lib.dg_graph_destroy(None) == dg.DG_EINVAL
    assert b"null" in lib.dg_last_error() or lib.dg_last_error()


def test_struct_layouts_match_header(tmp_path):
    """The ctypes mirrors have the sizes and field offsets the C compiler gives."""
    fields = {"dg_config": dg.Config, "dg_batch_stats": dg.BatchStats, "dg_kernel_prof": dg.KernelProf,
              "dg_server_config": dg.ServerConfig, "dg_request": dg.Request, "dg_result": dg.Result}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "dg.h"', "int main(void) {"]
    for cname, cls in fields.items():
        lines.append(f'printf("%zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("%zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    want = []
    for cls in fields.values():
        want.append(ctypes.sizeof(cls))
        want.extend(getattr(cls, f).offset for f, _ in cls._fields_)
    assert got == want
