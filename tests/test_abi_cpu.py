"""Host-side checks of the C-ABI library that need no GPU: it loads, exports
every entry point include/gmco.h declares, its ctypes structs match the C
layout, and argument errors are reported without touching a device."""
import ctypes as C
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gmco.h")


def _lib():
    from paper_1904_01567_amd import _binding
    if not os.path.exists(_binding.LIB_PATH):
        pytest.skip("libgmco.so not built (python -m paper_1904_01567_amd.build)")
    return _binding, _binding.load_library()


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(gmco_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_what_binding_lists():
    from paper_1904_01567_amd import _binding
    assert _declared() == sorted(_binding.EXPORTS)


def test_library_exports_every_declared_symbol():
    _, lib = _lib()
    out = subprocess.run(["nm", "-D", "--defined-only", _binding_path()], capture_output=True,
                         text=True, check=True).stdout
    syms = set(re.findall(r"\bT\s+(gmco_\w+)", out))
    for name in _declared():
        assert name in syms, name
        assert hasattr(lib, name)


def _binding_path():
    from paper_1904_01567_amd import _binding
    return _binding.LIB_PATH


def test_ctypes_layout_matches_header():
    b, _ = _lib()
    src = r'''
#include <stdio.h>
#include <stddef.h>
#include "gmco.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu\n", sizeof(gmco_opts), sizeof(gmco_case), sizeof(gmco_run),
         sizeof(gmco_run_info), sizeof(gmco_plan_metrics), sizeof(gmco_tuning), sizeof(gmco_select_opts));
  printf("%zu %zu %zu\n", offsetof(gmco_plan_metrics, D90_pct), offsetof(gmco_plan_metrics, status),
         offsetof(gmco_case, dose_rate));
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        cfile = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(cfile, "w").write(src)
        subprocess.run(["gcc", "-I", os.path.dirname(HEADER), cfile, "-o", exe], check=True)
        lines = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split("\n")
    sizes = [int(v) for v in lines[0].split()]
    offs = [int(v) for v in lines[1].split()]
    assert sizes == [C.sizeof(b.gmco_opts), C.sizeof(b.gmco_case), C.sizeof(b.gmco_run),
                     C.sizeof(b.gmco_run_info), C.sizeof(b.gmco_plan_metrics), C.sizeof(b.gmco_tuning),
                     C.sizeof(b.gmco_select_opts)]
    assert offs == [b.gmco_plan_metrics.D90_pct.offset, b.gmco_plan_metrics.status.offset,
                    b.gmco_case.dose_rate.offset]


def test_strerror_and_null_arguments():
    b, lib = _lib()
    assert lib.gmco_strerror(0) == b"ok"
    assert lib.gmco_strerror(-1) == b"invalid argument"
    assert lib.gmco_strerror(-4) == b"call out of order"
    assert lib.gmco_destroy(None) == 0
    assert lib.gmco_create(None, None) == -1
    assert lib.gmco_set_stream(None, None) == -1
    assert lib.gmco_load_case(None, None) == -1
    assert lib.gmco_optimize(None, None, None) == -1
    assert lib.gmco_last_error(None) == b"null context"


def test_create_rejects_bad_options_before_touching_a_device():
    b, lib = _lib()
    ctx = C.c_void_p()
    for opts in (b.gmco_opts(0, 7, 10, 8), b.gmco_opts(0, 0, 0, 8), b.gmco_opts(0, 0, 33, 8),
                 b.gmco_opts(0, 0, 10, 0)):
        assert lib.gmco_create(C.byref(ctx), C.byref(opts)) == -1
        assert not ctx.value


def test_create_without_gpu_reports_no_device():
    b, lib = _lib()
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except ImportError:
        pass
    ctx = C.c_void_p()
    rc = lib.gmco_create(C.byref(ctx), C.byref(b.gmco_opts(0, 0, 10, 8)))
    assert rc == -6
    assert not ctx.value
