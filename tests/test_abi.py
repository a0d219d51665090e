"""CPU-only checks of the C ABI: the library loads, exports every function the
header declares, validates arguments before touching the GPU, and its structures
match the binding's layouts.  No compute call needs a GPU here."""
import ctypes
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pauliwht.h")

pw = pytest.importorskip("paper_2601_00761_amd")


def declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"PW_API\s+[\w\s\*]+?\b(pw_\w+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    names = declared()
    assert len(names) >= 30
    lib = ctypes.CDLL(pw.lib_path())
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", pw.lib_path()], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (pw_\w+)", out))
    assert set(names) <= exported
    # nothing but the C ABI is exported
    assert exported == set(names), sorted(exported - set(names))


def test_struct_layouts_match_binding(tmp_path):
    # compile the header with the host C compiler and compare sizes and offsets
    prog = tmp_path / "layout.c"
    prog.write_text("""
#include <stdio.h>
#include <stddef.h>
#include "pauliwht.h"
int main(void) {
  printf("%zu %zu %zu %zu\\n", sizeof(pw_xres), sizeof(pw_result), sizeof(pw_mixed_result), sizeof(pw_state_ref));
  printf("%zu %zu %zu %zu\\n", offsetof(pw_xres, nu), offsetof(pw_result, nu_cnt), offsetof(pw_result, gap),
         offsetof(pw_mixed_result, families));
  return 0;
}
""")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-I" + os.path.join(ROOT, "include"), str(prog), "-o", str(exe)])
    a, b = subprocess.check_output([str(exe)], text=True).split("\n")[:2]
    sizes = [int(v) for v in a.split()]
    offs = [int(v) for v in b.split()]
    assert sizes == [ctypes.sizeof(pw.pw_xres), ctypes.sizeof(pw.pw_result), ctypes.sizeof(pw.pw_mixed_result),
                     ctypes.sizeof(pw.pw_state_ref)]
    assert offs == [pw.pw_xres.nu.offset, pw.pw_result.nu_cnt.offset, pw.pw_result.gap.offset,
                    pw.pw_mixed_result.families.offset]
    assert pw.XRES_DTYPE.itemsize == sizes[0] == 64


def test_version_and_argument_validation_without_gpu():
    assert "gfx950" in pw.pw_version()
    with pytest.raises(pw.PWError) as e:
        pw.pw_workspace_size(0, pw.PW_C64, 1)
    assert e.value.status == 2 and "outside" in str(e.value)
    with pytest.raises(pw.PWError) as e:
        pw.pw_workspace_size(20, 7, 1)
    assert e.value.status == 1
    with pytest.raises(pw.PWError) as e:
        pw.pw_workspace_size(20, pw.PW_C64, 0)
    assert e.value.status == 2
    assert pw.pw_workspace_size(20, pw.PW_C64, 64) > 64 * (1 << 19) * 8
    assert pw.pw_made_param_count(30, 256) == 30 * 256 + 256 + 256 * 256 + 256 + 256 * 30 + 30 + 900
    with pytest.raises(pw.PWError) as e:
        pw.pw_made_param_count(1, 256)
    assert e.value.status == 2
    with pytest.raises(pw.PWError) as e:
        pw.pw_made_param_count(10, 100)
    assert e.value.status == 8


def test_null_context_is_rejected_before_any_hip_call():
    L = pw._L
    assert L.pw_ctx_destroy(None) == 1
    assert L.pw_exact(None, 1e-7, None) == 1
    assert L.pw_set_moments(None, 2) == 1
    assert L.pw_timing_enable(None, 1) == 1
    assert "null context" in pw.pw_last_error()


def test_no_gpu_reports_hip_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(pw.PWError) as e:
        pw.pw_ctx_create(0)
    assert e.value.status == 6


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True)
    assert r.returncode == 2 and "one GPU" in r.stderr
