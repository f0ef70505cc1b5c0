"""Host-side checks of the C-ABI library: it loads, exports every declared symbol, and its
structs have the layout the C compiler gives them. No compute call is made (no GPU here)."""
import ctypes
import os
import re
import subprocess

import pytest

from conftest import ROOT
from paper_1602_02350_amd import binding

HEADER = os.path.join(ROOT, "include", "scs.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(scs_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libscs.so not built")
    return binding.load_library()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 12
    assert set(names) == set(binding.EXPORTED)
    for n in names:
        assert getattr(lib, n) is not None


def test_struct_layout_matches_the_c_compiler(tmp_path, lib):
    src = tmp_path / "probe.c"
    src.write_text('#include "scs.h"\n#include <stdio.h>\n#include <stddef.h>\n'
                   'int main(void){printf("%zu %zu %zu %zu\\n", sizeof(scs_opts), sizeof(scs_report),'
                   ' offsetof(scs_opts, seed), offsetof(scs_report, ms_solve)); return 0;}\n')
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    assert int(out[0]) == ctypes.sizeof(binding.ScsOpts)
    assert int(out[1]) == ctypes.sizeof(binding.ScsReport)
    assert int(out[2]) == binding.ScsOpts.seed.offset
    assert int(out[3]) == binding.ScsReport.ms_solve.offset


def test_defaults_and_status_strings(lib):
    o = binding.ScsOpts()
    lib.scs_opts_default(ctypes.byref(o))
    assert (o.oversample, o.batch, o.average, o.precision) == (5, 64, 1, binding.PREC_FP32)
    for code in [0, -1, -2, -3, -4, 1, 2, 3]:
        assert lib.scs_status_string(code).decode() != "unknown status"


def test_argument_validation_needs_no_device(lib):
    """Null pointers and bad sizes are rejected on the host before any device work."""
    assert lib.scs_svrg_solve(None, None, 10, 4, 4, None, 1.0, 0, 1e-6, None, None, None) == binding.EINVAL
    o = binding.ScsOpts()
    lib.scs_opts_default(ctypes.byref(o))
    assert lib.scs_sketch_build(None, None, 10, 4, 4, 2, ctypes.byref(o), None, None, None) == binding.EINVAL


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    monkeypatch.setattr(binding, "_lib", None)
    with pytest.raises(FileNotFoundError):
        binding.load_library(str(tmp_path / "libscs.so"))
