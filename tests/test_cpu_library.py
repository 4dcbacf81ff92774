"""Host-side checks that need no GPU: the C ABI library loads and exports every
entry point declared in include/adres.h, the ctypes parameter block has the C
layout, and the binding refuses to run without a GPU (no CPU fallback)."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_1806_10841_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "adres.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(adres_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(binding.LIB_PATH)
    names = _declared()
    assert len(names) >= 12
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # the binding wraps exactly the declared calls
    assert sorted(binding._SIGS) == names


def test_params_layout_matches_c(tmp_path):
    fields = [f[0] for f in binding.Params._fields_]
    src = tmp_path / "layout.c"
    body = "".join(f'printf("{f} %zu\\n", offsetof(adres_params, {f}));' for f in fields)
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "adres.h"\n'
                   f'int main(void){{{body} printf("size %zu\\n", sizeof(adres_params)); return 0;}}\n')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    c_off = dict(line.split() for line in out if line)
    for f in fields:
        assert int(c_off[f]) == getattr(binding.Params, f).offset, f
    assert int(c_off["size"]) == ctypes.sizeof(binding.Params)


def test_no_cpu_fallback():
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_1806_10841_amd import inputs
    with pytest.raises(RuntimeError):
        binding.Context(inputs.workload("c1"))


def test_binding_refuses_wrong_dtype_or_shape():
    """The binding checks dtype and extents before any call: a float32 position array, a
    transposed or short one, a (3, n_mol) array where frames (n_frames, 3, n_mol) are
    expected, or a histogram shorter than the bins would let the kernels read or write
    outside the allocation."""
    torch = pytest.importorskip("torch")
    chk = binding.check_tensor
    ok = torch.zeros((3, 8), dtype=torch.float64)
    chk(ok, torch.float64, (3, 8))
    with pytest.raises(TypeError):
        chk(ok.float(), torch.float64, (3, 8))
    with pytest.raises(ValueError):
        chk(torch.zeros((8, 3), dtype=torch.float64), torch.float64, (3, 8))
    with pytest.raises(ValueError):
        chk(torch.zeros((3, 7), dtype=torch.float64), torch.float64, (3, 8))
    with pytest.raises(ValueError):
        chk(ok.t(), torch.float64, (8, 3))                 # not contiguous
    with pytest.raises(ValueError):
        chk(torch.zeros((3, 8), dtype=torch.float64), torch.float64, (2, 3, 8))
    chk(torch.zeros((5, 3, 8), dtype=torch.float64), torch.float64, (5, 3, 8))
    chk(torch.zeros(14, dtype=torch.int64), torch.int64, (None,), min_numel=14)
    with pytest.raises(ValueError):
        chk(torch.zeros(13, dtype=torch.int64), torch.int64, (None,), min_numel=14)
    with pytest.raises(TypeError):
        binding._ptr(ok)                                   # a host tensor is refused outright
