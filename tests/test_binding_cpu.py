"""The Python binding's argument checks (host side, no GPU): element extents
of BLAS-shaped operands, what a call touches (A and B not read when alpha = 0
or k = 0; C not touched on a quick return), and the rejection of host
tensors, wrong dtypes, non-contiguous views and short buffers before the
library sees a pointer.  Invalid sizes or flags are left to the library,
which reports them as info codes."""
import numpy as np
import pytest
import torch

from paper_2109_13406_amd import binding as b


def test_extents():
    # A 5x3 (ld 5), B = op^T of 4x3 (ld 4), C 5x4 (ld 5)
    assert b._gemm_extents("N", "T", 5, 4, 3, 5, 4, 5) == (15, 12, 20)
    assert b._gemm_extents(b"t", b"n", 5, 4, 3, 3, 3, 6) == (3 * 4 + 3, 3 * 3 + 3, 6 * 3 + 5)
    assert b._gemm_extents("N", "N", 5, 4, 3, 4, 3, 5) is None      # lda < m
    assert b._gemm_extents("X", "N", 5, 4, 3, 5, 3, 5) is None      # bad flag
    assert b._gemm_extents("N", "N", -1, 4, 3, 5, 3, 5) is None
    assert b._gemm_extents("N", "N", 0, 4, 3, 1, 3, 1) == (0, 3 * 3 + 3, 0)
    assert b._syrk_extents("L", "T", 4, 3, 3, 4) == (3 * 3 + 3, 4 * 3 + 4)
    assert b._syrk_extents("Q", "T", 4, 3, 3, 4) is None


def test_touches():
    ext = (1, 1, 1)
    assert b._touches(ext, False, False, 3, 5, 4) == (True, True)
    assert b._touches(ext, True, True, 3, 5, 4) == (False, False)   # quick return
    assert b._touches(ext, True, False, 3, 5, 4) == (False, True)   # C <- beta C
    assert b._touches(ext, False, True, 0, 5, 4) == (False, False)  # k = 0, beta = 1
    assert b._touches(ext, False, False, 3, 0, 4) == (0, 0)
    assert b._touches(None, False, False, 3, 5, 4) == (0, 0)


def test_device_arguments_rejected_before_the_library():
    x = torch.zeros(64, dtype=torch.float64)
    with pytest.raises(ValueError, match="CUDA"):
        b.mpdd_Rgemm(None, "N", "N", 4, 4, 4, 1.0, (x, x), 4, (x, x), 4, 0.0, (x, x), 4)
    y = torch.zeros(64, dtype=torch.float32)
    with pytest.raises(ValueError, match="dtype"):
        b._dev(y, 16, "A")
    with pytest.raises(TypeError):
        b._dev(np.zeros(16), 16, "A")
    # untouched arguments and raw pointers pass unchecked
    assert b._dev(x, 0, "A") == x.data_ptr()
    assert b._dev(12345, 10 ** 9, "A") == 12345
    assert b._dev(None, 16, "A") is None


def test_host_pairs_checked():
    a = np.zeros((4, 2))
    assert b._host_pairs(a, 4, "A") == a.ctypes.data
    with pytest.raises(ValueError, match="touches"):
        b._host_pairs(a, 5, "A")
    with pytest.raises(ValueError, match="contiguous"):
        b._host_pairs(np.zeros((4, 4))[:, ::2], 1, "A")
    with pytest.raises(ValueError, match="touches"):
        b.mpdd_Rgemm_host(None, "N", "N", 3, 3, 3, 1.0, np.zeros(16), 3, np.zeros(18), 3, 0.0,
                          np.zeros(18), 3)


def test_library_extent_helper_matches_binding(tmp_path):
    """The host-pointer calls size every copy with one C++ helper
    (csrc/extent.hpp); it must give the same extents as the binding's check,
    ld*(cols-1) + rows, and 0 for an empty matrix."""
    import os
    import subprocess
    cases = [(5, 5, 3), (8195, 8192, 8192), (7, 3, 1), (4, 0, 5), (4, 3, 0), (1, 1, 1),
             (1100, 1000, 137)]
    src = tmp_path / "extent_main.cpp"
    inc = os.path.join(os.path.dirname(b.__file__), "csrc")
    body = "".join(f'  std::printf("%zu\\n", mpdd::blas_extent({ld}, {r}, {c}));\n'
                   for ld, r, c in cases)
    src.write_text('#include <cstdio>\n#include "extent.hpp"\nint main() {\n' + body + "}\n")
    exe = tmp_path / "extent_main"
    subprocess.run(["g++", "-std=c++17", "-I", inc, str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    assert got == [b._extent(r, c, ld) for ld, r, c in cases]
