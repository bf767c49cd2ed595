"""C-ABI contract checks that need no GPU: the library loads, every entry
point declared in include/gevp.h is exported, and the host-side helpers
(status strings, block size, option defaults) behave as documented."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gevp.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gevp_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_1007_4400_amd import gevp

    lib = gevp.load()
    names = _declared()
    assert "gevp_solve" in names and "gevp_backward" in names and "gevp_create" in names
    for name in names:
        assert hasattr(lib, name), name


def test_status_strings():
    from paper_1007_4400_amd import gevp

    for s in range(9):
        assert gevp.status_string(s)
    assert "positive definite" in gevp.status_string(gevp.GEVP_ERR_NOT_HPD)


def test_block_size_defaults():
    from paper_1007_4400_amd import gevp

    lib = gevp.load()
    o = gevp.make_opts()
    # nex = max(16, ceil(0.15 nev)) rounded up to a multiple of 16, capped at n
    assert lib.gevp_block_size(ctypes.byref(o), 8192, 820) == 820 + 128
    assert lib.gevp_block_size(ctypes.byref(o), 256, 16) == 32
    assert lib.gevp_block_size(ctypes.byref(o), 20, 16) == 20
    assert lib.gevp_block_size(ctypes.byref(o), 20, 0) == 0
    o.nex = 40
    assert lib.gevp_block_size(ctypes.byref(o), 1000, 100) == 140


def test_create_without_gpu_fails_cleanly():
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_1007_4400_amd import gevp

    with pytest.raises(gevp.GevpError):
        gevp.Handle(0)


def test_workspace_size_query_needs_no_gpu():
    from paper_1007_4400_amd import gevp

    skw = 6 * 128 * 2 ** 20  # six fixed split-K slots
    b8192 = gevp.workspace_size(8192, 820, gevp.make_opts(precision="bf16x3"))
    # at least A, B copies, L and C (4 n^2 complex128) and the split-BF16 copy of C
    assert b8192 >= 4 * 16 * 8192 ** 2 + 8 * 8192 ** 2 + skw
    assert b8192 < 6 * 16 * 8192 ** 2 + skw
    assert gevp.workspace_size(256, 16) < gevp.workspace_size(512, 16) < b8192
    # a low-precision filter needs its copies on top of the FP64 workspace
    assert gevp.workspace_size(2048, 205, gevp.make_opts(precision="fp32")) > \
        gevp.workspace_size(2048, 205)
    with pytest.raises(gevp.GevpError):
        gevp.workspace_size(10, 11)
