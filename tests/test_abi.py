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

    for s in range(8):
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
