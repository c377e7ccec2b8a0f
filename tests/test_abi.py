"""Host-side checks of the C ABI library (no GPU calls)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "tmx.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char \*)\s*\*?\s*(tmx_\w+)\s*\(", src, re.M)))


def test_header_declares_the_boundary():
    names = declared_symbols()
    for must in ["tmx_create", "tmx_load_gauge", "tmx_load_clover", "tmx_apply_D", "tmx_apply_mhat",
                 "tmx_apply_mdagm", "tmx_solve", "tmx_multishift_solve", "tmx_pc_train"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_2212_06635_amd.tmx as tmx

    lib = ctypes.CDLL(tmx.LIB_PATH)
    missing = [n for n in declared_symbols() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_has_same_names():
    import paper_2212_06635_amd.tmx as tmx

    for n in declared_symbols():
        assert hasattr(tmx.lib, n)


def test_no_oracle_in_product_path():
    """The HIP library and its binding never load the CPU oracle."""
    pkg = os.path.join(ROOT, "paper_2212_06635_amd")
    for dp, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dp, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt and "tmx_oracle" not in txt, f


def test_force_buffers_are_checked_before_any_call():
    """The force entry points write V * 36 complex128 values through a plain
    pointer: the binding passes on only contiguous complex128 GPU tensors of
    at least the needed size, and refuses host arrays, other dtypes, short or
    strided tensors before the library is called (no GPU needed to refuse)."""
    import numpy as np
    import pytest
    import torch

    import paper_2212_06635_amd.tmx as tmx

    n = 64
    with pytest.raises(ValueError, match="torch tensor"):
        tmx.check_device_complex128(np.zeros(n, dtype=np.complex128), n, "force")
    with pytest.raises(ValueError, match="complex128"):
        tmx.check_device_complex128(torch.zeros(2 * n, dtype=torch.float64), n, "force")
    with pytest.raises(ValueError, match="complex128"):
        tmx.check_device_complex128(torch.zeros(n, dtype=torch.complex64), n, "force")
    with pytest.raises(ValueError, match="on the GPU"):
        tmx.check_device_complex128(torch.zeros(n, dtype=torch.complex128), n, "force")


def test_set_allocator_marshals_without_a_context():
    """The allocator entry point takes two C function pointers and a user
    pointer; with no context it refuses before touching anything."""
    import paper_2212_06635_amd.tmx as tmx

    a = tmx.ALLOC_FN(lambda n, u: None)
    r = tmx.RELEASE_FN(lambda p, u: None)
    assert tmx.lib.tmx_set_allocator(None, a, r, None) == tmx.TMX_EINVAL
    assert tmx.lib.tmx_set_allocator(None, tmx.NO_ALLOC, tmx.NO_RELEASE, None) == tmx.TMX_EINVAL
