"""The C-ABI library loads and exports every symbol the public header declares (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "recon.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(recon_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1504_02591_amd import native
    if not os.path.exists(native.lib_path()):
        pytest.fail("librecon.so is not built; run __graft_entry__.build()")
    return native.load()


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("recon_plan", "recon_paint", "recon_solve", "recon_iterate", "recon_shift"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), f"{name} declared in recon.h but not exported"


def test_binding_covers_every_declared_symbol():
    from paper_1504_02591_amd import native
    assert set(declared_functions()) <= set(native.EXPORTED)


def test_workspace_size_validates_parameters(lib):
    from paper_1504_02591_amd import native
    p = native.Params()
    p.n, p.batch, p.box_len = 64, 1, 1000.0
    p.bias, p.growth, p.smooth_r, p.mask_tau = 1.0, 0.7, 10.0, 0.1
    good = lib.recon_workspace_bytes(ctypes.byref(p))
    n3, cn = 64 ** 3, 33 * 64 * 64
    assert good >= 2 * n3 * 8 + 5 * cn * 8 + 3 * n3 * 4
    for field, bad in (("n", 48), ("n", 2048), ("batch", 0), ("box_len", -1.0), ("bias", 0.0),
                       ("growth", -0.1), ("smooth_r", float("nan"))):
        q = native.Params()
        ctypes.pointer(q)[0] = p
        setattr(q, field, bad)
        assert lib.recon_workspace_bytes(ctypes.byref(q)) == 0, field
    q = native.Params()
    ctypes.pointer(q)[0] = p
    q.flags = native.NO_RANDOMS
    assert 0 < lib.recon_workspace_bytes(ctypes.byref(q)) < good


def test_error_strings(lib):
    for code in (0, 1, -1, -2, -3, -4, -5):
        assert lib.recon_strerror(code)
    assert lib.recon_plan(None, None, None, 0, None) == -1
