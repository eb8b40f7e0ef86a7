"""The ctypes binding rejects bad buffers before any call reaches the library (CPU only).

A plan object is built without a workspace and pointed at torch's "meta" device, with a stub in
place of the loaded library that fails the test if any C entry point is reached: every wrong
dtype, size or device must raise TypeError / ValueError in the binding itself.
"""
import pytest
import torch

from paper_1504_02591_amd import native


class _NoCalls:
    def __getattr__(self, name):
        raise AssertionError(f"C entry point {name} was reached")


def _plan(n=8, batch=1, max_objects=100, cnn_half=False):
    p = object.__new__(native.Plan)
    p.lib = _NoCalls()
    p.handle = None
    p.device = torch.device("meta")
    p.n, p.batch, p.randoms = n, batch, True
    p.cnn_n = n // 2 if cnn_half else n
    p.params = native.Params()
    p.params.max_objects = max_objects
    p._painted = None
    return p


def meta(*shape, dtype=torch.float32):
    return torch.empty(shape, dtype=dtype, device="meta")


def test_shift_checks_offsets_and_outputs():
    p = _plan(batch=2)
    pos = meta(10, 3)
    with pytest.raises(ValueError):
        p.shift(native.GAL, pos)                                   # batch 2 needs offsets
    with pytest.raises(TypeError):
        p.shift(native.GAL, pos, offsets=meta(3, dtype=torch.int32))
    with pytest.raises(ValueError):
        p.shift(native.GAL, pos, offsets=meta(4, dtype=torch.int64))
    with pytest.raises(ValueError):
        p.shift(native.GAL, pos, offsets=torch.zeros(3, dtype=torch.int64))   # host tensor
    off = meta(3, dtype=torch.int64)
    with pytest.raises(TypeError):
        p.shift(native.GAL, pos, offsets=off, want_pos=True, out_pos=meta(10, 3, dtype=torch.float64))
    with pytest.raises(ValueError):
        p.shift(native.GAL, pos, offsets=off, want_pos=True, out_pos=torch.zeros(10, 3))
    with pytest.raises(ValueError):
        p.shift(native.GAL, pos, offsets=off, want_pos=True, out_pos=meta(9, 3))
    with pytest.raises(ValueError):
        p.shift(native.GAL, pos, offsets=off, out_disp=meta(11, 3))
    with pytest.raises(ValueError):
        p.shift(5, pos, offsets=off)


def test_paint_checks():
    p = _plan(batch=2)
    pos = meta(10, 3)
    with pytest.raises(ValueError):
        p.paint(native.GAL, pos)
    with pytest.raises(ValueError):
        p.paint(native.GAL, pos, offsets=meta(2, dtype=torch.int64))
    with pytest.raises(ValueError):
        p.paint(7, pos, offsets=meta(3, dtype=torch.int64))
    with pytest.raises(TypeError):
        p.paint(native.GAL, meta(10, 3, dtype=torch.float16), offsets=meta(3, dtype=torch.int64))
    with pytest.raises(ValueError):
        p.paint(native.GAL, pos, w=meta(9), offsets=meta(3, dtype=torch.int64))


def test_solve_checks_network_parameters():
    p = _plan()
    with pytest.raises(ValueError):
        p.solve(native.START_LEARNED, meta(native.CNN_PARAMS - 1))
    with pytest.raises(TypeError):
        p.solve(native.START_LEARNED, meta(native.CNN_PARAMS, dtype=torch.bfloat16))
    with pytest.raises(ValueError):
        p.solve(native.START_LEARNED, torch.zeros(native.CNN_PARAMS))
    with pytest.raises(TypeError):
        p.solve(native.START_LEARNED, [0.0] * native.CNN_PARAMS)


def test_train_step_checks_moments_and_gradient():
    p = _plan()
    th = meta(native.CNN_PARAMS)
    f = meta(1, 8, 8, 8)
    good = meta(native.CNN_PARAMS)
    with pytest.raises(ValueError):
        p.cnn_train_step(th, None, good, 1, 1e-3, f, f, f)          # Adam without m
    with pytest.raises(ValueError):
        p.cnn_train_step(th, meta(10), good, 1, 1e-3, f, f, f)
    with pytest.raises(TypeError):
        p.cnn_train_step(th, good, meta(native.CNN_PARAMS, dtype=torch.float64), 1, 1e-3, f, f, f)
    with pytest.raises(ValueError):
        p.cnn_train_step(th, good, torch.zeros(native.CNN_PARAMS), 1, 1e-3, f, f, f)
    with pytest.raises(ValueError):
        p.cnn_train_step(th, None, None, 0, 0.0, f, f, f, grad_out=meta(5))
    with pytest.raises(TypeError):
        p.cnn_train_step(th, None, None, 0, 0.0, f, f, f, grad_out=meta(native.CNN_PARAMS, dtype=torch.int32))


def test_brick_order_shift_only_for_the_unchanged_painted_tensor():
    p = _plan()
    pos = torch.zeros(10, 3)
    off = None
    p._painted = (native.RAN, pos, pos._version, off, None)
    assert p._as_painted(native.RAN, pos, None)
    assert not p._as_painted(native.GAL, pos, None)                 # other catalogue kind
    assert not p._as_painted(native.RAN, pos.clone(), None)         # equal contents, other tensor
    assert not p._as_painted(native.RAN, pos, torch.zeros(2, dtype=torch.int64))
    pos.add_(1.0)                                                    # changed in place since the paint
    assert not p._as_painted(native.RAN, pos, None)
