"""FP64 oracle of the learned-start network -- test infrastructure only.

The learned start is not part of the paper: it replaces the radial part of the
starting displacement (the quantity the FFTA starts of eq. (approx1) and
eq. (approx2) approximate) by the output of a small periodic 3D CNN, after
which the iteration of Sec. 5.1 runs unchanged.  This module defines that
network plainly so the GPU kernels can be checked against it.

Network (all convolutions periodic, cross-correlation, taps t = (dz+1)*9 + (dy+1)*3 + (dx+1)):
  x0 = [delta_s, S_U u_p, r_x, r_y, r_z, 0, 0, 0]           (8 channels per cell)
  a1 = relu(conv(x0; W1 [16][27][8],  b1 [16]))
  a2 = relu(conv(a1; W2 [16][27][16], b2 [16]))
  y  =      conv(a2; W3 [1][27][16],  b3 [1])
  Delta u = y / S_U,   Psi_0 = Psi_p + Delta u r_hat
Training loss: L = mean_p (y - S_U Delta u*)^2.
Parameter vector (float32 on the device): W1, b1, W2, b2, W3, b3 in that order.

The network may also run on the (n/2)^3 grid (restrict, forward, prolong): coarse
nodes are every other fine node, r_hat is taken at the coarse nodes.

bf16=True rounds x0, the weights, a1 and a2 to bfloat16 (round to nearest even)
where the GPU stores them in bfloat16; sums stay in float64.  Parity unpinned
against the paper (the paper has no network); pinned here against
scipy.ndimage.correlate and central finite differences.

conv() writes the convolution with array shifts; conv_loops() computes the same
definition with plain C loops (oracle/cnn_conv.c, built by the repository's build
step) for grids where the array form is too slow (256^3), and is pinned to conv().
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

S_U = 0.1
C_IN, C_HID = 8, 16
SHAPES = [("W1", (C_HID, 27, C_IN)), ("b1", (C_HID,)), ("W2", (C_HID, 27, C_HID)), ("b2", (C_HID,)),
          ("W3", (1, 27, C_HID)), ("b3", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)
TAPS = [(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    out, off = {}, 0
    for name, shp in SHAPES:
        size = int(np.prod(shp))
        out[name] = theta[off:off + size].reshape(shp)
        off += size
    return out


def pack(p):
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def init_params(seed):
    """He-style initial weights; the radial channel of the last layer starts near the FFTA-2 map."""
    rng = np.random.default_rng(seed)
    p = {}
    p["W1"] = rng.standard_normal((C_HID, 27, C_IN)) * np.sqrt(2.0 / (27 * 5))
    p["W1"][:, :, 5:] = 0.0
    p["b1"] = np.zeros(C_HID)
    p["W2"] = rng.standard_normal((C_HID, 27, C_HID)) * np.sqrt(2.0 / (27 * C_HID))
    p["b2"] = np.zeros(C_HID)
    p["W3"] = rng.standard_normal((1, 27, C_HID)) * np.sqrt(1.0 / (27 * C_HID))
    p["b3"] = np.zeros(1)
    return pack(p)


def bf16(x):
    """Round float64 values to bfloat16 (round to nearest, ties to even), returned as float64.

    On the float32 bit pattern u: add 0x7FFF plus the lowest kept bit, clear the 16 dropped bits
    (uint32 arithmetic, in place)."""
    u = np.array(x, dtype=np.float32).view(np.uint32)
    lsb = u >> 16
    lsb &= 1
    u += np.uint32(0x7FFF)
    u += lsb
    del lsb
    u &= np.uint32(0xFFFF0000)
    return u.view(np.float32).astype(np.float64)


def shift(f, d):
    """g(p) = f(p + d) on the periodic grid (arrays [..., z, y, x])."""
    dx, dy, dz = d
    return np.roll(f, shift=(-dz, -dy, -dx), axis=(-3, -2, -1))


def conv(x, w, b):
    """out[o](p) = b[o] + sum_t sum_i w[o, t, i] x[i](p + d_t); x [C_in, n, n, n]."""
    out = np.zeros((w.shape[0],) + x.shape[1:])
    for t, d in enumerate(TAPS):
        xs = shift(x, d)
        out += np.einsum("oi,izyx->ozyx", w[:, t, :], xs)
    return out + b.reshape(-1, 1, 1, 1)


_CONV_LIB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libcnn_conv.so")
_conv_handle = None


def _conv_lib():
    global _conv_handle
    if _conv_handle is None:
        if not os.path.exists(_CONV_LIB):
            raise RuntimeError(f"{_CONV_LIB} is missing; build it with __graft_entry__.build()")
        lib = ctypes.CDLL(_CONV_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.conv3_periodic.argtypes = [dp, ctypes.c_int, ctypes.c_int, dp, dp, ctypes.c_int, dp]
        lib.conv3_periodic.restype = ctypes.c_int
        _conv_handle = lib
    return _conv_handle


def conv_loops(x, w, b):
    """conv(x, w, b) by plain FP64 loops in C (same definition; channels moved last for the loops)."""
    cout, _, cin = w.shape
    n = x.shape[-1]
    if x.shape != (cin, n, n, n) or cout > 64:
        raise ValueError("conv_loops: x must be [C_in, n, n, n] and C_out <= 64")
    xl = np.ascontiguousarray(np.moveaxis(np.asarray(x, dtype=np.float64), 0, -1))
    wl = np.ascontiguousarray(w, dtype=np.float64)
    bl = np.ascontiguousarray(b, dtype=np.float64)
    out = np.empty((n, n, n, cout))
    dp = ctypes.POINTER(ctypes.c_double)
    rc = _conv_lib().conv3_periodic(xl.ctypes.data_as(dp), cin, n, wl.ctypes.data_as(dp), bl.ctypes.data_as(dp),
                                    cout, out.ctypes.data_as(dp))
    if rc != 0:
        raise RuntimeError("conv_loops failed")
    return np.ascontiguousarray(np.moveaxis(out, -1, 0))


def conv_input_grad(g, w):
    """Gradient of sum(g * conv(x)) with respect to x: sum_t w[o,t,i] g[o](p - d_t)."""
    out = np.zeros((w.shape[2],) + g.shape[1:])
    for t, d in enumerate(TAPS):
        gs = shift(g, tuple(-v for v in d))
        out += np.einsum("oi,ozyx->izyx", w[:, t, :], gs)
    return out


def conv_weight_grad(g, x):
    """Gradient of sum(g * conv(x)) with respect to w[o,t,i]: sum_p g[o](p) x[i](p + d_t)."""
    return np.stack([np.einsum("ozyx,izyx->oi", g, shift(x, d)) for d in TAPS], axis=1)


def inputs(delta, u_p, rhat):
    z = np.zeros_like(delta)
    return np.stack([delta, S_U * u_p, rhat[0], rhat[1], rhat[2], z, z, z])


def forward(theta, delta, u_p, rhat, bf16_mode=False, conv_fn=conv):
    """Returns (y, cache); y is the scaled correction S_U * Delta u on the grid."""
    p = unpack(theta)
    q = (lambda a: bf16(a)) if bf16_mode else (lambda a: a)
    x0 = q(inputs(delta, u_p, rhat))
    a1 = q(np.maximum(conv_fn(x0, q(p["W1"]), p["b1"]), 0.0))
    a2 = q(np.maximum(conv_fn(a1, q(p["W2"]), p["b2"]), 0.0))
    y = conv_fn(a2, q(p["W3"]), p["b3"])[0]
    return y, dict(x0=x0, a1=a1, a2=a2, p=p, q=q)


def loss_and_grad(theta, delta, u_p, rhat, target_du, bf16_mode=False):
    """Mean-squared loss against S_U * target and its gradient with respect to theta."""
    y, c = forward(theta, delta, u_p, rhat, bf16_mode)
    p, q = c["p"], c["q"]
    n = y.size
    r = y - S_U * target_du
    loss = float(np.sum(r * r) / n)
    dy = (2.0 / n) * r[None]
    g = {"W3": conv_weight_grad(dy, c["a2"]), "b3": dy.sum(axis=(1, 2, 3))}
    d2 = conv_input_grad(dy, q(p["W3"])) * (c["a2"] > 0)
    d2 = q(d2)
    g["W2"] = conv_weight_grad(d2, c["a1"])
    g["b2"] = d2.sum(axis=(1, 2, 3))
    d1 = conv_input_grad(d2, q(p["W2"])) * (c["a1"] > 0)
    d1 = q(d1)
    g["W1"] = conv_weight_grad(d1, c["x0"])
    g["b1"] = d1.sum(axis=(1, 2, 3))
    return loss, pack(g)


def restrict(f):
    """Full-weighting restriction of a periodic node field [..., n, n, n] to [..., n/2, n/2, n/2].

    Coarse node J sits on fine node 2J; per axis the weights are 1/4, 1/2, 1/4 on
    fine nodes 2J-1, 2J, 2J+1 (the standard multigrid restriction, exact on linear
    functions and the adjoint of linear prolongation up to the factor 2^-3).
    """
    g = np.asarray(f, dtype=np.float64)
    for ax in (-3, -2, -1):
        g = 0.25 * np.roll(g, 1, axis=ax) + 0.5 * g + 0.25 * np.roll(g, -1, axis=ax)
    return g[..., ::2, ::2, ::2]


def prolong(c):
    """Linear prolongation of a periodic node field [..., m, m, m] to [..., 2m, 2m, 2m].

    Fine node 2J copies coarse node J; fine node 2J+1 takes the mean of coarse nodes J and J+1,
    axis by axis (trilinear interpolation between coarse nodes).
    """
    g = np.asarray(c, dtype=np.float64)
    for ax in (-3, -2, -1):
        mid = 0.5 * (g + np.roll(g, -1, axis=ax))
        shape = list(g.shape)
        shape[ax] *= 2
        out = np.empty(shape)
        sl_even = [slice(None)] * g.ndim
        sl_odd = [slice(None)] * g.ndim
        sl_even[ax] = slice(0, None, 2)
        sl_odd[ax] = slice(1, None, 2)
        out[tuple(sl_even)] = g
        out[tuple(sl_odd)] = mid
        g = out
    return g


def half_grid_correction(theta, delta, u_p, rhat_coarse, bf16_mode=False, conv_fn=conv):
    """Delta u on the fine grid when the network runs on the (n/2)^3 grid (one level)."""
    return coarse_grid_correction(theta, delta, u_p, rhat_coarse, 1, bf16_mode, conv_fn)


def coarse_grid_correction(theta, delta, u_p, rhat_coarse, levels, bf16_mode=False, conv_fn=conv):
    """Delta u on the fine grid when the network runs on the (n/2^levels)^3 grid: restrict delta_s and
    u_p levels times, evaluate the network there (r_hat of the coarse nodes), prolong y / S_U levels
    times."""
    d, u = delta, u_p
    for _ in range(levels):
        d, u = restrict(d), restrict(u)
    y, _ = forward(theta, d, u, rhat_coarse, bf16_mode, conv_fn)
    out = y / S_U
    for _ in range(levels):
        out = prolong(out)
    return out


def adam_step(theta, m, v, grad, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015) with bias correction; step counts from 1."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
