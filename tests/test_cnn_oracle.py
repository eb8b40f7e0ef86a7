"""Pins of the learned-start network oracle (library routines, adjointness, finite differences)."""
import numpy as np
import pytest
from scipy import ndimage

from oracle import cnn_oracle as C
from oracle import recon_oracle as O


def test_single_channel_conv_is_periodic_correlation():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((1, 6, 7, 8))
    w = rng.standard_normal((1, 27, 1))
    ker = np.zeros((3, 3, 3))
    for t, (dx, dy, dz) in enumerate(C.TAPS):
        ker[dz + 1, dy + 1, dx + 1] = w[0, t, 0]
    ref = ndimage.correlate(x[0], ker, mode="wrap")
    np.testing.assert_allclose(C.conv(x, w, np.zeros(1))[0], ref, atol=1e-12)


def test_multichannel_conv_sums_channel_correlations():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((3, 5, 5, 5))
    w = rng.standard_normal((2, 27, 3))
    b = rng.standard_normal(2)
    out = C.conv(x, w, b)
    for o in range(2):
        ref = b[o] + sum(ndimage.correlate(x[i], np.transpose(w[o, :, i].reshape(3, 3, 3), (0, 1, 2)), mode="wrap")
                         for i in range(3))
        np.testing.assert_allclose(out[o], ref, atol=1e-11)


def test_input_gradient_is_adjoint_of_conv():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((4, 6, 6, 6))
    g = rng.standard_normal((5, 6, 6, 6))
    w = rng.standard_normal((5, 27, 4))
    lhs = np.sum(g * C.conv(x, w, np.zeros(5)))
    rhs = np.sum(C.conv_input_grad(g, w) * x)
    assert abs(lhs - rhs) < 1e-9 * abs(lhs)
    gw = C.conv_weight_grad(g, x)
    assert abs(np.sum(gw * w) - lhs) < 1e-9 * abs(lhs)


def test_loss_gradient_matches_central_differences():
    rng = np.random.default_rng(4)
    n = 6
    delta = rng.standard_normal((n, n, n)) * 0.3
    u_p = rng.standard_normal((n, n, n)) * 5
    rhat = O.line_of_sight(n, 60.0, (0, 0, 0), (31.0, 17.0, -40.0))
    target = rng.standard_normal((n, n, n))
    theta = C.init_params(5)
    theta[C.N_PARAMS - 1] = 0.3
    loss, grad = C.loss_and_grad(theta, delta, u_p, rhat, target)
    idx = rng.choice(np.flatnonzero(np.abs(grad) > 1e-6), 40, replace=False)
    h = 1e-5
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (C.loss_and_grad(tp, delta, u_p, rhat, target)[0] - C.loss_and_grad(tm, delta, u_p, rhat, target)[0]) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-6 + 1e-5 * abs(grad[i]), i


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(6)
    x = np.concatenate([rng.standard_normal(10000) * 10, [0.0, -0.0, 1.0, 1.00390625, 1.01171875, 3.4e38]])
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(C.bf16(x), ref)


def test_first_adam_step_moves_by_lr_times_sign():
    rng = np.random.default_rng(7)
    theta = rng.standard_normal(100)
    g = rng.standard_normal(100)
    g = np.where(np.abs(g) < 0.05, 0.05, g)
    new, m, v = C.adam_step(theta, np.zeros(100), np.zeros(100), g, 1, 1e-3)
    np.testing.assert_allclose(new - theta, -1e-3 * np.sign(g), rtol=1e-6)


def test_adam_steps_hand_values():
    """Pins adam_step past the first step (Kingma & Ba 2015, Algorithm 1): theta_0 = 0.5, lr = 0.01,
    gradients 0.2, -0.1, 0.4.  By hand:
      step 1: m = 0.02,   v = 4e-5,         m^ = 0.2,          v^ = 0.04
      step 2: m = 0.008,  v = 4.996e-5,     m^ = 0.008/0.19,   v^ = 4.996e-5/0.001999
      step 3: m = 0.0472, v = 2.0991004e-4, m^ = 0.0472/0.271, v^ = 2.0991004e-4/0.002997001
    and theta_t = theta_{t-1} - lr m^ / (sqrt(v^) + 1e-8)."""
    theta, m, v = np.array([0.5]), np.zeros(1), np.zeros(1)
    hand = [(0.02, 4e-5, 0.4900000005),
            (0.008, 4.996e-5, 0.4873366302718676),
            (0.0472, 2.0991004e-4, 0.4807555145179949)]
    for step, (g, (m_e, v_e, th_e)) in enumerate(zip((0.2, -0.1, 0.4), hand), start=1):
        theta, m, v = C.adam_step(theta, m, v, np.array([g]), step, 0.01)
        np.testing.assert_allclose(m, m_e, rtol=1e-12)
        np.testing.assert_allclose(v, v_e, rtol=1e-12)
        np.testing.assert_allclose(theta, th_e, rtol=1e-12)


def test_adam_constant_gradient_moves_by_lr_every_step():
    """With a constant gradient g the bias-corrected moments are exactly g and g^2 at every step, so
    each update is lr g / (|g| + eps): a wrong bias-correction power fails from step 2 on."""
    theta, m, v = np.zeros(3), np.zeros(3), np.zeros(3)
    g = np.array([0.3, -2.0, 5e-3])
    for step in range(1, 11):
        new, m, v = C.adam_step(theta, m, v, g, step, 1e-3)
        np.testing.assert_allclose(new - theta, -1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-9)
        theta = new


@pytest.mark.parametrize("cin,cout", [(8, 16), (16, 16), (16, 1)])
def test_loop_convolution_equals_array_convolution(cin, cout):
    """The C loops (conv_loops, used on 256^3 grids) compute the same periodic convolution as conv."""
    rng = np.random.default_rng(cin * 100 + cout)
    n = 12
    x = rng.standard_normal((cin, n, n, n))
    w = rng.standard_normal((cout, 27, cin))
    b = rng.standard_normal(cout)
    np.testing.assert_allclose(C.conv_loops(x, w, b), C.conv(x, w, b), rtol=0, atol=1e-12)


def test_parameter_layout():
    assert C.N_PARAMS == 16 * 27 * 8 + 16 + 16 * 27 * 16 + 16 + 27 * 16 + 1
    theta = np.arange(C.N_PARAMS, dtype=np.float64)
    np.testing.assert_array_equal(C.pack(C.unpack(theta)), theta)


def test_restriction_of_cosines_has_closed_form():
    # per axis: R cos(theta i) at node 2J = cos(2 theta J) cos^2(theta / 2)
    n = 16
    i = np.arange(n)
    kx, ky, kz = 1, 3, 5
    th = 2 * np.pi * np.array([kx, ky, kz]) / n
    f = (np.cos(th[2] * i)[:, None, None] * np.cos(th[1] * i)[None, :, None] * np.cos(th[0] * i)[None, None, :])
    j = np.arange(n // 2)
    ref = (np.cos(2 * th[2] * j)[:, None, None] * np.cos(2 * th[1] * j)[None, :, None]
           * np.cos(2 * th[0] * j)[None, None, :]) * np.prod(np.cos(th / 2) ** 2)
    np.testing.assert_allclose(C.restrict(f), ref, atol=1e-13)
    np.testing.assert_allclose(C.restrict(np.full((n, n, n), 2.5)), 2.5, atol=1e-14)


def test_prolongation_of_cosines_has_closed_form():
    # per axis: fine 2J -> cos(phi J); fine 2J+1 -> cos(phi (J + 1/2)) cos(phi / 2)
    m = 8
    j = np.arange(m)
    phi = 2 * np.pi * np.array([2, 1, 3]) / m

    def axis(p):
        out = np.empty(2 * m)
        out[0::2] = np.cos(p * j)
        out[1::2] = np.cos(p * (j + 0.5)) * np.cos(p / 2)
        return out

    c = np.cos(phi[2] * j)[:, None, None] * np.cos(phi[1] * j)[None, :, None] * np.cos(phi[0] * j)[None, None, :]
    ref = axis(phi[2])[:, None, None] * axis(phi[1])[None, :, None] * axis(phi[0])[None, None, :]
    np.testing.assert_allclose(C.prolong(c), ref, atol=1e-13)


def test_restriction_is_scaled_adjoint_of_prolongation():
    rng = np.random.default_rng(8)
    f = rng.standard_normal((12, 12, 12))
    g = rng.standard_normal((6, 6, 6))
    lhs = 8.0 * np.sum(C.restrict(f) * g)
    rhs = np.sum(f * C.prolong(g))
    assert abs(lhs - rhs) < 1e-10 * abs(rhs)


def test_prolongation_then_restriction_of_smooth_field_is_close():
    # full weighting of a linear interpolant keeps coarse nodes to second order in k h
    m = 16
    j = np.arange(m)
    c = np.sin(2 * np.pi * j / m)[None, None, :] * np.ones((m, m, 1))
    rp = C.restrict(C.prolong(c))
    assert np.max(np.abs(rp - c)) < (2 * np.pi / m) ** 2
