"""Pins of the oracle's learned-preconditioner network: the convolution against
scipy's correlate2d, GELU against its erf definition and known values, the
hand-written gradient against central differences, the transposed convolution
by the adjoint identity, and the first Adam step."""
import math

import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import net as N
from paper_2007_10411_amd import inputs as I


def test_param_layout_matches_input_generator():
    nf = 4
    th = I.net_init_params(nf, seed=3)
    assert th.size == N.param_count(nf) == 4 * 16 * 9 + 16 * 16 * 9 * 2 + 16 * 4 * 9 + 16 * 3 + 4
    layers = N.unpack(th, nf)
    assert np.array_equal(N.pack(layers), th)
    assert [W.shape for W, _ in layers] == [s[0] for s in I.net_layer_shapes(nf)]


@pytest.mark.parametrize("d", [1, 2, 3])
def test_conv_equals_scipy_correlate_with_zero_padding(d):
    """A dilated 3x3 kernel is the (2d+1) x (2d+1) kernel with zeros between taps."""
    rng = np.random.Generator(np.random.PCG64(1))
    x = rng.normal(size=(3, 9, 11))
    W = rng.normal(size=(5, 3, 3, 3))
    b = rng.normal(size=5)
    out = N.conv(x, W, b, d)
    for co in range(5):
        ref = b[co]
        for ci in range(3):
            Kd = np.zeros((2 * d + 1, 2 * d + 1))
            Kd[::d, ::d] = W[co, ci]
            ref = ref + correlate2d(x[ci], Kd, mode="same", boundary="fill", fillvalue=0.0)
        assert np.allclose(out[co], ref, rtol=1e-13, atol=1e-13)


def test_gelu_definition_and_values():
    xs = np.linspace(-6, 6, 101)
    ref = np.array([0.5 * x * (1 + math.erf(x / math.sqrt(2))) for x in xs])
    assert np.allclose(N.gelu(xs), ref, rtol=1e-15, atol=1e-300)
    assert abs(N.gelu(np.array(1.0)) - 0.8413447460685429) < 1e-15       # Phi(1)
    assert np.allclose(N.gelu(xs) - N.gelu(-xs), xs, atol=1e-15)          # x Phi(x) - (-x) Phi(-x) = x
    h = 1e-6
    fd = (N.gelu(xs + h) - N.gelu(xs - h)) / (2 * h)
    assert np.allclose(N.gelu_grad(xs), fd, atol=1e-8)


@pytest.mark.parametrize("d", [1, 4])
def test_transposed_convolution_is_the_adjoint(d):
    rng = np.random.Generator(np.random.PCG64(2))
    x = rng.normal(size=(4, 6, 11))
    W = rng.normal(size=(16, 4, 3, 3))
    g = rng.normal(size=(16, 6, 11))
    lhs = float(np.sum(g * (N.conv(x, W, np.zeros(16), d))))
    rhs = float(np.sum(N.conv_grad_input(g, W, x.shape, d) * x))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    gW, gb = N.conv_grad_weight(g, x, d)
    # <g, conv_W(x)> is linear in W: its gradient is gW
    dW = rng.normal(size=W.shape)
    assert abs(float(np.sum(g * N.conv(x, dW, np.zeros(16), d))) - float(np.sum(gW * dW))) <= 1e-12 * abs(lhs)


def _pairs(nf=4, nz=5, nx=6, B=2, seed=4):
    rng = np.random.Generator(np.random.PCG64(seed))
    R = [rng.normal(size=(nf, nz, 1, nx)) * np.array([1.0, 0.5, 1e-3, 2.0])[:, None, None, None] for _ in range(B)]
    DU = [rng.normal(size=(nf, nz, 1, nx)) for _ in range(B)]
    return R, DU


@pytest.mark.parametrize("dils", [(1, 1, 1, 1), (1, 2, 3, 1)])
def test_loss_gradient_matches_central_differences(dils):
    nf, dt = 4, 2.0
    th = I.net_init_params(nf, seed=5, out_scale=1.0)
    th = th + np.random.Generator(np.random.PCG64(6)).normal(scale=0.05, size=th.size)   # nonzero biases
    R, DU = _pairs()
    loss, g = N.loss_and_grad(th, R, DU, dt, dils)
    rng = np.random.Generator(np.random.PCG64(7))
    idx = rng.choice(th.size, size=60, replace=False)
    for k in idx:
        h = 1e-6 * max(1.0, abs(th[k]))
        tp, tm = th.copy(), th.copy()
        tp[k] += h
        tm[k] -= h
        fd = (N.loss_and_grad(tp, R, DU, dt, dils)[0] - N.loss_and_grad(tm, R, DU, dt, dils)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(abs(g).max(), 1e-12) + 1e-7 * abs(g[k]), (k, fd, g[k])


def test_forward_reduces_to_diagonal_guess_with_zero_network():
    nf, dt = 4, 2.0
    th = np.zeros(N.param_count(nf))
    R, _ = _pairs()
    z = N.forward(th, R[0], dt)
    assert np.allclose(z, 0.5 * dt * R[0], rtol=0, atol=0)


def test_field_scale_is_the_global_rms():
    r = np.zeros((4, 3, 1, 5))
    r[0] = 2.0
    s = N.field_scale(r[:, :, 0, :])
    assert np.allclose(s, 1.0)                 # sqrt(mean) = sqrt(4 / 4)
    assert np.all(N.field_scale(np.zeros((4, 3, 5))) == 1.0)
    # positively homogeneous: z(a r) = a z(r)
    th = I.net_init_params(4, seed=2, out_scale=1.0)
    rr = np.random.Generator(np.random.PCG64(3)).normal(size=(4, 5, 1, 6))
    assert np.allclose(N.forward(th, 3.0 * rr, 2.0), 3.0 * N.forward(th, rr, 2.0), rtol=1e-12)


def test_first_adam_step_is_lr_times_sign():
    rng = np.random.Generator(np.random.PCG64(8))
    th = rng.normal(size=50)
    g = rng.normal(size=50)
    new, m, v = N.adam_step(th, g, np.zeros(50), np.zeros(50), 1, 1e-3)
    assert np.allclose(th - new, 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12)


# ---- 3D network (3 x 3 x 3 kernels) ---------------------------------------- #
def test_param_layout_3d():
    nf = 5
    th = I.net_init_params(nf, seed=3, dim=3)
    assert th.size == N.param_count(nf, 3) == (5 * 16 + 16 * 16 * 2 + 16 * 5) * 27 + 16 * 3 + 5
    assert [W.shape for W, _ in N.unpack(th, nf, 3)] == [s[0] for s in I.net_layer_shapes(nf, 3)]


def test_conv3d_equals_scipy_correlate_with_zero_padding():
    from scipy.signal import correlate
    rng = np.random.Generator(np.random.PCG64(21))
    x = rng.normal(size=(3, 5, 6, 7))
    W = rng.normal(size=(4, 3, 3, 3, 3))
    b = rng.normal(size=4)
    out = N.conv(x, W, b)
    for co in range(4):
        ref = b[co] + sum(correlate(x[ci], W[co, ci], mode="same") for ci in range(3))
        assert np.allclose(out[co], ref, rtol=1e-13, atol=1e-13)


def test_conv3d_transpose_adjoint_identity():
    rng = np.random.Generator(np.random.PCG64(22))
    x = rng.normal(size=(3, 4, 5, 6))
    W = rng.normal(size=(2, 3, 3, 3, 3))
    g = rng.normal(size=(2, 4, 5, 6))
    lhs = float(np.sum(N.conv(x, W, np.zeros(2)) * g))
    rhs = float(np.sum(x * N.conv_grad_input(g, W, x.shape)))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_loss_gradient_3d_matches_central_differences():
    from paper_2007_10411_amd.inputs import thermal_neutral_3d
    prob = thermal_neutral_3d(6, 5, 4)
    nf = prob.nf
    rng = np.random.Generator(np.random.PCG64(23))
    th = I.net_init_params(nf, seed=4, out_scale=1.0, dim=3) + rng.normal(scale=0.05, size=N.param_count(nf, 3))
    R = [rng.normal(size=prob.shape)]
    DU = [rng.normal(size=prob.shape)]
    lo, go = N.loss_and_grad(th, R, DU, prob.dt)
    o = 0
    for ws, bs in N.param_shapes(nf, 3):          # one weight and one bias of every layer
        nw = int(np.prod(ws))
        for idx in (o + int(rng.integers(nw)), o + nw + int(rng.integers(bs[0]))):
            h = 1e-6
            tp, tm = th.copy(), th.copy()
            tp[idx] += h
            tm[idx] -= h
            fd = (N.loss_and_grad(tp, R, DU, prob.dt)[0] - N.loss_and_grad(tm, R, DU, prob.dt)[0]) / (2 * h)
            assert abs(fd - go[idx]) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(go).max()), (idx, fd, go[idx])
        o += nw + bs[0]
