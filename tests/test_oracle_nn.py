"""Pins of the oracle of the learned-preconditioner network (CPU only).

* 3D convolution (stride 1 and 2, zero padding) against a direct sum written
  with numpy slicing, independent of the C loops;
* adjoint identities: <conv(x), g> = <x, conv_data^T(g)> = <w, grad_w>, and
  the bias gradient is the sum of g;
* linear upsampling reproduces linear fields and its adjoint satisfies
  <up(c), f> = <c, up^T(f)>;
* the full backward pass against central finite differences of the loss;
* Adam: the closed-form first step lr g / (|g| + eps), constant-gradient
  steps, and a second step computed by hand.
"""
import numpy as np
import pytest

import oracle
from oracle import nnet

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def direct_conv(x, w, b, s):
    """x [Ci][Z][Y][X], w [Co][Ci][3][3][3] -> [Co][Zo][Yo][Xo] by explicit taps."""
    Ci, Z, Y, X = x.shape
    Co = w.shape[0]
    xp = np.zeros((Ci, Z + 2, Y + 2, X + 2))
    xp[:, 1:-1, 1:-1, 1:-1] = x
    Zo, Yo, Xo = (Z - 1) // s + 1, (Y - 1) // s + 1, (X - 1) // s + 1
    y = np.zeros((Co, Zo, Yo, Xo)) + b[:, None, None, None]
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                patch = xp[:, dz:dz + s * (Zo - 1) + 1:s, dy:dy + s * (Yo - 1) + 1:s, dx:dx + s * (Xo - 1) + 1:s]
                y += np.tensordot(w[:, :, dz, dy, dx], patch, axes=(1, 0))
    return y


@pytest.mark.parametrize("s,dims", [(1, (5, 4, 6)), (2, (5, 4, 6)), (2, (7, 6, 3))])
def test_conv_matches_direct_sum(s, dims):
    rng = np.random.default_rng(11)
    x = rng.standard_normal((3,) + dims)
    w = rng.standard_normal((2, 3, 3, 3, 3))
    b = rng.standard_normal(2)
    y = oracle.conv3d_fwd(x[None], w, b, stride=s)[0]
    np.testing.assert_allclose(y, direct_conv(x, w, b, s), rtol=1e-13, atol=1e-12)


@pytest.mark.parametrize("s", [1, 2])
def test_conv_adjoint_identities(s):
    rng = np.random.default_rng(12)
    x = rng.standard_normal((1, 4, 7, 5, 6))
    w = rng.standard_normal((3, 4, 3, 3, 3))
    y = oracle.conv3d_fwd(x, w, None, stride=s)
    g = rng.standard_normal(y.shape)
    lhs = float((y * g).sum())
    gx = oracle.conv3d_bwd_data(g, w, x.shape, stride=s)
    gw, gb = oracle.conv3d_bwd_weight(x, g, 3, stride=s)
    assert abs(lhs - float((x * gx).sum())) <= 1e-11 * abs(lhs) + 1e-10
    assert abs(lhs - float((w * gw).sum())) <= 1e-11 * abs(lhs) + 1e-10
    np.testing.assert_allclose(gb, g.sum(axis=(0, 2, 3, 4)), rtol=1e-13)


def test_upsample_linear_exact_and_adjoint():
    rng = np.random.default_rng(13)
    fine = (9, 8, 7)
    coarse = nnet.down_dims(fine)
    assert coarse == (5, 4, 4)
    # a linear field sampled on the coarse grid (coarse o at fine 2o)
    a = rng.standard_normal(4)
    kz, jy, ix = np.meshgrid(*[np.arange(n) for n in coarse], indexing="ij")
    c = (a[0] + a[1] * 2 * kz + a[2] * 2 * jy + a[3] * 2 * ix)[None]
    f = nnet.upsample(c, fine)
    kz, jy, ix = np.meshgrid(*[np.arange(n) for n in fine], indexing="ij")
    lin = a[0] + a[1] * kz + a[2] * jy + a[3] * ix
    # exact everywhere except past the last coarse point (copies there)
    inner = (slice(None), slice(0, 9), slice(0, 7), slice(0, 7))
    np.testing.assert_allclose(f[inner], lin[None][inner], rtol=1e-13, atol=1e-12)
    cc = rng.standard_normal((3,) + coarse)
    ff = rng.standard_normal((3,) + fine)
    lhs = float((nnet.upsample(cc, fine) * ff).sum())
    rhs = float((cc * nnet.upsample_adj(ff, coarse)).sum())
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


@pytest.mark.parametrize("levels,ch,dims", [(3, (4, 6, 8), (5, 7, 6)), (4, (3, 4, 5, 6), (9, 8, 9))])
def test_backward_matches_finite_differences(levels, ch, dims):
    rng = np.random.default_rng(14)
    theta = nnet.init_params(levels, ch, seed=3)
    theta = theta + 0.01 * rng.standard_normal(theta.size)   # nonzero biases too
    inp = rng.standard_normal((2,) + dims)
    tgt = rng.standard_normal(dims)
    mask = np.zeros(dims, dtype=bool)
    mask[:, :, 0] = True

    def L(th):
        y, _ = nnet.forward(th, levels, ch, inp)
        return nnet.loss(y, tgt, mask)[0]

    y, cache = nnet.forward(theta, levels, ch, inp)
    _, gy = nnet.loss(y, tgt, mask)
    g = nnet.backward(theta, levels, ch, cache, gy)
    assert g.shape == theta.shape
    idx = rng.choice(theta.size, 40, replace=False)
    h = 1e-6
    worst = 0.0
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (L(tp) - L(tm)) / (2 * h)
        worst = max(worst, abs(fd - g[i]) / (abs(fd) + 1e-3 * np.abs(g).max()))
    assert worst < 1e-5, worst


def test_planted_backward_mistake_fails_the_check(monkeypatch):
    """A wrong upsampling adjoint in the backward pass is caught by the
    finite-difference comparison (the check has teeth)."""
    levels, ch, dims = 3, (3, 4, 5), (5, 5, 5)
    rng = np.random.default_rng(15)
    theta = nnet.init_params(levels, ch, seed=4)
    inp = rng.standard_normal((2,) + dims)
    tgt = rng.standard_normal(dims)
    orig = nnet.upsample_adj
    monkeypatch.setattr(nnet, "upsample_adj", lambda f, d: 0.5 * orig(f, d))
    y, cache = nnet.forward(theta, levels, ch, inp)
    _, gy = nnet.loss(y, tgt, None)
    g = nnet.backward(theta, levels, ch, cache, gy)
    h = 1e-6
    worst = 0.0
    for i in range(0, 60, 3):   # first-layer weights: part of their gradient comes through the decoder
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (nnet.loss(nnet.forward(tp, levels, ch, inp)[0], tgt, None)[0]
              - nnet.loss(nnet.forward(tm, levels, ch, inp)[0], tgt, None)[0]) / (2 * h)
        worst = max(worst, abs(fd - g[i]) / (abs(fd) + 1e-12))
    assert worst > 1e-2


def test_bf16_rounding_ties_to_even():
    """The storage rounding used to mirror BF16 activations: 8 significant
    bits, ties to even."""
    v = np.array([1.0, 1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, 1 + 2.0 ** -7, -2.5, 3.0e38, 1e-40])
    r = nnet.bf16(v)
    np.testing.assert_array_equal(r[:5], [1.0, 1.0, 1 + 2.0 ** -6, 1 + 2.0 ** -7, -2.5])
    assert abs(r[5] - 3.0e38) <= 3.0e38 * 2.0 ** -8
    x = np.random.default_rng(3).standard_normal(1000)
    assert np.all(np.abs(nnet.bf16(x) - x) <= np.abs(x) * 2.0 ** -8)


# ------------------------------------------------------------------- Adam
def test_adam_first_step_closed_form():
    """From m = v = 0 the bias-corrected moments are g and g^2, so the first
    update is lr g / (|g| + eps) for every parameter, whatever the scale."""
    rng = np.random.default_rng(21)
    th = rng.standard_normal(50)
    g = rng.standard_normal(50) * 10.0 ** rng.uniform(-6, 3, 50)
    lr, eps = 2e-3, 1e-8
    t1, m1, v1 = nnet.adam(th, g, np.zeros(50), np.zeros(50), 1, lr)
    np.testing.assert_allclose(t1, th - lr * g / (np.abs(g) + eps), rtol=0, atol=1e-15)
    np.testing.assert_allclose(m1, 0.1 * g, rtol=1e-15)
    np.testing.assert_allclose(v1, 0.001 * g * g, rtol=1e-14)


def test_adam_constant_gradient_moves_lr_per_step():
    """With a constant gradient m_t = (1 - b1^t) g and v_t = (1 - b2^t) g^2,
    so every bias-corrected step is again lr g / (|g| + eps)."""
    th0 = np.array([0.3, -1.2, 4.0])
    g = np.array([0.5, -2e-3, 7.0])
    th, m, v = th0.copy(), np.zeros(3), np.zeros(3)
    for t in range(1, 8):
        th, m, v = nnet.adam(th, g, m, v, t, 1e-2)
    np.testing.assert_allclose(th, th0 - 7 * 1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-13)


def test_adam_second_step_by_hand():
    """g1 = 1 then g2 = -1: m2 = 0.9 * 0.1 - 0.1 = -0.01, 1 - 0.9^2 = 0.19,
    so mhat = -1/19; v2 = 0.999 * 0.001 + 0.001 = 0.001999 = 1 - 0.999^2, so
    vhat = 1.  Steps: -lr / (1 + eps), then +lr / (19 (1 + eps)).
    g1 = 2 then g2 = 0: mhat = 0.18 / 0.19 = 18/19, vhat = 0.003996 / 0.001999."""
    lr, eps = 0.1, 1e-8
    th, m, v = nnet.adam([1.0, 1.0], [1.0, 2.0], [0.0, 0.0], [0.0, 0.0], 1, lr)
    th, m, v = nnet.adam(th, [-1.0, 0.0], m, v, 2, lr)
    exp0 = 1.0 - lr / (1.0 + eps) + lr / (19.0 * (1.0 + eps))
    exp1 = 1.0 - lr * 2.0 / (2.0 + eps) - lr * (18.0 / 19.0) / (np.sqrt(0.003996 / 0.001999) + eps)
    np.testing.assert_allclose(th, [exp0, exp1], rtol=1e-14)
    np.testing.assert_allclose(m, [-0.01, 0.18], rtol=1e-13)
    np.testing.assert_allclose(v, [0.001999, 0.003996], rtol=1e-13)


def test_network_gradient_check_detects_wiring_errors():
    """The GPU network's gradients are judged per layer against 3x the
    oracle's own sensitivity to sub-FP32 perturbations before each BF16
    rounding (nn_cases.sensitivity).  That tolerance must still catch a
    wrongly wired network: taps flipped in one layer (convolution instead of
    cross-correlation), the two input channels swapped, or the input mirrored
    along x each move the output by more than 0.1 relative and some layer's
    weight gradient by more than 0.3, and by more than 3x the sensitivity."""
    import nn_cases
    dims = (29, 22, 19)
    theta, inp, tgt, mask = nn_cases.net_case(11, dims)
    y0, _, g0 = nn_cases.oracle_grads(theta, inp, tgt, mask)
    sens = nn_cases.sensitivity(theta, inp, tgt, mask, g0)
    assert max(sens.values()) < 0.1
    specs = nnet.layer_specs(nn_cases.LEVELS, nn_cases.CH)

    def flipped(layer):
        th, o = theta.copy(), 0
        for name, ci, co, s, relu in specs:
            nw = co * ci * 27
            if name == layer:
                th[o:o + nw] = th[o:o + nw].reshape(co, ci, 3, 3, 3)[:, :, ::-1, ::-1, ::-1].ravel()
            o += nw + co
        return th

    planted = {
        "taps flipped in enc1": (flipped("enc1"), inp),
        "taps flipped in dec1": (flipped("dec1"), inp),
        "input channels swapped": (theta, inp[::-1].copy()),
        "input mirrored along x": (theta, inp[:, :, :, ::-1].copy()),
    }
    for what, (th, x) in planted.items():
        y1, _, g1 = nn_cases.oracle_grads(th, x, tgt, mask)
        dev = dict(nn_cases.layer_rel(g1, g0))
        caught = [k for k in dev if dev[k] > 0.3 and dev[k] > 3 * sens[k]]
        print(what, "output", np.linalg.norm(y1 - y0) / np.linalg.norm(y0), "layers caught", caught)
        assert np.linalg.norm(y1 - y0) > 0.1 * np.linalg.norm(y0), what
        assert caught, what
