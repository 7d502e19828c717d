"""Oracle of the learned preconditioner network (FP64, CPU).

TEST INFRASTRUCTURE ONLY (same rule as the rest of ``oracle``).

The learned preconditioner maps a normalised residual plus a node feature
(log-permeability) to an error estimate.  The network is a 3D convolutional
encoder-decoder with ``levels`` resolution levels, channel widths
``ch[0..levels-1]``, 3x3x3 kernels with zero padding 1, ReLU activations,
stride-2 convolutions going down, linear upsampling going up and additive
skip connections.  Layers, in parameter order:

* ``enc0a``: in -> ch0, ``enc0b``: ch0 -> ch0 (gives e0);
* for l = 1 .. levels-1: ``down_l`` (stride 2) ch[l-1] -> ch[l], then
  ``enc_l`` ch[l] -> ch[l] (gives e_l);
* for l = levels-2 .. 0: ``dec_l`` ch[l+1] -> ch[l] on the upsampled
  d_{l+1} (d_{levels-1} = e_{levels-1}); d_l = relu(dec_l(up(d_{l+1}))) + e_l;
* ``out``: ch0 -> 1, no activation.

A stride-2 convolution of a grid of n points gives floor((n-1)/2)+1 points;
coarse point o sits on fine point 2o.  Linear upsampling copies coarse values
to even fine points and averages the two coarse neighbours at odd ones (or
copies the last one past the end).

The loss is the mean squared error over free (non-Dirichlet) nodes of output
channel 0 against the target.  Parameters are given as a flat FP64 vector:
per layer W[cout][ci][kz][ky][kx] (cross-correlation weights, the layout of
``conv3d_fwd``) followed by b[cout].

Arrays here are [C][z][y][x] (one sample); the GPU path stores the same
tensors channels-last with x fastest.

Training updates the parameters with Adam (Kingma and Ba), ``adam`` below.

Pins: ``tests/test_oracle_nn.py`` checks the convolutions against direct
sums, the adjoint identities of convolution and upsampling, exactness of
the upsampling on linear fields, the full backward pass against central
finite differences of the loss, and Adam against its closed-form first
step, constant-gradient steps and a second step worked by hand.
"""
from __future__ import annotations

import numpy as np

from . import conv3d_fwd, conv3d_bwd_data, conv3d_bwd_weight


def layer_specs(levels: int, ch, cin: int = 2):
    """[(name, cin, cout, stride, relu)] in parameter order."""
    assert 2 <= levels <= len(ch)
    L = [("enc0a", cin, ch[0], 1, True), ("enc0b", ch[0], ch[0], 1, True)]
    for l in range(1, levels):
        L.append(("down%d" % l, ch[l - 1], ch[l], 2, True))
        L.append(("enc%d" % l, ch[l], ch[l], 1, True))
    for l in range(levels - 2, -1, -1):
        L.append(("dec%d" % l, ch[l + 1], ch[l], 1, True))
    L.append(("out", ch[0], 1, 1, False))
    return L


def n_params(levels, ch, cin=2):
    return sum(co * ci * 27 + co for _, ci, co, _, _ in layer_specs(levels, ch, cin))


def unpack(theta, levels, ch, cin=2):
    out, o = [], 0
    for name, ci, co, s, relu in layer_specs(levels, ch, cin):
        w = np.asarray(theta[o:o + co * ci * 27], dtype=np.float64).reshape(co, ci, 3, 3, 3)
        o += co * ci * 27
        b = np.asarray(theta[o:o + co], dtype=np.float64)
        o += co
        out.append((name, w, b, s, relu))
    return out


def down_dims(d):
    return tuple((n - 1) // 2 + 1 for n in d)


def _up_matrix(nf: int, nc: int) -> np.ndarray:
    """1D linear upsampling matrix [nf][nc]."""
    U = np.zeros((nf, nc))
    for i in range(nf):
        if i % 2 == 0:
            U[i, i // 2] = 1.0
        elif (i + 1) // 2 >= nc:
            U[i, i // 2] = 1.0
        else:
            U[i, i // 2] = 0.5
            U[i, (i + 1) // 2] = 0.5
    return U


def upsample(c: np.ndarray, fine_dims) -> np.ndarray:
    """[C][z][y][x] coarse -> fine (tensor product of 1D linear maps)."""
    Z, Y, X = fine_dims
    Uz, Uy, Ux = (_up_matrix(Z, c.shape[1]), _up_matrix(Y, c.shape[2]), _up_matrix(X, c.shape[3]))
    return np.einsum("zk,yj,xi,ckji->czyx", Uz, Uy, Ux, c, optimize=True)


def upsample_adj(f: np.ndarray, coarse_dims) -> np.ndarray:
    Z, Y, X = coarse_dims
    Uz, Uy, Ux = (_up_matrix(f.shape[1], Z), _up_matrix(f.shape[2], Y), _up_matrix(f.shape[3], X))
    return np.einsum("zk,yj,xi,czyx->ckji", Uz, Uy, Ux, f, optimize=True)


def bf16(a):
    """Round to the nearest BF16 value (ties to even), returned as float64.
    Used to state the storage precision of the GPU network; the pins run the
    oracle without it."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return u.view(np.float32).astype(np.float64)


def _conv(x, w, b, s):
    return conv3d_fwd(x[None], w, b, stride=s, pad=1)[0]


def forward(theta, levels, ch, inp: np.ndarray, cin: int = 2, act_round=None):
    """inp [cin][z][y][x] -> (out [z][y][x], cache).  act_round, if given, is
    applied to every stored activation (each hidden layer output, each
    upsampled tensor and each skip sum), as a network that keeps its
    activations in a narrower type does."""
    layers = unpack(theta, levels, ch, cin)
    cache = {"in": inp, "pre": [], "act": []}
    rnd = act_round if act_round is not None else (lambda a: a)

    def run(x, k):
        name, w, b, s, relu = layers[k]
        pre = _conv(x, w, b, s)
        cache["pre"].append(pre)
        cache["act"].append(x)
        return rnd(np.maximum(pre, 0.0)) if relu else pre

    h = run(inp, 0)
    e = [run(h, 1)]
    li = 2
    for l in range(1, levels):
        h = run(e[-1], li)
        e.append(run(h, li + 1))
        li += 2
    d = e[-1]
    for l in range(levels - 2, -1, -1):
        u = rnd(upsample(d, e[l].shape[1:]))
        d = rnd(run(u, li) + e[l])
        li += 1
    y = run(d, li)
    cache["e"] = e
    return y[0], cache


def loss(y0, target, mask):
    free = ~mask if mask is not None else np.ones_like(y0, dtype=bool)
    nf = max(1, int(free.sum()))
    diff = np.where(free, y0 - target, 0.0)
    return float((diff * diff).sum() / nf), 2.0 * diff / nf


def backward(theta, levels, ch, cache, gy0: np.ndarray, cin: int = 2, grad_round=None):
    """Gradient of sum(gy0 * out) with respect to theta (flat, parameter order).
    grad_round, if given, is applied to each layer's pre-activation gradient
    before it enters the two convolution gradients."""
    layers = unpack(theta, levels, ch, cin)
    grads = [None] * len(layers)
    rnd = grad_round if grad_round is not None else (lambda a: a)

    def back(k, gout):
        """gout: gradient w.r.t. the layer's output after its activation."""
        name, w, b, s, relu = layers[k]
        pre, x = cache["pre"][k], cache["act"][k]
        g = rnd(gout * (pre > 0) if relu else gout)
        gw, gb = conv3d_bwd_weight(x[None], g[None], 3, stride=s, pad=1)
        grads[k] = (gw, gb)
        return conv3d_bwd_data(g[None], w, (1,) + x.shape, stride=s, pad=1)[0]

    e = cache["e"]
    nl = len(layers)
    k = nl - 1
    gd = back(k, gy0[None])
    ge = [np.zeros_like(t) for t in e]
    for l in range(0, levels - 1):
        k -= 1
        ge[l] += gd                      # skip path of d_l = relu(dec_l(.)) + e_l
        gu = back(k, gd)                 # through dec_l
        gd = upsample_adj(gu, e[l + 1].shape[1:])
    ge[levels - 1] += gd
    for l in range(levels - 1, 0, -1):
        k = 2 * l + 1
        gh = back(k, ge[l])              # enc_l
        ge[l - 1] += back(k - 1, gh)     # down_l
    gh = back(1, ge[0])
    back(0, gh)
    flat = []
    for gw, gb in grads:
        flat.append(gw.ravel())
        flat.append(gb.ravel())
    return np.concatenate(flat)


def init_params(levels, ch, cin=2, seed=0):
    """He-normal weights, zero biases, output layer scaled by 0.1."""
    rng = np.random.default_rng(seed)
    out = []
    for name, ci, co, s, relu in layer_specs(levels, ch, cin):
        sd = np.sqrt(2.0 / (27 * ci)) * (0.1 if name == "out" else 1.0)
        out.append(rng.standard_normal(co * ci * 27) * sd)
        out.append(np.zeros(co))
    return np.concatenate(out)


def adam(theta, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, Algorithm 1), plain per-element loop
    in FP64.  step is the 1-based update count t.  Returns new (theta, m, v):

    m_t = beta1 m + (1 - beta1) g,  v_t = beta2 v + (1 - beta2) g^2,
    mhat = m_t / (1 - beta1^t),  vhat = v_t / (1 - beta2^t),
    theta_t = theta - lr mhat / (sqrt(vhat) + eps).

    The gradient is the minibatch mean (callers pass the summed gradient
    times 1 / batch)."""
    th = np.array(theta, dtype=np.float64, copy=True).ravel()
    g = np.asarray(grad, dtype=np.float64).ravel()
    m1 = np.array(m, dtype=np.float64, copy=True).ravel()
    v1 = np.array(v, dtype=np.float64, copy=True).ravel()
    c1 = 1.0 - beta1 ** step
    c2 = 1.0 - beta2 ** step
    for i in range(th.size):
        m1[i] = beta1 * m1[i] + (1.0 - beta1) * g[i]
        v1[i] = beta2 * v1[i] + (1.0 - beta2) * g[i] * g[i]
        mhat = m1[i] / c1
        vhat = v1[i] / c2
        th[i] = th[i] - lr * mhat / (np.sqrt(vhat) + eps)
    return th, m1, v1
