"""Network parity cases and the reference gradients they are judged by,
shared by the oracle pins and the GPU parity tests.

The GPU network stores activations and layer gradients in BF16.  Two
computations that differ only in FP32 summation order round some stored
values to neighbouring BF16 values (one BF16 ulp, 2^-8 relative); next to a
ReLU gate such a step can flip the gate, and the flips compound through the
layers, so no a-priori elementwise bound separates correct from wrong.  The
tolerance is taken instead from the oracle's own sensitivity: the per-layer
deviation of oracle runs whose stored values are perturbed, before rounding,
by a relative amount below FP32 accumulation error (uniform in +-2^-16).
"""
import numpy as np

from oracle import nnet

LEVELS = 4
CH = (16, 32, 48, 64)
NOISE_REL = 2.0 ** -16
NOISE_RUNS = 4


def net_case(seed, dims):
    """BF16 parameters (initialisation plus small noise so that biases are
    nonzero), a two-channel input, a target and a Dirichlet-row mask."""
    X, Y, Z = dims
    theta = nnet.bf16(nnet.init_params(LEVELS, CH, seed=seed))
    rng = np.random.default_rng(seed)
    theta = nnet.bf16(theta + 0.02 * rng.standard_normal(theta.size))
    inp = nnet.bf16(rng.standard_normal((2, Z, Y, X)))
    tgt = nnet.bf16(rng.standard_normal((Z, Y, X)))
    mask = np.zeros((Z, Y, X), dtype=bool)
    mask[:, 0, :] = True
    return theta, inp, tgt, mask


def oracle_grads(theta, inp, tgt, mask, rnd=nnet.bf16):
    """Output, loss and parameter gradient of the oracle network with storage
    rounding rnd at the points where the GPU stores BF16."""
    y, cache = nnet.forward(theta, LEVELS, CH, inp, act_round=rnd)
    lo, gy = nnet.loss(y, tgt, mask)
    return y, lo, nnet.backward(theta, LEVELS, CH, cache, gy, grad_round=rnd)


def layer_rel(a, b):
    """Per layer (name, ||a - b|| / ||b||) over weights and biases."""
    out, o = [], 0
    for name, ci, co, s, relu in nnet.layer_specs(LEVELS, CH):
        nw = co * ci * 27 + co
        out.append((name, float(np.linalg.norm(a[o:o + nw] - b[o:o + nw]) / max(np.linalg.norm(b[o:o + nw]), 1e-30))))
        o += nw
    return out


def sensitivity(theta, inp, tgt, mask, ref_grad):
    """Largest per-layer deviation from ref_grad over NOISE_RUNS oracle runs
    with sub-FP32 perturbations before each BF16 rounding."""
    worst = {}
    for k in range(NOISE_RUNS):
        rng = np.random.default_rng(1000 + k)

        def noisy(a):
            return nnet.bf16(a * (1.0 + NOISE_REL * rng.uniform(-1.0, 1.0, a.shape)))

        _, _, g = oracle_grads(theta, inp, tgt, mask, noisy)
        for name, r in layer_rel(g, ref_grad):
            worst[name] = max(worst.get(name, 0.0), r)
    return worst
