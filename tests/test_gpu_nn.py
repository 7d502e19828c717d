"""Parity of the learned-preconditioner kernels with the oracle, and the
learned solve.

Convolutions: BF16 operands (exact in FP32 products) with FP32
accumulation over K = 27 Cin terms (forward), 27 Cout (data gradient) or
the output voxels (weight gradient).  The rounding bound of such a sum is
K u sum|terms| with u = 2^-24, checked element by element against the FP64
oracle on the same BF16 values.

Network: the GPU keeps activations and layer gradients in BF16; the oracle
runs with the same storage rounding (oracle.nnet.bf16 at the same points),
so the two differ only by FP32 accumulation order and the BF16 values it
flips (one BF16 ulp, 2^-8 relative, each): output within 2e-3 relative (L2),
weight gradients within 5e-2 per layer (the deepest layers sum over a few
dozen voxels, where a flipped BF16 value next to zero also flips a ReLU
gate, so a few flips move them by percents; a wiring error moves them by
order one).  The grids keep 36 and 60 voxels on the coarsest level.

Learned solve: every answer is judged by the true FP64 residual; the
pressure must match the plain FP64 answer to 1e-8 relative.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import nnet
from gpu_util import print_case

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def bits(v):
    """BF16 bit patterns of values that are already BF16-representable."""
    return (np.ascontiguousarray(v, dtype=np.float32).view(np.uint32) >> 16).astype(np.uint16)


def cl(a):
    """[C][z][y][x] -> channels-last [voxel][C] (x fastest)."""
    return np.ascontiguousarray(np.moveaxis(a, 0, -1).reshape(-1, a.shape[0]))


def rand_bf16(seed, shape, scale=1.0):
    return nnet.bf16(scale * synth.random_field(seed, int(np.prod(shape))).reshape(shape))


CASES = [(8, 16, 1, (9, 7, 5)), (16, 16, 1, (17, 9, 6)), (16, 32, 2, (17, 9, 6)),
         (32, 48, 2, (9, 9, 5)), (48, 32, 1, (9, 5, 5)), (64, 64, 1, (5, 5, 3)),
         (16, 8, 1, (11, 6, 4))]


@pytest.mark.parametrize("cin,cout,s,din", CASES)
def test_conv_forward_parity(hts, cin, cout, s, din):
    print_case("conv fwd", cin, cout, s, din)
    X, Y, Z = din
    x = rand_bf16(1, (cin, Z, Y, X))
    w = rand_bf16(2, (cout, cin, 3, 3, 3), 0.2)
    b = nnet.bf16(synth.random_field(3, cout))
    y = hts.conv3d(0, cin, cout, s, din, x=bits(cl(x)), w=bits(w), bias=b)
    ref = oracle.conv3d_fwd(x[None], w, b, stride=s)[0]
    bound = oracle.conv3d_fwd(np.abs(x)[None], np.abs(w), np.abs(b), stride=s)[0]
    err = np.abs(y - cl(ref))
    assert np.all(err <= 27 * cin * U32 * cl(bound) + 1e-30), err.max()


# Grids of at least 32768 output voxels take the LDS-tiled kernel (stride 1,
# halo tile within 64 KB) or the one-gather-per-step kernel (stride 2, or
# 64 input channels); the small CASES take the split-K kernel.  Ragged tiles
# on every axis.
LARGE = [(16, 16, 1, (41, 33, 25)), (8, 16, 1, (37, 35, 27)), (48, 32, 1, (33, 33, 31)),
         (16, 32, 2, (129, 65, 33)), (64, 16, 1, (34, 33, 30))]


@pytest.mark.parametrize("cin,cout,s,din", LARGE)
def test_conv_forward_parity_large(hts, cin, cout, s, din):
    test_conv_forward_parity(hts, cin, cout, s, din)


@pytest.mark.parametrize("cin,cout,s,din", CASES)
def test_conv_data_gradient_parity(hts, cin, cout, s, din):
    print_case("conv bwd data", cin, cout, s, din)
    X, Y, Z = din
    dout = tuple((n - 1) // s + 1 for n in din)
    g = rand_bf16(4, (cout, dout[2], dout[1], dout[0]))
    w = rand_bf16(5, (cout, cin, 3, 3, 3), 0.2)
    gx = hts.conv3d(1, cin, cout, s, din, w=bits(w), g=bits(cl(g)))
    ref = oracle.conv3d_bwd_data(g[None], w, (1, cin, Z, Y, X), stride=s)[0]
    bound = oracle.conv3d_bwd_data(np.abs(g)[None], np.abs(w), (1, cin, Z, Y, X), stride=s)[0]
    err = np.abs(gx - cl(ref))
    assert np.all(err <= 27 * cout * U32 * cl(bound) + 1e-30), err.max()


# Stride 1 on at least 32768 voxels: the data gradient runs as the LDS-tiled
# forward kernel with mirrored offsets.
LARGE_DATA = [(16, 16, 1, (41, 33, 25)), (16, 48, 1, (33, 33, 31)), (8, 32, 1, (37, 35, 27)),
              (48, 16, 1, (34, 33, 30))]


@pytest.mark.parametrize("cin,cout,s,din", LARGE_DATA)
def test_conv_data_gradient_parity_large(hts, cin, cout, s, din):
    test_conv_data_gradient_parity(hts, cin, cout, s, din)


@pytest.mark.parametrize("cin,cout,s,din", CASES + [(16, 16, 1, (33, 21, 9))])
def test_conv_weight_gradient_parity(hts, cin, cout, s, din):
    print_case("conv bwd weight", cin, cout, s, din)
    X, Y, Z = din
    dout = tuple((n - 1) // s + 1 for n in din)
    nout = int(np.prod(dout))
    x = rand_bf16(6, (cin, Z, Y, X))
    g = rand_bf16(7, (cout, dout[2], dout[1], dout[0]))
    gw, gb = hts.conv3d(2, cin, cout, s, din, x=bits(cl(x)), w=np.zeros((cout, cin, 3, 3, 3), np.uint16),
                        g=bits(cl(g)))
    rw, rb = oracle.conv3d_bwd_weight(x[None], g[None], 3, stride=s)
    bw, bb = oracle.conv3d_bwd_weight(np.abs(x)[None], np.abs(g)[None], 3, stride=s)
    assert np.all(np.abs(gw - rw) <= nout * U32 * bw + 1e-30), np.abs(gw - rw).max()
    assert np.all(np.abs(gb - rb) <= nout * U32 * bb + 1e-30)


def small_net(hts, seed=0):
    return hts.Net(levels=4, channels=(16, 32, 48, 64), seed=seed)


def net_case(seed, dims):
    X, Y, Z = dims
    theta = nnet.bf16(nnet.init_params(4, (16, 32, 48, 64), seed=seed))
    rng = np.random.default_rng(seed)
    theta = nnet.bf16(theta + 0.02 * rng.standard_normal(theta.size))   # nonzero biases
    inp = nnet.bf16(rng.standard_normal((2, Z, Y, X)))
    tgt = nnet.bf16(rng.standard_normal((Z, Y, X)))
    mask = np.zeros((Z, Y, X), dtype=bool)
    mask[:, 0, :] = True
    return theta, inp, tgt, mask


@pytest.mark.parametrize("dims", [(33, 25, 17), (29, 22, 19)])
def test_network_forward_and_gradient_parity(hts, dims):
    print_case("network", dims)
    X, Y, Z = dims
    theta, inp, tgt, mask = net_case(11, dims)
    net = small_net(hts)
    net.set_params(theta)
    assert np.array_equal(net.get_params(), theta)
    out, lv, g = net.eval(dims, cl(inp), target=tgt.ravel(), mask=mask.ravel(), grad=True)
    y, cache = nnet.forward(theta, 4, (16, 32, 48, 64), inp, act_round=nnet.bf16)
    lo, gy = nnet.loss(y, tgt, mask)
    go = nnet.backward(theta, 4, (16, 32, 48, 64), cache, gy, grad_round=nnet.bf16)
    yr = y.ravel()
    print("out rel", np.linalg.norm(out - yr) / np.linalg.norm(yr), "loss", lv, lo)
    assert np.linalg.norm(out - yr) <= 2e-3 * np.linalg.norm(yr)
    assert lv == pytest.approx(lo, rel=5e-3)
    o = 0
    for name, ci, co, s, relu in nnet.layer_specs(4, (16, 32, 48, 64)):
        nw = co * ci * 27 + co
        a, b = g[o:o + nw], go[o:o + nw]
        r = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
        print(name, "grad rel", r)
        assert r <= 5e-2, name
        o += nw


def test_save_load_roundtrip(hts, tmp_path):
    print_case("save/load")
    a = small_net(hts, seed=1)
    b = small_net(hts, seed=2)
    assert not np.array_equal(a.get_params(), b.get_params())
    a.save(tmp_path / "n.bin")
    b.load(tmp_path / "n.bin")
    assert np.array_equal(a.get_params(), b.get_params())
    c = hts.Net(levels=3, channels=(16, 32, 48))
    with pytest.raises(hts.HtsError):
        c.load(tmp_path / "n.bin")


# ----------------------------------------------------------- learned solves
NC = (32, 32, 16)


def mesh_of(hts, seed, o):
    return hts.from_scenario(synth.config5(seed, ncells=NC, n_steps=4), opts=o)


@pytest.fixture(scope="module")
def trained(hts):
    """Network trained on pairs harvested from 4 draws (the last held out)."""
    print_case("harvest + train", NC)
    o = hts.default_opts()
    ms = [mesh_of(hts, 5000 + i, o) for i in range(4)]
    net = hts.Net(levels=4, channels=(16, 32, 48, 64), seed=7)
    net.harvest(ms, 3, synth.DAY, 8)
    st = net.train(epochs=6, lr=2e-3, batch=4, val_draws=1)
    print("train", st)
    return net, st


def test_training_reduces_loss(hts, trained):
    net, st = trained
    assert st["pairs"] >= 40
    assert np.isfinite(st["val_loss"])
    assert st["loss_last"] < st["loss_first"]


def solve_steps(hts, seed, o, steps=2):
    m = mesh_of(hts, seed, o)
    stats = []
    for _ in range(steps):
        code, st = m.solve_step(synth.DAY, o)
        stats.append(st)
    return m.get_state(0)[0], stats


def test_learned_solve_matches_fp64_and_reports_gain(hts, trained):
    net, _ = trained
    seed = 5100          # a draw the network never saw
    print_case("learned solve", seed)
    P64, s64 = solve_steps(hts, seed, hts.default_opts(rtol=1e-8))
    o = hts.default_opts(rtol=1e-8, mode=hts.MODE_LEARNED)
    o.nn = net.h.value
    PL, sL = solve_steps(hts, seed, o)
    for st in sL:
        assert st["status"] == [0, 0]
        assert st["relres"][0] <= 1e-8
    assert np.linalg.norm(PL - P64) <= 1e-8 * np.linalg.norm(P64)
    it64 = sum(s["iters"][0] for s in s64)
    itL = sum(s["iters"][0] for s in sL)
    fb = sum(s["fallbacks"] for s in sL)
    ms64 = sum(s["time_ms"][0] for s in s64)
    msL = sum(s["time_ms"][0] for s in sL)
    print("pressure iterations: multigrid %d, learned %d (fallbacks %d); ms %.2f vs %.2f"
          % (it64, itL, fb, ms64, msL))


def test_sabotaged_network_falls_back(hts):
    """Random weights give directions that do not reduce the residual: the
    solve switches to the V-cycle and still meets the FP64 residual."""
    print_case("fallback")
    net = hts.Net(levels=4, channels=(16, 32, 48, 64), seed=3)
    th = net.get_params()
    net.set_params(np.random.default_rng(0).standard_normal(th.size))
    o = hts.default_opts(rtol=1e-8, mode=hts.MODE_LEARNED)
    o.nn = net.h.value
    P64, _ = solve_steps(hts, 5101, hts.default_opts(rtol=1e-8), steps=1)
    PL, sL = solve_steps(hts, 5101, o, steps=1)
    assert sL[0]["fallbacks"] >= 1
    assert sL[0]["status"] == [0, 0]
    assert sL[0]["relres"][0] <= 1e-8
    assert np.linalg.norm(PL - P64) <= 1e-8 * np.linalg.norm(P64)
