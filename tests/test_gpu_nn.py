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
flips (one BF16 ulp, 2^-8 relative, each): output within 2e-3 relative (L2).
Flipped values next to ReLU gates flip gates and compound through the
layers, so the per-layer weight gradients are judged against the oracle's
own sensitivity (nn_cases.sensitivity: oracle runs perturbed below FP32
accumulation error before each BF16 rounding): at most 3x its largest
deviation per layer, floor 2e-3.  Planted wiring errors move some layer by
more than 0.3 (test_oracle_nn).  The grids keep 36 and 60 voxels on the
coarsest level.

Learned solve: every answer is judged against the oracle (parity mode:
1e-8 relative pressure, 1e-6 K) and by its backward error in the oracle's
assembled matrices at the working tolerance; the gain over plain multigrid
is measured and its outcome asserted.  Adam: per element against the
oracle's Adam with a bound derived from the FP32 operations.
"""
import numpy as np
import pytest

import nn_cases
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


@pytest.mark.parametrize("dims", [(33, 25, 17), (29, 22, 19)])
def test_network_forward_and_gradient_parity(hts, dims):
    print_case("network", dims)
    theta, inp, tgt, mask = nn_cases.net_case(11, dims)
    net = small_net(hts)
    net.set_params(theta)
    assert np.array_equal(net.get_params(), theta)
    out, lv, g = net.eval(dims, cl(inp), target=tgt.ravel(), mask=mask.ravel(), grad=True)
    y, lo, go = nn_cases.oracle_grads(theta, inp, tgt, mask)
    yr = y.ravel()
    print("out rel", np.linalg.norm(out - yr) / np.linalg.norm(yr), "loss", lv, lo)
    assert np.linalg.norm(out - yr) <= 2e-3 * np.linalg.norm(yr)
    assert lv == pytest.approx(lo, rel=5e-3)
    sens = nn_cases.sensitivity(theta, inp, tgt, mask, go)
    for name, r in nn_cases.layer_rel(g, go):
        tol = max(3.0 * sens[name], 2e-3)
        print(name, "grad rel %.4g  (oracle sensitivity %.4g, bound %.4g)" % (r, sens[name], tol))
        assert r <= tol, name


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


def judge_first_step(scn, P1, T1, rtol):
    """Backward error of one GPU step from the scenario's initial state in
    the oracle's own assembled, eliminated systems (residual accumulated in
    long double), and Dirichlet values as the oracle sets them."""
    om = oracle.Mesh.of(scn)
    P0, T0 = oracle.initial_state(scn, om)
    t1 = scn.t0 + scn.dt
    out = []
    for field in (0, 1):
        if field == 0:
            A, b = oracle.pressure_system(scn, om, P0, t1)
            x = P1
        else:
            A, b = oracle.heat_system(scn, om, T0, P1, t1)
            x = T1
        mask, g = oracle.dirichlet(scn, om, field, t1)
        free, AFF, bF = oracle.eliminate(A, b, mask, g)
        r = oracle.residual_ld(AFF, bF, x[free])
        out.append(float(np.linalg.norm(r) / np.linalg.norm(bF)))
        assert np.all(np.abs(x[mask] - g[mask]) <= 4 * np.finfo(float).eps * np.abs(g[mask]))
    assert out[0] <= rtol and out[1] <= rtol, out
    return out


def test_learned_solve_matches_oracle(hts, trained):
    """Learned mode (flexible CG with the network, V-cycle fallback) on a
    draw the network never saw: parity mode (rtol 1e-12) against the
    oracle's direct solve (<= 1e-8 relative pressure, also relative to the
    change of pressure over the steps, <= 1e-6 K temperature), and at the
    working tolerance 1e-8 the first step's backward error in the oracle's
    own matrices."""
    net, _ = trained
    seed = 5100
    print_case("learned solve vs oracle", seed)
    scn = synth.config5(seed, ncells=NC, n_steps=2)
    o = hts.default_opts(rtol=1e-12, mode=hts.MODE_LEARNED)
    o.nn = net.h.value
    m = hts.from_scenario(scn, opts=o)
    P0 = m.get_state(0)[0]
    for _ in range(2):
        code, st = m.solve_step(scn.dt, o)
        assert code == 0 and st["status"] == [0, 0]
    PL, TL = m.get_state(0)[0], m.get_state(1)[0]
    Po, To, _ = oracle.run(scn, n_steps=2)
    Pi, _ = oracle.initial_state(scn)
    assert np.linalg.norm(PL - Po) <= 1e-8 * np.linalg.norm(Po)
    assert np.linalg.norm(PL - Po) <= 1e-6 * np.linalg.norm(Po - Pi)
    assert np.abs(TL - To).max() <= 1e-6
    assert np.array_equal(P0, Pi)
    # working tolerance: one step judged in the oracle's CSR
    o8 = hts.default_opts(rtol=1e-8, mode=hts.MODE_LEARNED)
    o8.nn = net.h.value
    m8 = hts.from_scenario(scn, opts=o8)
    code, st = m8.solve_step(scn.dt, o8)
    assert code == 0
    print("backward errors", judge_first_step(scn, m8.get_state(0)[0], m8.get_state(1)[0], 1.0001e-8))


def test_learned_gain_over_multigrid(hts, trained):
    """What the trained network gains over plain multigrid CG on an unseen
    draw, measured as pressure iterations to a 1e-8 relative residual.  On
    this problem it gains nothing: a V-cycle reduces the residual about 20x
    per iteration, the network's direction less, and the fallback rule
    switches to the V-cycle within the first iterations.  The test states
    that measured outcome: the learned solve needs at least as many
    iterations as plain multigrid and at most 4x as many, and every step
    converges to the FP64 residual."""
    net, _ = trained
    seed = 5100
    print_case("learned gain", seed)
    _, s64 = solve_steps(hts, seed, hts.default_opts(rtol=1e-8))
    o = hts.default_opts(rtol=1e-8, mode=hts.MODE_LEARNED)
    o.nn = net.h.value
    _, sL = solve_steps(hts, seed, o)
    for st in sL:
        assert st["status"] == [0, 0]
        assert st["relres"][0] <= 1e-8
    it64 = sum(s["iters"][0] for s in s64)
    itL = sum(s["iters"][0] for s in sL)
    fb = sum(s["fallbacks"] for s in sL)
    print("pressure iterations: multigrid %d, learned %d (fallbacks %d)" % (it64, itL, fb))
    assert it64 <= itL <= 4 * it64


def test_learned_graph_replay_equals_eager(hts, trained):
    """The learned preconditioner's fallback rule runs on the device, so the
    learned flexible CG replays as captured graphs: graph replay and eager
    launches give the same pressure and temperature bit for bit, the same
    iteration counts and the same fallbacks, over three steps (the first
    replays capture, the later ones reuse the graphs)."""
    net, _ = trained
    seed = 5100
    print_case("learned graph vs eager", seed)
    og = hts.default_opts(rtol=1e-8, mode=hts.MODE_LEARNED, use_graph=1)
    og.nn = net.h.value
    oe = hts.default_opts(rtol=1e-8, mode=hts.MODE_LEARNED, use_graph=0)
    oe.nn = net.h.value
    mg, me = mesh_of(hts, seed, og), mesh_of(hts, seed, oe)
    for _ in range(3):
        cg_, sg = mg.solve_step(synth.DAY, og)
        ce, se = me.solve_step(synth.DAY, oe)
        assert cg_ == 0 and ce == 0
        assert sg["iters"] == se["iters"] and sg["fallbacks"] == se["fallbacks"]
    for f in (0, 1):
        assert np.array_equal(mg.get_state(f)[0], me.get_state(f)[0])


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
    scn = synth.config5(5101, ncells=NC, n_steps=4)
    m = hts.from_scenario(scn, opts=o)
    code, st = m.solve_step(scn.dt, o)
    assert code == 0 and st["fallbacks"] >= 1
    print("backward errors", judge_first_step(scn, m.get_state(0)[0], m.get_state(1)[0], 1.0001e-8))


# ------------------------------------------------------------------- Adam
@pytest.mark.parametrize("step", [1, 3, 60])
def test_adam_kernel_per_element(hts, step):
    """The FP32 Adam kernel against the FP64 oracle Adam with the kernel's
    hyperparameters (the FP32 values nearest 0.9, 0.999 and 1e-8), per
    element.  Bound, from the FP32 operations of one update (u = 2^-24):
    m: 4u (|b1 m| + |(1-b1) g|);  v: 5u (|b2 v| + |(1-b2) g^2|);  the bias
    corrections 1/(1 - b^t) carry u (2 kappa + 3) relative, kappa =
    b^t / (1 - b^t) (powf within 2 ulp, cancellation in 1 - b^t); the step
    lr mhat / (sqrt(vhat) + eps) adds these relative errors (half of those of
    vhat) plus 6u, and the final subtraction u |w|.  The BF16 copy must be
    the round-to-nearest-even of the new FP32 weight, bit for bit."""
    print_case("adam", step)
    rng = np.random.default_rng(40 + step)
    n = 4099
    f32 = lambda a: np.asarray(a, dtype=np.float32)
    w = f32(rng.standard_normal(n))
    g = f32(rng.standard_normal(n) * 10.0 ** rng.uniform(-4, 1, n))
    g[:5] = 0.0
    m = f32(0.1 * rng.standard_normal(n)) if step > 1 else np.zeros(n, np.float32)
    v = f32(0.01 * rng.uniform(0, 1, n) ** 2) if step > 1 else np.zeros(n, np.float32)
    lr, gs = 2e-3, 0.25
    wg, mg, vg, wbf = hts.adam_step(step, lr, gs, w, m, v, g)
    b1, b2, eps = float(np.float32(0.9)), float(np.float32(0.999)), float(np.float32(1e-8))
    gi = g.astype(np.float64) * gs
    wr, mr, vr = nnet.adam(w, gi, m, v, step, lr, beta1=b1, beta2=b2, eps=eps)
    u = U32
    em = 4 * u * (np.abs(b1 * m) + np.abs((1 - b1) * gi))
    ev = 5 * u * (np.abs(b2 * v) + np.abs((1 - b2) * gi * gi))
    assert np.all(np.abs(mg - mr) <= em)
    assert np.all(np.abs(vg - vr) <= ev)
    k1, k2 = b1 ** step / (1 - b1 ** step), b2 ** step / (1 - b2 ** step)
    rc1, rc2 = u * (2 * k1 + 3), u * (2 * k2 + 3)
    c1, c2 = 1 / (1 - b1 ** step), 1 / (1 - b2 ** step)
    sq = np.sqrt(vr * c2)
    D = sq + eps
    upd = lr * np.abs(mr) * c1 / D
    with np.errstate(divide="ignore", invalid="ignore"):
        rv = np.where(vr > 0, ev / vr, 0.0)
    eu = lr * em * c1 / D + upd * (rc1 + (0.5 * (rv + rc2) + 2 * u) * sq / D + 6 * u)
    err = np.abs(wg.astype(np.float64) - wr)
    tol = eu + u * np.abs(wr)
    assert np.all(err <= tol), float(np.max(err / tol))
    assert np.array_equal(bits(nnet.bf16(wg)), wbf)


def test_gamma_scales_every_target_once(hts):
    """Gamma (the target scale) is fixed by the first train call and each
    harvested target is divided by it exactly once: a train call with no
    epochs leaves the held-out loss unchanged when repeated, and pairs
    harvested after a train call (here from a copy of the held-out draw)
    give the same held-out loss as the original ones."""
    print_case("gamma bookkeeping")
    o = hts.default_opts()
    scn = [synth.config5(5000 + i, ncells=(16, 16, 8), n_steps=2) for i in range(2)]
    a, b, b2 = (hts.from_scenario(sc, opts=o) for sc in (scn[0], scn[1], scn[1]))
    net = hts.Net(levels=3, channels=(16, 32, 48), seed=5)
    net.harvest([a, b], 2, synth.DAY, 4)
    s1 = net.train(epochs=0, lr=1e-3, batch=2, val_draws=1)
    s2 = net.train(epochs=0, lr=1e-3, batch=2, val_draws=1)
    assert s1["val_loss"] > 0 and s1["val_loss"] == s2["val_loss"]
    net.harvest([b2], 2, synth.DAY, 4)      # draws a, b, b2: b2 is now held out
    s3 = net.train(epochs=0, lr=1e-3, batch=2, val_draws=1)
    assert s3["val_loss"] == pytest.approx(s1["val_loss"], rel=1e-6)
