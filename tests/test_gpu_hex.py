"""Time stepping on general hexahedral meshes (node coordinates given per
node, box topology) against the oracle.

Parity mode as for the box meshes: the GPU solves to 1e-12 and the oracle to
the FP64 floor; these small terrain-following cases are mass dominated
(heat) or have kappa near 1e3 (pressure), so the FP64 bound is 1e-10
relative; the FP32-refined path is judged at 1e-8 relative (pressure) and
1e-6 K (temperature).  A mesh whose coordinates are the box's own must give
the box mesh's answer (different arithmetic, the same matrices), and graph
replay, batching and eager stepping must agree bit for bit.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import print_case

pytestmark = pytest.mark.gpu


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def run_gpu(hts, scn, steps, **opt):
    o = hts.default_opts(**opt)
    m = hts.from_scenario(scn, opts=o)
    stats = []
    for _ in range(steps):
        code, st = m.solve_step(scn.dt, o)
        stats.append(st)
    return m, m.get_state(0)[0], m.get_state(1)[0], stats


def box_coords(scn):
    ax = [scn.origin[d] + scn.extent[d] * np.arange(n + 1) / n for d, n in enumerate(scn.ncells)]
    Z, Y, X = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    return np.stack([X.reshape(-1), Y.reshape(-1), Z.reshape(-1)], axis=1)


@pytest.mark.parametrize("mode", [0, 1])
def test_terrain_aquifer_small_steps(hts, mode):
    print_case("hex terrain aquifer mode", mode)
    scn = synth.aquifer_hex(ncells=(24, 20, 8), n_steps=2)
    m, P, T, stats = run_gpu(hts, scn, 2, rtol=1e-12, mode=mode)
    Po, To, _ = oracle.run(scn, n_steps=2)
    print("stats", stats)
    for st in stats:
        assert st["status"] == [0, 0], st
    if mode == 0:
        assert rel(P, Po) <= 1e-10
        assert rel(T, To) <= 1e-10
        assert np.abs(T - To).max() <= 1e-7
    else:
        assert rel(P, Po) <= 1e-8
        assert np.abs(T - To).max() <= 1e-6


def test_box_coordinates_give_the_box_answer(hts):
    print_case("hex box coordinates vs box mesh")
    scn = synth.aquifer_hex(ncells=(20, 16, 6), n_steps=2)
    scn.coords = box_coords(scn)
    _, P, T, _ = run_gpu(hts, scn, 2, rtol=1e-12)
    scn.coords = None
    _, Pb, Tb, _ = run_gpu(hts, scn, 2, rtol=1e-12)
    assert rel(P, Pb) <= 1e-10
    assert np.abs(T - Tb).max() <= 1e-7


@pytest.mark.parametrize("mode", [0, 1])
def test_graph_replay_matches_eager(hts, mode):
    print_case("hex graph replay mode", mode)
    scn = synth.aquifer_hex(ncells=(20, 16, 6), n_steps=3)
    out = []
    for g in (0, 1):
        o = hts.default_opts(rtol=1e-10, mode=mode, use_graph=g)
        m = hts.from_scenario(scn, opts=o)
        for _ in range(3):
            m.solve_step(scn.dt, o)
        out.append((m.get_state(0)[0], m.get_state(1)[0]))
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1])


def test_batched_equals_solo(hts):
    print_case("hex batch vs solo")
    scns = [synth.aquifer_hex(seed=s, ncells=n, n_steps=2)
            for s, n in ((1, (16, 12, 6)), (2, (24, 20, 8)), (3, (20, 18, 5)))]
    o = hts.default_opts(rtol=1e-10)
    ms = [hts.from_scenario(s, opts=o) for s in scns]
    code, _ = hts.advance(ms, 2, scns[0].dt, o)
    assert code == 0
    for s, m in zip(scns, ms):
        solo = hts.from_scenario(s, opts=o)
        hts.advance([solo], 2, s.dt, o)
        assert np.array_equal(solo.get_state(0)[0], m.get_state(0)[0])
        assert np.array_equal(solo.get_state(1)[0], m.get_state(1)[0])


def test_hex_and_box_meshes_do_not_share_a_batch(hts):
    print_case("hex + box batch refused")
    a = synth.aquifer_hex(ncells=(8, 8, 4), n_steps=1)
    b = synth.aquifer_hex(ncells=(8, 8, 4), n_steps=1)
    b.coords = None
    o = hts.default_opts()
    ms = [hts.from_scenario(a, opts=o), hts.from_scenario(b, opts=o)]
    with pytest.raises(hts.HtsError, match="general hexahedral"):
        hts.advance(ms, 1, a.dt, o)


def test_line_terms_refused(hts):
    print_case("hex line terms refused")
    scn = synth.aquifer_hex(ncells=(8, 8, 4), n_steps=1)
    m = hts.from_scenario(scn)
    with pytest.raises(hts.HtsError, match="box mesh"):
        m.add_line_source(250.0, 250.0, 20.0, 80.0, hts.LINE_HEAT, synth.timefn(10.0))
