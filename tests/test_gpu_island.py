"""Site-style boundary data on the GPU (Section 3.3): seasonal surface
temperature, geothermal Neumann inflow at the bottom, square-wave pile
temperatures, hydrostatic pressure with a lateral gradient, and the soil
table's hydraulic conductivity and bulk thermal values.

Parity with the oracle as in the other solver tests: the GPU solves to 1e-12
and the oracle to the FP64 floor; FP64 within 1e-10 relative, the
FP32-refined path within 1e-8 (pressure) and 1e-6 K (temperature).
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import print_case
from test_oracle_pins import geotherm_exact, geotherm_scn

pytestmark = pytest.mark.gpu


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("p", [1, 2])
def test_layered_geotherm_fixed_point(hts, p):
    """A step from the steady layered geotherm returns it (the Neumann
    inflow balances conduction exactly in the finite element space)."""
    n = (12, 8, 16) if p == 1 else (6, 4, 8)
    print_case("geotherm fixed point p", p, n)
    s = geotherm_scn(p, n=n)
    o = hts.default_opts(rtol=1e-13)
    m = hts.from_scenario(s, opts=o)
    om = oracle.Mesh.of(s)
    X, Y, Z = om.coords()
    T0 = geotherm_exact(Z)
    m.set_state(1, T0, s.t0)
    code, st = m.solve_step(s.dt, o)
    T1, _ = m.get_state(1)
    assert st["status"] == [0, 0], st
    assert np.abs(T1 - T0).max() <= 1e-9


@pytest.mark.parametrize("ncells,degree,mode", [((32, 20, 8), 1, 0), ((32, 20, 8), 1, 1),
                                                ((40, 25, 10), 1, 0), ((16, 10, 4), 2, 0)])
def test_island_small_steps(hts, ncells, degree, mode):
    """Three daily steps of the island-style pile field against the oracle."""
    print_case("island", ncells, "p", degree, "mode", mode)
    scn = synth.island(ncells=ncells, degree=degree, n_steps=3)
    o = hts.default_opts(rtol=1e-12, mode=mode)
    m = hts.from_scenario(scn, opts=o)
    stats = []
    for _ in range(3):
        code, st = m.solve_step(scn.dt, o)
        stats.append(st)
    P, t = m.get_state(0)
    T, _ = m.get_state(1)
    Po, To, to = oracle.run(scn, n_steps=3)
    print("stats", stats)
    assert t == pytest.approx(to)
    for st in stats:
        assert st["status"] == [0, 0], st
    # the piles are at their summer temperature and the column is warming
    assert T.max() == pytest.approx(288.55 + 13.0)
    if mode == 0:
        assert rel(P, Po) <= 1e-10
        assert rel(T, To) <= 1e-10
        assert np.abs(T - To).max() <= 1e-7
    else:
        assert rel(P, Po) <= 1e-8
        assert np.abs(T - To).max() <= 1e-6


# ------------------------------------------------ graded (rectilinear) meshes
@pytest.mark.parametrize("mode", [0, 1])
def test_island_graded_small_steps(hts, mode):
    """Three steps of the island field on a mesh refined around the building
    footprints and over the pile depth (Fig. 10b style grading)."""
    print_case("island graded mode", mode)
    scn = synth.island(ncells=(32, 20, 10), n_steps=3, graded=True)
    o = hts.default_opts(rtol=1e-12, mode=mode)
    m = hts.from_scenario(scn, opts=o)
    for _ in range(3):
        code, st = m.solve_step(scn.dt, o)
        assert st["status"] == [0, 0], st
    P, t = m.get_state(0)
    T, _ = m.get_state(1)
    Po, To, to = oracle.run(scn, n_steps=3)
    if mode == 0:
        assert rel(P, Po) <= 1e-10
        assert rel(T, To) <= 1e-10
        assert np.abs(T - To).max() <= 1e-7
    else:
        assert rel(P, Po) <= 1e-8
        assert np.abs(T - To).max() <= 1e-6


def test_graded_well_pair_steps(hts):
    """The layered aquifer's well pair (injection-line operator) on graded
    cells, refined around the wells; the separable heat preconditioner too."""
    print_case("c2 graded well pair")
    scn = synth.config2(ncells=(24, 20, 10), n_steps=2)
    scn.edges = (synth.graded_edges(0.0, 500.0, 24, [(120.0, 380.0)], ratio=4.0),
                 synth.graded_edges(0.0, 500.0, 20, [(200.0, 300.0)]),
                 synth.graded_edges(0.0, 100.0, 10, [(60.0, 100.0)], ratio=2.0))
    Po, To, to = oracle.run(scn, n_steps=2)
    for hp in (1, 2):
        o = hts.default_opts(rtol=1e-12, heat_precond=hp)
        m = hts.from_scenario(scn, opts=o)
        for _ in range(2):
            code, st = m.solve_step(scn.dt, o)
            assert st["status"] == [0, 0], st
        P, _ = m.get_state(0)
        T, _ = m.get_state(1)
        assert rel(P, Po) <= 1e-10
        assert rel(T, To) <= 1e-10


def test_graded_geotherm_fixed_point(hts):
    """The layered geotherm on graded cells stays fixed on the GPU too."""
    from test_oracle_pins import GEO_LAYERS
    print_case("graded geotherm")
    gx, gy = np.array([0.0, 4.0, 13.0, 30.0]), np.array([0.0, 15.0, 20.0])
    gz = np.array([0.0, 3.0, 15.0, 19.0, 30.0, 31.0, 36.0, 40.0])
    s = geotherm_scn(1, n=(3, 2, 7))
    s.edges = (gx, gy, gz)
    zc = 0.5 * (gz[1:] + gz[:-1])[np.arange(s.ncell) // 6]
    s.lambda_bulk = np.select([zc < a[1] for a in GEO_LAYERS], [a[2] for a in GEO_LAYERS])
    o = hts.default_opts(rtol=1e-13)
    m = hts.from_scenario(s, opts=o)
    X, Y, Z = oracle.Mesh.of(s).coords()
    T0 = geotherm_exact(Z)
    m.set_state(1, T0, s.t0)
    code, st = m.solve_step(s.dt, o)
    T1, _ = m.get_state(1)
    assert st["status"] == [0, 0], st
    assert np.abs(T1 - T0).max() <= 1e-9


@pytest.mark.parametrize("p", [1, 2])
def test_graded_and_uniform_meshes_in_one_batch(hts, p):
    """A batch mixing a graded and a uniform mesh launches the graded kernel
    instances for both; each instance still gives its solo answer bit for
    bit."""
    print_case("graded + uniform batch p", p)
    q = 3 - p   # degree 2: half the cells per axis
    scns = [synth.island(ncells=(12 * q, 8 * q, 4 * q), n_steps=2, graded=True, degree=p),
            synth.island(ncells=(10 * q, 6 * q, 4 * q), n_steps=2, degree=p)]
    o = hts.default_opts(rtol=1e-10)
    solo = []
    for s in scns:
        m = hts.from_scenario(s, opts=o)
        hts.advance([m], 2, s.dt, o)
        solo.append((m.get_state(0)[0], m.get_state(1)[0]))
    ms = [hts.from_scenario(s, opts=o) for s in scns]
    hts.advance(ms, 2, scns[0].dt, o)
    for m, (P, T) in zip(ms, solo):
        assert np.array_equal(m.get_state(0)[0], P)
        assert np.array_equal(m.get_state(1)[0], T)


@pytest.mark.parametrize("p", [1, 2])
def test_graded_graph_replay_matches_eager(hts, p):
    """Captured-graph replay on a graded mesh gives the eager answer bit for
    bit (both precisions of the inner solves)."""
    print_case("graded graph replay p", p)
    q = 3 - p
    scn = synth.island(ncells=(12 * q, 8 * q, 4 * q), n_steps=3, graded=True, degree=p)
    for mode in (0, 1):
        out = []
        for g in (0, 1):
            o = hts.default_opts(rtol=1e-10, mode=mode, use_graph=g)
            m = hts.from_scenario(scn, opts=o)
            for _ in range(3):
                code, st = m.solve_step(scn.dt, o)
                assert st["status"] == [0, 0], st
            out.append((m.get_state(0)[0], m.get_state(1)[0]))
        assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


@pytest.mark.parametrize("mode", [0, 1])
def test_island_q2_graded_steps(hts, mode):
    """The graded island on 27-node cells (mid-edge nodes at the cell
    midpoints): three steps against the oracle."""
    print_case("island q2 graded mode", mode)
    scn = synth.island(ncells=(16, 10, 5), n_steps=3, degree=2, graded=True)
    o = hts.default_opts(rtol=1e-12, mode=mode)
    m = hts.from_scenario(scn, opts=o)
    for _ in range(3):
        code, st = m.solve_step(scn.dt, o)
        assert st["status"] == [0, 0], st
    P, _ = m.get_state(0)
    T, _ = m.get_state(1)
    Po, To, to = oracle.run(scn, n_steps=3)
    if mode == 0:
        assert rel(P, Po) <= 1e-10
        assert rel(T, To) <= 1e-10
    else:
        assert rel(P, Po) <= 1e-8
        assert np.abs(T - To).max() <= 1e-6


@pytest.mark.parametrize("mode", [0, 1])
def test_graded_q2_column_at_midpoint(hts, mode):
    """A Dirichlet column on degree-2 graded axes lands on the nearest node,
    which is a cell midpoint here (x = 0.7 -> 0.65); one step against the
    oracle."""
    from test_oracle_pins import small_scn
    print_case("graded q2 column at a midpoint, mode", mode)
    s = small_scn(n=(4, 3, 3), p=2)
    s.edges = (np.array([0.0, 0.3, 1.0, 2.2, 3.0]), np.array([0.0, 1.0, 5.0, 8.0]),
               np.array([0.0, 0.1, 0.5, 1.0]))
    s.dir_columns = [synth.DirColumn(synth.TEMPERATURE, 0.7, 3.0, 0.0, 1.0, synth.timefn(300.0))]
    Po, To, _ = oracle.run(s, n_steps=1)
    o = hts.default_opts(rtol=1e-12, mode=mode)
    m = hts.from_scenario(s, opts=o)
    code, st = m.solve_step(s.dt, o)
    assert st["status"] == [0, 0], st
    T, _ = m.get_state(1)
    X, Y, Z = oracle.Mesh.of(s).coords()
    assert np.all(T[(X == 0.65) & (Y == 3.0)] == 300.0)
    if mode == 0:
        assert rel(T, To) <= 1e-10 and np.abs(T - To).max() <= 1e-7
    else:
        assert np.abs(T - To).max() <= 1e-6
