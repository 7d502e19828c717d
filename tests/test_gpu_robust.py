"""Failure handling and resumption of the time step (transactional steps).

* A non-finite right-hand side (a NaN in the volume heat source, which the
  library copies as given) makes the heat solve break down: the step returns
  HTS_ERR_BREAKDOWN and neither field nor the time advances, in FP64 and in
  FP32-refined mode.
* Checkpoint / resume: the state, the two previous time levels and the heat
  preconditioner's spectral estimates read back after three steps and set
  on a fresh mesh of the same scenario continue bit for bit like the
  uninterrupted run.
* Changing the time-step size keeps at most two pressure multigrid
  hierarchies; steps that alternate between three sizes give the same bits
  as fresh meshes that only ever see one size (given the same two levels).
* The extrapolated initial guess: the previous levels are the states one
  and two steps earlier, setting a state forgets them (the next step is
  then the plain one bit for bit), and extrapolated steps meet the same
  residual test in fewer iterations, with answers within the solver
  tolerance of the plain ones.
"""
import numpy as np
import pytest

import synth
from gpu_util import print_case

pytestmark = pytest.mark.gpu

NC = (24, 20, 12)


def copy_levels(dst, src):
    """The previous time levels of src, set on dst (level 1 first)."""
    for f in (0, 1):
        for level in (1, 2):
            dst.set_previous_state(f, *src.get_previous_state(f, level), level=level)


def scenario(n_steps=6):
    return synth.config2(ncells=NC, n_steps=n_steps)


@pytest.mark.parametrize("mode", [0, 1])
def test_nan_source_is_breakdown_and_state_unchanged(hts, mode):
    print_case("nan source breakdown, mode", mode)
    s = scenario()
    o = hts.default_opts(mode=mode, rtol=1e-8)
    m = hts.from_scenario(s, opts=o)
    code, _ = m.solve_step(s.dt, o)
    assert code == 0
    P, tP = m.get_state(0)
    T, tT = m.get_state(1)
    src = np.zeros(s.ncell)
    src[s.ncell // 2] = np.nan
    m.set_volume_source(src)
    code, st = m.solve_step(s.dt, o, raise_on_error=False)
    assert code == -6, (code, st)
    P2, tP2 = m.get_state(0)
    T2, tT2 = m.get_state(1)
    assert np.array_equal(P, P2) and np.array_equal(T, T2) and tP == tP2 and tT == tT2
    # a finite source again: the step goes through from the kept state
    m.set_volume_source(np.zeros(s.ncell))
    code, st = m.solve_step(s.dt, o)
    assert code == 0 and max(st["relres"]) <= 1e-8


@pytest.mark.parametrize("mode", [0, 1])
def test_checkpoint_resume_is_bit_exact(hts, mode):
    print_case("checkpoint resume, mode", mode)
    s = scenario()
    o = hts.default_opts(mode=mode, rtol=1e-8)
    a = hts.from_scenario(s, opts=o)
    for _ in range(5):
        assert a.solve_step(s.dt, o)[0] == 0
    b = hts.from_scenario(s, opts=o)
    for _ in range(3):
        assert b.solve_step(s.dt, o)[0] == 0
    P, t = b.get_state(0)
    T, _ = b.get_state(1)
    for f in (0, 1):
        for level in (1, 2):
            assert b.get_previous_state(f, level)[1] == s.dt
    spec = b.get_heat_spectrum()
    assert spec[0] == s.dt and spec[1] > 0 and spec[2] > 0
    c = hts.from_scenario(s, initial=False, opts=o)
    c.set_state(0, P, t)
    c.set_state(1, T, t)
    copy_levels(c, b)
    c.set_heat_spectrum(spec)
    del b
    for _ in range(2):
        assert c.solve_step(s.dt, o)[0] == 0
    assert np.array_equal(a.get_state(0)[0], c.get_state(0)[0])
    assert np.array_equal(a.get_state(1)[0], c.get_state(1)[0])
    assert a.get_state(0)[1] == c.get_state(0)[1]


def test_alternating_step_sizes_match_fresh_meshes(hts):
    print_case("dt sequence, hierarchy cache")
    s = scenario()
    o = hts.default_opts(rtol=1e-8)
    dts = [synth.DAY, 0.5 * synth.DAY, 2.0 * synth.DAY, synth.DAY, 0.5 * synth.DAY]
    m = hts.from_scenario(s, opts=o)
    P0, t0 = m.get_state(0)
    T0, _ = m.get_state(1)
    for dt in dts:
        # the same step from the same state on a mesh that only sees this dt
        f = hts.from_scenario(s, initial=False, opts=o)
        P, t = m.get_state(0)
        T, _ = m.get_state(1)
        f.set_state(0, P, t)
        f.set_state(1, T, t)
        copy_levels(f, m)
        assert f.solve_step(dt, o)[0] == 0
        assert m.solve_step(dt, o)[0] == 0
        assert np.array_equal(m.get_state(0)[0], f.get_state(0)[0])
        assert np.array_equal(m.get_state(1)[0], f.get_state(1)[0])
        del f


@pytest.mark.parametrize("mode", [0, 1])
def test_extrapolated_initial_guess(hts, mode):
    print_case("extrapolated initial guess, mode", mode)
    s = scenario(n_steps=6)
    ox = hts.default_opts(mode=mode, rtol=1e-8)
    op = hts.default_opts(mode=mode, rtol=1e-8, extrapolate=0)
    a = hts.from_scenario(s, opts=ox)
    b = hts.from_scenario(s, opts=op)
    assert a.get_previous_state(0) == (None, 0.0)
    its = {0: [0, 0], 1: [0, 0]}
    P_older = None
    for k in range(6):
        P_before = a.get_state(0)[0]
        ca, sa = a.solve_step(s.dt, ox)
        cb, sb = b.solve_step(s.dt, op)
        assert ca == 0 and cb == 0 and max(sa["relres"]) <= 1e-8 and max(sb["relres"]) <= 1e-8
        # the previous level is the state one step earlier, bit for bit
        Pp, dtp = a.get_previous_state(0)
        assert dtp == s.dt and np.array_equal(Pp, P_before)
        Ppp, dtpp = a.get_previous_state(0, 2)
        if P_older is None:
            assert Ppp is None and dtpp == 0.0
        else:
            assert dtpp == s.dt and np.array_equal(Ppp, P_older)
        P_older = P_before
        if k >= 2:
            for f in (0, 1):
                its[f][0] += sa["iters"][f]
                its[f][1] += sb["iters"][f]
        # both answers solve the same systems to 1e-8: they agree to about
        # that relative level (kappa ~ 1e3 for pressure)
        for f in (0, 1):
            x, y = a.get_state(f)[0], b.get_state(f)[0]
            assert np.linalg.norm(x - y) <= 1e-6 * np.linalg.norm(y)
    print("iterations over steps 3-6 (extrapolated, plain):", its)
    assert its[0][0] + its[1][0] < its[0][1] + its[1][1]
    # setting the state forgets the previous level: the next step is the
    # plain step from that state
    c = hts.from_scenario(s, initial=False, opts=ox)
    d = hts.from_scenario(s, initial=False, opts=op)
    for m in (c, d):
        for f in (0, 1):
            m.set_state(f, *a.get_state(f))
    assert c.get_previous_state(1) == (None, 0.0)
    assert c.solve_step(s.dt, ox)[0] == 0 and d.solve_step(s.dt, op)[0] == 0
    for f in (0, 1):
        assert np.array_equal(c.get_state(f)[0], d.get_state(f)[0])


@pytest.mark.parametrize("mode", [0, 1])
def test_extrapolation_is_exact_for_quadratic_histories(hts, mode):
    """Previous levels set on a quadratic in time through the state S and the
    answer P* of the next step (any step sizes): the quadratic extrapolation
    (Lagrange form at t^n - h1 - h2, t^n - h1, t^n) reproduces P*, so the
    pressure solve starts converged; with level 2 forgotten, levels on a
    line through S and P* do the same for the linear extrapolation."""
    print_case("exact extrapolation, mode", mode)
    s = scenario(n_steps=2)
    o = hts.default_opts(mode=mode, rtol=1e-8)
    a = hts.from_scenario(s, opts=o)
    S, t0 = a.get_state(0)
    T0, _ = a.get_state(1)
    assert a.solve_step(s.dt, o)[0] == 0
    Pstar = a.get_state(0)[0]
    dt, h1, h2 = s.dt, 0.7 * s.dt, 1.6 * s.dt
    rng = np.random.default_rng(4)
    # X(tau) = S + alpha tau + beta tau^2 with X(dt) = P*
    beta = 0.3 * (Pstar - S) / dt ** 2 * rng.uniform(0.5, 1.5, S.size)
    alpha = (Pstar - S - beta * dt ** 2) / dt
    X = lambda tau: S + alpha * tau + beta * tau ** 2
    for levels in (2, 1):
        b = hts.from_scenario(s, initial=False, opts=o)
        b.set_state(0, S, t0)
        b.set_state(1, T0, t0)
        if levels == 2:
            b.set_previous_state(0, X(-h1), h1, level=1)
            b.set_previous_state(0, X(-h1 - h2), h2, level=2)
        else:
            lin = lambda tau: S + (Pstar - S) / dt * tau
            b.set_previous_state(0, lin(-h1), h1, level=1)
        code, st = b.solve_step(dt, o)
        assert code == 0, st
        print("levels", levels, "pressure iterations", st["iters"][0], "relres", st["relres"][0])
        assert st["iters"][0] == 0, st
        P = b.get_state(0)[0]
        assert np.linalg.norm(P - Pstar) <= 1e-8 * np.linalg.norm(Pstar)
