"""Solver parity of the HIP time stepping with the oracle.

Parity mode: the GPU solves to a tight residual (1e-12) and the oracle solves
to the FP64 floor.  Forward error <= kappa * residual, and these small cases
have kappa well below 1e2 (heat, mass dominated) or about 1e3 (pressure), so
the FP64 bound is 1e-10 relative.  The mixed-precision path is judged by the
same true FP64 residual; its bounds are 1e-6 K (temperature, max abs) and
1e-8 relative (pressure).  The backward error of every GPU answer is also
checked in the oracle's own CSR matrices.
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
    P, t = m.get_state(0)
    T, _ = m.get_state(1)
    return m, P, T, t, stats


def test_c1_steady_pressure_exact(hts):
    print_case("c1 steady pressure")
    scn = synth.config1()
    m = hts.from_scenario(scn, opts=hts.default_opts(rtol=1e-13))
    P, _ = m.get_state(0)
    om = oracle.Mesh.of(scn)
    X, Y, Z = om.coords()
    Pex = 1e5 + scn.rho_w * scn.g * (100.0 - Z) + 1e4 * (1.0 - X / 100.0)
    assert np.abs(P - Pex).max() <= 1e-10 * np.abs(Pex).max()


def test_c1_full_run_fp64(hts):
    print_case("c1 full run fp64")
    scn = synth.config1()
    m, P, T, t, stats = run_gpu(hts, scn, scn.n_steps, rtol=1e-13)
    Po, To, to = oracle.run(scn)
    print("stats", stats[0], stats[-1])
    assert t == pytest.approx(to)
    assert rel(P, Po) <= 1e-10
    assert rel(T, To) <= 1e-10
    assert np.abs(T - To).max() <= 1e-8
    for st in stats:
        assert st["status"] == [0, 0]
        assert st["relres"][1] <= 1e-13


@pytest.mark.parametrize("mode", [0, 1])
def test_c2_small_steps(hts, mode):
    """Layered aquifer with a well pair, coarse grid, 3 steps."""
    print_case("c2 small mode", mode)
    scn = synth.config2(ncells=(24, 24, 12), n_steps=3)
    rtol = 1e-12 if mode == 0 else 1e-12
    m, P, T, t, stats = run_gpu(hts, scn, 3, rtol=rtol, mode=mode)
    Po, To, to = oracle.run(scn, n_steps=3)
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


def test_backward_error_in_oracle_matrices(hts):
    """The oracle's own CSR residual of the GPU answer meets the tolerance."""
    print_case("backward error")
    scn = synth.config2(ncells=(20, 16, 10), n_steps=1)
    o = hts.default_opts(rtol=1e-8)
    m = hts.from_scenario(scn, opts=o)
    P0, _ = m.get_state(0)
    T0, _ = m.get_state(1)
    code, st = m.solve_step(scn.dt, o)
    P1, _ = m.get_state(0)
    T1, _ = m.get_state(1)
    om = oracle.Mesh.of(scn)
    t1 = scn.t0 + scn.dt
    A, b = oracle.pressure_system(scn, om, P0, t1)
    mask, g = oracle.dirichlet(scn, om, 0, t1)
    free, AFF, bF = oracle.eliminate(A, b, mask, g)
    r = oracle.residual_ld(AFF, bF, P1[free])
    assert np.linalg.norm(r) <= 1.0001e-8 * np.linalg.norm(bF)
    assert np.abs(P1[mask] - g[mask]).max() == 0.0
    H, hb = oracle.heat_system(scn, om, T0, P1, t1)
    mask, g = oracle.dirichlet(scn, om, 1, t1)
    free, HFF, hF = oracle.eliminate(H, hb, mask, g)
    r = oracle.residual_ld(HFF, hF, T1[free])
    assert np.linalg.norm(r) <= 1.0001e-8 * np.linalg.norm(hF)


def test_c4_instance_dirichlet_columns(hts):
    print_case("c4 instance")
    scn = synth.config4_instance(5, n_override=16, n_steps=2)
    m, P, T, t, stats = run_gpu(hts, scn, 2, rtol=1e-12)
    Po, To, to = oracle.run(scn, n_steps=2)
    print("stats", stats)
    assert rel(P, Po) <= 1e-10
    assert rel(T, To) <= 1e-10
    assert np.abs(T - To).max() <= 1e-7


def test_c3_small_piles(hts):
    print_case("c3 small")
    scn = synth.config3(ncells=(24, 24, 12), n_steps=2)
    m, P, T, t, stats = run_gpu(hts, scn, 2, rtol=1e-12)
    Po, To, to = oracle.run(scn, n_steps=2)
    print("stats", stats)
    assert rel(P, Po) <= 1e-10
    assert rel(T, To) <= 1e-10
    assert np.abs(T - To).max() <= 1e-7


@pytest.mark.parametrize("mode", [0, 1])
def test_c3_q2_small_piles(hts, mode):
    """Q2 variant of the pile field (27-node cells, 3-point Gauss)."""
    print_case("c3 q2 small mode", mode)
    scn = synth.config3(degree=2, ncells=(12, 12, 6), n_steps=2)
    m, P, T, t, stats = run_gpu(hts, scn, 2, rtol=1e-12, mode=mode)
    Po, To, to = oracle.run(scn, n_steps=2)
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


def test_c2_q2_well_pair(hts):
    """Q2 layered aquifer with the injection/extraction wells (line operator
    of the injection enthalpy term on 27-node cells)."""
    print_case("c2 q2 small")
    scn = synth.config2(ncells=(14, 12, 6), n_steps=2)
    scn.degree = 2
    m, P, T, t, stats = run_gpu(hts, scn, 2, rtol=1e-12)
    Po, To, to = oracle.run(scn, n_steps=2)
    print("stats", stats)
    assert rel(P, Po) <= 1e-10
    assert rel(T, To) <= 1e-10
    assert np.abs(T - To).max() <= 1e-7


@pytest.mark.parametrize("B", [1e5, 1e9])
def test_q2_multigrid_rate(hts, B):
    """The Q2 -> Q1 p-multigrid keeps a mesh-independent rate whatever the
    scale of the operator (regression: residual restricted onto eliminated
    Dirichlet vertices of the Q1 level was injected back as a correction)."""
    print_case("q2 multigrid rate B", B)
    scn = synth.config2(ncells=(14, 12, 6), n_steps=1)
    scn.degree, scn.B_poro = 2, B
    for hp in (0, 1):
        o = hts.default_opts(rtol=1e-8, heat_precond=hp)
        m = hts.from_scenario(scn, opts=o)
        code, st = m.solve_step(scn.dt, o)
        print("heat_precond", hp, st)
        assert st["iters"][0] <= 20
        assert st["iters"][1] <= 30


@pytest.mark.parametrize("mode,hp", [(0, 1), (1, 1), (0, 0)])
def test_graph_replay_matches_eager_bitwise(hts, mode, hp):
    """Captured Krylov chunks replayed over several steps (with the eager
    right-hand sides, outer corrections and host checks between replays)
    give exactly the eager answer, step after step."""
    print_case("graph replay mode", mode, "heat_precond", hp)
    scn = synth.config2(ncells=(24, 20, 10), n_steps=4)
    res = []
    for g in (0, 1):
        o = hts.default_opts(rtol=1e-10, mode=mode, heat_precond=hp, use_graph=g)
        m = hts.from_scenario(scn, opts=o)
        states = []
        for _ in range(4):
            code, st = m.solve_step(scn.dt, o)
            states.append((m.get_state(0)[0], m.get_state(1)[0], st["iters"]))
        res.append(states)
    for (P0, T0, i0), (P1, T1, i1) in zip(*res):
        assert i0 == i1
        assert np.array_equal(P0, P1)
        assert np.array_equal(T0, T1)


def test_graph_replay_batched(hts):
    """Batched instances of uneven size advance identically with and without
    captured graphs."""
    print_case("graph replay batched")
    scns = [synth.config4_instance(i, n_override=n, n_steps=3) for i, n in [(0, 12), (1, 17), (2, 9)]]
    out = []
    for g in (0, 1):
        o = hts.default_opts(rtol=1e-10, use_graph=g)
        ms = [hts.from_scenario(s, opts=o) for s in scns]
        hts.advance(ms, 3, scns[0].dt, o)
        out.append([(m.get_state(0)[0], m.get_state(1)[0]) for m in ms])
    for (P0, T0), (P1, T1) in zip(*out):
        assert np.array_equal(P0, P1)
        assert np.array_equal(T0, T1)


@pytest.mark.parametrize("mode", [0, 1])
def test_tensor_mass_heat_preconditioner(hts, mode):
    """The separable mass preconditioner for the heat solve gives the oracle's
    answer (FP64 1e-10, mixed 1e-6 K) in fewer iterations than
    Chebyshev-Jacobi, also with Dirichlet pile columns in a batch."""
    print_case("tensor mass mode", mode)
    scn = synth.config2(ncells=(24, 24, 12), n_steps=3)
    m, P, T, t, stats = run_gpu(hts, scn, 3, rtol=1e-12, mode=mode, heat_precond=2)
    _, _, _, _, st_cheb = run_gpu(hts, scn, 3, rtol=1e-12, mode=mode, heat_precond=1)
    Po, To, to = oracle.run(scn, n_steps=3)
    print("tensor", stats, "cheb", st_cheb)
    if mode == 0:
        assert rel(T, To) <= 1e-10
    assert np.abs(T - To).max() <= (1e-7 if mode == 0 else 1e-6)
    assert sum(s["iters"][1] for s in stats) < sum(s["iters"][1] for s in st_cheb)
    scns = [synth.config4_instance(i, n_override=n, n_steps=2) for i, n in [(0, 12), (1, 17)]]
    o = hts.default_opts(rtol=1e-12, mode=mode, heat_precond=2)
    ms = [hts.from_scenario(sc, opts=o) for sc in scns]
    hts.advance(ms, 2, scns[0].dt, o)
    for mm, sc in zip(ms, scns):
        Po, To, _ = oracle.run(sc, n_steps=2)
        assert np.abs(mm.get_state(1)[0] - To).max() <= (1e-7 if mode == 0 else 1e-6)


def test_not_converged_is_transactional(hts):
    print_case("transactional")
    scn = synth.config2(ncells=(16, 16, 8), n_steps=1)
    o = hts.default_opts(rtol=1e-8)
    m = hts.from_scenario(scn, opts=o)
    P0, t0 = m.get_state(0)
    T0, _ = m.get_state(1)
    bad = hts.default_opts(rtol=1e-14, max_iter=1)
    code, st = m.solve_step(scn.dt, bad, raise_on_error=False)
    assert code == -5
    P1, t1 = m.get_state(0)
    T1, _ = m.get_state(1)
    assert t1 == t0 and np.array_equal(P1, P0) and np.array_equal(T1, T0)
    # a good step afterwards still works
    code, st = m.solve_step(scn.dt, o)
    assert code == 0


def test_batched_equals_solo_bitwise(hts):
    print_case("batched == solo")
    scns = [synth.config4_instance(i, n_override=n, n_steps=2) for i, n in [(0, 12), (1, 17), (2, 9)]]
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


def test_cached_batch_is_dropped_when_a_mesh_changes(hts):
    """hts_advance keeps the batch of a mesh list between calls; changing a
    member's boundary data must rebuild it.  Two calls of one step equal one
    call of two steps bit for bit, and after a change the batch answers like
    freshly created meshes with the new data."""
    print_case("batch cache")
    scns = [synth.config4_instance(i, n_override=n, n_steps=3) for i, n in [(0, 12), (1, 9)]]
    o = hts.default_opts(rtol=1e-10)
    a = [hts.from_scenario(s, opts=o) for s in scns]
    b = [hts.from_scenario(s, opts=o) for s in scns]
    hts.advance(a, 2, scns[0].dt, o)
    hts.advance(b, 1, scns[0].dt, o)
    hts.advance(b, 1, scns[0].dt, o)
    for ma, mb in zip(a, b):
        assert np.array_equal(ma.get_state(1)[0], mb.get_state(1)[0])
    # a new Dirichlet face on the second mesh, then one more step
    hot = synth.timefn(330.0)
    b[1].set_face_bc(synth.TEMPERATURE, 5, synth.DIRICHLET, hot)
    hts.advance(b, 1, scns[0].dt, o)
    s1 = scns[1]
    s1.bcs = list(s1.bcs) + [synth.FaceBC(synth.TEMPERATURE, 5, synth.DIRICHLET, hot)]
    c = [hts.from_scenario(scns[0], opts=o), hts.from_scenario(s1, opts=o)]
    for m, src in zip(c, a):
        for f in (0, 1):
            m.set_state(f, src.get_state(f)[0], src.get_state(f)[1])
            for level in (1, 2):
                m.set_previous_state(f, *src.get_previous_state(f, level), level=level)
    # the unchanged mesh keeps the heat preconditioner's estimates of its
    # first step; the changed one estimates again (as its fresh copy does)
    c[0].set_heat_spectrum(a[0].get_heat_spectrum())
    hts.advance(c, 1, scns[0].dt, o)
    for mb, mc in zip(b, c):
        assert np.array_equal(mb.get_state(0)[0], mc.get_state(0)[0])
        assert np.array_equal(mb.get_state(1)[0], mc.get_state(1)[0])
    T1 = b[1].get_state(1)[0]
    assert np.isclose(T1.max(), 330.0)


def test_heat_spectral_estimates_against_the_oracle(hts):
    """The heat preconditioner's estimates after one step: the largest
    eigenvalue of D^-1 A without convection and the imaginary extent of the
    convection part, D^-1 (A - A_0) (A_0 the operator with the Darcy flux
    removed), against the oracle's matrices (ARPACK on the assembled,
    eliminated systems).  Power iteration approaches the extremes from
    below; the bounds leave room for its 12 steps."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    print_case("heat spectrum vs oracle")
    scn = synth.config2(ncells=(24, 24, 12), n_steps=1)
    o = hts.default_opts(rtol=1e-10)
    m = hts.from_scenario(scn, opts=o)
    P0, _ = m.get_state(0)
    T0, _ = m.get_state(1)
    assert m.solve_step(scn.dt, o)[0] == 0
    dt_s, lsym, lfull, beta = m.get_heat_spectrum()
    assert dt_s == scn.dt
    P1, _ = m.get_state(0)
    om = oracle.Mesh.of(scn)
    t1 = scn.t0 + scn.dt
    X, Y, Z = om.coords()
    Phyd = P1[0] + scn.rho_w * scn.g * (Z[0] - Z)       # no Darcy flux
    H, hb = oracle.heat_system(scn, om, T0, P1, t1)
    H0, _ = oracle.heat_system(scn, om, T0, Phyd, t1)
    mask, g = oracle.dirichlet(scn, om, 1, t1)
    free, HF, _ = oracle.eliminate(H, hb, mask, g)
    _, H0F, _ = oracle.eliminate(H0, hb, mask, g)
    dinv = sp.diags(1.0 / H0F.diagonal())
    ls = abs(spla.eigs(dinv @ H0F, k=1, which="LM", return_eigenvectors=False)[0])
    C = dinv @ (HF - H0F)
    b_ex = abs(spla.eigs(C, k=1, which="LM", return_eigenvectors=False)[0])
    print("lmax symmetric %.5g (oracle %.5g), imaginary extent %.5g (oracle %.5g)" % (lsym, ls, beta, b_ex))
    assert 0.9 * ls <= lsym <= 1.02 * ls
    assert 0.8 * b_ex <= beta <= 1.05 * b_ex
