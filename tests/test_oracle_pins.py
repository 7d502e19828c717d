"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test ties one part of the oracle to something other than itself:

* element matrices  -> closed-form Kronecker products of the 1D Lagrange
  mass / stiffness / convection matrices (Q1 and Q2);
* global assembly   -> an independent NumPy Kronecker assembly on tiny meshes;
* invariants        -> K 1 = 0, 1^T M 1 = int c, symmetry of the pressure
  matrix, <C x, x> = 0 for a uniform flux with x = 0 on the boundary,
  partition-of-unity sums of the face / line / gravity load vectors;
* pressure Eq. 3 + gravity sign + Darcy flux -> the uniform Darcy-flow case
  (exact linear P_h, q_h = k dp/L at every quadrature point);
* heat Eq. 4 conduction -> a linear steady profile kept exactly by stepping;
* mass + backward Euler -> erfc semi-infinite conduction, O(h^2 + dt);
* advection         -> the Ogata-Banks solution, observed convergence;
* spatial order     -> manufactured solutions: L2 ratio ~4 (Q1), ~8 (Q2);
* balances          -> total stored heat / fluid equals the sources and
  boundary fluxes for insulated boxes;
* injection enthalpy -> one step's stored heat equals h c_w (Q/L) times the
  line integral of (T_inj - T^{n+1}), both evaluated with an independent
  Lagrange basis and Gauss rule; a state at T_inj stays there while the
  well pair drives flow; extraction wells add no heat term;
* solvers           -> sparse LU on small systems.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from scipy.special import erfc, erfcx

import oracle
import synth
from oracle import Mesh

# ---------------------------------------------------------------- 1D forms
def m1(p, h):
    if p == 1:
        return h / 6.0 * np.array([[2.0, 1.0], [1.0, 2.0]])
    return h / 30.0 * np.array([[4.0, 2.0, -1.0], [2.0, 16.0, 2.0], [-1.0, 2.0, 4.0]])


def k1(p, h):
    if p == 1:
        return 1.0 / h * np.array([[1.0, -1.0], [-1.0, 1.0]])
    return 1.0 / (3.0 * h) * np.array([[7.0, -8.0, 1.0], [-8.0, 16.0, -8.0], [1.0, -8.0, 7.0]])


def c1(p):
    """int N_a N_b' over one cell (independent of h)."""
    if p == 1:
        return np.array([[-0.5, 0.5], [-0.5, 0.5]])
    return np.array([[-3.0, 4.0, -1.0], [-4.0, 0.0, 4.0], [1.0, -4.0, 3.0]]) / 6.0


def kron3(ax, ay, az):
    # local numbering a = ax + (p+1)(ay + (p+1) az): z slowest -> kron(z, y, x)
    return np.kron(az, np.kron(ay, ax))


def elem_closed(p, h, cm, cs, beta):
    hx, hy, hz = h
    M = kron3(m1(p, hx), m1(p, hy), m1(p, hz))
    K = (kron3(k1(p, hx), m1(p, hy), m1(p, hz)) + kron3(m1(p, hx), k1(p, hy), m1(p, hz))
         + kron3(m1(p, hx), m1(p, hy), k1(p, hz)))
    Cv = (beta[0] * kron3(c1(p), m1(p, hy), m1(p, hz)) + beta[1] * kron3(m1(p, hx), c1(p), m1(p, hz))
          + beta[2] * kron3(m1(p, hx), m1(p, hy), c1(p)))
    return cm * M + cs * K + Cv


def small_scn(n=(3, 4, 2), p=1, L=(3.0, 8.0, 1.0), seed=0):
    rng = np.random.default_rng(seed)
    nc = n[0] * n[1] * n[2]
    return synth.Scenario("t", (0.0, 0.0, 0.0), L, n, p,
                          permeability=10 ** rng.uniform(-12, -10, nc),
                          porosity=rng.uniform(0.2, 0.35, nc),
                          lambda_solid=np.full(nc, 2.5), rhoc_solid=np.full(nc, 2e6))


# ------------------------------------------------------- element matrices
@pytest.mark.parametrize("p", [1, 2])
def test_element_matrix_kronecker(p):
    m = Mesh((1.0, -2.0, 0.5), (3.0, 8.0, 1.0), (3, 4, 2), p)
    h = (1.0, 2.0, 0.5)
    nc = m.ncell
    rng = np.random.default_rng(1)
    cm, cs = rng.uniform(1, 2, nc), rng.uniform(1, 2, nc)
    for cell in [(0, 0, 0), (2, 3, 1), (1, 2, 0)]:
        c = cell[0] + 3 * (cell[1] + 4 * cell[2])
        Ae = oracle.element_matrix(m, cell, mass=cm, stiff=cs)
        ref = elem_closed(p, h, cm[c], cs[c], (0, 0, 0))
        assert np.allclose(Ae, ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())


@pytest.mark.parametrize("p", [1, 2])
def test_element_advection_uniform_flux(p):
    """P linear and hydrostatic in z: q_h is uniform and the convection
    element matrix is the Kronecker form with beta = scale * q."""
    m = Mesh((0.0, 0.0, 0.0), (3.0, 8.0, 1.0), (3, 4, 2), p)
    X, Y, Z = m.coords()
    rho_g, kk, scale = 9810.0, 2e-9, 3.0
    gx, gy = -700.0, 250.0
    P = 1e5 + gx * X + gy * Y + rho_g * (1.0 - Z)
    k = np.full(m.ncell, kk)
    q = np.array([-kk * gx, -kk * gy, 0.0])
    Ae = oracle.element_matrix(m, (1, 2, 1), kvel=k, P=P, adv_scale=scale, rho_g=rho_g)
    ref = elem_closed(p, (1.0, 2.0, 0.5), 0.0, 0.0, scale * q)
    assert np.allclose(Ae, ref, rtol=1e-11, atol=1e-11 * np.abs(ref).max())


# ----------------------------------------------- independent assembly
def numpy_assembly(m: Mesh, cm, cs, beta):
    """Independent global assembly: Kronecker element matrices + scatter."""
    p = m.p
    n1 = p + 1
    NX, NY, NZ = m.dims
    h = tuple(m.L[d] / m.n[d] for d in range(3))
    rows, cols, vals = [], [], []
    for cz in range(m.n[2]):
        for cy in range(m.n[1]):
            for cx in range(m.n[0]):
                c = cx + m.n[0] * (cy + m.n[1] * cz)
                Ae = elem_closed(p, h, cm[c], cs[c], beta)
                g = [(p * cx + ax) + NX * ((p * cy + ay) + NY * (p * cz + az))
                     for az in range(n1) for ay in range(n1) for ax in range(n1)]
                for a in range(n1 ** 3):
                    for b in range(n1 ** 3):
                        rows.append(g[a]); cols.append(g[b]); vals.append(Ae[a, b])
    return sp.csr_matrix((vals, (rows, cols)), shape=(m.nnode, m.nnode))


@pytest.mark.parametrize("p", [1, 2])
def test_global_assembly_vs_numpy(p):
    m = Mesh((0.0, 0.0, 0.0), (3.0, 8.0, 1.0), (3, 4, 2), p)
    rng = np.random.default_rng(3)
    cm, cs = rng.uniform(1, 2, m.ncell), rng.uniform(1, 2, m.ncell)
    A = oracle.assemble(m, mass=cm, stiff=cs)
    B = numpy_assembly(m, cm, cs, (0, 0, 0))
    assert abs(A - B).max() <= 1e-13 * abs(B).max()


# ------------------------------------------------------------- invariants
@pytest.mark.parametrize("p", [1, 2])
def test_stiffness_kernel_and_mass_total(p):
    s = small_scn(p=p)
    m = Mesh.of(s)
    k, lam, cT = oracle.coefficients(s)
    K = oracle.assemble(m, stiff=k)
    M = oracle.assemble(m, mass=cT)
    one = np.ones(m.nnode)
    assert np.abs(K @ one).max() <= 1e-13 * abs(K).max()
    vol = np.prod(m.L) / m.ncell
    assert math.isclose(one @ (M @ one), vol * cT.sum(), rel_tol=1e-13)
    # pressure matrix symmetric
    A, _ = oracle.pressure_system(s, m, np.zeros(m.nnode), s.dt)
    assert abs(A - A.T).max() <= 1e-13 * abs(A).max()


@pytest.mark.parametrize("p", [1, 2])
def test_convection_skew_for_uniform_flux(p):
    m = Mesh((0.0, 0.0, 0.0), (3.0, 3.0, 3.0), (3, 3, 3), p)
    X, Y, Z = m.coords()
    rho_g, kk = 9810.0, 1e-9
    P = 1e5 - 300.0 * X + 120.0 * Y + rho_g * (3.0 - Z) - 50.0 * Z
    Cm = oracle.assemble(m, kvel=np.full(m.ncell, kk), P=P, adv_scale=4e6, rho_g=rho_g)
    NX, NY, NZ = m.dims
    I = np.arange(m.nnode)
    i, j, kz = I % NX, (I // NX) % NY, I // (NX * NY)
    bnd = (i == 0) | (i == NX - 1) | (j == 0) | (j == NY - 1) | (kz == 0) | (kz == NZ - 1)
    x = np.random.default_rng(4).standard_normal(m.nnode)
    x[bnd] = 0.0
    assert abs(x @ (Cm @ x)) <= 1e-12 * abs(Cm).max() * (x @ x)
    # rows sum to zero: constant fields are not advected
    assert np.abs(Cm @ np.ones(m.nnode)).max() <= 1e-12 * abs(Cm).max()


@pytest.mark.parametrize("p", [1, 2])
def test_load_vector_sums(p):
    m = Mesh((1.0, 2.0, -3.0), (3.0, 8.0, 2.0), (3, 4, 3), p)
    X, Y, Z = m.coords()
    f = np.random.default_rng(5).uniform(1, 2, m.ncell)
    vol = np.prod(m.L) / m.ncell
    assert math.isclose(oracle.load_cell(m, f).sum(), vol * f.sum(), rel_tol=1e-13)
    g = np.random.default_rng(6).uniform(1, 2, m.ncell)
    lg = oracle.load_gradz(m, g)
    assert abs(lg.sum()) <= 1e-13 * np.abs(lg).max()
    assert math.isclose(lg @ Z, vol * g.sum(), rel_tol=1e-12)     # int g d(z)/dz
    areas = [8 * 2, 8 * 2, 3 * 2, 3 * 2, 3 * 8, 3 * 8]
    for face in range(6):
        lf = oracle.load_face(m, face, 2.5)
        assert math.isclose(lf.sum(), 2.5 * areas[face], rel_tol=1e-13)
        # supported on that face only
        coord = [X, X, Y, Y, Z, Z][face]
        target = [1.0, 4.0, 2.0, 10.0, -3.0, -1.0][face]
        assert np.all(np.abs(coord[lf != 0] - target) < 1e-12)
    ll = oracle.load_line(m, 2.3, 5.1, -2.6, -1.2, 3.0)
    assert math.isclose(ll.sum(), 3.0 * 1.4, rel_tol=1e-13)
    assert math.isclose(ll @ Z, 3.0 * 0.5 * ((-1.2) ** 2 - (-2.6) ** 2), rel_tol=1e-12)
    assert math.isclose(ll @ X, 3.0 * 1.4 * 2.3, rel_tol=1e-12)
    Ml = oracle.line_mass(m, 2.3, 5.1, -2.6, -1.2, 3.0)
    one = np.ones(m.nnode)
    assert math.isclose(one @ (Ml @ one), 3.0 * 1.4, rel_tol=1e-13)
    # int z^2 along the line = (z1^3 - z0^3)/3 (exact for p >= 1 on z*z with x=z)
    assert math.isclose(Z @ (Ml @ Z), 3.0 * ((-1.2) ** 3 - (-2.6) ** 3) / 3.0, rel_tol=1e-12)


def test_dirichlet_column_on_node():
    s = synth.config4_instance(0, n_override=20, n_steps=1)
    m = Mesh.of(s)
    mask, g = oracle.dirichlet(s, m, synth.TEMPERATURE, 0.0)
    X, Y, Z = m.coords()
    col = s.dir_columns[0]
    sel = (np.abs(X - col.x) < 1e-9) & (np.abs(Y - col.y) < 1e-9) & (Z >= 170 - 1e-9)
    assert sel.sum() == 4        # z = 170, 180, 190, 200 on a 10 m node spacing
    assert mask[sel].all()
    assert np.allclose(g[sel], col.value[1])


# ---------------------------------------------------------- Darcy, Eq. 3
def test_uniform_darcy_flow_exact():
    """Config-1 pressure: hydrostatic + linear drop is the exact solution;
    q_h = (k dp / L, 0, 0) at every Gauss point (gravity sign, Eq. 3 loads)."""
    s = synth.config1()
    m = Mesh.of(s)
    P, _ = oracle.initial_state(s, m)
    X, Y, Z = m.coords()
    Pex = 1e5 + s.rho_w * s.g * (100.0 - Z) + 1e4 * (1.0 - X / 100.0)
    assert np.abs(P - Pex).max() <= 1e-12 * np.abs(Pex).max()
    k = s.permeability[0] / s.mu_w
    q = oracle.flux_qp(m, 2, np.full(m.ncell, k), P, s.rho_w * s.g)
    assert np.allclose(q[:, :, 0], k * 1e4 / 100.0, rtol=1e-9)
    assert np.abs(q[:, :, 1:]).max() <= 1e-9 * k * 1e4 / 100.0


@pytest.mark.parametrize("p", [1, 2])
def test_transient_pressure_keeps_hydrostatic(p):
    """Hydrostatic pressure is a steady state of Eq. 3 (q = 0)."""
    s = small_scn(p=p)
    s.B_poro = 1e5
    hyd = synth.hydrostatic(1.0, 1e5, s.rho_w, s.g)
    s.bcs = [synth.FaceBC(synth.PRESSURE, 0, synth.DIRICHLET, hyd)]
    m = Mesh.of(s)
    X, Y, Z = m.coords()
    P0 = oracle.tf_value(hyd, X, Y, Z, 0.0)
    P1 = oracle.solve_pressure(s, m, P0, s.dt)
    assert np.abs(P1 - P0).max() <= 1e-11 * np.abs(P0).max()


# ------------------------------------------------------------ heat, Eq. 4
@pytest.mark.parametrize("p", [1, 2])
def test_linear_conduction_profile_exact(p):
    """Linear T between two Dirichlet faces, insulated elsewhere, flux
    perpendicular to the gradient: every step reproduces it exactly."""
    n = (6, 3, 2)
    nc = np.prod(n)
    s = synth.Scenario("lin", (0.0, 0.0, 0.0), (30.0, 10.0, 4.0), n, p,
                       permeability=np.full(nc, 1e-11), porosity=np.full(nc, 0.25),
                       lambda_solid=np.full(nc, 2.0), rhoc_solid=np.full(nc, 2e6))
    lin = synth.timefn(c0=300.0, cx=-0.5)
    s.bcs = [synth.FaceBC(synth.TEMPERATURE, 0, synth.DIRICHLET, lin),
             synth.FaceBC(synth.TEMPERATURE, 1, synth.DIRICHLET, lin)]
    m = Mesh.of(s)
    X, Y, Z = m.coords()
    T0 = 300.0 - 0.5 * X
    P = 1e5 - 200.0 * Y + s.rho_w * s.g * (4.0 - Z)         # q along y only
    T = T0.copy()
    for it in range(3):
        T = oracle.solve_heat(s, m, T, P, (it + 1) * s.dt)
    assert np.abs(T - T0).max() <= 1e-12 * 300.0


def _rod(n, p, L, lam=1.0, cT=1e6, q0=0.0, c_w=4.18e6):
    """A 1D rod n x 1 x 1 with lambda, c_T fixed (porosity 0)."""
    s = synth.Scenario("rod", (0.0, 0.0, 0.0), (L, 1.0, 1.0), (n, 1, 1), p,
                       permeability=np.full(n, 1e-12), porosity=np.zeros(n),
                       lambda_solid=np.full(n, lam), rhoc_solid=np.full(n, cT), c_w=c_w)
    m = Mesh.of(s)
    X, Y, Z = m.coords()
    k = 1e-12 / s.mu_w
    P = 1e5 - (q0 / k) * X + s.rho_w * s.g * (1.0 - Z)        # q = (q0, 0, 0)
    return s, m, X, P


def _l2(m, u, fex):
    nq = 4
    vals = oracle.eval_qp(m, nq, u)
    gx, gw = oracle.gauss01(nq)
    hx = m.L[0] / m.n[0]
    err = 0.0
    cells = np.arange(m.ncell)
    cx = cells % m.n[0]
    for q in range(nq ** 3):
        qx, qy, qz = q % nq, (q // nq) % nq, q // (nq * nq)
        x = m.x0[0] + (cx + gx[qx]) * hx
        w = gw[qx] * gw[qy] * gw[qz] * np.prod(m.L) / m.ncell
        err += np.sum(w * (vals[cells * nq ** 3 + q] - fex(x)) ** 2)
    return math.sqrt(err)


def _run_rod(n, p, steps, t0, t1, exact, L, lam, cT, q0):
    s, m, X, P = _rod(n, p, L, lam, cT, q0)
    s.dt = (t1 - t0) / steps
    s.bcs = [synth.FaceBC(synth.TEMPERATURE, 0, synth.DIRICHLET, synth.timefn(exact(0.0, 1.0))),
             synth.FaceBC(synth.TEMPERATURE, 1, synth.DIRICHLET, synth.timefn(exact(L, t1)))]
    T = exact(X, t0)
    t = t0
    for _ in range(steps):
        t += s.dt
        T = oracle.solve_heat(s, m, T, P, t)
    return _l2(m, T, lambda x: exact(x, t1))


def test_erfc_semi_infinite_conduction_converges():
    """Mass + backward Euler + conduction: T = Ts + (T0-Ts) erf(x / 2 sqrt(a t))."""
    lam, cT, Ts, T0, L = 1.0, 1e6, 300.0, 280.0, 12.0
    a = lam / cT

    def exact(x, t):
        return Ts + (T0 - Ts) * (1.0 - erfc(np.asarray(x) / (2.0 * np.sqrt(a * t))))

    t0, t1 = 2e5, 1.0e6
    errs = [_run_rod(n, 1, st, t0, t1, exact, L, lam, cT, 0.0)
            for n, st in [(24, 4), (48, 16), (96, 64)]]
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert errs[2] < 2e-3 * abs(T0 - Ts) * math.sqrt(L)
    assert 3.2 < r1 < 4.8 and 3.4 < r2 < 4.6, (errs, r1, r2)


def test_ogata_banks_advection_converges():
    """Advection with the Darcy flux (Eq. 4): Ogata-Banks solution with
    thermal velocity v = c_w q / c_T and D = lambda / c_T."""
    lam, cT, c_w, L = 1.0, 1e6, 4.18e6, 16.0
    D = lam / cT
    v = 2e-6
    q0 = v * cT / c_w
    T0, Tin = 280.0, 300.0

    def exact(x, t):
        x = np.asarray(x, dtype=float)
        s = 2.0 * np.sqrt(D * t)
        z2 = (x + v * t) / s
        second = np.exp(v * x / D - z2 ** 2) * erfcx(z2)
        return T0 + 0.5 * (Tin - T0) * (erfc((x - v * t) / s) + second)

    t0, t1 = 3e5, 1.5e6
    errs = [_run_rod(n, 1, st, t0, t1, exact, L, lam, cT, q0)
            for n, st in [(32, 4), (64, 16), (128, 64)]]
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.0 < r1 < 5.0 and 3.4 < r2 < 4.6, (errs, r1, r2)
    # transport direction: a flipped advection term converges to a wrong
    # solution; the finest error must be small in absolute terms
    assert errs[2] < 5e-3 * (Tin - T0) * math.sqrt(L)


@pytest.mark.parametrize("p,ratio", [(1, 4.0), (2, 8.0)])
def test_manufactured_solution_order(p, ratio):
    """-div(k grad u) = f, u = sin(pi x) sin(pi y) sin(pi z) e^{x}, cellwise k
    (smooth k sampled at cell centres for Q1; constant for Q2)."""
    def run(n):
        m = Mesh((0.0, 0.0, 0.0), (1.0, 1.0, 1.0), (n, n, n), p)
        nq = 4
        gx, gw = oracle.gauss01(nq)
        h = 1.0 / n
        cells = np.arange(m.ncell)
        cx, cy, cz = cells % n, (cells // n) % n, cells // (n * n)
        if p == 1:
            kf = lambda x, y, z: 1.0 + 0.5 * x * y + 0.25 * z
            kgrad = lambda x, y, z: (0.5 * y, 0.5 * x, 0.25 + 0.0 * z)
        else:
            kf = lambda x, y, z: 1.5 + 0.0 * x
            kgrad = lambda x, y, z: (0.0 * x, 0.0 * x, 0.0 * x)
        kc = kf((cx + 0.5) * h, (cy + 0.5) * h, (cz + 0.5) * h)
        fq = np.zeros((m.ncell, nq ** 3))
        for q in range(nq ** 3):
            qx, qy, qz = q % nq, (q // nq) % nq, q // (nq * nq)
            x, y, z = (cx + gx[qx]) * h, (cy + gx[qy]) * h, (cz + gx[qz]) * h
            S = np.sin(np.pi * x) * np.sin(np.pi * y) * np.sin(np.pi * z)
            ex = np.exp(x)
            u = S * ex
            sx, sy, sz = np.sin(np.pi * x), np.sin(np.pi * y), np.sin(np.pi * z)
            cxp, cyp, czp = np.cos(np.pi * x), np.cos(np.pi * y), np.cos(np.pi * z)
            ux = np.pi * cxp * sy * sz * ex + u
            uy = np.pi * sx * cyp * sz * ex
            uz = np.pi * sx * sy * czp * ex
            lap = (-3 * np.pi ** 2) * u + 2 * np.pi * cxp * sy * sz * ex + u
            # f = -div(k grad u) with the smooth k; the discrete problem
            # samples k at cell centres (an O(h^2) consistency error)
            kx, ky, kz_ = kgrad(x, y, z)
            fq[:, q] = -(kf(x, y, z) * lap + kx * ux + ky * uy + kz_ * uz)
        A = oracle.assemble(m, stiff=kc)
        b = oracle.load_qp(m, nq, fq.reshape(-1))
        NX = p * n + 1
        I = np.arange(m.nnode)
        i, j, kz = I % NX, (I // NX) % NX, I // (NX * NX)
        mask = (i == 0) | (i == NX - 1) | (j == 0) | (j == NX - 1) | (kz == 0) | (kz == NX - 1)
        u = oracle.solve_field(A, b, mask, np.zeros(m.nnode), symmetric=True)
        vals = oracle.eval_qp(m, nq, u).reshape(m.ncell, nq ** 3)
        err = 0.0
        for q in range(nq ** 3):
            qx, qy, qz = q % nq, (q // nq) % nq, q // (nq * nq)
            x, y, z = (cx + gx[qx]) * h, (cy + gx[qy]) * h, (cz + gx[qz]) * h
            ue = np.sin(np.pi * x) * np.sin(np.pi * y) * np.sin(np.pi * z) * np.exp(x)
            err += np.sum(gw[qx] * gw[qy] * gw[qz] * h ** 3 * (vals[:, q] - ue) ** 2)
        return math.sqrt(err)

    ns = [4, 8, 16] if p == 1 else [2, 4, 8]
    e = [run(n) for n in ns]
    assert abs(e[1] / e[2] - ratio) < 0.2 * ratio, e
    assert e[0] > e[1] > e[2]


# ---------------------------------------------------------------- balances
@pytest.mark.parametrize("p", [1, 2])
def test_heat_energy_balance_insulated(p):
    """Insulated box with a volume source and a Neumann face flux:
    sum_i [M_cT (T^{n+1} - T^n)]_i = h int f - h q_TN |face| (no advection)."""
    s = small_scn(p=p)
    s.permeability[:] = 0.0
    s.heat_source = np.random.default_rng(7).uniform(0, 30, s.ncell)
    s.bcs = [synth.FaceBC(synth.TEMPERATURE, 3, synth.NEUMANN, synth.timefn(0.4))]
    m = Mesh.of(s)
    k, lam, cT = oracle.coefficients(s)
    T0 = 290.0 + np.random.default_rng(8).uniform(-1, 1, m.nnode)
    P = np.zeros(m.nnode)
    T1 = oracle.solve_heat(s, m, T0, P, s.dt)
    Mc = oracle.assemble(m, mass=cT)
    stored = np.ones(m.nnode) @ (Mc @ (T1 - T0))
    vol = np.prod(m.L) / m.ncell
    expect = s.dt * vol * s.heat_source.sum() - s.dt * 0.4 * (3.0 * 1.0)
    assert math.isclose(stored, expect, rel_tol=1e-10)


@pytest.mark.parametrize("p", [1, 2])
def test_pressure_mass_balance_well(p):
    """No Dirichlet data, a well of rate Q and a Neumann inflow: stored fluid
    sum_i [M (P^{n+1}-P^n)]_i = hB (Q - q_N |face|); gravity adds nothing."""
    s = small_scn(p=p)
    s.B_poro = 1e5
    s.lines = [synth.LineSource(1.3, 5.2, 0.2, 0.9, synth.LINE_WELL, synth.timefn(2e-4))]
    s.bcs = [synth.FaceBC(synth.PRESSURE, 5, synth.NEUMANN, synth.timefn(-1e-6))]
    m = Mesh.of(s)
    A, b = oracle.pressure_system(s, m, np.full(m.nnode, 2e5), s.dt)
    P1 = spla.spsolve(A.tocsc(), b)
    M = oracle.assemble(m, mass=np.ones(m.ncell))
    stored = np.ones(m.nnode) @ (M @ (P1 - 2e5))
    expect = s.dt * s.B_poro * (2e-4 + 1e-6 * 3.0 * 8.0)
    assert math.isclose(stored, expect, rel_tol=1e-9)


# ------------------------------------------ injection enthalpy (Eq. 4, C8)
def _lagrange_1d(p, t):
    """Values of the p+1 equispaced Lagrange basis functions on [0, 1] at t."""
    nodes = np.linspace(0.0, 1.0, p + 1)
    out = np.ones((p + 1,) + np.shape(t))
    for a in range(p + 1):
        for b in range(p + 1):
            if b != a:
                out[a] = out[a] * (t - nodes[b]) / (nodes[a] - nodes[b])
    return out


def _fe_eval(s, u, x, y, z):
    """Value of the finite element function with node values u at one point
    (uniform box), by the tensor Lagrange basis of the cell containing it."""
    p = s.degree
    NX, NY, NZ = s.nodes_per_dim
    pt = (x, y, z)
    idx, loc = [], []
    for d in range(3):
        h = s.extent[d] / s.ncells[d]
        c = min(int((pt[d] - s.origin[d]) // h), s.ncells[d] - 1)
        idx.append(c)
        loc.append(_lagrange_1d(p, (pt[d] - s.origin[d] - c * h) / h))
    val = 0.0
    for c_ in range(p + 1):
        for b in range(p + 1):
            for a in range(p + 1):
                n = (p * idx[0] + a) + NX * ((p * idx[1] + b) + NY * (p * idx[2] + c_))
                val += loc[0][a] * loc[1][b] * loc[2][c_] * u[n]
    return val


def _stored(s, cT, u):
    """int c_T u dV with a 4-point Gauss rule per direction in every cell
    (exact for the tensor degree-2 functions with cellwise c_T)."""
    gx, gw = np.polynomial.legendre.leggauss(4)
    gx, gw = 0.5 * (gx + 1.0), 0.5 * gw
    h = [s.extent[d] / s.ncells[d] for d in range(3)]
    tot = 0.0
    nx, ny, nz = s.ncells
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                acc = 0.0
                for qz, wz in zip(gx, gw):
                    for qy, wy in zip(gx, gw):
                        for qx, wx in zip(gx, gw):
                            acc += wx * wy * wz * _fe_eval(
                                s, u, s.origin[0] + (i + qx) * h[0], s.origin[1] + (j + qy) * h[1],
                                s.origin[2] + (k + qz) * h[2])
                tot += cT[i + nx * (j + ny * k)] * acc * h[0] * h[1] * h[2]
    return tot


def _line_integral(s, u, x, y, z0, z1):
    """int_{z0}^{z1} u(x, y, z) dz, 4-point Gauss on each cell piece."""
    hz = s.extent[2] / s.ncells[2]
    cuts = sorted({z0, z1} | {s.origin[2] + k * hz for k in range(s.ncells[2] + 1) if z0 < s.origin[2] + k * hz < z1})
    gx, gw = np.polynomial.legendre.leggauss(4)
    tot = 0.0
    for a, b in zip(cuts[:-1], cuts[1:]):
        for q, w in zip(gx, gw):
            tot += 0.5 * (b - a) * w * _fe_eval(s, u, x, y, a + 0.5 * (b - a) * (q + 1.0))
    return tot


@pytest.mark.parametrize("p", [1, 2])
def test_injection_enthalpy_energy_balance(p):
    """Insulated box without flow (zero permeability), one injection well
    (Q > 0, water at T_inj) and one extraction well.  Summing Eq. 4 over all
    test functions (partition of unity) leaves the heat stored in one step
    equal to the enthalpy the injected water brings in minus what it takes up
    at the new temperature along the screen:
        int c_T (T^{n+1} - T^n) dV = h c_w (Q / L) int_line (T_inj - T^{n+1}) dz,
    while the extraction well adds no heat term.  Both sides are evaluated
    here from the node values with an independent Lagrange basis and Gauss
    rule; a missing factor h or c_w, a flipped sign, a wrong per-metre rate or
    a heat term at the extraction well breaks the equality."""
    s = small_scn(p=p)
    s.permeability[:] = 0.0
    Q, Tin, z0, z1 = 2e-4, 320.0, 0.2, 0.9
    s.lines = [synth.LineSource(1.3, 5.2, z0, z1, synth.LINE_WELL, synth.timefn(Q), T_inj=Tin),
               synth.LineSource(2.1, 2.7, 0.1, 0.8, synth.LINE_WELL, synth.timefn(-3e-4), T_inj=400.0)]
    m = Mesh.of(s)
    k, lam, cT = oracle.coefficients(s)
    T0 = 290.0 + np.random.default_rng(9).uniform(-1, 1, m.nnode)
    T1 = oracle.solve_heat(s, m, T0, np.zeros(m.nnode), s.dt)
    stored = _stored(s, cT, T1 - T0)
    inflow = s.dt * s.c_w * Q / (z1 - z0) * (Tin * (z1 - z0) - _line_integral(s, T1, 1.3, 5.2, z0, z1))
    assert abs(inflow) > 1e3 * abs(s.dt * s.c_w * Q) * 1e-9
    assert math.isclose(stored, inflow, rel_tol=1e-9)
    # the extraction well alone leaves the stored heat unchanged
    s.lines = s.lines[1:]
    T2 = oracle.solve_heat(s, m, T0, np.zeros(m.nnode), s.dt)
    assert abs(_stored(s, cT, T2 - T0)) <= 1e-9 * s.dt * s.c_w * Q * 1.0


@pytest.mark.parametrize("p", [1, 2])
def test_injection_at_ambient_temperature_keeps_state(p):
    """A box at T_inj everywhere, held at T_inj on its faces, with an
    injection / extraction well pair driving Darcy flow: the injected water
    is at the temperature of the rock, so T stays T_inj (conduction and
    advection of a constant vanish, and the line terms c_w s+ (T_inj - T)
    cancel only if the matrix and load parts carry the same h, weights and
    sign)."""
    s = small_scn(p=p)
    Tin = 305.0
    s.lines = [synth.LineSource(1.3, 5.2, 0.2, 0.9, synth.LINE_WELL, synth.timefn(2e-4), T_inj=Tin),
               synth.LineSource(2.1, 2.7, 0.1, 0.8, synth.LINE_WELL, synth.timefn(-2e-4), T_inj=Tin)]
    s.bcs = [synth.FaceBC(synth.TEMPERATURE, f, synth.DIRICHLET, synth.timefn(Tin)) for f in range(6)]
    m = Mesh.of(s)
    P0 = np.full(m.nnode, 2e5)
    P1 = oracle.solve_pressure(s, m, P0, s.dt)
    k, lam, cT = oracle.coefficients(s)
    q = oracle.flux_qp(m, p + 1, k, P1, s.rho_w * s.g)
    assert np.abs(q).max() > 1e-9           # the wells do drive a flow
    T1 = oracle.solve_heat(s, m, np.full(m.nnode, Tin), P1, s.dt)
    assert np.abs(T1 - Tin).max() <= 1e-10 * Tin
    # water injected 10 K warmer moves the same state (the pin is not vacuous)
    s.lines[0] = synth.LineSource(1.3, 5.2, 0.2, 0.9, synth.LINE_WELL, synth.timefn(2e-4), T_inj=Tin + 10.0)
    T2 = oracle.solve_heat(s, m, np.full(m.nnode, Tin), P1, s.dt)
    assert np.abs(T2 - Tin).max() > 1e-3


# ------------------------------------------------- site-style boundary data
GEO_LAYERS = ((0.0, 15.0, 2.97), (15.0, 30.0, 1.5), (30.0, 40.0, 2.2))


def geotherm_scn(p, n=(3, 2, 8), q=0.0891, T_top=287.45):
    """Conduction-only 40 m column: bulk conductivity in three layers whose
    interfaces lie on cell faces, the surface temperature held at T_top and
    a geothermal inflow q through the bottom (Section 3.3 boundary data)."""
    nc = n[0] * n[1] * n[2]
    k = np.arange(nc) // (n[0] * n[1])
    zc = (k + 0.5) * 40.0 / n[2]
    lam = np.select([zc < a[1] for a in GEO_LAYERS], [a[2] for a in GEO_LAYERS])
    rng = np.random.default_rng(11)
    s = synth.Scenario("geo", (0.0, 0.0, 0.0), (30.0, 20.0, 40.0), n, p,
                       permeability=None, porosity=None, lambda_solid=None, rhoc_solid=None,
                       hydraulic_conductivity=np.zeros(nc), lambda_bulk=lam,
                       rhoc_bulk=rng.uniform(2.0e6, 3.5e6, nc))
    s.bcs = [synth.FaceBC(synth.TEMPERATURE, 5, synth.DIRICHLET, synth.timefn(T_top)),
             synth.FaceBC(synth.TEMPERATURE, 4, synth.NEUMANN, synth.timefn(-q))]
    return s


def geotherm_exact(Z, q=0.0891, T_top=287.45):
    """Steady conduction with an upward flux q: -lambda dT/dz = q, so
    T(z) = T_top + q int_z^top dz'/lambda(z'), piecewise linear."""
    Z = np.asarray(Z, dtype=float)
    acc = np.zeros_like(Z)
    for a, b, lam in GEO_LAYERS:
        acc += np.clip(b - np.maximum(a, Z), 0.0, None) / lam
    return T_top + q * acc


@pytest.mark.parametrize("p", [1, 2])
def test_layered_geotherm_is_a_fixed_point(p):
    """The piecewise-linear steady geotherm lies in the finite element space
    when the layer interfaces are cell faces, so a backward-Euler step from it
    returns it: this fixes the sign and size of the Neumann flux term of
    Eq. 4, the per-cell conductivity of the stiffness and the Dirichlet lift."""
    s = geotherm_scn(p)
    m = Mesh.of(s)
    X, Y, Z = m.coords()
    T0 = geotherm_exact(Z)
    T1 = oracle.solve_heat(s, m, T0, np.zeros(m.nnode), s.dt)
    assert np.abs(T1 - T0).max() <= 1e-10
    # the same column with the flux sign flipped moves away from it
    s.bcs[1] = synth.FaceBC(synth.TEMPERATURE, 4, synth.NEUMANN, synth.timefn(0.0891))
    T2 = oracle.solve_heat(s, m, T0, np.zeros(m.nnode), s.dt)
    assert np.abs(T2 - T0).max() > 1e-4


def test_hydraulic_conductivity_and_bulk_values():
    """A conductivity K [m/s] is K_i rho_w g / mu_w, and bulk thermal values
    equal to the mixture of solid and water give the same systems."""
    s = small_scn(n=(4, 3, 3))
    s.B_poro = 1e5
    s.lines = [synth.LineSource(1.3, 5.2, 0.2, 0.9, synth.LINE_WELL, synth.timefn(2e-4), T_inj=300.0)]
    phi = s.porosity
    s2 = s.replace(permeability=None, porosity=None, lambda_solid=None, rhoc_solid=None,
                   hydraulic_conductivity=s.permeability * s.rho_w * s.g / s.mu_w,
                   lambda_bulk=(1 - phi) * s.lambda_solid + phi * s.lambda_w,
                   rhoc_bulk=(1 - phi) * s.rhoc_solid + phi * s.c_w)
    m = Mesh.of(s)
    X, Y, Z = m.coords()
    P0 = 1e5 + s.rho_w * s.g * (1.0 - Z)
    A1, b1 = oracle.pressure_system(s, m, P0, s.dt)
    A2, b2 = oracle.pressure_system(s2, m, P0, s.dt)
    assert abs(A1 - A2).max() <= 1e-12 * abs(A1).max()
    assert np.abs(b1 - b2).max() <= 1e-12 * np.abs(b1).max()
    P1 = P0 - 3.0 * X
    H1, h1 = oracle.heat_system(s, m, np.full(m.nnode, 290.0), P1, s.dt)
    H2, h2 = oracle.heat_system(s2, m, np.full(m.nnode, 290.0), P1, s.dt)
    assert abs(H1 - H2).max() <= 1e-12 * abs(H1).max()
    assert np.abs(h1 - h2).max() <= 1e-12 * np.abs(h1).max()


def test_island_scenario_layout():
    """The island generator: Table 3 classes by depth, bedrock top between
    70 and 80 m, piles on the 20 m lattice 60 m long from the surface."""
    s = synth.island(ncells=(64, 40, 20), n_steps=1)
    nx, ny, nz = s.ncells
    lam = s.lambda_bulk.reshape(nz, ny, nx)
    depth = 100.0 - (np.arange(nz) + 0.5) * 100.0 / nz
    rock = lam == 2.97
    assert not rock[depth < 70.0].any() and rock[depth > 80.0].all()
    assert (lam[depth < 8.0] == 2.2).all()
    K = s.hydraulic_conductivity.reshape(nz, ny, nx)
    assert np.all(np.abs(np.log10(K[depth > 80.0]) + 6.0) < 2.0)
    assert len(s.dir_columns) > 20
    for c in s.dir_columns:
        assert c.x % 20.0 == 0.0 and c.y % 20.0 == 0.0
        assert 60.0 <= c.x <= 580.0 and 60.0 <= c.y <= 340.0
        assert (c.z0, c.z1) == (40.0, 100.0)


def test_ates_scenario_layout():
    """The injection benchmark analogue: Table 1 values, the aquifer between
    100 and 200 m depth, the wellbore on the axis over the aquifer only, and
    an injection rate equal to the wellbore flux times its surface."""
    s = synth.ates(ncells=(8, 8, 30), n_steps=1)
    nx, ny, nz = s.ncells
    K = s.hydraulic_conductivity.reshape(nz, ny, nx)
    depth = 300.0 - (np.arange(nz) + 0.5) * 10.0
    aq = (depth > 100.0) & (depth < 200.0)
    assert np.all(K[aq] == 1e-6) and np.all(K[~aq] == 1e-10)
    assert np.all(s.lambda_bulk == 1.2) and np.all(s.rhoc_bulk == 1.2e6) and s.c_w == 1e6
    (w,) = s.lines
    assert (w.x, w.y, w.z0, w.z1) == (20.0, 20.0, 100.0, 200.0) and w.T_inj == 288.15
    assert w.rate[1] == pytest.approx(0.001 * 2 * np.pi * 0.1 * 100.0)
    (c,) = s.dir_columns
    assert (c.x, c.y, c.z0, c.z1) == (20.0, 20.0, 100.0, 200.0) and c.value[1] == 288.15
    m = Mesh.of(s)
    X, Y, Z = m.coords()
    T0 = oracle.tf_value(s.T0, X, Y, Z, 0.0)
    assert T0.max() == pytest.approx(293.15) and T0.min() == pytest.approx(278.15)


# ------------------------------------------------ graded (rectilinear) meshes
GX = np.array([0.0, 7.0, 20.0, 31.0, 45.0, 60.0, 70.0, 81.0, 100.0])
GY = np.array([0.0, 12.0, 25.0, 50.0, 60.0, 64.0, 80.0, 100.0])
GZ = np.array([0.0, 5.0, 15.0, 22.0, 30.0, 45.0, 60.0, 63.0, 75.0, 100.0])


@pytest.mark.parametrize("p", [1, 2])
def test_graded_uniform_darcy_flow_exact(p):
    """Hydrostatic pressure plus a linear drop stays exact on graded cells,
    and q_h = (k dp / L, 0, 0) at every Gauss point."""
    s = synth.config1()
    s.degree = p
    s.ncells = (GX.size - 1, GY.size - 1, GZ.size - 1)
    nc = int(np.prod(s.ncells))
    s.permeability, s.porosity = np.full(nc, 1e-12), np.full(nc, 0.3)
    s.lambda_solid, s.rhoc_solid = np.full(nc, 2.5), np.full(nc, 2e6)
    s.heat_source = None
    s.edges = (GX, GY, GZ)
    m = Mesh.of(s)
    P, _ = oracle.initial_state(s, m)
    X, Y, Z = m.coords()
    if p == 1:
        assert np.allclose(np.unique(X), GX) and np.allclose(np.unique(Z), GZ)
    else:   # every edge plus the cell midpoints
        assert np.allclose(np.unique(X)[0::2], GX) and np.allclose(np.unique(X)[1::2], 0.5 * (GX[1:] + GX[:-1]))
    Pex = 1e5 + s.rho_w * s.g * (100.0 - Z) + 1e4 * (1.0 - X / 100.0)
    assert np.abs(P - Pex).max() <= 1e-12 * np.abs(Pex).max()
    k = 1e-12 / s.mu_w
    q = oracle.flux_qp(m, 2, np.full(m.ncell, k), P, s.rho_w * s.g)
    assert np.allclose(q[:, :, 0], k * 1e4 / 100.0, rtol=1e-9)
    assert np.abs(q[:, :, 1:]).max() <= 1e-9 * k * 1e4 / 100.0


def test_graded_layered_geotherm_is_a_fixed_point():
    """The layered geotherm of the uniform test on graded cells whose z-edges
    include the layer interfaces (15 m, 30 m): still in the finite element
    space, so a step returns it."""
    gx, gy = np.array([0.0, 4.0, 13.0, 30.0]), np.array([0.0, 15.0, 20.0])
    gz = np.array([0.0, 3.0, 15.0, 19.0, 30.0, 31.0, 36.0, 40.0])
    s = geotherm_scn(1, n=(3, 2, 7))
    s.edges = (gx, gy, gz)
    k = np.arange(s.ncell) // 6
    zc = 0.5 * (gz[1:] + gz[:-1])[k]
    s.lambda_bulk = np.select([zc < a[1] for a in GEO_LAYERS], [a[2] for a in GEO_LAYERS])
    m = Mesh.of(s)
    X, Y, Z = m.coords()
    T0 = geotherm_exact(Z)
    T1 = oracle.solve_heat(s, m, T0, np.zeros(m.nnode), s.dt)
    assert np.abs(T1 - T0).max() <= 1e-10


@pytest.mark.parametrize("p", [1, 2])
def test_graded_heat_energy_balance(p):
    """Insulated graded box: the stored heat equals the volume source over the
    actual cell volumes minus the Neumann flux over the whole face."""
    s = small_scn(n=(4, 3, 3), p=p)
    s.edges = (np.array([0.0, 0.3, 1.0, 2.2, 3.0]), np.array([0.0, 1.0, 5.0, 8.0]),
               np.array([0.0, 0.1, 0.5, 1.0]))
    s.permeability[:] = 0.0
    s.heat_source = np.random.default_rng(7).uniform(0, 30, s.ncell)
    s.bcs = [synth.FaceBC(synth.TEMPERATURE, 3, synth.NEUMANN, synth.timefn(0.4))]
    m = Mesh.of(s)
    T0 = 290.0 + np.random.default_rng(8).uniform(-1, 1, m.nnode)
    T1 = oracle.solve_heat(s, m, T0, np.zeros(m.nnode), s.dt)
    k, lam, cT = oracle.coefficients(s)
    Mc = oracle.assemble(m, mass=cT)
    stored = np.ones(m.nnode) @ (Mc @ (T1 - T0))
    ex, ey, ez = s.edges
    V = (np.diff(ez)[:, None, None] * np.diff(ey)[None, :, None] * np.diff(ex)[None, None, :]).reshape(-1)
    expect = s.dt * (V * s.heat_source).sum() - s.dt * 0.4 * (3.0 * 1.0)
    assert math.isclose(stored, expect, rel_tol=1e-10)


def test_graded_dirichlet_column_nearest_node():
    """On a graded axis a column goes to the nearest node, the higher one on
    a tie."""
    s = small_scn(n=(4, 3, 3))
    s.edges = (np.array([0.0, 0.3, 1.0, 2.2, 3.0]), np.array([0.0, 1.0, 5.0, 8.0]),
               np.array([0.0, 0.1, 0.5, 1.0]))
    s.dir_columns = [synth.DirColumn(synth.TEMPERATURE, 0.7, 3.0, 0.0, 1.0, synth.timefn(300.0))]
    m = Mesh.of(s)
    mask, g = oracle.dirichlet(s, m, synth.TEMPERATURE, 0.0)
    X, Y, Z = m.coords()
    sel = (X == 1.0) & (Y == 5.0)   # 0.7 is nearer 1.0 than 0.3; 3.0 ties 1.0 and 5.0
    assert mask.sum() == 4 and mask[sel].all() and np.all(g[sel] == 300.0)


def test_graded_q2_dirichlet_column_takes_mid_edge_nodes():
    """On degree-2 graded axes the cell midpoints are nodes too: x = 0.7 goes
    to the midpoint 0.65 of the cell [0.3, 1.0], y = 3.0 is the midpoint of
    [1, 5], and the column holds all seven z nodes of [0, 1]."""
    s = small_scn(n=(4, 3, 3), p=2)
    s.edges = (np.array([0.0, 0.3, 1.0, 2.2, 3.0]), np.array([0.0, 1.0, 5.0, 8.0]),
               np.array([0.0, 0.1, 0.5, 1.0]))
    s.dir_columns = [synth.DirColumn(synth.TEMPERATURE, 0.7, 3.0, 0.0, 1.0, synth.timefn(300.0))]
    m = Mesh.of(s)
    mask, g = oracle.dirichlet(s, m, synth.TEMPERATURE, 0.0)
    X, Y, Z = m.coords()
    sel = (X == 0.65) & (Y == 3.0)
    assert sel.sum() == 7 and mask.sum() == 7 and mask[sel].all() and np.all(g[sel] == 300.0)
    assert np.allclose(np.sort(Z[sel]), [0.0, 0.05, 0.1, 0.3, 0.5, 0.75, 1.0])


@pytest.mark.parametrize("p", [1, 2])
def test_graded_convection_skew_for_uniform_flux(p):
    """On graded cells a linear P still gives a uniform Darcy flux, so the
    convection matrix stays skew on fields vanishing at the boundary and
    annihilates constants (the per-cell 1/h of the gradients)."""
    m = Mesh((0.0, 0.0, 0.0), (3.0, 3.0, 3.0), (4, 3, 5), p,
             (np.array([0.0, 0.2, 1.1, 2.0, 3.0]), np.array([0.0, 1.7, 2.2, 3.0]),
              np.array([0.0, 0.5, 0.9, 1.0, 2.4, 3.0])))
    X, Y, Z = m.coords()
    rho_g, kk = 9810.0, 1e-9
    P = 1e5 - 300.0 * X + 120.0 * Y + rho_g * (3.0 - Z) - 50.0 * Z
    Cm = oracle.assemble(m, kvel=np.full(m.ncell, kk), P=P, adv_scale=4e6, rho_g=rho_g)
    NX, NY, NZ = m.dims
    I = np.arange(m.nnode)
    i, j, kz = I % NX, (I // NX) % NY, I // (NX * NY)
    bnd = (i == 0) | (i == NX - 1) | (j == 0) | (j == NY - 1) | (kz == 0) | (kz == NZ - 1)
    x = np.random.default_rng(4).standard_normal(m.nnode)
    x[bnd] = 0.0
    assert abs(x @ (Cm @ x)) <= 1e-12 * abs(Cm).max() * (x @ x)
    assert np.abs(Cm @ np.ones(m.nnode)).max() <= 1e-12 * abs(Cm).max()
    # and a linear field is advected at the uniform flux: C x = (q . grad x) * (row sums of M)
    q = np.array([300.0, -120.0, 50.0]) * kk * 4e6
    M = oracle.assemble(m, mass=np.ones(m.ncell))
    lin = 2.0 * X - 1.0 * Y + 0.5 * Z
    assert np.allclose(Cm @ lin, (q @ np.array([2.0, -1.0, 0.5])) * (M @ np.ones(m.nnode)),
                       rtol=1e-10, atol=1e-10 * abs(Cm @ lin).max())


def test_island_graded_layout():
    """The graded island keeps its piles and materials per cell and refines
    about 3:1 over the footprints and the top 70 m."""
    s = synth.island(ncells=(64, 40, 20), n_steps=1, graded=True)
    ex, ey, ez = s.edges
    assert ex[0] == 0.0 and ex[-1] == 640.0 and ez[-1] == 100.0
    hx, hz = np.diff(ex), np.diff(ez)
    assert 2.0 < hx.max() / hx.min() < 3.5 and 2.0 < hz.max() / hz.min() < 3.5
    assert hz[-1] < hz[0]      # finer at the top, where the piles are
    u = synth.island(ncells=(64, 40, 20), n_steps=1)
    assert [(c.x, c.y) for c in s.dir_columns] == [(c.x, c.y) for c in u.dir_columns]


# ----------------------------------------------------------------- solvers
def test_iterative_solvers_match_lu():
    s = small_scn(n=(6, 5, 4))
    s.B_poro = 1e5
    m = Mesh.of(s)
    A, b = oracle.pressure_system(s, m, np.full(m.nnode, 1e5), s.dt)
    xd = spla.spsolve(A.tocsc(), b)
    x1, it, rr = oracle.pcg(A, b, rtol=1e-13)
    assert rr <= 1e-13 and np.abs(x1 - xd).max() <= 1e-9 * np.abs(xd).max()
    X, Y, Z = m.coords()
    P = 1e5 - 3.0 * X + s.rho_w * s.g * (1.0 - Z)
    H, hb = oracle.heat_system(s, m, np.full(m.nnode, 290.0), P, s.dt)
    xh = spla.spsolve(H.tocsc(), hb)
    x2, it, rr = oracle.gmres(H, hb, m=20, rtol=1e-13)
    assert rr <= 1e-13 and np.abs(x2 - xh).max() <= 1e-9 * np.abs(xh).max()


def test_refinement_reaches_fp64_floor():
    s = synth.config1()
    m = Mesh.of(s)
    A, b = oracle.pressure_system(s, m, None, s.dt, steady=True)
    mask, g = oracle.dirichlet(s, m, synth.PRESSURE, s.dt)
    free, AFF, bF = oracle.eliminate(A, b, mask, g)
    u = oracle.solve(AFF, bF, symmetric=True)
    r = oracle.residual_ld(AFF, bF, u)
    assert np.linalg.norm(r) <= 1e-15 * np.linalg.norm(bF) * 10


@pytest.mark.parametrize("deg", [1, 2])
@pytest.mark.parametrize("field", [0, 1])
def test_operator_rows_match_assembled_operator(deg, field):
    """Row-by-row evaluation (used for sampled checks of meshes too large to
    assemble) equals the assembled, eliminated operator; the absolute variant
    bounds it and equals |A| |x| where no element entries cancel."""
    s = synth.config2(ncells=(7, 6, 4), n_steps=1)
    s.degree = deg
    m = oracle.Mesh.of(s)
    rng = np.random.default_rng(5)
    X, Y, Z = m.coords()
    P = 1e5 + s.rho_w * s.g * (s.extent[2] - Z) - 20.0 * X + rng.standard_normal(m.nnode)
    x = rng.standard_normal(m.nnode)
    A = oracle.operator(s, field, P=P if field else None)
    mask, _ = oracle.dirichlet(s, m, field, s.t0 + s.dt)
    full = oracle.reduced_apply(A, mask, x)
    rows = np.unique(np.concatenate([rng.choice(m.nnode, 200, replace=False), np.nonzero(mask)[0][:20]]))
    y = oracle.operator_rows(s, field, rows, x, P=P if field else None)
    np.testing.assert_allclose(y, full[rows], rtol=1e-12, atol=1e-12 * np.abs(full).max())
    yb = oracle.operator_rows(s, field, rows, x, P=P if field else None, absolute=True)
    Aabs = abs(A.tocsr())
    ref = np.where(mask, np.abs(x), Aabs @ np.where(mask, 0.0, np.abs(x)))[rows]
    assert np.all(yb >= ref * (1 - 1e-12))
    assert np.all(yb >= np.abs(y) * (1 - 1e-12))
