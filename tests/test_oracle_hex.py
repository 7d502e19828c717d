"""Pins of the oracle on general hexahedra (the box topology with arbitrary
node coordinates: each cell the isoparametric image of the unit cube,
Section 3.3 / Fig. 10b meshes), CPU only.

* node coordinates of a box (uniform or graded) reproduce the box matrices;
* a rigid motion of all coordinates leaves mass, stiffness and convection
  unchanged (gravity off, the pressure moved with the mesh);
* patch tests on a terrain-following mesh of curved cells: K 1 = 0, and the
  rows of K x_d vanish at interior nodes for the coordinate fields x, y, z
  (linear fields are in the trilinear space; with the cofactor form of the
  gradients the 2-point rule integrates those rows exactly);
* the mass matrix sums to the mesh volume, obtained independently from the
  divergence theorem over the bilinear boundary faces, V = (1/3) sum_f
  int x . n dA; the gravity load against the nodal z equals the volume too;
* a constant Darcy flux gives a convection matrix whose symmetric part
  vanishes on interior rows (int q . grad(N_a N_b) = boundary terms), with a
  rule exact for its polynomial degree (3 points);
* face loads sum to the face areas (planar side faces of known area).
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")

N = (6, 5, 4)
ORG, EXT = (0.0, 0.0, 0.0), (500.0, 400.0, 100.0)


def box_xyz(m):
    X, Y, Z = m.coords()
    return np.stack([X, Y, Z], axis=1)


def terrain():
    return oracle.Mesh(ORG, EXT, N, 1, xyz=synth.terrain_coords(ORG, EXT, N, top_amp=12.0, bottom_amp=7.0,
                                                                shear=0.08))


def coeffs(m, seed=0):
    rng = np.random.default_rng(seed)
    return rng.uniform(1.0, 3.0, m.ncell), rng.uniform(0.5, 2.0, m.ncell), rng.uniform(0.5, 1.5, m.ncell)


def rel(a, b):
    return abs(a - b).max() / max(abs(b).max(), 1e-300)


@pytest.mark.parametrize("graded", [False, True])
def test_box_coordinates_reproduce_box_matrices(graded):
    edges = None
    if graded:
        edges = tuple(np.cumsum(np.r_[0.0, np.random.default_rng(d).uniform(0.5, 1.5, N[d])]) for d in range(3))
        edges = tuple(ORG[d] + EXT[d] * e / e[-1] for d, e in enumerate(edges))
    box = oracle.Mesh(ORG, EXT, N, 1, edges)
    gen = oracle.Mesh(ORG, EXT, N, 1, xyz=box_xyz(box))
    cm, cs, kv = coeffs(box)
    P = np.random.default_rng(3).uniform(1e5, 2e5, box.nnode)
    for kw in (dict(mass=cm), dict(stiff=cs), dict(kvel=kv, P=P, adv_scale=2.0, rho_g=9810.0)):
        assert rel(oracle.assemble(gen, **kw).toarray(), oracle.assemble(box, **kw).toarray()) <= 1e-12
    assert rel(oracle.load_gradz(gen, cs), oracle.load_gradz(box, cs)) <= 1e-12
    for f in range(6):
        assert rel(oracle.load_face(gen, f, 1.0), oracle.load_face(box, f, 1.0)) <= 1e-12


def test_rigid_motion_invariance():
    m = terrain()
    c, s_ = np.cos(0.7), np.sin(0.7)
    Rz = np.array([[c, -s_, 0.0], [s_, c, 0.0], [0.0, 0.0, 1.0]])
    Rx = np.array([[1.0, 0.0, 0.0], [0.0, np.cos(0.4), -np.sin(0.4)], [0.0, np.sin(0.4), np.cos(0.4)]])
    R = Rx @ Rz
    moved = oracle.Mesh(ORG, EXT, N, 1, xyz=m.xyz @ R.T + np.array([30.0, -20.0, 5.0]))
    cm, cs, kv = coeffs(m)
    P = 1e5 + 50.0 * m.xyz[:, 0] - 30.0 * m.xyz[:, 2] + 0.01 * m.xyz[:, 1] ** 2   # moves with the mesh
    for kw in (dict(mass=cm), dict(stiff=cs), dict(kvel=kv, P=P, adv_scale=1.5, rho_g=0.0)):
        assert rel(oracle.assemble(moved, **kw).toarray(), oracle.assemble(m, **kw).toarray()) <= 1e-11


def interior(m):
    NX, NY, NZ = m.dims
    I = np.arange(m.nnode)
    i, j, k = I % NX, (I // NX) % NY, I // (NX * NY)
    return (i > 0) & (i < NX - 1) & (j > 0) & (j < NY - 1) & (k > 0) & (k < NZ - 1)


def test_terrain_patch_test():
    m = terrain()
    K = oracle.assemble(m, stiff=np.ones(m.ncell))
    scale = abs(K).sum(axis=1).max()
    assert abs(K @ np.ones(m.nnode)).max() <= 1e-13 * scale
    inn = interior(m)
    for d in range(3):
        r = K @ m.xyz[:, d]
        assert abs(r[inn]).max() <= 1e-12 * scale * abs(m.xyz[:, d]).max(), d
        # boundary rows carry the outward flux of grad x_d and do not vanish
        assert abs(r[~inn]).max() > 1e-6 * scale


def divergence_volume(m):
    """(1/3) sum over boundary faces of int x . n dA, each bilinear face by a
    2 x 2 Gauss rule (exact: x . (t1 x t2) has degree <= 3 per variable)."""
    NX, NY, NZ = m.dims
    X = m.xyz.reshape(NZ, NY, NX, 3)
    g = 0.5 + np.array([-0.5, 0.5]) / np.sqrt(3.0)
    V = 0.0
    faces = [(X[:, :, 0], -1), (X[:, :, -1], +1), (X[:, 0, :], +1), (X[:, -1, :], -1),
             (X[0, :, :], -1), (X[-1, :, :], +1)]
    # orientation: the parametrisation (first, second index) of each face
    # sheet with the sign that makes (d/ds x d/dt) point outward
    for F, sgn in faces:
        for a in range(F.shape[0] - 1):
            for b in range(F.shape[1] - 1):
                p00, p01, p10, p11 = F[a, b], F[a, b + 1], F[a + 1, b], F[a + 1, b + 1]
                for s in g:
                    for t in g:
                        x = (1 - s) * (1 - t) * p00 + (1 - s) * t * p01 + s * (1 - t) * p10 + s * t * p11
                        ds = (1 - t) * (p10 - p00) + t * (p11 - p01)
                        dt = (1 - s) * (p01 - p00) + s * (p11 - p10)
                        V += 0.25 * sgn * np.dot(x, np.cross(dt, ds))
    return V / 3.0


def test_terrain_mass_and_gravity_give_the_volume():
    m = terrain()
    V = divergence_volume(m)
    assert V == pytest.approx(np.prod(EXT), rel=0.05)   # the warp keeps the volume roughly
    M = oracle.assemble(m, mass=np.ones(m.ncell))
    assert np.ones(m.nnode) @ (M @ np.ones(m.nnode)) == pytest.approx(V, rel=1e-12)
    gz = oracle.load_gradz(m, np.ones(m.ncell))
    assert gz @ m.xyz[:, 2] == pytest.approx(V, rel=1e-12)


def test_terrain_constant_flux_convection_is_skew_inside():
    m = terrain()
    a = np.array([3.0, -2.0, 1.5])
    P = m.xyz @ a                                   # linear pressure: constant flux
    C = oracle.assemble(m, kvel=np.ones(m.ncell), P=P, adv_scale=1.0, rho_g=0.0, nq=3).toarray()
    inn = interior(m)
    S = C + C.T
    scale = abs(C).max()
    assert abs(S[np.ix_(inn, inn)]).max() <= 1e-11 * scale
    assert abs(C @ np.ones(m.nnode)).max() <= 1e-11 * scale   # q . grad(1) = 0
    # the flux is -grad P (k = 1): C x_d at interior rows = -a_d int N_a
    Mrow = oracle.assemble(m, mass=np.ones(m.ncell), nq=3) @ np.ones(m.nnode)
    for d in range(3):
        r = C @ m.xyz[:, d]
        assert abs(r[inn] + a[d] * Mrow[inn]).max() <= 1e-10 * abs(a[d] * Mrow).max()


def test_terrain_face_loads_sum_to_face_areas():
    m = terrain()
    Lx, Ly, Lz = EXT
    # side faces stay planar rectangles in x and y; their heights follow the
    # top and bottom surfaces, so compare with the divergence-free check:
    # the x faces are planes x = 0 and x = Lx, and their area is the
    # integral of (top - bottom) along y there
    assert oracle.load_face(m, 4, 1.0).sum() >= Lx * Ly * (1 - 1e-12)   # curved bottom: at least the plane
    for f, x in ((0, 0.0), (1, Lx)):
        NX, NY, NZ = m.dims
        X = m.xyz.reshape(NZ, NY, NX, 3)
        col = X[:, :, 0 if f == 0 else -1, :]
        assert np.allclose(col[..., 0], x)
        yv = col[0, :, 1]
        h = col[-1, :, 2] - col[0, :, 2]
        area = np.sum(0.5 * (h[1:] + h[:-1]) * np.diff(yv))   # h is linear between nodes
        assert oracle.load_face(m, f, 1.0).sum() == pytest.approx(area, rel=1e-12)
