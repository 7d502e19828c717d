"""Parity of the HIP operator application (hts_apply_operator) with the
oracle's assembled matrices, element by element.

FP64: |y - y_oracle| <= 1e-13 max|y_oracle| (rounding of a ~200-term sum).
FP32: |y - y_oracle|_i <= 64 eps32 (|A| |x|)_i, the forward error bound of an
inner product evaluated in single precision (coefficients, inputs and the
accumulation each rounded once; 64 covers the sum length).
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import synth
from gpu_util import print_case, to_dev

pytestmark = pytest.mark.gpu

EPS32 = np.finfo(np.float32).eps


def small_cases():
    c = []
    c.append(("c1", synth.config1()))
    c.append(("c2_small", synth.config2(ncells=(20, 18, 9), n_steps=1)))
    c.append(("c3_small", synth.config3(ncells=(33, 17, 12), n_steps=1)))
    c.append(("c4_small", synth.config4_instance(3, n_override=19, n_steps=1)))
    s = synth.config2(ncells=(17, 9, 5), n_steps=1)
    s.name = "odd_17x9x5"
    c.append((s.name, s))
    # several Q1 tiles along x and y (31 x 15 owned node columns) with ragged
    # tails, wells crossing tile edges
    s = synth.config2(ncells=(70, 33, 6), n_steps=1)
    s.name = "tiles_70x33x6"
    c.append((s.name, s))
    # Q2: the same scenarios on 27-node cells (cellwise data unchanged)
    c.append(("c3_q2_small", synth.config3(degree=2, ncells=(17, 16, 5), n_steps=1)))
    s = synth.config2(ncells=(19, 16, 6), n_steps=1)
    s.degree, s.name = 2, "c2_q2_small"
    c.append((s.name, s))
    s = synth.config4_instance(3, n_override=11, n_steps=1)
    s.degree, s.name = 2, "c4_q2_small"
    c.append((s.name, s))
    # graded (rectilinear) Q1 meshes: wells, line heat sources, Dirichlet
    # columns and Neumann faces on non-uniform cells
    s = synth.config2(ncells=(20, 18, 9), n_steps=1)
    s.edges = (synth.graded_edges(0.0, 500.0, 20, [(120.0, 380.0)], ratio=4.0),
               synth.graded_edges(0.0, 500.0, 18, [(200.0, 300.0)]),
               synth.graded_edges(0.0, 100.0, 9, [(60.0, 100.0)], ratio=2.0))
    s.name = "c2_graded"
    c.append((s.name, s))
    s = synth.config3(ncells=(33, 17, 12), n_steps=1)
    s.edges = (synth.graded_edges(0.0, 1000.0, 33, [(250.0, 750.0)]),
               synth.graded_edges(0.0, 1000.0, 17, [(250.0, 750.0)]),
               synth.graded_edges(0.0, 200.0, 12, [(160.0, 200.0)]))
    s.name = "c3_graded"
    c.append((s.name, s))
    c.append(("island_graded", synth.island(ncells=(32, 20, 10), n_steps=1, graded=True)))
    s = synth.island(ncells=(16, 10, 5), n_steps=1, degree=2, graded=True)
    s.name = "island_q2_graded"
    c.append((s.name, s))
    s = synth.config3(degree=2, ncells=(17, 16, 5), n_steps=1)
    s.edges = (synth.graded_edges(0.0, 1000.0, 17, [(250.0, 750.0)]),
               synth.graded_edges(0.0, 1000.0, 16, [(250.0, 750.0)]),
               synth.graded_edges(0.0, 200.0, 5, [(160.0, 200.0)]))
    s.name = "c3_q2_graded"
    c.append((s.name, s))
    # general hexahedra: terrain-following cells over several 15 x 15 tiles
    # with ragged tails, and a box mesh with randomly jittered interior nodes
    c.append(("aquifer_hex_tiles", synth.aquifer_hex(ncells=(40, 33, 6), n_steps=1)))
    s = synth.aquifer_hex(ncells=(17, 9, 5), n_steps=1)
    s.coords = jittered_coords(s, 0.12, seed=5)
    s.name = "jitter_hex"
    c.append((s.name, s))
    return c


def jittered_coords(scn, frac, seed):
    """Box node coordinates with every interior node moved by up to frac
    of a cell width along each axis (boundary nodes stay on their faces)."""
    nx, ny, nz = scn.ncells
    ax = [scn.origin[d] + scn.extent[d] * np.arange(n + 1) / n for d, n in enumerate(scn.ncells)]
    Z, Y, X = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    xyz = np.stack([X.reshape(-1), Y.reshape(-1), Z.reshape(-1)], axis=1)
    rng = np.random.default_rng(seed)
    k, j, i = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
    inner = ((i > 0) & (i < nx) & (j > 0) & (j < ny) & (k > 0) & (k < nz)).reshape(-1)
    h = np.array([scn.extent[d] / scn.ncells[d] for d in range(3)])
    xyz[inner] += frac * h * rng.uniform(-1.0, 1.0, (int(inner.sum()), 3))
    return xyz


def _mesh(hts, scn):
    return hts.from_scenario(scn, initial=False)


def _oracle_reduced(scn, field, P=None, steady=None):
    m = oracle.Mesh.of(scn)
    A = oracle.operator(scn, field, P=P, steady=steady)
    mask, g = oracle.dirichlet(scn, m, field, scn.t0 + scn.dt)
    return A, mask


@pytest.mark.parametrize("name,scn", small_cases(), ids=[c[0] for c in small_cases()])
@pytest.mark.parametrize("field", [0, 1])
def test_apply_parity(hts, name, scn, field):
    import torch
    print_case("apply", name, "field", field)
    m = _mesh(hts, scn)
    om = oracle.Mesh.of(scn)
    rng = np.random.default_rng(11)
    P = None
    if field == 1:
        X, Y, Z = om.coords()
        # a pressure field with a realistic gradient (hydrostatic + drop + noise)
        P = 1e5 + scn.rho_w * scn.g * (scn.extent[2] - Z) - 20.0 * X + 5.0 * rng.standard_normal(om.nnode)
        m.set_state(0, P, scn.t0)
    A, mask = _oracle_reduced(scn, field, P=P)
    x = rng.standard_normal(om.nnode)
    y_ref = oracle.reduced_apply(A, mask, x)
    for prec in (0, 1):
        dt = "float64" if prec == 0 else "float32"
        xd = to_dev(x, dt)
        yd = torch.zeros_like(xd)
        m.apply_operator(field, prec, scn.dt, xd, yd)
        torch.cuda.synchronize()
        y = yd.double().cpu().numpy()
        if prec == 0:
            tol = 1e-13 * np.abs(y_ref).max()
            err = np.abs(y - y_ref)
            assert err.max() <= tol, (name, field, err.max() / np.abs(y_ref).max())
        else:
            if field == 1:
                # the FP32 heat operator reads the pressure as the FP32-rounded
                # piezometric head P + rho_w g z (relative to node 0); the
                # reference uses that same rounded pressure in FP64; z is the
                # node height above node 0 (k dz on a uniform axis)
                NX, NY = om.dims[0], om.dims[1]
                kz = np.arange(om.nnode) // (NX * NY)
                dz = scn.extent[2] / (scn.degree * scn.ncells[2])
                box = getattr(scn, "edges", None) is None and getattr(scn, "coords", None) is None
                zk = kz * dz if box else Z - Z[0]
                rg = scn.rho_w * scn.g
                phi32 = ((P - P[0]) + rg * zk).astype(np.float32)
                Pt = phi32.astype(np.float64) - rg * zk + P[0]
                A, _ = _oracle_reduced(scn, field, P=Pt)
                y_ref = oracle.reduced_apply(A, mask, x)
            Aabs = abs(A.tocsr())
            xm = np.where(mask, 0.0, np.abs(x))
            bound = 64 * EPS32 * (Aabs @ xm)
            bound = np.where(mask, EPS32 * np.abs(x), bound) + 1e-30
            err = np.abs(y - y_ref)
            assert np.all(err <= bound), (name, field, np.max(err / bound))


def test_apply_steady_pressure(hts):
    scn = synth.config1()
    print_case("apply steady c1")
    import torch
    m = _mesh(hts, scn)
    A, mask = _oracle_reduced(scn, 0, steady=True)
    x = np.random.default_rng(3).standard_normal(m.nnode)
    y_ref = oracle.reduced_apply(A, mask, x)
    xd = to_dev(x)
    yd = torch.zeros_like(xd)
    m.apply_operator(0, 0, 0.0, xd, yd)          # dt <= 0 selects the steady operator
    torch.cuda.synchronize()
    assert np.abs(yd.cpu().numpy() - y_ref).max() <= 1e-13 * np.abs(y_ref).max()


def test_apply_is_bitwise_reproducible(hts):
    import torch
    scn = synth.config2(ncells=(20, 18, 9), n_steps=1)
    print_case("apply reproducible")
    m = _mesh(hts, scn)
    x = to_dev(np.random.default_rng(5).standard_normal(m.nnode))
    y1 = torch.zeros_like(x)
    y2 = torch.zeros_like(x)
    m.apply_operator(1, 0, scn.dt, x, y1)
    m.apply_operator(1, 0, scn.dt, x, y2)
    torch.cuda.synchronize()
    assert torch.equal(y1, y2)
