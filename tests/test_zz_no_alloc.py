"""The allocation-free operator entry point against hts_apply_operator.

hts_apply_operator_noalloc runs the same kernels on the same data with its
buffers in a static device array, so its result must equal that of
hts_apply_operator bit for bit, for both fields and precisions, on Q1, Q2,
graded and general hexahedral meshes.  Two calls in a row share the array: the second, on a
smaller mesh, must not see anything of the first.  A mesh whose buffers do
not fit is refused before any device work, and a changed mesh must be
prepared again by the allocating path first.
"""
import numpy as np
import pytest

import synth
from gpu_util import print_case, to_dev

pytestmark = pytest.mark.gpu


def cases():
    return [("aquifer 40x36x20 Q1", synth.config2(ncells=(40, 36, 20), n_steps=1)),
            ("aquifer 17x13x9 Q1", synth.config2(ncells=(17, 13, 9), n_steps=1)),
            ("piles 24x24x12 Q2", synth.config3(degree=2, ncells=(24, 24, 12), n_steps=1)),
            ("island graded 32x20x8 Q1", synth.island(ncells=(32, 20, 8), n_steps=1, graded=True, degree=1)),
            ("terrain hexahedra 20x16x8 Q1", synth.aquifer_hex(ncells=(20, 16, 8), n_steps=1))]


def check(hts, label, scn, rng):
    import torch
    m = hts.from_scenario(scn)
    n = m.nnode
    for field in (0, 1):
        for prec in (0, 1):
            print_case("noalloc", label, "field", field, "prec", prec)
            dt = "float64" if prec == 0 else "float32"
            x = to_dev(rng.standard_normal(n), dt)
            y1 = torch.full_like(x, np.nan)
            y2 = torch.full_like(x, -7.0)
            m.apply_operator(field, prec, scn.dt, x, y1)
            m.apply_operator_noalloc(field, prec, scn.dt, x, y2)
            torch.cuda.synchronize()
            a, b = y1.cpu().numpy(), y2.cpu().numpy()
            assert np.all(np.isfinite(a))
            assert np.array_equal(a.view(np.uint8), b.view(np.uint8)), (label, field, prec)
    return m


def test_noalloc_matches_apply_operator(hts):
    rng = np.random.default_rng(3)
    for label, scn in cases():        # the second case is smaller than the first
        check(hts, label, scn, rng)


def test_noalloc_refuses_unprepared_and_oversized(hts):
    import torch
    s = synth.config2(ncells=(16, 16, 8), n_steps=1)
    m = hts.from_scenario(s, initial=False)
    m.set_state(0, np.full(m.nnode, 2e5), 0.0)
    x = torch.zeros(m.nnode, dtype=torch.float64, device="cuda:0")
    y = torch.zeros_like(x)
    with pytest.raises(hts.HtsError):
        m.apply_operator_noalloc(0, 0, s.dt, x, y)      # not prepared yet
    m.apply_operator(0, 0, s.dt, x, y)                  # prepares the mesh data
    m.apply_operator_noalloc(0, 0, s.dt, x, y)
    # a mesh of 12.8 M nodes: its FP32 heat pressure alone exceeds the scratch
    nc = (320, 320, 124)
    big = synth.Scenario("big", (0.0, 0.0, 0.0), (1000.0, 1000.0, 200.0), nc, 1,
                         permeability=np.full(nc[0] * nc[1] * nc[2], 1e-12),
                         porosity=np.full(nc[0] * nc[1] * nc[2], 0.3),
                         lambda_solid=np.full(nc[0] * nc[1] * nc[2], 2.5),
                         rhoc_solid=np.full(nc[0] * nc[1] * nc[2], 2e6))
    mb = hts.from_scenario(big)
    xb = torch.zeros(mb.nnode, dtype=torch.float32, device="cuda:0")
    yb = torch.zeros_like(xb)
    mb.apply_operator(1, 1, big.dt, xb, yb)
    with pytest.raises(hts.HtsError):
        mb.apply_operator_noalloc(1, 1, big.dt, xb, yb)
    torch.cuda.synchronize()
