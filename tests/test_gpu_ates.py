"""Three-dimensional analogue of the hot-water injection benchmark (Section 2,
Table 1): three formations, a wellbore injecting through the aquifer and
held at the injection temperature there, Table 1 materials (bulk values,
water heat capacity 1e6 J/m^3/K).

Parity with the oracle as in the other solver tests: the GPU solves to 1e-12
and the oracle to the FP64 floor; FP64 within 1e-10 relative, the
FP32-refined path within 1e-8 (pressure) and 1e-6 K (temperature).
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import print_case

pytestmark = pytest.mark.gpu


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("ncells,degree,mode", [((16, 16, 24), 1, 0), ((16, 16, 24), 1, 1),
                                                ((20, 12, 30), 1, 0), ((8, 8, 12), 2, 0)])
def test_ates_small_steps(hts, ncells, degree, mode):
    """Three daily injection steps against the oracle."""
    print_case("ates", ncells, "p", degree, "mode", mode)
    scn = synth.ates(ncells=ncells, degree=degree, n_steps=3)
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
    # injection raises the pressure at the wellbore above hydrostatic
    assert P.max() > 1e5 + scn.rho_w * scn.g * 200.0 + 1e5
    if mode == 0:
        assert rel(P, Po) <= 1e-10
        assert rel(T, To) <= 1e-10
        assert np.abs(T - To).max() <= 1e-7
    else:
        assert rel(P, Po) <= 1e-8
        assert np.abs(T - To).max() <= 1e-6
