"""The autotuner changes only how FFT sub-transforms are grouped into workgroups and how many
right-hand sides a spreading pass takes: results before and after tuning agree to rounding, in one
dimension (one pass and two passes) and two."""
import numpy as np
import pytest

import workloads as W

from gpu_util import dev, host, nodes_dev, rel

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("M,d,precision", [((5000,), 1, "f32"), ((5000,), 1, "f64"), ((96,), 1, "f64"),
                                           ((48, 40), 2, "f32")])
def test_autotuned_plan_matches_untuned(M, d, precision):
    from paper_1811_05335_amd import NfftPlan
    g = W.rng(41)
    N = 3 * int(np.prod(M)) // 2
    x = W.uniform_nodes(g, N, d)
    fh = dev(W.complex_normal(g, (2,) + M), precision)
    f = dev(W.complex_normal(g, (2, N)), precision)
    P = NfftPlan(M, nodes_dev(x), sigma=2.0, m=4, precision=precision, rho=1e-8, max_rhs=2)
    before = [host(P.trafo(fh)), host(P.adjoint(f))]
    rows = P.autotune(reps=3)
    # 0: the default shape won; both passes of a direction are default or both are set
    assert all(v in (0, 1, 2, 4, 8, 16) for k, v in rows.items() if k != "spread_rhs")
    # right-hand sides per spreading pass: tuned among 1 and max_rhs = 2
    assert rows["spread_rhs"] in (1, 2)
    assert (rows["to_grid_0"] == 0) == (rows["to_grid_1"] == 0)
    assert (rows["to_coeff_0"] == 0) == (rows["to_coeff_1"] == 0)
    after = [host(P.trafo(fh)), host(P.adjoint(f))]
    tol = 1e-14 if precision == "f64" else 1e-6
    for a, b in zip(after, before):
        assert rel(a, b) <= tol
    P.close()
