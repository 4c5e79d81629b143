"""The 1-D mass model at 1e6 and 1e7 events stored in FP32, evaluated by the
mixed and the FP64 kernels at random parameter points within +-3 standard
deviations of the generating values, against the oracle on the same
(FP32-valued) events.  Reports the largest and the median errors of the NLL
and of each gradient component."""
import numpy as np
import pytest

import oracle
from paper_2505_12414_amd import datagen as G
from paper_2505_12414_amd import uml
from paper_2505_12414_amd import workloads as W

from gpu_common import TOL, random_points, say, sigmas
from oracle_pool import oracle_points, workers

pytestmark = pytest.mark.gpu

CASES = [(1_000_000, 1000), (10_000_000, 1000)]


@pytest.mark.timeout(1200)
@pytest.mark.parametrize("n,k", CASES, ids=[f"{c[0]}x{c[1]}" for c in CASES])
def test_random_points_mixed_and_fp64(n, k, tmp_path):
    desc = W.mass1d()
    x32 = G.gen_mass1d(n, 77, dtype=np.float32)
    x64 = x32.astype(np.float64)
    om = oracle.Model(desc)
    sig = sigmas(om, x64, om.theta0)
    pts = random_points(om.theta0, sig, om.free, k, seed=n % 9973)
    say(f"case random points n={n} k={k}: oracle on {workers()} processes")
    ref = oracle_points(desc, x64, pts, tmp_path)
    assert all(r[2] == 0 for r in ref)
    for precision in ("fp64", "mixed"):
        um = uml.Model(desc, precision)
        ud = uml.Data(um, x32)
        rel, gerr = [], []
        for th, (nll_o, g_o, _) in zip(pts, ref):
            nll_g, g_g = uml.uml_eval_nll_grad(um, ud, th)
            rel.append(abs(nll_g - nll_o) / abs(nll_o))
            gerr.append(np.abs(g_g - g_o) * sig)  # sig is over the free parameters
        rel, gerr = np.array(rel), np.array(gerr)
        say(f"  {precision}: NLL rel err max {rel.max():.2e} median {np.median(rel):.2e}; "
            f"grad err/sigma max {gerr.max(0)} median {np.median(gerr, 0)}")
        t = TOL[precision]
        assert rel.max() <= t["nll"]
        assert gerr.max() <= t["grad_sigma"]
