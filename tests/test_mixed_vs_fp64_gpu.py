"""The mixed-precision event kernel (FP32 per event, FP64 sums) against the
FP64 kernel on the same FP32-valued events, at 50 random points within +-3
standard deviations, at the sizes where a coherent per-event rounding error
would be largest in units of sigma.  The FP64 kernel is itself held to the
oracle at 1e-8 sigma (test_parity_gpu); this test measures what the FP32
arithmetic adds, per parameter, and prints it (run with -s for the table)."""
import numpy as np
import pytest

import oracle
from paper_2505_12414_amd import datagen as G
from paper_2505_12414_amd import uml
from paper_2505_12414_amd import workloads as W

from gpu_common import TOL, random_points, say, sigmas

pytestmark = pytest.mark.gpu

CASES = [("angmass4d", W.angmass4d, G.gen_angmass4d, 1_000_000),
         ("angmass4d", W.angmass4d, G.gen_angmass4d, 4_000_000),
         ("mass1d", W.mass1d, G.gen_mass1d, 10_000_000),
         ("mass1d", W.mass1d, G.gen_mass1d, 50_000_000)]


@pytest.mark.timeout(600)
@pytest.mark.parametrize("name,mk,gen,n", CASES, ids=[f"{c[0]}-{c[3]}" for c in CASES])
def test_mixed_against_fp64(name, mk, gen, n):
    desc = mk()
    x = gen(n, 2024, dtype=np.float32)
    om = oracle.Model(desc)
    sig = sigmas(om, x.astype(np.float64), om.theta0)
    pts = random_points(om.theta0, sig, om.free, 50, seed=11)
    say(f"case mixed-vs-fp64 {name} n={n}")
    mm = uml.Model(desc, "mixed")
    dm = uml.Data(mm, x)
    m64 = uml.Model(desc, "fp64")
    d64 = uml.Data(m64, x.astype(np.float64))
    gerr, rel = [], []
    for th in pts:
        n1, g1 = uml.uml_eval_nll_grad(mm, dm, th)
        n2, g2 = uml.uml_eval_nll_grad(m64, d64, th)
        gerr.append(np.abs(g1 - g2) * sig)
        rel.append(abs(n1 - n2) / abs(n2))
    gerr, rel = np.array(gerr), np.array(rel)
    say(f"  {name} n={n:.0e} points=50: grad err/sigma max {gerr.max():.2e} "
        f"median-of-max {np.median(gerr.max(1)):.2e} nll rel max {rel.max():.2e}")
    say("  per-parameter max " + np.array2string(gerr.max(0), precision=1, max_line_width=220))
    assert rel.max() <= TOL["mixed"]["nll"]
    assert gerr.max() <= TOL["mixed"]["grad_sigma"]
