"""The P-wave's event-only terms precomputed once per dataset (stored as
extra columns) against the kernel that recomputes them: the same terms from
the same device arithmetic give bitwise the same NLL, gradient and fits; and
the precomputed variant matches the oracle."""
import numpy as np
import pytest

import oracle
from paper_2505_12414_amd import uml
from paper_2505_12414_amd import workloads as W

from gpu_common import assert_parity, compare, random_points, rng_events, say, sigmas

pytestmark = pytest.mark.gpu

MODELS = [
    ("angmass4d", W.angmass4d, 30_001),
    ("pwave3d", lambda: W.pwave3d((0.45, 0.12, -0.23, 0.31, -0.17, 0.08, -0.11, 0.05)), 20_001),
]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name,mk,n", MODELS, ids=[m[0] for m in MODELS])
@pytest.mark.parametrize("weighted", [False, True], ids=["unweighted", "weighted"])
def test_precomputed_terms_equal_recomputed(name, mk, n, precision, weighted):
    desc = mk()
    dtype = np.float32 if precision == "mixed" else np.float64
    x = rng_events(desc, n, 61, dtype)
    w = np.random.default_rng(2).uniform(0.5, 1.5, n).astype(dtype) if weighted else None
    ua = uml.Model(desc, precision)
    ub = uml.Model(desc, precision, precompute=True)
    assert "Q" in ub.describe()
    da, db = uml.Data(ua, x, weights=w), uml.Data(ub, x, weights=w)
    om = oracle.Model(desc)
    sig = sigmas(om, x.astype(np.float64), om.theta0)
    say(f"case precompute {name} precision={precision} weighted={weighted}")
    for th in random_points(om.theta0, sig, om.free, 4, seed=5):
        a, b = uml.uml_eval_nll_grad(ua, da, th), uml.uml_eval_nll_grad(ub, db, th)
        assert a[0] == b[0] and np.array_equal(a[1], b[1])
    rel, gerr, _ = compare(desc, precision, x, th, w=w, um=ub, ud=db, om=om, sig=sig,
                           tag=f"precompute-{name}")
    assert_parity(rel, gerr, precision, f"precompute-{name}")


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_precomputed_fit_and_generation(precision):
    desc = W.angmass4d()
    ua = uml.Model(desc, precision)
    ub = uml.Model(desc, precision, precompute=True)
    da, db = uml.Data.generate(ua, 25_000, 8), uml.Data.generate(ub, 25_000, 8)
    assert np.array_equal(da.download(), db.download())
    ra, rb = uml.uml_fit(ua, da), uml.uml_fit(ub, db)
    assert ra["status"] == rb["status"] == 0
    assert np.array_equal(ra["theta"], rb["theta"]) and np.array_equal(ra["errors"], rb["errors"])


def test_precomputed_model_in_the_server():
    ub = uml.Model(W.angmass4d(), "mixed", precompute=True)
    srv = uml.Server(ub, max_slots=4)
    sizes = [900, 12000, 3000, 40000]
    tickets = {srv.submit_generated(n, 70 + i): i for i, n in enumerate(sizes)}
    srv.drain()
    res = srv.poll(max_results=10)
    srv.close()
    for r in res:
        i = tickets[r["ticket"]]
        alone = uml.uml_fit(ub, uml.Data.generate(ub, sizes[i], 70 + i))
        assert r["status"] == 0 and np.array_equal(r["theta"], alone["theta"])
