"""Serving loop: continuous batching with memory-budget admission; each fit
in the mix equals, bit for bit, the same fit run alone."""
import time

import numpy as np
import pytest

from paper_2505_12414_amd import datagen as G
from paper_2505_12414_amd import uml
from paper_2505_12414_amd import workloads as W

from gpu_common import say

pytestmark = pytest.mark.gpu


def toys(k, seed0, lo=500, hi=20000):
    rng = np.random.default_rng(seed0)
    sizes = np.exp(rng.uniform(np.log(lo), np.log(hi), k)).astype(int)
    return [G.gen_angmass4d(int(n), seed0 + 1 + i, dtype=np.float32) for i, n in enumerate(sizes)]


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_server_results_equal_lone_fits(precision):
    desc = W.angmass4d()
    um = uml.Model(desc, precision)
    events = toys(24, 100)
    if precision == "fp64":
        events = [e.astype(np.float64) for e in events]
    srv = uml.Server(um, max_slots=6, hbm_budget=256 << 20)
    say(f"case server mix precision={precision}")
    tickets = {}
    for i, ev in enumerate(events):
        tickets[srv.submit(ev)] = i
        if i % 5 == 4:
            time.sleep(0.002)   # requests keep arriving while others run
    srv.drain()
    res = srv.poll(max_results=100)
    st = srv.stats()
    srv.close()
    assert len(res) == len(events) and st["finished"] == len(events)
    assert st["iterations"] > 0
    for r in res:
        i = tickets[r["ticket"]]
        d = uml.Data(um, events[i])
        alone = uml.uml_fit(um, d, um.theta0)
        assert r["status"] == alone["status"] == 0, (i, r["status_name"])
        assert np.array_equal(r["theta"], alone["theta"]), i
        assert np.array_equal(r["errors"], alone["errors"]), i
        assert r["nll"] == alone["nll"] and r["n_iter"] == alone["n_iter"]
        assert r["latency_s"] > 0


def test_admission_respects_the_memory_budget():
    desc = W.angmass4d()
    um = uml.Model(desc, "mixed")
    events = toys(12, 7, 20000, 40000)
    budget = 6 << 20   # room for about two of these requests at a time
    srv = uml.Server(um, max_slots=64, hbm_budget=budget)
    for ev in events:
        srv.submit(ev)
    peak = 0
    t0 = time.time()
    while time.time() - t0 < 60:
        st = srv.stats()
        peak = max(peak, st["resident_bytes"])
        assert st["resident_bytes"] <= budget
        if st["finished"] == len(events):
            break
        time.sleep(0.001)
    res = srv.poll(max_results=100)
    srv.close()
    assert len(res) == len(events) and all(r["status"] == 0 for r in res)
    assert 0 < peak <= budget
    say(f"  peak resident {peak} of budget {budget}")


def test_over_budget_and_bad_requests():
    desc = W.angmass4d()
    um = uml.Model(desc, "mixed")
    srv = uml.Server(um, max_slots=4, hbm_budget=1 << 20)
    with pytest.raises(uml.UmlError) as e:
        srv.submit(G.gen_angmass4d(200000, 3))
    assert e.value.code == uml.UML_E_BUDGET
    bad = G.gen_angmass4d(1000, 4)
    bad[0, 5] = 7.0
    with pytest.raises(uml.UmlError) as e:
        srv.submit(bad)
    assert e.value.code == uml.UML_E_EVENT_DOMAIN
    # an unphysical start finishes at once; its neighbours are unaffected
    good = [G.gen_angmass4d(3000, 10 + i) for i in range(3)]
    start_bad = um.theta0.copy()
    start_bad[0] = 3.0
    t_bad = srv.submit(G.gen_angmass4d(3000, 20), start=start_bad)
    t_good = [srv.submit(ev) for ev in good]
    srv.drain()
    res = {r["ticket"]: r for r in srv.poll(max_results=10)}
    srv.close()
    assert res[t_bad]["status_name"] == "pdf_nonpositive"
    for t, ev in zip(t_good, good):
        alone = uml.uml_fit(um, uml.Data(um, ev), um.theta0)
        assert np.array_equal(res[t]["theta"], alone["theta"])
