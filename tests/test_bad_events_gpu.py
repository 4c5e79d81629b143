"""The count of events outside the domain of Eq. 1's logarithm (P <= 0 or
not finite) from the library, against the oracle's count on the same events
and parameter point."""
import math

import numpy as np
import pytest

import oracle
from paper_2505_12414_amd import uml
from paper_2505_12414_amd import workloads as W

from gpu_common import rng_events, say

pytestmark = pytest.mark.gpu


def _ambiguous(om, x64, th, rel):
    """Events whose density lies within rel of zero, relative to the largest
    density over the sample: there an FP32 evaluation may decide the sign
    differently from the oracle's FP64 one."""
    p = om.pdf(x64, th)
    return int(np.sum(np.abs(p) <= rel * np.max(np.abs(p))))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_bad_event_count_matches_oracle(precision):
    desc = W.pwave3d()
    dtype = np.float32 if precision == "mixed" else np.float64
    x = rng_events(desc, 50021, 9, dtype)
    x64 = x.astype(np.float64)
    um = uml.Model(desc, precision)
    ud = uml.Data(um, x)
    om = oracle.Model(desc)
    # F_L > 1 or a large S-term makes the angular rate negative in part of
    # the space
    for th in ([1.6, 0, 0, 0, 0, 0, 0, 0.0], [0.7, 0.9, -0.5, 0.6, 0.0, 0.0, 0.0, 0.4]):
        th = np.array(th)
        _, _, _, bad_o = om.nll(x64, th)
        say(f"case bad events precision={precision} theta={th.tolist()} oracle {bad_o}")
        assert bad_o > 0
        nll, g = uml.uml_eval_nll_grad(um, ud, th)
        assert nll == math.inf and np.all(g == 0)
        bad_g = uml.uml_eval_bad_events(um, ud, th)
        if precision == "fp64":
            assert bad_g == bad_o
        else:
            assert abs(bad_g - bad_o) <= _ambiguous(om, x64, th, 1e-6)
    # inside the domain: no bad events, and the count agrees with a finite NLL
    th = om.theta0
    assert uml.uml_eval_bad_events(um, ud, th) == 0
    assert math.isfinite(uml.uml_eval_nll_grad(um, ud, th)[0])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_bad_event_count_outside_parameter_domain(precision):
    """A fraction outside [0, 1] or a width <= 0: every event counts."""
    desc = W.mass1d()
    dtype = np.float32 if precision == "mixed" else np.float64
    n = 3001
    um = uml.Model(desc, precision)
    ud = uml.Data(um, rng_events(desc, n, 3, dtype))
    for th in ([5.28, 0.02, -1.5, 1.2], [5.28, -0.02, -1.5, 0.3]):
        say(f"case bad events outside the domain precision={precision} theta={th}")
        assert uml.uml_eval_bad_events(um, ud, np.array(th)) == n


def test_fit_reports_bad_event_count():
    """A fit whose start point has P <= 0 somewhere stops at once and
    reports how many events are outside the logarithm's domain."""
    desc = W.pwave3d()
    x = rng_events(desc, 20011, 4, np.float64)
    um = uml.Model(desc, "fp64")
    ud = uml.Data(um, x)
    om = oracle.Model(desc)
    start = np.array([1.6, 0, 0, 0, 0, 0, 0, 0.0])
    _, _, _, bad_o = om.nll(x, start)
    say(f"case fit with a non-positive start: oracle count {bad_o}")
    r = uml.uml_fit(um, ud, start=start)
    assert r["status_name"] == "pdf_nonpositive"
    assert r["n_bad_events"] == bad_o
