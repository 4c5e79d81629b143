"""Pseudo-experiments drawn on the device against the oracle's generator:
the same counter-based stream and the same sampling procedure give the same
events (FP64 storage: equal to rounding; FP32 storage: the oracle's values
rounded by the storage rule).  At 1e7 events, sampled events are drawn by the
oracle one by one."""
import numpy as np
import pytest

import oracle
from paper_2505_12414_amd import uml
from paper_2505_12414_amd import workloads as W

from gpu_common import cheb_desc, exp_desc, gauss_desc, mix_desc, say

pytestmark = pytest.mark.gpu

MODELS = [
    ("mass1d", W.mass1d),
    ("angmass4d", W.angmass4d),
    ("pwave3d", lambda: W.pwave3d((0.45, 0.12, -0.23, 0.31, -0.17, 0.08, -0.11, 0.05))),
    ("gauss", lambda: gauss_desc(mu=5.3, sigma=0.1)),
    ("exp", exp_desc),
    ("cheb4", lambda: cheb_desc((0.1, -0.2, 0.05, 0.1))),
    ("mix3", lambda: mix_desc(3)),
    ("mix4", lambda: mix_desc(4)),
    ("shared_leaf", lambda: shared_leaf_desc()),
]


def shared_leaf_desc():
    """f1 G(m) + (1 - f1) (f2 G(m) + (1 - f2) E(m)) with the one Gaussian node
    under both sums (drawn from either branch)."""
    return {"dims": [{"name": "m", "lo": 5.0, "hi": 5.6}],
            "params": [{"name": "mu", "value": 5.28}, {"name": "s", "value": 0.03},
                       {"name": "lambda", "value": -1.2}, {"name": "f1", "value": 0.35},
                       {"name": "f2", "value": 0.6}],
            "nodes": [{"kind": "gauss", "dims": [0], "params": [0, 1]},
                      {"kind": "exp", "dims": [0], "params": [2]},
                      {"kind": "sum", "children": [0, 1], "params": [4]},
                      {"kind": "sum", "children": [0, 2], "params": [3]}],
            "root": 3}


def storage(x64, desc, precision):
    """The library's storage of FP64 values: FP64 as is; FP32 the nearest
    value, moved one step inwards if rounding left the range."""
    if precision == "fp64":
        return x64
    out = x64.astype(np.float32)
    for d, dim in enumerate(desc["dims"]):
        f = out[d]
        up = f.astype(np.float64) > dim["hi"]
        f[up] = np.nextafter(f[up], np.float32(-np.inf))
        dn = f.astype(np.float64) < dim["lo"]
        f[dn] = np.nextafter(f[dn], np.float32(np.inf))
    return out


def compare(got, want, precision, tag):
    if precision == "fp64":
        scale = np.maximum(np.abs(want), 1.0)
        err = np.abs(got - want) / scale
        say(f"  {tag}: max rel diff {err.max():.2e}")
        assert err.max() <= 1e-13, tag
    else:
        diff = got != want
        ulps = np.abs(got.view(np.int32).astype(np.int64) - want.view(np.int32).astype(np.int64))
        say(f"  {tag}: {int(diff.sum())} of {diff.size} FP32 values differ, max {int(ulps.max())} ulp")
        assert ulps.max() <= 1, tag
        assert diff.sum() <= 1e-4 * diff.size, tag


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name,mk", MODELS, ids=[m[0] for m in MODELS])
def test_generated_events_equal_oracle(name, mk, precision):
    desc = mk()
    um = uml.Model(desc, precision)
    om = oracle.Model(desc)
    n, seed = 50_001, 777
    say(f"case generate {name} precision={precision} n={n}")
    d = uml.Data.generate(um, n, seed)
    got = d.download()
    x, bad = om.generate(n, seed)
    assert bad == 0
    compare(got, storage(x, desc, precision), precision, name)


def test_generation_at_1e7_events_sampled():
    desc = W.angmass4d()
    um = uml.Model(desc, "mixed")
    om = oracle.Model(desc)
    n, seed = 10_000_000, 4242
    say(f"case generate angmass4d n={n}")
    got = uml.Data.generate(um, n, seed).download()
    idx = np.sort(np.random.default_rng(1).choice(n, 3000, replace=False))
    want = np.stack([om.generate(1, seed, i0=int(i))[0][:, 0] for i in idx], axis=1)
    compare(got[:, idx], storage(want, desc, "mixed"), "mixed", "1e7 sampled")


@pytest.mark.parametrize("n", [300_000, 600_000])
def test_generation_with_several_events_per_lane_sampled(n):
    """Launches of 3e5 and 6e5 events draw two and four events per lane (the
    lanes take the next event of their block as each one completes): sampled
    events still equal the oracle's."""
    desc = W.angmass4d()
    um = uml.Model(desc, "fp64")
    om = oracle.Model(desc)
    seed = 515
    say(f"case generate angmass4d n={n} (several events per lane)")
    got = uml.Data.generate(um, n, seed).download()
    idx = np.sort(np.random.default_rng(n).choice(n, 1000, replace=False))
    idx[-1] = n - 1  # the last event of the last, partial block
    want = np.stack([om.generate(1, seed, i0=int(i))[0][:, 0] for i in idx], axis=1)
    compare(got[:, idx], want, "fp64", f"{n} sampled")


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_fit_to_generated_toy_equals_fit_to_uploaded_toy(precision):
    """Events drawn on the device and the same events uploaded from the host
    give the same fit, bit for bit."""
    desc = W.angmass4d()
    um = uml.Model(desc, precision)
    d = uml.Data.generate(um, 20_000, 99)
    x = d.download()
    r1 = uml.uml_fit(um, d)
    r2 = uml.uml_fit(um, uml.Data(um, x))
    assert r1["status"] == 0
    assert np.array_equal(r1["theta"], r2["theta"]) and np.array_equal(r1["errors"], r2["errors"])


def test_generation_errors():
    desc = W.mass1d()
    um = uml.Model(desc, "mixed")
    th = um.theta0.copy()
    th[3] = 1.5                                  # fraction outside [0, 1]
    with pytest.raises(uml.UmlError) as e:
        uml.Data.generate(um, 100, 1, theta=th)
    assert e.value.code == uml.UML_E_INVALID
    g = uml.Model(gauss_desc(mu=4.0, sigma=0.01), "mixed")   # window 100 sigma away
    with pytest.raises(uml.UmlError) as e:
        uml.Data.generate(g, 64, 1)
    assert e.value.code == uml.UML_E_GENERATION
