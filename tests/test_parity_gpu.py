"""GPU parity: NLL and gradient from the HIP kernels (through the C ABI)
against the oracle on the same seeded events and parameter points."""
import math

import numpy as np
import pytest

import oracle
from paper_2505_12414_amd import uml
from paper_2505_12414_amd import workloads as W

from gpu_common import (TOL, assert_parity, cheb_desc, compare, exp_desc, gauss_desc, mix_desc,
                        random_points, rng_events, say, sig4d_desc, sigmas)
from oracle_pool import oracle_points, workers

pytestmark = pytest.mark.gpu

FAMILIES = [
    ("mass1d", W.mass1d, 100003),
    ("angmass4d", W.angmass4d, 50001),
    ("pwave3d", lambda: W.pwave3d((0.6, 0.05, -0.1, 0.1, 0.08, -0.05, 0.03, -0.02)), 30001),
    ("sig4d", sig4d_desc, 30001),
    ("gauss", gauss_desc, 20011),
    ("exp", exp_desc, 20011),
    ("cheb1", lambda: cheb_desc((0.3,)), 20011),
    ("cheb2", lambda: cheb_desc((0.1, 0.05)), 20011),
    ("cheb3", lambda: cheb_desc((0.1, -0.2, 0.05)), 20011),
    ("cheb4", lambda: cheb_desc((0.1, -0.2, 0.05, 0.1)), 20011),
    # three and four components: the max-shifted mixture of the event kernel
    ("mix3", lambda: mix_desc(3), 20011),
    ("mix4", lambda: mix_desc(4), 20011),
]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name,mk,n", FAMILIES, ids=[f[0] for f in FAMILIES])
def test_nll_and_gradient_match_oracle(name, mk, n, precision):
    desc = mk()
    dtype = np.float32 if precision == "mixed" else np.float64
    x = rng_events(desc, n, 1000 + n, dtype)
    om = oracle.Model(desc)
    um = uml.Model(desc, precision)
    ud = uml.Data(um, x)
    th0 = om.theta0
    sig = sigmas(om, x.astype(np.float64), th0)
    for k, th in enumerate([th0] + random_points(th0, sig, om.free, 3, seed=7)):
        tag = f"{name}[{k}]"
        rel, gerr, vals = compare(desc, precision, x, th, um=um, ud=ud, om=om, sig=sig, tag=tag)
        say(f"  nll rel err {rel:.2e}  grad err/sigma max {gerr.max():.2e}")
        assert_parity(rel, gerr, precision, tag)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_weighted_4d(precision):
    desc = W.angmass4d()
    dtype = np.float32 if precision == "mixed" else np.float64
    x = rng_events(desc, 40009, 77, dtype)
    w = np.random.default_rng(3).uniform(0.5, 1.5, x.shape[1]).astype(dtype)
    om = oracle.Model(desc)
    th = om.theta0.copy()
    th[0] += 0.02
    th[17] -= 0.01
    rel, gerr, _ = compare(desc, precision, x, th, w=w, om=om, tag="weighted4d")
    assert_parity(rel, gerr, precision, "weighted4d")


@pytest.mark.parametrize("precision,tile", [("mixed", 1024), ("fp64", 512)])
def test_edge_sizes(precision, tile):
    """Empty data, one event and sizes around one tile (smallest data sets use
    the smallest tiles: 4 events per lane in mixed mode, 2 in FP64)."""
    desc = W.mass1d()
    dtype = np.float32 if precision == "mixed" else np.float64
    um = uml.Model(desc, precision)
    om = oracle.Model(desc)
    th = om.theta0
    for n in [0, 1, 3, tile - 1, tile, tile + 1, 2 * tile + 5]:
        x = rng_events(desc, max(n, 1), 500 + n, dtype)[:, :n]
        say(f"case edge n={n} precision={precision}")
        ud = uml.Data(um, x)
        nll_g, g_g = uml.uml_eval_nll_grad(um, ud, th)
        if n == 0:
            assert nll_g == 0.0 and np.all(g_g == 0.0)
            continue
        nll_o, g_o, _, _ = om.nll(x.astype(np.float64), th, order=1)
        tol = 1e-12 if precision == "fp64" else 1e-6
        assert abs(nll_g - nll_o) <= tol * max(1.0, abs(nll_o))
        assert np.allclose(g_g, g_o, rtol=1e-10 if precision == "fp64" else 1e-4,
                           atol=(1e-9 if precision == "fp64" else 2e-3) * math.sqrt(n) / 0.02)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_nonpositive_density_and_domain(precision):
    desc = W.pwave3d()
    dtype = np.float32 if precision == "mixed" else np.float64
    x = rng_events(desc, 5003, 9, dtype)
    um = uml.Model(desc, precision)
    ud = uml.Data(um, x)
    th = np.array([2.5, 0, 0, 0, 0, 0, 0, 0.0])  # F_L > 1: negative rate somewhere
    say(f"case nonpositive precision={precision}")
    with pytest.raises(uml.UmlError) as e:
        uml.uml_eval_nll_grad(um, ud, th, allow_nonpositive=False)
    assert e.value.code == uml.UML_E_PDF_NONPOSITIVE
    nll, g = uml.uml_eval_nll_grad(um, ud, th)
    assert nll == math.inf and np.all(g == 0)
    # outside the domain: fraction > 1 and sigma <= 0
    d1 = W.mass1d()
    um1 = uml.Model(d1, precision)
    ud1 = uml.Data(um1, rng_events(d1, 1000, 3, dtype))
    for th in ([5.28, 0.02, -1.5, 1.2], [5.28, -0.02, -1.5, 0.3]):
        nll, g = uml.uml_eval_nll_grad(um1, ud1, np.array(th))
        assert nll == math.inf and np.all(g == 0)
    # the good point still evaluates afterwards
    nll, _ = uml.uml_eval_nll_grad(um1, ud1, np.array([5.28, 0.02, -1.5, 0.3]))
    assert math.isfinite(nll)


def test_events_outside_range_are_rejected():
    desc = W.mass1d()
    um = uml.Model(desc, "fp64")
    x = rng_events(desc, 100, 1, np.float64)
    x[0, 17] = 5.7
    with pytest.raises(uml.UmlError) as e:
        uml.Data(um, x)
    assert e.value.code == uml.UML_E_EVENT_DOMAIN
    x[0, 17] = np.nan
    with pytest.raises(uml.UmlError) as e:
        uml.Data(um, x)
    assert e.value.code == uml.UML_E_EVENT_DOMAIN


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_repeated_evaluations_are_bitwise_identical(precision):
    desc = W.angmass4d()
    dtype = np.float32 if precision == "mixed" else np.float64
    x = rng_events(desc, 200003, 5, dtype)
    um = uml.Model(desc, precision)
    ud = uml.Data(um, x)
    th = um.theta0
    say(f"case determinism precision={precision}")
    ref = uml.uml_eval_nll_grad(um, ud, th)
    for _ in range(5):
        got = uml.uml_eval_nll_grad(um, ud, th)
        assert got[0] == ref[0] and np.array_equal(got[1], ref[1])
    # a second handle on the same events gives the same bits
    ud2 = uml.Data(um, x)
    got = uml.uml_eval_nll_grad(um, ud2, th)
    assert got[0] == ref[0] and np.array_equal(got[1], ref[1])


def test_device_entry_point_with_torch_tensors():
    import torch
    desc = W.angmass4d()
    x = rng_events(desc, 100000, 6, np.float32)
    um = uml.Model(desc, "mixed")
    ud = uml.Data(um, torch.from_numpy(x).cuda())   # device-source upload
    ref = uml.uml_eval_nll_grad(um, ud, um.theta0)
    d_theta = torch.tensor(um.theta0, dtype=torch.float64, device="cuda")
    d_out = torch.empty(1 + um.n_free, dtype=torch.float64, device="cuda")
    say("case device entry point")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        uml.uml_eval_nll_grad_dev(um, ud, d_theta, d_out)
    s.synchronize()
    out = d_out.cpu().numpy()
    assert out[0] == ref[0] and np.array_equal(out[1:], ref[1])


FULL = [
    ("angmass4d", W.angmass4d, 1_000_000, "mixed", 50),
    ("angmass4d", W.angmass4d, 1_000_000, "fp64", 10),
    ("mass1d", W.mass1d, 1_000_000, "mixed", 50),
    ("mass1d", W.mass1d, 10_000_000, "mixed", 50),
    ("mass1d", W.mass1d, 10_000_000, "fp64", 10),
    # larger tiles (32 and 64 events per thread) and the sizes where a
    # coherent per-event error would be largest in units of sigma
    ("angmass4d", W.angmass4d, 4_000_000, "mixed", 20),
    ("mass1d", W.mass1d, 50_000_000, "mixed", 20),
]


@pytest.mark.timeout(600)
@pytest.mark.parametrize("name,mk,n,precision,k", FULL,
                         ids=[f"{f[0]}-{f[2]}-{f[3]}" for f in FULL])
def test_full_size_parity(name, mk, n, precision, k, tmp_path):
    """The benchmark sizes, in the launch configuration the benchmark times,
    at k random points within +-3 standard deviations (the oracle's values
    from parallel CPU processes); the largest error over the points is
    asserted."""
    desc = mk()
    dtype = np.float32 if precision == "mixed" else np.float64
    x = rng_events(desc, n, 2024, dtype)
    x64 = x.astype(np.float64)
    om = oracle.Model(desc)
    sig = sigmas(om, x64, om.theta0)
    pts = random_points(om.theta0, sig, om.free, k, seed=11)
    say(f"case full-{name}-{n}-{precision}: {k} points, oracle on {workers()} processes")
    ref = oracle_points(desc, x64, pts, tmp_path)
    um = uml.Model(desc, precision)
    ud = uml.Data(um, x)
    rel, gerr = [], []
    for th, (nll_o, g_o, bad) in zip(pts, ref):
        assert bad == 0
        nll_g, g_g = uml.uml_eval_nll_grad(um, ud, th)
        rel.append(abs(nll_g - nll_o) / abs(nll_o))
        gerr.append(np.abs(g_g - g_o) * sig)
    rel, gerr = np.array(rel), np.array(gerr)
    say(f"  nll rel err max {rel.max():.2e}  grad err/sigma max {gerr.max():.2e} "
        f"per parameter {np.round(gerr.max(0), 7).tolist()}")
    t = TOL[precision]
    assert rel.max() <= t["nll"]
    assert gerr.max() <= t["grad_sigma"]
