"""Device-resident BFGS fits: fitted values and uncertainties against the
oracle's fit, closed-form MLEs, batch-vs-alone identity, failure statuses."""
import math

import numpy as np
import pytest

import oracle
from paper_2505_12414_amd import uml
from paper_2505_12414_amd import workloads as W

from gpu_common import gauss_desc, rng_events, say

pytestmark = pytest.mark.gpu


def compare_fits(r, ro, free, tol_sigma, tol_err, tag):
    sig = ro["errors"]  # oracle errors, free order
    th_g = r["theta"][free]
    th_o = ro["theta"][free]
    pulls = np.abs(th_g - th_o) / sig
    err_rel = np.abs(r["errors"][free] - sig) / sig
    say(f"  {tag}: max |dtheta|/sigma {pulls.max():.2e}, max |dsigma|/sigma {err_rel.max():.2e}, "
        f"iter {r['n_iter']} eval {r['n_eval']} status {r['status_name']}")
    assert r["status"] == 0, r["status_name"]
    assert pulls.max() <= tol_sigma, (tag, pulls)
    assert err_rel.max() <= tol_err, (tag, err_rel)


def test_c1_mass_fit_fp64_converges_and_matches_oracle():
    """1-D mass fit, 1e4 events, FP64, 4 free parameters started 5% off."""
    desc = W.mass1d()
    x = rng_events(desc, 10_000, 2025, np.float64)
    start = np.array(W.mass1d_start())
    um = uml.Model(desc, "fp64")
    ud = uml.Data(um, x)
    say("case c1 default options")
    r = uml.uml_fit(um, ud, start)                      # EDM < 1e-6, the config's rule
    assert r["status"] == 0 and r["edm"] < 1e-6
    om = oracle.Model(desc)
    ro = om.fit(x, start=start, edm_tol=1e-12, polish=1)
    assert ro["status"] == 0
    free = om.free
    # at EDM < 1e-6 the fitted values sit within ~sqrt(2 EDM) ~ 1.4e-3 sigma
    pulls = np.abs(r["theta"][free] - ro["theta"][free]) / ro["errors"]
    assert pulls.max() < 2e-3
    # converged tightly (plus one Newton step) both agree to 1e-6 sigma
    say("case c1 tight")
    r2 = uml.uml_fit(um, ud, start, edm_tol=1e-12, polish=1)
    compare_fits(r2, ro, free, 1e-6, 1e-9, "c1-fp64")
    assert abs(r2["nll"] - ro["nll"]) <= 1e-12 * abs(ro["nll"])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_4d_fit_matches_oracle(precision):
    desc = W.angmass4d()
    dtype = np.float32 if precision == "mixed" else np.float64
    x = rng_events(desc, 60_000, 77, dtype)
    um = uml.Model(desc, precision)
    ud = uml.Data(um, x)
    start = um.theta0.copy()
    start[0] += 0.02
    start[17] -= 0.02
    say(f"case 4d fit precision={precision}")
    # mixed mode: the per-point FP32 rounding of the constants puts a floor
    # of ~(2^-24 sqrt(N))^2 under the EDM, so converge to 1e-8 there
    r = uml.uml_fit(um, ud, start, edm_tol=1e-10 if precision == "fp64" else 1e-8, polish=1)
    om = oracle.Model(desc)
    ro = om.fit(x.astype(np.float64), start=start, edm_tol=1e-12, polish=1)
    assert ro["status"] == 0
    compare_fits(r, ro, om.free, 1e-5 if precision == "fp64" else 1e-3,
                 1e-8 if precision == "fp64" else 1e-4, f"4d-{precision}")


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_weighted_fit_sandwich_covariance(precision):
    """Weighted 4-D fit with the sandwich covariance H^-1 W2 H^-1: errors and
    matrix against the oracle's H and W2 at the fitted point."""
    desc = W.angmass4d()
    dtype = np.float32 if precision == "mixed" else np.float64
    n = 40_000
    x = rng_events(desc, n, 313, dtype)
    w = np.random.default_rng(314).uniform(0.5, 1.5, n).astype(dtype)
    um = uml.Model(desc, precision)
    ud = uml.Data(um, x, weights=w)
    say(f"case weighted sandwich fit precision={precision}")
    r = uml.uml_fit(um, ud, um.theta0, edm_tol=1e-10 if precision == "fp64" else 1e-8,
                    cov_kind=uml.UML_COV_SANDWICH)
    assert r["status"] == 0, r["status_name"]
    rh = uml.uml_fit(um, ud, um.theta0, edm_tol=1e-10 if precision == "fp64" else 1e-8)
    assert np.array_equal(r["theta"], rh["theta"])   # the covariance choice does not move the fit
    om = oracle.Model(desc)
    f = om.free
    x64, w64 = x.astype(np.float64), w.astype(np.float64)
    _, _, h, _ = om.nll(x64, r["theta"], w=w64, order=2)
    w2, bad = om.w2(x64, r["theta"], w64)
    assert bad == 0
    C = np.linalg.inv(h[np.ix_(f, f)])
    V = C @ w2[np.ix_(f, f)] @ C
    s_or = np.sqrt(np.diag(V))
    rel = np.abs(r["errors"][f] - s_or) / s_or
    tol = 1e-8 if precision == "fp64" else 1e-3
    say(f"  max |dsigma|/sigma {rel.max():.2e}; sandwich/HESSE error ratios "
        f"{np.round(r['errors'][f] / rh['errors'][f], 3).tolist()}")
    assert rel.max() <= tol
    assert np.max(np.abs(r["cov"] - V) / np.outer(s_or, s_or)) <= tol
    # w ~ U(0.5, 1.5): E[w] = 1, E[w^2] = 13/12, so the sandwich errors exceed
    # the inverse-Hessian ones by about sqrt(13/12) = 1.04
    ratio = r["errors"][f] / rh["errors"][f]
    assert np.all((ratio > 1.0) & (ratio < 1.1)), ratio


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_newton_fit_matches_oracle(precision):
    """Newton iterations with the analytic Hessian: the same minimum as the
    oracle's fit, reached in a few iterations."""
    desc = W.angmass4d()
    dtype = np.float32 if precision == "mixed" else np.float64
    x = rng_events(desc, 60_000, 77, dtype)
    um = uml.Model(desc, precision)
    ud = uml.Data(um, x)
    start = um.theta0.copy()
    start[0] += 0.02
    start[17] -= 0.02
    say(f"case 4d newton fit precision={precision}")
    r = uml.uml_fit(um, ud, start, edm_tol=1e-10 if precision == "fp64" else 1e-8,
                    method=uml.UML_METHOD_NEWTON)
    om = oracle.Model(desc)
    ro = om.fit(x.astype(np.float64), start=start, edm_tol=1e-12, polish=1)
    assert ro["status"] == 0
    compare_fits(r, ro, om.free, 1e-5 if precision == "fp64" else 1e-3,
                 1e-8 if precision == "fp64" else 1e-4, f"4d-newton-{precision}")
    assert r["n_iter"] <= 6


def test_newton_c1_mass_fit():
    desc = W.mass1d()
    x = rng_events(desc, 10_000, 2025, np.float64)
    start = np.array(W.mass1d_start())
    um = uml.Model(desc, "fp64")
    ud = uml.Data(um, x)
    say("case c1 newton")
    r = uml.uml_fit(um, ud, start, edm_tol=1e-12, method=uml.UML_METHOD_NEWTON)
    om = oracle.Model(desc)
    ro = om.fit(x, start=start, edm_tol=1e-12, polish=1)
    compare_fits(r, ro, om.free, 1e-6, 1e-8, "c1-newton")


def test_gaussian_fit_reaches_closed_form_mle():
    rng = np.random.default_rng(4)
    x = rng.normal(5.28, 0.02, 20_000).reshape(1, -1)
    um = uml.Model(gauss_desc(), "fp64")
    ud = uml.Data(um, x)
    r = uml.uml_fit(um, ud, np.array([5.29, 0.024]), edm_tol=1e-14, polish=1)
    assert r["status"] == 0
    sd = x.std()
    assert abs(r["theta"][0] - x.mean()) <= 1e-8 * sd
    assert abs(r["theta"][1] - sd) <= 1e-8 * sd
    assert r["errors"][0] == pytest.approx(sd / math.sqrt(x.shape[1]), rel=1e-6)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_equals_alone_bitwise(precision):
    desc = W.angmass4d()
    dtype = np.float32 if precision == "mixed" else np.float64
    um = uml.Model(desc, precision)
    sizes = [500, 3_000, 17_000, 70_000]
    datas = [uml.Data(um, rng_events(desc, n, 900 + n, dtype)) for n in sizes]
    starts = np.tile(um.theta0, (len(sizes), 1))
    starts[:, 0] += 0.01
    say(f"case batch precision={precision}")
    batch = uml.uml_fit_batch(um, datas, starts)
    for d, st, rb in zip(datas, starts, batch):
        ra = uml.uml_fit(um, d, st)
        assert ra["status"] == rb["status"] == 0
        assert np.array_equal(ra["theta"], rb["theta"]) and np.array_equal(ra["errors"], rb["errors"])
        assert ra["nll"] == rb["nll"] and ra["n_iter"] == rb["n_iter"]


def test_failure_statuses():
    desc = W.pwave3d()
    um = uml.Model(desc, "fp64")
    ud = uml.Data(um, rng_events(desc, 2000, 3, np.float64))
    # a start point with P <= 0 somewhere
    r = uml.uml_fit(um, ud, np.array([2.5, 0, 0, 0, 0, 0, 0, 0.0]))
    assert r["status_name"] == "pdf_nonpositive"
    # an iteration cap
    desc1 = W.mass1d()
    um1 = uml.Model(desc1, "fp64")
    ud1 = uml.Data(um1, rng_events(desc1, 5000, 8, np.float64))
    r = uml.uml_fit(um1, ud1, np.array(W.mass1d_start()), max_iter=1, edm_tol=1e-14)
    assert r["status_name"] == "max_iter" and r["n_iter"] == 1
