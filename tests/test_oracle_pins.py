"""Pins for the oracle: each test ties it to something other than itself --
library routines (scipy's truncated distributions), closed forms, quadrature,
the paper's printed constants, invariants and finite differences."""
import math
import os

import numpy as np
import pytest
from scipy import optimize, stats

import oracle
from paper_2505_12414_amd import datagen as G
from paper_2505_12414_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))


def gauss_model(lo, hi, mu, sigma):
    return {"dims": [{"name": "m", "lo": lo, "hi": hi}],
            "params": [{"name": "mu", "value": mu}, {"name": "sigma", "value": sigma}],
            "nodes": [{"kind": "gauss", "dims": [0], "params": [0, 1]}], "root": 0}


def exp_model(lo, hi, lam):
    return {"dims": [{"name": "m", "lo": lo, "hi": hi}],
            "params": [{"name": "lambda", "value": lam}],
            "nodes": [{"kind": "exp", "dims": [0], "params": [0]}], "root": 0}


def cheb_model(lo, hi, coeffs):
    return {"dims": [{"name": "x", "lo": lo, "hi": hi}],
            "params": [{"name": f"c{j+1}", "value": c} for j, c in enumerate(coeffs)],
            "nodes": [{"kind": "cheb", "dims": [0], "params": list(range(len(coeffs)))}],
            "root": 0}


def gl_composite(lo, hi, panels, order=20):
    t, w = np.polynomial.legendre.leggauss(order)
    edges = np.linspace(lo, hi, panels + 1)
    a, b = edges[:-1, None], edges[1:, None]
    x = (0.5 * (b - a) * t[None, :] + 0.5 * (a + b)).ravel()
    ww = (0.5 * (b - a) * w[None, :]).ravel()
    return x, ww


def trap_periodic(lo, hi, n):
    x = lo + (hi - lo) * np.arange(n) / n
    return x, np.full(n, (hi - lo) / n)


# --------------------------------------------------------------------------
# single PDFs against library routines, quadrature and closed forms
# --------------------------------------------------------------------------

@pytest.mark.parametrize("lo,hi,mu,sigma", [
    (5.0, 5.6, 5.28, 0.02),     # the mass window of the workloads
    (5.0, 7.0, 5.28, 0.06),     # the paper's mass fit (Table 1)
    (5.0, 5.6, 4.90, 0.05),     # both edges above the mean: erfc branch
    (5.0, 5.6, 5.75, 0.04),     # both edges below the mean: erfc branch
])
def test_gauss_matches_scipy_truncnorm(lo, hi, mu, sigma):
    m = oracle.Model(gauss_model(lo, hi, mu, sigma))
    x = np.linspace(lo, hi, 101)
    ref = stats.truncnorm.pdf(x, (lo - mu) / sigma, (hi - mu) / sigma, loc=mu, scale=sigma)
    got = m.pdf(x)
    assert np.allclose(got, ref, rtol=1e-10, atol=0)


@pytest.mark.parametrize("lam", [-1.5, -1.0, 2.5, -7.0, 1e-7, -3e-9])
def test_exp_matches_scipy_truncexpon(lam):
    lo, hi = 5.0, 5.6
    m = oracle.Model(exp_model(lo, hi, lam))
    x = np.linspace(lo, hi, 77)
    rate = abs(lam)
    if lam < 0:
        ref = stats.truncexpon.pdf(x, b=(hi - lo) * rate, loc=lo, scale=1.0 / rate)
    else:
        ref = stats.truncexpon.pdf(hi - x, b=(hi - lo) * rate, loc=0.0, scale=1.0 / rate)
    assert np.allclose(m.pdf(x), ref, rtol=1e-9, atol=0)


def test_exp_zero_slope_is_uniform_and_continuous():
    lo, hi = 5.0, 7.0
    x = np.array([[5.0, 5.3, 6.1, 6.9, 7.0]])
    p0 = oracle.Model(exp_model(lo, hi, 0.0))
    assert np.allclose(p0.pdf(x), 0.5, rtol=1e-15)
    n0, g0, h0, _ = p0.nll(x, order=2)
    for eps in (1e-12, -1e-12, 1e-9):
        pe = oracle.Model(exp_model(lo, hi, eps))
        ne, ge, he, _ = pe.nll(x, order=2)
        # d NLL / d lambda = -sum (x - E[x]); at lambda = 0, E[x] = (lo+hi)/2
        assert abs(ne - n0) < 1e-8
        assert abs(ge[0] - g0[0]) < 1e-8
        assert abs(he[0, 0] - h0[0, 0]) < 1e-8
    assert g0[0] == pytest.approx(-np.sum(x - 6.0), abs=1e-14)
    assert h0[0, 0] == pytest.approx(5 * 4.0 / 12.0, rel=1e-14)   # N * Var(uniform)


@pytest.mark.parametrize("coeffs", [(0.1, 0.05), (0.3,), (0.1, -0.2, 0.05, 0.1), (0.0, 0.0, 0.3)])
@pytest.mark.parametrize("lo,hi", [(-1.0, 1.0), (-math.pi, math.pi), (5.0, 5.6)])
def test_cheb_normalisation_and_shape(coeffs, lo, hi):
    m = oracle.Model(cheb_model(lo, hi, coeffs))
    x, w = gl_composite(lo, hi, 4)
    assert abs(np.sum(w * m.pdf(x)) - 1.0) < 1e-13
    # shape: T_j(cos t) = cos(j t), so p(x) is proportional to 1 + sum c_j cos(j acos u)
    xs = np.linspace(lo, hi, 33)
    u = np.clip((2 * xs - lo - hi) / (hi - lo), -1, 1)
    shape = 1 + sum(c * np.cos((j + 1) * np.arccos(u)) for j, c in enumerate(coeffs))
    p = m.pdf(xs)
    assert np.allclose(p / p[16], shape / shape[16], rtol=1e-13)


PWAVE_POINTS = [
    (0.6, 0, 0, 0, 0, 0, 0, 0),
    (0.7, 0.0, -0.1, -0.2, 0.1, 0.0, 0.0, 0.0),
    (0.45, 0.12, -0.23, 0.31, -0.17, 0.08, -0.11, 0.05),
]


def pwave_grid(nc=12, nphi=16):
    c, wc = np.polynomial.legendre.leggauss(nc)
    ph, wph = trap_periodic(-math.pi, math.pi, nphi)
    C1, C2, P = np.meshgrid(c, c, ph, indexing="ij")
    Wt = wc[:, None, None] * wc[None, :, None] * wph[None, None, :]
    return np.stack([C1.ravel(), C2.ravel(), P.ravel()]), Wt.ravel()


@pytest.mark.parametrize("ang", PWAVE_POINTS)
def test_pwave_unit_norm_and_moments(ang):
    m = oracle.Model(W.pwave3d(ang))
    x, w = pwave_grid()
    p = m.pdf(x)
    assert abs(np.sum(w * p) - 1.0) < 1e-14
    FL, S3, S4, S5, AFB, S7, S8, S9 = ang
    cl, ck, ph = x
    sl, sk = np.sqrt(1 - cl ** 2), np.sqrt(1 - ck ** 2)

    def E(t):
        return np.sum(w * p * t)
    # Hand-derived moments of the decay rate: each angular observable is
    # picked out by one weight function (integrals of powers of sin/cos).
    assert E(cl) == pytest.approx(2.0 / 3.0 * AFB, abs=1e-14)
    assert E(ck ** 2) == pytest.approx((1 + 2 * FL) / 5.0, abs=1e-14)
    assert E(sk ** 2 * sl ** 2 * np.cos(2 * ph)) == pytest.approx(0.32 * S3, abs=1e-14)
    assert E(sk ** 2 * sl ** 2 * np.sin(2 * ph)) == pytest.approx(0.32 * S9, abs=1e-14)
    assert E(2 * sk * ck * 2 * sl * cl * np.cos(ph)) == pytest.approx(0.32 * S4, abs=1e-14)
    assert E(2 * sk * ck * 2 * sl * cl * np.sin(ph)) == pytest.approx(0.32 * S8, abs=1e-14)
    assert E(2 * sk * ck * sl * np.cos(ph)) == pytest.approx(0.4 * S5, abs=1e-14)
    assert E(2 * sk * ck * sl * np.sin(ph)) == pytest.approx(0.4 * S7, abs=1e-14)


def load_listing4():
    rows = {}
    with open(os.path.join(HERE, "golden", "pwave_listing4.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            name, val, mult = line.split()[:3]
            rows[name] = (float(val), mult)
    return rows


def test_pwave_matches_paper_printed_constants():
    """The density and its parameter derivatives equal the per-event terms with
    the prefactors the paper prints for its precompute kernel."""
    K = load_listing4()
    assert K["t_S9"][0] == pytest.approx(9 / (32 * math.pi), rel=1e-15)
    rng = np.random.default_rng(5)
    x = np.stack([rng.uniform(-1, 1, 50), rng.uniform(-1, 1, 50),
                  rng.uniform(-math.pi, math.pi, 50)])
    cl, ck, ph = x
    sl, sk = np.sqrt(1 - cl ** 2), np.sqrt(1 - ck ** 2)
    fac = {
        "t_S9": np.sin(2 * ph) * (1 - cl ** 2) * (1 - ck ** 2),
        "t_S8": np.sin(ph) * ck * sk * cl * sl,
        "t_S7": np.sin(ph) * sl * ck * sk,
        "t_AFB": cl * (1 - ck ** 2),
        "t_S5": np.cos(ph) * sl * ck * sk,
        "t_S4": np.cos(ph) * ck * sk * cl * sl,
        "t_S3": np.cos(2 * ph) * (1 - cl ** 2) * (1 - ck ** 2),
        "t_mFL": (2 * cl ** 2 - 1) * ck ** 2,
        "t_a": (2 * cl ** 2 - 1) * (1 - ck ** 2),
        "t_b": (1 - ck ** 2),
        "t_FL": ck ** 2,
    }
    m = oracle.Model(W.pwave3d())
    for ang in PWAVE_POINTS:
        FL, S3, S4, S5, AFB, S7, S8, S9 = ang
        mult = {"S9": S9, "S8": S8, "S7": S7, "AFB": AFB, "S5": S5, "S4": S4, "S3": S3,
                "-FL": -FL, "1-FL": 1 - FL, "FL": FL}
        ref = sum(K[k][0] * mult[K[k][1]] * fac[k] for k in fac)
        assert np.allclose(m.pdf(x, np.array(ang, float)), ref, rtol=1e-13, atol=1e-15)
    # derivative with respect to each S_k, per event: -d/dS_k of -ln P = (1/P) dP/dS_k
    th = np.array(PWAVE_POINTS[2], float)
    for i in range(x.shape[1]):
        xi = x[:, i:i + 1]
        _, g, _, _ = m.nll(xi, th, order=1)
        P = m.pdf(xi, th)[0]
        dP = -g * P
        name = ["S3", "S4", "S5", "AFB", "S7", "S8", "S9"]
        for k, nm in enumerate(name):
            assert dP[k + 1] == pytest.approx(K["t_" + nm][0] * fac["t_" + nm][i], abs=1e-14)
        dFL = -K["t_mFL"][0] * fac["t_mFL"][i] - K["t_a"][0] * fac["t_a"][i] \
            - K["t_b"][0] * fac["t_b"][i] + K["t_FL"][0] * fac["t_FL"][i]
        assert dP[0] == pytest.approx(dFL, abs=1e-14)


# --------------------------------------------------------------------------
# composite models
# --------------------------------------------------------------------------

def test_mass_model_nll_matches_scipy():
    desc = W.mass1d()
    m = oracle.Model(desc)
    x = G.gen_mass1d(2000, 11)
    for th in ([5.28, 0.02, -1.5, 0.3], [5.29, 0.025, -0.7, 0.45], [5.1, 0.05, 1.2, 0.1]):
        mu, sg, lam, f = th
        g = stats.truncnorm.pdf(x[0], (5.0 - mu) / sg, (5.6 - mu) / sg, loc=mu, scale=sg)
        if lam < 0:
            e = stats.truncexpon.pdf(x[0], b=0.6 * -lam, loc=5.0, scale=-1 / lam)
        else:
            e = stats.truncexpon.pdf(5.6 - x[0], b=0.6 * lam, loc=0.0, scale=1 / lam)
        ref = -math.fsum(np.log(f * g + (1 - f) * e))
        got, _, _, bad = m.nll(x, np.array(th))
        assert bad == 0
        assert got == pytest.approx(ref, rel=1e-12)


def angmass_grid():
    xm, wm = gl_composite(5.0, 5.6, 60)
    c, wc = np.polynomial.legendre.leggauss(6)
    # phi carries both trigonometric (signal) and polynomial (background) terms
    ph, wph = gl_composite(-math.pi, math.pi, 2, 14)
    M, C1, C2, P = np.meshgrid(xm, c, c, ph, indexing="ij")
    Wt = (wm[:, None, None, None] * wc[None, :, None, None] * wc[None, None, :, None]
          * wph[None, None, None, :])
    return np.stack([M.ravel(), C1.ravel(), C2.ravel(), P.ravel()]), Wt.ravel()


@pytest.mark.parametrize("seed", [0, 1])
def test_angmass4d_normalisation(seed):
    m = oracle.Model(W.angmass4d())
    x, w = angmass_grid()
    th = np.array(W.angmass4d_truth_vector())
    if seed:
        rng = np.random.default_rng(seed)
        th[:8] += rng.uniform(-0.05, 0.05, 8)
        th[8] += 0.01
        th[9] *= 1.3
        th[10] = 0.8
        th[11:17] += rng.uniform(-0.05, 0.05, 6)
        th[17] = 0.55
    assert abs(np.sum(w * m.pdf(x, th)) - 1.0) < 1e-12


def test_sum_and_prod_compose_factors():
    """Sum and product nodes combine independently evaluated factors."""
    d4 = W.angmass4d()
    m4 = oracle.Model(d4)
    th = np.array(W.angmass4d_truth_vector())
    th[17] = 0.37
    rng = np.random.default_rng(3)
    x = np.stack([rng.uniform(5.0, 5.6, 40), rng.uniform(-1, 1, 40), rng.uniform(-1, 1, 40),
                  rng.uniform(-math.pi, math.pi, 40)])
    pw = oracle.Model(W.pwave3d(th[:8])).pdf(x[1:])
    g = stats.truncnorm.pdf(x[0], (5.0 - th[8]) / th[9], (5.6 - th[8]) / th[9], loc=th[8],
                            scale=th[9])
    e = stats.truncexpon.pdf(x[0], b=0.6 * -th[10], loc=5.0, scale=-1 / th[10])
    cb = [oracle.Model(cheb_model(lo, hi, th[11 + 2 * d:13 + 2 * d])).pdf(x[1 + d])
          for d, (lo, hi) in enumerate([(-1, 1), (-1, 1), (-math.pi, math.pi)])]
    ref = 0.37 * pw * g + 0.63 * cb[0] * cb[1] * cb[2] * e
    assert np.allclose(m4.pdf(x, th), ref, rtol=1e-12)


# --------------------------------------------------------------------------
# closed-form maximum-likelihood estimates
# --------------------------------------------------------------------------

def test_gaussian_closed_form_mle_gradient_and_hessian():
    """Gauss far inside [5.0, 5.6] (edges 14 and 16 sigma away): the MLE is the
    sample mean and the biased sample standard deviation, the gradient vanishes
    there and the Hessian is diag(N/s^2, 2N/s^2)."""
    rng = np.random.default_rng(21)
    x = rng.normal(5.28, 0.02, 5000).reshape(1, -1)
    n = x.shape[1]
    mean, sd = x.mean(), x.std()
    m = oracle.Model(gauss_model(5.0, 5.6, 5.28, 0.02))
    _, g, h, _ = m.nll(x, np.array([mean, sd]), order=2)
    assert abs(g[0]) * sd / math.sqrt(n) < 1e-9
    assert abs(g[1]) * sd / math.sqrt(n) < 1e-9
    assert h[0, 0] == pytest.approx(n / sd ** 2, rel=1e-9)
    assert h[1, 1] == pytest.approx(2 * n / sd ** 2, rel=1e-9)
    assert abs(h[0, 1]) < 1e-6 * h[0, 0]
    r = m.fit(x, start=[5.29, 0.023], edm_tol=1e-14, polish=1)
    assert r["status"] == 0
    assert r["theta"][0] == pytest.approx(mean, abs=1e-9 * sd)
    assert r["theta"][1] == pytest.approx(sd, abs=1e-9 * sd)
    assert r["errors"][0] == pytest.approx(sd / math.sqrt(n), rel=1e-8)


def trunc_exp_moment(lam, lo, hi, k):
    """E[x^k] for a density proportional to exp(lam x) on [lo, hi], by
    Gauss-Legendre quadrature (exact to rounding for this smooth integrand)."""
    t, w = gl_composite(lo, hi, 4)
    e = w * np.exp(lam * (t - lo))
    return math.fsum(e * t ** k) / math.fsum(e)


def trunc_exp_mean(lam, lo, hi):
    return trunc_exp_moment(lam, lo, hi, 1)


def test_exponential_mle_is_moment_root():
    lo, hi = 5.0, 5.6
    x = G.gen_mass1d(4000, 5, fsig=0.0)
    mbar = x.mean()
    lam_hat = optimize.brentq(lambda l: trunc_exp_mean(l, lo, hi) - mbar, -20, 20, xtol=1e-15)
    m = oracle.Model(exp_model(lo, hi, -1.0))
    r = m.fit(x, start=[-1.0], edm_tol=1e-16, polish=2)
    assert r["theta"][0] == pytest.approx(lam_hat, abs=1e-8)
    # H = N Var_lambda(x), by quadrature
    ex = trunc_exp_mean(lam_hat, lo, hi)
    ex2 = trunc_exp_moment(lam_hat, lo, hi, 2)
    _, _, h, _ = m.nll(x, np.array([lam_hat]), order=2)
    assert h[0, 0] == pytest.approx(x.shape[1] * (ex2 - ex * ex), rel=1e-9)


def test_fraction_mle_and_sum_rule():
    """With the shapes fixed the NLL is convex in f; the root of
    sum (g - e)/P = 0 (scipy densities, brentq) is the MLE, and at it the
    responsibilities sum to N: sum_i g_i / P_i = N."""
    x = G.gen_mass1d(3000, 9)
    mu, sg, lam = 5.28, 0.02, -1.5
    g = stats.truncnorm.pdf(x[0], (5.0 - mu) / sg, (5.6 - mu) / sg, loc=mu, scale=sg)
    e = stats.truncexpon.pdf(x[0], b=0.6 * -lam, loc=5.0, scale=-1 / lam)
    f_hat = optimize.brentq(lambda f: np.sum((g - e) / (f * g + (1 - f) * e)), 1e-6, 1 - 1e-6,
                            xtol=1e-15)
    assert np.sum(g / (f_hat * g + (1 - f_hat) * e)) == pytest.approx(x.shape[1], rel=1e-12)
    desc = W.mass1d()
    for k in range(3):
        desc["params"][k]["fixed"] = True
    m = oracle.Model(desc)
    r = m.fit(x, start=[mu, sg, lam, 0.4], edm_tol=1e-16, polish=2)
    assert r["theta"][3] == pytest.approx(f_hat, abs=1e-10)


# --------------------------------------------------------------------------
# derivatives against finite differences
# --------------------------------------------------------------------------

def richardson_grad(fun, th, steps):
    g = np.zeros(th.size)
    for k in range(th.size):
        def d(h):
            tp, tm = th.copy(), th.copy()
            tp[k] += h
            tm[k] -= h
            return (fun(tp) - fun(tm)) / (2 * h)
        h = steps[k]
        g[k] = (4 * d(h / 2) - d(h)) / 3
    return g


FD_CASES = [
    ("mass1d", lambda: W.mass1d(), lambda: G.gen_mass1d(48, 3),
     [5.283, 0.021, -1.3, 0.31], [2e-5, 2e-6, 1e-4, 1e-5]),
    ("angmass4d", lambda: W.angmass4d(mu_fixed=False),
     lambda: G.gen_angmass4d(48, 4, dtype=np.float64),
     W.angmass4d_truth_vector(), [1e-5] * 8 + [2e-5, 2e-6, 1e-4] + [1e-5] * 6 + [1e-5]),
    ("pwave3d", lambda: W.pwave3d(PWAVE_POINTS[2]), lambda: G.gen_pwave3d(48, 5, PWAVE_POINTS[2]),
     list(PWAVE_POINTS[2]), [1e-5] * 8),
    ("cheb4", lambda: cheb_model(-1.0, 2.0, (0.1, -0.2, 0.05, 0.1)),
     lambda: np.linspace(-1.0, 2.0, 31).reshape(1, -1), [0.1, -0.2, 0.05, 0.1], [1e-5] * 4),
]


@pytest.mark.parametrize("name,mk,gen,th,steps", FD_CASES, ids=[c[0] for c in FD_CASES])
def test_gradient_and_hessian_match_finite_differences(name, mk, gen, th, steps):
    m = oracle.Model(mk())
    x = gen()
    th = np.array(th, dtype=np.float64)
    steps = np.array(steps)
    nll, g, h, bad = m.nll(x, th, order=2)
    assert bad == 0
    gfd = richardson_grad(lambda t: m.nll(x, t)[0], th, steps)
    scale = np.abs(g) + np.sqrt(np.abs(np.diag(h)))   # gradient scale per parameter
    assert np.all(np.abs(g - gfd) <= 1e-7 * scale), (g, gfd)
    hfd = np.stack([richardson_grad(lambda t: m.nll(x, t, order=1)[1][k], th, steps)
                    for k in range(th.size)])
    hs = np.sqrt(np.outer(np.abs(np.diag(h)), np.abs(np.diag(h)))) + np.abs(h)
    assert np.all(np.abs(h - hfd) <= 1e-6 * hs)
    assert np.allclose(h, h.T, rtol=1e-12, atol=1e-12 * np.max(np.abs(h)))


@pytest.mark.parametrize("name,mk,gen,th,steps", FD_CASES[:2], ids=[c[0] for c in FD_CASES[:2]])
def test_w2_matches_finite_difference_scores(name, mk, gen, th, steps):
    """W2 = sum w^2 s s^T, with each event's score s = d ln P / d theta taken
    by Richardson central differences of its log-density alone."""
    m = oracle.Model(mk())
    x = gen()
    th = np.array(th, dtype=np.float64)
    n = x.shape[1]
    w = np.random.default_rng(3).uniform(0.5, 1.5, n)
    w2, bad = m.w2(x, th, w)
    assert bad == 0
    S = np.stack([richardson_grad(lambda t: math.log(m.pdf(x[:, i:i + 1], t)[0]), th, np.array(steps))
                  for i in range(n)])
    w2_fd = (S.T * w ** 2) @ S
    scale = np.sqrt(np.outer(np.diag(w2_fd), np.diag(w2_fd))) + 1e-300
    assert np.max(np.abs(w2 - w2_fd) / scale) < 1e-6


def test_sandwich_variance_of_weighted_gaussian_mean():
    """Gauss with sigma fixed, far inside [5.0, 5.6]: the weighted MLE of mu is
    the weighted mean, and H^-1 W2 H^-1 is sum w^2 (x - mu)^2 / (sum w)^2, the
    usual variance estimate of a weighted mean."""
    rng = np.random.default_rng(8)
    n = 4000
    x = rng.normal(5.28, 0.02, n).reshape(1, -1)
    w = rng.uniform(0.5, 1.5, n)
    desc = gauss_model(5.0, 5.6, 5.28, 0.02)
    desc["params"][1]["fixed"] = True
    m = oracle.Model(desc)
    mu = math.fsum(w * x[0]) / math.fsum(w)
    th = np.array([mu, 0.02])
    _, g, h, _ = m.nll(x, th, w=w, order=2)
    assert abs(g[0]) * 0.02 / math.sqrt(n) < 1e-9
    w2, _ = m.w2(x, th, w)
    var = w2[0, 0] / h[0, 0] ** 2
    assert var == pytest.approx(math.fsum(w ** 2 * (x[0] - mu) ** 2) / math.fsum(w) ** 2, rel=1e-10)


# --------------------------------------------------------------------------
# weights, invalid points
# --------------------------------------------------------------------------

def test_unit_weights_bitwise_and_constant_weights_scale():
    m = oracle.Model(W.angmass4d())
    x = G.gen_angmass4d(500, 8, dtype=np.float64)
    n0, g0, h0, _ = m.nll(x, order=2)
    n1, g1, h1, _ = m.nll(x, w=np.ones(500), order=2)
    assert n0 == n1 and np.array_equal(g0, g1) and np.array_equal(h0, h1)
    n2, g2, h2, _ = m.nll(x, w=np.full(500, 2.5), order=2)
    assert n2 == pytest.approx(2.5 * n0, rel=1e-13)
    assert np.allclose(g2, 2.5 * g0, rtol=1e-12, atol=1e-9)
    assert np.allclose(h2, 2.5 * h0, rtol=1e-12, atol=1e-6)


def test_nonpositive_density_gives_infinite_nll_and_count():
    m = oracle.Model(W.pwave3d())
    x = G.gen_pwave3d(400, 2)
    th = np.array([2.5, 0, 0, 0, 0, 0, 0, 0])   # F_L > 1 makes the rate negative somewhere
    nll, g, _, bad = m.nll(x, th, order=1)
    assert bad > 0 and nll == math.inf and np.all(g == 0)
    p = m.pdf(x, th)
    assert bad == int(np.sum(~(p > 0)))


def test_fraction_outside_unit_interval_is_outside_the_domain():
    m = oracle.Model(W.mass1d())
    x = G.gen_mass1d(100, 4)
    for f in (-0.01, 1.2):
        nll, _, _, bad = m.nll(x, np.array([5.28, 0.02, -1.5, f]), order=1)
        assert nll == math.inf and bad == 100
    for f in (0.0, 1.0):   # the closed ends are valid mixtures
        nll, _, _, bad = m.nll(x, np.array([5.28, 0.02, -1.5, f]))
        assert bad == 0 and math.isfinite(nll)


# --------------------------------------------------------------------------
# pseudo-experiment generation: the counter-based generator against NumPy's
# Philox bit generator, samples against library distribution functions and
# closed-form moments, fits to generated toys against their generating values
# --------------------------------------------------------------------------

@pytest.mark.parametrize("ctr,key", [
    ([0, 0, 0, 0], [0, 0]),
    ([5, 0, 0, 0], [7, 9]),
    ([2 ** 64 - 1, 3, 0, 0], [12345, 2 ** 63 + 11]),   # carry into the second word
    ([17, 2 ** 40, 5, 1], [2 ** 64 - 1, 2 ** 64 - 1]),
])
def test_philox_matches_numpy_bit_generator(ctr, key):
    """NumPy's Philox (4 x 64 bits, 10 rounds) advances its 256-bit counter
    before each block: its first four words are the block of counter + 1."""
    bg = np.random.Philox(counter=np.array(ctr, dtype=np.uint64), key=np.array(key, dtype=np.uint64))
    ref = [int(v) for v in bg.random_raw(8)]
    c = list(ctr)
    for blk in range(2):
        k = 0
        while True:   # counter + 1 with carry
            c[k] = (c[k] + 1) % 2 ** 64
            if c[k] != 0:
                break
            k += 1
        assert oracle.philox4x64(c, key) == ref[4 * blk:4 * blk + 4]


def ks_pvalue(x, cdf):
    return stats.kstest(x, cdf).pvalue


def test_generated_gaussian_and_exponential_follow_their_distributions():
    lo, hi = 5.0, 5.6
    g = oracle.Model(gauss_model(lo, hi, 5.3, 0.1))       # both edges inside 3 sigma
    x, bad = g.generate(100000, 11)
    assert bad == 0 and x.min() >= lo and x.max() <= hi
    tn = stats.truncnorm((lo - 5.3) / 0.1, (hi - 5.3) / 0.1, loc=5.3, scale=0.1)
    assert ks_pvalue(x[0], tn.cdf) > 1e-3
    e = oracle.Model(exp_model(lo, hi, -3.0))
    x, bad = e.generate(100000, 12)
    te = stats.truncexpon((hi - lo) * 3.0, loc=lo, scale=1 / 3.0)
    assert bad == 0 and ks_pvalue(x[0], te.cdf) > 1e-3
    e0 = oracle.Model(exp_model(lo, hi, 0.0))           # lambda = 0: uniform
    x, _ = e0.generate(100000, 13)
    assert ks_pvalue(x[0], stats.uniform(lo, hi - lo).cdf) > 1e-3


@pytest.mark.parametrize("coeffs", [(0.3,), (0.1, 0.05), (0.1, -0.2, 0.05, 0.1)])
def test_generated_chebyshev_follows_its_distribution(coeffs):
    lo, hi = -1.0, 2.0
    m = oracle.Model(cheb_model(lo, hi, coeffs))
    x, bad = m.generate(100000, 21)
    assert bad == 0
    series = np.polynomial.chebyshev.Chebyshev([1.0, *coeffs], domain=[lo, hi])
    prim = series.integ(lbnd=lo)
    norm = prim(hi)
    assert ks_pvalue(x[0], lambda v: prim(v) / norm) > 1e-3


def test_generated_mass_mixture_follows_its_distribution():
    lo, hi, mu, sg, lam, f = 5.0, 5.6, 5.28, 0.02, -1.5, 0.3
    m = oracle.Model(W.mass1d())
    x, bad = m.generate(200000, 31)
    tn = stats.truncnorm((lo - mu) / sg, (hi - mu) / sg, loc=mu, scale=sg)
    te = stats.truncexpon((hi - lo) * -lam, loc=lo, scale=1 / -lam)
    # the exponential of the model rises or falls with lambda: e^{lam x} with
    # lam < 0 falls, which is the truncated exponential of rate -lam
    assert bad == 0 and ks_pvalue(x[0], lambda v: f * tn.cdf(v) + (1 - f) * te.cdf(v)) > 1e-3


@pytest.mark.parametrize("ang", PWAVE_POINTS, ids=["fl-only", "workload", "all"])
def test_generated_pwave_moments(ang):
    """Sample moments of generated angles against the closed forms (within
    five standard errors of the sample)."""
    m = oracle.Model(W.pwave3d(ang))
    x, bad = m.generate(400000, 41)
    assert bad == 0
    FL, S3, S4, S5, AFB, S7, S8, S9 = ang
    cl, ck, ph = x
    sl, sk = np.sqrt(1 - cl ** 2), np.sqrt(1 - ck ** 2)
    for t, want in [(cl, 2.0 / 3.0 * AFB), (ck ** 2, (1 + 2 * FL) / 5.0),
                    (sk ** 2 * sl ** 2 * np.cos(2 * ph), 0.32 * S3),
                    (sk ** 2 * sl ** 2 * np.sin(2 * ph), 0.32 * S9),
                    (4 * sk * ck * sl * cl * np.cos(ph), 0.32 * S4),
                    (4 * sk * ck * sl * cl * np.sin(ph), 0.32 * S8),
                    (2 * sk * ck * sl * np.cos(ph), 0.4 * S5),
                    (2 * sk * ck * sl * np.sin(ph), 0.4 * S7)]:
        se = t.std() / math.sqrt(t.size)
        assert abs(t.mean() - want) < 5 * se, (t.mean(), want, se)


def test_fits_to_generated_toys_are_unbiased():
    """Oracle fits of 200 generated mass-model toys: pulls of mean ~0 and
    width ~1 for every parameter."""
    m = oracle.Model(W.mass1d())
    truth = m.theta0.copy()
    pulls = []
    for k in range(200):
        x, bad = m.generate(2000, 1000 + k)
        assert bad == 0
        r = m.fit(x, start=truth)
        assert r["status"] == 0
        pulls.append((r["theta"] - truth) / r["errors"])
    p = np.array(pulls)
    assert np.all(np.abs(p.mean(0)) < 0.3), p.mean(0)
    assert np.all(np.abs(p.std(0) - 1.0) < 0.2), p.std(0)
