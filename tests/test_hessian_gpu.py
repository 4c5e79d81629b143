"""GPU parity of the Hessian pass (H, W2, NLL, gradient) against the oracle,
and the torch.autograd binding against finite differences."""
import numpy as np
import pytest

import oracle
from paper_2505_12414_amd import uml
from paper_2505_12414_amd import workloads as W

from gpu_common import (cheb_desc, exp_desc, gauss_desc, mix_desc, random_points, rng_events, say,
                        sig4d_desc, sigmas)

pytestmark = pytest.mark.gpu

TOL_H = {"fp64": 1e-10, "mixed": 2e-5}

FAMILIES = [
    ("mass1d", W.mass1d, 20011),
    ("angmass4d", W.angmass4d, 20011),
    ("angmass4d_mufree", lambda: W.angmass4d(mu_fixed=False), 20011),
    ("pwave3d", lambda: W.pwave3d((0.6, 0.05, -0.1, 0.1, 0.08, -0.05, 0.03, -0.02)), 20011),
    ("sig4d", sig4d_desc, 20011),
    ("gauss", gauss_desc, 5003),
    ("exp", exp_desc, 5003),
    ("cheb3", lambda: cheb_desc((0.1, -0.2, 0.05)), 5003),
]


def oracle_hessian(om, x, th, w=None):
    _, _, h, _ = om.nll(x, th, w=w, order=2)
    f = om.free
    return h[np.ix_(f, f)]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name,mk,n", FAMILIES, ids=[f[0] for f in FAMILIES])
def test_hessian_matches_oracle(name, mk, n, precision):
    desc = mk()
    dtype = np.float32 if precision == "mixed" else np.float64
    x = rng_events(desc, n, 300 + n, dtype)
    x64 = x.astype(np.float64)
    om = oracle.Model(desc)
    um = uml.Model(desc, precision)
    ud = uml.Data(um, x)
    sig = sigmas(om, x64, om.theta0)
    for k, th in enumerate([om.theta0] + random_points(om.theta0, sig, om.free, 2, seed=3)):
        say(f"case hessian {name}[{k}] precision={precision}")
        nll_g, g_g, h_g = uml.uml_eval_hessian(um, ud, th)
        nll_o, g_o, _, _ = om.nll(x64, th, order=1)
        h_o = oracle_hessian(om, x64, th)
        scale = np.sqrt(np.outer(np.abs(np.diag(h_o)), np.abs(np.diag(h_o))))  # H need not be positive here
        err = np.max(np.abs(h_g - h_o) / scale)
        say(f"  H err {err:.2e}  nll rel {abs(nll_g - nll_o) / abs(nll_o):.2e}")
        assert err <= TOL_H[precision]
        assert abs(nll_g - nll_o) <= (1e-12 if precision == "fp64" else 1e-6) * abs(nll_o)
        assert np.all(np.abs(g_g - g_o[om.free]) * sig <= (1e-8 if precision == "fp64" else 1e-4))
        # the eval kernel and the Hessian pass agree on NLL and gradient
        nll_e, g_e = uml.uml_eval_nll_grad(um, ud, th)
        assert abs(nll_e - nll_g) <= (1e-12 if precision == "fp64" else 2e-6) * abs(nll_o)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("ncomp", [3, 4])
def test_hessian_of_three_and_four_components(ncomp, precision):
    """Mixtures of three and four components (nested sums): five and six
    matrix products per Hessian tile, so two of its waves take a second one.
    H is compared entry by entry on the scale sqrt(|H_aa H_bb|); the NLL and
    gradient of the Hessian pass and of the event kernel against the oracle
    (gradient in units of each parameter's standard deviation)."""
    desc = mix_desc(ncomp)
    dtype = np.float32 if precision == "mixed" else np.float64
    n = 20011
    x = rng_events(desc, n, 300 + n, dtype)
    x64 = x.astype(np.float64)
    om = oracle.Model(desc)
    um = uml.Model(desc, precision)
    ud = uml.Data(um, x)
    sig = sigmas(om, x64, om.theta0)
    gtol = 1e-8 if precision == "fp64" else 1e-4
    for k, th in enumerate([om.theta0] + random_points(om.theta0, sig, om.free, 2, seed=5)):
        say(f"case hessian of {ncomp} components [{k}] precision={precision}")
        nll_g, g_g, h_g = uml.uml_eval_hessian(um, ud, th)
        nll_o, g_o, _, _ = om.nll(x64, th, order=1)
        h_o = oracle_hessian(om, x64, th)
        scale = np.sqrt(np.outer(np.abs(np.diag(h_o)), np.abs(np.diag(h_o))))
        err = np.max(np.abs(h_g - h_o) / scale)
        say(f"  H err {err:.2e}  nll rel {abs(nll_g - nll_o) / abs(nll_o):.2e}")
        assert err <= TOL_H[precision]
        assert abs(nll_g - nll_o) <= (1e-12 if precision == "fp64" else 1e-6) * abs(nll_o)
        assert np.all(np.abs(g_g - g_o[om.free]) * sig <= gtol)
        nll_e, g_e = uml.uml_eval_nll_grad(um, ud, th)
        assert abs(nll_e - nll_o) <= (1e-12 if precision == "fp64" else 1e-6) * abs(nll_o)
        assert np.all(np.abs(g_e - g_o[om.free]) * sig <= gtol)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_weighted_hessian_and_w2(precision):
    desc = W.angmass4d()
    dtype = np.float32 if precision == "mixed" else np.float64
    n = 3001
    x = rng_events(desc, n, 91, dtype)
    w = np.random.default_rng(1).uniform(0.5, 1.5, n).astype(dtype)
    x64, w64 = x.astype(np.float64), w.astype(np.float64)
    om = oracle.Model(desc)
    um = uml.Model(desc, precision)
    ud = uml.Data(um, x, weights=w)
    th = om.theta0.copy()
    th[1] += 0.03
    say(f"case weighted hessian precision={precision}")
    nll_g, g_g, h_g, w2_g = uml.uml_eval_hessian(um, ud, th, want_w2=True)
    h_o = oracle_hessian(om, x64, th, w64)
    scale = np.sqrt(np.outer(np.abs(np.diag(h_o)), np.abs(np.diag(h_o))))  # H need not be positive here
    assert np.max(np.abs(h_g - h_o) / scale) <= TOL_H[precision]
    # W2 = sum w^2 s s^T from the oracle's per-event scores
    f = om.free
    w2_o = np.zeros((f.sum(), f.sum()))
    for i in range(n):
        _, gi, _, _ = om.nll(x64[:, i:i + 1], th, order=1)
        si = -gi[f]
        w2_o += w64[i] ** 2 * np.outer(si, si)
    s2 = np.sqrt(np.outer(np.diag(w2_o), np.diag(w2_o)))
    assert np.max(np.abs(w2_g - w2_o) / s2) <= TOL_H[precision]


def test_hessian_is_deterministic():
    desc = W.angmass4d()
    x = rng_events(desc, 50000, 5, np.float32)
    um = uml.Model(desc, "mixed")
    ud = uml.Data(um, x)
    a = uml.uml_eval_hessian(um, ud, um.theta0)
    b = uml.uml_eval_hessian(um, ud, um.theta0)
    assert a[0] == b[0] and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])


def test_autograd_gradcheck_and_gradgradcheck():
    import torch
    from paper_2505_12414_amd import autograd
    desc = W.angmass4d(mu_fixed=False)
    x = rng_events(desc, 400, 12, np.float64)
    um = uml.Model(desc, "fp64")
    ud = uml.Data(um, x)
    th = torch.tensor(um.theta0, dtype=torch.float64, device="cuda", requires_grad=True)
    say("case autograd gradcheck")
    f = lambda t: autograd.nll(t, um, ud)
    assert torch.autograd.gradcheck(f, (th,), eps=1e-6, atol=1e-5, rtol=1e-4)
    assert torch.autograd.gradgradcheck(f, (th,), eps=1e-6, atol=1e-4, rtol=1e-3)
    # value and gradient equal the C ABI's
    v = f(th)
    (g,) = torch.autograd.grad(v, th)
    nll_c, g_c = uml.uml_eval_nll_grad(um, ud, um.theta0)
    assert v.item() == nll_c and np.array_equal(g.cpu().numpy(), g_c)
