"""Datasets that borrow the caller's device columns (UML_DATA_BORROW): the same
results, bit for bit, as a copied dataset of the same values (NLL, gradient,
Hessian, fit), the device-side domain check, and the argument checks."""
import numpy as np
import pytest
import torch

from paper_2505_12414_amd import datagen as G
from paper_2505_12414_amd import uml
from paper_2505_12414_amd import workloads as W

from gpu_common import say

pytestmark = pytest.mark.gpu


def _pair(desc, precision, x, w=None):
    m = uml.Model(desc, precision)
    t = torch.tensor(x, device="cuda")
    tw = None if w is None else torch.tensor(w, device="cuda")
    copied = uml.Data(m, x, weights=w)
    borrowed = uml.Data(m, t, weights=tw, borrow=True)
    return m, copied, borrowed


@pytest.mark.parametrize("precision,weighted", [("mixed", False), ("mixed", True), ("fp64", False)])
def test_borrowed_equals_copied(precision, weighted):
    desc = W.angmass4d()
    n = 40_000  # a multiple of 4: every row starts on a 16-byte boundary
    dt = np.float32 if precision == "mixed" else np.float64
    x = G.gen_angmass4d(n, 17, dtype=dt)
    w = np.random.default_rng(3).uniform(0.5, 1.5, n).astype(dt) if weighted else None
    say(f"case borrow precision={precision} weighted={weighted}")
    m, a, b = _pair(desc, precision, x, w)
    th = np.asarray(W.angmass4d_truth_vector())
    th[9] *= 1.05
    na, ga = uml.uml_eval_nll_grad(m, a, th)
    nb, gb = uml.uml_eval_nll_grad(m, b, th)
    assert na == nb and np.array_equal(ga, gb)
    ha = uml.uml_eval_hessian(m, a, th)[2]
    hb = uml.uml_eval_hessian(m, b, th)[2]
    assert np.array_equal(ha, hb)
    fa = uml.uml_fit(m, a, th)
    fb = uml.uml_fit(m, b, th)
    assert fa["status_name"] == fb["status_name"] == "converged"
    assert np.array_equal(fa["theta"], fb["theta"]) and np.array_equal(fa["errors"], fb["errors"])
    # the values read back are the caller's
    assert np.array_equal(b.download(), x)


def test_borrowed_domain_and_arguments():
    desc = W.mass1d()
    n = 4096
    x = G.gen_mass1d(n, 5, dtype=np.float32)
    m = uml.Model(desc, "mixed")
    bad = x.copy()
    bad[0, 100] = 7.0  # outside [5.0, 5.6]
    with pytest.raises(uml.UmlError) as e:
        uml.Data(m, torch.tensor(bad, device="cuda"), borrow=True)
    assert e.value.code == uml.UML_E_EVENT_DOMAIN
    nan = x.copy()
    nan[0, 7] = np.nan
    with pytest.raises(uml.UmlError) as e:
        uml.Data(m, torch.tensor(nan, device="cuda"), borrow=True)
    assert e.value.code == uml.UML_E_EVENT_DOMAIN
    # storage type other than the model's
    with pytest.raises(uml.UmlError) as e:
        uml.Data(m, torch.tensor(x.astype(np.float64), device="cuda"), borrow=True)
    assert e.value.code == uml.UML_E_INVALID
    # a row that does not start on a 16-byte boundary (offset by one event)
    big = torch.tensor(np.concatenate([x[:, :1], x], axis=1), device="cuda")
    with pytest.raises(uml.UmlError) as e:
        uml.Data(m, big[:, 1:], borrow=True)
    assert e.value.code == uml.UML_E_INVALID
    # host memory cannot be borrowed
    with pytest.raises(ValueError):
        uml.Data(m, x, borrow=True)
    # a model storing precomputed terms
    mp = uml.Model(W.angmass4d(), "mixed", precompute=True)
    x4 = G.gen_angmass4d(n, 6, dtype=np.float32)
    with pytest.raises(uml.UmlError) as e:
        uml.Data(mp, torch.tensor(x4, device="cuda"), borrow=True)
    assert e.value.code == uml.UML_E_UNSUPPORTED
