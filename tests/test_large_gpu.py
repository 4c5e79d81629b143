"""The largest inputs: datasets whose columns pass 2^31 bytes, tens of
thousands of tiles, checked through properties that hold at any size (the
oracle cannot evaluate them in seconds):
  * additivity: the NLL and gradient of a dataset equal the sums over its two
    parts, split at a tile boundary (both parts tile their events as the whole
    does, so every tile's partial sums are the same numbers and only the FP64
    order in which the tiles are added differs);
  * the allocation-free entry point gives the same bits as the dataset path;
  * evaluations repeat bit for bit.
Events are drawn on the device (uniform inside each dimension's range); at
these sizes the event values do not matter to the properties."""
import numpy as np
import pytest
import torch

from paper_2505_12414_amd import uml
from paper_2505_12414_amd import workloads as W

from gpu_common import say

pytestmark = pytest.mark.gpu


def _uniform_events(desc, n, dtype, seed):
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    rows = []
    for d in desc["dims"]:
        lo, hi = d["lo"], d["hi"]
        if dtype == torch.float32:  # the range's ends as storable values inside [lo, hi]
            lo32, hi32 = np.float32(lo), np.float32(hi)
            if float(lo32) < lo:
                lo32 = np.nextafter(lo32, np.float32(np.inf))
            if float(hi32) > hi:
                hi32 = np.nextafter(hi32, np.float32(-np.inf))
            lo_s, hi_s = float(lo32), float(hi32)
        else:
            lo_s, hi_s = lo, hi
        u = torch.rand(n, generator=g, device="cuda", dtype=dtype)
        rows.append(torch.clamp(lo_s + (hi_s - lo_s) * u, min=lo_s, max=hi_s))
    return torch.stack(rows)


CASES = [("mass1d", W.mass1d, 600_000_017, "mixed"),     # 2.4 GB of events, 36622 tiles
         ("mass1d", W.mass1d, 300_000_001, "fp64"),      # 2.4 GB
         ("angmass4d", W.angmass4d, 100_000_004, "mixed")]  # 1.6 GB (rows 16-byte aligned)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("name,mk,n,precision", CASES, ids=[f"{c[0]}-{c[2]}-{c[3]}" for c in CASES])
def test_large_additivity_and_noalloc(name, mk, n, precision):
    desc = mk()
    dt = torch.float32 if precision == "mixed" else torch.float64
    say(f"case large {name} n={n} precision={precision}")
    x = _uniform_events(desc, n, dt, 7)
    m = uml.Model(desc, precision)
    th = m.theta0.copy()
    free = [i for i, p in enumerate(desc["params"]) if not p.get("fixed", False)]
    th[free[0]] += 1e-3 * (abs(th[free[0]]) + 1.0)
    full = uml.Data(m, x, borrow=True)
    nll, g = uml.uml_eval_nll_grad(m, full, th)
    assert np.isfinite(nll) and np.all(np.isfinite(g))
    again = uml.uml_eval_nll_grad(m, full, th)
    assert again[0] == nll and np.array_equal(again[1], g)
    tile = 64 * 256  # events per tile at these sizes (64 per thread), the same for the parts
    h = (n // 2) // tile * tile
    a = uml.Data(m, x[:, :h])
    na, ga = uml.uml_eval_nll_grad(m, a, th)
    del a
    b = uml.Data(m, x[:, h:])
    nb, gb = uml.uml_eval_nll_grad(m, b, th)
    del b
    gd = np.abs(g - (ga + gb)) / (np.abs(ga) + np.abs(gb))
    say(f"  nll {nll:.15e} parts {na + nb:.15e} rel {abs(nll - (na + nb)) / abs(nll):.2e}; "
        f"gradient rel max {gd.max():.2e}")
    assert abs(nll - (na + nb)) <= 1e-12 * abs(nll)
    assert np.all(gd <= 1e-12)
    # the allocation-free entry point on the same columns
    d_theta = torch.tensor(th, dtype=torch.float64, device="cuda")
    d_out = torch.empty(1 + m.n_free, dtype=torch.float64, device="cuda")
    cols = [x[k].data_ptr() for k in range(x.shape[0])]
    uml.uml_eval_nll_grad_noalloc(m, n, cols, None, d_theta, d_out)
    torch.cuda.synchronize()
    out = d_out.cpu().numpy()
    assert out[0] == nll and np.array_equal(out[1:], g)
