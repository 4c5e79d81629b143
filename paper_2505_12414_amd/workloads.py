"""Model descriptions and truth values of the benchmark workloads.

Plain data only.  A model description is a dict of dimensions, parameters
and a node tree over the PDF catalogue (Gaussian, exponential, Chebyshev
series, P-wave angular density, products, sums with a fraction), the same
structure the paper's control file builds with its dimension, parameter and
PDF objects (Listing 6).
"""
import math

MASS_LO, MASS_HI = 5.0, 5.6


def _p(name, value, lo=-1e30, hi=1e30, fixed=False):
    return {"name": name, "value": float(value), "lo": float(lo), "hi": float(hi),
            "fixed": bool(fixed)}


# 1-D mass fit: f*Gauss(m; mu, sigma) + (1-f)*Exp(m; lambda) on [5.0, 5.6].
MASS1D_TRUTH = {"mu": 5.28, "sigma": 0.02, "lambda": -1.5, "fsig": 0.3}


def mass1d(mu=5.28, sigma=0.02, lam=-1.5, fsig=0.3, lo=MASS_LO, hi=MASS_HI):
    return {
        "dims": [{"name": "m", "lo": lo, "hi": hi}],
        "params": [_p("mu", mu, lo, hi), _p("sigma", sigma, 1e-4, 1.0),
                   _p("lambda", lam, -10.0, 10.0), _p("fsig", fsig, 0.0, 1.0)],
        "nodes": [{"kind": "gauss", "dims": [0], "params": [0, 1]},
                  {"kind": "exp", "dims": [0], "params": [2]},
                  {"kind": "sum", "children": [0, 1], "params": [3]}],
        "root": 2,
    }


def mass1d_start(truth=MASS1D_TRUTH, lo=MASS_LO, hi=MASS_HI):
    """Start 5% off truth: sigma, lambda and f scaled by 1.05; mu moved by 5%
    of the window (a literal 1.05*mu would sit outside the signal peak)."""
    return [truth["mu"] + 0.05 * (hi - lo), 1.05 * truth["sigma"],
            1.05 * truth["lambda"], 1.05 * truth["fsig"]]


ANG_NAMES = ["FL", "S3", "S4", "S5", "AFB", "S7", "S8", "S9"]
ANG_TRUTH = (0.7, 0.0, -0.1, -0.2, 0.1, 0.0, 0.0, 0.0)
CHEB_TRUTH = ((0.1, 0.05), (0.1, 0.05), (0.1, 0.05))


def angmass4d(ang=ANG_TRUTH, mu=5.28, sigma=0.02, lam=-1.5, cheb=CHEB_TRUTH, fsig=0.4,
              mu_fixed=True, lo=MASS_LO, hi=MASS_HI):
    """Signal P-wave(ctl, ctk, phi) x Gauss(m), background
    Cheb(ctl) x Cheb(ctk) x Cheb(phi) x Exp(m), signal fraction fsig.
    Parameter order: FL S3 S4 S5 AFB S7 S8 S9 mu sigma lambda
    cl1 cl2 ck1 ck2 cp1 cp2 fsig (18; mu fixed by default -> 17 free)."""
    params = [_p(n, v, -1.0, 1.0) for n, v in zip(ANG_NAMES, ang)]
    params += [_p("mu", mu, lo, hi, fixed=mu_fixed), _p("sigma", sigma, 1e-4, 1.0),
               _p("lambda", lam, -10.0, 10.0)]
    for d, name in enumerate(("cl", "ck", "cp")):
        params += [_p(f"{name}1", cheb[d][0], -1.0, 1.0), _p(f"{name}2", cheb[d][1], -1.0, 1.0)]
    params.append(_p("fsig", fsig, 0.0, 1.0))
    return {
        "dims": [{"name": "m", "lo": lo, "hi": hi},
                 {"name": "ctl", "lo": -1.0, "hi": 1.0},
                 {"name": "ctk", "lo": -1.0, "hi": 1.0},
                 {"name": "phi", "lo": -math.pi, "hi": math.pi}],
        "params": params,
        "nodes": [{"kind": "pwave", "dims": [1, 2, 3], "params": list(range(8))},
                  {"kind": "gauss", "dims": [0], "params": [8, 9]},
                  {"kind": "prod", "children": [0, 1]},
                  {"kind": "cheb", "dims": [1], "params": [11, 12]},
                  {"kind": "cheb", "dims": [2], "params": [13, 14]},
                  {"kind": "cheb", "dims": [3], "params": [15, 16]},
                  {"kind": "exp", "dims": [0], "params": [10]},
                  {"kind": "prod", "children": [3, 4, 5, 6]},
                  {"kind": "sum", "children": [2, 7], "params": [17]}],
        "root": 8,
    }


def angmass4d_truth_vector():
    v = list(ANG_TRUTH) + [5.28, 0.02, -1.5]
    for c in CHEB_TRUTH:
        v += list(c)
    return v + [0.4]


def pwave3d(ang=(0.6, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0)):
    """The paper's angular fit (Sec. 3.3): the P-wave density alone, 8 parameters."""
    return {
        "dims": [{"name": "ctl", "lo": -1.0, "hi": 1.0},
                 {"name": "ctk", "lo": -1.0, "hi": 1.0},
                 {"name": "phi", "lo": -math.pi, "hi": math.pi}],
        "params": [_p(n, v, -1.0, 1.0) for n, v in zip(ANG_NAMES, ang)],
        "nodes": [{"kind": "pwave", "dims": [0, 1, 2], "params": list(range(8))}],
        "root": 0,
    }
