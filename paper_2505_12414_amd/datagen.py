"""Seeded synthetic event generators.

The MoreFit paper benchmarks on pseudo-experiments drawn from the fitted
models themselves (Sec. 3.1; accept-reject generation, Sec. 2.5).  These
generators produce such events for the tests, the benchmark and the serving
workload.  Both the GPU path and the oracle consume their output; neither
side's arithmetic lives here: nothing below computes a normalisation, a
logarithm or a derivative.  The samplers use numpy's PCG64 generator:

* Gaussian in a window: numpy normal draws, rejected outside the window;
* exponential in a window: numpy exponential draws measured from the window
  edge the density decays away from, rejected beyond the other edge;
* Chebyshev-shaped and P-wave angular shapes: accept-reject against a
  constant envelope (for the P-wave shape, the bound the paper's PDF class
  returns for generation, Listing 7), evaluating only the unnormalised shape.

Events come back as a structure of arrays, shape (ndim, n), in the requested
storage dtype.
"""
import math

import numpy as np


def _rng(seed):
    return np.random.Generator(np.random.PCG64(int(seed)))


def to_storage(x, lo, hi, dtype):
    """Rounds to the storage type, keeping every value inside [lo, hi]
    (a range edge such as pi need not be representable in that type)."""
    y = np.asarray(x).astype(dtype)
    lo_t = np.asarray(lo, dtype=dtype)
    if lo_t < lo:
        lo_t = np.nextafter(lo_t, np.asarray(np.inf, dtype=dtype))
    hi_t = np.asarray(hi, dtype=dtype)
    if hi_t > hi:
        hi_t = np.nextafter(hi_t, np.asarray(-np.inf, dtype=dtype))
    return np.clip(y, lo_t, hi_t)


def trunc_normal(rng, n, mu, sigma, lo, hi):
    out = np.empty(n, dtype=np.float64)
    k = 0
    while k < n:
        draw = rng.normal(mu, sigma, size=max(2 * (n - k), 1024))
        draw = draw[(draw >= lo) & (draw <= hi)]
        take = min(n - k, draw.size)
        out[k:k + take] = draw[:take]
        k += take
    return out


def trunc_exponential(rng, n, lam, lo, hi):
    """Density proportional to exp(lam * x) on [lo, hi]."""
    if lam == 0.0:
        return rng.uniform(lo, hi, size=n)
    out = np.empty(n, dtype=np.float64)
    k = 0
    while k < n:
        t = rng.exponential(1.0 / abs(lam), size=max(2 * (n - k), 1024))
        t = t[t <= hi - lo]
        x = lo + t if lam < 0 else hi - t
        take = min(n - k, x.size)
        out[k:k + take] = x[:take]
        k += take
    return out


def cheb_shape(rng, n, coeffs, lo, hi):
    """Density proportional to 1 + sum_j c_j T_j(u), u mapped from [lo, hi]."""
    env = 1.0 + sum(abs(c) for c in coeffs)
    out = np.empty(n, dtype=np.float64)
    k = 0
    while k < n:
        m = max(2 * (n - k), 1024)
        x = rng.uniform(lo, hi, size=m)
        u = (2.0 * x - lo - hi) / (hi - lo)
        shape = np.ones(m)
        t_prev, t_cur = np.ones(m), u
        for c in coeffs:
            shape += c * t_cur
            t_prev, t_cur = t_cur, 2.0 * u * t_cur - t_prev
        keep = x[rng.uniform(0.0, env, size=m) < shape]
        take = min(n - k, keep.size)
        out[k:k + take] = keep[:take]
        k += take
    return out


def pwave_shape(rng, n, FL, S3, S4, S5, AFB, S7, S8, S9):
    """(cos theta_l, cos theta_K, phi) distributed as the P-wave decay rate."""
    env = 9.0 / (32.0 * math.pi) * (4.0 + abs(S3) + abs(S4) + abs(S5) + 4.0 / 3.0 * abs(AFB)
                                    + abs(S7) + abs(S8) + abs(S9))
    out = np.empty((3, n), dtype=np.float64)
    k = 0
    while k < n:
        m = max(4 * (n - k), 4096)
        cl = rng.uniform(-1.0, 1.0, size=m)
        ck = rng.uniform(-1.0, 1.0, size=m)
        ph = rng.uniform(-math.pi, math.pi, size=m)
        sl2, sk2 = 1.0 - cl * cl, 1.0 - ck * ck
        sl, sk = np.sqrt(sl2), np.sqrt(sk2)
        c2l = 2.0 * cl * cl - 1.0
        shape = 9.0 / (32.0 * math.pi) * (
            0.75 * (1.0 - FL) * sk2 + FL * ck * ck + 0.25 * (1.0 - FL) * sk2 * c2l
            - FL * ck * ck * c2l + S3 * sk2 * sl2 * np.cos(2 * ph)
            + S4 * (2 * sk * ck) * (2 * sl * cl) * np.cos(ph)
            + S5 * (2 * sk * ck) * sl * np.cos(ph) + AFB * 4.0 / 3.0 * sk2 * cl
            + S7 * (2 * sk * ck) * sl * np.sin(ph) + S8 * (2 * sk * ck) * (2 * sl * cl) * np.sin(ph)
            + S9 * sk2 * sl2 * np.sin(2 * ph))
        keep = rng.uniform(0.0, env, size=m) < shape
        take = min(n - k, int(keep.sum()))
        out[0, k:k + take] = cl[keep][:take]
        out[1, k:k + take] = ck[keep][:take]
        out[2, k:k + take] = ph[keep][:take]
        k += take
    return out


def gen_mass1d(n, seed, mu=5.28, sigma=0.02, lam=-1.5, fsig=0.3, lo=5.0, hi=5.6,
               dtype=np.float64):
    """f*Gauss + (1-f)*Exp on [lo, hi]; returns shape (1, n)."""
    rng = _rng(seed)
    is_sig = rng.uniform(size=n) < fsig
    ns = int(is_sig.sum())
    m = np.empty(n, dtype=np.float64)
    m[is_sig] = trunc_normal(rng, ns, mu, sigma, lo, hi)
    m[~is_sig] = trunc_exponential(rng, n - ns, lam, lo, hi)
    return to_storage(m, lo, hi, dtype).reshape(1, n)


ANGLES_LO = (-1.0, -1.0, -math.pi)
ANGLES_HI = (1.0, 1.0, math.pi)


def gen_angmass4d(n, seed, ang=(0.7, 0.0, -0.1, -0.2, 0.1, 0.0, 0.0, 0.0), mu=5.28,
                  sigma=0.02, lam=-1.5, cheb=((0.1, 0.05),) * 3, fsig=0.4, mlo=5.0,
                  mhi=5.6, dtype=np.float32):
    """Signal P-wave(angles) x Gauss(m) with fraction fsig, background
    Chebyshev(ctl) x Chebyshev(ctk) x Chebyshev(phi) x Exp(m).
    Returns shape (4, n): rows m, cos theta_l, cos theta_K, phi."""
    rng = _rng(seed)
    is_sig = rng.uniform(size=n) < fsig
    ns = int(is_sig.sum())
    nb = n - ns
    x = np.empty((4, n), dtype=np.float64)
    x[0, is_sig] = trunc_normal(rng, ns, mu, sigma, mlo, mhi)
    x[1:, is_sig] = pwave_shape(rng, ns, *ang)
    x[0, ~is_sig] = trunc_exponential(rng, nb, lam, mlo, mhi)
    for d in range(3):
        x[1 + d, ~is_sig] = cheb_shape(rng, nb, cheb[d], ANGLES_LO[d], ANGLES_HI[d])
    lo = (mlo,) + ANGLES_LO
    hi = (mhi,) + ANGLES_HI
    return np.stack([to_storage(x[d], lo[d], hi[d], dtype) for d in range(4)])


def gen_pwave3d(n, seed, ang=(0.6, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0), dtype=np.float64):
    """The paper's angular workload (Sec. 3.3): P-wave density only."""
    rng = _rng(seed)
    x = pwave_shape(rng, n, *ang)
    return np.stack([to_storage(x[d], ANGLES_LO[d], ANGLES_HI[d], dtype) for d in range(3)])


def uniform_weights(n, seed, lo=0.5, hi=1.5, dtype=np.float32):
    """Per-event weights w ~ U(lo, hi), independent of the events."""
    return _rng(seed).uniform(lo, hi, size=n).astype(dtype)


def gen_mix1d(n, seed, ncomp, dtype=np.float64):
    """The 1-D mixtures of three and four components used by the parity
    tests, as nested sums on [5.0, 5.6]:
        f1 G(5.25, 0.02) + (1 - f1) [f2 G(5.35, 0.04) + (1 - f2) E(-1.5)]       (3)
        f1 G(5.25, 0.02) + (1 - f1) [f2 G(5.35, 0.04)
                                     + (1 - f2) (f3 E(-1.5) + (1 - f3) C(0.2))]  (4)
    with f1 = 0.3, f2 = 0.4, f3 = 0.5.  Each event picks its component by
    the fractions, then draws from it; returns shape (1, n)."""
    lo, hi = 5.0, 5.6
    rng = _rng(seed)
    u = rng.uniform(size=(3, n))
    g1 = u[0] < 0.3
    g2 = ~g1 & (u[1] < 0.4)
    rest = ~g1 & ~g2
    ex = rest & (u[2] < 0.5) if ncomp == 4 else rest
    ch = rest & ~ex
    m = np.empty(n, dtype=np.float64)
    m[g1] = trunc_normal(rng, int(g1.sum()), 5.25, 0.02, lo, hi)
    m[g2] = trunc_normal(rng, int(g2.sum()), 5.35, 0.04, lo, hi)
    m[ex] = trunc_exponential(rng, int(ex.sum()), -1.5, lo, hi)
    if ncomp == 4:
        m[ch] = cheb_shape(rng, int(ch.sum()), (0.2,), lo, hi)
    return to_storage(m, lo, hi, dtype).reshape(1, n)
