"""Offline model compile for encrypted KAN inference (host side, no GPU).

Turns trained (here: seeded random) KAN weights into the HE-friendly layer
description the library consumes (Method):
  * SiLU Approximation: range [max(mu-5 sigma, x_min), min(mu+5 sigma, x_max)]
    from Chebyshev's inequality, then a weighted least-squares fit (weight 10
    inside mu +- 3 sigma, 1 outside) in the Chebyshev basis of that range;
  * B-spline Basis Approximation: the g+2k+1 knots, the bound R used to scale
    comparison inputs into [-1, 1] (an explicit product by 1/(2R), or folded
    into the first stage when levels are short), and PolyComp as a composite
    of the odd sign-approximating polynomials f_n (final 1/2 folded into the
    last stage);
  * calibration statistics per layer from seeded inputs propagated through
    the HE-friendly network in plain FP64 (hidden layers get a grid fitted to
    their input range).
"""
from dataclasses import dataclass, field
from math import comb

import numpy as np
from numpy.polynomial import chebyshev as cheb


@dataclass
class KanLayer:
    n_in: int
    n_out: int
    g: int
    k: int
    knots: np.ndarray
    wb: np.ndarray
    ws: np.ndarray
    c: np.ndarray
    silu_coeffs: np.ndarray
    silu_lo: float
    silu_hi: float
    R: float
    comp: list = field(default_factory=list)
    comp_prescale: float = 0.0


def knot_vector(lo, hi, g, k):
    h = (hi - lo) / g
    return np.array([lo + float(j - k) * h for j in range(g + 2 * k + 1)])


def sign_poly(n):
    """f_n(x) = sum_{i<=n} C(2i,i) 4^-i x (1-x^2)^i as odd-power coefficients."""
    num = [0] * (n + 1)
    den = 4 ** n
    for i in range(n + 1):
        w = comb(2 * i, i) * 4 ** (n - i)
        for j in range(i + 1):
            num[j] += w * comb(i, j) * (-1) ** j
    return [v / den for v in num]


def comparison_stages(degrees, R, fold=True):
    stages = [sign_poly((d - 1) // 2) for d in degrees]
    if fold:
        inv = 1.0 / (2.0 * R)
        stages[0] = [a * inv ** (2 * i + 1) for i, a in enumerate(stages[0])]
    stages[-1] = [a * 0.5 for a in stages[-1]]
    return [np.asarray(s, np.float64) for s in stages]


def boot_cos_coeffs(K, r, degree):
    """EvalMod's series for a bootstrapping plan (he_boot_desc): the Chebyshev
    interpolant of cos(2 pi (y - 1/4) / 2^r) on [-K, K] at the degree + 1
    Chebyshev points (chebinterpolate), so that r double-angle steps give
    sin(2 pi y)."""
    return list(cheb.chebinterpolate(lambda u: np.cos(2.0 * np.pi * (K * u - 0.25) / 2.0 ** r), degree))


def silu_range(mu, sd, lo, hi):
    return max(mu - 5.0 * sd, lo), min(mu + 5.0 * sd, hi)


def silu(x):
    return x / (1.0 + np.exp(-x))


def _u(x, lo, hi):
    return (2.0 * x - (lo + hi)) / (hi - lo)


def fit_silu(lo, hi, degree, mu, sd, n=4001):
    """The paper's fit (SiLU Approximation): weighted least squares on n uniform
    samples of the range, weight 10 inside mu +- 3 sigma and 1 outside."""
    x = np.linspace(lo, hi, n)
    sw = np.sqrt(np.where(np.abs(x - mu) <= 3.0 * sd, 10.0, 1.0))
    A = cheb.chebvander(_u(x, lo, hi), degree) * sw[:, None]
    return np.linalg.lstsq(A, silu(x) * sw, rcond=None)[0]


def fit_silu_ols(lo, hi, degree, n=4001):
    """Ordinary least squares on the same uniform samples (every weight 1):
    the least-squares comparator of the SiLU Approximation experiments."""
    x = np.linspace(lo, hi, n)
    return np.linalg.lstsq(cheb.chebvander(_u(x, lo, hi), degree), silu(x), rcond=None)[0]


def remez(f, lo, hi, degree, grid=100001, iters=60, tol=1e-12):
    """Minimax polynomial of `degree` for f on [lo, hi] in the Chebyshev basis
    of the range, by the Remez exchange: solve p(x_j) + (-1)^j E = f(x_j) on
    degree + 2 reference points, move the references to the alternating
    extrema of the error on a dense grid, repeat until the largest error
    equals |E| to `tol` (relative).  Returns (coefficients, max error)."""
    n = degree
    j = np.arange(n + 2)
    ref = np.sort(np.cos(np.pi * j / (n + 1)))            # Chebyshev extrema in [-1, 1]
    xs = np.linspace(-1.0, 1.0, grid)
    fx = f(lo + (xs + 1.0) * (hi - lo) / 2.0)
    c, err = None, None
    for _ in range(iters):
        fr = f(lo + (ref + 1.0) * (hi - lo) / 2.0)
        A = np.hstack([cheb.chebvander(ref, n), ((-1.0) ** j)[:, None]])
        sol = np.linalg.solve(A, fr)
        c, E = sol[:-1], sol[-1]
        e = fx - cheb.chebval(xs, c)
        err = float(np.abs(e).max())
        if err - abs(E) <= tol * err:
            break
        # one extremum per run of equal sign, then keep n + 2 alternating ones
        # around the largest (multi-point exchange)
        sgn = np.sign(e)
        sgn[sgn == 0] = 1.0
        cut = np.flatnonzero(np.diff(sgn) != 0) + 1
        runs = np.split(np.arange(grid), cut)
        ext = np.array([r[np.argmax(np.abs(e[r]))] for r in runs])
        while len(ext) > n + 2:
            # drop the smaller end, never the global maximum
            if abs(e[ext[0]]) <= abs(e[ext[-1]]):
                ext = ext[1:]
            else:
                ext = ext[:-1]
        if len(ext) < n + 2:
            break
        ref = xs[ext]
    return c, err


def fit_silu_remez(lo, hi, degree):
    """Minimax (Remez) fit of SiLU on the range: the Remez comparator."""
    return remez(silu, lo, hi, degree)[0]


def silu_fit_comparison(lo, hi, degree, samples, n=4001):
    """Weighted least squares (mu, sigma of `samples`), ordinary least squares
    and Remez minimax at one degree and range, each measured by the RMSE over
    the range's n uniform points, the RMSE over `samples` (the activation
    distribution) and the largest error on the range."""
    samples = np.asarray(samples, np.float64)
    mu, sd = float(samples.mean()), float(samples.std())
    x = np.linspace(lo, hi, n)
    inside = samples[(samples >= lo) & (samples <= hi)]
    out = {}
    for name, c in (("wls", fit_silu(lo, hi, degree, mu, sd, n)), ("ols", fit_silu_ols(lo, hi, degree, n)),
                    ("remez", fit_silu_remez(lo, hi, degree))):
        eu = cheb.chebval(_u(x, lo, hi), c) - silu(x)
        ed = cheb.chebval(_u(inside, lo, hi), c) - silu(inside)
        out[name] = {"rmse_uniform": float(np.sqrt(np.mean(eu ** 2))),
                     "rmse_data": float(np.sqrt(np.mean(ed ** 2))), "max_err": float(np.abs(eu).max())}
    return out


def _soft_step(v, stages):
    for a in stages:
        v = sum(ai * v ** (2 * i + 1) for i, ai in enumerate(a))
    return v + 0.5


def plain_layer(x, L: KanLayer):
    """The HE-friendly layer on plain FP64 arrays, x: (batch, n_in)."""
    t = L.knots
    r = L.g + 2 * L.k + 1
    u = (2.0 * x - (L.silu_lo + L.silu_hi)) / (L.silu_hi - L.silu_lo)
    yb = cheb.chebval(u, L.silu_coeffs) @ L.wb.T
    xe = x[:, :, None]
    sc = L.comp_prescale if L.comp_prescale else 1.0
    B = _soft_step((xe - t[None, None, :r - 1]) * sc, L.comp) * _soft_step((t[None, None, 1:r] - xe) * sc, L.comp)
    for j in range(1, L.k + 1):
        n = r - 1 - j
        B = ((xe - t[:n]) / (t[j:j + n] - t[:n]) * B[:, :, :n]
             + (t[j + 1:j + 1 + n] - xe) / (t[j + 1:j + 1 + n] - t[1:1 + n]) * B[:, :, 1:n + 1])
    ys = np.einsum("bim,oim->bo", B, L.ws[:, :, None] * L.c)
    return yb + ys


def plain_forward(x, layers):
    x = np.atleast_2d(np.asarray(x, np.float64))
    for L in layers:
        x = plain_layer(x, L)
    return x


def compile_kan(raw_layers, calib, silu_degree, comp_degrees, first_grid, silu_fixed_range=None, prescale=True):
    """raw_layers: [{wb, ws, c, g, k}], calib: (n, n_in) calibration inputs."""
    out = []
    x = np.asarray(calib, np.float64)
    for li, raw in enumerate(raw_layers):
        n_out, n_in = raw["wb"].shape
        mu, sd, lo, hi = float(x.mean()), float(x.std()), float(x.min()), float(x.max())
        grid = first_grid if li == 0 else (lo, hi)
        knots = knot_vector(grid[0], grid[1], raw["g"], raw["k"])
        slo, shi = silu_fixed_range if silu_fixed_range is not None else silu_range(mu, sd, lo, hi)
        degree = silu_degree[li] if hasattr(silu_degree, "__len__") else silu_degree
        coeffs = fit_silu(slo, shi, degree, mu, sd)
        R = max(float(np.abs(knots).max()), 1.1 * float(np.abs(x).max()))
        L = KanLayer(n_in, n_out, raw["g"], raw["k"], knots, raw["wb"], raw["ws"], raw["c"], coeffs, slo, shi, R,
                     comparison_stages(comp_degrees[li], R, fold=not prescale),
                     1.0 / (2.0 * R) if prescale else 0.0)
        out.append(L)
        x = plain_layer(x, L)
    return out
