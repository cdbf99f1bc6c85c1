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


def silu_range(mu, sd, lo, hi):
    return max(mu - 5.0 * sd, lo), min(mu + 5.0 * sd, hi)


def fit_silu(lo, hi, degree, mu, sd, n=4001):
    x = np.linspace(lo, hi, n)
    y = x / (1.0 + np.exp(-x))
    sw = np.sqrt(np.where(np.abs(x - mu) <= 3.0 * sd, 10.0, 1.0))
    A = cheb.chebvander((2.0 * x - (lo + hi)) / (hi - lo), degree) * sw[:, None]
    return np.linalg.lstsq(A, y * sw, rcond=None)[0]


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
