"""Plain FP64 KAN references and the oracle-side model compile.

TEST INFRASTRUCTURE ONLY (tests/, the smoke check and the CPU-baseline leg of
the benchmark); the product package never imports this module.

Three things live here, each written from the paper:

* the exact KAN ("O3"): phi(x) = w_b silu(x) + w_s spline(x) per edge with
  spline(x) = sum_m c_m B_{m,k}(x) from the Cox-de Boor recursion
  (Preliminaries, the KAN equations and the B-spline recursion);
* the HE-friendly circuit in FP64 ("O2"): the same network with silu replaced
  by the fitted Chebyshev polynomial (Method, SiLU Approximation) and the
  indicator of the order-0 basis replaced by products of comparison
  polynomials followed by the order-k recursion (Method, B-spline Basis
  Approximation, Algorithm 2), evaluated slot-free on plain arrays;
* the offline model compile: approximation range from Chebyshev's inequality,
  weighted least-squares SiLU fit, knot vectors, comparison composite,
  bound R, lazy-combination weights W' and the Algorithm 3 permutation.
"""
from dataclasses import dataclass, field
from fractions import Fraction
from math import comb

import numpy as np
from numpy.polynomial import chebyshev as C


def silu(x):
    """silu(x) = x / (1 + e^-x)  (Preliminaries, KAN base function b(x))."""
    return x / (1.0 + np.exp(-x))


# --------------------------------------------------------------------------
# B-splines
# --------------------------------------------------------------------------
def make_knots(lo, hi, g, k):
    """r = g+2k+1 uniform knots t_1..t_r (returned 0-based) with
    t_p = lo + (p-1-k) h, h = (hi-lo)/g, so [lo, hi] = [t_{k+1}, t_{g+k+1}] and
    there are g+k order-k bases (Method, lazy combination: C is n_i x (g+k))."""
    h = (hi - lo) / g
    return np.array([lo + float(p - 1 - k) * h for p in range(1, g + 2 * k + 2)], np.float64)


def bspline_exact(x, t, k):
    """Cox-de Boor: B_{m,0} = 1 on [t_m, t_{m+1}), then
    B_{m,j} = (x-t_m)/(t_{m+j}-t_m) B_{m,j-1} + (t_{m+j+1}-x)/(t_{m+j+1}-t_{m+1}) B_{m+1,j-1}.
    x: any shape; returns shape x.shape + (len(t)-1-k,)."""
    x = np.asarray(x, np.float64)[..., None]
    B = ((x >= t[:-1]) & (x < t[1:])).astype(np.float64)
    for j in range(1, k + 1):
        n = len(t) - 1 - j
        left = (x - t[:n]) / (t[j:j + n] - t[:n]) * B[..., :n]
        right = (t[j + 1:j + 1 + n] - x) / (t[j + 1:j + 1 + n] - t[1:1 + n]) * B[..., 1:n + 1]
        B = left + right
    return B


# --------------------------------------------------------------------------
# comparison composite (PolyComp)
# --------------------------------------------------------------------------
def fn_odd_coeffs(n):
    """Odd power coefficients [a1, a3, ..., a_{2n+1}] of
    f_n(x) = sum_{i=0}^{n} 4^-i C(2i,i) x (1-x^2)^i  (Cheon, Kim, Kim, Lee, Lee,
    Asiacrypt 2020), an odd map of [-1,1] onto itself that sharpens sign(x)."""
    a = [Fraction(0)] * (n + 1)
    for i in range(n + 1):
        ci = Fraction(comb(2 * i, i), 4 ** i)
        for j in range(i + 1):
            a[j] += ci * comb(i, j) * (-1) ** j
    return [float(v) for v in a]


DEG_TO_N = {3: 1, 5: 2, 7: 3}


def composite_stages(degrees, R, fold=True):
    """Stage coefficient lists for S(v) = (F(v/(2R)) + 1)/2, F = f_{n_d} o ... o f_{n_1}:
    the final 1/2 is folded into the last stage and the evaluator adds 1/2.
    With fold=True the 1/(2R) input scaling is folded into the first stage
    (saves a level, fine for small R); otherwise the comparison input is
    multiplied by 1/(2R) explicitly, as Algorithm 2 writes it."""
    stages = [list(fn_odd_coeffs(DEG_TO_N[d])) for d in degrees]
    if fold:
        s = 1.0 / (2.0 * R)
        stages[0] = [a * s ** (2 * i + 1) for i, a in enumerate(stages[0])]
    stages[-1] = [a * 0.5 for a in stages[-1]]
    return [np.array(st, np.float64) for st in stages]


def eval_odd(v, a):
    """sum_i a_i v^(2i+1)."""
    v = np.asarray(v, np.float64)
    return sum(ai * v ** (2 * i + 1) for i, ai in enumerate(a))


def polycomp(v, stages):
    """S(v): 1 for v >> 0, 0 for v << 0, 1/2 at v = 0 (PolyComp(v, 0))."""
    for a in stages:
        v = eval_odd(v, a)
    return v + 0.5


# --------------------------------------------------------------------------
# model description
# --------------------------------------------------------------------------
@dataclass
class Layer:
    """One KANLayer n_in -> n_out with the HE-friendly constants."""
    n_in: int
    n_out: int
    g: int
    k: int
    knots: np.ndarray       # g+2k+1
    wb: np.ndarray          # (n_out, n_in) base weights
    ws: np.ndarray          # (n_out, n_in) spline scales
    c: np.ndarray           # (n_out, n_in, g+k) spline coefficients (per edge)
    silu_coeffs: np.ndarray # Chebyshev coefficients on [silu_lo, silu_hi]
    silu_lo: float
    silu_hi: float
    R: float
    comp: list = field(default_factory=list)  # stage coefficient arrays
    comp_prescale: float = 0.0  # explicit 1/(2R) product before PolyComp (0: folded into stage 0)


def exact_kan(x, layers):
    """O3: the exact KAN (true silu, exact Cox-de Boor). x: (batch, n_in)."""
    x = np.atleast_2d(np.asarray(x, np.float64))
    for L in layers:
        B = bspline_exact(x, L.knots, L.k)                    # (b, n_in, g+k)
        spline = np.einsum("oim,bim->boi", L.c, B)            # (b, n_out, n_in)
        x = np.einsum("oi,bi->bo", L.wb, silu(x)) + np.einsum("oi,boi->bo", L.ws, spline)
    return x


def soft_bspline(x, L):
    """Algorithm 2 on plain values: the order-0 basis from two comparisons,
    B^0_m = S(x - t_{m+1}) * S(t_{m+2} - x) for m < g+2k, then k rounds of
    B^j_m = (x-t_{m+1})/(t_{m+j+1}-t_{m+1}) B^{j-1}_m
          + (t_{m+j+2}-x)/(t_{m+j+2}-t_{m+2}) B^{j-1}_{m+1}."""
    t = L.knots
    x = np.asarray(x, np.float64)[..., None]
    r = L.g + 2 * L.k + 1
    sc = L.comp_prescale if L.comp_prescale else 1.0
    B = polycomp((x - t[: r - 1]) * sc, L.comp) * polycomp((t[1:r] - x) * sc, L.comp)
    for j in range(1, L.k + 1):
        n = r - 1 - j
        a1 = 1.0 / (t[j:j + n] - t[:n])
        a2 = 1.0 / (t[j + 1:j + 1 + n] - t[1:1 + n])
        B = a1 * (x - t[:n]) * B[..., :n] + a2 * (t[j + 1:j + 1 + n] - x) * B[..., 1:n + 1]
    return B


def silu_poly(x, L):
    u = (2.0 * np.asarray(x, np.float64) - (L.silu_lo + L.silu_hi)) / (L.silu_hi - L.silu_lo)
    return C.chebval(u, L.silu_coeffs)


def he_friendly_layer(x, L):
    s = silu_poly(x, L)
    B = soft_bspline(x, L)
    return np.einsum("oi,bi->bo", L.wb, s) + np.einsum("oi,oim,bim->bo", L.ws, L.c, B)


def he_friendly_kan(x, layers):
    """O2: the HE-friendly circuit in FP64. x: (batch, n_in)."""
    x = np.atleast_2d(np.asarray(x, np.float64))
    for L in layers:
        x = he_friendly_layer(x, L)
    return x


# --------------------------------------------------------------------------
# offline compile
# --------------------------------------------------------------------------
def approx_range(mu, sigma, xmin, xmax):
    """[max(mu-5 sigma, x_min), min(mu+5 sigma, x_max)] (Method, SiLU
    Approximation, Chebyshev's inequality with eps = 5 sigma)."""
    return max(mu - 5.0 * sigma, xmin), min(mu + 5.0 * sigma, xmax)


def wls_weights(x, mu, sigma):
    """w_i = 10 inside [mu-3 sigma, mu+3 sigma], 1 outside."""
    return np.where(np.abs(x - mu) <= 3.0 * sigma, 10.0, 1.0)


def wls_fit_silu(lo, hi, deg, mu, sigma, n=4001):
    """Weighted least squares min sum_i w_i (y_i - f(x_i))^2 over uniform samples
    of the range, f in the Chebyshev basis of [lo, hi]."""
    x = np.linspace(lo, hi, n)
    y = silu(x)
    w = wls_weights(x, mu, sigma)
    u = (2.0 * x - (lo + hi)) / (hi - lo)
    V = C.chebvander(u, deg)
    sw = np.sqrt(w)
    coef, *_ = np.linalg.lstsq(V * sw[:, None], y * sw, rcond=None)
    return coef


def choose_R(knots, xs):
    """R = max(max_p |t_p|, 1.1 max |x|) over the calibration inputs."""
    return max(float(np.max(np.abs(knots))), 1.1 * float(np.max(np.abs(xs))))


def alg3_permutation(n_r, n_c):
    """Algorithm 3: P[j_r][j_c] = 1 for j_c = (c-1) n_r + r, j_r = (r-1) n_c + c
    (1-based r <= n_r, c <= n_c).  Returned as a dense 0/1 matrix."""
    Pm = np.zeros((n_r * n_c, n_r * n_c))
    for r in range(1, n_r + 1):
        for c in range(1, n_c + 1):
            jc = (c - 1) * n_r + r
            jr = (r - 1) * n_c + c
            Pm[jr - 1][jc - 1] = 1.0
    return Pm


def alg3_index(n_r, n_c):
    """The same permutation as an index map: column j_c of W' P is column
    j_r(j_c) of W' (0-based)."""
    idx = np.zeros(n_r * n_c, np.int64)
    for r in range(1, n_r + 1):
        for c in range(1, n_c + 1):
            idx[(c - 1) * n_r + r - 1] = (r - 1) * n_c + c - 1
    return idx


def lazy_weights(L):
    """W' (n_out x n_in (g+k)), W'[o, i (g+k) + m] = w_s[o,i] c[o,i,m]: the spline
    coefficients folded into the following linear layer (lazy combination)."""
    nb = L.g + L.k
    Wp = (L.ws[:, :, None] * L.c).reshape(L.n_out, L.n_in * nb)
    return Wp


def fused_weights(L, n_blk):
    """W_f = W' P laid out for the ColTile basis vector with blocks of n_blk slots:
    W_f[o, m n_blk + i] = W'[o, i (g+k) + m] for i < n_in, zero for padded
    inputs i >= n_in."""
    nb = L.g + L.k
    Wp = lazy_weights(L)
    idx = alg3_index(L.n_in, nb)
    Wperm = Wp[:, idx]                                         # columns in ColTile order, block width n_in
    Wf = np.zeros((L.n_out, nb * n_blk))
    for m in range(nb):
        Wf[:, m * n_blk:m * n_blk + L.n_in] = Wperm[:, m * L.n_in:(m + 1) * L.n_in]
    return Wf


def compile_model(raw_layers, x_calib, degrees_silu, comp_degrees, first_grid, silu_fixed_range=None,
                  prescale=True):
    """Build the HE-friendly layer list.

    raw_layers: list of dicts {wb, ws, c, g, k} (weights only).
    x_calib: (n, n_in) calibration inputs propagated layer by layer through
    the HE-friendly circuit to get each layer's input statistics.
    first_grid: (lo, hi) grid of the first layer; hidden layers take the
    range [min, max] of their calibration inputs (a data-fitted grid).
    comp_degrees: per layer list of composite stage degrees (3, 5 or 7).
    prescale: multiply comparison inputs by 1/(2R) explicitly (one level)
    instead of folding the factor into the first stage."""
    layers = []
    x = np.asarray(x_calib, np.float64)
    for li, raw in enumerate(raw_layers):
        n_out, n_in = raw["wb"].shape
        g, k = raw["g"], raw["k"]
        mu, sd = float(x.mean()), float(x.std())
        xmin, xmax = float(x.min()), float(x.max())
        lo, hi = first_grid if li == 0 else (xmin, xmax)
        knots = make_knots(lo, hi, g, k)
        if silu_fixed_range is not None:
            slo, shi = silu_fixed_range
        else:
            slo, shi = approx_range(mu, sd, xmin, xmax)
        coef = wls_fit_silu(slo, shi, degrees_silu[li], mu, sd)
        R = choose_R(knots, x)
        L = Layer(n_in, n_out, g, k, knots, raw["wb"], raw["ws"], raw["c"], coef, slo, shi, R,
                  composite_stages(comp_degrees[li], R, fold=not prescale),
                  1.0 / (2.0 * R) if prescale else 0.0)
        layers.append(L)
        x = he_friendly_layer(x, L)
    return layers
