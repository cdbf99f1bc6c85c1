"""The SiLU approximation comparators of the paper's SiLU experiments (host
side, no GPU): the weighted least-squares fit the method uses, ordinary
least squares and Remez minimax, at one degree and range.

Pins: the Remez exchange reproduces the closed-form minimax approximation of
x^(n+1) on [-1, 1] (x^(n+1) - 2^-n T_(n+1), error 2^-n) and equioscillates on
SiLU; ordinary least squares equals numpy's unweighted Chebyshev fit; and
each method is best at the measure it optimises (least squares: the RMSE
over the uniform samples; the weighted fit: the weighted objective; Remez:
the largest error), so a slip in any of them fails an ordering."""
import numpy as np
import pytest
from numpy.polynomial import chebyshev as cheb

from paper_2409_07751_amd import compile as pc

# the three approximation ranges and degrees the paper's experiments state
# (5-sigma ranges of its three image data sets; degrees 10, 10 and 15)
RANGES = [(-12.4, 14.74, 10), (-9.77, 11.01, 10), (-11.90, 10.99, 15)]


@pytest.mark.parametrize("n", [1, 3, 6, 10, 15])
def test_remez_closed_form(n):
    c, err = pc.remez(lambda x: x ** (n + 1), -1.0, 1.0, n)
    assert abs(err - 2.0 ** -n) <= 1e-6 * 2.0 ** -n  # the exchange works on a grid of 100001 points
    want = np.zeros(n + 2)
    want[n + 1] = -2.0 ** -n
    want = cheb.chebsub(cheb.poly2cheb(np.eye(n + 2)[n + 1]), want)[:n + 1]
    assert np.abs(c - want).max() < 1e-7


@pytest.mark.parametrize("lo,hi,deg", RANGES)
def test_remez_equioscillates_on_silu(lo, hi, deg):
    c, err = pc.remez(pc.silu, lo, hi, deg)
    x = np.linspace(-1.0, 1.0, 200001)
    e = pc.silu(lo + (x + 1.0) * (hi - lo) / 2.0) - cheb.chebval(x, c)
    assert abs(np.abs(e).max() - err) <= 2e-5 * err
    # deg + 2 alternating extrema of (almost) equal magnitude
    s = np.sign(e)
    runs = np.split(np.arange(len(x)), np.flatnonzero(np.diff(s) != 0) + 1)
    peaks = np.array([np.abs(e[r]).max() for r in runs])
    assert len(runs) >= deg + 2
    assert (peaks[np.argsort(peaks)[-(deg + 2):]] >= err * (1 - 1e-4)).all()


def test_ols_is_the_unweighted_chebyshev_fit():
    lo, hi, deg = RANGES[0]
    x = np.linspace(lo, hi, 4001)
    want = cheb.chebfit((2 * x - (lo + hi)) / (hi - lo), pc.silu(x), deg)
    assert np.abs(pc.fit_silu_ols(lo, hi, deg) - want).max() < 1e-9


@pytest.mark.parametrize("lo,hi,deg", RANGES)
def test_each_fit_wins_its_own_measure(lo, hi, deg):
    mu, sd = (lo + hi) / 2, (hi - lo) / 10
    samples = np.random.default_rng(0).normal(mu, sd, 100000)
    r = pc.silu_fit_comparison(lo, hi, deg, samples)
    assert r["ols"]["rmse_uniform"] <= min(r["wls"]["rmse_uniform"], r["remez"]["rmse_uniform"])
    assert r["remez"]["max_err"] <= min(r["wls"]["max_err"], r["ols"]["max_err"]) * (1 + 1e-9)
    # the weighted objective on the uniform samples
    x = np.linspace(lo, hi, 4001)
    w = np.where(np.abs(x - samples.mean()) <= 3 * samples.std(), 10.0, 1.0)
    u = (2 * x - (lo + hi)) / (hi - lo)
    obj = {m: float(np.sum(w * (cheb.chebval(u, c) - pc.silu(x)) ** 2)) for m, c in
           (("wls", pc.fit_silu(lo, hi, deg, samples.mean(), samples.std())), ("ols", pc.fit_silu_ols(lo, hi, deg)),
            ("remez", pc.fit_silu_remez(lo, hi, deg)))}
    assert obj["wls"] <= min(obj["ols"], obj["remez"])
    # where the data is dense the weighted fit is the closest of the three
    assert r["wls"]["rmse_data"] <= min(r["ols"]["rmse_data"], r["remez"]["rmse_data"])
