"""Pins for risk-aware stopping and the ||A||_F denominator (CPU only).

The Corollary of §3.3: with G having independent N(0, 1/c) entries and
xi = (1 + delta) sqrt(1 - 2 sqrt(-ln(alpha) / c)),
P[ ||G(A - CUR)||_F / ||A||_F < xi eps  and  ||A - CUR||_F / ||A||_F > (1 + delta) eps ] <= alpha.
The oracle's Gaussian G has unit variance, so the estimate the Corollary bounds is
rho_A = ||S^col||_F / (sqrt(c) ||A||_F) (the denominator the §5 footnote mentions).
"""
import math

import numpy as np
import pytest

from oracle.icur import exact_relative_error, iterative_cur, risk_aware_factor
from oracle.rng import g_scale
from paper_2509_21963_amd import workloads as W


@pytest.mark.parametrize("kind", [0, 1, 2])
def test_denominator_a_is_the_rescaled_estimate(kind):
    # the denominator changes only when the loop stops: with a fixed rank both runs pick
    # the same indices and the estimates differ by the closed-form factor
    A, _ = W.planted_geometric(300, 200, 20.0, seed=1)
    ga = iterative_cur(A, 1e-300, 10, kind=kind, seed=2, max_rank=40)
    a = iterative_cur(A, 1e-300, 10, kind=kind, seed=2, max_rank=40, denominator="A")
    assert ga["I"] == a["I"] and ga["J"] == a["J"]
    c = 11
    factor = np.linalg.norm(ga["X0"]) / (g_scale(kind, c) * np.linalg.norm(A))
    assert a["rho"] == pytest.approx(ga["rho"] * factor, rel=1e-12)
    # before any index is chosen rho_A = ||G A||_F / (s ||A||_F): near 1, since
    # E ||G x||^2 = s^2 ||x||^2 and ||G A||_F^2 sums c n such terms
    first = iterative_cur(A, 10.0, 10, kind=kind, seed=2, denominator="A")
    assert first["rank"] == 0 and first["rho"] == pytest.approx(factor, rel=1e-12)
    assert 0.7 < factor < 1.4


def _failures(A, tol, b, alpha, n_runs):
    bad = 0
    for s in range(n_runs):
        o = iterative_cur(A, tol, b, seed=s, alpha=alpha, denominator="A")
        bad += exact_relative_error(A, o["I"], o["J"], o["U"]) > tol
    return bad


def test_corollary_failure_rate():
    # a spectrum that decays slowly per block, so the estimate crosses tol close to the
    # true error: without the adjustment the estimator alone misses now and then
    # (7 of 60 runs here), with xi (alpha = 0.1, c = 22, xi = 0.5941) the rate of
    # stopping with a true error above tol stays within the Corollary's alpha
    A = W.planted(300, 200, 10.0 ** (-np.arange(200) / 60.0), 0)
    n_runs, tol, alpha = 60, 0.05, 0.1
    assert risk_aware_factor(alpha, 0.0, 22) == pytest.approx(0.5941, abs=1e-4)
    plain = _failures(A, tol, 20, 0.0, n_runs)
    adjusted = _failures(A, tol, 20, alpha, n_runs)
    assert plain >= 3
    assert adjusted <= alpha * n_runs + 3 * math.sqrt(n_runs * alpha * (1 - alpha))


def test_risk_aware_stopping_is_for_the_gaussian_sketch_only():
    A = np.random.default_rng(0).standard_normal((50, 40))
    for kind in (1, 2):
        with pytest.raises(ValueError):
            iterative_cur(A, 1e-2, 10, kind=kind, alpha=0.2)
    iterative_cur(A, 1e-2, 10, kind=0, alpha=0.2)
