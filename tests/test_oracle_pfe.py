"""Pins of the Neuberger partial-fraction coefficients (Eq. (1.2), Fig. 1).

The closed form is independent of the pole/weight formulas:
  sqrt(x) sum_s w_s/(x + sigma_s)
      = [(1+sqrt x)^{2N} - (1-sqrt x)^{2N}] / [(1+sqrt x)^{2N} + (1-sqrt x)^{2N}].
"""
import json
import os

import numpy as np
import pytest

from oracle import pfe


def closed_form(x, n):
    r = np.sqrt(x)
    a, b = (1 + r) ** (2 * n), (1 - r) ** (2 * n)
    return (a - b) / (a + b)


@pytest.mark.parametrize("n", [1, 2, 10, 20, 30, 58])
def test_closed_form(n):
    sigma, w = pfe.neuberger(n)
    x = np.logspace(-4, 2, 301)
    lhs = np.sqrt(x) * pfe.pfe_scalar(x, sigma, w)
    assert np.allclose(lhs, closed_form(x, n), rtol=1e-13, atol=0)


@pytest.mark.parametrize("n", [10, 30, 58])
def test_unit_point_and_inversion_symmetry(n):
    sigma, w = pfe.neuberger(n)
    assert abs(pfe.pfe_scalar(1.0, sigma, w) - 1.0) < 1e-14
    x = np.logspace(-3, 0, 50)
    r1 = np.sqrt(x) * pfe.pfe_scalar(x, sigma, w)
    r2 = np.sqrt(1 / x) * pfe.pfe_scalar(1 / x, sigma, w)
    assert np.allclose(r1, r2, rtol=1e-13)
    assert np.all(sigma > 0) and np.all(w > 0) and np.all(np.diff(sigma) > 0)


def test_one_pole_is_two_over_one_plus_x():
    # N = 1: theta = pi/4, sigma = 1, w = 2
    sigma, w = pfe.neuberger(1)
    assert np.allclose(sigma, [1.0]) and np.allclose(w, [2.0])


def test_accuracy_grows_with_poles_as_fig1():
    """More poles, smaller error of x^{-1/2} on a fixed spectral window; the
    paper's 10 -> 1e-2 and 58 -> 1e-10 (Fig. 1 caption) hold on [1e-2, 1]."""
    facts = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_facts.json")))
    x = np.logspace(-2, 0, 2001)
    errs = {}
    for n in (10, 20, 30, 58):
        sigma, w = pfe.neuberger(n)
        errs[n] = np.max(np.abs(np.sqrt(x) * pfe.pfe_scalar(x, sigma, w) - 1.0))
    assert errs[10] > errs[20] > errs[30] > errs[58]
    for p in facts["pfe_accuracy"]["points"]:
        assert errs[p["n_shift"]] < 5 * p["accuracy"]
