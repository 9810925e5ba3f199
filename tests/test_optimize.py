"""Pins of the Davidon cubic-interpolation search (host logic, no GPU)."""
import math

import pytest

from paper_2407_16032_amd.optimize import cubic_step, davidon_maximize, davidon_minimize


def test_cubic_step_is_exact_for_a_cubic():
    # f = (x - 1.3)^2 (x + 4): its interpolant is itself, so one step lands on 1.3
    f = lambda x: (x - 1.3) ** 2 * (x + 4.0)
    g = lambda x: 2 * (x - 1.3) * (x + 4.0) + (x - 1.3) ** 2
    x = cubic_step(0.0, f(0.0), g(0.0), 3.0, f(3.0), g(3.0))
    assert x == pytest.approx(1.3, abs=1e-12)
    # and for a quadratic (vanishing cubic term)
    f2 = lambda x: (x - 0.7) ** 2
    g2 = lambda x: 2 * (x - 0.7)
    assert cubic_step(-1.0, f2(-1.0), g2(-1.0), 2.0, f2(2.0), g2(2.0)) == pytest.approx(0.7, abs=1e-12)


def test_minimum_of_cosine():
    out = davidon_minimize(lambda x: (math.cos(x), -math.sin(x)), 2.0, 4.5, tol=1e-10, gtol=1e-12)
    assert out["x"] == pytest.approx(math.pi, abs=1e-9)
    assert len(out["evaluations"]) <= 10


def test_quartic_and_bracket_shrinks():
    c = 0.1
    xs = 2.0 - (c / 4.0) ** (1.0 / 3.0)
    out = davidon_minimize(lambda x: ((x - 2.0) ** 4 + c * x, 4 * (x - 2.0) ** 3 + c), 0.0, 5.0, tol=1e-8,
                           maxit=60)
    assert out["x"] == pytest.approx(xs, abs=1e-6)
    a, b = out["bracket"]
    assert a <= xs <= b


def test_maximize_and_bad_bracket():
    out = davidon_maximize(lambda x: (-(x - 6.26) ** 2 + 0.05 * (x - 6.26) ** 3, -2 * (x - 6.26)
                                      + 0.15 * (x - 6.26) ** 2), 3.0, 8.0, tol=1e-9)
    assert out["x"] == pytest.approx(6.26, abs=1e-7)
    with pytest.raises(ValueError):
        davidon_minimize(lambda x: (x * x, 2 * x), 1.0, 2.0)
