"""Pins of the limited QUICK face value and the convection-diffusion residual."""
import itertools

import numpy as np
import pytest

import wlsynth
from oracle import Grid
from oracle.flux import conv_diff, quick_limited


# ---------------------------------------------------------------- limiter
def test_limiter_exact_on_linear_data():
    rng = np.random.default_rng(1)
    c = rng.normal(size=100)
    a = rng.normal(size=100)
    # u_far = c - a, d = c + a  =>  face value c + a/2
    np.testing.assert_allclose(quick_limited(c - a, c, c + a), c + a / 2, atol=1e-14)


def test_limiter_bounded_and_odd():
    rng = np.random.default_rng(2)
    far, c, d = rng.normal(size=(3, 10000))
    q = quick_limited(far, c, d)
    lo, hi = np.minimum(c, d), np.maximum(c, d)
    assert np.all(q >= lo - 1e-15) and np.all(q <= hi + 1e-15)
    np.testing.assert_array_equal(quick_limited(-far, -c, -d), -q)


def test_limiter_upwind_at_extremum():
    # c is a local maximum -> first-order upwind value c
    far = np.array([0.0, 1.0, -2.0])
    c = np.array([1.0, 3.0, 0.5])
    d = np.array([0.5, 2.0, -1.0])
    np.testing.assert_array_equal(quick_limited(far, c, d), c)


# ------------------------------------------------------------- residual
def _brute_R(n, periodic, u, nu):
    """Pure-Python loops over faces, written from the flux definition."""
    nd = len(n)
    shape = tuple(N + 2 for N in n)

    def get(a, I):
        J = list(I)
        for k in range(nd):
            if periodic[k]:
                J[k] = 1 + (J[k] - 1) % n[k]
            elif not 0 <= J[k] <= n[k] + 1:
                return None
        return float(a[tuple(J)])

    def off(I, k, s):
        J = list(I)
        J[k] += s
        return tuple(J)

    def inside(I, i, j):
        # far point must be a domain value along j (no ghost), see the flux docstring
        if periodic[j]:
            return True
        top = n[j] + 1 if j == i else n[j]
        return 1 <= I[j] <= top

    def med(x, y, z):
        return sorted([x, y, z])[1]

    def phi(i, j, I):
        adv = 0.5 * (get(u[j], I) + get(u[j], off(I, i, -1)))
        fI = off(I, j, -2) if adv >= 0 else off(I, j, +1)
        if adv >= 0:
            far, c, d = get(u[i], fI), get(u[i], off(I, j, -1)), get(u[i], I)
        else:
            far, c, d = get(u[i], fI), get(u[i], I), get(u[i], off(I, j, -1))
        if far is None or not inside(fI, i, j):
            Q = 0.5 * (get(u[i], I) + get(u[i], off(I, j, -1)))
        else:
            Q = med(c, (5 * c + 2 * d - far) / 6, med(c, d, 10 * c - 9 * far))
        return adv * Q - nu * (get(u[i], I) - get(u[i], off(I, j, -1)))

    R = [np.zeros(shape) for _ in range(nd)]
    for i in range(nd):
        ranges = []
        for k in range(nd):
            lo = 2 if (k == i and not periodic[k]) else 1
            ranges.append(range(lo, n[k] + 1))
        for I in itertools.product(*ranges):
            R[i][I] = sum(phi(i, j, I) - phi(i, j, off(I, j, +1)) for j in range(nd))
    return R


@pytest.mark.parametrize("n,per", [((7, 6), (False, False)), ((6, 5), (True, False)),
                                   ((5, 4, 4), (False, True, False)), ((4, 4, 5), (True, True, True))])
def test_residual_matches_brute_force(n, per):
    g = Grid(n, per)
    u = [wlsynth.random_field(g.shape, seed=11, comp=i) + (0.3 if i == 0 else -0.1)
         for i in range(len(n))]
    nu = 0.07
    R = conv_diff(g, u, nu)
    Rb = _brute_R(n, per, u, nu)
    for i in range(len(n)):
        np.testing.assert_allclose(R[i], Rb[i], atol=1e-13, rtol=0)


@pytest.mark.parametrize("per", [(False, False, False), (True, True, True)])
def test_uniform_field_has_zero_residual(per):
    g = Grid((8, 6, 4), per)
    u = [np.full(g.shape, v) for v in (0.7, -0.2, 0.1)]
    for R in conv_diff(g, u, 0.05):
        assert np.all(R == 0.0)


def test_periodic_momentum_conservation():
    g = Grid((8, 8, 8), (True, True, True))
    u = [wlsynth.random_field(g.shape, seed=3, comp=i) for i in range(3)]
    for R in conv_diff(g, u, 0.1):
        assert abs(R[g.interior()].sum()) < 1e-12


def test_couette_shear_is_steady():
    # u_x = y (linear shear), v = 0: an exact steady solution -> R = 0 away from walls
    g = Grid((8, 10), (True, False))
    y = np.arange(12) - 0.5
    u = [np.tile(y, (10, 1)), np.zeros(g.shape)]
    R = conv_diff(g, u, 0.3)
    assert np.abs(R[0][1:9, 2:10]).max() < 1e-13
    assert np.abs(R[1]).max() == 0.0
