"""Pins of body geometry, rigid motion, measure and force integrals."""
import math

import numpy as np
import pytest

import wlsynth
from oracle import Grid
from oracle.body import cell_points, forces, measure, sdf_normal_velocity


def test_box_sdf_known_points():
    b = wlsynth.Body("box", center=(0.0, 0.0), half_extent=(2.0, 1.0))
    X = [np.array([3.0, 3.0, 0.0, 1.5, -2.5]), np.array([0.0, 2.0, 0.0, 0.2, -1.0])]
    d, n, _ = sdf_normal_velocity(b, X, 0.0)
    np.testing.assert_allclose(d, [1.0, math.sqrt(2.0), -1.0, -0.5, 0.5], atol=1e-15)
    np.testing.assert_allclose(n[0], [1.0, 1 / math.sqrt(2), 0.0, 1.0, -1.0], atol=1e-15)
    np.testing.assert_allclose(n[1], [0.0, 1 / math.sqrt(2), 1.0, 0.0, 0.0], atol=1e-15)


def test_sphere_sdf_and_unit_normal():
    b = wlsynth.Body("sphere", center=(1.0, 2.0, 3.0), radius=2.0)
    rng = np.random.default_rng(0)
    X = [rng.uniform(-5, 5, 200) for _ in range(3)]
    d, n, V = sdf_normal_velocity(b, X, 0.0)
    r = np.sqrt((X[0] - 1) ** 2 + (X[1] - 2) ** 2 + (X[2] - 3) ** 2)
    np.testing.assert_allclose(d, r - 2.0, atol=1e-14)
    np.testing.assert_allclose(n[0] ** 2 + n[1] ** 2 + n[2] ** 2, 1.0, atol=1e-14)
    for v in V:
        assert np.all(v == 0.0)


@pytest.mark.parametrize("kind", ["sphere", "box"])
def test_rigid_velocity_transports_the_sdf(kind):
    # for rigid motion d(x, t) is advected: dd/dt + V . grad d = 0 (FD in time and space)
    b = wlsynth.Body(kind, center=(10.0, 8.0), radius=3.0, half_extent=(4.0, 1.0),
                     heave_amp=2.0, pitch_amp=0.4, freq=0.05, phase_h=0.3, phase_p=1.9,
                     pivot_offset=(-1.5, 0.0), spin_omega=0.02)
    rng = np.random.default_rng(3)
    X = [rng.uniform(4, 16, 400), rng.uniform(3, 13, 400)]
    t, h = 3.7, 1e-5
    d, n, V = sdf_normal_velocity(b, X, t)
    dp, _, _ = sdf_normal_velocity(b, X, t + h)
    dm, _, _ = sdf_normal_velocity(b, X, t - h)
    ddt = (dp - dm) / (2 * h)
    # keep points away from kinks of the box SDF
    grad = []
    for k in range(2):
        Xp = [x.copy() for x in X]
        Xm = [x.copy() for x in X]
        Xp[k] += h
        Xm[k] -= h
        grad.append((sdf_normal_velocity(b, Xp, t)[0] - sdf_normal_velocity(b, Xm, t)[0]) / (2 * h))
    smooth = np.abs(grad[0] - n[0]) + np.abs(grad[1] - n[1]) < 1e-6
    assert smooth.sum() > 200
    res = ddt + V[0] * n[0] + V[1] * n[1]
    assert np.abs(res[smooth]).max() < 1e-6


def test_mu0_volume_fraction_matches_area():
    R = 8.0
    g = Grid((48, 48))
    b = wlsynth.Body("sphere", center=(24.3, 23.8), radius=R)
    m0, m1, V = measure(g, b, 0.0)
    for i in range(2):
        solid = np.sum(1.0 - m0[i][g.interior()])
        assert solid == pytest.approx(math.pi * R * R, rel=5e-3)


def test_forces_linear_pressure_on_circle():
    R = 8.0
    g = Grid((48, 48))
    b = wlsynth.Body("sphere", center=(24.0, 24.0), radius=R)
    X = cell_points(g)
    G = (0.3, -0.7)
    p = G[0] * X[0] + G[1] * X[1]
    u = [np.full(g.shape, 1.0), np.zeros(g.shape)]
    Fp, Fv = forces(g, b, 0.0, u, p, nu=0.1)
    # -closed surface integral of p n = -(grad p) * area
    np.testing.assert_allclose(Fp, [-G[0] * math.pi * R * R, -G[1] * math.pi * R * R], rtol=1e-2)
    assert np.abs(Fv).max() < 1e-12
    Fp0, _ = forces(g, b, 0.0, u, np.full(g.shape, 5.0), nu=0.1)
    assert np.abs(Fp0).max() < 1e-10 * 5.0 * 2 * math.pi * R


def test_forces_viscous_constant_strain_integrates_to_zero():
    g = Grid((40, 40))
    b = wlsynth.Body("sphere", center=(20.0, 20.0), radius=6.0)
    y = np.arange(42) - 0.5
    u = [np.tile(0.2 * y, (42, 1)), np.zeros(g.shape)]
    _, Fv = forces(g, b, 0.0, u, np.zeros(g.shape), nu=0.5)
    assert np.abs(Fv).max() < 1e-12
