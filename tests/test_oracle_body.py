"""Pins of body geometry, rigid motion, measure and force integrals."""
import math

import numpy as np
import pytest

import wlsynth
from oracle import Grid
from oracle.body import cell_points, face_points, forces, measure, sdf_normal_velocity


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


@pytest.mark.parametrize("comp", [0, 1])
def test_forces_viscous_quadratic_shear_on_circle(comp):
    # u_comp = (other coordinate)^2: S has one off-diagonal entry equal to that
    # coordinate, whose divergence is the unit vector e_comp, so by the divergence
    # theorem F_v = 2 nu (area) e_comp (central differences are exact on a quadratic)
    R, nu = 8.0, 0.3
    g = Grid((48, 48))
    b = wlsynth.Body("sphere", center=(24.2, 23.7), radius=R)
    other = 1 - comp
    u = [np.zeros(g.shape), np.zeros(g.shape)]
    X = face_points(g, comp)
    u[comp] = (X[other] - b.center[other]) ** 2
    _, Fv = forces(g, b, 0.0, u, np.zeros(g.shape), nu=nu)
    expect = np.zeros(2)
    expect[comp] = 2 * nu * math.pi * R * R
    assert abs(Fv[comp] - expect[comp]) < 1e-2 * expect[comp]
    assert abs(Fv[other]) < 1e-3 * expect[comp]


def test_forces_viscous_quadratic_shear_on_sphere():
    R, nu = 7.0, 0.2
    g = Grid((32, 32, 32))
    b = wlsynth.Body("sphere", center=(16.1, 15.8, 16.3), radius=R)
    X = face_points(g, 0)
    u = [(X[1] - b.center[1]) ** 2, np.zeros(g.shape), np.zeros(g.shape)]
    _, Fv = forces(g, b, 0.0, u, np.zeros(g.shape), nu=nu)
    expect = 2 * nu * 4.0 / 3.0 * math.pi * R ** 3
    assert abs(Fv[0] - expect) < 1e-2 * expect
    assert np.abs(Fv[1:]).max() < 1e-3 * expect


def test_translating_body_motion():
    b = wlsynth.Body("sphere", center=(10.0, 8.0), radius=2.0, velocity=(0.7, -0.2))
    assert b.moving
    X = [np.array([12.0, 10.0]), np.array([8.0, 8.5])]
    t = 3.0
    d, _, V = sdf_normal_velocity(b, X, t)
    c = (10.0 + 0.7 * t, 8.0 - 0.2 * t)
    np.testing.assert_allclose(d, np.hypot(X[0] - c[0], X[1] - c[1]) - 2.0, atol=1e-14)
    np.testing.assert_array_equal(V[0], 0.7)
    np.testing.assert_array_equal(V[1], -0.2)


# ---------------------------------------------------------------------------
# gridded signed distance
# ---------------------------------------------------------------------------
def _plane_body(ndim, normal, offset, h=0.7, pitch=0.0):
    nrm = np.asarray(normal, dtype=np.float64)
    nrm = nrm / np.linalg.norm(nrm)
    sdf, origin = wlsynth.sampled_sdf(lambda X: sum(nrm[k] * X[k] for k in range(ndim)) - offset, 6.0, h, ndim)
    ctr = (20.0, 20.0, 20.0)[:ndim]
    return wlsynth.Body("grid", center=ctr, sdf_grid=sdf, grid_origin=origin, grid_h=h, pitch_amp=pitch,
                        phase_p=math.pi / 2), nrm


@pytest.mark.parametrize("ndim", [2, 3])
def test_grid_sdf_exact_on_a_linear_field(ndim):
    # multilinear interpolation and central/one-sided differences are exact on a
    # linear function: d and n equal the plane's at any point of the sampled box
    normal = (0.3, -0.8, 0.52)[:ndim]
    b, nrm = _plane_body(ndim, normal, 0.4)
    rng = np.random.default_rng(5)
    Xb = [rng.uniform(-5.9, 5.9, 500) for _ in range(ndim)]
    X = [Xb[k] + b.center[k] for k in range(ndim)]
    d, n, V = sdf_normal_velocity(b, X, 0.0)
    np.testing.assert_allclose(d, sum(nrm[k] * Xb[k] for k in range(ndim)) - 0.4, atol=1e-12)
    for k in range(ndim):
        np.testing.assert_allclose(n[k], nrm[k], atol=1e-12)
        assert np.all(V[k] == 0.0)


def test_grid_sdf_rotated_normal_follows_the_body():
    b, nrm = _plane_body(2, (1.0, 0.0), 0.0, pitch=0.5)
    X = [np.array([20.5, 21.0]), np.array([20.2, 19.1])]
    d, n, _ = sdf_normal_velocity(b, X, 0.0)
    np.testing.assert_allclose(n[0], math.cos(0.5), atol=1e-12)
    np.testing.assert_allclose(n[1], math.sin(0.5), atol=1e-12)


def test_grid_sdf_interpolates_the_samples_and_is_fluid_outside():
    rng = np.random.default_rng(2)
    sdf = rng.normal(size=(5, 6, 4))
    b = wlsynth.Body("grid", center=(0.0, 0.0, 0.0), sdf_grid=sdf, grid_origin=(1.0, 2.0, 3.0), grid_h=0.5)
    I = np.array([0, 4, 2, 3]), np.array([0, 5, 1, 4]), np.array([0, 3, 2, 1])
    X = [1.0 + 0.5 * I[0], 2.0 + 0.5 * I[1], 3.0 + 0.5 * I[2]]
    d, _, _ = sdf_normal_velocity(b, X, 0.0)
    np.testing.assert_allclose(d, sdf[I], atol=1e-14)
    d, n, _ = sdf_normal_velocity(b, [np.array([0.9]), np.array([3.0]), np.array([4.0])], 0.0)
    assert np.isinf(d[0]) and d[0] > 0


def test_grid_sdf_sampled_velocity_adds_to_the_rigid_one():
    sdf, origin = wlsynth.sampled_sdf(lambda X: np.hypot(X[0], X[1]) - 3.0, 6.0, 0.5, 2)
    vg = np.stack([np.full(sdf.shape, 0.25), np.full(sdf.shape, -0.5)])
    b = wlsynth.Body("grid", center=(10.0, 10.0), sdf_grid=sdf, vel_grid=vg, grid_origin=origin, grid_h=0.5,
                     velocity=(1.0, 0.0))
    _, _, V = sdf_normal_velocity(b, [np.array([11.0]), np.array([9.0])], 0.0)
    np.testing.assert_allclose([V[0][0], V[1][0]], [1.25, -0.5], atol=1e-15)


@pytest.mark.parametrize("ndim", [2, 3])
def test_grid_sdf_sphere_moments_converge_second_order(ndim):
    # the sampled sphere reproduces the analytic sphere's mu0, mu1 and V with an
    # O(h^2) error: halving the sample spacing cuts it by about 4
    R = 6.0
    n = (32, 32) if ndim == 2 else (24, 24, 24)
    ctr = (16.3, 15.6, 12.2)[:ndim] if ndim == 2 else (12.3, 11.6, 12.2)
    g = Grid(n)
    ref = wlsynth.Body("sphere", center=ctr, radius=R, spin_omega=0.05)
    m0r, m1r, Vr = measure(g, ref, 0.0)
    # V is cut off at d = 2 + eps: faces within 0.1 of the cut may fall on either side
    keep = []
    for i in range(ndim):
        d, _, _ = sdf_normal_velocity(ref, face_points(g, i), 0.0)
        keep.append(np.abs(d - 3.0) > 0.1)
    errs = []
    for h in (0.8, 0.4):
        gb = wlsynth.grid_sphere_body(R, h, ndim, ctr, spin_omega=0.05)
        m0, m1, V = measure(g, gb, 0.0)
        e = 0.0
        for i in range(ndim):
            e = max(e, float(np.max(np.abs(m0[i] - m0r[i]))))
            for j in range(ndim):
                e = max(e, float(np.max(np.abs(m1[i][j] - m1r[i][j]))))
            e = max(e, float(np.max(np.abs(V[i] - Vr[i])[keep[i]])))
        errs.append(e)
    assert errs[1] < 1e-2
    assert errs[0] / errs[1] > 3.0, errs
