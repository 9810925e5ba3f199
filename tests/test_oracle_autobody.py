"""Pins of the oracle's general bodies (mapped parts and signed-distance arithmetic).

The paper's AutoBody takes any signed distance and coordinate map and derives
the normal and the body velocity from their derivatives; bodies combine by the
arithmetic of signed distances (applications section: body = big + small,
sphere - plane).  These tests pin the oracle's general evaluation against
closed forms: the rigid bodies' direct formulas, an isotropically scaled
sphere, the material derivative of the map, and areas/volumes of combined
shapes."""
import math

import numpy as np
import pytest

import wlsynth
from oracle import Grid
from oracle.body import face_points, measure, part_general, part_map, sdf_normal_velocity


def _pts(ndim, lo, hi, n=400, seed=1):
    rng = np.random.default_rng(seed)
    return [rng.uniform(lo, hi, n) for _ in range(ndim)]


@pytest.mark.parametrize("kind", ["sphere", "box"])
@pytest.mark.parametrize("ndim", [2, 3])
def test_general_equals_rigid_formulas(kind, ndim):
    # a rigid map (S = 1) through the complex-step path reproduces the direct
    # closed forms of d, n and V
    b = wlsynth.Body(kind, center=(10.0, 9.0, 8.0)[:ndim], radius=3.0, half_extent=(3.0, 2.0, 2.5),
                     heave_amp=0.7, pitch_amp=0.3, freq=0.05, phase_p=0.4, spin_omega=0.02,
                     pivot_offset=(0.6, -0.3, 0.2), velocity=(0.2, -0.1, 0.05), heave_dir=(0.3, 1.0, -0.2))
    X = _pts(ndim, 4.0, 16.0)
    d, n, V = sdf_normal_velocity(b, X, 2.7)
    d2, n2, V2 = part_general(b, X, 2.7)
    np.testing.assert_allclose(d2, d, atol=1e-12)
    for k in range(ndim):
        np.testing.assert_allclose(n2[k], n[k], atol=1e-12)
        np.testing.assert_allclose(V2[k], V[k], atol=1e-12)


@pytest.mark.parametrize("ndim", [2, 3])
def test_general_box_normal_on_its_faces(ndim):
    # points exactly on a face (d = 0, between the edges) take the face normal in
    # both evaluations
    b = wlsynth.Body("box", center=(10.0, 9.0, 8.0)[:ndim], half_extent=(4.0, 3.0, 2.0))
    # on the +y face, on the +x face, the centre (the +z face in 3-D), inside
    X = [np.array([10.5, 14.0, 10.0, 7.5]), np.array([12.0, 8.5, 9.0, 9.0])]
    if ndim == 3:
        X.append(np.array([8.0, 8.0, 10.0, 8.0]))
    d, n, _ = sdf_normal_velocity(b, X, 0.0)
    d2, n2, _ = part_general(b, X, 0.0)
    np.testing.assert_array_equal(d[:2], 0.0)
    np.testing.assert_allclose(d2, d, atol=1e-15)
    for k in range(ndim):
        np.testing.assert_allclose(n2[k], n[k], atol=1e-15)
    np.testing.assert_allclose([n2[1][0], n2[0][1]], [1.0, 1.0], atol=1e-15)


def test_general_equals_rigid_formulas_grid():
    sdf, origin = wlsynth.sampled_sdf(lambda X: np.hypot(X[0], X[1]) - 3.0, 6.0, 0.5, 2)
    b = wlsynth.Body("grid", center=(10.0, 10.0), sdf_grid=sdf, grid_origin=origin, grid_h=0.5,
                     pitch_amp=0.4, freq=0.1, spin_omega=0.03)
    X = _pts(2, 5.0, 15.0)
    d, n, V = sdf_normal_velocity(b, X, 1.1)
    d2, n2, V2 = part_general(b, X, 1.1)
    fin = np.isfinite(d)
    assert fin.sum() > 100
    np.testing.assert_allclose(d2[fin], d[fin], atol=1e-12)
    assert np.all(np.isinf(d2[~fin]))
    for k in range(2):
        np.testing.assert_allclose(n2[k][fin], n[k][fin], atol=1e-12)
        np.testing.assert_allclose(V2[k], V[k], atol=1e-12)


@pytest.mark.parametrize("ndim", [2, 3])
def test_scaled_sphere_distance_and_velocity(ndim):
    # x_b = S(t) (x - P): the body is the sphere of radius R/S about P, and a
    # material point moves radially with x' = -(x - P) S'/S
    R, a, f, ph = 4.0, 0.2, 0.03, 0.3
    b = wlsynth.Body("sphere", center=(12.0, 11.0, 10.0)[:ndim], radius=R, scale_amp=(a, a, a),
                     freq=f, phase_s=ph)
    t = 3.3
    S = 1.0 + a * math.sin(2 * math.pi * f * t + ph)
    Sd = a * 2 * math.pi * f * math.cos(2 * math.pi * f * t + ph)
    X = _pts(ndim, 5.0, 18.0)
    r = [X[k] - b.center[k] for k in range(ndim)]
    rn = np.sqrt(sum(v * v for v in r))
    d, n, V = part_general(b, X, t)
    np.testing.assert_allclose(d, rn - R / S, atol=1e-12)
    for k in range(ndim):
        np.testing.assert_allclose(n[k], r[k] / rn, atol=1e-12)
        np.testing.assert_allclose(V[k], -r[k] * Sd / S, atol=1e-12)


def test_velocity_is_the_material_derivative_of_the_map():
    # the point x + V dt maps, at t + dt, to the body-frame point x maps to at t:
    # the mismatch is O(dt^2) with V and O(dt) without it
    b = wlsynth.Body("box", center=(10.0, 9.0, 8.0), half_extent=(2.0, 3.0, 1.5), heave_amp=0.8,
                     heave_dir=(0.2, 0.5, 1.0), pitch_amp=0.5, freq=0.07, phase_p=0.9, spin_omega=0.04,
                     scale_amp=(0.15, -0.1, 0.2), phase_s=0.2, velocity=(0.3, 0.1, -0.2),
                     pivot_offset=(0.4, 0.1, -0.3))
    X = _pts(3, 5.0, 15.0, n=50)
    t = 1.9
    _, _, V = part_general(b, X, t)
    x0 = part_map(b, X, t)
    errs = {}
    for dt in (1e-3, 5e-4):
        x1 = part_map(b, [X[k] + V[k] * dt for k in range(3)], t + dt)
        x1s = part_map(b, X, t + dt)
        errs[dt] = (max(np.max(np.abs(x1[k] - x0[k])) for k in range(3)),
                    max(np.max(np.abs(x1s[k] - x0[k])) for k in range(3)))
    (e1, s1), (e2, s2) = errs[1e-3], errs[5e-4]
    assert e1 / e2 > 3.5          # second order with V
    assert s1 / s2 < 2.2          # first order without it
    assert e1 < 1e-3 * s1


# second moment of the cosine kernel, int s^2 K(s) ds over [-1, 1] = 1/3 - 2/pi^2: a
# smoothed closed curve of total turning 2 pi encloses pi * M2 * eps^2 more than its
# area (integration by parts of the first moment of H(-d) - (1 - mu0(d)))
M2 = 1.0 / 3.0 - 2.0 / math.pi ** 2


def _solid_area(g, body, comp=0):
    m0, _, _ = measure(g, body, 0.0)
    inner = g.interior()
    return float(np.sum(1.0 - m0[comp][inner]))


def test_union_of_two_circles_area():
    # the fluid fraction's complement integrates to the union's area (lens formula)
    R, c = 6.0, 7.0
    g = Grid((48, 40))
    a = wlsynth.Body("sphere", center=(20.3, 19.6), radius=R)
    b = wlsynth.Body("sphere", center=(20.3 + c, 19.6), radius=R)
    u = wlsynth.combine(a, ("union", b))
    lens = 2 * R * R * math.acos(c / (2 * R)) - 0.5 * c * math.sqrt(4 * R * R - c * c)
    exact = 2 * math.pi * R * R - lens + math.pi * M2
    area = _solid_area(g, u)
    assert abs(area - exact) < 5e-4 * exact, (area, exact)
    # either part alone has the circle's area; the union is not their sum
    one = math.pi * R * R + math.pi * M2
    assert abs(_solid_area(g, a) - one) < 2e-4 * one


def test_circle_minus_half_plane_is_a_half_disk():
    R = 7.0
    g = Grid((40, 40))
    a = wlsynth.Body("sphere", center=(20.2, 19.7), radius=R)
    cut = wlsynth.Body("plane", center=(20.2, 19.7), normal=(0.0, -2.0))  # removes y < centre
    body = wlsynth.combine(a, ("subtract", cut))
    area = _solid_area(g, body)
    exact = 0.5 * math.pi * R * R + math.pi * M2
    # the convex corners add a little: max of two distances underestimates the
    # distance off a corner
    assert abs(area - exact) < 3e-3 * exact, (area, exact)
    # intersecting with the opposite half space is the same body, face for face
    keep = wlsynth.Body("plane", center=(20.2, 19.7), normal=(0.0, 2.0))
    body2 = wlsynth.combine(a, ("intersect", keep))
    for i in range(2):
        X = face_points(g, i)
        d1, n1, _ = sdf_normal_velocity(body, X, 0.0)
        d2, n2, _ = sdf_normal_velocity(body2, X, 0.0)
        np.testing.assert_allclose(d1, d2, atol=1e-13)
        for k in range(2):
            np.testing.assert_allclose(n1[k], n2[k], atol=1e-13)


def test_hollow_hemisphere_volume():
    # a shell of half thickness s about the sphere R, minus the half space below
    # its centre: (2/3) pi ((R+s)^3 - (R-s)^3)
    R, s = 7.0, 1.5
    g = Grid((24, 24, 24))
    ctr = (12.2, 11.9, 12.1)
    shell = wlsynth.Body("sphere", center=ctr, radius=R, shell=s)
    cut = wlsynth.Body("plane", center=ctr, normal=(0.0, 0.0, -1.0))
    body = wlsynth.combine(shell, ("subtract", cut))
    vol = _solid_area(g, body, comp=2)
    exact = 2.0 / 3.0 * math.pi * ((R + s) ** 3 - (R - s) ** 3)
    # smoothing of a thin curved shell with two sharp rims: a few percent at this
    # resolution (a missing shell, a union for the cut or |d| without the offset
    # would be off by 35 % to 100 %)
    assert abs(vol - exact) < 2.5e-2 * exact, (vol, exact)
    # the full shell is about twice the half
    full = _solid_area(g, shell, comp=2)
    assert abs(full - 2 * vol) < 2.5e-2 * full


def test_union_order_and_self_union():
    a = wlsynth.Body("sphere", center=(10.0, 10.0), radius=3.0, spin_omega=0.1)
    b = wlsynth.Body("box", center=(13.0, 9.0), half_extent=(2.0, 1.0), velocity=(0.2, 0.0))
    X = _pts(2, 4.0, 18.0)
    ab = sdf_normal_velocity(wlsynth.combine(a, ("union", b)), X, 0.5)
    ba = sdf_normal_velocity(wlsynth.combine(b, ("union", a)), X, 0.5)
    np.testing.assert_allclose(ab[0], ba[0], atol=1e-13)
    da, na, Va = part_general(a, X, 0.5)
    aa = sdf_normal_velocity(wlsynth.combine(a, ("union", a)), X, 0.5)
    np.testing.assert_allclose(aa[0], da, atol=1e-14)
    for k in range(2):
        np.testing.assert_allclose(aa[2][k], Va[k], atol=1e-14)
    # the winning part supplies the velocity: the box's translation where it is nearer
    nearer_b = sdf_normal_velocity(b, X, 0.5)[0] < da
    np.testing.assert_allclose(ab[2][0][nearer_b], 0.2, atol=1e-14)
    np.testing.assert_allclose(ab[2][1][nearer_b], 0.0, atol=1e-14)
