"""Pins of the BDIM blend's first-moment term and of the body velocity term.

Near a planar wall the convolution the BDIM meta-equation is built from can be
evaluated directly: with V = 0 and a fluid update that is linear in the signed
distance, f~ = G d, the kernel-weighted average over the fluid side is

    int K_eps(t) G (d - t) H(d - t) dt,

which the blend must reproduce exactly (central differences are exact on a
linear field).  The integral is taken by adaptive quadrature here, independent
of the closed-form moments, so a sign, a factor, n_i in place of n_j, or a
one-sided gradient in the mu1 term fails it.
"""
import math

import numpy as np
import pytest
from scipy.integrate import quad

import wlsynth
from oracle import Grid
from oracle.body import face_points, measure, sdf_normal_velocity
from oracle.moments import kernel_eps
from oracle.solver import bdim


def _exact_convolution(d, G, eps):
    if d <= -eps:
        return 0.0
    top = min(d, eps)
    val, _ = quad(lambda t: kernel_eps(t, eps) * G * (d - t), -eps, top, epsabs=1e-15, epsrel=1e-13,
                  limit=200)
    if d > eps:  # the kernel vanishes beyond eps: the rest of the integral is 0
        pass
    return float(val)


@pytest.mark.parametrize("theta", [0.0, math.pi / 2, 0.61])
@pytest.mark.parametrize("eps", [1.0, 1.5])
def test_bdim_planar_wall_equals_exact_convolution(theta, eps):
    g = Grid((40, 40))
    # a thick box rotated by theta: near its +x face the signed distance is that
    # plane's (the other faces are far from the tested band)
    b = wlsynth.Body("box", center=(9.3, 20.2), half_extent=(13.0, 200.0), pitch_amp=theta,
                     phase_p=math.pi / 2)
    G = (0.7, -1.3)
    m0, m1, V = measure(g, b, 0.0, eps)
    ft, dist = [], []
    for i in range(2):
        X = face_points(g, i)
        d, n, _ = sdf_normal_velocity(b, X, 0.0)
        dist.append(d)
        ft.append(G[i] * d)
    zero = [np.zeros(g.shape)] * 2
    out = bdim(g, ft, zero, m0, m1)
    tested = 0
    for i in range(2):
        for I0 in range(2, 39):
            for I1 in range(2, 39):
                d = float(dist[i][I0, I1])
                if abs(d) >= eps + 0.5 or (m0[i][I0, I1] == 0.0 and d > -eps):
                    continue  # outside the band, or a face the solid cut zeroed
                ref = _exact_convolution(d, G[i], eps)
                assert abs(out[i][I0, I1] - ref) <= 1e-12 * (1.0 + abs(G[i] * d)), (i, I0, I1, d)
                if abs(d) < eps:
                    tested += 1
    assert tested >= 40


def test_bdim_mu1_term_is_needed_for_the_wall():
    # the same wall without the first moment misses the convolution by O(mu1 G):
    # the pin above is sensitive to that term
    g = Grid((40, 40))
    b = wlsynth.Body("box", center=(9.3, 20.2), half_extent=(13.0, 200.0))
    m0, m1, _ = measure(g, b, 0.0)
    X = face_points(g, 1)
    d, _, _ = sdf_normal_velocity(b, X, 0.0)
    ft = [np.zeros(g.shape), 1.0 * d]
    zero = [np.zeros(g.shape)] * 2
    with_m1 = bdim(g, ft, zero, m0, m1)[1]
    no_m1 = bdim(g, ft, zero, m0, [[np.zeros(g.shape)] * 2] * 2)[1]
    band = (np.abs(d) < 0.9) & (np.asarray(m0[1]) > 0)
    assert np.max(np.abs(with_m1[band] - no_m1[band])) > 0.05
