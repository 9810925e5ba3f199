"""Pins of the Taylor-Green vortex on its symmetric subdomain (paper, performance
section: the benchmark runs on one eighth of the triple-periodic box with
symmetry conditions).  Symmetry planes are the slip faces with U = 0: the normal
face velocity is 0 and tangential ghosts mirror the interior."""
import math

import numpy as np
import pytest

import wlsynth
from oracle import Sim


def _run(w, amp, steps, dt, periodic, u0=None):
    s = Sim(w.n, w.U, w.nu, periodic=periodic, tol=1e-14 * amp, itmax=64)
    s.set_velocity([amp * a for a in (u0 if u0 is not None else wlsynth.initial_velocity(w))])
    for _ in range(steps):
        s.dt = dt
        s.step()
    return s


def test_symmetric_subdomain_equals_the_periodic_box_in_the_linear_limit():
    # At a tiny amplitude convection is negligible (its effect is amp / (nu kappa)
    # relative), and diffusion and projection on the octant with mirror conditions
    # reproduce the periodic box of twice the side restricted to that octant.
    N = 8
    half = wlsynth.tgv_sym_3d(N=N, Re=100.0)
    full = wlsynth.Workload("tgv_full", (2 * N,) * 3, (0.0, 0.0, 0.0), half.nu, periodic=(True,) * 3,
                            noise=0.0, init="tgv")
    # the same mode sampled on the full box: k = pi / N there as well
    k = math.pi / N
    u0 = []
    for i in range(3):
        X = wlsynth.face_coords(full.n, i)
        if i == 0:
            f = -np.sin(k * X[0]) * np.cos(k * X[1]) * np.cos(k * X[2])
        elif i == 1:
            f = np.cos(k * X[0]) * np.sin(k * X[1]) * np.cos(k * X[2])
        else:
            f = np.zeros(X[0].shape)
        u0.append(f)
    amp = 1e-10
    a = _run(half, amp, 5, 0.4, (False,) * 3)
    b = _run(full, amp, 5, 0.4, (True,) * 3, u0=u0)
    # the octant of the full box: faces 0..N+1 of the half grid are faces 0..N+1 there
    for i in range(3):
        ref = b.u[i][: N + 2, : N + 2, : N + 2]
        got = a.u[i]
        inner = tuple(slice(1, N + 1) for _ in range(3))
        scale = float(np.max(np.abs(ref[inner])))
        if i < 2:
            assert scale > 0.5 * amp
            np.testing.assert_allclose(got[inner], ref[inner], rtol=0, atol=1e-7 * scale)
        else:
            assert float(np.max(np.abs(got[inner]))) < 1e-6 * amp
    # and the flow really decayed: the comparison is not of the initial field
    assert float(np.max(np.abs(a.u[0]))) < 0.97 * amp


def test_symmetric_subdomain_early_decay_rate():
    # ln E_nu - ln E_2nu = 2 nu lam_h t with lam_h = 12 sin^2(kappa/2): a cell-centred
    # cosine under mirror conditions and a face-centred sine under zero normal
    # velocity are exact eigenvectors of the discrete Laplacian, as in the periodic box
    N = 16
    k = math.pi / N
    lam = 12 * math.sin(k / 2) ** 2
    out = {}
    for Re in (40.0, 20.0):
        w = wlsynth.tgv_sym_3d(N=N, Re=Re)
        s = Sim(w.n, w.U, w.nu, periodic=(False,) * 3, tol=1e-11, itmax=64)
        s.set_velocity(wlsynth.initial_velocity(w))
        E0 = s.ke()
        T = 0.5 / k
        while s.t < T - 1e-12:
            s.dt = min(0.25, T - s.t)
            s.step()
        out[Re] = (math.log(s.ke() / E0), s.t, w.nu)
    nu = out[40.0][2]
    assert out[20.0][2] == pytest.approx(2 * nu)
    d = out[40.0][0] - out[20.0][0]
    assert d == pytest.approx(2 * nu * lam * out[40.0][1], rel=0.02)


def test_symmetric_tgv_initial_field_is_discretely_divergence_free():
    from oracle.poisson import divergence
    w = wlsynth.tgv_sym_3d(N=12)
    s = Sim(w.n, w.U, w.nu, periodic=(False,) * 3)
    s.set_velocity(wlsynth.initial_velocity(w))
    z = divergence(s.grid, s.u)
    assert float(np.max(np.abs(z))) < 1e-14
    # the normal velocity vanishes on every symmetry plane
    N = w.n[0]
    for i in range(3):
        sl = [slice(None)] * 3
        for idx in (1, N + 1):
            sl[i] = idx
            assert float(np.max(np.abs(s.u[i][tuple(sl)]))) < 1e-15
