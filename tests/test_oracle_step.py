"""Pins of the full oracle step: exact solutions, invariants and special cases."""
import math

import numpy as np
import pytest

import wlsynth
from oracle import Grid, Sim
from oracle import poisson as P
from oracle.solver import apply_bc, bdim, cfl, exit_plane


def _run_tgv2d(N, Re=100.0, kut=1.0):
    k = 2 * math.pi / N
    nu = 1.0 / (k * Re)
    s = Sim((N, N), (0.0, 0.0), nu, periodic=(True, True), tol=1e-10, itmax=64)
    s.set_velocity(wlsynth.tgv2d_exact(N, nu, 0.0))
    T = kut / k
    while s.t < T - 1e-12:
        s.dt = min(s.dt, T - s.t)
        s.step()
    ex = wlsynth.tgv2d_exact(N, nu, s.t)
    g = s.grid
    num = sum(np.sum((s.u[i][g.interior()] - ex[i][g.interior()]) ** 2) for i in range(2))
    den = sum(np.sum(ex[i][g.interior()] ** 2) for i in range(2))
    return math.sqrt(num / den)


@pytest.mark.slow
def test_tgv2d_convergence_order():
    # the 2-D Taylor-Green vortex is an exact Navier-Stokes solution
    e = [_run_tgv2d(N) for N in (32, 64, 128)]
    orders = [math.log2(e[i] / e[i + 1]) for i in range(2)]
    assert min(orders) >= 1.8, (e, orders)
    assert e[-1] < 1e-4


def test_tgv3d_early_decay_rate():
    # Difference of two runs (nu and 2 nu): ln E_nu - ln E_2nu = 2 nu lam_h t with the
    # discrete eigenvalue lam_h = 12 sin^2(kappa/2) of the initial mode.
    N = 16
    k = 2 * math.pi / N
    lam = 12 * math.sin(k / 2) ** 2
    out = {}
    for nu in (0.02, 0.04):
        w = wlsynth.Workload("tgv", (N, N, N), (0.0, 0.0, 0.0), nu, periodic=(True,) * 3,
                             noise=0.0, init="tgv")
        s = Sim(w.n, w.U, nu, periodic=w.periodic, tol=1e-11, itmax=64)
        s.set_velocity(wlsynth.initial_velocity(w))
        E0 = s.ke()
        T = 0.5 / k
        while s.t < T - 1e-12:
            s.dt = min(0.25, T - s.t)
            s.step()
        out[nu] = (math.log(s.ke() / E0), s.t)
    d = out[0.02][0] - out[0.04][0]
    expect = 2 * 0.02 * lam * out[0.02][1]
    assert d == pytest.approx(expect, rel=0.02)


@pytest.mark.parametrize("n,per", [((32, 16), (False, False)), ((12, 8, 8), (False, False, False)),
                                   ((16, 16), (True, True))])
def test_freestream_is_preserved_exactly(n, per):
    U = (1.0, 0.0) if len(n) == 2 else (1.0, 0.0, 0.0)
    if all(per):
        U = (0.4, -0.3)
    s = Sim(n, U, 0.05, periodic=per)
    for _ in range(100 if len(n) == 2 else 20):
        s.step()
    for i in range(len(n)):
        assert np.all(s.u[i] == U[i])


def test_cfl_uniform_flow():
    g = Grid((8, 8, 8))
    u = [np.full(g.shape, v) for v in (0.5, -0.25, 0.125)]
    nu = 0.01
    assert cfl(g, u, nu) == 1.0 / (0.875 + 5 * nu)
    u = [np.zeros(g.shape) for _ in range(3)]
    assert cfl(g, u, 0.0) == 10.0


def test_bdim_special_cases():
    g = Grid((6, 5))
    rng = np.random.default_rng(0)
    ft = [rng.normal(size=g.shape) for _ in range(2)]
    V = [rng.normal(size=g.shape) for _ in range(2)]
    one = [np.ones(g.shape)] * 2
    zero2 = [[np.zeros(g.shape)] * 2] * 2
    out = bdim(g, ft, V, one, zero2)
    for i in range(2):
        np.testing.assert_array_equal(out[i], V[i] + ft[i])
    out = bdim(g, ft, V, [np.zeros(g.shape)] * 2, zero2)
    for i in range(2):
        np.testing.assert_array_equal(out[i], V[i])


def test_bc_closed_form():
    g = Grid((5, 4, 3), (False, True, False))
    rng = np.random.default_rng(3)
    u = [rng.normal(size=g.shape) for _ in range(3)]
    U = (1.0, 0.5, -0.25)
    apply_bc(g, U, u)
    # normal faces
    assert np.all(u[0][[0, 1, 6]] == 1.0)
    assert np.all(u[2][:, :, [0, 1, 4]] == -0.25)
    # periodic axis 1 for every component
    for i in range(3):
        np.testing.assert_array_equal(u[i][:, 0], u[i][:, 4])
        np.testing.assert_array_equal(u[i][:, 5], u[i][:, 1])
    # tangential zero-gradient ghosts
    np.testing.assert_array_equal(u[1][0], u[1][1])
    np.testing.assert_array_equal(u[1][6], u[1][5])
    np.testing.assert_array_equal(u[0][:, :, 0], u[0][:, :, 1])


def test_convective_exit_conserves_mass():
    g = Grid((10, 6, 4))
    rng = np.random.default_rng(2)
    u0 = [1.0 + 0.1 * rng.normal(size=g.shape) for _ in range(3)]
    e = exit_plane(g, (1.0, 0.0, 0.0), u0, 0.4)
    assert abs(e.sum() - 6 * 4 * 1.0) < 1e-12
    # without noise the exit value is the advected one
    u0 = [np.ones(g.shape), np.zeros(g.shape), np.zeros(g.shape)]
    np.testing.assert_array_equal(exit_plane(g, (1.0, 0.0, 0.0), u0, 0.4), 1.0)


def test_circle_flow_mirror_symmetry():
    w = wlsynth.circle_2d(n=(64, 32), R=5.0, center=(16.0, 16.0))
    s = Sim(w.n, w.U, w.nu, w.body, tol=1e-10)
    for _ in range(20):
        s.step()
    u, v = s.u
    # u symmetric, v antisymmetric about y = 16 (face rows of v sit at y = I - 1)
    np.testing.assert_allclose(u[1:-1, 1:33], u[1:-1, 1:33][:, ::-1], atol=1e-12)
    np.testing.assert_allclose(v[1:-1, 1:34], -v[1:-1, 1:34][:, ::-1], atol=1e-12)


def test_step_divergence_free_after_projection():
    w = wlsynth.sphere_3d(n=(32, 16, 16), D=6.0, center=(8.0, 8.0, 8.0))
    s = Sim(w.n, w.U, w.nu, w.body, convective_exit=True, tol=1e-8)
    s.set_velocity(wlsynth.initial_velocity(w))
    for _ in range(3):
        st = s.step()
        assert st["div_linf"] < 1e-8
        assert all(v >= 1 for v in st["vcycles"])


@pytest.mark.parametrize("ndim", [2, 3])
def test_freestream_around_a_body_translating_with_it(ndim):
    # A body moving at the free-stream velocity leaves uniform flow uniform: the
    # fluid update f~ = u0 + dt R - V vanishes wherever V is set (R = 0 on a uniform
    # field), mu0 f~ + mu1 grad f~ = f~ = U far away, so u* = U on every face, the
    # divergence is 0 and no pressure is needed.  Exact in floating point.
    if ndim == 2:
        U = (1.0, 0.0)
        body = wlsynth.Body("sphere", center=(20.0, 12.3), radius=4.0, velocity=U)
        n, steps = (160, 24), 100
    else:
        U = (1.0, 0.0, 0.0)
        body = wlsynth.Body("box", center=(10.0, 8.2, 7.9), half_extent=(2.0, 3.0, 2.5), velocity=U,
                            pitch_amp=0.3, phase_p=math.pi / 2)
        n, steps = (48, 16, 16), 20
    s = Sim(n, U, 0.03, body, convective_exit=True)
    for _ in range(steps):
        st = s.step()
        assert st["vcycles"] == (0, 0)
    assert s.t > 0.8 * steps * 0.85  # the body really travelled
    for i in range(ndim):
        assert np.all(s.u[i] == U[i])
    # the same body at rest in the stream is not uniform: the pin is not vacuous
    rest = wlsynth.Body(body.kind, center=body.center, radius=body.radius, half_extent=body.half_extent)
    s2 = Sim(n, U, 0.03, rest, convective_exit=True)
    s2.step()
    assert np.max(np.abs(s2.u[0] - U[0])) > 0.1
