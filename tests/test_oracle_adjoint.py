"""Pin of the oracle's complex-step rollout gradient against central finite differences."""
import pytest

import wlsynth
from oracle import adjoint as A


def test_complex_step_gradient_matches_central_differences():
    w = wlsynth.rotating_cylinder_2d(n=(48, 24), D=6.0, center=(14.0, 12.0), xi=0.8)
    xi, R = 0.8, 3.0
    steps, win = 12, 6
    J, gx, gR, dts = A.gradient(w, xi, R, steps, win)
    # the objective is piecewise smooth (limiter branches, solid-face cut): FD needs a
    # step small enough not to cross a kink; it then agrees with the complex step
    h = 1e-6
    Jp, _ = A.objective(w, xi + h, R, steps, win, dts)
    Jm, _ = A.objective(w, xi - h, R, steps, win, dts)
    assert gx == pytest.approx((Jp - Jm) / (2 * h), rel=1e-7, abs=1e-9)
    Jp, _ = A.objective(w, xi, R + h, steps, win, dts)
    Jm, _ = A.objective(w, xi, R - h, steps, win, dts)
    assert gR == pytest.approx((Jp - Jm) / (2 * h), rel=1e-7, abs=1e-9)
    # spinning changes the drag: the derivative is not trivially zero
    assert abs(gx) > 1e-4 and abs(gR) > 1e-4


def test_complex_step_with_live_cfl_matches_central_differences():
    # with the time steps following the flow (dt = 1/(max outflux + 5 nu) each step),
    # the complex step carries the derivative through the argmax cell of the outflux;
    # central differences of the live-CFL rollout agree, and the result differs from
    # the frozen-schedule derivative
    w = wlsynth.rotating_cylinder_2d(n=(48, 24), D=6.0, center=(14.0, 12.0), xi=0.8)
    xi, R = 0.8, 3.0
    steps, win = 12, 6
    J, gx, gR, dts = A.gradient_cfl(w, xi, R, steps, win)
    h = 1e-6
    Jp, dp = A.objective(w, xi + h, R, steps, win)
    Jm, dm = A.objective(w, xi - h, R, steps, win)
    assert dp != dts  # the steps really move with xi
    assert gx == pytest.approx((Jp - Jm) / (2 * h), rel=1e-6, abs=1e-9)
    Jp, _ = A.objective(w, xi, R + h, steps, win)
    Jm, _ = A.objective(w, xi, R - h, steps, win)
    assert gR == pytest.approx((Jp - Jm) / (2 * h), rel=1e-6, abs=1e-9)
    _, fx, fR, _ = A.gradient(w, xi, R, steps, win)
    assert abs(gx - fx) > 1e-6 * abs(fx)


def test_rotcyl_radius_step_crosses_no_cut():
    # Central differences of the 512 x 256 rotating-cylinder objective at h = 1e-3
    # in R disagree with the exact derivative by a few 1e-3; no face changes sides of
    # the solid cut (mu0 < 1e-6) or of the body velocity's cutoff (d < 2 + eps)
    # between R - 1e-3 and R + 1e-3, so those jumps are not the cause.
    import numpy as np
    from oracle import Grid
    from oracle.body import MU0_CUT, face_points, sdf_normal_velocity
    from oracle.moments import mu0
    w = wlsynth.rotating_cylinder_2d()
    g = Grid(w.n)
    R, h = float(w.body.radius), 1e-3
    for i in range(2):
        X = face_points(g, i)
        ds = []
        for RR in (R - h, R + h):
            b = wlsynth.Body("sphere", center=w.body.center, radius=RR)
            ds.append(sdf_normal_velocity(b, X, 0.0)[0])
        assert np.array_equal(mu0(ds[0], 1.0) < MU0_CUT, mu0(ds[1], 1.0) < MU0_CUT)
        assert np.array_equal(ds[0] < 3.0, ds[1] < 3.0)
