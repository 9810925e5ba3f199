"""Davidon optimisation of a rotation rate driven by the discrete adjoint with
live time steps (paper, applications section: the control cylinders' spin is
optimised from C_P and its exact derivative with Davidon's method).  Objective:
the Magnus lift efficiency -mean C_L / mean C_D of a spinning circle, which has
an interior optimum in the rotation rate."""
import sys

import numpy as np
import pytest

import wlsynth

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _problem(steps=120, win=60):
    from paper_2407_16032_amd.adjoint import RotatingCylinderDrag
    w = wlsynth.rotating_cylinder_2d(n=(96, 48), D=12.0, center=(30.0, 24.0), xi=1.0)
    return RotatingCylinderDrag(w, wlsynth.initial_velocity(w), steps, win, ckpt=20, prec="f64", tol=1e-10,
                                live_dt=True, objective="lift_to_drag")


def test_lift_to_drag_gradient_matches_central_differences():
    prob = _problem()
    R = 6.0
    J, gx, gR = prob.value_and_grad(1.2, R)
    # with the time steps live, J is smooth only between switches of the CFL's
    # argmax cell and of limiter branches: central differences need a step below
    # their spacing (at h = 1e-4 or 1e-5 they average over switches)
    h = 1e-6
    fx = (prob.value(1.2 + h, R) - prob.value(1.2 - h, R)) / (2 * h)
    fR = (prob.value(1.2, R + h) - prob.value(1.2, R - h)) / (2 * h)
    _say("J %.8f  dJ/dxi %.8f fd %.8f  dJ/dR %.8f fd %.8f" % (J, gx, fx, gR, fR))
    assert gx == pytest.approx(fx, rel=1e-4, abs=1e-7)
    assert gR == pytest.approx(fR, rel=1e-3, abs=1e-6)
    prob.sim.close()


def test_davidon_finds_the_best_rotation_rate():
    from paper_2407_16032_amd.optimize import optimize_rotation_rate
    prob = _problem()
    R = 6.0
    out = optimize_rotation_rate(prob, R, 1.0, 2.5, maximize=True, tol=0.02, maxit=10)
    for e in out["log"]:
        _say("  xi %.5f  J %.6f  dJ/dxi %+.6f  (%.1f s)" % (e["xi"], e["J"], e["dJ_dxi"], e["seconds"]))
    xs = out["x"]
    _say("optimum xi %.5f J %.6f after %d evaluations" % (xs, out["f"], len(out["evaluations"])))
    assert len(out["evaluations"]) <= 12
    assert abs(out["g"]) < 0.1 * max(abs(out["log"][0]["dJ_dxi"]), abs(out["log"][1]["dJ_dxi"]))
    # the optimum beats a scan of the interval
    scan = [prob.value(x, R) for x in np.linspace(1.0, 2.5, 7)]
    _say("  scan", ["%.5f" % v for v in scan])
    assert out["f"] >= max(scan) - 1e-3 * abs(max(scan))
    prob.sim.close()
