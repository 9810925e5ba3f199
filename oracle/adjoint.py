"""Reference gradient of a rollout objective by the complex-step method (test infrastructure).

The paper differentiates the whole solver with forward-mode dual numbers.
The same exact derivative of the FP64 oracle is obtained here with a complex
perturbation: J(theta + i h) = J + i h J'(theta) + O(h^2), so J' = Im J(theta + i h)/h
to rounding for h = 1e-30 (Squire & Trapp 1998).  Branches (limiter medians,
masks) follow the real part, i.e. the derivative is the one of the forward
branch.

Objective (rotating-cylinder case): J = mean over a window of steps of the
drag coefficient C_D = 2 (F_p + F_v)_x / (U^2 A_ref), A_ref = D = 2R, for a
circle of radius R spinning at Omega = xi U / R (xi = D Omega / (2U)).  The time
steps are frozen to the schedule of the unperturbed run.
"""
from __future__ import annotations

import copy

import numpy as np

import wlsynth

from .solver import Sim

H_CS = 1e-30


def rotcyl_body(w, xi, R):
    b = copy.copy(w.body)
    b.radius = R
    b.spin_omega = xi * w.U[0] / R
    return b


def objective(w, xi, R, steps, window_start, dt_schedule=None, tol=1e-12, itmax=200, u0=None):
    """J and the time-step schedule of the run (real part)."""
    body = rotcyl_body(w, xi, R)
    s = Sim(w.n, w.U, w.nu, body, periodic=w.periodic_mask(), tol=tol, itmax=itmax)
    s.set_velocity(wlsynth.initial_velocity(w) if u0 is None else u0)
    if dt_schedule is not None:
        s.dt = dt_schedule[0]
        s.dt_schedule = dt_schedule
    dts, cds = [], []
    for k in range(steps):
        dts.append(float(np.real(s.dt)))
        s.step()
        if k >= window_start:
            Fp, Fv = s.forces()
            cds.append(2.0 * (Fp[0] + Fv[0]) / (w.U[0] ** 2 * 2.0 * R))
    return np.mean(cds), dts


def gradient_cfl(w, xi, R, steps, window_start, tol=1e-12):
    """(J, dJ/dxi, dJ/dR) by complex step with the CFL time steps live: each step's
    dt follows the perturbed velocity through the largest outflux, so the
    derivative includes the dependence of the time steps on the flow."""
    J, dts = objective(w, xi, R, steps, window_start, tol=tol)
    Jx, _ = objective(w, xi + 1j * H_CS, R, steps, window_start, tol=tol)
    JR, _ = objective(w, xi, R + 1j * H_CS, steps, window_start, tol=tol)
    return float(np.real(J)), float(np.imag(Jx) / H_CS), float(np.imag(JR) / H_CS), dts


def gradient(w, xi, R, steps, window_start, tol=1e-12):
    """(J, dJ/dxi, dJ/dR) of the FP64 oracle by complex step, time steps frozen."""
    J, dts = objective(w, xi, R, steps, window_start, tol=tol)
    Jx, _ = objective(w, xi + 1j * H_CS, R, steps, window_start, dts, tol=tol)
    JR, _ = objective(w, xi, R + 1j * H_CS, steps, window_start, dts, tol=tol)
    return float(np.real(J)), float(np.imag(Jx) / H_CS), float(np.imag(JR) / H_CS), dts
