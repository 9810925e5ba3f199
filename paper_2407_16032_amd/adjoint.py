"""Reverse-mode gradient of a force objective of a rollout, as a torch.autograd.Function.

The paper differentiates the solver by running it on dual numbers (software
design section; the rotating-cylinder example of the results).  Here the
forward rollout runs the HIP step, keeping checkpoints of (u, p, t) every
``ckpt`` steps; backward re-runs each segment forward from its checkpoint to
recover the states, then walks the steps in reverse with the library's
discrete adjoint (``wl_adj_step``), seeding each state of the averaging window
with the force functional's adjoint (``wl_adj_forces``).  Only marshalling
and the checkpoint schedule live here; every step and transpose runs in the
HIP library.

Objective (rotating cylinder): J = mean over the window of the drag
coefficient C_D = 2 F_x / (U^2 A_ref), A_ref = 2 R, for a circle of radius R
spinning counter-clockwise at omega = xi U / R (xi = D omega / (2 U)); or
(``objective="lift_to_drag"``) the Magnus lift efficiency J = -mean C_L / mean C_D
(C_L = 2 F_y / (U^2 A_ref); counter-clockwise spin in a +x stream lifts toward -y).  The
time steps are either frozen to the schedule recorded by the first forward run,
or (``live_dt``) follow the CFL rule in every run, and the gradient then includes
their dependence on the flow (``wl_adj_step_cfl``).
"""
from __future__ import annotations

import copy
from typing import List, Optional

import torch

from .sim import Simulation


class RotatingCylinderDrag:
    """Window-mean drag of a spinning circle and its gradient in (xi, R).

    ``w`` is a rotating-cylinder workload (grid, U, nu, body centre); ``u0`` the
    initial velocity arrays (indexed [x, y]); ``steps`` and ``window_start`` as in
    the forward rollout; ``ckpt`` the checkpoint interval; ``tol``/``itmax`` the
    multigrid settings of forward and adjoint solves.
    """

    def __init__(self, w, u0, steps: int, window_start: int, ckpt: int = 20, prec: str = "f64",
                 tol: float = 1e-12, itmax: int = 200, device="cuda:0", live_dt: bool = False,
                 objective: str = "drag"):
        self.w = w
        self.u0 = u0
        self.steps = int(steps)
        self.win = int(window_start)
        if not 0 <= self.win < self.steps:
            raise ValueError("window_start must be in [0, steps)")
        self.ckpt = max(1, int(ckpt))
        self.tol = tol
        self.U = float(w.U[0])
        self.sim = Simulation(w.n, w.U, w.nu, self._body(1.0, float(w.body.radius)), periodic=w.periodic_mask(),
                              prec=prec, tol=tol, itmax=itmax, device=device, adjoint=True)
        self.dts: Optional[List[float]] = None
        self.live_dt = bool(live_dt)
        if objective not in ("drag", "lift_to_drag"):
            raise ValueError("objective must be 'drag' or 'lift_to_drag'")
        self.objective = objective
        self.means = (0.0, 0.0)  # window means of C_D and C_L of the last forward run
        self.last_dts: Optional[List[float]] = None  # the schedule of the last forward run
        self.stats = {}

    def _body(self, xi: float, R: float):
        b = copy.copy(self.w.body)
        b.radius = R
        b.spin_omega = xi * self.U / R
        return b

    def _start(self, xi: float, R: float):
        s = self.sim
        s.body_update(self._body(xi, R))
        s.set_velocity(self.u0)
        s.field("p").zero_()
        frozen = self.dts is not None and not self.live_dt
        s.set_time(0.0, self.dts[0] if frozen else s.desc.dt0)

    def _coefs(self, R: float):
        fp, fv = self.sim.forces()
        q = self.U ** 2 * 2.0 * R
        return 2.0 * (fp[0] + fv[0]) / q, 2.0 * (fp[1] + fv[1]) / q

    def value(self, xi: float, R: float, record: bool = False):
        """J and, if ``record``, the checkpoints of the run (dict step -> state)."""
        s = self.sim
        self._start(xi, R)
        ckpts = {}
        dts = []
        cds, cls = [], []
        for k in range(self.steps):
            t, dt = s.time()
            if self.dts is not None and not self.live_dt:
                dt = self.dts[k]
                s.set_time(t, dt)
            if record and k % self.ckpt == 0:
                ckpts[k] = s.save_state()
            dts.append(dt)
            s.step()
            if k >= self.win:
                cd, cl = self._coefs(R)
                cds.append(cd)
                cls.append(cl)
        if self.dts is None:
            self.dts = dts
        self.last_dts = dts
        mcd, mcl = sum(cds) / len(cds), sum(cls) / len(cls)
        self.means = (mcd, mcl)
        J = mcd if self.objective == "drag" else -mcl / mcd
        return (J, ckpts) if record else J

    def value_and_grad(self, xi: float, R: float):
        """(J, dJ/dxi, dJ/dR) with the frozen time-step schedule."""
        J, ckpts = self.value(xi, R, record=True)
        return (J,) + self.gradient(xi, R, J, ckpts)

    def gradient(self, xi: float, R: float, J: float, ckpts):
        """(dJ/dxi, dJ/dR) by the reverse sweep over the checkpoints of value(record=True)."""
        s = self.sim
        dts = self.last_dts if self.live_dt else self.dts
        s.body_update(self._body(xi, R))
        nwin = self.steps - self.win
        weight = 1.0 / (nwin * self.U ** 2 * R)  # d(mean C)/dF of each window state
        if self.objective == "drag":
            ex = (1.0, 0.0, 0.0)
        else:  # J = -Lbar / Dbar: dJ/dCD_k = (Lbar / Dbar^2) / n, dJ/dCL_k = -(1 / Dbar) / n
            mcd, mcl = self.means
            ex = (mcl / mcd ** 2, -1.0 / mcd, 0.0)
        s.adj_reset()
        adj_cycles = 0
        fwd_cycles = 0
        for s0 in reversed(sorted(ckpts)):
            s1 = min(s0 + self.ckpt, self.steps)
            # recompute the segment's states s0 .. s1
            s.load_state(ckpts[s0], dts[s0])
            states = [s.save_state()]
            for n in range(s0, s1):
                s.set_time(s.time()[0], dts[n])
                st = s.step()
                fwd_cycles += sum(st["vcycles"])
                states.append(s.save_state())
            for n in range(s1 - 1, s0 - 1, -1):
                if n >= self.win:  # C_D of the state after step n
                    s.load_state(states[n + 1 - s0])
                    s.adj_forces(ex, weight)
                s.load_state(states[n - s0], dts[n])
                # step 0 starts from dt0; every later step's dt is the CFL step of its state
                st = s.adj_step_cfl(n > 0, self.tol) if self.live_dt else s.adj_step(self.tol)
                adj_cycles += sum(st["adj_vcycles"])
                fwd_cycles += sum(st["vcycles"])
        dR_w, dW = s.adj_body_grad()
        omega = xi * self.U / R
        dxi = dW * self.U / R
        # the drag's reference area 2R gives the direct term -J/R; the ratio has none
        dR = dR_w - dW * omega / R - (J / R if self.objective == "drag" else 0.0)
        self.stats = {"adj_vcycles": adj_cycles, "recompute_vcycles": fwd_cycles}
        return dxi, dR


class _DragFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, problem):
        xi, R = (float(v) for v in theta.detach().cpu().tolist())
        J, ckpts = problem.value(xi, R, record=True)
        ctx.problem, ctx.ckpts, ctx.args = problem, ckpts, (xi, R, J)
        return theta.new_tensor(J)

    @staticmethod
    def backward(ctx, gJ):
        xi, R, J = ctx.args
        dxi, dR = ctx.problem.gradient(xi, R, J, ctx.ckpts)
        ctx.ckpts = None
        return gJ * gJ.new_tensor([dxi, dR]), None


def rotating_cylinder_drag(theta: torch.Tensor, problem: RotatingCylinderDrag) -> torch.Tensor:
    """J(theta) for theta = (xi, R) as a differentiable torch scalar: forward runs
    the rollout keeping checkpoints, backward runs the checkpointed reverse sweep."""
    return _DragFn.apply(theta, problem)
