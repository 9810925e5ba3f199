"""The BDIM projection time step in FP64 (test infrastructure; see ``oracle/__init__``).

One step n -> n+1 (paper, numerical-methods section: explicit
predictor-corrector, each stage projected; performance section: routines
measure!, conv_diff!, BDIM!, BC!, exitBC!, project!, CFL!, scale_u!):

  measure at t_n if the body moves; u0 = u
  predictor: f = u0 + dt R(u0) - V;  u* = V + mu0 f + sum_j mu1_ij (f[I+e_j]-f[I-e_j])/2
             BC (convective exit computed here from u0); project with x0 = p dt
  corrector: f = u0 + dt R(u') - V;  u** = (u' + V + mu0 f + mu1 . grad f)/2
             BC (exit plane held); project with x0 = p dt/2
  t += dt;  dt = min(dt_max, 1/(max_I sigma[I] + 5 nu)),
            sigma[I] = sum_i max(0, u_i[I+e_i]) + max(0, -u_i[I])

Projection: z = div u, solve A x = z, u_i -= L_i (x[I]-x[I-e_i]), p = x/(w dt).

Boundary conditions (reading of "slip by default, convective outlet or
periodic"): along a non-periodic axis i the normal faces 0, 1, N+1 of u_i
take U_i; tangential ghosts copy the nearest interior value; periodic axes
copy across the period.  Axes are processed in order 0..n-1 for every
component.  Convective exit on +x (predictor only, then held):
u_x[N+1] = u0_x[N+1] - dt U_x (u0_x[N+1] - u0_x[N]), then a uniform shift so
that the exit flux equals the inlet flux (FP64 sums).
"""
from __future__ import annotations

import math

import numpy as np

from . import body as _body
from . import flux as _flux
from . import poisson as _poisson
from .grid import Grid


def apply_bc(grid: Grid, U, u, exit_plane=None):
    nd = grid.ndim
    for i in range(nd):
        a = u[i]
        for k in range(nd):
            N = grid.n[k]

            def at(idx):
                s = [slice(None)] * nd
                s[k] = idx
                return tuple(s)

            if grid.periodic[k]:
                a[at(0)] = a[at(N)]
                a[at(N + 1)] = a[at(1)]
            elif k == i:
                for idx in (0, 1, N + 1):
                    a[at(idx)] = U[i]
                if exit_plane is not None and i == 0:
                    s = [N + 1] + [slice(1, grid.n[m] + 1) for m in range(1, nd)]
                    a[tuple(s)] = exit_plane
            else:
                a[at(0)] = a[at(1)]
                a[at(N + 1)] = a[at(N)]
    return u


def exit_plane(grid: Grid, U, u0, dt):
    N = grid.n[0]
    inner = tuple(slice(1, grid.n[m] + 1) for m in range(1, grid.ndim))
    ue = u0[0][(N + 1,) + inner]
    ub = u0[0][(N,) + inner]
    e = ue - dt * U[0] * (ue - ub)
    count = e.size
    inlet = np.sum(np.full(e.shape, float(U[0])))
    shift = (inlet - np.sum(e)) / count
    return e + shift


def bdim(grid: Grid, ft, V, m0, m1):
    out = []
    for i in range(grid.ndim):
        acc = V[i] + m0[i] * ft[i]
        for j in range(grid.ndim):
            fp, vp = grid.shift(ft[i], j, +1)
            fm, vm = grid.shift(ft[i], j, -1)
            grad = np.where(vp & vm, 0.5 * (fp - fm), 0.0)
            acc = acc + m1[i][j] * grad
        out.append(acc)
    return out


def cfl(grid: Grid, u, nu, dt_max=10.0, cfl_nu=5.0):
    """CFL step from the largest outflux sigma over the interior cells.  The maximum
    is taken at one cell (the first in x-fastest order among equal real parts), so
    a complex-step perturbation of u carries through sigma at that cell into the
    step: the derivative of the min/max map on its active branch."""
    s = grid.zeros(np.result_type(*u))
    for i in range(grid.ndim):
        s = s + np.maximum(0.0, grid.sh(u[i], i, +1)) + np.maximum(0.0, -u[i])
    si = s[grid.interior()].T          # x fastest in C order
    smax = si.flat[int(np.argmax(np.real(si)))]
    denom = smax + cfl_nu * nu
    if np.real(denom) <= 0.0:
        return dt_max
    dt = 1.0 / denom
    if np.real(dt) >= dt_max:
        return dt_max
    return float(dt) if np.isrealobj(dt) else dt


class Sim:
    """FP64 reference simulation (state lives in padded numpy arrays)."""

    def __init__(self, n, U, nu, body=None, periodic=None, convective_exit=False, eps=1.0,
                 dt0=0.25, dt_max=10.0, cfl_nu=5.0, tol=1e-6, itmax=32, pcg_iters=6):
        self.grid = Grid(n, periodic)
        g = self.grid
        self.U = tuple(float(v) for v in U)
        self.nu = float(nu)
        self.body = body if (body is not None and body.kind != "none") else None
        self.exit = bool(convective_exit)
        self.eps = float(eps)
        self.dt = float(dt0)
        self.dt_max = float(dt_max)
        self.cfl_nu = float(cfl_nu)
        self.tol = float(tol)
        self.itmax = int(itmax)
        self.pcg_iters = int(pcg_iters)
        self.t = 0.0
        self.dt_schedule = None          # frozen time steps (list), else CFL
        self.u = [np.full(g.shape, self.U[i]) for i in range(g.ndim)]
        self.p = g.zeros()
        self.exit_e = None
        self.stats = []
        self.measure(0.0)

    # -- set-up -------------------------------------------------------------
    def measure(self, t):
        g = self.grid
        self.mu0, self.mu1, self.V = _body.measure(g, self.body, t, self.eps)
        self.L = _poisson.boundary_zeroed(g, self.mu0)
        self.levels = _poisson.build_levels(g, self.L)

    def set_velocity(self, u):
        self.u = [np.array(a, dtype=np.float64, copy=True) for a in u]
        apply_bc(self.grid, self.U, self.u)

    # -- pieces of the step ---------------------------------------------------
    def conv_diff(self, u):
        return _flux.conv_diff(self.grid, u, self.nu)

    def project(self, w, tol=None):
        g = self.grid
        z = _poisson.divergence(g, self.u)
        x = (self.p * (w * self.dt)).astype(np.result_type(self.p, z, self.L[0], self.dt))
        st = _poisson.solve(self.levels, x, z, self.tol if tol is None else tol, self.itmax,
                            self.pcg_iters)
        for i in range(g.ndim):
            upd = self.L[i] * (x - g.sh(x, i, -1))
            self.u[i] = self.u[i] - np.where(g.interior_mask(), upd, 0.0)
        self.p = x / (w * self.dt)
        self.x = x
        return st

    def step(self, remeasure=True):
        g = self.grid
        dt = self.dt
        if self.body is not None and remeasure and self.body.moving:
            self.measure(self.t)
        u0 = [a.copy() for a in self.u]
        # predictor
        R = self.conv_diff(u0)
        ft = [u0[i] + dt * R[i] - self.V[i] for i in range(g.ndim)]
        self.u = bdim(g, ft, self.V, self.mu0, self.mu1)
        self.exit_e = exit_plane(g, self.U, u0, dt) if self.exit else None
        apply_bc(g, self.U, self.u, self.exit_e)
        s1 = self.project(1.0)
        apply_bc(g, self.U, self.u, self.exit_e)
        # corrector
        R = self.conv_diff(self.u)
        ft = [u0[i] + dt * R[i] - self.V[i] for i in range(g.ndim)]
        b = bdim(g, ft, self.V, self.mu0, self.mu1)
        self.u = [0.5 * (self.u[i] + b[i]) for i in range(g.ndim)]
        apply_bc(g, self.U, self.u, self.exit_e)
        s2 = self.project(0.5)
        apply_bc(g, self.U, self.u, self.exit_e)
        self.t += dt
        self.dt = cfl(g, self.u, self.nu, self.dt_max, self.cfl_nu)
        if self.dt_schedule is not None and len(self.stats) + 1 < len(self.dt_schedule):
            self.dt = self.dt_schedule[len(self.stats) + 1]
        st = {"dt": dt, "t": self.t, "vcycles": (s1["vcycles"], s2["vcycles"]),
              "res_linf": (s1["res_linf"], s2["res_linf"]),
              "div_linf": float(np.max(np.abs(_poisson.divergence(g, self.u)[
                  self.levels[0].active]))) if self.levels[0].active.any() else 0.0}
        self.stats.append(st)
        return st

    def forces(self):
        if self.body is None:
            return np.zeros(self.grid.ndim), np.zeros(self.grid.ndim)
        return _body.forces(self.grid, self.body, self.t, self.u, self.p, self.nu, self.eps,
                            active=self.levels[0].active)

    def ke(self):
        """Kinetic energy sum of u_i^2/2 over the interior faces (diagnostic)."""
        g = self.grid
        return 0.5 * sum(float(np.sum(self.u[i][g.interior()] ** 2)) for i in range(g.ndim))
