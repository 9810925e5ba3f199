"""Variable-coefficient Poisson operator and geometric multigrid (test infrastructure).

The paper's numerical-methods section: the projection leads to a Poisson
equation with spatially varying coefficients, solved by geometric multigrid;
the profiling section adds that a Jacobi-preconditioned conjugate-gradient
(PCG) smoother is used inside it; the software-design section shows the
coefficient array ``c`` (here L) applied as u_i[I] -= L_i[I](x[I]-x[I-e_i]).

Operator on interior cells (the divergence of L grad x):
    (A x)[I] = sum_i L_i[I+e_i](x[I+e_i]-x[I]) - L_i[I](x[I]-x[I-e_i]),
with periodic wrap, and rows of cells whose diagonal
D = -sum_i (L_i[I] + L_i[I+e_i]) vanishes set to zero (solid cells; iD = 0).

Readings used (the paper names the method only):
  * residual restriction = sum over the 2^n children; prolongation =
    piecewise-constant injection; coarse coefficients L_c = 1/2 * sum of the
    2^(n-1) fine faces covering the coarse face;
  * coarsen while every interior size is even and the coarse minimum >= 4;
  * V(0,1) cycle: restrict, recurse, PCG(k) on the coarse level, correct;
    the solve alternates one V-cycle and one fine PCG(k) until the max-norm
    of the residual is below tol (zero cycles if it already is), at most
    itmax cycles;
  * all inner products and norms are FP64 sums;
  * A has the constants (on the connected active cells) in its null space,
    since every boundary is Neumann or periodic, so each PCG sweep starts by
    removing the residual's mean over the active cells (projection onto the
    range of A).  This is exact for a consistent system and keeps rounding
    from driving the solution along the null space.
"""
from __future__ import annotations

import numpy as np

from .grid import Grid


class Level:
    def __init__(self, grid: Grid, L):
        self.grid = grid
        self.L = L
        g = grid
        D = g.zeros()
        for i in range(g.ndim):
            D = D - (L[i] + g.sh(L[i], i, +1))
        D = np.where(g.interior_mask(), D, 0.0)
        self.D = D
        self.iD = np.where(D != 0.0, 1.0 / np.where(D != 0.0, D, 1.0), 0.0)
        self.active = self.iD != 0.0


def boundary_zeroed(grid: Grid, mu0):
    """L_i = mu0_i with the non-periodic boundary and ghost faces along i set to 0."""
    L = []
    for i in range(grid.ndim):
        a = mu0[i].copy()
        N = grid.n[i]
        if not grid.periodic[i]:
            idx = [slice(None)] * grid.ndim
            for k in (0, 1, N + 1):
                idx[i] = k
                a[tuple(idx)] = 0.0
        L.append(a)
    return L


def coarsen_L(gf: Grid, Lf, gc: Grid):
    Lc = []
    for i in range(gf.ndim):
        a = gc.zeros(Lf[i].dtype)
        src = Lf[i]
        # along i: fine face index 2J-1 for J = 1..Nc+1
        sl = [slice(None)] * gf.ndim
        sl[i] = slice(1, gf.n[i] + 2, 2)
        src = src[tuple(sl)]
        # along the other axes: sum the two children of every interior coarse index
        for k in range(gf.ndim):
            if k == i:
                continue
            sl = [slice(None)] * gf.ndim
            sl[k] = slice(1, gf.n[k] + 1)
            s = src[tuple(sl)]
            shp = list(s.shape)
            shp[k:k + 1] = [gc.n[k], 2]
            src = s.reshape(shp).sum(axis=k + 1)
        dst = [slice(1, gc.n[k] + 1) for k in range(gf.ndim)]
        dst[i] = slice(1, gc.n[i] + 2)
        a[tuple(dst)] = 0.5 * src
        Lc.append(a)
    return Lc


def build_levels(grid: Grid, L):
    levels = [Level(grid, L)]
    g = grid
    while g.coarsenable():
        gc = g.coarse()
        levels.append(Level(gc, coarsen_L(g, levels[-1].L, gc)))
        g = gc
    return levels


def apply_A(lev: Level, x):
    g = lev.grid
    out = g.zeros()
    for i in range(g.ndim):
        Lp = g.sh(lev.L[i], i, +1)
        out = out + Lp * (g.sh(x, i, +1) - x) - lev.L[i] * (x - g.sh(x, i, -1))
    return np.where(lev.active, out, 0.0)


def dot(a, b):
    # bilinear (no conjugation), so complex-step derivatives pass through the solve
    return np.sum(a * b)


def restrict(gf: Grid, gc: Grid, r):
    s = r[gf.interior()]
    shp = []
    for Nc in gc.n:
        shp += [Nc, 2]
    s = s.reshape(shp).sum(axis=tuple(range(1, 2 * gf.ndim, 2)))
    out = gc.zeros(r.dtype)
    out[gc.interior()] = s
    return out


def prolong(gf: Grid, xc):
    s = xc[tuple(slice(1, N + 1) for N in (v // 2 for v in gf.n))]
    for k in range(gf.ndim):
        s = np.repeat(s, 2, axis=k)
    out = gf.zeros(xc.dtype)
    out[gf.interior()] = s
    return out


def pcg(lev: Level, x, r, iters):
    """Jacobi-preconditioned CG on A x = b, given x and r = b - A x (updated in place)."""
    act = lev.active
    if act.any():
        r[act] -= np.mean(r[act])
    z = lev.iD * r
    e = z.copy()
    rho = dot(r, z)
    if rho == 0.0:
        return
    for it in range(iters):
        q = apply_A(lev, e)
        sigma = dot(e, q)
        if abs(sigma) < 1e-300:
            return
        alpha = rho / sigma
        x += alpha * e
        r -= alpha * q
        if it == iters - 1:
            return
        z = lev.iD * r
        rho_new = dot(r, z)
        if rho_new == 0.0:
            return
        e = z + (rho_new / rho) * e
        rho = rho_new


def vcycle(levels, l, x, r, iters):
    f, c = levels[l], levels[l + 1]
    rc = np.where(c.active, restrict(f.grid, c.grid, r), 0.0)
    xc = c.grid.zeros(rc.dtype)
    if l + 2 < len(levels):
        vcycle(levels, l + 1, xc, rc, iters)
    pcg(c, xc, rc, iters)
    e = prolong(f.grid, xc)
    x += e
    r -= apply_A(f, e)


def residual(lev: Level, x, z):
    return np.where(lev.active, z - apply_A(lev, x), 0.0)


def solve(levels, x, z, tol, itmax=32, iters=6):
    """Multigrid solve of A x = z in place; returns a stats dict."""
    fine = levels[0]
    r = residual(fine, x, z)
    res0 = float(np.max(np.abs(r)))
    n = 0
    res = res0
    while res >= tol and n < itmax:
        if len(levels) > 1:
            vcycle(levels, 0, x, r, iters)
        pcg(fine, x, r, iters)
        n += 1
        res = float(np.max(np.abs(r)))
    return {"vcycles": n, "res0_linf": res0, "res_linf": res,
            "res_l2": float(np.sqrt(np.sum(np.abs(r) ** 2))), "converged": res < tol, "r": r}


def divergence(grid: Grid, u):
    z = grid.zeros()
    for i in range(grid.ndim):
        z = z + (grid.sh(u[i], i, +1) - u[i])
    return np.where(grid.interior_mask(), z, 0.0)
