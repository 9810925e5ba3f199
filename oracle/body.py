"""Analytic rigid bodies, ``measure`` and force integrals (test infrastructure).

The paper's AutoBody holds a signed-distance function and a coordinate map;
``measure!`` turns them into the signed distance d, normal n and body
velocity V at the velocity points and then into the kernel moments.  This
oracle covers rigid bodies: a circle/sphere, a box, or a signed distance
sampled on a grid, moved by a uniform translation, heave along e_y and a
rotation about e_z through a pivot.

Body description (``wlsynth.Body``): centre c(t) = center + velocity t +
A_h sin(2 pi f t + phi_h) e_y; angle theta(t) = A_p sin(2 pi f t + phi_p) +
Omega t about e_z through P(t) = c(t) + pivot_offset.  A world point x maps to
the body frame by x_b = Rot(-theta)(x - P) + pivot_offset; the shape is centred
at the origin of that frame; SDF < 0 inside.  The rigid velocity is
V = dc/dt + theta' e_z x (x - P).

Gridded signed distance (reading; the paper's AutoBody takes any SDF and gets
the normal by automatic differentiation, a sampled SDF has no derivative of
its own): d(x_b) is the trilinear (bilinear in 2-D) interpolant of the samples;
the normal is the interpolant, with the same weights, of the per-sample
gradient taken by central differences of the samples (one-sided at the
grid's edges), normalised; a point outside the sampled box is fluid beyond the
kernel's reach (d = +inf).  Both are exact for a linear distance field.

General bodies (the paper's AutoBody: any SDF and any coordinate map, with
every geometric property taken from derivatives, which the paper obtains by
automatic differentiation).  A body is a chain of parts, each a shape (sphere,
box, plane, gridded SDF, optionally hollowed to |SDF| - shell) seen through its
own map x_b = S(t) * Rot(-theta(t)) (x - P(t)) + pivot_offset.  Reading of the
measured quantities: with g the world gradient of SDF(x_b(x, t)),
n = g / |g| and d = SDF / |g| (the map need not preserve distances; the ratio
is the distance to first order, and equals the SDF when the map is rigid);
V = -J^{-1} dx_b/dt with J = dx_b/dx (the velocity of the material point that
the map holds fixed).  The oracle takes g, J and dx_b/dt by the complex step
(exact derivatives, independent of any hand derivation).  Parts combine in
order by the arithmetic of signed distances (the paper's body = a + b, a - b):
union keeps the nearer part, intersection the farther, subtraction compares
with the negated part; the winning part supplies d, n and V (n and d negated
for a subtracted part); ties keep the earlier parts.
"""
from __future__ import annotations

import math

import numpy as np

from .moments import kernel_eps, mu0, mu1

# moments below this value are treated as zero (the face is solid): reading of
# the paper's unspecified handling of cells with vanishing Poisson diagonal
MU0_CUT = 1e-6


def _vec3(v):
    v = list(v) if v is not None else []
    return [v[k] if k < len(v) else 0.0 for k in range(3)]


def heave_direction(body):
    e = _vec3(getattr(body, "heave_dir", ()))
    m = math.sqrt(sum(v * v for v in e))
    return [0.0, 1.0, 0.0] if m == 0.0 else [v / m for v in e]


def motion(body, t):
    """(c, P, theta, cdot, omega) at time t (numpy scalars, so that complex parameters
    carry complex-step derivatives)."""
    w = 2.0 * math.pi * body.freq
    vel = _vec3(getattr(body, "velocity", ()))
    eh = heave_direction(body)
    c = _vec3(body.center)
    hv = body.heave_amp * np.sin(w * t + body.phase_h)
    hd = body.heave_amp * w * np.cos(w * t + body.phase_h)
    c = [c[k] + vel[k] * t + hv * eh[k] for k in range(3)]
    po = _vec3(body.pivot_offset)
    P = [c[k] + po[k] for k in range(3)]
    theta = body.pitch_amp * np.sin(w * t + body.phase_p) + body.spin_omega * t
    cdot = [vel[k] + hd * eh[k] for k in range(3)]
    omega = body.pitch_amp * w * np.cos(w * t + body.phase_p) + body.spin_omega
    return c, P, theta, cdot, omega


def sdf_normal_velocity(body, X, t):
    """Signed distance, unit normal (list) and rigid velocity (list) at points X.

    X is a list of ndim coordinate arrays.  Normal = gradient of the SDF; for
    the box inside region, the face of largest q = |x_b| - h wins (first axis
    on ties); sign(0) counts as +.
    """
    if getattr(body, "composite", False):
        return general_eval(body, X, t)
    ndim = len(X)
    c, P, theta, cdot, omega = motion(body, t)
    po = list(body.pivot_offset) + [0.0] * 3
    ct, st = np.cos(theta), np.sin(theta)
    rx = X[0] - P[0]
    ry = X[1] - P[1]
    # body frame coordinates
    xb = [ct * rx + st * ry + po[0], -st * rx + ct * ry + po[1]]
    if ndim == 3:
        xb.append(X[2] - P[2] + po[2])
    if body.kind == "sphere":
        r = np.sqrt(sum(v * v for v in xb))
        d = r - body.radius
        safe = np.where(r > 0, r, 1.0)
        nb = [np.where(r > 0, v / safe, 1.0 if k == 0 else 0.0) for k, v in enumerate(xb)]
    elif body.kind == "box":
        h = list(body.half_extent)
        q = [np.abs(xb[k]) - h[k] for k in range(ndim)]
        o = [np.maximum(qk, 0.0) for qk in q]
        olen = np.sqrt(sum(v * v for v in o))
        qmax = q[0]
        for k in range(1, ndim):
            qmax = np.maximum(qmax, q[k])
        d = olen + np.minimum(qmax, 0.0)
        sgn = [np.where(xb[k] >= 0, 1.0, -1.0) for k in range(ndim)]
        # inside: first axis attaining the max of q
        arg = np.zeros(d.shape, dtype=np.int64)
        best = q[0].copy()
        for k in range(1, ndim):
            better = q[k] > best
            arg = np.where(better, k, arg)
            best = np.where(better, q[k], best)
        outside = olen > 0
        safe = np.where(outside, olen, 1.0)
        nb = [np.where(outside, sgn[k] * o[k] / safe, np.where(arg == k, sgn[k], 0.0))
              for k in range(ndim)]
    elif body.kind == "grid":
        d, nb, Vs = grid_sdf(body, xb)
    else:
        raise ValueError("unknown body kind %r" % body.kind)
    # rotate the normal back to the world frame
    n = [ct * nb[0] - st * nb[1], st * nb[0] + ct * nb[1]]
    if ndim == 3:
        n.append(nb[2])
    V = [cdot[0] - omega * ry, cdot[1] + omega * rx]
    if ndim == 3:
        V.append(np.zeros_like(rx) + cdot[2])
    if body.kind == "grid" and Vs is not None:
        V = [V[k] + Vs[k] for k in range(ndim)]
    return d, n, V


def _trilinear(samples, u):
    """Multilinear interpolant of ``samples`` (indexed [i, j(, k)]) at fractional
    sample coordinates u (list of arrays, all inside [0, n-1])."""
    nd = len(u)
    shape = samples.shape
    i0 = [np.clip(np.floor(u[k]).astype(np.int64), 0, shape[k] - 2) for k in range(nd)]
    fr = [u[k] - i0[k] for k in range(nd)]
    out = np.zeros(np.shape(u[0]))
    for corner in range(1 << nd):
        wgt = np.ones(np.shape(u[0]))
        idx = []
        for k in range(nd):
            bit = (corner >> k) & 1
            wgt = wgt * (fr[k] if bit else 1.0 - fr[k])
            idx.append(i0[k] + bit)
        out = out + wgt * samples[tuple(idx)]
    return out


def grid_sdf(body, xb):
    """Signed distance, unit normal (body frame) and sampled velocity (list or None)
    of a gridded body at body-frame points xb (see the module docstring)."""
    nd = len(xb)
    s = np.asarray(body.sdf_grid, dtype=np.float64)
    if s.ndim != nd or min(s.shape) < 2:
        raise ValueError("sdf_grid must have ndim axes of at least 2 samples")
    h = float(body.grid_h)
    o = list(body.grid_origin) + [0.0] * 3
    u = [(np.asarray(xb[k], dtype=np.float64) - o[k]) / h for k in range(nd)]
    inside = np.ones(np.shape(u[0]), dtype=bool)
    for k in range(nd):
        inside &= (u[k] >= 0.0) & (u[k] <= s.shape[k] - 1)
    uc = [np.where(inside, u[k], 0.0) for k in range(nd)]
    d = np.where(inside, _trilinear(s, uc), np.inf)
    # per-sample gradient: central differences, one-sided at the edges
    grads = np.gradient(s, h, edge_order=1) if nd > 1 else [np.gradient(s, h, edge_order=1)]
    gn = [_trilinear(grads[k], uc) for k in range(nd)]
    mag = np.sqrt(sum(v * v for v in gn))
    ok = inside & (mag > 0)
    safe = np.where(ok, mag, 1.0)
    nb = [np.where(ok, gn[k] / safe, 1.0 if k == 0 else 0.0) for k in range(nd)]
    Vs = None
    if getattr(body, "vel_grid", None) is not None:
        vg = np.asarray(body.vel_grid, dtype=np.float64)
        Vs = [np.where(inside, _trilinear(vg[k], uc), 0.0) for k in range(nd)]
    return d, nb, Vs


# ---------------------------------------------------------------------------
# general bodies: complex-step derivatives of map and SDF, and their arithmetic
# ---------------------------------------------------------------------------
_CS = 1e-30  # complex step


def _cabs(z):
    return np.where(np.real(z) < 0, -z, z)


def _cmax_first(a, b):
    """max by real part; a tie keeps a."""
    return np.where(np.real(b) > np.real(a), b, a)


def part_map(part, X, t):
    """Body-frame coordinates x_b of world points X (list of ndim arrays) at time t.
    Complex inputs carry complex-step derivatives."""
    nd = len(X)
    _, P, theta, _, _ = motion(part, t)
    w = 2.0 * math.pi * part.freq
    sa = _vec3(getattr(part, "scale_amp", ()))
    S = [1.0 + sa[k] * np.sin(w * t + getattr(part, "phase_s", 0.0)) for k in range(3)]
    po = _vec3(part.pivot_offset)
    ct, st = np.cos(theta), np.sin(theta)
    rx = X[0] - P[0]
    ry = X[1] - P[1]
    xb = [S[0] * (ct * rx + st * ry) + po[0], S[1] * (-st * rx + ct * ry) + po[1]]
    if nd == 3:
        xb.append(S[2] * (X[2] - P[2]) + po[2])
    return xb


def shape_sdf(part, xb):
    """Signed distance of an analytic shape (before any hollowing), complex-capable."""
    nd = len(xb)
    if part.kind == "sphere":
        return np.sqrt(sum(v * v for v in xb)) - part.radius
    if part.kind == "box":
        h = _vec3(part.half_extent)
        q = [_cabs(xb[k]) - h[k] for k in range(nd)]
        o = [np.where(np.real(qk) > 0.0, qk, 0.0 * qk) for qk in q]
        olen = np.sqrt(sum(v * v for v in o))
        qmax = q[0]
        for k in range(1, nd):
            qmax = _cmax_first(qmax, q[k])
        # on a face (qmax = 0, no positive q) the inner branch is taken, so the
        # derivative there is the face normal, as the rigid formulas define it
        return olen + np.where(np.real(qmax) <= 0.0, qmax, 0.0 * qmax)
    if part.kind == "plane":
        nrm = _vec3(part.normal)[:nd]
        m = math.sqrt(sum(v * v for v in nrm))
        return sum((nrm[k] / m) * xb[k] for k in range(nd)) - part.radius
    raise ValueError("no analytic SDF for kind %r" % part.kind)


def part_general(part, X, t):
    """d, n, V of one part at world points X (general evaluation)."""
    nd = len(X)
    X = [np.asarray(x, dtype=np.float64) for x in X]
    xb = part_map(part, X, t)
    # J[j][k] = d x_b_j / d x_k and d x_b / dt by the complex step
    J = [[None] * nd for _ in range(nd)]
    for k in range(nd):
        Xk = [X[m] + (1j * _CS if m == k else 0.0) for m in range(nd)]
        xbk = part_map(part, Xk, t)
        for j in range(nd):
            J[j][k] = np.imag(xbk[j]) / _CS
    xbt = part_map(part, X, t + 1j * _CS)
    dxdt = [np.imag(v) / _CS for v in xbt]
    shell = float(getattr(part, "shell", 0.0))
    Vs = None
    if part.kind == "grid":
        dt_, nb, Vs = grid_sdf(part, xb)
        if shell > 0.0:
            sg = np.where(dt_ < 0.0, -1.0, 1.0)
            nb = [sg * v for v in nb]
            dt_ = np.abs(dt_) - shell
        g = [sum(J[j][k] * nb[j] for j in range(nd)) for k in range(nd)]
    else:
        def f(xx):
            v = shape_sdf(part, xx)
            return _cabs(v) - shell if shell > 0.0 else v
        dt_ = np.real(f(xb))
        g = []
        for k in range(nd):
            Xk = [X[m] + (1j * _CS if m == k else 0.0) for m in range(nd)]
            g.append(np.imag(f(part_map(part, Xk, t))) / _CS)
        if part.kind == "sphere":
            # the centre: the body-frame normal is e_x there (as for the rigid sphere)
            r0 = np.sqrt(sum(np.real(v) ** 2 for v in xb)) == 0.0
            if np.any(r0):
                nb0 = [1.0 if j == 0 else 0.0 for j in range(nd)]
                sg = 1.0
                g = [np.where(r0, sg * sum(J[j][k] * nb0[j] for j in range(nd)), g[k]) for k in range(nd)]
    gm = np.sqrt(sum(v * v for v in g))
    ok = gm > 0.0
    safe = np.where(ok, gm, 1.0)
    d = np.where(ok, dt_ / safe, dt_)
    n = [np.where(ok, g[k] / safe, 1.0 if k == 0 else 0.0) for k in range(nd)]
    # V = -J^{-1} dx_b/dt, point by point
    Jm = np.stack([np.stack([np.broadcast_to(J[j][k], d.shape) for k in range(nd)], axis=-1)
                   for j in range(nd)], axis=-2)
    rhs = np.stack([np.broadcast_to(v, d.shape) for v in dxdt], axis=-1)[..., None]
    sol = np.linalg.solve(Jm, rhs)[..., 0]
    V = [-sol[..., k] for k in range(nd)]
    if Vs is not None:
        V = [V[k] + Vs[k] for k in range(nd)]
    return d, n, V


def general_eval(body, X, t):
    """d, n, V of a chain of parts combined by signed-distance arithmetic."""
    parts = body.parts()
    d, n, V = part_general(parts[0], X, t)
    for p in parts[1:]:
        db, nb, Vb = part_general(p, X, t)
        if p.op == "union":
            take = db < d
        elif p.op == "intersect":
            take = db > d
        elif p.op == "subtract":
            db = -db
            nb = [-v for v in nb]
            take = db > d
        else:
            raise ValueError("unknown op %r" % p.op)
        d = np.where(take, db, d)
        n = [np.where(take, nb[k], n[k]) for k in range(len(n))]
        V = [np.where(take, Vb[k], V[k]) for k in range(len(V))]
    return d, n, V


def face_points(grid, comp):
    axes = []
    for a, N in enumerate(grid.n):
        I = np.arange(N + 2, dtype=np.float64)
        axes.append(I - 1.0 if a == comp else I - 0.5)
    return np.meshgrid(*axes, indexing="ij")


def cell_points(grid):
    axes = [np.arange(N + 2, dtype=np.float64) - 0.5 for N in grid.n]
    return np.meshgrid(*axes, indexing="ij")


def measure(grid, body, t, eps=1.0):
    """mu0 (list n), mu1 (list n of lists n), V (list n) on every padded face.

    mu0_i = mu0(d), mu1_ij = mu1(d) n_j, V_i = body velocity where d < 2 + eps
    else 0.  Faces with mu0 < MU0_CUT are solid: mu0 = mu1 = 0 there.
    Without a body: mu0 = 1, mu1 = 0, V = 0.
    """
    nd = grid.ndim
    if body is None or body.kind == "none":
        m0 = [np.ones(grid.shape) for _ in range(nd)]
        m1 = [[np.zeros(grid.shape) for _ in range(nd)] for _ in range(nd)]
        V = [np.zeros(grid.shape) for _ in range(nd)]
        return m0, m1, V
    m0, m1, V = [], [], []
    for i in range(nd):
        X = face_points(grid, i)
        d, n, Vb = sdf_normal_velocity(body, X, t)
        a0 = mu0(d, eps)
        a1 = mu1(d, eps)
        solid = a0 < MU0_CUT
        a0 = np.where(solid, 0.0, a0)
        a1 = np.where(solid, 0.0, a1)
        m0.append(a0)
        m1.append([a1 * n[j] for j in range(nd)])
        V.append(np.where(d < 2.0 + eps, Vb[i], 0.0))
    return m0, m1, V


def forces(grid, body, t, u, p, nu, eps=1.0, active=None):
    """Pressure and viscous force on the body (FP64 sums over interior cells).

    Surface integrals become volume sums weighted by the smoothed delta
    K_eps(d) at the cell centres:  F_p = -sum (p - pbar) n K_eps,
    F_v = sum 2 nu S n K_eps with S = (grad u + grad u^T)/2 from central
    differences at the cell centre (face values averaged to the centre).
    The pressure is defined up to a constant; pbar is its mean over the
    cells passed as ``active`` (all interior cells if None), which fixes the gauge.
    """
    nd = grid.ndim
    Xc = cell_points(grid)
    d, n, _ = sdf_normal_velocity(body, Xc, t)
    w = kernel_eps(d, eps)
    inner = grid.interior_mask()
    w = np.where(inner, w, 0.0)
    act = inner if active is None else active
    p = p - np.mean(p[act])
    Fp = np.array([-np.sum(p * n[i] * w) for i in range(nd)])
    # velocity gradient at cell centres: G[i][j] = d u_i / d x_j
    G = [[None] * nd for _ in range(nd)]
    for i in range(nd):
        ui = u[i]
        up = grid.sh(ui, i, +1)
        ubar = 0.5 * (ui + up)            # u_i averaged to the cell centre
        for j in range(nd):
            if j == i:
                G[i][j] = up - ui
            else:
                G[i][j] = 0.5 * (grid.sh(ubar, j, +1) - grid.sh(ubar, j, -1))
    Fv = np.zeros(nd, dtype=np.result_type(u[0], p, w))
    for i in range(nd):
        acc = np.zeros(grid.shape)
        for j in range(nd):
            S = 0.5 * (G[i][j] + G[j][i])
            acc = acc + S * n[j]
        Fv[i] = np.sum(2.0 * nu * acc * w)
    return Fp, Fv
