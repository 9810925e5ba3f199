"""Convection-diffusion residual R(u) with the limited QUICK scheme (test infrastructure).

The paper's numerical-methods section: finite volumes on the staggered grid,
second-order central differences for diffusion, a flux-limited QUICK scheme
for convection, no explicit turbulence model.

For component i, the control volume of face u_i[I] has, on its lower side
along j, the flux

    Phi_ij[I] = a_ij Q_lim - nu (u_i[I] - u_i[I - e_j]),
    a_ij      = (u_j[I] + u_j[I - e_i]) / 2          (advecting velocity)

and R_i[I] = sum_j (Phi_ij[I] - Phi_ij[I + e_j]) on the unknown faces; R = 0
elsewhere.  Q_lim uses the upwind triple (far, c, d) along j: for a >= 0,
(u_i[I-2e_j], u_i[I-e_j], u_i[I]); for a < 0, (u_i[I+e_j], u_i[I], u_i[I-e_j]).
Reading of "flux-limited QUICK": the kappa = 1/3 upwind-biased face value
q = (5c + 2d - far)/6 clamped by a median-form universal limiter,
Q_lim = median(c, q, median(c, d, c + 9 (c - far))).  The far point must lie
inside the domain on a non-periodic axis j (cells 1..N_j when j != i, faces
1..N_j+1 when j == i, i.e. no ghost value); otherwise the central average
(u_i[I] + u_i[I-e_j])/2 is used.  This keeps the scheme mirror-symmetric at
the two ends of every axis.
"""
from __future__ import annotations

import numpy as np


def median3(a, b, c):
    return np.maximum(np.minimum(a, b), np.minimum(np.maximum(a, b), c))


def quick_limited(far, c, d):
    q = (5.0 * c + 2.0 * d - far) / 6.0
    return median3(c, q, median3(c, d, c + 9.0 * (c - far)))


def far_valid(grid, i, j, k):
    """Is I + k e_j inside the domain for component i (see module docstring)?"""
    N = grid.n[j]
    shp = [1] * grid.ndim
    shp[j] = -1
    if grid.periodic[j]:
        ok = np.ones(N + 2, dtype=bool)
    else:
        I = np.arange(N + 2) + k
        ok = (I >= 1) & (I <= (N + 1 if j == i else N))
    return np.broadcast_to(ok.reshape(shp), grid.shape)


def flux_ij(grid, u, i, j, nu):
    """Phi_ij at every padded index (entries never used by R may be garbage)."""
    a = 0.5 * (u[j] + grid.sh(u[j], i, -1))
    ui = u[i]
    m1 = grid.sh(ui, j, -1)
    m2 = grid.sh(ui, j, -2)
    p1 = grid.sh(ui, j, +1)
    v2 = far_valid(grid, i, j, -2)
    v1 = far_valid(grid, i, j, +1)
    up = a >= 0.0
    far = np.where(up, m2, p1)
    c = np.where(up, m1, ui)
    d = np.where(up, ui, m1)
    ok = np.where(up, v2, v1)
    Q = np.where(ok, quick_limited(far, c, d), 0.5 * (ui + m1))
    return a * Q - nu * (ui - m1)


def conv_diff(grid, u, nu):
    """R_i on the unknown faces of every component (list of padded arrays)."""
    R = []
    for i in range(grid.ndim):
        acc = grid.zeros()
        for j in range(grid.ndim):
            phi = flux_ij(grid, u, i, j, nu)
            acc = acc + (phi - grid.sh(phi, j, +1))
        R.append(np.where(grid.unknown_mask(i), acc, 0.0))
    return R
