"""Pins of the multigrid Poisson solve: dense direct solve, FFT solve, invariants."""
import itertools

import numpy as np
import pytest

import wlsynth
from oracle import Grid
from oracle import poisson as P
from oracle.body import measure
from oracle.solver import Sim


def _levels(n, periodic, body=None):
    g = Grid(n, periodic)
    m0, _, _ = measure(g, body, 0.0)
    L = P.boundary_zeroed(g, m0)
    return g, P.build_levels(g, L)


def _dense_matrix(g, L):
    """Assemble A cell by cell from the flux-form definition (pure Python)."""
    nd = g.ndim
    cells = list(itertools.product(*[range(1, N + 1) for N in g.n]))
    index = {c: k for k, c in enumerate(cells)}
    A = np.zeros((len(cells), len(cells)))
    for c in cells:
        row = index[c]
        for i in range(nd):
            for s in (+1, -1):
                nb = list(c)
                nb[i] += s
                face = list(c)
                if s > 0:
                    face[i] += 1          # upper face of c is the lower face of c + e_i
                coef = L[i][tuple(face)]
                if g.periodic[i]:
                    nb[i] = 1 + (nb[i] - 1) % g.n[i]
                elif not 1 <= nb[i] <= g.n[i]:
                    assert coef == 0.0
                    continue
                A[row, index[tuple(nb)]] += coef
                A[row, row] -= coef
    return cells, A


@pytest.mark.parametrize("n,body", [
    ((8, 8), wlsynth.Body("sphere", center=(4.0, 4.2), radius=1.7)),
    ((16, 12), wlsynth.Body("sphere", center=(7.3, 6.0), radius=3.5)),
    ((8, 8, 8), wlsynth.Body("sphere", center=(4.0, 4.0, 4.3), radius=2.2)),
    ((8, 8, 8), wlsynth.Body("box", center=(4.0, 4.0, 4.0), half_extent=(1.5, 2.5, 1.0),
                              pitch_amp=0.3, phase_p=1.0, freq=0.1)),
])
def test_multigrid_matches_dense_solve(n, body):
    g, levels = _levels(n, None, body)
    cells, A = _dense_matrix(g, levels[0].L)
    active = np.array([levels[0].active[c] for c in cells])
    # masked rows of the dense matrix are exactly the decoupled solid cells
    assert np.all(A[~active][:, active] == 0) and np.all(A[active][:, ~active] == 0)
    rng = np.random.default_rng(5)
    zv = rng.normal(size=len(cells)) * active
    zv[active] -= zv[active].mean()
    Aa = A[np.ix_(active, active)]
    xa = np.linalg.lstsq(Aa, zv[active], rcond=None)[0]
    z = g.zeros()
    for k, c in enumerate(cells):
        z[c] = zv[k]
    x = g.zeros()
    st = P.solve(levels, x, z, tol=1e-13, itmax=200)
    assert st["converged"]
    xm = np.array([x[c] for c in cells])[active]
    np.testing.assert_allclose(xm - xm.mean(), xa - xa.mean(), atol=1e-10)
    # the dense operator equals apply_A on a random vector
    v = g.zeros()
    v[g.interior()] = rng.normal(size=g.n)
    Av = P.apply_A(levels[0], v)
    dv = A @ np.array([v[c] for c in cells])
    np.testing.assert_allclose(np.array([Av[c] for c in cells])[active], dv[active], atol=1e-12)


def test_periodic_constant_coefficient_matches_fft():
    N = 32
    g, levels = _levels((N, N, N), (True, True, True))
    rng = np.random.default_rng(9)
    zi = rng.normal(size=(N, N, N))
    zi -= zi.mean()
    z = g.zeros()
    z[g.interior()] = zi
    x = g.zeros()
    st = P.solve(levels, x, z, tol=1e-12, itmax=100)
    assert st["converged"]
    k = np.fft.fftfreq(N) * N
    s = [4 * np.sin(np.pi * kk / N) ** 2 for kk in np.meshgrid(k, k, k, indexing="ij")]
    lam = -(s[0] + s[1] + s[2])
    lam[0, 0, 0] = 1.0
    xh = np.fft.fftn(zi) / lam
    xh[0, 0, 0] = 0.0
    xf = np.real(np.fft.ifftn(xh))
    xs = x[g.interior()]
    np.testing.assert_allclose(xs - xs.mean(), xf, atol=1e-10)


def test_operator_symmetric_and_negative():
    body = wlsynth.Body("sphere", center=(8.0, 6.0), radius=3.1)
    g, levels = _levels((16, 12), None, body)
    rng = np.random.default_rng(1)
    a, b = g.zeros(), g.zeros()
    a[g.interior()] = rng.normal(size=g.n)
    b[g.interior()] = rng.normal(size=g.n)
    act = levels[0].active
    a *= act
    b *= act
    lev = levels[0]
    assert abs(P.dot(P.apply_A(lev, a), b) - P.dot(a, P.apply_A(lev, b))) < 1e-12
    assert P.dot(P.apply_A(lev, a), a) < 0


@pytest.mark.parametrize("n,periodic", [((7, 6, 5), (False, True, False)), ((9, 7), (True, False))])
def test_energy_is_minus_the_face_sum(n, periodic):
    """e.Ae = -sum over faces of L_f (e_i - e_j)^2 on every level: A holds the face
    coefficients off the diagonal and minus their sum on it.  Faces are walked one by
    one (a periodic axis closes through face 1, a non-periodic boundary face has
    L = 0); the GPU's sigma pass of the PCG smoother sums this form."""
    nd = len(n)
    body = wlsynth.Body("sphere", center=tuple(0.5 * N + 0.3 for N in n), radius=1.9)
    g, levels = _levels(n, periodic, body)
    rng = np.random.default_rng(7)
    for lev in levels:
        gl = lev.grid
        e = gl.zeros()
        e[gl.interior()] = rng.normal(size=gl.n)
        lhs = P.dot(P.apply_A(lev, e), e)
        rhs = 0.0
        for c in itertools.product(*[range(1, N + 1) for N in gl.n]):
            for i in range(nd):
                lo = list(c)
                lo[i] -= 1                # face c along i joins cell c - e_i and cell c
                if lo[i] == 0:
                    if not gl.periodic[i]:
                        assert lev.L[i][c] == 0.0
                        continue
                    lo[i] = gl.n[i]
                rhs -= lev.L[i][c] * (e[c] - e[tuple(lo)]) ** 2
        assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(rhs)), (gl.n, lhs, rhs)


def test_coarse_coefficients_rediscretise_constant_L():
    # constant L = 1 -> coarse interior L = 2^(n-2)
    for n in [(16, 8), (8, 8, 8)]:
        g, levels = _levels(n, None)
        nd = len(n)
        for lev in levels[1:]:
            gc = lev.grid
            for i in range(nd):
                sl = [slice(1, N + 1) for N in gc.n]
                sl[i] = slice(2, gc.n[i] + 1)
                np.testing.assert_array_equal(lev.L[i][tuple(sl)], 2.0 ** (nd - 2))
                sl[i] = 1
                assert np.all(lev.L[i][tuple(sl)] == 0)


def test_level_counts():
    for n, k in [((128, 64), 5), ((128, 128, 128), 6), ((256, 128, 128), 6), ((512, 256), 7)]:
        g = Grid(n)
        cnt = 1
        while g.coarsenable():
            g = g.coarse()
            cnt += 1
        assert cnt == k


def test_projection_leaves_divergence_below_tolerance():
    w = wlsynth.circle_2d(n=(64, 32), R=5.0, center=(16.0, 16.0))
    s = Sim(w.n, w.U, w.nu, w.body, tol=1e-9)
    # solid faces (mu0 = 0) carry the body velocity 0, as after the BDIM blend
    u = [(wlsynth.random_field(s.grid.shape, seed=4, comp=i, amp=0.2) + w.U[i]) * s.mu0[i]
         for i in range(2)]
    s.set_velocity(u)
    s.dt = 0.3
    st = s.project(1.0)
    assert st["converged"]
    z = P.divergence(s.grid, s.u)
    assert np.abs(z[s.levels[0].active]).max() < 1e-9
    # the multigrid convergence factor per cycle is below 0.5 here
    assert st["vcycles"] <= 30
