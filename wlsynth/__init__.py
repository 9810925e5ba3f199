"""Seeded synthetic inputs shared by the oracle and the HIP path.

This module holds no arithmetic of the solver itself: only the workload
descriptions (grid sizes, viscosity, body geometry and motion parameters),
a counter-based random generator, and closed-form initial velocity fields
sampled at the staggered face positions.

Layout convention used by every array produced here (numpy, float64):
component ``i`` of a velocity field is an array of shape ``(N0+2, N1+2[, N2+2])``
indexed ``[I0, I1, I2]`` over the padded grid (one ghost layer per side).
Cell ``I`` has its centre at ``x = I - 1/2`` (grid units, h = 1) and
``u_i[I]`` sits on the lower ``i``-face of cell ``I``, i.e. at ``x_i = I_i - 1``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence, Tuple

import numpy as np

# ---------------------------------------------------------------------------
# counter-based SplitMix64 (Steele, Lea & Flood 2014, "Fast splittable
# pseudorandom number generators"); state_k = seed + (k+1)*gamma, then the
# published 64-bit finaliser.
# ---------------------------------------------------------------------------
_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(counter: np.ndarray, seed: int = 0) -> np.ndarray:
    """64-bit SplitMix64 output for each counter value (uint64 array)."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (counter.astype(np.uint64) + np.uint64(1)) * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(counter: np.ndarray, seed: int = 0) -> np.ndarray:
    """Doubles in [0, 1) from the top 53 bits of SplitMix64."""
    return (splitmix64(counter, seed) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def face_noise(shape: Sequence[int], comp: int, amp: float, seed: int = 0) -> np.ndarray:
    """iid U[-amp, amp) per (component, padded linear index), x fastest."""
    shape = tuple(int(s) for s in shape)
    size = int(np.prod(shape))
    # linear index with axis 0 (x) fastest
    lin = np.arange(size, dtype=np.uint64).reshape(shape[::-1]).T
    counter = np.uint64(comp) * np.uint64(size) + lin
    return (2.0 * uniform01(counter, seed) - 1.0) * amp


# ---------------------------------------------------------------------------
# bodies and workloads
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class Body:
    """One part of a body (the fields mirror ``wl_body_desc``).

    ``kind`` is 'none', 'sphere' (circle in 2-D), 'box', 'grid' or 'plane'.

    Map of the part from world to body frame:
    x_b = S(t) * Rot(-theta(t)) (x - P(t)) + pivot_offset, with
    P(t) = center + velocity*t + heave_amp*sin(2 pi freq t + phase_h) e_h + pivot_offset
    (e_h = heave_dir normalised, e_y when zero), theta(t) = pitch_amp*sin(2 pi freq t +
    phase_p) + spin_omega*t about e_z, S_a(t) = 1 + scale_amp[a]*sin(2 pi freq t + phase_s).

    'grid': the signed distance is sampled in the body frame, sample (i, j[, k]) of
    ``sdf_grid`` (numpy, indexed [i, j(, k)], x first) sitting at
    ``grid_origin + (i, j, k) * grid_h``; ``vel_grid`` (optional, shape (ndim,) +
    sdf_grid.shape) adds a sampled velocity to the map's.  'plane': the half space
    normal . x_b - radius <= 0.  ``shell`` > 0 makes the part hollow.

    Parts chain through ``next``; each later part combines with the ones before it
    by ``op`` ('union', 'intersect', 'subtract').
    """
    kind: str = "none"
    center: Tuple[float, ...] = (0.0, 0.0, 0.0)
    radius: float = 0.0
    half_extent: Tuple[float, ...] = (0.0, 0.0, 0.0)
    heave_amp: float = 0.0
    pitch_amp: float = 0.0
    freq: float = 0.0
    phase_h: float = 0.0
    phase_p: float = 0.0
    pivot_offset: Tuple[float, ...] = (0.0, 0.0, 0.0)
    spin_omega: float = 0.0
    velocity: Tuple[float, ...] = (0.0, 0.0, 0.0)
    heave_dir: Tuple[float, ...] = (0.0, 0.0, 0.0)
    scale_amp: Tuple[float, ...] = (0.0, 0.0, 0.0)
    phase_s: float = 0.0
    normal: Tuple[float, ...] = (0.0, 0.0, 0.0)
    shell: float = 0.0
    sdf_grid: Optional[np.ndarray] = None
    vel_grid: Optional[np.ndarray] = None
    grid_origin: Tuple[float, ...] = (0.0, 0.0, 0.0)
    grid_h: float = 1.0
    op: str = "union"
    next: Optional["Body"] = None

    def parts(self):
        """The chain of parts starting here."""
        out, b = [], self
        while b is not None:
            out.append(b)
            b = b.next
        return out

    def _part_moving(self) -> bool:
        return (self.heave_amp != 0.0 or self.pitch_amp != 0.0 or self.spin_omega != 0.0
                or any(v != 0.0 for v in self.velocity)
                or (self.freq != 0.0 and any(v != 0.0 for v in self.scale_amp)))

    @property
    def moving(self) -> bool:
        return self.kind != "none" and any(p._part_moving() for p in self.parts())

    @property
    def composite(self) -> bool:
        """True when the body needs the general evaluation (several parts, a plane, a
        hollow part or a scaled map)."""
        for p in self.parts():
            if p.kind == "plane" or p.shell != 0.0 or any(v != 0.0 for v in p.scale_amp):
                return True
        return self.next is not None


def combine(first: Body, *rest) -> Body:
    """A body made of ``first`` and the (op, part) pairs of ``rest`` in order; the parts
    are copied so the arguments stay unchained."""
    head = dataclasses.replace(first, next=None)
    tail = head
    for op, part in rest:
        nxt = dataclasses.replace(part, op=op, next=None)
        tail.next = nxt
        tail = nxt
    return head


@dataclasses.dataclass
class Workload:
    name: str
    n: Tuple[int, ...]                 # interior cells per axis (x first)
    U: Tuple[float, ...]               # free-stream velocity
    nu: float
    body: Body = dataclasses.field(default_factory=Body)
    periodic: Tuple[bool, ...] = ()
    convective_exit: bool = False
    steps: int = 100
    tol: float = 1e-6
    noise: float = 1e-3                # amplitude relative to |U|
    init: str = "uniform"              # 'uniform' or 'tgv'
    L: float = 1.0                     # length scale used for coefficients

    @property
    def ndim(self) -> int:
        return len(self.n)

    @property
    def cells(self) -> int:
        return int(np.prod(self.n))

    def periodic_mask(self) -> Tuple[bool, ...]:
        if self.periodic:
            return tuple(self.periodic)
        return tuple(False for _ in self.n)


def circle_2d(n=(128, 64), R=8.0, center=(32.0, 32.0), Re=250.0, steps=100, tol=1e-6) -> Workload:
    """2-D circle in uniform inflow (the small parity case)."""
    D = 2 * R
    return Workload("circle2d_%dx%d" % tuple(n), tuple(n), (1.0, 0.0), D / Re,
                    Body("sphere", center=tuple(center), radius=R), steps=steps, tol=tol, L=D)


def tgv_3d(N=128, Re=1600.0, steps=500, tol=1e-6) -> Workload:
    """Periodic Taylor-Green vortex box, kappa = 2 pi / N, U = 1, Re = U/(kappa nu)."""
    kappa = 2 * math.pi / N
    return Workload("tgv3d_%d" % N, (N, N, N), (0.0, 0.0, 0.0), 1.0 / (kappa * Re),
                    periodic=(True, True, True), steps=steps, tol=tol, noise=0.0, init="tgv",
                    L=N / (2 * math.pi))


def tgv_sym_3d(N=512, Re=1600.0, steps=100, tol=1e-5) -> Workload:
    """Taylor-Green vortex on the symmetric subdomain (one eighth of the periodic
    box of side 2N): N^3 cells spanning [0, pi/kappa]^3 with kappa = pi / N, symmetry
    (slip, U = 0) on every face, the paper's signs u = -sin cos cos, v = cos sin cos,
    w = 0, U = 1, Re = U / (kappa nu)."""
    kappa = math.pi / N
    return Workload("tgvsym3d_%d" % N, (N, N, N), (0.0, 0.0, 0.0), 1.0 / (kappa * Re),
                    periodic=(False, False, False), steps=steps, tol=tol, noise=0.0, init="tgv_sym",
                    L=1.0 / kappa)


def sphere_3d(n=(256, 128, 128), D=32.0, center=(64.0, 64.0, 64.0), Re=3700.0, steps=1000,
              tol=1e-6) -> Workload:
    return Workload("sphere3d_%dx%dx%d" % tuple(n), tuple(n), (1.0, 0.0, 0.0), D / Re,
                    Body("sphere", center=tuple(center), radius=D / 2), convective_exit=True,
                    steps=steps, tol=tol, L=D)


def rotating_cylinder_2d(n=(512, 256), D=32.0, center=(128.0, 128.0), Re=200.0, xi=1.0,
                         steps=400, tol=1e-12) -> Workload:
    """Rotation rate xi = (1/2) D Omega / U (counter-clockwise)."""
    omega = 2.0 * xi * 1.0 / D
    return Workload("rotcyl2d_%dx%d" % tuple(n), tuple(n), (1.0, 0.0), D / Re,
                    Body("sphere", center=tuple(center), radius=D / 2, spin_omega=omega),
                    steps=steps, tol=tol, L=D)


def rotcyl_xi0(seed: int = 0) -> float:
    """Seeded rotation rate in [0, 2) for the rotating-cylinder gradient case."""
    return 2.0 * float(uniform01(np.array([0], dtype=np.uint64), seed=seed)[0])


def plate_3d(scale: int = 1, steps=200, tol=1e-5) -> Workload:
    """Heaving-pitching flat plate; scale=1 is 768x384x384 cells (113 M).

    Chord c = 64/scale, thickness 4/scale (min 2), span 2c, heave 0.25 c,
    pitch 20 degrees about the quarter chord, pitch leading heave by 90 degrees,
    Strouhal f (2 h0)/U = 0.3, Re = U c / nu = 5000.
    """
    n = (768 // scale, 384 // scale, 384 // scale)
    c = 64.0 / scale
    th = max(4.0 / scale, 2.0)
    h0 = 0.25 * c
    f = 0.3 / (2 * h0)
    ctr = (n[0] / 4.0, n[1] / 2.0, n[2] / 2.0)
    body = Body("box", center=ctr, half_extent=(c / 2, th / 2, c), heave_amp=h0,
                pitch_amp=math.radians(20.0), freq=f, phase_h=0.0, phase_p=math.pi / 2,
                pivot_offset=(-c / 4, 0.0, 0.0))
    return Workload("plate3d_%dx%dx%d" % n, n, (1.0, 0.0, 0.0), c / 5000.0, body,
                    convective_exit=True, steps=steps, tol=tol, L=c)


def jelly_3d(n: int = 32, Re: float = 500.0, U: float = 1.0, steps: int = 100, tol: float = 1e-6) -> Workload:
    """A pulsing jellyfish-like bell (paper, applications section: a hollow sphere
    whose map scales x and y harmonically and heaves it along z, minus a half space
    that moves with the same heave), in a downward stream -U e_z.  Radius R = 2n/3,
    shell half thickness 1, angular frequency 2U/R, scale amplitude 0.1.  The bell
    is centred in x and y of a (3n, 3n, 4n + n/2) box instead of on the corner of a
    quarter domain with symmetry planes (the margins keep the reach of the pulsing
    bell clear of the side and top faces)."""
    R = 2.0 * n / 3.0
    hgt = 4.0 * n - 2.0 * R
    w = 2.0 * U / R
    f = w / (2.0 * math.pi)
    cx = cy = 1.5 * n
    # sphere: x_b = A(t) (x - P) with A_xy = 1 - 0.1 cos(w t) and the centre at
    # P_z = hgt + R/4 - (R/4)(cos w t + sin w t)
    bell = Body("sphere", center=(cx, cy, hgt + R / 4.0), radius=R, shell=1.0,
                scale_amp=(0.1, 0.1, 0.0), phase_s=-math.pi / 2.0, freq=f,
                heave_amp=math.sqrt(2.0) * R / 4.0, heave_dir=(0.0, 0.0, -1.0), phase_h=math.pi / 4.0)
    # half space z_b > 0 removed, its plane at P_z = hgt - (R/4) sin w t
    cut = Body("plane", center=(cx, cy, hgt), normal=(0.0, 0.0, 1.0), freq=f,
               heave_amp=R / 4.0, heave_dir=(0.0, 0.0, -1.0))
    body = combine(bell, ("subtract", cut))
    nz = 4 * n + n // 2
    return Workload("jelly3d_%dx%dx%d" % (3 * n, 3 * n, nz), (3 * n, 3 * n, nz), (0.0, 0.0, -U),
                    U * R / Re, body, steps=steps, tol=tol, L=R)


def sampled_sdf(fn, half_width: float, h: float, ndim: int):
    """Samples of a body-frame signed distance ``fn(list of coordinate arrays)`` on the
    grid origin + (i, j, k) h covering [-half_width, half_width]^ndim.  Returns
    (samples indexed [i, j(, k)], origin tuple)."""
    n = int(math.ceil(2.0 * half_width / h)) + 1
    origin = -0.5 * (n - 1) * h
    ax = origin + h * np.arange(n, dtype=np.float64)
    X = np.meshgrid(*([ax] * ndim), indexing="ij")
    return np.ascontiguousarray(fn(X), dtype=np.float64), (origin,) * ndim


def grid_sphere_body(R: float, h: float, ndim: int, center, margin: float = 5.0, **motion) -> Body:
    """A 'grid' body holding samples of the sphere (circle) distance |x_b| - R."""
    sdf, origin = sampled_sdf(lambda X: np.sqrt(sum(x * x for x in X)) - R, R + margin, h, ndim)
    return Body("grid", center=tuple(center), sdf_grid=sdf, grid_origin=origin, grid_h=h, **motion)


# ---------------------------------------------------------------------------
# initial velocity fields (inputs, sampled at face positions)
# ---------------------------------------------------------------------------
def face_coords(n: Sequence[int], comp: int):
    """Coordinates of the padded face points of component ``comp``."""
    axes = []
    for a, N in enumerate(n):
        I = np.arange(N + 2, dtype=np.float64)
        axes.append(I - 1.0 if a == comp else I - 0.5)
    return np.meshgrid(*axes, indexing="ij")


def initial_velocity(w: Workload, seed: int = 0):
    """Initial face velocities (list of padded float64 arrays).

    'uniform': u = U + U[-1e-3, 1e-3)*|U| iid noise (seeded SplitMix64).
    'tgv': u = sin(kx)cos(ky)cos(kz), v = -cos(kx)sin(ky)cos(kz), w = 0, k = 2 pi / N.
    'tgv_sym': the same mode with the opposite signs and k = pi / N (the grid is one
    eighth of the periodic box).
    """
    shape = tuple(N + 2 for N in w.n)
    out = []
    if w.init in ("tgv", "tgv_sym"):
        k = (math.pi if w.init == "tgv_sym" else 2 * math.pi) / w.n[0]
        sg = -1.0 if w.init == "tgv_sym" else 1.0
        for i in range(w.ndim):
            X = face_coords(w.n, i)
            if i == 0:
                f = sg * np.sin(k * X[0]) * np.cos(k * X[1])
            elif i == 1:
                f = -sg * np.cos(k * X[0]) * np.sin(k * X[1])
            else:
                f = np.zeros(shape)
            if w.ndim == 3 and i < 2:
                f = f * np.cos(k * X[2])
            out.append(np.ascontiguousarray(f))
        return out
    Umag = math.sqrt(sum(u * u for u in w.U))
    for i in range(w.ndim):
        f = np.full(shape, float(w.U[i]))
        if w.noise > 0:
            f = f + face_noise(shape, i, w.noise * Umag, seed)
        out.append(f)
    return out


def tgv2d_exact(n: int, nu: float, t: float, U: float = 1.0):
    """2-D Taylor-Green closed form at the face points of a periodic n x n grid."""
    k = 2 * math.pi / n
    F = math.exp(-2 * nu * k * k * t)
    X0 = face_coords((n, n), 0)
    X1 = face_coords((n, n), 1)
    u = U * np.sin(k * X0[0]) * np.cos(k * X0[1]) * F
    v = -U * np.cos(k * X1[0]) * np.sin(k * X1[1]) * F
    return [u, v]


def random_field(shape, seed: int, comp: int = 0, amp: float = 1.0):
    """Generic seeded test field U[-amp, amp)."""
    return face_noise(shape, comp, amp, seed)


# ---------------------------------------------------------------------------
# initial weights of the learned multigrid guess (an input: drawn here, used by
# both the oracle and the HIP path)
# ---------------------------------------------------------------------------
PG_SHAPES = [(27, 3, 16), (16,), (27, 16, 16), (16,), (27, 16, 1), (1,)]


def pg_init_weights(seed: int = 0, zero_output: bool = False) -> np.ndarray:
    """Kaiming-uniform weights (bound sqrt(6 / fan_in), fan_in = 27 c_in), zero biases,
    flat float32 in the order W1 b1 W2 b2 W3 b3 with W[tap][c_in][c_out].
    zero_output: W3 = 0, so the untrained net predicts no change (the plain warm start)."""
    parts = []
    k = 0
    for li, shp in enumerate(PG_SHAPES):
        n = int(np.prod(shp))
        if len(shp) == 3 and zero_output and li == len(PG_SHAPES) - 2:
            parts.append(np.zeros(n, dtype=np.float32))
        elif len(shp) == 3:
            bound = float(np.sqrt(6.0 / (27 * shp[1])))
            counter = np.arange(k, k + n, dtype=np.uint64)
            parts.append(((2.0 * uniform01(counter, seed + 12345) - 1.0) * bound).astype(np.float32))
        else:
            parts.append(np.zeros(n, dtype=np.float32))
        k += n
    return np.concatenate(parts)


def pg_split(flat):
    """Flat parameter vector -> [W1, b1, W2, b2, W3, b3] float64 arrays."""
    out = []
    k = 0
    for shp in PG_SHAPES:
        n = int(np.prod(shp))
        out.append(np.asarray(flat[k:k + n], dtype=np.float64).reshape(shp))
        k += n
    return out
