"""Helpers shared by the GPU parity tests (the HIP path vs the FP64 oracle)."""
import math

import numpy as np

import oracle
import wlsynth

# parity bars (rel-L2 of velocity over the interior faces)
FP64_STEP = 1e-12
FP32_STEP = 1e-5
FP32_10STEP = 1e-4
CD_REL = 5e-3


def small_cases():
    """Small workloads the oracle finishes in seconds (shapes of the paper's cases)."""
    circle = wlsynth.circle_2d()                                       # 128 x 64, R = 8
    sphere = wlsynth.sphere_3d(n=(64, 32, 32), D=12.0, center=(16.0, 16.0, 16.0))
    tgv = wlsynth.tgv_3d(N=32)
    plate = wlsynth.plate_3d(scale=8)                                  # 96 x 48 x 48, moving
    rot = wlsynth.rotating_cylinder_2d(n=(96, 48), D=12.0, center=(30.0, 24.0), xi=1.0)
    # 64^3 = 2^18 cells: the fine level runs the tiled (z-marching) multigrid kernels,
    # with tiles both inside and outside the body box (sphere) and periodic wraps (TGV)
    sphere_t = wlsynth.sphere_3d(n=(64, 64, 64), D=16.0, center=(24.0, 32.0, 32.0))
    tgv_t = wlsynth.tgv_3d(N=64)
    return {"circle2d": circle, "sphere3d": sphere, "tgv3d": tgv, "plate3d": plate, "rotcyl2d": rot,
            "sphere3d_tiled": sphere_t, "tgv3d_tiled": tgv_t}


def make_pair(w, prec, tol, itmax=200, seed=0, solver_path="auto"):
    from paper_2407_16032_amd import Simulation
    u0 = wlsynth.initial_velocity(w, seed=seed)
    body = w.body if w.body.kind != "none" else None
    ref = oracle.Sim(w.n, w.U, w.nu, body, periodic=w.periodic_mask(),
                     convective_exit=w.convective_exit, tol=min(tol, 1e-12), itmax=itmax)
    ref.set_velocity(u0)
    gpu = Simulation(w.n, w.U, w.nu, body, periodic=w.periodic_mask(), convective_exit=w.convective_exit,
                     prec=prec, tol=tol, itmax=itmax, device="cuda:0", solver_path=solver_path)
    gpu.set_velocity(u0)
    return ref, gpu


def rel_l2(got, ref, grid, comps=None):
    comps = range(grid.ndim) if comps is None else comps
    I = grid.interior()
    num = sum(float(np.sum((got[i][I] - ref[i][I]) ** 2)) for i in comps)
    den = sum(float(np.sum(ref[i][I] ** 2)) for i in comps)
    return math.sqrt(num / den) if den > 0 else math.sqrt(num)


def gauge_free(a, mask):
    v = a[mask]
    return v - v.mean()
