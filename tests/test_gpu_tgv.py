"""Taylor-Green vortex cases on the GPU: the periodic 128^3 box (the TGV
configuration's size) and the symmetric subdomain (one eighth of the periodic
box with symmetry planes, the paper's benchmark geometry), against the oracle
and against the discrete decay rate of the initial mode."""
import math
import sys

import numpy as np
import pytest

import wlsynth
from gpu_util import FP32_STEP, FP64_STEP, make_pair, rel_l2

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("N,prec", [(32, "f64"), (32, "f32"), (64, "f32"), (64, "f64")])
def test_symmetric_tgv_steps(N, prec):
    _say("tgv sym steps", N, prec)
    w = wlsynth.tgv_sym_3d(N=N, Re=1600.0)
    ref, gpu = make_pair(w, prec, 1e-13 if prec == "f64" else 1e-6)
    for _ in range(2):
        ref.step()
        gpu.step()
    err = rel_l2(gpu.get("u"), ref.u, ref.grid)
    _say("  rel-L2", err)
    assert err <= (FP64_STEP if prec == "f64" else FP32_STEP), err
    gpu.close()


def test_periodic_tgv_128_one_step_fp64():
    _say("tgv 128^3 periodic, one FP64 step")
    w = wlsynth.tgv_3d(N=128)
    ref, gpu = make_pair(w, "f64", 1e-13)
    ref.step()
    gpu.step()
    err = rel_l2(gpu.get("u"), ref.u, ref.grid)
    _say("  rel-L2", err)
    assert err <= FP64_STEP, err
    gpu.close()


def _decay(w, nu):
    from paper_2407_16032_amd import Simulation
    sim = Simulation(w.n, w.U, nu, None, periodic=w.periodic_mask(), prec="f32", tol=1e-6, itmax=64,
                     device="cuda:0")
    sim.set_velocity(wlsynth.initial_velocity(w))

    def ke():
        u = sim.get("u")
        inner = tuple(slice(1, n + 1) for n in w.n)
        return 0.5 * sum(float(np.sum(u[i][inner] ** 2)) for i in range(3))

    E0 = ke()
    kappa = (math.pi if w.init == "tgv_sym" else 2 * math.pi) / w.n[0]
    T = 0.5 / kappa
    t = 0.0
    while t < T - 1e-12:
        sim.set_time(t, min(0.25, T - t))
        t = sim.step()["t"]
    out = math.log(ke() / E0), t
    sim.close()
    return out


@pytest.mark.parametrize("which", ["periodic", "symmetric"])
def test_tgv_128_early_decay_rate_fp32(which):
    # ln E_nu - ln E_2nu = 2 nu lam_h t while kappa U t <= 1/2, lam_h = 12 sin^2(kappa/2):
    # the difference of two runs cancels the limiter's own dissipation to first order
    _say("tgv 128^3 decay", which)
    w = wlsynth.tgv_3d(N=128) if which == "periodic" else wlsynth.tgv_sym_3d(N=128, Re=1600.0)
    kappa = (math.pi if w.init == "tgv_sym" else 2 * math.pi) / w.n[0]
    lam = 12 * math.sin(kappa / 2) ** 2
    a, t = _decay(w, w.nu)
    b, _ = _decay(w, 2 * w.nu)
    expect = 2 * w.nu * lam * t
    _say("  ln E difference %.6e, closed form %.6e" % (a - b, expect))
    assert a - b == pytest.approx(expect, rel=0.02)
