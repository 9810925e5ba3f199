"""The HIP discrete adjoint (through the C ABI) against the oracle's complex-step
gradient, central differences of the HIP forward, and a one-step transpose check."""
import json
import os
import sys

import numpy as np
import pytest
import torch

import wlsynth
from oracle import adjoint as OA

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _case():
    # spinning circle, 48 x 24 cells, R = 3: small enough for the complex-step oracle
    return wlsynth.rotating_cylinder_2d(n=(48, 24), D=6.0, center=(14.0, 12.0), xi=0.8)


XI, R, STEPS, WIN = 0.8, 3.0, 12, 6


@pytest.fixture(scope="module")
def oracle_grad():
    w = _case()
    J, gx, gR, dts = OA.gradient(w, XI, R, STEPS, WIN)
    return J, gx, gR, dts


def _problem(ckpt, dts=None, prec="f64", tol=1e-12):
    from paper_2407_16032_amd.adjoint import RotatingCylinderDrag
    w = _case()
    prob = RotatingCylinderDrag(w, wlsynth.initial_velocity(w), STEPS, WIN, ckpt=ckpt, prec=prec, tol=tol)
    prob.dts = None if dts is None else list(dts)
    return prob


@pytest.mark.parametrize("ckpt", [1, 5, 20])
def test_adjoint_gradient_matches_oracle_complex_step(oracle_grad, ckpt):
    J0, gx0, gR0, dts = oracle_grad
    _say("adjoint vs complex step, ckpt", ckpt)
    prob = _problem(ckpt, dts)
    J, gx, gR = prob.value_and_grad(XI, R)
    _say("  J %.12g / %.12g  dxi %.10g / %.10g  dR %.10g / %.10g" % (J, J0, gx, gx0, gR, gR0), prob.stats)
    assert J == pytest.approx(J0, rel=1e-10)
    assert gx == pytest.approx(gx0, rel=1e-6, abs=1e-10)
    assert gR == pytest.approx(gR0, rel=1e-6, abs=1e-10)
    prob.sim.close()


def test_adjoint_gradient_matches_gpu_central_differences():
    _say("adjoint vs central differences of the HIP forward")
    prob = _problem(4)
    J, gx, gR = prob.value_and_grad(XI, R)  # records the frozen schedule
    h = 1e-6
    fx = (prob.value(XI + h, R) - prob.value(XI - h, R)) / (2 * h)
    fR = (prob.value(XI, R + h) - prob.value(XI, R - h)) / (2 * h)
    _say("  dxi %.10g fd %.10g   dR %.10g fd %.10g" % (gx, fx, gR, fR))
    assert gx == pytest.approx(fx, rel=1e-5, abs=1e-8)
    assert gR == pytest.approx(fR, rel=1e-5, abs=1e-8)
    prob.sim.close()


def test_autograd_function_backward():
    from paper_2407_16032_amd.adjoint import rotating_cylinder_drag
    _say("autograd.Function")
    prob = _problem(5)
    theta = torch.tensor([XI, R], dtype=torch.float64, requires_grad=True)
    J = rotating_cylinder_drag(theta, prob)
    J.backward()
    J2, gx, gR = prob.value_and_grad(XI, R)
    assert float(J.detach()) == pytest.approx(J2, rel=1e-12)
    np.testing.assert_allclose(theta.grad.numpy(), [gx, gR], rtol=1e-9, atol=1e-14)
    prob.sim.close()


def _dot(a, b):
    return float(sum(torch.sum(x.double() * y.double()) for x, y in zip(a, b)))


def _to_oracle(t):
    """(comp, 1, py, nx+2) GPU-layout tensor -> list of [x, y] float64 arrays."""
    a = t.detach().to("cpu", torch.float64).numpy()
    return [a[c, 0].T.copy() for c in range(a.shape[0])]


def test_one_step_transpose_dot_product():
    """<ubar, J du> + <pbar, J_p du> = <J^T (ubar, pbar), du> for one step (FP64).

    J du comes exactly from the complex step of the oracle's step (the HIP forward
    equals it to rounding), and approximately from central differences of the HIP
    step.  The step is only piecewise smooth: the limiter's medians switch where two
    arguments are (nearly) equal, and a finite step h |du| crosses the near-ties of
    the 1e-3 inflow noise unless h is tiny; exact ties (a ghost face and its source,
    or the rigidly spinning solid, where u = V is constant along one axis) are kept
    by admissible directions, which satisfy the boundary conditions and vanish near
    the body.
    """
    import oracle
    from paper_2407_16032_amd import Simulation
    _say("one-step transpose")
    w = _case()
    body = OA.rotcyl_body(w, XI, R)
    sim = Simulation(w.n, w.U, w.nu, body, prec="f64", tol=1e-13, itmax=300, device="cuda:0", adjoint=True)
    sim.set_velocity(wlsynth.initial_velocity(w))
    for _ in range(3):
        sim.step()
    base = sim.save_state()
    t0, dt = base[2]
    dev = base[0].device
    gen = torch.Generator().manual_seed(7)
    shp = base[0].shape  # (D, 1, py, nx + 2)
    far = torch.zeros(shp, dtype=torch.bool)
    yy, xx = torch.meshgrid(torch.arange(shp[2], dtype=torch.float64), torch.arange(shp[3], dtype=torch.float64),
                            indexing="ij")
    cx, cy = w.body.center[0], w.body.center[1]
    for c in range(2):  # faces of component c: x = I - 1 along c, I - 1/2 across
        fx = xx - (1.0 if c == 0 else 0.5)
        fy = yy - (1.0 if c == 1 else 0.5)
        far[c, 0] = torch.sqrt((fx - cx) ** 2 + (fy - cy) ** 2) > R + 4.0
    raw = torch.randn(shp, generator=gen, dtype=torch.float64) * far
    sim.load_state((base[0] + raw.to(dev), base[1], base[2]))
    sim.apply_bc()
    du = sim.field("u").clone() - base[0]  # the boundary-condition-consistent direction
    ubar = torch.randn(shp, generator=gen, dtype=torch.float64).to(dev)
    act = sim.field("iD") != 0
    pbar = torch.randn(sim.field("p").shape, generator=gen, dtype=torch.float64).to(dev)
    pbar = torch.where(act, pbar, torch.zeros_like(pbar))
    pbar[act] -= pbar[act].mean()  # the pressure's gauge is not a function of u

    # exact J du: complex step of the oracle's step from the same state
    ref = oracle.Sim(w.n, w.U, w.nu, body, tol=1e-13, itmax=300)
    hc = 1e-30
    u_np, du_np = _to_oracle(base[0]), _to_oracle(du)
    ref.u = [u_np[c] + 1j * hc * du_np[c] for c in range(2)]
    ref.p = _to_oracle(base[1])[0]
    ref.t, ref.dt = t0, dt
    ref.step()
    ub_np, pb_np = _to_oracle(ubar), _to_oracle(pbar)[0]
    lhs_cs = sum(float(np.sum(ub_np[c] * np.imag(ref.u[c]))) for c in range(2)) / hc
    lhs_cs += float(np.sum(pb_np * np.imag(ref.p))) / hc

    def run(sign, h):
        sim.load_state((base[0] + sign * h * du, base[1], (t0, dt)))
        sim.step()
        return sim.field("u").clone(), sim.field("p").clone()

    h = 1e-8
    up, pp = run(+1, h)
    um, pm = run(-1, h)
    lhs_fd = _dot([ubar], [(up - um) / (2 * h)]) + _dot([pbar], [(pp - pm) / (2 * h)])
    sim.adj_reset()
    sim.load_state(base, dt)
    sim.field("adj_u").copy_(ubar)
    sim.field("adj_p").copy_(pbar)
    st = sim.adj_step(1e-13)
    rhs = _dot([sim.field("adj_u").clone()], [du])
    _say("  complex step %.15g  central diff %.15g  adjoint %.15g" % (lhs_cs, lhs_fd, rhs), st)
    # the adjoint solves stop at a residual of 1e-13: agreement to ~1e-9
    assert rhs == pytest.approx(lhs_cs, rel=1e-8)
    assert rhs == pytest.approx(lhs_fd, rel=1e-4)
    assert float(sim.field("adj_p").abs().max()) == 0.0
    sim.close()


def test_adjoint_needs_buffers_and_no_exit():
    from paper_2407_16032_amd import Simulation
    from paper_2407_16032_amd._lib import WlError
    w = _case()
    sim = Simulation(w.n, w.U, w.nu, OA.rotcyl_body(w, XI, R), prec="f64", device="cuda:0")
    with pytest.raises(WlError, match="UNSUPPORTED"):
        sim.adj_reset()
    sim.close()
    sim = Simulation(w.n, w.U, w.nu, None, prec="f32", device="cuda:0", convective_exit=True, adjoint=True)
    with pytest.raises(WlError, match="UNSUPPORTED"):
        sim.adj_step()
    sim.close()


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "rotcyl_512x256_gradient.json")


@pytest.mark.skipif(not os.path.exists(GOLDEN), reason="oracle gradient not generated (tests/golden/make_rotcyl_gradient.py)")
def test_rotcyl_512x256_gradient_matches_oracle():
    """Full-size case: 512 x 256, D = 32, Re = 200, seeded xi, 400 steps, window 200..399,
    checkpoints every 20 steps; the oracle's complex-step gradient was stored by a script
    that calls only the oracle."""
    from paper_2407_16032_amd.adjoint import RotatingCylinderDrag
    with open(GOLDEN) as f:
        ref = json.load(f)
    w = wlsynth.rotating_cylinder_2d()
    assert w.name == ref["workload"]
    _say("rotating cylinder 512x256, 400 steps")
    prob = RotatingCylinderDrag(w, wlsynth.initial_velocity(w), ref["steps"], ref["window_start"], ckpt=20,
                                prec="f64", tol=ref["tol"], itmax=200)
    prob.dts = list(ref["dt_schedule"])
    J, gx, gR = prob.value_and_grad(ref["xi"], ref["R"])
    _say("  J %.12g / %.12g  dxi %.10g / %.10g  dR %.10g / %.10g" % (J, ref["J"], gx, ref["dJ_dxi"], gR,
                                                                   ref["dJ_dR"]), prob.stats)
    assert J == pytest.approx(ref["J"], rel=1e-9)
    assert gx == pytest.approx(ref["dJ_dxi"], rel=1e-6, abs=1e-9)
    assert gR == pytest.approx(ref["dJ_dR"], rel=1e-6, abs=1e-9)
    prob.sim.close()


def test_rotcyl_512x256_fd_steps():
    """Central differences of the full-size objective at the configuration's h = 1e-3
    and at h = 1e-5, against the oracle's complex-step gradient.  At h = 1e-5 both
    derivatives meet the 1e-3 gate; at h = 1e-3 dJ/dxi does (6.7e-4) and dJ/dR is
    off by 4.3e-3: J is piecewise smooth in R at that scale (limiter branches), so
    the wide step's figure is recorded and bounded, not gated at 1e-3."""
    from paper_2407_16032_amd.adjoint import RotatingCylinderDrag
    with open(GOLDEN) as f:
        ref = json.load(f)
    w = wlsynth.rotating_cylinder_2d()
    prob = RotatingCylinderDrag(w, wlsynth.initial_velocity(w), ref["steps"], ref["window_start"], ckpt=20,
                                prec="f64", tol=ref["tol"], itmax=200)
    prob.dts = list(ref["dt_schedule"])
    xi, R = ref["xi"], ref["R"]
    rel = {}
    for h in (1e-3, 1e-5):
        fx = (prob.value(xi + h, R) - prob.value(xi - h, R)) / (2 * h)
        fR = (prob.value(xi, R + h) - prob.value(xi, R - h)) / (2 * h)
        rel[h] = (abs(fx - ref["dJ_dxi"]) / abs(ref["dJ_dxi"]), abs(fR - ref["dJ_dR"]) / abs(ref["dJ_dR"]))
        _say("  h %.0e: dJ/dxi rel %.2e  dJ/dR rel %.2e" % (h, rel[h][0], rel[h][1]))
    assert rel[1e-5][0] < 1e-3 and rel[1e-5][1] < 1e-3
    assert rel[1e-3][0] < 1e-3
    assert rel[1e-3][1] < 1e-2
    prob.sim.close()


@pytest.mark.parametrize("ckpt", [1, 5])
def test_adjoint_with_live_time_steps_matches_oracle(ckpt):
    # time steps follow the CFL rule in every run: the gradient includes the steps'
    # dependence on the flow (wl_adj_step_cfl), against the oracle's complex step of
    # the live-CFL rollout
    from paper_2407_16032_amd.adjoint import RotatingCylinderDrag
    w = _case()
    J0, gx0, gR0, dts0 = OA.gradient_cfl(w, XI, R, STEPS, WIN)
    _say("live-dt adjoint vs complex step, ckpt", ckpt)
    prob = RotatingCylinderDrag(w, wlsynth.initial_velocity(w), STEPS, WIN, ckpt=ckpt, prec="f64", tol=1e-12,
                                live_dt=True)
    J, gx, gR = prob.value_and_grad(XI, R)
    _say("  J %.12g / %.12g  dxi %.10g / %.10g  dR %.10g / %.10g" % (J, J0, gx, gx0, gR, gR0))
    np.testing.assert_allclose(prob.last_dts, dts0, rtol=1e-10)
    assert J == pytest.approx(J0, rel=1e-10)
    assert gx == pytest.approx(gx0, rel=1e-6, abs=1e-10)
    assert gR == pytest.approx(gR0, rel=1e-6, abs=1e-10)
    # and it is not the frozen-schedule derivative
    _, fx, _, _ = OA.gradient(w, XI, R, STEPS, WIN)
    assert abs(gx - fx) > 1e-4 * abs(fx)
    prob.sim.close()


def test_adjoint_with_live_time_steps_matches_gpu_central_differences():
    from paper_2407_16032_amd.adjoint import RotatingCylinderDrag
    w = _case()
    prob = RotatingCylinderDrag(w, wlsynth.initial_velocity(w), STEPS, WIN, ckpt=4, prec="f64", tol=1e-12,
                                live_dt=True)
    J, gx, gR = prob.value_and_grad(XI, R)
    h = 1e-6
    fx = (prob.value(XI + h, R) - prob.value(XI - h, R)) / (2 * h)
    fR = (prob.value(XI, R + h) - prob.value(XI, R - h)) / (2 * h)
    _say("  live dt: dxi %.10g fd %.10g   dR %.10g fd %.10g" % (gx, fx, gR, fR))
    assert gx == pytest.approx(fx, rel=1e-5, abs=1e-8)
    assert gR == pytest.approx(fR, rel=1e-5, abs=1e-8)
    prob.sim.close()


def test_adjoint_fp32_variant(oracle_grad):
    # the same reverse sweep with FP32 fields (FP64 dots): its error against the FP64
    # oracle's complex-step gradient is reported and bounded
    J0, gx0, gR0, dts = oracle_grad
    prob = _problem(5, dts, prec="f32", tol=1e-6)
    J, gx, gR = prob.value_and_grad(XI, R)
    ex, eR = abs(gx - gx0) / abs(gx0), abs(gR - gR0) / abs(gR0)
    _say("  FP32 adjoint: J rel %.2e  dJ/dxi rel %.2e  dJ/dR rel %.2e" % (abs(J - J0) / abs(J0), ex, eR))
    assert abs(J - J0) < 1e-4 * abs(J0)
    assert ex < 2e-2 and eR < 2e-2
    prob.sim.close()
