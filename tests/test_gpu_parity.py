"""Parity of the HIP path (through the C ABI) with the FP64 oracle on the same inputs."""
import sys

import numpy as np
import torch
import pytest

import oracle
import wlsynth
from oracle import poisson as OP
from oracle.flux import conv_diff
from oracle.solver import apply_bc

from gpu_util import CD_REL, FP32_10STEP, FP32_STEP, FP64_STEP, gauge_free, make_pair, rel_l2, small_cases

pytestmark = pytest.mark.gpu
CASES = small_cases()


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("name", ["circle2d", "sphere3d", "plate3d", "rotcyl2d"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_measure_and_coefficients(name, prec):
    _say("measure", name, prec)
    w = CASES[name]
    ref, gpu = make_pair(w, prec, 1e-6)
    tol = 1e-13 if prec == "f64" else 2e-7
    g = ref.grid
    mu0 = gpu.get("mu0")
    for i in range(g.ndim):
        np.testing.assert_allclose(mu0[i], ref.L[i], atol=tol, rtol=0)
    mu1 = gpu.get("mu1")
    V = gpu.get("V")
    for i in range(g.ndim):
        np.testing.assert_allclose(V[i], ref.V[i], atol=tol, rtol=0)
        for j in range(g.ndim):
            np.testing.assert_allclose(mu1[i * g.ndim + j], ref.mu1[i][j], atol=tol, rtol=0)
    assert len(gpu.levels()) == len(ref.levels)
    for l, lev in enumerate(ref.levels):
        Lg = gpu.get("L", l)
        for i in range(g.ndim):
            np.testing.assert_allclose(Lg[i], lev.L[i], atol=4 * tol * 2 ** l, rtol=0)
        iD = gpu.get("iD", l)[0]
        act = lev.active
        assert np.array_equal(iD != 0, act)
        np.testing.assert_allclose(iD[act], lev.iD[act], rtol=1e-12 if prec == "f64" else 1e-5)
    gpu.close()


def test_measure_moving_body_at_later_time():
    w = CASES["plate3d"]
    ref, gpu = make_pair(w, "f64", 1e-6)
    for t in (3.7, 41.0):
        ref.measure(t)
        gpu.measure(t)
        mu0 = gpu.get("mu0")
        V = gpu.get("V")
        for i in range(3):
            np.testing.assert_allclose(mu0[i], ref.L[i], atol=1e-13, rtol=0)
            np.testing.assert_allclose(V[i], ref.V[i], atol=1e-13, rtol=0)
    gpu.close()


@pytest.mark.parametrize("name", ["circle2d", "sphere3d", "tgv3d"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_conv_diff(name, prec):
    _say("conv_diff", name, prec)
    w = CASES[name]
    ref, gpu = make_pair(w, prec, 1e-6)
    g = ref.grid
    # a rough field: initial field plus seeded noise, boundary conditions applied on both sides
    u = [ref.u[i] + wlsynth.random_field(g.shape, seed=7, comp=i, amp=0.3) for i in range(g.ndim)]
    ref.set_velocity(u)
    gpu.set_velocity(u)
    R = conv_diff(g, ref.u, ref.nu)
    Rg = gpu.conv_diff()
    Rg = gpu.get("f")
    scale = max(float(np.abs(R[i]).max()) for i in range(g.ndim))
    tol = 1e-13 if prec == "f64" else 3e-6
    for i in range(g.ndim):
        np.testing.assert_allclose(Rg[i], R[i], atol=tol * scale, rtol=0)
    gpu.close()


@pytest.mark.parametrize("name", ["sphere3d", "tgv3d", "circle2d"])
def test_boundary_conditions(name):
    w = CASES[name]
    ref, gpu = make_pair(w, "f64", 1e-6)
    g = ref.grid
    u = [wlsynth.random_field(g.shape, seed=5, comp=i) for i in range(g.ndim)]
    gpu.set("u", u)
    gpu.apply_bc()
    apply_bc(g, ref.U, u)
    got = gpu.get("u")
    for i in range(g.ndim):
        np.testing.assert_array_equal(got[i], u[i])
    gpu.close()


@pytest.mark.parametrize("name", ["circle2d", "sphere3d", "tgv3d"])
def test_poisson_solve(name):
    _say("poisson", name)
    w = CASES[name]
    ref, gpu = make_pair(w, "f64", 1e-12)
    g = ref.grid
    lev = ref.levels[0]
    rng = np.random.default_rng(3)
    z = g.zeros()
    z[g.interior()] = rng.normal(size=g.n)
    z = np.where(lev.active, z, 0.0)
    z[lev.active] -= z[lev.active].mean()
    x = g.zeros()
    st = OP.solve(ref.levels, x, z, tol=1e-11, itmax=200)
    assert st["converged"]
    import torch
    rhs = gpu.scalar_buffer()          # pressure-layout device arrays
    xg = gpu.scalar_buffer()
    zz = torch.as_tensor(z, dtype=torch.float64)
    zz = zz.transpose(0, 1).unsqueeze(0) if g.ndim == 2 else zz.permute(2, 1, 0)
    rhs.copy_(zz.to(rhs.device))
    sg = gpu.poisson_solve(rhs=rhs, x=xg, tol=1e-11, itmax=200)
    assert sg["converged"], sg
    xa = xg.cpu().numpy()
    xa = xa[0].T if g.ndim == 2 else xa.transpose(2, 1, 0)
    np.testing.assert_allclose(gauge_free(xa, lev.active), gauge_free(x, lev.active), atol=1e-8)
    # same number of cycles up to rounding-order effects
    assert abs(sg["vcycles"] - st["vcycles"]) <= 1
    gpu.close()


@pytest.mark.parametrize("name", ["circle2d", "sphere3d", "tgv3d", "plate3d", "rotcyl2d", "sphere3d_tiled",
                                  "tgv3d_tiled"])
def test_one_step_fp64(name):
    _say("step f64", name)
    w = CASES[name]
    ref, gpu = make_pair(w, "f64", 1e-13)
    ref.tol = 1e-13
    s_ref = ref.step()
    s_gpu = gpu.step()
    err = rel_l2(gpu.get("u"), ref.u, ref.grid)
    _say("  rel-L2 u", err, s_ref["vcycles"], s_gpu["vcycles"])
    assert err <= FP64_STEP
    act = ref.levels[0].active
    p_err = np.abs(gauge_free(gpu.get("p")[0], act) - gauge_free(ref.p, act)).max()
    assert p_err <= 1e-9 * max(1.0, np.abs(ref.p[act]).max())
    assert abs(s_gpu["dt_next"] - ref.dt) <= 1e-12 * ref.dt
    gpu.close()


@pytest.mark.parametrize("name", ["circle2d", "sphere3d", "tgv3d", "plate3d", "sphere3d_tiled", "tgv3d_tiled"])
def test_one_step_fp32(name):
    _say("step f32", name)
    w = CASES[name]
    ref, gpu = make_pair(w, "f32", 1e-6)
    ref.tol = 1e-13
    ref.step()
    gpu.step()
    err = rel_l2(gpu.get("u"), ref.u, ref.grid)
    _say("  rel-L2 u", err)
    assert err <= FP32_STEP
    gpu.close()


@pytest.mark.parametrize("name", ["sphere3d_tiled", "tgv3d_tiled"])
@pytest.mark.parametrize("path", ["tiles", "flat", "generic"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_one_step_other_solver_paths(name, path, prec):
    """By default the 64^3 cases run both PCG passes of the fine level as flat
    vector passes (2^18 cells, rows of whole 16-byte vectors; the tests above);
    here the fine level runs z-marching tiles, the flat passes forced, or the
    generic kernels."""
    _say("step", prec, name, path)
    w = CASES[name]
    ref, gpu = make_pair(w, prec, 1e-13 if prec == "f64" else 1e-6, solver_path=path)
    ref.tol = 1e-13
    ref.step()
    gpu.step()
    err = rel_l2(gpu.get("u"), ref.u, ref.grid)
    _say("  rel-L2 u", err)
    assert err <= (FP64_STEP if prec == "f64" else FP32_STEP)
    gpu.close()


@pytest.mark.parametrize("n,periodic", [((130, 18, 14), (True, False, True)), ((75, 18, 17), (False, False, False)),
                                         ((66, 11, 17), (False, True, False))])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_one_step_ragged_3d_grids(n, periodic, prec):
    """The 3-D flux shares face fluxes between neighbouring lanes and planes in bricks
    of 63 columns: grids of two or three bricks with a ragged last one, periodic and
    bounded axes and a body, one step against the oracle."""
    _say("ragged step", prec, n, periodic)
    # radius 2 keeps the body's reach (radius + 3) 3 cells from every bounded wall
    body = wlsynth.Body("sphere", center=(0.3 * n[0], 0.5 * n[1] + 0.2, 0.5 * n[2] - 0.3), radius=2.0)
    w = wlsynth.Workload("ragged", n, (1.0, 0.0, 0.0), 0.02, body, periodic=periodic,
                         convective_exit=not periodic[0], tol=1e-13)
    ref, gpu = make_pair(w, prec, 1e-13 if prec == "f64" else 1e-6)
    ref.tol = 1e-13
    ref.step()
    gpu.step()
    err = rel_l2(gpu.get("u"), ref.u, ref.grid)
    _say("  rel-L2 u", err)
    assert err <= (FP64_STEP if prec == "f64" else FP32_STEP)
    gpu.close()


@pytest.mark.parametrize("n,bx", [((61, 12, 12), 0.3), ((62, 12, 11), 0.3), ((63, 11, 12), 0.3), ((124, 10, 9), 0.3),
                                  ((63, 12, 12), None)])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_one_step_x_brick_edges(n, bx, prec):
    """Bricks of 63 columns against the x extent on a bounded x axis: padded rows of
    exactly 63, 64, 65 and 126 columns (one brick with its supply lane past the
    row; a last brick of one ghost column; of an interior column and the ghost; two
    full bricks).  The first and last brick of each row take the fast loads with the
    general form's boundary rules per lane; one step against the oracle, with the
    body near the inlet or (bx None) 8 cells from the outlet (y and z periodic, so
    that only the x walls bound the body's reach)."""
    _say("x brick edges", prec, n, bx)
    cx = 0.3 * n[0] if bx is not None else n[0] - 8.0
    body = wlsynth.Body("sphere", center=(cx, 0.5 * n[1] + 0.2, 0.5 * n[2] - 0.3), radius=2.0)
    w = wlsynth.Workload("xedges", n, (1.0, 0.0, 0.0), 0.02, body, periodic=(False, True, True),
                         convective_exit=True, tol=1e-13)
    ref, gpu = make_pair(w, prec, 1e-13 if prec == "f64" else 1e-6)
    ref.tol = 1e-13
    ref.step()
    gpu.step()
    err = rel_l2(gpu.get("u"), ref.u, ref.grid)
    _say("  rel-L2 u", err)
    assert err <= (FP64_STEP if prec == "f64" else FP32_STEP)
    gpu.close()


def test_solver_paths_agree_on_a_large_grid():
    """256 x 128 x 128 sphere wake in FP64: the fine level takes the flat passes
    (automatic), the z-marching tiles or the generic kernels, and the first coarse
    level (128 x 64 x 64) tiles or generic kernels; one step of each agrees to
    the solver tolerance (sums differ only in rounding order)."""
    from paper_2407_16032_amd import Simulation
    w = wlsynth.sphere_3d()
    u0 = wlsynth.initial_velocity(w)
    out = {}
    for path in ("auto", "tiles", "flat", "generic"):
        _say("large grid FP64 step", path)
        gpu = Simulation(w.n, w.U, w.nu, w.body, convective_exit=True, prec="f64", tol=1e-11, itmax=64,
                         device="cuda:0", solver_path=path)
        gpu.set_velocity(u0)
        st = gpu.step()
        assert st["converged"], st
        out[path] = gpu.get("u")
        gpu.close()
    g = oracle.Grid(w.n)
    for path in ("tiles", "flat", "generic"):
        err = rel_l2(out[path], out["auto"], g)
        _say("  rel-L2 u", path, "vs auto", err)
        assert err <= 1e-10


@pytest.mark.parametrize("name", ["circle2d", "sphere3d"])
def test_ten_steps_fp32(name):
    _say("10 steps f32", name)
    w = CASES[name]
    ref, gpu = make_pair(w, "f32", 1e-6)
    ref.tol = 1e-13
    for _ in range(10):
        ref.step()
        gpu.step()
    err = rel_l2(gpu.get("u"), ref.u, ref.grid)
    _say("  rel-L2 u", err)
    assert err <= FP32_10STEP
    gpu.close()


def test_drag_coefficient_window_circle():
    # 2-D circle, 128 x 64, R = 8, Re = 250: mean C_D over steps 51-100 (A_ref = D = 16)
    _say("drag window")
    w = CASES["circle2d"]
    ref, gpu = make_pair(w, "f32", 1e-6)
    ref.tol = 1e-10
    cd_r, cd_g = [], []
    for k in range(100):
        ref.step()
        gpu.step()
        if k >= 50:
            fp, fv = ref.forces()
            cd_r.append(2 * (fp[0] + fv[0]) / 16.0)
            gp, gv = gpu.forces()
            cd_g.append(2 * (gp[0] + gv[0]) / 16.0)
    mr, mg = float(np.mean(cd_r)), float(np.mean(cd_g))
    _say("  mean C_D oracle %.6f gpu %.6f" % (mr, mg))
    assert abs(mg - mr) <= CD_REL * abs(mr)
    gpu.close()


def test_forces_fp64_match():
    w = CASES["sphere3d"]
    ref, gpu = make_pair(w, "f64", 1e-13)
    ref.tol = 1e-13
    ref.step()
    gpu.step()
    fp, fv = ref.forces()
    gp, gv = gpu.forces()
    np.testing.assert_allclose(gp, fp, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(gv, fv, rtol=1e-9, atol=1e-12)
    gpu.close()


def test_moving_plate_three_steps_fp64():
    # the per-step re-measure of a moving body only rewrites the body's bounding box
    _say("3 steps f64 plate")
    w = CASES["plate3d"]
    ref, gpu = make_pair(w, "f64", 1e-13)
    ref.tol = 1e-13
    for _ in range(3):
        ref.step()
        gpu.step()
    err = rel_l2(gpu.get("u"), ref.u, ref.grid)
    _say("  rel-L2 u", err)
    assert err <= FP64_STEP
    mu0 = gpu.get("mu0")
    for i in range(3):
        np.testing.assert_allclose(mu0[i], ref.L[i], atol=1e-13, rtol=0)
    gpu.close()


def test_large_grid_projection_is_divergence_free():
    # 256 x 128 x 128 sphere wake (tiled multigrid kernels on the fine and first coarse
    # levels): after a step, max|div u| over active cells is below the tolerance
    _say("large grid divergence")
    import torch
    from paper_2407_16032_amd import Simulation
    w = wlsynth.sphere_3d()
    gpu = Simulation(w.n, w.U, w.nu, w.body, convective_exit=True, prec="f32", tol=1e-5, device="cuda:0")
    gpu.set_velocity(wlsynth.initial_velocity(w))
    for _ in range(2):
        st = gpu.step()
        assert st["converged"], st
    u = gpu.field("u")
    iD = gpu.field("iD")[0]
    div = (u[0][1:-1, 1:-1, 2:] - u[0][1:-1, 1:-1, 1:-1]) + (u[1][1:-1, 2:, 1:-1] - u[1][1:-1, 1:-1, 1:-1]) + \
        (u[2][2:, 1:-1, 1:-1] - u[2][1:-1, 1:-1, 1:-1])
    act = iD[1:-1, 1:-1, 1:-1] != 0
    d = float(div[act].abs().max())
    _say("  max |div u| =", d, "tol", w.tol)
    # the corrector's residual tolerance holds for x; div u = r up to FP32 rounding of u
    assert d < 2 * w.tol
    gpu.close()


def test_full_size_plate_fp32():
    """The benchmark's workload and launch configuration (768 x 384 x 384 heaving plate,
    FP32, automatic solver path): after two steps the solves converged, the velocity is
    divergence-free to the solver tolerance on active cells, and mu0 at sampled faces
    (inside the body box and elsewhere) matches the oracle's moment of the signed
    distance evaluated face by face at the last measure time."""
    _say("full-size plate")
    from paper_2407_16032_amd import Simulation
    from oracle import moments
    from oracle.body import MU0_CUT, sdf_normal_velocity
    w = wlsynth.plate_3d()
    gpu = Simulation(w.n, w.U, w.nu, w.body, convective_exit=True, prec="f32", tol=w.tol, device="cuda:0")
    gpu.set_velocity(wlsynth.initial_velocity(w))
    st = gpu.step()
    assert st["converged"], st
    t_meas, _ = gpu.time()
    st = gpu.step()  # re-measures the moving plate at t_meas
    assert st["converged"], st
    u = gpu.field("u")
    iD = gpu.field("iD")[0]
    div = (u[0][1:-1, 1:-1, 2:] - u[0][1:-1, 1:-1, 1:-1]) + (u[1][1:-1, 2:, 1:-1] - u[1][1:-1, 1:-1, 1:-1]) + \
        (u[2][2:, 1:-1, 1:-1] - u[2][1:-1, 1:-1, 1:-1])
    d = float(div[iD[1:-1, 1:-1, 1:-1] != 0].abs().max())
    _say("  max |div u| =", d)
    assert d < 2 * w.tol
    del div
    lo, hi = gpu.body_box(0)
    mu0 = gpu.field("mu0")
    rng = np.random.default_rng(3)
    n = w.n
    for comp in range(3):
        for inside in (True, False):
            I = []
            for a in range(3):
                # interior faces: 2..N along the component's own axis, 1..N across
                a0, a1 = (2 if a == comp else 1), n[a]
                if inside:
                    a0, a1 = max(a0, lo[a]), min(a1, hi[a])
                I.append(rng.integers(a0, a1 + 1, size=4000))
            got = mu0[comp][torch.as_tensor(I[2]), torch.as_tensor(I[1]), torch.as_tensor(I[0])]
            got = got.double().cpu().numpy()
            X = [I[a] - (1.0 if a == comp else 0.5) for a in range(3)]
            dist, _, _ = sdf_normal_velocity(w.body, [x.astype(np.float64) for x in X], t_meas)
            want = moments.mu0(dist, 1.0)
            want = np.where(want < MU0_CUT, 0.0, want)
            keep = np.abs(want - MU0_CUT) > 1e-5  # a face at the solid cut may fall either way
            err = np.abs(got - want)[keep].max()
            _say("  mu0 comp %d %s box: %d faces, max err %.2e" % (comp, "in" if inside else "any", keep.sum(), err))
            assert err < 1e-6
    gpu.close()


@pytest.mark.parametrize("name", ["plate3d", "rotcyl2d"])
def test_boxed_remeasure_matches_a_full_measure(name):
    """After several steps of a moving body, whose per-step re-measure updates the
    coefficients of every level only near the body, the stored L and iD equal those
    of a full-domain measure at the same time, on every level."""
    _say("boxed re-measure", name)
    from paper_2407_16032_amd import Simulation
    w = CASES[name]
    sims = [Simulation(w.n, w.U, w.nu, w.body, periodic=w.periodic_mask(), convective_exit=w.convective_exit,
                       prec="f64", tol=1e-8, device="cuda:0") for _ in range(2)]
    sims[0].set_velocity(wlsynth.initial_velocity(w))
    for _ in range(3):
        sims[0].step()
    t, _ = sims[0].time()
    sims[0].step()  # re-measures at its start time t
    sims[1].measure(t)
    for lvl in range(len(sims[0].levels())):
        for fname in ("L", "iD"):
            a, b = (s.field(fname, lvl).double().cpu().numpy() for s in sims)
            np.testing.assert_array_equal(a, b, err_msg="%s level %d" % (fname, lvl))
    for s in sims:
        s.close()


@pytest.mark.parametrize("name", ["plate3d", "sphere3d_tiled", "circle2d"])
def test_coefficients_are_body_free_outside_the_body_box(name):
    """The kernels evaluate L, iD (every level) and mu0, mu1, V (fine level) in closed
    form outside the body box; check that the stored fields hold exactly those values
    there, for a moving body after several re-measures."""
    _say("body box", name)
    import torch
    from paper_2407_16032_amd import Simulation
    w = CASES[name]
    gpu = Simulation(w.n, w.U, w.nu, w.body, periodic=w.periodic_mask(), convective_exit=w.convective_exit,
                     prec="f64", tol=1e-8, device="cuda:0")
    gpu.set_velocity(wlsynth.initial_velocity(w))
    for _ in range(3):
        gpu.step()
    D = len(w.n)
    per = w.periodic_mask() if w.periodic_mask() else [False] * D
    levels = gpu.levels()
    for lvl, n in enumerate(levels):
        lo, hi = gpu.body_box(lvl)
        Lstd = float(2 ** ((D - 2) * lvl))
        # padded index grids, axis order of the arrays (components, z, y, x) -> (x, y[, z])
        L = gpu.field("L", lvl).double().cpu().numpy()
        iD = gpu.field("iD", lvl).double().cpu().numpy()[0]
        if D == 2:
            L = L[:, 0].transpose(0, 2, 1)
            iD = iD[0].T
        else:
            L = L.transpose(0, 3, 2, 1)
            iD = iD.transpose(2, 1, 0)
        idx = np.meshgrid(*[np.arange(N + 2) for N in n], indexing="ij")

        def outside(margin):
            if lo[0] > hi[0]:
                return np.ones(idx[0].shape, dtype=bool)
            m = np.zeros(idx[0].shape, dtype=bool)
            for a in range(D):
                m |= (idx[a] < lo[a] - margin) | (idx[a] > hi[a] + margin)
            return m

        interior = np.ones(idx[0].shape, dtype=bool)
        for a in range(D):
            interior &= (idx[a] >= 1) & (idx[a] <= n[a])
        # L on the faces of interior cells (face index 1..N along its own axis)
        for a in range(D):
            face = interior.copy()
            expect = np.where(per[a] | ((idx[a] >= 2) & (idx[a] <= n[a])), Lstd, 0.0)
            m = face & outside(0)
            np.testing.assert_array_equal(L[a][m], expect[m])
        cnt = np.full(idx[0].shape, 2 * D)
        for a in range(D):
            if not per[a]:
                cnt = cnt - (idx[a] == 1) - (idx[a] == n[a])
        m = interior & outside(1)
        np.testing.assert_array_equal(iD[m], (1.0 / (-(Lstd * cnt)))[m])
        _say("  level %d n %s box %s..%s: %d interior cells checked" % (lvl, n, lo, hi, int(m.sum())))
        if lvl == 0 and w.body.kind != "none":
            for fname in ("mu1", "V"):
                f = gpu.field(fname).double().cpu().numpy()
                f = f[:, 0].transpose(0, 2, 1) if D == 2 else f.transpose(0, 3, 2, 1)
                m = outside(0)
                for comp in range(f.shape[0]):
                    assert np.all(f[comp][m] == 0.0), (fname, comp)
    gpu.close()


@pytest.mark.parametrize("mode", ["single", "two_stage", "auto"])
@pytest.mark.parametrize("name", ["tgv3d", "sphere3d"])
def test_one_step_fp64_every_partial_sum_path(name, mode):
    # the flat levels' per-block partial sums totalled by one separate launch or by
    # two (forced on these small grids) and the default (the consumers add them):
    # the same step to FP64 rounding and the same V-cycle counts
    _say("reduce path", name, mode)
    w = CASES[name]
    from paper_2407_16032_amd import Simulation
    u0 = wlsynth.initial_velocity(w, seed=0)
    body = w.body if w.body.kind != "none" else None
    ref = oracle.Sim(w.n, w.U, w.nu, body, periodic=w.periodic_mask(), convective_exit=w.convective_exit,
                     tol=1e-13, itmax=200)
    ref.set_velocity(u0)
    gpu = Simulation(w.n, w.U, w.nu, body, periodic=w.periodic_mask(), convective_exit=w.convective_exit,
                     prec="f64", tol=1e-13, itmax=200, device="cuda:0", reduce_mode=mode)
    gpu.set_velocity(u0)
    st_r = ref.step()
    st_g = gpu.step()
    err = rel_l2(gpu.get("u"), ref.u, ref.grid)
    _say("  rel-L2", err, st_g["vcycles"], st_r["vcycles"])
    assert err <= FP64_STEP, err
    assert all(abs(a - b) <= 1 for a, b in zip(st_g["vcycles"], st_r["vcycles"]))
    gpu.close()
