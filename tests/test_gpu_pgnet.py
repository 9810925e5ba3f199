"""Learned multigrid initial guess: BF16 MFMA kernels vs the FP64 conv-net oracle,
and the guided solve inside the step."""
import sys

import numpy as np
import pytest
import torch

import wlsynth
from oracle import pgnet as N

from gpu_util import make_pair, rel_l2

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _box_tensor(a, C):
    """[c, X, Y, Z] float64 interior -> bf16 device [P, C] channels-last with a zero halo."""
    c, X, Y, Z = a.shape
    out = np.zeros((Z + 2, Y + 2, X + 2, C), dtype=np.float32)
    out[1:-1, 1:-1, 1:-1, :c] = a.transpose(3, 2, 1, 0)
    return torch.tensor(out.reshape(-1, C)).to(torch.bfloat16).cuda()


def _box_scalar(a, dtype):
    X, Y, Z = a.shape
    out = np.zeros((Z + 2, Y + 2, X + 2), dtype=dtype)
    out[1:-1, 1:-1, 1:-1] = a.transpose(2, 1, 0)
    return torch.tensor(out.reshape(-1)).cuda()


def _unbox(y, n):
    X, Y, Z = n
    return y.cpu().numpy().reshape(Z + 2, Y + 2, X + 2)[1:-1, 1:-1, 1:-1].transpose(2, 1, 0)


def _sim():
    from paper_2407_16032_amd import Simulation
    w = wlsynth.sphere_3d(n=(64, 32, 32), D=12.0, center=(16.0, 16.0, 16.0))
    return w, Simulation(w.n, w.U, w.nu, w.body, convective_exit=True, prec="f32", tol=1e-6,
                         device="cuda:0", learned_guess=True)


def _weights(seed=0):
    flat = wlsynth.pg_init_weights(seed).copy()
    rng = np.random.default_rng(seed + 1)
    # non-zero biases so that every path of the kernels is exercised
    for k, n in [(1296, 16), (1296 + 16 + 6912, 16), (8672, 1)]:
        flat[k:k + n] = rng.uniform(-0.1, 0.1, n).astype(np.float32)
    return flat


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def test_forward_matches_oracle():
    _say("pg forward")
    w, sim = _sim()
    flat = _weights()
    sim.pg_set_weights(flat)
    n = (20, 18, 16)
    rng = np.random.default_rng(3)
    x = N.bf16_round(rng.normal(size=(3,) + n))
    y_ref, _ = N.forward(wlsynth.pg_split(flat), x, bf16=True)
    y = _unbox(sim.pg_forward(_box_tensor(x, 4), n), n)
    err = _rel(y, y_ref)
    _say("  forward rel err", err)
    assert err < 1e-2
    sim.close()


def test_gradients_and_adam_match_oracle():
    _say("pg gradients")
    w, sim = _sim()
    flat = _weights(2)
    sim.pg_set_weights(flat)
    sim.pg_mode(0, lr=1e-3)
    n = (24, 20, 16)
    rng = np.random.default_rng(5)
    x = N.bf16_round(rng.normal(size=(3,) + n))
    t = rng.normal(size=n)
    m = np.zeros(n, bool)
    m[3:-3, 3:-3, 3:-3] = rng.random((n[0] - 6, n[1] - 6, n[2] - 6)) > 0.1
    params = wlsynth.pg_split(flat)
    y_ref, cache = N.forward(params, x, bf16=True)
    loss_ref, dy = N.loss_and_grad(y_ref, t, m)
    g_ref = N.backward(params, cache, dy, bf16=True)
    g, loss = sim.pg_train_step(_box_tensor(x, 4), _box_scalar(t, np.float32),
                                _box_scalar(m.astype(np.uint8), np.uint8), n, apply=False)
    _say("  loss gpu %.6f oracle %.6f" % (loss, loss_ref))
    assert loss == pytest.approx(loss_ref, rel=2e-2)
    gs = wlsynth.pg_split(g)
    for k, name in enumerate(["W1", "b1", "W2", "b2", "W3"]):
        err = _rel(gs[k], g_ref[k])
        _say("  grad %s rel err %.3e" % (name, err))
        assert err < 2e-2, name
    # the loss is invariant to a constant output shift: d loss / d b3 = sum dy = 0 exactly;
    # on the GPU it is the sum of the BF16-rounded dy
    _say("  grad b3 gpu %.3e oracle %.3e" % (gs[5][0], g_ref[5][0]))
    assert abs(g_ref[5][0]) < 1e-12 and abs(gs[5][0]) < 1e-3
    # one Adam step on the master weights with the GPU's own gradient
    g2, _ = sim.pg_train_step(_box_tensor(x, 4), _box_scalar(t, np.float32),
                              _box_scalar(m.astype(np.uint8), np.uint8), n, apply=True)
    new = sim.pg_get_weights()
    ref = N.adam([flat.astype(np.float64)], [g2.astype(np.float64)], {}, lr=1e-3)[0]
    np.testing.assert_allclose(new, ref, rtol=1e-5, atol=1e-8)
    sim.close()


def test_guided_solves_converge_and_match_plain_run():
    # the learned guess only changes the multigrid starting point: both runs meet the
    # same residual tolerance, so the velocities agree to the solver tolerance
    _say("pg guided step")
    from paper_2407_16032_amd import Simulation
    w, sim = _sim()
    sim.pg_set_weights(wlsynth.pg_init_weights(0))
    sim.pg_mode(2, lr=1e-3, train_iters=2, crops=2, seed=7)
    plain = Simulation(w.n, w.U, w.nu, w.body, convective_exit=True, prec="f32", tol=1e-6, device="cuda:0")
    u0 = wlsynth.initial_velocity(w)
    sim.set_velocity(u0)
    plain.set_velocity(u0)
    for k in range(12):
        s1 = sim.step()
        s2 = plain.step()
        assert s1["converged"] and s2["converged"]
    st = sim.pg_stats()
    _say("  stats", st)
    assert st["train_steps"] == 2 * (2 * 12 - 2)
    assert st["snapshots"] == 2 * (2 * 12 - 2)
    assert np.isfinite(st["loss"])
    g = sim.grid if hasattr(sim, "grid") else None
    a = sim.get("u")
    b = plain.get("u")
    import oracle
    grid = oracle.Grid(w.n)
    err = rel_l2(a, b, grid)
    _say("  rel-L2 guided vs plain", err)
    assert err < 1e-4
    sim.close()
    plain.close()


def test_trained_guess_gain_over_plain_warm_start():
    """What the online-trained net gains over the plain warm start x0 = p w dt.

    Sphere wake, 128 x 64 x 64 (tiled multigrid), FP32, tolerance 1e-6: a learned run
    trains online for 40 steps (starting from a zero output layer, i.e. from the
    plain warm start), then runs 20 guided steps; a plain run takes the same steps.
    Multigrid decides on every guess (it is used only if its initial residual is below
    the warm start's), so the guided solves need no more cycles than the plain ones
    beyond what the slightly different flows explain; the V-cycles saved per step
    (possibly zero) are reported.
    """
    _say("pg gain")
    from paper_2407_16032_amd import Simulation
    w = wlsynth.sphere_3d(n=(128, 64, 64), D=16.0, center=(32.0, 32.0, 32.0))
    kw = dict(convective_exit=True, prec="f32", tol=1e-6, device="cuda:0")
    learned = Simulation(w.n, w.U, w.nu, w.body, learned_guess=True, **kw)
    plain = Simulation(w.n, w.U, w.nu, w.body, **kw)
    u0 = wlsynth.initial_velocity(w)
    learned.set_velocity(u0)
    plain.set_velocity(u0)
    learned.pg_set_weights(wlsynth.pg_init_weights(0, zero_output=True))
    learned.pg_mode(2, lr=1e-3, train_iters=2, crops=2, seed=3)
    for k in range(40):
        learned.step()
        plain.step()
    learned.pg_mode(1)
    vl, vp = [], []
    for k in range(20):
        a = learned.step()
        b = plain.step()
        assert a["converged"] and b["converged"]
        vl.append(sum(a["vcycles"]))
        vp.append(sum(b["vcycles"]))
    st = learned.pg_stats()
    gain = float(np.mean(vp) - np.mean(vl))
    _say("  V-cycles/step plain %.2f learned %.2f saved %.2f; guesses used %d of %d; last loss %.4g"
         % (np.mean(vp), np.mean(vl), gain, st["guesses_used"], st["guesses_tried"], st["loss"]))
    assert st["guesses_tried"] > 0
    assert np.mean(vl) <= np.mean(vp) + 0.5
    learned.close()
    plain.close()
