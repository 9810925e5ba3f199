"""The coarse part of each multigrid cycle replayed from a captured HIP graph
against plain launches of the same kernels.

Every solve runs several cycles, so a step replays the graph several times with
the solver's own launches and read-backs between the replays; velocity,
pressure and the solver statistics must agree bit for bit after every step.
The moving plate changes its body box (a launch argument) as it heaves, which
must select a newly captured graph rather than replay a stale one.
"""
import sys

import numpy as np
import pytest

import wlsynth
from gpu_util import small_cases

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _cases():
    c = small_cases()
    return {
        "plate3d_f32": (c["plate3d"], "f32", "auto"),
        "plate3d_f64": (c["plate3d"], "f64", "auto"),
        "tgv3d_f32": (c["tgv3d"], "f32", "auto"),
        "sphere3d_tiled_f32_tiles": (c["sphere3d_tiled"], "f32", "tiles"),
        "sphere3d_f64_generic": (c["sphere3d"], "f64", "generic"),
        "jelly3d_f32": (wlsynth.jelly_3d(n=12), "f32", "auto"),
    }


CASES = _cases()


@pytest.mark.parametrize("name", sorted(CASES))
def test_graph_replay_matches_plain_launches(name):
    from paper_2407_16032_amd import Simulation
    w, prec, path = CASES[name]
    _say("vcycle graph", name, w.n)
    u0 = wlsynth.initial_velocity(w, seed=5)
    body = w.body if w.body.kind != "none" else None
    sims = {}
    for graph in ("on", "off"):
        s = Simulation(w.n, w.U, w.nu, body, periodic=w.periodic_mask(), convective_exit=w.convective_exit,
                       prec=prec, tol=1e-5 if prec == "f32" else 1e-10, itmax=64, device="cuda:0",
                       solver_path=path, vcycle_graph=graph)
        s.set_velocity(u0)
        sims[graph] = s
    for k in range(5):
        a, b = sims["on"].step(), sims["off"].step()
        assert a == b, (k, a, b)
        ua, ub = sims["on"].get("u"), sims["off"].get("u")
        for c in range(3):
            assert np.array_equal(ua[c], ub[c]), (k, c, float(np.max(np.abs(ua[c] - ub[c]))))
        assert np.array_equal(sims["on"].get("p"), sims["off"].get("p")), k
        _say("  step", k, "vcycles", a["vcycles"], "identical")
    for s in sims.values():
        s.close()
