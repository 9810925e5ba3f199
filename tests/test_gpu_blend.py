"""The BDIM blend applied inside the 3-D flux launch against the separate blend
pass over every face.

Outside the body box the coefficients are body-free (mu0 = L with L = 0 or 1 on
the fine level, mu1 = 0, V = 0), so the flux launch blends those faces with the
same operations the separate pass uses, and a launch over the box blends the
rest from the f~ the flux launch kept near the box.  Both forms must give the
same velocity and pressure bit for bit, step after step: no body, a static body
near a periodic wrap, a moving plate, a deforming mapped body and the
symmetric-subdomain TGV, in FP32 and FP64.
"""
import sys

import numpy as np
import pytest
import torch

import wlsynth
from gpu_util import small_cases

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _cases():
    c = small_cases()
    # a sphere 4.2 cells from z = 0 of a periodic z axis: the body box (reach + 3
    # cells) takes in the ghost plane 0, so the box's blend reads f~ across the wrap
    wrap = wlsynth.Workload("wrapz", (70, 24, 40), (1.0, 0.0, 0.0), 0.02,
                            wlsynth.Body("sphere", center=(20.3, 12.2, 4.2), radius=2.0),
                            periodic=(False, False, True), convective_exit=True)
    return {
        "tgv3d_f32": (c["tgv3d"], "f32"),
        "sphere3d_f32": (c["sphere3d"], "f32"),
        "plate3d_f32": (c["plate3d"], "f32"),
        "plate3d_f64": (c["plate3d"], "f64"),
        "wrapz_f64": (wrap, "f64"),
        "wrapz_f32": (wrap, "f32"),
        "jelly3d_f32": (wlsynth.jelly_3d(n=12), "f32"),
        "tgvsym_f32": (wlsynth.tgv_sym_3d(N=48), "f32"),
    }


CASES = _cases()


@pytest.mark.parametrize("name", sorted(CASES))
def test_blend_in_flux_matches_the_separate_pass(name):
    from paper_2407_16032_amd import Simulation
    w, prec = CASES[name]
    _say("blend", name, w.n)
    u0 = wlsynth.initial_velocity(w, seed=3)
    body = w.body if w.body.kind != "none" else None
    sims = {}
    for mode in ("auto", "separate"):
        s = Simulation(w.n, w.U, w.nu, body, periodic=w.periodic_mask(), convective_exit=w.convective_exit,
                       prec=prec, tol=1e-5 if prec == "f32" else 1e-10, itmax=64, device="cuda:0",
                       blend_mode=mode)
        s.set_velocity(u0)
        sims[mode] = s
    for k in range(4):
        st = {m: s.step() for m, s in sims.items()}
        a, b = st["auto"], st["separate"]
        assert a["dt"] == b["dt"] and a["vcycles"] == b["vcycles"], (k, a, b)
        ua, ub = sims["auto"].get("u"), sims["separate"].get("u")
        pa, pb = sims["auto"].get("p"), sims["separate"].get("p")
        for c in range(3):
            assert np.array_equal(ua[c], ub[c]), (k, c, float(np.max(np.abs(ua[c] - ub[c]))))
        assert np.array_equal(pa, pb), (k, float(np.max(np.abs(pa - pb))))
        _say("  step", k, "dt", a["dt"], "vcycles", a["vcycles"], "identical")
    for s in sims.values():
        s.close()
