"""The allocation-free force entry point (wl_forces_static, static device scratch)
against wl_forces, through the C ABI: two calls in a row on simulations of
different sizes, the second smaller, and a repeat on the first."""
import sys

import numpy as np
import pytest

import wlsynth
from gpu_util import make_pair

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _both(gpu):
    fp, fv = gpu.forces()
    sp, sv = gpu.forces_static()
    return np.array(fp + fv), np.array(sp + sv)


def _check(a, b):
    scale = max(float(np.max(np.abs(a))), 1e-300)
    np.testing.assert_allclose(b, a, rtol=0, atol=1e-12 * scale)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_forces_static_matches_forces(prec):
    big = wlsynth.sphere_3d(n=(96, 48, 48), D=14.0, center=(30.0, 24.0, 24.0))
    small = wlsynth.circle_2d(n=(64, 32), R=5.0, center=(16.0, 16.0))
    _say("no-alloc forces", prec, big.name)
    _, g1 = make_pair(big, prec, 1e-6)
    for _ in range(3):
        g1.step()
    ref1, got1 = _both(g1)
    assert np.any(ref1 != 0.0)
    _check(ref1, got1)
    _say("no-alloc forces", prec, small.name, "(smaller grid, same scratch)")
    _, g2 = make_pair(small, prec, 1e-6)
    for _ in range(3):
        g2.step()
    ref2, got2 = _both(g2)
    _check(ref2, got2)
    # the first simulation again: nothing of the second call's partials is left over
    ref1b, got1b = _both(g1)
    np.testing.assert_array_equal(ref1b, ref1)
    _check(ref1b, got1b)
    g1.close()
    g2.close()


def test_forces_static_without_body_is_zero():
    w = wlsynth.tgv_3d(N=16)
    _, g = make_pair(w, "f64", 1e-8)
    fp, fv = g.forces_static()
    assert fp == [0.0, 0.0, 0.0] and fv == [0.0, 0.0, 0.0]
    g.close()
