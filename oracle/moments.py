"""BDIM kernel and its zeroth and first moments (test infrastructure).

The paper's numerical-methods section describes the meta-equation as the
fluid and body equations convolved with a kernel of thickness eps built from
the signed distance d.  Reading used: the cosine kernel
K(s) = (1 + cos(pi s))/2 on |s| < 1 (unit integral), s = d/eps, and

    mu0(d) = int_{-1}^{s} K,              (0 deep in the body, 1 in the fluid)
    mu1(d) = -eps int_{-1}^{s} s' K(s') ds'

written out in closed form below.
"""
from __future__ import annotations

import numpy as np


def kernel(s):
    s = np.asarray(s)
    return np.where(np.abs(np.real(s)) < 1.0, 0.5 * (1.0 + np.cos(np.pi * s)), 0.0)


def kernel_eps(d, eps=1.0):
    """Smoothed surface delta K(d/eps)/eps."""
    return kernel(np.asarray(d) / eps) / eps


def mu0(d, eps=1.0):
    """Zeroth moment; exactly 0 / 1 beyond the kernel support (|s| >= 1), where the
    closed form would otherwise carry the rounding of sin(pi)."""
    s = np.clip(np.asarray(d) / eps, -1.0, 1.0)
    inner = 0.5 * (1.0 + s) + np.sin(np.pi * s) / (2.0 * np.pi)
    rs = np.real(s)
    return np.where(rs >= 1.0, 1.0, np.where(rs <= -1.0, 0.0, inner))


def mu1(d, eps=1.0):
    """First moment; exactly 0 beyond the kernel support, where the integral of s K
    over the whole symmetric support vanishes."""
    s = np.clip(np.asarray(d) / eps, -1.0, 1.0)
    inner = eps * (0.25 * (1.0 - s * s)
                   - (s * np.sin(np.pi * s) + (1.0 + np.cos(np.pi * s)) / np.pi) / (2.0 * np.pi))
    return np.where(np.abs(np.real(s)) >= 1.0, 0.0, inner)
