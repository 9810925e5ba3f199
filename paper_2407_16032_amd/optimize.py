"""Davidon's cubic-interpolation search for the optimum of a function of one
parameter from its values and exact derivatives.

The paper optimises the spin of its control cylinders this way (applications
section, optimized control cylinders): C_P and dC_P/dxi are evaluated at points
bracketing the optimum, and inverse cubic interpolation shrinks the interval in
a few iterations.  Here the derivative comes from the library's discrete adjoint
(``adjoint.RotatingCylinderDrag``).  The interpolant is the cubic that matches
the values and slopes at both ends of the bracket (Davidon's method; Hermite
interpolation); its interior stationary point with positive curvature is the
next evaluation, safeguarded toward the bracket's middle.
"""
from __future__ import annotations

import math
from typing import Callable, Dict, List, Tuple

FG = Callable[[float], Tuple[float, float]]


def cubic_step(a: float, fa: float, ga: float, b: float, fb: float, gb: float) -> float:
    """Minimiser in (a, b) of the cubic with values fa, fb and slopes ga, gb at a, b.

    In s = (x - a) / (b - a) the cubic is p(s) = fa + ga h s + c2 s^2 + c3 s^3 with
    h = b - a, c3 = (ga + gb) h - 2 (fb - fa), c2 = fb - fa - ga h - c3; p'(s) = 0 is a
    quadratic whose root with p'' > 0 is taken.  With ga < 0 < gb such a root lies in
    (0, 1)."""
    h = b - a
    c3 = (ga + gb) * h - 2.0 * (fb - fa)
    c2 = fb - fa - ga * h - c3
    # p'(s) = ga h + 2 c2 s + 3 c3 s^2
    A, B, C = 3.0 * c3, 2.0 * c2, ga * h
    if abs(A) < 1e-14 * (abs(B) + abs(C)):
        s = -C / B  # the quadratic case (the cubic term vanishes)
    else:
        disc = B * B - 4.0 * A * C
        if disc < 0.0:
            disc = 0.0
        # the root where p'' = 2 c2 + 6 c3 s = B + 2 A s is positive; written without
        # cancellation (q and C / q)
        q = -0.5 * (B + math.copysign(math.sqrt(disc), B))
        roots = [q / A, C / q] if q != 0.0 else [-B / (2.0 * A)]
        s = None
        for r in roots:
            if B + 2.0 * A * r > 0.0 and 0.0 <= r <= 1.0:
                s = r
        if s is None:
            s = 0.5
    return a + s * h


def davidon_minimize(fg: FG, a: float, b: float, tol: float = 1e-3, gtol: float = 0.0, maxit: int = 20,
                     safeguard: float = 1e-3) -> Dict:
    """Minimise f on [a, b] given fg(x) -> (f(x), f'(x)) with f'(a) < 0 < f'(b).

    Each iteration evaluates the cubic interpolant's minimiser (kept at least
    ``safeguard`` of the bracket away from its ends) and replaces the end whose
    slope has the same sign; when three steps in a row have not halved the bracket
    (one end converging while the other stays put) the next point is the midpoint.
    Stops when the bracket is shorter than ``tol``, when |f'| <= gtol at the new
    point, or after ``maxit`` evaluations.  Returns the best point, its value and
    slope, the evaluations in order and the final bracket."""
    fa, ga = fg(a)
    fb, gb = fg(b)
    hist: List[Tuple[float, float, float]] = [(a, fa, ga), (b, fb, gb)]
    if not (ga < 0.0 < gb):
        raise ValueError("the bracket must satisfy f'(a) < 0 < f'(b) (got %g, %g)" % (ga, gb))
    it = 0
    widths = [b - a]
    while b - a > tol and it < maxit:
        if len(widths) >= 4 and widths[-1] > 0.5 * widths[-4]:
            x = 0.5 * (a + b)
            widths = [b - a]
        else:
            x = cubic_step(a, fa, ga, b, fb, gb)
            lo, hi = a + safeguard * (b - a), b - safeguard * (b - a)
            x = min(max(x, lo), hi)
        fx, gx = fg(x)
        hist.append((x, fx, gx))
        it += 1
        if gx > 0.0:
            b, fb, gb = x, fx, gx
        else:
            a, fa, ga = x, fx, gx
        widths.append(b - a)
        if abs(gx) <= gtol:
            break
    best = min(hist, key=lambda e: e[1])
    return {"x": best[0], "f": best[1], "g": best[2], "evaluations": hist, "bracket": (a, b),
            "iterations": it}


def davidon_maximize(fg: FG, a: float, b: float, **kw) -> Dict:
    """Maximise f on [a, b] (f'(a) > 0 > f'(b)) by minimising -f."""
    out = davidon_minimize(lambda x: tuple(-v for v in fg(x)), a, b, **kw)
    out["f"], out["g"] = -out["f"], -out["g"]
    out["evaluations"] = [(x, -f, -g) for x, f, g in out["evaluations"]]
    return out


def optimize_rotation_rate(problem, R: float, a: float, b: float, maximize: bool = True, **kw) -> Dict:
    """Davidon search over the rotation rate xi in [a, b] of a rotating-cylinder
    problem (``adjoint.RotatingCylinderDrag``): each evaluation runs the forward
    rollout with checkpoints and the reverse sweep, giving J(xi) and dJ/dxi.  The
    evaluations carry their wall time."""
    import time
    log = []

    def fg(xi):
        t0 = time.perf_counter()
        J, gx, _ = problem.value_and_grad(xi, R)
        log.append({"xi": xi, "J": J, "dJ_dxi": gx, "seconds": time.perf_counter() - t0})
        return J, gx

    out = (davidon_maximize if maximize else davidon_minimize)(fg, a, b, **kw)
    out["log"] = log
    return out
