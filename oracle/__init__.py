"""FP64 CPU oracle of one BDIM projection time step (WaterLily.jl method).

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow reference the HIP
path is checked against.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it; the product library never
does, and it shares no code with the HIP kernels.

It follows the paper's numerical-methods section: the BDIM meta-equation
(convolution of the fluid momentum equation with the body equation through a
kernel of half-width eps, built from the signed distance and normal), a
staggered uniform Cartesian finite-volume grid with one ghost layer
(``inside(p)`` excludes ghosts), second-order central differences for pressure
and diffusion, a flux-limited QUICK convective scheme, an explicit
predictor-corrector step with a pressure projection after each stage, a
geometric multigrid Poisson solver with a PCG smoother, and an adaptive CFL
time step.  Where the paper gives no formula, the reading used is stated in
each function's docstring.

Modules
-------
grid      padded index helpers (periodic wrap, validity masks)
moments   BDIM kernel K and its moments mu0, mu1
body      analytic bodies, rigid motion, ``measure``, force integrals
flux      limited QUICK face value and the convection-diffusion residual R(u)
poisson   variable-coefficient Poisson operator, multigrid V-cycle, PCG smoother
solver    BDIM blend, boundary conditions, projection, CFL, the full step
pgnet     the learned multigrid initial guess (an extension): conv net, its
          backward pass and Adam, on BF16-rounded inputs, in FP64
adjoint   the rollout objective's exact derivative by complex step (the paper
          differentiates the solver with dual numbers)
"""
from .grid import Grid
from .moments import kernel, mu0, mu1
from .solver import Sim

__all__ = ["Grid", "Sim", "kernel", "mu0", "mu1"]
