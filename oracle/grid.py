"""Padded staggered grid helpers (test infrastructure; see ``oracle/__init__``).

Grid convention (paper, software-design section: ``inside(p)`` skips one
ghost layer per side; numerical-methods section: uniform cells, h = 1):
interior cells ``I_d = 1..N_d`` inside a padded array ``0..N_d+1``.  Cell ``I``
is centred at ``x = I - 1/2``; velocity component ``u_i[I]`` sits on the lower
``i``-face of cell ``I``.
"""
from __future__ import annotations

import numpy as np


class Grid:
    def __init__(self, n, periodic=None):
        self.n = tuple(int(v) for v in n)
        self.ndim = len(self.n)
        if periodic is None or len(periodic) == 0:
            periodic = (False,) * self.ndim
        self.periodic = tuple(bool(p) for p in periodic)
        self.shape = tuple(N + 2 for N in self.n)

    # -- index maps ---------------------------------------------------------
    def src(self, axis: int, k: int):
        """Source index of ``I + k`` along ``axis`` for every padded ``I``.

        Periodic axes wrap into ``1..N``; otherwise indices outside ``0..N+1``
        are flagged invalid (and clipped so that gathering stays in range).
        """
        N = self.n[axis]
        I = np.arange(N + 2) + k
        if self.periodic[axis]:
            return 1 + np.mod(I - 1, N), np.ones(N + 2, dtype=bool)
        valid = (I >= 0) & (I <= N + 1)
        return np.clip(I, 0, N + 1), valid

    def shift(self, a: np.ndarray, axis: int, k: int):
        """``b[I] = a[I + k e_axis]`` and a validity mask of the same shape."""
        idx, valid = self.src(axis, k)
        b = np.take(a, idx, axis=axis)
        shp = [1] * self.ndim
        shp[axis] = -1
        return b, np.broadcast_to(valid.reshape(shp), a.shape)

    def sh(self, a: np.ndarray, axis: int, k: int) -> np.ndarray:
        return self.shift(a, axis, k)[0]

    # -- index sets ---------------------------------------------------------
    def interior(self):
        return tuple(slice(1, N + 1) for N in self.n)

    def interior_mask(self) -> np.ndarray:
        m = np.zeros(self.shape, dtype=bool)
        m[self.interior()] = True
        return m

    def unknown_mask(self, comp: int) -> np.ndarray:
        """Faces of component ``comp`` whose value the momentum update computes.

        All interior cells, except that along a non-periodic ``comp`` axis the
        two boundary faces (index 1 and N+1) are prescribed, so ``2..N``.
        """
        m = np.zeros(self.shape, dtype=bool)
        sl = []
        for a, N in enumerate(self.n):
            if a == comp and not self.periodic[a]:
                sl.append(slice(2, N + 1))
            else:
                sl.append(slice(1, N + 1))
        m[tuple(sl)] = True
        return m

    def zeros(self, dtype=np.float64) -> np.ndarray:
        return np.zeros(self.shape, dtype=dtype)

    def coarsenable(self) -> bool:
        """Multigrid coarsening rule: every interior size even, coarse min >= 4."""
        return all(N % 2 == 0 for N in self.n) and min(self.n) // 2 >= 4

    def coarse(self) -> "Grid":
        return Grid(tuple(N // 2 for N in self.n), self.periodic)
