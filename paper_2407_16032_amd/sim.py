"""Python face of the C ABI: a Simulation whose workspace is one torch device tensor.

Only marshalling lives here; every step of the method runs in the HIP library.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence

import torch

from . import _lib as L


def _part_desc(body, ndim, dtype, device, keep) -> L.BodyDesc:
    b = L.BodyDesc()
    b.kind = L.BODY_KIND[body.kind]
    for k, v in enumerate(tuple(body.center)[:3]):
        b.center[k] = v
    # a field the body object does not carry keeps its zero default (no motion)
    b.radius = float(getattr(body, "radius", 0.0))
    for name in ("heave_amp", "pitch_amp", "freq", "phase_h", "phase_p", "spin_omega", "phase_s", "shell"):
        setattr(b, name, float(getattr(body, name, 0.0)))
    for name in ("half_extent", "pivot_offset", "velocity", "heave_dir", "scale_amp", "normal", "grid_origin"):
        arr = getattr(b, name)
        for k, v in enumerate(tuple(getattr(body, name, ()))[:3]):
            arr[k] = float(v)
    b.op = L.BODY_OP[getattr(body, "op", "union")]
    sdf = getattr(body, "sdf_grid", None)
    if sdf is not None:
        import numpy as np
        s = np.asarray(sdf, dtype=np.float64)
        for k in range(ndim):
            b.grid_n[k] = s.shape[k]
        b.grid_h = float(body.grid_h)
        # device copy, x fastest (the library reads it at creation / body update)
        ts = torch.from_numpy(np.ascontiguousarray(s.T)).to(device=device, dtype=dtype)
        keep.append(ts)
        b.sdf_grid = ts.data_ptr()
        vg = getattr(body, "vel_grid", None)
        if vg is not None:
            v = np.asarray(vg, dtype=np.float64)
            tv = torch.from_numpy(np.ascontiguousarray(np.stack([v[c].T for c in range(ndim)]))).to(
                device=device, dtype=dtype)
            keep.append(tv)
            b.vel_grid = tv.data_ptr()
    return b


def _body_desc(body, ndim=3, dtype=torch.float32, device="cpu", keep=None) -> L.BodyDesc:
    """The head of a chain of wl_body_desc parts; ``keep`` collects the objects that
    must stay alive while the library reads the chain (parts and sample arrays)."""
    keep = [] if keep is None else keep
    if body is None or getattr(body, "kind", "none") == "none":
        b = L.BodyDesc()
        b.kind = 0
        keep.append(b)
        return b
    parts = body.parts() if hasattr(body, "parts") else [body]
    descs = [_part_desc(p, ndim, dtype, device, keep) for p in parts]
    for k in range(len(descs) - 1):
        descs[k].next = C.pointer(descs[k + 1])
    keep.extend(descs)
    return descs[0]


class Simulation:
    """BDIM projection solver on one GPU (fields live in ``self.workspace``).

    Parameters mirror ``wl_sim_desc`` / ``wl_body_desc`` in include/wlmi.h.
    ``body`` is any object with the attributes of ``wl_body_desc`` (kind is
    'none', 'sphere', 'box', 'grid' or 'plane'), optionally chained through
    ``parts()`` (``wlsynth.Body``).
    """

    def __init__(self, n: Sequence[int], U: Sequence[float], nu: float, body=None,
                 periodic: Sequence[bool] = (), convective_exit: bool = False, prec: str = "f32",
                 eps: float = 1.0, dt0: float = 0.25, dt_max: float = 10.0, cfl_nu: float = 5.0,
                 tol: float = 1e-6, itmax: int = 32, pcg_iters: int = 6, device="cuda:0",
                 stream: Optional[torch.cuda.Stream] = None, learned_guess: bool = False,
                 adjoint: bool = False, solver_path: str = "auto", L_ref: float = 1.0,
                 reduce_mode: str = "auto", blend_mode: str = "auto", vcycle_graph: str = "auto"):
        self.lib = L.load()
        nd = len(n)
        d = L.SimDesc()
        d.ndim = nd
        for k in range(nd):
            d.n[k] = int(n[k])
            d.U[k] = float(U[k])
        d.nu = float(nu)
        d.L = float(L_ref)
        d.periodic_mask = sum((1 << k) for k, p in enumerate(periodic) if p)
        d.convective_exit = 1 if convective_exit else 0
        d.prec = L.WL_F64 if prec == "f64" else L.WL_F32
        d.eps, d.dt0, d.dt_max, d.cfl_nu_coef = eps, dt0, dt_max, cfl_nu
        d.mg_tol, d.mg_itmax, d.pcg_iters = tol, itmax, pcg_iters
        d.learned_guess = 1 if learned_guess else 0
        d.adjoint = 1 if adjoint else 0
        d.solver_path = {"auto": 0, "tiles": 1, "flat": 2, "generic": 3}[solver_path]
        d.reduce_mode = {"auto": 0, "single": 1, "two_stage": 2}[reduce_mode]
        d.blend_mode = {"auto": 0, "separate": 1}[blend_mode]
        d.vcycle_graph = {"auto": 0, "off": 1, "on": 2}[vcycle_graph]
        self.desc = d
        self.ndim = nd
        self.n = tuple(int(v) for v in n)
        self.dtype = torch.float64 if prec == "f64" else torch.float32
        self.device = torch.device(device)
        self._keep = []
        self.bdesc = _body_desc(body, nd, self.dtype, self.device, self._keep)
        nbytes = self.lib.wl_workspace_bytes(C.byref(d), C.byref(self.bdesc))
        if nbytes == 0:
            raise L.WlError("invalid simulation description: %s" % self.lib.wl_last_error().decode())
        # workspace: one caller-owned allocation (torch), 256-byte aligned
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        self._off = (-base) % 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        L.check(self.lib.wl_sim_create(C.byref(d), C.byref(self.bdesc), C.c_void_p(base + self._off),
                                       C.c_size_t(nbytes), C.c_void_p(self.stream.cuda_stream),
                                       C.byref(h)), "wl_sim_create")
        self._h = h
        # the library holds its own copies of the body now
        torch.cuda.synchronize(self.device)
        self._keep = [self.bdesc]

    # ------------------------------------------------------------------ life
    def close(self):
        if getattr(self, "_h", None):
            self.lib.wl_sim_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------- the method
    def measure(self, t: float):
        L.check(self.lib.wl_measure_body(self._h, float(t)), "wl_measure_body")

    def step(self, remeasure: bool = True) -> dict:
        st = L.StepStats()
        L.check(self.lib.wl_step(self._h, 1 if remeasure else 0, C.byref(st)), "wl_step")
        return {"dt": st.dt, "t": st.t, "dt_next": st.dt_next, "vcycles": (st.vcycles[0], st.vcycles[1]),
                "res0_linf": (st.res0_linf[0], st.res0_linf[1]),
                "res_linf": (st.res_linf[0], st.res_linf[1]), "res_l2": (st.res_l2[0], st.res_l2[1]),
                "div_linf": st.div_linf, "converged": bool(st.converged)}

    def apply_bc(self):
        L.check(self.lib.wl_apply_bc(self._h), "wl_apply_bc")

    def conv_diff(self):
        L.check(self.lib.wl_conv_diff(self._h), "wl_conv_diff")
        return self.field("f")

    def project(self, w: float) -> dict:
        st = L.SolveStats()
        L.check(self.lib.wl_project(self._h, float(w), C.byref(st)), "wl_project")
        return self._solve_dict(st)

    def poisson_solve(self, rhs: Optional[torch.Tensor] = None, x: Optional[torch.Tensor] = None,
                      tol: float = 0.0, itmax: int = 0) -> dict:
        st = L.SolveStats()
        rp = C.c_void_p(rhs.data_ptr()) if rhs is not None else None
        xp = C.c_void_p(x.data_ptr()) if x is not None else None
        L.check(self.lib.wl_poisson_solve(self._h, rp, xp, float(tol), int(itmax), C.byref(st)),
                "wl_poisson_solve")
        return self._solve_dict(st)

    @staticmethod
    def _solve_dict(st) -> dict:
        return {"vcycles": st.vcycles, "res0_linf": st.res0_linf, "res_linf": st.res_linf,
                "res_l2": st.res_l2, "converged": bool(st.converged)}

    def forces(self):
        fp = (C.c_double * 3)()
        fv = (C.c_double * 3)()
        L.check(self.lib.wl_forces(self._h, fp, fv), "wl_forces")
        return list(fp)[:self.ndim], list(fv)[:self.ndim]

    def forces_static(self):
        """wl_forces through the allocation-free entry point (static device scratch)."""
        fp = (C.c_double * 3)()
        fv = (C.c_double * 3)()
        L.check(self.lib.wl_forces_static(self._h, fp, fv), "wl_forces_static")
        return list(fp)[:self.ndim], list(fv)[:self.ndim]

    # ------------------------------------------------------------- state
    def field(self, name: str, level: int = 0) -> torch.Tensor:
        """Zero-copy view (components, pz, py, nx+2) into the workspace."""
        ptr = C.c_void_p()
        shape = (C.c_int64 * 4)()
        strides = (C.c_int64 * 4)()
        L.check(self.lib.wl_field(self._h, L.FIELDS[name], int(level), C.byref(ptr), shape, strides),
                "wl_field")
        esz = torch.tensor([], dtype=self.dtype).element_size()
        off = (ptr.value - self.workspace.data_ptr())
        assert off % esz == 0
        flat = self.workspace.view(self.dtype) if self.workspace.numel() % esz == 0 else \
            self.workspace[: (self.workspace.numel() // esz) * esz].view(self.dtype)
        return flat.as_strided(tuple(shape), tuple(strides), off // esz)

    def scalar_buffer(self) -> torch.Tensor:
        """A new zeroed device array in the pressure layout, returned as the
        (pz, py, nx+2) view of a (pz, py, px) allocation; pass it to poisson_solve."""
        v = self.field("p")
        pz, py, nxp = v.shape[1], v.shape[2], v.shape[3]
        px = v.stride(2)
        store = torch.zeros((pz, py, px), dtype=self.dtype, device=self.device)
        return store[:, :, :nxp]

    def levels(self):
        nl = C.c_int()
        L.check(self.lib.wl_levels(self._h, C.byref(nl), 0, None), "wl_levels")
        out = []
        for l in range(nl.value):
            nn = (C.c_int64 * 3)()
            L.check(self.lib.wl_levels(self._h, None, l, nn), "wl_levels")
            out.append(tuple(nn)[:self.ndim])
        return out

    def profile(self, enable: bool = True, groups=None):
        """Per-launch event timing of every kernel group, or only of the named ones."""
        if groups is None or not enable:
            L.check(self.lib.wl_profile(self._h, 1 if enable else 0), "wl_profile")
            return
        mask = 0
        for name in groups:
            mask |= 1 << L.KERNELS.index(name)
        L.check(self.lib.wl_profile_groups(self._h, mask), "wl_profile_groups")

    def profile_read(self) -> dict:
        out = {}
        for k, name in enumerate(L.KERNELS):
            ms = C.c_double()
            n = C.c_int64()
            L.check(self.lib.wl_profile_read(self._h, k, C.byref(ms), C.byref(n)), "wl_profile_read")
            out[name] = (ms.value, n.value)
        return out

    # ------------------------------------------------ learned initial guess
    def pg_set_weights(self, flat):
        import numpy as np
        w = np.ascontiguousarray(flat, dtype=np.float32)
        assert w.size == L.PG_PARAMS
        L.check(self.lib.wl_pg_set_weights(self._h, w.ctypes.data_as(C.POINTER(C.c_float))), "wl_pg_set_weights")

    def pg_get_weights(self):
        import numpy as np
        w = np.zeros(L.PG_PARAMS, dtype=np.float32)
        L.check(self.lib.wl_pg_get_weights(self._h, w.ctypes.data_as(C.POINTER(C.c_float))), "wl_pg_get_weights")
        return w

    def pg_mode(self, mode: int, lr: float = 1e-3, train_iters: int = 1, crops: int = 2, seed: int = 0):
        L.check(self.lib.wl_pg_mode(self._h, int(mode), float(lr), int(train_iters), int(crops), int(seed)),
                "wl_pg_mode")

    @staticmethod
    def _box(n):
        return (C.c_int64 * 3)(*[int(v) for v in n])

    def pg_forward(self, x_box: torch.Tensor, n) -> torch.Tensor:
        """x_box: bfloat16 device tensor [P, 4] on the box n (with halo); returns y [P] float32."""
        y = torch.zeros(x_box.shape[0], dtype=torch.float32, device=self.device)
        L.check(self.lib.wl_pg_forward(self._h, C.c_void_p(x_box.data_ptr()), self._box(n),
                                       C.c_void_p(y.data_ptr())), "wl_pg_forward")
        torch.cuda.synchronize(self.device)
        return y

    def pg_train_step(self, x_box, target, mask, n, apply: bool = False):
        import numpy as np
        g = np.zeros(L.PG_PARAMS, dtype=np.float32)
        loss = C.c_double()
        L.check(self.lib.wl_pg_train_step(self._h, C.c_void_p(x_box.data_ptr()), C.c_void_p(target.data_ptr()),
                                          C.c_void_p(mask.data_ptr()), self._box(n),
                                          g.ctypes.data_as(C.POINTER(C.c_float)), C.byref(loss),
                                          1 if apply else 0), "wl_pg_train_step")
        return g, loss.value

    def pg_stats(self):
        loss = C.c_double()
        steps = C.c_int64()
        snaps = C.c_int64()
        used = C.c_int64()
        tried = C.c_int64()
        L.check(self.lib.wl_pg_stats(self._h, C.byref(loss), C.byref(steps), C.byref(snaps), C.byref(used),
                                     C.byref(tried)), "wl_pg_stats")
        return {"loss": loss.value, "train_steps": steps.value, "snapshots": snaps.value,
                "guesses_used": used.value, "guesses_tried": tried.value}

    # ---------------------------------------------------- discrete adjoint
    def body_update(self, body):
        keep = []
        self.bdesc = _body_desc(body, self.ndim, self.dtype, self.device, keep)
        L.check(self.lib.wl_body_update(self._h, C.byref(self.bdesc)), "wl_body_update")
        torch.cuda.synchronize(self.device)

    def body_box(self, level: int = 0):
        """(lo, hi) padded index box of a level outside of which coefficients are body-free."""
        lo = (C.c_int * 3)()
        hi = (C.c_int * 3)()
        L.check(self.lib.wl_body_box(self._h, int(level), lo, hi), "wl_body_box")
        return tuple(lo)[:self.ndim], tuple(hi)[:self.ndim]

    def adj_reset(self):
        L.check(self.lib.wl_adj_reset(self._h), "wl_adj_reset")

    def adj_forces(self, direction, weight: float) -> float:
        d = (C.c_double * 3)(*[float(v) for v in (list(direction) + [0.0, 0.0])[:3]])
        val = C.c_double()
        L.check(self.lib.wl_adj_forces(self._h, d, float(weight), C.byref(val)), "wl_adj_forces")
        return val.value

    def adj_step(self, tol: float = 0.0) -> dict:
        fst = L.StepStats()
        ast = (L.SolveStats * 2)()
        L.check(self.lib.wl_adj_step(self._h, float(tol), C.byref(fst), ast), "wl_adj_step")
        return {"dt": fst.dt, "vcycles": (fst.vcycles[0], fst.vcycles[1]),
                "adj_vcycles": (ast[0].vcycles, ast[1].vcycles),
                "adj_res_linf": (ast[0].res_linf, ast[1].res_linf)}

    def adj_step_cfl(self, dt_from_cfl: bool, tol: float = 0.0) -> dict:
        """Reverse of one step whose dt follows the CFL rule; also returns dt_bar."""
        fst = L.StepStats()
        ast = (L.SolveStats * 2)()
        dtb = C.c_double()
        L.check(self.lib.wl_adj_step_cfl(self._h, float(tol), 1 if dt_from_cfl else 0, C.byref(dtb), C.byref(fst),
                                         ast), "wl_adj_step_cfl")
        return {"dt": fst.dt, "vcycles": (fst.vcycles[0], fst.vcycles[1]), "dt_bar": dtb.value,
                "adj_vcycles": (ast[0].vcycles, ast[1].vcycles),
                "adj_res_linf": (ast[0].res_linf, ast[1].res_linf)}

    def adj_body_grad(self):
        dR = C.c_double()
        dW = C.c_double()
        L.check(self.lib.wl_adj_body_grad(self._h, C.byref(dR), C.byref(dW)), "wl_adj_body_grad")
        return dR.value, dW.value

    def save_state(self):
        """Device copies of (u, p) and the clock: a checkpoint."""
        return (self.field("u").clone(), self.field("p").clone(), self.time())

    def load_state(self, state, dt_next: Optional[float] = None):
        u, p, (t, dt) = state
        self.field("u").copy_(u)
        self.field("p").copy_(p)
        self.set_time(t, dt if dt_next is None else dt_next)

    def set_time(self, t: float, dt_next: float):
        L.check(self.lib.wl_set_time(self._h, float(t), float(dt_next)), "wl_set_time")

    def sim_time(self) -> float:
        """Convective time t |U| / L."""
        ts = C.c_double()
        L.check(self.lib.wl_sim_time(self._h, C.byref(ts)), "wl_sim_time")
        return ts.value

    def time(self):
        t = C.c_double()
        dt = C.c_double()
        L.check(self.lib.wl_get_time(self._h, C.byref(t), C.byref(dt)), "wl_get_time")
        return t.value, dt.value

    # convenience converters between the padded [comp][z][y][x] views and
    # per-component arrays indexed [x, y(, z)]
    def get(self, name: str, level: int = 0):
        v = self.field(name, level)
        torch.cuda.synchronize(self.device)
        out = []
        for c in range(v.shape[0]):
            a = v[c]
            a = a[0].transpose(0, 1) if self.ndim == 2 else a.permute(2, 1, 0)
            out.append(a.to("cpu", torch.float64).numpy().copy())
        return out

    def set(self, name: str, arrays, level: int = 0):
        v = self.field(name, level)
        for c, arr in enumerate(arrays):
            t = torch.as_tensor(arr, dtype=self.dtype)
            t = t.transpose(0, 1).unsqueeze(0) if self.ndim == 2 else t.permute(2, 1, 0)
            v[c].copy_(t.to(self.device))
        torch.cuda.synchronize(self.device)

    def set_velocity(self, arrays):
        self.set("u", arrays)
        self.apply_bc()
