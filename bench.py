#!/usr/bin/env python3
"""Throughput of the FP32 BDIM projection step on one MI355X.

Metric: ns per grid point per time step (lower is better), with the MG
V-cycles per step and the HBM-roofline fraction of the dominant kernel.

Default workload: the heaving-pitching flat plate, 768 x 384 x 384 cells
(113 M), chord 64 cells, Re = 5000, body re-measured every step, convective
exit, FP32 fields with FP64 reductions, multigrid to a residual max-norm of
1e-5.  Synthetic input: uniform inflow plus seeded 1e-3 noise.

Usage: python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-cpu-baseline]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E

# the paper's own figure for a workload measured here (another machine's: context)
PAPER_NS = {"tgv512sym": {"value": 1.57, "unit": "ns/point/step", "hardware": "NVIDIA H100 64 GB, FP32",
                          "workload": "TGV Re = 1600, 512^3 cells on the symmetric subdomain, 100 steps",
                          "source": "paper, performance section (benchmarks)"}}


def workloads():
    import wlsynth
    return {
        "plate3d": wlsynth.plate_3d(scale=1),
        "tgv3d": wlsynth.tgv_3d(N=128),
        "tgv512sym": wlsynth.tgv_sym_3d(N=512),
        "sphere3d": wlsynth.sphere_3d(),
        "circle2d": wlsynth.circle_2d(),
    }


def kernel_bytes(name, ndim, cells, faces, esize, has_body, pcg_iters, box_cells=None, box_faces=None,
                 tiled=False, flat=False, fused=False):
    """Algorithmic bytes of one launch of the kernels as built: each field the pass
    needs is read once, each output written once.

    cells = interior cells of the fine level, faces = padded points per component.
    Coefficient fields (L, iD on cells; V, mu0, mu1 on faces) are only needed inside
    the body box (box_cells / box_faces): outside it the kernels evaluate their
    body-free closed form.  On tiled levels (3-D, large) pass A does not store q and
    pass B recomputes it from e (pass B then needs L and iD in the box); the flat
    form of the fine level (``flat``) moves the same fields.  With ``fused`` (3-D
    steps) the flux launch writes the blended velocity outside the body box and f~
    only near it, and the blend launch covers the box's faces alone.
    """
    n = ndim
    bc = cells if box_cells is None else box_cells
    bf = faces if box_faces is None else box_faces
    if name == "pcg_a":
        # reads r, and e_old except in the first sweep; writes e_new (and q on the generic
        # path); iD, L (n) in the box
        fields = (1 + (pcg_iters - 1) / pcg_iters) + (1 if (tiled or flat) else 2)
        return (fields * cells + (1 + n) * bc) * esize
    if name == "pcg_b":
        if tiled or flat:  # reads e, x, r; writes x, r; iD and L (n) in the box
            return (5 * cells + (1 + n) * bc) * esize
        return ((4 + 2) * cells + bc) * esize    # reads e, q, x, r; writes x, r; iD in the box
    if name == "divres":
        return ((n + 1 + 2) * cells + (n + 1) * bc) * esize   # u (n), p; writes x, r; L (n), iD in the box
    if name == "project":
        return ((n + 1 + n + 1) * cells + n * bc) * esize     # u (n), x; writes u (n), p; L (n) in the box
    if name == "prolong":
        return ((1 / 2 ** n + 2 + 2) * cells + (n + 1) * bc) * esize  # x_c, x, r; writes x, r; L, iD in the box
    if name == "restrict":
        return (1 + 2 / 2 ** n) * cells * esize      # r; writes r_c, x_c
    if name == "flux":
        # average of predictor (u = u0: n) and corrector (u, u0: 2n); writes f, or with
        # ``fused`` u (n); V (n) in the box, and with ``fused`` f there too
        box = ((2 if fused else 1) * n * bf) if has_body else 0
        return ((1.5 * n + n) * faces + box) * esize
    if name == "bdim":
        body = (n + n + n * n) * bf if has_body else 0     # V, mu0, mu1 in the box
        if fused:                                          # f, u (corrector), writes u: in the box
            return ((n + 0.5 * n + n) * bf + body) * esize
        return ((n + 0.5 * n + n) * faces + body) * esize  # f, u (corrector); writes u
    if name == "cfl":
        return n * cells * esize
    return None


def fine_level_flat(n, esize=4, solver_path="auto"):
    """The fine level takes the flat passes when it is 3-D with >= 2^14 cells and
    rows of whole 16-byte vectors, unless the solver path asks for tiles or the
    generic kernels (the library's rule)."""
    return (len(n) == 3 and solver_path in ("auto", "flat") and n[0] % (16 // esize) == 0
            and n[0] * n[1] * n[2] >= (1 << 14))


def fine_level_tiled(n):
    """The library tiles a 3-D level (64 x 8 columns marching 32 planes, fewer down
    to 8 while the level has under 1024 tiles) when n0 >= 32, n1 >= 8, it has
    >= 2^18 cells and at most 8192 tiles."""
    if len(n) != 3:
        return False
    cols = -(-n[0] // 64) * -(-n[1] // 8)
    depth = 32
    while depth > 8 and cols * -(-n[2] // depth) < 1024:
        depth //= 2
    tiles = cols * -(-n[2] // depth)
    return n[0] >= 32 and n[1] >= 8 and n[0] * n[1] * n[2] >= (1 << 18) and tiles <= 8192


def model_bytes(name, ndim, cells, esize):
    """Bytes of one launch by the fixed algorithmic model of the method (values per
    fine cell, dense coefficients): PCG pass A reads r, e, L (ndim) and writes e, q
    (7 in 3-D, 6 in 2-D); pass B reads x, e, r, q, iD and writes x, r (7);
    restriction 1 + 1/2^ndim; prolongation + increment 7 + 1/2^ndim.  None for
    kernels the model prices only as part of a fused pass."""
    per = {"pcg_a": 4 + ndim, "pcg_b": 7, "restrict": 1 + 1 / 2 ** ndim, "prolong": 7 + 1 / 2 ** ndim}.get(name)
    return None if per is None else per * cells * esize


def box_counts(sim, n):
    """Interior cells and padded faces inside the fine level's body box."""
    lo, hi = sim.body_box(0)
    if lo[0] > hi[0]:
        return 0, 0
    cells = faces = 1
    for a, N in enumerate(n):
        cells *= max(0, min(hi[a], N) - max(lo[a], 1) + 1)
        faces *= max(0, min(hi[a], N + 1) - max(lo[a], 0) + 1)
    return cells, faces


def cpu_sample_workload(w_name):
    """The bounded CPU sample of a workload: the same case at 1/3 of the linear size
    (plate: 256 x 128 x 128 cells)."""
    import wlsynth
    if w_name == "plate3d":
        return wlsynth.plate_3d(scale=3)
    if w_name == "tgv3d":
        return wlsynth.tgv_3d(N=64)
    if w_name == "tgv512sym":
        return wlsynth.tgv_sym_3d(N=128)
    if w_name == "sphere3d":
        return wlsynth.sphere_3d(n=(128, 64, 64), D=16.0, center=(32.0, 32.0, 32.0))
    return wlsynth.circle_2d()


def _oracle_sample_step(job):
    """One FP64 oracle step of the CPU sample (runs in a worker process)."""
    w_name, seed = job
    import wlsynth
    import oracle
    w = cpu_sample_workload(w_name)
    body = w.body if w.body.kind != "none" else None
    s = oracle.Sim(w.n, w.U, w.nu, body, periodic=w.periodic_mask(), convective_exit=w.convective_exit,
                   tol=w.tol)
    s.set_velocity(wlsynth.initial_velocity(w, seed=seed))
    t0 = time.perf_counter()
    s.step()
    return time.perf_counter() - t0, w.cells, w.name


def run_cpu_baseline(w_name):
    """The FP64 oracle (numpy) on a bounded sample, timed on this host's cores in
    worker processes that never touch the GPU: one step alone (one thread), then one
    step per worker on all cores at once (up to 16 workers, independent seeds); the
    all-core aggregate is the reported value."""
    import multiprocessing as mp
    ncpu = os.cpu_count() or 1
    workers = max(1, min(16, ncpu))
    old = os.environ.get("OMP_NUM_THREADS")
    os.environ["OMP_NUM_THREADS"] = "1"  # the workers' numpy: one thread each
    try:
        ctx = mp.get_context("spawn")
        with ctx.Pool(1) as pool:
            dt1, cells, name = pool.map(_oracle_sample_step, [(w_name, 0)])[0]
        print("[bench] oracle, one core: %.1f s for one step of %d cells" % (dt1, cells), file=sys.stderr,
              flush=True)
        with ctx.Pool(workers) as pool:
            res = pool.map(_oracle_sample_step, [(w_name, k) for k in range(workers)], chunksize=1)
    finally:
        if old is None:
            del os.environ["OMP_NUM_THREADS"]
        else:
            os.environ["OMP_NUM_THREADS"] = old
    slowest = max(r[0] for r in res)
    agg = slowest / (workers * cells) * 1e9
    print("[bench] oracle, %d cores: %d steps in parallel, slowest %.1f s" % (workers, workers, slowest),
          file=sys.stderr, flush=True)
    return {"value": round(agg, 2), "unit": "ns/point/step", "cores": workers, "kind": "oracle",
            "sample": "one FP64 step of %s (%d cells) per worker, %d single-threaded numpy workers at once on "
                      "%d host CPUs; aggregate = slowest step / (workers x cells)" % (name, cells, workers, ncpu),
            "host_cpu_count": ncpu,
            "single_core": {"value": round(dt1 / cells * 1e9, 2), "unit": "ns/point/step", "cores": 1,
                            "seconds": round(dt1, 2)}}


def step_byte_model(ndim, has_body, k):
    """Algorithmic bytes per fine cell of one whole FP32 step by the fixed model of the
    method: 4 (F + 105.4 k) in 3-D (F = 79 with a body, 55 without) and 4 (52 + 115.3 k)
    in 2-D, k = V-cycles per step (both solves)."""
    if ndim == 3:
        return 4.0 * ((79.0 if has_body else 55.0) + 105.4 * k)
    return 4.0 * (52.0 + 115.3 * k)


def code_text(src):
    """C++ source without its comments, each line stripped, blank lines dropped:
    two texts that differ only in comments or layout give the same code text."""
    out, i, n = [], 0, len(src)
    while i < n:
        ch = src[i]
        if ch in "\"'":  # string or character literal, copied whole
            j = i + 1
            while j < n and src[j] != ch:
                j += 2 if src[j] == "\\" else 1
            out.append(src[i:j + 1])
            i = j + 1
        elif src.startswith("//", i):
            j = src.find("\n", i)
            i = n if j < 0 else j
        elif src.startswith("/*", i):
            j = src.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        else:
            out.append(ch)
            i += 1
    lines = (ln.strip() for ln in "".join(out).split("\n"))
    return "\n".join(ln for ln in lines if ln)


def kernel_source_hash():
    """Hash of the code (comments and layout aside) of the step's kernels and of
    the host code that launches them."""
    import hashlib
    h = hashlib.sha256()
    for f in ("wl_kernels.hpp", "wl_device.hpp", "wlmi.hip"):
        with open(os.path.join(ROOT, "paper_2407_16032_amd", "csrc", f), encoding="utf-8") as fh:
            h.update(code_text(fh.read()).encode("utf-8"))
    return h.hexdigest()[:16]


def measured_traffic(workload, kernel):
    """HBM bytes per launch from the committed PMC summary, only if the kernel sources
    are unchanged since the counters were taken (else None)."""
    path = os.path.join(ROOT, "profiles", "pmc_%s.md" % workload)
    if not os.path.exists(path):
        return None
    key = {"pcg_a": "k_pcg_a_flat_fine", "pcg_b": "k_pcg_b_flat_fine", "flux": "k_flux_reuse_mean"}.get(kernel)
    src, val = None, None
    with open(path) as f:
        for line in f:
            if line.startswith("kernel-source-sha256-16:"):
                src = line.split(":", 1)[1].strip()
            if key and line.startswith("traffic_bytes " + key + " "):
                val = float(line.split()[2])
    if src != kernel_source_hash():
        return None
    return val


def copy_probe(nbytes):
    """A plain device-to-device copy of known size: reads and writes nbytes each. Its
    FETCH_SIZE / WRITE_SIZE counter values calibrate the counters of the solver kernels."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record()
    b.copy_(a)
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop)
    print(json.dumps({"copy_bytes": nbytes, "ms": ms, "GBps_read_plus_write": 2 * nbytes / (ms * 1e-3) / 1e9}))


def run_adjoint(args):
    """The rotating-cylinder gradient case: 512 x 256 cells, D = 32, Re = 200, xi
    seeded in [0, 2), 400 steps, mean C_D over steps 200..399, FP64 with multigrid to
    1e-12, checkpoints every 20 steps.  Times the forward rollout (with checkpoints)
    and the reverse sweep, and checks the gradient against central differences of
    the HIP forward (h = 1e-3) and, if stored, the oracle's complex-step gradient."""
    import torch
    import wlsynth
    from paper_2407_16032_amd.adjoint import RotatingCylinderDrag
    w = wlsynth.rotating_cylinder_2d()
    xi, R = wlsynth.rotcyl_xi0(0), float(w.body.radius)
    steps = args.steps if args.steps_given else 400
    win = steps // 2
    golden = os.path.join(ROOT, "tests", "golden", "rotcyl_512x256_gradient.json")
    ref = None
    if os.path.exists(golden) and steps == 400:
        with open(golden) as f:
            ref = json.load(f)
    prob = RotatingCylinderDrag(w, wlsynth.initial_velocity(w), steps, win, ckpt=20, prec="f64", tol=1e-12,
                                itmax=200)
    if ref is not None:
        prob.dts = list(ref["dt_schedule"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J, ckpts = prob.value(xi, R, record=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    gx, gR = prob.gradient(xi, R, J, ckpts)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    print("[bench] adjoint: J %.10g dJ/dxi %.10g dJ/dR %.10g  forward %.2f s  reverse %.2f s" % (
        J, gx, gR, t1 - t0, t2 - t1), file=sys.stderr, flush=True)
    h = 1e-3
    fx = (prob.value(xi + h, R) - prob.value(xi - h, R)) / (2 * h)
    fR = (prob.value(xi, R + h) - prob.value(xi, R - h)) / (2 * h)
    # J is only piecewise smooth at small scales (limiter branches switch as the
    # parameters move), so a smaller step is also reported
    h2 = 1e-5
    fx2 = (prob.value(xi + h2, R) - prob.value(xi - h2, R)) / (2 * h2)
    fR2 = (prob.value(xi, R + h2) - prob.value(xi, R - h2)) / (2 * h2)
    out = {
        "metric": "adjoint / forward cost ratio (rotating-cylinder drag gradient, FP64)",
        "value": round((t2 - t1) / (t1 - t0), 3),
        "unit": "ratio",
        "n_gpus": 1, "steps": steps, "higher_is_better": False, "dtype": "f64", "data": "synthetic",
        "config": {"workload": w.name, "cells": w.cells, "xi": xi, "R": R, "window_start": win,
                   "checkpoint_every": 20, "mg_tol": 1e-12},
        "forward_s": round(t1 - t0, 3), "reverse_s": round(t2 - t1, 3),
        "J": J, "dJ_dxi": gx, "dJ_dR": gR,
        "fd_h": h, "fd_dJ_dxi": fx, "fd_dJ_dR": fR,
        "rel_vs_fd": [abs(gx - fx) / abs(fx), abs(gR - fR) / abs(fR)],
        "fd_h2": h2, "fd2_dJ_dxi": fx2, "fd2_dJ_dR": fR2,
        "rel_vs_fd2": [abs(gx - fx2) / abs(fx2), abs(gR - fR2) / abs(fR2)],
        "stats": prob.stats,
    }
    if ref is not None:
        out["oracle"] = {"J": ref["J"], "dJ_dxi": ref["dJ_dxi"], "dJ_dR": ref["dJ_dR"],
                         "rel": [abs(gx - ref["dJ_dxi"]) / abs(ref["dJ_dxi"]),
                                 abs(gR - ref["dJ_dR"]) / abs(ref["dJ_dR"])]}
    print(json.dumps(out))
    prob.sim.close()


def run_learned(args):
    """The learned multigrid guess at its configuration: sphere wake 256 x 128 x 128,
    D = 32, Re = 3700, FP32, tolerance 1e-6; the net trains online on 2000 solver
    snapshots (1000 steps, one crop per solve, 2 Adam steps per solve, from a zero
    output layer), then guides the solves of 1000 evaluation steps with its weights
    frozen; a plain run takes the same 2000 steps.  Both meet the same residual
    tolerance in every solve; reported: ms and V-cycles per evaluation step."""
    import numpy as np
    import torch
    import wlsynth
    from paper_2407_16032_amd import Simulation
    w = wlsynth.sphere_3d()
    train = 1000
    evals = args.steps if args.steps_given else 1000
    kw = dict(convective_exit=True, prec="f32", tol=1e-6, itmax=32, device="cuda:0")
    u0 = wlsynth.initial_velocity(w)
    out = {}
    for mode in ("plain", "learned"):
        sim = Simulation(w.n, w.U, w.nu, w.body, learned_guess=(mode == "learned"), **kw)
        sim.set_velocity(u0)
        if mode == "learned":
            sim.pg_set_weights(wlsynth.pg_init_weights(0, zero_output=True))
            sim.pg_mode(2, lr=1e-3, train_iters=2, crops=1, seed=3)
        t0 = time.perf_counter()
        for k in range(train):
            sim.step()
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t0
        if mode == "learned":
            sim.pg_mode(1)
        vc, res = [], []
        t0 = time.perf_counter()
        for k in range(evals):
            st = sim.step()
            vc.append(sum(st["vcycles"]))
            res.append(max(st["res_linf"]))
        torch.cuda.synchronize()
        t_eval = time.perf_counter() - t0
        ent = {"ms_per_step": round(t_eval / evals * 1e3, 3), "vcycles_per_step": round(float(np.mean(vc)), 3),
               "max_final_residual": max(res), "first_steps_s": round(t_train, 2)}
        if mode == "learned":
            ent["pg"] = sim.pg_stats()
        out[mode] = ent
        print("[bench] %s: %.3f ms/step, %.3f V-cycles/step over %d steps (after %d steps, %.1f s)" % (
            mode, ent["ms_per_step"], ent["vcycles_per_step"], evals, train, t_train), file=sys.stderr, flush=True)
        sim.close()
        del sim
        torch.cuda.empty_cache()
    print(json.dumps({
        "metric": "learned multigrid guess: ms per step and V-cycles per step against the plain warm start",
        "value": out["learned"]["ms_per_step"], "unit": "ms/step", "n_gpus": 1, "steps": evals,
        "higher_is_better": False, "dtype": "f32", "data": "synthetic",
        "config": {"workload": w.name, "cells": w.cells, "mg_tol": 1e-6, "training_steps": train,
                   "snapshots": 2 * train, "evaluation_steps": evals},
        "plain": out["plain"], "learned": out["learned"],
        "vcycles_saved_per_step": round(out["plain"]["vcycles_per_step"] - out["learned"]["vcycles_per_step"], 3),
        "step_time_ratio": round(out["learned"]["ms_per_step"] / out["plain"]["ms_per_step"], 4)}))


def run_optimize(args):
    """Davidon optimisation of the rotation rate of the rotating-cylinder case
    (512 x 256 cells, D = 32, Re = 200, 400 steps, window 200..399, FP64) for the
    Magnus lift efficiency -mean C_L / mean C_D, each evaluation a forward rollout
    with checkpoints every 20 steps and the reverse sweep of the adjoint with live
    CFL time steps."""
    import torch
    import wlsynth
    from paper_2407_16032_amd.adjoint import RotatingCylinderDrag
    from paper_2407_16032_amd.optimize import optimize_rotation_rate
    w = wlsynth.rotating_cylinder_2d()
    R = float(w.body.radius)
    steps = args.steps if args.steps_given else 400
    prob = RotatingCylinderDrag(w, wlsynth.initial_velocity(w), steps, steps // 2, ckpt=20, prec="f64", tol=1e-10,
                                itmax=200, live_dt=True, objective="lift_to_drag")
    t0 = time.perf_counter()
    out = optimize_rotation_rate(prob, R, 1.0, 2.5, maximize=True, tol=0.01, maxit=10)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    for e in out["log"]:
        print("[bench] xi %.5f  J %.6f  dJ/dxi %+.6f  %.1f s" % (e["xi"], e["J"], e["dJ_dxi"], e["seconds"]),
              file=sys.stderr, flush=True)
    print(json.dumps({
        "metric": "Davidon optimisation of the rotation rate by the adjoint (live CFL steps)",
        "value": round(wall, 2), "unit": "s", "n_gpus": 1, "steps": steps, "higher_is_better": False,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": w.name, "objective": "-mean C_L / mean C_D over steps %d..%d" % (steps // 2, steps - 1),
                   "bracket": [1.0, 2.5], "R": R, "mg_tol": 1e-10},
        "xi_opt": out["x"], "J_opt": out["f"], "dJ_dxi_at_opt": out["g"], "evaluations": out["log"],
        "bracket_final": out["bracket"]}))
    prob.sim.close()


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--windows", type=int, default=3,
                    help="timed windows of --steps steps each; the value is their median")
    ap.add_argument("--workload", default="plate3d", choices=sorted(workloads().keys()))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--solver-path", default="auto", choices=["auto", "tiles", "flat", "generic"],
                    help="kernels of the large 3-D multigrid levels (same arithmetic)")
    ap.add_argument("--blend", default="auto", choices=["auto", "separate"],
                    help="BDIM blend inside the 3-D flux launch outside the body box (auto) or a separate pass")
    ap.add_argument("--vcycle-graph", default="auto", choices=["auto", "off", "on"],
                    help="replay the coarse part of each multigrid cycle from a HIP graph (auto: unless the body moves)")
    ap.add_argument("--no-profile", action="store_true", help="skip per-kernel event timing")
    ap.add_argument("--adjoint", action="store_true",
                    help="run the rotating-cylinder gradient case instead (adjoint vs forward cost)")
    ap.add_argument("--learned", action="store_true",
                    help="run the learned-guess case (sphere wake, online training) against plain multigrid")
    ap.add_argument("--optimize", action="store_true",
                    help="run the Davidon optimisation of the rotating cylinder's rate instead")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES bytes (calibrates HBM counters)")
    args = ap.parse_args()
    args.steps_given = any(a == "--steps" or a.startswith("--steps=") for a in sys.argv[1:])
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.gpus != 1:
        print("bench.py: the solver runs on one GPU (its multi-GPU domain decomposition is designed, not "
              "implemented); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    # the CPU baseline runs first, in worker processes, before this process touches the GPU
    cpu = None
    if not args.no_cpu_baseline and not args.adjoint and not args.optimize and not args.learned:
        print("[bench] timing the FP64 oracle on a bounded CPU sample", file=sys.stderr, flush=True)
        cpu = run_cpu_baseline(args.workload)

    import numpy as np
    import torch

    import wlsynth
    from paper_2407_16032_amd import Simulation

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.adjoint:
        run_adjoint(args)
        return
    if args.optimize:
        run_optimize(args)
        return
    if args.learned:
        run_learned(args)
        return
    w = workloads()[args.workload]
    body = w.body if w.body.kind != "none" else None
    print("[bench] workload %s (%d cells), building initial field" % (w.name, w.cells), file=sys.stderr,
          flush=True)
    sim = Simulation(w.n, w.U, w.nu, body, periodic=w.periodic_mask(), convective_exit=w.convective_exit,
                     prec="f32", tol=w.tol, itmax=32, device="cuda:0", solver_path=args.solver_path,
                     blend_mode=args.blend, vcycle_graph=args.vcycle_graph)
    sim.set_velocity(wlsynth.initial_velocity(w, seed=0))
    for k in range(args.warmup):
        sim.step()
    print("[bench] warmup done (%d steps)" % args.warmup, file=sys.stderr, flush=True)

    profile = not args.no_profile
    cells = w.cells
    faces = 1
    for N in w.n:
        faces *= N + 2
    bcells, bfaces = box_counts(sim, w.n)
    flat = fine_level_flat(w.n, 4, args.solver_path)
    tiled = flat or (args.solver_path != "generic" and fine_level_tiled(w.n))

    def launch_bytes(name):
        return kernel_bytes(name, w.ndim, cells, faces, 4, body is not None, 6, bcells, bfaces, tiled, flat,
                            fused=w.ndim == 3 and args.blend == "auto")

    # Breakdown: a few extra steps with an event pair around every launch (the
    # events cost a few per cent of the step, so these steps are not the timed ones)
    kernels = {}
    dominant = None
    if profile:
        nprof = min(args.steps, 5)
        sim.profile(True)
        for k in range(nprof):
            sim.step()
        torch.cuda.synchronize()
        prof = sim.profile_read()
        sim.profile(False)
        for name, (tms, cnt) in prof.items():
            if cnt == 0:
                continue
            b = launch_bytes(name)
            avg_ms = tms / cnt
            ent = {"total_ms_per_step": tms / nprof, "launches_per_step": cnt / nprof, "avg_us": avg_ms * 1e3}
            if b is not None:
                ent["GBps"] = b / (avg_ms * 1e-3) / 1e9
                if dominant is None or tms > kernels[dominant]["total_ms_per_step"] * nprof:
                    dominant = name
            kernels[name] = ent
        for name, ent in sorted(kernels.items(), key=lambda kv: -kv[1]["total_ms_per_step"]):
            print("[bench]   %-9s %8.3f ms/step %6.1f launches/step %9.1f us avg %s" % (
                name, ent["total_ms_per_step"], ent["launches_per_step"], ent["avg_us"],
                ("%7.0f GB/s" % ent["GBps"]) if "GBps" in ent else ""), file=sys.stderr, flush=True)

    # Timed region: events only around the dominant kernel's launches (its
    # average launch duration for the roofline), none around the rest; --windows
    # windows of exactly --steps steps, each bracketed by synchronisations
    if dominant is not None:
        sim.profile(True, groups=[dominant])
    stream = sim.stream
    vc, factors, windows = [], [], []
    for wi in range(args.windows):
        torch.cuda.synchronize()
        start = torch.cuda.Event(enable_timing=True)
        stop = torch.cuda.Event(enable_timing=True)
        start.record(stream)
        t0 = time.perf_counter()
        for k in range(args.steps):
            st = sim.step()
            vc.append(st["vcycles"][0] + st["vcycles"][1])
            for j in range(2):
                n_c = st["vcycles"][j]
                if n_c > 0 and st["res0_linf"][j] > 0 and st["res_linf"][j] > 0:
                    factors.append((st["res_linf"][j] / st["res0_linf"][j]) ** (1.0 / n_c))
        stop.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms = start.elapsed_time(stop)
        windows.append(ms / args.steps)
        print("[bench] window %d: %d steps, %.3f ms/step (wall %.3f ms/step), %.4f ns/pt/step"
              % (wi, args.steps, ms / args.steps, wall * 1e3 / args.steps, ms / args.steps * 1e6 / w.cells),
              file=sys.stderr, flush=True)
    ms_per_step = float(np.median(windows))
    ns_pt = ms_per_step * 1e6 / w.cells
    kmean = float(np.mean(vc))
    print("[bench] median of %d windows: %.3f ms/step, %.4f ns/pt/step, %.2f V-cycles/step"
          % (args.windows, ms_per_step, ns_pt, kmean), file=sys.stderr, flush=True)

    roof = None
    if dominant is not None:
        tms, cnt = sim.profile_read()[dominant]
        sim.profile(False)
        b = launch_bytes(dominant)
        avg_ms = tms / cnt
        ach = b / (avg_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": measured_traffic(w.name, dominant),
                "kernel": dominant, "bytes_per_launch": b, "avg_launch_us": round(avg_ms * 1e3, 2),
                "launches_timed": cnt, "dense_model_bytes_per_launch": model_bytes(dominant, w.ndim, cells, 4),
                "body_box_cells": bcells}
        print("[bench] %s over the timed region: %d launches, %.1f us avg, %.0f GB/s algorithmic"
              % (dominant, cnt, avg_ms * 1e3, ach), file=sys.stderr, flush=True)
        # one fine PCG iteration (passes A + B) on the bytes its kernels need,
        # durations from the breakdown steps
        if "pcg_a" in kernels and "pcg_b" in kernels:
            ba, bb = launch_bytes("pcg_a"), launch_bytes("pcg_b")
            ta, tb = kernels["pcg_a"]["avg_us"], kernels["pcg_b"]["avg_us"]
            gbs = (ba + bb) / ((ta + tb) * 1e-6) / 1e9
            roof["pcg_iteration"] = {"bytes": ba + bb, "us": round(ta + tb, 2), "achieved": round(gbs, 1),
                                     "frac": round(gbs / HBM_PEAK_GBS, 4),
                                     "dense_model_bytes": model_bytes("pcg_a", w.ndim, cells, 4)
                                     + model_bytes("pcg_b", w.ndim, cells, 4)}
        # the whole step by the fixed algorithmic model at the measured V-cycles per step
        per_cell = step_byte_model(w.ndim, body is not None, kmean)
        gbs = per_cell * cells / (ms_per_step * 1e-3) / 1e9
        roof["step"] = {"model_bytes_per_cell": round(per_cell, 1), "bytes": per_cell * cells,
                        "vcycles_per_step": round(kmean, 3), "achieved": round(gbs, 1),
                        "frac": round(gbs / HBM_PEAK_GBS, 4)}
        print("[bench] whole step by the byte model: %.0f B/cell, %.0f GB/s, %.3f of peak"
              % (per_cell, gbs, gbs / HBM_PEAK_GBS), file=sys.stderr, flush=True)

    out = {
        "metric": "ns per grid point per time step (FP32 BDIM step)",
        "value": round(ns_pt, 4),
        "unit": "ns/point/step",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "windows": args.windows,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": (round(ns_pt / PAPER_NS[args.workload]["value"], 4) if args.workload in PAPER_NS else None),
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "cells": w.cells,
                   "Re": round((math.sqrt(sum(u * u for u in w.U)) or 1.0) * w.L / w.nu, 1) if w.nu else None,
                   "mg_tol": w.tol, "moving_body": bool(body is not None and body.moving),
                   "convective_exit": w.convective_exit, "blend": args.blend, "vcycle_graph": args.vcycle_graph,
                   "parallelism": "single GPU"},
        "windows_ms_per_step": [round(v, 3) for v in windows],
        "vcycles_per_step": round(kmean, 3),
        "vcycle_factor": round(float(np.exp(np.mean(np.log(factors)))), 4) if factors else None,
        "roofline": roof,
        "kernels": kernels,
        "cpu_baseline": cpu,
    }
    if args.workload in PAPER_NS:
        out["paper_baseline"] = PAPER_NS[args.workload]
    print(json.dumps(out))
    sim.close()


if __name__ == "__main__":
    main()
