"""C-ABI contract checks that need no GPU: exports, struct layout, argument validation."""
import ctypes as C
import os
import re
import subprocess

import pytest

from paper_2407_16032_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wlmi.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(wl_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(L.LIB_PATH):
        pytest.fail("libwlmi.so not built; run __graft_entry__.build()")
    return L.load()


def test_library_exports_every_declared_symbol(lib):
    declared = _declared()
    assert set(declared) == set(L.EXPORTS)
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (wl_\w+)", out))
    missing = [s for s in declared if s not in exported]
    assert not missing, missing
    for s in declared:
        assert hasattr(lib, s)


def test_struct_layout_matches_header(tmp_path):
    prog = tmp_path / "layout.c"
    prog.write_text("""
#include <stdio.h>
#include <stddef.h>
#include "wlmi.h"
int main(void) {
  printf("%zu %zu %zu %zu\\n", sizeof(wl_sim_desc), sizeof(wl_body_desc), sizeof(wl_step_stats), sizeof(wl_solve_stats));
  printf("%zu %zu %zu %zu %zu\\n", offsetof(wl_sim_desc, nu), offsetof(wl_sim_desc, mg_tol), offsetof(wl_body_desc, spin_omega), offsetof(wl_step_stats, converged), offsetof(wl_sim_desc, adjoint));
  return 0;
}
""")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)], check=True)
    lines = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    sizes = [int(v) for v in lines[0].split()]
    offs = [int(v) for v in lines[1].split()]
    assert sizes == [C.sizeof(L.SimDesc), C.sizeof(L.BodyDesc), C.sizeof(L.StepStats), C.sizeof(L.SolveStats)]
    assert offs == [L.SimDesc.nu.offset, L.SimDesc.mg_tol.offset, L.BodyDesc.spin_omega.offset,
                    L.StepStats.converged.offset, L.SimDesc.adjoint.offset]


def _desc(n=(64, 32), prec=L.WL_F32):
    d = L.SimDesc()
    d.ndim = len(n)
    for k, v in enumerate(n):
        d.n[k] = v
    d.U[0] = 1.0
    d.nu = 0.01
    d.prec = prec
    return d


def test_workspace_bytes_and_validation(lib):
    d = _desc()
    b = L.BodyDesc()
    nb = lib.wl_workspace_bytes(C.byref(d), C.byref(b))
    assert nb > 0 and nb % 256 == 0
    d64 = _desc(prec=L.WL_F64)
    assert lib.wl_workspace_bytes(C.byref(d64), C.byref(b)) > nb
    bad = _desc()
    bad.ndim = 4
    assert lib.wl_workspace_bytes(C.byref(bad), C.byref(b)) == 0
    assert b"ndim" in lib.wl_last_error()
    small = _desc(n=(3, 32))
    assert lib.wl_workspace_bytes(C.byref(small), C.byref(b)) == 0
    ex = _desc()
    ex.convective_exit = 1
    ex.periodic_mask = 1
    assert lib.wl_workspace_bytes(C.byref(ex), C.byref(b)) == 0
    # a body too close to the boundary is rejected
    body = L.BodyDesc()
    body.kind = 1
    body.center[0], body.center[1] = 5.0, 16.0
    body.radius = 4.0
    assert lib.wl_workspace_bytes(C.byref(d), C.byref(body)) == 0
    body.center[0] = 20.0
    assert lib.wl_workspace_bytes(C.byref(d), C.byref(body)) == nb


@pytest.mark.parametrize("n", [(128, 64), (512, 256), (64, 32, 32), (96, 48, 48), (768, 384, 384),
                               (24, 20, 10), (6, 5)])
@pytest.mark.parametrize("prec", [L.WL_F32, L.WL_F64])
def test_workspace_plan_is_consistent(lib, n, prec):
    # wl_workspace_bytes dry-runs the field carving on the host and returns 0 if any
    # buffer of any multigrid level would be missing or outside the workspace
    d = _desc(n=n, prec=prec)
    nb = lib.wl_workspace_bytes(C.byref(d), None)
    assert nb > 0, lib.wl_last_error()
    cells = 1
    for v in n:
        cells *= v + 2
    assert nb >= cells * (4 if prec == L.WL_F32 else 8) * (5 * len(n) + len(n) ** 2 + 7)


@pytest.mark.parametrize("n", [(48, 24), (512, 256), (64, 32, 32)])
def test_adjoint_buffers_in_the_plan(lib, n):
    # desc.adjoint adds 8 D + D^2 + 4 fine-level fields (adjoint velocities, blend and
    # flux adjoints, mu0/mu1/V accumulators, the recorded step, x of both solves, pbar, rhs)
    D = len(n)
    for prec, esz in ((L.WL_F32, 4), (L.WL_F64, 8)):
        d = _desc(n=n, prec=prec)
        base = lib.wl_workspace_bytes(C.byref(d), None)
        d.adjoint = 1
        more = lib.wl_workspace_bytes(C.byref(d), None)
        assert more > base, lib.wl_last_error()
        px = ((n[0] + 2 + 15) // 16) * 16
        alloc = px * (n[1] + 2) * (n[2] + 2 if D == 3 else 1) + 16
        f0 = (alloc * esz + 255) // 256 * 256
        assert more - base == (8 * D + D * D + 4) * f0


def test_create_rejects_bad_arguments_before_any_gpu_work(lib):
    d = _desc()
    out = C.c_void_p()
    # NULL workspace
    st = lib.wl_sim_create(C.byref(d), None, None, 0, None, C.byref(out))
    assert st == 1 and not out.value
    # misaligned workspace pointer (never dereferenced: rejected first)
    st = lib.wl_sim_create(C.byref(d), None, C.c_void_p(0x1001), 1 << 30, None, C.byref(out))
    assert st == 1
    # too small workspace
    st = lib.wl_sim_create(C.byref(d), None, C.c_void_p(0x100000), 16, None, C.byref(out))
    assert st == 2
    assert lib.wl_step(None, 0, None) == 1
    assert lib.wl_sim_destroy(None) == 1
