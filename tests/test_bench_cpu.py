"""Host logic of bench.py (no GPU): the one-GPU rule, the traffic lookup that goes
stale with the kernel sources, and the byte model's invariants."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

PLATE = (768, 384, 384)
CELLS = 768 * 384 * 384
FACES = 770 * 386 * 386
BOX = 6967871


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def _fake_root(tmp_path, src_hash, value):
    (tmp_path / "profiles").mkdir()
    (tmp_path / "paper_2407_16032_amd").mkdir()
    os.symlink(os.path.join(ROOT, "paper_2407_16032_amd", "csrc"), tmp_path / "paper_2407_16032_amd" / "csrc")
    (tmp_path / "profiles" / "pmc_w.md").write_text(
        "# counters\n\nkernel-source-sha256-16: %s\n\ntraffic_bytes k_pcg_b_flat_fine %.4e\n" % (src_hash, value))


def test_traffic_is_reported_only_for_the_profiled_sources(tmp_path, monkeypatch):
    current = bench.kernel_source_hash()
    _fake_root(tmp_path, current, 3.25e9)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("w", "pcg_b") == pytest.approx(3.25e9)
    assert bench.measured_traffic("w", "pcg_a") is None       # no line for it
    assert bench.measured_traffic("other", "pcg_b") is None   # no summary


def test_traffic_goes_stale_when_the_sources_change(tmp_path, monkeypatch):
    _fake_root(tmp_path, "0" * 16, 3.25e9)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("w", "pcg_b") is None


def test_source_hash_ignores_comments_but_not_code():
    src = 'int f(int a) {\n  // twice a\n  return 2 * a; /* doubled */\n}\nconst char* s = "// kept";\n'
    same = 'int f(int a) {\n  return 2 * a;\n\n}  // end\nconst char* s = "// kept";\n'
    other = 'int f(int a) {\n  return 3 * a;\n}\nconst char* s = "// kept";\n'
    assert bench.code_text(src) == bench.code_text(same)
    assert bench.code_text(src) != bench.code_text(other)
    assert '"// kept"' in bench.code_text(src)


def test_flat_level_rule():
    assert bench.fine_level_flat(PLATE)
    assert bench.fine_level_flat((32, 32, 16))                  # 2^14 cells
    assert not bench.fine_level_flat((32, 16, 16))              # below 2^14 cells
    assert not bench.fine_level_flat((130, 18, 14))             # rows not whole 16-byte vectors
    assert not bench.fine_level_flat((512, 256))                # 2-D
    assert not bench.fine_level_flat(PLATE, solver_path="tiles")


def test_byte_model_invariants():
    kb = lambda name, box, flat=True, tiled=False: bench.kernel_bytes(  # noqa: E731
        name, 3, CELLS, FACES, 4, True, 6, box, None, tiled, flat)
    # outside the body box coefficients are closed form: a smaller box moves fewer bytes,
    # and no box at all leaves exactly the field traffic
    for name in ("pcg_a", "pcg_b", "prolong"):
        assert kb(name, BOX) < kb(name, CELLS)
        assert kb(name, 0) < kb(name, BOX)
    # the flat and tiled pass B recompute q: e, x, r in and x, r out, on a level of any size
    assert kb("pcg_b", 0) == 5 * CELLS * 4
    assert kb("pcg_b", 0, flat=True, tiled=False) == kb("pcg_b", 0, flat=False, tiled=True)
    # the generic pass B reads the stored q as well
    assert kb("pcg_b", 0, flat=False, tiled=False) == 6 * CELLS * 4
    # the dense fixed model (stored q, all coefficients) is an upper bound
    assert bench.model_bytes("pcg_b", 3, CELLS, 4) >= kb("pcg_b", BOX)


def test_byte_model_of_the_blend_in_the_flux_launch():
    # the 3-D step's flux launch writes the blended velocity instead of f~ (same
    # bytes) and f~ again within one face of the body box; the blend launch then
    # moves only the box's faces
    kb = lambda name, fused, body=True: bench.kernel_bytes(  # noqa: E731
        name, 3, CELLS, FACES, 4, body, 6, BOX, BOX, True, True, fused=fused)
    assert kb("flux", True) == kb("flux", False) + 3 * BOX * 4
    assert kb("flux", True, body=False) == kb("flux", False, body=False)
    assert kb("bdim", True) < kb("bdim", False)
    # outside the box nothing of the blend launch remains
    assert kb("bdim", True) == (3 + 1.5 + 3 + 3 + 3 + 9) * BOX * 4


def test_step_byte_model_matches_the_fixed_model():
    # 3-D with a body at k = 4 V-cycles: 4 (79 + 4 x 105.4) = 2002.4 bytes per cell
    assert bench.step_byte_model(3, True, 4.0) == pytest.approx(2002.4)
    assert bench.step_byte_model(3, False, 0.0) == pytest.approx(220.0)
    assert bench.step_byte_model(2, True, 2.0) == pytest.approx(4 * (52 + 230.6))


def test_cpu_baseline_reports_both_legs_and_the_core_count():
    out = bench.run_cpu_baseline("circle2d")
    assert out["kind"] == "oracle" and out["unit"] == "ns/point/step"
    assert out["host_cpu_count"] == os.cpu_count()
    assert 1 <= out["cores"] <= 16
    assert out["single_core"]["cores"] == 1
    assert out["value"] > 0 and out["single_core"]["value"] > 0
