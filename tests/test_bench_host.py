"""Host-side logic of bench.py: the algorithmic floor, the kernel-source
hash that keys recorded counters, and the lookup of those counters."""
import json
import os
import shutil
import types

import pytest

import bench


def _tile(ny, nx, sh, sw, n_terms=None):
    return types.SimpleNamespace(n_terms_y=ny, n_terms_x=nx, support_h=sh, support_w=sw,
                                 n_terms=n_terms if n_terms is not None else ny * nx, frame=640)


def test_step_floor_counts_twenty_bytes_plus_eight_per_term():
    ctx = types.SimpleNamespace(tiles=[_tile(3, 3, 638, 638), _tile(2, 3, 607, 638), _tile(1, 1, 10, 20)])
    want = (20 + 8 * 9) * 638 * 638 + (20 + 8 * 6) * 607 * 638 + (20 + 8) * 200
    assert bench.step_floor_bytes(ctx) == want


def _fake_root(tmp_path):
    root = tmp_path / "root"
    (root / "paper_1705_06603_amd" / "csrc").mkdir(parents=True)
    for f in ("fft_core.h", "kernels.h"):
        shutil.copy(os.path.join(bench.ROOT, "paper_1705_06603_amd", "csrc", f),
                    root / "paper_1705_06603_amd" / "csrc" / f)
    (root / "profiles").mkdir()
    return root


def test_source_hash_ignores_comments_but_not_code(tmp_path, monkeypatch):
    root = _fake_root(tmp_path)
    monkeypatch.setattr(bench, "ROOT", str(root))
    h0 = bench.kernel_source_hash()
    k = root / "paper_1705_06603_amd" / "csrc" / "kernels.h"
    text = k.read_text()
    k.write_text("// a comment line\n" + text.replace("namespace dbl {", "namespace dbl {  /* inline */", 1) + "\n\n")
    assert bench.kernel_source_hash() == h0
    k.write_text(text.replace("constexpr int kMaxK = 3;", "constexpr int kMaxK = 4;", 1))
    assert bench.kernel_source_hash() != h0


def test_measured_traffic_needs_matching_sources_and_launch_shape(tmp_path, monkeypatch):
    root = _fake_root(tmp_path)
    monkeypatch.setattr(bench, "ROOT", str(root))
    plan = types.SimpleNamespace(frame=640, col_waves=4, row_waves=4, tile_order=2)
    ctx = types.SimpleNamespace(plan=lambda: plan)
    rec = {"kernel_source_hash": bench.kernel_source_hash(),
           "kernels": {"col_H": [{"variant": {"frame": 640, "waves": 4, "tile_order": 0}, "bytes_per_launch": 11},
                                 {"variant": {"frame": 640, "waves": 4, "tile_order": 2}, "bytes_per_launch": 22}],
                       "row_update": [{"variant": {"frame": 640, "waves": 4}, "bytes_per_launch": 33}]}}
    (root / "profiles" / "combined_hbm_traffic.json").write_text(json.dumps(rec))
    assert bench.measured_traffic(ctx, "combined", "col_H") == 22
    assert bench.measured_traffic(ctx, "combined", "row_update") == 33
    assert bench.measured_traffic(ctx, "combined", "col_Ht") is None      # not recorded
    assert bench.measured_traffic(ctx, "batched", "col_H") is None        # no file
    plan.row_waves = 2
    assert bench.measured_traffic(ctx, "combined", "row_update") is None  # other launch shape
    rec["kernel_source_hash"] = "0" * 16
    (root / "profiles" / "combined_hbm_traffic.json").write_text(json.dumps(rec))
    assert bench.measured_traffic(ctx, "combined", "col_H") is None       # other sources


@pytest.mark.parametrize("text,want", [("640,4,4,heavy_first", (640, 4, 4, 2, 1)),
                                       ("320,2,4,column_major,4", (320, 2, 4, 0, 4))])
def test_parse_plan(text, want):
    p = bench.parse_plan(text)
    assert (p.frame, p.col_waves, p.row_waves, p.tile_order, p.tile_groups) == want


def test_more_than_one_gpu_is_refused_before_any_work():
    """The solver runs all tiles on one GPU: --gpus N > 1 exits with status 2
    and a JSON error line, before torch or the library is touched."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], cwd=root,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]
