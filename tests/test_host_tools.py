"""Host-side logic around the library (no GPU): the benchmark's byte model for the brick-sparse deposit
grids and the autotuner's handling of the tuning header."""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def brute_force_touched(pos, n, box_len, brick=16):
    """Bricks holding an object's base cell, and their upper neighbours, one object at a time."""
    nbs = n // brick
    seen = set()
    for p in pos.astype(np.float64):
        c = [int(np.floor(v * n / box_len)) % n for v in p]
        b = [v // brick for v in c]
        for dz in (0, 1):
            for dy in (0, 1):
                for dx in (0, 1):
                    seen.add(((b[2] + dz) % nbs, (b[1] + dy) % nbs, (b[0] + dx) % nbs))
    return len(seen)


def test_touched_bricks_matches_brute_force():
    import bench
    rng = np.random.default_rng(5)
    n, box = 64, 640.0
    clump = rng.random((300, 3)) * 60.0 + 200.0
    edge = rng.random((50, 3)) * 8.0 + np.array([632.0, 0.0, 300.0])      # wraps in x
    spread = rng.random((40, 3)) * box
    for pos in (clump, edge, spread, np.concatenate([clump, edge, spread])):
        assert bench.touched_bricks(pos, n, box) == brute_force_touched(pos, n, box)


def test_sparse_byte_model_counts_only_touched_bricks():
    import bench
    dense = bench.algorithmic_bytes(512, 1000, 50000)
    sparse = bench.algorithmic_bytes(512, 1000, 50000, bricks_g=100, bricks_r=200)
    brick_bytes = 16 ** 3 * 8
    cn = 257 * 512 * 512 * 8
    assert sparse["z_fwd_grid"] == 300 * brick_bytes + 2 * cn
    assert sparse["mask"] == 200 * brick_bytes + 2 * 512 ** 3
    # setup tiles: only the grid tiles with data are written by the forward z pass, only the mask's
    # tiles are read and written by the overdensity step
    tiles = (1000, 2000, 1500, 8192)
    tiled = bench.algorithmic_bytes(512, 1000, 50000, bricks_g=100, bricks_r=200, tiles=tiles)
    assert tiled["z_fwd_grid"] == 300 * brick_bytes + (3000 / 8192) * cn
    assert tiled["z_delta"] == (1500 / 8192) * (3 * cn + 512 ** 3)
    assert sparse["paint_grids"] == 300 * brick_bytes
    assert dense["z_fwd_grid"] == 2 * 512 ** 3 * 8 + 2 * cn


def test_autotuner_keeps_knobs_it_does_not_time():
    from paper_1504_02591_amd import autotune
    kept = autotune.other_knobs()
    text = "\n".join(kept)
    for knob in ("RECON_BRICK_NT", "RECON_BIN_BLOCKS", "RECON_OBJ_BATCH"):
        assert f"#define {knob}" in text
    for knob in autotune.KNOBS:
        assert f"#define {knob} " not in text
    # the deposit and reorder timings stay with their knobs
    assert any(l.startswith("// Deposit") for l in kept)
    assert any("reorder" in l for l in kept)
    assert not any(l.startswith("//   RECON_") or l.startswith("//   base") for l in kept)


def test_bench_refuses_more_than_one_gpu():
    """The benchmark measures one GPU: asked for more it exits with a message before touching a device."""
    import subprocess
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=60, cwd=ROOT)
    assert r.returncode == 2
    assert "single MI355X" in r.stderr
    assert r.stdout == ""


def test_every_timed_stage_has_a_byte_model():
    """Each stage the library's event profile reports on the benchmarked path carries algorithmic
    bytes in the benchmark's model, so its roofline fraction is reported; the exceptions are the
    tiny reductions and scans and the stages the benchmark never runs (the real-field forward z
    pass behind recon_set_delta, network training)."""
    import ctypes
    import bench
    from paper_1504_02591_amd import native
    lib = native.load()
    lib.recon_profile_kernel_name.restype = ctypes.c_char_p
    names = [lib.recon_profile_kernel_name(k) for k in range(64)]
    names = [s.decode() for s in names if s]
    assert "x_iter" in names and "shift" in names
    ab = bench.algorithmic_bytes(512, 1000, 50000, bricks_g=100, bricks_r=200)
    missing = {n for n in names if n not in ab and n + "_step" not in ab}
    assert missing <= {"reduce", "scan", "z_fwd_real", "cnn_bwd"}, missing


def test_autotuner_writes_one_size_and_keeps_the_others(tmp_path, monkeypatch):
    """Tuning at 256^3 (batch 64) rewrites only the _256 knobs and adds its timing block; the general
    knobs, their 512^3 timings and the deposit knobs stay."""
    import argparse
    import json
    import shutil
    from paper_1504_02591_amd import autotune
    header = tmp_path / "recon_tuning.h"
    shutil.copy(autotune.TUNING, header)
    monkeypatch.setattr(autotune, "TUNING", str(header))
    before = autotune.current()
    blocks_before = autotune.size_blocks()
    choice = dict(before)
    choice["RECON_TILE_X_256"] = 8 if before["RECON_TILE_X_256"] != 8 else 2
    json.dump({"n": 256, "batch": 64, "base": before, "choice": choice,
               "times": {"base": 2.0, f"RECON_TILE_X_256={choice['RECON_TILE_X_256']}": 1.9}},
              open(tmp_path / "result.json", "w"))
    autotune.cmd_write(argparse.Namespace(dir=str(tmp_path)))
    after = autotune.current()
    assert after["RECON_TILE_X_256"] == choice["RECON_TILE_X_256"]
    for k in autotune.KNOBS:
        if k != "RECON_TILE_X_256":
            assert after[k] == before[k], k
    blocks = autotune.size_blocks()
    assert 256 in blocks and "batch of 64" in blocks[256][0]
    for size, lines in blocks_before.items():
        if size != 256:
            assert blocks[size] == lines
    text = header.read_text()
    for knob in ("RECON_BRICK_NT", "RECON_BIN_BLOCKS", "RECON_OBJ_BATCH"):
        assert f"#define {knob}" in text
