"""Host-side parts of the benchmark (no GPU): the one-GPU contract and the
tile bookkeeping of its CPU baseline."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


def test_tile_run_segments_cover_each_tile_once():
    sys.path.insert(0, ROOT)
    import bench
    width, height, tiles_x = 3840, 2160, 480
    seen = {}
    for b in range(0, 480 * 270, 64):
        for rows, cols in bench.tile_run_segments(b, 64, tiles_x, width, height):
            assert rows.stop - rows.start == 8 and (cols.stop - cols.start) % 8 == 0
            for tx in range(cols.start // 8, cols.stop // 8):
                t = (rows.start // 8) * tiles_x + tx
                assert b <= t < b + 64
                seen[t] = seen.get(t, 0) + 1
    assert len(seen) == 480 * 270 and set(seen.values()) == {1}
