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


def test_summary_line_fits_the_record_and_ends_with_the_metric(tmp_path):
    """The printed line stays well under the 8 KB a log tail keeps, ends with
    the metric's ratio and its roofline, and the full sections go to the
    details file."""
    sys.path.insert(0, ROOT)
    import bench
    meth = {"gpixels_per_s": 23.123456, "ms": 0.0899, "texel_evals_per_pixel": 0.70533,
            "not_exact_fraction": 0.357, "waves_failed": 2100, "waves_ok": 20835, "unique_texels_per_wave": 46.123,
            "speedup_vs_bilinear4": 3.4257, "alu_frac": 0.29476}
    names = ["bilinear4", "stf1", "list", "box4x4", "box6x6", "mask", "mask_fbC", "mask_fbCplus", "list_k2",
             "list_no_split", "mask_no_split", "bilinear4_8x4", "list_8x4", "box4x4_8x4", "mask_8x4",
             "mask_fbCplus_8x4"]
    run = {"layer_gpixels_per_s": 40.123, "ms": 1.2345, "texel_evals_per_layer_pixel": 0.7,
           "mfma_tflops": 300.1, "mfma_frac": 0.12, "output_hbm_gb_per_s": 640.2}
    res = {"metric": "m", "value": 41.0, "unit": "Gpixels/s", "roofline": {"frac": 0.12, "traffic": 3.7e8},
           "cpu_baseline": {"value": 0.0024, "sample": "x" * 120}, "texel_evals_per_pixel": 0.711,
           "bilinear4": {"gpixels_per_s": 14.6}, "speedup_vs_bilinear4": 2.8, "decoder": {"psnr_db": 61.2},
           "bicubic_4k": {"workload": "w" * 200, "runs": {
               "bspline_list_k4": {"gpixels_per_s": 19.4, "texel_evals_per_pixel": 1.06, "ms": 0.4},
               "bspline_full16": {"gpixels_per_s": 4.48, "texel_evals_per_pixel": 16.0, "ms": 1.8},
               "bspline_speedup_vs_full16": 4.33}},
           "procedural_1080p": {"workload": "w" * 200, "roofline": {"frac": 0.29},
                                "methods": {n: dict(meth) for n in names},
                                "constant_texture_overhead": {n: {"ms": 0.02, "us_per_mpixel": 12.1}
                                                              for n in names[:6]},
                                "cpu_oracle": {"mpixels_per_s": 4.1}},
           "layers_4k": {"workload": "w" * 200, "layer_scales": [1.0] * 6,
                         "psnr_db": {"fp16": [60.123456] * 6, "bf16": [59.9] * 6},
                         "max_abs_fp16_vs_bf16": [2.1234e-3] * 6,
                         "runs": {f"{p}_{m}": dict(run) for p in ("fp16", "bf16") for m in ("list_k4", "bilinear4")},
                         "error_vs_fp64_procedural": {"fp16": {"max_abs": [1.23456e-3] * 6, "psnr_db": [60.1] * 6},
                                                      "bf16": {"max_abs": [2.3456e-3] * 6, "psnr_db": [59.8] * 6},
                                                      "reference": "r"}}}
    res["layers_4k"]["runs"]["fp16_speedup_vs_bilinear4"] = 2.7
    details = tmp_path / "d" / "details.json"
    line = json.dumps(bench.summary_line(res, str(details)))
    assert len(line) < 6000, len(line)
    keys = list(json.loads(line))
    assert keys[-4:] == ["texel_evals_per_pixel", "bilinear4", "speedup_vs_bilinear4", "roofline"]
    full = json.load(open(details))
    assert full["procedural_1080p"]["methods"]["list"]["waves_ok"] == 20835
    assert json.loads(line)["layers_4k"]["error_vs_fp64_procedural"]["bf16"]["max_abs"][0] == 2.35e-3
