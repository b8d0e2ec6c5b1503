"""Benchmark: collaborative vs 4-tap bilinear filtering with a learned texel decoder.

Workload (default): a 3840x2160 frame of four seeded perspective planes
textured by a learned decoder (latent grids 512^2 and 128^2 x 8 channels,
MLP 16-64-64-4) trained on the GPU against a 2048^2 procedural texture (32
sinusoids per channel).  One step = one filtered frame with List-exact
dedup (up to 4 texels per lane, so magnifying waves never overflow) and
one-tap STF for minifying pixels; the 4-tap baseline decodes all four
texels of every active pixel through the same MFMA decode.

Prints one JSON line.  Inputs are synthetic and resident in GPU memory
before timing starts.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

MLP_FLOP = 2 * (16 * 64 + 64 * 64 + 64 * 4)      # useful FLOP per decoded texel
PROC_SLOTS_PER_TERM = 8                       # 4 full-rate VALU + v_sin_f32 (quarter rate: 4 slots)
VALU_SLOT_PEAK = 256 * 4 * 32 * 2.4e9          # full-rate VALU lane-ops/s: 157.3 TFLOP/s fp32 / 2
PEAK_FP16_TFLOPS = 2500.0                          # MI355X dense fp16/bf16 MFMA


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--train-steps", type=int, default=20000)
    ap.add_argument("--batch", type=int, default=65536)
    ap.add_argument("--width", type=int, default=3840)
    ap.add_argument("--height", type=int, default=2160)
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target CPU time of the oracle baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precision", choices=["fp16", "bf16"], default="fp16")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one 256 MiB device copy first (scale for the HBM byte counters)")
    ap.add_argument("--no-procedural", action="store_true", help="skip the 1080p procedural-texture runs")
    ap.add_argument("--no-layers", action="store_true", help="skip the six-layer 4K runs")
    ap.add_argument("--no-bicubic", action="store_true", help="skip the bicubic 4K runs")
    ap.add_argument("--layers", type=int, default=6)
    ap.add_argument("--details", default=os.path.join("gpurun_out", "bench_details.json"),
                    help="file for the full per-method sections (the printed line carries a summary)")
    return ap.parse_args()


KERNEL_SOURCES = ["paper_2506_17770_amd/csrc/filter_decoder.hip", "paper_2506_17770_amd/csrc/filter_decoder.h",
                  "paper_2506_17770_amd/csrc/decoder_mlp.h",
                  "paper_2506_17770_amd/csrc/ctf_device.h", "paper_2506_17770_amd/csrc/ctf_internal.h",
                  "paper_2506_17770_amd/csrc/fallback.h"]
KERNEL_OBJECT = "filter_decoder.hip"   # the source the List kernel is compiled from
TRAFFIC_RECORD = "profiles/k_filter_dec_list_fp16_4k.json"


def kernel_compile_flags():
    """The hipcc flags the List kernel's source is compiled with (include
    paths left out: they name the checkout's location)."""
    import importlib.util
    spec = importlib.util.spec_from_file_location("ctf_hip_build_flags",
                                                  os.path.join(ROOT, "paper_2506_17770_amd", "build.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    flags = mod.HIPCC_FLAGS + mod.SOURCE_FLAGS.get(KERNEL_OBJECT, [])
    return [f for f in flags if not f.startswith("-I")]


def kernel_source_digest() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    h.update(" ".join(kernel_compile_flags()).encode())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per launch of the List kernel from the committed rocprofv3
    counter record, or None if the kernel sources changed since."""
    path = os.path.join(ROOT, TRAFFIC_RECORD)
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_source_sha256") != kernel_source_digest():
        return None
    return (rec["fetch_kib_per_launch"] * rec["fetch_scale"] + rec["write_kib_per_launch"] * rec["write_scale"]) * 1024


def timed(fn, stream, steps, warmup, torch):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for a, b in ev:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = [a.elapsed_time(b) for a, b in ev]
    return wall, per


def tile_run_segments(b, count, tiles_x, width, height):
    """Pixel slices (rows, cols) of tiles b .. b+count-1 (row-major tiles)."""
    segs = []
    t = b
    while t < b + count:
        ty, tx0 = divmod(t, tiles_x)
        tx1 = min(tiles_x, tx0 + (b + count - t))
        segs.append((slice(8 * ty, min(height, 8 * ty + 8)), slice(8 * tx0, min(width, 8 * tx1))))
        t += tx1 - tx0
    return segs


def cpu_baseline(args, sc, dec_params, l0, l1, H, tex_w, seed, gpu_out=None):
    """Oracle (float64 decoder, List k=4) on a bounded sample of tiles, all host
    threads; with ``gpu_out`` also the GPU frame's error against it on that
    sample (compared after the timed region)."""
    import oracle as O
    tiles_x = (sc.width + 7) // 8
    ntiles = tiles_x * ((sc.height + 7) // 8)
    otex = O.decoder_texture(tex_w, l0, l1, H, dec_params.astype(np.float64))
    meth = O.method(O.LIST, k=4)
    threads = os.cpu_count() or 1
    rng = np.random.default_rng(0)
    # calibrate on one tile row, then size the sample to the time budget
    t0 = time.perf_counter()
    O.filter(sc.uv, sc.duv, otex, meth, seed=seed, tiles=(ntiles // 2, ntiles // 2 + 64), stats=False)
    per_tile = (time.perf_counter() - t0) / 64
    n_sample = int(max(64, min(ntiles, args.cpu_seconds * threads / max(per_tile, 1e-6))))
    starts = np.sort(rng.choice(ntiles // 64, size=max(1, n_sample // 64), replace=False)) * 64
    chunks = np.array_split(starts, threads)

    kept = [[] for _ in chunks]

    def work(i, ch):
        for b in ch:
            o = O.filter(sc.uv, sc.duv, otex, meth, seed=seed, tiles=(int(b), int(b) + 64), stats=False)
            if gpu_out is not None:
                kept[i].append([(sl, o["out"][sl]) for sl in tile_run_segments(int(b), 64, tiles_x, sc.width,
                                                                                 sc.height)])

    t0 = time.perf_counter()
    ths = [threading.Thread(target=work, args=(i, c)) for i, c in enumerate(chunks) if len(c)]
    for t in ths:
        t.start()
    for t in ths:
        t.join()
    dt = time.perf_counter() - t0
    px = len(starts) * 64 * 64
    base = {"value": px / dt / 1e9, "unit": "Gpixels/s", "cores": len(ths), "kind": "oracle",
            "sample": f"{len(starts) * 64} of {ntiles} 8x8 tiles of the same frame (runs of 64 tiles), "
                      f"float64 decoder, List k=4 + STF, {dt:.1f} s wall"}
    if gpu_out is None:
        return base, None
    mx, se, n = 0.0, 0.0, 0
    for runs in kept:
        for segs in runs:
            for sl, ref in segs:
                d = gpu_out[sl].astype(np.float64) - ref
                mx = max(mx, float(np.abs(d).max()))
                se += float((d * d).sum())
                n += d.size
    mse = se / max(1, n)
    err = {"max_abs": mx, "psnr_db": 10 * math.log10(1.0 / mse) if mse > 0 else None, "values": n,
           "reference": "the oracle's frame on the same sample: float64 decoder from the same float32 "
                        "master parameters, float64 filtering; the GPU decodes in fp16 MFMA"}
    return base, err


def cpu_layer_errors(layer_tex, layer_vals, tex_w):
    """Per-layer error of the GPU decoders against the float64 procedural
    oracle over the whole tex_w^2 lattice: max abs and PSNR for each
    precision.  ``layer_tex``: (pqj, amp) per layer; ``layer_vals``: per layer
    {precision: float32 [tex_w^2][4] host array of decoded texels}."""
    import oracle as O
    ys, xs = np.mgrid[0:tex_w, 0:tex_w]
    xy = np.ascontiguousarray(np.stack([xs.ravel(), ys.ravel()], -1).astype(np.int32))
    threads = os.cpu_count() or 1
    parts = np.array_split(np.arange(xy.shape[0]), threads)
    out = {}
    t0 = time.perf_counter()
    for l, ((pqj, amp), vals) in enumerate(zip(layer_tex, layer_vals)):
        otex = O.sinusoid_texture(tex_w, pqj, amp)
        ref = np.empty((xy.shape[0], 4), np.float64)

        def work(ix):
            ref[ix] = otex.eval(xy[ix])

        ths = [threading.Thread(target=work, args=(ix,)) for ix in parts if ix.size]
        for t in ths:
            t.start()
        for t in ths:
            t.join()
        for pname, v in vals.items():
            d = v.astype(np.float64) - ref
            mse = float((d * d).mean())
            out.setdefault(pname, {"max_abs": [], "psnr_db": []})
            out[pname]["max_abs"].append(float(np.abs(d).max()))
            out[pname]["psnr_db"].append(10 * math.log10(1.0 / mse) if mse > 0 else None)
    out["reference"] = (f"float64 procedural oracle over all {tex_w}^2 texels of each layer, "
                        f"{len(parts)} threads, {time.perf_counter() - t0:.1f} s")
    return out


def cpu_oracle_procedural(sc, pqj, amp, single_s=2.0):
    """The oracle's List on the 1080p procedural frame: one thread on whole
    tile rows for about ``single_s`` seconds, then every tile row on all host
    threads."""
    import oracle as O
    otex = O.sinusoid_texture(2048, pqj, amp)
    meth = O.method(O.LIST)
    tiles_x, tiles_y = (sc.width + 7) // 8, (sc.height + 7) // 8

    def rows(rs):
        for r in rs:
            O.filter(sc.uv, sc.duv, otex, meth, seed=0, tiles=(r * tiles_x, (r + 1) * tiles_x), stats=False)

    t0 = time.perf_counter()
    n1 = 0
    while n1 < tiles_y and time.perf_counter() - t0 < single_s:
        rows([n1])
        n1 += 1
    dt1 = time.perf_counter() - t0
    threads = os.cpu_count() or 1
    parts = [list(range(tiles_y))[i::threads] for i in range(threads)]
    t0 = time.perf_counter()
    ths = [threading.Thread(target=rows, args=(p,)) for p in parts if p]
    for t in ths:
        t.start()
    for t in ths:
        t.join()
    dtn = time.perf_counter() - t0
    return {"method": "list", "single_thread_mpixels_per_s": n1 * tiles_x * 64 / dt1 / 1e6,
            "threads": len(ths), "mpixels_per_s": tiles_y * tiles_x * 64 / dtn / 1e6,
            "sample": f"one thread: {n1} of {tiles_y} tile rows ({dt1:.1f} s); {len(ths)} threads: all "
                      f"{tiles_y} tile rows ({dtn:.1f} s); float64 texels"}


def bench_procedural(ctx, ctf, cs, torch, args, stream):
    """1920x1080 four-plane frame, 2048^2 procedural texture (32 sinusoids per
    channel): every method through the per-lane kernel."""
    sc = cs.random_planes_scene(1920, 1080, 2048, 2048, seed=1)
    pqj, amp = cs.sinusoid_params(2048, 32, 64, seed=2)
    tex = ctx.sinusoid_texture(2048, pqj, amp)
    uv = torch.from_numpy(sc.uv).cuda()
    duv = torch.from_numpy(sc.duv).cuda()
    out = torch.empty((1080, 1920, 4), dtype=torch.float32, device="cuda")
    npx = 1920 * 1080
    res = {}
    for name, m in (("bilinear4", ctf.method(ctf.BILINEAR4)), ("stf1", ctf.method(ctf.STF1)),
                    ("list", ctf.method(ctf.LIST)), ("box4x4", ctf.method(ctf.BOX, box=(4, 4))),
                    ("box6x6", ctf.method(ctf.BOX, box=(6, 6))), ("mask", ctf.method(ctf.MASK)),
                    ("mask_fbC", ctf.method(ctf.MASK, fallback=ctf.FB_C)),
                    ("mask_fbCplus", ctf.method(ctf.MASK, fallback=ctf.FB_CPLUS)),
                    ("list_k2", ctf.method(ctf.LIST, k=2)),
                    ("list_no_split", ctf.method(ctf.LIST, split=ctf.SPLIT_OFF)),
                    ("mask_no_split", ctf.method(ctf.MASK, split=ctf.SPLIT_OFF)),
                    ("bilinear4_8x4", ctf.method(ctf.BILINEAR4, wave_shape=ctf.WAVE_8X4)),
                    ("list_8x4", ctf.method(ctf.LIST, wave_shape=ctf.WAVE_8X4)),
                    ("box4x4_8x4", ctf.method(ctf.BOX, box=(4, 4), wave_shape=ctf.WAVE_8X4)),
                    ("mask_8x4", ctf.method(ctf.MASK, wave_shape=ctf.WAVE_8X4)),
                    ("mask_fbCplus_8x4", ctf.method(ctf.MASK, fallback=ctf.FB_CPLUS, wave_shape=ctf.WAVE_8X4))):
        fs = ctf.frame_stats_buffer()
        ts = ctf.tile_stats_buffer(1920, 1080, meth=m)
        ctx.filter(uv, duv, tex, m, out=out, frame_stats=fs, tile_stats=ts)
        torch.cuda.synchronize()
        st = ctf.frame_stats_dict(fs)
        rec = ts.cpu().numpy().view(ctf.TILE_STATS_DTYPE).reshape(-1)
        used = rec["part"] != 0   # waves with at least one magnifying lane
        _, per = timed(lambda: ctx.filter(uv, duv, tex, m, out=out), stream, max(3, args.steps // 2), 2, torch)
        ms = float(np.mean(per))
        res[name] = {"gpixels_per_s": npx / (ms * 1e-3) / 1e9, "ms": ms,
                     "texel_evals_per_pixel": st["evals"] / npx,
                     "unique_texels_per_wave": float(rec["unique"][used].mean()) if used.any() else 0.0,
                     "not_exact_fraction": st["stf"] / max(1, st["active"]),
                     "waves_failed": st["tiles_fail"], "waves_ok": st["tiles_ok"]}
    # the dedup machinery's own cost: the same frame on a constant texture,
    # whose texel evaluation is free (time per Mpixel, as the paper states it)
    ctex = ctx.constant_texture(2048, 2048, (0.25, 0.5, 0.75, 1.0))
    overhead = {}
    for name, m in (("bilinear4", ctf.method(ctf.BILINEAR4)), ("stf1", ctf.method(ctf.STF1)),
                    ("list", ctf.method(ctf.LIST)), ("box4x4", ctf.method(ctf.BOX, box=(4, 4))),
                    ("box6x6", ctf.method(ctf.BOX, box=(6, 6))), ("mask", ctf.method(ctf.MASK))):
        _, per = timed(lambda: ctx.filter(uv, duv, ctex, m, out=out), stream, max(3, args.steps // 2), 2, torch)
        ms = float(np.mean(per))
        overhead[name] = {"ms": ms, "us_per_mpixel": ms * 1e3 / (npx / 1e6)}
    ctex.close()
    cpu = None if args.no_cpu_baseline else cpu_oracle_procedural(sc, pqj, amp)
    b4 = res["bilinear4"]["gpixels_per_s"]
    # ALU roofline of the texel evaluations: per term 4 full-rate VALU
    # instructions (two FMAs for the exact phase, fract, the accumulating FMA)
    # and one v_sin_f32 at quarter rate = 8 lane slots; peak = 256 CUs x 4
    # SIMDs x 32 lanes x 2.4 GHz (the fp32 vector rate, one FMA per lane slot)
    slots_per_eval = 4 * 32 * PROC_SLOTS_PER_TERM
    for v in res.values():
        v["speedup_vs_bilinear4"] = v["gpixels_per_s"] / b4
        evals = v["texel_evals_per_pixel"] * npx
        v["alu_frac"] = evals * slots_per_eval / (v["ms"] * 1e-3) / VALU_SLOT_PEAK
    lst = res["list"]
    achieved = lst["texel_evals_per_pixel"] * npx * slots_per_eval / (lst["ms"] * 1e-3)
    roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_SLOT_PEAK / 1e12, "unit": "T lane-slots/s",
            "frac": achieved / VALU_SLOT_PEAK, "kernel": "k_filter_simt<LIST, SINUSOIDS>",
            "work_per_launch": f"{lst['texel_evals_per_pixel'] * npx:.0f} texel evals x {slots_per_eval} slots"}
    tex.close()
    return {"workload": "1920x1080 four-plane frame, 2048^2 procedural texture (K=32 sinusoids "
                        "per channel, F=64), per-lane texel production; *_8x4: the paper's 8x4 tiles, "
                        "two per wave64", "roofline": roof, "methods": res,
            "constant_texture_overhead": overhead, "cpu_oracle": cpu}


def bench_layers(ctx, ctf, cs, torch, args, stream, sc, uv, duv):
    """Six material layers at 4K in one launch: layer l has its own texture
    (seed 11 + l) and decoder, and samples uv_l = s_l R(theta_l) uv."""
    n = args.layers
    tex_w, l0, l1, H = 2048, 512, 128, 64
    decs, psnr = [], {"fp16": [], "bf16": []}
    layer_tex, layer_vals = [], []
    ys, xs = np.mgrid[0:tex_w, 0:tex_w]
    xy = torch.from_numpy(np.stack([xs.ravel(), ys.ravel()], -1).astype(np.int32)).cuda()
    fp_bf_max = []
    t0 = time.perf_counter()
    for l in range(n):
        pqj, amp = cs.sinusoid_params(tex_w, 32, 64, seed=11 + l)
        target = ctx.sinusoid_texture(tex_w, pqj, amp)
        dec = ctx.decoder(l0, l1, H, tex_w, cs.decoder_init(l0, l1, H, seed=100 + l))
        if args.train_steps:
            dec.train(target, args.train_steps, batch=args.batch, lr=1e-3, seed=200 + l, precision=ctf.BF16)
        pv = target.eval(xy).double()
        vals = {}
        for pname, prec in (("fp16", ctf.FP16), ("bf16", ctf.BF16)):
            t = ctx.decoder_texture(dec, prec)
            vals[pname] = t.eval(xy)
            mse = float(((vals[pname].double() - pv) ** 2).mean())
            psnr[pname].append(10 * math.log10(1.0 / mse))
            t.close()
        fp_bf_max.append(float((vals["fp16"] - vals["bf16"]).abs().max()))
        layer_tex.append((pqj, amp))
        if not args.no_cpu_baseline:
            layer_vals.append({k: v.cpu().numpy() for k, v in vals.items()})
        del vals, pv
        target.close()
        decs.append(dec)
    train_s = time.perf_counter() - t0
    del xy
    mats = np.array([cs.layer_params(11, l)[2] for l in range(n)], np.float32)
    scales = [float(cs.layer_params(11, l)[0]) for l in range(n)]
    out = torch.empty((n, args.height, args.width, 4), dtype=torch.float32, device="cuda")
    npx = args.width * args.height
    res = {}
    for pname, prec in (("fp16", ctf.FP16), ("bf16", ctf.BF16)):
        texs = [ctx.decoder_texture(d, prec) for d in decs]
        for mname, m in (("list_k4", ctf.method(ctf.LIST, k=4)), ("bilinear4", ctf.method(ctf.BILINEAR4))):
            fs = ctf.frame_stats_buffer()
            ctx.filter_layers(uv, duv, texs, mats, m, seed=0, out=out, frame_stats=fs)
            torch.cuda.synchronize()
            st = ctf.frame_stats_dict(fs)
            _, per = timed(lambda: ctx.filter_layers(uv, duv, texs, mats, m, seed=0, out=out), stream,
                           max(3, args.steps // 2), 2, torch)
            ms = float(np.mean(per))
            tflops = st["evals"] * MLP_FLOP / (ms * 1e-3) / 1e12
            res[f"{pname}_{mname}"] = {
                "layer_gpixels_per_s": n * npx / (ms * 1e-3) / 1e9, "ms": ms,
                "texel_evals_per_layer_pixel": st["evals"] / (n * npx),
                "mfma_tflops": tflops, "mfma_frac": tflops / PEAK_FP16_TFLOPS,
                "output_hbm_gb_per_s": n * npx * 16 / (ms * 1e-3) / 1e9}
        for t in texs:
            t.close()
    for d in decs:
        d.close()
    for pname in ("fp16", "bf16"):
        res[f"{pname}_speedup_vs_bilinear4"] = (res[f"{pname}_list_k4"]["layer_gpixels_per_s"] /
                                                res[f"{pname}_bilinear4"]["layer_gpixels_per_s"])
    return {"workload": f"{args.width}x{args.height} four-plane frame, {n} layers in one launch, "
                        f"layer l: own 2048^2 procedural texture (seed 11+l) and learned decoder, "
                        "uv_l = s_l R(theta_l) uv, s_l ~ U[0.25, 4]",
            "layer_scales": scales, "psnr_db": psnr, "max_abs_fp16_vs_bf16": fp_bf_max,
            "train_seconds_total": train_s, "runs": res}, (layer_tex, layer_vals, tex_w)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    import ctf_synth as cs
    import paper_2506_17770_amd as ctf

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    prec = ctf.FP16 if args.precision == "fp16" else ctf.BF16
    tex_w, l0, l1, H, K, F = 2048, 512, 128, 64, 32, 64
    seed_scene, seed_tex, seed_stf, seed_dec = 1, 2, 0, 3

    log("bench: generating scene")
    sc = cs.random_planes_scene(args.width, args.height, tex_w, tex_w, seed=seed_scene)
    ctx = ctf.Context(0)
    pqj, amp = cs.sinusoid_params(tex_w, K, F, seed=seed_tex)
    target = ctx.sinusoid_texture(tex_w, pqj, amp)
    init = cs.decoder_init(l0, l1, H, seed=seed_dec)
    dec = ctx.decoder(l0, l1, H, tex_w, init)

    log(f"bench: training decoder, {args.train_steps} steps x {args.batch}")
    trace = torch.zeros(max(1, args.train_steps), device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if args.train_steps:
        dec.train(target, args.train_steps, batch=args.batch, lr=1e-3, seed=7, precision=ctf.BF16,
                  loss_trace=trace)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    tr = trace.cpu().numpy()
    log(f"bench: trained in {train_s:.1f} s, final loss {tr[-1]:.3e}")
    dtex = ctx.decoder_texture(dec, prec)

    # decoder quality over the whole 2048^2 lattice vs the procedural texture
    # (the GPU's float32 procedural texels, within 3e-7 of float64)
    ys, xs = np.mgrid[0:tex_w, 0:tex_w]
    xy = torch.from_numpy(np.stack([xs.ravel(), ys.ravel()], -1).astype(np.int32)).to(dev)
    dv = dtex.eval(xy)
    pv = target.eval(xy)
    mse = float(((dv.double() - pv.double()) ** 2).mean())
    psnr = 10 * math.log10(1.0 / mse) if mse > 0 else float("inf")
    max_abs = float((dv - pv).abs().max())
    init_tex = ctx.decoder_texture(ctx.decoder(l0, l1, H, tex_w, init), prec)
    mse0 = float(((init_tex.eval(xy).double() - pv.double()) ** 2).mean())
    psnr_init = 10 * math.log10(1.0 / mse0)
    del xy, dv, pv

    uv = torch.from_numpy(sc.uv).to(dev)
    duv = torch.from_numpy(sc.duv).to(dev)
    out = torch.empty((args.height, args.width, 4), dtype=torch.float32, device=dev)
    m_col = ctf.method(ctf.LIST, k=4)
    m_b4 = ctf.method(ctf.BILINEAR4)

    # statistics of the same frames (untimed runs)
    def stats(m):
        fs = ctf.frame_stats_buffer()
        ctx.filter(uv, duv, dtex, m, seed=seed_stf, out=out, frame_stats=fs)
        torch.cuda.synchronize()
        return ctf.frame_stats_dict(fs)

    s_col, s_b4 = stats(m_col), stats(m_b4)
    npx = args.width * args.height

    if args.calib_copy:
        src = torch.ones(64 * 2**20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("bench: calibration copy of 268435456 bytes done")
        del src, dst

    log("bench: timing")
    run_col = lambda: ctx.filter(uv, duv, dtex, m_col, seed=seed_stf, out=out)
    run_b4 = lambda: ctx.filter(uv, duv, dtex, m_b4, seed=seed_stf, out=out)
    wall_col, per_col = timed(run_col, stream, args.steps, args.warmup, torch)
    col_out = out.cpu().numpy()   # the collaborative frame, for the error against the oracle
    wall_b4, per_b4 = timed(run_b4, stream, args.steps, args.warmup, torch)
    ms_col = float(np.mean(per_col))
    ms_b4 = float(np.mean(per_b4))
    gpx_col = npx / (ms_col * 1e-3) / 1e9
    gpx_b4 = npx / (ms_b4 * 1e-3) / 1e9

    achieved = s_col["evals"] * MLP_FLOP / (ms_col * 1e-3) / 1e12
    roof = {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP16_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP16_TFLOPS, "traffic": measured_traffic(),
            "algorithmic_bytes": npx * 40,
            "kernel": "k_filter_dec_batch<LIST>", "work_per_launch": f"{s_col['evals']} decoded texels x {MLP_FLOP} FLOP"}
    achieved_b4 = s_b4["evals"] * MLP_FLOP / (ms_b4 * 1e-3) / 1e12

    res = {
        "metric": "Gpixels/s + texel evals/pixel, collaborative vs 4-tap bilinear, 4K, 1 GPU",
        "value": gpx_col, "unit": "Gpixels/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_col, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "fp16" if prec == ctf.FP16 else "bf16", "data": "synthetic",
        "config": {"workload": f"{args.width}x{args.height} four-plane frame, learned decoder "
                               f"(latents {l0}^2+{l1}^2 x8, MLP 16-{H}-{H}-4) on a {tex_w}^2 texture, "
                               "List dedup k=4 + one-tap STF vs 4-tap bilinear",
                   "width": args.width, "height": args.height, "train_steps": args.train_steps,
                   "batch": args.batch},
        "texel_evals_per_pixel": s_col["evals"] / npx,
        "bilinear4": {"gpixels_per_s": gpx_b4, "ms_per_step": ms_b4,
                      "texel_evals_per_pixel": s_b4["evals"] / npx, "mfma_tflops": achieved_b4},
        "speedup_vs_bilinear4": gpx_col / gpx_b4,
        "fallback_fraction": s_col["stf"] / max(1, s_col["active"]),
        "minify_fraction": s_col["minify"] / max(1, s_col["active"]),
        "mlp_rows_per_pixel": s_col["rows"] / npx,
        "decoder": {"psnr_db": psnr, "max_abs_err": max_abs, "psnr_db_untrained": psnr_init,
                    "train_seconds": train_s, "train_final_loss": float(tr[-1]) if args.train_steps else None,
                    # MLP work of training: forward + backward (two GEMMs per layer) = 3x the forward
                    "train_mlp_tflops": (args.train_steps * args.batch * 3 * MLP_FLOP / train_s / 1e12
                                         if args.train_steps and train_s > 0 else None),
                    "train_samples_per_s": args.train_steps * args.batch / train_s if train_s > 0 else None,
                    "reference": "GPU float32 procedural texels (within 3e-7 of float64)"},
        "wall_s": {"collaborative": wall_col, "bilinear4": wall_b4},
        "roofline": roof,
    }
    if not args.no_bicubic:
        log("bench: bicubic filters at 4K")
        bic = {}
        for fname, flt in (("bspline", ctf.FILTER_BSPLINE), ("catmull_rom", ctf.FILTER_CATMULL_ROM)):
            for mname, m in (("list_k4", ctf.method(ctf.LIST, k=4, filter=flt)),
                             ("full16", ctf.method(ctf.BILINEAR4, filter=flt))):
                st = stats(m)
                _, per = timed(lambda: ctx.filter(uv, duv, dtex, m, seed=seed_stf, out=out), stream,
                               max(3, args.steps // 2), 2, torch)
                ms = float(np.mean(per))
                tfl = st["evals"] * MLP_FLOP / (ms * 1e-3) / 1e12
                bic[f"{fname}_{mname}"] = {"gpixels_per_s": npx / (ms * 1e-3) / 1e9, "ms": ms,
                                           "texel_evals_per_pixel": st["evals"] / npx,
                                           "not_exact_fraction": st["stf"] / max(1, st["active"]),
                                           "mfma_tflops": tfl, "mfma_frac": tfl / PEAK_FP16_TFLOPS}
            bic[f"{fname}_speedup_vs_full16"] = (bic[f"{fname}_list_k4"]["gpixels_per_s"] /
                                                 bic[f"{fname}_full16"]["gpixels_per_s"])
        res["bicubic_4k"] = {"workload": "the 4K frame and fp16 decoder above with 4x4 bicubic footprints: List "
                                         "k=4 + one-tap draw by |w| vs all 16 taps decoded per pixel", "runs": bic}
    layer_data = None
    if not args.no_procedural:
        log("bench: 1080p procedural texture")
        res["procedural_1080p"] = bench_procedural(ctx, ctf, cs, torch, args, stream)
    if not args.no_layers and args.layers > 0:
        log(f"bench: {args.layers} layers at 4K")
        res["layers_4k"], layer_data = bench_layers(ctx, ctf, cs, torch, args, stream, sc, uv, duv)
    if not args.no_cpu_baseline:
        log("bench: cpu baseline")
        res["cpu_baseline"], res["frame_error_vs_fp64_oracle"] = cpu_baseline(
            args, sc, dec.params(), l0, l1, H, tex_w, seed_stf, gpu_out=col_out)
        if layer_data is not None and layer_data[1]:
            log("bench: layer decoders against the float64 procedural oracle")
            res["layers_4k"]["error_vs_fp64_procedural"] = cpu_layer_errors(*layer_data)
    print(json.dumps(summary_line(res, args.details)), flush=True)


def summary_line(res, details_path):
    """The printed record: the headline fields in full, each side section
    reduced to its key figures; the full sections go to ``details_path``."""
    line = {k: v for k, v in res.items() if k not in ("bicubic_4k", "procedural_1080p", "layers_4k")}
    if "bicubic_4k" in res:
        r = res["bicubic_4k"]["runs"]
        line["bicubic_4k"] = {k: (round(v, 3) if not isinstance(v, dict) else
                                  {"gpx": round(v["gpixels_per_s"], 2),
                                   "evals_px": round(v["texel_evals_per_pixel"], 3)})
                              for k, v in r.items()}
    if "procedural_1080p" in res:
        p = res["procedural_1080p"]
        line["procedural_1080p"] = {
            "roofline_frac_list": round(p["roofline"]["frac"], 4),
            "methods": {k: {"gpx": round(v["gpixels_per_s"], 2), "x_b4": round(v["speedup_vs_bilinear4"], 2),
                            "evals_px": round(v["texel_evals_per_pixel"], 3), "alu_frac": round(v["alu_frac"], 3),
                            "uniq_wave": round(v["unique_texels_per_wave"], 1),
                            "fb_frac": round(v["not_exact_fraction"], 3)}
                        for k, v in p["methods"].items()},
            "overhead_us_per_mpixel": {k: round(v["us_per_mpixel"], 2)
                                       for k, v in p["constant_texture_overhead"].items()}}
        if p.get("cpu_oracle"):
            line["procedural_1080p"]["cpu_oracle_mpixels_per_s"] = round(p["cpu_oracle"]["mpixels_per_s"], 3)
    if "layers_4k" in res:
        L = res["layers_4k"]
        s = {"psnr_db": {k: [round(x, 2) for x in v] for k, v in L["psnr_db"].items()},
             "max_abs_fp16_vs_bf16": [float(f"{x:.3g}") for x in L["max_abs_fp16_vs_bf16"]]}
        for k, v in L["runs"].items():
            s[k] = (round(v, 3) if not isinstance(v, dict) else
                    {"layer_gpx": round(v["layer_gpixels_per_s"], 2), "ms": round(v["ms"], 4),
                     "mfma_frac": round(v["mfma_frac"], 4)})
        if "error_vs_fp64_procedural" in L:
            e = L["error_vs_fp64_procedural"]
            s["error_vs_fp64_procedural"] = {
                k: {"max_abs": [float(f"{x:.3g}") for x in e[k]["max_abs"]],
                    "psnr_db": [round(x, 2) for x in e[k]["psnr_db"]]} for k in ("fp16", "bf16") if k in e}
        line["layers_4k"] = s
    try:
        d = os.path.dirname(details_path)
        if d:
            os.makedirs(d, exist_ok=True)
        with open(details_path, "w") as f:
            json.dump(res, f, indent=1)
        line["details"] = details_path
    except OSError as e:
        line["details"] = f"not written: {e}"
    # the metric's ratio and the figures it rests on, last on the line
    for k in ("texel_evals_per_pixel", "bilinear4", "speedup_vs_bilinear4", "roofline"):
        if k in line:
            line[k] = line.pop(k)
    return line


if __name__ == "__main__":
    main()
