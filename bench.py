"""Benchmark: DRR forward + backward views/s, batched vs per-view, one GPU.

Default workload: 200 000 radiative Gaussians (log-scales ~
N(log 0.02, 0.3)), 8 views of 512 x 512 at evenly spaced azimuths, L1 loss
against a target rendered from a perturbed copy of the scene.  One step =
the whole hot path for all views: preprocess, tile binning + radix sort,
forward blending, L1 upstream gradient, reverse blending, and the adjoint
of the projection to every Gaussian parameter.  Inputs are resident in HBM
before timing.

Batched: all views in one set of launches, the step captured as one HIP
graph and replayed (`value`; the same launches enqueued eagerly are
reported as "eager", and with --graph 0 they are the value).  Per-view: the
same kernels with one view per launch sequence, looped over the views,
enqueued eagerly.  Prints one JSON line.

--workload 5 is the training-scale case (1M Gaussians, 16 views of
512 x 512, anisotropic scales) whose step also runs the fused Adam update;
--store SLOTS switches to the stored-transmittance forward/backward.  Both
report the peak device memory of the step.  --loss eq11 takes the upstream
gradient from the full Eq. 11 objective (0.8 L1 + 0.2 SSIM term, fused
kernels) instead of L1 alone; every run also times that objective on its
own ("loss_eq11").

"acui_forward" is the forward-only scan of the ACUI-initialised model
(Sec. 3.3, Eq. 13 grid of 35^3 centres, 100 views of 512 x 512 over 0-180
degrees), batched and per view: the paper's inference measurement on a
synthetic stand-in.  --no-acui skips it, --only-acui runs nothing else.
"rgb_forward" compares the forward of the radiative model with that of the
RGB model with spherical-harmonics colour (Eq. 2, degree 3) on the
headline scene (Tab. 3a's comparison); --no-rgb skips it.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Algorithmic work of the blend kernels in VALU lane-operation cycles (a
# transcendental counts 4: quarter rate), per unit of work of the definition:
#   forward: 21 per evaluation (offset, exponent, exp, opacity, clamp, test,
#            transmittance update, accumulate);
#   backward: 35 per revisited evaluation (recompute alpha, recover T by
#            division, the 7 gradient terms) plus, per (Gaussian, wavefront)
#            with a contributing lane, 42 wavefront instructions (the 7-value
#            wavefront reduction and its atomics) = 42 x 64 lane slots.
LANE_OPS_EVAL_FWD = 21
LANE_OPS_EVAL_BWD = 35
WAVE_INSTR_REDUCTION = 42
WAVE = 64
# MI355X: 256 CUs x 64 FP32 lanes x 2.4 GHz = 39.3 T lane-operations/s without
# packed FP32 (what these scalar-FP32 kernels can issue); the published FP32
# vector peak, 157.3 TFLOP/s, counts an FMA as 2 and packed FP32 (2 per lane).
PEAK_LANE_OPS = 256 * 64 * 2.4e9
PEAK_FP32_TFLOPS = 157.3
PEAK_HBM_BPS = 8.0e12     # MI355X HBM3E
# Eq. 11 loss gradient, algorithmic bytes per pixel: image + target read twice
# (16), three SSIM derivative maps written then read (24), dl written (4)
LOSS_BYTES_PER_PX = 44


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", type=int, default=3)
    ap.add_argument("--tile", type=int, default=16)
    ap.add_argument("--lds", type=int, default=256)
    ap.add_argument("--persistent", type=int, default=0, help="persistent blending kernels (1/0)")
    ap.add_argument("--no-peaks", action="store_true",
                    help="skip the on-device HBM / VALU / LDS microbenchmarks")
    ap.add_argument("--autotune", action="store_true",
                    help="pick tile and LDS batch with the autotuner on this scene (timed fwd+bwd "
                         "steps over the 9 settings, before the benchmark) instead of --tile/--lds")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-per-view", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--graph", type=int, default=1,
                    help="time the batched step captured as one HIP graph (1/0; 1: that is the value)")
    ap.add_argument("--store", type=int, default=0, metavar="SLOTS",
                    help="stored-transmittance variant with SLOTS per pixel (0: divide back)")
    ap.add_argument("--adam", type=int, default=-1,
                    help="run the fused Adam update in every step (1/0; default: on for workload 5)")
    ap.add_argument("--loss", choices=("l1", "eq11"), default="l1",
                    help="upstream gradient of the step: L1 alone, or the Eq. 11 objective "
                         "(0.8 L1 + 0.2 SSIM term, fused kernels)")
    ap.add_argument("--fused", type=int, default=1,
                    help="1: the L1 gradient in the forward blend's launch and gradients written by "
                         "the projection adjoint (no clearing launch); 0: separate launches")
    ap.add_argument("--no-acui", action="store_true",
                    help="skip the forward-only scan of the ACUI-initialised model")
    ap.add_argument("--no-rgb", action="store_true",
                    help="skip the forward comparison with the RGB (spherical-harmonics) model")
    ap.add_argument("--only-acui", action="store_true",
                    help="run only the forward-only ACUI scan (prints its JSON object)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MB",
                    help="after timing, run 3 plain device copies of MB MiB (counter calibration)")
    return ap.parse_args()


def acui_forward(args, dev, stream, st) -> dict:
    """Forward-only scan of the ACUI-initialised model (the paper's inference
    measurement on a synthetic stand-in): centres on the Eq. 13 grid made by
    the library, attributes from the seeded generator, 100 views of 512 x 512
    evenly over 0-180 degrees.  One pass = preprocess + binning/sort +
    forward blending of all views; batched (one launch sequence) and per view
    (one launch sequence per view, the paper's one-projection-per-frame)."""
    import numpy as np
    import torch

    import scenes as S
    import paper_2403_04116_amd as P
    from paper_2403_04116_amd import _lib as X

    w = S.workload(6)
    n = X.xg_acui_count(S.ACUI_SIZE, S.ACUI_GRID, S.ACUI_D)
    attrs = S.attributes(n, w.log_scale_mean, w.log_scale_std, w.seeds["scene"])
    g = {k: torch.from_numpy(v).to(dev) for k, v in attrs.items()}
    g["means"] = P.acui_means(S.ACUI_SIZE, S.ACUI_GRID, S.ACUI_D, device=dev)
    D = S.DETECTOR_SIDE
    cams = P.cameras(w.angles, w.sizes, S.L_SO, S.L_SD, D, D)
    sid = int(stream.cuda_stream)
    gs = P.drr.gaussians_struct(g)
    frame = P.Frame(n, cams, st, device=dev)
    n_pairs = frame.fit_capacity(g)
    image, final_t, n_contrib = frame.new_outputs()
    names = ["preprocess", "bin_sort", "render_fwd"]
    rows = []

    def one_pass(record: bool):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)] if record else None
        calls = [lambda: P.xg_preprocess(frame.frame, gs, sid),
                 lambda: P.xg_bin_sort(frame.frame, sid),
                 lambda: P.xg_render_fwd(frame.frame, gs, image.data_ptr(), final_t.data_ptr(),
                                         n_contrib.data_ptr(), sid)]
        if record:
            ev[0].record(stream)
        for k, c in enumerate(calls):
            c()
            if record:
                ev[k + 1].record(stream)
        if record:
            rows.append(ev)

    for _ in range(args.warmup):
        one_pass(False)
    torch.cuda.synchronize()
    for _ in range(args.steps):
        one_pass(True)
    torch.cuda.synchronize()
    assert frame.status() == 0, "pair capacity exceeded in the ACUI scan"
    ms = float(np.mean([r[0].elapsed_time(r[3]) for r in rows]))
    stages = {nm: float(np.mean([r[k].elapsed_time(r[k + 1]) for r in rows])) for k, nm in enumerate(names)}
    out = {"workload": f"ACUI grid {S.ACUI_GRID[0]}^3 voxels, d={S.ACUI_D:g} (Eq. 13): {n} Gaussians, "
                       f"{w.n_views} views of 512x512 over 0-180 deg, forward only",
           "gaussians": n, "views": w.n_views, "pairs": int(n_pairs), "ms_per_pass": ms,
           "views_per_s": w.n_views / (ms * 1e-3), "stages_ms": stages,
           "paper_fps_context": "148 fps, one projection per frame, trained scenes, RTX 8000 (Tab. 1)"}
    if not args.no_per_view:
        frames = []
        off = 0
        for v in range(w.n_views):
            f = P.Frame(n, [cams[v]], st, device=dev)
            f.fit_capacity(g)
            npx = w.sizes[v][0] * w.sizes[v][1]
            frames.append((f, image[off:off + npx], final_t[off:off + npx], n_contrib[off:off + npx]))
            off += npx

        def per_view_pass():
            for f, im, ft, nc in frames:
                P.xg_preprocess(f.frame, gs, sid)
                P.xg_bin_sort(f.frame, sid)
                P.xg_render_fwd(f.frame, gs, im.data_ptr(), ft.data_ptr(), nc.data_ptr(), sid)

        per_view_pass()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = max(1, args.steps // 4)
        e0.record(stream)
        for _ in range(reps):
            per_view_pass()
        e1.record(stream)
        torch.cuda.synchronize()
        assert all(f.status() == 0 for f, *_ in frames)
        pv_ms = e0.elapsed_time(e1) / reps
        out["per_view"] = {"ms_per_pass": pv_ms, "views_per_s": w.n_views / (pv_ms * 1e-3),
                           "ms_per_view": pv_ms / w.n_views}
        out["batched_over_per_view"] = out["views_per_s"] / out["per_view"]["views_per_s"]
        del frames
    del frame
    torch.cuda.empty_cache()
    return out


def rgb_forward(args, dev, stream, st, w, g, cams) -> dict:
    """Forward of the radiative model against the comparison model (RGB
    Gaussians with degree-3 spherical-harmonics colour, Eq. 2) on the same
    scene and views: preprocess (+ colours), binning/sort, blend.  The
    paper's Tab. 3a ratio (2.1x inference) is this comparison on trained
    scenes."""
    import numpy as np
    import torch

    import scenes as S
    import paper_2403_04116_amd as P
    from paper_2403_04116_amd import _lib as X

    degree = 3
    sh = torch.from_numpy(S.sh_coefficients(w.n, degree, w.seeds["scene"] + 7)).to(dev)
    frame = P.Frame(w.n, cams, st, device=dev)
    frame.fit_capacity(g)
    sid = int(stream.cuda_stream)
    gs = P.drr.gaussians_struct(g)
    npx = frame.total_pixels
    img1 = torch.empty(npx, device=dev)
    img3 = torch.empty((3, npx), device=dev)
    ft = torch.empty(npx, device=dev)
    nc = torch.empty(npx, dtype=torch.int32, device=dev)
    drr = [lambda: P.xg_preprocess(frame.frame, gs, sid),
           lambda: P.xg_bin_sort(frame.frame, sid),
           lambda: P.xg_render_fwd(frame.frame, gs, img1.data_ptr(), ft.data_ptr(), nc.data_ptr(), sid)]
    rgb = [lambda: X.xg_preprocess_rgb(frame.frame, gs, sh.data_ptr(), degree, sid),
           lambda: P.xg_bin_sort(frame.frame, sid),
           lambda: X.xg_render_fwd_rgb(frame.frame, gs, img3.data_ptr(), ft.data_ptr(), nc.data_ptr(), sid)]

    def run(calls):
        for _ in range(args.warmup):
            for c in calls:
                c()
        torch.cuda.synchronize()
        rows = []
        for _ in range(args.steps):
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(len(calls) + 1)]
            ev[0].record(stream)
            for k, c in enumerate(calls):
                c()
                ev[k + 1].record(stream)
            rows.append(ev)
        torch.cuda.synchronize()
        total = float(np.mean([r[0].elapsed_time(r[-1]) for r in rows]))
        parts = [float(np.mean([r[k].elapsed_time(r[k + 1]) for r in rows])) for k in range(len(calls))]
        return total, parts

    d_ms, d_parts = run(drr)
    r_ms, r_parts = run(rgb)
    assert frame.status() == 0
    names = ["preprocess", "bin_sort", "render_fwd"]
    out = {"degree": degree, "views": w.n_views, "gaussians": w.n,
           "radiative_ms": d_ms, "rgb_ms": r_ms, "rgb_over_radiative": r_ms / d_ms,
           "radiative_views_per_s": w.n_views / (d_ms * 1e-3), "rgb_views_per_s": w.n_views / (r_ms * 1e-3),
           "radiative_stages_ms": dict(zip(names, d_parts)), "rgb_stages_ms": dict(zip(names, r_parts)),
           "paper_context": "Tab. 3a: 72 -> 148 fps (2.1x) from RGB to radiative, trained scenes"}
    del frame
    torch.cuda.empty_cache()
    return out


def kernel_source_hash() -> str:
    """Hash of the blend kernels' source file; a stored HBM-traffic figure is
    only reported while it matches."""
    import hashlib
    h = hashlib.sha256()
    for f in ("render.hip",):
        with open(os.path.join(ROOT, "paper_2403_04116_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_peaks(dev, stream) -> dict:
    """On-device ceilings from libxgpeaks.so (HIP events on `stream`):
    streaming copy and read of 1 GiB (HBM), independent scalar FP32 FMA
    chains (VALU issue rate in lane-operations/s), conflict-free 16-byte LDS
    reads (LDS bandwidth).  Best of 5 launches each."""
    import ctypes as C
    import torch
    lib = C.CDLL(os.path.join(ROOT, "paper_2403_04116_amd", "libxgpeaks.so"))
    for name, args in (("xgp_copy", [C.c_void_p, C.c_void_p, C.c_int64, C.c_int, C.c_void_p]),
                       ("xgp_read", [C.c_void_p, C.c_int64, C.c_void_p, C.c_int, C.c_void_p]),
                       ("xgp_valu", [C.c_void_p, C.c_int, C.c_int, C.c_void_p]),
                       ("xgp_lds", [C.c_void_p, C.c_int, C.c_int, C.c_void_p])):
        getattr(lib, name).argtypes = args
        getattr(lib, name).restype = C.c_int
    sid = C.c_void_p(int(stream.cuda_stream))
    cus = torch.cuda.get_device_properties(dev).multi_processor_count
    nbytes = 1 << 30
    src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    sink = torch.zeros(1 << 16, dtype=torch.float32, device=dev)

    def best_ms(fn, reps=5):
        assert fn() == 0
        torch.cuda.synchronize()
        out = []
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            torch.cuda.synchronize()
            out.append(e0.elapsed_time(e1))
        return min(out)

    n16 = nbytes // 16
    blocks = cus * 16
    copy_ms = best_ms(lambda: lib.xgp_copy(src.data_ptr(), dst.data_ptr(), n16, blocks, sid))
    read_ms = best_ms(lambda: lib.xgp_read(src.data_ptr(), n16, sink.data_ptr(), blocks, sid))
    iters = 8192
    wg = cus * 8
    valu_ms = best_ms(lambda: lib.xgp_valu(sink.data_ptr(), iters, wg, sid))
    lds_ms = best_ms(lambda: lib.xgp_lds(sink.data_ptr(), iters, wg, sid))
    del src, dst, sink
    torch.cuda.empty_cache()
    return {"cus": cus,
            "hbm_copy_GBps": 2 * nbytes / (copy_ms * 1e-3) / 1e9,
            "hbm_read_GBps": nbytes / (read_ms * 1e-3) / 1e9,
            "valu_T_lane_ops": wg * 256 * iters * 8 / (valu_ms * 1e-3) / 1e12,
            "lds_TBps": wg * 256 * iters * 16 / (lds_ms * 1e-3) / 1e12,
            "lds_B_per_clk_per_cu_at_2p4GHz": wg * 256 * iters * 16 / (lds_ms * 1e-3) / cus / 2.4e9}


# Lists by counting are used when every view has at most this many tiles
# (the library's limit); otherwise emission and the radix sort of the pairs.
BIN_MAX_TILES = 4096
BIN_ITEMS = 2048


def bin_sort_bytes(frame, w, n_items, n_kept, npairs, item_passes, pair_passes):
    """Bytes the binning stage must move: the item sort (key and value read
    and written per pass, the key histogram, the sorted counts), the count
    scan, then either the lists by counting (the kept items' slot, count and
    value read twice, the per-partition tile counts written, scanned and
    read, each pair written once, the tile ranges) or emission and the pair
    passes (each pair written, histogrammed, read and written per pass and
    read for the ranges)."""
    tile = frame.settings.tile
    view_tiles = [((wd + tile - 1) // tile) * ((ht + tile - 1) // tile) for wd, ht in w.sizes]
    pair_word = 4 if frame.layout.pair_index_bits else 8
    items = n_items * (4 + 24 * item_passes + 4) + 16 * n_kept + 8 * n_items
    if max(view_tiles) <= BIN_MAX_TILES:
        rows = w.n_views * ((w.n + BIN_ITEMS - 1) // BIN_ITEMS)
        return items + 2 * 16 * n_kept + 16 * rows * max(view_tiles) + pair_word * npairs \
            + 16 * frame.total_tiles
    return items + npairs * (pair_word + 4 + 2 * pair_word * pair_passes + 4) + 8 * frame.total_tiles


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the DRR path is built and "
              "measured on a single MI355X", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import scenes as S
    import paper_2403_04116_amd as P
    from paper_2403_04116_amd import _lib as X

    dev = torch.device("cuda:0")
    if args.only_acui:
        st = P.settings(tile=args.tile, lds_batch=args.lds, persistent=bool(args.persistent))
        print(json.dumps({"acui_forward": acui_forward(args, dev, torch.cuda.current_stream(), st)}))
        return
    w = S.workload(args.workload)
    use_adam = (args.workload == 5) if args.adam < 0 else bool(args.adam)
    g_np = S.scene(args.workload)
    tgt_np = S.perturb(g_np, w.seeds["perturb"])
    D = S.DETECTOR_SIDE
    cams = P.cameras(w.angles, w.sizes, S.L_SO, S.L_SD, D, D)
    st = P.settings(tile=args.tile, lds_batch=args.lds, persistent=bool(args.persistent))
    g = {k: torch.from_numpy(v).to(dev) for k, v in g_np.items()}
    gt_t = {k: torch.from_numpy(v).to(dev) for k, v in tgt_np.items()}
    npx = w.n_pixels
    scale = 1.0 / npx

    # target images (rendered once, outside timing)
    tframe = P.Frame(w.n, cams, st, device=dev)
    tframe.fit_capacity(gt_t)
    target, _, _ = tframe.render_fwd(gt_t)
    torch.cuda.synchronize()
    del tframe

    stream = torch.cuda.current_stream()
    del gt_t
    tuned = None
    if args.autotune:
        from paper_2403_04116_amd.autotune import autotune
        res = autotune(g, cams, target, scale, use_cache=False)
        best = res["settings"]
        args.tile, args.lds = int(best.tile), int(best.lds_batch)
        st = P.settings(tile=args.tile, lds_batch=args.lds, persistent=bool(args.persistent))
        tuned = {"tile": args.tile, "lds_batch": args.lds,
                 "ms_per_step": {f"{t}x{b}": round(v, 4) for (t, b), v in sorted(res["ms"].items())}}
    torch.cuda.empty_cache()
    torch.cuda.reset_peak_memory_stats()

    # ---- batched path -------------------------------------------------------
    opt = None
    if use_adam:
        from paper_2403_04116_amd.optim import FusedAdam
        opt = FusedAdam.from_activated(g)
        g = opt.act              # the renderer reads the optimiser's activated copies
    frame = P.Frame(w.n, cams, st, device=dev)
    n_pairs = frame.fit_capacity(g)
    store = frame.new_store(args.store) if args.store > 0 else None
    out = frame.new_outputs()
    dl = torch.empty(npx, dtype=torch.float32, device=dev)
    loss_val = torch.zeros(1, dtype=torch.float32, device=dev)
    grads = frame.new_grads(g)
    gs = P.drr.gaussians_struct(g)
    gr = P.XgGrads(*(grads[k].data_ptr() for k in P.drr.PARAMS))
    sid = int(stream.cuda_stream)
    image, final_t, n_contrib = out
    # per-stage HIP events on the launch stream: marks[k] follows stage k
    loss_stage = "l1_grad" if args.loss == "l1" else "loss_grad"
    fuse_l1 = bool(args.fused) and args.loss == "l1" and store is None
    write_grads = bool(args.fused)
    STAGES = ([] if write_grads else ["zero_grads"]) + ["preprocess", "bin_sort"] \
        + (["render_fwd_l1"] if fuse_l1 else ["render_fwd", loss_stage]) \
        + ["render_bwd", "preprocess_bwd"] + (["adam"] if opt is not None else [])
    marks = []

    def mark(record, row):
        if record:
            e = torch.cuda.Event(enable_timing=True)
            e.record(stream)
            row.append(e)

    def step_batched(record: bool):
        row = []
        mark(record, row)
        if not write_grads:
            grads.zero_()
            mark(record, row)
        P.xg_preprocess(frame.frame, gs, sid)
        mark(record, row)
        P.xg_bin_sort(frame.frame, sid)
        mark(record, row)
        if fuse_l1:
            X.xg_render_fwd_l1(frame.frame, gs, image.data_ptr(), final_t.data_ptr(),
                               n_contrib.data_ptr(), target.data_ptr(), scale, dl.data_ptr(), sid)
            mark(record, row)
        else:
            if store is None:
                P.xg_render_fwd(frame.frame, gs, image.data_ptr(), final_t.data_ptr(),
                                n_contrib.data_ptr(), sid)
            else:
                X.xg_render_fwd_store(frame.frame, gs, image.data_ptr(), final_t.data_ptr(),
                                      n_contrib.data_ptr(), store.view.data_ptr(), store.slots,
                                      store.view.numel(), sid)
            mark(record, row)
            if args.loss == "l1":
                P.xg_l1_grad(image.data_ptr(), target.data_ptr(), dl.data_ptr(), npx, scale, sid)
            else:
                X.xg_loss_grad(frame.frame, image.data_ptr(), target.data_ptr(), 0.2, dl.data_ptr(),
                               loss_val.data_ptr(), sid)
            mark(record, row)
        if store is None:
            X.xg_render_bwd_2d(frame.frame, dl.data_ptr(), final_t.data_ptr(), n_contrib.data_ptr(),
                               sid)
        else:
            X.xg_render_bwd_store_2d(frame.frame, dl.data_ptr(), final_t.data_ptr(),
                                     n_contrib.data_ptr(), store.view.data_ptr(), store.slots,
                                     store.view.numel(), sid)
        mark(record, row)
        if write_grads:
            X.xg_preprocess_bwd_write(frame.frame, gs, gr, sid)
        else:
            P.xg_preprocess_bwd(frame.frame, gs, gr, sid)
        mark(record, row)
        if opt is not None:
            opt.step(grads, sid, gate=frame.status_ptr())
            mark(record, row)
        if record:
            marks.append(row)

    def timed(fn, steps, warmup, **kw):
        for _ in range(warmup):
            fn(False, **kw) if kw else fn(False)
        torch.cuda.synchronize()
        s0 = torch.cuda.Event(enable_timing=True)
        s1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        s0.record(stream)
        for _ in range(steps):
            fn(True, **kw) if kw else fn(True)
        s1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        return s0.elapsed_time(s1) / steps, wall

    ms_batched, wall_b = timed(step_batched, args.steps, args.warmup)
    assert frame.status() == 0, "pair capacity exceeded during timing"
    hbm = {"peak_allocated": int(torch.cuda.max_memory_allocated()),
           "workspace": int(frame.ws.numel()),
           "store": int(store.view.numel()) if store is not None else 0,
           "optimizer_state": int(opt.m.numel() * 8 + sum(t.numel() * 4 for t in opt.raw.values()))
           if opt is not None else 0}
    stage_ms = {name: float(np.mean([row[k].elapsed_time(row[k + 1]) for row in marks]))
                for k, name in enumerate(STAGES)}
    fwd_ms = stage_ms["render_fwd_l1"] if fuse_l1 else stage_ms["render_fwd"]
    bwd_ms = stage_ms["render_bwd"]

    counts = frame.render_counts().double().sum(dim=1).cpu().numpy()
    evals, contribs, upto, reductions, bwd_visits, fwd_visits, fwd_lane_evals, bwd_lane_evals = \
        (float(x) for x in counts)
    fwd_ops = evals * LANE_OPS_EVAL_FWD
    bwd_ops = upto * LANE_OPS_EVAL_BWD + reductions * WAVE_INSTR_REDUCTION * WAVE
    if bwd_ms >= fwd_ms:
        dom, dom_ms, dom_ops = "k_render_bwd", bwd_ms, bwd_ops
    else:
        dom, dom_ms, dom_ops = "k_render_fwd", fwd_ms, fwd_ops
    achieved = dom_ops / (dom_ms * 1e-3)
    lanes = {
        "fwd_visits": fwd_visits, "fwd_active_lanes_per_visit": fwd_lane_evals / max(fwd_visits, 1),
        "bwd_visits": bwd_visits, "bwd_active_lanes_per_visit": bwd_lane_evals / max(bwd_visits, 1),
        "bwd_reductions": reductions, "bwd_contributing_lanes_per_reduction": contribs / max(reductions, 1),
    }

    # per-stage algorithmic work and fraction of the stage's roofline
    n_items = w.n * w.n_views
    n_kept = int((frame.ws_tensor(frame.layout.counts, torch.int32, n_items) > 0).sum())
    # header word 9 of the workspace: item-sort passes that moved data
    item_passes = int(frame.ws[36:40].view(torch.int32).item())
    npairs = frame.n_pairs()
    pair_passes = (max(frame.total_tiles - 1, 1).bit_length() + 7) // 8
    work = {
        "zero_grads": ("hbm", 48 * w.n),
        "preprocess": ("hbm", 48 * w.n + (64 + 4 + 8 + 32) * n_items),
        "bin_sort": ("hbm", bin_sort_bytes(frame, w, n_items, n_kept, npairs, item_passes, pair_passes)),
        "render_fwd": ("alu", fwd_ops),
        "render_fwd_l1": ("alu", fwd_ops),   # plus 12 bytes per pixel for the L1 epilogue
        "l1_grad": ("hbm", 12 * npx),
        "loss_grad": ("hbm", LOSS_BYTES_PER_PX * npx),
        "render_bwd": ("alu", bwd_ops),
        "preprocess_bwd": ("hbm", 32 * n_items + 144 * w.n),
        # per Gaussian: 11 raw scalars (means, log-scales, quaternion, opacity
        # logit) read x, grad, m, v and write x, m, v (28 B), the activated
        # scales and opacity written (16 B); per response feature read x, m, v
        # and write them (24 B); the intensity gradient read and the new
        # intensity written (8 B)
        "adam": ("hbm", w.n * (11 * 28 + 16 + 24 * (opt.n_features if opt is not None else 0) + 8)),
    }
    stages = {}
    for name in STAGES:
        bound, wk = work[name]
        ms = stage_ms[name]
        rate = wk / (ms * 1e-3)
        stages[name] = {"ms": ms, "bound": bound, "work": wk,
                        "unit": "bytes" if bound == "hbm" else "lane-op",
                        "frac": rate / (PEAK_HBM_BPS if bound == "hbm" else PEAK_LANE_OPS)}
    traffic = None
    tfile = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(tfile):
        try:
            tj = json.load(open(tfile))
            if (tj.get("kernel") == dom and tj.get("workload") == args.workload
                    and tj.get("source_hash") == kernel_source_hash()
                    and tj.get("tile") == args.tile and tj.get("lds_batch") == args.lds):
                traffic = tj.get("bytes_per_launch")
        except (OSError, ValueError):
            traffic = None

    # ---- the same batched step captured as one HIP graph --------------------
    graph = None
    if args.graph:
        from paper_2403_04116_amd.step import TrainStep
        ts = TrainStep(frame, g, target, scale, grads=grads, optimizer=opt, store=store)
        ts.capture()
        for _ in range(args.warmup):
            ts.replay()
        torch.cuda.synchronize()
        g0 = torch.cuda.Event(enable_timing=True)
        g1 = torch.cuda.Event(enable_timing=True)
        g0.record(stream)
        for _ in range(args.steps):
            ts.replay()
        g1.record(stream)
        torch.cuda.synchronize()
        assert ts.check(), "pair capacity exceeded during graph replay"
        ms_graph = g0.elapsed_time(g1) / args.steps
        graph = {"value": w.n_views / (ms_graph * 1e-3), "ms_per_step": ms_graph}
        del ts

    # ---- per-view path ------------------------------------------------------
    per_view = None
    if not args.no_per_view and store is None and opt is None:
        frames = []
        off = 0
        for v in range(w.n_views):
            f = P.Frame(w.n, [cams[v]], st, device=dev)
            f.fit_capacity(g)
            wv, hv = w.sizes[v]
            sl = slice(off, off + wv * hv)
            frames.append((f, image[sl], final_t[sl], n_contrib[sl], dl[sl], target[sl], wv * hv))
            off += wv * hv

        def step_per_view(record: bool):
            grads.zero_()
            for f, im, ft, nc, d, tg, n in frames:
                P.xg_preprocess(f.frame, gs, sid)
                P.xg_bin_sort(f.frame, sid)
                if args.fused:
                    X.xg_render_fwd_l1(f.frame, gs, im.data_ptr(), ft.data_ptr(), nc.data_ptr(),
                                       tg.data_ptr(), scale, d.data_ptr(), sid)
                else:
                    P.xg_render_fwd(f.frame, gs, im.data_ptr(), ft.data_ptr(), nc.data_ptr(), sid)
                    P.xg_l1_grad(im.data_ptr(), tg.data_ptr(), d.data_ptr(), n, scale, sid)
                # the views' gradients add up: cleared once, accumulated per view
                P.xg_render_bwd(f.frame, gs, d.data_ptr(), ft.data_ptr(), nc.data_ptr(), gr, sid)

        ms_pv, _ = timed(step_per_view, args.steps, args.warmup)
        per_view = {"value": w.n_views / (ms_pv * 1e-3), "ms_per_step": ms_pv}

    # The batched path is the step captured as one HIP graph and replayed
    # (each replay enqueues every stage of the step); without --graph, the
    # same launches enqueued eagerly.  Both are reported.
    eager = {"value": w.n_views / (ms_batched * 1e-3), "ms_per_step": ms_batched}
    ms_step = graph["ms_per_step"] if graph is not None else ms_batched
    value = w.n_views / (ms_step * 1e-3)

    # the radiation intensity response (Eq. 3, 16 features) on its own: forward
    # and adjoint over all Gaussians, HBM bound
    nf = 16
    feats = torch.randn(w.n, nf, device=dev) * 0.3
    wts = torch.ones(nf, device=dev)
    inten = torch.empty(w.n, device=dev)
    gfeat = torch.zeros(w.n, nf, device=dev)
    r_ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    for rep in range(3):
        if rep == 2:
            r_ev[0].record(stream)
        X.xg_rirf_fwd(feats.data_ptr(), wts.data_ptr(), w.n, nf, inten.data_ptr(), sid)
        if rep == 2:
            r_ev[1].record(stream)
        X.xg_rirf_bwd(feats.data_ptr(), wts.data_ptr(), w.n, nf, inten.data_ptr(), gfeat.data_ptr(), sid)
        if rep == 2:
            r_ev[2].record(stream)
    torch.cuda.synchronize()
    rf_ms, rb_ms = r_ev[0].elapsed_time(r_ev[1]), r_ev[1].elapsed_time(r_ev[2])
    rirf_bytes_f = w.n * (4 * nf + 4)
    rirf_bytes_b = w.n * (4 * nf + 4 + 8 * nf)
    rirf = {"n_features": nf, "fwd_ms": rf_ms, "bwd_ms": rb_ms,
            "fwd_frac_hbm": rirf_bytes_f / (rf_ms * 1e-3) / PEAK_HBM_BPS,
            "bwd_frac_hbm": rirf_bytes_b / (rb_ms * 1e-3) / PEAK_HBM_BPS}
    del feats, gfeat, inten

    # the Eq. 11 objective (0.8 L1 + 0.2 SSIM term) and its gradient on its own
    l_ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    for rep in range(4):
        if rep == 3:
            l_ev[0].record(stream)
        X.xg_loss_grad(frame.frame, image.data_ptr(), target.data_ptr(), 0.2, dl.data_ptr(),
                       loss_val.data_ptr(), sid)
        if rep == 3:
            l_ev[1].record(stream)
    torch.cuda.synchronize()
    l_ms = l_ev[0].elapsed_time(l_ev[1])
    loss_eq11 = {"ms": l_ms, "loss": float(loss_val.item()),
                 "frac_hbm": LOSS_BYTES_PER_PX * npx / (l_ms * 1e-3) / PEAK_HBM_BPS}

    if args.calibrate_copy > 0:
        # a plain copy of known size, for scaling the HBM byte counters
        nbytes = args.calibrate_copy << 20
        src = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    acui = None if args.no_acui else acui_forward(args, dev, stream, st)
    rgb = None if args.no_rgb else rgb_forward(args, dev, stream, st, w, g, cams)

    # ---- CPU baseline: the FP64 oracle on a bounded sample of views ---------
    cpu = None
    if not args.no_cpu:
        import oracle as O
        st_o = O.Settings(tile=args.tile)
        ocams = [O.camera(w.angles[v], S.L_SO, S.L_SD, w.sizes[v][0], w.sizes[v][1], D, D)
                 for v in range(w.n_views)]
        # the L1 targets are inputs of the step (the GPU renders them once,
        # outside timing): rendered here before the timed region too, for the
        # views the time budget can reach
        per_view_s = None
        targets = {}
        done_views = 0
        timed_s = 0.0
        # views in order, cycling, until the time budget is spent (at least one);
        # timed per view: pair emission + sort, binned forward, L1 upstream,
        # binned adjoint to every parameter -- the GPU step's work
        while True:
            v = done_views % w.n_views
            c = ocams[v]
            if v not in targets:
                prt = O.pairs(tgt_np, [c], st_o)
                targets[v] = O.render_binned(tgt_np, [c], st_o, prt["values"], prt["ranges"])["image"]
            t0 = time.perf_counter()
            pr = O.pairs(g_np, [c], st_o)
            r = O.render_binned(g_np, [c], st_o, pr["values"], pr["ranges"])
            up = (np.sign(r["image"] - targets[v]) * scale).astype(np.float32)
            O.backward(g_np, [c], st_o, up, binned=(pr["values"], pr["ranges"]))
            timed_s += time.perf_counter() - t0
            done_views += 1
            if timed_s >= args.cpu_seconds:
                break
        model = "unknown"
        try:
            for line in open("/proc/cpuinfo"):
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
        except OSError:
            pass
        cpu = {"value": done_views / timed_s, "unit": "views/s", "cores": O.threads(),
               "cpu_model": model, "kind": "oracle",
               "sample": f"{done_views} view passes (views 0..{w.n_views - 1} in turn; timed: pair "
                         f"emission + sort, binned forward, L1 upstream, binned adjoint, FP64; the "
                         f"targets rendered before timing), {timed_s:.1f} s timed"}

    if args.workload == 3:
        metric = "DRR fwd+bwd views/s at 512^2, 200k Gaussians; batched vs per-view, same GPU"
    else:
        metric = f"DRR fwd+bwd{'+Adam' if opt is not None else ''} views/s, {w.describe()}"
    res = {
        "metric": metric,
        "value": value,
        "unit": "views/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{w.describe()}, "
                               + ("L1" if args.loss == "l1" else "Eq.11 L1+SSIM (gamma 0.2)")
                               + ", fwd+bwd" + ("+Adam" if opt is not None else ""),
                   "gaussians": w.n, "views": w.n_views,
                   "detector": "x".join(map(str, w.sizes[0])) if len(set(w.sizes)) == 1 else "mixed",
                   "tile": args.tile, "lds_batch": args.lds, "persistent": bool(args.persistent),
                   "store_slots": args.store, "adam": opt is not None,
                   "path": "batched, one HIP graph per step" if graph is not None else "batched, eager",
                   "autotuned": tuned},
        "roofline": {"bound": "alu", "kernel": dom, "achieved": achieved / 1e12,
                     "peak": PEAK_LANE_OPS / 1e12, "unit": "T lane-op/s",
                     "frac": achieved / PEAK_LANE_OPS,
                     "frac_of_fp32_flops_peak": achieved / (PEAK_FP32_TFLOPS * 1e12),
                     "traffic": traffic, "launch_ms": dom_ms, "lane_ops_per_launch": dom_ops,
                     "work_model": f"fwd {LANE_OPS_EVAL_FWD}/evaluation; bwd {LANE_OPS_EVAL_BWD}/"
                                   f"revisited evaluation + {WAVE_INSTR_REDUCTION} x {WAVE} per "
                                   "(Gaussian, wavefront) reduction",
                     "note": "the model prices each reduction as a 6-level butterfly per value "
                             f"({WAVE_INSTR_REDUCTION} wavefront instructions); the backward's "
                             "reduce-scatter issues about 18 per entry, so the model's lane "
                             "operations exceed the instructions issued and frac can pass 1"},
        "cpu_baseline": cpu,
        "graph": graph,
        "eager": eager,
        "per_view": per_view,
        "batched_over_per_view": (value / per_view["value"]) if per_view else None,
        "kernels_ms": {"k_render_fwd": fwd_ms, "k_render_bwd": bwd_ms},
        "stages": stages,
        "rirf": rirf,
        "loss_eq11": loss_eq11,
        "acui_forward": acui,
        "rgb_forward": rgb,
        "work": {"pairs": n_pairs, "evals": evals, "contributors": contribs,
                 "revisited": upto, "reductions": reductions},
        "lanes": lanes,
        "evals_per_s": evals / (ms_step * 1e-3),
        "wall_s": wall_b,
        "kernel_source_hash": kernel_source_hash(),
        "hbm": hbm,
        "measured_peaks": None if args.no_peaks else measured_peaks(dev, stream),
    }
    print(json.dumps(res))


if __name__ == "__main__":
    main()
