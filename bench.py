"""Benchmark: frames/sec and seed x pixel updates/sec of Faster Mean-shift on one
MI355X, 512 x 512 frame, D = 32, in the three arithmetic forms (split BF16, FP32,
BF16 + FP32 replay).

One step = one fms_cluster call on one frame already resident in HBM: compaction
and normalisation, the seed rounds of the online seed policy (seed selection,
fused mean-shift iterations, window counts, pruning, coverage), and the labels.
Every call is bracketed by HIP events on the stream the library works on; the
figure is the median over the timed calls, after the warm-up calls.

Prints one JSON line.  ``value`` is the split BF16 form's frames/sec (it meets
the FP32 accuracy bar); the FP32 form (``value_fp32``), the BF16 + FP32 replay
form, update rates, every form's mode error against the FP64 oracle, the
roofline of the dominant kernel (live HIP-event timings from the library), the
128 x 128, 1024 x 1024 and 64-frame batched workloads, and the oracle's CPU
rate on the same frames (all threads and one thread) are carried alongside.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"bf16": 2500.0, "fp32": 157.3}  # MI355X dense MFMA
PEAK_HBM_GBPS = 8000.0  # MI355X HBM3E
# Bytes per pixel value a step of each form reads (the split form keeps two
# BF16 parts), and the MFMA peak it runs against.
STEP_BYTES = {"fp32": 4, "bf16": 2, "split": 4}
STEP_PEAK = {"fp32": "fp32", "bf16": "bf16", "split": "bf16"}


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="budget of the oracle CPU baseline")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--batch-frames", type=int, default=64,
                    help="frames of the uneven batched workload reported under 'batched' (0: skip)")
    ap.add_argument("--batch-steps", type=int, default=5)
    ap.add_argument("--only-frame", action="store_true",
                    help="time the 512x512 frame in both forms only (no other sections; for kernel traces)")
    ap.add_argument("--only-batch", action="store_true",
                    help="time the uneven batched workload only (for kernel traces)")
    ap.add_argument("--only-1024", action="store_true",
                    help="time the 1024x1024 precision workload only (for kernel traces)")
    ap.add_argument("--profile-batch", action="store_true",
                    help="with --profile-run: cluster the uneven batch (--batch-frames, split BF16) --steps "
                         "times instead of the single frame")
    ap.add_argument("--profile-form", choices=("all", "fp32", "bf16", "split"), default="all",
                    help="with --profile-run on the single frame: the arithmetic form(s) to run")
    ap.add_argument("--profile-side", type=int, choices=(512, 1024), default=512,
                    help="with --profile-run on the single frame: the 512x512 frame or the 1024x1024 "
                         "precision frame")
    ap.add_argument("--profile-steps", action="store_true",
                    help="with --profile-run: single fused steps of each form on the 512x512 frame at "
                         "128, 512, 2048 and 8192 active seeds (--steps launches each, in that order)")
    ap.add_argument("--profile-run", action="store_true",
                    help="for hardware-counter passes: one plain 256 MiB device copy (the byte-count "
                         "reference), then --steps frames of each form; prints a short summary only")
    return ap.parse_args()


def _profile_run(a):
    import torch

    import paper_2007_14283_amd as fms
    import synth
    ref = torch.empty(64 << 20, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(ref)
    ref.fill_(1.0)
    torch.cuda.synchronize()
    dst.copy_(ref)  # reads and writes exactly 256 MiB
    torch.cuda.synchronize()
    if a.profile_steps:
        frame = synth.make_frame(synth.PLAIN512)
        emb = torch.from_numpy(frame.emb).cuda()
        mask = torch.from_numpy(frame.mask).cuda()
        order = fms.seed_order(frame.n_fg, 0)
        for prec in (fms.FP32, fms.BF16_REFINE, fms.BF16_SPLIT):
            for m in STEP_SEEDS:
                for _ in range(a.steps):
                    fms.shift_seeds(emb, mask, order[:m], bandwidth=frame.bandwidth, precision=prec, max_iter=1,
                                    gamma=1.0, refine_iters=0)
        torch.cuda.synchronize()
        print(f"profile run: copy 256 MiB, then for fp32, bf16, split and m in {STEP_SEEDS}: "
              f"{a.steps} single steps each", flush=True)
        return
    if a.profile_batch:
        frames = [synth.make_frame(sp) for sp in synth.batch_specs(a.batch_frames)]
        inp = [{"emb": torch.from_numpy(f.emb).cuda(), "mask": torch.from_numpy(f.mask).cuda(),
                "bandwidth": f.bandwidth} for f in frames]
        for _ in range(a.steps):
            res = fms.cluster_batch(inp, precision=fms.BF16_SPLIT)
        torch.cuda.synchronize()
        print(f"profile run: copy 256 MiB, {a.steps} calls of the {len(frames)}-frame batch, "
              f"{sum(len(r[0]) for r in res)} modes", flush=True)
        return
    frame = synth.make_frame(synth.PLAIN512 if a.profile_side == 512 else synth.PRECISION1024)
    emb = torch.from_numpy(frame.emb).cuda()
    mask = torch.from_numpy(frame.mask).cuda()
    forms = {"fp32": (fms.FP32,), "bf16": (fms.BF16_REFINE,), "split": (fms.BF16_SPLIT,),
             "all": (fms.FP32, fms.BF16_REFINE, fms.BF16_SPLIT)}[a.profile_form]
    for prec in forms:
        for _ in range(a.steps):
            modes, _, st = fms.cluster(emb, mask, frame.bandwidth, precision=prec)
    torch.cuda.synchronize()
    print(f"profile run: copy 256 MiB, {a.steps} frames per form, {len(modes)} modes", flush=True)


def _time_calls(torch, call, steps, warmup):
    """Median milliseconds of `steps` calls, each bracketed by HIP events on
    the current stream (the stream the library enqueues on), after `warmup`
    untimed calls; also the wall time of the timed loop and the last result."""
    for _ in range(warmup):
        call()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    last = None
    res = []
    t0 = time.perf_counter()
    for e0, e1 in ev:
        e0.record()
        last = call()
        e1.record()
        res.append(last)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = sorted(e0.elapsed_time(e1) for e0, e1 in ev)
    med = 0.5 * (ms[(steps - 1) // 2] + ms[steps // 2])
    return med, wall, last, res


def _time_form(fms, torch, emb, mask, h, precision, steps, warmup):
    """Whole-frame throughput without instrumentation (median of event-timed
    calls), then the same number of frames again with per-launch kernel
    timing for the roofline figures."""
    agg = {"step_ms": [0.0, 0.0], "step_updates": [0, 0], "step_launches": [0, 0], "step_pixels": [0, 0],
           "updates": 0, "refine_updates": 0}
    med, wall, last, res = _time_calls(torch, lambda: fms.cluster(emb, mask, h, precision=precision), steps, warmup)
    for r in res:
        agg["updates"] += r[2]["seed_pixel_updates"]
        agg["refine_updates"] += r[2]["refine_updates"]
    agg["wall_s"] = wall
    dt = med * 1e-3 * steps
    for _ in range(steps):
        st = fms.cluster(emb, mask, h, precision=precision, timing=1)[2]
        for k in range(2):
            agg["step_ms"][k] += st["step_ms"][k]
            agg["step_updates"][k] += st["step_updates"][k]
            agg["step_launches"][k] += st["step_launches"][k]
            agg["step_pixels"][k] += st["step_pixels"][k]
    torch.cuda.synchronize()
    return dt, agg, last


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_shift_512x512_d32_traffic.txt")
KERNEL_SRC = [os.path.join(ROOT, "paper_2007_14283_amd", "csrc", n) for n in ("kernels.hip", "fms_internal.h")]


def kernel_source_hash():
    """SHA-256 over the kernel sources (kernels.hip, then fms_internal.h)."""
    import hashlib
    h = hashlib.sha256()
    for path in KERNEL_SRC:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _measured_traffic(form):
    """HBM bytes per launch of the fused step of a form (fp32, bf16, split) on
    the 512x512 frame, or of the split form on the 64-frame batch
    ("batch_split"), from the committed counter summary (FETCH_SIZE +
    WRITE_SIZE, scaled by a plain copy); None when the kernel sources have
    changed since the counters were taken, or for a case not measured."""
    try:
        text = open(TRAFFIC_FILE).read()
        src = kernel_source_hash()
    except OSError:
        return None
    if f"kernels_sha256: {src}" not in text:
        return None
    for line in text.splitlines():
        f = line.split()
        if len(f) == 3 and f[0] == "traffic_bytes_per_launch" and f[1] == form:
            return float(f[2])
    return None


def _roofline(agg, dim, n_fg, form, traffic_key=""):
    """Roofline of the dominant kernel, the fused step of the form with the
    larger summed duration (the BF16 form's replay runs FP32 steps).  Its
    algorithmic work: 4 D flops per seed-pixel update, and per launch the
    pixels of the frames it steps once (n x D x b bytes, b from STEP_BYTES;
    the library counts n per stepped frame) plus the active centres in and out
    (2 x N_act x D x 4, N_act taken as updates / n: exact for one frame, a
    size-weighted mean over a batch's frames, kilobytes against the pixels'
    megabytes either way).  A launch's floor is the larger of its MFMA
    and HBM times (the min of the two update rates); `bound` is the term that
    dominates the summed floors, and `frac` its achieved rate over its peak,
    which is the summed floor over the measured time."""
    k = 1 if agg["step_ms"][1] >= agg["step_ms"][0] else 0
    kform = form if k == 1 else "fp32"
    ms = agg["step_ms"][k]
    t = ms * 1e-3
    launches = max(1, agg["step_launches"][k])
    flops = agg["step_updates"][k] * 4.0 * dim  # 2D for the dot product + 2D for the masked sum
    seeds = agg["step_updates"][k] / max(1, n_fg)
    pixels = agg["step_pixels"][k]
    nbytes = pixels * dim * STEP_BYTES[kform] + 8.0 * dim * seeds
    peak_f = PEAK_TFLOPS[STEP_PEAK[kform]]
    t_mfma = flops / (peak_f * 1e12)
    t_hbm = nbytes / (PEAK_HBM_GBPS * 1e9)
    tflops = flops / t / 1e12 if t > 0 else 0.0
    gbps = nbytes / t / 1e9 if t > 0 else 0.0
    if t_hbm > t_mfma:
        bound, achieved, peak, unit = "hbm", gbps, PEAK_HBM_GBPS, "GB/s"
    else:
        bound, achieved, peak, unit = "mfma", tflops, peak_f, "TFLOP/s"
    return {"kernel": "k_shift_" + kform, "bound": bound, "achieved": achieved, "peak": peak, "unit": unit,
            "frac": achieved / peak, "traffic": _measured_traffic(traffic_key + kform),
            "algorithmic_bytes_per_launch": nbytes / launches, "flops_per_launch": flops / launches,
            "avg_launch_us": ms * 1e3 / launches, "launches": agg["step_launches"][k],
            "mean_active_seeds": seeds / launches,
            "mfma": {"achieved_tflops": tflops, "peak": peak_f, "frac": tflops / peak_f,
                     "issued_frac": tflops / peak_f * (2.5 if kform == "split" else 1.0)},
            "hbm": {"achieved_gbps": gbps, "peak": PEAK_HBM_GBPS, "frac": gbps / PEAK_HBM_GBPS}}


def _accuracy(gpu_modes, gpu_labels, o_modes, fg, o_fg_labels, band, tie_of, tol):
    """A GPU result against an oracle result: modes found within `tol`
    (mutual best), lost oracle modes, extra GPU modes, and label mismatches
    outside the exempt sets (bandwidth band, near ties within the band the
    largest error of the found modes allows, pixels of lost modes)."""
    import numpy as np

    from tests import parity
    mm = parity.match_modes(gpu_modes, o_modes)
    good = mm.errors <= tol
    found = set(mm.pairs[good, 1].tolist())
    lost = [k for k in range(len(o_modes)) if k not in found]
    max_err = float(mm.errors[good].max()) if good.any() else 0.0
    width = parity.BAND if tol < 1e-4 else parity.tie_band(max_err)
    gm = parity.ModeMatch(mm.pairs[good], mm.errors[good], int(len(gpu_modes) - good.sum()), len(lost))
    lc = parity.compare_labels_fg(gpu_labels, fg, o_fg_labels, band, tie_of(width), gm, lost)
    return {"modes": int(len(gpu_modes)), "oracle_modes": int(len(o_modes)), "found": len(found),
            "max_mode_err": max_err, "lost": len(lost), "extra": int(len(gpu_modes) - good.sum()),
            "label_mismatch": lc.mismatched, "label_exempt_mismatch": lc.mismatched_exempt,
            "tie_band": width}


def _batch_accuracy(frames, res, tol):
    """Five frames of the batch against their stored oracle results."""
    import numpy as np

    from tests import parity
    gold = parity.load_batch_oracle()
    out = {}
    for i, o in gold.items():
        if i >= len(frames):
            continue
        fg = np.flatnonzero(frames[i].mask.reshape(-1))
        out[str(i)] = _accuracy(res[i][0].cpu().numpy(), res[i][1].cpu().numpy(), o["modes"], fg, o["fg_labels"],
                                o["band"], lambda w, o=o, n=len(fg): o["tie"] | parity.near_tie_mask(
                                    n, o["near_idx"], o["near_gap"], w), tol)
        out[str(i)]["side"] = frames[i].spec.height
    return out


def _batched(fms, torch, a):
    """The batched form on the uneven multi-frame workload: every frame of the
    batch clustered by one fms_cluster_batch call, against the same frames
    clustered one call at a time in FP32 (the plain form)."""
    import synth
    specs = synth.batch_specs(a.batch_frames)
    frames = [synth.make_frame(sp) for sp in specs]
    inp = [{"emb": torch.from_numpy(f.emb).cuda(), "mask": torch.from_numpy(f.mask).cuda(),
            "bandwidth": f.bandwidth} for f in frames]
    torch.cuda.synchronize()
    nf = len(frames)
    sides = sorted({sp.height for sp in specs})
    out = {"workload": f"{nf} frames, side in {sides}, 10-300 cells, foreground 20-50%, sigma U(0.03, 0.1), "
                       f"D={specs[0].dim}, per-frame h; frame seeds 0..{nf - 1}",
           "frames": nf, "n_fg_total": int(sum(f.n_fg for f in frames)), "steps": a.batch_steps}
    for name, prec in (("bf16_refine", fms.BF16_REFINE), ("fp32", fms.FP32), ("bf16_split", fms.BF16_SPLIT)):
        # Two warm-up calls, the first result still held during the second,
        # so that the caching allocator holds the output tensors of two calls
        # before the timed loop (which keeps one result while making the next).
        res = fms.cluster_batch(inp, precision=prec)
        med, wall, res, allres = _time_calls(torch, lambda: fms.cluster_batch(inp, precision=prec), a.batch_steps, 1)
        upd = sum(r[2]["seed_pixel_updates"] + r[2]["refine_updates"] for rr in allres for r in rr)
        dt = med * 1e-3 * a.batch_steps
        st = fms.cluster_batch(inp, precision=prec, timing=1)[0][2]
        agg = {k: list(st[k]) for k in ("step_ms", "step_updates", "step_launches", "step_pixels")}
        out[name] = {"frames_per_s": nf * a.batch_steps / dt, "ms_per_batch": med,
                     "wall_ms_per_batch": 1e3 * wall / a.batch_steps,
                     "updates_per_s": upd / dt, "modes": int(sum(len(r[0]) for r in res)),
                     "roofline": _roofline(agg, specs[0].dim, out["n_fg_total"],
                                           {fms.FP32: "fp32", fms.BF16_REFINE: "bf16", fms.BF16_SPLIT: "split"}[prec],
                                           traffic_key="batch_"),
                     "vs_oracle": _batch_accuracy(frames, res, 1e-3 if prec == fms.BF16_REFINE else 1e-5)}
        del res, allres
    # Autotuned tiles: fms_autotune_batch on these frames (split BF16 form);
    # its entries serve the batch calls when whole calls got faster with them.
    t0 = time.perf_counter()
    tune = fms.autotune_batch(inp, precision=fms.BF16_SPLIT)
    tune_s = time.perf_counter() - t0
    res = fms.cluster_batch(inp, precision=fms.BF16_SPLIT)
    med, wall, res, _ = _time_calls(torch, lambda: fms.cluster_batch(inp, precision=fms.BF16_SPLIT),
                                    a.batch_steps, 1)
    dt = med * 1e-3 * a.batch_steps
    out["bf16_split_autotuned"] = {"frames_per_s": nf * a.batch_steps / dt, "ms_per_batch": med,
                                    "kept": tune["kept"], "tune_s": tune_s, "call_ms_default": tune["ms_default"],
                                    "call_ms_tuned": tune["ms_tuned"], "modes": int(sum(len(r[0]) for r in res)),
                                    "entries": [{k: e[k] for k in ("precision", "seeds", "tile_seeds", "tile_items",
                                                                   "tile_waves")} for e in tune["entries"]]}
    fms.clear_tuning()
    # The plain form: the same frames, one FP32 call each.
    for x in inp[:2]:
        fms.cluster(x["emb"], x["mask"], x["bandwidth"], precision=fms.FP32)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for x in inp:
        fms.cluster(x["emb"], x["mask"], x["bandwidth"], precision=fms.FP32)
    torch.cuda.synchronize()
    out["fp32_one_call_per_frame"] = {"frames_per_s": nf / (time.perf_counter() - t0)}
    for name in ("bf16_split", "bf16_refine", "fp32"):
        out[f"{name}_batched_vs_fp32_one_call_per_frame"] = (out[name]["frames_per_s"] /
                                                            out["fp32_one_call_per_frame"]["frames_per_s"])
    return out


def _differentiation(fms, torch, frame, seeds_used, reps=5):
    """The differentiable form on the 512x512 frame: T = 10 unrolled FP32
    steps from as many seeds as the policy used (the first positions of the
    seed order), then the gradient of sum_j y_T,j . t_j (random unit targets)
    with respect to the embeddings."""
    T = 10
    emb = torch.from_numpy(frame.emb).cuda().requires_grad_(True)
    mask = torch.from_numpy(frame.mask).cuda()
    seeds = fms.seed_order(frame.n_fg, 0)[:seeds_used].to(torch.int32)
    g = torch.Generator(device="cpu").manual_seed(0)
    targets = torch.randn((seeds_used, frame.spec.dim), generator=g)
    targets = (targets / targets.norm(dim=1, keepdim=True)).cuda()

    def step():
        emb.grad = None
        y = fms.unroll(emb, mask, seeds, T, frame.bandwidth)
        (y * targets).sum().backward()

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    # T forward steps and one backward contraction of the same shape.
    flops = (T + 1) * seeds_used * frame.n_fg * 4.0 * frame.spec.dim
    return {"workload": f"512x512 frame, D={frame.spec.dim}, T={T} unrolled FP32 steps from {seeds_used} seeds "
                        f"(the policy's seed count, first positions of the seed order), backward of "
                        f"sum(y_T . unit targets) to the embeddings",
            "seeds": seeds_used, "steps": T, "fwd_bwd_per_s": 1.0 / dt, "ms_fwd_bwd": 1e3 * dt,
            "tflops": flops / dt / 1e12}


def _precision1024(fms, torch, reps=10):
    """The precision workload: one 1024x1024 frame, 300 cells, D=32, in both
    forms, with the mode error of each against the stored FP64 oracle result
    (tests/golden/precision1024_oracle.npz, written from oracle/ alone), then
    both forms again with the autotuner's table for this frame."""
    import numpy as np

    import synth
    from tests import parity
    spec = synth.PRECISION1024
    f = synth.make_frame(spec)
    g = parity.load_precision1024()
    e = torch.from_numpy(f.emb).cuda()
    m = torch.from_numpy(f.mask).cuda()
    out = {"workload": f"one {spec.height}x{spec.width} frame, {spec.n_cells} cells (radii {spec.r_min}-{spec.r_max}), "
                       f"D={spec.dim}, sigma={spec.sigma}, h={f.bandwidth}, seed {spec.seed}",
           "n_fg": f.n_fg, "oracle_modes": int(len(g["modes"]))}
    fg = np.flatnonzero(f.mask.reshape(-1))
    for name, prec, tol in (("bf16_refine", fms.BF16_REFINE, 1e-3), ("fp32", fms.FP32, 1e-5),
                            ("bf16_split", fms.BF16_SPLIT, 1e-5)):
        med, _, last, _ = _time_calls(torch, lambda p=prec: fms.cluster(e, m, f.bandwidth, precision=p), reps, 1)
        modes, labels, st = last
        dt = med * 1e-3
        out[name] = {"frames_per_s": 1.0 / dt, "ms_per_frame": med, "modes": int(len(modes)), "tol": tol,
                     "vs_oracle": _accuracy(modes.cpu().numpy(), labels.cpu().numpy(), g["modes"], fg,
                                            g["fg_labels"], g["band"], lambda w: g["tie"] | parity.near_tie_mask(
                                                len(fg), g["near_idx"], g["near_gap"], w), tol),
                     "updates_per_s": (st["seed_pixel_updates"] + st["refine_updates"]) / dt}
    # The same frame with the decomposition table fms_autotune picks for it.
    for name, prec, tol in (("bf16_split", fms.BF16_SPLIT, 1e-5), ("fp32", fms.FP32, 1e-5)):
        t0 = time.perf_counter()
        res = fms.autotune(e, m, f.bandwidth, precision=prec)
        tune_s = time.perf_counter() - t0
        med, _, last, _ = _time_calls(torch, lambda p=prec: fms.cluster(e, m, f.bandwidth, precision=p), reps, 1)
        modes = last[0]
        fms.clear_tuning()
        mm = parity.match_modes(modes.cpu().numpy(), g["modes"])
        out[name + "_autotuned"] = {
            "frames_per_s": 1e3 / med, "tune_s": tune_s, "kept": res["kept"],
            "call_ms_default": res["ms_default"], "call_ms_tuned": res["ms_tuned"],
            "oracle_modes_within_tol": int(np.sum(mm.errors <= tol)), "unmatched_oracle": mm.unmatched_oracle,
            "entries": [{k: q[k] for k in ("precision", "seeds", "tile_seeds", "tile_items", "tile_waves")} |
                        {"us_tuned": round(q["us_per_step"], 2), "us_default": round(q["us_default"], 2)}
                        for q in res["entries"]]}
    return out


def _appendix_a(fms, torch, reps=5):
    """Appendix A overlap workload: 1000x1000, D=18, eight noise-free discs of
    diameter 250 pulled together (overlap 0.3), P = 0.95, h = 0.1."""
    import synth
    emb, mask, owner, _ = synth.overlap_circles(0.3)
    e = torch.from_numpy(emb).cuda()
    m = torch.from_numpy(mask).cuda()
    out = {"workload": "1000x1000, D=18 (padded to 32), 8 noise-free discs of diameter 250, overlap 0.3, "
                       "P=0.95, h=0.1", "n_fg": int(mask.sum()), "visible_discs": int(len(set(owner[owner >= 0])))}
    for name, prec in (("bf16_split", fms.BF16_SPLIT), ("bf16_refine", fms.BF16_REFINE), ("fp32", fms.FP32)):
        fms.cluster(e, m, 0.1, precision=prec, p_target=0.95)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            modes, _, _ = fms.cluster(e, m, 0.1, precision=prec, p_target=0.95)
        torch.cuda.synchronize()
        out[name] = {"frames_per_s": reps / (time.perf_counter() - t0), "modes": int(len(modes))}
    return out


def _online_n(fms, torch, n_frames=10):
    """N carried across a drifting synthetic 512x512 sequence (Sec. 3.2.4),
    for N_initial in {64, 128, 256} and H in {4, 8, 16}: mean time per frame,
    mean seeds per frame and the final N (Table 3 / Table 4 style)."""
    import synth
    seq = synth.drifting_sequence(synth.PLAIN512, n_frames)
    inp = [(torch.from_numpy(f.emb).cuda(), torch.from_numpy(f.mask).cuda(), f.bandwidth) for f in seq]
    torch.cuda.synchronize()
    rows = []
    for n0 in (64, 128, 256):
        for big_h in (4.0, 8.0, 16.0):
            n_state, seeds, t_tot = 0, 0, 0.0
            for e, m, h in inp:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, _, st = fms.cluster(e, m, h, precision=fms.BF16_SPLIT, n_initial=n0, big_h=big_h,
                                       n_state_in=n_state)
                torch.cuda.synchronize()
                t_tot += time.perf_counter() - t0
                n_state = st["n_state_out"]
                seeds += st["seeds_used"]
            rows.append({"n_initial": n0, "big_h": big_h, "ms_per_frame": 1e3 * t_tot / n_frames,
                         "seeds_per_frame": seeds / n_frames, "final_n": n_state})
    return {"workload": f"{n_frames} frames of the 512x512 generator, cells drifting (1, 2) px per frame, "
                        f"split BF16, N carried", "runs": rows}


def _autotune(fms, torch, emb, mask, h, steps):
    """The autotuner on the 512x512 frame: the decomposition it picks per
    active-seed count (fused step + reduction, tuned against default), and the
    split BF16 frame rate with the tuned table against the defaults."""
    t0 = time.perf_counter()
    res = fms.autotune(emb, mask, h, precision=fms.BF16_SPLIT)
    tune_s = time.perf_counter() - t0
    ent = res["entries"]
    rates = {}
    for name in ("default", "tuned", "default_again"):
        if name == "tuned":
            fms.autotune(emb, mask, h, precision=fms.BF16_SPLIT)
        else:
            fms.clear_tuning()
        fms.cluster(emb, mask, h, precision=fms.BF16_SPLIT)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fms.cluster(emb, mask, h, precision=fms.BF16_SPLIT)
        torch.cuda.synchronize()
        rates[name] = steps / (time.perf_counter() - t0)
    fms.clear_tuning()
    return {"tune_s": tune_s, "kept": res["kept"], "call_ms_default": res["ms_default"],
            "call_ms_tuned": res["ms_tuned"],
            "entries": [{k: e[k] for k in ("precision", "seeds", "tile_seeds", "tile_items", "tile_waves")} |
                        {"us_tuned": round(e["us_per_step"], 2), "us_default": round(e["us_default"], 2)}
                        for e in ent],
            "frames_per_s_default": 0.5 * (rates["default"] + rates["default_again"]),
            "frames_per_s_tuned": rates["tuned"]}


STEP_SEEDS = (128, 512, 2048, 8192)


def _step_scaling(fms, torch, emb, mask, frame, reps=5):
    """One fused step (no reduction) of each form at 128 to 8,192 active
    seeds on the 512x512 frame (the first positions of the seed order), timed
    with the library's kernel-bound events (fms_params.timing): median of
    `reps` launches.  TFLOP/s count the algorithmic 4 D flops per seed-pixel
    update; the split form issues 2.5 times as many on the matrix cores."""
    import numpy as np
    n = frame.n_fg
    order = fms.seed_order(n, 0).to(torch.int32)
    rows = []
    for name, prec, peak, issue in (("fp32", fms.FP32, 157.3, 1.0), ("bf16", fms.BF16_REFINE, 2500.0, 1.0),
                                    ("bf16_split", fms.BF16_SPLIT, 2500.0, 2.5)):
        k = 0 if prec == fms.FP32 else 1
        for m in STEP_SEEDS:
            ts = []
            for _ in range(reps + 1):
                st = fms.shift_seeds(emb, mask, order[:m], bandwidth=frame.bandwidth, precision=prec, max_iter=1,
                                     gamma=1.0, refine_iters=0, timing=1)["stats"]
                ts.append(st["step_ms"][k] / max(1, st["step_launches"][k]))
            us = 1e3 * float(np.median(ts[1:]))
            tf = m * n * 4.0 * frame.spec.dim / (us * 1e-6) / 1e12
            rows.append({"form": name, "active_seeds": m, "us": us, "tflops": tf, "frac": tf / peak,
                         "issued_frac": issue * tf / peak})
    return {"workload": "one fused step on the 512x512 frame, first positions of the seed order as centres",
            "peak_tflops": {"fp32": 157.3, "bf16": 2500.0}, "rows": rows}


def _cpu_threads():
    try:
        from threadpoolctl import threadpool_info
        info = threadpool_info()
        return max([int(i.get("num_threads", 1)) for i in info] or [1])
    except Exception:
        return os.cpu_count() or 1


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_rate(frame, reps, budget_s, threads=None):
    """Frames/s of the FP64 oracle on `frame`: up to `reps` runs, stopping
    once `budget_s` seconds are spent (at least one run); with `threads`, the
    BLAS pools are limited to that many threads.  Returns (rate, runs,
    result)."""
    from oracle import cluster as C
    ctx = None
    if threads is not None:
        from threadpoolctl import threadpool_limits
        ctx = threadpool_limits(threads)
    try:
        runs, t_cpu, res = 0, 0.0, None
        while runs == 0 or (t_cpu < budget_s and runs < reps):
            t0 = time.perf_counter()
            res = C.cluster(frame.emb, frame.mask, C.Params(bandwidth=frame.bandwidth))
            t_cpu += time.perf_counter() - t0
            runs += 1
    finally:
        if ctx is not None:
            ctx.unregister()
    return runs / t_cpu, runs, res


def _vs_oracle(modes, labels, res, thr, tol):
    """A single-frame GPU result against a live oracle result (_accuracy)."""
    import numpy as np

    from tests import parity
    fg = res.fg
    return _accuracy(modes.cpu().numpy(), labels.cpu().numpy(), res.modes, fg, np.asarray(res.labels).reshape(-1)[fg],
                     np.abs(res.best - thr) < parity.BAND, lambda w: np.abs(res.best - res.second) < w, tol)


def main():
    a = _args()
    if a.profile_run:
        _profile_run(a)
        return
    if a.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU per process here; --gpus must be 1"}))
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2007_14283_amd as fms
    import synth

    if a.only_batch:
        print(json.dumps({"batched": _batched(fms, torch, a)}), flush=True)
        return
    if a.only_1024:
        print(json.dumps({"precision_1024": _precision1024(fms, torch, reps=a.steps)}), flush=True)
        return

    spec = synth.PLAIN512
    frame = synth.make_frame(spec)
    h = frame.bandwidth
    emb = torch.from_numpy(frame.emb).cuda()
    mask = torch.from_numpy(frame.mask).cuda()
    torch.cuda.synchronize()

    dt_b, agg_b, last_b = _time_form(fms, torch, emb, mask, h, fms.BF16_REFINE, a.steps, a.warmup)
    print(f"bf16+replay: median {1e3 * dt_b / a.steps:.3f} ms per frame", file=sys.stderr, flush=True)
    dt_f, agg_f, last_f = _time_form(fms, torch, emb, mask, h, fms.FP32, a.steps, a.warmup)
    print(f"fp32: median {1e3 * dt_f / a.steps:.3f} ms per frame", file=sys.stderr, flush=True)
    dt_s, agg_s, last_s = _time_form(fms, torch, emb, mask, h, fms.BF16_SPLIT, a.steps, a.warmup)
    print(f"split bf16: median {1e3 * dt_s / a.steps:.3f} ms per frame", file=sys.stderr, flush=True)

    fps_b = a.steps / dt_b
    fps_f = a.steps / dt_f
    fps_s = a.steps / dt_s
    upd_b = (agg_b["updates"] + agg_b["refine_updates"]) / dt_b
    upd_f = agg_f["updates"] / dt_f
    upd_s = agg_s["updates"] / dt_s

    st_b = last_b[2]
    roof_s = _roofline(agg_s, spec.dim, frame.n_fg, "split")
    # The headline is the BF16 form that meets the 1e-3 mode-error bar with
    # the fewest frames lost to rounding: the split (hi/lo) BF16 form, which
    # runs every contraction on BF16 MFMA and returns the oracle's modes to
    # FP32 accuracy.  The plain BF16 form with its FP32 replay is reported
    # beside it ("bf16_refine"), and the FP32 form ("fp32", "value_fp32").
    out = {
        "metric": "frames/sec (BF16 on MFMA, at <= 1e-3 mode error) and seed-pixel updates/sec, 512x512 D=32; "
                  "vs FP32",
        "value": fps_s,
        "value_fp32": fps_f,
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * dt_s / a.steps,
        "wall_ms_per_step": 1e3 * agg_s["wall_s"] / a.steps,
        "timing": "median of the timed calls, each bracketed by HIP events on the library's stream",
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16 (hi/lo split) MFMA, f32 accumulate",
        "data": "synthetic",
        "config": {"workload": f"one {spec.height}x{spec.width} frame, {spec.n_cells} elliptic cells "
                               f"(radii {spec.r_min}-{spec.r_max}), D={spec.dim}, sigma={spec.sigma}, "
                               f"<=5% overlap, h={h}, seed {spec.seed}",
                   "form": "split BF16 (FMS_PREC_BF16_SPLIT)",
                   "n_fg": frame.n_fg, "bandwidth": h, "parallelism": "single GPU"},
        "updates_per_s": upd_s,
        "modes": int(len(last_s[0])),
        "speedup_vs_fp32": fps_s / fps_f,
        "fp32": {"frames_per_s": fps_f, "ms_per_frame": 1e3 * dt_f / a.steps, "updates_per_s": upd_f,
                 "modes": int(len(last_f[0])), "roofline": _roofline(agg_f, spec.dim, frame.n_fg, "fp32"),
                 "kernel_ms_per_frame": agg_f["step_ms"][0] / a.steps},
        "bf16_refine": {"frames_per_s": fps_b, "ms_per_frame": 1e3 * dt_b / a.steps, "updates_per_s": upd_b,
                        "modes": int(len(last_b[0])), "roofline": _roofline(agg_b, spec.dim, frame.n_fg, "bf16"),
                        "kernel_ms_per_frame": [agg_b["step_ms"][0] / a.steps, agg_b["step_ms"][1] / a.steps],
                        "replay": {k: st_b[k] for k in ("refine_steps", "refine_unconverged", "refine_step_diff",
                                                        "refine_gamma_cut", "refine_updates")}},
        "kernel_ms_per_frame": agg_s["step_ms"][1] / a.steps,
        "roofline": roof_s,
        "mfma_target": {"frac_target": 0.5, "frac": roof_s["mfma"]["frac"], "met": roof_s["mfma"]["frac"] >= 0.5,
                        "issued_frac": roof_s["mfma"]["issued_frac"],
                        "note": "algorithmic flops (4D per seed-pixel update) of the fused step on this frame over "
                                "dense BF16 MFMA peak, against the 0.5 utilisation target; the split form issues "
                                "2.5x those flops on the matrix cores"},
    }

    if a.only_frame:
        print(json.dumps(out), flush=True)
        return

    # The 128x128, D=16 workload (20 cells), both forms, same protocol.
    tiny = synth.make_frame(synth.TINY)
    te = torch.from_numpy(tiny.emb).cuda()
    tm = torch.from_numpy(tiny.mask).cuda()
    cfg1 = {"workload": f"one 128x128 frame, 20 elliptic cells (radii 4-12), D=16, sigma=0.05, h={tiny.bandwidth}, "
                        f"seed 0", "n_fg": tiny.n_fg}
    for name, prec in (("bf16_refine", fms.BF16_REFINE), ("fp32", fms.FP32), ("bf16_split", fms.BF16_SPLIT)):
        med, _, last, _ = _time_calls(torch, lambda p=prec: fms.cluster(te, tm, tiny.bandwidth, precision=p),
                                      a.steps, a.warmup)
        cfg1[name] = {"frames_per_s": 1e3 / med, "ms_per_frame": med, "modes": int(len(last[0])), "_last": last}
    out["plain_128"] = cfg1

    out["step_scaling"] = _step_scaling(fms, torch, emb, mask, frame)
    out["differentiation"] = _differentiation(fms, torch, frame, int(last_f[2]["seeds_used"]))
    print(f"differentiation: {out['differentiation']['ms_fwd_bwd']:.2f} ms forward+backward",
          file=sys.stderr, flush=True)

    out["precision_1024"] = _precision1024(fms, torch)
    out["autotune"] = _autotune(fms, torch, emb, mask, h, a.steps)
    out["appendix_a"] = _appendix_a(fms, torch)
    out["online_n"] = _online_n(fms, torch)

    if a.batch_frames > 0:
        out["batched"] = _batched(fms, torch, a)
        print(f"batched: {out['batched']['bf16_split']['frames_per_s']:.1f} frames/s (split BF16)",
              file=sys.stderr, flush=True)

    if not a.no_cpu:
        # The oracle as it stands, on the same frames: the 512x512 frame with
        # every BLAS thread (up to 3 runs within the time budget) and with one
        # thread (one run); the 128x128 frame 10 times each way.
        rate, runs, res = _oracle_rate(frame, 3, a.cpu_seconds)
        rate1, runs1, _ = _oracle_rate(frame, 1, 0.0, threads=1)
        trate, truns, tres = _oracle_rate(tiny, 10, a.cpu_seconds)
        trate1, truns1, _ = _oracle_rate(tiny, 10, a.cpu_seconds, threads=1)
        out["cpu_baseline"] = {"value": rate, "unit": "frames/s", "cores": _cpu_threads(), "kind": "oracle",
                               "sample": f"{runs} full runs on the same 512x512 frame (FP64 NumPy, all BLAS "
                                         f"threads)",
                               "cpu_model": _cpu_model(), "os_cpu_count": os.cpu_count(),
                               "blas_threads": _cpu_threads(),
                               "single_thread": {"value": rate1, "runs": runs1},
                               "plain_128": {"value": trate, "runs": truns, "single_thread": trate1,
                                             "single_thread_runs": truns1}}
        for name, last, tol in (("bf16_split", last_s, 1e-5), ("bf16", last_b, 1e-3), ("fp32", last_f, 1e-5)):
            out[f"{name}_vs_oracle"] = _vs_oracle(last[0], last[1], res, 1.0 - h, tol)
        for name, tol in (("bf16_refine", 1e-3), ("fp32", 1e-5), ("bf16_split", 1e-5)):
            last = cfg1[name]["_last"]
            cfg1[name]["vs_oracle"] = _vs_oracle(last[0], last[1], tres, 1.0 - tiny.bandwidth, tol)
    for name in ("bf16_refine", "fp32", "bf16_split"):
        cfg1[name].pop("_last", None)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
