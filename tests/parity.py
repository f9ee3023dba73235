"""Comparison of GPU results with the FP64 oracle (test infrastructure).

Modes are matched by mutual best cosine; the mode error is 1 - cos in FP64.
Labels are compared after remapping GPU mode indices through the matching and
must agree exactly except on two counted exempt sets: pixels whose best
similarity lies within BAND of the bandwidth threshold, and pixels whose best
and second-best similarities lie within BAND of each other (argmax near-ties;
for the BF16 form, within the band its largest mode error allows).

The BF16 bar (assert_bf16_bar): found modes within BF16_TOL, at most
BF16_LOST_FRAC of the oracle's modes lost (and as many extra), and each one
traced to a changed trajectory: the oracle's rounds are iterated again on
their own seed lists in the BF16 form, and a lost mode's own seed, or a seed
of its round or an earlier one, takes another outcome than in FP64 (the
arithmetic changed that trajectory, directly or through what it changed
later); an extra mode sits on a changed seed's endpoint or next to a lost
mode.
"""
from __future__ import annotations

import dataclasses

import numpy as np

BAND = 1e-4
BF16_TOL = 1e-3          # mode error bar of the BF16 form
BF16_LOST_FRAC = 0.02    # at most this share of the oracle's modes may be lost, each traced


def mode_error(a, b) -> np.ndarray:
    """1 - cos between matching rows, in FP64."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return 1.0 - np.sum(a * b, axis=1) / (np.linalg.norm(a, axis=1) * np.linalg.norm(b, axis=1))


@dataclasses.dataclass
class ModeMatch:
    pairs: np.ndarray        # (k, 2): (gpu index, oracle index)
    errors: np.ndarray       # 1 - cos for each pair
    unmatched_gpu: int
    unmatched_oracle: int

    @property
    def max_error(self) -> float:
        return float(self.errors.max()) if len(self.errors) else 0.0


def match_modes(gpu_modes, oracle_modes) -> ModeMatch:
    g = np.asarray(gpu_modes, np.float64)
    o = np.asarray(oracle_modes, np.float64)
    if len(g) == 0 or len(o) == 0:
        return ModeMatch(np.zeros((0, 2), np.int64), np.zeros(0), len(g), len(o))
    gn = g / np.linalg.norm(g, axis=1, keepdims=True)
    on = o / np.linalg.norm(o, axis=1, keepdims=True)
    s = gn @ on.T
    bg = np.argmax(s, axis=1)
    bo = np.argmax(s, axis=0)
    pairs = np.array([(i, bg[i]) for i in range(len(g)) if bo[bg[i]] == i], np.int64).reshape(-1, 2)
    err = 1.0 - s[pairs[:, 0], pairs[:, 1]] if len(pairs) else np.zeros(0)
    return ModeMatch(pairs, err, len(g) - len(pairs), len(o) - len(pairs))


@dataclasses.dataclass
class LabelCompare:
    n_fg: int
    mismatched: int           # mismatches outside the exempt sets
    exempt_band: int          # pixels within BAND of the bandwidth threshold
    exempt_tie: int           # argmax near-ties
    mismatched_exempt: int    # mismatches inside the exempt sets
    unmatched_mode_pixels: int


def tie_band(max_mode_error: float) -> float:
    """Width of the argmax near-tie set for modes within `max_mode_error`
    (1 - cos) of the oracle's: a unit mode that far off moves every
    similarity by at most |m' - m| = sqrt(2 * error), so a pixel's best and
    second-best modes can swap only where their similarities lie within
    twice that of each other.  Never below BAND."""
    return max(BAND, 2.0 * float(np.sqrt(2.0 * max(max_mode_error, 0.0))))


def compare_labels(gpu_labels, res, match: ModeMatch, thr: float, tie_width: float = BAND,
                   lost_modes=()) -> LabelCompare:
    """Compare GPU labels (H*W, -1 background) with the oracle result.
    tie_width: the argmax near-tie band; lost_modes: oracle modes the GPU
    result does not hold (their pixels are counted as exempt)."""
    ol = np.asarray(res.labels).reshape(-1)
    band = np.abs(res.best - thr) < BAND
    tie = np.abs(res.best - res.second) < tie_width
    return compare_labels_fg(gpu_labels, res.fg, ol[res.fg], band, tie, match, lost_modes)


def compare_labels_fg(gpu_labels, fg, o_fg, band, tie, match: ModeMatch, lost_modes=()) -> LabelCompare:
    """The same from the oracle's foreground labels and exempt masks (per
    foreground pixel, raster order)."""
    gl = np.asarray(gpu_labels).reshape(-1).astype(np.int64)
    bg_ok = np.all(gl[np.setdiff1d(np.arange(len(gl)), fg)] == -1)
    assert bg_ok, "background pixels must be labelled -1"
    remap = np.full(max(1, gl.max() + 1), -2, np.int64)
    for gi, oi in match.pairs:
        remap[gi] = oi
    g_fg = gl[fg]
    mapped = np.where(g_fg >= 0, remap[np.clip(g_fg, 0, None)], -1)
    o_fg = np.asarray(o_fg).astype(np.int64)
    exempt = band | tie
    if len(lost_modes):
        exempt = exempt | np.isin(o_fg, np.asarray(list(lost_modes), np.int64))
    unmatched = mapped == -2
    bad = (mapped != o_fg) & ~unmatched
    return LabelCompare(len(fg), int(np.count_nonzero(bad & ~exempt)), int(band.sum()), int(tie.sum()),
                        int(np.count_nonzero(bad & exempt)), int(unmatched.sum()))


def near_tie_mask(n: int, near_idx, near_gap, width: float) -> np.ndarray:
    """Per foreground pixel: best - second < width, from a stored sparse list
    of the pixels whose gap is small (golden files keep gaps below 0.02)."""
    m = np.zeros(n, bool)
    m[np.asarray(near_idx)[np.asarray(near_gap) < width]] = True
    return m


def load_precision1024():
    """The stored oracle result of the 1024x1024 precision workload
    (tests/golden/precision1024_oracle.npz, written by make_precision1024.py
    from oracle/ alone): a dict of modes, mode_counts, fg_labels, band, tie,
    bandwidth and stats."""
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "precision1024_oracle.npz")
    z = np.load(path)
    n = int(z["n_fg"])
    return {"modes": z["modes"], "mode_counts": z["mode_counts"], "fg_labels": z["fg_labels"].astype(np.int64),
            "band": np.unpackbits(z["band"])[:n].astype(bool), "tie": np.unpackbits(z["tie"])[:n].astype(bool),
            "near_idx": z["near_idx"], "near_gap": z["near_gap"], **_provenance(z, ""),
            "bandwidth": float(z["bandwidth"]), "stats": json.loads(bytes(z["stats"]).decode())}


def _provenance(z, pre):
    off = z[pre + "round_off"]
    seeds = z[pre + "round_seeds"]
    conv = np.unpackbits(z[pre + "round_conv"])[:off[-1]].astype(bool)
    iters = z[pre + "round_iters"].astype(np.int64)
    return {"round_seeds": [seeds[off[i]:off[i + 1]] for i in range(len(off) - 1)],
            "round_conv": [conv[off[i]:off[i + 1]] for i in range(len(off) - 1)],
            "round_iters": [iters[off[i]:off[i + 1]] for i in range(len(off) - 1)],
            "mode_round": z[pre + "mode_round"], "mode_local": z[pre + "mode_local"],
            "mode_iters": z[pre + "mode_iters"]}


def _golden(name):
    import os
    return np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", name))


def load_batch_oracle():
    """The stored oracle results of five frames of the uneven batching
    workload (tests/golden/batch_oracle.npz, written by make_batch_oracle.py
    from oracle/ alone): {frame index: dict as load_precision1024}."""
    import json
    z = _golden("batch_oracle.npz")
    out = {}
    for i in z["frames"].tolist():
        n = len(z[f"f{i}_fg_labels"])
        out[i] = {"modes": z[f"f{i}_modes"], "mode_counts": z[f"f{i}_mode_counts"],
                  "fg_labels": z[f"f{i}_fg_labels"].astype(np.int64),
                  "band": np.unpackbits(z[f"f{i}_band"])[:n].astype(bool),
                  "tie": np.unpackbits(z[f"f{i}_tie"])[:n].astype(bool),
                  "near_idx": z[f"f{i}_near_idx"], "near_gap": z[f"f{i}_near_gap"], **_provenance(z, f"f{i}_"),
                  "bandwidth": float(z[f"f{i}_bandwidth"]),
                  "stats": json.loads(bytes(z[f"f{i}_stats"]).decode())}
    return out


def load_host_prune():
    """The stored oracle result of the 256x256 frame clustered with 20,000
    seeds carried in (tests/golden/host_prune_oracle.npz, written by
    make_host_prune.py from oracle/ alone)."""
    import json
    z = _golden("host_prune_oracle.npz")
    n = int(z["n_fg"])
    return {"modes": z["modes"], "mode_counts": z["mode_counts"], "fg_labels": z["fg_labels"].astype(np.int64),
            "band": np.unpackbits(z["band"])[:n].astype(bool), "tie": np.unpackbits(z["tie"])[:n].astype(bool),
            "bandwidth": float(z["bandwidth"]), "n_state_in": int(z["n_state_in"]), **_provenance(z, ""),
            "stats": json.loads(bytes(z["stats"]).decode())}


def provenance_of(res):
    """The provenance fields of a live oracle result (as the golden files
    store them): per round the seeds, converged flags and step counts; per
    mode its round, index in that round and step count; the modes."""
    owner = [(r, a) for r, lg in enumerate(res.rounds) for a in lg.accepted]
    return {"round_seeds": [lg.seeds for lg in res.rounds], "round_conv": [lg.converged for lg in res.rounds],
            "round_iters": [lg.iters for lg in res.rounds], "mode_round": [q[0] for q in owner],
            "mode_local": [q[1] for q in owner], "mode_iters": [res.rounds[q[0]].iters[q[1]] for q in owner],
            "modes": res.modes}


def trace_bf16(F, emb, mask, h, prov, lost, extra_modes, **kw):
    """Trace the BF16 result's differences from the oracle's to changed
    trajectories.  Every oracle round up to the last one needed is iterated
    again on the oracle's own seed list in the BF16 form (fms_shift_seeds,
    kw: parameters of the clustering call that also apply to the step); a
    seed has diverged when its converged flag or step count differs from
    FP64.  A lost oracle mode is 'direct' when its own seed diverged (or
    ends farther than BF16_TOL from it), 'cascade' when another seed of its
    round or an earlier one diverged (a changed endpoint can be accepted in
    its place, or change the coverage that the later rounds' seeds come
    from), else unexplained.  An extra GPU mode is explained when it lies
    within BF16_TOL of a diverged seed's BF16 endpoint or within h of a lost
    mode (it took that mode's place)."""
    rounds = len(prov["round_seeds"])
    last = max([int(prov["mode_round"][k]) for k in lost], default=-1)
    if len(extra_modes):
        last = rounds - 1
    div_round, div_ends = [], []
    runs = {}
    for r in range(last + 1):
        print("[case] lockstep trace of round", r, len(prov["round_seeds"][r]), flush=True)
        g = F.shift_seeds(emb, mask, np.asarray(prov["round_seeds"][r], np.int32), bandwidth=h,
                          precision=F.BF16_REFINE, **kw)
        gc = g["converged"].cpu().numpy().astype(bool)
        gi = g["iters"].cpu().numpy()
        d = (gc != np.asarray(prov["round_conv"][r], bool)) | (gc & (gi != np.asarray(prov["round_iters"][r])))
        runs[r] = g
        div_round.append(int(d.sum()))
        if d.any():
            div_ends.append(g["endpoints"].cpu().numpy()[d & gc])
    ends = np.concatenate(div_ends) if div_ends else np.zeros((0, np.asarray(prov["modes"]).shape[1]))
    out = {"diverged_per_round": div_round, "lost": [], "extra": []}
    for k in lost:
        r, a = int(prov["mode_round"][k]), int(prov["mode_local"][k])
        g = runs[r]
        conv = bool(g["converged"][a].item())
        it = int(g["iters"][a].item())
        err = float(mode_error(g["endpoints"][a:a + 1].cpu().numpy(), prov["modes"][k:k + 1])[0])
        if (not conv) or it != int(prov["mode_iters"][k]) or err > BF16_TOL:
            why = "direct"
        elif sum(div_round[:r + 1]) > 0:
            why = "cascade"
        else:
            why = None
        out["lost"].append({"mode": int(k), "round": r, "converged": conv, "iters": it,
                            "oracle_iters": int(prov["mode_iters"][k]), "err": err, "why": why})
    lost_m = np.asarray(prov["modes"])[list(lost)] if len(lost) else np.zeros((0, ends.shape[1]))
    for gm in extra_modes:
        gm = np.asarray(gm, np.float64)[None, :]
        near_end = len(ends) and float(mode_error(np.repeat(gm, len(ends), 0), ends).min()) <= BF16_TOL
        near_lost = len(lost_m) and float(mode_error(np.repeat(gm, len(lost_m), 0), lost_m).min()) <= h
        out["extra"].append({"explained": bool(near_end or near_lost), "near_diverged_end": bool(near_end),
                             "near_lost_mode": bool(near_lost)})
    return out


def assert_bf16_bar(F, emb, mask, h, modes, labels_cmp, mm, prov, trace_kw=None):
    """The BF16 bar.  An oracle mode counts as found when a GPU mode matches
    it (mutual best) within BF16_TOL; lost oracle modes and extra GPU modes
    (matching none within BF16_TOL) may each be at most BF16_LOST_FRAC of the
    oracle's modes (at least one), and every one must be traced to a changed
    trajectory (trace_bf16); labels exact outside the exempt sets (the
    near-tie band from the largest error of the found modes, and the pixels
    of lost modes).  labels_cmp(tie_width, lost, match) returns the label
    comparison under the matching of the found modes (pixels of extra modes
    are not compared).  Returns (lost, extra, trace, label comparison)."""
    n_oracle = len(prov["modes"])
    good = mm.errors <= BF16_TOL
    found = set(mm.pairs[good, 1].tolist())
    lost = [k for k in range(n_oracle) if k not in found]
    gpu_good = set(mm.pairs[good, 0].tolist())
    g_modes = modes.cpu().numpy() if hasattr(modes, "cpu") else np.asarray(modes)
    extra = [g for g in range(len(g_modes)) if g not in gpu_good]
    max_err = float(mm.errors[good].max()) if good.any() else 0.0
    print(f"bf16 bar: {len(g_modes)} GPU / {n_oracle} oracle modes, found {len(found)} (max err "
          f"{max_err:.2e}), lost {lost}, extra {extra}", flush=True)
    cap = max(1, int(BF16_LOST_FRAC * n_oracle))
    assert len(lost) <= cap and len(extra) <= cap, (lost, extra)
    tr = trace_bf16(F, emb, mask, h, prov, lost, g_modes[extra], **(trace_kw or {})) if (lost or extra) else None
    if tr is not None:
        print("bf16 trace:", tr, flush=True)
        assert all(t["why"] for t in tr["lost"]), tr
        assert all(t["explained"] for t in tr["extra"]), tr
    good_mm = ModeMatch(mm.pairs[good], mm.errors[good], len(extra), len(lost))
    width = tie_band(max_err)
    lc = labels_cmp(width, lost, good_mm)
    print(f"bf16 bar: tie band {width:.1e}, labels {lc}", flush=True)
    assert lc.mismatched == 0
    return lost, extra, tr, lc
