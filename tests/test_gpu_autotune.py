"""GPU tests of the fused-step autotuner (fms_autotune, fms_autotune_batch,
fms_clear_tuning).  Single frames: the table it reports is well formed, a
tuned handle still matches the FP64 oracle
(FP32 modes within 1e-5, labels exact outside the exempt sets), a call after
tuning equals, bit for bit, the call that fixes the chosen decomposition
explicitly when the entries were kept and the default call when they were
not, and clearing the table restores the default path bit for bit.  Batches:
the table is well formed, a tuned batch still matches the oracle frame by
frame, and batch entries leave single-frame calls bit-identical."""
import dataclasses

import numpy as np
import pytest

import synth
from oracle import cluster as C
from tests import parity

pytestmark = pytest.mark.gpu

FP32_TOL = 1e-5
# A frame with fewer than 128 foreground pixels: one seed count, one entry.
TINY = dataclasses.replace(synth.MID, height=16, width=16, n_cells=2, r_min=3, r_max=6, seed=6)


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def F():
    import paper_2007_14283_amd as fms
    fms.library()
    yield fms
    fms.clear_tuning()


def _dev(frame):
    import torch
    return torch.from_numpy(frame.emb).cuda(), torch.from_numpy(frame.mask).cuda()


def test_autotune_table_is_well_formed(F):
    f = synth.make_frame(synth.MID)
    emb, mask = _dev(f)
    _say("autotune MID fp32 + bf16")
    for prec, forms in ((F.FP32, {0}), (F.BF16_REFINE, {0, 1})):
        res = F.autotune(emb, mask, f.bandwidth, precision=prec)
        print(res)
        ent = res["entries"]
        assert res["ms_default"] > 0 and res["ms_tuned"] > 0
        assert res["kept"] == (res["ms_tuned"] < res["ms_default"])
        assert {e["precision"] for e in ent} == forms
        seeds = sorted({e["seeds"] for e in ent})
        assert seeds == [m for m in (128, 512, 2048, 8192) if m <= f.n_fg]
        for e in ent:
            assert e["dim_padded"] == 32 and e["n_fg"] == f.n_fg
            assert e["tile_items"] in (256, 512, 1024) and e["tile_waves"] in (4, 8, 16)
            assert e["tile_seeds"] in ((32, 64, 128) if e["precision"] == 1 else (16, 32, 64))
            assert 0 < e["us_per_step"] <= e["us_default"] * 1.5
    F.clear_tuning()


def test_tuned_handle_matches_oracle(F):
    f = synth.make_frame(synth.MID)
    emb, mask = _dev(f)
    _say("tuned MID vs oracle")
    F.autotune(emb, mask, f.bandwidth, precision=F.FP32)
    modes, labels, st = F.cluster(emb, mask, f.bandwidth, precision=F.FP32)
    F.clear_tuning()
    o = C.cluster(f.emb, f.mask, C.Params(bandwidth=f.bandwidth))
    mm = parity.match_modes(modes.cpu().numpy(), o.modes)
    lc = parity.compare_labels(labels.cpu().numpy(), o, mm, 1.0 - f.bandwidth)
    assert mm.unmatched_gpu == 0 and mm.unmatched_oracle == 0 and mm.max_error <= FP32_TOL
    assert lc.mismatched == 0
    for k in ("rounds", "seeds_used", "iterations_total"):
        assert st[k] == o.stats[k], k


def test_tuned_call_equals_explicit_decomposition(F):
    f = synth.make_frame(TINY)
    assert f.n_fg < 128
    emb, mask = _dev(f)
    _say("tuned TINY vs explicit", f.n_fg)
    res = F.autotune(emb, mask, f.bandwidth, precision=F.FP32)
    ent = res["entries"]
    assert len(ent) == 1 and ent[0]["seeds"] == f.n_fg
    e = ent[0]
    m1, l1, _ = F.cluster(emb, mask, f.bandwidth, precision=F.FP32)
    F.clear_tuning()
    if res["kept"]:
        m2, l2, _ = F.cluster(emb, mask, f.bandwidth, precision=F.FP32, tile_seeds=e["tile_seeds"],
                              tile_items=e["tile_items"], tile_waves=e["tile_waves"])
    else:
        m2, l2, _ = F.cluster(emb, mask, f.bandwidth, precision=F.FP32)
    assert np.array_equal(m1.cpu().numpy(), m2.cpu().numpy())
    assert np.array_equal(l1.cpu().numpy(), l2.cpu().numpy())


def test_clear_restores_default_path(F):
    f = synth.make_frame(synth.MID)
    emb, mask = _dev(f)
    _say("clear restores default")
    F.clear_tuning()
    m0, l0, _ = F.cluster(emb, mask, f.bandwidth, precision=F.BF16_REFINE)
    F.autotune(emb, mask, f.bandwidth, precision=F.BF16_REFINE)
    F.clear_tuning()
    m1, l1, _ = F.cluster(emb, mask, f.bandwidth, precision=F.BF16_REFINE)
    assert np.array_equal(m0.cpu().numpy(), m1.cpu().numpy())
    assert np.array_equal(l0.cpu().numpy(), l1.cpu().numpy())


def test_autotune_rejects_empty_mask(F):
    import torch
    f = synth.make_frame(TINY)
    emb, mask = _dev(f)
    with pytest.raises(F.FmsError):
        F.autotune(emb, torch.zeros_like(mask), f.bandwidth)


# fms_autotune_batch: launches over all frames of a batch (three MID frames
# of different seeds and TINY).
def _batch():
    import torch
    specs = [synth.MID.with_seed(s) for s in (0, 1, 2)] + [TINY]
    frames = [synth.make_frame(sp) for sp in specs]
    inp = [{"emb": torch.from_numpy(f.emb).cuda(), "mask": torch.from_numpy(f.mask).cuda(),
            "bandwidth": f.bandwidth} for f in frames]
    return frames, inp


def test_autotune_batch_table_and_oracle(F):
    frames, inp = _batch()
    n_max = max(f.n_fg for f in frames)
    _say("autotune batch", [f.n_fg for f in frames])
    res = F.autotune_batch(inp, precision=F.FP32)
    print(res)
    ent = res["entries"]
    assert res["ms_default"] > 0 and res["ms_tuned"] > 0
    assert res["kept"] == (res["ms_tuned"] < res["ms_default"])
    assert {e["precision"] for e in ent} == {0}
    assert sorted({e["seeds"] for e in ent}) == [m for m in (128, 512, 2048) if m <= n_max]
    for e in ent:
        assert e["dim_padded"] == 32 and e["n_fg"] == n_max
        assert e["tile_items"] in (256, 512, 1024) and e["tile_waves"] in (4, 8, 16)
        assert 0 < e["us_per_step"] <= e["us_default"] * 1.5
    out = F.cluster_batch(inp, precision=F.FP32)
    F.clear_tuning()
    for f, (modes, labels, st) in zip(frames, out):
        o = C.cluster(f.emb, f.mask, C.Params(bandwidth=f.bandwidth))
        mm = parity.match_modes(modes.cpu().numpy(), o.modes)
        lc = parity.compare_labels(labels.cpu().numpy(), o, mm, 1.0 - f.bandwidth)
        assert mm.unmatched_gpu == 0 and mm.unmatched_oracle == 0 and mm.max_error <= FP32_TOL
        assert lc.mismatched == 0
        for k in ("rounds", "seeds_used", "iterations_total"):
            assert st[k] == o.stats[k], k


def test_batch_entries_leave_single_frame_calls_alone(F):
    frames, inp = _batch()
    f = frames[0]
    emb, mask = _dev(f)
    _say("batch entries vs single frame")
    F.clear_tuning()
    m0, l0, _ = F.cluster(emb, mask, f.bandwidth, precision=F.BF16_REFINE)
    F.autotune_batch(inp, precision=F.BF16_REFINE)
    m1, l1, _ = F.cluster(emb, mask, f.bandwidth, precision=F.BF16_REFINE)
    F.clear_tuning()
    assert np.array_equal(m0.cpu().numpy(), m1.cpu().numpy())
    assert np.array_equal(l0.cpu().numpy(), l1.cpu().numpy())


def test_autotune_batch_needs_two_frames(F):
    frames, inp = _batch()
    with pytest.raises(F.FmsError):
        F.autotune_batch(inp[:1])


def test_autotune_batch_with_an_empty_frame(F):
    import torch
    frames, inp = _batch()
    inp = [inp[0], dict(inp[3], mask=torch.zeros_like(inp[3]["mask"]))]
    _say("autotune batch with an empty frame")
    res = F.autotune_batch(inp, precision=F.FP32)
    assert res["entries"] and res["ms_default"] > 0
    out = F.cluster_batch(inp, precision=F.FP32)
    F.clear_tuning()
    assert len(out[1][0]) == 0 and bool((out[1][1] == -1).all())
