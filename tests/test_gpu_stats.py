"""GPU checks of the fused-step counters that fms_stats reports when
fms_params.timing is set (the inputs of the bench's roofline).  A step launch
that steps a frame reads that frame's n pixel rows once and updates every
active centre against them; a launch that takes the early stop reads and
counts nothing.  So, summed over a call, the pixel rows equal n times the
frame's iterations, and the updates equal the seed-pixel updates the call
reports, for one frame and for every frame of a batch."""
import dataclasses

import pytest

import synth

pytestmark = pytest.mark.gpu

SPECS = [
    synth.MID,
    dataclasses.replace(synth.MID, height=96, width=128, n_cells=10, sigma=0.03, seed=7),
    dataclasses.replace(synth.MID, height=24, width=20, n_cells=2, seed=5),
]


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def F():
    import paper_2007_14283_amd as fms
    fms.library()
    return fms


def _slot(F, precision):
    # Index 0 counts the FP32 step, index 1 the BF16 step (both BF16 forms).
    return 0 if precision == F.FP32 else 1


@pytest.mark.parametrize("form", ["fp32", "split"])
def test_step_counters_single_frame(F, form):
    import torch
    prec = F.FP32 if form == "fp32" else F.BF16_SPLIT
    f = synth.make_frame(synth.MID)
    _say("step counters, one frame", form, f.n_fg)
    _, _, st = F.cluster(torch.from_numpy(f.emb).cuda(), torch.from_numpy(f.mask).cuda(), f.bandwidth,
                         precision=prec, timing=1)
    k = _slot(F, prec)
    assert st["n_fg"] == f.n_fg
    assert st["step_launches"][k] >= st["iterations_total"] > 0
    assert st["step_launches"][1 - k] == 0
    assert st["step_pixels"][k] == f.n_fg * st["iterations_total"]
    assert st["step_updates"][k] == st["seed_pixel_updates"]
    assert st["step_pixels"][k] <= st["step_updates"][k] <= st["step_pixels"][k] * st["seeds_used"]
    assert st["step_ms"][k] > 0.0


@pytest.mark.parametrize("form", ["fp32", "split"])
def test_step_counters_batch(F, form):
    import torch
    prec = F.FP32 if form == "fp32" else F.BF16_SPLIT
    frames = [synth.make_frame(s) for s in SPECS]
    _say("step counters, batch", form, [f.n_fg for f in frames])
    inp = [{"emb": torch.from_numpy(f.emb).cuda(), "mask": torch.from_numpy(f.mask).cuda(),
            "bandwidth": f.bandwidth} for f in frames]
    res = F.cluster_batch(inp, precision=prec, timing=1)
    k = _slot(F, prec)
    call = res[0][2]  # the call's launch counters come with the first frame's statistics
    pixels = sum(f.n_fg * r[2]["iterations_total"] for f, r in zip(frames, res))
    updates = sum(r[2]["seed_pixel_updates"] for r in res)
    assert call["step_launches"][k] >= max(r[2]["iterations_total"] for r in res) > 0
    assert call["step_pixels"][k] == pixels
    assert call["step_updates"][k] == updates
    assert call["step_pixels"][k] <= call["step_launches"][k] * sum(f.n_fg for f in frames)
