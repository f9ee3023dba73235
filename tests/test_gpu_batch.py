"""GPU parity of the batched entry point (fms_cluster_batch): each frame of a
batch of uneven frames against the FP64 oracle run on that frame alone, and
against the single-frame call.  Same tolerances as the single-frame tests:
FP32 modes within 1e-5 (1 - cos), labels exact outside the counted exempt
sets; BF16 + FP32 replay: the BF16 bar of tests/parity.py per frame.  Also
five frames of the 64-frame uneven batching workload at full size (512^2 to
1024^2) against their stored oracle results."""
import dataclasses

import numpy as np
import pytest

import synth
from oracle import cluster as C
from tests import parity

pytestmark = pytest.mark.gpu

FP32_TOL = 1e-5
BF16_TOL = 1e-3

# D = 32 frames of different sizes, cell counts and noise (so different
# bandwidths by the same 99.9 % rule), one of them tiny.
SPECS = [
    synth.MID,
    dataclasses.replace(synth.MID, height=96, width=128, n_cells=10, sigma=0.03, seed=7),
    dataclasses.replace(synth.MID, height=64, width=160, n_cells=8, sigma=0.07, seed=11),
    dataclasses.replace(synth.MID, height=24, width=20, n_cells=2, seed=5),
]


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def F():
    import paper_2007_14283_amd as fms
    fms.library()
    return fms


@pytest.fixture(scope="module")
def frames():
    return [synth.make_frame(s) for s in SPECS]


@pytest.fixture(scope="module")
def oracles(frames):
    return [C.cluster(f.emb, f.mask, C.Params(bandwidth=f.bandwidth)) for f in frames]


def _inputs(frames, empty=()):
    import torch
    out = []
    for i, f in enumerate(frames):
        mask = torch.from_numpy(f.mask).cuda()
        if i in empty:
            mask = torch.zeros_like(mask)
        out.append({"emb": torch.from_numpy(f.emb).cuda(), "mask": mask, "bandwidth": f.bandwidth})
    return out


def test_batch_bandwidths_differ(frames):
    # The batch mixes bandwidths, so per-frame thresholds are exercised.
    assert len({f.bandwidth for f in frames}) >= 2


@pytest.mark.parametrize("precision", ["fp32", "split"])
def test_batch_fp32_matches_oracle(F, frames, oracles, precision):
    _say("batch", precision, [f.spec for f in frames])
    res = F.cluster_batch(_inputs(frames), precision=F.FP32 if precision == "fp32" else F.BF16_SPLIT)
    assert len(res) == len(frames)
    for f, o, (modes, labels, st) in zip(frames, oracles, res):
        mm = parity.match_modes(modes.cpu().numpy(), o.modes)
        lc = parity.compare_labels(labels.cpu().numpy(), o, mm, 1.0 - f.bandwidth)
        print(f"{f.spec.height}x{f.spec.width} h={f.bandwidth}: modes {len(modes)}/{len(o.modes)} "
              f"max err {mm.max_error:.2e} labels {lc}")
        assert mm.unmatched_gpu == 0 and mm.unmatched_oracle == 0
        assert mm.max_error <= FP32_TOL
        assert lc.mismatched == 0
        np.testing.assert_array_equal(mm.pairs[:, 0], mm.pairs[:, 1])
        for k in ("rounds", "seeds_used", "iterations_total", "n_discarded", "n_state_out", "seed_pixel_updates"):
            assert st[k] == o.stats[k], k
        np.testing.assert_array_equal(st["mode_counts"].cpu().numpy(), o.mode_counts)


def test_batch_equals_single_frame_calls(F, frames):
    _say("batch vs single", len(frames))
    inp = _inputs(frames)
    batch = F.cluster_batch(inp, precision=F.FP32)
    for x, (bm, bl, bst) in zip(inp, batch):
        sm, sl, sst = F.cluster(x["emb"], x["mask"], x["bandwidth"], precision=F.FP32)
        assert bm.shape == sm.shape
        err = 1.0 - np.sum(bm.cpu().double().numpy() * sm.cpu().double().numpy(), axis=1)
        assert err.size == 0 or err.max() <= FP32_TOL
        assert bst["rounds"] == sst["rounds"] and bst["seeds_used"] == sst["seeds_used"]
        diff = int((bl != sl).sum().item())
        assert diff == 0, diff


def test_batch_bf16_refine(F, frames, oracles):
    _say("batch bf16")
    inp = _inputs(frames)
    res = F.cluster_batch(inp, precision=F.BF16_REFINE)
    for f, o, x, (modes, labels, st) in zip(frames, oracles, inp, res):
        if len(o.modes) == 0:
            assert len(modes) == 0
            continue
        mm = parity.match_modes(modes.cpu().numpy(), o.modes)
        lab = labels.cpu().numpy()
        print(f"{f.spec.height}x{f.spec.width} h={f.bandwidth}")
        parity.assert_bf16_bar(F, x["emb"], x["mask"], f.bandwidth, modes, lambda w, lost, match: parity.compare_labels(
            lab, o, match, 1.0 - f.bandwidth, tie_width=w, lost_modes=lost), mm, parity.provenance_of(o))
        assert st["refine_steps"] >= 2


# Five frames of the uneven batching workload at their full size, clustered
# together in one call, against the oracle results stored for them
# (tests/golden/batch_oracle.npz, pinned in test_golden_batch.py).
@pytest.fixture(scope="module")
def golden():
    g = parity.load_batch_oracle()
    specs = synth.batch_specs(64)
    fr = {i: synth.make_frame(specs[i]) for i in g}
    return g, fr


@pytest.mark.parametrize("precision", ["fp32", "split"])
def test_batch_workload_frames_fp32(F, golden, precision):
    g, fr = golden
    idx = sorted(g)
    _say("batch workload frames", precision, idx)
    res = F.cluster_batch(_inputs([fr[i] for i in idx]), precision=F.FP32 if precision == "fp32" else F.BF16_SPLIT)
    for i, (modes, labels, st) in zip(idx, res):
        o, f = g[i], fr[i]
        fg = np.flatnonzero(f.mask.reshape(-1))
        mm = parity.match_modes(modes.cpu().numpy(), o["modes"])
        lc = parity.compare_labels_fg(labels.cpu().numpy(), fg, o["fg_labels"], o["band"], o["tie"], mm)
        print(f"frame {i} {f.spec.height}^2 h={f.bandwidth}: modes {len(modes)}/{len(o['modes'])} "
              f"max err {mm.max_error:.2e} labels {lc}")
        assert mm.unmatched_gpu == 0 and mm.unmatched_oracle == 0
        assert mm.max_error <= FP32_TOL
        assert lc.mismatched == 0
        np.testing.assert_array_equal(mm.pairs[:, 0], mm.pairs[:, 1])
        for k in ("rounds", "seeds_used", "iterations_total", "n_discarded", "n_state_out", "seed_pixel_updates"):
            assert st[k] == o["stats"][k], (i, k)
        np.testing.assert_array_equal(st["mode_counts"].cpu().numpy(), o["mode_counts"])


def test_batch_workload_frames_bf16(F, golden):
    g, fr = golden
    idx = sorted(g)
    _say("batch workload frames bf16", idx)
    inp = _inputs([fr[i] for i in idx])
    res = F.cluster_batch(inp, precision=F.BF16_REFINE)
    for i, x, (modes, labels, st) in zip(idx, inp, res):
        o, f = g[i], fr[i]
        fg = np.flatnonzero(f.mask.reshape(-1))
        mm = parity.match_modes(modes.cpu().numpy(), o["modes"])
        lab = labels.cpu().numpy()

        def labels_cmp(width, lost, match, o=o, fg=fg, lab=lab):
            tie = o["tie"] | parity.near_tie_mask(len(fg), o["near_idx"], o["near_gap"], width)
            return parity.compare_labels_fg(lab, fg, o["fg_labels"], o["band"], tie, match, lost)

        print(f"frame {i} {f.spec.height}^2 h={f.bandwidth}")
        parity.assert_bf16_bar(F, x["emb"], x["mask"], f.bandwidth, modes, labels_cmp, mm, o)


def test_batch_with_empty_frame(F, frames, oracles):
    _say("batch with an empty mask")
    res = F.cluster_batch(_inputs(frames, empty=(1,)), precision=F.FP32)
    modes, labels, st = res[1]
    assert len(modes) == 0
    assert int((labels != -1).sum().item()) == 0
    assert st["n_fg"] == 0
    for i in (0, 2, 3):
        mm = parity.match_modes(res[i][0].cpu().numpy(), oracles[i].modes)
        assert mm.unmatched_gpu == 0 and mm.unmatched_oracle == 0 and mm.max_error <= FP32_TOL


def test_batch_capacity_retry(F, frames, oracles):
    # k_max = 1 forces FMS_ERR_CAPACITY with the required total; the binding
    # grows the buffer and calls again.
    _say("batch capacity")
    res = F.cluster_batch(_inputs(frames), precision=F.FP32, k_max=1)
    assert [len(r[0]) for r in res] == [len(o.modes) for o in oracles]


def test_batch_of_one_is_the_single_frame_path(F, frames, oracles):
    _say("batch of one")
    (modes, labels, st), = F.cluster_batch(_inputs(frames[:1]), precision=F.FP32)
    mm = parity.match_modes(modes.cpu().numpy(), oracles[0].modes)
    assert mm.unmatched_gpu == 0 and mm.unmatched_oracle == 0 and mm.max_error <= FP32_TOL


def test_batch_nchw_layout(F, frames, oracles):
    import torch
    _say("batch nchw")
    inp = [{"emb": torch.from_numpy(f.emb).cuda().permute(2, 0, 1).contiguous(),
            "mask": torch.from_numpy(f.mask).cuda(), "bandwidth": f.bandwidth} for f in frames]
    res = F.cluster_batch(inp, layout="nchw", precision=F.FP32)
    for f, o, (modes, labels, st) in zip(frames, oracles, res):
        mm = parity.match_modes(modes.cpu().numpy(), o.modes)
        lc = parity.compare_labels(labels.cpu().numpy(), o, mm, 1.0 - f.bandwidth)
        assert mm.unmatched_gpu == 0 and mm.unmatched_oracle == 0 and mm.max_error <= FP32_TOL
        assert lc.mismatched == 0


def test_many_small_frames_equal_single_calls(F):
    # 96 small frames of 11 different shapes and seeds in one call (the grid's
    # frame dimension well beyond the CU count): every frame as its own call.
    import torch
    specs = [dataclasses.replace(synth.MID, height=24 + 4 * (k % 11), width=20 + 6 * (k % 7),
                                 n_cells=2 + k % 5, r_min=3, r_max=8, seed=100 + k) for k in range(96)]
    frames = [synth.make_frame(s) for s in specs]
    inp = [{"emb": torch.from_numpy(f.emb).cuda(), "mask": torch.from_numpy(f.mask).cuda(),
            "bandwidth": f.bandwidth} for f in frames]
    _say("96 small frames")
    res = F.cluster_batch(inp, precision=F.FP32)
    for x, (bm, bl, bst) in zip(inp, res):
        sm, sl, sst = F.cluster(x["emb"], x["mask"], x["bandwidth"], precision=F.FP32)
        assert bm.shape == sm.shape
        if len(sm):
            err = 1.0 - np.sum(bm.cpu().double().numpy() * sm.cpu().double().numpy(), axis=1)
            assert err.max() <= FP32_TOL
        assert int((bl != sl).sum().item()) == 0
        assert bst["rounds"] == sst["rounds"] and bst["seeds_used"] == sst["seeds_used"]
    # Every frame of the BF16 form gets modes and labels (the frames are too
    # many for oracle runs here; the bar is checked on the other batches).
    res = F.cluster_batch(inp, precision=F.BF16_REFINE)
    for f, (bm, bl, bst) in zip(frames, res):
        assert len(bm) >= 1 and bst["n_fg"] == f.n_fg
        assert int((bl >= 0).sum().item()) == f.n_fg


def test_batch_round_above_device_ranking_is_unsupported(F, frames):
    # A round of more than 16,384 seeds in one frame of a batch of two or
    # more frames (the device ranking's limit; single-frame calls prune such
    # rounds on the host) returns FMS_ERR_UNSUPPORTED.
    from tests.golden import make_host_prune as mhp
    from paper_2007_14283_amd import _binding as B
    big = synth.make_frame(mhp.SPEC)
    assert big.n_fg > 16384
    inp = _inputs([frames[0], big])
    inp[1]["n_state_in"] = 16385
    _say("batch round above 16384 seeds")
    with pytest.raises(F.FmsError) as ei:
        F.cluster_batch(inp, precision=F.FP32)
    assert ei.value.status == B.FMS_ERR_UNSUPPORTED
    # The handle still works afterwards.
    res = F.cluster_batch(_inputs(frames[:2]), precision=F.FP32)
    assert len(res) == 2 and len(res[0][0]) >= 1
