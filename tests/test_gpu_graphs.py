"""Iteration batches captured into HIP graphs (fms_params.graphs) against the
same calls launched kernel by kernel.

A call is deterministic, so every output must be bit-identical: modes, mode
counts, labels and the statistics.  Each case replays the handle's cached
graphs several times, with eager calls (and their synchronisations) in
between, and checks every replay."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

STAT_KEYS = ("rounds", "seeds_used", "iterations_total", "n_discarded", "n_state_out", "seed_pixel_updates",
             "refine_steps", "refine_unconverged", "n_uncovered")


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def F():
    import paper_2007_14283_amd as fms
    fms.library()
    return fms


def _same(a, b):
    ma, la, sa = a
    mb, lb, sb = b
    assert ma.shape == mb.shape
    assert np.array_equal(ma.cpu().numpy().view(np.uint32), mb.cpu().numpy().view(np.uint32))
    assert np.array_equal(la.cpu().numpy(), lb.cpu().numpy())
    assert np.array_equal(sa["mode_counts"].cpu().numpy(), sb["mode_counts"].cpu().numpy())
    for k in STAT_KEYS:
        assert sa[k] == sb[k], k


@pytest.mark.parametrize("spec", [synth.MID, synth.PLAIN512])
@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_graph_replays_equal_eager_calls(F, spec, precision):
    import torch
    f = synth.make_frame(spec)
    emb = torch.from_numpy(f.emb).cuda()
    mask = torch.from_numpy(f.mask).cuda()
    prec = F.FP32 if precision == "fp32" else F.BF16_REFINE
    _say("graphs", spec.height, spec.width, precision)
    eager = F.cluster(emb, mask, f.bandwidth, precision=prec)
    for rep in range(3):
        got = F.cluster(emb, mask, f.bandwidth, precision=prec, graphs=1)
        torch.cuda.synchronize()
        _same(got, eager)
        _same(F.cluster(emb, mask, f.bandwidth, precision=prec), eager)


def test_graph_replays_equal_eager_batch(F):
    import torch
    specs = synth.batch_specs(6)
    frames = [synth.make_frame(sp) for sp in specs]
    inp = [{"emb": torch.from_numpy(q.emb).cuda(), "mask": torch.from_numpy(q.mask).cuda(),
            "bandwidth": q.bandwidth} for q in frames]
    _say("graphs batch", [sp.height for sp in specs])
    eager = F.cluster_batch(inp, precision=F.BF16_REFINE)
    for rep in range(2):
        got = F.cluster_batch(inp, precision=F.BF16_REFINE, graphs=1)
        torch.cuda.synchronize()
        for a, b in zip(got, eager):
            _same(a, b)
