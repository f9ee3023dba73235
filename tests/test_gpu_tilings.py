"""GPU parity of every compiled work decomposition of the fused step: each
(seeds per group, waves per group) the library accepts, for each D class and
precision, clusters a small frame to the same result as the FP64 oracle
(FP32: modes within 1e-5 and labels exact outside the exempt sets; BF16 +
FP32 replay: the BF16 bar of tests/parity.py), and rounds large enough to take
the wide seed groups by default do too."""
import pytest

import synth
from oracle import cluster as C
from tests import parity

pytestmark = pytest.mark.gpu

FP32_TOL = 1e-5
_ORACLE = {}


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def F():
    import paper_2007_14283_amd as fms
    fms.library()
    return fms


def _case(spec, **kw):
    key = (spec, tuple(sorted(kw.items())))
    if key not in _ORACLE:
        f = synth.make_frame(spec)
        _ORACLE[key] = (f, C.cluster(f.emb, f.mask, C.Params(bandwidth=f.bandwidth, **kw)))
    return _ORACLE[key]


def _check(F, f, res, prec, **kw):
    import torch
    emb = torch.from_numpy(f.emb).cuda()
    mask = torch.from_numpy(f.mask).cuda()
    modes, labels, st = F.cluster(emb, mask, f.bandwidth, precision=prec, **kw)
    mm = parity.match_modes(modes.cpu().numpy(), res.modes)
    if prec in (F.FP32, F.BF16_SPLIT):
        lc = parity.compare_labels(labels.cpu().numpy(), res, mm, 1.0 - f.bandwidth)
        assert mm.unmatched_gpu == 0 and mm.unmatched_oracle == 0, kw
        assert mm.max_error <= FP32_TOL, kw
        assert lc.mismatched == 0, kw
        assert st["rounds"] == res.stats["rounds"] and st["seeds_used"] == res.stats["seeds_used"], kw
    else:
        lab = labels.cpu().numpy()
        parity.assert_bf16_bar(F, emb, mask, f.bandwidth, modes, lambda w, lost, match: parity.compare_labels(
            lab, res, match, 1.0 - f.bandwidth, tie_width=w, lost_modes=lost), mm, parity.provenance_of(res),
            {k: v for k, v in kw.items() if k.startswith("tile_")})


def _prec(F, precision):
    return {"fp32": F.FP32, "bf16": F.BF16_REFINE, "split": F.BF16_SPLIT}[precision]


@pytest.mark.parametrize("dim", [32, 64, 128])
@pytest.mark.parametrize("precision", ["fp32", "bf16", "split"])
def test_every_decomposition(F, dim, precision):
    spec = synth.FrameSpec(64, 80, 8, 5, 12, dim, 0.02, 0.05, 11 + dim)
    f, res = _case(spec)
    prec = _prec(F, precision)
    for seeds in (16, 32, 64, 128):
        for waves in (4, 8, 16):
            for items in (256, 1024):
                _say("tiling", dim, precision, seeds, waves, items)
                _check(F, f, res, prec, tile_seeds=seeds, tile_waves=waves, tile_items=items)


@pytest.mark.parametrize("precision", ["fp32", "bf16", "split"])
def test_large_rounds_take_wide_groups(F, precision):
    # A first round of 4096 seeds: the default decomposition switches to
    # 64-seed (FP32, split BF16) and 128-seed (BF16) groups for these launches.
    f, res = _case(synth.MID, n_initial=4096)
    _say("wide groups", precision, f.n_fg)
    _check(F, f, res, _prec(F, precision), n_initial=4096)
