"""GPU parity on the 1024x1024, 300-cell, D = 32 precision workload against the
stored FP64 oracle result (tests/golden/precision1024_oracle.npz, written from
oracle/ alone and pinned in test_golden_precision1024.py).  FP32 form: the same
modes in the same order within 1e-5 (1 - cos), the same window counts and
round statistics, labels exact outside the exempt sets.  BF16 + FP32 replay:
the BF16 bar of tests/parity.py (modes within 1e-3, at most 2 % of the
oracle's modes lost and each traced to its seed through the stored round
seed lists, labels exact outside the exempt sets)."""
import numpy as np
import pytest

import synth
from tests import parity

pytestmark = pytest.mark.gpu

FP32_TOL = 1e-5
BF16_TOL = 1e-3


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def F():
    import paper_2007_14283_amd as fms
    fms.library()
    return fms


@pytest.fixture(scope="module")
def case():
    f = synth.make_frame(synth.PRECISION1024)
    g = parity.load_precision1024()
    fg = np.flatnonzero(f.mask.reshape(-1))
    return f, g, fg


def _run(F, f, prec):
    import torch
    emb = torch.from_numpy(f.emb).cuda()
    mask = torch.from_numpy(f.mask).cuda()
    return F.cluster(emb, mask, f.bandwidth, precision=prec)


@pytest.mark.parametrize("precision", ["fp32", "split"])
def test_precision1024_fp32(F, case, precision):
    f, g, fg = case
    _say("1024x1024", precision, f.n_fg)
    modes, labels, st = _run(F, f, F.FP32 if precision == "fp32" else F.BF16_SPLIT)
    mm = parity.match_modes(modes.cpu().numpy(), g["modes"])
    lc = parity.compare_labels_fg(labels.cpu().numpy(), fg, g["fg_labels"], g["band"], g["tie"], mm)
    print(f"modes {len(modes)}/{len(g['modes'])} max err {mm.max_error:.2e} labels {lc}")
    assert mm.unmatched_gpu == 0 and mm.unmatched_oracle == 0
    assert mm.max_error <= FP32_TOL
    np.testing.assert_array_equal(mm.pairs[:, 0], mm.pairs[:, 1])
    assert lc.mismatched == 0
    for k in ("rounds", "seeds_used", "iterations_total", "n_discarded", "n_state_out", "seed_pixel_updates"):
        assert st[k] == g["stats"][k], k
    np.testing.assert_array_equal(st["mode_counts"].cpu().numpy(), g["mode_counts"])


def test_precision1024_bf16_refine(F, case):
    import torch
    f, g, fg = case
    _say("1024x1024 bf16")
    modes, labels, st = _run(F, f, F.BF16_REFINE)
    mm = parity.match_modes(modes.cpu().numpy(), g["modes"])
    emb = torch.from_numpy(f.emb).cuda()
    mask = torch.from_numpy(f.mask).cuda()
    lab = labels.cpu().numpy()

    def labels_cmp(width, lost, match):
        tie = g["tie"] | parity.near_tie_mask(len(fg), g["near_idx"], g["near_gap"], width)
        return parity.compare_labels_fg(lab, fg, g["fg_labels"], g["band"], tie, match, lost)

    parity.assert_bf16_bar(F, emb, mask, f.bandwidth, modes, labels_cmp, mm, g)
    print(f"replay: steps {st['refine_steps']}, unconverged {st['refine_unconverged']}, "
          f"step diff {st['refine_step_diff']}")
