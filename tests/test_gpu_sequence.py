"""GPU parity of two further workloads against the FP64 oracle and closed forms:

* a drifting synthetic sequence with N carried from frame to frame (the
  online seed-count policy across frames, Sec. 3.2.4): every frame's modes,
  labels and round statistics, including the carried N, equal the oracle's
  chain;
* the Appendix A overlap workload (1000 x 1000, D = 18, eight noise-free
  discs of diameter 250, P = 0.95): the modes are exactly the disc vectors of
  the visible discs and every foreground pixel takes its disc."""
import numpy as np
import pytest

import synth
from oracle import cluster as C
from tests import parity

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def F():
    import paper_2007_14283_amd as fms
    fms.library()
    return fms


def test_carried_n_over_a_drifting_sequence(F):
    import torch
    seq = synth.drifting_sequence(synth.MID, 4)
    n_gpu = n_or = 0
    for t, f in enumerate(seq):
        _say("sequence frame", t, "N in", n_gpu)
        emb = torch.from_numpy(f.emb).cuda()
        mask = torch.from_numpy(f.mask).cuda()
        modes, labels, st = F.cluster(emb, mask, f.bandwidth, precision=F.FP32, n_state_in=n_gpu)
        res = C.cluster(f.emb, f.mask, C.Params(bandwidth=f.bandwidth, n_state_in=n_or))
        mm = parity.match_modes(modes.cpu().numpy(), res.modes)
        lc = parity.compare_labels(labels.cpu().numpy(), res, mm, 1.0 - f.bandwidth)
        assert mm.unmatched_gpu == 0 and mm.unmatched_oracle == 0 and mm.max_error <= 1e-5
        assert lc.mismatched == 0
        for k in ("rounds", "seeds_used", "n_state_out"):
            assert st[k] == res.stats[k], (t, k)
        n_gpu, n_or = st["n_state_out"], res.stats["n_state_out"]


@pytest.mark.parametrize("overlap", [0.0, 0.3])
@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_appendix_a_discs(F, overlap, precision):
    import torch
    emb, mask, owner, centres = synth.overlap_circles(overlap)
    _say("appendix A", overlap, precision, int(mask.sum()))
    prec = F.FP32 if precision == "fp32" else F.BF16_REFINE
    modes, labels, st = F.cluster(torch.from_numpy(emb).cuda(), torch.from_numpy(mask).cuda(), 0.1,
                                  precision=prec, p_target=0.95)
    visible = np.unique(owner[owner >= 0])
    m = modes.cpu().double().numpy()
    c = centres[visible] / np.linalg.norm(centres[visible], axis=1, keepdims=True)
    assert len(m) == len(visible)
    sim = m @ c.T
    best = np.argmax(sim, axis=1)
    assert sorted(best.tolist()) == list(range(len(visible)))
    assert np.max(1.0 - sim[np.arange(len(m)), best]) <= 1e-6
    # Every foreground pixel takes its own disc's mode; background stays -1.
    lab = labels.cpu().numpy()
    disc_of_mode = visible[best]
    fg = owner >= 0
    np.testing.assert_array_equal(disc_of_mode[lab[fg]], owner[fg])
    assert np.all(lab[~fg] == -1)
