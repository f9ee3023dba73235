"""GPU parity on the 1024x1024, 300-cell, D = 32 precision workload against the
stored FP64 oracle result (tests/golden/precision1024_oracle.npz, written from
oracle/ alone and pinned in test_golden_precision1024.py).  FP32 form: the same
modes in the same order within 1e-5 (1 - cos), the same window counts and
round statistics, labels exact outside the exempt sets.  BF16 + FP32 refine:
every mode an FP64 fixed point up to the stopping rule (as the oracle's own
modes, 99 % within tol = h/1000, all within 10 tol) and >= 90 % of the
oracle's modes within 1e-3."""
import numpy as np
import pytest

import synth
from oracle import meanshift as ms
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


def test_precision1024_fp32(F, case):
    f, g, fg = case
    _say("1024x1024 fp32", f.n_fg)
    modes, labels, st = _run(F, f, F.FP32)
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
    f, g, fg = case
    _say("1024x1024 bf16")
    modes, labels, st = _run(F, f, F.BF16_REFINE)
    mm = parity.match_modes(modes.cpu().numpy(), g["modes"])
    e = f.emb.reshape(-1, f.emb.shape[-1])[fg].astype(np.float64)
    x = e / np.linalg.norm(e, axis=1, keepdims=True)
    m = modes.cpu().double().numpy()
    m = m / np.linalg.norm(m, axis=1, keepdims=True)
    tol = f.bandwidth / 1000
    _, resid, _ = ms.shift(m, x, 1.0 - f.bandwidth)
    within = int(np.sum(mm.errors <= BF16_TOL))
    print(f"bf16: {len(m)} modes, {within}/{len(g['modes'])} oracle modes within 1e-3, "
          f"max err {mm.max_error:.2e}, max residual {resid.max():.2e}")
    assert np.mean(resid < tol) >= 0.99 and np.all(resid < 10 * tol)
    assert within >= 0.9 * len(g["modes"])
