"""Pins of the stored oracle results of the uneven batching workload
(tests/golden/batch_oracle.npz, five frames) and of the 20,000-seed frame
(tests/golden/host_prune_oracle.npz) against their frames, without re-running
the oracle (CPU only).  Each stored result must be one the method can return:
every mode a fixed point of the FP64 step (Eq. 8, 10, 11) up to the stopping
rule of Sec. 3.2.1, modes outside each other's window (the pruning of
Alg. 2), labels the FP64 argmax over the modes (Alg. 2) outside the stored
exempt sets, window counts recomputed, and the per-mode provenance (round,
seed, step count) consistent with the seed lists and the statistics."""
import numpy as np
import pytest

import synth
from oracle import meanshift as ms
from tests import parity


def _x(frame):
    fg = np.flatnonzero(frame.mask.reshape(-1))
    e = frame.emb.reshape(-1, frame.emb.shape[-1])[fg].astype(np.float64)
    return e / np.linalg.norm(e, axis=1, keepdims=True)


def _pin(frame, g):
    x = _x(frame)
    m = g["modes"]
    h = g["bandwidth"]
    thr, tol = 1.0 - h, h / 1000
    assert h == frame.bandwidth
    assert len(x) == g["stats"]["n_fg"] == len(g["fg_labels"])
    assert len(m) == len(g["mode_counts"]) >= 1
    # Fixed points up to the stopping rule: a seed stops once its last move is
    # below tol, so one more step may still move it a little.
    _, delta, _ = ms.shift(m, x, thr)
    assert np.sum(delta >= tol) <= max(1, int(0.02 * len(m)))
    assert np.all(delta < 10 * tol)
    s = m @ m.T
    np.fill_diagonal(s, -1.0)
    assert np.all(s < thr)
    lab = np.empty(len(x), np.int64)
    counts = np.zeros(len(m), np.int64)
    for i0 in range(0, len(x), 65536):
        sx = x[i0:i0 + 65536] @ m.T
        lab[i0:i0 + 65536] = np.argmax(sx, axis=1)
        counts += np.sum(sx >= thr, axis=0)
    exempt = g["band"] | g["tie"]
    assert np.array_equal(lab[~exempt], g["fg_labels"][~exempt])
    assert np.array_equal(counts, g["mode_counts"])
    return x


@pytest.fixture(scope="module")
def batch():
    g = parity.load_batch_oracle()
    specs = synth.batch_specs(64)
    return g, {i: synth.make_frame(specs[i]) for i in g}


def test_batch_frames_cover_the_sizes(batch):
    g, fr = batch
    assert sorted({fr[i].spec.height for i in g}) == [512, 768, 1024]
    assert len({g[i]["bandwidth"] for i in g}) >= 3


@pytest.mark.parametrize("i", [1, 2, 3, 10, 15])
def test_batch_frame_result(batch, i):
    g, fr = batch
    o = g[i]
    x = _pin(fr[i], o)
    # Provenance: every mode's seed belongs to its round's list, the rounds'
    # lists add up to the seeds used, and the stored near-tie gaps are the
    # best-minus-second similarities.
    assert sum(len(r) for r in o["round_seeds"]) == o["stats"]["seeds_used"]
    assert len(o["round_seeds"]) == o["stats"]["rounds"]
    assert len(o["mode_round"]) == len(o["modes"])
    for k in range(len(o["modes"])):
        r, a = int(o["mode_round"][k]), int(o["mode_local"][k])
        assert 0 <= a < len(o["round_seeds"][r]) and 1 <= o["mode_iters"][k] <= 100
    assert np.all(np.diff(o["mode_round"]) >= 0)
    idx = o["near_idx"][:200]
    sx = np.sort(x[idx] @ o["modes"].T, axis=1)
    np.testing.assert_allclose(sx[:, -1] - sx[:, -2], o["near_gap"][:200], atol=1e-6)


def test_mode_seeds_reach_their_modes(batch):
    # One FP64 trajectory per stored mode, from its seed, for its stored step
    # count (Alg. 1's step for one point): it ends on the mode.  Frame 10.
    g, fr = batch
    o = g[10]
    x = _x(fr[10])
    thr = 1.0 - o["bandwidth"]
    for k in range(0, len(o["modes"]), 7):
        r, a = int(o["mode_round"][k]), int(o["mode_local"][k])
        y = x[int(o["round_seeds"][r][a])][None, :]
        for _ in range(int(o["mode_iters"][k])):
            y, _, _ = ms.shift(y, x, thr)
        assert 1.0 - float(y[0] @ o["modes"][k]) < 1e-12


def test_host_prune_result():
    from tests.golden import make_host_prune as mhp
    g = parity.load_host_prune()
    f = synth.make_frame(mhp.SPEC)
    _pin(f, g)
    assert g["n_state_in"] == 20000 and g["stats"]["seeds_used"] == 20000 and g["stats"]["rounds"] == 1
