"""Pins of the oracle's unrolled mean shift and its gradient (oracle/unroll.py),
checked against FP64 central finite differences and closed-form properties.
CPU only."""
import numpy as np
import pytest

from oracle import meanshift as ms
from oracle import unroll as U


def _clusters(seed, n_per=20, k=3, dim=5, spread=0.15):
    rng = np.random.default_rng(seed)
    centres = rng.normal(size=(k, dim))
    pts = np.concatenate([c + spread * rng.normal(size=(n_per, dim)) for c in centres])
    scale = rng.uniform(0.5, 2.0, size=(len(pts), 1))  # raw rows: not unit length
    return pts * scale


def _case(min_margin=1e-4, h=0.3, steps=3, seeds=(0, 7, 21, 33, 50)):
    # A seeded small problem whose similarities stay clear of the threshold at
    # every step, so finite differences cannot flip a window membership.
    for seed in range(200):
        e = _clusters(seed)
        seeds = np.array(seeds)
        _, _, _, margin = U.forward(e, seeds, h, steps)
        if margin > min_margin:
            return e, seeds, h, steps
    raise AssertionError("no case with a clear margin")


def _fd(e, seeds, h, steps, targets, eps=1e-7):
    g = np.zeros_like(e)
    for i in range(e.shape[0]):
        for d in range(e.shape[1]):
            ep = e.copy()
            em = e.copy()
            ep[i, d] += eps
            em[i, d] -= eps
            g[i, d] = (U.loss(ep, seeds, h, steps, targets) - U.loss(em, seeds, h, steps, targets)) / (2 * eps)
    return g


def test_forward_is_the_plain_step_repeated():
    e, seeds, h, steps = _case()
    x = e / np.linalg.norm(e, axis=1, keepdims=True)
    y = x[seeds]
    for _ in range(steps):
        y, _, _ = ms.shift(y, x, 1.0 - h)
    got, _, _, _ = U.forward(e, seeds, h, steps)
    np.testing.assert_allclose(got, y, atol=1e-15)


def test_gradient_matches_finite_differences():
    e, seeds, h, steps = _case()
    rng = np.random.default_rng(1)
    targets = rng.normal(size=(len(seeds), e.shape[1]))
    targets /= np.linalg.norm(targets, axis=1, keepdims=True)
    ga = U.grad(e, seeds, h, steps, targets)
    gf = _fd(e, seeds, h, steps, targets)
    assert np.max(np.abs(gf)) > 1e-3  # a non-trivial gradient
    np.testing.assert_allclose(ga, gf, atol=1e-7, rtol=1e-6)


def test_gradient_is_orthogonal_to_each_row_and_scales_inversely():
    e, seeds, h, steps = _case()
    g = np.ones((len(seeds), e.shape[1]))
    ga = U.grad(e, seeds, h, steps, g)
    np.testing.assert_allclose(np.sum(ga * e, axis=1), 0.0, atol=1e-12)
    ga2 = U.grad(2.0 * e, seeds, h, steps, g)
    np.testing.assert_allclose(ga2, ga / 2.0, atol=1e-14)


def test_rows_outside_every_last_window_get_no_gradient():
    # Seeds in two of the three clusters: the third cluster's rows are in no
    # window.
    e, seeds, h, steps = _case(seeds=(0, 7, 21, 33))
    x = e / np.linalg.norm(e, axis=1, keepdims=True)
    _, y_prev, _, _ = U.forward(e, seeds, h, steps)
    member = np.any(y_prev @ x.T >= 1.0 - h, axis=0)
    assert (~member).any() and member.any()
    ga = U.grad(e, seeds, h, steps, np.ones((len(seeds), e.shape[1])))
    assert np.all(ga[~member] == 0.0)
    assert np.all(np.linalg.norm(ga[member], axis=1) > 0.0)


def test_single_step_closed_form():
    # One seed, one step: y = normalize(sum of the members of its window), and
    # dL/de_i for a member i is (I - x x^T)(I - y y^T) g / (|V| |e_i|).
    e, seeds, h, _ = _case(steps=1)
    s0 = seeds[:1]
    x = e / np.linalg.norm(e, axis=1, keepdims=True)
    w = (x[s0] @ x.T >= 1.0 - h)[0]
    v = x[w].sum(axis=0)
    y = v / np.linalg.norm(v)
    g = np.arange(1.0, e.shape[1] + 1.0)[None, :]
    gv = (g[0] - (g[0] @ y) * y) / np.linalg.norm(v)
    want = np.zeros_like(e)
    for i in np.nonzero(w)[0]:
        want[i] = (gv - (gv @ x[i]) * x[i]) / np.linalg.norm(e[i])
    np.testing.assert_allclose(U.grad(e, s0, h, 1, g), want, atol=1e-14)


def test_planted_mistake_is_caught():
    # Dropping the projection of the renormalisation must break the
    # finite-difference agreement.
    e, seeds, h, steps = _case()
    rng = np.random.default_rng(2)
    targets = rng.normal(size=(len(seeds), e.shape[1]))
    x = e / np.linalg.norm(e, axis=1, keepdims=True)
    y, y_prev, vnorm, _ = U.forward(e, seeds, h, steps)
    gv_wrong = targets / vnorm[:, None]
    w = (y_prev @ x.T >= 1.0 - h).astype(float)
    gx = w.T @ gv_wrong
    wrong = (gx - np.sum(gx * x, axis=1, keepdims=True) * x) / np.linalg.norm(e, axis=1, keepdims=True)
    gf = _fd(e, seeds, h, steps, targets)
    assert np.max(np.abs(wrong - gf)) > 1e-3


def test_steps_must_be_positive():
    e, seeds, h, _ = _case()
    with pytest.raises(ValueError):
        U.forward(e, seeds, h, 0)


def crop_case(size=64):
    """The differentiation workload's finite-difference crop: the size x size
    window (on a grid of size) with the most foreground of the 512x512, D = 32
    frame; 128 seeds from the seed order, T = 10 steps.  Seeds whose FP64
    trajectory comes within 1e-5 of a window edge get a zero target (a
    perturbation could flip one of their memberships)."""
    import synth
    from oracle import seed_order as so
    frame = synth.make_frame(synth.PLAIN512)
    best = None
    for y0 in range(0, frame.spec.height - size + 1, size):
        for x0 in range(0, frame.spec.width - size + 1, size):
            c = int(frame.mask[y0:y0 + size, x0:x0 + size].sum())
            if best is None or c > best[0]:
                best = (c, y0, x0)
    _, y0, x0 = best
    emb = frame.emb[y0:y0 + size, x0:x0 + size].reshape(-1, frame.emb.shape[-1])
    mask = frame.mask[y0:y0 + size, x0:x0 + size].reshape(-1)
    e = emb[mask != 0].astype(np.float64)
    h, steps = frame.bandwidth, 10
    seeds = so.seed_order(len(e), 0)[:128].astype(np.int64)
    x = e / np.linalg.norm(e, axis=1, keepdims=True)
    y = x[seeds]
    marg = np.full(len(seeds), np.inf)
    for _ in range(steps):
        s = y @ x.T
        marg = np.minimum(marg, np.min(np.abs(s - (1.0 - h)), axis=1))
        v = (s >= 1.0 - h).astype(np.float64) @ x
        y = v / np.linalg.norm(v, axis=1, keepdims=True)
    rng = np.random.default_rng(0)
    targets = rng.normal(size=(len(seeds), e.shape[1]))
    targets /= np.linalg.norm(targets, axis=1, keepdims=True)
    targets[marg < 1e-5] = 0.0
    coords = np.stack([rng.integers(0, len(e), 200), rng.integers(0, e.shape[1], 200)], axis=1)
    return e, seeds, h, steps, targets, coords


def fd_at(e, seeds, h, steps, targets, coords, eps=1e-6):
    """FP64 central differences of L = sum_j y_T,j . target_j at the given
    (row, dimension) coordinates of the raw embeddings.  With |L| ~ 10 the
    rounding of the quotient is about 1e-16 |L| / eps ~ 1e-9; the kept seeds
    sit at least 1e-5 from every window edge, ten times the perturbation."""
    out = np.empty(len(coords))
    for k, (i, d) in enumerate(coords):
        ep = e.copy()
        em = e.copy()
        ep[i, d] += eps
        em[i, d] -= eps
        out[k] = (U.loss(ep, seeds, h, steps, targets) - U.loss(em, seeds, h, steps, targets)) / (2 * eps)
    return out


def test_gradient_matches_finite_differences_on_the_crop():
    # The differentiation workload at its own size (64 x 64 crop of the
    # 512 x 512, D = 32 frame, 128 seeds, T = 10): the oracle gradient equals
    # FP64 central differences at 200 sampled coordinates.
    e, seeds, h, steps, targets, coords = crop_case()
    assert np.count_nonzero(np.any(targets != 0, axis=1)) >= 100
    ga = U.grad(e, seeds, h, steps, targets)
    gf = fd_at(e, seeds, h, steps, targets, coords)
    got = ga[coords[:, 0], coords[:, 1]]
    assert np.count_nonzero(np.abs(gf) > 1e-3) >= 20  # many non-trivial entries
    np.testing.assert_allclose(got, gf, atol=1e-8, rtol=1e-5)


def test_stored_finite_differences_match_the_oracle_gradient():
    # tests/golden/unroll_fd.npz (the GPU test's reference) holds the crop
    # case's seeds, targets and coordinates and FP64 differences that equal
    # the oracle gradient there.
    import os
    z = np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "unroll_fd.npz"))
    e, seeds, h, steps, targets, coords = crop_case()
    np.testing.assert_array_equal(z["seeds"], seeds)
    np.testing.assert_array_equal(z["coords"], coords)
    np.testing.assert_array_equal(z["targets"], targets)
    assert float(z["bandwidth"]) == h and int(z["steps"]) == steps
    ga = U.grad(e, seeds, h, steps, targets)
    np.testing.assert_allclose(ga[coords[:, 0], coords[:, 1]], z["fd"], atol=1e-8, rtol=1e-5)
