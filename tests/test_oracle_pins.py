"""Pins for the FP64 oracle: each test ties the oracle to something other than
itself (published values, closed forms, invariants, brute force, special
cases), chosen so that a dropped term, a wrong sign or index, or a transposed
operand fails at least one of them."""
import math
import os

import numpy as np
import pytest

import synth
from oracle import cluster as C
from oracle import meanshift as ms
from oracle import osop
from oracle import seed_order as so

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _unit(v):
    v = np.asarray(v, np.float64)
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


# ---------------------------------------------------------------- seed order

def test_splitmix64_published_outputs():
    with open(os.path.join(GOLDEN, "splitmix64.txt")) as fh:
        rows = [ln.split() for ln in fh if ln.strip() and not ln.startswith("#")]
    assert rows
    for r in rows:
        seed, outs = int(r[0]), [int(v) for v in r[1:]]
        assert so.splitmix64_stream(seed, len(outs)) == outs


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 7, 16, 17, 255, 256, 257, 1000, 4097])
def test_seed_order_is_a_permutation(n):
    p = so.seed_order(n, 12345)
    assert sorted(p.tolist()) == list(range(n))


def test_seed_order_vectorised_matches_scalar_definition():
    for n in (1, 9, 100, 513):
        p = so.seed_order(n, 99)
        assert all(int(p[j]) == so.position_to_ordinal(j, n, 99) for j in range(n))


def test_feistel_round_is_invertible():
    # A Feistel network is a bijection whatever the round function: undo the
    # rounds in reverse order and get the input back.
    keys = so.splitmix64_stream(5, so.ROUNDS)
    b = 6
    mask = (1 << b) - 1
    for x in range(1 << (2 * b)):
        y = so.feistel_encrypt(x, b, keys)
        left, right = y >> b, y & mask
        for key in reversed(keys):
            left, right = right ^ (so.mix64(left ^ key) & mask), left
        assert (left << b) | right == x


def test_seed_order_depends_on_seed_and_is_spread():
    n = 1000
    firsts = [int(so.seed_order(n, s)[0]) for s in range(400)]
    assert len(set(firsts)) > 300          # distinct first picks across seeds
    hist = np.bincount(np.array(firsts) * 4 // n, minlength=4)
    assert hist.min() > 60                  # roughly even over the frame


# ---------------------------------------------------------------- OSOP closed forms

def test_eq14_at_paper_circle_example():
    # Sec. 4.1 Results: 64 seeds sufficed for the 10-cluster circle data
    # (no background, r = 1), matching the theoretical curve of Eq. 14.
    p64 = osop.p_all_seeded(64, 10, 1.0)
    assert 0.98 < p64 < 0.995
    nm = osop.n_min(0.99, 10, 1.0)
    assert 64 < nm < 70


@pytest.mark.parametrize("p,i,r", [(0.99, 10, 1.0), (0.99, 20, 0.3), (0.99, 100, 0.4),
                                   (0.99, 300, 0.4), (0.95, 8, 0.39), (0.5, 3, 0.2)])
def test_eq19_inverts_eq14(p, i, r):
    nm = osop.n_min(p, i, r)
    assert osop.p_all_seeded(nm, i, r) == pytest.approx(p, rel=1e-12)
    assert osop.p_all_seeded(math.floor(nm), i, r) < p <= osop.p_all_seeded(math.ceil(nm), i, r)


@pytest.mark.parametrize("p,i,r,want", [(0.99, 10, 1.0, 65.52), (0.99, 20, 0.3, 502.60),
                                        (0.99, 100, 0.4, 2296.74), (0.99, 300, 0.4, 7722.81),
                                        (0.95, 8, 0.39, 101.10)])
def test_eq19_values(p, i, r, want):
    # Eq. 19 worked out separately (to two decimals) for the circle data of
    # Sec. 4.1 (I = 10, r = 1), the workloads of this hot path (I = 20, 100,
    # 300 at 30-40 % foreground) and the Appendix A setting (P = 0.95, I = 8).
    assert osop.n_min(p, i, r) == pytest.approx(want, abs=1e-2)


def test_eq15_chain_equals_eq19_at_half():
    # Eq. 15-18 solve (1 - (1 - 1/(2I))^N)^I = P for N; solve it by bisection
    # and compare with Eq. 19 at r = 1/2.
    for p, i in ((0.99, 10), (0.95, 8), (0.9, 50)):
        lo, hi = 0.0, 1e7
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if (1 - (1 - 1 / (2 * i)) ** mid) ** i < p:
                lo = mid
            else:
                hi = mid
        assert osop.n_min(p, i, 0.5) == pytest.approx(hi, rel=1e-9)
        assert osop.p_upper_half(hi, i) == pytest.approx(p, rel=1e-9)


def _exact_all_seeded(n, i, r):
    # Inclusion-exclusion over the multinomial draw of n seeds into i equal
    # instances (probability r / i each) plus background.
    return sum((-1) ** j * math.comb(i, j) * (1 - j * r / i) ** n for j in range(i + 1))


def test_eq14_is_the_independence_upper_bound():
    # The "instance k is seeded" events are negatively associated, so Eq. 14
    # (their product) bounds the exact probability from above (Sec. 3.2.2 calls
    # it an upper bound); for a single instance it is exact.
    for n, i, r in ((10, 5, 0.6), (40, 8, 0.4), (200, 20, 0.3), (64, 10, 1.0)):
        assert _exact_all_seeded(n, i, r) <= osop.p_all_seeded(n, i, r) + 1e-15
    for n, r in ((3, 0.2), (10, 0.5)):
        assert osop.p_all_seeded(n, 1, r) == pytest.approx(1 - (1 - r) ** n, rel=1e-14)


def test_eq14_exact_probability_by_monte_carlo():
    rng = np.random.Generator(np.random.PCG64(7))
    n, i, r, trials = 12, 4, 0.6, 40000
    probs = np.r_[np.full(i, r / i), 1 - r]
    draws = rng.multinomial(n, probs, size=trials)
    est = np.mean(np.all(draws[:, :i] > 0, axis=1))
    exact = _exact_all_seeded(n, i, r)
    assert abs(est - exact) < 4 * math.sqrt(exact * (1 - exact) / trials)
    assert exact < osop.p_all_seeded(n, i, r)


def test_controller_transitions():
    # Sec. 3.2.4: double while N < L N_min; next frame N - N_min when N > H N_min.
    assert osop.wants_more_seeds(128, 100.0, 2.0)
    assert not osop.wants_more_seeds(200, 100.0, 2.0)
    assert not osop.wants_more_seeds(256, 100.0, 2.0)
    assert osop.wants_more_seeds(128, None, 2.0)
    assert osop.next_frame_seeds(1000, 100.0, 8.0) == 900
    assert osop.next_frame_seeds(800, 100.0, 8.0) == 800
    assert osop.next_frame_seeds(1000, 100.2, 8.0) == 899
    assert osop.next_frame_seeds(128, None, 8.0) == 128
    assert osop.n_min(0.99, 0, 0.3) is None
    assert osop.n_min(0.99, 2, 0.9) < osop.n_min(0.99, 3, 0.9)
    assert osop.n_min(0.99, 1, 1.0) == 1.0


# ---------------------------------------------------------------- mean-shift step

def _clustered(rng, k, per, dim, noise):
    centres = np.eye(dim)[:k]
    x = np.repeat(centres, per, axis=0) + noise * rng.standard_normal((k * per, dim))
    return _unit(x), np.repeat(np.arange(k), per)


def _margin_ok(x, ends, thr, margin=1e-9):
    for y in (x, ends):
        if np.min(np.abs(y @ x.T - thr)) < margin:
            return False
    return True


@pytest.mark.parametrize("dim", [2, 3, 16])
def test_iterate_matches_alg1_brute_force(dim):
    # Random unit rows: the two sides sum the window members in different
    # orders, so their centres may differ in the last bits (the bit-exact
    # comparison is test_iterate_matches_alg1_bit_exact).
    rng = np.random.Generator(np.random.PCG64(dim))
    thr, tol = 0.9, 1e-4
    for _ in range(20):
        if dim == 2:
            ang = np.r_[rng.normal(0.0, 0.15, 20), rng.normal(1.6, 0.15, 20)]
            x = np.stack([np.cos(ang), np.sin(ang)], 1)
        else:
            x, _lab = _clustered(rng, 3, 14, dim, 0.25)
        ends, its = ms.classic(x, thr, tol, 100)
        if _margin_ok(x, ends, thr):
            break
    it = ms.iterate(x, np.arange(len(x)), thr, tol, 1.0, 100)
    assert it["converged"].all()
    np.testing.assert_allclose(it["endpoints"], ends, rtol=0, atol=1e-12)
    np.testing.assert_array_equal(it["iters"], its)


def _dyadic_clusters(seed=0, k=3, per=14, dim=16):
    # Unit rows whose entries are all +-1/4 (dim = 16): a base sign pattern per
    # cluster with 0-4 signs flipped.  Any sum of such rows, and the sum of the
    # squares of its entries, is exact in FP64 whatever the order, so Alg. 1's
    # Python loops and the matrix products of the parallel iteration form the
    # same window sums bit for bit, and a correctly rounded square root and
    # division then give the same centres.
    rng = np.random.default_rng(seed)
    base = rng.choice([-0.25, 0.25], size=(k, dim))
    rows = []
    for b in base:
        for _ in range(per):
            v = b.copy()
            v[rng.choice(dim, rng.integers(0, 5), replace=False)] *= -1
            rows.append(v)
    return np.array(rows)


DYADIC_THR, DYADIC_TOL = 0.6, 1e-4


def test_iterate_matches_alg1_bit_exact():
    # Every vector a seed (Alg. 1) against the parallel iteration of Alg. 2 on
    # the same starts: identical endpoints and step counts, bit for bit.
    x = _dyadic_clusters()
    ends, its = ms.classic(x, DYADIC_THR, DYADIC_TOL, 100)
    assert its.max() >= 5 and len(set(its.tolist())) >= 4  # non-trivial trajectories
    it = ms.iterate(x, np.arange(len(x)), DYADIC_THR, DYADIC_TOL, 1.0, 100)
    assert it["converged"].all()
    np.testing.assert_array_equal(it["endpoints"], ends)
    np.testing.assert_array_equal(it["iters"], its)


def test_gamma_stop_is_strict():
    # Sec. 3.2.3 stops a round once MORE than gamma of its seeds have
    # converged.  Pick seeds so that exactly gamma * m of them converge first
    # (Alg. 1 gives each start's step count): the round must go on until the
    # slow one converges too, with Alg. 1's endpoints; one step earlier would
    # discard it.
    x = _dyadic_clusters()
    ends, its = ms.classic(x, DYADIC_THR, DYADIC_TOL, 100)
    fast = np.flatnonzero(its == 3)[:9]
    slow = np.flatnonzero(its >= 6)[:1]
    assert len(fast) == 9 and len(slow) == 1
    for seeds, gamma in ((np.r_[fast[:1], slow], 0.5), (np.r_[fast, slow], 0.9)):
        it = ms.iterate(x, seeds, DYADIC_THR, DYADIC_TOL, gamma, 100)
        assert it["converged"].all(), (gamma, it["iters"])
        assert it["steps"] == its[slow[0]]
        np.testing.assert_array_equal(it["iters"], its[seeds])
        np.testing.assert_array_equal(it["endpoints"], ends[seeds])
    # Just past the boundary the stop does come: 9 of 10 converged with
    # gamma < 0.9 ends the round after the fast seeds' last step.
    it = ms.iterate(x, np.r_[fast, slow], DYADIC_THR, DYADIC_TOL, 0.89, 100)
    assert it["steps"] == 3 and it["converged"].sum() == 9


def test_window_counts_brute_force():
    rng = np.random.Generator(np.random.PCG64(1))
    x = _unit(rng.standard_normal((50, 4)))
    y = _unit(rng.standard_normal((7, 4)))
    thr = 0.3
    brute = [sum(1 for p in x if sum(a * b for a, b in zip(q, p)) >= thr) for q in y]
    np.testing.assert_array_equal(ms.window_counts(y, x, thr), brute)


def test_flat_kernel_boundary_is_inclusive():
    # Eq. 11: k_h = 1 when d <= h.  x1 sits exactly at cosine 0.5 from the
    # seed (d = h = 0.5 exactly in binary), so it is a member.
    x = np.array([[1.0, 0.0], [0.5, math.sqrt(0.75)], [0.0, 1.0]])
    yn, delta, members = ms.shift(x[:1], x, 0.5)
    assert members[0] == 2
    np.testing.assert_allclose(yn[0], _unit(x[0] + x[1]), atol=1e-15)


def test_coverage_boundary_is_inclusive():
    # A pixel is covered when it lies inside a mode's window, boundary
    # included (Eq. 11's d <= h).  With the mode (1, 0) the similarity is the
    # first coordinate exactly: 0.5 = 1 - h is covered, 0.5 - 2^-40 is not.
    modes = np.array([[1.0, 0.0]])
    a = 0.5 - 2.0 ** -40
    x = np.array([[0.5, math.sqrt(0.75)], [a, math.sqrt(1.0 - a * a)], [1.0, 0.0], [0.0, 1.0]])
    assert ms.covered_by(x, modes, 0.5).tolist() == [True, False, True, False]
    assert ms.covered_by(x, np.zeros((0, 2)), 0.5).tolist() == [False] * 4


def test_later_round_seeds_skip_covered_pixels():
    # The policy seeds only pixels that are neither used nor within h of a
    # mode found in an earlier round: every round after the first takes the
    # first such positions of the seed order.  Coverage is recomputed here
    # from the modes the earlier rounds accepted, and it must have skipped
    # positions (it changes the seeds).
    f = synth.make_frame(synth.TINY)
    res = C.cluster(f.emb, f.mask, C.Params(bandwidth=f.bandwidth))
    assert len(res.rounds) >= 2
    thr = 1.0 - f.bandwidth
    order = so.seed_order(f.n_fg, 0)
    used = np.zeros(f.n_fg, bool)
    covered = np.zeros(f.n_fg, bool)
    skipped_by_cover = 0
    for rnd in res.rounds:
        want = len(rnd.positions)
        ok = ~used[order] & ~covered[order]
        expect = np.flatnonzero(ok)[:want]
        np.testing.assert_array_equal(rnd.positions, expect)
        skipped_by_cover += int(np.count_nonzero(covered[order[:expect[-1] + 1]] & ~used[order[:expect[-1] + 1]]))
        used[rnd.seeds] = True
        for a in rnd.accepted:
            m = rnd.endpoints[a]
            covered |= np.einsum("nd,d->n", res.x, m) >= thr
    assert skipped_by_cover > 0


def test_tight_clusters_closed_form():
    # Separated tight clusters: every within-cluster similarity is above 1-h and
    # every cross one far below, so each mode is the normalised cluster sum,
    # reached in one jump and confirmed in the next step, and labels are the
    # cluster ids.
    rng = np.random.Generator(np.random.PCG64(3))
    x, lab = _clustered(rng, 5, 40, 8, 0.03)
    res = C.cluster(x.astype(np.float64), None, C.Params(bandwidth=0.1, n_initial=64))
    assert len(res.modes) == 5
    want = np.stack([_unit(x[lab == k].sum(0)) for k in range(5)])
    match = np.argmax(res.modes @ want.T, axis=1)
    assert sorted(match.tolist()) == list(range(5))
    np.testing.assert_allclose(res.modes, want[match], atol=1e-14)
    for rnd in res.rounds:
        assert set(rnd.iters.tolist()) == {2}
    np.testing.assert_array_equal(match[res.labels], lab)


def test_positive_row_scale_leaves_result_bit_identical():
    f = synth.make_frame(synth.TINY)
    rng = np.random.Generator(np.random.PCG64(11))
    scale = np.ldexp(1.0, rng.integers(-6, 7, f.emb.shape[:2]))[..., None]
    p = C.Params(bandwidth=f.bandwidth)
    a = C.cluster(f.emb.astype(np.float64), f.mask, p)
    b = C.cluster(f.emb.astype(np.float64) * scale, f.mask, p)
    np.testing.assert_array_equal(a.modes, b.modes)
    np.testing.assert_array_equal(a.labels, b.labels)


def test_symmetric_arc_mode_on_the_circle():
    # D = 2: points placed symmetrically about angle phi have their window mean
    # on the ray at phi (Sec. 4.1 circle data); windows are arcs of half-width
    # arccos(1 - h).
    phi, psi = 0.7, 0.7 + math.pi / 2
    ks = np.arange(-6, 7)
    pts = [(math.cos(a), math.sin(a)) for a in np.r_[phi + 0.02 * ks, psi + 0.03 * ks]]
    res = C.cluster(np.array(pts), None, C.Params(bandwidth=0.1, n_initial=16))
    ang = sorted(math.atan2(m[1], m[0]) for m in res.modes)
    assert len(ang) == 2
    assert ang[0] == pytest.approx(phi, abs=1e-14)
    assert ang[1] == pytest.approx(psi, abs=1e-14)


def test_circle_simulation_finds_ten_clusters():
    pts, lab = synth.circle_points(0)
    res = C.cluster(pts, None, C.Params(bandwidth=0.1, n_initial=64))
    assert len(res.modes) == 10
    fgl = res.labels
    for k in range(10):
        assert len(set(fgl[lab == k].tolist())) == 1
    assert res.stats["n_min"] == pytest.approx(osop.n_min(0.99, 10, 1.0))


def test_prune_order_and_suppression():
    e = _unit(np.array([[1.0, 0.0], [1.0, 0.01], [0.0, 1.0], [0.01, 1.0]]))
    counts = np.array([10, 10, 5, 7])
    positions = np.array([3, 1, 0, 2])
    # Visit order: (10, pos 1) -> idx 1, (10, pos 3) -> idx 0, 7 -> idx 3, 5 -> idx 2.
    assert ms.prune(e, counts, positions, np.zeros((0, 2)), 0.9) == [1, 3]
    # An existing mode blocks its neighbours.
    assert ms.prune(e, counts, positions, np.array([[0.0, 1.0]]), 0.9) == [1]


def test_assign_ties_go_to_lowest_mode():
    m = np.array([[0.0, 1.0], [1.0, 0.0], [1.0, 0.0]])
    x = np.array([[1.0, 0.0], [0.0, 1.0], [math.sqrt(0.5), math.sqrt(0.5)]])
    lab, best, second = ms.assign(x, m)
    assert lab.tolist() == [1, 0, 0]
    assert best[0] == 1.0 and second[0] == 1.0


def test_normalise_rejects_bad_rows():
    with pytest.raises(ms.BadInput):
        ms.normalise(np.array([[0.0, 0.0], [1.0, 0.0]]))
    with pytest.raises(ms.BadInput):
        ms.normalise(np.array([[np.nan, 1.0]]))


# ---------------------------------------------------------------- whole pipeline

@pytest.fixture(scope="module")
def mid_result():
    f = synth.make_frame(synth.MID)
    return f, C.cluster(f.emb, f.mask, C.Params(bandwidth=f.bandwidth))


def test_modes_are_fixed_points(mid_result):
    f, res = mid_result
    thr = 1 - f.bandwidth
    yn, delta, _ = ms.shift(res.modes, res.x, thr)
    assert np.all(delta < f.bandwidth / 1000)
    assert np.max(np.abs(yn - res.modes)) < 1e-12


def test_modes_are_mutually_outside_windows(mid_result):
    f, res = mid_result
    s = res.modes @ res.modes.T
    np.fill_diagonal(s, -1)
    assert s.max() < 1 - f.bandwidth


def test_known_centres_are_found(mid_result):
    # Every generated cell with at least 100 single-owner pixels has a mode
    # within 5e-3 cosine distance of its centre (mode noise is ~sigma sqrt(D/m)).
    f, res = mid_result
    own, sec = f.owner.reshape(-1), f.second.reshape(-1)
    for k in range(len(f.centres)):
        if np.count_nonzero((own == k) & (sec < 0)) >= 100:
            assert 1 - np.max(res.modes @ f.centres[k]) < 5e-3


def test_labels_background_and_range(mid_result):
    f, res = mid_result
    lab = res.labels
    assert np.all(lab[f.mask.reshape(-1) == 0] == -1)
    fgl = lab[f.mask.reshape(-1) != 0]
    assert fgl.min() >= 0 and fgl.max() < len(res.modes)


def test_round_seeds_follow_the_seed_order(mid_result):
    f, res = mid_result
    order = so.seed_order(f.n_fg, 0)
    first = res.rounds[0]
    np.testing.assert_array_equal(first.seeds, order[:len(first.seeds)])
    used = np.concatenate([r.seeds for r in res.rounds])
    assert len(set(used.tolist())) == len(used)


def test_empty_mask():
    f = synth.make_frame(synth.TINY)
    res = C.cluster(f.emb, np.zeros_like(f.mask), C.Params(bandwidth=0.1))
    assert len(res.modes) == 0 and np.all(res.labels == -1)
    assert res.stats["n_state_out"] == 128


# ---------------------------------------------------------------- planted mistakes

def _pins_catch(monkeypatch, broken_shift):
    monkeypatch.setattr(ms, "shift", broken_shift)
    failures = 0
    for fn in (test_tight_clusters_closed_form, test_flat_kernel_boundary_is_inclusive):
        try:
            fn()
        except AssertionError:
            failures += 1
    return failures


def test_planted_mistakes_are_caught(monkeypatch):
    real = ms.shift

    def strict(y, x, thr):  # '>' instead of '>='
        return real(y, x, np.nextafter(thr, 2.0))

    def unnormalised(y, x, thr):  # mean without renormalisation
        yn, d, m = real(y, x, thr)
        w = (np.asarray(y) @ x.T) >= thr
        v = (w.astype(float) @ x) / m[:, None]
        return v, 1 - np.sum(y * v, 1), m

    def drops_first_member(y, x, thr):  # a dropped term
        return real(y, x[1:], thr)

    for bad in (strict, unnormalised, drops_first_member):
        assert _pins_catch(monkeypatch, bad) >= 1, bad.__name__


def _failures(fns):
    failures = 0
    for fn in fns:
        try:
            fn()
        except AssertionError:
            failures += 1
    return failures


def test_planted_coverage_and_stop_mistakes_are_caught(monkeypatch):
    real_cov, real_it = ms.covered_by, ms.iterate
    cover_pins = (test_coverage_boundary_is_inclusive, test_later_round_seeds_skip_covered_pixels)

    def cover_strict(x, modes, thr):  # '>' instead of '>='
        return real_cov(x, modes, np.nextafter(thr, 2.0))

    def cover_nothing(x, modes, thr):  # coverage never applied
        return np.zeros(len(x), bool)

    for bad in (cover_strict, cover_nothing):
        monkeypatch.setattr(ms, "covered_by", bad)
        assert _failures(cover_pins) >= 1, bad.__name__
    monkeypatch.setattr(ms, "covered_by", real_cov)

    def stop_inclusive(x, seeds, thr, tol, gamma, max_iter, trace=False):  # '>=' instead of '>'
        return real_it(x, seeds, thr, tol, gamma - 1e-9, max_iter, trace)

    monkeypatch.setattr(ms, "iterate", stop_inclusive)
    assert _failures((test_gamma_stop_is_strict,)) >= 1
