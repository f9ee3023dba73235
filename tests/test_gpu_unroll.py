"""GPU parity of the differentiable form (fms_unroll / fms_unroll_backward via
torch.autograd) against the FP64 oracle of oracle/unroll.py, whose gradient is
itself pinned to FP64 finite differences.

Seeds whose oracle trajectory came within BAND = 1e-5 of a window edge are
exempt (FP32 and FP64 may take different membership decisions there: the
FP32 rounding of a 32-term dot product of unit vectors, and of the
renormalised centres, stays below about 2e-6, so 1e-5 leaves a margin); they
get a zero target, and the gradient is compared on the pixels that sit at
least BAND from the edge of every remaining seed's last window.  Tolerances: y_T
within 1e-5 (1 - cos); gradients within 1e-4 of the largest oracle entry
plus 1e-3 relative."""
import numpy as np
import pytest

import synth
from oracle import unroll as U
from oracle import seed_order as so

pytestmark = pytest.mark.gpu

BAND = 1e-5
STEPS = 10


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def F():
    import paper_2007_14283_amd as fms
    fms.library()
    return fms


@pytest.fixture(scope="module")
def frame512():
    return synth.make_frame(synth.PLAIN512)


def _crop(frame, size=64):
    # The size x size window with the most foreground among a fixed grid.
    best = None
    for y0 in range(0, frame.spec.height - size + 1, size):
        for x0 in range(0, frame.spec.width - size + 1, size):
            c = int(frame.mask[y0:y0 + size, x0:x0 + size].sum())
            if best is None or c > best[0]:
                best = (c, y0, x0)
    _, y0, x0 = best
    emb = np.ascontiguousarray(frame.emb[y0:y0 + size, x0:x0 + size])
    mask = np.ascontiguousarray(frame.mask[y0:y0 + size, x0:x0 + size])
    return emb, mask


def _trajectory_margins(x, seeds, h, steps):
    # Per-seed smallest |y_{t-1} . x_i - (1 - h)| over all steps (FP64).
    thr = 1.0 - h
    y = x[seeds]
    marg = np.full(len(seeds), np.inf)
    for _ in range(steps):
        s = y @ x.T
        marg = np.minimum(marg, np.min(np.abs(s - thr), axis=1))
        v = (s >= thr).astype(np.float64) @ x
        y = v / np.linalg.norm(v, axis=1, keepdims=True)
    return marg


def _compare(F, emb_np, mask_np, h, n_seeds, layout="nhwc"):
    import torch
    fg = np.flatnonzero(mask_np.reshape(-1))
    e_fg = emb_np.reshape(-1, emb_np.shape[-1])[fg].astype(np.float64)
    x = e_fg / np.linalg.norm(e_fg, axis=1, keepdims=True)
    n = len(fg)
    seeds = so.seed_order(n, 0)[:min(n_seeds, n)].astype(np.int64)
    marg = _trajectory_margins(x, seeds, h, STEPS)
    keep = marg >= BAND
    rng = np.random.default_rng(0)
    targets = rng.normal(size=(len(seeds), emb_np.shape[-1]))
    targets /= np.linalg.norm(targets, axis=1, keepdims=True)
    targets[~keep] = 0.0

    emb = torch.from_numpy(emb_np).cuda()
    if layout == "nchw":
        emb = emb.permute(2, 0, 1).contiguous()
    emb.requires_grad_(True)
    mask = torch.from_numpy(mask_np).cuda()
    y = F.unroll(emb, mask, torch.from_numpy(seeds.astype(np.int32)), STEPS, h, layout=layout)
    loss = (y * torch.from_numpy(targets).float().cuda()).sum()
    loss.backward()
    g = emb.grad.detach()
    if layout == "nchw":
        g = g.permute(1, 2, 0)
    g = g.cpu().double().numpy().reshape(-1, emb_np.shape[-1])

    y_or, y_prev, _, _ = U.forward(e_fg, seeds, h, STEPS)
    err = 1.0 - np.sum(y.detach().cpu().double().numpy() * y_or, axis=1)
    g_or = U.grad(e_fg, seeds, h, STEPS, targets)
    # Pixels clear of every kept seed's last window edge.
    s_last = y_prev[keep] @ x.T
    clear = np.all(np.abs(s_last - (1.0 - h)) >= BAND, axis=0)
    print(f"n={n} seeds={len(seeds)} exempt seeds={int((~keep).sum())} exempt pixels={int((~clear).sum())} "
          f"max y err (kept)={err[keep].max():.2e}")
    return g, g_or, fg, clear, err, keep


def test_unroll_crop_forward_and_gradient(F, frame512):
    emb, mask = _crop(frame512)
    _say("unroll crop 64x64", int(mask.sum()))
    g, g_or, fg, clear, err, keep = _compare(F, emb, mask, frame512.bandwidth, 128)
    assert keep.sum() >= 0.8 * len(keep)
    assert err[keep].max() <= 1e-5
    scale = np.abs(g_or).max()
    assert scale > 0
    np.testing.assert_allclose(g[fg][clear], g_or[clear], atol=1e-4 * scale, rtol=1e-3)
    bg = np.setdiff1d(np.arange(g.shape[0]), fg)
    assert np.all(g[bg] == 0.0)


def test_unroll_nchw_layout(F, frame512):
    emb, mask = _crop(frame512)
    _say("unroll crop nchw")
    g, g_or, fg, clear, err, keep = _compare(F, emb, mask, frame512.bandwidth, 64, layout="nchw")
    scale = np.abs(g_or).max()
    np.testing.assert_allclose(g[fg][clear], g_or[clear], atol=1e-4 * scale, rtol=1e-3)


def test_unroll_full_512_frame(F, frame512):
    _say("unroll 512x512")
    g, g_or, fg, clear, err, keep = _compare(F, frame512.emb, frame512.mask, frame512.bandwidth, 256)
    assert err[keep].max() <= 1e-5
    scale = np.abs(g_or).max()
    np.testing.assert_allclose(g[fg][clear], g_or[clear], atol=1e-4 * scale, rtol=1e-3)


def test_unroll_rejects_bad_seed(F, frame512):
    import torch
    emb, mask = _crop(frame512)
    n = int(mask.sum())
    with pytest.raises(F.FmsError):
        F.unroll(torch.from_numpy(emb).cuda(), torch.from_numpy(mask).cuda(),
                 torch.tensor([0, n], dtype=torch.int32), 2, frame512.bandwidth)


def test_unroll_gradient_matches_finite_differences(F, frame512):
    # The GPU gradient on the differentiation workload's crop against FP64
    # central differences at 200 sampled coordinates (tests/golden/unroll_fd.npz,
    # written from oracle/ alone and pinned in test_oracle_unroll.py): FP32
    # against FP64, within 1e-4 of the largest difference plus 1e-3 relative.
    import os

    import torch
    z = np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "unroll_fd.npz"))
    emb_np, mask_np = _crop(frame512)
    fg = np.flatnonzero(mask_np.reshape(-1))
    _say("unroll finite differences", len(fg), len(z["fd"]))
    emb = torch.from_numpy(emb_np).cuda().requires_grad_(True)
    mask = torch.from_numpy(mask_np).cuda()
    y = F.unroll(emb, mask, torch.from_numpy(z["seeds"].astype(np.int32)), int(z["steps"]), float(z["bandwidth"]))
    (y * torch.from_numpy(z["targets"]).float().cuda()).sum().backward()
    g = emb.grad.detach().cpu().double().numpy().reshape(-1, emb_np.shape[-1])
    rows, dims = z["coords"][:, 0], z["coords"][:, 1]
    got = g[fg[rows], dims]
    fd = z["fd"]
    tol = 1e-4 * np.abs(fd).max() + 1e-3 * np.abs(fd)
    print(f"max |gpu - fd| {np.abs(got - fd).max():.2e}, largest |fd| {np.abs(fd).max():.2e}")
    assert np.count_nonzero(np.abs(fd) > 1e-3) >= 20
    assert np.all(np.abs(got - fd) <= tol)
