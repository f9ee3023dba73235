"""Synthetic embedding frames shaped like the paper's microscopy workloads.

Recipe (stated once here, repeated in the design notes):

* Cell centres ``c_k`` are unit vectors drawn from an isotropic normal and
  rejection-sampled so that every earlier centre has ``c_k . c_j < 0.5`` (the
  paper's blobs are mutually "orthogonal or opposite", Sec. 4.1 Design).
* Cells are ellipses: centre uniform over the frame, semi-axes uniform in
  ``[r_min, r_max]`` (independently), angle uniform in ``[0, pi)``.  They are
  painted in index order; ``owner`` is the last cell covering a pixel and
  ``second`` the owner before it.
* A pixel owned by one cell starts at ``c_owner``; a pixel on an overlap starts
  at the normalised mix ``normalize(c_owner + c_second)``.  Then per-component
  Gaussian noise of standard deviation ``sigma`` is added and the vector is
  normalised again (the make_blobs convention of Sec. 4.1).
* Background pixels carry random unit vectors, so a masking mistake shows up;
  ``mask = owner >= 0``.
* With ``overlap_cap`` set, a cell is re-placed (up to 100 tries, keeping the
  try with the smallest share) when it would push the overlap share of the
  foreground above the cap.
* The bandwidth of a frame is the smallest of 0.10, 0.15, ..., 0.30 whose
  cosine cap ``cos >= 1 - h`` holds 99.9 % of the single-owner pixels around
  their own centre; the paper's h = 0.1 (Sec. 4.1 Design) is kept wherever it
  fits.

Everything is drawn from ``numpy.random.Generator(PCG64(seed))`` in a fixed
order, so a (spec, seed) pair always gives the same frame.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

BANDWIDTH_LADDER = (0.10, 0.15, 0.20, 0.25, 0.30)


@dataclasses.dataclass(frozen=True)
class FrameSpec:
    height: int
    width: int
    n_cells: int
    r_min: float
    r_max: float
    dim: int
    sigma: float
    overlap_cap: Optional[float] = None
    seed: int = 0

    def with_seed(self, seed: int) -> "FrameSpec":
        return dataclasses.replace(self, seed=seed)


@dataclasses.dataclass
class Frame:
    spec: FrameSpec
    emb: np.ndarray        # (H, W, D) float32, pixel-major (NHWC)
    mask: np.ndarray       # (H, W) uint8, 1 = foreground
    owner: np.ndarray      # (H, W) int32, -1 = background
    second: np.ndarray     # (H, W) int32, -1 = none
    centres: np.ndarray    # (n_cells, D) float64, unit rows
    bandwidth: float
    n_fg: int
    overlap_share: float

    @property
    def shape(self):
        return self.emb.shape


# Presets.  Sizes follow the paper's frames (512^2 HeLa, 1024^2 GOWT1, Sec. 4.2)
# and the workloads named for this hot path.
TINY = FrameSpec(128, 128, 20, 4, 12, 16, 0.05, None, 0)
PLAIN512 = FrameSpec(512, 512, 100, 8, 30, 32, 0.08, 0.05, 0)
PRECISION1024 = FrameSpec(1024, 1024, 300, 8, 30, 32, 0.08, 0.05, 0)
# A parity-test frame the oracle finishes in seconds: several pixel tiles,
# a ragged tail, D = 32.
MID = FrameSpec(192, 160, 24, 6, 16, 32, 0.05, 0.05, 3)


def _unit_rows(v: np.ndarray) -> np.ndarray:
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def _draw_centres(rng: np.random.Generator, k: int, dim: int, max_dot: float = 0.5) -> np.ndarray:
    out = np.zeros((k, dim))
    got = 0
    tries = 0
    while got < k:
        c = _unit_rows(rng.standard_normal(dim)[None, :])[0]
        tries += 1
        if got == 0 or np.max(out[:got] @ c) < max_dot or tries > 1000 * k:
            out[got] = c
            got += 1
    return out


def _ellipse_mask(h, w, cy, cx, a, b, ang):
    r = int(math.ceil(max(a, b))) + 1
    y0, y1 = max(0, int(math.floor(cy)) - r), min(h, int(math.floor(cy)) + r + 1)
    x0, x1 = max(0, int(math.floor(cx)) - r), min(w, int(math.floor(cx)) + r + 1)
    if y0 >= y1 or x0 >= x1:
        return (0, 0, 0, 0), np.zeros((0, 0), bool)
    yy, xx = np.mgrid[y0:y1, x0:x1]
    dy, dx = yy - cy, xx - cx
    ca, sa = math.cos(ang), math.sin(ang)
    u = (dx * ca + dy * sa) / a
    v = (-dx * sa + dy * ca) / b
    return (y0, y1, x0, x1), (u * u + v * v) <= 1.0


def _choose_bandwidth(emb64, owner, second, centres) -> float:
    excl = (owner >= 0) & (second < 0)
    if not np.any(excl):
        return BANDWIDTH_LADDER[0]
    x = emb64[excl]
    c = centres[owner[excl]]
    cosv = np.sum(x * c, axis=1) / np.linalg.norm(x, axis=1)
    q = np.quantile(cosv, 0.001)
    for h in BANDWIDTH_LADDER:
        if 1.0 - h <= q:
            return h
    return BANDWIDTH_LADDER[-1]


def make_frame(spec: FrameSpec) -> Frame:
    rng = np.random.Generator(np.random.PCG64(spec.seed))
    H, W, D = spec.height, spec.width, spec.dim
    centres = _draw_centres(rng, spec.n_cells, D)
    owner = np.full((H, W), -1, np.int32)
    second = np.full((H, W), -1, np.int32)
    n_fg = 0
    n_ov = 0
    for k in range(spec.n_cells):
        a = rng.uniform(spec.r_min, spec.r_max)
        b = rng.uniform(spec.r_min, spec.r_max)
        ang = rng.uniform(0.0, math.pi)
        best = None
        for _ in range(100 if spec.overlap_cap is not None else 1):
            cy, cx = rng.uniform(0, H), rng.uniform(0, W)
            box, m = _ellipse_mask(H, W, cy, cx, a, b, ang)
            y0, y1, x0, x1 = box
            o = owner[y0:y1, x0:x1]
            s = second[y0:y1, x0:x1]
            add_fg = int(np.count_nonzero(m & (o < 0)))
            add_ov = int(np.count_nonzero(m & (o >= 0) & (s < 0)))
            share = (n_ov + add_ov) / max(1, n_fg + add_fg)
            if best is None or share < best[0]:
                best = (share, box, m, add_fg, add_ov)
            if spec.overlap_cap is None or share <= spec.overlap_cap:
                break
        share, (y0, y1, x0, x1), m, add_fg, add_ov = best
        if m.size:
            o = owner[y0:y1, x0:x1]
            s = second[y0:y1, x0:x1]
            s[m] = o[m]
            o[m] = k
            n_fg += add_fg
            n_ov += add_ov
    fg = owner >= 0
    base = np.zeros((H, W, D))
    own = owner[fg]
    sec = second[fg]
    v = centres[own]
    mix = sec >= 0
    v[mix] = _unit_rows(v[mix] + centres[sec[mix]])
    base[fg] = v
    noise = rng.standard_normal((int(fg.sum()), D)) * spec.sigma
    base[fg] = _unit_rows(base[fg] + noise)
    nbg = H * W - int(fg.sum())
    base[~fg] = _unit_rows(rng.standard_normal((nbg, D)))
    h = _choose_bandwidth(base, owner, second, centres)
    nf = int(fg.sum())
    ov = int(np.count_nonzero(fg & (second >= 0)))
    return Frame(spec, base.astype(np.float32), fg.astype(np.uint8), owner, second, centres, h,
                 nf, ov / max(1, nf))


def batch_specs(n_frames: int = 64, dim: int = 32) -> List[FrameSpec]:
    """Uneven multi-frame batch: side in {256, 512, 768, 1024}, 10-300 cells,
    foreground 20-50 % (reached by scaling the radii), sigma in U(0.03, 0.1).
    Frame f is drawn from seed f."""
    out = []
    for f in range(n_frames):
        rng = np.random.Generator(np.random.PCG64(10_000 + f))
        side = int(rng.choice([256, 512, 768, 1024]))
        cells = int(rng.integers(10, 301))
        fg = float(rng.uniform(0.2, 0.5))
        sigma = float(rng.uniform(0.03, 0.1))
        area = -math.log(1.0 - fg) * side * side / cells
        r = math.sqrt(area / math.pi)
        out.append(FrameSpec(side, side, cells, max(2.0, 0.6 * r), max(3.0, 1.4 * r), dim, sigma,
                             0.05, f))
    return out


def drifting_sequence(spec: FrameSpec, n_frames: int, drift=(1, 2)) -> List[Frame]:
    """A synthetic video: the cells of ``make_frame(spec)`` translated by
    ``drift`` pixels (dy, dx) per frame with wrap-around, each frame with fresh
    per-component noise (seed spec.seed * 1000 + t) and fresh background
    vectors.  The cell vectors, shapes and the bandwidth stay those of frame 0,
    as for one cell line over a time-lapse."""
    f0 = make_frame(spec)
    H, W, D = spec.height, spec.width, spec.dim
    out = [f0]
    for t in range(1, n_frames):
        rng = np.random.Generator(np.random.PCG64(spec.seed * 1000 + t))
        owner = np.roll(f0.owner, (t * drift[0], t * drift[1]), axis=(0, 1))
        second = np.roll(f0.second, (t * drift[0], t * drift[1]), axis=(0, 1))
        fg = owner >= 0
        base = np.zeros((H, W, D))
        v = f0.centres[owner[fg]]
        sec = second[fg]
        mix = sec >= 0
        v[mix] = _unit_rows(v[mix] + f0.centres[sec[mix]])
        base[fg] = _unit_rows(v + rng.standard_normal((int(fg.sum()), D)) * spec.sigma)
        base[~fg] = _unit_rows(rng.standard_normal((H * W - int(fg.sum()), D)))
        nf = int(fg.sum())
        ov = int(np.count_nonzero(fg & (second >= 0)))
        out.append(Frame(spec, base.astype(np.float32), fg.astype(np.uint8), owner, second, f0.centres,
                         f0.bandwidth, nf, ov / max(1, nf)))
    return out


def circle_points(seed: int = 0, n: int = 1500, noise: float = 0.02):
    """Two concentric circles with 10 clusters (Sec. 4.1 Data): returns an
    (n, 2) float32 point set and the cluster id of each point.  Clusters sit at
    ten distinct angles, alternating between the radius-1 and radius-0.5
    circle; radii are jittered by +-5 % and Gaussian noise is added."""
    rng = np.random.Generator(np.random.PCG64(seed))
    k = np.arange(n) % 10
    ang = 2 * math.pi * k / 10
    radius = np.where(k % 2 == 0, 1.0, 0.5) * rng.uniform(0.95, 1.05, n)
    pts = np.stack([radius * np.cos(ang), radius * np.sin(ang)], 1) + rng.standard_normal((n, 2)) * noise
    return pts.astype(np.float32), k.astype(np.int32)


def blob_points(n: int, seed: int = 0, dim: int = 18, sigma: float = 0.01):
    """Ten 18-D blobs whose centres are mutually orthogonal or opposite
    (+-e_0 ... +-e_4), per-component noise 0.01 (Sec. 4.1 Design)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    centres = np.zeros((10, dim))
    for c in range(10):
        centres[c, c // 2] = 1.0 if c % 2 == 0 else -1.0
    lab = rng.integers(0, 10, n)
    pts = centres[lab] + rng.standard_normal((n, dim)) * sigma
    return pts.astype(np.float32), lab.astype(np.int32)


def overlap_circles(overlap: float, seed: int = 0, side: int = 1000, dim: int = 18,
                    diameter: float = 250.0):
    """Appendix A workload: eight noise-free discs of diameter 250 on a
    side x side frame; ``overlap`` in [0, 1) pulls the discs together so that
    neighbouring discs intersect more.  Returns (emb, mask, owner, centres)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    centres = _draw_centres(rng, 8, dim, 0.3)
    rad = diameter / 2
    step = diameter * (1.0 - overlap)
    cy0, cx0 = side / 2 - 0.5 * step, side / 2 - 1.5 * step
    owner = np.full((side, side), -1, np.int32)
    yy, xx = np.mgrid[0:side, 0:side]
    for k in range(8):
        cy = cy0 + (k // 4) * step
        cx = cx0 + (k % 4) * step
        owner[(yy - cy) ** 2 + (xx - cx) ** 2 <= rad * rad] = k
    emb = _unit_rows(rng.standard_normal((side, side, dim)))
    fg = owner >= 0
    emb[fg] = centres[owner[fg]]
    return emb.astype(np.float32), fg.astype(np.uint8), owner, centres
