"""Faster Mean-shift (arXiv 2007.14283) on MI355X: Python binding of libfms.so.

Cosine, flat-kernel mean shift over per-pixel embeddings (Eq. 8-11), seeds
iterated in parallel with early stopping (Sec. 3.2.3) under the online seed
optimisation policy (Sec. 3.2.2, 3.2.4), then mode pruning and pixel
assignment (Alg. 2).  Every step runs in the library's HIP kernels; this module
only marshals arguments.  PyTorch provides device memory and the stream.

    modes, labels, stats = cluster(emb, mask, bandwidth=0.2)

``emb`` is a float32 GPU tensor, (H, W, D) by default or (D, H, W) with
``layout="nchw"``; ``mask`` is an (H, W) GPU tensor (nonzero = foreground) or
None.
"""
from __future__ import annotations

import ctypes
import dataclasses
from typing import Dict, Optional

from . import _binding as B

__all__ = ["Params", "FmsError", "FP32", "BF16_REFINE", "BF16_SPLIT", "cluster", "cluster_batch", "shift_seeds", "unroll",
           "autotune", "autotune_batch", "clear_tuning", "seed_order", "default_params", "library"]

FP32 = B.FMS_PREC_FP32
BF16_REFINE = B.FMS_PREC_BF16_REFINE
BF16_SPLIT = B.FMS_PREC_BF16_SPLIT


class FmsError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        lib = B.load()
        msg = lib.fms_status_string(status).decode()
        super().__init__(f"{what}: {msg} (status {status})" if what else f"{msg} (status {status})")
        self.status = status


@dataclasses.dataclass
class Params:
    bandwidth: float = 0.1
    conv_tol: float = 0.0
    gamma: float = 0.9
    big_l: float = 2.0
    big_h: float = 8.0
    p_target: float = 0.99
    seed: int = 0
    n_initial: int = 128
    n_state_in: int = 0
    max_iter: int = 100
    max_rounds: int = 32
    precision: int = FP32
    refine_iters: int = 2
    timing: int = 0
    tile_seeds: int = 0
    tile_items: int = 0
    tile_chunks: int = 0
    tile_waves: int = 0
    graphs: int = 0

    def to_c(self) -> B.FmsParams:
        c = B.FmsParams()
        for f in dataclasses.fields(self):
            setattr(c, f.name, getattr(self, f.name))
        return c


def library():
    """The loaded libfms.so (raises when it is not built)."""
    return B.load()


def default_params() -> Params:
    c = B.FmsParams()
    library().fms_default_params(ctypes.byref(c))
    return Params(**{f.name: getattr(c, f.name) for f in dataclasses.fields(Params)})


_handles: Dict[int, ctypes.c_void_p] = {}


def _handle(device_index: int) -> ctypes.c_void_p:
    h = _handles.get(device_index)
    if h is None:
        h = ctypes.c_void_p()
        st = library().fms_create(ctypes.byref(h), device_index)
        if st != B.FMS_OK:
            raise FmsError(st, "fms_create")
        _handles[device_index] = h
    return h


def _params(params: Optional[Params], kw) -> Params:
    p = dataclasses.replace(params) if params is not None else Params()
    for k, v in kw.items():
        if not hasattr(p, k):
            raise TypeError(f"unknown parameter {k!r}")
        setattr(p, k, v)
    return p


def _frame_args(emb, layout: str):
    import torch
    if not isinstance(emb, torch.Tensor) or not emb.is_cuda:
        raise TypeError("emb must be a GPU tensor")
    if emb.dtype != torch.float32:
        raise TypeError("emb must be float32")
    if emb.dim() != 3:
        raise ValueError("emb must be 3-D")
    if layout == "nhwc":
        h, w, d = emb.shape
        if emb.stride(0) != w * emb.stride(1):
            emb = emb.contiguous()
        ps, cs = emb.stride(1), emb.stride(2)
    elif layout == "nchw":
        d, h, w = emb.shape
        if emb.stride(1) != w * emb.stride(2):
            emb = emb.contiguous()
        ps, cs = emb.stride(2), emb.stride(0)
    else:
        raise ValueError("layout must be 'nhwc' or 'nchw'")
    return emb, h, w, d, ps, cs


def _mask_arg(mask, h, w, device):
    import torch
    if mask is None:
        return None, None
    if not isinstance(mask, torch.Tensor):
        raise TypeError("mask must be a tensor or None")
    m = mask.to(device=device, dtype=torch.uint8).reshape(h * w).contiguous()
    return m, m.data_ptr()


def _stream_ptr(device):
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def cluster(emb, mask=None, bandwidth: Optional[float] = None, *, layout: str = "nhwc",
            params: Optional[Params] = None, k_max: int = 4096, **kw):
    """Cluster one frame.  Returns (modes [K, D] float32, labels [H, W] int32,
    stats dict with ``mode_counts`` added)."""
    import torch
    if bandwidth is not None:
        kw["bandwidth"] = bandwidth
    p = _params(params, kw)
    emb, h, w, d, ps, cs = _frame_args(emb, layout)
    dev = emb.device
    m, mptr = _mask_arg(mask, h, w, dev)
    lib = library()
    hdl = _handle(dev.index if dev.index is not None else torch.cuda.current_device())
    cp = p.to_c()
    while True:
        modes = torch.empty((max(k_max, 1), d), dtype=torch.float32, device=dev)
        counts = torch.empty((max(k_max, 1),), dtype=torch.int32, device=dev)
        labels = torch.empty((h, w), dtype=torch.int32, device=dev)
        nm = ctypes.c_int32(0)
        stats = B.FmsStats()
        st = lib.fms_cluster(hdl, _stream_ptr(dev), ctypes.c_void_p(emb.data_ptr()), ps, cs,
                             ctypes.c_void_p(mptr) if mptr else None, h, w, d, ctypes.byref(cp),
                             ctypes.c_void_p(modes.data_ptr()), ctypes.c_void_p(counts.data_ptr()), k_max,
                             ctypes.byref(nm), ctypes.c_void_p(labels.data_ptr()), ctypes.byref(stats))
        if st == B.FMS_ERR_CAPACITY and nm.value > k_max:
            k_max = nm.value
            continue
        if st != B.FMS_OK:
            raise FmsError(st, "fms_cluster")
        break
    k = nm.value
    out = stats.as_dict()
    out["mode_counts"] = counts[:k]
    return modes[:k], labels, out


def cluster_batch(frames, *, layout: str = "nhwc", params: Optional[Params] = None, k_max: int = 0, **kw):
    """Cluster a batch of frames of one embedding width D in one call
    (fms_cluster_batch).  ``frames``: sequence of dicts with ``emb`` (GPU
    float32, (H, W, D) or (D, H, W) per ``layout``), ``mask`` (GPU (H, W) or
    None), ``bandwidth`` and optionally ``n_state_in``.  Returns a list of
    (modes [K_f, D], labels [H, W], stats dict with ``mode_counts``) per frame."""
    import torch
    p = _params(params, kw)
    frames = list(frames)
    if not frames:
        return []
    lib = library()
    cframes = (B.FmsFrame * len(frames))()
    keep = []
    dev = None
    d0 = None
    outs = []
    for i, fr in enumerate(frames):
        emb, h, w, d, ps, cs = _frame_args(fr["emb"], layout)
        if d0 is None:
            d0, dev = d, emb.device
        elif d != d0 or emb.device != dev:
            raise ValueError("every frame of a batch needs the same D and device")
        m, mptr = _mask_arg(fr.get("mask"), h, w, dev)
        labels = torch.empty((h, w), dtype=torch.int32, device=dev)
        keep += [emb, m, labels]
        cf = cframes[i]
        cf.emb = emb.data_ptr()
        cf.pixel_stride, cf.channel_stride = ps, cs
        cf.mask = mptr if mptr else None
        cf.height, cf.width = h, w
        cf.bandwidth = float(fr["bandwidth"])
        cf.n_state_in = int(fr.get("n_state_in", 0))
        cf.labels = labels.data_ptr()
        outs.append(labels)
    hdl = _handle(dev.index if dev.index is not None else torch.cuda.current_device())
    cp = p.to_c()
    n = len(frames)
    k_max = max(k_max, 256 * n)
    while True:
        modes = torch.empty((k_max, d0), dtype=torch.float32, device=dev)
        counts = torch.empty((k_max,), dtype=torch.int32, device=dev)
        offs = (ctypes.c_int32 * (n + 1))()
        stats = (B.FmsStats * n)()
        st = lib.fms_cluster_batch(hdl, _stream_ptr(dev), n, cframes, d0, ctypes.byref(cp),
                                   ctypes.c_void_p(modes.data_ptr()), ctypes.c_void_p(counts.data_ptr()), k_max,
                                   offs, stats)
        if st == B.FMS_ERR_CAPACITY and offs[n] > k_max:
            k_max = offs[n]
            continue
        if st != B.FMS_OK:
            raise FmsError(st, "fms_cluster_batch")
        break
    res = []
    for i in range(n):
        a, b = offs[i], offs[i + 1]
        sd = stats[i].as_dict()
        sd["mode_counts"] = counts[a:b]
        res.append((modes[a:b], outs[i], sd))
    return res


_UNROLL_FN = None


def autotune(emb, mask=None, bandwidth: Optional[float] = None, *, layout: str = "nhwc",
             params: Optional[Params] = None, **kw):
    """Time the fused step's work decompositions on this frame (fms_autotune)
    and keep the fastest in the device's handle for later calls that leave
    the tiling to the library, when whole calls on the frame get faster with
    them.  Returns {"entries": [dicts], "kept": bool, "ms_default": x,
    "ms_tuned": y}."""
    import torch
    if bandwidth is not None:
        kw["bandwidth"] = bandwidth
    p = _params(params, kw)
    emb, h, w, d, ps, cs = _frame_args(emb, layout)
    dev = emb.device
    m, mptr = _mask_arg(mask, h, w, dev)
    fr = B.FmsFrame()
    fr.emb = emb.data_ptr()
    fr.pixel_stride, fr.channel_stride = ps, cs
    fr.mask = mptr if mptr else None
    fr.height, fr.width = h, w
    fr.bandwidth = float(p.bandwidth)
    fr.n_state_in = 0
    fr.labels = None
    entries = (B.FmsTuneEntry * 16)()
    count = ctypes.c_int32(0)
    report = B.FmsTuneReport()
    lib = library()
    hdl = _handle(dev.index if dev.index is not None else torch.cuda.current_device())
    cp = p.to_c()
    st = lib.fms_autotune(hdl, _stream_ptr(dev), ctypes.byref(fr), d, ctypes.byref(cp), entries, 16,
                          ctypes.byref(count), ctypes.byref(report))
    if st != B.FMS_OK:
        raise FmsError(st, "fms_autotune")
    return {"entries": [entries[i].as_dict() for i in range(count.value)], "kept": bool(report.kept),
            "ms_default": float(report.ms_default), "ms_tuned": float(report.ms_tuned)}


def autotune_batch(frames, *, layout: str = "nhwc", params: Optional[Params] = None, **kw):
    """fms_autotune_batch: time the fused step's work decompositions on
    launches spanning all ``frames`` (dicts as for ``cluster_batch``, at
    least two) and keep the fastest in the device's handle for later batch
    calls that leave the tiling to the library, when whole batch calls get
    faster with them.  Returns {"entries": [dicts], "kept": bool,
    "ms_default": x, "ms_tuned": y}."""
    import torch
    p = _params(params, kw)
    frames = list(frames)
    cframes = (B.FmsFrame * len(frames))()
    keep = []
    dev = d0 = None
    for i, fr in enumerate(frames):
        emb, h, w, d, ps, cs = _frame_args(fr["emb"], layout)
        if d0 is None:
            d0, dev = d, emb.device
        elif d != d0 or emb.device != dev:
            raise ValueError("every frame of a batch needs the same D and device")
        m, mptr = _mask_arg(fr.get("mask"), h, w, dev)
        keep += [emb, m]
        cf = cframes[i]
        cf.emb = emb.data_ptr()
        cf.pixel_stride, cf.channel_stride = ps, cs
        cf.mask = mptr if mptr else None
        cf.height, cf.width = h, w
        cf.bandwidth = float(fr["bandwidth"])
        cf.n_state_in = 0
        cf.labels = None
    entries = (B.FmsTuneEntry * 16)()
    count = ctypes.c_int32(0)
    report = B.FmsTuneReport()
    lib = library()
    hdl = _handle(dev.index if dev.index is not None else torch.cuda.current_device())
    cp = p.to_c()
    st = lib.fms_autotune_batch(hdl, _stream_ptr(dev), len(frames), cframes, d0, ctypes.byref(cp), entries, 16,
                                ctypes.byref(count), ctypes.byref(report))
    if st != B.FMS_OK:
        raise FmsError(st, "fms_autotune_batch")
    return {"entries": [entries[i].as_dict() for i in range(count.value)], "kept": bool(report.kept),
            "ms_default": float(report.ms_default), "ms_tuned": float(report.ms_tuned)}


def clear_tuning(device=None):
    """Forget the tuned decompositions of the device's handle."""
    import torch
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    st = library().fms_clear_tuning(_handle(dev.index if dev.index is not None else torch.cuda.current_device()))
    if st != B.FMS_OK:
        raise FmsError(st, "fms_clear_tuning")


def _unroll_function():
    """torch.autograd.Function around fms_unroll / fms_unroll_backward (built
    on first use so that importing this package does not import torch)."""
    global _UNROLL_FN
    if _UNROLL_FN is not None:
        return _UNROLL_FN
    import torch

    class Unroll(torch.autograd.Function):
        @staticmethod
        def forward(ctx, emb, mask, seeds, steps, bandwidth, layout):
            e, h, w, d, ps, cs = _frame_args(emb.detach(), layout)
            dev = e.device
            m, mptr = _mask_arg(mask, h, w, dev)
            sd = torch.as_tensor(seeds).to(device=dev, dtype=torch.int32).contiguous()
            ns = int(sd.numel())
            y = torch.empty((ns, d), dtype=torch.float32, device=dev)
            yp = torch.empty_like(y)
            vn = torch.empty((ns,), dtype=torch.float32, device=dev)
            hdl = _handle(dev.index if dev.index is not None else torch.cuda.current_device())
            st = library().fms_unroll(hdl, _stream_ptr(dev), ctypes.c_void_p(e.data_ptr()), ps, cs,
                                      ctypes.c_void_p(mptr) if mptr else None, h, w, d,
                                      ctypes.c_void_p(sd.data_ptr()), ns, steps, bandwidth,
                                      ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(yp.data_ptr()),
                                      ctypes.c_void_p(vn.data_ptr()))
            if st != B.FMS_OK:
                raise FmsError(st, "fms_unroll")
            ctx.save_for_backward(e, y, yp, vn)
            ctx.geom = (m, mptr, h, w, d, ps, cs, ns, bandwidth, hdl, tuple(emb.shape))
            return y

        @staticmethod
        def backward(ctx, gy):
            e, y, yp, vn = ctx.saved_tensors
            m, mptr, h, w, d, ps, cs, ns, bandwidth, hdl, shape = ctx.geom
            gy = gy.to(dtype=torch.float32).contiguous()
            grad = torch.empty_like(e)
            st = library().fms_unroll_backward(hdl, _stream_ptr(e.device), ctypes.c_void_p(e.data_ptr()), ps, cs,
                                               ctypes.c_void_p(mptr) if mptr else None, h, w, d, ns, bandwidth,
                                               ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(yp.data_ptr()),
                                               ctypes.c_void_p(vn.data_ptr()), ctypes.c_void_p(gy.data_ptr()),
                                               ctypes.c_void_p(grad.data_ptr()))
            if st != B.FMS_OK:
                raise FmsError(st, "fms_unroll_backward")
            return grad.reshape(shape), None, None, None, None, None

    _UNROLL_FN = Unroll
    return Unroll


def unroll(emb, mask, seeds, steps: int = 10, bandwidth: float = 0.1, *, layout: str = "nhwc"):
    """y_T of ``steps`` unrolled FP32 mean-shift steps from ``seeds``
    (foreground ordinals), every seed taking all steps; differentiable with
    respect to ``emb`` through torch.autograd (fms_unroll_backward).  Returns
    [m, D] float32."""
    return _unroll_function().apply(emb, mask, seeds, int(steps), float(bandwidth), layout)


def shift_seeds(emb, mask, seeds, *, layout: str = "nhwc", params: Optional[Params] = None, **kw):
    """One round of the parallel seed iteration on explicit seeds (foreground
    ordinals).  Returns a dict with endpoints [m, D], iters, converged,
    counts and stats."""
    import torch
    p = _params(params, kw)
    emb, h, w, d, ps, cs = _frame_args(emb, layout)
    dev = emb.device
    m, mptr = _mask_arg(mask, h, w, dev)
    sd = torch.as_tensor(seeds).to(device=dev, dtype=torch.int32).contiguous()
    ns = int(sd.numel())
    endpoints = torch.empty((max(ns, 1), d), dtype=torch.float32, device=dev)
    iters = torch.empty((max(ns, 1),), dtype=torch.int32, device=dev)
    conv = torch.empty((max(ns, 1),), dtype=torch.uint8, device=dev)
    counts = torch.empty((max(ns, 1),), dtype=torch.int32, device=dev)
    stats = B.FmsStats()
    lib = library()
    hdl = _handle(dev.index if dev.index is not None else torch.cuda.current_device())
    cp = p.to_c()
    st = lib.fms_shift_seeds(hdl, _stream_ptr(dev), ctypes.c_void_p(emb.data_ptr()), ps, cs,
                             ctypes.c_void_p(mptr) if mptr else None, h, w, d,
                             ctypes.c_void_p(sd.data_ptr()), ns, ctypes.byref(cp),
                             ctypes.c_void_p(endpoints.data_ptr()), ctypes.c_void_p(iters.data_ptr()),
                             ctypes.c_void_p(conv.data_ptr()), ctypes.c_void_p(counts.data_ptr()),
                             ctypes.byref(stats))
    if st != B.FMS_OK:
        raise FmsError(st, "fms_shift_seeds")
    return {"endpoints": endpoints[:ns], "iters": iters[:ns], "converged": conv[:ns],
            "counts": counts[:ns], "stats": stats.as_dict()}


def seed_order(n: int, seed: int = 0, device=None):
    """The library's seed order: a permutation of range(n) as an int32 tensor."""
    import torch
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    out = torch.empty((max(n, 1),), dtype=torch.int32, device=dev)
    hdl = _handle(dev.index if dev.index is not None else torch.cuda.current_device())
    st = library().fms_seed_order(hdl, _stream_ptr(dev), n, seed, ctypes.c_void_p(out.data_ptr()))
    if st != B.FMS_OK:
        raise FmsError(st, "fms_seed_order")
    torch.cuda.current_stream(dev).synchronize()
    return out[:n]
