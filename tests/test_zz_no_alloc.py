"""fms_shift_seeds_noalloc (the entry point for callers that cannot allocate)
against fms_shift_seeds through the C ABI: the same endpoints, step counts,
converged flags, window counts and statistics, on two calls in a row, the
second on a smaller frame with fewer seeds (the fixed buffer keeps the first
call's contents), and its limits rejected on the host."""
import ctypes

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import paper_2007_14283_amd as fms
    fms.library()
    return fms


def _call(F, name, frame, seeds, **kw):
    import torch
    from paper_2007_14283_amd import _binding as B
    lib = F.library()
    h = F._handle(0)
    emb = torch.from_numpy(frame.emb).cuda()
    mask = torch.from_numpy(frame.mask).cuda()
    hgt, wid, dim = frame.emb.shape
    sd = torch.from_numpy(np.asarray(seeds, np.int32)).cuda()
    m = len(seeds)
    ep = torch.full((max(m, 1), dim), float("nan"), device="cuda")
    it = torch.full((max(m, 1),), -7, dtype=torch.int32, device="cuda")
    cv = torch.full((max(m, 1),), 9, dtype=torch.uint8, device="cuda")
    ct = torch.full((max(m, 1),), -7, dtype=torch.int32, device="cuda")
    p = F.Params(bandwidth=frame.bandwidth, **kw).to_c()
    st = B.FmsStats()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = getattr(lib, name)(h, stream, ctypes.c_void_p(emb.data_ptr()), dim, 1, ctypes.c_void_p(mask.data_ptr()),
                            hgt, wid, dim, ctypes.c_void_p(sd.data_ptr()), m, ctypes.byref(p),
                            ctypes.c_void_p(ep.data_ptr()), ctypes.c_void_p(it.data_ptr()),
                            ctypes.c_void_p(cv.data_ptr()), ctypes.c_void_p(ct.data_ptr()), ctypes.byref(st))
    torch.cuda.synchronize()
    return rc, ep[:m].cpu().numpy(), it[:m].cpu().numpy(), cv[:m].cpu().numpy(), ct[:m].cpu().numpy(), st.as_dict()


def _seeds(frame, m, key):
    rng = np.random.Generator(np.random.PCG64(key))
    return rng.choice(frame.n_fg, size=m, replace=False).astype(np.int32)


def _same(F, frame, seeds):
    print(f"[case] noalloc vs shift_seeds: {frame.spec.height}x{frame.spec.width}, n {frame.n_fg}, "
          f"{len(seeds)} seeds", flush=True)
    a = _call(F, "fms_shift_seeds", frame, seeds)
    b = _call(F, "fms_shift_seeds_noalloc", frame, seeds)
    assert a[0] == 0 and b[0] == 0, (a[0], b[0])
    np.testing.assert_array_equal(b[1], a[1])
    for k in (2, 3, 4):
        np.testing.assert_array_equal(b[k], a[k])
    for k in ("n_fg", "seeds_used", "iterations_total", "seed_pixel_updates", "n_discarded"):
        assert b[5][k] == a[5][k], k
    assert a[3].sum() > 0.8 * len(seeds)


def test_two_calls_second_smaller(F):
    big = synth.make_frame(synth.PLAIN512)
    small = synth.make_frame(synth.MID)
    _same(F, big, _seeds(big, 1024, 1))
    _same(F, small, _seeds(small, 200, 2))


def test_limits_rejected(F):
    from paper_2007_14283_amd import _binding as B
    small = synth.make_frame(synth.MID)
    rc = _call(F, "fms_shift_seeds_noalloc", small, np.zeros(4097, np.int32))[0]
    assert rc == B.FMS_ERR_UNSUPPORTED
    rc = _call(F, "fms_shift_seeds_noalloc", small, _seeds(small, 8, 3), precision=F.BF16_SPLIT)[0]
    assert rc == B.FMS_ERR_UNSUPPORTED
    # A frame with more foreground pixels than the fixed buffer holds: found
    # on the GPU, reported as unsupported.
    wide = synth.make_frame(synth.FrameSpec(512, 512, 600, 20, 40, 16, 0.02, None, 4))
    assert wide.n_fg > 131072
    rc = _call(F, "fms_shift_seeds_noalloc", wide, _seeds(wide, 16, 4))[0]
    assert rc == B.FMS_ERR_UNSUPPORTED
    # The buffer is still usable afterwards.
    _same(F, small, _seeds(small, 64, 5))
