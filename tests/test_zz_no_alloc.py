"""The allocation-free histogram entry point (apo_histogram_u8_noalloc,
device-resident scratch) against the allocating one (apo_histogram_u8),
both called through the C ABI: equal counts on two calls in a row, the
second on a smaller input, then on the full-size blob image, an unaligned
start and the degenerate sizes (one pixel, no pixels); each also against
numpy's bincount."""
import ctypes as C

import numpy as np
import pytest

import gen
from gpu_common import need_gpu

pytestmark = pytest.mark.gpu


def _both(apo, torch, dev):
    """Counts of the allocating call (host uint64) and of the allocation-free
    call (device uint64, copied back after a synchronisation)."""
    L = apo.lib()
    s = torch.cuda.current_stream()
    ref = np.zeros(256, np.uint64)
    assert L.apo_histogram_u8(C.c_void_p(dev.data_ptr()), dev.numel(),
                              ref.ctypes.data_as(C.POINTER(C.c_uint64)),
                              C.c_void_p(s.cuda_stream)) == 0
    out = torch.full((256,), -1, dtype=torch.int64, device="cuda")
    assert L.apo_histogram_u8_noalloc(C.c_void_p(dev.data_ptr()), dev.numel(),
                                      C.c_void_p(out.data_ptr()), C.c_void_p(s.cuda_stream)) == 0
    torch.cuda.synchronize()
    return ref.astype(np.int64), out.cpu().numpy()


def test_noalloc_histogram_equals_allocating_one():
    apo = need_gpu()
    import torch
    cases = [("random 3M", 3 << 20, 0, 11), ("random 200k, smaller", 200_003, 0, 12),
             ("unaligned start", 1_000_001, 5, 13), ("one pixel", 1, 0, 14),
             ("no pixels", 0, 0, 15)]
    for name, n, off, seed in cases:
        print(f"[noalloc] {name}: n={n} offset={off}", flush=True)
        host = np.random.default_rng(seed).integers(0, 256, size=n + off, dtype=np.uint8)
        dev = torch.from_numpy(host).cuda()
        ref, got = _both(apo, torch, dev[off:] if n > 0 else dev)
        want = np.bincount(host[off:], minlength=256)
        assert np.array_equal(ref, want), name
        assert np.array_equal(got, ref), name
    print("[noalloc] blob 4096x4096, then a 512x512 blob image", flush=True)
    for size in (4096, 512):
        img = gen.blob_image(size, size, seed=2)
        dev = torch.from_numpy(img).cuda().reshape(-1)
        ref, got = _both(apo, torch, dev)
        assert np.array_equal(ref, np.bincount(img.reshape(-1), minlength=256))
        assert np.array_equal(got, ref)


def test_noalloc_histogram_argument_checks():
    apo = need_gpu()
    import torch
    L = apo.lib()
    img = torch.zeros(16, dtype=torch.uint8, device="cuda")
    out = torch.zeros(257, dtype=torch.int64, device="cuda")
    assert L.apo_histogram_u8_noalloc(C.c_void_p(img.data_ptr()), 16, None, None) == -1
    assert L.apo_histogram_u8_noalloc(C.c_void_p(img.data_ptr()), 16,
                                      C.c_void_p(out.data_ptr() + 4), None) == -1
    assert L.apo_histogram_u8_noalloc(None, 16, C.c_void_p(out.data_ptr()), None) == -1
    assert L.apo_histogram_u8_noalloc(C.c_void_p(img.data_ptr()), 1 << 32,
                                      C.c_void_p(out.data_ptr()), None) == -6
