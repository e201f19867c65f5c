"""The allocation-free entry point ils_smooth_noalloc (spectra in the
library's own device array) against ils_smooth (plan workspace), through the
C ABI: two calls in a row, the second on a smaller frame, and the size limit.
Both run the same kernels on the same tables, so the outputs are compared
bit for bit; the smaller frame is also held to the FP64 oracle's bar."""
import ctypes
import sys

import numpy as np
import pytest

from oracle.ils import ils_channels
from synth import voronoi_image

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.skip("no GPU")
    return _t


def _noalloc(torch, f, lam, p, eps, N):
    from paper_2003_07504_amd import _lib
    L = _lib.load()
    C, H, W = f.shape
    out = torch.full_like(f, float("nan"))
    st = torch.cuda.current_stream().cuda_stream
    rc = L.ils_smooth_noalloc(ctypes.c_void_p(f.data_ptr()), H, W, C, lam, p, eps, N,
                              ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(st))
    assert rc == 0, rc
    return out


def test_noalloc_matches_smooth_two_calls(torch):
    from paper_2003_07504_amd import ils
    cases = [(1080, 1920, 3, 400, 1.0, 0.8, 4), (256, 256, 1, 40, 2.0, 0.5, 10)]
    for i, (H, W, C, K, lam, p, N) in enumerate(cases):
        _say(f"noalloc call {i}: {H}x{W}x{C} lambda={lam} p={p} N={N}")
        f_np = voronoi_image(H, W, C, K, 0.05, seed=70 + i)
        f = torch.from_numpy(f_np).cuda()
        got = _noalloc(torch, f, lam, p, 1e-4, N)
        plan = ils.Plan(H, W, C)
        ref = plan.smooth(f, lam, p, 1e-4, N)
        torch.cuda.synchronize()
        assert plan.last_error() == 0
        plan.close()
        g, r = got.cpu().numpy(), ref.cpu().numpy()
        assert np.isfinite(g).all()
        assert np.array_equal(g, r), float(np.max(np.abs(g - r)))
        if H * W <= 65536:
            o = ils_channels(f_np.astype(np.float64), lam, p, 1e-4, N)
            d = g.astype(np.float64) - o
            assert np.max(np.abs(d)) <= 1e-4
            assert np.linalg.norm(d) / np.linalg.norm(o) <= 1e-5


def test_noalloc_rejects_frames_beyond_its_array(torch):
    from paper_2003_07504_amd import _lib
    L = _lib.load()
    assert L.ils_noalloc_max_bytes() == (64 - 4) << 20
    # 3840 x 2160 RGB needs 2 * 3 * 2160 * 1936 * 8 bytes of spectra: rejected before any enqueue
    f = torch.zeros((3, 2160, 3840), dtype=torch.float32, device="cuda")
    rc = L.ils_smooth_noalloc(ctypes.c_void_p(f.data_ptr()), 2160, 3840, 3, 1.0, 0.8, 1e-4, 4,
                              ctypes.c_void_p(f.data_ptr()), None)
    assert rc == -3
    assert L.ils_smooth_noalloc(None, 64, 64, 1, 1.0, 0.8, 1e-4, 4, None, None) == -1
    # N = 0 is a copy
    x = torch.rand((1, 64, 96), device="cuda")
    y = torch.empty_like(x)
    rc = L.ils_smooth_noalloc(ctypes.c_void_p(x.data_ptr()), 64, 96, 1, 1.0, 0.8, 1e-4, 0,
                              ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0
    torch.cuda.synchronize()
    assert torch.equal(x, y)
