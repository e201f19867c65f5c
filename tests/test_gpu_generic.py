"""The runtime-length passes (sizes whose row or column length has no
compiled four-step split) in batches: frames of such sizes mixed with
compiled sizes in one batched call give bitwise the results of single-frame
calls, on eager calls and on graph replays; and the detail-enhancement blend
of their final pass against the oracle."""
import sys

import numpy as np
import pytest

from oracle import ils as O
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


@pytest.fixture(scope="module")
def ils(torch):
    from paper_2003_07504_amd import ils as m
    return m


def test_batch_mixes_runtime_and_compiled_lengths(torch, ils):
    sizes = [(768, 1024, 3), (480, 640, 1), (450, 600, 3), (768, 1024, 1), (81, 54, 2), (480, 640, 3)]
    params = [(1.0, 0.8, 4), (2.0, 0.5, 4), (0.7, 0.9, 3), (1.5, 0.6, 4), (1.0, 0.8, 5), (1.2, 0.7, 4)]
    fs = [torch.from_numpy(voronoi_image(H, W, C, max(4, H * W // 5000), 0.05, seed=900 + i)).cuda()
          for i, (H, W, C) in enumerate(sizes)]
    single = ils.Plan(768, 1024, 3)
    want = [single.smooth(f, lam, p, 1e-4, N).cpu().numpy() for f, (lam, p, N) in zip(fs, params)]
    single.close()
    for graph in (False, True):
        plan = ils.Plan(768, 1024, 3, max_frames=len(fs), graph=graph)
        for rep in range(3):
            _say(f"batch graph={graph} rep={rep}")
            outs = plan.smooth_batch([(f, lam, p, 1e-4, N) for f, (lam, p, N) in zip(fs, params)])
            torch.cuda.synchronize()
            assert plan.last_error() == 0
            for i, (o, w) in enumerate(zip(outs, want)):
                assert np.array_equal(o.cpu().numpy(), w), (graph, rep, i)
        plan.close()


def test_runtime_length_detail_enhance(torch, ils):
    H, W, C, k = 450, 600, 3, 3.0
    _say(f"detail enhance {H}x{W}x{C} k={k}")
    f = voronoi_image(H, W, C, 50, 0.05, seed=77)
    ref = O.detail_enhance(f.astype(np.float64), O.ils_channels(f, 1.0, 0.8, 1e-4, 4), k)
    plan = ils.Plan(H, W, C)
    out = plan.detail_enhance(torch.from_numpy(f).cuda(), 1.0, 0.8, 1e-4, 4, k)
    torch.cuda.synchronize()
    assert plan.last_error() == 0
    d = out.cpu().numpy().astype(np.float64) - ref
    # the blend scales the smoothing error by |1 - k| = 2
    assert np.max(np.abs(d)) <= 2e-4 and np.linalg.norm(d) / np.linalg.norm(ref) <= 2e-5
    plan.close()
