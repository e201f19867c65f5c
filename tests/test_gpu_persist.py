"""The persistent single-launch pass sequence (sizes compiled with one)
against one launch per pass, through the C ABI: bitwise equal outputs for
single frames (Charbonnier and Welsch penalties, u0 != f, detail
enhancement) and for batches (frames of mixed channel counts in one class,
graph replays); no wait gives up in a normal run; and a wait limit of 1 us
makes the kernel give up and end, reported by ils_last_error."""
import sys

import numpy as np
import pytest

from synth import voronoi_image

pytestmark = [
    pytest.mark.gpu,
    pytest.mark.skip(reason="the persistent single-launch path is switched off: its first launches on the "
                            "MI355X did not end (twice, the second time with waits bounded by the real-time "
                            "clock), cause not found; ils_plan_set_persistent(plan, 1) returns "
                            "ILS_ERR_INVALID_ARG"),
]


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


SIZES = [(256, 256, 1, 40), (480, 640, 3, 60), (720, 1280, 1, 180), (1080, 1920, 3, 400), (2160, 3840, 3, 800)]


@pytest.mark.parametrize("H,W,C,K", SIZES, ids=[f"{s[0]}x{s[1]}x{s[2]}" for s in SIZES])
def test_persistent_matches_per_pass(torch, ils, H, W, C, K):
    f = torch.from_numpy(voronoi_image(H, W, C, K, 0.05, seed=H + C)).cuda()
    u0 = torch.clamp(f + 0.01 * torch.randn_like(f), 0, 1).contiguous()
    plan = ils.Plan(H, W, C)
    res = {}
    for on in (False, True):
        _say(f"{H}x{W}x{C} persistent={on}")
        plan.set_persistent(on)
        res[on] = [plan.smooth(f, 1.0, 0.8, 1e-4, 4).cpu().numpy(),
                   plan.smooth_welsch(f, 20.0, 10 / 255, 3).cpu().numpy(),
                   plan.iterate_from(f, u0, 2.0, 0.5, 1e-4, 2).cpu().numpy(),
                   plan.detail_enhance(f, 1.0, 0.8, 1e-4, 1, 3.0).cpu().numpy()]
        torch.cuda.synchronize()
        assert plan.last_error() == 0
    for i, (a, b) in enumerate(zip(res[False], res[True])):
        assert np.isfinite(b).all(), i
        assert np.array_equal(a, b), (i, float(np.max(np.abs(a - b))))
    plan.close()


def test_persistent_batch_mixed_channels(torch, ils):
    """1080p grey and RGB frames of one class (one persistent launch per
    part, channel prefix sums on the device), and 256^2 grey frames, against
    single calls with one launch per pass, on eager calls and graph replays."""
    specs = [(1080, 1920, 3), (1080, 1920, 1), (1080, 1920, 3), (256, 256, 1), (256, 256, 1), (1080, 1920, 1)]
    fs = [torch.from_numpy(voronoi_image(H, W, C, 100, 0.05, seed=300 + i)).cuda() for i, (H, W, C) in enumerate(specs)]
    params = [(1.0, 0.8, 4), (1.5, 0.6, 4), (0.7, 0.9, 4), (1.0, 0.8, 4), (2.0, 0.5, 4), (1.2, 0.7, 4)]
    single = ils.Plan(1080, 1920, 3)
    single.set_persistent(False)
    want = [single.smooth(f, lam, p, 1e-4, N).cpu().numpy() for f, (lam, p, N) in zip(fs, params)]
    single.close()
    for graph in (False, True):
        plan = ils.Plan(1080, 1920, 3, max_frames=len(fs), graph=graph)
        plan.set_persistent(True)
        for rep in range(3):
            _say(f"persistent batch graph={graph} rep={rep}")
            outs = plan.smooth_batch([(f, lam, p, 1e-4, N) for f, (lam, p, N) in zip(fs, params)])
            torch.cuda.synchronize()
            assert plan.last_error() == 0
            for i, (o, w) in enumerate(zip(outs, want)):
                assert np.array_equal(o.cpu().numpy(), w), (graph, rep, i)
        plan.close()


def test_wait_limit_gives_up_and_ends(torch, ils):
    """A wait limit of 1 us: items run without waiting for the items they
    depend on, the kernel ends, and ils_last_error reports it once."""
    f = torch.from_numpy(voronoi_image(1080, 1920, 3, 400, 0.05, seed=5)).cuda()
    plan = ils.Plan(1080, 1920, 3)
    plan.set_persistent(True)
    plan._lib.ils_plan_set_wait_limit(plan._h, 1)
    _say("wait limit 1 us")
    plan.smooth(f, 1.0, 0.8, 1e-4, 4)
    torch.cuda.synchronize()
    assert plan.last_error() != 0
    assert plan.last_error() == 0  # read and cleared
    plan._lib.ils_plan_set_wait_limit(plan._h, 0)
    u = plan.smooth(f, 1.0, 0.8, 1e-4, 4)
    torch.cuda.synchronize()
    assert plan.last_error() == 0
    plan.set_persistent(False)
    v = plan.smooth(f, 1.0, 0.8, 1e-4, 4)
    torch.cuda.synchronize()
    assert np.array_equal(u.cpu().numpy(), v.cpu().numpy())
    plan.close()
