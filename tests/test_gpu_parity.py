"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerance for the whole iteration: max-abs <= 1e-4 and relative L2 <= 1e-5
on [0, 1] images.  Single passes are compared with float64 NumPy transforms
of the same definitions."""
import sys

import numpy as np
import pytest

from oracle import ils as O
from synth import voronoi_image, batch_mix

pytestmark = pytest.mark.gpu

MAX_ABS = 1e-4
REL_L2 = 1e-5


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


def _errs(u_gpu, u_ref):
    d = u_gpu.astype(np.float64) - u_ref
    return float(np.max(np.abs(d))), float(np.linalg.norm(d) / np.linalg.norm(u_ref))


def _gpu_smooth(torch, ils, f, lam, p, eps, N):
    ft = torch.from_numpy(f).cuda()
    plan = ils.Plan(f.shape[-2], f.shape[-1], f.shape[0] if f.ndim == 3 else 1)
    u = plan.smooth(ft, lam, p, eps, N)
    torch.cuda.synchronize()
    assert plan.last_error() == 0
    out = u.cpu().numpy()
    plan.close()
    return out


# Sizes whose row or column length has no compiled split (runtime-length
# passes): H generic; both generic; odd W/2 = 27 with H = 81; the maximum
# column length 4096; the maximum row length W/2 = 4096.
GENERIC_STAGE_SHAPES = [(768, 1024, 1), (450, 600, 2), (81, 54, 1), (4096, 8, 1), (6, 8192, 1)]


# ------------------------------------------------------------ single passes
@pytest.mark.parametrize("H,W,C", [(8, 8, 1), (16, 16, 2), (90, 120, 1), (256, 256, 1), (1080, 1920, 1),
                                   (2160, 3840, 1), (480, 640, 1), (720, 1280, 1)] + GENERIC_STAGE_SHAPES)
def test_stage_rhs_spectrum(torch, ils, H, W, C):
    _say(f"stage rhs H={H} W={W} C={C}")
    lam, p, eps = 1.3, 0.7, 1e-4
    f = voronoi_image(H, W, C, max(4, H * W // 5000), 0.05, seed=H + W)
    u0 = np.clip(f + 0.01 * np.random.default_rng(1).standard_normal(f.shape), 0, 1).astype(np.float32)
    plan = ils.Plan(H, W, C)
    spec = plan.debug_rhs_spectrum(torch.from_numpy(f).cuda(), torch.from_numpy(u0).cuda(), lam, p, eps)
    torch.cuda.synchronize()
    got = spec.cpu().numpy().astype(np.complex128)
    c = O.charbonnier_c0(p, eps)
    kap = lam * c / 2
    u = u0.astype(np.float64)
    mx = O.mu_update(O.grad_x(u), p, eps, c) / c
    my = O.mu_update(O.grad_y(u), p, eps, c) / c
    d = (np.roll(mx, 1, axis=-1) - mx) + (np.roll(my, 1, axis=-2) - my)
    r = f.astype(np.float64) + kap * d
    exp = 2.0 * np.fft.rfft(r, axis=-1)
    rel = np.linalg.norm(got - exp) / np.linalg.norm(exp)
    assert rel < 3e-6, rel
    plan.close()


@pytest.mark.parametrize("H,W,C", [(8, 8, 1), (16, 16, 1), (90, 120, 2), (256, 256, 1), (1080, 1920, 1),
                                   (2160, 3840, 1), (480, 640, 1), (720, 1280, 1)] + GENERIC_STAGE_SHAPES)
def test_stage_column_solve(torch, ils, H, W, C):
    _say(f"stage column H={H} W={W} C={C}")
    lam, p, eps = 0.9, 0.8, 1e-4
    rng = np.random.default_rng(H * 7 + W)
    x = (rng.standard_normal((C, H, W // 2 + 1)) + 1j * rng.standard_normal((C, H, W // 2 + 1))).astype(np.complex64)
    plan = ils.Plan(H, W, C)
    out = plan.debug_column_solve(torch.from_numpy(x).cuda(), W, lam, p, eps)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.complex128)
    kap = lam * O.charbonnier_c0(p, eps) / 2
    sx = 4 * np.sin(np.pi * np.arange(W // 2 + 1) / W) ** 2
    sy = 4 * np.sin(np.pi * np.arange(H) / H) ** 2
    den = 2.0 * H * W * (1 + kap * (sx[None, :] + sy[:, None]))
    exp = H * np.fft.ifft(np.fft.fft(x.astype(np.complex128), axis=-2) / den, axis=-2)
    rel = np.linalg.norm(got - exp) / np.linalg.norm(exp)
    assert rel < 3e-6, rel
    plan.close()


@pytest.mark.parametrize("H,W,C", [(8, 8, 1), (16, 16, 1), (90, 120, 2), (256, 256, 1), (1080, 1920, 1),
                                   (2160, 3840, 1), (480, 640, 1), (720, 1280, 1)] + GENERIC_STAGE_SHAPES)
def test_stage_row_inverse(torch, ils, H, W, C):
    _say(f"stage row inverse H={H} W={W} C={C}")
    rng = np.random.default_rng(H * 3 + W)
    x = (rng.standard_normal((C, H, W // 2 + 1)) + 1j * rng.standard_normal((C, H, W // 2 + 1))).astype(np.complex64)
    plan = ils.Plan(H, W, C)
    out = plan.debug_row_inverse(torch.from_numpy(x).cuda(), W)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.float64)
    exp = W * np.fft.irfft(x.astype(np.complex128), n=W, axis=-1)
    rel = np.linalg.norm(got - exp) / np.linalg.norm(exp)
    assert rel < 3e-6, rel
    plan.close()


# ------------------------------------------------------------ end to end
CASES = [
    # (H, W, C, K, sigma, lam, p, N, seed)   configs: 256^2 grey; 1080p RGB
    (256, 256, 1, 40, 0.05, 1.0, 0.8, 4, 0),
    (1080, 1920, 3, 400, 0.05, 1.0, 0.8, 4, 1),
    (8, 8, 1, 4, 0.05, 1.0, 0.8, 4, 11),
    (16, 16, 2, 6, 0.05, 2.0, 0.5, 4, 12),
    (90, 120, 2, 10, 0.05, 1.5, 0.6, 3, 13),
    (60, 96, 1, 8, 0.08, 0.7, 1.0, 6, 14),
    (2, 4, 1, 2, 0.05, 1.0, 0.8, 2, 15),
    (480, 640, 3, 60, 0.05, 0.5, 0.9, 4, 16),
    (720, 1280, 1, 180, 0.05, 2.0, 0.5, 4, 17),
    (540, 720, 1, 70, 0.05, 1.0, 0.8, 5, 18),
    # p outside the configs' [0.5, 1]: the paper's p = 0.2 (lambda = 0.5,
    # N = 10; c0 ~ 796, kappa ~ 199) and 1 < p < 2
    (256, 256, 1, 40, 0.05, 0.5, 0.2, 10, 21),
    (1080, 1920, 3, 400, 0.05, 0.5, 0.2, 10, 22),
    (256, 256, 1, 40, 0.05, 1.0, 1.5, 4, 23),
    (1080, 1920, 3, 400, 0.05, 1.0, 1.5, 4, 24),
    # runtime-length passes: 1024 x 768 RGB (H = 768), 800 x 600 (H = 600,
    # W/2 = 400), odd W/2, and the maximum lengths
    (768, 1024, 3, 100, 0.05, 1.0, 0.8, 4, 25),
    (600, 800, 1, 60, 0.05, 2.0, 0.5, 4, 26),
    (81, 54, 2, 8, 0.05, 1.0, 0.8, 4, 27),
    (4096, 8, 1, 20, 0.05, 1.0, 0.8, 4, 28),
    (6, 8192, 1, 20, 0.05, 1.0, 0.8, 4, 29),
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}x{c[1]}x{c[2]}_p{c[6]}" for c in CASES])
def test_end_to_end_parity(torch, ils, case):
    H, W, C, K, sig, lam, p, N, seed = case
    _say(f"e2e H={H} W={W} C={C} lam={lam} p={p} N={N} seed={seed}")
    f = voronoi_image(H, W, C, K, sig, seed)
    got = _gpu_smooth(torch, ils, f, lam, p, 1e-4, N)
    ref = O.ils_channels(f.astype(np.float64), lam, p, 1e-4, N, workers=8)
    ma, rl = _errs(got, ref)
    _say(f"  max_abs={ma:.3e} rel_l2={rl:.3e}")
    assert ma <= MAX_ABS and rl <= REL_L2


def test_config4_crop_parity(torch, ils):
    """4K RGB frame (2000 cells, sigma 0.08); its 256 x 256 crop smoothed as
    an image of its own at lam = 2, p = 0.5, N = 10."""
    _say("config4 crop 256x256 from 4K, N=10")
    f = voronoi_image(2160, 3840, 3, 2000, 0.08, seed=5000)[:, :256, :256].copy()
    got = _gpu_smooth(torch, ils, f, 2.0, 0.5, 1e-4, 10)
    ref = O.ils_channels(f.astype(np.float64), 2.0, 0.5, 1e-4, 10)
    ma, rl = _errs(got, ref)
    _say(f"  max_abs={ma:.3e} rel_l2={rl:.3e}")
    assert ma <= MAX_ABS and rl <= REL_L2


def test_config4_full_frame_channel_parity(torch, ils):
    """One channel of the full 4K frame at lam = 2, p = 0.5, N = 10, whole
    frame against the oracle (plus a fixed 256 x 256 window)."""
    _say("config4 full 4K channel, N=10")
    f = voronoi_image(2160, 3840, 1, 2000, 0.08, seed=5000)
    got = _gpu_smooth(torch, ils, f, 2.0, 0.5, 1e-4, 10)
    ref = O.ils_channels(f.astype(np.float64), 2.0, 0.5, 1e-4, 10, workers=8)
    ma, rl = _errs(got, ref)
    wa, _ = _errs(got[:, 1000:1256, 2000:2256], ref[:, 1000:1256, 2000:2256])
    _say(f"  max_abs={ma:.3e} rel_l2={rl:.3e} window_max={wa:.3e}")
    assert ma <= MAX_ABS and rl <= REL_L2 and wa <= MAX_ABS


# ------------------------------------------------------- special cases
def test_p2_single_mode_closed_form(torch, ils):
    _say("p=2 closed form")
    H, W = 90, 120
    y = np.arange(H)[:, None]
    x = np.arange(W)[None, :]
    lam = 1.5
    outs = []
    for kx, ky in [(1, 0), (0, 3), (7, 5), (60, 45)]:
        mode = np.cos(2 * np.pi * (kx * x / W + ky * y / H) + 0.3)
        f = (0.5 + 0.2 * mode).astype(np.float32)[None]
        got = _gpu_smooth(torch, ils, f, lam, 2.0, 1e-4, 4)
        gain = 1 / (1 + 4 * lam * (np.sin(np.pi * kx / W) ** 2 + np.sin(np.pi * ky / H) ** 2))
        exp = 0.5 + 0.2 * gain * (f[0].astype(np.float64) - 0.5) / 0.2
        outs.append(np.max(np.abs(got[0] - exp)))
    assert max(outs) < 2e-6, outs


def test_lambda0_and_N0_copy_exactly(torch, ils):
    _say("lambda=0 / N=0 copy")
    f = voronoi_image(90, 120, 2, 10, 0.05, seed=3)
    assert np.array_equal(_gpu_smooth(torch, ils, f, 0.0, 0.8, 1e-4, 4), f)
    assert np.array_equal(_gpu_smooth(torch, ils, f, 1.0, 0.8, 1e-4, 0), f)


def test_constant_image_and_mean(torch, ils):
    _say("constant image, mean preservation")
    f = np.full((1, 256, 256), 0.37, dtype=np.float32)
    got = _gpu_smooth(torch, ils, f, 2.0, 0.6, 1e-4, 4)
    assert np.max(np.abs(got - 0.37)) < 1e-6
    g = voronoi_image(480, 640, 3, 60, 0.05, seed=4)
    u = _gpu_smooth(torch, ils, g, 1.0, 0.8, 1e-4, 4)
    assert np.max(np.abs(u.mean(axis=(1, 2), dtype=np.float64) - g.mean(axis=(1, 2), dtype=np.float64))) < 1e-6


def test_in_place_and_determinism(torch, ils):
    _say("in place + determinism")
    f = voronoi_image(256, 256, 3, 40, 0.05, seed=5)
    ft = torch.from_numpy(f).cuda()
    plan = ils.Plan(256, 256, 3)
    a = plan.smooth(ft, 1.0, 0.8, 1e-4, 4)
    b = plan.smooth(ft, 1.0, 0.8, 1e-4, 4)
    g = ft.clone()
    plan.smooth(g, 1.0, 0.8, 1e-4, 4, out=g)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    assert torch.equal(a, g)
    plan.close()


def test_iterate_from_matches_oracle(torch, ils):
    _say("iterate_from (one-iteration map from a candidate)")
    f = voronoi_image(256, 256, 3, 40, 0.05, seed=6)
    v = O.ils_channels(f.astype(np.float64), 1.0, 0.8, 1e-4, 2).astype(np.float32)
    plan = ils.Plan(256, 256, 3)
    t = plan.iterate_from(torch.from_numpy(f).cuda(), torch.from_numpy(v).cuda(), 1.0, 0.8, 1e-4, 1)
    torch.cuda.synchronize()
    ref = O.ils_channels(f.astype(np.float64), 1.0, 0.8, 1e-4, 1, u0=v.astype(np.float64))
    ma, rl = _errs(t.cpu().numpy(), ref)
    assert ma <= MAX_ABS and rl <= REL_L2
    plan.close()


def test_rms_diff(torch, ils):
    _say("rms_diff")
    rng = np.random.default_rng(9)
    a = [torch.from_numpy(rng.random(s).astype(np.float32)).cuda() for s in [(3, 90, 120), (1, 256, 256), (7,)]]
    b = [torch.from_numpy(rng.random(t.shape).astype(np.float32)).cuda() for t in a]
    plan = ils.Plan(256, 256, 3)
    r = plan.rms_diff(a, b).cpu().numpy()
    exp = [np.sqrt(np.mean((x.cpu().numpy().astype(np.float64) - y.cpu().numpy()) ** 2)) for x, y in zip(a, b)]
    assert np.allclose(r, exp, rtol=1e-6)
    plan.close()


def test_plan_limits_and_workspace(torch, ils):
    _say("plan limits")
    from paper_2003_07504_amd._lib import IlsError
    plan = ils.Plan(256, 256, 1)
    f = torch.zeros((1, 480, 640), device="cuda")
    with pytest.raises(IlsError):
        plan.smooth(f, 1.0, 0.8)
    g = torch.zeros((2, 256, 256), device="cuda")
    with pytest.raises(IlsError):
        plan.smooth(g, 1.0, 0.8)
    h = torch.zeros((1, 254, 256), device="cuda")  # 254 = 2 x 127: not 2/3/5-smooth
    with pytest.raises(IlsError):
        plan.smooth(h, 1.0, 0.8)
    plan.close()


# ---------------------------------------------------------------- batch
def test_batch_matches_single_frames(torch, ils):
    """Uneven sizes in one call; each frame equals its single-frame result
    bitwise (same kernels, same order of arithmetic), and the oracle."""
    _say("batch of mixed sizes")
    sizes = [(480, 640), (720, 1280), (256, 256), (90, 120)]
    specs = batch_mix(n=8, seed=2, sizes=sizes)
    frames = [(torch.from_numpy(s.image()).cuda(), s.lam, s.p, s.eps, s.N) for s in specs]
    singles = []
    for f, lam, p, eps, N in frames:
        single = ils.Plan(f.shape[1], f.shape[2], f.shape[0])
        singles.append(single.smooth(f, lam, p, eps, N))
        torch.cuda.synchronize()
        single.close()
    plan = ils.Plan(720, 1280, 3, max_frames=8)
    # the batch runs as a captured graph: replay it several times with eager
    # work and synchronisation in between, checking every replay
    for rep in range(3):
        outs = plan.smooth_batch(frames)
        torch.cuda.synchronize()
        assert plan.last_error() == 0
        for u, o, s in zip(singles, outs, specs):
            assert torch.equal(u, o), (rep, s.H, s.W, s.C)
        junk = torch.randn(1 << 20, device="cuda").sum()  # eager work between replays
        torch.cuda.synchronize()
        del junk
    s = specs[0]
    ref = O.ils_channels(frames[0][0].cpu().numpy().astype(np.float64), s.lam, s.p, s.eps, s.N)
    ma, rl = _errs(outs[0].cpu().numpy(), ref)
    assert ma <= MAX_ABS and rl <= REL_L2
    plan.close()
    # the same batch without graph capture
    plan = ils.Plan(720, 1280, 3, max_frames=8, graph=False)
    outs = plan.smooth_batch(frames)
    torch.cuda.synchronize()
    for u, o in zip(singles, outs):
        assert torch.equal(u, o)
    plan.close()


def test_batch_graph_changes_with_structure(torch, ils):
    """A different batch structure re-captures; a repeated one replays with new
    frame contents and parameters."""
    _say("batch graph re-capture / replay with new data")
    plan = ils.Plan(256, 256, 3, max_frames=4)
    a = [torch.from_numpy(voronoi_image(256, 256, 1, 20, 0.05, seed=70 + i)).cuda() for i in range(4)]
    for k, (n, lam) in enumerate([(2, 1.0), (3, 1.5), (3, 0.7), (2, 2.0)]):
        frames = [(a[(i + k) % 4], lam, 0.8, 1e-4, 4) for i in range(n)]
        outs = plan.smooth_batch(frames)
        torch.cuda.synchronize()
        for (f, lm, p, eps, N), o in zip(frames, outs):
            single = ils.Plan(256, 256, 1)
            u = single.smooth(f, lm, p, eps, N)
            torch.cuda.synchronize()
            assert torch.equal(u, o), (k, n)
            single.close()
    plan.close()


def test_batch_mix_full_size(torch, ils):
    """The 64-frame uneven-size batch at its real sizes (640x480 .. 3840x2160,
    grey and RGB, per-frame lambda and p): every frame equals its single-frame
    result bitwise and keeps the mean of each channel; two small frames are
    compared with the oracle."""
    _say("full uneven-size batch (64 frames)")
    specs = batch_mix(n=64, seed=2)
    frames = [(torch.from_numpy(s.image()).cuda(), s.lam, s.p, s.eps, s.N) for s in specs]
    plan = ils.Plan(2160, 3840, 3, max_frames=64)
    outs = plan.smooth_batch(frames)
    torch.cuda.synchronize()
    assert plan.last_error() == 0
    single = ils.Plan(2160, 3840, 3)
    for i, ((f, lam, p, eps, N), o, s) in enumerate(zip(frames, outs, specs)):
        u = single.smooth(f, lam, p, eps, N)
        torch.cuda.synchronize()
        assert torch.equal(u, o), (i, s.H, s.W, s.C)
        dm = (o.double().mean(dim=(1, 2)) - f.double().mean(dim=(1, 2))).abs().max().item()
        assert dm < 2e-6, (i, dm)
    checked = 0
    for (f, lam, p, eps, N), o, s in zip(frames, outs, specs):
        if s.H == 480 and checked < 2:
            ref = O.ils_channels(f.cpu().numpy().astype(np.float64), lam, p, eps, N, workers=8)
            ma, rl = _errs(o.cpu().numpy(), ref)
            _say(f"  {s.W}x{s.H}x{s.C} lam={lam:.3f} p={p:.3f}: max_abs={ma:.3e} rel_l2={rl:.3e}")
            assert ma <= MAX_ABS and rl <= REL_L2
            checked += 1
    assert checked == 2
    single.close()
    plan.close()


# ------------------------------------------------------------ tile shapes (autotuner)
@pytest.mark.parametrize("H,W,C", [(1080, 1920, 3), (720, 1280, 1), (2160, 3840, 1)])
def test_tile_shapes_are_bitwise_equal(torch, ils, H, W, C):
    """Every compiled row-band / column-tile shape gives the same bits, in
    single and batched calls, and the tuner picks one of them."""
    nr, nc = ils.shape_variants(H, W)
    _say(f"tile shapes H={H} W={W} C={C}: {nr} row x {nc} column")
    f = [voronoi_image(H, W, C, 400, 0.05, seed=77 + i) for i in range(2)]
    ft = [torch.from_numpy(x).cuda() for x in f]
    plan = ils.Plan(H, W, C, max_frames=2)
    ref = None
    for r in range(nr):
        for c in range(nc):
            plan.set_shapes(H, W, C, r, c)
            u = plan.smooth(ft[0], 1.0, 0.8, 1e-4, 4)
            ub = plan.smooth_batch([(ft[0], 1.0, 0.8, 1e-4, 4), (ft[1], 1.7, 0.6, 1e-4, 3)])
            torch.cuda.synchronize()
            assert plan.last_error() == 0
            got = (u.cpu().numpy(), ub[0].cpu().numpy(), ub[1].cpu().numpy())
            assert np.array_equal(got[0], got[1]), (r, c)
            if ref is None:
                ref = got
            else:
                for a, b in zip(got, ref):
                    assert np.array_equal(a, b), (r, c)
    plan.close()
    fresh = ils.Plan(H, W, C)
    rt, ct = fresh.tune(H, W, C)
    assert 0 <= rt < nr and 0 <= ct < nc
    assert fresh.tune(H, W, C) == (rt, ct)
    u = fresh.smooth(ft[0], 1.0, 0.8, 1e-4, 4)
    torch.cuda.synchronize()
    assert np.array_equal(u.cpu().numpy(), ref[0])
    with pytest.raises(Exception):
        fresh.set_shapes(H, W, C, nr, 0)
    fresh.close()


def test_tune_cache_file_is_read_and_written(torch, ils, tmp_path, monkeypatch):
    """ILS_TUNE_CACHE: a stored choice (rows per band, columns per tile) is
    taken without timing; a newly tuned size is appended."""
    cache = tmp_path / "tune.txt"
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    nr, nc = ils.shape_variants(720, 1280)
    assert nr > 1 and nc > 1
    # find the band height / tile width of shape index 1 by forcing it on a plan
    cache.write_text(f"{arch} 720 1280 1 0 0\n")  # no such shape: ignored
    monkeypatch.setenv("ILS_TUNE_CACHE", str(cache))
    plan = ils.Plan(720, 1280, 1)
    r, c = plan.tune(720, 1280, 1)  # tuned now (the stored line named no compiled shape)
    plan.close()
    lines = cache.read_text().split("\n")
    last = [ln for ln in lines if ln.strip()][-1].split()
    assert last[:4] == [arch, "720", "1280", "1"]
    g, s = int(last[4]), int(last[5])
    assert g > 0 and s > 0
    # a fresh plan reads the appended line and returns the same shapes untimed
    plan = ils.Plan(720, 1280, 1)
    assert plan.tune(720, 1280, 1) == (r, c)
    plan.close()


def test_nan_in_input_propagates_and_leaves_other_frames_alone(torch, ils):
    """NaN in f is not checked for: it spreads through the transforms of its
    own channel; the other channel of the frame and the other frame of a batch
    are unaffected and equal their clean results."""
    H, W = 64, 96
    f = voronoi_image(H, W, 2, 8, 0.05, seed=3)
    g = voronoi_image(H, W, 2, 8, 0.05, seed=4)
    bad = f.copy()
    bad[0, 10, 20] = np.nan
    plan = ils.Plan(H, W, 2, max_frames=2)
    ft, gt, bt = (torch.from_numpy(x).cuda() for x in (f, g, bad))
    clean_f = plan.smooth(ft, 1.0, 0.8, 1e-4, 4).cpu().numpy()
    clean_g = plan.smooth(gt, 1.0, 0.8, 1e-4, 4).cpu().numpy()
    outs = plan.smooth_batch([(bt, 1.0, 0.8, 1e-4, 4), (gt, 1.0, 0.8, 1e-4, 4)])
    torch.cuda.synchronize()
    a, b = outs[0].cpu().numpy(), outs[1].cpu().numpy()
    assert np.isnan(a[0]).all()
    assert np.array_equal(a[1], clean_f[1])
    assert np.array_equal(b, clean_g)
    plan.close()


def test_batch_order_does_not_change_results(torch, ils):
    """Each frame's result is independent of its position in the batch."""
    sizes = [(90, 120, 1), (64, 96, 3), (90, 120, 3), (64, 96, 1)]
    fs = [torch.from_numpy(voronoi_image(H, W, C, 8, 0.05, seed=60 + i)).cuda() for i, (H, W, C) in enumerate(sizes)]
    params = [(1.0, 0.8, 4), (2.0, 0.5, 3), (0.7, 1.0, 4), (1.3, 0.6, 2)]
    plan = ils.Plan(90, 120, 3, max_frames=4)
    frames = [(fs[i], params[i][0], params[i][1], 1e-4, params[i][2]) for i in range(4)]
    first = [o.cpu().numpy() for o in plan.smooth_batch(frames)]
    order = [2, 0, 3, 1]
    second = plan.smooth_batch([frames[i] for i in order])
    torch.cuda.synchronize()
    for j, i in enumerate(order):
        assert np.array_equal(second[j].cpu().numpy(), first[i]), i
    plan.close()


def test_corrupt_tune_cache_is_ignored(torch, ils, tmp_path, monkeypatch):
    cache = tmp_path / "tune.txt"
    cache.write_text("garbage line\n\x00\x01 not numbers 7 7\ngfx950 1080 1920\n")
    monkeypatch.setenv("ILS_TUNE_CACHE", str(cache))
    f = voronoi_image(90, 120, 1, 8, 0.05, seed=1)
    plan = ils.Plan(90, 120, 1)
    u = plan.smooth(torch.from_numpy(f).cuda(), 1.0, 0.8, 1e-4, 4)
    torch.cuda.synchronize()
    assert plan.last_error() == 0
    ref = O.ils_channels(f.astype(np.float64), 1.0, 0.8, 1e-4, 4)
    assert _errs(u.cpu().numpy(), ref)[0] <= MAX_ABS
    plan.close()
