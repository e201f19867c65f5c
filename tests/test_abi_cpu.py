"""C-ABI checks that need no GPU: the library loads, exports every function
include/ils.h declares, and rejects invalid arguments before any HIP call."""
import ctypes
import math
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ils.h")
NET_HEADER = os.path.join(ROOT, "include", "ils_net.h")


def _declared(path=HEADER):
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ils_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    from paper_2003_07504_amd import _lib
    return _lib.load()


def test_header_declares_expected_entry_points():
    names = _declared()
    for required in ("ils_plan_create", "ils_smooth", "ils_plan_destroy", "ils_smooth_batch"):
        assert required in names


def test_every_declared_symbol_is_exported(L):
    from paper_2003_07504_amd import _lib
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (ils_[a-z_0-9]+)$", out, flags=re.M))
    for name in _declared():
        assert name in exported, name
        assert name in _lib.SIGNATURES, name
        getattr(L, name)


def test_every_surrogate_symbol_is_exported(L):
    from paper_2003_07504_amd import _lib, surrogate
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (ils_[a-z_0-9]+)$", out, flags=re.M))
    names = _declared(NET_HEADER)
    assert "ils_net_train_step" in names and "ils_surrogate_infer" in names
    for name in names:
        assert name in exported, name
        assert name in surrogate._SIGS, name


def test_surrogate_validation_without_gpu(L):
    from paper_2003_07504_amd import surrogate
    lib = surrogate._lib()
    assert lib.ils_net_param_count() == 5 * 32 * 9 + 32 + 4 * (32 * 32 * 9 + 32) + 32 * 3 * 9 + 3
    assert lib.ils_net_workspace_bytes(0, 8, 8) == 0
    assert lib.ils_net_workspace_bytes(16, 256, 256) > 16 * 256 * 256 * 32 * 2 * 5
    h = ctypes.c_void_p()
    assert lib.ils_net_create(ctypes.byref(h), 1, 8, 8, None, 1 << 30, None) == -3
    assert lib.ils_net_create(None, 1, 8, 8, None, 0, None) == -1
    assert lib.ils_net_forward(None, None, None, None, 1, 8, 8, None) == -1
    assert lib.ils_net_train_step(None, None, None, None, None, 1, 8, 8, 1e-3, None) == -1
    assert lib.ils_net_destroy(None) == 0
    assert len(surrogate.init_params(0)) == lib.ils_net_param_count()


def test_smooth_signature_order_matches_header():
    text = open(HEADER).read()
    m = re.search(r"int ils_smooth\(([^)]*)\)", text)
    params = [p.split()[-1].lstrip("*") for p in m.group(1).replace("\n", " ").split(",")]
    assert params == ["plan", "f", "H", "W", "C", "lambda", "p", "eps", "N", "out"]


def test_status_strings(L):
    for code in (0, -1, -2, -3, -4, -5):
        assert L.ils_status_string(code)
    assert L.ils_status_string(0) == b"ok"


@pytest.mark.parametrize("H,W", [(256, 256), (1080, 1920), (2160, 3840), (480, 640), (720, 1280), (8, 8),
                                 (16, 16), (90, 120), (768, 1024), (600, 800), (450, 600), (81, 54),
                                 (4096, 8192), (1000, 1920)])
def test_config_sizes_supported(L, H, W):
    assert L.ils_size_supported(H, W) == 1


@pytest.mark.parametrize("H,W", [(1080, 1921), (7, 8), (1, 8), (8, 1), (1080, 14), (1000, 1918), (543, 1024),
                                 (4374, 16), (16, 8194), (8192, 8), (8, 2)])
def test_unsupported_sizes(L, H, W):
    assert L.ils_size_supported(H, W) == 0


def test_every_235_smooth_length_up_to_4096_is_supported(L):
    def smooth(n):
        for q in (2, 3, 5):
            while n % q == 0:
                n //= q
        return n == 1
    for n in range(0, 4200):
        assert L.ils_length_supported(n) == (1 if (2 <= n <= 4096 and smooth(n)) else 0), n


def test_compiled_lengths_are_235_smooth(L):
    for n in range(1, 2200):
        if L.ils_length_supported(n):
            m = n
            for q in (2, 3, 5):
                while m % q == 0:
                    m //= q
            assert m == 1, n


@pytest.mark.parametrize("args,code", [
    ((1080, 1920, 3, 1.0, 0.8, 1e-4, 4), 0),
    ((1080, 1920, 3, 0.0, 0.8, 1e-4, 4), 0),
    ((1080, 1920, 3, 1.0, 2.0, 1e-4, 0), 0),
    ((1080, 1920, 0, 1.0, 0.8, 1e-4, 4), -1),
    ((1080, 1920, 3, -1.0, 0.8, 1e-4, 4), -1),
    ((1080, 1920, 3, math.nan, 0.8, 1e-4, 4), -1),
    ((1080, 1920, 3, math.inf, 0.8, 1e-4, 4), -1),
    ((1080, 1920, 3, 1.0, 0.0, 1e-4, 4), -1),
    ((1080, 1920, 3, 1.0, 2.5, 1e-4, 4), -1),
    ((1080, 1920, 3, 1.0, math.nan, 1e-4, 4), -1),
    ((1080, 1920, 3, 1.0, 0.8, 0.0, 4), -1),
    ((1080, 1920, 3, 1.0, 0.8, -1e-4, 4), -1),
    ((1080, 1920, 3, 1.0, 0.8, 1e-4, -1), -1),
    ((1, 1920, 3, 1.0, 0.8, 1e-4, 4), -1),
    ((1080, 1921, 3, 1.0, 0.8, 1e-4, 4), -2),
    ((1001, 1920, 3, 1.0, 0.8, 1e-4, 4), -2),
])
def test_check_args(L, args, code):
    assert L.ils_check_args(*args) == code


def test_null_plan_and_pointers_rejected(L):
    assert L.ils_smooth(None, None, 8, 8, 1, 1.0, 0.8, 1e-4, 4, None) == -1
    assert L.ils_iterate_from(None, None, None, 8, 8, 1, 1.0, 0.8, 1e-4, 1, None) == -1
    assert L.ils_smooth_batch(None, None, 1) == -1
    assert L.ils_plan_destroy(None) == 0
    assert L.ils_plan_set_stream(None, None) == -1
    assert L.ils_last_error(None) == -1
    assert L.ils_rms_diff(None, None, None, None, 1, None) == -1
    assert L.ils_debug_rhs_spectrum(None, None, None, 8, 8, 1, 1.0, 0.8, 1e-4, None) == -1
    assert L.ils_enqueue_pass(None, 1, None, None, 8, 8, 1, 1.0, 0.8, 1e-4) == -1


def test_plan_create_rejects_bad_arguments_before_hip(L):
    h = ctypes.c_void_p()
    assert L.ils_plan_create(None, 8, 8, 1, 1, None, 0, None, 0) == -1
    assert L.ils_plan_create(ctypes.byref(h), 1, 8, 1, 1, None, 0, None, 0) == -1
    assert L.ils_plan_create(ctypes.byref(h), 8, 8, 1, 1, None, 1 << 30, None, 0) == -3
    assert L.ils_plan_create(ctypes.byref(h), 8, 8, 1, 1, ctypes.c_void_p(4096 + 8), 1 << 30, None, 0) == -3
    assert L.ils_plan_create(ctypes.byref(h), 8, 8, 1, 1, ctypes.c_void_p(4096), 16, None, 0) == -3
    # the workspace must hold one frame of the largest size (batches are checked per call)
    one = L.ils_workspace_bytes(1080, 1920, 3, 1)
    assert L.ils_plan_create(ctypes.byref(h), 1080, 1920, 3, 8, ctypes.c_void_p(4096), one - 256, None, 0) == -3
    assert L.ils_plan_create(ctypes.byref(h), 8, 8, 1, 1, ctypes.c_void_p(4096), 1 << 30, None, 7) == -1
    assert h.value is None


def test_workspace_bytes(L):
    one = L.ils_workspace_bytes(1080, 1920, 3, 1)
    # two half spectra, rows padded to 976 complex values, plus the 1 MiB header
    assert one == (1 << 20) + 2 * 3 * 1080 * 976 * 8
    assert L.ils_workspace_bytes(1080, 1920, 3, 4) == (1 << 20) + 4 * 2 * 3 * 1080 * 976 * 8
    assert L.ils_workspace_bytes(0, 1920, 3, 1) == 0
    from paper_2003_07504_amd._lib import IlsFrame
    arr = (IlsFrame * 2)()
    arr[0] = IlsFrame(None, None, 480, 640, 1, 1.0, 0.8, 1e-4, 4, None)
    arr[1] = IlsFrame(None, None, 1080, 1920, 3, 1.0, 0.8, 1e-4, 4, None)
    assert L.ils_batch_workspace_bytes(arr, 2) == (1 << 20) + 2 * 480 * 336 * 8 + 2 * 3 * 1080 * 976 * 8


@pytest.mark.parametrize("H,W,nr,nc", [(1080, 1920, 6, 4), (2160, 3840, 3, 2), (256, 256, 1, 1), (480, 640, 1, 4),
                                       (768, 1024, 1, 1), (450, 600, 1, 1)])
def test_shape_variants(L, H, W, nr, nc):
    from paper_2003_07504_amd import ils
    assert ils.shape_variants(H, W) == (nr, nc)


def test_shape_entry_points_reject_bad_arguments(L):
    r, c = ctypes.c_int(), ctypes.c_int()
    assert L.ils_shape_variants(1080, 1921, ctypes.byref(r), ctypes.byref(c)) == -2
    assert L.ils_shape_variants(1080, 1920, None, None) == -1
    assert L.ils_plan_tune(None, 1080, 1920, 3, ctypes.byref(r), ctypes.byref(c)) == -1
    assert L.ils_plan_set_shapes(None, 1080, 1920, 3, 0, 0) == -1


def test_frame_struct_layout_matches_c(tmp_path):
    """ctypes mirror of ils_frame has the C compiler's size and offsets."""
    from paper_2003_07504_amd._lib import IlsFrame
    src = tmp_path / "layout.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "ils.h"\n'
                   'int main(void) { printf("%zu %zu %zu %zu %zu\\n", sizeof(ils_frame), '
                   'offsetof(ils_frame, N), offsetof(ils_frame, u0), offsetof(ils_frame, penalty), '
                   'offsetof(ils_frame, gamma)); return 0; }\n')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    assert got == [ctypes.sizeof(IlsFrame), IlsFrame.N.offset, IlsFrame.u0.offset, IlsFrame.penalty.offset,
                   IlsFrame.gamma.offset]


def test_welsch_entry_point_rejects_null_plan(L):
    assert L.ils_smooth_welsch(None, None, 8, 8, 1, 20.0, 0.04, 10, None) == -1


def test_application_entry_points_reject_bad_arguments(L):
    assert L.ils_detail_enhance(None, None, 8, 8, 1, 1.0, 0.8, 1e-4, 4, 3.0, None) == -1
    assert L.ils_smooth_luminance(None, None, 8, 8, 1.0, 0.8, 1e-4, 4, 0.0, None) == -1
    assert L.ils_energy(None, None, None, 8, 8, 1, 1.0, 0.8, 1e-4, None) == -1
    assert L.ils_energy_welsch(None, None, None, 8, 8, 1, 1.0, 0.04, None) == -1
    assert L.ils_luminance_workspace_bytes(1080, 1920) == (1 << 20) + 1080 * 976 * 16 + 2 * 1080 * 1920 * 4
    assert L.ils_luminance_workspace_bytes(1080, 1921) == 0
    assert L.ils_luminance_workspace_bytes(1080, 1920) <= L.ils_workspace_bytes(1080, 1920, 3, 1)


def test_iterate_from_c_rejects_null_plan(L):
    assert L.ils_iterate_from_c(None, None, None, 8, 8, 1, 1.0, 0.8, 1e-4, 201.0, 4, None) == -1


def test_tone_map_rejects_null_plan(L):
    assert L.ils_tone_map(None, None, 8, 8, 10.0, 1.0, 1e-4, 4, 100.0, 1.0, None) == -1
