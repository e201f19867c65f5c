"""Python binding of the ILS library: argument marshalling only.

Every step of the smoothing runs in the HIP kernels of libils.so; PyTorch
provides device memory (the workspace and the images) and the stream.
"""
from __future__ import annotations

import ctypes
from typing import NamedTuple, Sequence

import torch

from ._lib import PENALTY_CHARBONNIER, PENALTY_WELSCH, IlsFrame, check, load

__all__ = ["Plan", "smooth", "size_supported", "workspace_bytes"]


def _as_chw(t: torch.Tensor, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on a GPU device")
    if t.dtype != torch.float32:
        raise ValueError(f"{name} must be float32")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.dim() == 2:
        return t.unsqueeze(0)
    if t.dim() != 3:
        raise ValueError(f"{name} must be (H, W) or (C, H, W)")
    return t


def size_supported(H: int, W: int) -> bool:
    return bool(load().ils_size_supported(int(H), int(W)))


def workspace_bytes(max_H: int, max_W: int, max_C: int = 3, max_frames: int = 1) -> int:
    return int(load().ils_workspace_bytes(max_H, max_W, max_C, max_frames))


def _stream_ptr(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


class Plan:
    """A plan and its workspace for frames up to max_H x max_W x max_C;
    max_frames frames may be resident in one batched call."""

    def __init__(self, max_H: int, max_W: int, max_C: int = 3, max_frames: int = 1, device=None,
                 ws_bytes: int | None = None, graph: bool = True):
        self._lib = load()
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        need = int(self._lib.ils_workspace_bytes(max_H, max_W, max_C, max_frames))
        if need == 0:
            raise ValueError("invalid plan limits")
        # default: room for max_frames frames of the largest size; a caller that
        # knows its batches may pass a smaller ws_bytes (at least one frame)
        ws_bytes = need if ws_bytes is None else max(int(ws_bytes),
                                                      int(self._lib.ils_workspace_bytes(max_H, max_W, max_C, 1)))
        self.workspace = torch.empty(ws_bytes, dtype=torch.uint8, device=self.device)
        self.max_H, self.max_W, self.max_C, self.max_frames = max_H, max_W, max_C, max_frames
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            check(self._lib.ils_plan_create(ctypes.byref(h), max_H, max_W, max_C, max_frames,
                                            ctypes.c_void_p(self.workspace.data_ptr()), ws_bytes,
                                            ctypes.c_void_p(_stream_ptr(self.device)), 0 if graph else 1),
                  "ils_plan_create")
        self._h = h

    # -- lifetime ----------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            torch.cuda.synchronize(self.device)
            self._lib.ils_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _bind_stream(self):
        check(self._lib.ils_plan_set_stream(self._h, ctypes.c_void_p(_stream_ptr(self.device))),
              "ils_plan_set_stream")

    def set_persistent(self, on: bool) -> None:
        """Use (True, the default) or not the single-launch pass sequence of
        the sizes compiled with one."""
        check(self._lib.ils_plan_set_persistent(self._h, 1 if on else 0), "ils_plan_set_persistent")

    def last_error(self) -> int:
        return int(self._lib.ils_last_error(self._h))

    PASS_KINDS = ("row_first", "row_mid", "row_final", "column")

    def profile_begin(self):
        check(self._lib.ils_profile_begin(self._h), "ils_profile_begin")

    def profile_end(self) -> dict:
        """{kind: (total_ms, launches)} for the launches since profile_begin."""
        tot = (ctypes.c_double * 4)()
        cnt = (ctypes.c_int * 4)()
        check(self._lib.ils_profile_end(self._h, tot, cnt), "ils_profile_end")
        return {k: (tot[i], cnt[i]) for i, k in enumerate(self.PASS_KINDS)}

    def enqueue_pass(self, kind: str, f: torch.Tensor, lam: float, p: float, eps: float = 1e-4,
                     out: torch.Tensor | None = None) -> None:
        """Enqueue one launch of one pass kind (see PASS_KINDS) of the
        sequence smooth() runs for f, on the workspace spectra (timing only:
        the spectra are left meaningless; the final pass writes out)."""
        fc = _as_chw(f, "f")
        oc = _as_chw(out if out is not None else torch.empty_like(f), "out")
        C, H, W = fc.shape
        self._bind_stream()
        check(self._lib.ils_enqueue_pass(self._h, self.PASS_KINDS.index(kind), ctypes.c_void_p(fc.data_ptr()),
                                         ctypes.c_void_p(oc.data_ptr()), H, W, C, float(lam), float(p),
                                         float(eps)), "ils_enqueue_pass")

    # -- tile shapes -------------------------------------------------------
    def tune(self, H: int, W: int, C: int) -> tuple[int, int]:
        """Time the tile shapes for this size now (if not yet) and return the
        chosen (row shape, column shape) indices."""
        r, c = ctypes.c_int(), ctypes.c_int()
        self._bind_stream()
        check(self._lib.ils_plan_tune(self._h, H, W, C, ctypes.byref(r), ctypes.byref(c)), "ils_plan_tune")
        return r.value, c.value

    def set_shapes(self, H: int, W: int, C: int, row_shape: int, col_shape: int) -> None:
        check(self._lib.ils_plan_set_shapes(self._h, H, W, C, int(row_shape), int(col_shape)), "ils_plan_set_shapes")

    # -- smoothing ---------------------------------------------------------
    def smooth(self, f: torch.Tensor, lam: float, p: float, eps: float = 1e-4, N: int = 4,
               out: torch.Tensor | None = None) -> torch.Tensor:
        """u^N of Algorithm 1 for a (H, W) or (C, H, W) float32 GPU tensor."""
        fc = _as_chw(f, "f")
        out = torch.empty_like(f) if out is None else out
        oc = _as_chw(out, "out")
        if oc.shape != fc.shape:
            raise ValueError("out must have the shape of f")
        C, H, W = fc.shape
        self._bind_stream()
        check(self._lib.ils_smooth(self._h, ctypes.c_void_p(fc.data_ptr()), H, W, C, float(lam), float(p),
                                   float(eps), int(N), ctypes.c_void_p(oc.data_ptr())), "ils_smooth")
        return out

    def smooth_welsch(self, f: torch.Tensor, lam: float, gamma: float, N: int = 10,
                      out: torch.Tensor | None = None) -> torch.Tensor:
        """u^N of Algorithm 1 with the Welsch penalty (Sec. 5, c = 2)."""
        fc = _as_chw(f, "f")
        out = torch.empty_like(f) if out is None else out
        oc = _as_chw(out, "out")
        if oc.shape != fc.shape:
            raise ValueError("out must have the shape of f")
        C, H, W = fc.shape
        self._bind_stream()
        check(self._lib.ils_smooth_welsch(self._h, ctypes.c_void_p(fc.data_ptr()), H, W, C, float(lam),
                                          float(gamma), int(N), ctypes.c_void_p(oc.data_ptr())),
              "ils_smooth_welsch")
        return out

    def detail_enhance(self, f: torch.Tensor, lam: float, p: float, eps: float = 1e-4, N: int = 4, k: float = 3.0,
                       out: torch.Tensor | None = None) -> torch.Tensor:
        """u + k (f - u) with u = u^N of Algorithm 1 (blend fused into the final pass)."""
        fc = _as_chw(f, "f")
        out = torch.empty_like(f) if out is None else out
        oc = _as_chw(out, "out")
        if oc.shape != fc.shape:
            raise ValueError("out must have the shape of f")
        C, H, W = fc.shape
        self._bind_stream()
        check(self._lib.ils_detail_enhance(self._h, ctypes.c_void_p(fc.data_ptr()), H, W, C, float(lam), float(p),
                                           float(eps), int(N), float(k), ctypes.c_void_p(oc.data_ptr())),
              "ils_detail_enhance")
        return out

    def smooth_luminance(self, f: torch.Tensor, lam: float, p: float, eps: float = 1e-4, N: int = 4,
                         k: float = 0.0, out: torch.Tensor | None = None) -> torch.Tensor:
        """Luminance-only smoothing of a (3, H, W) RGB frame (Sec. 3.4, option I)."""
        fc = _as_chw(f, "f")
        if fc.shape[0] != 3:
            raise ValueError("smooth_luminance needs a (3, H, W) RGB frame")
        out = torch.empty_like(f) if out is None else out
        oc = _as_chw(out, "out")
        if oc.shape != fc.shape:
            raise ValueError("out must have the shape of f")
        _, H, W = fc.shape
        self._bind_stream()
        check(self._lib.ils_smooth_luminance(self._h, ctypes.c_void_p(fc.data_ptr()), H, W, float(lam), float(p),
                                             float(eps), int(N), float(k), ctypes.c_void_p(oc.data_ptr())),
              "ils_smooth_luminance")
        return out

    def tone_map(self, f: torch.Tensor, lam: float = 10.0, p: float = 1.0, eps: float = 1e-4, N: int = 4,
                 contrast: float = 100.0, detail: float = 1.0, out: torch.Tensor | None = None) -> torch.Tensor:
        """Single-scale HDR tone mapping of a (3, H, W) linear RGB frame on log luminance."""
        fc = _as_chw(f, "f")
        if fc.shape[0] != 3:
            raise ValueError("tone_map needs a (3, H, W) RGB frame")
        out = torch.empty_like(f) if out is None else out
        oc = _as_chw(out, "out")
        if oc.shape != fc.shape:
            raise ValueError("out must have the shape of f")
        _, H, W = fc.shape
        self._bind_stream()
        check(self._lib.ils_tone_map(self._h, ctypes.c_void_p(fc.data_ptr()), H, W, float(lam), float(p), float(eps),
                                     int(N), float(contrast), float(detail), ctypes.c_void_p(oc.data_ptr())),
              "ils_tone_map")
        return out

    def tone_map_multiscale(self, f: torch.Tensor, lams: Sequence[float] = (0.125, 1.0, 8.0), p: float = 1.0,
                            eps: float = 1e-4, N: int = 4, contrast: float = 100.0,
                            weights: Sequence[float] = (1.0, 1.0, 1.0),
                            out: torch.Tensor | None = None) -> torch.Tensor:
        """Multi-scale HDR tone mapping of a (3, H, W) linear RGB frame on log
        luminance (one smoothing of log Y per lambda, detail layers between
        successive levels kept times `weights`)."""
        fc = _as_chw(f, "f")
        if fc.shape[0] != 3:
            raise ValueError("tone_map_multiscale needs a (3, H, W) RGB frame")
        if len(lams) != len(weights):
            raise ValueError("one weight per scale")
        out = torch.empty_like(f) if out is None else out
        oc = _as_chw(out, "out")
        if oc.shape != fc.shape:
            raise ValueError("out must have the shape of f")
        _, H, W = fc.shape
        K = len(lams)
        need = int(self._lib.ils_tone_map_multiscale_workspace_bytes(H, W, K))
        if need == 0 or need > self.workspace.numel():
            raise ValueError(f"the plan's workspace holds {self.workspace.numel()} bytes; multi-scale tone mapping "
                             f"of {H}x{W} with {K} scales needs {need}")
        la = (ctypes.c_float * K)(*[float(v) for v in lams])
        wa = (ctypes.c_float * K)(*[float(v) for v in weights])
        self._bind_stream()
        check(self._lib.ils_tone_map_multiscale(self._h, ctypes.c_void_p(fc.data_ptr()), H, W, la, wa, K, float(p),
                                                float(eps), int(N), float(contrast), ctypes.c_void_p(oc.data_ptr())),
              "ils_tone_map_multiscale")
        return out

    def energy(self, f: torch.Tensor, u: torch.Tensor, lam: float, p: float | None = None, eps: float = 1e-4,
               gamma: float | None = None) -> torch.Tensor:
        """Eq. (1) energy (float64 GPU scalar tensor): Charbonnier with p, or
        Welsch when gamma is given."""
        fc = _as_chw(f, "f")
        uc = _as_chw(u, "u")
        if uc.shape != fc.shape:
            raise ValueError("u must have the shape of f")
        C, H, W = fc.shape
        e = torch.empty((), dtype=torch.float64, device=self.device)
        self._bind_stream()
        if gamma is not None:
            check(self._lib.ils_energy_welsch(self._h, ctypes.c_void_p(fc.data_ptr()), ctypes.c_void_p(uc.data_ptr()),
                                              H, W, C, float(lam), float(gamma), ctypes.c_void_p(e.data_ptr())),
                  "ils_energy_welsch")
        else:
            check(self._lib.ils_energy(self._h, ctypes.c_void_p(fc.data_ptr()), ctypes.c_void_p(uc.data_ptr()),
                                       H, W, C, float(lam), float(p), float(eps), ctypes.c_void_p(e.data_ptr())),
                  "ils_energy")
        return e

    def iterate_from(self, f: torch.Tensor, u0: torch.Tensor, lam: float, p: float, eps: float = 1e-4,
                     N: int = 1, out: torch.Tensor | None = None, c: float | None = None) -> torch.Tensor:
        """N iterations of Eqs. (7)-(9) from u^0 = u0 with data term f (c = c0
        unless c is given; c >= c0)."""
        fc = _as_chw(f, "f")
        uc = _as_chw(u0, "u0")
        if uc.shape != fc.shape:
            raise ValueError("u0 must have the shape of f")
        out = torch.empty_like(f) if out is None else out
        oc = _as_chw(out, "out")
        C, H, W = fc.shape
        self._bind_stream()
        if c is not None:
            check(self._lib.ils_iterate_from_c(self._h, ctypes.c_void_p(fc.data_ptr()), ctypes.c_void_p(uc.data_ptr()),
                                               H, W, C, float(lam), float(p), float(eps), float(c), int(N),
                                               ctypes.c_void_p(oc.data_ptr())), "ils_iterate_from_c")
            return out
        check(self._lib.ils_iterate_from(self._h, ctypes.c_void_p(fc.data_ptr()), ctypes.c_void_p(uc.data_ptr()),
                                         H, W, C, float(lam), float(p), float(eps), int(N),
                                         ctypes.c_void_p(oc.data_ptr())), "ils_iterate_from")
        return out

    def smooth_batch(self, frames: Sequence[tuple], outs: Sequence[torch.Tensor] | None = None,
                     u0s: Sequence[torch.Tensor | None] | None = None) -> list[torch.Tensor]:
        """frames: sequence of (f, lam, p, eps, N) for the Charbonnier penalty
        or Welsch(f, lam, gamma, N) frames; returns the outputs."""
        n = len(frames)
        arr = (IlsFrame * n)()
        keep = []
        res = []
        for i, fr in enumerate(frames):
            if isinstance(fr, Welsch):
                f, lam, N = fr.f, fr.lam, fr.N
                p, eps, pen, gamma = 1.0, 1.0, PENALTY_WELSCH, float(fr.gamma)
            else:
                f, lam, p, eps, N = fr
                pen, gamma = PENALTY_CHARBONNIER, 0.0
            fc = _as_chw(f, f"frames[{i}].f")
            o = torch.empty_like(f) if outs is None else outs[i]
            oc = _as_chw(o, f"outs[{i}]")
            u0 = None if u0s is None else u0s[i]
            uc = None if u0 is None else _as_chw(u0, f"u0s[{i}]")
            C, H, W = fc.shape
            arr[i] = IlsFrame(fc.data_ptr(), oc.data_ptr(), H, W, C, float(lam), float(p), float(eps), int(N),
                              0 if uc is None else uc.data_ptr(), pen, gamma)
            keep.append((fc, oc, uc))
            res.append(o)
        need = int(self._lib.ils_batch_workspace_bytes(arr, n))
        if need > self.workspace.numel():
            raise ValueError(f"batch needs {need} workspace bytes, plan has {self.workspace.numel()}")
        self._bind_stream()
        check(self._lib.ils_smooth_batch(self._h, arr, n), "ils_smooth_batch")
        return res

    def rms_diff(self, a: Sequence[torch.Tensor], b: Sequence[torch.Tensor]) -> torch.Tensor:
        """Per-pair RMS of (a_i - b_i) as a float32 GPU tensor of length n."""
        n = len(a)
        pa = (ctypes.c_void_p * n)(*[t.data_ptr() for t in a])
        pb = (ctypes.c_void_p * n)(*[t.data_ptr() for t in b])
        cnt = (ctypes.c_longlong * n)(*[t.numel() for t in a])
        for x, y in zip(a, b):
            if x.shape != y.shape or x.dtype != torch.float32 or y.dtype != torch.float32:
                raise ValueError("rms_diff needs float32 pairs of equal shape")
            if not (x.is_contiguous() and y.is_contiguous()):
                raise ValueError("rms_diff needs contiguous tensors")
        out = torch.empty(n, dtype=torch.float32, device=self.device)
        self._bind_stream()
        check(self._lib.ils_rms_diff(self._h, pa, pb, cnt, n, ctypes.c_void_p(out.data_ptr())), "ils_rms_diff")
        return out

    # -- single passes ----------------------------------------------------
    def debug_rhs_spectrum(self, f, u0, lam, p, eps=1e-4) -> torch.Tensor:
        fc = _as_chw(f, "f")
        uc = _as_chw(u0, "u0")
        C, H, W = fc.shape
        spec = torch.empty((C, H, W // 2 + 1), dtype=torch.complex64, device=f.device)
        self._bind_stream()
        check(self._lib.ils_debug_rhs_spectrum(self._h, ctypes.c_void_p(fc.data_ptr()), ctypes.c_void_p(uc.data_ptr()),
                                               H, W, C, float(lam), float(p), float(eps),
                                               ctypes.c_void_p(spec.data_ptr())), "ils_debug_rhs_spectrum")
        return spec

    def debug_column_solve(self, spec_in: torch.Tensor, W: int, lam, p, eps=1e-4) -> torch.Tensor:
        if spec_in.dtype != torch.complex64 or not spec_in.is_contiguous() or spec_in.dim() != 3:
            raise ValueError("spec_in must be contiguous complex64 (C, H, W/2+1)")
        C, H, Wh = spec_in.shape
        if Wh != W // 2 + 1:
            raise ValueError("spec_in width must be W/2+1")
        out = torch.empty_like(spec_in)
        self._bind_stream()
        check(self._lib.ils_debug_column_solve(self._h, ctypes.c_void_p(spec_in.data_ptr()), H, W, C, float(lam),
                                               float(p), float(eps), ctypes.c_void_p(out.data_ptr())),
              "ils_debug_column_solve")
        return out

    def debug_row_inverse(self, spec: torch.Tensor, W: int) -> torch.Tensor:
        if spec.dtype != torch.complex64 or not spec.is_contiguous() or spec.dim() != 3:
            raise ValueError("spec must be contiguous complex64 (C, H, W/2+1)")
        C, H, Wh = spec.shape
        out = torch.empty((C, H, W), dtype=torch.float32, device=spec.device)
        self._bind_stream()
        check(self._lib.ils_debug_row_inverse(self._h, ctypes.c_void_p(spec.data_ptr()), H, W, C,
                                              ctypes.c_void_p(out.data_ptr())), "ils_debug_row_inverse")
        return out


class Welsch(NamedTuple):
    """A frame of a batched call smoothed with the Welsch penalty."""
    f: torch.Tensor
    lam: float
    gamma: float
    N: int = 10


def shape_variants(H: int, W: int) -> tuple[int, int]:
    """Number of compiled (row, column) tile shapes for a supported size."""
    r, c = ctypes.c_int(), ctypes.c_int()
    check(load().ils_shape_variants(H, W, ctypes.byref(r), ctypes.byref(c)), "ils_shape_variants")
    return r.value, c.value


_plans: dict = {}


def smooth(f: torch.Tensor, lam: float, p: float, eps: float = 1e-4, N: int = 4,
           out: torch.Tensor | None = None) -> torch.Tensor:
    """One-call convenience: smooth with a plan cached per (device, size)."""
    fc = _as_chw(f, "f")
    C, H, W = fc.shape
    key = (f.device.index, H, W, C)
    plan = _plans.get(key)
    if plan is None:
        plan = _plans[key] = Plan(H, W, C, 1, device=f.device)
    return plan.smooth(f, lam, p, eps, N, out)
