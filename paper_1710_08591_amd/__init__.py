"""MI355X FFT beamformer: Python binding of libfftbf (torch tensors in, torch tensors out).

The functions here only check tensors and marshal pointers into the C ABI of
include/fftbf.h; every step of the beamformer runs in the library's HIP
kernels on the caller's current torch stream.  Importing this package does
not load the library; the first call does, and fails loudly if it has not
been built.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional

import numpy as np

from ._lib import (bf_server_stats, BF_OK, BF_ERR_INVALID_ARGUMENT, BF_ERR_UNSUPPORTED, BF_ERR_OUT_OF_MEMORY,
                   BF_ERR_DEVICE, BF_ERR_REJECTED, BF_ERR_EVICTED, BF_ERR_NOT_READY,
                   BF_PREC_FP32, BF_PREC_FP16_MFMA, BF_PREC_FP8_MFMA, BF_OUT_INTENSITY,
                   BF_OUT_COMPLEX, BFError, LibraryMissing, bf_plan_desc, check, lib)

__all__ = [
    "Plan", "plan_create", "plan_destroy", "beamform_fft", "form_tied_beams", "form_tied_beams_v",
    "accumulate_intensity", "Regrid", "Regrid2D", "localize", "Server", "lib", "BFError", "LibraryMissing",
    "BF_PREC_FP32", "BF_PREC_FP16_MFMA", "BF_PREC_FP8_MFMA", "BF_OUT_INTENSITY", "BF_OUT_COMPLEX",
]


def _torch():
    import torch
    return torch


def _stream_handle(stream=None) -> C.c_void_p:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t) -> C.c_void_p:
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def _need(t, dtype, name: str):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on the GPU")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


class Plan:
    """A beamforming plan: lattice geometry, precision, clamp table (bf_plan_create)."""

    def __init__(self, n_ew: int = 4, n_ns: int = 16, m_ew: Optional[int] = None,
                 m_ns: Optional[int] = None, n_pol: int = 1, n_chan: int = 1, block: int = 16,
                 ns_select: Optional[np.ndarray] = None, pol_sum: bool = False,
                 precision: int = BF_PREC_FP32, d_over_lambda: Optional[np.ndarray] = None):
        m_ew = n_ew if m_ew is None else m_ew
        m_ns = 2 * n_ns if m_ns is None else m_ns
        keep = 0
        self._sel = None
        self._dl = None
        d = bf_plan_desc()
        d.n_ew, d.n_ns, d.m_ew, d.m_ns = n_ew, n_ns, m_ew, m_ns
        d.n_pol, d.n_chan, d.block = n_pol, n_chan, block
        d.pol_sum, d.precision = int(bool(pol_sum)), int(precision)
        if ns_select is not None:
            self._sel = np.ascontiguousarray(ns_select, dtype=np.int32)
            if self._sel.ndim != 2 or self._sel.shape[0] != n_chan:
                raise ValueError("ns_select must be [n_chan][n_ns_keep]")
            keep = self._sel.shape[1]
            d.ns_select = self._sel.ctypes.data_as(C.POINTER(C.c_int32))
        if d_over_lambda is not None:
            self._dl = np.ascontiguousarray(d_over_lambda, dtype=np.float64)
            if self._dl.shape != (n_chan, 2):
                raise ValueError("d_over_lambda must be [n_chan][2]")
            d.d_over_lambda = self._dl.ctypes.data_as(C.POINTER(C.c_double))
        d.n_ns_keep = keep
        self.desc = d
        self.n_ew, self.n_ns, self.m_ew, self.m_ns = n_ew, n_ns, m_ew, m_ns
        self.n_pol, self.n_chan, self.block = n_pol, n_chan, block
        self.keep = keep if keep else m_ns
        self.pol_sum = bool(pol_sum)
        self.precision = int(precision)
        h = C.c_void_p()
        check(lib().bf_plan_create(C.byref(d), C.byref(h)), "bf_plan_create")
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            check(lib().bf_plan_destroy(self.handle), "bf_plan_destroy")
            self.handle = None

    def __del__(self):
        try:
            if getattr(self, "handle", None):
                lib().bf_plan_destroy(self.handle)
                self.handle = None
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def volts_shape(self, n_time: int):
        return (n_time, self.n_chan, self.n_pol, self.n_ns, self.n_ew)

    def out_shape(self, n_time: int, kind: int = BF_OUT_INTENSITY):
        if kind == BF_OUT_COMPLEX:
            return (n_time, self.n_chan, self.n_pol, self.m_ew, self.m_ns)
        nb = n_time // self.block
        if self.pol_sum:
            return (nb, self.n_chan, self.m_ew, self.keep)
        return (nb, self.n_chan, self.n_pol, self.m_ew, self.keep)


def plan_create(**kw) -> Plan:
    return Plan(**kw)


def plan_destroy(plan: Plan) -> None:
    plan.close()


def beamform_fft(plan: Plan, volts, taper=None, kind: int = BF_OUT_INTENSITY, out=None, stream=None,
                 gains=None):
    """FFT beams of ``volts`` (uint8 [t][chan][pol][n_ns][n_ew]) -> intensities or complex beams.

    taper: real float32 [n_ns][n_ew] weights (bf_beamform_fft); gains: complex64
    [n_ns][n_ew] per-antenna gains (bf_beamform_fft_gains).  At most one."""
    torch = _torch()
    _need(volts, torch.uint8, "volts")
    n_time = volts.shape[0]
    if tuple(volts.shape) != plan.volts_shape(n_time):
        raise ValueError(f"volts shape {tuple(volts.shape)} != {plan.volts_shape(n_time)}")
    if taper is not None and gains is not None:
        raise ValueError("pass a real taper or complex gains, not both")
    if taper is not None:
        _need(taper, torch.float32, "taper")
        if tuple(taper.shape) != (plan.n_ns, plan.n_ew):
            raise ValueError("taper must be [n_ns][n_ew]")
    if gains is not None:
        _need(gains, torch.complex64, "gains")
        if tuple(gains.shape) != (plan.n_ns, plan.n_ew):
            raise ValueError("gains must be [n_ns][n_ew]")
    shape = plan.out_shape(n_time, kind)
    dt = torch.complex64 if kind == BF_OUT_COMPLEX else torch.float32
    if out is None:
        out = torch.empty(shape, dtype=dt, device=volts.device)
    else:
        _need(out, dt, "out")
        if tuple(out.shape) != shape:
            raise ValueError(f"out shape {tuple(out.shape)} != {shape}")
    if gains is not None:
        check(lib().bf_beamform_fft_gains(plan.handle, _ptr(volts), n_time, _ptr(gains), kind, _ptr(out),
                                          _stream_handle(stream)), "bf_beamform_fft_gains")
    else:
        check(lib().bf_beamform_fft(plan.handle, _ptr(volts), n_time, _ptr(taper), kind, _ptr(out),
                                    _stream_handle(stream)), "bf_beamform_fft")
    return out


def _dircos(dircos):
    torch = _torch()
    _need(dircos, torch.float64, "dircos")
    if dircos.ndim != 2 or dircos.shape[1] != 2:
        raise ValueError("dircos must be [n_point][2]")
    return dircos.shape[0]


def form_tied_beams(plan: Plan, fft_beams, chan_lo: int, n_chan_sub: int, dircos,
                    kind: int = BF_OUT_INTENSITY, out=None, stream=None):
    """Tied-array beams interpolated from complex FFT beams [t][chan][pol][m_ew][m_ns]."""
    torch = _torch()
    _need(fft_beams, torch.complex64, "fft_beams")
    n_time = fft_beams.shape[0]
    if tuple(fft_beams.shape) != (n_time, plan.n_chan, plan.n_pol, plan.m_ew, plan.m_ns):
        raise ValueError("fft_beams must be [t][n_chan][n_pol][m_ew][m_ns]")
    n_point = _dircos(dircos)
    if kind == BF_OUT_COMPLEX:
        shape, dt = (n_time, n_chan_sub, plan.n_pol, n_point), torch.complex64
    elif plan.pol_sum:
        shape, dt = (n_time // plan.block, n_chan_sub, n_point), torch.float32
    else:
        shape, dt = (n_time // plan.block, n_chan_sub, plan.n_pol, n_point), torch.float32
    if out is None:
        out = torch.empty(shape, dtype=dt, device=fft_beams.device)
    else:
        _need(out, dt, "out")
        if tuple(out.shape) != shape:
            raise ValueError(f"out shape {tuple(out.shape)} != {shape}")
    check(lib().bf_form_tied_beams(plan.handle, _ptr(fft_beams), n_time, chan_lo, n_chan_sub, _ptr(dircos),
                                   n_point, kind, _ptr(out), _stream_handle(stream)), "bf_form_tied_beams")
    return out


def form_tied_beams_v_noalloc(plan: Plan, volts, chan_lo: int, n_chan_sub: int, dircos, out, taper=None,
                              stream=None):
    """form_tied_beams_v through bf_form_tied_beams_v_noalloc: the library's
    static device scratch as the workspace, no allocation in the call
    (``out`` must be given)."""
    torch = _torch()
    _need(volts, torch.uint8, "volts")
    n_time = volts.shape[0]
    if tuple(volts.shape) != plan.volts_shape(n_time):
        raise ValueError("volts shape does not match the plan")
    if taper is not None:
        _need(taper, torch.float32, "taper")
    n_point = _dircos(dircos)
    shape = ((n_time // plan.block, n_chan_sub, n_point) if plan.pol_sum
             else (n_time // plan.block, n_chan_sub, plan.n_pol, n_point))
    _need(out, torch.float32, "out")
    if tuple(out.shape) != shape:
        raise ValueError(f"out shape {tuple(out.shape)} != {shape}")
    check(lib().bf_form_tied_beams_v_noalloc(plan.handle, _ptr(volts), n_time, _ptr(taper), chan_lo, n_chan_sub,
                                             _ptr(dircos), n_point, _ptr(out), _stream_handle(stream)),
          "bf_form_tied_beams_v_noalloc")
    return out


def tied_workspace_size(plan: Plan, n_chan_sub: int, chunk_samples: int) -> int:
    """Bytes of workspace form_tied_beams_v needs per chunk of samples (other lattices than 4 x 16)."""
    return int(lib().bf_tied_workspace_size(plan.handle, n_chan_sub, chunk_samples))


def form_tied_beams_v(plan: Plan, volts, chan_lo: int, n_chan_sub: int, dircos, taper=None, out=None,
                      stream=None, workspace=None):
    """Tied-array beam intensities straight from voltages (FFT beams formed on chip).

    The 4 x 16 lattice (block a multiple of 16) runs one fused kernel.  Other
    lattices pass each chunk's complex FFT beams through ``workspace`` (a
    device tensor; by default one of up to 256 MiB, at least one block, is
    allocated here)."""
    torch = _torch()
    _need(volts, torch.uint8, "volts")
    n_time = volts.shape[0]
    if tuple(volts.shape) != plan.volts_shape(n_time):
        raise ValueError("volts shape does not match the plan")
    if taper is not None:
        _need(taper, torch.float32, "taper")
    n_point = _dircos(dircos)
    if plan.pol_sum:
        shape = (n_time // plan.block, n_chan_sub, n_point)
    else:
        shape = (n_time // plan.block, n_chan_sub, plan.n_pol, n_point)
    if out is None:
        out = torch.empty(shape, dtype=torch.float32, device=volts.device)
    else:
        _need(out, torch.float32, "out")
    if plan.n_ns == 16 and plan.m_ew == 4 and plan.block % 16 == 0:
        check(lib().bf_form_tied_beams_v(plan.handle, _ptr(volts), n_time, _ptr(taper), chan_lo, n_chan_sub,
                                         _ptr(dircos), n_point, _ptr(out), _stream_handle(stream)),
              "bf_form_tied_beams_v")
        return out
    if workspace is None:
        per_block = tied_workspace_size(plan, n_chan_sub, plan.block)
        n_blk = max(1, n_time // plan.block)
        nbytes = per_block * max(1, min(n_blk, (256 << 20) // max(per_block, 1)))
        workspace = torch.empty(max(nbytes, 16), dtype=torch.uint8, device=volts.device)
    check(lib().bf_form_tied_beams_v_ws(plan.handle, _ptr(volts), n_time, _ptr(taper), chan_lo, n_chan_sub,
                                        _ptr(dircos), n_point, _ptr(workspace),
                                        workspace.numel() * workspace.element_size(), _ptr(out),
                                        _stream_handle(stream)),
          "bf_form_tied_beams_v_ws")
    return out


def accumulate_intensity(z, block: int, out=None, add: bool = False, stream=None):
    """sum over blocks of |z|^2 for complex64 z [t][series] (bf_accumulate_intensity)."""
    torch = _torch()
    _need(z, torch.complex64, "z")
    if z.ndim != 2:
        raise ValueError("z must be [n_time][n_series]")
    n_time, n_series = z.shape
    shape = (n_time // block if block > 0 else 0, n_series)
    if out is None:
        if add:
            raise ValueError("add=True needs an existing out")
        out = torch.empty(shape, dtype=torch.float32, device=z.device)
    else:
        _need(out, torch.float32, "out")
        if tuple(out.shape) != shape:
            raise ValueError(f"out shape {tuple(out.shape)} != {shape}")
    check(lib().bf_accumulate_intensity(_ptr(z), n_time, n_series, block, int(add), _ptr(out),
                                        _stream_handle(stream)), "bf_accumulate_intensity")
    return out


def localize(plan: Plan, fft_intensity, n_window: int = 10, n_iter: int = 6, stream=None):
    """Newton localisation per row of unclamped FFT-beam intensities (bf_localize).

    Returns (sin_theta float64, peak float32), shaped like the intensities
    without their last (N-S beam) axis."""
    torch = _torch()
    _need(fft_intensity, torch.float32, "fft_intensity")
    shape = ((plan.n_chan, plan.m_ew, plan.m_ns) if plan.pol_sum
             else (plan.n_chan, plan.n_pol, plan.m_ew, plan.m_ns))
    if tuple(fft_intensity.shape[1:]) != shape:
        raise ValueError(f"fft_intensity must be [n_blk]{list(shape)}")
    n_blk = fft_intensity.shape[0]
    out_shape = (n_blk,) + shape[:-1]
    st = torch.empty(out_shape, dtype=torch.float64, device=fft_intensity.device)
    pk = torch.empty(out_shape, dtype=torch.float32, device=fft_intensity.device)
    check(lib().bf_localize(plan.handle, _ptr(fft_intensity), n_blk, int(n_window), int(n_iter), _ptr(st),
                            _ptr(pk), _stream_handle(stream)), "bf_localize")
    return st, pk


class Regrid:
    """Achromatic beams regridded from FFT-beam intensities (bf_regrid_*).

    window: optional real N-S window [n_ns] for the optimally windowed beam;
    n_taps: 0 for the exact dense kernel, 1..8 for the compact kernel."""

    def __init__(self, plan: Plan, sin_theta: np.ndarray, window: Optional[np.ndarray] = None, n_taps: int = 0):
        st = np.ascontiguousarray(sin_theta, dtype=np.float64).ravel()
        win = None
        if window is not None:
            win = np.ascontiguousarray(window, dtype=np.float64).ravel()
            if len(win) != plan.n_ns:
                raise ValueError("window must have n_ns entries")
        h = C.c_void_p()
        check(lib().bf_regrid_create(plan.handle, st.ctypes.data_as(C.c_void_p), len(st),
                                     None if win is None else win.ctypes.data_as(C.c_void_p), int(n_taps),
                                     C.byref(h)), "bf_regrid_create")
        self.handle = h
        self.n_target = len(st)
        # the plan's intensity layout: the polarisation axis is absent when it sums them
        self.plan_shape = ((plan.n_chan, plan.m_ew, plan.m_ns) if plan.pol_sum
                           else (plan.n_chan, plan.n_pol, plan.m_ew, plan.m_ns))

    def close(self):
        if getattr(self, "handle", None):
            lib().bf_regrid_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __call__(self, fft_intensity, out=None, stream=None):
        """Regrid [n_blk][n_chan]([n_pol])[m_ew][m_ns] intensities to [..][n_target]."""
        torch = _torch()
        _need(fft_intensity, torch.float32, "fft_intensity")
        n_blk = fft_intensity.shape[0]
        if tuple(fft_intensity.shape[1:]) != self.plan_shape:
            raise ValueError(f"fft_intensity must be [n_blk]{list(self.plan_shape)}")
        shape = (n_blk,) + self.plan_shape[:-1] + (self.n_target,)
        if out is None:
            out = torch.empty(shape, dtype=torch.float32, device=fft_intensity.device)
        else:
            _need(out, torch.float32, "out")
            if tuple(out.shape) != shape:
                raise ValueError(f"out shape {tuple(out.shape)} != {shape}")
        check(lib().bf_regrid_intensity(self.handle, _ptr(fft_intensity), n_blk, _ptr(out),
                                        _stream_handle(stream)), "bf_regrid_intensity")
        return out


class Regrid2D(Regrid):
    """Pointed beams at 2-D pointings from FFT-beam intensities of a plan with
    an E-W axis padded to 8 beams (bf_regrid_create_2d)."""

    def __init__(self, plan: Plan, dircos: np.ndarray):
        d = np.ascontiguousarray(dircos, dtype=np.float64)
        if d.ndim != 2 or d.shape[1] != 2:
            raise ValueError("dircos must be [n_point][2]")
        h = C.c_void_p()
        check(lib().bf_regrid_create_2d(plan.handle, d.ctypes.data_as(C.c_void_p), d.shape[0], C.byref(h)),
              "bf_regrid_create_2d")
        self.handle = h
        self.n_target = d.shape[0]
        self.plan_shape = ((plan.n_chan, plan.m_ew, plan.m_ns) if plan.pol_sum
                           else (plan.n_chan, plan.n_pol, plan.m_ew, plan.m_ns))

    def __call__(self, fft_intensity, out=None, stream=None):
        """Regrid [n_blk][n_chan]([n_pol])[8][m_ns] intensities to [n_blk][n_chan]([n_pol])[n_point]."""
        torch = _torch()
        _need(fft_intensity, torch.float32, "fft_intensity")
        n_blk = fft_intensity.shape[0]
        if tuple(fft_intensity.shape[1:]) != self.plan_shape:
            raise ValueError(f"fft_intensity must be [n_blk]{list(self.plan_shape)}")
        shape = (n_blk,) + self.plan_shape[:-2] + (self.n_target,)
        if out is None:
            out = torch.empty(shape, dtype=torch.float32, device=fft_intensity.device)
        else:
            _need(out, torch.float32, "out")
            if tuple(out.shape) != shape:
                raise ValueError(f"out shape {tuple(out.shape)} != {shape}")
        check(lib().bf_regrid_intensity(self.handle, _ptr(fft_intensity), n_blk, _ptr(out),
                                        _stream_handle(stream)), "bf_regrid_intensity")
        return out


class Server:
    """Tied-beam server over a device voltage ring (bf_server_*).

    ``plan`` must be an FP32 4 x 16 lattice plan with block 16.  Requests are
    admitted against ``hbm_budget`` bytes of device memory and executed by
    batched launches on the server's own stream; call ``pump()`` often.
    """

    def __init__(self, plan: Plan, ring_samples: int = 65536, hbm_budget: int = 16 << 30,
                 blocks_per_tile: int = 32, max_tiles_per_launch: int = 8192):
        h = C.c_void_p()
        check(lib().bf_server_create(plan.handle, ring_samples, hbm_budget, blocks_per_tile,
                                     max_tiles_per_launch, C.byref(h)), "bf_server_create")
        self.handle = h
        self.n_chan, self.n_pol = plan.n_chan, plan.n_pol
        self.ring_samples = ring_samples
        self._shapes = {}

    def close(self):
        if getattr(self, "handle", None):
            lib().bf_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def now(self) -> float:
        return lib().bf_server_now(self.handle)

    def ring(self):
        """(device pointer, ring_samples, head)."""
        p, n, h = C.c_void_p(), C.c_int64(), C.c_int64()
        check(lib().bf_server_ring(self.handle, C.byref(p), C.byref(n), C.byref(h)), "bf_server_ring")
        return p.value, n.value, h.value

    def advance(self, n_samples: int, src=None, force: bool = False) -> int:
        """Append samples (uint8 tensor [n][n_chan][n_pol][16][4] on the GPU, or None)."""
        if src is not None:
            _need(src, _torch().uint8, "src")
            if src.shape[0] != n_samples:
                raise ValueError("src must hold n_samples samples")
        return lib().bf_server_advance(self.handle, n_samples, _ptr(src), int(force), _stream_handle())

    def submit(self, dircos: np.ndarray, chan_lo: int, n_chan: int, n_time: int,
               arrival: Optional[float] = None) -> int:
        d = np.ascontiguousarray(dircos, dtype=np.float64)
        if d.ndim != 2 or d.shape[1] != 2:
            raise ValueError("dircos must be [n_point][2]")
        rid = C.c_int64()
        t = self.now() if arrival is None else float(arrival)
        st = lib().bf_server_submit(self.handle, d.shape[0], chan_lo, n_chan, n_time,
                                    d.ctypes.data_as(C.c_void_p), t, C.byref(rid))
        check(st, "bf_server_submit")
        self._shapes[rid.value] = (n_time // 16, n_chan, self.n_pol, d.shape[0])
        return rid.value

    def try_submit(self, dircos, chan_lo, n_chan, n_time, arrival=None):
        """Like submit, but returns (status, id) instead of raising."""
        try:
            return BF_OK, self.submit(dircos, chan_lo, n_chan, n_time, arrival)
        except BFError as e:
            return e.status, 0

    def pump(self) -> None:
        check(lib().bf_server_pump(self.handle), "bf_server_pump")

    def poll(self, rid: int):
        """(status, latency seconds): BF_OK when finished, BF_ERR_NOT_READY while running."""
        lat = C.c_double(-1.0)
        st = lib().bf_server_poll(self.handle, rid, C.byref(lat))
        return st, lat.value

    def result(self, rid: int):
        """Copy a finished request's intensities into a new tensor [blk][chan][pol][point]."""
        torch = _torch()
        out = torch.empty(self._shapes[rid], dtype=torch.float32, device="cuda")
        check(lib().bf_server_copy_result(self.handle, rid, _ptr(out), _stream_handle()), "bf_server_copy_result")
        return out

    def release(self, rid: int) -> int:
        st = lib().bf_server_release(self.handle, rid)
        if st == BF_OK:
            self._shapes.pop(rid, None)
        return st

    def cancel(self, rid: int) -> None:
        check(lib().bf_server_cancel(self.handle, rid), "bf_server_cancel")

    def stats(self) -> dict:
        s = bf_server_stats()
        check(lib().bf_server_stats_get(self.handle, C.byref(s)), "bf_server_stats_get")
        return {k: getattr(s, k) for k, _ in s._fields_}

    def wait(self, rid: int, timeout_s: float = 60.0):
        """Pump until the request finishes; returns (status, latency)."""
        import time
        t0 = time.perf_counter()
        while True:
            self.pump()
            st, lat = self.poll(rid)
            if st != BF_ERR_NOT_READY:
                return st, lat
            if time.perf_counter() - t0 > timeout_s:
                raise TimeoutError(f"request {rid} not finished after {timeout_s} s")
