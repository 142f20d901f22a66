"""Seeded synthetic workloads for the FFT beamformer.

This module creates inputs only.  It contains none of the beamforming
arithmetic (no decode, no transform, no squaring, no weights); both the
FP64 oracle and the GPU library take what it produces as plain inputs.

Every voltage byte is a pure integer function of (seed, t, chan, pol,
antenna), evaluated with 64-bit integer operations only, so the numpy
backend (used on the host for any slice) and the torch backend (used to
fill gigabytes directly in device memory) produce bit-identical bytes.

Signal model (Preliminaries, "Antennas and Visibilities", eq:feed): each
antenna sees receiver noise plus plane waves from point sources, the
source term carrying the phase e^{+i 2 pi u_a . n} with u_a the antenna
position in wavelengths.  On a lattice with spacing d the phase of
antenna (a_ew, a_ns) is 2 pi (a_ew y_ew + a_ns y_ns) with y = (d/lambda)
sin(theta) per axis.

Recipe (integer only):
  * hash: the 32-bit "lowbias32" integer hash (C. Wellons, "Prospecting
    for hash functions", 2018) keyed by (seed, stream, t) and indexed by
    (chan, pol, antenna).
  * noise: each component is popcount(16 random bits) - 8, a binomial
    B(16, 1/2) - 8 with sigma = 2 exactly, range [-8, 8].
  * source k: complex amplitude s_k(t, chan, pol) drawn the same way
    (sigma 2 per component), scaled by SNR_k / sqrt(n_ant) in Q12 fixed
    point, times a phasor from a 1024-entry Q14 cos/sin table indexed by
    the top 10 bits of the Q32 phase frac(a_ew y_ew + a_ns y_ns).
  * sum in Q26, round half up, clip to [-7, 7], pack as two's-complement
    nibbles: real part in the high nibble, imaginary in the low nibble.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence

import numpy as np

MASK32 = 0xFFFFFFFF
STREAM_NOISE = 1
STREAM_SOURCE = 2

# --------------------------------------------------------------------------
# integer hashing, identical for numpy int64 arrays and torch int64 tensors
# --------------------------------------------------------------------------


def _mul32(x, c: int):
    """(x * c) mod 2^32 for 0 <= x < 2^32, without int64 overflow."""
    c_lo = c & 0xFFFF
    c_hi = c >> 16
    return (x * c_lo + (((x * c_hi) & 0xFFFF) << 16)) & MASK32


def lowbias32(x):
    x = x ^ (x >> 16)
    x = _mul32(x, 0x7FEB352D)
    x = x ^ (x >> 15)
    x = _mul32(x, 0x846CA68B)
    x = x ^ (x >> 16)
    return x


def _popcount16(v):
    v = v - ((v >> 1) & 0x5555)
    v = (v & 0x3333) + ((v >> 2) & 0x3333)
    v = (v + (v >> 4)) & 0x0F0F
    return (v + (v >> 8)) & 0x1F


def _time_key(seed: int, stream: int, t):
    k = lowbias32((seed * 0x9E37 + stream * 0x85EB + 0x1234567) & MASK32)
    return lowbias32((t + k) & MASK32)


def _gauss_pair(x):
    """Two integer 'Gaussians' (sigma 2, range [-8, 8]) from 32 hash bits."""
    return _popcount16(x & 0xFFFF) - 8, _popcount16(x >> 16) - 8


# --------------------------------------------------------------------------
# workload description
# --------------------------------------------------------------------------


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    n_ew: int
    n_ns: int
    n_chan: int
    n_pol: int
    n_time: int
    m_ew: int
    m_ns: int
    block: int
    seed: int
    # sources: y_ew, y_ns per source for channel 0 geometry is derived from
    # direction cosines and the per-channel d/lambda table
    src_dircos: tuple = ()          # ((n_ew, n_ns), ...) direction cosines
    src_snr: tuple = ()             # amplitude SNR per source
    src_lattice: tuple = ()         # ((A_ew, A_ns), ...) lattice-aligned y = A/M
    dl_lo: float = 0.5              # d/lambda at the lowest channel
    dl_hi: float = 0.5              # d/lambda at the highest channel
    n_ns_keep: int = 0              # 0 -> no clamp (keep all m_ns beams)

    @property
    def n_ant(self) -> int:
        return self.n_ew * self.n_ns

    @property
    def frame_bytes(self) -> int:
        return self.n_ew * self.n_ns

    @property
    def keep(self) -> int:
        return self.n_ns_keep if self.n_ns_keep else self.m_ns

    @property
    def antenna_samples(self) -> int:
        return self.n_time * self.n_chan * self.n_pol * self.n_ant

    def d_over_lambda(self) -> np.ndarray:
        """[n_chan][2] (ew, ns) antenna spacing in wavelengths, linear in channel."""
        if self.n_chan == 1:
            dl = np.array([self.dl_lo])
        else:
            dl = self.dl_lo + (self.dl_hi - self.dl_lo) * np.arange(self.n_chan) / (self.n_chan - 1)
        return np.stack([dl, dl], axis=1).astype(np.float64)

    def ns_select(self) -> Optional[np.ndarray]:
        """Clamp table [n_chan][n_ns_keep] int32 (None when unclamped).

        Nearest FFT beam (round half even) to n_ns_keep fixed targets
        sin(theta_j) = -1 + (j + 1/2) * 2 / n_ns_keep, at the channel's
        N-S spacing; beam A points at sin(theta_A) = A lambda / (M d).
        """
        if not self.n_ns_keep:
            return None
        return clamp_table(self.d_over_lambda()[:, 1], self.m_ns, self.n_ns_keep)

    def source_y(self) -> np.ndarray:
        """[n_src][n_chan][2] pointings y = (d/lambda) sin(theta) per axis."""
        dl = self.d_over_lambda()
        ys = []
        for (nw, nn) in self.src_dircos:
            ys.append(np.stack([dl[:, 0] * nw, dl[:, 1] * nn], axis=1))
        for (aw, an) in self.src_lattice:
            ys.append(np.tile(np.array([aw / self.m_ew, an / self.m_ns]), (self.n_chan, 1)))
        if not ys:
            return np.zeros((0, self.n_chan, 2))
        return np.stack(ys, axis=0)

    def snr(self) -> np.ndarray:
        return np.asarray(list(self.src_snr), dtype=np.float64)


def clamp_table(dl_ns: np.ndarray, m_ns: int, n_keep: int) -> np.ndarray:
    j = np.arange(n_keep, dtype=np.float64)
    s = -1.0 + (j + 0.5) * 2.0 / n_keep
    a = np.rint(m_ns * dl_ns[:, None] * s[None, :]).astype(np.int64)  # rint = half even
    return np.mod(a, m_ns).astype(np.int32)


def _uniform(rng: np.random.Generator, lo, hi, n):
    return tuple(float(v) for v in rng.uniform(lo, hi, n))


def make_workload(name: str) -> Workload:
    """The five named workloads (tiny, CHIME-shaped, tied, mixed, serving)."""
    if name in ("c1", "c4"):
        rng = np.random.default_rng(1)
        a_ew = int(rng.integers(0, 4))
        a_ns = int(rng.integers(0, 32))
        return Workload(name, 4, 16, 1, 1, 1024, 4, 32, 16, 1,
                        src_snr=(20.0,), src_lattice=((a_ew, a_ns),))
    if name == "c2":
        rng = np.random.default_rng(2)
        dirs = tuple(zip(_uniform(rng, -1, 1, 8), _uniform(rng, -1, 1, 8)))
        snr = _uniform(rng, 5, 50, 8)
        return Workload(name, 4, 256, 256, 2, 16384, 4, 512, 16, 2,
                        src_dircos=dirs, src_snr=snr, dl_lo=0.4, dl_hi=0.8,
                        n_ns_keep=256)
    if name == "c3":
        rng = np.random.default_rng(3)
        dirs = ((float(rng.uniform(-1, 1)), float(rng.uniform(-1, 1))),)
        return Workload(name, 4, 16, 1, 1, 1024, 4, 32, 16, 3,
                        src_dircos=dirs, src_snr=(20.0,))
    if name == "c5":
        rng = np.random.default_rng(5)
        dirs = tuple(zip(_uniform(rng, -1, 1, 4), _uniform(rng, -1, 1, 4)))
        snr = _uniform(rng, 5, 50, 4)
        return Workload(name, 4, 16, 256, 1, 65536, 4, 32, 16, 5,
                        src_dircos=dirs, src_snr=snr, dl_lo=0.4, dl_hi=0.8)
    raise KeyError(name)


def custom_workload(n_ew=4, n_ns=16, n_chan=1, n_pol=1, n_time=64, m_ew=None, m_ns=None,
                    block=16, seed=0, n_src=1, snr=20.0, n_ns_keep=0, dl=(0.5, 0.5)) -> Workload:
    """A free-form workload of the same recipe (for edge-case tests)."""
    rng = np.random.default_rng(seed + 1000)
    dirs = tuple(zip(_uniform(rng, -1, 1, n_src), _uniform(rng, -1, 1, n_src)))
    return Workload("custom", n_ew, n_ns, n_chan, n_pol, n_time,
                    m_ew or n_ew, m_ns or 2 * n_ns, block, seed,
                    src_dircos=dirs, src_snr=tuple([snr] * n_src),
                    dl_lo=dl[0], dl_hi=dl[1], n_ns_keep=n_ns_keep)


# --------------------------------------------------------------------------
# tapers and pointings (inputs to the method)
# --------------------------------------------------------------------------


def gaussian_taper(n_ew: int, n_ns: int, width: float = 0.4) -> np.ndarray:
    """[n_ns][n_ew] float32 separable Gaussian, sigma = width * aperture."""
    def ax(n):
        a = np.arange(n, dtype=np.float64)
        return np.exp(-0.5 * ((a - (n - 1) / 2.0) / (width * n)) ** 2)
    return (ax(n_ns)[:, None] * ax(n_ew)[None, :]).astype(np.float32)


def half_sine_taper(n_ew: int, n_ns: int, shifted: bool = False) -> np.ndarray:
    """[n_ns][n_ew] float32 half-sine window per axis."""
    def ax(n):
        a = np.arange(n, dtype=np.float64)
        return np.sin(np.pi * (a + 1) / (n + 1)) if shifted else np.sin(np.pi * (a + 0.5) / n)
    return (ax(n_ns)[:, None] * ax(n_ew)[None, :]).astype(np.float32)


def pointings(n_point: int, seed: int) -> np.ndarray:
    """[n_point][2] direction cosines (ew, ns) uniform in [-1, 1)^2, float64."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=(n_point, 2))


# --------------------------------------------------------------------------
# voltage generation
# --------------------------------------------------------------------------

_PH_BITS = 10
_cos_tab = np.rint(np.cos(2 * np.pi * np.arange(1 << _PH_BITS) / (1 << _PH_BITS)) * (1 << 14)).astype(np.int64)
_sin_tab = np.rint(np.sin(2 * np.pi * np.arange(1 << _PH_BITS) / (1 << _PH_BITS)) * (1 << 14)).astype(np.int64)


def _source_tables(w: Workload, chans: np.ndarray):
    """Per source: amplitude (Q12) and phasor tables (Q14) [n_src][nc][n_ns][n_ew]."""
    ys = w.source_y()[:, chans, :] if len(w.src_snr) else np.zeros((0, len(chans), 2))
    amp = np.rint(w.snr() / math.sqrt(w.n_ant) * (1 << 12)).astype(np.int64)
    yfx = np.mod(np.rint(ys * 2.0 ** 32).astype(np.int64), 1 << 32)  # Q32 turns
    a_ns = np.arange(w.n_ns, dtype=np.int64)[:, None]
    a_ew = np.arange(w.n_ew, dtype=np.int64)[None, :]
    ph = (a_ew[None, None] * yfx[:, :, 0, None, None] + a_ns[None, None] * yfx[:, :, 1, None, None]) & MASK32
    idx = ph >> (32 - _PH_BITS)
    return amp, _cos_tab[idx], _sin_tab[idx]


def volts(w: Workload, t0: int = 0, nt: Optional[int] = None,
          chans: Optional[Sequence[int]] = None, pols: Optional[Sequence[int]] = None,
          backend: str = "numpy", device=None, out=None):
    """Voltage bytes [nt][nc][np][n_ns][n_ew] uint8 for the requested slice.

    backend "numpy" returns a numpy array; backend "torch" returns (or
    fills ``out``, a uint8 tensor of the full slice shape) a torch tensor on
    ``device``, computed in chunks of time.
    """
    nt = w.n_time - t0 if nt is None else nt
    chans = np.arange(w.n_chan) if chans is None else np.asarray(chans, dtype=np.int64)
    pols = np.arange(w.n_pol) if pols is None else np.asarray(pols, dtype=np.int64)
    amp, pc, ps = _source_tables(w, chans)
    if backend == "numpy":
        return _volts_chunk(np, w, np.arange(t0, t0 + nt, dtype=np.int64), chans, pols, amp, pc, ps)
    import torch
    dev = torch.device(device if device is not None else "cuda")
    shape = (nt, len(chans), len(pols), w.n_ns, w.n_ew)
    if out is None:
        out = torch.empty(shape, dtype=torch.uint8, device=dev)
    assert tuple(out.shape) == shape and out.dtype == torch.uint8
    tc = torch.as_tensor(chans, device=dev)
    tp = torch.as_tensor(pols, device=dev)
    tpc = torch.as_tensor(pc, device=dev)
    tps = torch.as_tensor(ps, device=dev)
    per_t = len(chans) * len(pols) * w.n_ant
    step = max(1, min(nt, (1 << 24) // max(per_t, 1)))
    for s in range(0, nt, step):
        e = min(nt, s + step)
        tt = torch.arange(t0 + s, t0 + e, dtype=torch.int64, device=dev)
        out[s:e] = _volts_chunk(torch, w, tt, tc, tp, amp, tpc, tps)
    return out


def _volts_chunk(xp, w: Workload, t, chans, pols, amp, pc, ps):
    nt, nc, npol = len(t), len(chans), len(pols)
    t5 = t.reshape(nt, 1, 1, 1, 1)
    c5 = chans.reshape(1, nc, 1, 1, 1)
    p5 = pols.reshape(1, 1, npol, 1, 1)
    if xp is np:
        ant = np.arange(w.n_ant, dtype=np.int64).reshape(1, 1, 1, w.n_ns, w.n_ew)
    else:
        ant = xp.arange(w.n_ant, dtype=xp.int64, device=t.device).reshape(1, 1, 1, w.n_ns, w.n_ew)
    # receiver noise, one 32-bit hash per complex sample
    key = _time_key(w.seed, STREAM_NOISE, t5)
    idx = (c5 * w.n_pol + p5) * w.n_ant + ant
    nre, nim = _gauss_pair(lowbias32(key ^ idx))
    re = nre << 26
    im = nim << 26
    # point sources: s_k(t, chan, pol) * amp_k * exp(+i 2 pi (a . y_k))
    if len(amp):
        skey = _time_key(w.seed, STREAM_SOURCE, t5)
        for k in range(len(amp)):
            sidx = ((k * w.n_chan + c5) * w.n_pol + p5)
            sre, sim = _gauss_pair(lowbias32(skey ^ sidx))
            pck = pc[k].reshape(1, nc, 1, w.n_ns, w.n_ew)
            psk = ps[k].reshape(1, nc, 1, w.n_ns, w.n_ew)
            a = int(amp[k])
            re = re + a * (sre * pck - sim * psk)
            im = im + a * (sre * psk + sim * pck)
    half = 1 << 25
    vre = (re + half) >> 26
    vim = (im + half) >> 26
    if xp is np:
        vre = np.clip(vre, -7, 7)
        vim = np.clip(vim, -7, 7)
        return (((vre & 0xF) << 4) | (vim & 0xF)).astype(np.uint8)
    vre = vre.clamp(-7, 7)
    vim = vim.clamp(-7, 7)
    return (((vre & 0xF) << 4) | (vim & 0xF)).to(xp.uint8)


def point_source_volts(n_ew: int, n_ns: int, q_ew: int, q_ns: int, n_time: int,
                       amp: int = 7) -> np.ndarray:
    """Noise-free lattice-aligned source [n_time][1][1][n_ns][n_ew] uint8.

    y = (q_ew / 4, q_ns / 4) turns per antenna spacing, so each antenna
    sees amp * i^(q_ew a_ew + q_ns a_ns): exactly representable nibbles.
    """
    a_ns = np.arange(n_ns)[:, None]
    a_ew = np.arange(n_ew)[None, :]
    q = (q_ew * a_ew + q_ns * a_ns) % 4
    re = np.choose(q, [amp, 0, -amp, 0])
    im = np.choose(q, [0, amp, 0, -amp])
    b = (((re & 0xF) << 4) | (im & 0xF)).astype(np.uint8)
    return np.broadcast_to(b, (n_time, 1, 1, n_ns, n_ew)).copy()


def pack_nibbles(re: np.ndarray, im: np.ndarray) -> np.ndarray:
    """Pack integer components in [-8, 7] as (re << 4) | im nibbles."""
    re = np.asarray(re, dtype=np.int64)
    im = np.asarray(im, dtype=np.int64)
    if re.min(initial=0) < -8 or re.max(initial=0) > 7 or im.min(initial=0) < -8 or im.max(initial=0) > 7:
        raise ValueError("components outside the 4-bit range")
    return (((re & 0xF) << 4) | (im & 0xF)).astype(np.uint8)


def random_complex_series(n_time: int, n_series: int, seed: int) -> np.ndarray:
    """[n_time][n_series] complex64 Gaussian series (input to the intensity accumulator)."""
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((n_time, n_series, 2)).astype(np.float32)
    return z.view(np.complex64)[..., 0]


# --------------------------------------------------------------------------
# serving request stream
# --------------------------------------------------------------------------


@dataclasses.dataclass(frozen=True)
class Request:
    rid: int
    arrival_s: float
    n_point: int
    n_time: int
    chan_lo: int
    n_chan: int
    dircos: np.ndarray   # [n_point][2]


def request_stream(n_req: int, seed: int = 5, rate_hz: float = 200.0, n_chan_total: int = 256,
                   t_min: int = 1024, t_max: int = 65536, p_max: int = 256,
                   c_min: int = 8, c_max: int = 256, block: int = 16):
    """Poisson arrivals with log-uniform pointings, duration and channel count."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, n_req)
    arr = np.cumsum(gaps)
    out = []
    for i in range(n_req):
        p = int(np.clip(np.floor(np.exp(rng.uniform(0, np.log(p_max + 1)))), 1, p_max))
        t = int(np.exp(rng.uniform(np.log(t_min), np.log(t_max))))
        t = int(np.clip((t // block) * block, t_min, t_max))
        c = int(np.clip(np.floor(np.exp(rng.uniform(np.log(c_min), np.log(c_max + 1)))), c_min, c_max))
        lo = int(rng.integers(0, n_chan_total - c + 1))
        d = rng.uniform(-1.0, 1.0, size=(p, 2))
        out.append(Request(i, float(arr[i]), p, t, lo, c, d))
    return out
