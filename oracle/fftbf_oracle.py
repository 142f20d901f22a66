"""Plain, slow FP64 oracle of the FFT-beamforming hot path (test infrastructure).

This module is test infrastructure.  It is imported only by tests, by the
smoke check and by the benchmark's CPU-baseline leg; the GPU library never
uses it and the two share no code.

Every routine is the plain definition of what the hot path computes,
written in numpy float64/complex128 with no FFT, no blocking and no
fusion.  Paper: K. W. Masui et al., "Algorithms for FFT Beamforming Radio
Interferometers" (arXiv:1710.08591).

Conventions (readings of the paper, shared with the GPU library by
specification only):

* voltages ``volts[t][chan][pol][a_ns][a_ew]`` uint8, each byte two's
  complement nibbles, real part high nibble, imaginary part low nibble.
* the 2-D lattice is separable: antenna (a_ew, a_ns), beam (A_ew, A_ns),
  transform lengths (m_ew, m_ns), normalisation 1/sqrt(n_ew n_ns).
* FFT beams: the inner sum of eq. e:fftbeamform (Sec. "Redundant arrays
  and Fourier transform beamforming"), with weights e:w_A^a,
  ``B[A] = n^-1/2 sum_a h_a eta_a exp(-i 2 pi A a / M)`` per axis,
  zero padding when M > n (the same section).
* sculpting: eta_a -> h_a eta_a, the naive windowed beam of Sec.
  "Controlling beam shape with windowing" (w_nw^a ~ h^a w_p^a).
* intensities: |B|^2 summed (not averaged) over blocks of ``block``
  consecutive samples, the sum over t of eq. e:bf / e:fftbeamform with
  the 1/n_samp factor and the c^2/(k_B nu^2) unit factor dropped.
* tied-array (pointed) beams: the factorisable pointed weights of eq.
  e:c_pointed, w_p^a = n^-1/2 exp(-i 2 pi a (d/lambda) sin(theta_p)),
  per axis, at y = (d/lambda) sin(theta) per axis.
"""
from __future__ import annotations

import math
from typing import Optional

import numpy as np

__all__ = [
    "decode_int4", "dft_matrix", "fft_beams", "intensity", "beamform_fft",
    "pointed_weights", "tied_beams", "tied_intensity", "accumulate_intensity",
    "visibilities", "beam_power_from_visibilities", "stacked_visibilities",
    "beam_power_from_stacked", "stacked_from_beams", "regrid_weights_paper",
    "interp_weights", "interpolate_beams", "rel_power_error",
    "window_autocorr", "optimal_window_norm", "optimal_window_lag_weights",
    "optimal_window_weights", "compact_taps", "regrid_intensity",
    "baseline_moi", "pointed_power_and_slope", "localize_row", "localize",
    "regrid_intensity_2d",
]


# ---------------------------------------------------------------- decode ---

def _weights(h) -> np.ndarray:
    """Per-antenna weights as given: real windows (Sec. "Controlling beam
    shape with windowing") stay real, complex per-antenna gains
    e^{gamma + i psi} (eq. e:vis_pert, Sec. "Non-redundancy") stay complex."""
    h = np.asarray(h)
    return h.astype(np.complex128) if np.iscomplexobj(h) else h.astype(np.float64)


def decode_int4(volts: np.ndarray) -> np.ndarray:
    """uint8 voltages -> complex128 (two's complement nibbles, re high).

    The antenna signal eta_a[t] of eq. e:Vab as digitised samples; the
    4+4-bit encoding is not in the paper (reading: two's complement, real
    part in the high nibble).
    """
    b = np.asarray(volts, dtype=np.uint8).astype(np.int64)
    hi = (b >> 4) & 0xF
    lo = b & 0xF
    re = np.where(hi >= 8, hi - 16, hi)
    im = np.where(lo >= 8, lo - 16, lo)
    return re.astype(np.float64) + 1j * im.astype(np.float64)


# ------------------------------------------------------------- FFT beams ---

def dft_matrix(n: int, m: int) -> np.ndarray:
    """[m][n] weights n^-1/2 exp(-i 2 pi A a / m) of eq. e:w_A^a.

    The phase index (A a) mod m is reduced in integers before the
    exponential so that every entry is accurate to FP64 rounding.
    """
    A = np.arange(m)[:, None]
    a = np.arange(n)[None, :]
    k = (A * a) % m
    return np.exp(-2j * np.pi * k / m)


def fft_beams(eta: np.ndarray, m_ew: int, m_ns: int, taper: Optional[np.ndarray] = None) -> np.ndarray:
    """Complex FFT beams [..., m_ew, m_ns] from complex voltages [..., n_ns, n_ew].

    Direct evaluation of the inner sum of eq. e:fftbeamform on the 2-D
    lattice (separable phase, normalisation 1/sqrt(n_ew n_ns)), after the
    per-antenna window h (Sec. "Controlling beam shape with windowing").
    Zero padding to m > n is implicit: antennas beyond n contribute zero.
    For m < n the same weights over all n antennas are the cyclic
    co-adding of the same section (antennas with equal a mod m share a
    phase); the normalisation stays n^-1/2.
    """
    n_ns, n_ew = eta.shape[-2], eta.shape[-1]
    x = eta if taper is None else eta * _weights(taper)
    w_ew = dft_matrix(n_ew, m_ew)            # [m_ew][n_ew]
    w_ns = dft_matrix(n_ns, m_ns)            # [m_ns][n_ns]
    # B[..., A_ew, A_ns] = sum_{a_ns, a_ew} w_ew[A_ew, a_ew] w_ns[A_ns, a_ns] x[..., a_ns, a_ew]
    y = np.matmul(x, w_ew.T)                 # [..., n_ns, m_ew]
    y = np.swapaxes(y, -1, -2)               # [..., m_ew, n_ns]
    b = np.matmul(y, w_ns.T)                 # [..., m_ew, m_ns]
    return b / math.sqrt(n_ew * n_ns)


def intensity(z: np.ndarray, block: int) -> np.ndarray:
    """|z|^2 summed over consecutive blocks of the leading (time) axis.

    The time sum of eq. e:bf (and of eq. e:fftbeamform) over n_samp =
    ``block`` samples, without the 1/n_samp factor.
    """
    t = z.shape[0]
    if t % block:
        raise ValueError("time length is not a multiple of the block")
    p = z.real ** 2 + z.imag ** 2
    return p.reshape((t // block, block) + z.shape[1:]).sum(axis=1)


def beamform_fft(volts: np.ndarray, m_ew: int, m_ns: int, block: int,
                 taper: Optional[np.ndarray] = None, ns_select: Optional[np.ndarray] = None,
                 pol_sum: bool = False) -> np.ndarray:
    """FFT-beam intensities [blk][chan][pol][m_ew][keep] in float64.

    volts: uint8 [t][chan][pol][n_ns][n_ew].  ``ns_select`` [chan][keep]
    picks which N-S beams are kept per channel (the clamp of a chromatic
    beam grid, Sec. "Redundant arrays ...": beam positions depend on
    wavelength, e:theta_A).  ``pol_sum`` adds the polarisations.
    """
    b = fft_beams(decode_int4(volts), m_ew, m_ns, taper)
    i = intensity(b, block)                  # [blk][chan][pol][m_ew][m_ns]
    if ns_select is not None:
        sel = np.asarray(ns_select)
        i = np.stack([i[:, c, :, :, :][..., sel[c]] for c in range(i.shape[1])], axis=1)
    if pol_sum:
        i = i.sum(axis=2, keepdims=False)
    return i


# ---------------------------------------------------- tied-array beams ---

def pointed_weights(n: int, y: np.ndarray) -> np.ndarray:
    """[P][n] factorisable pointed weights of eq. e:c_pointed at y = (d/lambda) sin(theta)."""
    a = np.arange(n)[None, :]
    return np.exp(-2j * np.pi * a * np.asarray(y, dtype=np.float64)[:, None]) / math.sqrt(n)


def tied_beams(volts: np.ndarray, dircos: np.ndarray, d_over_lambda: np.ndarray,
               taper: Optional[np.ndarray] = None, chans=None) -> np.ndarray:
    """Tied-array beams by direct phased sum, [t][chan][pol][P] complex.

    B_p[t] = sum_a h_a eta_a[t] w_p^a with the product of per-axis pointed
    weights (eq. e:c_pointed), y_axis = (d/lambda)_chan * dircos_axis.
    volts: uint8 [t][chan][pol][n_ns][n_ew]; dircos [P][2] (ew, ns);
    d_over_lambda [n_chan_total][2]; ``chans`` lists the channel of each
    slice in ``volts`` (default: 0..n-1).
    """
    eta = decode_int4(volts)
    if taper is not None:
        eta = eta * _weights(taper)
    n_t, n_c, n_p, n_ns, n_ew = eta.shape
    chans = np.arange(n_c) if chans is None else np.asarray(chans)
    dircos = np.asarray(dircos, dtype=np.float64)
    out = np.empty((n_t, n_c, n_p, dircos.shape[0]), dtype=np.complex128)
    for ci in range(n_c):
        dl = np.asarray(d_over_lambda, dtype=np.float64)[chans[ci]]
        w_ew = pointed_weights(n_ew, dl[0] * dircos[:, 0])   # [P][n_ew]
        w_ns = pointed_weights(n_ns, dl[1] * dircos[:, 1])   # [P][n_ns]
        # sum_{a_ns,a_ew} w_ns[p,a_ns] w_ew[p,a_ew] eta[t,c,pol,a_ns,a_ew]
        out[:, ci] = np.einsum("pn,pe,tqne->tqp", w_ns, w_ew, eta[:, ci])
    return out


def tied_intensity(volts, dircos, d_over_lambda, block, taper=None, chans=None) -> np.ndarray:
    """[blk][chan][pol][P] float64 intensities of the direct phased-sum beams."""
    return intensity(tied_beams(volts, dircos, d_over_lambda, taper, chans), block)


def accumulate_intensity(z: np.ndarray, block: int, prev: Optional[np.ndarray] = None) -> np.ndarray:
    """sum over blocks of |z|^2 for a complex series [t][series] (+ prev if given)."""
    i = intensity(np.asarray(z, dtype=np.complex128), block)
    return i if prev is None else i + np.asarray(prev, dtype=np.float64)


# ----------------------------------------- visibility-space formulation ---
# These are independent routes to the same beams, used to pin the oracle.

def visibilities(eta: np.ndarray) -> np.ndarray:
    """V_ab = sum_t eta_a[t] eta_b[t]^* over the leading axis (eq. e:Vab, summed).

    eta: complex [t][n]; returns [n][n].
    """
    n = eta.shape[1]
    v = np.zeros((n, n), dtype=np.complex128)
    for a in range(n):
        for b in range(n):
            v[a, b] = np.sum(eta[:, a] * np.conj(eta[:, b]))
    return v


def beam_power_from_visibilities(v: np.ndarray, pos: np.ndarray, m: np.ndarray,
                                 h: Optional[np.ndarray] = None) -> np.ndarray:
    """b_A = (1/n) sum_ab h_a h_b e^{-i 2 pi A.(a-b)/M} V_ab (eq. e:b2n-1, 2-D).

    pos: [n][2] integer lattice coordinates (ew, ns) of each antenna;
    m: (m_ew, m_ns).  Returns [m_ew][m_ns].
    """
    n = v.shape[0]
    h = np.ones(n) if h is None else np.asarray(h, dtype=np.float64)
    out = np.zeros((m[0], m[1]))
    for A0 in range(m[0]):
        for A1 in range(m[1]):
            s = 0.0 + 0.0j
            for a in range(n):
                for b in range(n):
                    ph = A0 * (pos[a, 0] - pos[b, 0]) / m[0] + A1 * (pos[a, 1] - pos[b, 1]) / m[1]
                    s += h[a] * h[b] * np.exp(-2j * np.pi * ph) * v[a, b]
            out[A0, A1] = (s / n).real
    return out


def stacked_visibilities(v: np.ndarray, n: int) -> np.ndarray:
    """Redundancy-stacked visibilities of a linear array (eq. e:b_V_delta).

    Returns a dict-like array indexed by delta + n - 1, delta in
    [-(n-1), n-1]; alpha runs over [max(0, -delta), min(n, n - delta)),
    an exclusive upper limit (the n - |delta| redundant pairs).
    """
    out = np.zeros(2 * n - 1, dtype=np.complex128)
    for d in range(-(n - 1), n):
        for al in range(max(0, -d), min(n, n - d)):
            out[d + n - 1] += v[al + d, al]
    return out


def beam_power_from_stacked(vt: np.ndarray, n: int, m: int) -> np.ndarray:
    """b_A = (1/n) sum_delta e^{-i 2 pi A delta / M} V~_delta (eq. e:b2n-1)."""
    d = np.arange(-(n - 1), n)
    A = np.arange(m)[:, None]
    return (np.exp(-2j * np.pi * A * d[None, :] / m) @ vt).real / n


def stacked_from_beams(b: np.ndarray, n: int, m: int) -> np.ndarray:
    """V~_delta = (n/M) sum_A e^{+i 2 pi delta A / M} b_A (eq. e:inv_b2n-1)."""
    d = np.arange(-(n - 1), n)[:, None]
    A = np.arange(m)[None, :]
    return (n / m) * (np.exp(2j * np.pi * d * A / m) @ b)


def regrid_weights_paper(n: int, m: int, y: float) -> np.ndarray:
    """Intensity regridding weights w^A_p of eq. e:bp_max_arbitrary, [M].

    w^A = (1/M) sin((2n-1) pi y_A) / sin(pi y_A), y_A = y - A/M, with the
    removable singularity (2n-1)/M at integer y_A.
    """
    ya = y - np.arange(m) / m
    s = np.sin(np.pi * ya)
    num = np.sin((2 * n - 1) * np.pi * ya)
    near = np.abs(s) < 1e-12
    w = np.where(near, (2 * n - 1) * np.cos((2 * n - 1) * np.pi * ya) / np.where(near, np.cos(np.pi * ya), 1.0),
                 num / np.where(near, 1.0, s))
    return w / m


def window_autocorr(h: np.ndarray) -> np.ndarray:
    """Auto-convolution of the window, R_delta = sum_alpha h^{alpha+delta} conj(h^alpha),
    for delta = -(n-1) .. n-1 (index delta + n - 1); the sum over redundant
    pairs in eq. e:w_opt."""
    h = np.asarray(h, dtype=np.complex128)
    n = len(h)
    out = np.zeros(2 * n - 1, dtype=np.complex128)
    for d in range(-(n - 1), n):
        al = np.arange(max(0, -d), min(n, n - d))        # alpha with 0 <= alpha + d < n
        out[d + n - 1] = np.sum(h[al + d] * np.conj(h[al]))
    return out


def optimal_window_norm(h: np.ndarray) -> float:
    """The normalisation N of the optimally windowed beam (eq. e:w_opt).

    The paper leaves N to be computed numerically.  Reading: N makes the
    beam's noise equal to the unwindowed pointed beam's when the visibility
    noise is dominated by the auto-correlations (eq. e:var_bV): each of the
    n - |delta| redundant visibilities of lag delta carries the weight
    w^delta, so sum_delta (n - |delta|) |w^delta|^2 must equal the pointed
    beam's sum_delta (n - |delta|) / n^2 = 1.  With
    w^delta = R_delta e^{-i 2 pi delta y} / (n N (n - |delta|)) that gives
    N = (1/n) sqrt(sum_delta |R_delta|^2 / (n - |delta|)).  N = 1 for h = 1.
    """
    r = window_autocorr(h)
    n = len(h)
    lag = np.arange(-(n - 1), n)
    return float(np.sqrt(np.sum(np.abs(r) ** 2 / (n - np.abs(lag)))) / n)


def optimal_window_lag_weights(h: np.ndarray, y) -> np.ndarray:
    """Lag-domain weights w_ow^delta of eq. e:w_opt, delta = -(n-1) .. n-1
    (last axis), for a scalar or an array of steerings y.

    w_ow^delta = w_p^delta R_delta / (N (n - |delta|)) with the pointed lag
    weight w_p^delta = (1/n) e^{-i 2 pi delta y} (the weights that make
    sum_delta w_p^delta V~_delta the pointed beam of eq. e:b2n-1 at y), so
    that the beam is b = sum_delta w^delta V~_delta.
    """
    n = len(h)
    lag = np.arange(-(n - 1), n)
    wp = np.exp(-2j * np.pi * np.multiply.outer(np.asarray(y, dtype=np.float64), lag)) / n
    return wp * window_autocorr(h) / (optimal_window_norm(h) * (n - np.abs(lag)))


def optimal_window_weights(h: np.ndarray, m: int, y) -> np.ndarray:
    """FFT-beam weights w_ow^A of eq. e:wA_windowed: [M] for a scalar y,
    [T][M] for an array; real for a real window.

    Lag weights mapped to the FFT-beam basis by eq. e:wA_from_wdelta,
    w^A = (n/M) sum_delta e^{+i 2 pi delta A / M} w^delta (valid for
    M >= 2n - 1).  The paper's second form carries n/(M N) in front; with
    h = 1 that would be n times the pointed regridding weights of eq.
    e:bp_max_arbitrary, so the reading kept here is the first form, whose
    prefactor works out to 1/(M N).
    """
    n = len(h)
    lag = np.arange(-(n - 1), n)
    wd = optimal_window_lag_weights(h, y)                          # [..., 2n-1]
    e = np.exp(2j * np.pi * np.outer(np.arange(m), lag) / m)       # [M][2n-1]
    w = (n / m) * wd @ e.T
    if np.isrealobj(h):
        assert np.max(np.abs(w.imag)) < 1e-9 * max(1.0, np.max(np.abs(w.real)))
        return w.real
    return w


def compact_taps(w: np.ndarray, y: float, k: int):
    """Compact k-tap version of a regridding kernel (Sec. "Controlling beam
    shape with windowing": a few weights around the pointing approximate the
    full set).

    Reading: keep the k FFT beams nearest the pointing on the circular beam
    grid, A = round(y M) - (k-1)//2 + j mod M for j < k (round half to even),
    with their full-kernel weights unchanged; every other weight is zero.
    Returns (first tap index mod M, [k] weights).
    """
    m = len(w)
    first = int(np.round(y * m)) - (k - 1) // 2
    idx = (first + np.arange(k)) % m
    return first % m, np.asarray(w)[idx]


def regrid_intensity(b: np.ndarray, weights: np.ndarray) -> np.ndarray:
    """Regridded beams sum_A w^A b_A: b [..., M] intensities, weights [T][M] -> [..., T]."""
    return np.asarray(b, dtype=np.float64) @ np.asarray(weights, dtype=np.float64).T


def baseline_moi(n: int) -> int:
    """sum over lags of delta^2 (n - |delta|) for a linear array: the moment
    of inertia of the baseline distribution (eq. e:baseline_MOI), summed term
    by term."""
    return sum(d * d * (n - abs(d)) for d in range(-(n - 1), n))


def pointed_power_and_slope(b: np.ndarray, beams: np.ndarray, n: int, m: int, y: float):
    """(b_p(y), d b_p / dy) from FFT-beam intensities b over the listed beams.

    b_p(y) = sum_A w^A(y) b_A with the regridding weights of eq.
    e:bp_max_arbitrary written as their lag sum,
    w^A(y) = (1/M) sum_{|delta|<n} e^{+i 2 pi delta (A/M - y)}, and its
    derivative in y term by term.
    """
    lag = np.arange(-(n - 1), n)
    ph = np.exp(2j * np.pi * np.outer(np.asarray(beams) / m - y, lag))     # [K][2n-1]
    w = ph.sum(axis=1).real / m
    dw = (ph * (-2j * np.pi * lag)).sum(axis=1).real / m
    bb = np.asarray(b, dtype=np.float64)[np.asarray(beams)]
    return float(w @ bb), float(dw @ bb)


def localize_row(b: np.ndarray, n: int, d_over_lambda: float, n_window: int, n_iter: int):
    """Newton's-method estimate of a point source's sin(theta) from one row of
    M FFT-beam intensities of a linear array (Sec. "Localization").

    Steps, in the paper's order:
    * initial guess: the beam of strongest detection, y_0 = A_0 / M
      (A_0 = first index of the maximum);
    * sums truncated to the n_window beams nearest A_0 on the circular grid
      (the paper keeps the ~10 beams around the source; n_window = M keeps
      all), A = A_0 - (n_window - 1)//2 + j mod M;
    * update with the curvature replaced by its value at the maximum (the
      baseline moment of inertia, eq. e:baseline_MOI), in y = (d/lambda) sin(theta):
          y <- y + n^2 b_p'(y) / (4 pi^2 MOI b_p(y)),
      i.e. the first form of the paper's final estimator (its second form
      prints n^3 where the substitution gives n^2);
    * n_iter updates; an update is not taken (and the iteration stops) when
      b_p(y) <= 0 or when it would leave [y_0 - 1/M, y_0 + 1/M] (the maximum
      lies within half a beam spacing of the strongest beam, so a step beyond
      one spacing is heading for a sidelobe).
    Returns (sin(theta) estimate with y wrapped to [-1/2, 1/2), b_p at it).
    """
    b = np.asarray(b, dtype=np.float64)
    m = len(b)
    a0 = int(np.argmax(b))
    beams = (a0 - (n_window - 1) // 2 + np.arange(n_window)) % m
    moi = baseline_moi(n)
    y0 = a0 / m
    y = y0
    for _ in range(n_iter):
        p, dp = pointed_power_and_slope(b, beams, n, m, y)
        if not p > 0:
            break
        y_new = y + n * n * dp / (4 * np.pi ** 2 * moi * p)
        if abs(y_new - y0) > 1.0 / m:
            break
        y = y_new
    p, _ = pointed_power_and_slope(b, beams, n, m, y)
    yw = (y + 0.5) % 1.0 - 0.5
    return yw / d_over_lambda, p


def localize(intensity: np.ndarray, n: int, d_over_lambda_ns: np.ndarray, n_window: int, n_iter: int,
             chans=None):
    """localize_row over every row of [blk][chan][..][M] intensities; returns
    (sin(theta) [blk][chan][..], peak [blk][chan][..])."""
    x = np.asarray(intensity, dtype=np.float64)
    chans = np.arange(x.shape[1]) if chans is None else np.asarray(chans)
    st = np.empty(x.shape[:-1])
    pk = np.empty(x.shape[:-1])
    for idx in np.ndindex(*x.shape[:-1]):
        st[idx], pk[idx] = localize_row(x[idx], n, float(d_over_lambda_ns[chans[idx[1]]]), n_window, n_iter)
    return st, pk


def regrid_intensity_2d(b: np.ndarray, y_ew: np.ndarray, y_ns: np.ndarray, n_ew: int, n_ns: int) -> np.ndarray:
    """Pointed-beam intensities at 2-D pointings from FFT-beam intensities
    b [..., M_ew, M_ns]: eq. e:bp_max_arbitrary on each axis (the lattice is
    separable), b_p = sum_{A_ew, A_ns} w^{A_ew}(y_ew) w^{A_ns}(y_ns) b_A.
    Exact when M >= 2n - 1 on both axes.  Returns [..., P]."""
    m_ew, m_ns = b.shape[-2], b.shape[-1]
    out = np.empty(b.shape[:-2] + (len(y_ew),))
    for p in range(len(y_ew)):
        w = np.outer(regrid_weights_paper(n_ew, m_ew, float(y_ew[p])), regrid_weights_paper(n_ns, m_ns, float(y_ns[p])))
        out[..., p] = np.tensordot(np.asarray(b, dtype=np.float64), w, axes=([-2, -1], [0, 1]))
    return out


def interp_weights(n: int, m: int, y: np.ndarray) -> np.ndarray:
    """[P][M] complex weights c_A(y) = (1/M) sum_{a<n} e^{+i 2 pi a (A/M - y)}.

    The voltage-domain counterpart of the regridding of eq.
    e:bp_max_arbitrary: substituting the zero-padded inverse transform
    eta_a = (sqrt(n)/M) sum_A B_A e^{+i 2 pi A a / M} (a < n) into the
    pointed beam of eq. e:c_pointed gives B_p = sum_A c_A(y) B_A exactly
    for M >= n.  The weights are the minimum-norm choice (support a < n).
    Summed term by term (no closed form, so no 0/0).
    """
    y = np.asarray(y, dtype=np.float64)[:, None, None]
    A = np.arange(m)[None, :, None]
    a = np.arange(n)[None, None, :]
    return np.exp(2j * np.pi * a * (A / m - y)).sum(axis=2) / m


def interpolate_beams(b: np.ndarray, y_ew: np.ndarray, y_ns: np.ndarray, n_ew: int, n_ns: int) -> np.ndarray:
    """Tied beams [..., P] from complex FFT beams [..., m_ew, m_ns] by interpolation."""
    m_ew, m_ns = b.shape[-2], b.shape[-1]
    c_ew = interp_weights(n_ew, m_ew, y_ew)      # [P][m_ew]
    c_ns = interp_weights(n_ns, m_ns, y_ns)      # [P][m_ns]
    return np.einsum("pe,pn,...en->...p", c_ew, c_ns, b)


def rel_power_error(got: np.ndarray, ref: np.ndarray) -> float:
    """max over beams of |got - ref| / ref (reference powers must be > 0)."""
    ref = np.asarray(ref, dtype=np.float64)
    got = np.asarray(got, dtype=np.float64)
    return float(np.max(np.abs(got - ref) / ref))
