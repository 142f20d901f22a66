"""Regridding FFT-beam intensities to arbitrary N-S steering angles on the GPU
(eq. e:bp_max_arbitrary) against the FP64 oracle.

The reference is the plain definition the regridding reaches exactly for
M >= 2n - 1: the intensity of the directly phased beam whose E-W direction is
the E-W FFT beam's own (y_ew = e/4, a channel-dependent dircos) and whose N-S
direction is the target's sin(theta) in every channel.

Tolerance of the chain (FFT beams, then regridding): each FFT-beam intensity
may carry the FP32 path's 1e-5 relative error, and the regridding is a fixed
linear map with weights of both signs, so the bound carried to a regridded
beam is 1e-5 * sum_A |w^A| b_A (at most ~11x the beam itself for n = 256 on
noise-dominated skies).  The contraction on its own is held to FP32
dot-product rounding of its inputs.
"""
import numpy as np
import pytest

import oracle as orc
import synthgen as sg
from tests.helpers import TOL_FP32, by_time_chunks, c2_wide_regions, rel_err

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _targets(n, seed):
    rng = np.random.default_rng(seed)
    st = rng.uniform(-1.0, 1.0, n)
    st[0] = 0.0                                   # zenith: an on-grid beam for every channel
    if n > 2:
        st[1], st[2] = -1.0, 1.0                  # the horizon at both ends
    return st


def _propagated_scale(w, v, sin_t, taper, pol_sum):
    """sum_A |w^A| b_A over the oracle's unclamped FFT-beam intensities."""
    b = orc.beamform_fft(v, w.m_ew, w.m_ns, w.block, taper=taper)       # [blk][chan][pol][m_ew][M]
    if pol_sum:
        b = b.sum(axis=2, keepdims=True)
    dl = w.d_over_lambda()
    out = np.empty(b.shape[:-1] + (len(sin_t),))
    for c in range(b.shape[1]):
        W = np.stack([orc.regrid_weights_paper(w.n_ns, w.m_ns, dl[c, 1] * s) for s in sin_t])
        out[:, c] = b[:, c] @ np.abs(W).T
    return out[:, :, 0] if pol_sum else out


def _phased_reference(w, v, sin_t, taper, pol_sum):
    """[blk][chan][pg][4][T] by direct phased sums, channel by channel."""
    dl = w.d_over_lambda()
    n_blk = v.shape[0] // w.block
    out = np.empty((n_blk, w.n_chan, 1 if pol_sum else w.n_pol, w.m_ew, len(sin_t)))
    for c in range(w.n_chan):
        e = np.repeat(np.arange(w.m_ew), len(sin_t))
        dircos = np.stack([e / (w.m_ew * dl[c, 0]), np.tile(sin_t, w.m_ew)], axis=1)
        ti = orc.tied_intensity(v[:, c:c + 1], dircos, dl, w.block, taper=taper, chans=[c])[:, 0]
        if pol_sum:
            ti = ti.sum(axis=1, keepdims=True)
        out[:, c] = ti.reshape(n_blk, ti.shape[1], w.m_ew, len(sin_t))
    return out[:, :, 0] if pol_sum else out


CASES = [
    # n_ns, n_chan, n_pol, n_time, n_target, pol_sum, taper
    pytest.param(16, 6, 2, 1024, 37, False, True, id="4x16-2pol-taper-37"),
    pytest.param(64, 3, 2, 208, 65, True, False, id="4x64-polsum-ragged-rows-65"),
    pytest.param(256, 2, 1, 592, 130, False, False, id="4x256-3x3tiles-130"),
    pytest.param(32, 1, 1, 16, 1, False, False, id="4x32-one-block-one-target"),
]


@pytest.mark.parametrize("n_ns,n_chan,n_pol,n_time,n_target,pol_sum,taper", CASES)
def test_regrid_chain_matches_phased_beams(n_ns, n_chan, n_pol, n_time, n_target, pol_sum, taper):
    torch = _torch()
    import paper_1710_08591_amd as bf
    w = sg.custom_workload(n_ew=4, n_ns=n_ns, n_chan=n_chan, n_pol=n_pol, n_time=n_time, seed=n_ns + n_target,
                           n_src=2, snr=0.5, dl=(0.4, 0.8))
    tap = sg.gaussian_taper(4, n_ns) if taper else None
    v = sg.volts(w)
    plan = bf.Plan(n_ew=4, n_ns=n_ns, n_chan=n_chan, n_pol=n_pol, block=16, pol_sum=pol_sum,
                   d_over_lambda=w.d_over_lambda())
    st = _targets(n_target, n_ns)
    rg = bf.Regrid(plan, st)
    dev_tap = torch.from_numpy(tap).cuda() if taper else None
    fft_i = bf.beamform_fft(plan, torch.from_numpy(v).cuda(), taper=dev_tap)
    got = rg(fft_i)
    torch.cuda.synchronize()
    ref = _phased_reference(w, v, st, tap, pol_sum)
    scale = _propagated_scale(w, v, st, tap, pol_sum)
    assert got.shape == ref.shape == scale.shape
    assert np.all(np.abs(got.cpu().numpy() - ref) <= TOL_FP32 * scale)
    rg.close()
    plan.close()


@pytest.mark.parametrize("n_ns,n_blk,n_target", [(16, 5, 64), (128, 17, 63), (256, 33, 200)])
def test_regrid_kernel_on_oracle_intensities(n_ns, n_blk, n_target):
    """The contraction alone: oracle FFT intensities rounded to FP32 go in; the
    FP64 regridding of the same FP32 values is the reference, element by element
    within a dot-product rounding bound, and per beam within 1e-5."""
    torch = _torch()
    import paper_1710_08591_amd as bf
    n_chan, m = 3, 2 * n_ns
    w = sg.custom_workload(n_ew=4, n_ns=n_ns, n_chan=n_chan, n_pol=2, n_time=16 * n_blk, seed=7, n_src=3,
                           snr=1.0, dl=(0.3, 0.9))
    x = orc.beamform_fft(sg.volts(w), 4, m, 16).astype(np.float32)       # [blk][chan][pol][4][M]
    plan = bf.Plan(n_ew=4, n_ns=n_ns, n_chan=n_chan, n_pol=2, block=16, d_over_lambda=w.d_over_lambda())
    st = _targets(n_target, 3)
    rg = bf.Regrid(plan, st)
    got = rg(torch.from_numpy(x).cuda()).cpu().numpy()
    x64 = x.astype(np.float64)
    for c in range(n_chan):
        W = np.stack([orc.regrid_weights_paper(n_ns, m, w.d_over_lambda()[c, 1] * s) for s in st])   # [T][M]
        ref = x64[:, c] @ W.T
        scale = np.abs(x64[:, c]) @ np.abs(W).T
        assert np.all(np.abs(got[:, c] - ref) <= 2e-6 * scale)
        assert rel_err(got[:, c], ref) < TOL_FP32
    rg.close()
    plan.close()


def _window(kind, n):
    if kind == "sine":
        return np.sin(np.pi * (np.arange(n) + 1) / (n + 1))
    rng = np.random.default_rng(n)
    return 0.2 + rng.random(n)                     # real, asymmetric


def _oracle_case(n_ns, n_blk, n_chan=3, seed=7):
    w = sg.custom_workload(n_ew=4, n_ns=n_ns, n_chan=n_chan, n_pol=2, n_time=16 * n_blk, seed=seed, n_src=3,
                           snr=1.0, dl=(0.3, 0.9))
    x = orc.beamform_fft(sg.volts(w), 4, 2 * n_ns, 16).astype(np.float32)       # [blk][chan][pol][4][M]
    return w, x


@pytest.mark.parametrize("n_ns,n_blk,n_target,kind", [(16, 5, 40, "sine"), (64, 9, 100, "asym"),
                                                      (256, 6, 256, "sine")])
def test_regrid_windowed_kernel_on_oracle_intensities(n_ns, n_blk, n_target, kind):
    """Optimally windowed weights (eq. e:wA_windowed) generated on the device,
    applied to oracle FFT intensities, against the FP64 oracle weights."""
    torch = _torch()
    import paper_1710_08591_amd as bf
    m = 2 * n_ns
    w, x = _oracle_case(n_ns, n_blk)
    h = _window(kind, n_ns)
    plan = bf.Plan(n_ew=4, n_ns=n_ns, n_chan=3, n_pol=2, block=16, d_over_lambda=w.d_over_lambda())
    st = _targets(n_target, 5)
    rg = bf.Regrid(plan, st, window=h)
    got = rg(torch.from_numpy(x).cuda()).cpu().numpy()
    x64 = x.astype(np.float64)
    for c in range(3):
        W = orc.optimal_window_weights(h, m, w.d_over_lambda()[c, 1] * st)
        ref = orc.regrid_intensity(x64[:, c], W)
        scale = orc.regrid_intensity(np.abs(x64[:, c]), np.abs(W))
        assert np.all(np.abs(got[:, c] - ref) <= 2e-6 * scale)
        assert rel_err(got[:, c], ref) < TOL_FP32
    rg.close()
    plan.close()


@pytest.mark.parametrize("n_ns,k,kind", [(16, 1, None), (16, 5, "sine"), (64, 3, None), (64, 8, "asym"),
                                         (256, 5, "sine"), (128, 4, "sine")])
def test_regrid_compact_taps_on_oracle_intensities(n_ns, k, kind):
    """Compact k-tap kernels: the nearest-beam taps and their weights against
    the oracle's truncation of the full kernel, then the gather."""
    torch = _torch()
    import paper_1710_08591_amd as bf
    m = 2 * n_ns
    w, x = _oracle_case(n_ns, 11)
    h = _window(kind, n_ns) if kind else None
    plan = bf.Plan(n_ew=4, n_ns=n_ns, n_chan=3, n_pol=2, block=16, d_over_lambda=w.d_over_lambda())
    st = _targets(300, 9)                          # more targets than one pass of 256 threads
    rg = bf.Regrid(plan, st, window=h, n_taps=k)
    got = rg(torch.from_numpy(x).cuda()).cpu().numpy()
    assert got.shape == (11, 3, 2, 4, 300)
    x64 = x.astype(np.float64)
    for c in range(3):
        ref = np.empty(x64.shape[:1] + x64.shape[2:-1] + (len(st),))
        scale = np.empty_like(ref)
        ys = w.d_over_lambda()[c, 1] * st
        fulls = orc.optimal_window_weights(h, m, ys) if kind else None
        for t, y in enumerate(ys):
            full = fulls[t] if kind else orc.regrid_weights_paper(n_ns, m, y)
            first, taps = orc.compact_taps(full, y, k)
            idx = (first + np.arange(k)) % m
            ref[..., t] = x64[:, c][..., idx] @ taps
            scale[..., t] = np.abs(x64[:, c][..., idx]) @ np.abs(taps)
        assert np.all(np.abs(got[:, c] - ref) <= 1e-6 * scale)
    rg.close()
    plan.close()


def test_regrid_windowed_chain():
    """Voltages -> FP32 FFT intensities (no taper) -> optimally windowed
    beams with the dense and the 5-tap kernels, against the oracle's beams
    regridded in FP64, to the FP32 bar carried through the weights."""
    torch = _torch()
    import paper_1710_08591_amd as bf
    n_ns, m = 64, 128
    w = sg.custom_workload(n_ew=4, n_ns=n_ns, n_chan=4, n_pol=2, n_time=512, seed=31, n_src=3, snr=5.0,
                           dl=(0.4, 0.8))
    v = sg.volts(w)
    plan = bf.Plan(n_ew=4, n_ns=n_ns, n_chan=4, n_pol=2, block=16, d_over_lambda=w.d_over_lambda())
    fft_i = bf.beamform_fft(plan, torch.from_numpy(v).cuda())
    b = orc.beamform_fft(v, 4, m, 16)
    h = _window("sine", n_ns)
    st = _targets(77, 2)
    for k in (0, 5):
        rg = bf.Regrid(plan, st, window=h, n_taps=k)
        got = rg(fft_i).cpu().numpy()
        for c in range(4):
            W = np.zeros((len(st), m))
            ys = w.d_over_lambda()[c, 1] * st
            fulls = orc.optimal_window_weights(h, m, ys)
            for t, y in enumerate(ys):
                full = fulls[t]
                if k:
                    first, taps = orc.compact_taps(full, y, k)
                    W[t, (first + np.arange(k)) % m] = taps
                else:
                    W[t] = full
            ref = orc.regrid_intensity(b[:, c], W)
            scale = orc.regrid_intensity(b[:, c], np.abs(W))
            assert np.all(np.abs(got[:, c] - ref) <= TOL_FP32 * scale)
        rg.close()
    plan.close()


def test_regrid_at_zenith_is_the_fft_beam():
    """sin(theta) = 0 is the position of FFT beam A = 0 in every channel, so the
    regridded beam (a sum over all M beams: weight (2n-1)/M on A = 0 and
    -(-1)^A/M elsewhere) reproduces b_0 to FP32 rounding."""
    torch = _torch()
    import paper_1710_08591_amd as bf
    w = sg.custom_workload(n_ew=4, n_ns=64, n_chan=4, n_pol=1, n_time=320, seed=21, snr=3.0, dl=(0.4, 0.8))
    plan = bf.Plan(n_ew=4, n_ns=64, n_chan=4, block=16, d_over_lambda=w.d_over_lambda())
    rg = bf.Regrid(plan, np.array([0.0]))
    fft_i = bf.beamform_fft(plan, torch.from_numpy(sg.volts(w)).cuda())
    got = rg(fft_i)[..., 0]
    assert rel_err(got.cpu().numpy(), fft_i[..., 0].cpu().numpy()) < TOL_FP32
    rg.close()
    plan.close()


def test_regrid_empty_and_validation():
    torch = _torch()
    import paper_1710_08591_amd as bf
    plan = bf.Plan(n_ew=4, n_ns=16, n_chan=2, block=16)
    rg = bf.Regrid(plan, np.array([0.1, -0.2]))
    empty = torch.empty((0, 2, 1, 4, 32), dtype=torch.float32, device="cuda")
    assert rg(empty).shape == (0, 2, 1, 4, 2)
    with pytest.raises(ValueError):
        rg(torch.empty((1, 2, 1, 4, 16), dtype=torch.float32, device="cuda"))
    rg.close()
    # a clamped plan does not hold all M beams; an unpadded N-S axis is not exact
    clamped = bf.Plan(n_ew=4, n_ns=16, n_chan=1, block=16, ns_select=np.arange(16, dtype=np.int32)[None])
    with pytest.raises(bf.BFError) as e:
        bf.Regrid(clamped, np.array([0.0]))
    assert e.value.status == bf.BF_ERR_INVALID_ARGUMENT
    with pytest.raises(bf.BFError) as e:
        bf.Regrid(plan, np.zeros(0))
    assert e.value.status == bf.BF_ERR_INVALID_ARGUMENT
    with pytest.raises(bf.BFError) as e:
        bf.Regrid(plan, np.array([np.nan]))
    assert e.value.status == bf.BF_ERR_INVALID_ARGUMENT
    for kw in ({"n_taps": 9}, {"n_taps": -1}, {"window": np.zeros(16)}, {"window": np.full(16, np.inf)}):
        with pytest.raises(bf.BFError) as e:
            bf.Regrid(plan, np.array([0.0]), **kw)
        assert e.value.status == bf.BF_ERR_INVALID_ARGUMENT
    with pytest.raises(ValueError):
        bf.Regrid(plan, np.array([0.0]), window=np.ones(8))
    clamped.close()
    plan.close()


def _c2_regrid_wide(w, v, got, weights_for):
    """(largest error over 1e-5 sum_A |w^A| b_A, largest per-beam relative
    error) of regridded CHIME-shaped outputs ``got`` [blk][chan][pol][4][T]
    over the full-size comparison set; the reference is the oracle's
    regridding (weights_for(channel) -> [T][M]) of its own FFT-beam
    intensities."""
    prop = beam = 0.0
    cache = {}
    for idx, vs, chans in c2_wide_regions(w, v):
        b = by_time_chunks(lambda x: orc.beamform_fft(x, 4, 512, 16), vs)     # [nb][nc][pol][4][512]
        g = got[idx].cpu().numpy()
        for ci, c in enumerate(chans):
            if c not in cache:
                cache[c] = weights_for(int(c))
            W = cache[c]
            ref = orc.regrid_intensity(b[:, ci], W)
            scale = orc.regrid_intensity(b[:, ci], np.abs(W))
            d = np.abs(g[:, ci] - ref)
            prop = max(prop, float(np.max(d / (TOL_FP32 * scale))))
            beam = max(beam, float(np.max(d / ref)))
    return prop, beam


def test_regrid_c2_shape_sampled():
    """CHIME-shaped lattice (4 x 256, 256 channels, 2 pols, 16384 samples), all
    512 N-S beams regridded to 256 achromatic targets, in the launch
    configuration the benchmark times.  Sampled (block, channel) outputs
    against direct phased beams, and the full-size comparison set (every
    channel and both polarisations of the first and the last block, one
    channel over all blocks) against the oracle's regridding of its own
    FFT-beam intensities.  The bar is the propagated FP32 bar; the per-beam
    relative error is printed beside it."""
    torch = _torch()
    import paper_1710_08591_amd as bf
    w = sg.make_workload("c2")
    plan = bf.Plan(n_ew=4, n_ns=256, n_chan=256, n_pol=2, block=16, d_over_lambda=w.d_over_lambda())
    st = np.linspace(-0.95, 0.95, 256)
    rg = bf.Regrid(plan, st)
    v = sg.volts(w, backend="torch", device="cuda")
    fft_i = bf.beamform_fft(plan, v)
    got = rg(fft_i)
    torch.cuda.synchronize()
    del fft_i
    assert got.shape == (1024, 256, 2, 4, 256)
    rng = np.random.default_rng(4)
    picks = [(0, 0), (1023, 255)] + [(int(rng.integers(1024)), int(rng.integers(256))) for _ in range(3)]
    dl = w.d_over_lambda()
    for blk, c in picks:
        vs = sg.volts(w, blk * 16, 16, chans=[c])
        e = np.repeat(np.arange(4), len(st))
        dircos = np.stack([e / (4 * dl[c, 0]), np.tile(st, 4)], axis=1)
        ref = orc.tied_intensity(vs, dircos, dl, 16, chans=[c])[0, 0].reshape(2, 4, len(st))
        b = orc.beamform_fft(vs, 4, 512, 16)[0, 0]                              # [pol][4][512]
        W = orc.regrid_weights_paper(256, 512, dl[c, 1] * st[:, None])          # [T][512]
        scale = b @ np.abs(W).T
        assert np.all(np.abs(got[blk, c].cpu().numpy() - ref) <= TOL_FP32 * scale)
    prop, beam = _c2_regrid_wide(w, v, got, lambda c: orc.regrid_weights_paper(256, 512, dl[c, 1] * st[:, None]))
    print(f"4x256 regrid to 256 targets, full size: error / (1e-5 sum|w|b) {prop:.3f}, "
          f"max per-beam rel error {beam:.3e}")
    assert prop <= 1.0
    rg.close()
    plan.close()
    del v, got
    torch.cuda.empty_cache()


@pytest.mark.parametrize("n_taps", [0, 5])
def test_windowed_regrid_c2_shape_sampled(n_taps):
    """The optimally windowed beams (half-sine window) on the CHIME-shaped
    lattice at full size, dense and with the compact 5-tap kernel, in the
    launch configuration the benchmark times; sampled (block, channel)
    outputs against the oracle's windowed weights applied to its own FFT-beam
    intensities."""
    torch = _torch()
    import paper_1710_08591_amd as bf
    w = sg.make_workload("c2")
    plan = bf.Plan(n_ew=4, n_ns=256, n_chan=256, n_pol=2, block=16, d_over_lambda=w.d_over_lambda())
    st = np.linspace(-0.95, 0.95, 256)
    h = np.sin(np.pi * (np.arange(256) + 1) / 257)
    rg = bf.Regrid(plan, st, window=h, n_taps=n_taps)
    v = sg.volts(w, backend="torch", device="cuda")
    fft_i = bf.beamform_fft(plan, v)
    del v
    got = rg(fft_i)
    torch.cuda.synchronize()
    assert got.shape == (1024, 256, 2, 4, 256)
    rng = np.random.default_rng(6)
    dl = w.d_over_lambda()
    for blk, c in [(0, 0), (1023, 255)] + [(int(rng.integers(1024)), int(rng.integers(256))) for _ in range(2)]:
        b = orc.beamform_fft(sg.volts(w, blk * 16, 16, chans=[c]), 4, 512, 16)[0, 0]
        ys = dl[c, 1] * st
        full = orc.optimal_window_weights(h, 512, ys)
        W = np.zeros_like(full)
        for t, y in enumerate(ys):
            if n_taps:
                first, taps = orc.compact_taps(full[t], y, n_taps)
                W[t, (first + np.arange(n_taps)) % 512] = taps
            else:
                W[t] = full[t]
        ref = orc.regrid_intensity(b, W)
        scale = orc.regrid_intensity(b, np.abs(W))
        assert np.all(np.abs(got[blk, c].cpu().numpy() - ref) <= TOL_FP32 * scale)
    rg.close()
    plan.close()
    del fft_i, got
    torch.cuda.empty_cache()


@pytest.mark.parametrize("n_blk", [1, 3, 11])
def test_regrid_compact_taps_ragged_row_tiles(n_blk):
    """Compact taps on pol-summed intensities, so a channel has 4 n_blk rows:
    1, 3 and 11 blocks leave the last workgroup's row tile short (4, 12 and
    44 rows against tiles of 8)."""
    torch = _torch()
    import paper_1710_08591_amd as bf
    n_ns, k = 64, 5
    m = 2 * n_ns
    w, x = _oracle_case(n_ns, n_blk, seed=13)
    xs = x.sum(axis=2)                                            # [blk][chan][4][M]: the pol-summed rows
    plan = bf.Plan(n_ew=4, n_ns=n_ns, n_chan=3, n_pol=2, block=16, pol_sum=True, d_over_lambda=w.d_over_lambda())
    st = _targets(70, 5)
    rg = bf.Regrid(plan, st, n_taps=k)
    got = rg(torch.from_numpy(np.ascontiguousarray(xs)).cuda()).cpu().numpy()
    assert got.shape == (n_blk, 3, 4, 70)
    x64 = xs.astype(np.float64)
    for c in range(3):
        ys = w.d_over_lambda()[c, 1] * st
        for t, y in enumerate(ys):
            first, taps = orc.compact_taps(orc.regrid_weights_paper(n_ns, m, y), y, k)
            idx = (first + np.arange(k)) % m
            ref = x64[:, c][..., idx] @ taps
            scale = np.abs(x64[:, c][..., idx]) @ np.abs(taps)
            assert np.all(np.abs(got[:, c, :, t] - ref) <= 1e-6 * scale)
    rg.close()
    plan.close()
