"""GPU parity of the FP32 FFT beamformer against the FP64 oracle (through the C ABI)."""
import numpy as np
import pytest

import oracle as orc
import synthgen as sg
from tests.helpers import TOL_FP32, c2_wide_worst, peak_err, plan_for, rel_err

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _run(w, v_np, taper=None, kind=0, pol_sum=False, clamp=True, block=None):
    torch = _torch()
    import paper_1710_08591_amd as bf
    plan = plan_for(w, pol_sum=pol_sum, clamp=clamp, block=block)
    v = torch.from_numpy(np.ascontiguousarray(v_np)).cuda()
    h = None if taper is None else torch.from_numpy(taper).cuda()
    out = bf.beamform_fft(plan, v, taper=h, kind=kind)
    torch.cuda.synchronize()
    plan.close()
    return out.cpu().numpy()


def test_c1_parity():
    w = sg.make_workload("c1")
    v = sg.volts(w)
    got = _run(w, v)
    ref = orc.beamform_fft(v, w.m_ew, w.m_ns, w.block)
    assert got.shape == ref.shape == (64, 1, 1, 4, 32)
    assert rel_err(got, ref) < TOL_FP32


def test_c1_taper_parity():
    w = sg.make_workload("c3")
    v = sg.volts(w)
    h = sg.gaussian_taper(w.n_ew, w.n_ns)
    got = _run(w, v, taper=h)
    ref = orc.beamform_fft(v, w.m_ew, w.m_ns, w.block, taper=h)
    assert rel_err(got, ref) < TOL_FP32


@pytest.mark.parametrize("n_ns", [16, 32, 64, 128, 256])
@pytest.mark.parametrize("taper", [False, True])
def test_shapes_parity(n_ns, taper):
    """Every supported N-S length, 2 channels x 2 pols, several blocks."""
    w = sg.custom_workload(n_ew=4, n_ns=n_ns, n_chan=2, n_pol=2, n_time=48, seed=n_ns, n_src=2, snr=4.0)
    v = sg.volts(w)
    h = sg.half_sine_taper(4, n_ns, shifted=True) if taper else None
    got = _run(w, v, taper=h, clamp=False)
    ref = orc.beamform_fft(v, w.m_ew, w.m_ns, w.block, taper=h)
    assert rel_err(got, ref) < TOL_FP32


@pytest.mark.parametrize("q", [(0, 0), (1, 2), (3, 1), (2, 3)])
def test_point_source_closed_form_gpu(q):
    """Noise-free lattice-aligned source: compare with the Dirichlet closed form."""
    n_ew, n_ns = 4, 16
    v = sg.point_source_volts(n_ew, n_ns, q[0], q[1], 32, 7)
    w = sg.custom_workload(n_ew=n_ew, n_ns=n_ns, n_time=32, n_src=0)
    got = _run(w, v, clamp=False)[0, 0, 0]
    de = np.array([(np.sin(n_ew * np.pi * d) ** 2 / np.sin(np.pi * d) ** 2) if abs(np.sin(np.pi * d)) > 1e-9 else n_ew ** 2
                   for d in q[0] / 4 - np.arange(4) / 4])
    dn = np.array([(np.sin(n_ns * np.pi * d) ** 2 / np.sin(np.pi * d) ** 2) if abs(np.sin(np.pi * d)) > 1e-9 else n_ns ** 2
                   for d in q[1] / 4 - np.arange(32) / 32])
    ref = 16 * 49 / 64 * de[:, None] * dn[None, :]
    assert peak_err(got, ref) < TOL_FP32
    # even N-S offsets from the peak stay at (rounding-level) zero
    pk = q[1] * 8
    row = got[q[0]]
    assert np.all(row[(pk + np.arange(2, 32, 2)) % 32] <= 1e-5 * row.max())


def test_clamp_and_pol_sum():
    w = sg.custom_workload(n_ew=4, n_ns=64, n_chan=3, n_pol=2, n_time=32, seed=9, n_ns_keep=64, dl=(0.4, 0.8))
    v = sg.volts(w)
    got = _run(w, v)
    ref = orc.beamform_fft(v, w.m_ew, w.m_ns, w.block, ns_select=w.ns_select())
    assert rel_err(got, ref) < TOL_FP32
    unc = _run(w, v, clamp=False)
    sel = w.ns_select()
    for c in range(3):                      # clamp is a bitwise selection
        assert np.array_equal(got[:, c], unc[:, c][..., sel[c]])
    ps = _run(w, v, pol_sum=True)
    refp = orc.beamform_fft(v, w.m_ew, w.m_ns, w.block, ns_select=sel, pol_sum=True)
    assert ps.shape == refp.shape
    assert rel_err(ps, refp) < TOL_FP32


@pytest.mark.parametrize("n_ns,n_time", [(16, 1), (16, 5), (16, 17), (16, 64), (256, 3), (256, 21)])
def test_complex_beams_ragged(n_ns, n_time):
    """Complex FFT beams for every sample, including a ragged last chunk
    (four frames side by side per wavefront at n_ns = 16, one at 256)."""
    w = sg.custom_workload(n_ew=4, n_ns=n_ns, n_chan=2, n_pol=2, n_time=n_time, seed=3)
    v = sg.volts(w)
    got = _run(w, v, kind=1, clamp=False)
    ref = orc.fft_beams(orc.decode_int4(v), 4, 2 * n_ns)
    assert got.shape == ref.shape
    assert np.max(np.abs(got - ref)) / np.max(np.abs(ref)) < 1e-6


@pytest.mark.parametrize("n_ns", [64, 128, 256])
@pytest.mark.parametrize("weights", ["window", "gains"])
def test_weighted_partial_last_workgroup(n_ns, weights):
    """With per-antenna weights several wavefronts share a workgroup and its
    table of weights, one (block, channel, polarisation group) each: 9 tasks
    (3 blocks x 3 channels) leave the last workgroup partly empty, for
    intensities per polarisation and summed, and for complex beams with a
    ragged last chunk."""
    torch = _torch()
    import paper_1710_08591_amd as bf
    rng = np.random.default_rng(n_ns)
    if weights == "window":
        wt = sg.half_sine_taper(4, n_ns, shifted=True)
        ref_wt = wt
    else:
        wt = (np.exp(rng.normal(size=(n_ns, 4)) * 0.3 + 1j * rng.uniform(-np.pi, np.pi, (n_ns, 4)))
              ).astype(np.complex64)
        ref_wt = wt.astype(np.complex128)
    wd = torch.from_numpy(wt).cuda()
    kw = {"taper": wd} if weights == "window" else {"gains": wd}
    for n_pol, n_time in [(1, 48), (2, 48), (1, 37)]:
        w = sg.custom_workload(n_ew=4, n_ns=n_ns, n_chan=3, n_pol=n_pol, n_time=n_time, seed=60 + n_ns,
                               n_src=2, snr=5.0)
        v = sg.volts(w)
        plan = plan_for(w, clamp=False, pol_sum=n_pol == 2)
        vt = torch.from_numpy(v).cuda()
        if n_time == 37:
            got = bf.beamform_fft(plan, vt, kind=bf.BF_OUT_COMPLEX, **kw).cpu().numpy()
            ref = orc.fft_beams(orc.decode_int4(v), 4, 2 * n_ns, taper=ref_wt)
            assert got.shape == ref.shape
            assert np.max(np.abs(got - ref)) / np.max(np.abs(ref)) < 1e-5
        else:
            got = bf.beamform_fft(plan, vt, **kw).cpu().numpy()
            ref = orc.beamform_fft(v, 4, 2 * n_ns, w.block, taper=ref_wt, pol_sum=n_pol == 2)
            assert got.shape == ref.shape
            assert rel_err(got, ref) < TOL_FP32
        plan.close()


def test_block_sizes():
    w = sg.custom_workload(n_ew=4, n_ns=32, n_chan=1, n_pol=1, n_time=96, seed=4)
    v = sg.volts(w)
    for blk in (4, 8, 32, 48):
        got = _run(w, v, clamp=False, block=blk)
        ref = orc.beamform_fft(v, w.m_ew, w.m_ns, blk)
        assert rel_err(got, ref) < TOL_FP32


def test_block_sizes_odd_pass_count():
    """Blocks whose frames take an odd number of passes (four frames side by
    side per pass at n_ns = 16: blocks of 4, 12 and 20 samples), and short
    blocks at n_ns = 256 (one frame per pass)."""
    w = sg.custom_workload(n_ew=4, n_ns=16, n_chan=2, n_pol=2, n_time=120, seed=14)
    v = sg.volts(w)
    for blk in (4, 12, 20):
        got = _run(w, v, clamp=False, block=blk)
        ref = orc.beamform_fft(v, w.m_ew, w.m_ns, blk)
        assert rel_err(got, ref) < TOL_FP32
    w = sg.custom_workload(n_ew=4, n_ns=256, n_chan=1, n_pol=1, n_time=24, seed=15)
    v = sg.volts(w)
    for blk in (4, 12):
        got = _run(w, v, clamp=False, block=blk)
        ref = orc.beamform_fft(v, w.m_ew, w.m_ns, blk)
        assert rel_err(got, ref) < TOL_FP32


def test_extreme_values():
    """All antennas at -8 - 8i (the most negative nibble) and +7 + 7i."""
    torch = _torch()
    for b in (0x88, 0x77):
        w = sg.custom_workload(n_ew=4, n_ns=256, n_time=16, n_src=0)
        v = np.full((16, 1, 1, 256, 4), b, dtype=np.uint8)
        got = _run(w, v, clamp=False)
        ref = orc.beamform_fft(v, 4, 512, 16)
        assert peak_err(got, ref) < TOL_FP32


def test_empty_and_errors():
    torch = _torch()
    import paper_1710_08591_amd as bf
    w = sg.make_workload("c1")
    plan = plan_for(w)
    v = torch.zeros((0, 1, 1, 16, 4), dtype=torch.uint8, device="cuda")
    out = bf.beamform_fft(plan, v)
    assert out.shape == (0, 1, 1, 4, 32)
    v = torch.zeros((24, 1, 1, 16, 4), dtype=torch.uint8, device="cuda")
    with pytest.raises(bf.BFError) as e:
        bf.beamform_fft(plan, v, out=torch.full((1, 1, 1, 4, 32), 7.0, device="cuda"))
    assert e.value.status == bf.BF_ERR_INVALID_ARGUMENT
    plan.close()


def test_repeatable_bitwise():
    torch = _torch()
    import paper_1710_08591_amd as bf
    w = sg.custom_workload(n_ew=4, n_ns=256, n_chan=4, n_pol=2, n_time=256, seed=8)
    plan = plan_for(w, clamp=False)
    v = torch.from_numpy(sg.volts(w)).cuda()
    a = bf.beamform_fft(plan, v)
    b = bf.beamform_fft(plan, v)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    plan.close()


def test_c2_full_size_sampled():
    """The CHIME-shaped workload at full size, in the launch configuration the
    benchmark times, against the oracle: every channel and both polarisations
    of the first and the last block (each channel's own clamp table, eq.
    e:theta_A), and one channel over all 1024 blocks."""
    torch = _torch()
    import paper_1710_08591_amd as bf
    w = sg.make_workload("c2")
    plan = plan_for(w)
    v = sg.volts(w, backend="torch", device="cuda")
    out = bf.beamform_fft(plan, v)
    torch.cuda.synchronize()
    assert out.shape == (1024, 256, 2, 4, 256)
    sel = w.ns_select()
    worst = c2_wide_worst(w, v, out, lambda x, ch: orc.beamform_fft(x, w.m_ew, w.m_ns, 16, ns_select=sel[ch]))
    print(f"4x256 FP32, full size: max rel beam-power error {worst:.3e}")
    assert worst < TOL_FP32
    plan.close()
    del v, out
    torch.cuda.empty_cache()


def test_window_c2_full_size():
    """The per-antenna Gaussian window (width 0.4 of the aperture per axis) on
    the CHIME-shaped workload at full size, in the launch configuration the
    benchmark times, against the oracle over the full-size comparison set."""
    torch = _torch()
    import paper_1710_08591_amd as bf
    w = sg.make_workload("c2")
    plan = plan_for(w)
    h = sg.gaussian_taper(w.n_ew, w.n_ns)
    v = sg.volts(w, backend="torch", device="cuda")
    out = bf.beamform_fft(plan, v, taper=torch.from_numpy(np.ascontiguousarray(h, dtype=np.float32)).cuda())
    torch.cuda.synchronize()
    sel = w.ns_select()
    h64 = np.asarray(h, dtype=np.float32).astype(np.float64)
    worst = c2_wide_worst(w, v, out, lambda x, ch: orc.beamform_fft(x, w.m_ew, w.m_ns, 16, taper=h64,
                                                                      ns_select=sel[ch]))
    print(f"4x256 FP32 with window, full size: max rel beam-power error {worst:.3e}")
    assert worst < TOL_FP32
    plan.close()
    del v, out
    torch.cuda.empty_cache()
