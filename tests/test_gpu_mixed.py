"""Mixed-precision (FP16 / FP8 MFMA) beamformer against the FP64 oracle.

The target is <= 1e-3 relative beam power per variant (the int4 inputs are
exact in both formats; the DFT coefficients are split into two FP16 or three
scaled FP8 terms, accumulation in FP32).
"""
import numpy as np
import pytest

import oracle as orc
import synthgen as sg
from tests.helpers import c2_wide_worst, plan_for, rel_err

pytestmark = pytest.mark.gpu

TOL_MIXED = 1e-3


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _run(w, v, prec, pol_sum=False, clamp=True, block=None):
    torch = _torch()
    import paper_1710_08591_amd as bf
    plan = plan_for(w, precision=prec, pol_sum=pol_sum, clamp=clamp, block=block)
    out = bf.beamform_fft(plan, torch.from_numpy(np.ascontiguousarray(v)).cuda())
    torch.cuda.synchronize()
    plan.close()
    return out.cpu().numpy()


@pytest.mark.parametrize("prec", [1, 2])
def test_c4_variant_error(prec):
    """Same bytes as the tiny workload; per-variant relative beam-power error."""
    w = sg.make_workload("c4")
    v = sg.volts(w)
    ref = orc.beamform_fft(v, w.m_ew, w.m_ns, w.block)
    got = _run(w, v, prec)
    err = rel_err(got, ref)
    print(f"precision {prec}: max rel beam-power error {err:.3e}")
    assert err < TOL_MIXED
    if prec == 1:
        assert err < 1e-5          # FP16 hi+lo is FP32-grade


@pytest.mark.parametrize("prec", [1, 2])
def test_mixed_channels_pols_clamp(prec):
    w = sg.custom_workload(n_ew=4, n_ns=16, n_chan=3, n_pol=2, n_time=160, seed=31, n_src=3, snr=6.0,
                           n_ns_keep=20, dl=(0.4, 0.8))
    v = sg.volts(w)
    ref = orc.beamform_fft(v, 4, 32, 16, ns_select=w.ns_select())
    assert rel_err(_run(w, v, prec), ref) < TOL_MIXED
    refp = orc.beamform_fft(v, 4, 32, 16, ns_select=w.ns_select(), pol_sum=True)
    assert rel_err(_run(w, v, prec, pol_sum=True), refp) < TOL_MIXED
    ref32 = orc.beamform_fft(v, 4, 32, 32, ns_select=w.ns_select())
    assert rel_err(_run(w, v, prec, block=32), ref32) < TOL_MIXED


@pytest.mark.parametrize("prec", [1, 2])
def test_mixed_point_source_and_extremes(prec):
    for q in [(0, 0), (1, 2), (3, 3)]:
        v = sg.point_source_volts(4, 16, q[0], q[1], 32, 7)
        w = sg.custom_workload(n_ew=4, n_ns=16, n_time=32, n_src=0)
        got = _run(w, v, prec, clamp=False)
        ref = orc.beamform_fft(v, 4, 32, 16)
        assert np.max(np.abs(got - ref)) / ref.max() < TOL_MIXED
    for b in (0x88, 0x77, 0x8F):
        v = np.full((16, 1, 1, 16, 4), b, dtype=np.uint8)
        got = _run(w, v, prec, clamp=False)
        ref = orc.beamform_fft(v, 4, 32, 16)
        assert np.max(np.abs(got - ref)) / ref.max() < TOL_MIXED


def test_mixed_repeatable_and_unsupported():
    torch = _torch()
    import paper_1710_08591_amd as bf
    w = sg.custom_workload(n_ew=4, n_ns=16, n_chan=4, n_pol=2, n_time=256, seed=2)
    v = torch.from_numpy(sg.volts(w)).cuda()
    plan = plan_for(w, precision=2, clamp=False)
    a = bf.beamform_fft(plan, v)
    b = bf.beamform_fft(plan, v)
    assert torch.equal(a, b)
    with pytest.raises(bf.BFError) as e:
        bf.beamform_fft(plan, v, taper=torch.ones((16, 4), device="cuda"))
    assert e.value.status == bf.BF_ERR_UNSUPPORTED
    plan.close()
    with pytest.raises(bf.BFError) as e:
        bf.Plan(n_ns=32, m_ew=8, precision=1)
    assert e.value.status == bf.BF_ERR_UNSUPPORTED
    with pytest.raises(bf.BFError) as e:
        bf.Plan(n_ns=64, m_ns=32, precision=2)
    assert e.value.status == bf.BF_ERR_UNSUPPORTED


@pytest.mark.parametrize("prec", [1, 2])
def test_mix256_chime_lattice_parity(prec):
    """Stage 1 of 512 = 32 x 16 on the matrix cores (FP16: exact E-W sums and
    two-term coefficients; FP8: exact int4 columns and three stacked terms),
    stage 2 in FP32, on the 4 x 256 lattice with a clamp, summed pols, and
    one block of 48 samples without a clamp."""
    w = sg.custom_workload(n_ew=4, n_ns=256, n_chan=3, n_pol=2, n_time=48, seed=77, n_src=4, snr=10.0,
                           n_ns_keep=256, dl=(0.4, 0.8))
    v = sg.volts(w)
    ref = orc.beamform_fft(v, 4, 512, 16, ns_select=w.ns_select())
    got = _run(w, v, prec)
    err = rel_err(got, ref)
    print(f"4x256 precision {prec}: max rel beam-power error {err:.3e}")
    assert err < (1e-5 if prec == 1 else TOL_MIXED)
    refp = orc.beamform_fft(v, 4, 512, 16, ns_select=w.ns_select(), pol_sum=True)
    assert rel_err(_run(w, v, prec, pol_sum=True), refp) < TOL_MIXED
    unc = _run(w, v, prec, clamp=False, block=48)
    assert rel_err(unc, orc.beamform_fft(v, 4, 512, 48)) < TOL_MIXED


@pytest.mark.parametrize("prec", [1, 2])
def test_mix256_extremes_and_point_source(prec):
    """Constant extreme voltages (-8 - 8i, 7 + 7i, 1 - 8i) and a lattice-aligned
    point source of amplitude 7, against the oracle's peak power."""
    w = sg.custom_workload(n_ew=4, n_ns=256, n_time=16, n_src=0)
    for b in (0x88, 0x77, 0x18):
        v = np.full((16, 1, 1, 256, 4), b, dtype=np.uint8)
        got = _run(w, v, prec, clamp=False)
        ref = orc.beamform_fft(v, 4, 512, 16)
        assert np.max(np.abs(got - ref)) / ref.max() < TOL_MIXED
    v = sg.point_source_volts(4, 256, 1, 3, 16, 7)
    got = _run(w, v, prec, clamp=False)
    ref = orc.beamform_fft(v, 4, 512, 16)
    assert np.max(np.abs(got - ref)) / ref.max() < TOL_MIXED


@pytest.mark.parametrize("prec", [1, 2])
def test_mix256_c2_full_size_sampled(prec):
    """The CHIME-shaped workload at full size through the FP16- and FP8-MFMA
    plans, in the launch configuration the benchmark times, against the
    oracle: every channel and both polarisations of the first and the last
    block, and one channel over all 1024 blocks.  The bar is the
    mixed-precision 1e-3; FP16 (exact data, two-term coefficients, FP32
    stage 2) is meant to stay within the FP32 bar (1e-5) as well, which the
    second assertion holds it to."""
    torch = _torch()
    import paper_1710_08591_amd as bf
    w = sg.make_workload("c2")
    plan = plan_for(w, precision=prec)
    v = sg.volts(w, backend="torch", device="cuda")
    out = bf.beamform_fft(plan, v)
    torch.cuda.synchronize()
    assert out.shape == (1024, 256, 2, 4, 256)
    sel = w.ns_select()
    worst = c2_wide_worst(w, v, out, lambda x, ch: orc.beamform_fft(x, w.m_ew, w.m_ns, 16, ns_select=sel[ch]))
    print(f"4x256 precision {prec}, full size: max rel beam-power error {worst:.3e}")
    assert worst < TOL_MIXED
    if prec == 1:
        assert worst < 1e-5
    plan.close()
    del v, out
    torch.cuda.empty_cache()


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_lattice4x16_scaled_full_size_sampled(prec):
    """The scaled 4 x 16 workload of the precision comparison (2 pol, 256
    channels, 16384 samples) at full size, each precision in the launch
    configuration the benchmark times; sampled outputs against the oracle."""
    torch = _torch()
    import paper_1710_08591_amd as bf
    w = sg.Workload("lattice4x16_scaled", 4, 16, 256, 2, 16384, 4, 32, 16, 6,
                    src_dircos=((0.3, -0.2), (-0.7, 0.5)), src_snr=(10.0, 30.0), dl_lo=0.4, dl_hi=0.8)
    v = sg.volts(w, backend="torch", device="cuda")
    plan = bf.Plan(n_ew=4, n_ns=16, n_pol=2, n_chan=256, block=16, precision=prec)
    out = bf.beamform_fft(plan, v)
    torch.cuda.synchronize()
    assert out.shape == (1024, 256, 2, 4, 32)
    rng = np.random.default_rng(2)
    picks = [(0, 0, 0), (1023, 255, 1)] + [tuple(int(x) for x in (rng.integers(1024), rng.integers(256),
                                                                  rng.integers(2))) for _ in range(4)]
    worst = 0.0
    for blk, c, p in picks:
        vs = sg.volts(w, blk * 16, 16, chans=[c], pols=[p])
        ref = orc.beamform_fft(vs, 4, 32, 16)[0, 0, 0]
        worst = max(worst, rel_err(out[blk, c, p].cpu().numpy(), ref))
    assert worst < (1e-5 if prec < 2 else TOL_MIXED), worst
    plan.close()
    del v, out
    torch.cuda.empty_cache()


@pytest.mark.parametrize("scale", [1.0, 40.0, 1e-3])
def test_mix256_window_parity(scale):
    """Per-antenna real weights on the FP16 matrix-core path at the 4 x 256
    lattice (Sec. "Controlling beam shape with windowing"): the windowed E-W
    sums are split into FP16 hi + lo terms, so the result is held to the FP32
    bar.  Weights scaled by 40 and 1e-3 test the per-wavefront power-of-two
    scaling that keeps the low terms in FP16's normal range."""
    w = sg.custom_workload(n_ew=4, n_ns=256, n_chan=3, n_pol=2, n_time=48, seed=91, n_src=3, snr=12.0,
                           n_ns_keep=256, dl=(0.4, 0.8))
    v = sg.volts(w)
    h = (sg.gaussian_taper(4, 256) * scale).astype(np.float32)
    torch = _torch()
    import paper_1710_08591_amd as bf
    vt = torch.from_numpy(v).cuda()
    ht = torch.from_numpy(h).cuda()
    h64 = h.astype(np.float64)
    for pol_sum in (False, True):
        plan = plan_for(w, precision=1, pol_sum=pol_sum)
        got = bf.beamform_fft(plan, vt, taper=ht).cpu().numpy()
        plan.close()
        ref = orc.beamform_fft(v, 4, 512, 16, taper=h64, ns_select=w.ns_select(), pol_sum=pol_sum)
        err = rel_err(got, ref)
        print(f"4x256 FP16 MFMA with window x{scale}, pol_sum={pol_sum}: max rel beam-power error {err:.3e}")
        assert err < 1e-5
    plan = plan_for(w, precision=2)
    with pytest.raises(bf.BFError) as e:
        bf.beamform_fft(plan, vt, taper=ht)
    assert e.value.status == bf.BF_ERR_UNSUPPORTED
    plan.close()


def test_mix256_window_c2_full_size():
    """The Gaussian window on the CHIME-shaped workload at full size through the
    FP16 matrix-core plan, against the oracle over the full-size comparison
    set, held to the FP32 bar."""
    torch = _torch()
    import paper_1710_08591_amd as bf
    w = sg.make_workload("c2")
    plan = plan_for(w, precision=1)
    h = sg.gaussian_taper(w.n_ew, w.n_ns).astype(np.float32)
    v = sg.volts(w, backend="torch", device="cuda")
    out = bf.beamform_fft(plan, v, taper=torch.from_numpy(h).cuda())
    torch.cuda.synchronize()
    sel = w.ns_select()
    h64 = h.astype(np.float64)
    worst = c2_wide_worst(w, v, out, lambda x, ch: orc.beamform_fft(x, w.m_ew, w.m_ns, 16, taper=h64,
                                                                      ns_select=sel[ch]))
    print(f"4x256 FP16 MFMA with window, full size: max rel beam-power error {worst:.3e}")
    assert worst < 1e-5
    plan.close()
    del v, out
    torch.cuda.empty_cache()


@pytest.mark.parametrize("scale", [1.0, 40.0, 1e-3])
def test_mix16_window_parity(scale):
    """Per-antenna real weights on the FP16 matrix-core path of the 4 x 16
    lattice: the C3-shaped Gaussian window (width 0.4 of the aperture) on the
    tiny workload's bytes, and a half-sine window over several channels, pols
    and a clamp, held to the FP32 bar; scaled weights test the per-wavefront
    power-of-two scaling."""
    torch = _torch()
    import paper_1710_08591_amd as bf
    w = sg.make_workload("c3")
    v = sg.volts(w)
    h = (sg.gaussian_taper(4, 16) * scale).astype(np.float32)
    plan = plan_for(w, precision=1)
    got = bf.beamform_fft(plan, torch.from_numpy(v).cuda(), taper=torch.from_numpy(h).cuda()).cpu().numpy()
    plan.close()
    ref = orc.beamform_fft(v, 4, 32, 16, taper=h.astype(np.float64))
    err = rel_err(got, ref)
    print(f"C3 shape, FP16 MFMA with window x{scale}: max rel beam-power error {err:.3e}")
    assert err < 1e-5
    w2 = sg.custom_workload(n_ew=4, n_ns=16, n_chan=3, n_pol=2, n_time=96, seed=23, n_src=2, snr=8.0,
                            n_ns_keep=20, dl=(0.4, 0.8))
    v2 = sg.volts(w2)
    h2 = (sg.half_sine_taper(4, 16, shifted=True) * scale).astype(np.float32)
    for pol_sum in (False, True):
        plan = plan_for(w2, precision=1, pol_sum=pol_sum)
        got = bf.beamform_fft(plan, torch.from_numpy(v2).cuda(), taper=torch.from_numpy(h2).cuda()).cpu().numpy()
        plan.close()
        ref = orc.beamform_fft(v2, 4, 32, 16, taper=h2.astype(np.float64), ns_select=w2.ns_select(),
                               pol_sum=pol_sum)
        assert rel_err(got, ref) < 1e-5


# ---- 4 x 32, 4 x 64, 4 x 128: polyphase split onto the 16 -> 32 products ----

@pytest.mark.parametrize("n_ns", [32, 64, 128])
@pytest.mark.parametrize("prec", [1, 2])
def test_mixp_lattice_parity(n_ns, prec):
    """n = 16 R positions (R = 2, 4, 8) on the matrix cores: R zero-padded
    16 -> 32 products per E-W beam (FP16: exact E-W sums, two-term
    coefficients; FP8: exact first-stage E-W sums, three stacked terms), the
    twiddles W_M^{a0 m} and the R-point DFT in FP32 (eq. e:fftbeamform).
    Several channels with their own clamp tables, both pols and summed pols,
    6 blocks of 16 (a run of 4 and a ragged run of 2) and 3 blocks of 32."""
    w = sg.custom_workload(n_ew=4, n_ns=n_ns, n_chan=3, n_pol=2, n_time=96, seed=40 + n_ns, n_src=3, snr=8.0,
                           n_ns_keep=n_ns + n_ns // 4, dl=(0.4, 0.8))
    v = sg.volts(w)
    m = 2 * n_ns
    tol = 1e-5 if prec == 1 else TOL_MIXED
    for pol_sum in (False, True):
        ref = orc.beamform_fft(v, 4, m, 16, ns_select=w.ns_select(), pol_sum=pol_sum)
        err = rel_err(_run(w, v, prec, pol_sum=pol_sum), ref)
        print(f"4x{n_ns} precision {prec}, pol_sum={pol_sum}: max rel beam-power error {err:.3e}")
        assert err < tol
    ref32 = orc.beamform_fft(v, 4, m, 32, ns_select=w.ns_select())
    assert rel_err(_run(w, v, prec, block=32), ref32) < tol
    # no clamp: every one of the 2 n beams
    w1 = sg.custom_workload(n_ew=4, n_ns=n_ns, n_chan=2, n_pol=1, n_time=48, seed=7 + n_ns, n_src=2, snr=10.0)
    v1 = sg.volts(w1)
    assert rel_err(_run(w1, v1, prec, clamp=False), orc.beamform_fft(v1, 4, m, 16)) < tol


@pytest.mark.parametrize("n_ns", [32, 64, 128])
@pytest.mark.parametrize("prec", [1, 2])
def test_mixp_point_source_and_extremes(n_ns, prec):
    """Lattice-aligned point sources and constant extreme bytes (-8 / +7
    nibbles) through the polyphase matrix-core kernels."""
    w = sg.custom_workload(n_ew=4, n_ns=n_ns, n_time=32, n_src=0)
    tol = 1e-5 if prec == 1 else TOL_MIXED
    for q in [(0, 0), (1, 2), (3, 3)]:
        v = sg.point_source_volts(4, n_ns, q[0], q[1], 32, 7)
        got = _run(w, v, prec, clamp=False)
        ref = orc.beamform_fft(v, 4, 2 * n_ns, 16)
        assert np.max(np.abs(got - ref)) / ref.max() < tol
    for b in (0x88, 0x77, 0x8F):
        v = np.full((16, 1, 1, n_ns, 4), b, dtype=np.uint8)
        got = _run(w, v, prec, clamp=False)
        ref = orc.beamform_fft(v, 4, 2 * n_ns, 16)
        assert np.max(np.abs(got - ref)) / ref.max() < tol


@pytest.mark.parametrize("n_ns", [32, 64, 128])
@pytest.mark.parametrize("scale", [1.0, 1e-3])
def test_mixp_window_parity(n_ns, scale):
    """Per-antenna real weights on the FP16 polyphase path (Sec. "Controlling
    beam shape with windowing"): windowed E-W sums split into FP16 hi + lo,
    three products per tile, per-wavefront power-of-two scaling; held to the
    FP32 bar.  An FP8 plan refuses a window."""
    torch = _torch()
    import paper_1710_08591_amd as bf
    w = sg.custom_workload(n_ew=4, n_ns=n_ns, n_chan=2, n_pol=2, n_time=64, seed=60 + n_ns, n_src=2, snr=10.0,
                           n_ns_keep=n_ns, dl=(0.45, 0.9))
    v = sg.volts(w)
    vt = torch.from_numpy(v).cuda()
    for h in (sg.gaussian_taper(4, n_ns) * scale, sg.half_sine_taper(4, n_ns, shifted=True) * scale):
        h = h.astype(np.float32)
        ht = torch.from_numpy(h).cuda()
        for pol_sum in (False, True):
            plan = plan_for(w, precision=1, pol_sum=pol_sum)
            got = bf.beamform_fft(plan, vt, taper=ht).cpu().numpy()
            plan.close()
            ref = orc.beamform_fft(v, 4, 2 * n_ns, 16, taper=h.astype(np.float64), ns_select=w.ns_select(),
                                   pol_sum=pol_sum)
            err = rel_err(got, ref)
            print(f"4x{n_ns} FP16 MFMA with window x{scale}, pol_sum={pol_sum}: {err:.3e}")
            assert err < 1e-5
    plan = plan_for(w, precision=2)
    with pytest.raises(bf.BFError) as e:
        bf.beamform_fft(plan, vt, taper=ht)
    assert e.value.status == bf.BF_ERR_UNSUPPORTED
    plan.close()


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_lattice4x16_pol_pairs_across_workgroups(prec):
    """The 4 x 16 kernels place the two polarisations of a frame line 8
    workgroups apart; with 5 channels and 20 blocks the grid has a part
    that is a multiple of 16 and a tail in plain order (50 workgroups for
    the matrix-core kernels, 200 for FP32), and every (block, channel, pol)
    must still land in its own slot."""
    w = sg.custom_workload(n_ew=4, n_ns=16, n_chan=5, n_pol=2, n_time=320, seed=77, n_src=2, snr=5.0)
    v = sg.volts(w)
    ref = orc.beamform_fft(v, 4, 32, 16)
    got = _run(w, v, prec, clamp=False)
    assert got.shape == ref.shape == (20, 5, 2, 4, 32)
    assert rel_err(got, ref) < (1e-5 if prec < 2 else TOL_MIXED)
    # each polarisation slot differs from the other (a swapped pair would match the wrong one)
    assert rel_err(got[:, :, 0], ref[:, :, 1]) > 1e-2
