"""The E-W axis zero-padded to M_ew = 8 (>= 2 n_ew - 1) and exact 2-D intensity
regridding (eq. e:bp_max_arbitrary on both axes) on the GPU, against the FP64
oracle.  The odd E-W beams come from a second pass over the voltages with the
per-antenna factors W_8^{a_ew}."""
import numpy as np
import pytest

import oracle as orc
import synthgen as sg
from tests.helpers import TOL_FP32, rel_err

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _plan(bf, w, m_ew=8, pol_sum=False, sel=None):
    return bf.Plan(n_ew=4, n_ns=w.n_ns, m_ew=m_ew, n_chan=w.n_chan, n_pol=w.n_pol, block=16, pol_sum=pol_sum,
                   ns_select=sel, d_over_lambda=w.d_over_lambda())


@pytest.mark.parametrize("n_ns,window", [(16, None), (64, "real"), (256, None), (128, "gains"), (256, "real"),
                                          (256, "gains")])
def test_ew8_beams_parity(n_ns, window):
    torch = _torch()
    import paper_1710_08591_amd as bf
    w = sg.custom_workload(n_ew=4, n_ns=n_ns, n_chan=3, n_pol=2, n_time=96, seed=n_ns, n_src=2, snr=6.0)
    v = sg.volts(w)
    plan = _plan(bf, w)
    kw, h = {}, None
    if window == "real":
        h = sg.gaussian_taper(4, n_ns)
        kw["taper"] = torch.from_numpy(h).cuda()
    elif window == "gains":
        rng = np.random.default_rng(2)
        h = np.exp(0.2 * rng.normal(size=(n_ns, 4)) + 1j * rng.uniform(-3, 3, (n_ns, 4))).astype(np.complex64)
        kw["gains"] = torch.from_numpy(h).cuda()
    got = bf.beamform_fft(plan, torch.from_numpy(v).cuda(), **kw).cpu().numpy()
    ref = orc.beamform_fft(v, 8, 2 * n_ns, 16, taper=None if h is None else h.astype(
        np.complex128 if np.iscomplexobj(h) else np.float64))
    assert got.shape == ref.shape == (6, 3, 2, 8, 2 * n_ns)
    assert rel_err(got, ref) < TOL_FP32
    z = bf.beamform_fft(plan, torch.from_numpy(v[:21]).cuda(), kind=bf.BF_OUT_COMPLEX, **kw).cpu().numpy()
    zr = orc.fft_beams(orc.decode_int4(v[:21]), 8, 2 * n_ns, taper=None if h is None else h.astype(
        np.complex128 if np.iscomplexobj(h) else np.float64))
    assert np.max(np.abs(z - zr)) < 1e-5 * np.max(np.abs(zr))
    plan.close()


@pytest.mark.parametrize("n_ns,keep,pol_sum", [(32, 20, True), (256, 200, True), (256, 256, False)])
def test_ew8_clamp_and_pol_sum(n_ns, keep, pol_sum):
    """Clamped and polarisation-summed padded-E-W intensities; at n_ns = 256
    one launch forms the even and the odd E-W beams."""
    torch = _torch()
    import paper_1710_08591_amd as bf
    w = sg.custom_workload(n_ew=4, n_ns=n_ns, n_chan=3, n_pol=2, n_time=64, seed=9 + n_ns, n_ns_keep=keep)
    v = sg.volts(w)
    plan = _plan(bf, w, pol_sum=pol_sum, sel=w.ns_select())
    got = bf.beamform_fft(plan, torch.from_numpy(v).cuda()).cpu().numpy()
    ref = orc.beamform_fft(v, 8, 2 * n_ns, 16, ns_select=w.ns_select(), pol_sum=pol_sum)
    assert got.shape == ref.shape == ((4, 3, 8, keep) if pol_sum else (4, 3, 2, 8, keep))
    assert rel_err(got, ref) < TOL_FP32
    plan.close()


def _abs_scale(b, y_ew, y_ns, n_ew, n_ns):
    """sum over beams of |w_ew| |w_ns| |b|: the size of the regridding sum."""
    m_ew, m_ns = b.shape[-2], b.shape[-1]
    out = np.empty(b.shape[:-2] + (len(y_ew),))
    for p in range(len(y_ew)):
        wgt = np.outer(np.abs(orc.regrid_weights_paper(n_ew, m_ew, y_ew[p])),
                       np.abs(orc.regrid_weights_paper(n_ns, m_ns, y_ns[p])))
        out[..., p] = np.tensordot(np.abs(b), wgt, axes=([-2, -1], [0, 1]))
    return out


@pytest.mark.parametrize("n_ns,n_point,pol_sum", [(16, 37, False), (64, 64, True), (256, 300, False)])
def test_regrid2d_kernel_on_oracle_intensities(n_ns, n_point, pol_sum):
    torch = _torch()
    import paper_1710_08591_amd as bf
    n_blk = 9 if n_ns < 256 else 3
    w = sg.custom_workload(n_ew=4, n_ns=n_ns, n_chan=3, n_pol=2, n_time=16 * n_blk, seed=5, n_src=3, snr=2.0,
                           dl=(0.4, 0.9))
    x = orc.beamform_fft(sg.volts(w), 8, 2 * n_ns, 16, pol_sum=pol_sum).astype(np.float32)
    plan = _plan(bf, w, pol_sum=pol_sum)
    dirs = sg.pointings(n_point, 4)
    rg = bf.Regrid2D(plan, dirs)
    got = rg(torch.from_numpy(x).cuda()).cpu().numpy()
    dl = w.d_over_lambda()
    x64 = x.astype(np.float64)
    assert got.shape == x.shape[:-2] + (n_point,)
    for c in range(3):
        ye, yn = dl[c, 0] * dirs[:, 0], dl[c, 1] * dirs[:, 1]
        ref = orc.regrid_intensity_2d(x64[:, c], ye, yn, 4, n_ns)
        scale = _abs_scale(x64[:, c], ye, yn, 4, n_ns)
        assert np.all(np.abs(got[:, c] - ref) <= 2e-6 * scale)
    rg.close()
    plan.close()


def test_regrid2d_chain_equals_phased_beams():
    """Voltages -> FP32 FFT beams on the 8 x 32 padded grid -> 2-D regridding,
    against the direct phased beams at the same pointings (the plain
    definition the method reaches exactly), to the FP32 bar carried through
    the weights."""
    torch = _torch()
    import paper_1710_08591_amd as bf
    w = sg.custom_workload(n_ew=4, n_ns=16, n_chan=4, n_pol=2, n_time=256, seed=12, n_src=3, snr=5.0,
                           dl=(0.4, 0.8))
    v = sg.volts(w)
    plan = _plan(bf, w)
    dirs = np.concatenate([sg.pointings(50, 7), [[0.0, 0.0], [0.99, -0.99]]], axis=0)
    fft_i = bf.beamform_fft(plan, torch.from_numpy(v).cuda())
    rg = bf.Regrid2D(plan, dirs)
    got = rg(fft_i).cpu().numpy()
    ref = orc.tied_intensity(v, dirs, w.d_over_lambda(), 16)
    b = orc.beamform_fft(v, 8, 32, 16)
    dl = w.d_over_lambda()
    for c in range(4):
        scale = _abs_scale(b[:, c], dl[c, 0] * dirs[:, 0], dl[c, 1] * dirs[:, 1], 4, 16)
        assert np.all(np.abs(got[:, c] - ref[:, c]) <= TOL_FP32 * scale)
    rg.close()
    plan.close()


def test_ew8_unsupported_paths():
    torch = _torch()
    import paper_1710_08591_amd as bf
    w = sg.custom_workload(n_ew=4, n_ns=16, n_chan=2, n_pol=1, n_time=64, seed=1)
    plan8 = _plan(bf, w)
    plan4 = _plan(bf, w, m_ew=4)
    with pytest.raises(bf.BFError) as e:
        bf.Regrid2D(plan4, np.zeros((3, 2)))
    assert e.value.status == bf.BF_ERR_UNSUPPORTED
    with pytest.raises(bf.BFError) as e:
        bf.form_tied_beams_v(plan8, torch.from_numpy(sg.volts(w)).cuda(), 0, 2,
                             torch.zeros((3, 2), dtype=torch.float64, device="cuda"))
    assert e.value.status == bf.BF_ERR_UNSUPPORTED
    with pytest.raises(bf.BFError) as e:
        bf.Plan(n_ew=4, n_ns=16, m_ew=8, block=16, precision=bf.BF_PREC_FP16_MFMA)
    assert e.value.status == bf.BF_ERR_UNSUPPORTED
    with pytest.raises(bf.BFError) as e:
        bf.Server(plan8, ring_samples=1024, hbm_budget=1 << 24, blocks_per_tile=4, max_tiles_per_launch=16)
    assert e.value.status == bf.BF_ERR_UNSUPPORTED
    plan8.close()
    plan4.close()


def test_regrid2d_c2_shape_sampled():
    """CHIME-shaped lattice with the E-W axis padded to 8 (4 x 256 antennas,
    8 x 512 beams, 256 channels, 2 pols, 16384 samples), 256 2-D pointings;
    sampled (block, channel) outputs against the direct phased beams."""
    torch = _torch()
    import paper_1710_08591_amd as bf
    w = sg.make_workload("c2")
    plan = bf.Plan(n_ew=4, n_ns=256, m_ew=8, n_chan=256, n_pol=2, block=16, d_over_lambda=w.d_over_lambda())
    dirs = sg.pointings(256, 12)
    rg = bf.Regrid2D(plan, dirs)
    v = sg.volts(w, backend="torch", device="cuda")
    fft_i = bf.beamform_fft(plan, v)
    del v
    got = rg(fft_i)
    torch.cuda.synchronize()
    assert got.shape == (1024, 256, 2, 256)
    rng = np.random.default_rng(6)
    dl = w.d_over_lambda()
    for blk, c in [(0, 0), (1023, 255)] + [(int(rng.integers(1024)), int(rng.integers(256))) for _ in range(2)]:
        vs = sg.volts(w, blk * 16, 16, chans=[c])
        ref = orc.tied_intensity(vs, dirs, dl, 16, chans=[c])[0, 0]
        b = orc.beamform_fft(vs, 8, 512, 16)[0, 0]
        scale = _abs_scale(b, dl[c, 0] * dirs[:, 0], dl[c, 1] * dirs[:, 1], 4, 256)
        assert np.all(np.abs(got[blk, c].cpu().numpy() - ref) <= TOL_FP32 * scale)
    rg.close()
    plan.close()
    del fft_i, got
    torch.cuda.empty_cache()


@pytest.mark.parametrize("block", [4, 48])
def test_ew8_fused_block_lengths(block):
    """The one-launch padded-E-W kernel of the 4 x 256 lattice (the N-S
    transform of the four E-W antenna columns, then all eight E-W beams per
    N-S beam); blocks of 4 and 48 samples (several blocks per channel, the
    frame prefetch crossing block and polarisation boundaries) against the
    oracle."""
    torch = _torch()
    import paper_1710_08591_amd as bf
    w = sg.custom_workload(n_ew=4, n_ns=256, n_chan=2, n_pol=2, n_time=96, seed=block, n_src=2, snr=5.0)
    v = sg.volts(w)
    plan = bf.Plan(n_ew=4, n_ns=256, m_ew=8, n_chan=2, n_pol=2, block=block, d_over_lambda=w.d_over_lambda())
    got = bf.beamform_fft(plan, torch.from_numpy(v).cuda()).cpu().numpy()
    plan.close()
    ref = orc.beamform_fft(v, 8, 512, block)
    assert got.shape == ref.shape == (96 // block, 2, 2, 8, 512)
    assert rel_err(got, ref) < TOL_FP32


@pytest.mark.parametrize("window", [None, "real", "gains"])
def test_ew8_fused_partial_workgroup(window):
    """The one-launch padded-E-W kernels of the 4 x 256 lattice with a task
    count that leaves the last workgroup partly empty (5 blocks x 3 channels
    x 1 polarisation = 15 tasks for four-wavefront workgroups), a clamp to
    200 N-S beams, unwindowed, with a real window and with complex gains."""
    torch = _torch()
    import paper_1710_08591_amd as bf
    w = sg.custom_workload(n_ew=4, n_ns=256, n_chan=3, n_pol=1, n_time=80, seed=31, n_src=2, snr=5.0,
                           n_ns_keep=200)
    v = sg.volts(w)
    sel = w.ns_select()
    plan = _plan(bf, w, sel=sel)
    kw, h = {}, None
    if window == "real":
        h = sg.gaussian_taper(4, 256)
        kw["taper"] = torch.from_numpy(h).cuda()
    elif window == "gains":
        rng = np.random.default_rng(5)
        h = np.exp(0.2 * rng.normal(size=(256, 4)) + 1j * rng.uniform(-3, 3, (256, 4))).astype(np.complex64)
        kw["gains"] = torch.from_numpy(h).cuda()
    got = bf.beamform_fft(plan, torch.from_numpy(v).cuda(), **kw).cpu().numpy()
    plan.close()
    ref = orc.beamform_fft(v, 8, 512, 16, ns_select=sel, taper=None if h is None else h.astype(
        np.complex128 if np.iscomplexobj(h) else np.float64))
    assert got.shape == ref.shape == (5, 3, 1, 8, 200)
    assert rel_err(got, ref) < TOL_FP32
