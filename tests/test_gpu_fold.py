"""Cyclic co-adding (fewer N-S beams than antennas, Sec. "Redundant arrays and
Fourier transform beamforming") in the FP32 beamformer, against the FP64
oracle, whose beams use the weights n^-1/2 e^{-i 2 pi A a / M} over all n
antennas."""
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


def _plan(bf, w, m_ns, pol_sum=False):
    return bf.Plan(n_ew=4, n_ns=w.n_ns, m_ns=m_ns, n_chan=w.n_chan, n_pol=w.n_pol, block=16, pol_sum=pol_sum,
                   d_over_lambda=w.d_over_lambda())


@pytest.mark.parametrize("n_ns,m_ns,window", [(32, 16, False), (64, 16, True), (256, 16, False),
                                              (256, 128, True), (256, 128, False), (128, 32, False),
                                              (256, 32, True), (256, 64, False), (256, 64, True),
                                              (128, 16, False), (128, 16, True), (64, 32, False)])
def test_fold_parity(n_ns, m_ns, window):
    torch = _torch()
    import paper_1710_08591_amd as bf
    w = sg.custom_workload(n_ew=4, n_ns=n_ns, n_chan=3, n_pol=2, n_time=80, seed=n_ns + m_ns, n_src=2, snr=4.0)
    v = sg.volts(w)
    plan = _plan(bf, w, m_ns)
    h = sg.gaussian_taper(4, n_ns) if window else None
    got = bf.beamform_fft(plan, torch.from_numpy(v).cuda(),
                          taper=None if h is None else torch.from_numpy(h).cuda()).cpu().numpy()
    ref = orc.beamform_fft(v, 4, m_ns, 16, taper=h)
    assert got.shape == ref.shape == (5, 3, 2, 4, m_ns)
    assert rel_err(got, ref) < TOL_FP32
    plan.close()


def test_fold_complex_and_pol_sum():
    torch = _torch()
    import paper_1710_08591_amd as bf
    w = sg.custom_workload(n_ew=4, n_ns=128, n_chan=2, n_pol=2, n_time=48, seed=3, n_src=1, snr=9.0)
    v = sg.volts(w)
    plan = _plan(bf, w, 32)
    z = bf.beamform_fft(plan, torch.from_numpy(v[:19]).cuda(), kind=bf.BF_OUT_COMPLEX).cpu().numpy()
    zr = orc.fft_beams(orc.decode_int4(v[:19]), 4, 32)
    assert z.shape == zr.shape == (19, 2, 2, 4, 32)
    assert np.max(np.abs(z - zr)) < 1e-5 * np.max(np.abs(zr))
    plan.close()
    plan = _plan(bf, w, 64, pol_sum=True)
    got = bf.beamform_fft(plan, torch.from_numpy(v).cuda()).cpu().numpy()
    ref = orc.beamform_fft(v, 4, 64, 16, pol_sum=True)
    assert got.shape == ref.shape == (3, 2, 4, 64)
    assert rel_err(got, ref) < TOL_FP32
    plan.close()


@pytest.mark.parametrize("n_ns,m_ns", [(256, 64), (64, 16), (256, 128), (64, 32)])
def test_fold_complex_even_columns(n_ns, m_ns):
    """Complex beams with cyclic co-adding, with and without a window, and a
    ragged last chunk (19 samples): only the even pass-1 columns are formed;
    pass 2 takes only those at m_ns = 16, 64 and 128 (at 128 with G = 8, two
    frames per pass), and at m_ns = 32 runs the odd columns' tasks on unused
    data whose results are never stored."""
    torch = _torch()
    import paper_1710_08591_amd as bf
    w = sg.custom_workload(n_ew=4, n_ns=n_ns, n_chan=2, n_pol=2, n_time=19, seed=7 + m_ns, n_src=2, snr=6.0)
    v = sg.volts(w)
    vt = torch.from_numpy(v).cuda()
    plan = _plan(bf, w, m_ns)
    for h in (None, sg.gaussian_taper(4, n_ns)):
        z = bf.beamform_fft(plan, vt, kind=bf.BF_OUT_COMPLEX,
                            taper=None if h is None else torch.from_numpy(h).cuda()).cpu().numpy()
        zr = orc.fft_beams(orc.decode_int4(v), 4, m_ns, taper=h)
        assert z.shape == zr.shape == (19, 2, 2, 4, m_ns)
        assert np.max(np.abs(z - zr)) < 1e-5 * np.max(np.abs(zr))
    plan.close()


def test_fold_unsupported_paths():
    torch = _torch()
    import paper_1710_08591_amd as bf
    w = sg.custom_workload(n_ew=4, n_ns=256, n_chan=1, n_pol=1, n_time=32, seed=1)
    vt = torch.from_numpy(sg.volts(w)).cuda()
    plan = _plan(bf, w, 16)                                      # 16-fold
    with pytest.raises(bf.BFError) as e:
        bf.beamform_fft(plan, vt, taper=torch.ones((256, 4), device="cuda"))
    assert e.value.status == bf.BF_ERR_UNSUPPORTED
    with pytest.raises(bf.BFError) as e:
        bf.beamform_fft(plan, vt, gains=torch.ones((256, 4), dtype=torch.complex64, device="cuda"))
    assert e.value.status == bf.BF_ERR_UNSUPPORTED
    with pytest.raises(bf.BFError) as e:
        bf.Regrid(plan, np.zeros(3))
    assert e.value.status == bf.BF_ERR_UNSUPPORTED
    plan.close()
    w2 = sg.custom_workload(n_ew=4, n_ns=128, n_chan=1, n_pol=1, n_time=32, seed=1)
    plan = _plan(bf, w2, 64)
    beams = bf.beamform_fft(plan, torch.from_numpy(sg.volts(w2)).cuda(), kind=bf.BF_OUT_COMPLEX)
    with pytest.raises(bf.BFError) as e:
        bf.form_tied_beams(plan, beams, 0, 1, torch.zeros((2, 2), dtype=torch.float64, device="cuda"))
    assert e.value.status == bf.BF_ERR_UNSUPPORTED
    plan.close()
