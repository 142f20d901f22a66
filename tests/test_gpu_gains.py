"""Complex per-antenna gains (eq. e:vis_pert, Sec. "Non-redundancy") through
the FP32 FFT beamformer, against the FP64 oracle."""
import numpy as np
import pytest

import oracle as orc
import synthgen as sg
from tests.helpers import TOL_FP32, c2_wide_worst, plan_for, rel_err

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _gains(n_ns, n_ew, seed, amp=0.3, phase=np.pi):
    rng = np.random.default_rng(seed)
    return (np.exp(rng.normal(size=(n_ns, n_ew)) * amp + 1j * rng.uniform(-phase, phase, (n_ns, n_ew)))
            ).astype(np.complex64)


def _run(w, v, g, kind=0, clamp=False, pol_sum=False):
    torch = _torch()
    import paper_1710_08591_amd as bf
    plan = plan_for(w, clamp=clamp, pol_sum=pol_sum)
    out = bf.beamform_fft(plan, torch.from_numpy(v).cuda(), kind=kind,
                          gains=None if g is None else torch.from_numpy(g).cuda())
    torch.cuda.synchronize()
    plan.close()
    return out.cpu().numpy()


@pytest.mark.parametrize("n_ns", [16, 32, 64, 128, 256])
def test_gains_parity(n_ns):
    w = sg.custom_workload(n_ew=4, n_ns=n_ns, n_chan=3, n_pol=2, n_time=160 if n_ns < 256 else 48,
                           seed=n_ns, n_src=2, snr=5.0)
    v = sg.volts(w)
    g = _gains(n_ns, 4, n_ns)
    got = _run(w, v, g)
    ref = orc.beamform_fft(v, 4, 2 * n_ns, 16, taper=g.astype(np.complex128))
    assert got.shape == ref.shape
    assert rel_err(got, ref) < TOL_FP32


def test_gains_complex_output_clamp_polsum():
    w = sg.custom_workload(n_ew=4, n_ns=64, n_chan=2, n_pol=2, n_time=37, seed=5, n_src=1, snr=8.0,
                           n_ns_keep=40)
    v = sg.volts(w)
    g = _gains(64, 4, 9)
    import paper_1710_08591_amd as bf
    z = _run(w, v, g, kind=bf.BF_OUT_COMPLEX)
    ref = orc.fft_beams(orc.decode_int4(v), 4, 128, taper=g.astype(np.complex128))
    assert np.max(np.abs(z - ref)) < 1e-5 * np.max(np.abs(ref))
    vb = v[:32]
    got = _run(w, vb, g, clamp=True, pol_sum=True)
    ref = orc.beamform_fft(vb, 4, 128, 16, taper=g.astype(np.complex128), ns_select=w.ns_select(), pol_sum=True)
    assert rel_err(got, ref) < TOL_FP32


def test_real_gains_equal_the_window():
    torch = _torch()
    import paper_1710_08591_amd as bf
    w = sg.custom_workload(n_ew=4, n_ns=256, n_chan=2, n_pol=1, n_time=64, seed=3, snr=3.0)
    v = sg.volts(w)
    h = sg.gaussian_taper(4, 256)
    plan = plan_for(w, clamp=False)
    vt = torch.from_numpy(v).cuda()
    a = bf.beamform_fft(plan, vt, taper=torch.from_numpy(h).cuda())
    b = bf.beamform_fft(plan, vt, gains=torch.from_numpy(h.astype(np.complex64)).cuda())
    assert rel_err(b.cpu().numpy(), a.cpu().numpy()) < 1e-6
    plan.close()


@pytest.mark.parametrize("shift", [1, 7, -3])
def test_phase_ramp_gains_shift_the_beams(shift):
    """g_a = e^{+i 2 pi a_ns D / M}: the N-S beams move by D (the shift theorem)."""
    w = sg.custom_workload(n_ew=4, n_ns=128, n_chan=2, n_pol=1, n_time=64, seed=4, n_src=2, snr=10.0)
    v = sg.volts(w)
    a_ns = np.arange(128)[:, None] * np.ones((1, 4))
    g = np.exp(2j * np.pi * a_ns * shift / 256).astype(np.complex64)
    plain = _run(w, v, None)
    ramp = _run(w, v, g)
    assert rel_err(ramp, np.roll(plain, shift, axis=-1)) < 2e-6


def test_gains_errors():
    torch = _torch()
    import paper_1710_08591_amd as bf
    w = sg.make_workload("c1")
    v = torch.from_numpy(sg.volts(w)).cuda()
    plan = plan_for(w)
    with pytest.raises(ValueError):
        bf.beamform_fft(plan, v, taper=torch.ones((16, 4), device="cuda"),
                        gains=torch.ones((16, 4), dtype=torch.complex64, device="cuda"))
    st = bf.lib().bf_beamform_fft_gains(plan.handle, bf._ptr(v), 1024, None, 0,
                                        bf._ptr(torch.empty((64, 1, 1, 4, 32), device="cuda")), None)
    assert st == bf.BF_ERR_INVALID_ARGUMENT
    plan.close()
    mixed = bf.Plan(n_ew=4, n_ns=16, block=16, precision=bf.BF_PREC_FP16_MFMA)
    with pytest.raises(bf.BFError) as e:
        bf.beamform_fft(mixed, v, gains=torch.ones((16, 4), dtype=torch.complex64, device="cuda"))
    assert e.value.status == bf.BF_ERR_UNSUPPORTED
    mixed.close()


def test_gains_c2_full_size_sampled():
    """Complex per-antenna gains on the CHIME-shaped workload at full size, in
    the launch configuration the benchmark times, against the oracle with the
    same gains over the full-size comparison set (every channel and both
    polarisations of the first and the last block, one channel over every
    block)."""
    torch = _torch()
    import paper_1710_08591_amd as bf
    w = sg.make_workload("c2")
    plan = plan_for(w)
    grng = np.random.default_rng(17)
    gains = np.exp(0.1 * grng.normal(size=(w.n_ns, w.n_ew)) + 0.1j * grng.normal(size=(w.n_ns, w.n_ew)))
    g64 = gains.astype(np.complex64)
    v = sg.volts(w, backend="torch", device="cuda")
    out = bf.beamform_fft(plan, v, gains=torch.from_numpy(g64).cuda())
    torch.cuda.synchronize()
    sel = w.ns_select()
    g = g64.astype(np.complex128)
    worst = c2_wide_worst(w, v, out, lambda x, ch: orc.beamform_fft(x, w.m_ew, w.m_ns, 16, taper=g,
                                                                      ns_select=sel[ch]))
    print(f"4x256 FP32 with complex gains, full size: max rel beam-power error {worst:.3e}")
    assert worst < TOL_FP32
    plan.close()
    del v, out
    torch.cuda.empty_cache()
