"""Mixed-precision (FP16 / FP8 MFMA) beamformer against the FP64 oracle.

The target is <= 1e-3 relative beam power per variant (the int4 inputs are
exact in both formats; the DFT coefficients are split into two FP16 or three
scaled FP8 terms, accumulation in FP32).
"""
import numpy as np
import pytest

import oracle as orc
import synthgen as sg
from tests.helpers import plan_for, rel_err

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
        bf.Plan(n_ns=32, precision=1)
    assert e.value.status == bf.BF_ERR_UNSUPPORTED


def test_mix256_chime_lattice_parity():
    """The two-stage FP16 MFMA transform on the 4 x 256 lattice (512 = 32 x 16)."""
    w = sg.custom_workload(n_ew=4, n_ns=256, n_chan=3, n_pol=2, n_time=48, seed=77, n_src=4, snr=10.0,
                           n_ns_keep=256, dl=(0.4, 0.8))
    v = sg.volts(w)
    ref = orc.beamform_fft(v, 4, 512, 16, ns_select=w.ns_select())
    got = _run(w, v, 1)
    err = rel_err(got, ref)
    print(f"4x256 FP16 MFMA: max rel beam-power error {err:.3e}")
    assert err < TOL_MIXED
    refp = orc.beamform_fft(v, 4, 512, 16, ns_select=w.ns_select(), pol_sum=True)
    assert rel_err(_run(w, v, 1, pol_sum=True), refp) < TOL_MIXED
    unc = _run(w, v, 1, clamp=False, block=48)
    assert rel_err(unc, orc.beamform_fft(v, 4, 512, 48)) < TOL_MIXED


def test_mix256_extremes_and_point_source():
    w = sg.custom_workload(n_ew=4, n_ns=256, n_time=16, n_src=0)
    for b in (0x88, 0x77, 0x18):
        v = np.full((16, 1, 1, 256, 4), b, dtype=np.uint8)
        got = _run(w, v, 1, clamp=False)
        ref = orc.beamform_fft(v, 4, 512, 16)
        assert np.max(np.abs(got - ref)) / ref.max() < TOL_MIXED
    v = sg.point_source_volts(4, 256, 1, 3, 16, 7)
    got = _run(w, v, 1, clamp=False)
    ref = orc.beamform_fft(v, 4, 512, 16)
    assert np.max(np.abs(got - ref)) / ref.max() < TOL_MIXED
