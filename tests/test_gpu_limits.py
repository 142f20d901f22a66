"""Calls at the documented maximum sizes, against the FP64 oracle on sampled
outputs, and one past each limit (rejected before any launch)."""
import numpy as np
import pytest

import oracle as orc
import synthgen as sg
from tests.helpers import TOL_FP32, plan_for, rel_err

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def test_tied_beams_4096_pointings():
    torch = _torch()
    import paper_1710_08591_amd as bf
    w = sg.custom_workload(n_ew=4, n_ns=16, n_chan=2, n_pol=1, n_time=32, seed=61, n_src=2, snr=8.0,
                           dl=(0.4, 0.8))
    v = sg.volts(w)
    plan = plan_for(w, clamp=False)
    vt = torch.from_numpy(v).cuda()
    dirs = sg.pointings(4096, 62)
    d = torch.from_numpy(dirs).cuda()
    got_v = bf.form_tied_beams_v(plan, vt, 0, 2, d).cpu().numpy()
    beams = bf.beamform_fft(plan, vt, kind=bf.BF_OUT_COMPLEX)
    got_b = bf.form_tied_beams(plan, beams, 0, 2, d).cpu().numpy()
    assert got_v.shape == got_b.shape == (2, 2, 1, 4096)
    pick = np.random.default_rng(3).choice(4096, 64, replace=False)
    ref = orc.tied_intensity(v, dirs[pick], w.d_over_lambda(), 16)
    assert rel_err(got_v[..., pick], ref) < TOL_FP32
    assert rel_err(got_b[..., pick], ref) < TOL_FP32
    with pytest.raises(bf.BFError) as e:
        bf.form_tied_beams_v(plan, vt, 0, 2, torch.from_numpy(sg.pointings(4097, 1)).cuda())
    assert e.value.status == bf.BF_ERR_UNSUPPORTED
    plan.close()


def test_regrid_65536_targets():
    torch = _torch()
    import paper_1710_08591_amd as bf
    w = sg.custom_workload(n_ew=4, n_ns=16, n_chan=1, n_pol=1, n_time=32, seed=63, n_src=2, snr=2.0)
    x = orc.beamform_fft(sg.volts(w), 4, 32, 16).astype(np.float32)
    plan = bf.Plan(n_ew=4, n_ns=16, block=16, d_over_lambda=w.d_over_lambda())
    st = np.linspace(-1.0, 1.0, 65536)
    rg = bf.Regrid(plan, st)
    got = rg(torch.from_numpy(x).cuda()).cpu().numpy()
    assert got.shape == (2, 1, 1, 4, 65536)
    pick = np.random.default_rng(4).choice(65536, 300, replace=False)
    W = np.stack([orc.regrid_weights_paper(16, 32, w.d_over_lambda()[0, 1] * s) for s in st[pick]])
    ref = orc.regrid_intensity(x.astype(np.float64), W)
    assert rel_err(got[..., pick], ref) < TOL_FP32
    with pytest.raises(bf.BFError) as e:
        bf.Regrid(plan, np.zeros(65537))
    assert e.value.status == bf.BF_ERR_INVALID_ARGUMENT
    rg.close()
    plan.close()


def test_localize_largest_window_and_iterations():
    torch = _torch()
    import paper_1710_08591_amd as bf
    w = sg.custom_workload(n_ew=4, n_ns=64, n_chan=2, n_pol=2, n_time=48, seed=65, n_src=2, snr=30.0)
    x = orc.beamform_fft(sg.volts(w), 4, 128, 16).astype(np.float32)
    plan = bf.Plan(n_ew=4, n_ns=64, n_chan=2, n_pol=2, block=16, d_over_lambda=w.d_over_lambda())
    st, pk = bf.localize(plan, torch.from_numpy(x).cuda(), n_window=64, n_iter=64)
    ref_st, ref_pk = orc.localize(x.astype(np.float64), 64, w.d_over_lambda()[:, 1], 64, 64)
    assert np.max(np.abs(st.cpu().numpy() - ref_st)) < 1e-9
    assert np.max(np.abs(pk.cpu().numpy() - ref_pk) / ref_pk) < 1e-6
    plan.close()
