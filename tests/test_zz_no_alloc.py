"""bf_form_tied_beams_v_noalloc (the library's static device scratch as the
workspace, no allocation in the call) against bf_form_tied_beams_v_ws (a
caller workspace): the same kernels, so the same beams, on two calls in a row,
the second smaller; and against the oracle's direct phased sums."""
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


def test_noalloc_matches_workspace_entry_point():
    torch = _torch()
    import paper_1710_08591_amd as bf
    # 4 x 256 lattice, 8 channels, 2 pols: 4 MiB of FFT beams per block, so
    # the 64 MiB static scratch takes 16 blocks per chunk and 512 samples (32
    # blocks) go in two chunks
    w = sg.custom_workload(n_ew=4, n_ns=256, n_chan=8, n_pol=2, n_time=512, seed=101, n_src=2, snr=15.0,
                           dl=(0.4, 0.8))
    v = sg.volts(w)
    vt = torch.from_numpy(v).cuda()
    dl = w.d_over_lambda()
    dirs = np.concatenate([sg.pointings(20, 102), [[0.0, 0.0]]], axis=0)
    d = torch.from_numpy(dirs).cuda()
    plan = plan_for(w, clamp=False)
    assert bf.tied_workspace_size(plan, 8, 16) == 4 << 20
    # first call: every channel and sample
    out1 = torch.full((32, 8, 2, 21), -1.0, dtype=torch.float32, device="cuda")
    bf.form_tied_beams_v_noalloc(plan, vt, 0, 8, d, out1)
    ref1 = bf.form_tied_beams_v(plan, vt, 0, 8, d)
    torch.cuda.synchronize()
    assert torch.equal(out1, ref1)
    c = 5
    r = orc.tied_intensity(v[-16:, c:c + 1], dirs, dl, 16, chans=[c])
    assert rel_err(out1[-1:, c:c + 1].cpu().numpy(), r) < TOL_FP32
    # second call, smaller: channels 1..3, the first 256 samples, with a window
    h = torch.from_numpy(sg.gaussian_taper(4, 256)).cuda()
    v2 = vt[:256].contiguous()
    out2 = torch.full((16, 3, 2, 21), -1.0, dtype=torch.float32, device="cuda")
    bf.form_tied_beams_v_noalloc(plan, v2, 1, 3, d, out2, taper=h)
    ref2 = bf.form_tied_beams_v(plan, v2, 1, 3, d, taper=h)
    torch.cuda.synchronize()
    assert torch.equal(out2, ref2)
    r2 = orc.tied_intensity(v[:16, 2:3], dirs, dl, 16, taper=sg.gaussian_taper(4, 256), chans=[2])
    assert rel_err(out2[:1, 1:2].cpu().numpy(), r2) < TOL_FP32
    plan.close()


def test_noalloc_limit_and_fused_lattice():
    """A channel range whose one block of beams exceeds the static scratch is
    refused before any launch; on the 4 x 16 lattice the call is the fused
    kernel (no workspace) and equals bf_form_tied_beams_v."""
    torch = _torch()
    import paper_1710_08591_amd as bf
    plan = bf.Plan(n_ew=4, n_ns=256, n_chan=130, n_pol=2, block=16)
    assert bf.tied_workspace_size(plan, 130, 16) > 64 << 20
    vt = torch.zeros((16, 130, 2, 256, 4), dtype=torch.uint8, device="cuda")
    d = torch.zeros((3, 2), dtype=torch.float64, device="cuda")
    out = torch.empty((1, 130, 2, 3), dtype=torch.float32, device="cuda")
    with pytest.raises(bf.BFError) as e:
        bf.form_tied_beams_v_noalloc(plan, vt, 0, 130, d, out)
    assert e.value.status == bf.BF_ERR_INVALID_ARGUMENT
    plan.close()
    w = sg.custom_workload(n_ew=4, n_ns=16, n_chan=3, n_pol=1, n_time=64, seed=9, dl=(0.4, 0.8))
    v = torch.from_numpy(sg.volts(w)).cuda()
    plan = plan_for(w, clamp=False)
    d = torch.from_numpy(sg.pointings(10, 3)).cuda()
    out = torch.empty((4, 3, 1, 10), dtype=torch.float32, device="cuda")
    bf.form_tied_beams_v_noalloc(plan, v, 0, 3, d, out)
    assert torch.equal(out, bf.form_tied_beams_v(plan, v, 0, 3, d))
    plan.close()
