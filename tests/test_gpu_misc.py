"""GPU parity of the intensity accumulator and the tied-array beams."""
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


@pytest.mark.parametrize("n_time,n_series,block", [(64, 7, 16), (48, 1000, 3), (16, 64, 16), (5, 3, 1),
                                                   (44, 33, 11), (40, 5, 10)])
def test_accumulate_intensity(n_time, n_series, block):
    torch = _torch()
    import paper_1710_08591_amd as bf
    z = sg.random_complex_series(n_time, n_series, seed=n_series)
    zt = torch.from_numpy(z).cuda()
    out = bf.accumulate_intensity(zt, block)
    ref = orc.accumulate_intensity(z.astype(np.complex128), block)
    assert rel_err(out.cpu().numpy(), ref) < TOL_FP32
    out2 = bf.accumulate_intensity(zt, block, out=out.clone(), add=True)
    assert rel_err(out2.cpu().numpy(), 2 * ref) < TOL_FP32


def _tied_case(w, n_point, seed, taper):
    torch = _torch()
    import paper_1710_08591_amd as bf
    v = sg.volts(w)
    h = sg.gaussian_taper(w.n_ew, w.n_ns) if taper else None
    dirs = sg.pointings(n_point, seed)
    plan = plan_for(w, clamp=False)
    vt = torch.from_numpy(v).cuda()
    ht = None if h is None else torch.from_numpy(h).cuda()
    beams = bf.beamform_fft(plan, vt, taper=ht, kind=bf.BF_OUT_COMPLEX)
    d = torch.from_numpy(dirs).cuda()
    return plan, v, vt, h, ht, dirs, d, beams


@pytest.mark.parametrize("taper", [False, True])
def test_c3_tied_beams_from_fft_beams(taper):
    """64 arbitrary pointings on the 4 x 16 lattice vs the direct phased sum."""
    torch = _torch()
    import paper_1710_08591_amd as bf
    w = sg.make_workload("c3")
    plan, v, vt, h, ht, dirs, d, beams = _tied_case(w, 64, 3, taper)
    got = bf.form_tied_beams(plan, beams, 0, 1, d).cpu().numpy()
    ref = orc.tied_intensity(v, dirs, w.d_over_lambda(), w.block, taper=h)
    assert got.shape == ref.shape == (64, 1, 1, 64)
    assert rel_err(got, ref) < TOL_FP32
    gotc = bf.form_tied_beams(plan, beams, 0, 1, d, kind=bf.BF_OUT_COMPLEX).cpu().numpy()
    refc = orc.tied_beams(v, dirs, w.d_over_lambda(), taper=h)
    assert np.max(np.abs(gotc - refc)) / np.max(np.abs(refc)) < 1e-5
    plan.close()


@pytest.mark.parametrize("taper", [False, True])
def test_c3_tied_beams_from_voltages(taper):
    torch = _torch()
    import paper_1710_08591_amd as bf
    w = sg.make_workload("c3")
    plan, v, vt, h, ht, dirs, d, beams = _tied_case(w, 64, 3, taper)
    got = bf.form_tied_beams_v(plan, vt, 0, 1, d, taper=ht).cpu().numpy()
    ref = orc.tied_intensity(v, dirs, w.d_over_lambda(), w.block, taper=h)
    assert rel_err(got, ref) < TOL_FP32
    plan.close()


@pytest.mark.parametrize("scale", [3.5, 1e-3, 40.0])
def test_tied_from_voltages_window_scaling(scale):
    """The matrix-core interpolation scales the FFT beams by a power of two
    chosen from the window's largest weight (so its FP16 high and low terms
    neither overflow nor fall below the normal range): windows far above and
    below 1, extreme voltages, both polarisations summed."""
    torch = _torch()
    import paper_1710_08591_amd as bf
    w = sg.custom_workload(n_ew=4, n_ns=16, n_chan=3, n_pol=2, n_time=160, seed=23, n_src=2, snr=30.0,
                           dl=(0.4, 0.8))
    v = sg.volts(w)
    rng = np.random.default_rng(1)
    v[:16] = rng.choice(np.array([0x88, 0x77, 0x78, 0x87], dtype=np.uint8), size=v[:16].shape)   # |re|, |im| >= 7
    h = (sg.gaussian_taper(4, 16) * scale).astype(np.float32)
    plan = plan_for(w, clamp=False, pol_sum=True)
    dirs = np.concatenate([sg.pointings(40, 3), [[0.0, 0.0]]], axis=0)
    got = bf.form_tied_beams_v(plan, torch.from_numpy(v).cuda(), 0, 3, torch.from_numpy(dirs).cuda(),
                               taper=torch.from_numpy(h).cuda()).cpu().numpy()
    ref = orc.tied_intensity(v, dirs, w.d_over_lambda(), 16, taper=h).sum(axis=2)
    assert got.shape == ref.shape
    assert rel_err(got, ref) < TOL_FP32
    plan.close()


@pytest.mark.parametrize("scale", [1e4, 1e-4])
def test_tied_from_fft_beams_scaling_and_fallback(scale):
    """Tied beams from stored complex FFT beams on the matrix cores scale each
    sample by its own power of two (stored beams have no fixed bound): beams
    formed with a window far above or below 1 must still match the oracle;
    an unaligned view of the beams takes the FP32 vector kernel and must give
    the same beams to the FP32 bar."""
    torch = _torch()
    import paper_1710_08591_amd as bf
    w = sg.custom_workload(n_ew=4, n_ns=16, n_chan=3, n_pol=2, n_time=96, seed=41, n_src=2, snr=20.0,
                           dl=(0.4, 0.8))
    v = sg.volts(w)
    h = (sg.gaussian_taper(4, 16) * scale).astype(np.float32)
    plan = plan_for(w, clamp=False)
    beams = bf.beamform_fft(plan, torch.from_numpy(v).cuda(), taper=torch.from_numpy(h).cuda(),
                            kind=bf.BF_OUT_COMPLEX)
    dirs = np.concatenate([sg.pointings(70, 9), [[0.0, 0.0]]], axis=0)
    d = torch.from_numpy(dirs).cuda()
    got = bf.form_tied_beams(plan, beams, 0, 3, d).cpu().numpy()
    ref = orc.tied_intensity(v, dirs, w.d_over_lambda(), 16, taper=h)
    assert rel_err(got, ref) < TOL_FP32
    # an 8-byte-aligned (not 16) copy of the beams: the vector-ALU path
    buf = torch.empty(beams.numel() + 1, dtype=torch.complex64, device="cuda")
    shifted = buf[1:].view(beams.shape)
    shifted.copy_(beams)
    assert shifted.data_ptr() % 16 == 8
    got2 = bf.form_tied_beams(plan, shifted, 0, 3, d).cpu().numpy()
    assert rel_err(got2, ref) < TOL_FP32
    plan.close()


@pytest.mark.parametrize("n_time,block", [(368, 16), (352, 32)])
def test_tied_from_fft_beams_pol_sum_ragged_quads(n_time, block):
    """Tied beams from stored FFT beams on the matrix cores with both
    polarisations summed, and sample counts that leave the last quad of
    16-sample groups partly empty, over two workgroup spans (368) or with
    blocks of two groups (352): the next group's beams are loaded while the
    current quad is interpolated, stepping through (quad, polarisation)."""
    torch = _torch()
    import paper_1710_08591_amd as bf
    w = sg.custom_workload(n_ew=4, n_ns=16, n_chan=2, n_pol=2, n_time=n_time, seed=71, n_src=2, snr=20.0,
                           dl=(0.4, 0.8))
    v = sg.volts(w)
    plan = plan_for(w, clamp=False, pol_sum=True, block=block)
    beams = bf.beamform_fft(plan, torch.from_numpy(v).cuda(), kind=bf.BF_OUT_COMPLEX)
    assert beams.data_ptr() % 16 == 0          # the matrix-core kernel
    dirs = np.concatenate([sg.pointings(40, 72), [[0.0, 0.0]]], axis=0)
    got = bf.form_tied_beams(plan, beams, 0, 2, torch.from_numpy(dirs).cuda()).cpu().numpy()
    ref = orc.tied_intensity(v, dirs, w.d_over_lambda(), block).sum(axis=2)
    assert got.shape == ref.shape
    assert rel_err(got, ref) < TOL_FP32
    plan.close()


def test_tied_on_grid_and_odd_counts():
    """On-grid pointings reproduce the FFT beams; ragged pointing tiles; channel subsets."""
    torch = _torch()
    import paper_1710_08591_amd as bf
    w = sg.custom_workload(n_ew=4, n_ns=16, n_chan=5, n_pol=2, n_time=64, seed=17, dl=(0.4, 0.8))
    v = sg.volts(w)
    plan = plan_for(w, clamp=False)
    vt = torch.from_numpy(v).cuda()
    dl = w.d_over_lambda()
    A = [(1, 3), (0, 0), (3, 31), (2, 16)]
    c = 3
    dirs = np.array([[a / 4 / dl[c, 0], b / 32 / dl[c, 1]] for a, b in A])
    dirs = np.concatenate([dirs, sg.pointings(67, 5)], axis=0)         # 71 pointings: 2 tiles
    d = torch.from_numpy(dirs).cuda()
    beams = bf.beamform_fft(plan, vt, kind=bf.BF_OUT_COMPLEX)
    got = bf.form_tied_beams(plan, beams, 2, 3, d).cpu().numpy()       # channels 2..4
    ref = orc.tied_intensity(v[:, 2:5], dirs, dl, 16, chans=[2, 3, 4])
    assert rel_err(got, ref) < TOL_FP32
    fb = orc.beamform_fft(v, 4, 32, 16)
    for i, (a, b) in enumerate(A):
        assert rel_err(got[:, 1, :, i], fb[:, c, :, a, b]) < TOL_FP32
    gv = bf.form_tied_beams_v(plan, vt, 2, 3, d).cpu().numpy()
    assert rel_err(gv, ref) < TOL_FP32
    plan.close()


def test_tied_beams_benchmark_configuration_sampled():
    """Tied beams as the benchmark times them: the 4 x 16 lattice, 256
    channels, 16384 samples, 64 pointings, from voltages and from stored
    complex FFT beams; sampled (block, channel) outputs against the oracle's
    direct phased sums."""
    torch = _torch()
    import paper_1710_08591_amd as bf
    w = sg.make_workload("c5")
    vt = sg.volts(w, 0, 16384, backend="torch", device="cuda")
    plan = bf.Plan(n_ew=4, n_ns=16, n_chan=256, block=16, d_over_lambda=w.d_over_lambda())
    dirs = sg.pointings(64, 11)
    d = torch.from_numpy(dirs).cuda()
    got_v = bf.form_tied_beams_v(plan, vt, 0, 256, d)
    beams = bf.beamform_fft(plan, vt, kind=bf.BF_OUT_COMPLEX)
    got_b = bf.form_tied_beams(plan, beams, 0, 256, d)
    torch.cuda.synchronize()
    assert got_v.shape == got_b.shape == (1024, 256, 1, 64)
    rng = np.random.default_rng(4)
    dl = w.d_over_lambda()
    for blk, c in [(0, 0), (1023, 255)] + [(int(rng.integers(1024)), int(rng.integers(256))) for _ in range(3)]:
        vs = sg.volts(w, blk * 16, 16, chans=[c])
        ref = orc.tied_intensity(vs, dirs, dl, 16, chans=[c])[0, 0, 0]
        assert rel_err(got_v[blk, c, 0].cpu().numpy(), ref) < TOL_FP32
        assert rel_err(got_b[blk, c, 0].cpu().numpy(), ref) < TOL_FP32
    plan.close()
    del vt, beams, got_v, got_b
    torch.cuda.empty_cache()


@pytest.mark.parametrize("n_ns", [64, 128, 256])
def test_tied_from_fft_beams_large_lattices(n_ns):
    """Tied beams from stored complex FFT beams of the 4 x 64, 4 x 128 and
    4 x 256 lattices (m_ns = 128, 256, 512) on the FP32 matrix cores, against
    the oracle's direct phased sums (eq. e:c_pointed; exact for M >= n):
    ragged pointing tiles, on-grid pointings that must reproduce FFT beams,
    a channel subset, per-pol and summed intensities, blocks of 16 and 32,
    complex output with a sample count that is not a multiple of 4."""
    torch = _torch()
    import paper_1710_08591_amd as bf
    m = 2 * n_ns
    w = sg.custom_workload(n_ew=4, n_ns=n_ns, n_chan=4, n_pol=2, n_time=96, seed=80 + n_ns, n_src=3, snr=15.0,
                           dl=(0.4, 0.8))
    v = sg.volts(w)
    dl = w.d_over_lambda()
    c = 2
    grid = [(1, 3), (0, 0), (3, m - 1), (2, m // 2)]
    dirs = np.array([[a / 4 / dl[c, 0], b / m / dl[c, 1]] for a, b in grid])
    dirs = np.concatenate([dirs, sg.pointings(29, 81)], axis=0)           # 33 pointings: 3 tiles of 16
    d = torch.from_numpy(dirs).cuda()
    vt = torch.from_numpy(v).cuda()
    plan = plan_for(w, clamp=False)
    beams = bf.beamform_fft(plan, vt, kind=bf.BF_OUT_COMPLEX)
    assert beams.data_ptr() % 16 == 0
    got = bf.form_tied_beams(plan, beams, 1, 3, d).cpu().numpy()         # channels 1..3
    ref = orc.tied_intensity(v[:, 1:4], dirs, dl, 16, chans=[1, 2, 3])
    err = rel_err(got, ref)
    print(f"4x{n_ns} tied from stored beams: {err:.3e}")
    assert got.shape == ref.shape
    assert err < TOL_FP32
    fb = orc.beamform_fft(v, 4, m, 16)
    for i, (a, b) in enumerate(grid):
        assert rel_err(got[:, c - 1, :, i], fb[:, c, :, a, b]) < TOL_FP32
    gotc = bf.form_tied_beams(plan, beams[:93], 0, 4, d, kind=bf.BF_OUT_COMPLEX).cpu().numpy()
    refc = orc.tied_beams(v[:93], dirs, dl)
    assert np.max(np.abs(gotc - refc)) / np.max(np.abs(refc)) < 1e-5
    plan.close()
    for block in (16, 32):
        plan = plan_for(w, clamp=False, pol_sum=True, block=block)
        got = bf.form_tied_beams(plan, beams, 0, 4, d).cpu().numpy()
        ref = orc.tied_intensity(v, dirs, dl, block).sum(axis=2)
        assert got.shape == ref.shape
        assert rel_err(got, ref) < TOL_FP32
        plan.close()
    # the 16-byte alignment these lattices need
    buf = torch.empty(beams.numel() + 1, dtype=torch.complex64, device="cuda")
    shifted = buf[1:].view(beams.shape)
    plan = plan_for(w, clamp=False)
    with pytest.raises(bf.BFError) as e:
        bf.form_tied_beams(plan, shifted, 0, 1, d)
    assert e.value.status == bf.BF_ERR_INVALID_ARGUMENT
    plan.close()


@pytest.mark.parametrize("n_ns", [32, 64, 256])
def test_tied_from_voltages_other_lattices(n_ns):
    """Tied beams from voltages on the 4 x 32, 4 x 64 and 4 x 256 lattices:
    each chunk of whole blocks is beamformed (FP32, complex, with the window)
    into the caller's workspace and interpolated from there.  A workspace of
    one or two blocks forces several chunks; a channel subset, summed pols,
    blocks of 32 and the too-small-workspace error."""
    torch = _torch()
    import paper_1710_08591_amd as bf
    w = sg.custom_workload(n_ew=4, n_ns=n_ns, n_chan=4, n_pol=2, n_time=96, seed=90 + n_ns, n_src=3, snr=15.0,
                           dl=(0.4, 0.8))
    v = sg.volts(w)
    dl = w.d_over_lambda()
    vt = torch.from_numpy(v).cuda()
    dirs = np.concatenate([sg.pointings(20, 91), [[0.0, 0.0]]], axis=0)
    d = torch.from_numpy(dirs).cuda()
    h = sg.gaussian_taper(4, n_ns)
    ht = torch.from_numpy(h).cuda()
    plan = plan_for(w, clamp=False)
    ref = orc.tied_intensity(v[:, 1:4], dirs, dl, 16, chans=[1, 2, 3])
    got = bf.form_tied_beams_v(plan, vt, 1, 3, d).cpu().numpy()                 # one chunk
    assert got.shape == ref.shape
    err = rel_err(got, ref)
    print(f"4x{n_ns} tied from voltages: {err:.3e}")
    assert err < TOL_FP32
    one = bf.tied_workspace_size(plan, 3, 16)
    for blocks in (1, 2):
        ws = torch.empty(blocks * one + 8, dtype=torch.uint8, device="cuda")     # 6 or 3 chunks
        got = bf.form_tied_beams_v(plan, vt, 1, 3, d, workspace=ws).cpu().numpy()
        assert rel_err(got, ref) < TOL_FP32
    refh = orc.tied_intensity(v, dirs, dl, 16, taper=h)
    goth = bf.form_tied_beams_v(plan, vt, 0, 4, d, taper=ht).cpu().numpy()
    assert rel_err(goth, refh) < TOL_FP32
    with pytest.raises(bf.BFError) as e:
        bf.form_tied_beams_v(plan, vt, 1, 3, d, workspace=torch.empty(one - 16, dtype=torch.uint8, device="cuda"))
    assert e.value.status == bf.BF_ERR_INVALID_ARGUMENT
    plan.close()
    plan = plan_for(w, clamp=False, pol_sum=True, block=32)
    ws = torch.empty(bf.tied_workspace_size(plan, 4, 32), dtype=torch.uint8, device="cuda")
    got = bf.form_tied_beams_v(plan, vt, 0, 4, d, workspace=ws).cpu().numpy()
    ref = orc.tied_intensity(v, dirs, dl, 32).sum(axis=2)
    assert got.shape == ref.shape
    assert rel_err(got, ref) < TOL_FP32
    plan.close()


def test_tied_from_voltages_workspace_empty_and_errors():
    """Empty calls return without launching; shape and workspace errors are
    reported before any launch (4 x 64 lattice, workspace path)."""
    torch = _torch()
    import paper_1710_08591_amd as bf
    import paper_1710_08591_amd._lib as L
    w = sg.custom_workload(n_ew=4, n_ns=64, n_chan=2, n_pol=1, n_time=32, seed=3)
    plan = plan_for(w, clamp=False)
    vt = torch.from_numpy(sg.volts(w)).cuda()
    d = torch.zeros((2, 2), dtype=torch.float64, device="cuda")
    out = torch.full((2, 2, 1, 2), 7.0, dtype=torch.float32, device="cuda")
    ws = torch.empty(bf.tied_workspace_size(plan, 2, 32), dtype=torch.uint8, device="cuda")
    lib = L.lib()
    ptr = lambda t: bf._ptr(t)  # noqa: E731
    # n_time, n_point or n_chan_sub zero: OK, nothing written
    for nt, npnt, ncs in ((0, 2, 2), (32, 0, 2), (32, 2, 0)):
        st = lib.bf_form_tied_beams_v_ws(plan.handle, ptr(vt), nt, None, 0, ncs, ptr(d), npnt, ptr(ws),
                                         ws.numel(), ptr(out), None)
        assert st == bf.BF_OK
        st = lib.bf_form_tied_beams_v_noalloc(plan.handle, ptr(vt), nt, None, 0, ncs, ptr(d), npnt, ptr(out), None)
        assert st == bf.BF_OK
    torch.cuda.synchronize()
    assert bool((out == 7.0).all())
    # a sample count that is not a multiple of the block, a workspace below one block
    assert lib.bf_form_tied_beams_v_ws(plan.handle, ptr(vt), 24, None, 0, 2, ptr(d), 2, ptr(ws), ws.numel(),
                                       ptr(out), None) == bf.BF_ERR_INVALID_ARGUMENT
    assert lib.bf_form_tied_beams_v_ws(plan.handle, ptr(vt), 32, None, 0, 2, ptr(d), 2, ptr(ws),
                                       bf.tied_workspace_size(plan, 2, 16) - 8, ptr(out), None) \
        == bf.BF_ERR_INVALID_ARGUMENT
    # channel range outside the plan
    assert lib.bf_form_tied_beams_v_noalloc(plan.handle, ptr(vt), 32, None, 1, 2, ptr(d), 2, ptr(out), None) \
        == bf.BF_ERR_INVALID_ARGUMENT
    plan.close()
