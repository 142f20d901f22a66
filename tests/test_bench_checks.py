"""The benchmark's sampled-parity machinery on the CPU: the measurement legs
record output slices, and the oracle leg fills in the errors.  Here the
'measured' slices are oracle values with a known perturbation, so the
reported errors must equal that perturbation."""
import numpy as np

import bench
import oracle as orc
import synthgen as sg


def test_oracle_leg_fills_in_sampled_errors():
    w = sg.make_workload("c2")
    dl, sel = w.d_over_lambda(), w.ns_select()
    checks = bench.OracleChecks()
    blk, c, p = 3, 17, 1
    vs = sg.volts(w, blk * 16, 16, chans=[c], pols=[p])
    ref = orc.beamform_fft(vs, 4, 512, 16)[0, 0, 0][:, sel[c]]
    r_fft = {}
    checks.add(r_fft, "err", "fft_rel", ref * (1 + 3e-7), v=vs, m_ew=4, m_ns=512, index=(0, 0, 0), sel=sel[c])
    vs2 = sg.volts(w, blk * 16, 16, chans=[c])
    st = np.linspace(-0.9, 0.9, 6)
    dircos = np.stack([np.repeat(np.arange(4), 6) / (4 * dl[c, 0]), np.tile(st, 4)], axis=1)
    t_ref = orc.tied_intensity(vs2, dircos, dl, 16, chans=[c])[0, 0].reshape(2, 4, 6)
    r_tied = {}
    checks.add(r_tied, "err", "tied_rel", t_ref, v=vs2, dircos=dircos, dl=dl, c=c, shape=(2, 4, 6))
    b = orc.beamform_fft(vs2, 4, 512, 16)[0, 0]
    W = np.stack([orc.regrid_weights_paper(256, 512, dl[c, 1] * s) for s in st])
    r_rg = {}
    checks.add(r_rg, "err", "regrid_prop", orc.regrid_intensity(b, W), v=vs2, m_ew=4, m_ns=512,
               weights="paper", n_ns=256, ys=dl[c, 1] * st)
    x = orc.beamform_fft(vs2, 4, 512, 16)
    lst, _ = orc.localize(x, 256, dl[:, 1], 10, 6, chans=[c])
    r_loc = {}
    checks.add(r_loc, "err", "localize_abs", lst + 2e-9, v=vs2, m_ew=4, m_ns=512, n_ns=256, dl_ns=dl[:, 1],
               c=c, n_window=10, n_iter=6)
    rec = bench.cpu_baseline(0.05, checks)
    assert rec["kind"] == "oracle" and rec["value"] > 0
    assert rec["parity_slices_checked"] == 4
    assert abs(r_fft["err"] - 3e-7) < 1e-12
    assert r_tied["err"] == 0.0 and r_rg["err"] == 0.0
    assert abs(r_loc["err"] - 2e-9) < 1e-15


def test_failing_side_measurement_is_reported_not_raised():
    def boom():
        raise RuntimeError("no device")
    assert bench._leg(boom) == {"error": "RuntimeError: no device"}


def test_whole_block_checks_use_each_channels_clamp_table():
    """add_blocks compares every channel and polarisation of whole blocks,
    each channel with its own kept beams; a perturbation of one channel's
    slice is what the oracle leg reports, and the CPU statement is filled in."""
    import torch
    w = sg.custom_workload(n_ew=4, n_ns=8, n_chan=3, n_pol=2, n_time=32, seed=9, n_ns_keep=8, dl=(0.4, 0.8))
    v = sg.volts(w)
    sel = w.ns_select()
    assert not all(np.array_equal(sel[0], sel[c]) for c in range(3))
    ref = orc.beamform_fft(v, 4, 16, 16, ns_select=sel)                       # [2][3][2][4][8]
    got = ref.copy()
    got[1, 2, 1] *= 1 + 5e-7
    checks = bench.OracleChecks()
    rec = {}
    checks.add_blocks(rec, "err", torch.from_numpy(got), w)
    out = bench.cpu_baseline(0.05, checks, seconds_1t=0.05)
    assert out["parity_slices_checked"] == 2 * 3 * 2
    assert abs(rec["err"] - 5e-7) < 1e-12
    assert out["value_1_thread"] is None or out["value_1_thread"] > 0
    for k in ("cpu_model", "nproc", "cpus_allowed", "thread_env", "blas_pools"):
        assert k in out
