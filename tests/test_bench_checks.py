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
