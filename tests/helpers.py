"""Shared test helpers: plans from workloads, tolerances, comparisons."""
import numpy as np

# FP32 path: beam powers within 1e-5 relative of the FP64 oracle (per beam
# for noise-dominated data; against the peak for noise-free sources).
TOL_FP32 = 1e-5


def rel_err(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.max(np.abs(got - ref) / ref))


def peak_err(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))


def plan_for(w, precision=0, pol_sum=False, clamp=True, block=None):
    import paper_1710_08591_amd as bf
    sel = w.ns_select() if clamp else None
    return bf.Plan(n_ew=w.n_ew, n_ns=w.n_ns, m_ew=w.m_ew, m_ns=w.m_ns, n_pol=w.n_pol, n_chan=w.n_chan,
                   block=block or w.block, ns_select=sel, pol_sum=pol_sum, precision=precision,
                   d_over_lambda=w.d_over_lambda())


# ---- full-size comparison set of the CHIME-shaped workload ----------------
# Every channel and both polarisations of the first and the last block (all
# 256 per-channel clamp tables), and one channel, both polarisations, over
# every block of the 16384 samples.
C2_WIDE_CHAN = 137


def c2_wide_regions(w, v_gpu, chan=C2_WIDE_CHAN):
    """[(output index, voltages [t][chan][pol][n_ns][n_ew], channel numbers)].

    The voltages of the two whole blocks are generated on the host by the
    seeded generator and checked byte for byte against the device copy; the
    single channel's 16384 samples are copied from the device (the same
    generator's device backend), with their first and last blocks checked
    against the host generator."""
    import synthgen as sg
    b = w.block
    last = w.n_time // b - 1
    regions = []
    for blk in (0, last):
        vs = sg.volts(w, blk * b, b)
        assert np.array_equal(vs, v_gpu[blk * b:(blk + 1) * b].cpu().numpy())
        regions.append(((slice(blk, blk + 1),), vs, np.arange(w.n_chan)))
    vc = v_gpu[:, chan:chan + 1].cpu().numpy()
    assert np.array_equal(vc[:b], sg.volts(w, 0, b, chans=[chan]))
    assert np.array_equal(vc[-b:], sg.volts(w, w.n_time - b, b, chans=[chan]))
    regions.append(((slice(None), slice(chan, chan + 1)), vc, np.array([chan])))
    return regions


def by_time_chunks(fn, v, chunk=4096):
    """fn over consecutive time chunks of v (a multiple of the block), joined
    along the block axis: blocks are independent, so this is fn(v) with
    bounded host memory."""
    return np.concatenate([fn(v[i:i + chunk]) for i in range(0, v.shape[0], chunk)], axis=0)


def c2_wide_worst(w, v_gpu, out, ref_fn, err=None):
    """Largest error of out against ref_fn(voltages, channels) over the
    full-size comparison set (rel_err by default)."""
    err = err or rel_err
    worst = 0.0
    for idx, vs, chans in c2_wide_regions(w, v_gpu):
        ref = by_time_chunks(lambda x: ref_fn(x, chans), vs)
        worst = max(worst, err(out[idx].cpu().numpy(), ref))
    return worst
