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
