"""The tied-beam server on the GPU: results against the FP64 oracle, alone vs in a mix,
memory-budget admission, ring leases, wrap-around and cancellation."""
import numpy as np
import pytest

import oracle as orc
import synthgen as sg
from tests.helpers import TOL_FP32, rel_err

pytestmark = pytest.mark.gpu

RING = 4096
N_CHAN = 32


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _setup(budget=64 << 20, n_pol=1):
    torch = _torch()
    import paper_1710_08591_amd as bf
    w = sg.custom_workload(n_ew=4, n_ns=16, n_chan=N_CHAN, n_pol=n_pol, n_time=4 * RING, seed=55, n_src=3,
                           snr=8.0, dl=(0.4, 0.8))
    plan = bf.Plan(n_ew=4, n_ns=16, n_chan=N_CHAN, n_pol=n_pol, block=16, d_over_lambda=w.d_over_lambda())
    srv = bf.Server(plan, ring_samples=RING, hbm_budget=budget, blocks_per_tile=4, max_tiles_per_launch=256)
    plan.close()
    return w, srv


def _write(srv, w, t0, n):
    torch = _torch()
    src = sg.volts(w, t0, n, backend="torch", device="cuda")
    return srv.advance(n, src)


def _oracle(w, rid_args, head):
    dircos, lo, nc, nt = rid_args
    v = sg.volts(w, head - nt, nt, chans=list(range(lo, lo + nc)))
    return orc.tied_intensity(v, dircos, w.d_over_lambda(), 16, chans=list(range(lo, lo + nc)))


def test_alone_equals_mixed_and_matches_oracle():
    import paper_1710_08591_amd as bf
    w, srv = _setup()
    assert _write(srv, w, 0, RING) == bf.BF_OK
    head = RING
    a_args = (sg.pointings(37, 1), 3, 5, 1024)
    ra = srv.submit(a_args[0], *a_args[1:])
    st, lat = srv.wait(ra)
    assert st == bf.BF_OK and lat > 0
    alone = srv.result(ra).cpu().numpy()
    assert alone.shape == (64, 5, 1, 37)
    assert rel_err(alone, _oracle(w, a_args, head)) < TOL_FP32
    assert srv.release(ra) == bf.BF_OK
    # the same request again, submitted among others of uneven shapes
    others = [(sg.pointings(200, 2), 0, 32, 2048), (sg.pointings(1, 3), 31, 1, 4096),
              (sg.pointings(64, 4), 10, 12, 512), (sg.pointings(65, 5), 2, 7, 3072)]
    ids = [srv.submit(o[0], *o[1:]) for o in others[:2]]
    rb = srv.submit(a_args[0], *a_args[1:])
    ids += [srv.submit(o[0], *o[1:]) for o in others[2:]]
    for i in ids + [rb]:
        st, _ = srv.wait(i)
        assert st == bf.BF_OK
    mixed = srv.result(rb).cpu().numpy()
    assert np.array_equal(alone, mixed)              # bitwise: tiles do not depend on the batch
    for i, o in zip(ids, others):
        assert rel_err(srv.result(i).cpu().numpy(), _oracle(w, o, head)) < TOL_FP32
        assert srv.release(i) == bf.BF_OK
    s = srv.stats()
    assert s["completed"] == 6 and s["rejected"] == 0 and s["launches"] >= 2
    srv.close()


def test_budget_lease_wrap_cancel():
    import paper_1710_08591_amd as bf
    w, srv = _setup(budget=1 << 20)
    assert _write(srv, w, 0, RING) == bf.BF_OK
    # over the 1 MiB budget: 256 pointings x 32 channels x 256 blocks x 4 B
    st, _ = srv.try_submit(sg.pointings(256, 6), 0, 32, 4096)
    assert st == bf.BF_ERR_REJECTED and srv.stats()["rejected"] == 1
    # a window longer than the ring, or not yet written
    st, _ = srv.try_submit(sg.pointings(2, 6), 0, 1, 2 * RING)
    assert st == bf.BF_ERR_EVICTED
    # lease: a live request's window may not be overwritten
    args = (sg.pointings(8, 7), 4, 2, 2048)
    r1 = srv.submit(args[0], *args[1:])
    assert _write(srv, w, RING, 2048) == bf.BF_OK          # overwrites [0, 2048): not leased
    head = RING + 2048
    assert _write(srv, w, head, 16) == bf.BF_ERR_NOT_READY  # would hit the lease on [2048, 4096)
    st, _ = srv.wait(r1)
    assert st == bf.BF_OK
    assert rel_err(srv.result(r1).cpu().numpy(), _oracle(w, args, RING)) < TOL_FP32
    assert srv.release(r1) == bf.BF_OK
    # the writer moves on; a window that straddles the ring's wrap
    assert _write(srv, w, head, 1024) == bf.BF_OK
    head += 1024                                            # 7168: slots wrap at 4096
    args2 = (sg.pointings(70, 8), 20, 3, 4096)
    r2 = srv.submit(args2[0], *args2[1:])
    st, _ = srv.wait(r2)
    assert st == bf.BF_OK
    assert rel_err(srv.result(r2).cpu().numpy(), _oracle(w, args2, head)) < TOL_FP32
    assert srv.release(r2) == bf.BF_OK
    # forced overwrite evicts a live request; cancel stops one
    r3 = srv.submit(sg.pointings(3, 9), 0, 32, 4096)
    r4 = srv.submit(sg.pointings(3, 9), 0, 32, 512)
    srv.cancel(r4)
    assert srv.advance(32, None, force=True) == bf.BF_OK
    assert srv.poll(r3)[0] == bf.BF_ERR_EVICTED
    for r in (r3, r4):
        for _ in range(100000):
            srv.pump()
            if srv.release(r) == bf.BF_OK:
                break
    assert srv.stats()["budget_used"] == 0
    srv.close()


def test_two_pols():
    import paper_1710_08591_amd as bf
    w, srv = _setup(n_pol=2)
    assert _write(srv, w, 0, RING) == bf.BF_OK
    args = (sg.pointings(5, 11), 6, 4, 256)
    r = srv.submit(args[0], *args[1:])
    assert srv.wait(r)[0] == bf.BF_OK
    got = srv.result(r).cpu().numpy()
    v = sg.volts(w, RING - 256, 256, chans=list(range(6, 10)))
    ref = orc.tied_intensity(v, args[0], w.d_over_lambda(), 16, chans=list(range(6, 10)))
    assert got.shape == ref.shape == (16, 4, 2, 5)
    assert rel_err(got, ref) < TOL_FP32
    srv.close()
