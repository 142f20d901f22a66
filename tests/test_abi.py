"""The C-ABI library loads, exports every declared symbol, and validates on the host.

These run without a GPU: no call here reaches a kernel or the HIP runtime.
"""
import ctypes as C

import pytest

from paper_1710_08591_amd import _lib as L


def test_exports_every_declared_symbol():
    lib = L.lib()
    names = L.declared_symbols()
    assert "bf_beamform_fft" in names and "bf_form_tied_beams" in names
    assert "bf_accumulate_intensity" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings():
    lib = L.lib()
    assert lib.bf_status_string(L.BF_OK) == b"ok"
    assert b"invalid" in lib.bf_status_string(L.BF_ERR_INVALID_ARGUMENT)
    assert lib.bf_version().startswith(b"fftbf")


def _desc(**kw):
    d = L.bf_plan_desc()
    vals = dict(n_ew=4, n_ns=16, m_ew=4, m_ns=32, n_pol=1, n_chan=1, block=16, n_ns_keep=0,
                pol_sum=0, precision=0)
    vals.update(kw)
    for k, v in vals.items():
        setattr(d, k, v)
    return d


@pytest.mark.parametrize("kw,status", [
    (dict(n_ns=0), L.BF_ERR_INVALID_ARGUMENT),
    (dict(block=0), L.BF_ERR_INVALID_ARGUMENT),
    (dict(m_ns=8), L.BF_ERR_UNSUPPORTED),                 # cyclic co-adding below 16 beams
    (dict(m_ew=2), L.BF_ERR_INVALID_ARGUMENT),            # E-W transform shorter than the array
    (dict(n_ns=64, m_ns=48), L.BF_ERR_UNSUPPORTED),
    (dict(n_ns=64, m_ns=32, precision=1), L.BF_ERR_UNSUPPORTED),
    (dict(n_ns=64, m_ns=32, m_ew=8), L.BF_ERR_UNSUPPORTED),
    (dict(n_ns=64, m_ns=32, n_ns_keep=16), L.BF_ERR_UNSUPPORTED),
    (dict(m_ew=8, precision=1), L.BF_ERR_UNSUPPORTED),
    (dict(n_ew=2, m_ew=2), L.BF_ERR_UNSUPPORTED),
    (dict(n_ns=24, m_ns=48), L.BF_ERR_UNSUPPORTED),
    (dict(n_ns=512, m_ns=1024), L.BF_ERR_UNSUPPORTED),
    (dict(m_ns=33), L.BF_ERR_UNSUPPORTED),
    (dict(n_pol=3), L.BF_ERR_UNSUPPORTED),
    (dict(precision=7), L.BF_ERR_INVALID_ARGUMENT),
    (dict(n_ns_keep=8), L.BF_ERR_INVALID_ARGUMENT),   # a clamp without a table
    (dict(block=6), L.BF_ERR_UNSUPPORTED),
])
def test_plan_create_rejects_before_touching_the_device(kw, status):
    lib = L.lib()
    h = C.c_void_p(123)
    st = lib.bf_plan_create(C.byref(_desc(**kw)), C.byref(h))
    assert st == status, lib.bf_last_error()
    assert h.value is None
    assert len(lib.bf_last_error()) > 0


def test_plan_create_rejects_out_of_range_clamp_table():
    lib = L.lib()
    sel = (C.c_int32 * 4)(0, 5, 32, 1)
    d = _desc(n_ns_keep=4)
    d.ns_select = C.cast(sel, C.POINTER(C.c_int32))
    h = C.c_void_p()
    assert lib.bf_plan_create(C.byref(d), C.byref(h)) == L.BF_ERR_INVALID_ARGUMENT
    assert b"ns_select" in lib.bf_last_error()


def test_null_arguments():
    lib = L.lib()
    assert lib.bf_plan_create(None, None) == L.BF_ERR_INVALID_ARGUMENT
    assert lib.bf_beamform_fft(None, None, 16, None, 0, None, None) == L.BF_ERR_INVALID_ARGUMENT
    assert lib.bf_plan_destroy(None) == L.BF_OK
    assert lib.bf_form_tied_beams(None, None, 16, 0, 1, None, 1, 0, None, None) == L.BF_ERR_INVALID_ARGUMENT
    assert lib.bf_form_tied_beams_v(None, None, 16, None, 0, 1, None, 1, None, None) == L.BF_ERR_INVALID_ARGUMENT
    assert lib.bf_form_tied_beams_v_ws(None, None, 16, None, 0, 1, None, 1, None, 0, None, None) \
        == L.BF_ERR_INVALID_ARGUMENT
    assert lib.bf_form_tied_beams_v_noalloc(None, None, 16, None, 0, 1, None, 1, None, None) \
        == L.BF_ERR_INVALID_ARGUMENT
    assert b"NULL plan" in lib.bf_last_error()
    assert lib.bf_tied_workspace_size(None, 4, 16) == 0


@pytest.mark.parametrize("args,status", [
    ((None, 15, 1, 16, 0, None, None), L.BF_ERR_INVALID_ARGUMENT),    # ragged n_time
    ((None, 32, 1, 0, 0, None, None), L.BF_ERR_INVALID_ARGUMENT),     # block 0
    ((None, 32, 1, 16, 2, None, None), L.BF_ERR_INVALID_ARGUMENT),    # add not 0/1
    ((None, -16, 1, 16, 0, None, None), L.BF_ERR_INVALID_ARGUMENT),
    ((None, 32, 4, 16, 0, None, None), L.BF_ERR_INVALID_ARGUMENT),    # NULL buffers
    ((None, 0, 4, 16, 0, None, None), L.BF_OK),                       # empty: nothing to do
    ((C.c_void_p(12), 32, 4, 16, 0, C.c_void_p(16), None), L.BF_ERR_INVALID_ARGUMENT),  # misaligned z
])
def test_accumulate_validation(args, status):
    lib = L.lib()
    assert lib.bf_accumulate_intensity(*args) == status


def test_native_driver_rejects_bad_arguments():
    """The C-ABI driver is built beside the library and validates its
    arguments before touching the device."""
    import os
    import subprocess
    exe = os.path.join(os.path.dirname(L.__file__), "fftbf_bench")
    assert os.path.exists(exe)
    r = subprocess.run([exe, "--n-ns", "-4"], capture_output=True, text=True, timeout=60)
    assert r.returncode == 2 and "invalid arguments" in r.stderr
    r = subprocess.run([exe, "--keep", "9999"], capture_output=True, text=True, timeout=60)
    assert r.returncode == 2
    r = subprocess.run([exe, "--random", "2"], capture_output=True, text=True, timeout=60)
    assert r.returncode == 2 and "invalid arguments" in r.stderr
    r = subprocess.run([exe, "--tied", "5000"], capture_output=True, text=True, timeout=60)
    assert r.returncode == 2 and "invalid arguments" in r.stderr
    r = subprocess.run([exe, "--copy", "2"], capture_output=True, text=True, timeout=60)
    assert r.returncode == 2 and "invalid arguments" in r.stderr
    r = subprocess.run([exe, "--issue", "3"], capture_output=True, text=True, timeout=60)
    assert r.returncode == 2 and "invalid arguments" in r.stderr
