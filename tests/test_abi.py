"""Host-side checks of the C ABI (no GPU needed): the built library exports
every entry point include/rdcnn.h declares, and argument validation returns the
documented status codes before any device work is issued."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in sorted(os.listdir(os.path.join(ROOT, "include")))
           if f.endswith(".h")]


def _declared():
    names = set()
    for h in HEADERS:
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"^[A-Za-z_][\w \t\*]*?\b(rdcnn_\w+)\s*\(", text, flags=re.M))
    return sorted(names)


def test_header_declares_entry_points():
    names = _declared()
    assert "rdcnn_create" in names and "rdcnn_step" in names and "rdcnn_read" in names


def test_library_exports_every_declared_symbol():
    from paper_2102_10340_amd import _lib
    missing = [n for n in _declared() if not hasattr(_lib.lib, n)]
    assert not missing, missing


@pytest.fixture(scope="module")
def L():
    from paper_2102_10340_amd import _lib
    return _lib


def _params(L, **kw):
    g = dict(dt=0.1, a=0.0, b=1.0, eps=-0.1, c=1.0, k3=1.0, Du=0.05, Dv=1.0)
    g.update(kw)
    return L.Params.from_mapping(g)


def test_create_rejects_bad_arguments(L):
    h = ctypes.c_void_p()
    p = _params(L)
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    cases = [
        dict(rows=0), dict(cols=-3), dict(bc=7), dict(x=None), dict(b0=None),
        dict(b1=fake.value + 0), dict(ka=float("nan")), dict(rows=1 << 15, cols=1 << 15),
    ]
    for c in cases:
        args = dict(rows=4, cols=4, bc=1, x=0x2000, ka=1.0, b0=0x3000, b1=0x4000)
        args.update(c)
        if "b1" in c:
            args["b0"] = args["b1"]  # aliasing buffers
        rc = L.lib.rdcnn_create(ctypes.byref(h), args["rows"], args["cols"], args["bc"],
                                ctypes.byref(p), args["x"], args["ka"], args["b0"], args["b1"], None)
        assert rc == L.EINVAL, (c, rc)
        assert L.last_error()
        assert not h.value
    assert L.lib.rdcnn_create(None, 4, 4, 1, ctypes.byref(p), 0x2000, 1.0, 0x3000, 0x4000, None) == L.EINVAL
    bad = _params(L, Du=float("inf"))
    assert L.lib.rdcnn_create(ctypes.byref(h), 4, 4, 1, ctypes.byref(bad), 0x2000, 1.0, 0x3000,
                              0x4000, None) == L.EINVAL
    assert L.lib.rdcnn_create(ctypes.byref(h), 4, 4, 1, None, 0x2000, 1.0, 0x3000, 0x4000,
                              None) == L.EINVAL


def test_model_create_rejects_bad_arguments(L):
    h = ctypes.c_void_p()
    gs = (ctypes.c_float * 5)(0.5, 0.037, 0.06, 0.2, 0.1)
    bad = (ctypes.c_float * 5)(0.5, float("nan"), 0.06, 0.2, 0.1)
    args = (0x2000, 0x3000, 0x4000, 0x5000, None)
    assert L.lib.rdcnn_model_create(ctypes.byref(h), 7, 8, 8, 0, gs, 5, *args) == L.EINVAL
    assert L.lib.rdcnn_model_create(ctypes.byref(h), 1, 8, 8, 0, gs, 4, *args) == L.EINVAL
    assert L.lib.rdcnn_model_create(ctypes.byref(h), 2, 8, 8, 0, gs, 5, *args) == L.EINVAL
    assert L.lib.rdcnn_model_create(ctypes.byref(h), 1, 8, 8, 0, bad, 5, *args) == L.EINVAL
    assert L.lib.rdcnn_model_create(ctypes.byref(h), 1, 0, 8, 0, gs, 5, *args) == L.EINVAL
    assert L.lib.rdcnn_model_create(ctypes.byref(h), 1, 8, 8, 5, gs, 5, *args) == L.EINVAL
    assert L.lib.rdcnn_model_create(ctypes.byref(h), 1, 8, 8, 0, gs, 5, None, 0x3000, 0x4000,
                                    0x5000, None) == L.EINVAL
    assert L.lib.rdcnn_model_create(ctypes.byref(h), 1, 8, 8, 0, gs, 5, 0x2000, 0x3000, 0x4000,
                                    0x4000, None) == L.EINVAL
    assert L.lib.rdcnn_model_create(None, 1, 8, 8, 0, gs, 5, *args) == L.EINVAL
    assert not h.value


def test_null_handle_calls_fail_cleanly(L):
    assert L.lib.rdcnn_step(None, 5) == L.EINVAL
    assert L.lib.rdcnn_read(None, None, None, 1) == L.EINVAL
    assert L.lib.rdcnn_write_state(None, None, None) == L.EINVAL
    assert L.lib.rdcnn_set_params(None, None) == L.EINVAL
    assert L.lib.rdcnn_current(None, None) == L.EINVAL
    assert L.lib.rdcnn_set_kernel(None, 0, 0, 0, 0) == L.EINVAL
    assert L.lib.rdcnn_destroy(None) == L.OK
    assert L.lib.rdcnn_batch_stats(None, None, None, 0.0, 0.0, 0x1000) == L.EINVAL
    assert L.lib.rdcnn_batch_use_lds(None, 1) == L.EINVAL
    assert L.lib.rdcnn_batch_lds_instances(None, None) == L.EINVAL
    assert L.lib.rdcnn_step_record_even(None, 4, 0x1000) == L.EINVAL
    assert L.lib.rdcnn_adjoint_even(None, 0x1000, 4, 0x2000, 0x3000, 0x4000) == L.EINVAL
    assert L.lib.rdcnn_batch_step_record_even(None, 4, 0x1000) == L.EINVAL
    assert L.lib.rdcnn_batch_adjoint_even(None, 0x1000, 4, 0x2000, 0x3000, 0xFF, 0x4000) == L.EINVAL
    assert L.lib.rdcnn_step_bwd(None, 0x1000, 4, 0x2000, 0x3000, 0x4000) == L.EINVAL
    assert L.lib.rdcnn_step_record_sparse(None, 4, 0x1000) == L.EINVAL
    assert L.lib.rdcnn_step_checkpoints(None, 4, 2, 0x1000) == L.EINVAL
    assert L.lib.rdcnn_set_check_finite(None, 1) == L.EINVAL
    assert L.lib.rdcnn_batch_read(None, 0x1000) == L.EINVAL
    assert L.lib.rdcnn_batch_set_check_finite(None, 1) == L.EINVAL
    assert L.lib.rdcnn_batch_set_shared_grad(None, 1) == L.EINVAL
    v = ctypes.c_int()
    assert L.lib.rdcnn_pass_config(None, ctypes.byref(v), ctypes.byref(v), ctypes.byref(v),
                                   ctypes.byref(v)) == L.EINVAL
    assert "NULL" in L.last_error()


def test_status_codes_match_header(L):
    """The Python constants are the header's enum values."""
    text = open(os.path.join(ROOT, "include", "rdcnn.h")).read()
    for name in ("OK", "EINVAL", "EHIP", "ENONFINITE", "ESTATE", "ENOMEM"):
        m = re.search(r"RDCNN_%s\s*=\s*(-?\d+)" % name, text)
        assert m and int(m.group(1)) == getattr(L, name), name


def test_error_is_raised_as_exception(L):
    with pytest.raises(L.RDCNNError) as e:
        L.check(L.lib.rdcnn_step(None, 1))
    assert e.value.code == L.EINVAL
