"""The C-ABI library: loads without a GPU, exports every symbol include/smp.h
declares, and validates arguments on the host (no compute calls here)."""

import ctypes
import os
import re

import pytest

from paper_1610_06656_amd import _lib
from conftest import ROOT, gpu_available

HEADER = os.path.join(ROOT, "include", "smp.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libsmp.so is not built (run __graft_entry__.build())")
    return _lib.load()


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(smp_[a-z_0-9]+)\s*\(", src)))


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), f"{n} declared in smp.h but not exported"
    assert set(names) == set(_lib.EXPORTS), "binding and header disagree"


def test_struct_layouts_match_header():
    # smp_params: 3 int64, 6 int32, double, uint64, 2 int32 -> 72 bytes
    assert ctypes.sizeof(_lib.SmpParams) == 72
    assert ctypes.sizeof(_lib.SmpOmega) == 4 * 8 + 10 * 8
    assert ctypes.sizeof(_lib.SmpJobResult) == 2 * 4 + 2 * 8
    assert ctypes.sizeof(_lib.SmpServerStats) == 3 * 8 + 2 * 4 + 8 + 8


@pytest.mark.skipif(gpu_available(), reason="checks the behaviour without a GPU")
def test_server_entry_points_without_gpu(lib):
    h = ctypes.c_void_p()
    assert lib.smp_server_create(0, 4, 0, ctypes.byref(h)) == _lib.SMP_ERR_INVALID_ARG   # no device
    assert lib.smp_server_create(0, 0, 0, ctypes.byref(h)) == _lib.SMP_ERR_INVALID_ARG   # workers < 1
    jid = ctypes.c_uint64()
    p = _params()
    assert lib.smp_server_submit(None, ctypes.byref(p), None, 0, None, 0, None, None, None,
                                 ctypes.byref(jid)) == _lib.SMP_ERR_INVALID_ARG
    assert lib.smp_server_try_submit(None, ctypes.byref(p), None, 0, None, 0, None, None, None,
                                     ctypes.byref(jid)) == _lib.SMP_ERR_INVALID_ARG
    assert lib.smp_server_wait(None, 1, None) == _lib.SMP_ERR_INVALID_ARG
    lib.smp_server_destroy(None)
    # an empty batch needs no device
    assert lib.smp_solve_batch(0, 0, None, None, None, None, None, None, None, None, 4, 0, None) == _lib.SMP_OK


def _params(**kw):
    from paper_1610_06656_amd.api import make_params
    base = dict(d=1000, n1=50, n2=60, k=20, r=5, T=3)
    base.update(kw)
    return make_params(**base)


@pytest.mark.parametrize("bad", [
    dict(d=0), dict(n1=0), dict(k=0), dict(k=5000), dict(r=0), dict(r=51), dict(r=33, n1=100, n2=100),
    dict(T=-1), dict(m=-1.0), dict(m=float("inf")), dict(prec=7), dict(omega_mode=3), dict(init_iters=-2),
    dict(b_is_a=True),                       # n1 != n2
    dict(T=200, omega_mode=1),               # more than 255 subsets
])
def test_invalid_params_rejected(lib, bad):
    p = _params(**bad)
    assert lib.smp_check_params(ctypes.byref(p)) == _lib.SMP_ERR_INVALID_ARG
    assert len(lib.smp_last_error(None)) > 0
    size = ctypes.c_size_t(0)
    assert lib.smp_workspace_size(ctypes.byref(p), ctypes.byref(size)) == _lib.SMP_ERR_INVALID_ARG


def test_valid_params_and_workspace(lib):
    p = _params()
    assert lib.smp_check_params(ctypes.byref(p)) == _lib.SMP_OK
    size = ctypes.c_size_t(0)
    assert lib.smp_workspace_size(ctypes.byref(p), ctypes.byref(size)) == _lib.SMP_OK
    small = size.value
    p2 = _params(d=200_000, n1=2000, n2=2000, k=400, r=10)
    assert lib.smp_workspace_size(ctypes.byref(p2), ctypes.byref(size)) == _lib.SMP_OK
    assert size.value > small
    # the sketches alone are (n1 + n2) k FP32
    assert size.value > 4000 * 400 * 4


@pytest.mark.parametrize("prec", [1, 2])
def test_workspace_does_not_grow_with_d_through_pi(lib, prec):
    """Alg. 1 step 2 draws Pi, the pass does not keep it: the stored-Pi BF16
    pass holds one bounded window of Pi (at most 128 MiB) and the FP8
    fragment pass one window of Pi and data fragments (at most about
    512 MiB), so from d = 10^6 to d = 10^7 the workspace grows only by what
    depends on d through the split-K partials and nothing else (it is the
    same here)."""
    size = ctypes.c_size_t(0)
    sizes = []
    for d in (1_000_000, 4_000_000, 10_000_000):
        p = _params(d=d, n1=4096, n2=4096, k=1024, r=20, prec=prec)
        assert lib.smp_workspace_size(ctypes.byref(p), ctypes.byref(size)) == _lib.SMP_OK
        sizes.append(size.value)
    assert sizes[0] == sizes[1] == sizes[2]
    # a full k x d Pi at d = 10^7 would be 20 GB (BF16) / 10 GB (FP8) alone
    assert sizes[2] < 2_000_000_000


def test_noalloc_estimate_without_context(lib):
    p = _params()
    assert lib.smp_estimate_noalloc(None, ctypes.byref(p), None, None, None, None, None) == _lib.SMP_ERR_INVALID_ARG


def test_status_strings(lib):
    for s in range(8):
        assert lib.smp_status_str(s) and lib.smp_status_str(s) != b"unknown status"
    assert lib.smp_status_str(0) == b"ok"


def test_null_pointers_rejected_before_launch(lib):
    assert lib.smp_create(None, 0, None) == _lib.SMP_ERR_INVALID_ARG
    p = _params()
    assert lib.smp_sketch(None, ctypes.byref(p), None, 0, None, 0, None, None, None, None) == _lib.SMP_ERR_INVALID_ARG
    assert lib.smp_solve(None, ctypes.byref(p), None, 0, None, 0, None, None, None) == _lib.SMP_ERR_INVALID_ARG
    assert lib.smp_set_timing(None, 1) == _lib.SMP_ERR_INVALID_ARG
    ms = (ctypes.c_float * 5)()
    assert lib.smp_stage_times(None, ms, 5) == _lib.SMP_ERR_INVALID_ARG


@pytest.mark.skipif(gpu_available(), reason="checks the no-device path")
def test_create_without_device_fails_cleanly(lib):
    h = ctypes.c_void_p()
    assert lib.smp_create(ctypes.byref(h), 0, None) == _lib.SMP_ERR_INVALID_ARG


def test_binding_has_no_cpu_fallback(monkeypatch, tmp_path):
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        _lib.load()
