"""The C-ABI library loads and exports every entry point its header declares
(no compute call: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

import paper_1202_4748_amd as lbf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "lbfss.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lb2?_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(lbf.library_path()):
        from paper_1202_4748_amd import build
        build.build()
    return lbf.lib()


def test_every_declared_symbol_exported(L):
    names = declared()
    assert set(names) == set(lbf.EXPORTS)
    for n in names:
        assert hasattr(L, n), n


def test_strerror(L):
    for code in (0, -1, -2, -3, -4, -5, 7):
        assert isinstance(L.lb_strerror(code), bytes)
    assert b"unstable" in L.lb_strerror(lbf.LB_EUNSTABLE)


def test_invalid_arguments_rejected_before_device(L):
    """Parameter validation happens on the host, before any HIP call."""
    h = ctypes.c_void_p()
    good = lbf.make_params(a=0.0, b=0.1, kappa=0.1, kT=1e-4, tau=1.0)
    for L_, p in [(3, good), (2000, good),
                  (16, lbf.make_params(tau=0.5)), (16, lbf.make_params(kT=-1.0)),
                  (16, lbf.make_params(kappa=-0.1)), (16, lbf.make_params(b=-1.0)),
                  (16, lbf.make_params(rho_c=0.0)), (16, lbf.make_params(init_sigma=-1.0)),
                  (16, lbf.make_params(sample_every=-1)), (16, lbf.make_params(n_levels=-2)),
                  (16, lbf.make_params(hist_bins=-1)), (16, lbf.make_params(hist_bins=4097, hist_range=1.0)),
                  (16, lbf.make_params(hist_bins=10, hist_range=0.0)),
                  (16, lbf.make_params(hist_bins=10, hist_range=float("inf"))),
                  (16, lbf.make_params(sample_every=5, sk3_stride=-1)),
                  # the paper's model: FP32 storage, one tau, no force switch
                  (16, lbf.make_params(eq_pressure=True, storage="fp16")),
                  (16, lbf.make_params(eq_pressure=True, force_off=True)),
                  (16, lbf.make_params(eq_pressure=True, tau_bulk=1.2)),
                  (16, lbf.make_params(eq_pressure=True, tau_ghost=0.9))]:
        assert L.lb_create(L_, ctypes.byref(p), 1, ctypes.byref(h)) == lbf.LB_EINVAL
    bad = lbf.make_params()
    bad.storage = 7
    assert L.lb_create(16, ctypes.byref(bad), 1, ctypes.byref(h)) == lbf.LB_EINVAL
    # mixed storage in one batch
    Ls = (ctypes.c_int * 2)(8, 8)
    P = (lbf.Params * 2)(lbf.make_params(storage="fp32"), lbf.make_params(storage="fp16"))
    S = (ctypes.c_uint64 * 2)(1, 2)
    assert L.lb_create_batch(2, Ls, P, S, ctypes.byref(h)) == lbf.LB_EINVAL
    assert L.lb_step(None, 1) == lbf.LB_EINVAL
    assert L.lb_sync(None) == lbf.LB_EINVAL
    assert L.lb_histogram(None, 0, None) == lbf.LB_EINVAL
    assert L.lb_hist_estimates(None, 0, None) == lbf.LB_EINVAL
    assert L.lb_sk3(None, 0, None, None) == lbf.LB_EINVAL
    assert L.lb_sk3_shells(None, 0, None, None, None, None) == lbf.LB_EINVAL
    assert L.lb_oz_fit(None, 0, 1.0, 0, None) == lbf.LB_EINVAL
    h2 = ctypes.c_void_p()
    for L_, p2 in [(3, lbf.Params2(0, 0, 0, 1, 0, 1, 0, 0, 0)), (4096, lbf.Params2(0, 0, 0, 1, 0, 1, 0, 0, 0)),
                   (16, lbf.Params2(0, 0, 0, 1, 0, 0.5, 0, 0, 0)), (16, lbf.Params2(0, -1, 0, 1, 0, 1, 0, 0, 0)),
                   (16, lbf.Params2(0, 0, 0, 1, 0, 1, 0, -1, 0))]:
        assert L.lb2_create(L_, ctypes.byref(p2), 1, ctypes.byref(h2)) == lbf.LB_EINVAL
    assert L.lb2_step(None, 1) == lbf.LB_EINVAL
    assert L.lb2_spectra(None, 0, None, None, None, None, None, None) == lbf.LB_EINVAL
    # batches: at least one replica, one sampling period
    arr = (lbf.Params2 * 2)(lbf.Params2(0, 0, 0, 1, 0, 1, 0, 5, 0), lbf.Params2(0, 0, 0, 1, 0, 1, 0, 10, 0))
    seeds = (ctypes.c_uint64 * 2)(1, 2)
    assert L.lb2_create_batch(0, 16, arr, seeds, ctypes.byref(h2)) == lbf.LB_EINVAL
    assert L.lb2_create_batch(2, 16, arr, seeds, ctypes.byref(h2)) == lbf.LB_EINVAL
    assert L.lb2_create_batch(2, 3, arr, seeds, ctypes.byref(h2)) == lbf.LB_EINVAL
    bad_flag = lbf.make_params()
    bad_flag.flags = 4
    assert L.lb_create(16, ctypes.byref(bad_flag), 1, ctypes.byref(h)) == lbf.LB_EINVAL
    # the model must agree across a batch
    P3 = (lbf.Params * 2)(lbf.make_params(eq_pressure=True), lbf.make_params())
    assert L.lb_create_batch(2, Ls, P3, S, ctypes.byref(h)) == lbf.LB_EINVAL
    # sk3_stride must agree across a batch
    Ls2 = (ctypes.c_int * 2)(8, 8)
    P2 = (lbf.Params * 2)(lbf.make_params(sample_every=2, sk3_stride=1), lbf.make_params(sample_every=2))
    assert L.lb_create_batch(2, Ls2, P2, (ctypes.c_uint64 * 2)(1, 2), ctypes.byref(h)) == lbf.LB_EINVAL
    L.lb_destroy(None)


def test_new_calls_check_arguments_on_host(L):
    """lb_philox and lb_set_step reject bad arguments before any HIP call."""
    assert L.lb_philox(-1, None, None, None, None, None) == lbf.LB_EINVAL
    assert L.lb_philox(3, None, None, None, None, None) == lbf.LB_EINVAL
    assert L.lb_philox((1 << 24) + 1, None, None, None, None, None) == lbf.LB_EINVAL
    assert L.lb_philox(0, None, None, None, None, None) == lbf.LB_OK
    assert L.lb_set_step(None, 5) == lbf.LB_EINVAL
