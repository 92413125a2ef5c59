"""lb_fields_static, the field export that allocates no device memory (its
FP64 staging is a static device array of 2^22 doubles per GPU), against
lb_fields through the C ABI: the same bits on consecutive calls, the second
with a smaller replica, then a larger one again; sizes beyond the array are
refused before any device work."""
import ctypes

import numpy as np
import pytest

import workloads
from gpu_util import require_gpu, say

pytestmark = pytest.mark.gpu

M0 = workloads.MODEL


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if a is not None else None


def _static(lbf, sim, replica, rho=True, j=True, f=False):
    N = sim.Ls[replica] ** 3
    r = np.full(N, np.nan) if rho else None
    jj = np.full(3 * N, np.nan) if j else None
    ff = np.full(19 * N, np.nan) if f else None
    rc = lbf.lib().lb_fields_static(sim._h, replica, _dp(r), _dp(jj), _dp(ff))
    return rc, r, jj, ff


def _same(lbf, sim, replica, rho, j, f):
    rc, r, jj, ff = _static(lbf, sim, replica, rho, j, f)
    assert rc == lbf.LB_OK, lbf.lib().lb_strerror(rc)
    ref = sim.fields(replica, rho=rho, j=j, f=f)
    if rho:
        assert np.array_equal(r, ref["rho"])
    if j:
        assert np.array_equal(jj.reshape(3, -1), ref["j"])
    if f:
        assert np.array_equal(ff.reshape(19, -1), ref["f"])


def test_static_export_matches_lb_fields():
    lbf = require_gpu()
    say("no-alloc export: L=40 fp32 with f, then L=12 fp16 batch replica, then L=40 again")
    a = lbf.Sim(40, 5, **M0)            # 23 * 40^3 = 1.47e6 doubles of the 4.19e6
    a.step(7)
    _same(lbf, a, 0, True, True, True)
    b = lbf.Sim.batch([16, 12], [6, 7], [dict(M0, storage="fp16"), dict(M0, storage="fp16", a=0.01)])
    b.step(5)
    _same(lbf, b, 1, True, False, False)   # smaller: 12^3 doubles
    _same(lbf, b, 0, False, True, True)
    a.step(3)
    _same(lbf, a, 0, True, True, True)     # the array holds the last call's contents: nothing leaks


def test_static_export_refuses_sizes_beyond_the_array():
    lbf = require_gpu()
    say("no-alloc export: size limit")
    big = lbf.Sim(64, 1, **M0)     # 23 * 64^3 = 6.0e6 > 2^22 with f; 4 * 64^3 = 1.0e6 without
    rc, *_ = _static(lbf, big, 0, True, True, True)
    assert rc == lbf.LB_EINVAL
    _same(lbf, big, 0, True, True, False)
    r = np.zeros(64 ** 3)
    assert lbf.lib().lb_fields_static(big._h, 1, _dp(r), None, None) == lbf.LB_EINVAL   # no such replica
