"""Parts of the C ABI around the step: lb_info, lb_step's count argument,
the caller's stream (lb_set_stream) and the device allocator
(lb_set_allocator; the Python binding routes allocations through PyTorch's
caching allocator, the library's own default is hipMalloc).  None of them
may change a result: the state depends only on (L, parameters, seed, step
count)."""
import numpy as np
import pytest

import workloads
from gpu_util import require_gpu, say

pytestmark = pytest.mark.gpu

M0 = workloads.MODEL


def test_info_reports_the_handle():
    lbf = require_gpu()
    sim = lbf.Sim.batch([12, 8], [1, 2], [dict(M0), dict(M0)])
    i = sim.info()
    assert i["n_replicas"] == 2 and i["storage"] == lbf.LB_FP32
    assert i["total_sites"] == 12 ** 3 + 8 ** 3
    # at least the two population buffers
    assert i["device_bytes"] >= 2 * 19 * 4 * i["total_sites"]
    assert i["step"] == 0
    sim.step(7)
    assert sim.info()["step"] == 7
    p = sim.plan()
    assert (i["kernel"], i["tile_x"], i["tile_y"], i["tile_z"]) == (p["kernel"], p["tile_x"], p["tile_y"], p["tile_z"])


def test_plan_changes_release_their_tables():
    """Switching plans frees the tile tables it no longer needs (the rows
    table and, for FP32 64 x 8 plans, the 64 x 4 table of their sample
    steps): device memory is the same after any number of switches."""
    lbf = require_gpu()
    sim = lbf.Sim(64, 4, sample_every=5, **M0)
    plans = [("rows", (64, 8, 16)), ("rows", (64, 4, 16)), ("split", (0, 0, 0)), ("rows", (64, 8, 32)),
             ("fused", (32, 8, 16))]
    sim.set_plan(*plans[0])
    sim.step(5)
    first = None
    for rnd in range(3):
        for k, t in plans:
            sim.set_plan(k, t)
            sim.step(5)
        b = sim.info()["device_bytes"]
        first = b if first is None else first
        assert b == first, (rnd, b, first)


def test_step_count_zero_and_negative():
    lbf = require_gpu()
    sim = lbf.Sim(8, 3, **M0)
    sim.step(4)
    before = sim.fields(f=True)["f"]
    sim.step(0)
    assert sim.info()["step"] == 4
    assert np.array_equal(sim.fields(f=True)["f"], before)
    with pytest.raises(lbf.LBError) as e:
        sim.step(-1)
    assert e.value.code == lbf.LB_EINVAL
    assert sim.info()["step"] == 4


def test_stream_and_allocator_do_not_change_results():
    """The same lattice on the library's own stream with PyTorch's
    allocator, on a PyTorch side stream, and with hipMalloc (the library's
    default, selected by passing no allocator), moved between streams half
    way: identical populations."""
    import torch
    lbf = require_gpu()
    L, seed, steps = 20, 41, 16
    prm = dict(M0, sample_every=4)
    say("own stream, torch allocator")
    ref = lbf.Sim(L, seed, **prm)
    ref.step(steps)
    f_ref = ref.fields(f=True)["f"]
    m_ref = ref.moments()

    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        say("torch side stream")
        a = lbf.Sim(L, seed, **prm)
        a.step(steps)
        side.synchronize()
        f_a = a.fields(f=True)["f"]

    lib = lbf.lib()
    hooks = lbf._torch_hooks
    assert hooks and hooks is not True
    try:
        # null function pointers: back to the library's own hipMalloc/hipFree
        assert lib.lb_set_allocator(lbf._ALLOC_T(), lbf._FREE_T(), None) == lbf.LB_OK
        say("hipMalloc, from the side stream to the library's own after half the steps")
        with torch.cuda.stream(side):
            b = lbf.Sim(L, seed, **prm)
            b.step(steps // 2)
        assert lib.lb_set_stream(b._h, None) == lbf.LB_OK  # synchronises the side stream first
        b.step(steps - steps // 2)
        f_b = b.fields(f=True)["f"]
        m_b = b.moments()
        del b
    finally:
        assert lib.lb_set_allocator(hooks[0], hooks[1], None) == lbf.LB_OK
    assert np.array_equal(f_a, f_ref)
    assert np.array_equal(f_b, f_ref)
    assert m_b["mass"] == m_ref["mass"] and m_b["levels"] == m_ref["levels"]


def test_d2q9_stream_does_not_change_results():
    """The D2Q9 handle (lb2_set_stream): on its own stream, on a PyTorch side
    stream, and moved from the side stream back to its own half way, with the
    spectra sampled: identical populations and spectra."""
    import torch
    lbf = require_gpu()
    L, seed, steps = 24, 43, 18
    prm = dict(a=0.03, b=0.5, kappa=0.01, rho_c=1.0, kT=1e-5, tau=0.8, init_sigma=0.02, sample_every=3)
    say("d2q9 own stream")
    ref = lbf.Sim2D(L, seed, **prm)
    ref.step(steps)
    f_ref = ref.fields(f=True)["f"]
    s_ref = ref.spectra()
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        say("d2q9 torch side stream, back to its own after half the steps")
        b = lbf.Sim2D(L, seed, **prm)
        b.step(steps // 2)
    assert lbf.lib().lb2_set_stream(b._h, None) == lbf.LB_OK  # synchronises the side stream first
    b.step(steps - steps // 2)
    f_b = b.fields(f=True)["f"]
    s_b = b.spectra()
    assert np.array_equal(f_b, f_ref)
    assert s_b["n_samples"] == s_ref["n_samples"] == steps // 3
    for k in ("S", "Jx", "Jy"):
        assert np.array_equal(s_b[k], s_ref[k]), k
