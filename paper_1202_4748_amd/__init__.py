"""Python binding of the lbfss C ABI (``include/lbfss.h``).

Argument marshalling only: every step of the method runs in the HIP kernels
of ``liblbfss.so``.  When PyTorch with a GPU is present, device memory comes
from PyTorch's caching allocator and work is ordered on PyTorch's current
stream; otherwise the library uses hipMalloc and its own stream.

There is no CPU fallback: without the compiled library (or without a GPU)
creating a simulation raises.
"""
import ctypes
import os

import numpy as np

from .build import LIB as _LIB_PATH

Q = 19
LB_OK, LB_EINVAL, LB_ENOMEM, LB_EDEVICE, LB_EUNSTABLE, LB_ESTATE = 0, -1, -2, -3, -4, -5
LB_FP32, LB_FP16 = 0, 1
LB_FORCE_OFF = 1
LB_EQ_PRESSURE = 2
LB_KERNEL_SPLIT, LB_KERNEL_FUSED, LB_KERNEL_STAGED, LB_KERNEL_ROWS = 0, 1, 2, 3
LB_MAX_LEVELS = 16

EXPORTS = ("lb_create", "lb_create_batch", "lb_step", "lb_sync", "lb_moments", "lb_fields",
           "lb_set_populations", "lb_reset_moments", "lb_set_stream", "lb_set_allocator",
           "lb_set_plan", "lb_get_plan", "lb_tune", "lb_info", "lb_destroy", "lb_strerror",
           "lb_histogram", "lb_hist_estimates", "lb_sk3_shells", "lb_sk3", "lb_oz_fit",
           "lb_set_step", "lb_philox", "lb_fields_static",
           "lb2_create", "lb2_create_batch", "lb2_step", "lb2_sync", "lb2_set_stream", "lb2_fields", "lb2_set_populations",
           "lb2_spectra", "lb2_reset_spectra", "lb2_destroy")


class Params(ctypes.Structure):
    _fields_ = [("a", ctypes.c_double), ("b", ctypes.c_double), ("kappa", ctypes.c_double),
                ("rho_c", ctypes.c_double), ("kT", ctypes.c_double), ("tau", ctypes.c_double),
                ("init_sigma", ctypes.c_double), ("storage", ctypes.c_int32),
                ("sample_every", ctypes.c_int32), ("n_levels", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("series_capacity", ctypes.c_int32),
                ("hist_bins", ctypes.c_int32), ("hist_range", ctypes.c_double),
                ("sk3_stride", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("tau_bulk", ctypes.c_double), ("tau_ghost", ctypes.c_double)]


class Params2(ctypes.Structure):
    _fields_ = [("a", ctypes.c_double), ("b", ctypes.c_double), ("kappa", ctypes.c_double),
                ("rho_c", ctypes.c_double), ("kT", ctypes.c_double), ("tau", ctypes.c_double),
                ("init_sigma", ctypes.c_double), ("sample_every", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class OzT(ctypes.Structure):
    _fields_ = [("chi", ctypes.c_double), ("xi", ctypes.c_double), ("C0", ctypes.c_double),
                ("A", ctypes.c_double), ("B", ctypes.c_double), ("n_used", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class HistEst(ctypes.Structure):
    _fields_ = [("Lb", ctypes.c_int32), ("reserved", ctypes.c_int32), ("P0", ctypes.c_double),
                ("chi_center", ctypes.c_double), ("m_max", ctypes.c_double), ("P_max", ctypes.c_double),
                ("chi_peak", ctypes.c_double), ("chi_var", ctypes.c_double), ("chi_var_low", ctypes.c_double),
                ("m_fit", ctypes.c_double), ("chi_fit", ctypes.c_double)]


class LevelSums(ctypes.Structure):
    _fields_ = [("Lb", ctypes.c_int32), ("reserved", ctypes.c_int32), ("n_boxes", ctypes.c_int64),
                ("sum_m", ctypes.c_double), ("sum_m2", ctypes.c_double), ("sum_m3", ctypes.c_double),
                ("sum_m4", ctypes.c_double), ("sum_abs_m", ctypes.c_double), ("sum_E", ctypes.c_double),
                ("sum_E2", ctypes.c_double)]


class MomentsT(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("n_samples", ctypes.c_int64), ("mass", ctypes.c_double),
                ("momentum", ctypes.c_double * 3), ("L", ctypes.c_int32), ("n_levels", ctypes.c_int32),
                ("n_k", ctypes.c_int32), ("series_len", ctypes.c_int32),
                ("series_record", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("level", LevelSums * LB_MAX_LEVELS)]


class InfoT(ctypes.Structure):
    _fields_ = [("n_replicas", ctypes.c_int32), ("storage", ctypes.c_int32),
                ("total_sites", ctypes.c_int64), ("device_bytes", ctypes.c_int64),
                ("step", ctypes.c_int64), ("kernel", ctypes.c_int32), ("tile_x", ctypes.c_int32),
                ("tile_y", ctypes.c_int32), ("tile_z", ctypes.c_int32),
                ("graph_steps", ctypes.c_int32), ("device", ctypes.c_int32)]


class Plan(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int32), ("tile_x", ctypes.c_int32), ("tile_y", ctypes.c_int32),
                ("tile_z", ctypes.c_int32), ("graph_steps", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


_lib = None
_ALLOC_T = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_T = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)
_torch_hooks = None


def library_path():
    return _LIB_PATH


def lib():
    """Load liblbfss.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(f"{_LIB_PATH} is missing: build it with paper_1202_4748_amd/build.py "
                           "(or __graft_entry__.build())")
    L = ctypes.CDLL(_LIB_PATH)
    vp, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)
    i32 = ctypes.c_int
    L.lb_create.argtypes = [i32, ctypes.POINTER(Params), ctypes.c_uint64, ctypes.POINTER(vp)]
    L.lb_create_batch.argtypes = [i32, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(Params),
                                  ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(vp)]
    L.lb_step.argtypes = [vp, ctypes.c_int64]
    L.lb_sync.argtypes = [vp]
    L.lb_moments.argtypes = [vp, i32, ctypes.POINTER(MomentsT), dp, dp]
    L.lb_fields.argtypes = [vp, i32, dp, dp, dp]
    L.lb_set_populations.argtypes = [vp, i32, dp]
    L.lb_reset_moments.argtypes = [vp]
    L.lb_set_stream.argtypes = [vp, vp]
    L.lb_set_allocator.argtypes = [_ALLOC_T, _FREE_T, vp]
    L.lb_set_plan.argtypes = [vp, ctypes.POINTER(Plan)]
    L.lb_get_plan.argtypes = [vp, ctypes.POINTER(Plan)]
    L.lb_tune.argtypes = [vp, i32, ctypes.POINTER(Plan)]
    L.lb_info.argtypes = [vp, ctypes.POINTER(InfoT)]
    L.lb_destroy.argtypes = [vp]
    L.lb_destroy.restype = None
    L.lb_histogram.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_uint64)]
    L.lb_hist_estimates.argtypes = [vp, i32, ctypes.POINTER(HistEst)]
    L.lb_sk3_shells.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64), dp, dp]
    L.lb_sk3.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_int64), dp]
    L.lb_oz_fit.argtypes = [vp, i32, ctypes.c_double, i32, ctypes.POINTER(OzT)]
    L.lb_set_step.argtypes = [vp, ctypes.c_int64]
    L.lb_fields_static.argtypes = [vp, i32, dp, dp, dp]
    u32p, fp = ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_float)
    L.lb_philox.argtypes = [ctypes.c_int64, u32p, u32p, u32p, fp, fp]
    L.lb2_create.argtypes = [i32, ctypes.POINTER(Params2), ctypes.c_uint64, ctypes.POINTER(vp)]
    L.lb2_create_batch.argtypes = [i32, i32, ctypes.POINTER(Params2), ctypes.POINTER(ctypes.c_uint64),
                                   ctypes.POINTER(vp)]
    L.lb2_step.argtypes = [vp, ctypes.c_int64]
    L.lb2_sync.argtypes = [vp]
    L.lb2_set_stream.argtypes = [vp, vp]
    L.lb2_fields.argtypes = [vp, i32, dp, dp, dp]
    L.lb2_set_populations.argtypes = [vp, i32, dp]
    L.lb2_spectra.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_int64), dp, dp, dp, dp, dp]
    L.lb2_reset_spectra.argtypes = [vp]
    L.lb2_destroy.argtypes = [vp]
    L.lb2_destroy.restype = None
    L.lb_strerror.argtypes = [i32]
    L.lb_strerror.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("lb_destroy", "lb_strerror", "lb2_destroy"):
            getattr(L, name).restype = i32
    _lib = L
    return L


class LBError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__(f"{where}: {lib().lb_strerror(code).decode()} ({code})")


def _check(code, where):
    if code != LB_OK:
        raise LBError(code, where)


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if a is not None else None


def _use_torch():
    """Route device allocations through PyTorch's caching allocator (once)."""
    global _torch_hooks
    if _torch_hooks is not None:
        return _torch_hooks is not False
    try:
        import torch
        if not torch.cuda.is_available():
            _torch_hooks = False
            return False
    except Exception:
        _torch_hooks = False
        return False

    def _alloc(nbytes, _ctx):
        dev = torch.cuda.current_device()
        return torch.cuda.caching_allocator_alloc(int(nbytes), dev, torch.cuda.current_stream(dev))

    def _free(ptr, _ctx):
        torch.cuda.caching_allocator_delete(ptr)

    _torch_hooks = (_ALLOC_T(_alloc), _FREE_T(_free))
    _check(lib().lb_set_allocator(_torch_hooks[0], _torch_hooks[1], None), "lb_set_allocator")
    return True


def make_params(a=0.0, b=0.0, kappa=0.0, rho_c=1.0, kT=0.0, tau=1.0, init_sigma=1e-3,
                storage="fp32", sample_every=0, n_levels=0, force_off=False, series_capacity=0,
                hist_bins=0, hist_range=0.0, sk3_stride=0, tau_bulk=0.0, tau_ghost=0.0, eq_pressure=False):
    st = {"fp32": LB_FP32, "fp16": LB_FP16, LB_FP32: LB_FP32, LB_FP16: LB_FP16}[storage]
    return Params(a, b, kappa, rho_c, kT, tau, init_sigma, st, sample_every, n_levels,
                  (LB_FORCE_OFF if force_off else 0) | (LB_EQ_PRESSURE if eq_pressure else 0),
                  series_capacity, int(hist_bins), float(hist_range),
                  int(sk3_stride), 0, float(tau_bulk), float(tau_ghost))


class Sim:
    """A handle of one or more replicas advanced together on the GPU.

    ``Sim(L, seed, **params)`` is one lattice; ``Sim.batch(Ls, seeds,
    params_list)`` many replicas of possibly different sizes and parameters.
    """

    def __init__(self, L=None, seed=0, _handle=None, _Ls=None, **params):
        L_ = lib()
        self._torch = _use_torch()
        if _handle is not None:
            self._h = _handle
            self.Ls = list(_Ls)
        else:
            h = ctypes.c_void_p()
            p = make_params(**params)
            _check(L_.lb_create(int(L), ctypes.byref(p), ctypes.c_uint64(seed), ctypes.byref(h)),
                   "lb_create")
            self._h = h
            self.Ls = [int(L)]
            self._hb = [int(params.get("hist_bins", 0))]
        if self._torch:
            import torch
            cs = torch.cuda.current_stream().cuda_stream
            if cs:  # the legacy default stream is not shared; the library keeps its own
                _check(L_.lb_set_stream(self._h, ctypes.c_void_p(cs)), "lb_set_stream")

    @classmethod
    def batch(cls, Ls, seeds, params_list):
        L_ = lib()
        _use_torch()
        n = len(Ls)
        arrL = (ctypes.c_int * n)(*[int(v) for v in Ls])
        arrP = (Params * n)(*[make_params(**p) for p in params_list])
        arrS = (ctypes.c_uint64 * n)(*[int(s) for s in seeds])
        h = ctypes.c_void_p()
        _check(L_.lb_create_batch(n, arrL, arrP, arrS, ctypes.byref(h)), "lb_create_batch")
        sim = cls(_handle=h, _Ls=Ls)
        sim._hb = [int(p.get("hist_bins", 0)) for p in params_list]
        return sim

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            try:
                _lib.lb_destroy(h)
            finally:
                self._h = None

    def close(self):
        self.__del__()

    def step(self, n=1):
        _check(lib().lb_step(self._h, int(n)), "lb_step")

    def sync(self):
        _check(lib().lb_sync(self._h), "lb_sync")

    def fields(self, replica=0, rho=True, j=True, f=False):
        N = self.Ls[replica] ** 3
        r = np.zeros(N) if rho else None
        jj = np.zeros(3 * N) if j else None
        ff = np.zeros(Q * N) if f else None
        _check(lib().lb_fields(self._h, replica, _dp(r), _dp(jj), _dp(ff)), "lb_fields")
        out = {}
        if rho:
            out["rho"] = r
        if j:
            out["j"] = jj.reshape(3, N)
        if f:
            out["f"] = ff.reshape(Q, N)
        return out

    def set_populations(self, f, replica=0):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(-1)
        _check(lib().lb_set_populations(self._h, replica, _dp(f)), "lb_set_populations")

    def set_step(self, t):
        """Set the step counter (the populations held are then f(r, t))."""
        _check(lib().lb_set_step(self._h, int(t)), "lb_set_step")

    def moments(self, replica=0, series=False):
        m = MomentsT()
        L = self.Ls[replica]
        nk = max(L // 2 - 1, 0)
        sk = np.zeros(3 * max(nk, 1))
        # first call learns the series size
        _check(lib().lb_moments(self._h, replica, ctypes.byref(m), _dp(sk), None), "lb_moments")
        ser = None
        if series and m.series_len > 0:
            buf = np.zeros(m.series_len * m.series_record)
            _check(lib().lb_moments(self._h, replica, ctypes.byref(m), _dp(sk), _dp(buf)), "lb_moments")
            ser = buf.reshape(m.series_len, m.series_record)
        levels = []
        for i in range(m.n_levels):
            lv = m.level[i]
            levels.append({"Lb": lv.Lb, "n_boxes": lv.n_boxes, "m": lv.sum_m, "m2": lv.sum_m2,
                           "m3": lv.sum_m3, "m4": lv.sum_m4, "abs_m": lv.sum_abs_m, "E": lv.sum_E,
                           "E2": lv.sum_E2})
        return {"step": m.step, "n_samples": m.n_samples, "mass": m.mass,
                "momentum": np.array(m.momentum[:]), "L": m.L, "levels": levels,
                "sk": sk[:3 * nk].reshape(3, nk), "series": ser}

    def histogram(self, replica=0):
        """Counts [n_levels, hist_bins + 2] of the box order parameter per level
        (coarsest first): the bins, then below -hist_range, then at or above."""
        m = self.moments(replica)
        nlev = len(m["levels"])
        n = nlev * (self._hb[replica] + 2)
        buf = np.zeros(max(n, 1), dtype=np.uint64)
        _check(lib().lb_histogram(self._h, int(replica), buf.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))),
               "lb_histogram")
        return buf[:n].reshape(nlev, -1)

    def hist_estimates(self, replica=0):
        """Per level (coarsest first): P0, chi_center, m_max, P_max, chi_peak,
        chi_var, chi_var_low (see lb_hist_est in include/lbfss.h)."""
        nlev = len(self.moments(replica)["levels"])
        arr = (HistEst * max(nlev, 1))()
        _check(lib().lb_hist_estimates(self._h, int(replica), arr), "lb_hist_estimates")
        return [{k: getattr(arr[i], k) for k, _ in HistEst._fields_ if k != "reserved"} for i in range(nlev)]

    def sk3(self, replica=0):
        """Shell sums of the 3D structure factor: n_samples, and per shell
        (index = shell, 0 is k = 0) modes, mean k^2, mean lattice Laplacian
        symbol, sum_C (over modes and samples) and mean_C."""
        L_ = lib()
        ns = ctypes.c_int32()
        _check(L_.lb_sk3_shells(self._h, int(replica), ctypes.byref(ns), None, None, None), "lb_sk3_shells")
        n = ns.value
        modes = np.zeros(n, dtype=np.int64)
        k2 = np.zeros(n)
        lap = np.zeros(n)
        _check(L_.lb_sk3_shells(self._h, int(replica), ctypes.byref(ns),
                                modes.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _dp(k2), _dp(lap)),
               "lb_sk3_shells")
        sums = np.zeros(n)
        nsamp = ctypes.c_int64()
        _check(L_.lb_sk3(self._h, int(replica), ctypes.byref(nsamp), _dp(sums)), "lb_sk3")
        with np.errstate(invalid="ignore", divide="ignore"):
            mean = sums / (modes * max(nsamp.value, 1))
        return {"n_samples": nsamp.value, "modes": modes, "k2": k2, "lap": lap, "sum_C": sums, "mean_C": mean}

    def oz_fit(self, replica=0, k_max=1.0, lattice=False):
        o = OzT()
        _check(lib().lb_oz_fit(self._h, int(replica), float(k_max), int(bool(lattice)), ctypes.byref(o)), "lb_oz_fit")
        return {k: getattr(o, k) for k, _ in OzT._fields_ if k != "reserved"}

    def reset_moments(self):
        _check(lib().lb_reset_moments(self._h), "lb_reset_moments")

    def set_plan(self, kernel="fused", tile=(32, 8, 32), graph_steps=0):
        k = {"split": LB_KERNEL_SPLIT, "fused": LB_KERNEL_FUSED, "staged": LB_KERNEL_STAGED,
             "rows": LB_KERNEL_ROWS}[kernel]
        p = Plan(k, tile[0], tile[1], tile[2], graph_steps, 0)
        _check(lib().lb_set_plan(self._h, ctypes.byref(p)), "lb_set_plan")

    def plan(self):
        p = Plan()
        _check(lib().lb_get_plan(self._h, ctypes.byref(p)), "lb_get_plan")
        return p.as_dict()

    def tune(self, steps=20):
        p = Plan()
        _check(lib().lb_tune(self._h, int(steps), ctypes.byref(p)), "lb_tune")
        return p.as_dict()

    def info(self):
        i = InfoT()
        _check(lib().lb_info(self._h, ctypes.byref(i)), "lb_info")
        return {k: getattr(i, k) for k, _ in i._fields_}


def philox(ctr, key):
    """The device generator of the noise on given counters: ctr [n, 4] and key
    [n, 2] (uint32) -> words [n, 4] (uint32), uniforms [n, 4] and Box-Muller
    normals [n, 4] (float32), as the step kernels form them (lb_philox)."""
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    key = np.ascontiguousarray(key, dtype=np.uint32).reshape(-1, 2)
    if ctr.shape[0] != key.shape[0]:
        raise ValueError("ctr and key need the same number of rows")
    n = ctr.shape[0]
    words = np.zeros((n, 4), dtype=np.uint32)
    uni = np.zeros((n, 4), dtype=np.float32)
    nrm = np.zeros((n, 4), dtype=np.float32)
    u32p, fp = ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_float)
    _use_torch()
    _check(lib().lb_philox(n, ctr.ctypes.data_as(u32p), key.ctypes.data_as(u32p), words.ctypes.data_as(u32p),
                           uni.ctypes.data_as(fp), nrm.ctypes.data_as(fp)), "lb_philox")
    return words, uni, nrm


class Sim2D:
    """The paper's own D2Q9 model (Sec. III A) on an L x L lattice: the
    Ginzburg-Landau pressure in a modified equilibrium, local-sound-speed
    noise covariance (see the lb2_* section of include/lbfss.h).
    ``Sim2D.batch(L, seeds, params_list)`` holds many replicas of one L."""

    def __init__(self, L=None, seed=0, a=0.0, b=0.0, kappa=0.0, rho_c=1.0, kT=0.0, tau=1.0, init_sigma=1e-3,
                 sample_every=0, _handle=None, _n=1):
        L_ = lib()
        _use_torch()
        self.L = int(L)
        self.n = int(_n)
        if _handle is not None:
            self._h = _handle
        else:
            p = Params2(a, b, kappa, rho_c, kT, tau, init_sigma, int(sample_every), 0)
            h = ctypes.c_void_p()
            _check(L_.lb2_create(self.L, ctypes.byref(p), ctypes.c_uint64(seed), ctypes.byref(h)), "lb2_create")
            self._h = h
        if _use_torch():
            import torch
            cs = torch.cuda.current_stream().cuda_stream
            if cs:  # as Sim: torch's current stream unless it is the legacy default one
                _check(L_.lb2_set_stream(self._h, ctypes.c_void_p(cs)), "lb2_set_stream")

    @classmethod
    def batch(cls, L, seeds, params_list):
        L_ = lib()
        _use_torch()
        n = len(seeds)
        keys = ("a", "b", "kappa", "rho_c", "kT", "tau", "init_sigma", "sample_every")
        dflt = dict(a=0.0, b=0.0, kappa=0.0, rho_c=1.0, kT=0.0, tau=1.0, init_sigma=1e-3, sample_every=0)
        arrP = (Params2 * n)(*[Params2(*[dict(dflt, **p)[k] for k in keys[:7]],
                                       int(dict(dflt, **p)["sample_every"]), 0) for p in params_list])
        arrS = (ctypes.c_uint64 * n)(*[int(s) for s in seeds])
        h = ctypes.c_void_p()
        _check(L_.lb2_create_batch(n, int(L), arrP, arrS, ctypes.byref(h)), "lb2_create_batch")
        return cls(L, _handle=h, _n=n)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            try:
                _lib.lb2_destroy(h)
            finally:
                self._h = None

    def step(self, n=1):
        _check(lib().lb2_step(self._h, int(n)), "lb2_step")

    def sync(self):
        _check(lib().lb2_sync(self._h), "lb2_sync")

    def fields(self, f=False, replica=0):
        N = self.L * self.L
        rho, j = np.zeros(N), np.zeros(2 * N)
        ff = np.zeros(9 * N) if f else None
        _check(lib().lb2_fields(self._h, int(replica), _dp(rho), _dp(j), _dp(ff)), "lb2_fields")
        out = {"rho": rho, "j": j.reshape(2, N)}
        if f:
            out["f"] = ff.reshape(9, N)
        return out

    def set_populations(self, f, replica=0):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(-1)
        _check(lib().lb2_set_populations(self._h, int(replica), _dp(f)), "lb2_set_populations")

    def spectra(self, replica=0):
        """Sums over samples of the spectra, each [ky, kx]: S, Jx, Jy, Jpar,
        Jperp; and n_samples."""
        N = self.L * self.L
        arr = [np.zeros(N) for _ in range(5)]
        n = ctypes.c_int64()
        _check(lib().lb2_spectra(self._h, int(replica), ctypes.byref(n), *[_dp(a) for a in arr]), "lb2_spectra")
        out = {k: a.reshape(self.L, self.L) for k, a in zip(("S", "Jx", "Jy", "Jpar", "Jperp"), arr)}
        out["n_samples"] = n.value
        return out

    def reset_spectra(self):
        _check(lib().lb2_reset_spectra(self._h), "lb2_reset_spectra")
