"""FP64 CPU oracle of the fluctuating non-ideal D3Q19 lattice-Boltzmann step.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the HIP library (``paper_1202_4748_amd``) and neither imports the other.

The stepping code is plain C (``lbfss_oracle.c``, compiled by ``build.py``);
the observables are plain numpy (``moments.py``).
"""
import ctypes
import os

import numpy as np

from . import build as _build

Q = 19

_lib = None


class _Params(ctypes.Structure):
    _fields_ = [("a", ctypes.c_double), ("b", ctypes.c_double), ("kappa", ctypes.c_double),
                ("rho_c", ctypes.c_double), ("kT", ctypes.c_double), ("tau", ctypes.c_double),
                ("force_off", ctypes.c_int), ("tau_bulk", ctypes.c_double), ("tau_ghost", ctypes.c_double)]


def lib():
    """Load (building first if needed) the oracle shared library."""
    global _lib
    if _lib is not None:
        return _lib
    path = _build.library()
    if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
        _build.build(sanitize=path == _build.LIB_SAN)
    L = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    L.orc_lattice.argtypes = [ctypes.POINTER(ctypes.c_int), dp, dp, dp]
    L.orc_philox.argtypes = [u32p, u32p, u32p]
    L.orc_uniform.argtypes = [ctypes.c_uint32]
    L.orc_uniform.restype = ctypes.c_double
    L.orc_site_normals.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int, dp]
    L.orc_gradient.argtypes = [ctypes.c_int, dp, dp]
    L.orc_laplacian.argtypes = [ctypes.c_int, dp, dp]
    L.orc_fields.argtypes = [ctypes.c_int, dp, dp, dp]
    L.orc_chem_potential.argtypes = [ctypes.c_int, ctypes.POINTER(_Params), dp, dp]
    L.orc_force.argtypes = [ctypes.c_int, ctypes.POINTER(_Params), dp, dp, dp]
    L.orc_collide_site.argtypes = [ctypes.POINTER(_Params), dp, dp, dp, dp]
    L.orc_collide_site.restype = ctypes.c_int
    L.orc_init.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_uint64, dp]
    L.orc_step.argtypes = [ctypes.c_int, ctypes.POINTER(_Params), ctypes.c_uint64, ctypes.c_uint64,
                           dp, dp, ctypes.c_int]
    L.orc_step.restype = ctypes.c_int
    L.orc_max_threads.restype = ctypes.c_int
    _lib = L
    return L


def _dp(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def params(a=0.0, b=0.0, kappa=0.0, rho_c=1.0, kT=0.0, tau=1.0, force_off=False, tau_bulk=0.0, tau_ghost=0.0,
           **_ignored):
    """tau_bulk, tau_ghost: relaxation times of moment 4 and of moments 10..18
    (0: the same as tau)."""
    return _Params(a, b, kappa, rho_c, kT, tau, 1 if force_off else 0, tau_bulk, tau_ghost)


def lattice():
    """(c[19,3] int, w[19], basis[19(a),19(i)], norms[19]) as the oracle holds them."""
    c = (ctypes.c_int * (Q * 3))()
    w = np.zeros(Q)
    T = np.zeros((Q, Q))
    n = np.zeros(Q)
    lib().orc_lattice(c, _dp(w), _dp(T), _dp(n))
    return np.array(c[:], dtype=np.int64).reshape(Q, 3), w, T, n


def philox(ctr, key):
    """Philox4x32-10 words for a 4-word counter and 2-word key."""
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (ctypes.c_uint32 * 4)()
    lib().orc_philox(c, k, o)
    return list(o)


def uniform(word):
    return lib().orc_uniform(int(word) & 0xFFFFFFFF)


def site_normals(seed, site, step, domain=0):
    g = np.zeros(16)
    lib().orc_site_normals(seed, site, step, domain, _dp(g))
    return g if domain == 0 else g[:4]


def gradient(psi):
    S = round(psi.size ** (1 / 3))
    psi = np.ascontiguousarray(psi, dtype=np.float64).reshape(-1)
    g = np.zeros(3 * psi.size)
    lib().orc_gradient(S, _dp(psi), _dp(g))
    return g.reshape(3, -1)


def laplacian(psi):
    S = round(psi.size ** (1 / 3))
    psi = np.ascontiguousarray(psi, dtype=np.float64).reshape(-1)
    out = np.zeros(psi.size)
    lib().orc_laplacian(S, _dp(psi), _dp(out))
    return out


def chem_potential(rho, prm):
    S = round(rho.size ** (1 / 3))
    rho = np.ascontiguousarray(rho, dtype=np.float64).reshape(-1)
    mu = np.zeros(rho.size)
    lib().orc_chem_potential(S, ctypes.byref(prm), _dp(rho), _dp(mu))
    return mu


def force(rho, mu, prm):
    S = round(rho.size ** (1 / 3))
    rho = np.ascontiguousarray(rho, dtype=np.float64).reshape(-1)
    mu = np.ascontiguousarray(mu, dtype=np.float64).reshape(-1)
    F = np.zeros(3 * rho.size)
    lib().orc_force(S, ctypes.byref(prm), _dp(rho), _dp(mu), _dp(F))
    return F.reshape(3, -1)


def collide_site(prm, f, F, g=None):
    f = np.ascontiguousarray(f, dtype=np.float64)
    F = np.ascontiguousarray(F, dtype=np.float64)
    out = np.zeros(Q)
    gp = _dp(np.ascontiguousarray(g, dtype=np.float64)) if g is not None else None
    rc = lib().orc_collide_site(ctypes.byref(prm), _dp(f), _dp(F), gp, _dp(out))
    if rc != 0:
        raise FloatingPointError("oracle collision unstable (rho <= 0 or non-finite)")
    return out


def fields(f):
    """rho[N], j[3,N] of post-streaming populations f[19,N] (Eq. (mom))."""
    N = f.shape[1]
    S = round(N ** (1 / 3))
    f = np.ascontiguousarray(f, dtype=np.float64)
    rho = np.zeros(N)
    j = np.zeros(3 * N)
    lib().orc_fields(S, _dp(f), _dp(rho), _dp(j))
    return rho, j.reshape(3, N)


def default_threads():
    env = os.environ.get("OMP_NUM_THREADS")
    return int(env) if env else max(1, os.cpu_count() or 1)


class Sim:
    """One periodic S^3 lattice advanced by the oracle.

    ``f`` holds the post-streaming populations f_i(r, t) as [19, S^3] doubles,
    site = x + S*(y + S*z); ``t`` is the step counter used by the noise.
    """

    def __init__(self, S, seed, a=0.0, b=0.0, kappa=0.0, rho_c=1.0, kT=0.0, tau=1.0,
                 init_sigma=1e-3, force_off=False, nthreads=None, f=None, t=0, tau_bulk=0.0, tau_ghost=0.0):
        self.S = int(S)
        self.N = self.S ** 3
        self.seed = int(seed)
        self.prm = params(a, b, kappa, rho_c, kT, tau, force_off, tau_bulk, tau_ghost)
        self.nthreads = int(nthreads or default_threads())
        self.t = int(t)
        if f is None:
            self.f = np.zeros((Q, self.N))
            lib().orc_init(self.S, rho_c, init_sigma, self.seed, _dp(self.f))
        else:
            self.f = np.ascontiguousarray(f, dtype=np.float64).reshape(Q, self.N).copy()
        self._buf = np.zeros_like(self.f)

    def step(self, n=1):
        for _ in range(int(n)):
            rc = lib().orc_step(self.S, ctypes.byref(self.prm), self.seed, self.t, _dp(self.f),
                                _dp(self._buf), self.nthreads)
            if rc != 0:
                raise FloatingPointError(f"oracle step {self.t} failed with code {rc}")
            self.f, self._buf = self._buf, self.f
            self.t += 1

    def fields(self):
        return fields(self.f)

    def rho(self):
        return self.fields()[0]
