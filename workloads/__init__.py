"""Seeded synthetic inputs shared by the oracle side and the GPU side of the
tests and the benchmark.  Parameter sets and random populations only: no
arithmetic of the method lives here.

The paper (Gross & Varnik) runs 2D D2Q9 simulations with parameter sets, not
datasets; these 3D workloads replace them (sizes, run lengths, parameters).
"""
import numpy as np

SEED = 20120221

# GL parameters of the reference model: critical-point search around a = 0
MODEL = dict(a=0.0, b=0.1, kappa=0.1, rho_c=1.0, kT=1e-4, tau=1.0, init_sigma=1e-3)

WORKLOADS = {
    # oracle-sized case: 16^3, 1000 steps
    "d3q19_16": dict(L=16, steps=1000, **MODEL),
    # 64^3 verification: Gaussian statics (b = 0, a > 0) against Ornstein-Zernike
    "d3q19_64_oz": dict(L=64, steps=20000, **{**MODEL, "a": 0.05, "b": 0.0}),
    "d3q19_64_crit": dict(L=64, steps=20000, **MODEL),
    # plain 256^3 throughput case
    "d3q19_256": dict(L=256, steps=5000, **MODEL),
    # 512^3 precision variant
    "d3q19_512_fp16": dict(L=512, steps=2000, storage="fp16", **MODEL),
    # the paper's own model (GL pressure in the equilibrium, local-sound-speed
    # noise) with the same parameters: on D3Q19 at 256^3, and on D2Q9 at the
    # paper's lattice size 256^2 and at the largest the library takes
    "d3q19_256_eq": dict(L=256, steps=5000, model="eq", **MODEL),
    "d2q9_256": dict(L=256, steps=5000, model="d2q9", **MODEL),
    "d2q9_2048": dict(L=2048, steps=1000, model="d2q9", **MODEL),
}


def sweep_replicas(seeds_per_point=4):
    """Finite-size sweep: L in {8,12,16,24,32,48} x a in {-0.02, -0.00667,
    0.00667, 0.02} x 4 seeds = 96 replicas (b = 0.1, kappa = 0.1, kT = 1e-4)."""
    Ls, seeds, params = [], [], []
    k = 0
    for L in (8, 12, 16, 24, 32, 48):
        for a in (-0.02, -0.02 / 3, 0.02 / 3, 0.02):
            for s in range(seeds_per_point):
                Ls.append(L)
                seeds.append(SEED + 1000 * k + s)
                params.append({**MODEL, "a": a})
            k += 1
    return Ls, seeds, params


def random_populations(L, seed, rho_c=1.0, drho=0.02, u=0.02, neq=0.01):
    """A generic far-from-equilibrium state, [19, L^3] doubles, built from
    random numbers only: the rest weights times (rho_c + a density field of
    standard deviation drho + independent per-population parts of standard
    deviation neq), plus, on each pair of opposite velocities, one random
    number of standard deviation 6 u added to one and taken from the other
    (a site momentum of about u per axis)."""
    rng = np.random.default_rng(seed)
    N = L ** 3
    W = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
    f = W[:, None] * (rho_c + drho * rng.standard_normal(N)[None, :] + neq * rng.standard_normal((19, N)))
    odd = 6.0 * u * rng.standard_normal((9, N))
    f[1::2] += W[1::2, None] * odd   # velocities 1, 3, ..., 17 and their opposites 2, 4, ..., 18
    f[2::2] -= W[2::2, None] * odd
    return f
