"""Pins of the oracle's observables (block moments, axis structure factor)
against brute force and closed forms."""
import numpy as np
import pytest

from oracle import moments


def test_levels():
    assert moments.levels(64) == [32, 16, 8, 4, 2, 1]
    assert moments.levels(48) == [24, 12, 6, 3]
    assert moments.levels(12) == [6, 3]
    assert moments.levels(8) == [4, 2, 1]
    assert moments.levels(256, 2) == [128, 64]


def test_structure_factor_brute_force():
    """Axis S(k) from plane sums equals the O(N^2) direct sum of Eq. (G-comput)."""
    S = 6
    rng = np.random.default_rng(4)
    phi = rng.standard_normal(S ** 3)
    got = moments.axis_structure_factor(phi, S)
    z, y, x = np.meshgrid(np.arange(S), np.arange(S), np.arange(S), indexing="ij")
    r = [x.reshape(-1), y.reshape(-1), z.reshape(-1)]
    for axis in range(3):
        for m in range(1, S // 2):
            k = 2 * np.pi * m / S
            acc = 0j
            for s in range(S ** 3):
                acc += phi[s] * np.exp(-1j * k * r[axis][s])
            assert abs(got[axis, m - 1] - abs(acc) ** 2 / S ** 3) < 1e-12


def test_structure_factor_single_wave():
    S = 16
    z, y, x = np.meshgrid(np.arange(S), np.arange(S), np.arange(S), indexing="ij")
    for m0 in (1, 3, 7):
        phi = np.cos(2 * np.pi * m0 * y / S).reshape(-1)
        sk = moments.axis_structure_factor(phi, S)
        expect = np.zeros(S // 2 - 1)
        expect[m0 - 1] = S ** 3 / 4
        assert np.allclose(sk[1], expect, atol=1e-9)
        assert np.allclose(sk[0], 0, atol=1e-9) and np.allclose(sk[2], 0, atol=1e-9)


def test_block_sums_brute_force():
    S, L = 8, 2
    rng = np.random.default_rng(8)
    rho = 1 + 0.01 * rng.standard_normal(S ** 3)
    phi = moments.order_parameter(rho)
    got = moments.block_sums(phi, S, L)
    ms, Es = [], []
    for bz in range(0, S, L):
        for by in range(0, S, L):
            for bx in range(0, S, L):
                vals = [phi[x + S * (y + S * z)] for z in range(bz, bz + L)
                        for y in range(by, by + L) for x in range(bx, bx + L)]
                ms.append(sum(vals) / L ** 3)
                Es.append(sum(v * v for v in vals) / (2 * L ** 3))
    ms, Es = np.array(ms), np.array(Es)
    assert got["n"] == (S // L) ** 3
    for key, ref in (("m", ms.sum()), ("m2", (ms ** 2).sum()), ("m3", (ms ** 3).sum()),
                     ("m4", (ms ** 4).sum()), ("abs_m", np.abs(ms).sum()), ("E", Es.sum()),
                     ("E2", (Es ** 2).sum())):
        assert abs(got[key] - ref) < 1e-14 * max(1, abs(ref)) + 1e-18
    # boxes tile the lattice: the box means of phi sum to the global phi, 0
    assert abs(got["m"]) < 1e-13
    # L = 1 boxes are the sites (Sec. II B, below Eq. (mL))
    one = moments.block_sums(phi, S, 1)
    assert abs(one["m2"] - np.sum(phi ** 2)) < 1e-15


def test_binder_gaussian_zero():
    rng = np.random.default_rng(0)
    m = rng.standard_normal(2_000_000)
    assert abs(moments.binder(np.mean(m ** 2), np.mean(m ** 4))) < 5e-3
    assert abs(moments.binder(1.0, 1.0) - 2 / 3) < 1e-15     # two delta peaks at +-1
