"""Pins of the oracle's lattice tables: D3Q19 velocities, weights and the
moment basis (Sec. III A, the expansion f_i = T_ai w_i m_a / N_a)."""
import itertools
from fractions import Fraction

import numpy as np
import pytest

import oracle


def test_velocity_set_is_d3q19():
    c, w, _, _ = oracle.lattice()
    vs = {tuple(v) for v in c}
    expect = {(0, 0, 0)}
    for v in itertools.product((-1, 0, 1), repeat=3):
        if 1 <= sum(abs(x) for x in v) <= 2:
            expect.add(v)
    assert vs == expect and len(c) == 19
    # opposite pairs are stored next to each other (1,2), (3,4), ...
    for k in range(1, 19, 2):
        assert tuple(c[k]) == tuple(-c[k + 1])


def test_weights_isotropy():
    """sum w = 1, sum w c_a c_b = c_s^2 delta, fourth moments isotropic with
    c_s^4 (the conditions a second-order lattice equilibrium needs)."""
    c, w, _, _ = oracle.lattice()
    c = c.astype(float)
    assert abs(w.sum() - 1) < 1e-15
    for a in range(3):
        assert abs(np.sum(w * c[:, a])) < 1e-15
        for b in range(3):
            assert abs(np.sum(w * c[:, a] * c[:, b]) - (a == b) / 3) < 1e-15
            for g in range(3):
                assert abs(np.sum(w * c[:, a] * c[:, b] * c[:, g])) < 1e-15
                for d in range(3):
                    iso = ((a == b) * (g == d) + (a == g) * (b == d) + (a == d) * (b == g)) / 9
                    assert abs(np.sum(w * c[:, a] * c[:, b] * c[:, g] * c[:, d]) - iso) < 1e-15


def test_basis_weight_orthogonal_and_complete():
    c, w, T, n = oracle.lattice()
    G = (T * w) @ T.T
    assert np.allclose(G, np.diag(n), atol=1e-14)
    assert np.linalg.matrix_rank(T) == 19
    # completeness: sum_a e_a(c_i) e_a(c_j) / N_a = delta_ij / w_i
    Cm = T.T @ np.diag(1 / n) @ T
    assert np.allclose(Cm, np.diag(1 / w), atol=1e-12)
    # first four moments are density and momentum
    assert np.allclose(T[0], 1) and np.allclose(T[1:4], c.T)


def test_basis_norms_exact():
    """N_a as exact rationals: the oracle's norms are the squared weighted
    lengths of its basis vectors (integer-valued polynomials in c)."""
    c, w, T, n = oracle.lattice()
    wf = [Fraction(1, 3) if sum(abs(x) for x in v) == 0 else
          Fraction(1, 18) if sum(abs(x) for x in v) == 1 else Fraction(1, 36) for v in c]
    for a in range(19):
        assert np.allclose(T[a], np.round(T[a]))
        exact = sum(wf[i] * int(round(T[a, i])) ** 2 for i in range(19))
        assert abs(float(exact) - n[a]) < 1e-15


def _frac(s):
    num, _, den = s.partition("/")
    return Fraction(int(num), int(den or 1))


def test_noise_reading_matches_paper_d2q9():
    """The paper's noise covariance (Eq. (lbnoise)) at c_s^2 = 1/3 is diagonal
    with entries equal to the weighted norms of the D2Q9 analog of the basis
    (1, c, c^2-type stresses, cubic ghosts, the quartic mode).  This pins the
    reading 'variance of non-conserved moment a = 3 rho kT (1 - gamma^2) N_a'
    that the D3Q19 oracle applies with its own N_a."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "paper_lbnoise_d2q9.txt")
    paper = [_frac(line.split()[1]) for line in open(path)
             if line.strip() and not line.startswith("#")]
    cs = [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)]
    wq = [Fraction(4, 9)] + [Fraction(1, 9)] * 4 + [Fraction(1, 36)] * 4

    def e(v):
        x, y = v
        c2 = x * x + y * y
        return [3 * c2 - 2, x * x - y * y, x * y, (3 * c2 - 4) * x, (3 * c2 - 4) * y,
                9 * c2 * c2 - 15 * c2 + 2]

    E = [e(v) for v in cs]
    norms = [sum(wq[i] * E[i][a] ** 2 for i in range(9)) for a in range(6)]
    for a in range(6):
        for b in range(6):
            if a != b:
                assert sum(wq[i] * E[i][a] * E[i][b] for i in range(9)) == 0
    assert norms == paper
