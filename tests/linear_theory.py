"""Linearized theory of the fluctuating non-ideal LB step, used as a pin.

This is an independent route to the model's statics: instead of stepping the
nonlinear model in moment space (what the oracle and the GPU do), it writes
the step linearized around the uniform state f_i = w_i rho0, u = 0 as a
19x19 complex matrix per wave vector, in population space, and solves the
discrete Lyapunov equation for the stationary covariance.

  collision   f* = P f + gamma (I - P) f + 3 w_i c_i . F
              P_ij = w_i (1 + 3 c_i . c_j)      (projector on rho and j)
  force       F(k) = i G(k) [1/3 - rho0 (a + kappa Lam(k))] drho(k)
              G(k) = 3 sum_i w_i c_i sin(k . c_i), Lam(k) = 6 sum_i w_i (1 - cos k . c_i)
  noise       covariance 3 rho0 kT (1 - gamma^2) (W - P W) by the completeness
              of the moment basis (every non-conserved moment a gets variance
              proportional to its norm N_a, Eq. (lbnoise) at c_s^2 = 1/3)
  streaming   f_i(k, t+1) = exp(-i k . c_i) f*_i(k)

The stationary structure factor is S(k) = 1^T Sigma(k) 1 (per site).  Its
closed-form limits (checked in the tests) are: for the ideal lattice gas
(no force) S = 3 rho0 kT at every k; with the force and b = 0,
S(k) -> kT / a as k -> 0 (Ornstein-Zernike, Sec. II A, Eq. (CMF)).
"""
import numpy as np
import scipy.linalg

C = np.array([(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
              (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0), (1, 0, 1), (-1, 0, -1),
              (1, 0, -1), (-1, 0, 1), (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)], dtype=float)
W = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)


def grad_symbol(k):
    k = np.asarray(k, dtype=float)
    return 3.0 * (W * np.sin(C @ k)) @ C


def lap_symbol(k):
    k = np.asarray(k, dtype=float)
    return 6.0 * np.sum(W * (1.0 - np.cos(C @ k)))


def basis():
    """E[a, i] = e_a(c_i), the weight-orthogonal D3Q19 moment basis: 1, c,
    c^2 - 1, 3c_x^2 - c^2, c_y^2 - c_z^2, c_x c_y, c_y c_z, c_z c_x,
    (3c^2 - 5) c, (c_y^2 - c_z^2) c_x, (c_z^2 - c_x^2) c_y, (c_x^2 - c_y^2) c_z,
    3c^4 - 6c^2 + 1, (2c^2 - 3)(3c_x^2 - c^2), (2c^2 - 3)(c_y^2 - c_z^2)."""
    cx, cy, cz = C.T
    c2 = cx * cx + cy * cy + cz * cz
    return np.array([np.ones(19), cx, cy, cz, c2 - 1, 3 * cx * cx - c2, cy * cy - cz * cz,
                     cx * cy, cy * cz, cz * cx, (3 * c2 - 5) * cx, (3 * c2 - 5) * cy, (3 * c2 - 5) * cz,
                     (cy * cy - cz * cz) * cx, (cz * cz - cx * cx) * cy, (cx * cx - cy * cy) * cz,
                     3 * c2 * c2 - 6 * c2 + 1, (2 * c2 - 3) * (3 * cx * cx - c2), (2 * c2 - 3) * (cy * cy - cz * cz)])


def gammas(tau, tau_bulk=0.0, tau_ghost=0.0):
    """gamma_a = 1 - 1/tau_a per moment: bulk a = 4, shear 5..9, ghosts 10..18."""
    t = np.full(19, float(tau))
    if tau_bulk:
        t[4] = tau_bulk
    if tau_ghost:
        t[10:] = tau_ghost
    return 1.0 - 1.0 / t


def step_matrices(k, tau, a=0.0, kappa=0.0, rho0=1.0, kT=1.0, force_off=False, tau_bulk=0.0, tau_ghost=0.0):
    """(A, Qn): f(t+1) = A f(t) + D theta, with D theta of covariance Qn.
    Separate relaxation times relax moment a with gamma_a: the collision is
    sum_a gamma_a Pi_a with the projectors Pi_a = w e_a e_a^T / N_a."""
    E = basis()
    Nrm = (E * E * W).sum(axis=1)
    proj = [W[:, None] * np.outer(E[a], E[a]) / Nrm[a] for a in range(19)]
    gam_a = gammas(tau, tau_bulk, tau_ghost)
    gam = gam_a[5]
    P = W[:, None] * (1.0 + 3.0 * (C @ C.T))
    Cmat = P + sum(gam_a[a] * proj[a] for a in range(4, 19))
    Cmat = Cmat.astype(complex)
    if not force_off:
        G = grad_symbol(k)
        lam = lap_symbol(k)
        coef = 1.0 / 3.0 - rho0 * (a + kappa * lam)
        Fvec = 1j * G * coef                    # F = Fvec * drho, drho = sum_i f_i
        Cmat += 3.0 * np.outer(W * (C @ Fvec), np.ones(19))
    D = np.diag(np.exp(-1j * (C @ np.asarray(k, dtype=float))))
    A = D @ Cmat
    Wd = np.diag(W)
    Qn = 3.0 * rho0 * kT * sum((1.0 - gam_a[a] ** 2) * proj[a] @ Wd for a in range(4, 19))
    Qn = D @ Qn @ D.conj().T
    return A, Qn


def stationary_cov(k, tau, **kw):
    A, Qn = step_matrices(k, tau, **kw)
    if np.max(np.abs(np.linalg.eigvals(A))) > 1.0 - 1e-10:
        return None   # a conserved or frozen mode: no unique stationary state
    return scipy.linalg.solve_discrete_lyapunov(A, Qn)


def structure_factor(k, tau, **kw):
    """<|drho_k|^2> / N of the linearized model, or None for a mode without a
    unique stationary state."""
    Sig = stationary_cov(k, tau, **kw)
    if Sig is None:
        return None
    one = np.ones(19)
    return float(np.real(one @ Sig @ one))


def momentum_variance(k, tau, **kw):
    """<|j_alpha(k)|^2> / N, alpha = x, y, z."""
    Sig = stationary_cov(k, tau, **kw)
    if Sig is None:
        return None
    return np.array([float(np.real(C[:, d] @ Sig @ C[:, d])) for d in range(3)])


def axis_structure_factor(S, tau, **kw):
    """S(k_m) for k_m = 2 pi m / S along x, m = 1 .. S/2 - 1 (the three axes
    are equivalent by the cubic symmetry of the lattice)."""
    return np.array([structure_factor((2 * np.pi * m / S, 0.0, 0.0), tau, **kw)
                     for m in range(1, S // 2)])


_SK_CACHE = {}


def box_variance(S, L, tau, **kw):
    """<m_L^2> of the linearized model: the block average of edge L of the
    order parameter phi = drho / rho0 has variance
    N^-1 L^-6 sum_{k != 0} S(k) |B_L(k)|^2 / rho0^2 with the box Dirichlet sum
    B_L(k) = prod_alpha sum_{n<L} exp(i k_alpha n); k = 0 is excluded by mass
    conservation (Sec. II B, the discussion of Eq. (mL))."""
    rho0 = kw.get("rho0", 1.0)
    ks = 2 * np.pi * np.arange(S) / S
    total = 0.0
    n = np.arange(L)
    B1 = np.array([np.abs(np.sum(np.exp(1j * kk * n))) ** 2 for kk in ks])
    # S(k) on the full grid, using the cubic symmetry to avoid recomputation
    cache = _SK_CACHE.setdefault((S, tau, tuple(sorted(kw.items()))), {})
    for ix in range(S):
        for iy in range(S):
            for iz in range(S):
                if ix == iy == iz == 0:
                    continue
                w = B1[ix] * B1[iy] * B1[iz]
                if w < 1e-12:
                    continue
                key = tuple(sorted((min(ix, S - ix), min(iy, S - iy), min(iz, S - iz))))
                if key not in cache:
                    val = structure_factor((ks[ix], ks[iy], ks[iz]), tau, **kw)
                    cache[key] = val
                val = cache[key]
                if val is None:
                    continue
                total += val * w
    return total / (S ** 3 * L ** 6 * rho0 ** 2)
