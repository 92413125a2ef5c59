"""Oracle of the paper's model in three dimensions: the fluctuating non-ideal
lattice Boltzmann method with the Ginzburg-Landau thermodynamics carried by a
modified equilibrium (Sec. III A), on the D3Q19 lattice, written plainly in
numpy, FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

One time step t -> t+1 on a periodic L^3 lattice, site = x + L (y + L z):
  1. rho = sum_i f_i, j = sum_i c_i f_i                        Eq. (mom)
  2. derivatives of rho with the isotropic D3Q19 stencils
       d_a rho = 3 sum_i w_i c_ia rho(r + c_i),
       lap rho = 6 sum_i w_i [rho(r + c_i) - rho(r)]
  3. thermodynamics of the Landau free energy (Sec. II A, Eq. (landau-pot)) in
     d = rho - rho_c: f0 = a d^2/2 + b d^4/4, p0 = rho f0'(rho) - f0 (below
     Eq. (press-th)), c_s^2 = dp0/drho = rho (a + 3 b d^2)
  4. pressure tensor, Eq. (press-th), and the second moment of the
     equilibrium, Eq. (holdych-cond):
       P = (p0 - kappa rho lap rho - kappa/2 |grad rho|^2) I + kappa grad rho grad rho
       Pi = P + rho u u + nu (u grad rho + grad rho u + (u . grad rho) I),
       nu = (tau - 1/2)/3, u = j/rho
  5. equilibrium populations with the structure of the paper's explicit D2Q9
     equilibrium (the scalar pressure on the moving populations, the rest
     population takes what remains of rho):
       moving  f_i = w_i [3 p_iso + 3 c_i . j + 9/2 (c_i c_i - I/3) : (Pi - p_iso I)]
       rest    f_0 = rho - sum of the moving ones,
     p_iso = p0 - kappa rho lap rho - kappa/2 |grad rho|^2; for an ideal gas
     (p0 = rho/3, kappa = 0, nu terms dropped) this is the standard
     second-order equilibrium
  6. BGK relaxation of the 15 non-conserved moments of the weight-orthogonal
     basis, Eq. (lbe): m*_a = m_a - (m_a - m_a^eq)/tau + theta_a
  7. noise theta with the covariance fdt_moment_covariance gives for the
     local c_s^2 (pre-collision rho), times 3 rho kT (1/tau)(2 - 1/tau):
     the basis norms, except the (bulk, fourth-order ghost) pair, drawn
     through its Cholesky factor (noise_factor)
  8. f*_i = w_i sum_a e_a(c_i) m*_a / N_a, then f_i(r + c_i, t + 1) = f*_i(r)

Normals: the D3Q19 model's generator (Philox4x32-10, counter (site, step_lo,
call | domain << 16, step_hi), key (seed_lo, seed_hi), Box-Muller on word
pairs), calls 0..3 of a site give g_0..g_15, g_{a-4} drives moment a.
Initial state: rho = rho_c + sigma0 g (domain 1, call 0, first normal),
f_i = w_i rho (the lattice gas at rest), as in the force model.
"""
import numpy as np

from . import d2q9 as _d2

C = np.array([(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
              (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0), (1, 0, 1), (-1, 0, -1),
              (1, 0, -1), (-1, 0, 1), (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)])
W = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
Q = 19


def basis():
    """E[a, i] = e_a(c_i): 1, c, c^2 - 1, 3c_x^2 - c^2, c_y^2 - c_z^2,
    c_x c_y, c_y c_z, c_z c_x, (3c^2 - 5) c, (c_y^2 - c_z^2) c_x,
    (c_z^2 - c_x^2) c_y, (c_x^2 - c_y^2) c_z, 3c^4 - 6c^2 + 1,
    (2c^2 - 3)(3c_x^2 - c^2), (2c^2 - 3)(c_y^2 - c_z^2)."""
    cx, cy, cz = (C[:, k].astype(float) for k in range(3))
    c2 = cx * cx + cy * cy + cz * cz
    return np.array([np.ones(Q), cx, cy, cz, c2 - 1, 3 * cx * cx - c2, cy * cy - cz * cz,
                     cx * cy, cy * cz, cz * cx, (3 * c2 - 5) * cx, (3 * c2 - 5) * cy, (3 * c2 - 5) * cz,
                     (cy * cy - cz * cz) * cx, (cz * cz - cx * cx) * cy, (cx * cx - cy * cy) * cz,
                     3 * c2 * c2 - 6 * c2 + 1, (2 * c2 - 3) * (3 * cx * cx - c2), (2 * c2 - 3) * (cy * cy - cz * cz)])


E = basis()
NORM = (E * E * W).sum(axis=1)


def fdt_moment_covariance(C_, W_, E_, cs2):
    """Noise covariance of the linearised BGK step around rest, in the basis
    E_ and in units of 3 rho kT (1/tau)(2 - 1/tau), for a lattice (C_, W_)
    whose equilibrium carries the pressure p0(rho) on its moving populations
    (slope dp0/drho = cs2) and the momentum as 3 w_i c_i . j.

    Requiring the stationary covariance G of the populations to be the same
    at every wave vector makes it diagonal in population space (streaming
    multiplies population i by a phase), and mass and momentum conservation
    of the noise make G c_a and G 1 equilibrium perturbations; with
    <j j> = rho kT I this fixes g_i = 3 rho kT w_i on the moving populations
    and g_0 = rho kT / cs2 - 3 rho kT (1 - w_0) on the rest one (so that
    <drho^2> = rho kT / cs2).  The stationarity condition
    G = B G B^T + Theta with B = gamma I + (1 - gamma) E_eq then gives
    Theta = (1 - gamma^2)(G - C_eq), C_eq = rho kT (e_rho e_rho^T / cs2 +
    sum_a e_ja e_ja^T) the part of G carried by the conserved fields, with
    e_rho = d f^eq / d rho and e_ja = d f^eq / d j_a."""
    C_ = np.asarray(C_, dtype=float)
    W_ = np.asarray(W_, dtype=float)
    g = 3.0 * W_.copy()
    g[0] = 1.0 / cs2 - 3.0 * (1.0 - W_[0])
    e_rho = 3.0 * W_ * cs2
    e_rho[0] = 1.0 - e_rho[1:].sum()
    ceq = np.outer(e_rho, e_rho) / cs2
    for a in range(C_.shape[1]):
        e_j = 3.0 * W_ * C_[:, a]
        ceq += np.outer(e_j, e_j)
    return E_ @ (np.diag(g) - ceq) @ E_.T / 3.0


def noise_factor(cs2):
    """Cholesky factor of fdt_moment_covariance on this basis, in closed form:
    the diagonal is the basis norms N_a except the coupled (bulk a = 4,
    fourth-order ghost a = 16) pair, M_44 = 5/3 - 3 x, M_4,16 = 3 x - 1,
    M_16,16 = 3 - 3 x with x = cs2 (positive definite for x < 1/2).
    Returns (L44, L16_4, L16_16)."""
    x = np.asarray(cs2, dtype=float)
    L44 = np.sqrt(5.0 / 3.0 - 3.0 * x)
    L164 = (3.0 * x - 1.0) / L44
    L1616 = np.sqrt(3.0 - 3.0 * x - L164 * L164)
    return L44, L164, L1616


# --- operators ----------------------------------------------------------------
def shift(field, L, c):
    """field(r + c) on the periodic lattice (field flat, site = x + L (y + L z))."""
    return np.roll(field.reshape(L, L, L), shift=(-c[2], -c[1], -c[0]), axis=(0, 1, 2)).reshape(-1)


def gradient(rho, L):
    g = np.zeros((3, rho.size))
    for i in range(Q):
        s = shift(rho, L, C[i])
        for a in range(3):
            g[a] += 3 * W[i] * C[i, a] * s
    return g


def laplacian(rho, L):
    out = np.zeros(rho.size)
    for i in range(Q):
        out += 6 * W[i] * (shift(rho, L, C[i]) - rho)
    return out


def thermo(rho, a, b, rho_c):
    """p0 and c_s^2 of the Landau free energy at density rho."""
    d = rho - rho_c
    f0 = 0.5 * a * d * d + 0.25 * b * d ** 4
    mu0 = a * d + b * d ** 3
    return rho * mu0 - f0, rho * (a + 3 * b * d * d)


def second_moment(rho, j, grad, lap, prm):
    """(p_iso, Pi[3, 3, n]) of step 4."""
    a, b, kappa, rho_c, tau = prm["a"], prm["b"], prm["kappa"], prm["rho_c"], prm["tau"]
    p0, _ = thermo(rho, a, b, rho_c)
    u = j / rho
    nu = (tau - 0.5) / 3.0
    g2 = (grad * grad).sum(axis=0)
    p_iso = p0 - kappa * rho * lap - 0.5 * kappa * g2
    ug = (u * grad).sum(axis=0)
    Pi = np.empty((3, 3, rho.size))
    for al in range(3):
        for be in range(3):
            Pi[al, be] = (kappa * grad[al] * grad[be] + rho * u[al] * u[be]
                          + nu * (u[al] * grad[be] + grad[al] * u[be]))
        Pi[al, al] += p_iso + nu * ug
    return p_iso, Pi


def equilibrium(rho, j, grad, lap, prm):
    """Equilibrium populations [19, n] (steps 4 and 5)."""
    p_iso, Pi = second_moment(rho, j, grad, lap, prm)
    return equilibrium_from(rho, j, p_iso, Pi)


def equilibrium_from(rho, j, p_iso, Pi):
    """Step 5 for a given scalar pressure p_iso and second moment Pi."""
    Pp = Pi.copy()
    for al in range(3):
        Pp[al, al] -= p_iso
    f = np.empty((Q, rho.size))
    for i in range(1, Q):
        c = C[i].astype(float)
        qc = np.outer(c, c) - np.eye(3) / 3.0
        f[i] = W[i] * (3 * p_iso + 3 * (c @ j) + 4.5 * np.einsum("ab,abn->n", qc, Pp))
    f[0] = rho - f[1:].sum(axis=0)
    return f


def init(L, prm, seed):
    sites = np.arange(L ** 3)
    rho = prm["rho_c"] + prm.get("init_sigma", 1e-3) * _d2.normals(seed, sites, 0, domain=1, calls=1)[0]
    return W[:, None] * rho[None, :]


def step(f, L, prm, seed, t):
    """One step from the post-streaming populations f[19, L^3] at step t."""
    rho = f.sum(axis=0)
    j = C.T.astype(float) @ f
    m = E @ f
    meq = E @ equilibrium(rho, j, gradient(rho, L), laplacian(rho, L), prm)
    tau, kT = prm["tau"], prm["kT"]
    post = m - (m - meq) / tau
    post[0:4] = m[0:4]
    if kT > 0:
        _, cs2 = thermo(rho, prm["a"], prm["b"], prm["rho_c"])
        L44, L164, L1616 = noise_factor(cs2)
        g = _d2.normals(seed, np.arange(L ** 3), t, calls=4)
        sig = np.sqrt(3 * rho * kT * (1 / tau) * (2 - 1 / tau))
        for a in range(5, 19):
            if a != 16:
                post[a] += sig * np.sqrt(NORM[a]) * g[a - 4]
        post[4] += sig * L44 * g[0]
        post[16] += sig * (L164 * g[0] + L1616 * g[12])
    fpost = W[:, None] * (E.T @ (post / NORM[:, None]))
    out = np.empty_like(fpost)
    for i in range(Q):  # pull: f_i(r, t + 1) = f*_i(r - c_i)
        out[i] = shift(fpost[i], L, -C[i])
    return out


class Sim:
    def __init__(self, L, seed, **prm):
        self.L, self.seed = L, seed
        self.prm = dict(a=0.0, b=0.0, kappa=0.0, rho_c=1.0, kT=0.0, tau=1.0, init_sigma=1e-3)
        self.prm.update(prm)
        self.f = init(L, self.prm, seed)
        self.t = 0

    def step(self, n=1):
        for _ in range(n):
            self.f = step(self.f, self.L, self.prm, self.seed, self.t)
            self.t += 1

    def fields(self):
        return self.f.sum(axis=0), C.T.astype(float) @ self.f
