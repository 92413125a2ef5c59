"""Oracle of the paper's own model: the fluctuating non-ideal D2Q9 lattice
Boltzmann method with the Ginzburg-Landau thermodynamics carried by a
modified equilibrium (Sec. III A), written plainly in numpy, FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

One time step t -> t+1 on a periodic L x L lattice, site = x + L y:
  1. rho = sum_i f_i, j = sum_i c_i f_i                        Eq. (mom)
  2. derivatives of rho with the isotropic D2Q9 stencils
       d_a rho = 3 sum_i w_i c_ia rho(r + c_i),
       lap rho = 6 sum_i w_i [rho(r + c_i) - rho(r)]
  3. thermodynamics of the Landau free energy (Sec. II A, Eq. (landau-pot)) in
     the density deviation d = rho - rho_c:  f0 = a d^2/2 + b d^4/4,
     p0 = rho f0'(rho) - f0 (the pressure below Eq. (press-th)),
     c_s^2 = dp0/drho = rho (a + 3 b d^2)
  4. pressure tensor, Eq. (press-th):
       P_ab = (p0 - kappa rho lap rho - kappa/2 |grad rho|^2) delta_ab
              + kappa d_a rho d_b rho
  5. second moment of the equilibrium, Eq. (holdych-cond):
       Pi_ab = P_ab + rho u_a u_b + nu (u_a d_b rho + u_b d_a rho
               + u.grad rho delta_ab),  nu = (tau - 1/2)/3, u = j/rho
  6. the equilibrium in moment space (the weight-orthogonal basis below), as
     the paper's explicit equilibrium projects: rho, j, 3 tr Pi - 2 rho,
     Pi_xx - Pi_yy, Pi_xy, zero for the two third-order ghosts, and
     2 rho - 6 (p0 - kappa rho lap rho) - 3 kappa |grad rho|^2 for the
     fourth-order one (zero for an ideal gas, p0 = rho/3, kappa = 0)
  7. BGK relaxation of the six non-conserved moments, Eq. (lbe):
       m*_a = m_a - (m_a - m_a^eq)/tau + theta_a
  8. noise theta with the covariance of Eq. (lbnoise),
       Theta = 3 rho kT (1/tau)(2 - 1/tau) M(c_s^2),
       M diagonal 4(2 - 3 c_s^2), 4/9, 1/9, 2/3, 2/3, 16(5/4 - 3 c_s^2/4) on
       the moments 3..8, plus the coupling 12(c_s^2 - 1/3) of moments 3 and 8,
       drawn through its Cholesky factor from six standard normals
  9. f*_i = w_i sum_a e_a(c_i) m*_a / N_a, then f_i(r + c_i, t + 1) = f*_i(r)

The normals are those of the D3Q19 model's generator: Philox4x32-10 with
counter (site, step_lo, call | domain << 16, step_hi), key (seed_lo,
seed_hi), uniforms ((w >> 9) + 1/2) 2^-23, Box-Muller on word pairs; calls 0
and 1 give normals g_0..g_7, of which g_0..g_5 drive moments 3..8.  The
initial state is rho = rho_c + sigma0 g (domain 1, call 0, first normal),
u = 0, f = the equilibrium of that density.
"""
import numpy as np

C = np.array([(0, 0), (1, 0), (-1, 0), (0, 1), (0, -1), (1, 1), (-1, -1), (1, -1), (-1, 1)])
W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
Q = 9


def basis():
    """E[a, i] = e_a(c_i): 1, c_x, c_y, 3c^2 - 2, c_x^2 - c_y^2, c_x c_y,
    (3c^2 - 4) c_x, (3c^2 - 4) c_y, 9c^4 - 15c^2 + 2."""
    cx, cy = C[:, 0].astype(float), C[:, 1].astype(float)
    c2 = cx * cx + cy * cy
    return np.array([np.ones(Q), cx, cy, 3 * c2 - 2, cx * cx - cy * cy, cx * cy,
                     (3 * c2 - 4) * cx, (3 * c2 - 4) * cy, 9 * c2 * c2 - 15 * c2 + 2])


E = basis()
NORM = (E * E * W).sum(axis=1)


# --- random numbers ---------------------------------------------------------
M0, M1 = np.uint64(0xD2511F53), np.uint64(0xCD9E8D57)
K0, K1 = 0x9E3779B9, 0xBB67AE85
MASK = np.uint64(0xFFFFFFFF)


def philox(c0, c1, c2, c3, k0, k1):
    """Philox4x32-10 on arrays of counters (uint64 holding 32-bit words)."""
    c0, c1, c2, c3 = (np.asarray(v, dtype=np.uint64) & MASK for v in (c0, c1, c2, c3))
    for r in range(10):
        kk0 = np.uint64((k0 + r * K0) & 0xFFFFFFFF)
        kk1 = np.uint64((k1 + r * K1) & 0xFFFFFFFF)
        p0 = M0 * c0
        p1 = M1 * c2
        n0 = (p1 >> np.uint64(32)) ^ c1 ^ kk0
        n2 = (p0 >> np.uint64(32)) ^ c3 ^ kk1
        c0, c1, c2, c3 = n0 & MASK, p1 & MASK, n2 & MASK, p0 & MASK
    return c0, c1, c2, c3


def uniform(w):
    return ((np.asarray(w, dtype=np.uint64) >> np.uint64(9)).astype(np.float64) + 0.5) * (1.0 / 8388608.0)


def normals(seed, sites, step, domain=0, calls=2):
    """Standard normals [4 * calls, len(sites)] of the given sites and step."""
    sites = np.asarray(sites, dtype=np.uint64)
    k0, k1 = seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF
    out = []
    for j in range(calls):
        w = philox(sites, np.full_like(sites, step & 0xFFFFFFFF), np.full_like(sites, j | (domain << 16)),
                   np.full_like(sites, (step >> 32) & 0xFFFFFFFF), k0, k1)
        for p in range(2):
            u0, u1 = uniform(w[2 * p]), uniform(w[2 * p + 1])
            r = np.sqrt(-2.0 * np.log(u0))
            out += [r * np.cos(2 * np.pi * u1), r * np.sin(2 * np.pi * u1)]
    return np.array(out)


# --- operators ----------------------------------------------------------------
def shift(field, L, c):
    """field(r + c) on the periodic lattice (field flat, site = x + L y)."""
    return np.roll(field.reshape(L, L), shift=(-c[1], -c[0]), axis=(0, 1)).reshape(-1)


def gradient(rho, L):
    g = np.zeros((2, rho.size))
    for i in range(Q):
        s = shift(rho, L, C[i])
        g[0] += 3 * W[i] * C[i, 0] * s
        g[1] += 3 * W[i] * C[i, 1] * s
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


def eq_moments(rho, j, grad, lap, prm):
    """Equilibrium moments [9, n] (steps 3-6 of the module docstring)."""
    a, b, kappa, rho_c, tau = prm["a"], prm["b"], prm["kappa"], prm["rho_c"], prm["tau"]
    p0, _ = thermo(rho, a, b, rho_c)
    gx, gy = grad
    u = j / rho
    ux, uy = u
    nu = (tau - 0.5) / 3.0
    iso = p0 - kappa * rho * lap - 0.5 * kappa * (gx * gx + gy * gy)
    ug = ux * gx + uy * gy
    Pxx = iso + kappa * gx * gx + rho * ux * ux + nu * (2 * ux * gx + ug)
    Pyy = iso + kappa * gy * gy + rho * uy * uy + nu * (2 * uy * gy + ug)
    Pxy = kappa * gx * gy + rho * ux * uy + nu * (ux * gy + uy * gx)
    z = np.zeros_like(rho)
    # the fourth-order moment of the paper's explicit equilibrium (rest
    # weights 1/3, 1/12 and the gradient weights w^xx, w^yy, w^xy): the scalar
    # p0 - kappa rho lap rho and the squared gradients project onto it
    m8 = 2 * rho - 6 * (p0 - kappa * rho * lap) - 3 * kappa * (gx * gx + gy * gy)
    return np.array([rho, j[0], j[1], 3 * (Pxx + Pyy) - 2 * rho, Pxx - Pyy, Pxy, z, z, m8])


def noise_factor(cs2):
    """Cholesky factor entries of M(c_s^2) (the bracket of Eq. (lbnoise)) on
    the moments 3..8: returns (L33, L83, L88) of the coupled pair 3, 8 and the
    square roots of the four diagonal entries of moments 4..7."""
    A = 4 * (2 - 3 * cs2)
    Cc = 12 * (cs2 - 1.0 / 3.0)
    B = 16 * (1.25 - 0.75 * cs2)
    L33 = np.sqrt(A)
    L83 = Cc / L33
    L88 = np.sqrt(B - L83 * L83)
    return L33, L83, L88, np.sqrt(np.array([4 / 9, 1 / 9, 2 / 3, 2 / 3]))


def equilibrium(rho, j, L, prm):
    m = eq_moments(rho, j, gradient(rho, L), laplacian(rho, L), prm)
    return (W[:, None] * (E.T @ (m / NORM[:, None])))


def init(L, prm, seed):
    sites = np.arange(L * L)
    rho = prm["rho_c"] + prm.get("init_sigma", 1e-3) * normals(seed, sites, 0, domain=1, calls=1)[0]
    return equilibrium(rho, np.zeros((2, L * L)), L, prm)


def step(f, L, prm, seed, t):
    """One step from the post-streaming populations f[9, L*L] at step t."""
    rho = f.sum(axis=0)
    j = C.T.astype(float) @ f
    m = E @ f
    meq = eq_moments(rho, j, gradient(rho, L), laplacian(rho, L), prm)
    tau, kT = prm["tau"], prm["kT"]
    post = m - (m - meq) / tau
    post[0:3] = m[0:3]
    if kT > 0:
        _, cs2 = thermo(rho, prm["a"], prm["b"], prm["rho_c"])
        L33, L83, L88, dg = noise_factor(cs2)
        g = normals(seed, np.arange(L * L), t)
        sig = np.sqrt(3 * rho * kT * (1 / tau) * (2 - 1 / tau))
        post[3] += sig * L33 * g[0]
        post[4] += sig * dg[0] * g[1]
        post[5] += sig * dg[1] * g[2]
        post[6] += sig * dg[2] * g[3]
        post[7] += sig * dg[3] * g[4]
        post[8] += sig * (L83 * g[0] + L88 * g[5])
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
