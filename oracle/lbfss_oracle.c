/*
 * FP64 CPU oracle for the fluctuating non-ideal lattice-Boltzmann time step
 * (Gross & Varnik, "Simulation of static critical phenomena in non-ideal
 * fluids with the Lattice Boltzmann method").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the
 * GPU path is checked against.  Only the tests, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no source with
 * the HIP library and must never be used as a fallback for it.
 *
 * What it computes (paper, Sec. III A, Eq. (lbe) and Eq. (mom)):
 *   f_i(r + c_i, t + 1) = f_i(r, t) - [f_i - f_i^eq] / tau + theta_i
 * written in moment space (Sec. III A, the basis expansion following Eq. (mom))
 * on a periodic D3Q19 lattice.  Readings where the paper is silent or 2D-only:
 *   - lattice D3Q19 instead of the paper's D2Q9, c_s^2 = 1/3;
 *   - the Ginzburg-Landau thermodynamics (Sec. II A, Eqs. (fef), (landau-pot))
 *     enters as a body force F = -rho grad(mu) + c_s^2 grad(rho) with
 *     mu = a (rho - rho_c) + b (rho - rho_c)^3 - kappa lap(rho); the first term
 *     has divergence-of-pressure-tensor form (Sec. III A, the identity
 *     div P = rho grad(dF/dphi)), the second cancels the ideal-gas pressure of
 *     the lattice fluid; the force is applied with Guo's second-order scheme;
 *   - the noise covariance of Eq. (lbnoise) evaluated for an ideal-gas
 *     equilibrium (c_s^2 = 1/3) is diagonal: variance
 *     (rho kT / c_s^2) (1/tau)(2 - 1/tau) N_a on every non-conserved moment a;
 *   - one relaxation time tau for all non-conserved moments (BGK, Eq. (lbe));
 *   - Gaussian numbers from Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11)
 *     through the Box-Muller transform, keyed by (seed, step, site).
 *
 * Arrays: populations are f[q * N + site], site = x + S * (y + S * z),
 * N = S^3.  The state held between steps is the post-streaming population
 * f_i(r, t).  Everything is IEEE double.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define Q 19

/* D3Q19 velocities: rest, 6 axis neighbours, 12 face diagonals, in opposite
 * pairs (2k-1, 2k). */
static const int CV[Q][3] = {
    {0, 0, 0},
    {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
    {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

static const double CS2 = 1.0 / 3.0;

typedef struct {
    double a, b, kappa, rho_c, kT, tau;
    int force_off; /* 1: F = 0 (ideal lattice gas, used by the tests) */
    double tau_bulk, tau_ghost; /* relaxation times of moment 4 and of moments 10..18; 0 = tau */
} orc_params;

/* Relaxation time of moment a (>= 4): bulk (a = 4), shear (5..9, tau), ghosts
 * (10..18).  One tau for all is the BGK collision of Eq. (lbe); separate
 * rates are the multiple-relaxation-time form in which the paper sets all
 * of them to one value (Sec. III B). */
static double tau_of(const orc_params *p, int a) {
    if (a == 4 && p->tau_bulk > 0.0) return p->tau_bulk;
    if (a >= 10 && p->tau_ghost > 0.0) return p->tau_ghost;
    return p->tau;
}

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_EUNSTABLE = -4 };

static double weight(int i) {
    int c2 = CV[i][0] * CV[i][0] + CV[i][1] * CV[i][1] + CV[i][2] * CV[i][2];
    return c2 == 0 ? 1.0 / 3.0 : (c2 == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
}

/* Moment basis vector a evaluated at velocity c (a weight-orthogonal
 * polynomial basis: 1, c, bulk, two normal stresses, three shear stresses,
 * nine ghost moments). */
static double basis(int a, const int *c) {
    double x = c[0], y = c[1], z = c[2];
    double c2 = x * x + y * y + z * z;
    switch (a) {
    case 0: return 1.0;
    case 1: return x;
    case 2: return y;
    case 3: return z;
    case 4: return c2 - 1.0;
    case 5: return 3.0 * x * x - c2;
    case 6: return y * y - z * z;
    case 7: return x * y;
    case 8: return y * z;
    case 9: return z * x;
    case 10: return (3.0 * c2 - 5.0) * x;
    case 11: return (3.0 * c2 - 5.0) * y;
    case 12: return (3.0 * c2 - 5.0) * z;
    case 13: return (y * y - z * z) * x;
    case 14: return (z * z - x * x) * y;
    case 15: return (x * x - y * y) * z;
    case 16: return 3.0 * c2 * c2 - 6.0 * c2 + 1.0;
    case 17: return (2.0 * c2 - 3.0) * (3.0 * x * x - c2);
    case 18: return (2.0 * c2 - 3.0) * (y * y - z * z);
    }
    return 0.0;
}

static double T[Q][Q]; /* T[a][i] = e_a(c_i) */
static double NRM[Q];  /* N_a = sum_i w_i e_a(c_i)^2 */
static double WQ[Q];
static int tables_ready = 0;

static void tables(void) {
    if (tables_ready) return;
    for (int i = 0; i < Q; ++i) WQ[i] = weight(i);
    for (int a = 0; a < Q; ++a) {
        double n = 0.0;
        for (int i = 0; i < Q; ++i) {
            T[a][i] = basis(a, CV[i]);
            n += WQ[i] * T[a][i] * T[a][i];
        }
        NRM[a] = n;
    }
    tables_ready = 1;
}

/* Copies of the lattice tables, for the tests. */
void orc_lattice(int *c_out, double *w_out, double *basis_out, double *norms_out) {
    tables();
    for (int i = 0; i < Q; ++i) {
        for (int d = 0; d < 3; ++d) c_out[3 * i + d] = CV[i][d];
        w_out[i] = WQ[i];
    }
    for (int a = 0; a < Q; ++a) {
        norms_out[a] = NRM[a];
        for (int i = 0; i < Q; ++i) basis_out[a * Q + i] = T[a][i];
    }
}

/* ---------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon et al., SC'11): a 4x32-bit counter is permuted by  */
/* ten rounds of two 32x32->64 multiplications whose high halves are mixed  */
/* into the other two words with the round key; the 2x32-bit key advances  */
/* by the Weyl increments between rounds.                                   */
/* ---------------------------------------------------------------------- */
void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

/* Uniform number in (0,1) from the top 23 bits of a word, centred in its
 * bin: ((w >> 9) + 1/2) / 2^23.  Exactly representable in float and double. */
double orc_uniform(uint32_t w) { return ((double)(w >> 9) + 0.5) * (1.0 / 8388608.0); }

/* The random words of one site and step: counter (site, step_lo,
 * call | domain << 16, step_hi), key (seed_lo, seed_hi).  Domain 0 is the
 * collision noise (calls 0..3), domain 1 the initial density (call 0). */
static void site_words(uint64_t seed, uint64_t site, uint64_t step, int domain, int ncalls,
                       uint32_t *words) {
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int j = 0; j < ncalls; ++j) {
        uint32_t ctr[4] = {(uint32_t)site, (uint32_t)step, (uint32_t)j | ((uint32_t)domain << 16),
                           (uint32_t)(step >> 32)};
        orc_philox(ctr, key, words + 4 * j);
    }
}

/* Box-Muller on consecutive word pairs: g_{2p} = r cos(2 pi U_{2p+1}),
 * g_{2p+1} = r sin(2 pi U_{2p+1}), r = sqrt(-2 ln U_{2p}). */
static void box_muller(const uint32_t *words, int npairs, double *g) {
    for (int p = 0; p < npairs; ++p) {
        double u0 = orc_uniform(words[2 * p]);
        double u1 = orc_uniform(words[2 * p + 1]);
        double r = sqrt(-2.0 * log(u0));
        g[2 * p] = r * cos(2.0 * M_PI * u1);
        g[2 * p + 1] = r * sin(2.0 * M_PI * u1);
    }
}

/* The 16 standard normals of (seed, site, step) in domain 0, or the 4 of
 * domain 1. */
void orc_site_normals(uint64_t seed, uint64_t site, uint64_t step, int domain, double *g) {
    uint32_t words[16];
    int ncalls = domain == 0 ? 4 : 1;
    site_words(seed, site, step, domain, ncalls, words);
    box_muller(words, 2 * ncalls, g);
}

/* ---------------------------------------------------------------------- */
/* Lattice helpers                                                          */
/* ---------------------------------------------------------------------- */
static inline int64_t wrap(int64_t v, int S) {
    v %= S;
    return v < 0 ? v + S : v;
}
static inline int64_t site_of(int S, int64_t x, int64_t y, int64_t z) {
    return wrap(x, S) + (int64_t)S * (wrap(y, S) + (int64_t)S * wrap(z, S));
}

/* Isotropic D3Q19 difference operators (a reading; the paper defers its
 * discrete derivatives to its reference on the fluctuating model):
 *   grad psi(r) = (1/c_s^2) sum_i w_i c_i psi(r + c_i)
 *   lap  psi(r) = (2/c_s^2) sum_i w_i [psi(r + c_i) - psi(r)]            */
static void grad_at(int S, const double *psi, int x, int y, int z, double g[3]) {
    g[0] = g[1] = g[2] = 0.0;
    for (int i = 1; i < Q; ++i) {
        double v = psi[site_of(S, x + CV[i][0], y + CV[i][1], z + CV[i][2])];
        for (int d = 0; d < 3; ++d) g[d] += WQ[i] * CV[i][d] * v;
    }
    for (int d = 0; d < 3; ++d) g[d] /= CS2;
}
static double lap_at(int S, const double *psi, int x, int y, int z) {
    double c = psi[site_of(S, x, y, z)], acc = 0.0;
    for (int i = 1; i < Q; ++i)
        acc += WQ[i] * (psi[site_of(S, x + CV[i][0], y + CV[i][1], z + CV[i][2])] - c);
    return 2.0 * acc / CS2;
}

void orc_gradient(int S, const double *psi, double *g /* [3][N] */) {
    tables();
    int64_t N = (int64_t)S * S * S;
    for (int z = 0; z < S; ++z)
        for (int y = 0; y < S; ++y)
            for (int x = 0; x < S; ++x) {
                double v[3];
                grad_at(S, psi, x, y, z, v);
                int64_t s = site_of(S, x, y, z);
                for (int d = 0; d < 3; ++d) g[d * N + s] = v[d];
            }
}

void orc_laplacian(int S, const double *psi, double *out) {
    tables();
    for (int z = 0; z < S; ++z)
        for (int y = 0; y < S; ++y)
            for (int x = 0; x < S; ++x) out[site_of(S, x, y, z)] = lap_at(S, psi, x, y, z);
}

/* ---------------------------------------------------------------------- */
/* Hydrodynamic fields, Eq. (mom): rho = sum_i f_i, j = sum_i c_i f_i.      */
/* ---------------------------------------------------------------------- */
void orc_fields(int S, const double *f, double *rho, double *j /* [3][N] or NULL */) {
    tables();
    int64_t N = (int64_t)S * S * S;
    for (int64_t s = 0; s < N; ++s) {
        double r = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
        for (int i = 0; i < Q; ++i) {
            double v = f[i * N + s];
            r += v;
            jx += CV[i][0] * v;
            jy += CV[i][1] * v;
            jz += CV[i][2] * v;
        }
        if (rho) rho[s] = r;
        if (j) {
            j[s] = jx;
            j[N + s] = jy;
            j[2 * N + s] = jz;
        }
    }
}

/* Chemical potential of the Ginzburg-Landau free energy, Sec. II A,
 * Eqs. (fef), (landau-pot), as a function of the density:
 *   mu = a (rho - rho_c) + b (rho - rho_c)^3 - kappa lap(rho)             */
void orc_chem_potential(int S, const orc_params *p, const double *rho, double *mu) {
    tables();
    for (int z = 0; z < S; ++z)
        for (int y = 0; y < S; ++y)
            for (int x = 0; x < S; ++x) {
                int64_t s = site_of(S, x, y, z);
                double d = rho[s] - p->rho_c;
                mu[s] = p->a * d + p->b * d * d * d - p->kappa * lap_at(S, rho, x, y, z);
            }
}

/* Body force F = -rho grad(mu) + c_s^2 grad(rho). */
void orc_force(int S, const orc_params *p, const double *rho, const double *mu, double *F) {
    tables();
    int64_t N = (int64_t)S * S * S;
    for (int z = 0; z < S; ++z)
        for (int y = 0; y < S; ++y)
            for (int x = 0; x < S; ++x) {
                int64_t s = site_of(S, x, y, z);
                double gm[3], gr[3];
                grad_at(S, mu, x, y, z, gm);
                grad_at(S, rho, x, y, z, gr);
                for (int d = 0; d < 3; ++d)
                    F[d * N + s] = p->force_off ? 0.0 : -rho[s] * gm[d] + CS2 * gr[d];
            }
}

/* ---------------------------------------------------------------------- */
/* Collision of one site in moment space.                                  */
/*   m_a = sum_i e_a(c_i) f_i                                               */
/*   u = (j + F/2) / rho                                                    */
/*   conserved:   m*_0 = rho, m*_{1..3} = j + F                             */
/*   a >= 4:      m*_a = meq_a + gamma (m_a - meq_a) + (1 + gamma)/2 Psi_a   */
/*                       + sqrt(rho kT (1 - gamma^2) N_a / c_s^2) g_{a-4}    */
/*   gamma = 1 - 1/tau; (1/tau)(2 - 1/tau) = 1 - gamma^2 (Eq. (lbnoise))    */
/*   f*_i = w_i sum_a e_a(c_i) m*_a / N_a                                    */
/* meq and Psi are the moments of the second-order equilibrium and of Guo's */
/* forcing term; for this basis they vanish beyond the stresses.            */
/* Returns ORC_EUNSTABLE if rho <= 0 or a value is not finite.              */
/* ---------------------------------------------------------------------- */
int orc_collide_site(const orc_params *p, const double *f, const double *F, const double *g,
                     double *fout) {
    tables();
    double m[Q];
    for (int a = 0; a < Q; ++a) {
        double acc = 0.0;
        for (int i = 0; i < Q; ++i) acc += T[a][i] * f[i];
        m[a] = acc;
    }
    double rho = m[0];
    if (!(rho > 0.0) || !isfinite(rho)) return ORC_EUNSTABLE;
    double Fx = F[0], Fy = F[1], Fz = F[2];
    double ux = (m[1] + 0.5 * Fx) / rho, uy = (m[2] + 0.5 * Fy) / rho, uz = (m[3] + 0.5 * Fz) / rho;
    double u2 = ux * ux + uy * uy + uz * uz;
    double uF = ux * Fx + uy * Fy + uz * Fz;

    double meq[Q], psi[Q];
    for (int a = 0; a < Q; ++a) meq[a] = psi[a] = 0.0;
    meq[0] = rho;
    meq[1] = rho * ux;
    meq[2] = rho * uy;
    meq[3] = rho * uz;
    meq[4] = rho * u2;
    meq[5] = rho * (3.0 * ux * ux - u2);
    meq[6] = rho * (uy * uy - uz * uz);
    meq[7] = rho * ux * uy;
    meq[8] = rho * uy * uz;
    meq[9] = rho * uz * ux;
    psi[1] = Fx;
    psi[2] = Fy;
    psi[3] = Fz;
    psi[4] = 2.0 * uF;
    psi[5] = 2.0 * (3.0 * ux * Fx - uF);
    psi[6] = 2.0 * (uy * Fy - uz * Fz);
    psi[7] = ux * Fy + uy * Fx;
    psi[8] = uy * Fz + uz * Fy;
    psi[9] = uz * Fx + ux * Fz;

    double mpost[Q];
    mpost[0] = rho;
    mpost[1] = m[1] + Fx;
    mpost[2] = m[2] + Fy;
    mpost[3] = m[3] + Fz;
    for (int a = 4; a < Q; ++a) {
        double gam = 1.0 - 1.0 / tau_of(p, a);
        double sigma = sqrt(rho * p->kT * (1.0 - gam * gam) * NRM[a] / CS2);
        mpost[a] = meq[a] + gam * (m[a] - meq[a]) + 0.5 * (1.0 + gam) * psi[a] +
                   (g ? sigma * g[a - 4] : 0.0);
    }
    for (int i = 0; i < Q; ++i) {
        double acc = 0.0;
        for (int a = 0; a < Q; ++a) acc += T[a][i] * mpost[a] / NRM[a];
        fout[i] = WQ[i] * acc;
        if (!isfinite(fout[i])) return ORC_EUNSTABLE;
    }
    return ORC_OK;
}

/* ---------------------------------------------------------------------- */
/* Initial state: rho = rho_c + sigma0 g (first normal of domain 1 at step  */
/* 0), u = 0, f_i = w_i rho.                                                 */
/* ---------------------------------------------------------------------- */
void orc_init(int S, double rho_c, double sigma0, uint64_t seed, double *f) {
    tables();
    int64_t N = (int64_t)S * S * S;
    for (int64_t s = 0; s < N; ++s) {
        double g[4];
        orc_site_normals(seed, (uint64_t)s, 0, 1, g);
        double rho = rho_c + sigma0 * g[0];
        for (int i = 0; i < Q; ++i) f[i * N + s] = WQ[i] * rho;
    }
}

/* ---------------------------------------------------------------------- */
/* One full time step t -> t+1 (t is the step counter of the noise).        */
/*  1. rho, j from f(t)                                                      */
/*  2. mu, 3. F on the whole lattice                                         */
/*  4. collide every site, 5. stream: f_i(r + c_i, t+1) = f*_i(r)            */
/* nthreads > 1 splits the z planes of each pass over OpenMP threads.       */
/* ---------------------------------------------------------------------- */
int orc_step(int S, const orc_params *p, uint64_t seed, uint64_t t, const double *fin, double *fout,
             int nthreads) {
    tables();
    if (S < 1 || !(p->tau > 0.5) || (p->tau_bulk != 0.0 && !(p->tau_bulk > 0.5)) ||
        (p->tau_ghost != 0.0 && !(p->tau_ghost > 0.5)))
        return ORC_EINVAL;
    int64_t N = (int64_t)S * S * S;
    double *rho = (double *)malloc(sizeof(double) * N);
    double *mu = (double *)malloc(sizeof(double) * N);
    double *F = (double *)malloc(sizeof(double) * 3 * N);
    if (!rho || !mu || !F) {
        free(rho);
        free(mu);
        free(F);
        return ORC_EINVAL;
    }
    orc_fields(S, fin, rho, NULL);
    int status = ORC_OK;
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int z = 0; z < S; ++z)
        for (int y = 0; y < S; ++y)
            for (int x = 0; x < S; ++x) {
                int64_t s = site_of(S, x, y, z);
                double d = rho[s] - p->rho_c;
                mu[s] = p->a * d + p->b * d * d * d - p->kappa * lap_at(S, rho, x, y, z);
            }
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int z = 0; z < S; ++z)
        for (int y = 0; y < S; ++y)
            for (int x = 0; x < S; ++x) {
                int64_t s = site_of(S, x, y, z);
                double gm[3], gr[3];
                grad_at(S, mu, x, y, z, gm);
                grad_at(S, rho, x, y, z, gr);
                for (int d = 0; d < 3; ++d)
                    F[d * N + s] = p->force_off ? 0.0 : -rho[s] * gm[d] + CS2 * gr[d];
            }
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int z = 0; z < S; ++z)
        for (int y = 0; y < S; ++y)
            for (int x = 0; x < S; ++x) {
                int64_t s = site_of(S, x, y, z);
                double fl[Q], fpost[Q], Fl[3], g[16];
                for (int i = 0; i < Q; ++i) fl[i] = fin[i * N + s];
                for (int d = 0; d < 3; ++d) Fl[d] = F[d * N + s];
                orc_site_normals(seed, (uint64_t)s, t, 0, g);
                int rc = orc_collide_site(p, fl, Fl, g, fpost);
                if (rc != ORC_OK) {
#pragma omp atomic write
                    status = rc;
                }
                for (int i = 0; i < Q; ++i)
                    fout[i * N + site_of(S, x + CV[i][0], y + CV[i][1], z + CV[i][2])] = fpost[i];
            }
    free(rho);
    free(mu);
    free(F);
    return status;
}

/* Number of threads an OpenMP region of the oracle would use by default. */
int orc_max_threads(void) {
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
