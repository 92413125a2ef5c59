// The paper's own model on the D3Q19 lattice (Sec. III A): the Ginzburg-
// Landau thermodynamics carried by a modified equilibrium instead of a body
// force, BGK relaxation with one tau, and thermal noise whose covariance
// depends on the local sound speed.  A split step: the density pass of the
// force model, then one collide pass per site.
//
// Equilibrium (moments of f in the weight-orthogonal basis of the force
// model): rho, j, the second moment
//   Pi = P + rho u u + nu (u grad rho + grad rho u + (u . grad rho) I),
//   P  = p_iso I + kappa grad rho grad rho,  Eqs. (press-th), (holdych-cond),
//   p_iso = p0 - kappa rho lap rho - kappa/2 |grad rho|^2,
//   p0 = rho f0' - f0 of f0 = a d^2/2 + b d^4/4 (d = rho - rho_c),
// as m4 = tr Pi - rho, m5 = 3 Pi_xx - tr Pi, m6 = Pi_yy - Pi_zz, m7..m9 the
// off-diagonal Pi; zero third-order ghosts; m16 = rho - 3 p_iso (the
// pressure sits on the moving populations, the rest population takes the
// remainder of rho); m17 = m18 = 0.
//
// Noise: in units of 3 rho kT (1 - gamma^2), the basis norms N_a, except the
// coupled pair of the bulk moment 4 and the fourth-order ghost 16 with
// M_44 = 5/3 - 3 c^2, M_4,16 = 3 c^2 - 1, M_16,16 = 3 - 3 c^2 at the local
// c^2 = c_s^2 = rho (a + 3 b d^2), drawn through its Cholesky factor from the
// normals g0 and g12.  This is the noise that keeps the stationary population
// covariance the same at every wave vector (on D2Q9 the same construction
// gives the matrix of Eq. (lbnoise)); it exists for c_s^2 < 1/2.
#pragma once

#include "lbfss_step.hpp"

namespace lbfss {

// e_a(c_q) of the weight-orthogonal D3Q19 basis (as in the force model's
// collision): 1, c, c^2 - 1, 3c_x^2 - c^2, c_y^2 - c_z^2, c_x c_y, c_y c_z,
// c_z c_x, (3c^2 - 5) c, (c_y^2 - c_z^2) c_x, (c_z^2 - c_x^2) c_y,
// (c_x^2 - c_y^2) c_z, 3c^4 - 6c^2 + 1, (2c^2 - 3)(3c_x^2 - c^2),
// (2c^2 - 3)(c_y^2 - c_z^2).
__host__ __device__ constexpr int meq_basis(int a, int q) {
    const int x = cx_of(q), y = cy_of(q), z = cz_of(q);
    const int c2 = x * x + y * y + z * z;
    switch (a) {
    case 0: return 1;
    case 1: return x;
    case 2: return y;
    case 3: return z;
    case 4: return c2 - 1;
    case 5: return 3 * x * x - c2;
    case 6: return y * y - z * z;
    case 7: return x * y;
    case 8: return y * z;
    case 9: return z * x;
    case 10: return (3 * c2 - 5) * x;
    case 11: return (3 * c2 - 5) * y;
    case 12: return (3 * c2 - 5) * z;
    case 13: return (y * y - z * z) * x;
    case 14: return (z * z - x * x) * y;
    case 15: return (x * x - y * y) * z;
    case 16: return 3 * c2 * c2 - 6 * c2 + 1;
    case 17: return (2 * c2 - 3) * (3 * x * x - c2);
    default: return (2 * c2 - 3) * (y * y - z * z);
    }
}
// lattice weight in units of 1/36
__host__ __device__ constexpr int meq_w36(int q) { return q == 0 ? 12 : (q < 7 ? 2 : 1); }
// N_a = sum_q w_q e_a(c_q)^2, in units of 1/36
__host__ __device__ constexpr int meq_norm36(int a) {
    int s = 0;
    for (int q = 0; q < Q; ++q) s += meq_w36(q) * meq_basis(a, q) * meq_basis(a, q);
    return s;
}

// Both transforms as compile-time tables, so that the unrolled loops are
// plain constant-coefficient multiply-adds: the forward weights 36 w_q e_a(c_q)
// (integers) and the back-transform coefficients e_a(c_q) / N_a.
struct MeqTables {
    int fwd[Q][Q];     // [a][q]
    float back[Q][Q];  // [q][a]
};
__host__ __device__ constexpr MeqTables meq_tables() {
    MeqTables t{};
    for (int a = 0; a < Q; ++a)
        for (int q = 0; q < Q; ++q) {
            const int e = meq_basis(a, q);
            t.fwd[a][q] = meq_w36(q) * e;
            t.back[q][a] = e == 0 ? 0.0f : (float)e * (36.0f / (float)meq_norm36(a));
        }
    return t;
}

template <typename T, bool SNAP>
__global__ void __launch_bounds__(kBlock)
k_meq_collide(const RepDesc *__restrict__ desc, int nrep, int64_t total, const T *__restrict__ pop,
              T *__restrict__ pop_out, const float *__restrict__ drho, const uint64_t *__restrict__ step, int koff,
              int *__restrict__ err, float *__restrict__ snap) {
    const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (g >= total) return;
    const int r = find_rep(desc, nrep, g);
    const RepDesc &d = desc[r];
    const int64_t s = g - d.site_off;
    const Nbr n(s, d.L);
    float f[Q];
    pull(pop + Q * d.site_off, d.N, n, f);
    if constexpr (SNAP) write_snapshot(snap, total, g, f);

    // moments of the stored deviations r_q = f_q / w_q - rho_c: for a >= 1
    // they are the moments of f; m[0] is rho - rho_c.  Integer weights
    // (36 w_q e_a) and one correctly rounded division: the deviations of this
    // model are O(1) (its rest state keeps the mass on the rest population),
    // and FP32-rounded weights would bias the density of every site the same
    // way each step
    constexpr MeqTables tab = meq_tables();
    float m[Q];
#pragma unroll
    for (int a = 0; a < Q; ++a) {
        float acc = 0.0f;
#pragma unroll
        for (int q = 0; q < Q; ++q)
            if (tab.fwd[a][q] != 0) acc += (float)tab.fwd[a][q] * f[q];
        m[a] = acc / 36.0f;
    }
    const float dr = m[0];
    const float rho = d.rho_c + dr;
    const float jx = m[1], jy = m[2], jz = m[3];

    // derivatives of rho from the density pass (isotropic D3Q19 stencils)
    const float *drp = drho + d.site_off;
    const NbrAt R{drp, n};
    const Grad18 gr = grad18(R);
    const float lap = lap18(drp[s], R);
    const float gx = gr.gx, gy = gr.gy, gz = gr.gz;

    // thermodynamics and the second moment of the equilibrium
    const float inv_rho = 1.0f / rho;
    const float ux = jx * inv_rho, uy = jy * inv_rho, uz = jz * inv_rho;
    const float dd = dr;
    const float f0 = 0.5f * d.a * dd * dd + 0.25f * d.b * dd * dd * dd * dd;
    const float p0 = rho * (d.a * dd + d.b * dd * dd * dd) - f0;
    const float cs2 = rho * (d.a + 3.0f * d.b * dd * dd);
    const float tau = 1.0f / (1.0f - d.gamma);
    const float nu = (tau - 0.5f) * (1.0f / 3.0f);
    const float g2 = gx * gx + gy * gy + gz * gz;
    const float p_iso = p0 - d.kappa * rho * lap - 0.5f * d.kappa * g2;
    const float ug = ux * gx + uy * gy + uz * gz;
    const float iso = p_iso + nu * ug;
    const float Pxx = iso + d.kappa * gx * gx + rho * ux * ux + nu * (2.0f * ux * gx);
    const float Pyy = iso + d.kappa * gy * gy + rho * uy * uy + nu * (2.0f * uy * gy);
    const float Pzz = iso + d.kappa * gz * gz + rho * uz * uz + nu * (2.0f * uz * gz);
    const float Pxy = d.kappa * gx * gy + rho * ux * uy + nu * (ux * gy + gx * uy);
    const float Pyz = d.kappa * gy * gz + rho * uy * uz + nu * (uy * gz + gy * uz);
    const float Pzx = d.kappa * gz * gx + rho * uz * ux + nu * (uz * gx + gz * ux);
    const float tr = Pxx + Pyy + Pzz;
    float meq[Q];
#pragma unroll
    for (int a = 0; a < Q; ++a) meq[a] = 0.0f;
    meq[4] = tr - rho;
    meq[5] = 3.0f * Pxx - tr;
    meq[6] = Pyy - Pzz;
    meq[7] = Pxy;
    meq[8] = Pyz;
    meq[9] = Pzx;
    meq[16] = rho - 3.0f * p_iso;

    // BGK on the non-conserved moments, Eq. (lbe)
    const float gam = d.gamma, og = 1.0f - d.gamma;
#pragma unroll
    for (int a = 4; a < Q; ++a) m[a] = gam * m[a] + og * meq[a];

    bool bad = !(rho > 0.0f && rho < 1e30f);  // Sec. III B: rho must stay positive
    if (d.noise_amp > 0.0f) {
        // the pair (4, 16) has a covariance only for c_s^2 < 1/2
        bad |= !(cs2 < 0.5f);
        const float sig = d.noise_amp * __builtin_amdgcn_sqrtf(fmaxf(rho, 0.0f));
        const float L44 = __builtin_amdgcn_sqrtf(fmaxf(5.0f / 3.0f - 3.0f * cs2, 0.0f));
        const float L164 = (3.0f * cs2 - 1.0f) / L44;
        const float L1616 = __builtin_amdgcn_sqrtf(fmaxf(3.0f - 3.0f * cs2 - L164 * L164, 0.0f));
        const uint64_t t = *step + (uint64_t)koff;
        const SiteNoise noise{(uint32_t)s, (uint32_t)t, (uint32_t)(t >> 32), d.key0, d.key1};
        float gn[16];
#pragma unroll
        for (int call = 0; call < 4; ++call) {
            float v[4];
            noise(call, v);
#pragma unroll
            for (int k = 0; k < 4; ++k) gn[4 * call + k] = v[k];
        }
#pragma unroll
        for (int a = 5; a < Q; ++a) {
            if (a == 16) continue;
            constexpr float inv6 = 1.0f / 6.0f;  // sqrt(N_a) = sqrt(norm36) / 6
            m[a] += sig * (__builtin_sqrtf((float)meq_norm36(a)) * inv6) * gn[a - 4];
        }
        m[4] += sig * L44 * gn[0];
        m[16] += sig * (L164 * gn[0] + L1616 * gn[12]);
    }
    if (bad) *err = 1;

    // back-transform: r*_q = sum_a e_a(c_q) m*_a / N_a  (m*_0 = rho - rho_c)
    T *out = pop_out + Q * d.site_off;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        float v = m[0];
#pragma unroll
        for (int a = 1; a < Q; ++a)
            if (tab.back[q][a] != 0.0f) v += tab.back[q][a] * m[a];
        Store<T>::st(out + (int64_t)q * d.N, s, v);
    }
}

}  // namespace lbfss
