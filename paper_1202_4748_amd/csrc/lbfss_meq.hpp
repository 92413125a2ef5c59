// The paper's own model on the D3Q19 lattice (Sec. III A): the Ginzburg-
// Landau thermodynamics carried by a modified equilibrium instead of a body
// force, BGK relaxation with one tau, and thermal noise whose covariance
// depends on the local sound speed.  Two plans with the same arithmetic:
// the split plan (the density pass of the force model, then k_meq_collide)
// and the rows plan (k_meq_staged, one z-marching pass per tile).
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

#include "lbfss_fused.hpp"

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
// plain constant-coefficient multiply-adds.  The velocities come in opposite
// pairs (q, q + 1) for odd q, and every basis vector is even or odd under
// c -> -c (odd: the momentum a = 1..3 and the third-order ghosts a = 10..15),
// so the forward transform works on the nine pair sums (even moments) or
// differences (odd moments), and the back-transform forms one even and one
// odd part per pair: r*_q = E + O, r*_(q+1) = E - O.  The forward weights are
// the integers 36 w_q e_a(c_q); the back-transform coefficients e_a(c_q) / N_a.
__host__ __device__ constexpr bool meq_odd(int a) { return (a >= 1 && a <= 3) || (a >= 10 && a <= 15); }
struct MeqTables {
    int fwd0[Q];      // 36 w_0 e_a(0), the rest population (0 for odd a)
    int fwd[Q][9];    // [a][k]: 36 w_q e_a(c_q), q = 2k + 1
    float back0[Q];   // e_a(0) / N_a
    float back[9][Q]; // [k][a]: e_a(c_q) / N_a, q = 2k + 1
};
__host__ __device__ constexpr MeqTables meq_tables() {
    MeqTables t{};
    for (int a = 0; a < Q; ++a) {
        const int e0 = meq_basis(a, 0);
        t.fwd0[a] = meq_w36(0) * e0;
        t.back0[a] = e0 == 0 ? 0.0f : (float)e0 * (36.0f / (float)meq_norm36(a));
        for (int k = 0; k < 9; ++k) {
            const int e = meq_basis(a, 2 * k + 1);
            t.fwd[a][k] = meq_w36(2 * k + 1) * e;
            t.back[k][a] = e == 0 ? 0.0f : (float)e * (36.0f / (float)meq_norm36(a));
        }
    }
    return t;
}
// the pairing and the parities the tables rely on
__host__ __device__ constexpr bool meq_pairs_ok() {
    for (int k = 0; k < 9; ++k) {
        const int q = 2 * k + 1, p = q + 1;
        if (cx_of(p) != -cx_of(q) || cy_of(p) != -cy_of(q) || cz_of(p) != -cz_of(q)) return false;
        if (meq_w36(p) != meq_w36(q)) return false;
        for (int a = 0; a < Q; ++a)
            if (meq_basis(a, p) != (meq_odd(a) ? -1 : 1) * meq_basis(a, q)) return false;
    }
    for (int a = 0; a < Q; ++a)
        if (meq_odd(a) && meq_basis(a, 0) != 0) return false;
    return true;
}
static_assert(meq_pairs_ok(), "opposite velocity pairs and basis parities");

// nu = (tau - 1/2) / 3 of the Galilean correction, Eq. (holdych-cond)
__device__ __forceinline__ float meq_nu(const RepDesc &d) {
    const float tau = 1.0f / (1.0f - d.gamma);
    return (tau - 0.5f) * (1.0f / 3.0f);
}

// The collision of one site.  f holds its 19 pulled values (the stored
// deviations r_q = f_q / w_q - rho_c) and receives the post-collision ones;
// at(dx, dy, dz) is the density deviation of the density pass at a
// neighbour, centre its value at the site; s is the site index in its
// lattice and t the step (the noise counter).  Returns false where rho or
// the sound speed leaves its domain.  Both plans call this, so they round
// alike.
template <typename F>
__device__ __forceinline__ bool meq_collide_site(const RepDesc &d, float (&f)[Q], float centre, F &&at, uint32_t s,
                                                 uint64_t t, float nu) {
    // moments of the stored deviations: for a >= 1 they are the moments of
    // f; m[0] is rho - rho_c.  Integer weights (36 w_q e_a), and for the
    // conserved moments (rho, j) one correctly rounded division: the
    // deviations of this model are O(1) (its rest state keeps the mass on
    // the rest population), and FP32-rounded weights would bias the mass and
    // momentum of every site the same way each step.  The non-conserved
    // moments are relaxed and noised; a product with 1/36 serves them.
    constexpr MeqTables tab = meq_tables();
    float ps[9], pd[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        ps[k] = f[2 * k + 1] + f[2 * k + 2];
        pd[k] = f[2 * k + 1] - f[2 * k + 2];
    }
    float m[Q];
#pragma unroll
    for (int a = 0; a < Q; ++a) {
        float acc = 0.0f;
        if (tab.fwd0[a] != 0) acc += (float)tab.fwd0[a] * f[0];
#pragma unroll
        for (int k = 0; k < 9; ++k)
            if (tab.fwd[a][k] != 0) acc += (float)tab.fwd[a][k] * (meq_odd(a) ? pd[k] : ps[k]);
        m[a] = a < 4 ? acc / 36.0f : acc * (1.0f / 36.0f);
    }
    const float dr = m[0];
    const float rho = d.rho_c + dr;
    const float jx = m[1], jy = m[2], jz = m[3];

    // derivatives of rho from the density pass (isotropic D3Q19 stencils)
    const Grad18 gr = grad18(at);
    const float lap = lap18(centre, at);
    const float gx = gr.gx, gy = gr.gy, gz = gr.gz;

    // thermodynamics and the second moment of the equilibrium
    const float inv_rho = __builtin_amdgcn_rcpf(rho);  // hardware reciprocal, 1 ulp (as the force model)
    const float ux = jx * inv_rho, uy = jy * inv_rho, uz = jz * inv_rho;
    const float dd = dr;
    const float f0 = 0.5f * d.a * dd * dd + 0.25f * d.b * dd * dd * dd * dd;
    const float p0 = rho * (d.a * dd + d.b * dd * dd * dd) - f0;
    const float cs2 = rho * (d.a + 3.0f * d.b * dd * dd);
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
        const float L164 = (3.0f * cs2 - 1.0f) * __builtin_amdgcn_rcpf(L44);  // scales normals only
        const float L1616 = __builtin_amdgcn_sqrtf(fmaxf(3.0f - 3.0f * cs2 - L164 * L164, 0.0f));
        const SiteNoise noise{s, (uint32_t)t, (uint32_t)(t >> 32), d.key0, d.key1};
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

    // back-transform: r*_q = sum_a e_a(c_q) m*_a / N_a  (m*_0 = rho - rho_c),
    // the rest population, then the even and odd parts of each pair
    {
        float v = m[0];
#pragma unroll
        for (int a = 1; a < Q; ++a)
            if (tab.back0[a] != 0.0f) v += tab.back0[a] * m[a];
        f[0] = v;
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        float ev = m[0], od = 0.0f;
#pragma unroll
        for (int a = 1; a < Q; ++a) {
            if (tab.back[k][a] == 0.0f) continue;
            if (meq_odd(a)) od += tab.back[k][a] * m[a];
            else ev += tab.back[k][a] * m[a];
        }
        f[2 * k + 1] = ev + od;
        f[2 * k + 2] = ev - od;
    }
    return !bad;
}

// Split plan, pass 2 (after k_density): one site per thread.
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
    const float *drp = drho + d.site_off;
    const uint64_t t = *step + (uint64_t)koff;
    if (!meq_collide_site(d, f, drp[s], NbrAt{drp, n}, (uint32_t)s, t, meq_nu(d))) *err = 1;
    T *out = pop_out + Q * d.site_off;
#pragma unroll
    for (int q = 0; q < Q; ++q) Store<T>::st(out + (int64_t)q * d.N, s, f[q]);
}

// Rows plan: one z-marching pass per tile, no density pass.  The density
// needs a halo of one site only (the equilibrium takes grad rho and lap rho,
// there is no chemical potential), so for each population the workgroup
// stages the unshifted source rectangle of TY + 2 rows and TX + 8 columns
// from x0 - 4 (16-byte global-to-LDS loads, aligned when L is a multiple of
// 4; populations dealt round-robin to the waves).  The value pulled by the
// site at extended column ex (ex = x - x0 + 1) and row ey is the rectangle
// entry at row ey, column ex + 3 - cx_q.  Iteration p computes the densities
// of plane p on the tile and its halo into a ring of three LDS planes,
// issues the loads of plane p + 1, and collides plane p - 1, whose pulled
// values waited one iteration in registers; two barriers per plane.  The
// densities are drho_of of the same values the density pass pulls and the
// collision is meq_collide_site, so the result equals the split plan's.
template <int TX, int TY, bool SNAP>
__global__ void __launch_bounds__(TX * TY)
k_meq_staged(const RepDesc *__restrict__ desc, const FusedTile *__restrict__ tiles, const float *__restrict__ pop,
             float *__restrict__ pop_out, const uint64_t *__restrict__ step, int koff, int *__restrict__ err,
             float *__restrict__ snap, int64_t total) {
    constexpr int NT = TX * TY, NW = NT / 64;
    constexpr int EX = TX + 2, EP = EX * (TY + 2);  // a density plane with its one-site halo
    constexpr int CH = 4;                           // floats per 16-byte load
    constexpr int RW = TX + 2 * CH, CW = RW / CH, NL = CW * (TY + 2), NM = (NL + 63) / 64;
    static_assert(NT % 64 == 0 && 2 * (TX + 2) + 2 * TY <= NT, "one halo site per thread");
    __shared__ float s_stage[Q][CH * NL];
    __shared__ float s_rho[3][EP];
    auto rslot = [](int p) { return (p + 6) % 3; };  // p >= -6

    const FusedTile tl = tiles[xcd_tile(blockIdx.x, gridDim.x)];
    const RepDesc &d = desc[tl.rep];
    const int L = d.L;
    const uint32_t N = (uint32_t)d.N, LL = (uint32_t)(L * L);
    const float *base = pop + Q * d.site_off;
    float *obase = pop_out + Q * d.site_off;
    const uint64_t t = *step + (uint64_t)koff;
    const float nu = meq_nu(d);

    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int ix = tid % TX, iy = tid / TX;
    const int nx = tl.nx, ny = tl.ny;
    const bool inner = ix < nx && iy < ny;
    const uint32_t site_c = (uint32_t)(tl.x0 + (inner ? ix : 0) + (tl.y0 + (inner ? iy : 0)) * L);
    const int r_in = (iy + 1) * EX + (ix + 1);

    // the density halo site of this thread: the rows above and below the
    // tile, then the columns left and right of it
    const int ew = nx + 2;
    const bool has_h = tid < 2 * ew + 2 * ny;
    int hx = 0, hy = 0;
    if (has_h) {
        const int h = tid - 2 * ew;
        if (tid < ew) {
            hx = tid;
        } else if (tid < 2 * ew) {
            hy = ny + 1;
            hx = tid - ew;
        } else {
            hy = 1 + (h >> 1);
            hx = (h & 1) ? nx + 1 : 0;
        }
    }
    const int r_h = hy * EX + hx;

    // does this wave store populations (then 19 stores may be younger than
    // the staged loads when it next waits for them)
    const bool wave_stores = __builtin_amdgcn_readfirstlane((int)(__ballot(inner) != 0)) != 0;

    // the chunks this lane copies, one per 64-lane slice m of the NL chunks of
    // a population: byte offsets of its column and of its row for the three
    // y shifts (cy = -1, 0, 1)
    uint32_t r_col[NM], r_row[NM][3];
    bool r_on[NM];
    {
        const int lane = tid & 63;
#pragma unroll
        for (int m = 0; m < NM; ++m) {
            const int j = m * 64 + lane;
            r_on[m] = j < NL;
            const int ey = j / CW, k = j - (j / CW) * CW;
            r_col[m] = (uint32_t)(((tl.x0 - CH + CH * k) % L + L) % L) * 4u;
#pragma unroll
            for (int c = 0; c < 3; ++c)
                r_row[m][c] = (uint32_t)(((tl.y0 - 1 + ey - (c - 1)) % L + L) % L) * (uint32_t)L * 4u;
        }
    }
    auto issue = [&](int p) __attribute__((always_inline)) {
        const int zc = wrap_near(p, L);
        const uint32_t Zc = (uint32_t)zc * LL, Zm = (uint32_t)wrap_dec(zc, L) * LL,
                       Zp = (uint32_t)wrap_inc(zc, L) * LL;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            if (q % NW != wave) continue;
            const int cz = cz_of(q);
            const char *bq = (const char *)(base + (size_t)q * N + (cz > 0 ? Zm : (cz < 0 ? Zp : Zc)));
#pragma unroll
            for (int m = 0; m < NM; ++m)
                if (r_on[m])
                    __builtin_amdgcn_global_load_lds((gptr_t)(bq + r_row[m][cy_of(q) + 1] + r_col[m]),
                                                     (lptr_t)&s_stage[q][m * 64 * CH], 16, 0, 0);
        }
    };

    bool bad = false;
    bool stored_last = false;  // did the previous iteration issue stores (wave-uniform)
    float A[Q], B[Q];
    auto body = [&](int p, float(&ld)[Q], float(&cl)[Q]) __attribute__((always_inline)) {
        // 1. the staged rows of plane p have landed (the stores of the last
        //    collision, if any, are the only younger memory operations)
        if (stored_last) __builtin_amdgcn_s_waitcnt(vmcnt_wait(Q));  // the Q stores may still run
        else __builtin_amdgcn_s_waitcnt(vmcnt_wait(0));
        __syncthreads();
        {
            float *rs = s_rho[rslot(p)];
            if (inner) {
#pragma unroll
                for (int q = 0; q < Q; ++q) ld[q] = s_stage[q][(iy + 1) * RW + ix + CH - cx_of(q)];
                rs[r_in] = drho_of(ld);
            }
            if (has_h) {
                float h[Q];
#pragma unroll
                for (int q = 0; q < Q; ++q) h[q] = s_stage[q][hy * RW + hx + CH - 1 - cx_of(q)];
                rs[r_h] = drho_of(h);
            }
        }
        __syncthreads();
        // 2. prefetch plane p + 1
        if (p + 1 <= tl.z0 + tl.nz) issue(p + 1);
        // 3. collision of plane z = p - 1 (densities of z - 1, z, z + 1 in the ring)
        stored_last = false;
        const int z = p - 1;
        if (z >= tl.z0) {
            stored_last = wave_stores;
            if (inner) {
                const float *r0 = s_rho[rslot(z - 1)], *r1 = s_rho[rslot(z)], *r2 = s_rho[rslot(p)];
                auto at = [&](int dx, int dy, int dz) {
                    const float *pl = dz < 0 ? r0 : (dz > 0 ? r2 : r1);
                    return pl[r_in + dy * EX + dx];
                };
                const uint32_t s = site_c + (uint32_t)z * LL;
                if constexpr (SNAP) write_snapshot(snap, total, d.site_off + (int64_t)s, cl);
                bad |= !meq_collide_site(d, cl, r1[r_in], at, s, t, nu);
                float *oz = obase + (uint32_t)z * LL;
#pragma unroll
                for (int q = 0; q < Q; ++q) stb(oz + (size_t)q * N, site_c * 4u, cl[q]);
            }
        }
    };

    const int p0 = tl.z0 - 1, pend = tl.z0 + tl.nz;
    issue(p0);
    for (int p = p0; p <= pend; p += 2) {
        body(p, A, B);
        if (p + 1 <= pend) body(p + 1, B, A);
    }
    if (bad) *err = 1;
}

// tiles of the rows plan of this model: 256 threads, or 512 (64 x 8,
// 32 x 16: fewer staged halo rows per site, two workgroups per CU)
inline bool meq_tile_ok(int tx, int ty) {
    return (tx == 64 && ty == 4) || (tx == 32 && ty == 8) || (tx == 16 && ty == 16) || (tx == 64 && ty == 8) ||
           (tx == 32 && ty == 16);
}

template <bool SNAP>
void launch_meq_staged_snap(const RepDesc *desc, const FusedTile *tiles, int n_tiles, const float *in, float *out,
                            const uint64_t *step, int koff, int *err, int tx, int ty, hipStream_t stream, float *snap,
                            int64_t total) {
    if (tx == 64 && ty == 4)
        hipLaunchKernelGGL((k_meq_staged<64, 4, SNAP>), dim3(n_tiles), dim3(256), 0, stream, desc, tiles, in, out,
                           step, koff, err, snap, total);
    else if (tx == 16 && ty == 16)
        hipLaunchKernelGGL((k_meq_staged<16, 16, SNAP>), dim3(n_tiles), dim3(256), 0, stream, desc, tiles, in, out,
                           step, koff, err, snap, total);
    else if (tx == 64 && ty == 8)
        hipLaunchKernelGGL((k_meq_staged<64, 8, SNAP>), dim3(n_tiles), dim3(512), 0, stream, desc, tiles, in, out,
                           step, koff, err, snap, total);
    else if (tx == 32 && ty == 16)
        hipLaunchKernelGGL((k_meq_staged<32, 16, SNAP>), dim3(n_tiles), dim3(512), 0, stream, desc, tiles, in, out,
                           step, koff, err, snap, total);
    else
        hipLaunchKernelGGL((k_meq_staged<32, 8, SNAP>), dim3(n_tiles), dim3(256), 0, stream, desc, tiles, in, out,
                           step, koff, err, snap, total);
}

// snap: where the step also writes the sample snapshot of its input state,
// or null
inline void launch_meq_staged(const RepDesc *desc, const FusedTile *tiles, int n_tiles, const float *in, float *out,
                              const uint64_t *step, int koff, int *err, int tx, int ty, hipStream_t stream,
                              float *snap, int64_t total) {
    if (snap) launch_meq_staged_snap<true>(desc, tiles, n_tiles, in, out, step, koff, err, tx, ty, stream, snap, total);
    else launch_meq_staged_snap<false>(desc, tiles, n_tiles, in, out, step, koff, err, tx, ty, stream, snap, total);
}

}  // namespace lbfss
