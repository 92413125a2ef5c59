// Step kernels of the split plan (density pass, chemical-potential pass,
// collide pass), the initial state, and field import/export.
//
// Every kernel works on the handle's flattened site index g (all replicas
// back to back); the replica of g is found by binary search over site_off.
#pragma once

#include "lbfss_device.hpp"

namespace lbfss {

constexpr int kBlock = 256;

__device__ __forceinline__ int find_rep(const RepDesc *__restrict__ desc, int nrep, int64_t g) {
    int lo = 0, hi = nrep - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (desc[mid].site_off <= g) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Neighbour coordinates of a site with periodic wrap.
struct Nbr {
    int x, y, z, xm, xp;
    int Y0, Ym, Yp;  // y * L etc.
    int Z0, Zm, Zp;  // z * L * L etc.
    __device__ __forceinline__ Nbr(int64_t s, int L) {
        const int LL = L * L;
        z = (int)(s / LL);
        const int rem = (int)(s - (int64_t)z * LL);
        y = rem / L;
        x = rem - y * L;
        xm = wrap_dec(x, L);
        xp = wrap_inc(x, L);
        Y0 = y * L;
        Ym = wrap_dec(y, L) * L;
        Yp = wrap_inc(y, L) * L;
        Z0 = z * LL;
        Zm = wrap_dec(z, L) * LL;
        Zp = wrap_inc(z, L) * LL;
    }
    __device__ __forceinline__ Nbr(int x_, int y_, int z_, int L) : x(x_), y(y_), z(z_) {
        const int LL = L * L;
        xm = wrap_dec(x, L);
        xp = wrap_inc(x, L);
        Y0 = y * L;
        Ym = wrap_dec(y, L) * L;
        Yp = wrap_inc(y, L) * L;
        Z0 = z * LL;
        Zm = wrap_dec(z, L) * LL;
        Zp = wrap_inc(z, L) * LL;
    }
};

// Pull: r_q(x, t) = buf_q(x - c_q).
template <typename T>
__device__ __forceinline__ void pull(const T *__restrict__ base, int64_t N, const Nbr &n, float (&r)[Q]) {
    using S = Store<T>;
    r[0] = S::ld(base, n.x + n.Y0 + n.Z0);
    r[1] = S::ld(base + 1 * N, n.xm + n.Y0 + n.Z0);
    r[2] = S::ld(base + 2 * N, n.xp + n.Y0 + n.Z0);
    r[3] = S::ld(base + 3 * N, n.x + n.Ym + n.Z0);
    r[4] = S::ld(base + 4 * N, n.x + n.Yp + n.Z0);
    r[5] = S::ld(base + 5 * N, n.x + n.Y0 + n.Zm);
    r[6] = S::ld(base + 6 * N, n.x + n.Y0 + n.Zp);
    r[7] = S::ld(base + 7 * N, n.xm + n.Ym + n.Z0);
    r[8] = S::ld(base + 8 * N, n.xp + n.Yp + n.Z0);
    r[9] = S::ld(base + 9 * N, n.xm + n.Yp + n.Z0);
    r[10] = S::ld(base + 10 * N, n.xp + n.Ym + n.Z0);
    r[11] = S::ld(base + 11 * N, n.xm + n.Y0 + n.Zm);
    r[12] = S::ld(base + 12 * N, n.xp + n.Y0 + n.Zp);
    r[13] = S::ld(base + 13 * N, n.xm + n.Y0 + n.Zp);
    r[14] = S::ld(base + 14 * N, n.xp + n.Y0 + n.Zm);
    r[15] = S::ld(base + 15 * N, n.x + n.Ym + n.Zm);
    r[16] = S::ld(base + 16 * N, n.x + n.Yp + n.Zp);
    r[17] = S::ld(base + 17 * N, n.x + n.Ym + n.Zp);
    r[18] = S::ld(base + 18 * N, n.x + n.Yp + n.Zm);
}

// Isotropic gradient (1/c_s^2) sum_i w_i c_i psi(x + c_i) of a scalar, from
// its 18 neighbours; at(dx, dy, dz) returns psi at that offset.  Every
// kernel uses this one function, so all plans round identically.
struct Grad18 {
    float gx, gy, gz;
};

template <typename F>
__device__ __forceinline__ Grad18 grad18(F &&at) {
    const float pxp = at(1, 0, 0), pxm = at(-1, 0, 0);
    const float pyp = at(0, 1, 0), pym = at(0, -1, 0);
    const float pzp = at(0, 0, 1), pzm = at(0, 0, -1);
    const float ppo = at(1, 1, 0), mmo = at(-1, -1, 0);
    const float pmo = at(1, -1, 0), mpo = at(-1, 1, 0);
    const float pop = at(1, 0, 1), mom = at(-1, 0, -1);
    const float pom = at(1, 0, -1), mop = at(-1, 0, 1);
    const float opp = at(0, 1, 1), omm = at(0, -1, -1);
    const float opm = at(0, 1, -1), omp = at(0, -1, 1);
    Grad18 g;
    g.gx = (1.0f / 6.0f) * (pxp - pxm) + (1.0f / 12.0f) * ((ppo - mmo) + (pmo - mpo) + (pop - mom) + (pom - mop));
    g.gy = (1.0f / 6.0f) * (pyp - pym) + (1.0f / 12.0f) * ((ppo - mmo) + (mpo - pmo) + (opp - omm) + (opm - omp));
    g.gz = (1.0f / 6.0f) * (pzp - pzm) + (1.0f / 12.0f) * ((pop - mom) + (mop - pom) + (opp - omm) + (omp - opm));
    return g;
}

// Isotropic Laplacian (2/c_s^2) sum_i w_i [psi(x + c_i) - psi(x)].
template <typename F>
__device__ __forceinline__ float lap18(float centre, F &&at) {
    const float ax = at(1, 0, 0) + at(-1, 0, 0) + at(0, 1, 0) + at(0, -1, 0) + at(0, 0, 1) + at(0, 0, -1);
    const float dg = at(1, 1, 0) + at(-1, -1, 0) + at(1, -1, 0) + at(-1, 1, 0) + at(1, 0, 1) + at(-1, 0, -1) +
                     at(1, 0, -1) + at(-1, 0, 1) + at(0, 1, 1) + at(0, -1, -1) + at(0, 1, -1) + at(0, -1, 1);
    return (1.0f / 3.0f) * ax + (1.0f / 6.0f) * dg - 4.0f * centre;
}

// Chemical potential mu = a drho + b drho^3 - kappa lap(drho).
__device__ __forceinline__ float chem_potential(const RepDesc &d, float c, float lap) {
    return d.a * c + d.b * (c * c * c) - d.kappa * lap;
}

// Offset accessor on a flattened periodic lattice.
struct NbrAt {
    const float *p;
    const Nbr &n;
    __device__ __forceinline__ float operator()(int dx, int dy, int dz) const {
        const int x = dx > 0 ? n.xp : (dx < 0 ? n.xm : n.x);
        const int Y = dy > 0 ? n.Yp : (dy < 0 ? n.Ym : n.Y0);
        const int Z = dz > 0 ? n.Zp : (dz < 0 ? n.Zm : n.Z0);
        return p[x + Y + Z];
    }
};

// ---------------------------------------------------------------------------
// Initial state, domain 1 of the noise: drho = sigma0 g, g the first normal
// of Philox(site, 0, 1 << 16, 0).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock)
k_init_density(const RepDesc *__restrict__ desc, const float *__restrict__ sigma0, int nrep,
               int64_t total, float *__restrict__ drho) {
    const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (g >= total) return;
    const int r = find_rep(desc, nrep, g);
    const RepDesc &d = desc[r];
    const uint32_t s = (uint32_t)(g - d.site_off);
    const Words4 w = philox4x32_10(s, 0u, 1u << 16, 0u, d.key0, d.key1);
    drho[g] = sigma0[r] * (bm_radius(uniform01(w.v[0])) * cos_rev(uniform01(w.v[1])));
}

// f_i = w_i rho, u = 0: post-streaming r_i(x) = drho(x), stored pre-pull as
// buf_i(y) = drho(y + c_i).
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_init_populations(const RepDesc *__restrict__ desc, int nrep, int64_t total,
                   const float *__restrict__ drho, T *__restrict__ pop) {
    const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (g >= total) return;
    const int r = find_rep(desc, nrep, g);
    const RepDesc &d = desc[r];
    const int64_t s = g - d.site_off;
    const Nbr n(s, d.L);
    const float *dr = drho + d.site_off;
    T *base = pop + Q * d.site_off;
    const int N = (int)d.N;
    using S = Store<T>;
    // buf_q(y) = drho(y + c_q)
    S::st(base, s, dr[n.x + n.Y0 + n.Z0]);
    S::st(base + 1 * (int64_t)N, s, dr[n.xp + n.Y0 + n.Z0]);
    S::st(base + 2 * (int64_t)N, s, dr[n.xm + n.Y0 + n.Z0]);
    S::st(base + 3 * (int64_t)N, s, dr[n.x + n.Yp + n.Z0]);
    S::st(base + 4 * (int64_t)N, s, dr[n.x + n.Ym + n.Z0]);
    S::st(base + 5 * (int64_t)N, s, dr[n.x + n.Y0 + n.Zp]);
    S::st(base + 6 * (int64_t)N, s, dr[n.x + n.Y0 + n.Zm]);
    S::st(base + 7 * (int64_t)N, s, dr[n.xp + n.Yp + n.Z0]);
    S::st(base + 8 * (int64_t)N, s, dr[n.xm + n.Ym + n.Z0]);
    S::st(base + 9 * (int64_t)N, s, dr[n.xp + n.Ym + n.Z0]);
    S::st(base + 10 * (int64_t)N, s, dr[n.xm + n.Yp + n.Z0]);
    S::st(base + 11 * (int64_t)N, s, dr[n.xp + n.Y0 + n.Zp]);
    S::st(base + 12 * (int64_t)N, s, dr[n.xm + n.Y0 + n.Zm]);
    S::st(base + 13 * (int64_t)N, s, dr[n.xp + n.Y0 + n.Zm]);
    S::st(base + 14 * (int64_t)N, s, dr[n.xm + n.Y0 + n.Zp]);
    S::st(base + 15 * (int64_t)N, s, dr[n.x + n.Yp + n.Zp]);
    S::st(base + 16 * (int64_t)N, s, dr[n.x + n.Ym + n.Zm]);
    S::st(base + 17 * (int64_t)N, s, dr[n.x + n.Yp + n.Zm]);
    S::st(base + 18 * (int64_t)N, s, dr[n.x + n.Ym + n.Zp]);
}

// ---------------------------------------------------------------------------
// Split plan, pass 1: drho(x, t) of the pulled populations.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_density(const RepDesc *__restrict__ desc, int nrep, int64_t total, const T *__restrict__ pop,
          float *__restrict__ drho) {
    const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (g >= total) return;
    const int r = find_rep(desc, nrep, g);
    const RepDesc &d = desc[r];
    const Nbr n(g - d.site_off, d.L);
    float f[Q];
    pull(pop + Q * d.site_off, d.N, n, f);
    drho[g] = drho_of(f);
}

// Split plan, pass 2: mu = a drho + b drho^3 - kappa lap(drho).
__global__ void __launch_bounds__(kBlock)
k_chem_potential(const RepDesc *__restrict__ desc, int nrep, int64_t total,
                 const float *__restrict__ drho, float *__restrict__ mu) {
    const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (g >= total) return;
    const int r = find_rep(desc, nrep, g);
    const RepDesc &d = desc[r];
    const Nbr n(g - d.site_off, d.L);
    const float *dr = drho + d.site_off;
    const float c = dr[n.x + n.Y0 + n.Z0];
    mu[g] = chem_potential(d, c, lap18(c, NbrAt{dr, n}));
}

// Split plan, pass 3: force, collision, noise; the post-collision values are
// written in place of the site (pull streaming reads them next step).
// Sample snapshot written by a step kernel: density deviation and momentum
// of the pulled (pre-collision) populations of flattened site g, which are
// the state the previous step left (the functions k_snapshot uses, so both
// routes give the same bits).  Layout [4][total]: drho, jx, jy, jz.
__device__ __forceinline__ void write_snapshot(float *__restrict__ snap, int64_t total, int64_t g,
                                               const float (&r)[Q]) {
    float jx, jy, jz;
    momentum_of(r, jx, jy, jz);
    snap[g] = drho_of(r);
    snap[total + g] = jx;
    snap[2 * total + g] = jy;
    snap[3 * total + g] = jz;
}

template <typename T, bool SNAP>
__global__ void __launch_bounds__(kBlock)
k_collide(const RepDesc *__restrict__ desc, int nrep, int64_t total, const T *__restrict__ pop,
          T *__restrict__ pop_out, const float *__restrict__ drho, const float *__restrict__ mu,
          const uint64_t *__restrict__ step, int koff, int *__restrict__ err, float *__restrict__ snap) {
    const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (g >= total) return;
    const int r = find_rep(desc, nrep, g);
    const RepDesc &d = desc[r];
    const int64_t s = g - d.site_off;
    const Nbr n(s, d.L);
    const float *dr = drho + d.site_off;
    const float *mr = mu + d.site_off;
    float Fx = 0.f, Fy = 0.f, Fz = 0.f;
    if (!(d.flags & 1)) {
        // F = -rho grad(mu) + c_s^2 grad(drho) = grad of psi(y) = drho(y)/3 - rho(x) mu(y)
        const float rho_x = d.rho_c + dr[s];
        const NbrAt R{dr, n}, M{mr, n};
        const Grad18 gr = grad18([&](int dx, int dy, int dz) {
            return (1.0f / 3.0f) * R(dx, dy, dz) - rho_x * M(dx, dy, dz);
        });
        Fx = gr.gx;
        Fy = gr.gy;
        Fz = gr.gz;
    }
    float f[Q];
    pull(pop + Q * d.site_off, d.N, n, f);
    if constexpr (SNAP) write_snapshot(snap, total, g, f);
    const uint64_t t = *step + (uint64_t)koff;
    const SiteNoise noise{(uint32_t)s, (uint32_t)t, (uint32_t)(t >> 32), d.key0, d.key1};
    const float rho = collide_site(d, f, Fx, Fy, Fz, noise);
    if (!(rho > 0.0f && rho < 1e30f)) *err = 1;  // Sec. III B: rho must stay positive
    T *out = pop_out + Q * d.site_off;
#pragma unroll
    for (int q = 0; q < Q; ++q) Store<T>::st(out + q * d.N, s, f[q]);
}

// ---------------------------------------------------------------------------
// Fields out: rho, j and f of the pulled populations, in FP64.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_export(const RepDesc d, const T *__restrict__ pop, double *__restrict__ rho,
         double *__restrict__ j, double *__restrict__ f) {
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s >= d.N) return;
    const Nbr n(s, d.L);
    float r[Q];
    pull(pop, d.N, n, r);
    double acc = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const double w = q == 0 ? 1.0 / 3.0 : (q < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
        const double fq = w * ((double)d.rho_c + (double)r[q]);
        if (f) f[q * d.N + s] = fq;
        acc += fq;
        jx += cx_of(q) * fq;
        jy += cy_of(q) * fq;
        jz += cz_of(q) * fq;
    }
    if (rho) rho[s] = acc;
    if (j) {
        j[s] = jx;
        j[d.N + s] = jy;
        j[2 * d.N + s] = jz;
    }
}

// Fields in: post-streaming f (FP64) to the pre-pull storage,
// buf_q(y) = (f_q(y + c_q) - w_q rho_c) / w_q.
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_import(const RepDesc d, const double *__restrict__ f, T *__restrict__ pop) {
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s >= d.N) return;
    const Nbr n(s, d.L);
    const int L = d.L;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int x = (n.x + cx_of(q) + L) % L;
        const int y = (n.y + cy_of(q) + L) % L;
        const int z = (n.z + cz_of(q) + L) % L;
        const int64_t src = x + (int64_t)L * (y + (int64_t)L * z);
        const double w = q == 0 ? 1.0 / 3.0 : (q < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
        Store<T>::st(pop + q * d.N, s, (float)((f[q * d.N + src] - w * (double)d.rho_c) / w));
    }
}

__global__ void k_add_step(uint64_t *step, int64_t n) { *step += (uint64_t)n; }

// The generator of the noise on caller-given counters: per counter the four
// Philox4x32-10 words, their uniforms, and the Box-Muller normals of the word
// pairs (0, 1) and (2, 3) (radius from the even word, angle from the odd one),
// through the same device functions as the step kernels.
constexpr int64_t kPhiloxMax = int64_t(1) << 24;
__global__ void __launch_bounds__(kBlock)
k_philox_probe(int64_t n, const uint32_t *__restrict__ ctr, const uint32_t *__restrict__ key,
               uint32_t *__restrict__ words, float *__restrict__ uni, float *__restrict__ nrm) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const Words4 w = philox4x32_10(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3], key[2 * i],
                                   key[2 * i + 1]);
    float u[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        words[4 * i + k] = w.v[k];
        u[k] = uniform01(w.v[k]);
        uni[4 * i + k] = u[k];
    }
    const float r0 = bm_radius(u[0]), r1 = bm_radius(u[2]);
    nrm[4 * i] = r0 * cos_rev(u[1]);
    nrm[4 * i + 1] = r0 * sin_rev(u[1]);
    nrm[4 * i + 2] = r1 * cos_rev(u[3]);
    nrm[4 * i + 3] = r1 * sin_rev(u[3]);
}

}  // namespace lbfss
