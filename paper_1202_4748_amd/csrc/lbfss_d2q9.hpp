// The paper's own model (Sec. III A): fluctuating non-ideal D2Q9 lattice
// Boltzmann with the Ginzburg-Landau thermodynamics in a modified equilibrium
// (the pressure tensor of Eq. (press-th) imposed on the equilibrium's second
// moment, Eq. (holdych-cond)), BGK relaxation (Eq. (lbe)) and noise with the
// local-sound-speed covariance of Eq. (lbnoise), drawn through its Cholesky
// factor.
//
// Layout: populations [9][L^2] (site = x + L y), stored as deviations from
// the rest state of density rho_c, whose equilibrium puts all mass at rest
// (p0(rho_c) = 0): d_0 = f_0 - rho_c, d_i = f_i otherwise.  Moments are
// taken in the weight-orthogonal basis 1, c_x, c_y, 3c^2 - 2, c_x^2 - c_y^2,
// c_x c_y, (3c^2 - 4) c_x, (3c^2 - 4) c_y, 9c^4 - 15c^2 + 2 and handled as
// deviations from the rest state's moments (rho_c, 0, 0, -2 rho_c, 0, 0, 0, 0,
// 2 rho_c).  Velocity order: 0 (0,0); 1 (1,0) 2 (-1,0) 3 (0,1) 4 (0,-1);
// 5 (1,1) 6 (-1,-1) 7 (1,-1) 8 (-1,1).
#pragma once

#include "lbfss_fused.hpp"

namespace lbfss {

constexpr int Q2 = 9;

struct D2Desc {
    int32_t L, pad;
    float a, b, kappa, rho_c;
    float gamma;      // 1 - 1/tau
    float nu;         // (tau - 1/2) / 3
    float noise_amp;  // sqrt(3 kT (1/tau)(2 - 1/tau)); the noise scale is sqrt(rho) times this
    uint32_t key0, key1;
};

__host__ __device__ constexpr int c2x(int i) { return i == 1 || i == 5 || i == 7 ? 1 : (i == 2 || i == 6 || i == 8 ? -1 : 0); }
__host__ __device__ constexpr int c2y(int i) { return i == 3 || i == 5 || i == 8 ? 1 : (i == 4 || i == 6 || i == 7 ? -1 : 0); }
__host__ __device__ constexpr float w2(int i) { return i == 0 ? 4.0f / 9.0f : (i < 5 ? 1.0f / 9.0f : 1.0f / 36.0f); }

// e_a(c_i) and the norms N_a = sum_i w_i e_a^2
__host__ __device__ constexpr float e2(int a, int i) {
    const int cx = c2x(i), cy = c2y(i), cc = cx * cx + cy * cy;
    return a == 0 ? 1.0f
         : a == 1 ? (float)cx
         : a == 2 ? (float)cy
         : a == 3 ? (float)(3 * cc - 2)
         : a == 4 ? (float)(cx * cx - cy * cy)
         : a == 5 ? (float)(cx * cy)
         : a == 6 ? (float)((3 * cc - 4) * cx)
         : a == 7 ? (float)((3 * cc - 4) * cy)
                  : (float)(9 * cc * cc - 15 * cc + 2);
}
__host__ __device__ constexpr float n2(int a) {
    return a == 0 ? 1.0f : a <= 2 ? 1.0f / 3.0f : a == 3 ? 4.0f : a == 4 ? 4.0f / 9.0f : a == 5 ? 1.0f / 9.0f
         : a <= 7 ? 2.0f / 3.0f : 16.0f;
}

__device__ __forceinline__ int wrap2(int v, int L) { return v < 0 ? v + L : (v >= L ? v - L : v); }

// Pulled deviations of site (x, y): d_i(r - c_i).  The three source columns
// x - c_x and the three source rows y - c_y are wrapped once; each pull is
// then a 32-bit in-plane offset from the population's (uniform) base.
__device__ __forceinline__ void pull2(const float *__restrict__ pop, int L, int x, int y, float (&d)[Q2]) {
    const uint32_t N = (uint32_t)L * (uint32_t)L;
    const uint32_t col[3] = {(uint32_t)wrap2(x + 1, L), (uint32_t)x, (uint32_t)wrap2(x - 1, L)};  // c_x = -1, 0, 1
    const uint32_t row[3] = {(uint32_t)wrap2(y + 1, L) * (uint32_t)L, (uint32_t)y * (uint32_t)L,
                             (uint32_t)wrap2(y - 1, L) * (uint32_t)L};  // c_y = -1, 0, 1
#pragma unroll
    for (int i = 0; i < Q2; ++i) d[i] = pop[(size_t)i * N + (col[c2x(i) + 1] + row[c2y(i) + 1])];
}

__device__ __forceinline__ float drho2(const float (&d)[Q2]) {
    return ((d[0] + (d[1] + d[2])) + (d[3] + d[4])) + ((d[5] + d[6]) + (d[7] + d[8]));
}

// Opposite velocities come in pairs (q, q + 1) for q = 1, 3, 5, 7, and each
// basis vector is even or odd under c -> -c (odd: a = 1, 2, 6, 7), so the
// transforms work on pair sums and differences (checked at compile time).
__host__ __device__ constexpr bool k2_odd(int a) { return a == 1 || a == 2 || a == 6 || a == 7; }
__host__ __device__ constexpr bool k2_pairs_ok() {
    for (int k = 0; k < 4; ++k) {
        const int q = 2 * k + 1, p = q + 1;
        if (c2x(p) != -c2x(q) || c2y(p) != -c2y(q) || w2(p) != w2(q)) return false;
        for (int a = 0; a < Q2; ++a)
            if (e2(a, p) != (k2_odd(a) ? -e2(a, q) : e2(a, q))) return false;
    }
    for (int a = 0; a < Q2; ++a)
        if (k2_odd(a) && e2(a, 0) != 0.0f) return false;
    return true;
}
static_assert(k2_pairs_ok(), "opposite velocity pairs and basis parities");

// The collision of one site: d holds its nine pulled deviations and
// receives the post-collision ones (stored unshifted: the next step pulls);
// at(dx, dy) is the density deviation of a neighbour (the same sum drho2 of
// its pulled values); s is the site index, t the step (the noise counter).
// Moments, equilibrium, relaxation, noise, back-transform.  Returns false
// where rho or the noise covariance leaves its domain.
template <typename F>
__device__ __forceinline__ bool k2_collide_site(const D2Desc &D, float (&d)[Q2], F &&at, uint32_t s, uint64_t t) {
    // moment deviations, from the rest value and the pair sums (even
    // moments) or differences (odd moments)
    float ps[4], pd[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        ps[k] = d[2 * k + 1] + d[2 * k + 2];
        pd[k] = d[2 * k + 1] - d[2 * k + 2];
    }
    float m[Q2];
#pragma unroll
    for (int a = 0; a < Q2; ++a) {
        float v = 0.0f;
        if (e2(a, 0) != 0.0f) v += e2(a, 0) * d[0];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (e2(a, 2 * k + 1) != 0.0f) v += e2(a, 2 * k + 1) * (k2_odd(a) ? pd[k] : ps[k]);
        m[a] = v;
    }
    const float dr = drho2(d);  // the same sum as the density array
    const float rho = D.rho_c + dr;
    // isotropic stencils on the densities of the neighbours
    float gx = 0.0f, gy = 0.0f, lap = 0.0f;
#pragma unroll
    for (int i = 1; i < Q2; ++i) {
        const float v = at(c2x(i), c2y(i));
        gx += 3.0f * w2(i) * (float)c2x(i) * v;
        gy += 3.0f * w2(i) * (float)c2y(i) * v;
        lap += 6.0f * w2(i) * (v - dr);
    }
    // thermodynamics of the Landau potential in d = rho - rho_c
    const float d2 = dr * dr;
    const float p0 = rho * (D.a * dr + D.b * d2 * dr) - (0.5f * D.a * d2 + 0.25f * D.b * d2 * d2);
    const float cs2 = rho * (D.a + 3.0f * D.b * d2);
    // equilibrium moments (deviations from the rest state)
    const float inv_rho = __builtin_amdgcn_rcpf(rho);  // hardware reciprocal, 1 ulp
    const float ux = m[1] * inv_rho, uy = m[2] * inv_rho;
    const float g2 = gx * gx + gy * gy, ug = ux * gx + uy * gy;
    const float S = p0 - D.kappa * rho * lap;
    const float iso = S - 0.5f * D.kappa * g2;
    const float Pxx = iso + D.kappa * gx * gx + rho * ux * ux + D.nu * (2.0f * ux * gx + ug);
    const float Pyy = iso + D.kappa * gy * gy + rho * uy * uy + D.nu * (2.0f * uy * gy + ug);
    const float Pxy = D.kappa * gx * gy + rho * ux * uy + D.nu * (ux * gy + uy * gx);
    float meq[Q2];
    meq[3] = 3.0f * (Pxx + Pyy) - 2.0f * dr;
    meq[4] = Pxx - Pyy;
    meq[5] = Pxy;
    meq[6] = 0.0f;
    meq[7] = 0.0f;
    meq[8] = 2.0f * dr - 6.0f * S - 3.0f * D.kappa * g2;
#pragma unroll
    for (int a = 3; a < Q2; ++a) m[a] = meq[a] + D.gamma * (m[a] - meq[a]);
    // noise, Eq. (lbnoise), through the Cholesky factor of its c_s^2 block
    bool bad = !(rho > 0.0f);
    if (D.noise_amp > 0.0f) {
        const float A = 4.0f * (2.0f - 3.0f * cs2), C = 12.0f * (cs2 - 1.0f / 3.0f),
                    B = 16.0f * (1.25f - 0.75f * cs2);
        // the factor scales normals only: hardware square roots and
        // reciprocal (1 ulp) serve it
        const float L33 = __builtin_amdgcn_sqrtf(A), L83 = C * __builtin_amdgcn_rcpf(L33), R = B - L83 * L83;
        bad |= !(A > 0.0f) || !(R > 0.0f);
        const float L88 = __builtin_amdgcn_sqrtf(R);
        const float sig = D.noise_amp * __builtin_amdgcn_sqrtf(rho);
        const Words4 w0 = philox4x32_10(s, (uint32_t)t, 0u, (uint32_t)(t >> 32), D.key0, D.key1);
        const Words4 w1 = philox4x32_10(s, (uint32_t)t, 1u, (uint32_t)(t >> 32), D.key0, D.key1);
        const float r0 = bm_radius(uniform01(w0.v[0])), a0 = uniform01(w0.v[1]);
        const float r1 = bm_radius(uniform01(w0.v[2])), a1 = uniform01(w0.v[3]);
        const float r2 = bm_radius(uniform01(w1.v[0])), a2 = uniform01(w1.v[1]);
        const float g0 = r0 * cos_rev(a0), g1 = r0 * sin_rev(a0);
        const float g2n = r1 * cos_rev(a1), g3 = r1 * sin_rev(a1);
        const float g4 = r2 * cos_rev(a2), g5 = r2 * sin_rev(a2);
        m[3] += sig * L33 * g0;
        m[4] += sig * (2.0f / 3.0f) * g1;
        m[5] += sig * (1.0f / 3.0f) * g2n;
        m[6] += sig * 0.816496580927726f * g3;  // sqrt(2/3)
        m[7] += sig * 0.816496580927726f * g4;
        m[8] += sig * (L83 * g0 + L88 * g5);
    }
    // back to populations: the rest one, then an even and an odd part per pair
    float mn[Q2];
#pragma unroll
    for (int a = 0; a < Q2; ++a) mn[a] = m[a] * (1.0f / n2(a));
    {
        float v = 0.0f;
#pragma unroll
        for (int a = 0; a < Q2; ++a)
            if (e2(a, 0) != 0.0f) v += e2(a, 0) * mn[a];
        d[0] = w2(0) * v;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int q = 2 * k + 1;
        float ev = 0.0f, od = 0.0f;
#pragma unroll
        for (int a = 0; a < Q2; ++a) {
            if (e2(a, q) == 0.0f) continue;
            if (k2_odd(a)) od += e2(a, q) * mn[a];
            else ev += e2(a, q) * mn[a];
        }
        d[q] = w2(q) * (ev + od);
        d[q + 1] = w2(q) * (ev - od);
    }
    return !bad;
}

// One step on a K2TX x K2TY tile per workgroup (tiles at the edges of the
// lattice are partial, so any L works): every site pulls its nine values,
// the densities of the tile and of a one-site halo (pulled by the first
// threads) go to LDS, and after one barrier each site collides with the
// stencils read there.  The densities are drho2 of the same pulled values
// wherever they are formed, so the result does not depend on the tiling.
// Tiles are numbered x fastest and dealt to the XCDs in contiguous runs
// (xcd_tile), so the halo pulls of a tile find its neighbours' rows in the
// same L2.  64 x 4 tiles: 3% faster than 32 x 8 at 2048^2, 16 x 16 12% slower.
// A batch of replicas (one L, own parameters and seeds) is one launch: the
// tiles of replica r follow those of replica r - 1, each replica's
// populations a [9][L^2] block after the previous one's.
// BATCH = false (one replica, the latency-bound small lattices): the
// descriptor comes with the launch, no replica arithmetic, no descriptor load.
constexpr int K2TX = 64, K2TY = 4;
template <bool BATCH>
__global__ void __launch_bounds__(K2TX * K2TY)
k2_step_tiled(D2Desc D0, const D2Desc *__restrict__ descs, int tiles_per_rep, const float *__restrict__ pop_all,
              float *__restrict__ pop_out_all, uint64_t t, int *__restrict__ err) {
    constexpr int EX = K2TX + 2;
    static_assert(2 * (K2TX + 2) + 2 * K2TY <= K2TX * K2TY, "one halo site per thread");
    __shared__ float s_rho[EX * (K2TY + 2)];
    const int gtile = xcd_tile(blockIdx.x, gridDim.x);
    const int rep = BATCH ? gtile / tiles_per_rep : 0, tile = gtile - rep * tiles_per_rep;
    const D2Desc D = BATCH ? descs[rep] : D0;
    const int L = D.L;
    const int64_t N = (int64_t)L * L;
    const float *pop = pop_all + (int64_t)rep * Q2 * N;
    float *pop_out = pop_out_all + (int64_t)rep * Q2 * N;
    const int ntx = (L + K2TX - 1) / K2TX;
    const int x0 = (tile % ntx) * K2TX, y0 = (tile / ntx) * K2TY;
    const int nx = min(K2TX, L - x0), ny = min(K2TY, L - y0);
    const int tid = threadIdx.x, ix = tid % K2TX, iy = tid / K2TX;
    const bool inner = ix < nx && iy < ny;
    const int r_in = (iy + 1) * EX + ix + 1;
    float d[Q2];
    if (inner) {
        pull2(pop, L, x0 + ix, y0 + iy, d);
        s_rho[r_in] = drho2(d);
    }
    // halo: the rows above and below the tile, then the columns beside it
    const int ew = nx + 2;
    if (tid < 2 * ew + 2 * ny) {
        int hx = 0, hy = 0;
        if (tid < ew) {
            hx = tid;
        } else if (tid < 2 * ew) {
            hy = ny + 1;
            hx = tid - ew;
        } else {
            const int h = tid - 2 * ew;
            hy = 1 + (h >> 1);
            hx = (h & 1) ? nx + 1 : 0;
        }
        float h[Q2];
        pull2(pop, L, wrap2(x0 - 1 + hx, L), wrap2(y0 - 1 + hy, L), h);
        s_rho[hy * EX + hx] = drho2(h);
    }
    __syncthreads();
    if (!inner) return;
    const uint32_t s = (uint32_t)(x0 + ix) + (uint32_t)L * (uint32_t)(y0 + iy);
    const bool ok = k2_collide_site(D, d, [&](int dx, int dy) { return s_rho[r_in + dy * EX + dx]; }, s, t);
#pragma unroll
    for (int i = 0; i < Q2; ++i) pop_out[i * N + s] = d[i];
    if (!ok) *err = 1;
}

// Initial state: rho = rho_c + sigma0 g (generator domain 1, call 0), u = 0,
// the equilibrium of that density (gradients of the density array).
__global__ void __launch_bounds__(kBlock)
k2_init_density(D2Desc D, float sigma0, float *__restrict__ drho) {
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s >= (int64_t)D.L * D.L) return;
    const Words4 w = philox4x32_10((uint32_t)s, 0u, 1u << 16, 0u, D.key0, D.key1);
    drho[s] = sigma0 * (bm_radius(uniform01(w.v[0])) * cos_rev(uniform01(w.v[1])));
}

__global__ void __launch_bounds__(kBlock)
k2_init_populations(D2Desc D, const float *__restrict__ drho, float *__restrict__ pop) {
    const int L = D.L;
    const int64_t N = (int64_t)L * L;
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s >= N) return;
    const int x = (int)(s % L), y = (int)(s / L);
    const float dr = drho[s], rho = D.rho_c + dr;
    float gx = 0.0f, gy = 0.0f, lap = 0.0f;
#pragma unroll
    for (int i = 1; i < Q2; ++i) {
        const float v = drho[wrap2(x + c2x(i), L) + (int64_t)L * wrap2(y + c2y(i), L)];
        gx += 3.0f * w2(i) * (float)c2x(i) * v;
        gy += 3.0f * w2(i) * (float)c2y(i) * v;
        lap += 6.0f * w2(i) * (v - dr);
    }
    const float d2 = dr * dr;
    const float p0 = rho * (D.a * dr + D.b * d2 * dr) - (0.5f * D.a * d2 + 0.25f * D.b * d2 * d2);
    const float g2 = gx * gx + gy * gy;
    const float S = p0 - D.kappa * rho * lap, iso = S - 0.5f * D.kappa * g2;
    float m[Q2] = {dr, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    const float Pxx = iso + D.kappa * gx * gx, Pyy = iso + D.kappa * gy * gy;
    m[3] = 3.0f * (Pxx + Pyy) - 2.0f * dr;
    m[4] = Pxx - Pyy;
    m[5] = D.kappa * gx * gy;
    m[8] = 2.0f * dr - 6.0f * S - 3.0f * D.kappa * g2;
    // the state is read by pulling, f_i(r) = buffer_i(r - c_i)
#pragma unroll
    for (int i = 0; i < Q2; ++i) {
        float v = 0.0f;
#pragma unroll
        for (int a = 0; a < Q2; ++a)
            if (e2(a, i) != 0.0f) v += e2(a, i) * (m[a] * (1.0f / n2(a)));
        pop[i * N + wrap2(x - c2x(i), L) + (int64_t)L * wrap2(y - c2y(i), L)] = w2(i) * v;
    }
}

// Export: rho, j and the populations f_i in FP64 of the state at step t
// (post-streaming: f_i(r) = buffer_i(r - c_i)).
__global__ void __launch_bounds__(kBlock)
k2_export(D2Desc D, const float *__restrict__ pop, double *__restrict__ rho, double *__restrict__ j,
          double *__restrict__ f) {
    const int L = D.L;
    const int64_t N = (int64_t)L * L;
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s >= N) return;
    const int x = (int)(s % L), y = (int)(s / L);
    double r = 0.0, jx = 0.0, jy = 0.0;
#pragma unroll
    for (int i = 0; i < Q2; ++i) {
        const int xs = wrap2(x - c2x(i), L), ys = wrap2(y - c2y(i), L);
        const double v = (double)pop[i * N + xs + (int64_t)L * ys] + (i == 0 ? (double)D.rho_c : 0.0);
        r += v;
        jx += c2x(i) * v;
        jy += c2y(i) * v;
        if (f) f[i * N + s] = v;
    }
    if (rho) rho[s] = r;
    if (j) {
        j[s] = jx;
        j[N + s] = jy;
    }
}

// Import: the state f_i(r) at step t into the buffer, buffer_i(r - c_i) = f_i(r).
__global__ void __launch_bounds__(kBlock)
k2_import(D2Desc D, const double *__restrict__ f, float *__restrict__ pop) {
    const int L = D.L;
    const int64_t N = (int64_t)L * L;
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s >= N) return;
    const int x = (int)(s % L), y = (int)(s / L);
#pragma unroll
    for (int i = 0; i < Q2; ++i) {
        const int xs = wrap2(x - c2x(i), L), ys = wrap2(y - c2y(i), L);
        pop[i * N + xs + (int64_t)L * ys] = (float)(f[i * N + s] - (i == 0 ? (double)D.rho_c : 0.0));
    }
}

// Sampling: density deviation and momentum of the state, FP64 [3][L^2].
// (The sampling kernels take replica blockIdx.y of a batch.)
__global__ void __launch_bounds__(kBlock)
k2_snap(int L, const float *__restrict__ pop_all, double *__restrict__ out_all) {
    const int64_t N = (int64_t)L * L;
    const float *pop = pop_all + (int64_t)blockIdx.y * Q2 * N;
    double *out = out_all + (int64_t)blockIdx.y * 3 * N;
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s >= N) return;
    const int x = (int)(s % L), y = (int)(s / L);
    double r = 0.0, jx = 0.0, jy = 0.0;
#pragma unroll
    for (int i = 0; i < Q2; ++i) {
        const int xs = wrap2(x - c2x(i), L), ys = wrap2(y - c2y(i), L);
        const double v = (double)pop[i * N + xs + (int64_t)L * ys];
        r += v;
        jx += c2x(i) * v;
        jy += c2y(i) * v;
    }
    out[s] = r;
    out[N + s] = jx;
    out[2 * N + s] = jy;
}

// Row transforms X_c[y][kx] = sum_x v_c[y][x] e^{-2 pi i kx x / L}: one
// workgroup per (channel, row), twiddles cos, sin of 2 pi k / L.
__global__ void __launch_bounds__(kBlock)
k2_dft_rows(int L, const double *__restrict__ v_all, const double *__restrict__ twid, double2 *__restrict__ X_all) {
    __shared__ double row[2048], cs[2048], sn[2048];
    const double *v = v_all + (int64_t)blockIdx.y * 3 * L * L;
    double2 *X = X_all + (int64_t)blockIdx.y * 3 * L * L;
    const int64_t r = blockIdx.x;  // channel * L + y
    for (int x = threadIdx.x; x < L; x += kBlock) {
        row[x] = v[r * L + x];
        cs[x] = twid[x];
        sn[x] = twid[L + x];
    }
    __syncthreads();
    for (int kx = threadIdx.x; kx < L; kx += kBlock) {
        double re = 0.0, im = 0.0;
        int k = 0;
        for (int x = 0; x < L; ++x) {
            re += row[x] * cs[k];
            im -= row[x] * sn[k];
            k += kx;
            if (k >= L) k -= L;
        }
        X[r * L + kx] = make_double2(re, im);
    }
}

// Column transforms and accumulation, one thread per (ky, kx): per sample
// S += |rho_k|^2 / N, Jx, Jy += |j_a,k|^2 / N, and the projections of j_k on
// k (longitudinal) and across it (transverse); k = 0 has no direction (0).
__global__ void __launch_bounds__(kBlock)
k2_dft_cols(int L, const double2 *__restrict__ X_all, const double *__restrict__ twid, double *__restrict__ acc_all) {
    const int64_t N = (int64_t)L * L;
    const double2 *X = X_all + (int64_t)blockIdx.y * 3 * N;
    double *acc = acc_all + (int64_t)blockIdx.y * 5 * N;
    const int64_t o = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (o >= N) return;
    const int ky = (int)(o / L), kx = (int)(o - (int64_t)ky * L);
    double re[3] = {0, 0, 0}, im[3] = {0, 0, 0};
    int k = 0;
    for (int y = 0; y < L; ++y) {
        const double c = twid[k], sn = twid[L + k];
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            const double2 v = X[(int64_t)ch * N + (int64_t)y * L + kx];
            re[ch] += v.x * c + v.y * sn;
            im[ch] += v.y * c - v.x * sn;
        }
        k += ky;
        if (k >= L) k -= L;
    }
    const double inv = 1.0 / (double)N;
    const int mx = kx <= L / 2 ? kx : kx - L, my = ky <= L / 2 ? ky : ky - L;
    const double kn = sqrt((double)mx * mx + (double)my * my);
    const double hx = kn > 0 ? mx / kn : 0.0, hy = kn > 0 ? my / kn : 0.0;
    const double pr = hx * re[1] + hy * re[2], pi = hx * im[1] + hy * im[2];
    const double tr = -hy * re[1] + hx * re[2], ti = -hy * im[1] + hx * im[2];
    acc[o] += (re[0] * re[0] + im[0] * im[0]) * inv;
    acc[N + o] += (re[1] * re[1] + im[1] * im[1]) * inv;
    acc[2 * N + o] += (re[2] * re[2] + im[2] * im[2]) * inv;
    acc[3 * N + o] += (pr * pr + pi * pi) * inv;
    acc[4 * N + o] += (tr * tr + ti * ti) * inv;
}

// Power-of-two L: the same transforms as radix-2 FFTs, O(L^2 log L) per
// sample instead of O(L^3).  One line of L complex values in LDS, loaded in
// bit-reversed order, then the log2 L butterfly stages of length len = 2,
// 4, ..., L with the twiddles e^{-2 pi i k / L} (k = j L / len).  Up to three
// consecutive stages run together on groups of 2^M values held in registers:
// each value goes through the same butterflies, with the same twiddles, as
// in separate stages, with a barrier and an LDS round trip per pass instead
// of per stage.
__device__ __forceinline__ void k2_bfly(double2 &u, double2 &v, double c, double sn) {
    const double tr = v.x * c + v.y * sn, ti = v.y * c - v.x * sn;  // v e^{-i theta}
    v = make_double2(u.x - tr, u.y - ti);
    u = make_double2(u.x + tr, u.y + ti);
}

// Stages len, 2 len, ..., 2^(M-1) len on NL lines (line l at buf + l * stride):
// group g holds the values e_t = base + t half (half = len / 2, t < 2^M), and
// stage k pairs e_t with e_(t + 2^k) (bit k of t clear) at twiddle
// (j + (t mod 2^k) half) L / (2^k len), j = g mod half.
template <int NL, int M>
__device__ __forceinline__ void k2_fft_pass(double2 *buf, int stride, int L, int len,
                                            const double *__restrict__ twid) {
    constexpr int G = 1 << M;
    const int half = len >> 1, ng = L >> M;
    for (int b = threadIdx.x; b < NL * ng; b += kBlock) {
        const int line = b / ng, g = b - line * ng;
        const int grp = g / half, j = g - grp * half;
        double2 *ln = buf + line * stride + grp * (half << M) + j;
        double2 e[G];
#pragma unroll
        for (int t = 0; t < G; ++t) e[t] = ln[t * half];
#pragma unroll
        for (int k = 0; k < M; ++k) {
            const int st = L / (len << k);
#pragma unroll
            for (int t = 0; t < G; ++t) {
                if ((t >> k) & 1) continue;
                const int tw = (j + (t & ((1 << k) - 1)) * half) * st;
                k2_bfly(e[t], e[t + (1 << k)], twid[tw], twid[L + tw]);
            }
        }
#pragma unroll
        for (int t = 0; t < G; ++t) ln[t * half] = e[t];
    }
    __syncthreads();
}

// NL lines of L values side by side (line l at buf + l * stride), one
// barrier per pass for all of them.  Three stages per pass where the groups
// of eight still give every thread one (2048-point lines, the batches'
// twelve-line column passes), else two (a single 256-point line: 32 groups
// of eight would leave seven threads in eight idle).
template <int NL>
__device__ __forceinline__ void k2_fft_lines(double2 *buf, int stride, int L, const double *__restrict__ twid) {
    int len = 2, left = __builtin_ctz((unsigned)L);
    if (NL * L >= 8 * kBlock)
        for (; left >= 3; left -= 3, len <<= 3) k2_fft_pass<NL, 3>(buf, stride, L, len, twid);
    for (; left >= 2; left -= 2, len <<= 2) k2_fft_pass<NL, 2>(buf, stride, L, len, twid);
    if (left == 1) k2_fft_pass<NL, 1>(buf, stride, L, len, twid);
}

__device__ __forceinline__ void k2_fft_line(double2 *buf, int L, const double *__restrict__ twid) {
    k2_fft_lines<1>(buf, L, L, twid);
}

// Power-of-two L <= kK2LinesMaxL: the density deviation and momentum of the
// state (the sums of k2_snap, in its order) formed straight into bit-reversed
// LDS lines and their three row transforms side by side, one workgroup per
// (row, replica); k2_fft_cols3_acc then takes the columns.  The same values
// as k2_snap + k2_fft_rows, without the snapshot array and with a third of
// the barriers.
// ML: the largest L of the instance (its LDS lines).
constexpr int kK2LinesMaxL = 1024;
template <int ML>
__global__ void __launch_bounds__(kBlock)
k2_snap_fft_rows(int L, int logL, const float *__restrict__ pop_all, const double *__restrict__ twid,
                 double2 *__restrict__ X_all) {
    __shared__ double2 buf[3 * ML];
    const int64_t N = (int64_t)L * L;
    const float *pop = pop_all + (int64_t)blockIdx.y * Q2 * N;
    double2 *X = X_all + (int64_t)blockIdx.y * 3 * N;
    const int y = blockIdx.x;
    for (int x = threadIdx.x; x < L; x += kBlock) {
        double r = 0.0, jx = 0.0, jy = 0.0;
#pragma unroll
        for (int i = 0; i < Q2; ++i) {
            const int xs = wrap2(x - c2x(i), L), ys = wrap2(y - c2y(i), L);
            const double v = (double)pop[i * N + xs + (int64_t)L * ys];
            r += v;
            jx += c2x(i) * v;
            jy += c2y(i) * v;
        }
        const int br = (int)(__brev((unsigned)x) >> (32 - logL));
        buf[br] = make_double2(r, 0.0);
        buf[L + br] = make_double2(jx, 0.0);
        buf[2 * L + br] = make_double2(jy, 0.0);
    }
    __syncthreads();
    k2_fft_lines<3>(buf, L, L, twid);
    for (int kx = threadIdx.x; kx < L; kx += kBlock)
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) X[ch * N + (int64_t)y * L + kx] = buf[ch * L + kx];
}

// Row FFTs X_c[y][kx] of the snapshot: one workgroup per (channel, row).
__global__ void __launch_bounds__(kBlock)
k2_fft_rows(int L, int logL, const double *__restrict__ v_all, const double *__restrict__ twid,
            double2 *__restrict__ X_all) {
    __shared__ double2 buf[2048];
    const double *v = v_all + (int64_t)blockIdx.y * 3 * L * L;
    double2 *X = X_all + (int64_t)blockIdx.y * 3 * L * L;
    const int64_t r = blockIdx.x;  // channel * L + y
    for (int x = threadIdx.x; x < L; x += kBlock)
        buf[__brev((unsigned)x) >> (32 - logL)] = make_double2(v[r * L + x], 0.0);
    __syncthreads();
    k2_fft_line(buf, L, twid);
    for (int kx = threadIdx.x; kx < L; kx += kBlock) X[r * L + kx] = buf[kx];
}

// Column FFTs in place: X_c[ky][kx] from X_c[y][kx], one workgroup per
// (channel, CPW adjacent kx; each row read as CPW consecutive values), the
// butterflies of k2_fft_line on each column.
template <int CPW>
__global__ void __launch_bounds__(kBlock)
k2_fft_cols(int L, int logL, double2 *__restrict__ X_all, const double *__restrict__ twid) {
    __shared__ double2 buf[CPW * 2048];
    const int64_t N = (int64_t)L * L;
    double2 *X = X_all + (int64_t)blockIdx.y * 3 * N;
    const int per = L / CPW, ch = blockIdx.x / per, kx0 = (blockIdx.x - ch * per) * CPW;
    double2 *col = X + ch * N + kx0;
    for (int i = threadIdx.x; i < L * CPW; i += kBlock) {
        const int y = i / CPW, c = i - y * CPW;
        buf[c * L + (__brev((unsigned)y) >> (32 - logL))] = col[(int64_t)y * L + c];
    }
    __syncthreads();
    if constexpr (CPW == 1) k2_fft_line(buf, L, twid);
    else k2_fft_lines<CPW>(buf, L, L, twid);
    for (int i = threadIdx.x; i < L * CPW; i += kBlock) {
        const int ky = i / CPW, c = i - ky * CPW;
        col[(int64_t)ky * L + c] = buf[c * L + ky];
    }
}

// The spectra of mode (ky, kx) from its transformed channels (density, jx,
// jy), added to the accumulators at o = ky L + kx: |rho_k|^2, |jx_k|^2,
// |jy_k|^2 and the projections of j_k on k (longitudinal) and across it
// (transverse), each divided by N; k = 0 has no direction (0).
__device__ __forceinline__ void k2_spec_add(double *acc, int64_t N, int L, int ky, int kx, const double (&re)[3],
                                            const double (&im)[3]) {
    const int64_t o = (int64_t)ky * L + kx;
    const double inv = 1.0 / (double)N;
    const int mx = kx <= L / 2 ? kx : kx - L, my = ky <= L / 2 ? ky : ky - L;
    const double kn = sqrt((double)mx * mx + (double)my * my);
    const double hx = kn > 0 ? mx / kn : 0.0, hy = kn > 0 ? my / kn : 0.0;
    const double pr = hx * re[1] + hy * re[2], pi = hx * im[1] + hy * im[2];
    const double tr = -hy * re[1] + hx * re[2], ti = -hy * im[1] + hx * im[2];
    acc[o] += (re[0] * re[0] + im[0] * im[0]) * inv;
    acc[N + o] += (re[1] * re[1] + im[1] * im[1]) * inv;
    acc[2 * N + o] += (re[2] * re[2] + im[2] * im[2]) * inv;
    acc[3 * N + o] += (pr * pr + pi * pi) * inv;
    acc[4 * N + o] += (tr * tr + ti * ti) * inv;
}

// Accumulation of the spectra from the transformed channels, one thread per
// (ky, kx): the same sums as the direct transform's.
__global__ void __launch_bounds__(kBlock)
k2_spec_acc(int L, const double2 *__restrict__ X_all, double *__restrict__ acc_all) {
    const int64_t N = (int64_t)L * L;
    const double2 *X = X_all + (int64_t)blockIdx.y * 3 * N;
    double *acc = acc_all + (int64_t)blockIdx.y * 5 * N;
    const int64_t o = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (o >= N) return;
    const int ky = (int)(o / L), kx = (int)(o - (int64_t)ky * L);
    double re[3], im[3];
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        const double2 v = X[(int64_t)ch * N + o];
        re[ch] = v.x;
        im[ch] = v.y;
    }
    k2_spec_add(acc, N, L, ky, kx, re, im);
}

// Batches: the column transforms of CPW adjacent kx (three channels each,
// 3 CPW lines side by side; each row read as CPW consecutive values) and the
// spectra accumulated straight from LDS, without writing the columns back:
// per line the butterflies of k2_fft_cols, per mode the sums of k2_spec_acc.
template <int ML, int CPW>
__global__ void __launch_bounds__(kBlock)
k2_fft_cols3_acc(int L, int logL, const double2 *__restrict__ X_all, const double *__restrict__ twid,
                 double *__restrict__ acc_all) {
    __shared__ double2 buf[3 * CPW * ML];
    const int64_t N = (int64_t)L * L;
    const double2 *X = X_all + (int64_t)blockIdx.y * 3 * N;
    double *acc = acc_all + (int64_t)blockIdx.y * 5 * N;
    const int kx0 = blockIdx.x * CPW;
    for (int i = threadIdx.x; i < L * CPW; i += kBlock) {
        const int y = i / CPW, c = i - y * CPW;
        const int br = (int)(__brev((unsigned)y) >> (32 - logL));
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) buf[(ch * CPW + c) * L + br] = X[ch * N + (int64_t)y * L + kx0 + c];
    }
    __syncthreads();
    k2_fft_lines<3 * CPW>(buf, L, L, twid);
    for (int i = threadIdx.x; i < L * CPW; i += kBlock) {
        const int ky = i / CPW, c = i - ky * CPW;
        double re[3], im[3];
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            const double2 v = buf[(ch * CPW + c) * L + ky];
            re[ch] = v.x;
            im[ch] = v.y;
        }
        k2_spec_add(acc, N, L, ky, kx0 + c, re, im);
    }
}

}  // namespace lbfss
