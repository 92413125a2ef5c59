// Sample-step kernels: the observables of the finite-size-scaling analysis
// (Gross & Varnik, Sec. II B, Eqs. (mL), (ML), (chiL), (chiL-lowT), (CL)) and
// the structure factor along the lattice axes (Sec. IV A, Eq. (G-comput)),
// with the order parameter phi = (rho - rho0)/rho0, rho0 the global mean
// density (Sec. II A, Eq. (op)).
//
// All reductions are FP64 and run in a fixed order, so a replica's results
// are bit-identical whatever batch it is part of.  Each launch covers every
// replica of a handle: per-stage prefix arrays `cum` map a flattened item
// index to (replica, local item).
#pragma once

#include "lbfss_step.hpp"

namespace lbfss {

constexpr int kMaxLevels = 16;
constexpr int kMoments = 7;  // m, m^2, m^3, m^4, |m|, E, E^2
constexpr int kMaxHistBins = 4096;

struct SampDesc {
    int32_t L, Lmin, nlev, nb;   // nb = L / Lmin boxes per axis at the finest level
    int32_t n_k, series_cap, rec_len, pad;
    int32_t base_lev;            // finest level whose box sums are stored (-1: none)
    int32_t snap_lev;            // level of one-site boxes, read from the snapshot (-1: none)
    int32_t direct;              // base level summed straight from the snapshot (else separably)
    int32_t pad2;
    int64_t twid_off;            // 2 * L doubles: cos, sin of 2 pi k / L
    int64_t site_off;            // first site (snapshot index) of the replica
    int64_t rows_off;            // 4 * L^2 doubles: row sums of drho, jx, jy, jz, [4][z][y]
    int64_t cols_off;            // L^2 doubles: column sums of drho over y, [z][x]
    int64_t planes_off;          // 6 * L doubles: plane sums P_x, P_y, P_z of drho, P_z of jx, jy, jz
    int64_t a_off;               // 2 * L * L * nb: [2][z][y][bx]
    int64_t b_off;               // 2 * L * nb * nb: [2][z][by][bx]
    int64_t lev_off[kMaxLevels]; // 2 * (L/Lb)^3 each: [2][bz][by][bx], level 0 = L/2
    int32_t lev_L[kMaxLevels];   // box edge of each level
    int64_t chunk_first[kMaxLevels]; // first partial-sum chunk of each level
    int32_t chunk_count[kMaxLevels];
    int64_t acc_off;             // accumulators: nlev * 7 level sums, then 3 * n_k S(k) sums
    int64_t series_off;          // series_cap * rec_len doubles
    int64_t glob_off;            // 6 doubles: dbar, rhobar, mass, px, py, pz of the last reduction
    int32_t hist_bins;           // histogram bins per level (0: none)
    int32_t pad3;
    double hist_h, hist_inv_w;   // half-width h and bins / (2 h)
    int64_t hist_off;            // nlev * (hist_bins + 2) counters (uint64)
    int64_t levtot_off;          // nlev * 7 doubles: this sample's level sums
};

// A chunk of consecutive boxes of one (replica, level) reduced by one
// workgroup into one partial-sum row.
struct BoxChunk {
    int32_t rep, lev;
    int64_t first;
    int32_t count, pad;
};

__device__ __forceinline__ int find_cum(const int64_t *__restrict__ cum, int nrep, int64_t g) {
    int lo = 0, hi = nrep - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (cum[mid] <= g) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Deterministic FP64 sum over one 64-lane wave (fixed butterfly).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

// N deterministic FP64 sums over a 256-thread workgroup at once, each by
// the fixed tree v[t] += v[t + s], s = 128, 64, ..., 1: the two cross-wave
// halvings in LDS (sh holds N * kBlock doubles), then the wave butterfly,
// whose lane 0 adds the same pairs in the same order.  The sums are valid
// in thread 0 only.
template <int N>
__device__ __forceinline__ void block_sums(double (&v)[N], double *sh) {
    static_assert(kBlock == 256, "two cross-wave halvings, then one wave");
    const int t = threadIdx.x;
#pragma unroll
    for (int q = 0; q < N; ++q) sh[q * kBlock + t] = v[q];
    __syncthreads();
    if (t < 128)
#pragma unroll
        for (int q = 0; q < N; ++q) sh[q * kBlock + t] += sh[q * kBlock + t + 128];
    __syncthreads();
    if (t < 64)
#pragma unroll
        for (int q = 0; q < N; ++q) v[q] = wave_sum(sh[q * kBlock + t] + sh[q * kBlock + t + 64]);
    __syncthreads();
}

// 1. Snapshot of drho and j at every site (pulled populations), FP32.
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_snapshot(const RepDesc *__restrict__ desc, int nrep, int64_t total, const T *__restrict__ pop,
           float *__restrict__ snap) {
    const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (g >= total) return;
    const int r = find_rep(desc, nrep, g);
    const RepDesc &d = desc[r];
    const Nbr n(g - d.site_off, d.L);
    float f[Q];
    pull(pop + Q * d.site_off, d.N, n, f);
    float jx, jy, jz;
    momentum_of(f, jx, jy, jz);
    snap[g] = drho_of(f);
    snap[total + g] = jx;
    snap[2 * total + g] = jy;
    snap[3 * total + g] = jz;
}

// 2. Row sums over x of drho, jx, jy, jz: one 64-lane wave per (z, y) row.
__global__ void __launch_bounds__(kBlock)
k_rows(const SampDesc *__restrict__ sd, const int64_t *__restrict__ cum, int nrep, int64_t total_sites,
       const float *__restrict__ snap, double *__restrict__ ws) {
    const int64_t row = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= cum[nrep]) return;  // whole wave leaves together
    const int r = find_cum(cum, nrep, row);
    const SampDesc &s = sd[r];
    const int64_t lr = row - cum[r];
    const int L = s.L;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const int64_t base = s.site_off + lr * L;
    int x = lane;
    // four x chunks of the four channels loaded before they are added (same order)
    for (; x + 192 < L; x += 256) {
        float t[4][4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int c = 0; c < 4; ++c) t[u][c] = snap[c * total_sites + base + x + 64 * u];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[c] += (double)t[u][c];
    }
    for (; x < L; x += 64)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[c] += (double)snap[c * total_sites + base + x];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        double v = acc[c];
#pragma unroll
        for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
        acc[c] = v;
    }
    if (lane == 0) {
        const int64_t LL = (int64_t)L * L;
#pragma unroll
        for (int c = 0; c < 4; ++c) ws[s.rows_off + c * LL + lr] = acc[c];
    }
}

// 3. Column sums over y of drho for every (z, x): a workgroup takes 64
// consecutive columns (one per lane, so each load reads 64 consecutive
// values) and its four waves the four interleaved y phases y = k, k + 4, ...
// (the rows past the last multiple of four go to phase 0); the phase sums
// combine as (a0 + a1) + (a2 + a3).
__global__ void __launch_bounds__(kBlock)
k_cols(const SampDesc *__restrict__ sd, const int64_t *__restrict__ cum, int nrep,
       const float *__restrict__ snap, double *__restrict__ ws) {
    static_assert(kBlock == 4 * 64, "one wave per y phase");
    __shared__ double sh[4][64];
    const int lane = threadIdx.x & 63, k = threadIdx.x >> 6;
    const int64_t g = (int64_t)blockIdx.x * 64 + lane;
    const bool on = g < cum[nrep];
    double a = 0.0;
    int r = 0;
    int64_t li = 0;
    if (on) {
        r = find_cum(cum, nrep, g);
        const SampDesc &s = sd[r];
        li = g - cum[r];
        const int L = s.L;
        const uint32_t zi = (uint32_t)li / (uint32_t)L;  // li < L^2
        const int64_t z = zi, x = li - (int64_t)zi * L;
        const float *col = snap + s.site_off + x + (int64_t)L * L * z;
        int y = 0;
        // eight rows of this phase loaded before they are added (same order)
        for (; y + 31 < L; y += 32) {
            float t[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) t[u] = col[(int64_t)(y + 4 * u + k) * L];
#pragma unroll
            for (int u = 0; u < 8; ++u) a += (double)t[u];
        }
        for (; y + 3 < L; y += 4) a += (double)col[(int64_t)(y + k) * L];
        if (k == 0)
            for (; y < L; ++y) a += (double)col[(int64_t)y * L];
    }
    sh[k][lane] = a;
    __syncthreads();
    if (k == 0 && on) ws[sd[r].cols_off + li] = (sh[0][lane] + sh[1][lane]) + (sh[2][lane] + sh[3][lane]);
}

// 4. Plane sums: one 64-lane wave per (replica, plane family, n) over six
// families P_x, P_y, P_z of drho and P_z of jx, jy, jz; lane l adds the
// terms l, l + 64, ... in order, then a fixed butterfly.
__global__ void __launch_bounds__(kBlock)
k_planes(const SampDesc *__restrict__ sd, const int64_t *__restrict__ cum, int nrep, double *__restrict__ ws) {
    const int64_t g = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (g >= cum[nrep]) return;  // whole wave leaves together
    const int r = find_cum(cum, nrep, g);
    const SampDesc &s = sd[r];
    const int L = s.L;
    const int64_t li = g - cum[r];
    const int fam = (int)(li / L), n = (int)(li - (int64_t)fam * L);
    const int64_t LL = (int64_t)L * L;
    const double *src;
    int64_t stride;
    if (fam == 0) {        // P_x(n) = sum_z cols[z][n]
        src = ws + s.cols_off + n;
        stride = L;
    } else if (fam == 1) { // P_y(n) = sum_z rows[z][n]
        src = ws + s.rows_off + n;
        stride = L;
    } else {               // P_z(n) of channel fam - 2 = sum_y rows[c][n][y]
        src = ws + s.rows_off + (fam - 2) * LL + (int64_t)n * L;
        stride = 1;
    }
    double a = 0.0;
    for (int k = lane; k < L; k += 64) a += src[k * stride];
    a = wave_sum(a);
    if (lane == 0) ws[s.planes_off + li] = a;
}

// 5. Totals (one workgroup per replica): mass, momentum and the mean density
// deviation dbar that defines phi.
__global__ void __launch_bounds__(kBlock)
k_totals(const SampDesc *__restrict__ sd, const RepDesc *__restrict__ desc, int nrep, double *__restrict__ ws) {
    __shared__ double sh[4 * kBlock];
    const int r = blockIdx.x;
    const SampDesc &s = sd[r];
    const int L = s.L;
    double tot[4];
    for (int c = 0; c < 4; ++c) {
        const double *P = ws + s.planes_off + (int64_t)(2 + c) * L;
        double a = 0.0;
        for (int k = threadIdx.x; k < L; k += kBlock) a += P[k];
        tot[c] = a;
    }
    block_sums(tot, sh);
    if (threadIdx.x == 0) {
        const double N = (double)L * (double)L * (double)L;
        const double rho_c = (double)desc[r].rho_c;
        double *gl = ws + s.glob_off;
        gl[0] = tot[0] / N;
        gl[1] = rho_c + tot[0] / N;
        gl[2] = rho_c * N + tot[0];
        gl[3] = tot[1];
        gl[4] = tot[2];
        gl[5] = tot[3];
    }
}

// Base-level box sums straight from the snapshot: one thread per box of edge
// Lb <= 4 (at most 64 sites, z then y then x).
__global__ void __launch_bounds__(kBlock)
k_box_direct(const SampDesc *__restrict__ sd, const int64_t *__restrict__ cum, int nrep,
             const float *__restrict__ snap, double *__restrict__ ws) {
    const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (g >= cum[nrep]) return;
    const int r = find_cum(cum, nrep, g);
    const SampDesc &s = sd[r];
    const int L = s.L, Lb = s.lev_L[s.base_lev];
    const uint32_t nbl = (uint32_t)(L / Lb);
    const uint32_t li = (uint32_t)(g - cum[r]);  // < nbl^3 <= 2^27: 32-bit division
    const uint32_t bzy = li / nbl;
    const int64_t bx = li - bzy * nbl, bz = bzy / nbl, by = bzy - (uint32_t)bz * nbl;
    const float *src = snap + s.site_off + bx * Lb + (int64_t)L * (by * Lb + (int64_t)L * bz * Lb);
    double a1 = 0.0, a2 = 0.0;
    if (Lb == 2) {  // the common case: all eight sites loaded first, then added in order
        float t[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) t[u] = src[(u & 1) + (int64_t)L * (((u >> 1) & 1) + (int64_t)L * (u >> 2))];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const double v = (double)t[u];
            a1 += v;
            a2 += v * v;
        }
    } else {
        for (int dz = 0; dz < Lb; ++dz)
            for (int dy = 0; dy < Lb; ++dy)
                for (int dx = 0; dx < Lb; ++dx) {
                    const double v = (double)src[dx + (int64_t)L * (dy + (int64_t)L * dz)];
                    a1 += v;
                    a2 += v * v;
                }
    }
    const int64_t cnt = (int64_t)nbl * nbl * nbl;
    ws[s.lev_off[s.base_lev] + li] = a1;
    ws[s.lev_off[s.base_lev] + cnt + li] = a2;
}

// 5.-7. Box sums of drho and drho^2 at the finest level Lmin, separably:
// along x from the snapshot, then along y, then along z.
__global__ void __launch_bounds__(kBlock)
k_box_x(const SampDesc *__restrict__ sd, const int64_t *__restrict__ cum, int nrep,
        const float *__restrict__ snap, double *__restrict__ ws) {
    const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (g >= cum[nrep]) return;
    const int r = find_cum(cum, nrep, g);
    const SampDesc &s = sd[r];
    const int64_t li = g - cum[r];          // (z, y, bx)
    const int64_t row = li / s.nb, bx = li - row * s.nb;
    const float *src = snap + s.site_off + row * s.L + bx * s.Lmin;
    double a1 = 0.0, a2 = 0.0;
    for (int i = 0; i < s.Lmin; ++i) {
        const double v = (double)src[i];
        a1 += v;
        a2 += v * v;
    }
    const int64_t cnt = (int64_t)s.L * s.L * s.nb;
    ws[s.a_off + li] = a1;
    ws[s.a_off + cnt + li] = a2;
}

__global__ void __launch_bounds__(kBlock)
k_box_y(const SampDesc *__restrict__ sd, const int64_t *__restrict__ cum, int nrep, double *__restrict__ ws) {
    const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (g >= cum[nrep]) return;
    const int r = find_cum(cum, nrep, g);
    const SampDesc &s = sd[r];
    const int64_t li = g - cum[r];          // (z, by, bx)
    const int nb = s.nb;
    const int64_t z = li / ((int64_t)nb * nb);
    const int64_t rem = li - z * nb * nb;
    const int64_t by = rem / nb, bx = rem - by * nb;
    const int64_t cntA = (int64_t)s.L * s.L * nb;
    double a1 = 0.0, a2 = 0.0;
    for (int i = 0; i < s.Lmin; ++i) {
        const int64_t src = (z * s.L + by * s.Lmin + i) * nb + bx;
        a1 += ws[s.a_off + src];
        a2 += ws[s.a_off + cntA + src];
    }
    const int64_t cntB = (int64_t)s.L * nb * nb;
    ws[s.b_off + li] = a1;
    ws[s.b_off + cntB + li] = a2;
}

__global__ void __launch_bounds__(kBlock)
k_box_z(const SampDesc *__restrict__ sd, const int64_t *__restrict__ cum, int nrep, double *__restrict__ ws) {
    const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (g >= cum[nrep]) return;
    const int r = find_cum(cum, nrep, g);
    const SampDesc &s = sd[r];
    const int64_t li = g - cum[r];          // (bz, by, bx)
    const int nb = s.nb;
    const int64_t plane = (int64_t)nb * nb;
    const int64_t bz = li / plane, rem = li - bz * plane;
    const int64_t cntB = (int64_t)s.L * plane;
    double a1 = 0.0, a2 = 0.0;
    for (int i = 0; i < s.Lmin; ++i) {
        const int64_t src = (bz * s.Lmin + i) * plane + rem;
        a1 += ws[s.b_off + src];
        a2 += ws[s.b_off + cntB + src];
    }
    const int64_t dst = s.lev_off[s.nlev - 1];
    const int64_t cnt = plane * nb;
    ws[dst + li] = a1;
    ws[dst + cnt + li] = a2;
}

// 8. Coarser levels from a stored finer one.  Level l has 2^(l + 1) boxes
// per axis whatever L is, and a box sums its 8 children (z, then y, then x).
// One launch forms up to three levels per replica: a workgroup loads a cube
// of e^3 boxes (e = 2^nl <= 8) of level `fine` into LDS and forms the
// (e/2)^3, (e/4)^3, ... boxes of the levels fine - 1, ..., fine - nl above
// it, each written out and kept in LDS for the next.
struct CoarsenGroup {
    int32_t fine, nl;  // nl = 0: nothing for this replica in this launch
};

__global__ void __launch_bounds__(kBlock)
k_coarsen_cube(const SampDesc *__restrict__ sd, const int64_t *__restrict__ cum,
               const CoarsenGroup *__restrict__ grp, int nrep, double *__restrict__ ws) {
    __shared__ double cube[2][2][512];  // [buffer][sum of drho, of drho^2][box]
    const int64_t g = blockIdx.x;
    if (g >= cum[nrep]) return;  // whole workgroup
    const int r = find_cum(cum, nrep, g);
    const SampDesc &s = sd[r];
    const CoarsenGroup cg = grp[r];
    // every edge is a power of two: indices split by shifts (li < 2^27)
    const uint32_t li = (uint32_t)(g - cum[r]);
    const int ln = cg.nl, e = 1 << ln;
    const int lt = cg.fine - cg.nl + 1;  // log2 of the top-level boxes per axis
    const int64_t cz = li >> (2 * lt), cy = (li >> lt) & ((1u << lt) - 1), cx = li & ((1u << lt) - 1);
    {
        const int64_t nf = (int64_t)2 << cg.fine;
        const double *f1 = ws + s.lev_off[cg.fine], *f2 = f1 + nf * nf * nf;
        for (int i = threadIdx.x; i < e * e * e; i += kBlock) {
            const int dz = i >> (2 * ln), dy = (i >> ln) & (e - 1), dx = i & (e - 1);
            const int64_t src = (cx * e + dx) + nf * ((cy * e + dy) + nf * (cz * e + dz));
            cube[0][0][i] = f1[src];
            cube[0][1][i] = f2[src];
        }
    }
    __syncthreads();
    for (int k = 1; k <= cg.nl; ++k) {
        const int ef = e >> (k - 1), ec = e >> k;   // this cube's edge at the finer, coarser level
        const double *a = cube[(k - 1) & 1][0], *b = cube[(k - 1) & 1][1];
        double *oa = cube[k & 1][0], *ob = cube[k & 1][1];
        const int lev = cg.fine - k;
        const int64_t nc = (int64_t)2 << lev;
        const int lc = ln - k;  // log2 ec
        for (int i = threadIdx.x; i < ec * ec * ec; i += kBlock) {
            const int bz = i >> (2 * lc), by = (i >> lc) & (ec - 1), bx = i & (ec - 1);
            double a1 = 0.0, a2 = 0.0;
            for (int dz = 0; dz < 2; ++dz)
                for (int dy = 0; dy < 2; ++dy)
                    for (int dx = 0; dx < 2; ++dx) {
                        const int src = (2 * bx + dx) + ef * ((2 * by + dy) + ef * (2 * bz + dz));
                        a1 += a[src];
                        a2 += b[src];
                    }
            oa[i] = a1;
            ob[i] = a2;
            const int64_t dst = (cx * ec + bx) + nc * ((cy * ec + by) + nc * (cz * ec + bz));
            double *out = ws + s.lev_off[lev];
            out[dst] = a1;
            out[nc * nc * nc + dst] = a2;
        }
        __syncthreads();
    }
}

// 9. Partial sums over a chunk of boxes of m, m^2, m^3, m^4, |m|, E, E^2,
// and the chunk's contribution to the level's histogram of m (Sec. II C,
// Eq. (PL-def)): counted in LDS, then added to the device counters (integer
// sums, so the order of the additions cannot change them).
constexpr int kBoxesPerThread = 16;
constexpr int kChunkBoxes = kBlock * kBoxesPerThread;

__global__ void __launch_bounds__(kBlock)
k_level_partials(const SampDesc *__restrict__ sd, const BoxChunk *__restrict__ chunks,
                 const float *__restrict__ snap, double *__restrict__ ws, double *__restrict__ parts,
                 unsigned long long *__restrict__ hist) {
    __shared__ double sh[kMoments * kBlock];
    __shared__ unsigned int s_hist[kMaxHistBins + 2];
    const BoxChunk c = chunks[blockIdx.x];
    const SampDesc &s = sd[c.rep];
    const int nbins = s.hist_bins;  // uniform over the workgroup
    if (nbins > 0) {
        for (int i = threadIdx.x; i < nbins + 2; i += kBlock) s_hist[i] = 0u;
        __syncthreads();
    }
    const double *gl = ws + s.glob_off;
    const double dbar = gl[0], inv_rho0 = 1.0 / gl[1];
    const int Lb = s.lev_L[c.lev];
    const double n = (double)Lb * (double)Lb * (double)Lb;
    // box volume reciprocals, once per chunk (exact for power-of-two boxes)
    const double inv_n = 1.0 / n, inv_2n = 0.5 * inv_n;
    const int64_t nbl = s.L / Lb;
    const int64_t cnt = nbl * nbl * nbl;
    const bool from_snap = c.lev == s.snap_lev;  // one-site boxes: the snapshot itself
    const double *b1 = ws + s.lev_off[c.lev];
    const double *b2 = b1 + cnt;
    const float *sn = snap + s.site_off;
    double acc[kMoments] = {0, 0, 0, 0, 0, 0, 0};
    auto add_box = [&](double B1, double B2) __attribute__((always_inline)) {
        const double sphi = (B1 - n * dbar) * inv_rho0;
        const double sphi2 = (B2 - 2.0 * dbar * B1 + n * dbar * dbar) * inv_rho0 * inv_rho0;
        const double m = sphi * inv_n, E = sphi2 * inv_2n;
        const double m2 = m * m;
        acc[0] += m;
        acc[1] += m2;
        acc[2] += m2 * m;
        acc[3] += m2 * m2;
        acc[4] += fabs(m);
        acc[5] += E;
        acc[6] += E * E;
        if (nbins > 0) {
            const double kf = floor((m + s.hist_h) * s.hist_inv_w);
            // in range: its bin; below -h (or not a number): nbins; at or above h: nbins + 1
            const int idx = (kf >= 0.0 && kf < (double)nbins) ? (int)kf : (kf >= (double)nbins ? nbins + 1 : nbins);
            atomicAdd(&s_hist[idx], 1u);
        }
    };
    // a full chunk (every chunk of a level but its last): the thread's loads
    // issued together, eight at a time for the stored levels, then its boxes
    // added in the same order as the guarded loop below
    const int64_t i0 = c.first + threadIdx.x;
    if (c.count == kChunkBoxes && from_snap) {
        float v[kBoxesPerThread];
#pragma unroll
        for (int k = 0; k < kBoxesPerThread; ++k) v[k] = sn[i0 + k * kBlock];
#pragma unroll
        for (int k = 0; k < kBoxesPerThread; ++k) {
            const double B1 = (double)v[k];
            add_box(B1, B1 * B1);
        }
    } else if (c.count == kChunkBoxes) {
#pragma unroll
        for (int k0 = 0; k0 < kBoxesPerThread; k0 += 8) {
            double v1[8], v2[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                v1[k] = b1[i0 + (k0 + k) * kBlock];
                v2[k] = b2[i0 + (k0 + k) * kBlock];
            }
#pragma unroll
            for (int k = 0; k < 8; ++k) add_box(v1[k], v2[k]);
        }
    } else {
        for (int k = 0; k < kBoxesPerThread; ++k) {
            const int64_t i = (int64_t)k * kBlock + threadIdx.x;
            if (i >= c.count) break;
            if (from_snap) {
                const double B1 = (double)sn[c.first + i];
                add_box(B1, B1 * B1);
            } else {
                add_box(b1[c.first + i], b2[c.first + i]);
            }
        }
    }
    if (nbins > 0) {
        __syncthreads();
        unsigned long long *hl = hist + s.hist_off + (int64_t)c.lev * (nbins + 2);
        for (int i = threadIdx.x; i < nbins + 2; i += kBlock)
            if (s_hist[i]) atomicAdd(&hl[i], (unsigned long long)s_hist[i]);
    }
    block_sums(acc, sh);
    if (threadIdx.x == 0)
#pragma unroll
        for (int q = 0; q < kMoments; ++q) parts[(int64_t)blockIdx.x * kMoments + q] = acc[q];
}

// Axis structure factor S_a(k_m) = N^-1 |sum_n P_a(n) e^{-i k_m n}|^2 of phi,
// one 64-lane wave per (replica, axis, m), twiddles from the replica's FP64
// table (index m n mod L); lanes take n = l, l + 64, ..., then a butterfly.
__global__ void __launch_bounds__(kBlock)
k_structure_factor(const SampDesc *__restrict__ sd, const int64_t *__restrict__ cum, int nrep,
                   const double *__restrict__ ws, double *__restrict__ acc_all) {
    const int64_t g = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (g >= cum[nrep]) return;  // whole wave leaves together
    const int r = find_cum(cum, nrep, g);
    const SampDesc &s = sd[r];
    const int idx = (int)(g - cum[r]);
    const int L = s.L;
    const int a = idx / s.n_k, m = idx - a * s.n_k + 1;
    const double *planes = ws + s.planes_off + (int64_t)a * L;
    const double *cs = ws + s.twid_off, *sn = cs + L;
    const double *gl = ws + s.glob_off;
    const double rho0 = gl[1], off = (double)L * L * gl[0];  // plane sum of rho0 - rho_c
    double re = 0.0, im = 0.0;
    for (int n = lane; n < L; n += 64) {
        const double p = (planes[n] - off) / rho0;
        const int k = (int)(((int64_t)m * n) % L);
        re += p * cs[k];
        im -= p * sn[k];
    }
    re = wave_sum(re);
    im = wave_sum(im);
    if (lane == 0) {
        const double Nsites = (double)L * L * L;
        acc_all[s.acc_off + s.nlev * kMoments + idx] += (re * re + im * im) / Nsites;
    }
}

// 10. One workgroup per (replica, level): reduce the level's chunk partial
// sums in a fixed order, add them to the accumulators and keep this
// sample's level sums for the series record.
__global__ void __launch_bounds__(kBlock)
k_level_reduce(const SampDesc *__restrict__ sd, int max_nlev, double *__restrict__ ws,
               const double *__restrict__ parts, double *__restrict__ acc_all) {
    __shared__ double sh[kMoments * kBlock];
    const int r = blockIdx.x / max_nlev, lev = blockIdx.x - r * max_nlev;
    const SampDesc &s = sd[r];
    if (lev >= s.nlev) return;  // whole workgroup
    double *acc = acc_all + s.acc_off;
    // one pass over the chunks for all moments (each moment still adds its
    // chunks in the same order per thread, then the same block sum)
    double v[kMoments] = {0, 0, 0, 0, 0, 0, 0};
    const double *p0 = parts + s.chunk_first[lev] * kMoments;
    const int64_t nch = s.chunk_count[lev];
    int64_t k = threadIdx.x;
    // four of this thread's chunks loaded at a time, then added in order
    for (; k + 3 * kBlock < nch; k += 4 * kBlock) {
        double t[4][kMoments];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int q = 0; q < kMoments; ++q) t[u][q] = p0[(k + u * kBlock) * kMoments + q];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int q = 0; q < kMoments; ++q) v[q] += t[u][q];
    }
    for (; k < nch; k += kBlock) {
        const double *pk = p0 + k * kMoments;
#pragma unroll
        for (int q = 0; q < kMoments; ++q) v[q] += pk[q];
    }
    block_sums(v, sh);
    if (threadIdx.x == 0)
#pragma unroll
        for (int q = 0; q < kMoments; ++q) {
            ws[s.levtot_off + lev * kMoments + q] = v[q];
            acc[lev * kMoments + q] += v[q];
        }
}

// 11. Per replica (one thread each): append a series record, count the sample.
__global__ void k_finalize(const SampDesc *__restrict__ sd, int nrep, const double *__restrict__ ws,
                           double *__restrict__ series_all, int64_t *__restrict__ nsamp,
                           const uint64_t *__restrict__ step, int koff) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrep) return;
    const SampDesc &s = sd[r];
    const double *gl = ws + s.glob_off;
    const double *lt = ws + s.levtot_off;
    const int64_t k = nsamp[r];
    if (s.series_cap > 0) {
        double *rec = series_all + s.series_off + (k % s.series_cap) * s.rec_len;
        rec[0] = (double)(*step + (uint64_t)koff);
        rec[1] = gl[2];
        rec[2] = gl[3];
        rec[3] = gl[4];
        rec[4] = gl[5];
        for (int lev = 0; lev < s.nlev; ++lev) {
            const double nb = (double)(s.L / s.lev_L[lev]);
            const double nboxes = nb * nb * nb;
            for (int q = 0; q < kMoments; ++q) rec[5 + lev * kMoments + q] = lt[lev * kMoments + q] / nboxes;
        }
    }
    nsamp[r] = k + 1;
}

}  // namespace lbfss
