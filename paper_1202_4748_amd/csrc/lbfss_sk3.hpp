// Three-dimensional structure factor on sample steps (Sec. IV A, Eq.
// (G-comput)): C(k) = N^-1 |sum_r phi(r) e^{-i k.r}|^2 at every k = 2 pi m / L,
// reduced into shells s = floor(|m| + 1/2) (m folded into (-L/2, L/2]) for
// the Ornstein-Zernike analysis of Eq. (CMF).
//
// phi = (rho - rho0)/rho0 differs from the density deviation of the snapshot
// by a constant (k = 0 only) and the factor 1/rho0, so the transform runs on
// the snapshot and C is scaled by 1/(N rho0^2).  The transform is separable:
// a real-to-half-complex DFT along x (kx = 0..L/2), then complex DFTs along y
// and z, each a direct O(L) sum per output with an FP64 twiddle table (index
// (k n) mod L), so any L works.  Tiles of the input columns sit in LDS.  The
// shell sums reduce each shell's mode list in a fixed order, so they are
// deterministic; a half-space mode with 0 < kx < L/2 stands for itself and
// its mirror -k (weight 2).
#pragma once

#include "lbfss_step.hpp"

namespace lbfss {

constexpr int kSk3MaxL = 1024;

// x pass: one workgroup per (z, y) row of the replica.
__global__ void __launch_bounds__(kBlock)
k_sk3_x(int L, const float *__restrict__ drho, const double *__restrict__ twid, double2 *__restrict__ A) {
    __shared__ double row[kSk3MaxL], cs[kSk3MaxL], sn[kSk3MaxL];
    const int64_t r = blockIdx.x;
    for (int x = threadIdx.x; x < L; x += kBlock) {
        row[x] = (double)drho[r * L + x];
        cs[x] = twid[x];
        sn[x] = twid[L + x];
    }
    __syncthreads();
    const int Lh = L / 2 + 1;
    for (int kx = threadIdx.x; kx < Lh; kx += kBlock) {
        double re = 0.0, im = 0.0;
        int k = 0;
        for (int x = 0; x < L; ++x) {
            re += row[x] * cs[k];
            im -= row[x] * sn[k];
            k += kx;
            if (k >= L) k -= L;
        }
        A[r * Lh + kx] = make_double2(re, im);
    }
}

// Columns of KX consecutive kx per workgroup: L * KX complex values in LDS.
inline int sk3_tile(int L) { return L <= 256 ? 8 : (L <= 512 ? 4 : 2); }

// y pass (AXIS = 1): workgroup (z, kx tile); in[z][y][kx] -> out[z][ky][kx].
// z pass (AXIS = 2): workgroup (ky, kx tile); in[z][ky][kx] -> C[kz][ky][kx] =
// |X|^2 * scale, with scale = 1 / (N rho0^2) from the replica's totals.
template <int AXIS>
__global__ void __launch_bounds__(kBlock)
k_sk3_yz(int L, int KX, const double2 *__restrict__ in, double2 *__restrict__ out, double *__restrict__ C,
         const double *__restrict__ twid, const double *__restrict__ gl) {
    __shared__ double2 T[2048];
    __shared__ double cs[kSk3MaxL], sn[kSk3MaxL];
    const int Lh = L / 2 + 1;
    const int ntile = (Lh + KX - 1) / KX;
    const int a = blockIdx.x / ntile, kx0 = (blockIdx.x - a * ntile) * KX;
    // element (n, j) of the column tile: n runs along the transformed axis
    auto src = [&](int n, int j) -> int64_t {
        return AXIS == 1 ? ((int64_t)a * L + n) * Lh + kx0 + j : ((int64_t)n * L + a) * Lh + kx0 + j;
    };
    for (int e = threadIdx.x; e < L * KX; e += kBlock) {
        const int n = e / KX, j = e - n * KX;
        T[e] = (kx0 + j < Lh) ? in[src(n, j)] : make_double2(0.0, 0.0);
    }
    for (int x = threadIdx.x; x < L; x += kBlock) {
        cs[x] = twid[x];
        sn[x] = twid[L + x];
    }
    __syncthreads();
    double scale = 0.0;
    if (AXIS == 2) {
        const double rho0 = gl[1];
        scale = 1.0 / ((double)L * L * L * rho0 * rho0);
    }
    for (int o = threadIdx.x; o < L * KX; o += kBlock) {
        const int kk = o / KX, j = o - kk * KX;
        if (kx0 + j >= Lh) continue;
        double re = 0.0, im = 0.0;
        int k = 0;
        for (int n = 0; n < L; ++n) {
            const double2 v = T[n * KX + j];
            // v * e^{-i 2 pi kk n / L}
            re += v.x * cs[k] + v.y * sn[k];
            im += v.y * cs[k] - v.x * sn[k];
            k += kk;
            if (k >= L) k -= L;
        }
        if (AXIS == 1)
            out[((int64_t)a * L + kk) * Lh + kx0 + j] = make_double2(re, im);
        else
            C[((int64_t)kk * L + a) * Lh + kx0 + j] = (re * re + im * im) * scale;
    }
}

// Shell sums: one workgroup per shell s >= 1 of the replica; the modes of a
// shell are listed (half-space index (kz L + ky) Lh + kx, ascending).
// Workgroup 0 counts the sample.
__global__ void __launch_bounds__(kBlock)
k_sk3_shells(int L, const double *__restrict__ C, const int32_t *__restrict__ idx,
             const int64_t *__restrict__ off, double *__restrict__ acc, int64_t *__restrict__ nsamp3) {
    __shared__ double sh[kBlock];
    const int s = blockIdx.x;
    if (s == 0) {
        if (threadIdx.x == 0) *nsamp3 += 1;
        return;  // k = 0 is excluded
    }
    const int Lh = L / 2 + 1;
    const bool even = (L % 2) == 0;
    double v = 0.0;
    for (int64_t i = off[s] + threadIdx.x; i < off[s + 1]; i += kBlock) {
        const int32_t m = idx[i];
        const int kx = m % Lh;
        const double w = (kx == 0 || (even && kx == L / 2)) ? 1.0 : 2.0;
        v += w * C[m];
    }
    // fixed tree over the workgroup
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int h = kBlock / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) acc[s] += sh[0];
}

}  // namespace lbfss
