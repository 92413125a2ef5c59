// Three-dimensional structure factor on sample steps (Sec. IV A, Eq.
// (G-comput)): C(k) = N^-1 |sum_r phi(r) e^{-i k.r}|^2 at every k = 2 pi m / L,
// reduced into shells s = floor(|m| + 1/2) (m folded into (-L/2, L/2]) for
// the Ornstein-Zernike analysis of Eq. (CMF).
//
// phi = (rho - rho0)/rho0 differs from the density deviation of the snapshot
// by a constant (k = 0 only) and the factor 1/rho0, so the transform runs on
// the snapshot and C is scaled by 1/(N rho0^2).  The transform is separable:
// a real-to-half-complex transform along x (kx = 0..L/2), then complex ones
// along y and z, all in FP64 with a twiddle table: radix-2 FFTs in LDS when L
// is a power of two, otherwise direct O(L) sums per output (index (k n) mod
// L), so any L works.  Tiles of the input columns sit in LDS.  The
// shell sums reduce each shell's mode list in a fixed order, so they are
// deterministic; a half-space mode with 0 < kx < L/2 stands for itself and
// its mirror -k (weight 2).
#pragma once

#include <algorithm>

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

// Radix-2 FFT passes for power-of-two L (the same three passes, O(L log L)
// per column instead of O(L^2)): a tile of KT columns sits in LDS with the
// element order along the transformed axis bit-reversed, followed by log2 L
// in-place decimation-in-time butterfly stages (twiddle e^{-2 pi i q / m} =
// table entry q L / m).  AXIS 0: real rows of the snapshot -> A[row][kx],
// kx = 0..L/2; AXIS 1: A[z][y][kx] -> B[z][ky][kx]; AXIS 2: B[z][ky][kx] ->
// C[kz][ky][kx] = |X|^2 / (N rho0^2).
inline int sk3_fft_tile(int L) { return std::min(2048 / L, 64); }

// Stages m, 2m, ..., 2^(M-1) m of the tile (element n of column j at
// T[n KT + j]): group g of column j holds e_t = base + t half (half = m / 2,
// t < 2^M), stage k pairs e_t with e_(t + 2^k) (bit k of t clear) at twiddle
// index (q + (t mod 2^k) half) L / (2^k m), q = group mod half.
template <int M>
__device__ __forceinline__ void sk3_fft_pass(double2 *T, int L, int KT, int m, const double *cs, const double *sn) {
    constexpr int G = 1 << M;
    const int half = m >> 1, ng = (L >> M) * KT;
    for (int b = threadIdx.x; b < ng; b += kBlock) {
        const int j = b % KT, bb = b / KT;
        const int grp = bb / half, q = bb - grp * half;
        double2 *col = T + (grp * (half << M) + q) * KT + j;
        double2 e[G];
#pragma unroll
        for (int t = 0; t < G; ++t) e[t] = col[t * half * KT];
#pragma unroll
        for (int k = 0; k < M; ++k) {
            const int step = L / (m << k);
#pragma unroll
            for (int t = 0; t < G; ++t) {
                if ((t >> k) & 1) continue;
                const int w = (q + (t & ((1 << k) - 1)) * half) * step;
                const double wr = cs[w], wi = -sn[w];
                const double2 u = e[t], v = e[t + (1 << k)];
                const double tr = v.x * wr - v.y * wi, ti = v.x * wi + v.y * wr;
                e[t] = make_double2(u.x + tr, u.y + ti);
                e[t + (1 << k)] = make_double2(u.x - tr, u.y - ti);
            }
        }
#pragma unroll
        for (int t = 0; t < G; ++t) col[t * half * KT] = e[t];
    }
    __syncthreads();
}

template <int AXIS>
__global__ void __launch_bounds__(kBlock)
k_sk3_fft(int L, int log2L, int KT, const float *__restrict__ drho, const double2 *__restrict__ in,
          double2 *__restrict__ out, double *__restrict__ C, const double *__restrict__ twid,
          const double *__restrict__ gl) {
    __shared__ double2 T[2048];
    __shared__ double cs[kSk3MaxL], sn[kSk3MaxL];
    const int Lh = L / 2 + 1;
    // columns: AXIS 0 -> the L^2 rows; AXIS 1, 2 -> (outer index a, kx)
    const int64_t ncol = AXIS == 0 ? (int64_t)L * L : (int64_t)L * Lh;
    const int64_t c0 = (int64_t)blockIdx.x * KT;
    auto col_ok = [&](int j) { return c0 + j < ncol; };
    // address of element n of column c
    auto at = [&](int64_t c, int n) -> int64_t {
        if (AXIS == 0) return c * L + n;
        const int64_t a = c / Lh, kx = c - a * Lh;
        return AXIS == 1 ? (a * L + n) * Lh + kx : ((int64_t)n * L + a) * Lh + kx;
    };
    for (int e = threadIdx.x; e < L * KT; e += kBlock) {
        const int n = e / KT, j = e - n * KT;
        const int slot = (int)(__brev((unsigned)n) >> (32 - log2L)) * KT + j;
        double2 v = make_double2(0.0, 0.0);
        if (col_ok(j)) {
            if (AXIS == 0) v.x = (double)drho[at(c0 + j, n)];
            else v = in[at(c0 + j, n)];
        }
        T[slot] = v;
    }
    for (int x = threadIdx.x; x < L; x += kBlock) {
        cs[x] = twid[x];
        sn[x] = twid[L + x];
    }
    __syncthreads();
    // stages m = 2, 4, ..., L, up to three per pass on groups of 2^M values of
    // one column held in registers (each value through the same butterflies
    // with the same twiddles as stage by stage); three where the groups still
    // give every thread one
    int m = 2, left = log2L;
    if ((L >> 3) * KT >= kBlock)
        for (; left >= 3; left -= 3, m <<= 3) sk3_fft_pass<3>(T, L, KT, m, cs, sn);
    for (; left >= 2; left -= 2, m <<= 2) sk3_fft_pass<2>(T, L, KT, m, cs, sn);
    if (left == 1) sk3_fft_pass<1>(T, L, KT, m, cs, sn);
    double scale = 0.0;
    if (AXIS == 2) {
        const double rho0 = gl[1];
        scale = 1.0 / ((double)L * L * L * rho0 * rho0);
    }
    const int nout = AXIS == 0 ? Lh : L;
    for (int e = threadIdx.x; e < nout * KT; e += kBlock) {
        const int k = e / KT, j = e - k * KT;
        if (!col_ok(j)) continue;
        const double2 v = T[k * KT + j];
        const int64_t c = c0 + j;
        if (AXIS == 0) out[c * Lh + k] = v;
        else if (AXIS == 1) out[at(c, k)] = v;
        else C[at(c, k)] = (v.x * v.x + v.y * v.y) * scale;
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
