// Device building blocks of the fluctuating non-ideal D3Q19 lattice-Boltzmann
// step (Gross & Varnik, Sec. III A): counter-based noise, the moment-space
// collision with Guo forcing, and population storage.
//
// Populations live in device memory as the scaled deviation
//     r_i = (f_i - w_i rho_c) / w_i
// (FP32 or FP16), one [19][N] block per replica, N = L^3, site = x + L(y + L z).
// The scaling makes every population of a quiet fluid O(drho), which is what
// lets FP16 storage keep the fluctuations, and it leaves the moment
// transforms with small integer coefficients.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbfss {

constexpr int Q = 19;

// Per-replica constants, resident in device memory (one table per handle).
struct RepDesc {
    int32_t L;
    int32_t flags;     // LB_FORCE_OFF
    int64_t N;         // L^3
    int64_t site_off;  // first site of the replica in the handle's flattened sites
    float a, b, kappa, rho_c;
    float gamma;       // 1 - 1/tau of the shear moments 5..9
    float half1pg;     // (1 + gamma) / 2, the Guo source factor 1 - 1/(2 tau)
    float noise_amp;   // sqrt(kT (1 - gamma^2) / c_s^2)
    float gamma_b;     // the same three for the bulk moment 4 (its own time tau_bulk)
    float half1pg_b;
    float noise_amp_b;
    float gamma_g;     // ghost moments 10..18 (tau_ghost; no force source there)
    float noise_amp_g;
    uint32_t key0, key1;  // Philox key: seed low and high words
};

// ---------------------------------------------------------------------------
// Storage precision
// ---------------------------------------------------------------------------
template <typename T> struct Store;
template <> struct Store<float> {
    static __device__ __forceinline__ float ld(const float *p, int64_t i) { return p[i]; }
    static __device__ __forceinline__ void st(float *p, int64_t i, float v) { p[i] = v; }
};
template <> struct Store<__half> {
    static __device__ __forceinline__ float ld(const __half *p, int64_t i) {
        return __half2float(p[i]);
    }
    static __device__ __forceinline__ void st(__half *p, int64_t i, float v) {
        p[i] = __float2half_rn(v);
    }
};

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32 -> 64-bit products; each round's high halves are xor-ed with the
// other two counter words and the round key, the key advancing by the Weyl
// constants between rounds.
// ---------------------------------------------------------------------------
struct Words4 {
    uint32_t v[4];
};

// a ^ b ^ c as one three-input bitwise instruction (truth table 0x96); the
// compiler forms it from no expression by itself
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ Words4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        // one 32x32 -> 64-bit multiply-add instruction per product
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
        const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
        if (round < 2) {
            // the collision noise's first two rounds still mix wave-uniform
            // words (step, call, key): xor those on the scalar unit first
            c0 = hi1 ^ (c1 ^ k0);
            c2 = hi0 ^ (c3 ^ k1);
        } else {
            c0 = xor3(hi1, c1, k0);
            c2 = xor3(hi0, c3, k1);
        }
        c1 = lo1;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    Words4 w;
    w.v[0] = c0;
    w.v[1] = c1;
    w.v[2] = c2;
    w.v[3] = c3;
    return w;
}

// Uniform in (0,1): ((w >> 9) + 1/2) 2^-23.  The top 23 bits of w become the
// mantissa of a float in [1, 2) (one funnel shift puts the exponent of 1
// above them), and subtracting 1 - 2^-24 leaves (2 (w >> 9) + 1) 2^-24:
// exact, since the difference has at most 24 significant bits.
__device__ __forceinline__ float uniform01(uint32_t w) {
    return __uint_as_float(__builtin_amdgcn_alignbit(0x7Fu, w, 9u)) - 0.999999940395355224609375f;
}

// Box-Muller radius sqrt(-2 ln u) via the hardware base-2 logarithm.
__device__ __forceinline__ float bm_radius(float u0) {
    return __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(u0));
}

// Hardware sine and cosine take their argument in revolutions, which is
// exactly the Box-Muller angle 2 pi u.
__device__ __forceinline__ float cos_rev(float u) { return __builtin_amdgcn_cosf(u); }
__device__ __forceinline__ float sin_rev(float u) { return __builtin_amdgcn_sinf(u); }

// ---------------------------------------------------------------------------
// Collision of one site.
//
// r[19]  in:  pulled scaled deviations r_i(x, t);  out: post-collision r*_i.
// Moments of the basis (weight-orthogonal, norms N_a):
//   0: 1   1-3: c   4: c^2 - 1   5: 3cx^2 - c^2   6: cy^2 - cz^2
//   7-9: cx cy, cy cz, cz cx   10-12: (3c^2 - 5) c   13: (cy^2 - cz^2) cx
//   14: (cz^2 - cx^2) cy   15: (cx^2 - cy^2) cz   16: 3c^4 - 6c^2 + 1
//   17: (2c^2 - 3)(3cx^2 - c^2)   18: (2c^2 - 3)(cy^2 - cz^2)
// Velocities come in opposite pairs; even moments use pair sums, odd moments
// pair differences.  Pairs: X(1,2) Y(3,4) Z(5,6) A(7,8)=(1,1,0)
// B(9,10)=(1,-1,0) C(11,12)=(1,0,1) D(13,14)=(1,0,-1) E(15,16)=(0,1,1)
// F(17,18)=(0,1,-1).
// Returns the site density rho (<= 0 or NaN flags instability).
// ---------------------------------------------------------------------------
template <typename NoiseFn>
__device__ __forceinline__ float collide_site(const RepDesc &d, float (&r)[Q], float Fx, float Fy,
                                              float Fz, NoiseFn &&noise) {
    // weighted pair sums / differences: moments of the deviation f - w rho_c
    const float w1 = 1.0f / 18.0f, w2 = 1.0f / 36.0f;
    const float f0 = r[0] * (1.0f / 3.0f);
    const float sX = (r[1] + r[2]) * w1, dX = (r[1] - r[2]) * w1;
    const float sY = (r[3] + r[4]) * w1, dY = (r[3] - r[4]) * w1;
    const float sZ = (r[5] + r[6]) * w1, dZ = (r[5] - r[6]) * w1;
    const float sA = (r[7] + r[8]) * w2, dA = (r[7] - r[8]) * w2;
    const float sB = (r[9] + r[10]) * w2, dB = (r[9] - r[10]) * w2;
    const float sC = (r[11] + r[12]) * w2, dC = (r[11] - r[12]) * w2;
    const float sD = (r[13] + r[14]) * w2, dD = (r[13] - r[14]) * w2;
    const float sE = (r[15] + r[16]) * w2, dE = (r[15] - r[16]) * w2;
    const float sF = (r[17] + r[18]) * w2, dF = (r[17] - r[18]) * w2;

    const float sAx = sX + sY + sZ;
    const float sABCD = (sA + sB) + (sC + sD);
    const float sEF = sE + sF;
    const float sDg = sABCD + sEF;

    const float drho = f0 + sAx + sDg;
    const float jx = dX + (dA + dB) + (dC + dD);
    const float jy = dY + (dA - dB) + (dE + dF);
    const float jz = dZ + (dC - dD) + (dE - dF);

    const float m4 = sDg - f0;
    const float m5 = 2.0f * sX - sY - sZ + sABCD - 2.0f * sEF;
    const float m6 = sY - sZ + (sA + sB) - (sC + sD);
    const float m7 = sA - sB;
    const float m8 = sE - sF;
    const float m9 = sC - sD;
    const float dABCD = (dA + dB) + (dC + dD);
    const float m10 = dABCD - 2.0f * dX;
    const float m11 = (dA - dB) + (dE + dF) - 2.0f * dY;
    const float m12 = (dC - dD) + (dE - dF) - 2.0f * dZ;
    const float m13 = (dA + dB) - (dC + dD);
    const float m14 = (dB - dA) + (dE + dF);
    const float m15 = (dC - dD) - (dE - dF);
    const float m16 = f0 - 2.0f * sAx + sDg;
    const float m17 = sY + sZ - 2.0f * sX + sABCD - 2.0f * sEF;
    const float m18 = sZ - sY + (sA + sB) - (sC + sD);

    const float rho = d.rho_c + drho;
    const float inv_rho = __builtin_amdgcn_rcpf(rho);  // hardware reciprocal, 1 ulp
    const float ux = (jx + 0.5f * Fx) * inv_rho;
    const float uy = (jy + 0.5f * Fy) * inv_rho;
    const float uz = (jz + 0.5f * Fz) * inv_rho;
    const float uxx = ux * ux, uyy = uy * uy, uzz = uz * uz;
    const float u2 = uxx + uyy + uzz;
    const float uF = ux * Fx + uy * Fy + uz * Fz;

    // second-order equilibrium and Guo source moments (zero beyond a = 9);
    // moment 4 relaxes with the bulk time, 5..9 with tau, 10..18 with the ghost time
    const float g = d.gamma, og = 1.0f - d.gamma, h = d.half1pg;
    const float gg = d.gamma_g;
    float p4 = (1.0f - d.gamma_b) * (rho * u2) + d.gamma_b * m4 + d.half1pg_b * (2.0f * uF);
    float p5 = og * (rho * (3.0f * uxx - u2)) + g * m5 + h * (2.0f * (3.0f * ux * Fx - uF));
    float p6 = og * (rho * (uyy - uzz)) + g * m6 + h * (2.0f * (uy * Fy - uz * Fz));
    float p7 = og * (rho * ux * uy) + g * m7 + h * (ux * Fy + uy * Fx);
    float p8 = og * (rho * uy * uz) + g * m8 + h * (uy * Fz + uz * Fy);
    float p9 = og * (rho * uz * ux) + g * m9 + h * (uz * Fx + ux * Fz);
    float p10 = gg * m10, p11 = gg * m11, p12 = gg * m12;
    float p13 = gg * m13, p14 = gg * m14, p15 = gg * m15;
    float p16 = gg * m16, p17 = gg * m17, p18 = gg * m18;

    // thermal noise: sigma_a g_{a-4}, sigma_a = noise_amp sqrt(rho) sqrt(N_a);
    // generated and applied four normals (one Philox call) at a time
    {
        const float srho = __builtin_amdgcn_sqrtf(fmaxf(rho, 0.0f));
        const float amp = d.noise_amp * srho, amp_b = d.noise_amp_b * srho, amp_g = d.noise_amp_g * srho;
        float n[4];
        noise(0, n);  // normals 0..3 -> moments 4..7
        p4 += amp_b * 0.81649658092772603f * n[0];   // sqrt(N_4),  N = 2/3
        p5 += amp * 1.1547005383792515f * n[1];    // N = 4/3
        p6 += amp * 0.66666666666666667f * n[2];   // N = 4/9
        p7 += amp * 0.33333333333333333f * n[3];   // N = 1/9
        noise(1, n);  // normals 4..7 -> moments 8..11
        p8 += amp * 0.33333333333333333f * n[0];
        p9 += amp * 0.33333333333333333f * n[1];
        p10 += amp_g * 0.81649658092772603f * n[2];  // N = 2/3
        p11 += amp_g * 0.81649658092772603f * n[3];
        noise(2, n);  // normals 8..11 -> moments 12..15
        p12 += amp_g * 0.81649658092772603f * n[0];
        p13 += amp_g * 0.47140452079103169f * n[1];  // N = 2/9
        p14 += amp_g * 0.47140452079103169f * n[2];
        p15 += amp_g * 0.47140452079103169f * n[3];
        noise(3, n);  // normals 12..14 -> moments 16..18 (normal 15 unused)
        p16 += amp_g * 1.4142135623730951f * n[0];   // N = 2
        p17 += amp_g * 1.1547005383792515f * n[1];   // N = 4/3
        p18 += amp_g * 0.66666666666666667f * n[2];  // N = 4/9
    }

    // back-transform: r*_i = sum_a e_a(c_i) m*_a / N_a
    const float M0 = drho;
    const float M1 = 3.0f * (jx + Fx), M2 = 3.0f * (jy + Fy), M3 = 3.0f * (jz + Fz);
    const float M4 = 1.5f * p4, M5 = 0.75f * p5, M6 = 2.25f * p6;
    const float M7 = 9.0f * p7, M8 = 9.0f * p8, M9 = 9.0f * p9;
    const float M10 = 1.5f * p10, M11 = 1.5f * p11, M12 = 1.5f * p12;
    const float M13 = 4.5f * p13, M14 = 4.5f * p14, M15 = 4.5f * p15;
    const float M16 = 0.5f * p16, M17 = 0.75f * p17, M18 = 2.25f * p18;

    r[0] = M0 - M4 + M16;
    {
        const float ev = M0 + 2.0f * M5 - 2.0f * M16 - 2.0f * M17;
        const float od = M1 - 2.0f * M10;
        r[1] = ev + od;
        r[2] = ev - od;
    }
    {
        const float ev = M0 - M5 + M6 - 2.0f * M16 + M17 - M18;
        const float od = M2 - 2.0f * M11;
        r[3] = ev + od;
        r[4] = ev - od;
    }
    {
        const float ev = M0 - M5 - M6 - 2.0f * M16 + M17 + M18;
        const float od = M3 - 2.0f * M12;
        r[5] = ev + od;
        r[6] = ev - od;
    }
    const float base = M0 + M4 + M16;        // common even part of the 12 diagonals
    const float bxy = base + M5 + M6 + M17 + M18;  // (+-1,+-1,0)
    const float bxz = base + M5 - M6 + M17 - M18;  // (+-1,0,+-1)
    const float byz = base - 2.0f * M5 - 2.0f * M17;  // (0,+-1,+-1)
    {
        const float ev = bxy + M7;
        const float od = M1 + M2 + M10 + M11 + M13 - M14;
        r[7] = ev + od;
        r[8] = ev - od;
    }
    {
        const float ev = bxy - M7;
        const float od = M1 - M2 + M10 - M11 + M13 + M14;
        r[9] = ev + od;
        r[10] = ev - od;
    }
    {
        const float ev = bxz + M9;
        const float od = M1 + M3 + M10 + M12 - M13 + M15;
        r[11] = ev + od;
        r[12] = ev - od;
    }
    {
        const float ev = bxz - M9;
        const float od = M1 - M3 + M10 - M12 - M13 - M15;
        r[13] = ev + od;
        r[14] = ev - od;
    }
    {
        const float ev = byz + M8;
        const float od = M2 + M3 + M11 + M12 + M14 - M15;
        r[15] = ev + od;
        r[16] = ev - od;
    }
    {
        const float ev = byz - M8;
        const float od = M2 - M3 + M11 - M12 + M14 + M15;
        r[17] = ev + od;
        r[18] = ev - od;
    }
    return rho;
}

// Density deviation of pulled scaled deviations, in the same summation order
// as collide_site (so every kernel sees bit-identical densities).
__device__ __forceinline__ float drho_of(const float (&r)[Q]) {
    const float w1 = 1.0f / 18.0f, w2 = 1.0f / 36.0f;
    const float f0 = r[0] * (1.0f / 3.0f);
    const float sX = (r[1] + r[2]) * w1, sY = (r[3] + r[4]) * w1, sZ = (r[5] + r[6]) * w1;
    const float sA = (r[7] + r[8]) * w2, sB = (r[9] + r[10]) * w2;
    const float sC = (r[11] + r[12]) * w2, sD = (r[13] + r[14]) * w2;
    const float sE = (r[15] + r[16]) * w2, sF = (r[17] + r[18]) * w2;
    const float sAx = sX + sY + sZ;
    const float sDg = ((sA + sB) + (sC + sD)) + (sE + sF);
    return f0 + sAx + sDg;
}

// Momentum j = sum_i c_i w_i r_i of pulled scaled deviations.
__device__ __forceinline__ void momentum_of(const float (&r)[Q], float &jx, float &jy, float &jz) {
    const float w1 = 1.0f / 18.0f, w2 = 1.0f / 36.0f;
    const float dX = (r[1] - r[2]) * w1, dY = (r[3] - r[4]) * w1, dZ = (r[5] - r[6]) * w1;
    const float dA = (r[7] - r[8]) * w2, dB = (r[9] - r[10]) * w2;
    const float dC = (r[11] - r[12]) * w2, dD = (r[13] - r[14]) * w2;
    const float dE = (r[15] - r[16]) * w2, dF = (r[17] - r[18]) * w2;
    jx = dX + (dA + dB) + (dC + dD);
    jy = dY + (dA - dB) + (dE + dF);
    jz = dZ + (dC - dD) + (dE - dF);
}

// The collision normals of (site, step): Philox call j (counter (site,
// step_lo, j, step_hi)) gives normals 4j .. 4j+3 as the cos and sin of the
// Box-Muller pairs of its word pairs (0, 1) and (2, 3).
struct SiteNoise {
    uint32_t site, t_lo, t_hi, k0, k1;
    __device__ __forceinline__ void operator()(int j, float (&n)[4]) const {
        const Words4 w = philox4x32_10(site, t_lo, (uint32_t)j, t_hi, k0, k1);
        const float r0 = bm_radius(uniform01(w.v[0]));
        const float a0 = uniform01(w.v[1]);
        const float r1 = bm_radius(uniform01(w.v[2]));
        const float a1 = uniform01(w.v[3]);
        n[0] = r0 * cos_rev(a0);
        n[1] = r0 * sin_rev(a0);
        n[2] = r1 * cos_rev(a1);
        n[3] = (j == 3) ? 0.0f : r1 * sin_rev(a1);  // normal 15 is unused
    }
};

// Wrap-around neighbour coordinate for periodic boundaries.
__device__ __forceinline__ int wrap_dec(int v, int L) { return v == 0 ? L - 1 : v - 1; }
__device__ __forceinline__ int wrap_inc(int v, int L) { return v == L - 1 ? 0 : v + 1; }

// Velocity components of population q (same order as the public header).
__host__ __device__ constexpr int cx_of(int q) {
    return q == 1 ? 1 : q == 2 ? -1 : (q == 7 || q == 9 || q == 11 || q == 13) ? 1
           : (q == 8 || q == 10 || q == 12 || q == 14) ? -1 : 0;
}
__host__ __device__ constexpr int cy_of(int q) {
    return q == 3 ? 1 : q == 4 ? -1 : (q == 7 || q == 10 || q == 15 || q == 17) ? 1
           : (q == 8 || q == 9 || q == 16 || q == 18) ? -1 : 0;
}
__host__ __device__ constexpr int cz_of(int q) {
    return q == 5 ? 1 : q == 6 ? -1 : (q == 11 || q == 14 || q == 15 || q == 18) ? 1
           : (q == 12 || q == 13 || q == 16 || q == 17) ? -1 : 0;
}

}  // namespace lbfss
