// Fused step: one pass per time step.  A workgroup owns an x-y tile of one
// replica and marches through a range of z planes.  For each plane it pulls
// the populations of the tile plus a two-site halo to form the density in
// LDS (a four-plane ring), derives the chemical potential on the tile plus
// a one-site halo (a three-plane ring), and two planes behind that front
// collides the tile interior: force from the LDS stencils, pull, moment-space
// collision with Philox noise, store.  Densities of the halo are recomputed
// by neighbouring tiles instead of being exchanged, so there is no
// inter-workgroup synchronisation; the halo pulls mostly hit L2.
#pragma once

#include <array>
#include <vector>

#include "lbfss_step.hpp"

namespace lbfss {

struct FusedTile {
    int32_t rep, x0, y0, z0, nx, ny, nz, pad;
};

__device__ __forceinline__ int wrap_near(int v, int L) { return v < 0 ? v + L : (v >= L ? v - L : v); }

template <typename T>
__global__ void __launch_bounds__(kBlock)
k_fused(const RepDesc *__restrict__ desc, const FusedTile *__restrict__ tiles, const T *__restrict__ pop,
        T *__restrict__ pop_out, const uint64_t *__restrict__ step, int koff, int *__restrict__ err,
        int ep_max) {
    extern __shared__ float lds[];
    const FusedTile tl = tiles[blockIdx.x];
    const RepDesc &d = desc[tl.rep];
    const int L = d.L;
    const int EX = tl.nx + 4, EP = EX * (tl.ny + 4);
    const int MX = tl.nx + 2, MP = MX * (tl.ny + 2);
    float *rho_ring = lds;                 // 4 planes of EP (stride ep_max)
    float *mu_ring = lds + 4 * ep_max;     // 3 planes of MP (stride ep_max)
    const T *base = pop + Q * d.site_off;
    T *obase = pop_out + Q * d.site_off;
    const uint64_t t = *step + (uint64_t)koff;
    const bool force_on = !(d.flags & 1);
    bool bad = false;

    for (int p = tl.z0 - 2; p <= tl.z0 + tl.nz + 1; ++p) {
        // (a) density of plane p on the tile and its two-site halo
        {
            const int zp = wrap_near(p, L);
            float *rs = rho_ring + ((p + 8) & 3) * ep_max;
            for (int i = threadIdx.x; i < EP; i += kBlock) {
                const int ey = i / EX, ex = i - ey * EX;
                const Nbr n(wrap_near(tl.x0 - 2 + ex, L), wrap_near(tl.y0 - 2 + ey, L), zp, L);
                float f[Q];
                pull(base, d.N, n, f);
                rs[i] = drho_of(f);
            }
        }
        __syncthreads();
        // (b) chemical potential of plane p - 1 on the tile and a one-site halo
        if (p - 1 >= tl.z0 - 1) {
            const float *rz[3] = {rho_ring + ((p - 2 + 8) & 3) * ep_max, rho_ring + ((p - 1 + 8) & 3) * ep_max,
                                  rho_ring + ((p + 8) & 3) * ep_max};
            float *ms = mu_ring + ((p - 1 + 9) % 3) * ep_max;
            for (int i = threadIdx.x; i < MP; i += kBlock) {
                const int my = i / MX, mx = i - my * MX;
                const int c0 = (my + 1) * EX + (mx + 1);
                const float c = rz[1][c0];
                ms[i] = chem_potential(d, c, lap18(c, [&](int dx, int dy, int dz) {
                                           return rz[1 + dz][c0 + dy * EX + dx];
                                       }));
            }
        }
        __syncthreads();
        // (c) collide plane z = p - 2
        if (p - 2 >= tl.z0) {
            const int z = p - 2;
            const float *rz[3] = {rho_ring + ((z - 1 + 8) & 3) * ep_max, rho_ring + ((z + 8) & 3) * ep_max,
                                  rho_ring + ((z + 1 + 8) & 3) * ep_max};
            const float *mz[3] = {mu_ring + ((z - 1 + 9) % 3) * ep_max, mu_ring + ((z + 9) % 3) * ep_max,
                                  mu_ring + ((z + 1 + 9) % 3) * ep_max};
            const int npl = tl.nx * tl.ny;
            for (int i = threadIdx.x; i < npl; i += kBlock) {
                const int iy = i / tl.nx, ix = i - iy * tl.nx;
                const int x = tl.x0 + ix, y = tl.y0 + iy;
                float Fx = 0.f, Fy = 0.f, Fz = 0.f;
                if (force_on) {
                    const int rc0 = (iy + 2) * EX + (ix + 2);
                    const int mc0 = (iy + 1) * MX + (ix + 1);
                    const float rho_x = d.rho_c + rz[1][rc0];
                    const Grad18 gr = grad18([&](int dx, int dy, int dz) {
                        return (1.0f / 3.0f) * rz[1 + dz][rc0 + dy * EX + dx] -
                               rho_x * mz[1 + dz][mc0 + dy * MX + dx];
                    });
                    Fx = gr.gx;
                    Fy = gr.gy;
                    Fz = gr.gz;
                }
                const Nbr n(x, y, z, L);
                float f[Q];
                pull(base, d.N, n, f);
                const uint32_t s = (uint32_t)(x + n.Y0 + n.Z0);
                const SiteNoise noise{s, (uint32_t)t, (uint32_t)(t >> 32), d.key0, d.key1};
                const float rho = collide_site(d, f, Fx, Fy, Fz, noise);
                bad |= !(rho > 0.0f && rho < 1e30f);  // Sec. III B: rho must stay positive
#pragma unroll
                for (int q = 0; q < Q; ++q) Store<T>::st(obase + q * d.N, s, f[q]);
            }
        }
        __syncthreads();
    }
    if (bad) *err = 1;
}

// ---------------------------------------------------------------------------
// Host side: tile tables and launch.
// ---------------------------------------------------------------------------
inline int fused_ep_max(int tx, int ty) { return (tx + 4) * (ty + 4); }
constexpr int64_t kFusedLdsBytes = 65536;  // per workgroup: 4 density + 3 potential planes

inline int make_fused_tiles(const std::vector<RepDesc> &reps, int tx, int ty, int tz,
                            std::vector<FusedTile> &out) {
    if (tx < 1 || ty < 1 || tz < 1 || tx > 256 || ty > 256 || tz > 1024) return -1;
    if (7 * 4 * (int64_t)fused_ep_max(std::min(tx, 1024), std::min(ty, 1024)) > kFusedLdsBytes) return -1;
    out.clear();
    for (size_t r = 0; r < reps.size(); ++r) {
        const int L = reps[r].L;
        const int nx = std::min(tx, L), ny = std::min(ty, L), nz = std::min(tz, L);
        for (int z0 = 0; z0 < L; z0 += nz)
            for (int y0 = 0; y0 < L; y0 += ny)
                for (int x0 = 0; x0 < L; x0 += nx)
                    out.push_back(FusedTile{(int32_t)r, x0, y0, z0, std::min(nx, L - x0), std::min(ny, L - y0),
                                            std::min(nz, L - z0), 0});
    }
    return 0;
}

inline void default_fused_tile(const std::vector<RepDesc> &reps, int &tx, int &ty, int &tz) {
    int maxL = 0;
    for (const auto &d : reps) maxL = std::max(maxL, d.L);
    if (maxL >= 128) {
        tx = 64;
        ty = 16;
        tz = 32;
    } else if (maxL >= 64) {
        tx = 64;
        ty = 8;
        tz = 16;
    } else {
        tx = std::min(maxL, 32);
        ty = std::min(maxL, 8);
        tz = std::min(maxL, 16);
    }
}

inline std::vector<std::array<int, 3>> fused_tile_candidates(const std::vector<RepDesc> &reps) {
    int maxL = 0;
    for (const auto &d : reps) maxL = std::max(maxL, d.L);
    std::vector<std::array<int, 3>> c = {{64, 8, 16}, {64, 16, 32}, {64, 8, 64}, {32, 8, 32},
                                         {128, 8, 32}, {64, 4, 32},  {32, 16, 16}};
    if (maxL <= 64) c.push_back({maxL, std::min(maxL, 16), std::min(maxL, 16)});
    if (maxL <= 44) c.push_back({maxL, maxL, maxL});
    return c;
}

template <typename T>
void launch_fused(const RepDesc *desc, const FusedTile *tiles, int n_tiles, const T *in, T *out,
                  const uint64_t *step, int koff, int *err, int tx, int ty, hipStream_t stream) {
    const int ep = fused_ep_max(tx, ty);
    const size_t lds = sizeof(float) * (size_t)(7 * ep);
    hipLaunchKernelGGL(k_fused<T>, dim3(n_tiles), dim3(kBlock), lds, stream, desc, tiles, in, out, step, koff,
                       err, ep);
}

}  // namespace lbfss
