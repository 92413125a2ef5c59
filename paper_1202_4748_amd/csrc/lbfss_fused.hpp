// Fused step: one pass per time step.
//
// A workgroup owns an x-y tile of TX x TY sites of one replica (256
// threads; 128 for 16 x 8 tiles, 512 for 64 x 8) and marches through a
// range of z planes, one thread per tile site.
// For each plane p it
//   (a) pulls the 19 populations of its site into a register ring (three
//       planes deep) and puts the site density in an LDS ring; threads also
//       pull the two-site halo of the tile, for the density only;
//   (b) derives the chemical potential of plane p - 1 on the tile and a
//       one-site halo (LDS ring);
//   (c) collides plane p - 2 from the register ring: force from the LDS
//       stencils, moment-space collision with Philox noise, non-temporal
//       store.
// Populations are read from memory once per site; the halo pulls are
// interior pulls of a neighbouring tile, which the XCD-aware workgroup order
// schedules on the same XCD at the same time, so they are served by its L2.
// Address arithmetic is hoisted: per-plane offsets are wave-uniform and the
// in-plane offsets of a thread are computed once.
#pragma once

#include <algorithm>
#include <array>
#include <vector>

#include "lbfss_step.hpp"

namespace lbfss {

struct FusedTile {
    int32_t rep, x0, y0, z0, nx, ny, nz, pad;
};

__device__ __forceinline__ int wrap_near(int v, int L) { return v < 0 ? v + L : (v >= L ? v - L : v); }

// In-plane byte offsets of the nine (x, y) positions a pull touches, for a
// site at (x, y) of an L x L plane: centre, -x, +x, -y, +y and the four
// diagonals.  Plane bases live in wave-uniform pointers, so every load is a
// scalar base plus one of these 32-bit offsets.
struct PlaneOffs {
    uint32_t c, xm, xp, ym, yp, mm, pp, mp, pm;  // mm = (x-1, y-1), mp = (x-1, y+1), ...
    __device__ __forceinline__ void set(int x, int y, int L, uint32_t esize) {
        const uint32_t xm_ = wrap_dec(x, L), xp_ = wrap_inc(x, L);
        const uint32_t Y0 = y * L, Ym = wrap_dec(y, L) * L, Yp = wrap_inc(y, L) * L;
        c = (x + Y0) * esize;
        xm = (xm_ + Y0) * esize;
        xp = (xp_ + Y0) * esize;
        ym = (x + Ym) * esize;
        yp = (x + Yp) * esize;
        mm = (xm_ + Ym) * esize;
        pp = (xp_ + Yp) * esize;
        mp = (xm_ + Yp) * esize;
        pm = (xp_ + Ym) * esize;
    }
};

// A wave-uniform address pinned to scalar registers, so that an access at it
// plus a 32-bit lane offset keeps no 64-bit per-lane address alive.
template <typename P>
__device__ __forceinline__ P *sbase(P *p) {
    const uint64_t a = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
    return (P *)(((uint64_t)hi << 32) | lo);
}

template <typename T>
__device__ __forceinline__ float ldb(const T *p, uint32_t boff) {
    return Store<T>::ld((const T *)((const char *)p + boff), 0);
}
// Store of a post-collision value: non-temporal, so the written planes do
// not push out of L2 the source rows that neighbouring tiles still read as
// their halo (the next step reads these values, long after L2 turned over).
template <typename T>
__device__ __forceinline__ void stb(T *p, uint32_t boff, float v) {
    if constexpr (sizeof(T) == 4)
        __builtin_nontemporal_store(v, (float *)((char *)p + boff));
    else
        __builtin_nontemporal_store(__half_as_ushort(__float2half_rn(v)), (unsigned short *)((char *)p + boff));
}

// Pull of the 19 populations of a site of plane z: buf_q(x - c_q).  qz[q] is
// the base of population q shifted to plane z - cz_q (wave-uniform).
template <typename T>
__device__ __forceinline__ void pull_plane(const T *const (&qz)[Q], const PlaneOffs &o, float (&r)[Q]) {
    r[0] = ldb(qz[0], o.c);
    r[1] = ldb(qz[1], o.xm);
    r[2] = ldb(qz[2], o.xp);
    r[3] = ldb(qz[3], o.ym);
    r[4] = ldb(qz[4], o.yp);
    r[5] = ldb(qz[5], o.c);
    r[6] = ldb(qz[6], o.c);
    r[7] = ldb(qz[7], o.mm);
    r[8] = ldb(qz[8], o.pp);
    r[9] = ldb(qz[9], o.mp);
    r[10] = ldb(qz[10], o.pm);
    r[11] = ldb(qz[11], o.xm);
    r[12] = ldb(qz[12], o.xp);
    r[13] = ldb(qz[13], o.xm);
    r[14] = ldb(qz[14], o.xp);
    r[15] = ldb(qz[15], o.ym);
    r[16] = ldb(qz[16], o.yp);
    r[17] = ldb(qz[17], o.ym);
    r[18] = ldb(qz[18], o.yp);
}

// Workgroup index to tile index: each XCD (workgroups are dealt to the 8
// XCDs round-robin) gets one contiguous run of the tile table, whose tiles
// are ordered x fastest, then y, then z, so neighbouring tiles share an L2.
// s_waitcnt immediate (gfx9 encoding) that waits until at most n vector-memory
// operations of the wave are outstanding (loads and stores alike, completed
// in order), leaving the LDS and export counters free.  The staged kernels
// wait with n = Q after a collision: the Q population stores of the wave are
// then the only operations younger than the staged loads, which holds while
// the kernel uses no scratch memory (build.py refuses a build where it does).
constexpr unsigned vmcnt_wait(int n) { return (unsigned)((n & 15) | ((n >> 4) << 14) | (0x7 << 4) | (0xF << 8)); }
static_assert(vmcnt_wait(19) == 0x4F73 && vmcnt_wait(0) == 0x0F70, "s_waitcnt encoding");

__device__ __forceinline__ int xcd_tile(int b, int nt) {
    const int per = nt / 8;
    if (b >= per * 8) return b;
    return (b & 7) * per + (b >> 3);
}

template <typename T, int TX, int TY, bool RING, bool SNAP>
__global__ void __launch_bounds__(TX * TY)
k_fused(const RepDesc *__restrict__ desc, const FusedTile *__restrict__ tiles, const T *__restrict__ pop,
        T *__restrict__ pop_out, const uint64_t *__restrict__ step, int koff, int *__restrict__ err,
        float *__restrict__ snap, int64_t total) {
    constexpr int EX = TX + 4, EP = EX * (TY + 4);
    constexpr int MX = TX + 2, MP = MX * (TY + 2);
    __shared__ float s_rho[5][EP];
    __shared__ float s_mu[4][MP];

    const FusedTile tl = tiles[xcd_tile(blockIdx.x, gridDim.x)];
    const RepDesc &d = desc[tl.rep];
    const int L = d.L;
    const uint32_t N = (uint32_t)d.N, LL = (uint32_t)(L * L);
    const T *base = pop + Q * d.site_off;
    T *obase = pop_out + Q * d.site_off;
    const uint64_t t = *step + (uint64_t)koff;
    const bool force_on = !(d.flags & 1);

    const int tid = threadIdx.x;
    const int ix = tid % TX, iy = tid / TX;
    const int nx = tl.nx, ny = tl.ny;
    const bool inner = ix < nx && iy < ny;
    const int sx = tl.x0 + (inner ? ix : 0), sy = tl.y0 + (inner ? iy : 0);
    const uint32_t site_c = (uint32_t)(sx + sy * L);  // in-plane site index (noise counter)
    PlaneOffs io;
    io.set(sx, sy, L, sizeof(T));
    const int r_in = (iy + 2) * EX + (ix + 2);  // LDS density index of the site
    const int m_in = (iy + 1) * MX + (ix + 1);  // LDS potential index of the site

    // density halo: ring of the (nx+4) x (ny+4) extension, at most two sites
    // per thread; positions packed as (hy << 16) | hx, offsets formed per plane
    constexpr int NT = TX * TY;
    const int ew = nx + 4;
    const int nhalo = 4 * (nx + ny) + 16;
    auto halo_pos = [&](int h) {
        int hx, hy;
        if (h < 2 * ew) {
            hy = h / ew;
            hx = h - hy * ew;
        } else if (h < 4 * ew) {
            h -= 2 * ew;
            hy = ny + 2 + h / ew;
            hx = h - (h / ew) * ew;
        } else {
            h -= 4 * ew;
            hy = 2 + (h >> 2);
            const int k = h & 3;
            hx = k < 2 ? k : nx + k;
        }
        return (uint32_t)((hy << 16) | hx);
    };
    const bool has_h = tid < nhalo, has_h2 = tid + NT < nhalo;
    const uint32_t hp0 = has_h ? halo_pos(tid) : 0u;
    const uint32_t hp1 = has_h2 ? halo_pos(tid + NT) : 0u;
    auto halo_density = [&](const T *const (&qz)[Q], float *rs, uint32_t hp) {
        const int hx = hp & 0xffff, hy = hp >> 16;
        PlaneOffs ho;
        ho.set(wrap_near(tl.x0 - 2 + hx, L), wrap_near(tl.y0 - 2 + hy, L), L, sizeof(T));
        float h[Q];
        pull_plane(qz, ho, h);
        rs[hy * EX + hx] = drho_of(h);
    };

    // potential halo: ring of the (nx+2) x (ny+2) extension
    const int mw = nx + 2;
    const int nmhalo = 2 * (nx + ny) + 4;
    const bool has_mh = tid < nmhalo;
    int mhx = 0, mhy = 0;
    if (has_mh) {
        int h = tid;
        if (h < mw) {
            mhy = 0;
            mhx = h;
        } else if (h < 2 * mw) {
            mhy = ny + 1;
            mhx = h - mw;
        } else {
            h -= 2 * mw;
            mhy = 1 + (h >> 1);
            mhx = (h & 1) ? nx + 1 : 0;
        }
    }
    const int m_h = mhy * MX + mhx;
    const int r_mh = (mhy + 1) * EX + (mhx + 1);

    bool bad = false;
    float A[Q], B[Q], C[Q];

    auto body = [&](int p, float(&ld)[Q], float(&cl)[Q]) {
        // (a) density of plane p
        {
            const int zc = wrap_near(p, L);
            const uint32_t Zc = (uint32_t)zc * LL, Zm = (uint32_t)wrap_dec(zc, L) * LL,
                           Zp = (uint32_t)wrap_inc(zc, L) * LL;
            const T *qz[Q];
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int cz = cz_of(q);
                qz[q] = base + (size_t)q * N + (cz > 0 ? Zm : (cz < 0 ? Zp : Zc));
            }
            float *rs = s_rho[(p + 10) % 5];
            if (inner) {
                if (RING) {
                    pull_plane(qz, io, ld);
                    rs[r_in] = drho_of(ld);
                } else {
                    float f[Q];
                    pull_plane(qz, io, f);
                    rs[r_in] = drho_of(f);
                }
            }
            if (has_h) halo_density(qz, rs, hp0);
            if (has_h2) halo_density(qz, rs, hp1);
        }
        __syncthreads();
        // (b) chemical potential of plane p - 1
        if (p - 1 >= tl.z0 - 1) {
            const float *r0 = s_rho[(p - 2 + 10) % 5], *r1 = s_rho[(p - 1 + 10) % 5], *r2 = s_rho[(p + 10) % 5];
            float *ms = s_mu[(p - 1 + 8) & 3];
            auto mu_at = [&](int ri) {
                const float c = r1[ri];
                return chem_potential(d, c, lap18(c, [&](int dx, int dy, int dz) {
                                          const float *pl = dz < 0 ? r0 : (dz > 0 ? r2 : r1);
                                          return pl[ri + dy * EX + dx];
                                      }));
            };
            if (inner) ms[m_in] = mu_at(r_in);
            if (has_mh) ms[m_h] = mu_at(r_mh);
        }
        __syncthreads();
        // (c) collision of plane z = p - 2
        if (p - 2 >= tl.z0 && inner) {
            const int z = p - 2;
            float Fx = 0.f, Fy = 0.f, Fz = 0.f;
            if (force_on) {
                const float *rm = s_rho[(z - 1 + 10) % 5], *rc = s_rho[(z + 10) % 5], *rp = s_rho[(z + 1 + 10) % 5];
                const float *mm = s_mu[(z - 1 + 8) & 3], *mc = s_mu[(z + 8) & 3], *mp = s_mu[(z + 1 + 8) & 3];
                const float rho_x = d.rho_c + rc[r_in];
                const Grad18 gr = grad18([&](int dx, int dy, int dz) {
                    const float *rr = dz < 0 ? rm : (dz > 0 ? rp : rc);
                    const float *mu = dz < 0 ? mm : (dz > 0 ? mp : mc);
                    return (1.0f / 3.0f) * rr[r_in + dy * EX + dx] - rho_x * mu[m_in + dy * MX + dx];
                });
                Fx = gr.gx;
                Fy = gr.gy;
                Fz = gr.gz;
            }
            if (!RING) {  // pull plane z again (served by L2 / the last-level cache)
                const int zc = wrap_near(z, L);
                const uint32_t Zc = (uint32_t)zc * LL, Zm = (uint32_t)wrap_dec(zc, L) * LL,
                               Zp = (uint32_t)wrap_inc(zc, L) * LL;
                const T *qz[Q];
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    const int cz = cz_of(q);
                    qz[q] = base + (size_t)q * N + (cz > 0 ? Zm : (cz < 0 ? Zp : Zc));
                }
                pull_plane(qz, io, cl);
            }
            const uint32_t s = site_c + (uint32_t)z * LL;
            const SiteNoise noise{s, (uint32_t)t, (uint32_t)(t >> 32), d.key0, d.key1};
            if constexpr (SNAP) write_snapshot(snap, total, d.site_off + (int64_t)s, cl);
            const float rho = collide_site(d, cl, Fx, Fy, Fz, noise);
            bad |= !(rho > 0.0f && rho < 1e30f);  // Sec. III B: rho must stay positive
            T *oz = obase + (uint32_t)z * LL;
#pragma unroll
            for (int q = 0; q < Q; ++q) stb(oz + (size_t)q * N, io.c, cl[q]);
        }
    };

    const int p0 = tl.z0 - 2, pend = tl.z0 + tl.nz + 1;
    for (int p = p0; p <= pend; p += 3) {
        body(p, A, B);
        if (p + 1 <= pend) body(p + 1, B, C);
        if (p + 2 <= pend) body(p + 2, C, A);
    }
    if (bad) *err = 1;
}

// ---------------------------------------------------------------------------
// Staged variant (FP32 storage): the pulls of plane p + 1 (tile and halo) are
// issued as asynchronous global-to-LDS loads as soon as plane p has been
// consumed, so their latency hides behind the potential and collision
// phases of plane p; no registers hold loads in flight.  The arithmetic is
// the same function calls in the same order as k_fused.
// ---------------------------------------------------------------------------
typedef __attribute__((address_space(1))) const void *gptr_t;
typedef __attribute__((address_space(3))) void *lptr_t;

__device__ __forceinline__ uint32_t pull_off(int q, const PlaneOffs &o) {
    switch (q) {
    case 1: case 11: case 13: return o.xm;
    case 2: case 12: case 14: return o.xp;
    case 3: case 15: case 17: return o.ym;
    case 4: case 16: case 18: return o.yp;
    case 7: return o.mm;
    case 8: return o.pp;
    case 9: return o.mp;
    case 10: return o.pm;
    default: return o.c;
    }
}

//
// ROWS selects how plane p + 1 is staged.  false (FP32 only): every thread
// loads the 19 pulled values of its tile site, and threads of the first
// waves those of one halo site each (dword per lane, the slot of a value is
// its site).  true: for each population the workgroup copies the unshifted
// source rectangle that the pulls of the tile and its two-site halo read,
// TY + 4 rows of TX + 2 CH columns starting at x0 - CH, with CH = 4 floats
// or 8 halves per 16-byte load (aligned when L is a multiple of CH); the
// loads are spread over all waves, and a pulled value is then the
// rectangle entry at the site's row and at column ex + CH - 2 - cx_q.  The
// rows mode issues about a quarter of the load instructions for the same
// data.  Tiles of 512 threads (64 x 8) have eight waves; the rest four.
// 512-thread tiles fit two workgroups per CU (LDS and at most 128 VGPRs)
// in every instance the host launches; the build checks the VGPR count (a
// launch-bounds hint to the same effect made the compiler's code slower)
template <typename T, int TX, int TY, bool ROWS, bool SNAP>
__global__ void __launch_bounds__(TX * TY)
k_fused_staged(const RepDesc *__restrict__ desc, const FusedTile *__restrict__ tiles, const T *__restrict__ pop,
               T *__restrict__ pop_out, const uint64_t *__restrict__ step, int koff, int *__restrict__ err,
               float *__restrict__ snap, int64_t total) {
    static_assert(ROWS || sizeof(T) == 4, "the per-site staging copies whole dwords");
    constexpr int NT = TX * TY;
    constexpr int NW = NT / 64;
    constexpr int EX = TX + 4, EP = EX * (TY + 4);
    constexpr int MX = TX + 2, MP = MX * (TY + 2);
    constexpr int NH_MAX = 4 * (TX + TY) + 16;
    // per-site staging loads one halo site per thread; the rows staging only
    // reads halo values from LDS and lets a thread take a second halo site
    static_assert(NH_MAX <= NT || (ROWS && NH_MAX <= 2 * NT), "halo sites per thread");
    constexpr bool H2 = NH_MAX > NT;
    constexpr int NHW = (std::min(NH_MAX, NT) + 63) / 64;  // waves that load halo sites
    // rows mode: source rectangle of RW values per row (CH values in a 16-byte
    // chunk, CH columns of margin each side), CW chunks per row
    constexpr int CH = 16 / (int)sizeof(T);
    constexpr int RW = TX + 2 * CH, CW = RW / CH, NL = CW * (TY + 4), NM = (NL + 63) / 64;
    constexpr int NS = ROWS ? CH * NL : NT + NHW * 64;  // staged values per population
    // rings: densities of planes p - 2 .. p, potentials of p - 2 .. p - 1;
    // what the collision of plane z needs from plane z - 1 is taken into
    // registers one iteration earlier (psi_m), so those planes can go
    __shared__ T s_stage[Q][NS];
    __shared__ float s_rho[3][EP];
    __shared__ float s_mu[2][MP];
    auto rslot = [](int p) { return (p + 9) % 3; };  // p >= -2
    auto mslot = [](int p) { return (p + 8) & 1; };

    const FusedTile tl = tiles[xcd_tile(blockIdx.x, gridDim.x)];
    const RepDesc &d = desc[tl.rep];
    const int L = d.L;
    const uint32_t N = (uint32_t)d.N, LL = (uint32_t)(L * L);
    const T *base = pop + Q * d.site_off;
    T *obase = pop_out + Q * d.site_off;
    const uint64_t t = *step + (uint64_t)koff;
    const bool force_on = !(d.flags & 1);

    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int ix = tid % TX, iy = tid / TX;
    const int nx = tl.nx, ny = tl.ny;
    const bool inner = ix < nx && iy < ny;
    const int sx = tl.x0 + (inner ? ix : 0), sy = tl.y0 + (inner ? iy : 0);
    const uint32_t site_c = (uint32_t)(sx + sy * L);
    PlaneOffs io;
    io.set(sx, sy, L, sizeof(T));
    const int r_in = (iy + 2) * EX + (ix + 2);
    const int m_in = (iy + 1) * MX + (ix + 1);

    // density halo sites of this thread (h = tid, and h = tid + NT for wide
    // tiles, while h < nhalo): two rows above, two below, two columns each side
    const int ew = nx + 4;
    const int nhalo = 4 * (nx + ny) + 16;
    auto halo_pos = [&](int h, int &px, int &py) {
        if (h < 2 * ew) {
            py = h / ew;
            px = h - py * ew;
        } else if (h < 4 * ew) {
            h -= 2 * ew;
            py = ny + 2 + h / ew;
            px = h - (h / ew) * ew;
        } else {
            h -= 4 * ew;
            py = 2 + (h >> 2);
            const int k = h & 3;
            px = k < 2 ? k : nx + k;
        }
    };
    const bool has_h = tid < nhalo;
    int hx = 0, hy = 0;
    if (has_h) halo_pos(tid, hx, hy);
    const bool has_h2 = H2 && tid + NT < nhalo;
    int hx2 = 0, hy2 = 0;
    if (has_h2) halo_pos(tid + NT, hx2, hy2);
    const int r_h2 = hy2 * EX + hx2;
    PlaneOffs ho;
    ho.set(wrap_near(tl.x0 - 2 + hx, L), wrap_near(tl.y0 - 2 + hy, L), L, sizeof(T));
    const int r_h = hy * EX + hx;

    // potential halo
    const int mw = nx + 2;
    const int nmhalo = 2 * (nx + ny) + 4;
    const bool has_mh = tid < nmhalo;
    int mhx = 0, mhy = 0;
    if (has_mh) {
        int h = tid;
        if (h < mw) {
            mhy = 0;
            mhx = h;
        } else if (h < 2 * mw) {
            mhy = ny + 1;
            mhx = h - mw;
        } else {
            h -= 2 * mw;
            mhy = 1 + (h >> 1);
            mhx = (h & 1) ? nx + 1 : 0;
        }
    }
    const int m_h = mhy * MX + mhx;
    const int r_mh = (mhy + 1) * EX + (mhx + 1);

    // does this wave store populations (then 19 stores may be younger than
    // the staged loads when it next waits for them)
    const bool wave_stores = __builtin_amdgcn_readfirstlane((int)(__ballot(inner) != 0)) != 0;

    // rows mode: the chunks this lane copies, one per 64-lane slice m of the
    // NL chunks of a population: byte offsets of its column and of its
    // unshifted row; the rows one above or below (y shifts cy = -1, 1) are
    // wrapped from it where a load needs them
    uint32_t r_col[NM], r_row[NM];
    bool r_on[NM];
    const uint32_t row_bytes = (uint32_t)L * sizeof(T), plane_bytes = LL * sizeof(T);
    if (ROWS) {
        const int lane = tid & 63;
#pragma unroll
        for (int m = 0; m < NM; ++m) {
            const int j = m * 64 + lane;
            r_on[m] = j < NL;
            const int ey = j / CW, k = j - (j / CW) * CW;
            r_col[m] = (uint32_t)(((tl.x0 - CH + CH * k) % L + L) % L) * sizeof(T);
            r_row[m] = (uint32_t)(((tl.y0 - 2 + ey) % L + L) % L) * row_bytes;
        }
    }
    // byte offset of the source row of a pull with y shift cy (row - cy)
    auto row_of = [&](uint32_t r, int cy) {
        if (cy > 0) return r == 0 ? plane_bytes - row_bytes : r - row_bytes;
        if (cy < 0) return r + row_bytes == plane_bytes ? 0u : r + row_bytes;
        return r;
    };

    auto issue = [&](int p) __attribute__((always_inline)) {
        const int zc = wrap_near(p, L);
        const uint32_t Zc = (uint32_t)zc * LL, Zm = (uint32_t)wrap_dec(zc, L) * LL,
                       Zp = (uint32_t)wrap_inc(zc, L) * LL;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int cz = cz_of(q);
            const char *bq = (const char *)(base + (size_t)q * N + (cz > 0 ? Zm : (cz < 0 ? Zp : Zc)));
            if (ROWS) {
                if (q % NW != wave) continue;  // populations are dealt round-robin to the waves
#pragma unroll
                for (int m = 0; m < NM; ++m)
                    if (r_on[m])
                        __builtin_amdgcn_global_load_lds((gptr_t)(bq + (row_of(r_row[m], cy_of(q)) + r_col[m])),
                                                         (lptr_t)&s_stage[q][m * 64 * CH], 16, 0, 0);
            } else {
                __builtin_amdgcn_global_load_lds((gptr_t)(bq + pull_off(q, io)), (lptr_t)&s_stage[q][wave * 64], 4,
                                                 0, 0);
                if (wave < NHW)
                    __builtin_amdgcn_global_load_lds((gptr_t)(bq + pull_off(q, ho)),
                                                     (lptr_t)&s_stage[q][NT + wave * 64], 4, 0, 0);
            }
        }
    };
    // LDS slot of the pulled value q of the tile site / the halo site
    // (rows: column ex + CH - 2 - cx_q of the rectangle for extended column ex)
    auto slot_in = [&](int q) { return ROWS ? (iy + 2) * RW + ix + CH - cx_of(q) : tid; };
    auto slot_h = [&](int q) { return ROWS ? hy * RW + hx + CH - 2 - cx_of(q) : NT + tid; };
    auto slot_h2 = [&](int q) { return hy2 * RW + hx2 + CH - 2 - cx_of(q); };

    // psi(y) = drho(y) / 3 - rho(x) mu(y), the force's summand (one
    // expression for every use, so every plan rounds alike)
    auto psi = [](float dr, float rho_x, float mu) { return (1.0f / 3.0f) * dr - rho_x * mu; };
    // psi at the five neighbours in plane z - 1 of the next collision's site:
    // (0,0), (-1,0), (1,0), (0,-1), (0,1) in x, y
    float psi_m[5] = {0.f, 0.f, 0.f, 0.f, 0.f};

    bool bad = false;
    float A[Q], B[Q], C[Q];
    bool stored_last = false;  // did the previous iteration issue stores (wave-uniform)

    auto body = [&](int p, float(&ld)[Q], float(&cl)[Q]) __attribute__((always_inline)) {
        // 1. staged pulls of plane p have landed (stores of the last collision,
        //    if any, are the only younger memory operations)
        if (stored_last) __builtin_amdgcn_s_waitcnt(vmcnt_wait(Q));  // the Q stores may still run
        else __builtin_amdgcn_s_waitcnt(vmcnt_wait(0));
        __syncthreads();
        {
            float *rs = s_rho[rslot(p)];
            if (inner) {
#pragma unroll
                for (int q = 0; q < Q; ++q) ld[q] = Store<T>::ld(s_stage[q], slot_in(q));
                rs[r_in] = drho_of(ld);
                // the sample snapshot of the pulled state of plane p (its
                // collision comes two iterations later, at the register peak)
                if constexpr (SNAP)
                    if (p >= tl.z0 && p < tl.z0 + tl.nz) {
                        // plane bases of the four snapshot arrays in scalar
                        // registers, the lane's in-plane offset added per store
                        float jx, jy, jz;
                        momentum_of(ld, jx, jy, jz);
                        const float *sp = snap + d.site_off + (int64_t)p * LL;
                        const float v[4] = {drho_of(ld), jx, jy, jz};
#pragma unroll
                        for (int c = 0; c < 4; ++c)
                            *(float *)((char *)sbase(sp + c * total) + site_c * 4u) = v[c];
                    }
            }
            if (has_h) {
                float h[Q];
#pragma unroll
                for (int q = 0; q < Q; ++q) h[q] = Store<T>::ld(s_stage[q], slot_h(q));
                rs[r_h] = drho_of(h);
            }
            if (H2 && has_h2) {
                float h[Q];
#pragma unroll
                for (int q = 0; q < Q; ++q) h[q] = Store<T>::ld(s_stage[q], slot_h2(q));
                rs[r_h2] = drho_of(h);
            }
        }
        __syncthreads();
        // 2. prefetch plane p + 1
        if (p + 1 <= tl.z0 + tl.nz + 1) issue(p + 1);
        // 3. chemical potential of plane p - 1
        if (p - 1 >= tl.z0 - 1) {
            const float *r0 = s_rho[rslot(p - 2)], *r1 = s_rho[rslot(p - 1)], *r2 = s_rho[rslot(p)];
            float *ms = s_mu[mslot(p - 1)];
            auto mu_at = [&](int ri) {
                const float c = r1[ri];
                return chem_potential(d, c, lap18(c, [&](int dx, int dy, int dz) {
                                          const float *pl = dz < 0 ? r0 : (dz > 0 ? r2 : r1);
                                          return pl[ri + dy * EX + dx];
                                      }));
            };
            if (inner) ms[m_in] = mu_at(r_in);
            if (has_mh) ms[m_h] = mu_at(r_mh);
        }
        __syncthreads();
        // 4. collision of plane z = p - 2
        stored_last = false;
        if (p - 2 >= tl.z0) {
            stored_last = wave_stores;
            if (inner) {
                const int z = p - 2;
                float Fx = 0.f, Fy = 0.f, Fz = 0.f;
                if (force_on) {
                    const float *rc = s_rho[rslot(z)], *rp = s_rho[rslot(z + 1)];
                    const float *mc = s_mu[mslot(z)], *mp = s_mu[mslot(z + 1)];
                    const float rho_x = d.rho_c + rc[r_in];
                    const Grad18 gr = grad18([&](int dx, int dy, int dz) {
                        if (dz < 0) return psi_m[dy == 0 ? (dx == 0 ? 0 : (dx < 0 ? 1 : 2)) : (dy < 0 ? 3 : 4)];
                        const float *rr = dz > 0 ? rp : rc;
                        const float *mu = dz > 0 ? mp : mc;
                        return psi(rr[r_in + dy * EX + dx], rho_x, mu[m_in + dy * MX + dx]);
                    });
                    Fx = gr.gx;
                    Fy = gr.gy;
                    Fz = gr.gz;
                }
                const uint32_t s = site_c + (uint32_t)z * LL;
                const SiteNoise noise{s, (uint32_t)t, (uint32_t)(t >> 32), d.key0, d.key1};
                const float rho = collide_site(d, cl, Fx, Fy, Fz, noise);
                bad |= !(rho > 0.0f && rho < 1e30f);  // Sec. III B: rho must stay positive
                T *oz = obase + (uint32_t)z * LL;
#pragma unroll
                for (int q = 0; q < Q; ++q) stb(oz + (size_t)q * N, io.c, cl[q]);
            }
        }
        // 5. plane p - 2 seen from the next collision (plane p - 1), before
        //    the next iteration overwrites it
        if (force_on && inner && p - 1 >= tl.z0 && p - 1 < tl.z0 + tl.nz) {
            const float *rz = s_rho[rslot(p - 2)], *mz = s_mu[mslot(p - 2)];
            const float rho_n = d.rho_c + s_rho[rslot(p - 1)][r_in];
            psi_m[0] = psi(rz[r_in], rho_n, mz[m_in]);
            psi_m[1] = psi(rz[r_in - 1], rho_n, mz[m_in - 1]);
            psi_m[2] = psi(rz[r_in + 1], rho_n, mz[m_in + 1]);
            psi_m[3] = psi(rz[r_in - EX], rho_n, mz[m_in - MX]);
            psi_m[4] = psi(rz[r_in + EX], rho_n, mz[m_in + MX]);
        }
    };

    const int p0 = tl.z0 - 2, pend = tl.z0 + tl.nz + 1;
    issue(p0);
    for (int p = p0; p <= pend; p += 3) {
        body(p, A, B);
        if (p + 1 <= pend) body(p + 1, B, C);
        if (p + 2 <= pend) body(p + 2, C, A);
    }
    if (bad) *err = 1;
}

// ---------------------------------------------------------------------------
// Host side: tile tables and launch.
// ---------------------------------------------------------------------------
inline bool fused_tile_ok(int tx, int ty) {
    return (tx == 16 && ty == 16) || (tx == 32 && ty == 8) || (tx == 16 && ty == 8) || (tx == 64 && ty == 4);
}

inline int make_fused_tiles(const std::vector<RepDesc> &reps, int tx, int ty, int tz,
                            std::vector<FusedTile> &out) {
    if (tx < 1 || ty < 1 || tz < 1 || tz > 1024) return -1;
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
    tx = 32;
    ty = 8;
    // six z slabs per column on large lattices: 2 x 768 tiles at L = 256
    // fill 256 CUs holding three workgroups each in two even rounds
    tz = maxL >= 128 ? (maxL + 5) / 6 : std::min(maxL, 16);
}

inline std::vector<std::array<int, 3>> fused_tile_candidates(const std::vector<RepDesc> &reps) {
    int maxL = 0;
    for (const auto &d : reps) maxL = std::max(maxL, d.L);
    std::vector<std::array<int, 3>> c;
    std::vector<int> tzs{16, 32, 64};
    for (int n : {3, 6})
        if ((maxL + n - 1) / n > 16 && std::find(tzs.begin(), tzs.end(), (maxL + n - 1) / n) == tzs.end())
            tzs.push_back((maxL + n - 1) / n);
    for (int tz : tzs)
        if (tz <= std::max(maxL, 16)) {
            c.push_back({64, 4, tz});
            c.push_back({64, 8, tz});
            c.push_back({32, 8, tz});
            c.push_back({16, 16, tz});
            c.push_back({32, 16, tz});  // taken by the paper's model only
        }
    if (maxL < 16) c.push_back({16, 16, maxL});
    return c;
}

#ifndef LBFSS_FUSED_RING
#define LBFSS_FUSED_RING 1
#endif
constexpr bool kFusedRing = LBFSS_FUSED_RING;

template <typename T, bool SNAP>
void launch_fused_snap(const RepDesc *desc, const FusedTile *tiles, int n_tiles, const T *in, T *out,
                       const uint64_t *step, int koff, int *err, int tx, int ty, hipStream_t stream, float *snap,
                       int64_t total) {
#define LBFSS_LAUNCH_FUSED(TX_, TY_)                                                                             \
    hipLaunchKernelGGL((k_fused<T, TX_, TY_, kFusedRing, SNAP>), dim3(n_tiles), dim3(TX_ * TY_), 0, stream, desc, \
                       tiles, in, out, step, koff, err, snap, total)
    if (tx == 16 && ty == 16) LBFSS_LAUNCH_FUSED(16, 16);
    else if (tx == 16 && ty == 8) LBFSS_LAUNCH_FUSED(16, 8);
    else if (tx == 64 && ty == 4) LBFSS_LAUNCH_FUSED(64, 4);
    else LBFSS_LAUNCH_FUSED(32, 8);
#undef LBFSS_LAUNCH_FUSED
}

// snap: where the step also writes the sample snapshot of its input state,
// or null (a separate instance without the snapshot's registers)
template <typename T>
void launch_fused(const RepDesc *desc, const FusedTile *tiles, int n_tiles, const T *in, T *out,
                  const uint64_t *step, int koff, int *err, int tx, int ty, hipStream_t stream, float *snap,
                  int64_t total) {
    if (snap) launch_fused_snap<T, true>(desc, tiles, n_tiles, in, out, step, koff, err, tx, ty, stream, snap, total);
    else launch_fused_snap<T, false>(desc, tiles, n_tiles, in, out, step, koff, err, tx, ty, stream, snap, total);
}

inline bool staged_tile_ok(int tx, int ty) {
    return (tx == 16 && ty == 16) || (tx == 32 && ty == 8) || (tx == 16 && ty == 8);
}

// the rows staging also takes 64 x 4 tiles (two halo sites for some threads)
// and 64 x 8 tiles (512 threads: fewer halo rows per site; two workgroups
// per CU)
inline bool rows_tile_ok(int tx, int ty) {
    return staged_tile_ok(tx, ty) || (tx == 64 && ty == 4) || (tx == 64 && ty == 8);
}

// With FP32 storage the snapshot instance of the 512-thread rows kernel needs
// more than the 128 VGPRs of two workgroups per CU, so the sample steps of
// such a plan run on 64 x 4 tiles (three workgroups per CU; every tile shape
// gives the same bits), in three z slabs on large lattices.  Returns whether
// the plan (tx, ty, tz) takes such a table, and its shape.
inline bool rows_snap_tile(const std::vector<RepDesc> &reps, bool fp32, int tx, int ty, int tz, int &sx, int &sy,
                           int &sz) {
    if (!fp32 || tx * ty != 512) return false;
    int maxL = 0;
    for (const auto &d : reps) maxL = std::max(maxL, d.L);
    sx = 64;
    sy = 4;
    sz = maxL >= 128 ? (maxL + 2) / 3 : tz;
    return true;
}


template <typename T, bool ROWS, bool SNAP>
void launch_staged_snap(const RepDesc *desc, const FusedTile *tiles, int n_tiles, const T *in, T *out,
                        const uint64_t *step, int koff, int *err, int tx, int ty, hipStream_t stream, float *snap,
                        int64_t total) {
    if (tx == 16 && ty == 16)
        hipLaunchKernelGGL((k_fused_staged<T, 16, 16, ROWS, SNAP>), dim3(n_tiles), dim3(256), 0, stream, desc, tiles,
                           in, out, step, koff, err, snap, total);
    else if (tx == 16 && ty == 8)
        hipLaunchKernelGGL((k_fused_staged<T, 16, 8, ROWS, SNAP>), dim3(n_tiles), dim3(128), 0, stream, desc, tiles,
                           in, out, step, koff, err, snap, total);
    else if (ROWS && tx == 64 && ty == 4)
        hipLaunchKernelGGL((k_fused_staged<T, 64, 4, true, SNAP>), dim3(n_tiles), dim3(256), 0, stream, desc, tiles,
                           in, out, step, koff, err, snap, total);
    else if (ROWS && tx == 64 && ty == 8)
        hipLaunchKernelGGL((k_fused_staged<T, 64, 8, true, SNAP>), dim3(n_tiles), dim3(512), 0, stream, desc, tiles,
                           in, out, step, koff, err, snap, total);
    else
        hipLaunchKernelGGL((k_fused_staged<T, 32, 8, ROWS, SNAP>), dim3(n_tiles), dim3(256), 0, stream, desc, tiles,
                           in, out, step, koff, err, snap, total);
}

template <typename T, bool ROWS>
void launch_fused_staged(const RepDesc *desc, const FusedTile *tiles, int n_tiles, const T *in, T *out,
                         const uint64_t *step, int koff, int *err, int tx, int ty, hipStream_t stream, float *snap,
                         int64_t total) {
    if (snap)
        launch_staged_snap<T, ROWS, true>(desc, tiles, n_tiles, in, out, step, koff, err, tx, ty, stream, snap, total);
    else
        launch_staged_snap<T, ROWS, false>(desc, tiles, n_tiles, in, out, step, koff, err, tx, ty, stream, snap,
                                           total);
}

}  // namespace lbfss
