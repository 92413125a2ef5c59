/*
 * lbfss — fluctuating non-ideal lattice Boltzmann (D3Q19) on AMD Instinct
 * MI355X (gfx950).  C ABI: plain pointers and sizes, no C++ or framework types.
 *
 * The model is the Langevin lattice-Boltzmann method of Gross & Varnik,
 * "Simulation of static critical phenomena in non-ideal fluids with the
 * Lattice Boltzmann method", Sec. III A (Eqs. (lbe), (mom), (lbnoise)), with
 * the Ginzburg-Landau free energy of Sec. II A (Eqs. (fef), (landau-pot)),
 * on a periodic three-dimensional D3Q19 lattice.  One time step:
 *   1. rho = sum_i f_i, j = sum_i c_i f_i                         (Eq. (mom))
 *   2. mu  = a (rho - rho_c) + b (rho - rho_c)^3 - kappa lap(rho) (Sec. II A)
 *   3. F   = -rho grad(mu) + c_s^2 grad(rho)   (the non-ideal pressure as a
 *            force, div P = rho grad(dF/dphi), with the ideal lattice-gas
 *            pressure cancelled; c_s^2 = 1/3)
 *   4. moment-space BGK collision with Guo forcing, u = (j + F/2)/rho, one
 *      relaxation time tau for every non-conserved moment (Eq. (lbe)), or
 *      separate times for the bulk and ghost moments (tau_bulk, tau_ghost)
 *   5. Gaussian noise on the 15 non-conserved moments a with variance
 *      rho kT (1/tau_a)(2 - 1/tau_a) N_a / c_s^2 (Eq. (lbnoise) at c_s^2 = 1/3);
 *      the normals come from Philox4x32-10 (Salmon et al., SC'11) with key
 *      (seed_lo, seed_hi) and counter (site, step_lo, call, step_hi), call
 *      0..3, through Box-Muller on pairs of uniforms ((w >> 9) + 1/2) 2^-23
 *   6. streaming f_i(r + c_i, t + 1) = f*_i(r, t)
 * Observables of the finite-size-scaling analysis are accumulated on sample
 * steps: block order-parameter moments (Sec. II B, Eqs. (mL), (ML), (chiL),
 * (chiL-lowT), (CL)) and the structure factor along the lattice axes
 * (Sec. IV A, Eq. (G-comput)), with phi = (rho - rho0)/rho0 and rho0 the
 * global mean density (Sec. II A, Eq. (op)).
 *
 * Lattice layout seen through this interface: site = x + L*(y + L*z);
 * populations are [19][L^3] in the velocity order
 *   0 (0,0,0); 1 (1,0,0) 2 (-1,0,0) 3 (0,1,0) 4 (0,-1,0) 5 (0,0,1) 6 (0,0,-1);
 *   7 (1,1,0) 8 (-1,-1,0) 9 (1,-1,0) 10 (-1,1,0) 11 (1,0,1) 12 (-1,0,-1)
 *   13 (1,0,-1) 14 (-1,0,1) 15 (0,1,1) 16 (0,-1,-1) 17 (0,1,-1) 18 (0,-1,1)
 * with weights 1/3, 1/18 (axis), 1/36 (diagonal).  The populations passed
 * in and out are the post-streaming f_i(r, t) of the current step t.
 *
 * Errors: every int-returning call returns LB_OK (0) or a negative LB_E*
 * code; lb_strerror names it.  LB_EUNSTABLE is sticky: once a kernel has
 * met rho <= 0 or a non-finite value (the positivity condition of Sec. III B,
 * Eq. (den_fluct_constr)), every later synchronising call returns it.
 *
 * Threads: a handle must not be used from two threads at once.  Handles are
 * independent of each other.
 * Streams: all device work of a handle is ordered on one HIP stream (its own
 * unless lb_set_stream gives another).  lb_step is asynchronous; lb_sync,
 * lb_moments, lb_fields and lb_set_populations synchronise that stream.
 * Determinism: results depend only on (L, parameters, seed, step count) of
 * each replica, never on the batch it runs in, the launch plan or the stream.
 */
#ifndef LBFSS_H
#define LBFSS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    LB_OK = 0,
    LB_EINVAL = -1,    /* an argument is out of range or inconsistent */
    LB_ENOMEM = -2,    /* a device or host allocation failed */
    LB_EDEVICE = -3,   /* a HIP runtime call failed (no device, launch error) */
    LB_EUNSTABLE = -4, /* sticky: rho <= 0 or a non-finite value was met */
    LB_ESTATE = -5     /* the call is not valid in the handle's current state */
};

/* storage of the populations in device memory (compute is always FP32):
 * the deviation (f_i - w_i rho_c) / w_i in IEEE binary32 or binary16 */
enum { LB_FP32 = 0, LB_FP16 = 1 };

/* lb_params.flags */
enum {
    LB_FORCE_OFF = 1,   /* F = 0: the ideal lattice gas (a test of the noise) */
    LB_EQ_PRESSURE = 2  /* the paper's own model (Sec. III A) on D3Q19: no force; the
                         * non-ideal pressure tensor of Eq. (press-th) carried by the
                         * equilibrium, whose second moment is Eq. (holdych-cond) (the
                         * scalar pressure on the moving populations, the rest one takes
                         * the remainder of rho), BGK with one tau (tau_bulk = tau_ghost =
                         * 0), and noise with the local-sound-speed covariance that keeps
                         * the stationary population covariance independent of the wave
                         * vector (on D2Q9 it is Eq. (lbnoise)): on the bulk moment and the
                         * fourth-order ghost, M_44 = 5/3 - 3 c_s^2, M_4,16 = 3 c_s^2 - 1,
                         * M_16,16 = 3 - 3 c_s^2 in units of 3 rho kT (1/tau)(2 - 1/tau),
                         * c_s^2 = rho (a + 3 b (rho - rho_c)^2); c_s^2 >= 1/2 with kT > 0
                         * raises LB_EUNSTABLE.  Mass and momentum are conserved exactly.
                         * Plans: LB_KERNEL_SPLIT (a density pass and a collide pass) or
                         * LB_KERNEL_ROWS (one z-marching pass with a one-site density
                         * halo; tiles (64,4), (32,8), (16,16), (64,8), (32,16)); the two
                         * give identical results.  FP32 storage only (at rest this model
                         * keeps nearly all mass on the rest population, so the stored
                         * deviations are O(1)); not with LB_FORCE_OFF; equal in a batch. */
};

#define LB_MAX_LEVELS 16

typedef struct {
    double a;          /* r of Eq. (landau-pot): coefficient of (rho - rho_c) in mu */
    double b;          /* u of Eq. (landau-pot): coefficient of (rho - rho_c)^3, >= 0 */
    double kappa;      /* square-gradient coefficient of Eq. (fef), >= 0 */
    double rho_c;      /* reference density rho_c > 0 of the Landau potential */
    double kT;         /* noise temperature k_B T >= 0 of Eq. (lbnoise) */
    double tau;        /* relaxation time, > 1/2 */
    double init_sigma; /* standard deviation of the initial density, >= 0 */
    int32_t storage;   /* LB_FP32 or LB_FP16 */
    int32_t sample_every; /* > 0: sample after every such step; 0: never */
    int32_t n_levels;  /* block edges L_b = L / 2^l, l = 1..n_levels while integer; 0 = all */
    int32_t flags;     /* LB_FORCE_OFF, LB_EQ_PRESSURE or 0 */
    int32_t series_capacity; /* per-sample records kept (ring buffer); 0 = none */
    int32_t hist_bins; /* > 0: histogram every level's box values m over this many equal
                        * bins of [-hist_range, hist_range) (<= LB_MAX_HIST_BINS); 0 = none */
    double hist_range; /* half-width of the histogram, > 0 when hist_bins > 0 */
    int32_t sk3_stride; /* > 0: on the samples at steps that are multiples of
                         * sample_every * sk3_stride also accumulate the 3D structure
                         * factor by shells (lb_sk3); 0 = never; equal in a batch */
    int32_t reserved;   /* must be 0 */
    double tau_bulk;    /* relaxation time of the bulk moment c^2 - 1 (0: tau) */
    double tau_ghost;   /* relaxation time of the ghost moments 10..18 (0: tau); the paper
                         * sets all times to one value (Sec. III B), which is the default */
} lb_params;

#define LB_MAX_HIST_BINS 4096

typedef struct {
    int32_t Lb;        /* box edge */
    int32_t reserved;
    int64_t n_boxes;   /* boxes per sample, (L / Lb)^3 */
    /* sums over all boxes of all samples of m, m^2, m^3, m^4, |m|, E, E^2 with
     * m = Lb^-3 sum_box phi (Eq. (mL)) and E = (2 Lb^3)^-1 sum_box phi^2 */
    double sum_m, sum_m2, sum_m3, sum_m4, sum_abs_m, sum_E, sum_E2;
} lb_level_sums;

typedef struct {
    int64_t step;        /* steps taken so far (the step counter of the noise) */
    int64_t n_samples;   /* samples accumulated since creation or lb_reset_moments */
    double mass;         /* sum of rho over the lattice now (FP64 reduction) */
    double momentum[3];  /* sum of j over the lattice now */
    int32_t L;           /* lattice edge of the replica */
    int32_t n_levels;    /* entries used in level[] */
    int32_t n_k;         /* axis modes per axis, L/2 - 1 */
    int32_t series_len;  /* records held in the ring, min(n_samples, capacity) */
    int32_t series_record; /* doubles per record, 5 + 7 n_levels */
    int32_t reserved;
    lb_level_sums level[LB_MAX_LEVELS]; /* coarsest (L/2) first */
} lb_moments_t;

typedef struct {
    int32_t n_replicas;
    int32_t storage;
    int64_t total_sites;   /* sum of L^3 over replicas */
    int64_t device_bytes;  /* device memory held by the handle */
    int64_t step;
    int32_t kernel;        /* plan in use: LB_KERNEL_* */
    int32_t tile_x, tile_y, tile_z; /* tile of the fused kernel */
    int32_t graph_steps;   /* steps captured per graph replay, 0 = direct launches */
    int32_t device;        /* HIP device ordinal */
} lb_info_t;

/* launch plans (results do not depend on the plan) */
enum {
    LB_KERNEL_SPLIT = 0,  /* density pass, chemical-potential pass, collide pass (with
                           * LB_EQ_PRESSURE: density pass, collide pass) */
    LB_KERNEL_FUSED = 1,  /* one z-marching pass, density halo in LDS, pulls in registers */
    LB_KERNEL_STAGED = 2, /* as FUSED, the next plane's pulls staged asynchronously in LDS
                           * (FP32 storage; FP16 handles run FUSED) */
    LB_KERNEL_ROWS = 3    /* as STAGED, the staging copies the source rows of each population
                           * with 16-byte loads (FP32 or FP16 storage); every L a multiple
                           * of 4 (FP32) or 8 (FP16), else LB_EINVAL.  FP32 plans on 64 x 8
                           * tiles run their sample steps on 64 x 4 tiles (same results) */
};

typedef struct {
    int32_t kernel;      /* LB_KERNEL_SPLIT, _FUSED, _STAGED or _ROWS */
    int32_t tile_x;      /* fused: tile edge along x; (tile_x, tile_y) in {(32,8), (16,16),
                          * (16,8), (64,4), (64,8)}, (64,4) not staged, (64,8) rows only;
                          * with LB_EQ_PRESSURE rows only, in {(64,4), (32,8), (16,16),
                          * (64,8), (32,16)}; clamped to L */
    int32_t tile_y;      /* fused: tile edge along y */
    int32_t tile_z;      /* fused: planes marched by one workgroup */
    int32_t graph_steps; /* > 0: capture this many steps in a HIP graph and replay
                          * it, rounded up to a multiple of the sampling period
                          * (sample_every, times sk3_stride when set, doubled if odd;
                          * 2 without sampling); LB_EINVAL if the rounded value
                          * exceeds 100000; 0: launch kernels directly */
    int32_t reserved;
} lb_plan;

typedef struct lb_sim lb_sim; /* opaque, owned by the library */

/* One periodic L^3 lattice (L >= 4) of the model of Sec. III A (Eq. (lbe):
 * BGK relaxation of f towards f^eq plus the noise of Eq. (lbnoise)), with the
 * Ginzburg-Landau parameters of Sec. II A, Eqs. (fef) and (landau-pot): a, b
 * and kappa are the r, u and kappa there, rho_c the density about which the
 * Landau potential is expanded.  Initial state: rho = rho_c +
 * init_sigma g with g the first Box-Muller normal of Philox call
 * (site, 0, 1 << 16, 0), u = 0, f_i = w_i rho.  *out receives the handle
 * (owned by the library until lb_destroy); p is read during the call only.
 * Initial plan: LB_KERNEL_ROWS where every L allows it (else FUSED, or SPLIT
 * with LB_EQ_PRESSURE); when the largest L is at least 256 (FP32) on 64 x 8
 * tiles in four z slabs (six from L = 512), from 128 to 255 (FP32) on 64 x 4
 * tiles in three, from 128 (FP16) on 64 x 8 tiles in six, from 128
 * (LB_EQ_PRESSURE) on 64 x 8 tiles in eight, else on 32 x 8 tiles; direct
 * launches (lb_set_plan and lb_tune change it; results do not depend on it).
 * Errors: LB_EINVAL for L < 4, L > 1024, tau <= 1/2, kT < 0, kappa < 0,
 * b < 0, rho_c <= 0, init_sigma < 0, bad storage, flags, sample_every < 0,
 * n_levels < 0 or series_capacity < 0; LB_ENOMEM; LB_EDEVICE. */
int lb_create(int L, const lb_params *p, uint64_t seed, lb_sim **out);

/* n >= 1 replicas advanced together, replica r of edge L[r], parameters
 * p[r] and seed seeds[r].  All replicas must share storage and sample_every.
 * Each replica evolves exactly as it would alone under lb_create. */
int lb_create_batch(int n, const int *L, const lb_params *p, const uint64_t *seeds, lb_sim **out);

/* Advance every replica by n >= 0 steps (asynchronous on the handle's stream).
 * One step is Eq. (lbe) of Sec. III A: the moments rho, j of the pulled
 * populations (Eq. (mom)), the chemical potential and the force of steps 2-3
 * of the file preamble, the moment-space collision with the noise of
 * Eq. (lbnoise) drawn at the current step counter, and streaming; on steps
 * after which the counter is a multiple of sample_every the observables of
 * lb_moments are accumulated.  LB_EINVAL for n < 0 or a NULL handle; launch
 * failures return LB_EDEVICE; instability shows at the next synchronising
 * call (sticky LB_EUNSTABLE). */
int lb_step(lb_sim *s, int64_t n);

/* Wait for the handle's work; LB_EUNSTABLE if the sticky flag is set. */
int lb_sync(lb_sim *s);

/* Accumulated observables of one replica (synchronising): the block
 * order-parameter sums of Sec. II B (Eq. (mL) for m over boxes of edge L_b,
 * from which Eqs. (ML), (chiL), (chiL-lowT) and (CL) are formed; the Binder
 * ratio <m^4>/<m^2>^2 likewise) and the axis structure factor of Sec. IV A,
 * Eq. (G-comput), with phi = (rho - rho0)/rho0 of Eq. (op), plus the current
 * mass and momentum (FP64 sums).  out: caller-owned; LB_EINVAL for a bad
 * replica index.  sk, if not NULL,
 * receives 3 * n_k doubles: sk[a * n_k + m - 1] = sum over samples of
 * L^-3 |sum_r phi e^{-i k_m r_a}|^2, k_m = 2 pi m / L, axis a = x, y, z.
 * series, if not NULL, receives series_len records (oldest first) of
 * series_record doubles: step, mass, momentum x, y, z, then per level
 * (coarsest first) the box means of m, m^2, m^3, m^4, |m|, E, E^2. */
int lb_moments(lb_sim *s, int replica, lb_moments_t *out, double *sk, double *series);

/* Order-parameter distribution P_L(m) of every level (Sec. II C, Eq. (PL-def):
 * the histogram of the box values m_L^(b) over all boxes of all samples).
 * counts: caller-owned, n_levels * (hist_bins + 2) entries, levels in the
 * order of lb_moments_t.level (coarsest first); per level the hist_bins bins
 * (box value m in bin k = floor((m + h) * (hist_bins / (2 h))), h =
 * hist_range), then the number of values below -h, then the number at or
 * above h.  Counts are exact integers, so batch and plan never change them.
 * Synchronises.  LB_ESTATE if the replica was created with hist_bins = 0. */
int lb_histogram(lb_sim *sim, int replica, uint64_t *counts);

typedef struct {
    int32_t Lb;          /* box edge */
    int32_t reserved;
    double P0;           /* density P_L(0): the bin holding 0, or the mean of the two bins
                          * meeting at 0; densities are count / (all counted values * width) */
    double chi_center;   /* L_b^3 / (2 pi kT P0^2): Eq. (PL-highT) at m = 0 */
    double m_max;        /* |centre| of the fullest bin (lowest on ties): M_L as the
                          * position of the maximum of P_L (Sec. IV C) */
    double P_max;        /* density of that bin */
    double chi_peak;     /* L_b^3 / (8 pi kT P_max^2): Eq. (PL-lowT) at m = M_L (Sec. IV C) */
    double chi_var;      /* L_b^3 (<m^2> - <m>^2) / kT: Eq. (chiL), from the moment sums */
    double chi_var_low;  /* L_b^3 (<m^2> - <|m|>^2) / kT: Eq. (chiL-lowT) */
    double m_fit;        /* |centre| of a Gaussian fitted to the fullest peak (Sec. IV C):
                          * weighted least squares of ln(count) against a quadratic in m
                          * over the contiguous bins around the fullest one holding at
                          * least exp(-2) of its count, weights = counts */
    double chi_fit;      /* L_b^3 s^2 / kT, s^2 the fitted variance less w^2 / 12
                          * (Sheppard's correction for bins of width w); NaN (and m_fit
                          * NaN) when fewer than 3 bins qualify or the curvature is >= 0 */
} lb_hist_est;           /* a zero denominator (empty bin, kT = 0) gives +inf */

/* Susceptibility estimates of every level of a replica from its histogram and
 * moment sums; out: caller-owned, n_levels entries (coarsest first).
 * Synchronises.  LB_ESTATE if hist_bins = 0 or no sample was taken. */
int lb_hist_estimates(lb_sim *sim, int replica, lb_hist_est *out);

/* Three-dimensional structure factor (Sec. IV A, Eq. (G-comput)),
 * C(k) = N^-1 |sum_r phi e^{-i k.r}|^2 at every k = 2 pi m / L, summed over
 * shells s = floor(|m| + 1/2) with m folded into (-L/2, L/2]; shell 0 is
 * k = 0 (excluded, no modes).  Shell geometry of one replica: n_shells
 * (including shell 0), and, where the arrays are not NULL (n_shells entries
 * each), the number of modes, the mean continuum k^2 and the mean lattice
 * Laplacian symbol 6 sum_i w_i (1 - cos k.c_i) of every shell.
 * LB_ESTATE if the replica has sk3_stride = 0. */
int lb_sk3_shells(lb_sim *sim, int replica, int32_t *n_shells, int64_t *modes, double *k2_mean,
                  double *lap_mean);

/* Accumulated shell sums of C(k) (sum over the shell's modes and the samples
 * taken, n_samples of them) of one replica; sum_C has n_shells entries.
 * Synchronises.  LB_ESTATE if sk3_stride = 0. */
int lb_sk3(lb_sim *sim, int replica, int64_t *n_samples, double *sum_C);

typedef struct {
    double chi;      /* 1 / (kT A): C(0) = kT chi */
    double xi;       /* sqrt(B / A), NaN if B / A < 0 */
    double C0;       /* 1 / A */
    double A, B;     /* fit 1/C = A + B x */
    int32_t n_used;  /* shells in the fit */
    int32_t reserved;
} lb_oz_t;

/* Ornstein-Zernike fit of Eq. (CMF), C = kT chi / (1 + xi^2 k^2), to the
 * shell means C_s = sum_C / (modes n_samples): weighted least squares of
 * 1/C_s = A + B x_s over the shells s >= 1 with sqrt(mean k^2) <= k_max,
 * weight modes_s C_s^2; x = mean k^2 (x_lattice = 0) or the mean lattice
 * Laplacian symbol (x_lattice = 1), which Sec. IV A names as the k^2 of the
 * discrete model.  LB_ESTATE without samples or with fewer than 2 shells. */
int lb_oz_fit(lb_sim *sim, int replica, double k_max, int x_lattice, lb_oz_t *out);

/* Current fields of one replica copied to host memory owned by the caller
 * (synchronising); any pointer may be NULL.  rho and j are the moments of
 * Eq. (mom) (Sec. III A) of the post-streaming populations, summed in FP64:
 * rho: L^3 doubles, j: 3 L^3 ([3][L^3]), f: 19 L^3 ([19][L^3]) populations
 * f_i(r, t) in the velocity order above.  LB_EINVAL for a bad replica,
 * LB_ENOMEM when the device staging buffers cannot be had. */
int lb_fields(lb_sim *s, int replica, double *rho, double *j, double *f);

/* lb_fields for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same outputs, bit for bit, with the FP64 staging of the exported fields
 * in a static device array of 2^22 doubles (32 MiB) per GPU, held until the
 * process ends, instead of per-call allocations.  The requested outputs must
 * fit it: L^3 ((rho != NULL) + 3 (j != NULL) + 19 (f != NULL)) <= 2^22, else
 * LB_EINVAL (L <= 56 with f; L <= 101 for rho and j).  Every call on one GPU
 * shares that GPU's array: calls that overlap on one GPU (other threads,
 * other handles, other streams) race, so the caller serialises them.
 * Synchronising; errors as lb_fields. */
int lb_fields_static(lb_sim *s, int replica, double *rho, double *j, double *f);

/* Replace the populations of one replica by f ([19][L^3] doubles, post-
 * streaming, host memory), rounded to the storage precision.  The step
 * counter and accumulators are kept (synchronising). */
int lb_set_populations(lb_sim *s, int replica, const double *f);

/* Set the step counter of every replica to t >= 0: the populations held are
 * then the post-streaming f_i(r, t), and the next step draws the noise of
 * Eq. (lbnoise) from counters (site, t_lo, call, t_hi), t_lo and t_hi the low
 * and high 32-bit words of t.  With lb_fields (f) and lb_set_populations this
 * resumes a run exactly: a handle created with the same L, parameters and
 * seed, given the populations and step count of another, continues that run
 * bit for bit (FP32 and FP16 storage round-trip exactly through the FP64
 * populations).  A sample due on the current state is taken first; the state
 * at the new step is not sampled (sampling resumes after the next step that
 * ends on a multiple of sample_every); the accumulators are kept.
 * Synchronises.  LB_EINVAL for t < 0. */
int lb_set_step(lb_sim *s, int64_t t);

/* Zero every replica's accumulators, sample count and series. */
int lb_reset_moments(lb_sim *s);

/* Order all later device work of the handle on hip_stream (a hipStream_t;
 * NULL selects the handle's own stream).  Synchronises the previous stream. */
int lb_set_stream(lb_sim *s, void *hip_stream);

/* Device allocator used by handles created afterwards (process-wide; each
 * handle keeps the one it was created with until lb_destroy).  alloc(bytes,
 * ctx) returns device memory or NULL; free_(ptr, ctx) releases it.  Both
 * NULL restore hipMalloc / hipFree; exactly one NULL is LB_EINVAL.  Not
 * synchronised: call it while no other thread creates handles. */
int lb_set_allocator(void *(*alloc)(size_t, void *), void (*free_)(void *, void *), void *ctx);

/* Launch plan; LB_EINVAL for unknown kernels or tiles. */
int lb_set_plan(lb_sim *s, const lb_plan *plan);
int lb_get_plan(lb_sim *s, lb_plan *plan);

/* Autotuner: time each candidate plan (split; fused, staged and rows tiles
 * by z depth; each with and without graphs) over `steps` steps, time the
 * three fastest once more, keep the one with the best time and report it
 * in *best (may be NULL).  The timed steps are taken: the state advances by
 * their number (lb_info's step).  Results are plan-independent, so tuning
 * changes no result beyond that advance. */
int lb_tune(lb_sim *s, int steps, lb_plan *best);

int lb_info(lb_sim *s, lb_info_t *out);

/* Release every resource of the handle (NULL is ignored). */
void lb_destroy(lb_sim *s);

/* The generator of the noise of Eq. (lbnoise) (its Gaussian random
 * variables), on counters the caller chooses; for testing the step kernels'
 * random numbers against an independent implementation.  For i < n: ctr[4i..4i+3]
 * and key[2i..2i+1] (host memory) give the Philox4x32-10 counter and key;
 * words[4i..4i+3] receives the four output words, uniforms[4i..4i+3] their
 * uniforms ((w >> 9) + 1/2) 2^-23, normals[4i..4i+3] the Box-Muller pairs
 * sqrt(-2 ln u0) (cos 2 pi u1, sin 2 pi u1), then the same of (u2, u3), as the
 * step kernels form them (host memory, caller-owned; any output may be NULL).
 * The model's counters are (site, t_lo, call | domain << 16, t_hi) with key
 * (seed_lo, seed_hi): domain 0, calls 0..3 for the collision noise; domain 1,
 * call 0 at t = 0 for the initial density.  Runs on the current device on a
 * stream of its own and synchronises.  LB_EINVAL for n < 0, n > 2^24 or NULL
 * inputs with n > 0; LB_ENOMEM; LB_EDEVICE. */
int lb_philox(int64_t n, const uint32_t *ctr, const uint32_t *key, uint32_t *words, float *uniforms,
              float *normals);

/* Static description of an error code. */
const char *lb_strerror(int code);

/* ------------------------------------------------------------------------
 * The paper's own model (Sec. III A): fluctuating non-ideal D2Q9 lattice
 * Boltzmann on a periodic L x L lattice (site = x + L y), with the
 * Ginzburg-Landau thermodynamics carried by a modified equilibrium: its
 * second moment is the pressure tensor of Eq. (press-th) plus rho u u and the
 * Galilean correction of Eq. (holdych-cond); p0 = rho f0' - f0 with
 * f0 = a d^2/2 + b d^4/4, d = rho - rho_c; zero third-order ghost moments
 * and the fourth-order one 2 rho - 6 (p0 - kappa rho lap rho)
 * - 3 kappa |grad rho|^2 (the projection of the paper's explicit
 * equilibrium).  BGK relaxation, Eq. (lbe), with one tau; no body force, so
 * mass and momentum are conserved exactly.  Noise on the six non-conserved
 * moments with the covariance of Eq. (lbnoise) at the local squared sound
 * speed c_s^2 = rho (a + 3 b d^2), drawn through its Cholesky factor from
 * six normals of calls 0 and 1 of the same Philox generator (counter (site,
 * step_lo, call, step_hi), key (seed_lo, seed_hi)).  Velocity order:
 * 0 (0,0); 1 (1,0) 2 (-1,0) 3 (0,1) 4 (0,-1); 5 (1,1) 6 (-1,-1) 7 (1,-1)
 * 8 (-1,1).  Populations stored in FP32, arithmetic FP32, spectra FP64.
 * The calls follow the lb_* conventions (return codes, sticky LB_EUNSTABLE
 * for rho <= 0, a non-finite value or a covariance that is not positive
 * definite, i.e. c_s^2 >= 0.6).
 * ------------------------------------------------------------------------ */
typedef struct lb2_sim lb2_sim;

typedef struct {
    double a, b, kappa;  /* Landau r, u and the square-gradient coefficient */
    double rho_c;        /* reference density, > 0 */
    double kT;           /* noise temperature, >= 0 */
    double tau;          /* relaxation time, > 1/2 */
    double init_sigma;   /* standard deviation of the initial density, >= 0 */
    int32_t sample_every; /* > 0: accumulate the spectra after every such step */
    int32_t reserved;    /* must be 0 */
} lb2_params;

/* 4 <= L <= 2048.  The initial state is rho = rho_c + init_sigma g (Philox
 * domain 1, call 0, first normal), u = 0, the equilibrium of that density. */
int lb2_create(int L, const lb2_params *p, uint64_t seed, lb2_sim **out);

/* n >= 1 replicas of one lattice edge L in one handle, replica r with
 * parameters p[r] and seed seeds[r] (the paper averages over a few hundred
 * realizations, Sec. III B): each step is one launch over every replica's
 * tiles, and each replica evolves bit for bit as it does alone under
 * lb2_create.  All sample_every equal; n L^2 <= 2^31; else LB_EINVAL. */
int lb2_create_batch(int n, int L, const lb2_params *p, const uint64_t *seeds, lb2_sim **out);
int lb2_step(lb2_sim *s, int64_t n);   /* asynchronous; every replica */
int lb2_sync(lb2_sim *s);
/* Order all later device work of the handle on hip_stream (a hipStream_t;
 * NULL selects the handle's own stream), as lb_set_stream.  Synchronises
 * the previous stream; the caller keeps ownership of hip_stream, which must
 * outlive its use by the handle. */
int lb2_set_stream(lb2_sim *s, void *hip_stream);
/* rho (L^2), j ([2][L^2]) and f ([9][L^2]) of the current state of one
 * replica (0 for lb2_create); any may be NULL; caller-owned FP64 buffers;
 * synchronises.  LB_EINVAL for a bad replica index. */
int lb2_fields(lb2_sim *s, int replica, double *rho, double *j, double *f);
int lb2_set_populations(lb2_sim *s, int replica, const double *f);
/* Accumulated spectra of one replica over the samples, each [ky][kx] (L^2 doubles, k index
 * m in 0..L-1, wave number 2 pi m / L): S = <|drho_k|^2>/N, J_x, J_y =
 * <|j_a,k|^2>/N, J_par, J_perp = the same for the projections of j_k on the
 * direction of k (folded into (-L/2, L/2]) and across it (0 at k = 0):
 * sums over samples, n_samples of them.  Any array may be NULL. */
int lb2_spectra(lb2_sim *s, int replica, int64_t *n_samples, double *S, double *Jx, double *Jy, double *Jpar,
                double *Jperp);
int lb2_reset_spectra(lb2_sim *s);  /* every replica */
void lb2_destroy(lb2_sim *s);

#ifdef __cplusplus
}
#endif

#endif /* LBFSS_H */
