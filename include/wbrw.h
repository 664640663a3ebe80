/*
 * wbrw.h -- C ABI of the MI355X signed-particle Wigner branching random walk.
 *
 * The library advances ensembles of signed particles (x, k, sign) under the
 * Wigner branching random walk of Xiong & Shao ("The Wigner branching random
 * walk: efficient implementation and performance evaluation"): free flight
 * x += (hbar/m) k dt, jumps at a constant auxiliary rate gamma0 with exact
 * life-lengths (Sec. 3.2.1), kicks drawn from the majorant |F[V](2k)| of
 * Remark 3 (Sec. 4.2) with pair generation read as a probability (sp1) or as
 * a weight followed by a bootstrap filter (sp2, Sec. 3.3), periodic
 * annihilation on a uniform phase-space grid (Sec. 4.3, Alg. 3) and a density
 * readout (Eq. estimator, Sec. 2).  Every step runs in HIP kernels on one GPU.
 *
 * Memory: the caller owns all device memory.  wbrw_workspace_size() gives the
 * bytes of the single device workspace that wbrw_init() carves into particle
 * arrays, grids and control words; the library never allocates device memory
 * and never frees the workspace.  Host pointers in wbrw_config are read during
 * wbrw_init() only.
 *
 * Streams: every call enqueues work on the hip stream given to wbrw_init()
 * (NULL = legacy default stream) and returns without synchronising, except the
 * calls documented as synchronising.  A handle is not thread-safe.
 *
 * Errors: calls return WBRW_OK or a negative code.  Argument errors are
 * reported immediately.  Device-side conditions (capacity exceeded, family
 * depth limit) set sticky flags that the next synchronising call returns; the
 * ensemble is then invalid until the handle is re-initialised.
 *
 * Determinism: for a given configuration and seed, results are bit-identical
 * across runs and independent of launch shapes and of how many instances share
 * a handle (instance b is keyed by instance_offset + b).  Every sum over
 * particles is an exact integer sum: signs and sp2 weights in 2^-32 units,
 * tangents in 32.32 fixed point (each component D enters as trunc(D 2^32),
 * and a sum Q reads as (double)floor(Q / 2^32) + (Q mod 2^32) 2^-32), so no
 * result depends on the order in which the GPU adds them.
 */
#ifndef WBRW_H
#define WBRW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define WBRW_MAX_COMPONENTS 4

enum wbrw_status {
    WBRW_OK = 0,
    WBRW_EINVAL = -1,     /* invalid argument or configuration */
    WBRW_ECAPACITY = -2,  /* an instance outgrew its particle capacity */
    WBRW_EHIP = -3,       /* a HIP runtime call failed */
    WBRW_ESTATE = -4,     /* call not valid in this state (e.g. sticky device error) */
    WBRW_EDEPTH = -5,     /* a family tree within one step exceeded the depth limit */
    WBRW_ERANGE = -6      /* a non-finite position met at annihilation, or a tangent
                             component outside the fixed-point range |D| < 2^31 */
};

enum wbrw_strategy {
    WBRW_SP1 = 0,  /* pair generation with probability xi/gamma0 (Alg. 1, sp1 box) */
    WBRW_SP2 = 1   /* weighted pairs (Alg. 1, wp box) + bootstrap filter at annihilation */
};

enum wbrw_kernel_kind {
    WBRW_KERNEL_GAUSSIAN = 0,  /* V = H exp(-(x - x0)^2 / (2 w^2)), per-instance H, w, x0 */
    WBRW_KERNEL_TABLE = 1      /* tabulated |F[V](2q)| on uniform bins of q (shared by instances) */
};

/*
 * One component V_m of the potential (Eq. eq:M, Sec. 2).  The Wigner kernel
 * of a potential symmetric about its centre is
 *   V_W(x, q) = (2/(pi hbar)) F[V](2q) sin(2q r),  F[V](s) = int V(y) e^{-isy} dy
 * (Eq. wigner_kernel_Gaussian with the normalisation of Eq. Wigner_kernel),
 * with r = x1 - c (axis 0), x2 - c (axis 1) or x1 - x2 - c (axis 2), and the
 * kick acts along (1,0), (0,1) or (1,-1) respectively (Example 1).
 */
typedef struct wbrw_component {
    int32_t kind;            /* enum wbrw_kernel_kind */
    int32_t axis;            /* 0, 1 or 2 (only 0 when dim == 1) */
    double sign;             /* TABLE: sign of F[V] (+1 or -1) */
    double center;           /* TABLE: c */
    const double *table;     /* TABLE, host: |F[V](2 q_j)| >= 0 at bin midpoints, table_n values */
    int32_t table_n;         /* TABLE: number of bins, 1 .. 65536 */
    int32_t modulated;       /* GAUSSIAN: 1 = height H (mod_a + mod_b cos(mod_omega t + mod_phase)) */
    double q_lo, q_hi;       /* TABLE: kick range [q_lo, q_hi) */
    const double *H;         /* GAUSSIAN, host [n_instances]: barrier height (any sign, nonzero) */
    const double *width;     /* GAUSSIAN, host [n_instances]: w > 0 */
    const double *center_b;  /* GAUSSIAN, host [n_instances]: x0 */
    /* Time-varying height (Remark 1, Sec. 2): the kernel is evaluated at the
     * absolute time of each jump; a given gamma0 must be >= max_t xi_m(t) / 2. */
    double mod_a, mod_b, mod_omega, mod_phase;
    /* GAUSSIAN kick sampler: 0 = majorant |F[V](2q)| with pair probability
     * xi_hat |sin| / (2 gamma0) (Remark 3, Sec. 4.2); 1 = Alg. 4 (Sec. 4.2): pair
     * probability xi(x)/gamma0 from xi tabulated on 4097 points over |x - x0| in
     * [0, 8w] (midpoint quadrature, 8192 nodes) with linear interpolation, and
     * the kick by rejection from V_W^+(x, .) (at most 256 proposals; sp1 only,
     * static height, no tangents). */
    int32_t sampler;
    int32_t reserved2;
} wbrw_component;

typedef struct wbrw_config {
    int32_t dim;              /* 1: phase space (x, k); 2: (x1, x2, k1, k2) */
    int32_t strategy;         /* enum wbrw_strategy */
    int32_t n_components;     /* 1 .. WBRW_MAX_COMPONENTS */
    int32_t n_instances;      /* B, 1 .. 65536 independent ensembles */
    int32_t instance_offset;  /* instance b draws with key index instance_offset + b */
    int32_t track_tangent;    /* tangents d/d(H, w, x0) (dim 1, one static Gaussian component,
                                 majorant sampler).  0: none.  sp1: 1 = likelihood-ratio
                                 scores of the kick density and pair acceptance; 2 = the same
                                 for (H, w), and d/dx0 by derivative ghost pairs instead of
                                 the x0 score (finite variance).  sp2: 1 = pathwise weight
                                 derivatives with the kick-density score (finite variance);
                                 2 is rejected.  Ghosts branch by the sp1 rule. */
    uint32_t seed;            /* Philox key word */
    int32_t max_density_bins; /* largest nbins a later wbrw_density() may ask for */
    double hbar, mass;        /* free flight x += (hbar/mass) k dt */
    double dt;                /* time step */
    double gamma0;            /* > 0: auxiliary rate for every instance; <= 0: derived */
    double gamma_scale;       /* derived gamma0 = gamma_scale * max_m xi_m / 2 */
    wbrw_component comp[WBRW_MAX_COMPONENTS];
    const int64_t *N0;        /* host [n_instances]: initial particle counts (the sample size N_alpha) */
    const int64_t *capacity;  /* host [n_instances]: most particles an instance may hold, < 2^31 */
    int64_t ghost_capacity;   /* per instance, tangent ghosts (track_tangent only) */
    double init_mean_x[2], init_sigma_x[2], init_mean_k[2], init_sigma_k[2];
    const double *init_hist;  /* host [n_instances][N_h] or NULL: signed histogram d_nu of the
                                 initial Wigner function (cell order as the grid), sampled by
                                 Alg. 3 (Sec. 4.1) instead of the Gaussian f0 */
    double x_lo, x_hi;        /* annihilation grid and K box: every position axis */
    double k_lo, k_hi;        /* ... every wave-vector axis; offspring outside K are removed */
    int32_t nx, nk;           /* cells per position / wave-vector axis; N_h = nx nk (dim 1) or
                                 nx^2 nk^2 (dim 2) must be < 2^31 (sp2: < 2^30), else
                                 WBRW_EINVAL */
} wbrw_config;

typedef struct wbrw_stats {
    int64_t n;                /* particles held (sp1/sp2), excluding the ghost ensemble; with
                                 track_tangent 2 this includes the sign-0 derivative ghosts
                                 born since the last annihilation */
    int64_t n_ghost;          /* tangent ghosts held */
    int64_t events;           /* jumps so far */
    int64_t pairs;            /* offspring pairs generated so far */
    int64_t killed;           /* sp1: net sign removed by the K box; sp2: the same in 2^-32 units */
    int64_t escaped;          /* sp1: net sign outside the grid at annihilation; sp2: 2^-32 units */
    int64_t max_depth;        /* deepest family tree seen within one step */
    int64_t event_cap_hits;   /* particle-steps that reached the per-step jump cap (expected 0) */
    int64_t step;             /* steps completed */
    int64_t S_plus, S_minus;  /* sp2: last bootstrap's class weights, 2^-32 units */
    int64_t N_plus, N_minus;  /* sp2: last bootstrap's class sizes */
    int64_t particle_steps;   /* sum over steps of the particles held at the start of the step */
    double gamma0;            /* the instance's auxiliary rate */
    int64_t annihilations;    /* annihilations so far */
    int64_t triggered;        /* of those, run by wbrw_run_adaptive for the threshold alone */
} wbrw_stats_t;

/* Stages timed by the per-stage profiler. */
enum wbrw_stage {
    WBRW_STAGE_STREAM = 0,    /* clock test, free flight, event compaction */
    WBRW_STAGE_FAMILY = 1,    /* family trees of jumping particles */
    WBRW_STAGE_BIN = 2,       /* annihilation: cell sums */
    WBRW_STAGE_SCAN = 3,      /* annihilation: ordered scan */
    WBRW_STAGE_REGEN = 4,     /* annihilation: regeneration */
    WBRW_STAGE_BOOTSTRAP = 5, /* sp2 bootstrap filter */
    WBRW_STAGE_DENSITY = 6,   /* density readout */
    WBRW_STAGE_GHOST = 7,     /* tangent ghosts and ghost steps */
    WBRW_STAGE_EVENTS = 8,    /* step: ordered event list */
    WBRW_STAGE_PLACE = 9,     /* step: record placement */
    WBRW_STAGE_CLOSE = 10,    /* unused: the placement launch's first block closes the step */
    WBRW_STAGE_STEP = 11,     /* a whole step, all of its launches (brackets the others) */
    WBRW_STAGE_COUNT = 12
};

typedef struct wbrw_handle *wbrw_t;

/* Bytes of device workspace the configuration needs.  Host-only; no HIP calls.
 * Returns WBRW_EINVAL for an invalid configuration. */
int wbrw_workspace_size(const wbrw_config *cfg, size_t *bytes);

/* Validates cfg, lays the workspace out, derives gamma0 and the kernel
 * constants per instance (Sec. 4.2 Remark 3: xi_m = int |F[V_m](2q)| 2/(pi hbar) dq,
 * pair probability xi_m |sin| / (2 gamma0)), uploads them, and samples the
 * initial ensembles (x ~ N(mean_x, sigma_x), k ~ N(mean_k, sigma_k), sign +1,
 * id = index).  workspace: device pointer, 256-byte aligned, of at least
 * wbrw_workspace_size() bytes, owned by the caller and untouched by anyone
 * else until wbrw_destroy().  hip_stream: a hipStream_t or NULL.
 * Enqueues work; does not synchronise. */
int wbrw_init(const wbrw_config *cfg, void *workspace, size_t workspace_bytes,
              void *hip_stream, wbrw_t *out);

/* Advances every instance by nsteps time steps (Alg. 1 between t_l and
 * t_{l+1} = t_l + dt; Sec. 2).  Enqueues 4 kernels per step (streaming, event
 * list, families, record placement whose first block does the bookkeeping;
 * 8 with tangents, whose ghosts take a second such pass); no host
 * synchronisation. */
int wbrw_step(wbrw_t h, int32_t nsteps);

/* Annihilation (Sec. 4.3): particles outside the grid are removed (escaped
 * tally); sp1 sums the signs per cell exactly (Eq. signed_histogram) and
 * regenerates |n_nu| particles of sign sgn(n_nu) uniformly in each cell
 * (Alg. 3 without rounding); sp2 first applies the residual bootstrap to each
 * sign class (Alg. 2, Eqs. lambda and double_bootstrap), forms the cell value
 * of Eq. boostrap_histogram and rounds it stochastically (Alg. 3).  Output
 * order: ascending cell, then index within the cell.  No synchronisation. */
int wbrw_annihilate(wbrw_t h);

/* Runs nsteps steps with an annihilation after every step whose number is a
 * multiple of annihilate_every (steps counted from 0 at wbrw_init; 0 = never).
 * With use_graph != 0 (and a non-NULL stream) whole epochs of
 * annihilate_every steps + annihilation are captured once into a hipGraph and
 * replayed.  No synchronisation. */
int wbrw_run(wbrw_t h, int32_t nsteps, int32_t annihilate_every, int32_t use_graph);

/* Steps with resampling at the scheduled instants and whenever the particle
 * number is about to exceed a threshold (Sec. 5): after each of the nsteps
 * steps the ensemble is annihilated (as wbrw_annihilate) if the step count
 * is a multiple of annihilate_every (0 = no schedule) or if it holds more
 * than `limit` particles (0 = no threshold).  The decision is taken on the
 * device by the step's last kernel, and every annihilation kernel enqueued
 * after the step reads it, so a run needs no host round trip; with
 * use_graph != 0 (and a non-NULL stream) one step with its conditional
 * annihilation is captured once into a hipGraph and replayed.  A threshold
 * needs n_instances == 1 (instances must not resample each other);
 * track_tangent must be 0.  WBRW_EINVAL otherwise.  No synchronisation. */
int wbrw_run_adaptive(wbrw_t h, int32_t nsteps, int32_t annihilate_every, int64_t limit,
                      int32_t use_graph);

/* Position density (Eq. estimator with an indicator observable):
 * d_out[b * nbins + j] = sum_{particles of instance b in bin j} w / (N0_b dx),
 * dx = (hi - lo)/nbins over [lo, hi) of position axis `axis`; sp1 counts signs
 * exactly, sp2 sums weights in 2^-32 fixed point.  d_out: device, B*nbins
 * doubles, caller-owned.  nbins <= max_density_bins.  No synchronisation. */
int wbrw_density(wbrw_t h, int32_t axis, int32_t nbins, double lo, double hi, double *d_out);

/* Density readout that allocates nothing, for callers that cannot allocate
 * device memory (code under hipGraph capture, tight serving loops, harnesses
 * that forbid allocation).  Same result as wbrw_density, and nbins may exceed
 * max_density_bins: the per-XCD accumulators live in a library-owned device
 * array of 4 MiB (kXcd * n_instances * nbins int64 words, so
 * 8 * n_instances * nbins <= 524288, else WBRW_EINVAL) instead of the
 * workspace.  Each GPU holds one such array for the life of the process and
 * every call on that GPU shares it: the call clears it first, and calls that
 * overlap on one GPU (other streams or handles) race.  d_out: device,
 * caller-owned, B*nbins doubles.  No allocation, no synchronisation. */
int wbrw_density_noalloc(wbrw_t h, int32_t axis, int32_t nbins, double lo, double hi,
                         double *d_out);

/* Tangent density (track_tangent only): d_out[(b*3 + c) * nbins + j] =
 * sum over real particles and ghosts in bin j of D_c / (N0_b dx) (the sum in
 * 32.32 fixed point, see Determinism), an unbiased
 * estimate of the derivative of the density with respect to
 * theta = (H, w, x0) (likelihood-ratio scores; with track_tangent 2 the x0
 * part comes from derivative ghost pairs).  d_out: device, caller-owned.
 * No synchronisation. */
int wbrw_density_tangent(wbrw_t h, int32_t axis, int32_t nbins, double lo, double hi,
                         double *d_out);

/* Backward pass of the density (track_tangent only): grad_out[b*3 + c] =
 * sum_j g[b*nbins + j] d rho_bj / d theta_c, theta = (H, w, x0): the
 * per-particle tangents of real particles and ghosts are summed per bin j in
 * fixed point (as wbrw_density_tangent), then contracted with g over the bins
 * in ascending order and divided by N0_b dx.  nbins <= max_density_bins.
 * g, grad_out: device, caller-owned.  Same binning as wbrw_density.  No
 * synchronisation. */
int wbrw_density_vjp(wbrw_t h, int32_t axis, int32_t nbins, double lo, double hi,
                     const double *g, double *grad_out);

/* Checkpoint / resume.  wbrw_snapshot_size synchronises and gives the bytes a
 * snapshot of the current state needs (every instance's particles and ghosts,
 * counts, tallies, the step counter).  wbrw_snapshot copies that state into a
 * caller-owned device buffer (synchronises).  wbrw_restore makes a handle with
 * the same configuration continue exactly from a snapshot. */
int wbrw_snapshot_size(wbrw_t h, size_t *bytes);
int wbrw_snapshot(wbrw_t h, void *dst, size_t bytes);
int wbrw_restore(wbrw_t h, const void *src, size_t bytes);

/* Synchronises the stream, then writes instance b's statistics.  Returns a
 * sticky device error (WBRW_ECAPACITY, WBRW_EDEPTH, WBRW_ERANGE) if one was
 * raised. */
int wbrw_stats(wbrw_t h, int32_t b, wbrw_stats_t *out);

/* Synchronises and writes the particle count of instance b (ghost != 0: ghosts). */
int wbrw_count(wbrw_t h, int32_t b, int32_t ghost, int64_t *n);

/* Copies instance b's ensemble (ghost != 0: its tangent ghosts) into caller
 * device buffers, any of which may be NULL: x, k: [dim][n] doubles; sign: [n]
 * int8 (sp1 particles; ghosts in either strategy, where it is 0); w: [n]
 * doubles (sp2 particles only); id: [n] uint64 lineage ids; D: [n][3]
 * tangents (track_tangent only).  n must equal the current count
 * (wbrw_count).  WBRW_EINVAL if n differs or a requested field does not exist
 * for this ensemble.  Synchronises the handle's stream before and after. */
int wbrw_export(wbrw_t h, int32_t b, int32_t ghost, int64_t n, double *x, double *k,
                int8_t *sign, double *w, uint64_t *id, double *D);

/* Launch configuration of the plain step and annihilation: six int32,
 * {streaming blocks, family blocks, streaming threads per block, streaming
 * particles per thread, binning blocks, binning hash slots}.  The streaming
 * tile is always 2048 particles; the shapes offered are 256 x 8, 128 x 16
 * (1D only) and 512 x 4, the hash sizes 4096, 2048 and 8192 slots.  Results
 * do not depend on the configuration: every kernel's arithmetic and output
 * order are the same under all of them (the parallel scheme of Sec. 4 with
 * per-particle random streams). */
int wbrw_get_launch(wbrw_t h, int32_t *cfg);
/* cfg as above; WBRW_EINVAL for a shape or hash size not offered (for this
 * dimension) or a block count outside [1, 8192].  Synchronises the stream;
 * drops captured graphs. */
int wbrw_set_launch(wbrw_t h, const int32_t *cfg);

/* Autotuner.  Runs 2 * max(#streaming candidates, #family candidates) *
 * steps_per_candidate time steps of the handle's own ensemble (they are real
 * steps: results do not depend on launch shapes) while timing the streaming
 * kernel over its block shapes and grid sizes (blocks per compute unit) and
 * the family kernel over its grid sizes; for a plain sp1 ensemble it also
 * times the binning pass alone over its hash sizes and grids (its counts are
 * cleared and its escape tallies restored, so the ensemble and its stats are
 * unchanged).  Keeps the fastest of each.  chosen (host, may be NULL)
 * receives the launch configuration (wbrw_get_launch's six values).
 * Synchronises; drops captured graphs. */
int wbrw_autotune(wbrw_t h, int32_t steps_per_candidate, int32_t *chosen);

/* Per-stage timing with hip events recorded on the handle's stream around
 * every kernel of a stage and around every whole step (enable == 1 starts a
 * fresh measurement; enable == 2 the same with whole steps marked only, two
 * events per step; enable == 0 stops recording).  Not used inside graph
 * capture. */
int wbrw_profile(wbrw_t h, int32_t enable);

/* Synchronises, then writes for each stage s < WBRW_STAGE_COUNT the summed
 * kernel time in ms (ms[s]) and the number of timed launches (launches[s]). */
int wbrw_profile_read(wbrw_t h, double *ms, int64_t *launches);

/* Releases host-side state.  The workspace stays the caller's. */
int wbrw_destroy(wbrw_t h);

const char *wbrw_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* WBRW_H */
