/*
 * wbrw_oracle.c -- plain, slow, FP64 CPU oracle for the signed-particle
 * Wigner branching random walk (Xiong & Shao, "The Wigner branching random
 * walk: efficient implementation and performance evaluation").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * loads this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code with the HIP path: the HIP side
 * implements the same arithmetic independently, and parity tests compare the
 * two element by element.
 *
 * What it computes, in the paper's order:
 *   - Alg. 1 (Sec. 2): the branching random walk over one time step, with a
 *     constant auxiliary rate gamma0, so the life-length is exactly
 *     tau = -ln(1-u)/gamma0 (Sec. 3.2.1).  Jumps sample the kick from the
 *     majorant |F[V](2k)| of Remark 3 (Sec. 4.2, Eq. majorant_approach) and
 *     read xi/gamma0 * |sin| as the pair-generation probability (sp1 box of
 *     Alg. 1; Sec. 3.1) or as the pair weight (wp/sp2 box of Alg. 1).
 *   - Eq. signed_histogram (Sec. 4.3) + Alg. 3 (Sec. 4.1): sp1 annihilation
 *     (exact integer count per cell, regeneration uniformly in the cell).
 *   - Alg. 2 + Eqs. lambda / double_bootstrap (Sec. 3.3) and
 *     Eq. boostrap_histogram + the rounding step of Alg. 3: sp2 annihilation.
 *   - Eq. estimator (Sec. 2): the density readout.
 *   - Likelihood-ratio tangents of the density with respect to the Gaussian
 *     barrier's (H, w, x0) (the differentiation form).
 *
 * Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), keyed by
 * (seed, instance) with counter (id_lo, id_hi, step, tag|event|sub), so each
 * particle lineage owns its own stream.  Elementary functions (log, sin, cos)
 * are written out from their series so that both implementations perform the
 * same IEEE operations; build with -ffp-contract=off.
 *
 * Parity status of each function is listed in the header comment of that
 * function ("pinned by" lines name the tests that tie it to the paper or to
 * mathematics independent of this file).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;
typedef __int128 i128;

#define ORC_MAXM 4
#define ORC_EMAX 4096u /* event cap per particle-step (never reached at the configs) */

enum { TAG_STEP = 0, TAG_REGEN = 1, TAG_INIT = 2, TAG_BOOT = 3, TAG_ROUND = 4,
       TAG_CHILD = 5, TAG_GHOST = 6, TAG_HIST = 7, TAG_REJECT = 8, TAG_DERIV = 9 };
#define ORC_XI_N 4096      /* xi(r) grid intervals over r in [0, 8w] (Alg. 4 sampler) */
#define ORC_XI_Q 8192      /* midpoint quadrature nodes over q in [-8/w, 8/w) */
#define ORC_REJECT_MAX 256 /* proposals per kick before the pair is dropped */
enum { KIND_GAUSS = 0, KIND_TABLE = 1 };
enum { STRAT_SP1 = 0, STRAT_SP2 = 1 };

/* ------------------------------------------------------------------------ */
/* Configuration (mirrored by the ctypes Structure in oracle/oracle.py).     */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t dim;            /* 1: phase space (x,k); 2: (x1,x2,k1,k2) */
    int32_t strategy;       /* STRAT_SP1 or STRAT_SP2 */
    int32_t M;              /* kernel components */
    int32_t B;              /* instances */
    int32_t instance_offset;/* key index of instance 0 (lets one instance replay instance b) */
    int32_t track_tangent;  /* single Gaussian component.  sp1: 1 = LR tangents;
                             * 2 = the same for (H, w), and the x0 tangent by
                             * derivative ghost pairs (see deriv_pairs).
                             * sp2: 1 = pathwise weight tangents (see walk) */
    uint32_t seed;
    int32_t pad0;
    double hbar, mass, dt, gamma0, gamma_scale;
    int32_t comp_kind[ORC_MAXM];
    int32_t comp_axis[ORC_MAXM];   /* 0: e=(1,0) r=x1-c; 1: e=(0,1) r=x2-c; 2: e=(1,-1) r=x1-x2-c */
    double comp_sgn[ORC_MAXM];     /* table kind: sign of the Fourier transform */
    double comp_center[ORC_MAXM];  /* table kind: centre c */
    const double *table[ORC_MAXM]; /* table kind: |F[V_m](2 q_j)| at bin midpoints */
    int32_t table_n[ORC_MAXM];
    double table_qlo[ORC_MAXM], table_qhi[ORC_MAXM];
    const double *H, *width, *center; /* Gaussian kind: per instance, [B*M] */
    const int64_t *N0;                /* [B] */
    double init_mean_x[2], init_sigma_x[2], init_mean_k[2], init_sigma_k[2];
    double x_lo, x_hi, k_lo, k_hi;
    int32_t nx, nk;
    /* time-dependent Gaussian heights (Remark 1): H_m(t) = H_m (a + b cos(omega t + phase)) */
    int32_t time_dependent, pad1;
    double mod_a[ORC_MAXM], mod_b[ORC_MAXM], mod_omega[ORC_MAXM], mod_phase[ORC_MAXM];
    /* initial data: 0 = Gaussian f0 sampled exactly; 1 = signed histogram d_nu on
     * the grid ([B][N_h] values of the Wigner function), sampled by Alg. 3 */
    int32_t init_kind, pad2;
    const double *init_hist;
    /* kick sampler per component: 0 = majorant of Remark 3; 1 = Alg. 4
     * (xi(x) on a grid with linear interpolation, rejection from V_W^+) */
    int32_t sampler[ORC_MAXM];
} orc_config;

typedef struct {
    int64_t n, n_plus, n_minus, n_ghost;
    int64_t net;          /* sp1: sum of signs of real particles */
    int64_t escaped;      /* sp1: net sign removed at annihilation; sp2: Q32 weight */
    int64_t killed;       /* sp1: net sign of offspring outside K; sp2: Q32 weight */
    int64_t pairs, events, event_cap_hits, max_depth;
    int64_t S_plus, S_minus, N_plus, N_minus; /* last sp2 bootstrap */
    double gamma0;
    int64_t step;
    int64_t range_errors; /* tangent components outside the fixed-point range of fx_add */
    int64_t annihilations, triggered; /* orc_run_adaptive: annihilations, and those the
                                         threshold alone called for */
} orc_stats;

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 from its published definition.  Pinned by                   */
/* tests/test_oracle_rng.py (against rocRAND's host implementation).         */
/* ------------------------------------------------------------------------ */
void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; round++) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* 53-bit uniform on [0,1) from two 32-bit words. */
double orc_u01(uint32_t lo, uint32_t hi)
{
    uint64_t v = (((uint64_t)hi << 32) | (uint64_t)lo) >> 11;
    return (double)v * 0x1p-53;
}

/* Draw 4 words for (instance key, lineage id, step, tag, event, sub). */
static void rng4(uint32_t seed, uint32_t inst, uint64_t id, uint32_t step,
                 uint32_t tag, uint32_t event, uint32_t sub, uint32_t out[4])
{
    uint32_t ctr[4] = { (uint32_t)id, (uint32_t)(id >> 32), step,
                        (tag << 28) | ((event & 0xFFFFFu) << 8) | (sub & 0xFFu) };
    uint32_t key[2] = { seed, inst };
    orc_philox(ctr, key, out);
}

/* ------------------------------------------------------------------------ */
/* Elementary functions written out from their series.  Pinned by           */
/* tests/test_oracle_elementary.py (<= 2 ulp against numpy on wide ranges).  */
/* ------------------------------------------------------------------------ */
#define SQRT_HALF   0x1.6a09e667f3bcdp-1
#define LN2_HI      0x1.62e42fee00000p-1
#define LN2_LO      0x1.a39ef35793c76p-33
#define TWO_OVER_PI 0x1.45f306dc9c883p-1
#define PIO2_1      0x1.921fb54400000p+0
#define PIO2_2      0x1.0b4611a600000p-34
#define PIO2_3      0x1.3198a2e037073p-69
#define TWO_PI      0x1.921fb54442d18p+2
#define PI_D        0x1.921fb54442d18p+1

/* ln(y) for y > 0 normal: y = m 2^e, m in [sqrt(1/2), sqrt(2)),
 * ln m = 2 atanh(f), f = (m-1)/(m+1), series sum_{j=0}^{11} f^(2j)/(2j+1). */
double orc_dlog(double y)
{
    int e;
    double m = frexp(y, &e);
    if (m < SQRT_HALF) { m = m + m; e = e - 1; }
    double f = (m - 1.0) / (m + 1.0);
    double s = f * f;
    double p = 1.0 / 23.0;
    p = p * s + 1.0 / 21.0;
    p = p * s + 1.0 / 19.0;
    p = p * s + 1.0 / 17.0;
    p = p * s + 1.0 / 15.0;
    p = p * s + 1.0 / 13.0;
    p = p * s + 1.0 / 11.0;
    p = p * s + 1.0 / 9.0;
    p = p * s + 1.0 / 7.0;
    p = p * s + 1.0 / 5.0;
    p = p * s + 1.0 / 3.0;
    p = p * s + 1.0;
    double lm = (2.0 * f) * p;
    double de = (double)e;
    return de * LN2_HI + (de * LN2_LO + lm);
}

/* Cody-Waite reduction a = n pi/2 + r with a three-part pi/2. */
static double reduce_pio2(double a, int *quadrant)
{
    double n = rint(a * TWO_OVER_PI);
    double r = a - n * PIO2_1;
    r = r - n * PIO2_2;
    r = r - n * PIO2_3;
    *quadrant = (int)((long long)n & 3);
    return r;
}

/* Taylor series of sin to r^19 and cos to r^20, Horner form. */
static double sin_poly(double r)
{
    double s = r * r;
    double p = -1.0 / 121645100408832000.0;
    p = p * s + 1.0 / 355687428096000.0;
    p = p * s - 1.0 / 1307674368000.0;
    p = p * s + 1.0 / 6227020800.0;
    p = p * s - 1.0 / 39916800.0;
    p = p * s + 1.0 / 362880.0;
    p = p * s - 1.0 / 5040.0;
    p = p * s + 1.0 / 120.0;
    p = p * s - 1.0 / 6.0;
    return r + (r * s) * p;
}

static double cos_poly(double r)
{
    double s = r * r;
    double p = 1.0 / 2432902008176640000.0;
    p = p * s - 1.0 / 6402373705728000.0;
    p = p * s + 1.0 / 20922789888000.0;
    p = p * s - 1.0 / 87178291200.0;
    p = p * s + 1.0 / 479001600.0;
    p = p * s - 1.0 / 3628800.0;
    p = p * s + 1.0 / 40320.0;
    p = p * s - 1.0 / 720.0;
    p = p * s + 1.0 / 24.0;
    p = p * s - 1.0 / 2.0;
    return 1.0 + s * p;
}

double orc_dsin(double a)
{
    int q;
    double r = reduce_pio2(a, &q);
    switch (q) {
    case 0: return sin_poly(r);
    case 1: return cos_poly(r);
    case 2: return -sin_poly(r);
    default: return -cos_poly(r);
    }
}

double orc_dcos(double a)
{
    int q;
    double r = reduce_pio2(a, &q);
    switch (q) {
    case 0: return cos_poly(r);
    case 1: return -sin_poly(r);
    case 2: return -cos_poly(r);
    default: return sin_poly(r);
    }
}

/* Box-Muller: two standard normals from two uniforms. */
static void normal_pair(double u1, double u2, double *z1, double *z2)
{
    double R = sqrt(-2.0 * orc_dlog(1.0 - u1));
    double th = TWO_PI * u2;
    *z1 = R * orc_dcos(th);
    *z2 = R * orc_dsin(th);
}

/* ------------------------------------------------------------------------ */
/* Ensembles.                                                               */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t n, cap;
    double *x[2], *k[2];
    double *w;      /* sp2 weight */
    int8_t *sgn;    /* sp1 sign (+1/-1; 0 for a ghost) */
    uint64_t *id;
    double *D;      /* tangent, 3 per particle */
} ens_t;

typedef struct {
    double x[2], k[2];
    double t0;
    int sgn;
    double w;
    uint64_t id;
    double D[3];
} part_t;

static void ens_reserve(ens_t *E, int64_t need)
{
    if (need <= E->cap) return;
    int64_t cap = E->cap ? E->cap : 1024;
    while (cap < need) cap *= 2;
    for (int d = 0; d < 2; d++) {
        E->x[d] = (double *)realloc(E->x[d], (size_t)cap * sizeof(double));
        E->k[d] = (double *)realloc(E->k[d], (size_t)cap * sizeof(double));
    }
    E->w = (double *)realloc(E->w, (size_t)cap * sizeof(double));
    E->sgn = (int8_t *)realloc(E->sgn, (size_t)cap);
    E->id = (uint64_t *)realloc(E->id, (size_t)cap * sizeof(uint64_t));
    E->D = (double *)realloc(E->D, (size_t)cap * 3 * sizeof(double));
    E->cap = cap;
}

static void ens_free(ens_t *E)
{
    for (int d = 0; d < 2; d++) { free(E->x[d]); free(E->k[d]); }
    free(E->w); free(E->sgn); free(E->id); free(E->D);
    memset(E, 0, sizeof(*E));
}

static void ens_push(ens_t *E, const part_t *p)
{
    ens_reserve(E, E->n + 1);
    int64_t i = E->n++;
    for (int d = 0; d < 2; d++) { E->x[d][i] = p->x[d]; E->k[d][i] = p->k[d]; }
    E->w[i] = p->w; E->sgn[i] = (int8_t)p->sgn; E->id[i] = p->id;
    E->D[3 * i] = p->D[0]; E->D[3 * i + 1] = p->D[1]; E->D[3 * i + 2] = p->D[2];
}

static void ens_load(const ens_t *E, int64_t i, part_t *p)
{
    for (int d = 0; d < 2; d++) { p->x[d] = E->x[d][i]; p->k[d] = E->k[d][i]; }
    p->w = E->w[i]; p->sgn = E->sgn[i]; p->id = E->id[i];
    p->D[0] = E->D[3 * i]; p->D[1] = E->D[3 * i + 1]; p->D[2] = E->D[3 * i + 2];
    p->t0 = 0.0;
}

typedef struct {
    double H[ORC_MAXM], width[ORC_MAXM], center[ORC_MAXM];
    double xi[ORC_MAXM];   /* normaliser of the majorant, int |F[V_m](2q)| 2/(pi hbar) dq */
    double c[ORC_MAXM];    /* xi_m / (2 gamma0): pair probability per unit |sin| */
    double sq[ORC_MAXM];   /* Gaussian kind: std of the kick q, 1/(2w) */
    double gamma0;
    int64_t N0;
    uint32_t key_inst;
    double *xi_tab[ORC_MAXM];   /* Alg. 4 sampler: xi at r_j = j h, j = 0..ORC_XI_N */
    double xi_h[ORC_MAXM];
    ens_t real, ghost;
    orc_stats st;
} inst_t;

typedef struct {
    orc_config cfg;
    double *cum[ORC_MAXM];  /* table kind: cumulative sums, n+1 entries */
    double dq[ORC_MAXM];
    double xi_table[ORC_MAXM];
    inst_t *I;
    uint32_t step;          /* number of completed steps */
    double vfac;            /* hbar / mass */
    int ghost_pass;         /* stepping the ghost ensemble (sp1 branching rule) */
    int keep_cells;         /* test hook: keep the last sp2 annihilation's cell arrays */
    int64_t *kept[3];       /* [B][N_h] each: n~+, n~-, rounded signed count n_nu */
} orc_sim;

/* ------------------------------------------------------------------------ */
/* Kernel constants (Sec. 4.2, Eq. wigner_kernel_Gaussian and Remark 3).     */
/* For symmetric V about c, V_W(x,q) = (2/(pi hbar)) F[V](2q) sin(2q(x-c)),  */
/* derived from the definition Eq. Wigner_kernel with the non-unitary        */
/* transform F[V](s) = int V(y) e^{-isy} dy.  The majorant is                */
/* G(q) = (2/(pi hbar)) |F[V](2q)| with integral xi.  For the Gaussian       */
/* barrier F[V](s) = H w sqrt(2 pi) exp(-w^2 s^2/2), so xi = 2H/hbar and      */
/* G/xi is the normal law with std 1/(2w).                                   */
/* Pinned by tests/test_oracle_physics.py (pair rate against the closed-form */
/* xi(x), the printed 1.5 xi_check = 0.8706, and the Ehrenfest drift).        */
/* ------------------------------------------------------------------------ */
/* xi(r) = (1/2) int |V_W(x, q)| dq for the Gaussian barrier (Sec. 4.2), on
 * r_j = j h, h = 8w / ORC_XI_N, by the midpoint rule over q in [-8/w, 8/w)
 * with ORC_XI_Q nodes; Alg. 4 then interpolates it linearly. */
static void build_xi_table(inst_t *I, int m, double hbar)
{
    double w = I->width[m], H = fabs(I->H[m]);
    double h = (8.0 * w) / (double)ORC_XI_N;
    double qlo = -8.0 / w, dq = (16.0 / w) / (double)ORC_XI_Q;
    double pref = ((H * w) * sqrt(2.0 * PI_D)) / (PI_D * hbar);   /* (1/2)(2/(pi hbar)) F[V] prefactor */
    I->xi_h[m] = h;
    I->xi_tab[m] = (double *)malloc((ORC_XI_N + 1) * sizeof(double));
    for (int j = 0; j <= ORC_XI_N; j++) {
        double r = (double)j * h, acc = 0.0;
        for (int i = 0; i < ORC_XI_Q; i++) {
            double q = qlo + ((double)i + 0.5) * dq;
            acc += exp(-2.0 * ((w * w) * (q * q))) * fabs(sin(2.0 * q * r));
        }
        I->xi_tab[m][j] = (pref * acc) * dq;
    }
}

/* linear interpolation of xi at distance |r| from the centre; constant beyond the grid */
static double xi_interp(const inst_t *I, int m, double r)
{
    double a = fabs(r) / I->xi_h[m];
    if (!(a < (double)ORC_XI_N)) return I->xi_tab[m][ORC_XI_N];
    int j = (int)a;
    double t = a - (double)j;
    return I->xi_tab[m][j] + t * (I->xi_tab[m][j + 1] - I->xi_tab[m][j]);
}

static void setup_instance(orc_sim *S, int b)
{
    const orc_config *C = &S->cfg;
    inst_t *I = &S->I[b];
    double g = 0.0;
    for (int m = 0; m < C->M; m++) {
        if (C->comp_kind[m] == KIND_GAUSS) {
            I->H[m] = C->H[b * C->M + m];
            I->width[m] = C->width[b * C->M + m];
            I->center[m] = C->center[b * C->M + m];
            I->xi[m] = (2.0 * fabs(I->H[m])) / C->hbar;
            I->sq[m] = 0.5 / I->width[m];
            if (C->time_dependent) {   /* the largest xi_m over time bounds gamma0 from below */
                double amp = fabs(C->mod_a[m]) + fabs(C->mod_b[m]);
                double xmax = (2.0 * (fabs(I->H[m]) * amp)) / C->hbar;
                if (xmax > g) g = xmax;
            }
        } else {
            I->center[m] = C->comp_center[m];
            I->xi[m] = S->xi_table[m];
        }
        if (I->xi[m] > g) g = I->xi[m];
    }
    /* gamma0: given, else the smallest value with pair probability <= 1 */
    I->gamma0 = (C->gamma0 > 0.0) ? C->gamma0 : C->gamma_scale * (g / 2.0);
    for (int m = 0; m < C->M; m++) I->c[m] = I->xi[m] / (2.0 * I->gamma0);
    for (int m = 0; m < C->M; m++)
        if (C->sampler[m] == 1 && C->comp_kind[m] == KIND_GAUSS) build_xi_table(I, m, C->hbar);
    I->N0 = C->N0[b];
    I->key_inst = (uint32_t)(C->instance_offset + b);
    I->st.gamma0 = I->gamma0;
}

/* Initial ensemble: exact sampling of the positive Gaussian f0
 * (Sec. 5 test problems), all signs +1, id = index. */
static void init_instance(orc_sim *S, int b)
{
    const orc_config *C = &S->cfg;
    inst_t *I = &S->I[b];
    ens_reserve(&I->real, I->N0);
    for (int64_t j = 0; j < I->N0; j++) {
        part_t p;
        memset(&p, 0, sizeof(p));
        for (int d = 0; d < C->dim; d++) {
            uint32_t r[4];
            rng4(C->seed, I->key_inst, (uint64_t)j, 0, TAG_INIT, 0, (uint32_t)d, r);
            double z1, z2;
            normal_pair(orc_u01(r[0], r[1]), orc_u01(r[2], r[3]), &z1, &z2);
            p.x[d] = C->init_mean_x[d] + C->init_sigma_x[d] * z1;
            p.k[d] = C->init_mean_k[d] + C->init_sigma_k[d] * z2;
        }
        p.sgn = 1;
        p.w = 1.0;
        p.id = (uint64_t)j;
        ens_push(&I->real, &p);
    }
}

static void init_from_histogram(orc_sim *S, int b);
void orc_destroy(orc_sim *S);

orc_sim *orc_create(const orc_config *cfg)
{
    orc_sim *S = (orc_sim *)calloc(1, sizeof(orc_sim));
    S->cfg = *cfg;
    S->vfac = cfg->hbar / cfg->mass;
    for (int m = 0; m < cfg->M; m++) {
        if (cfg->comp_kind[m] != KIND_TABLE) continue;
        int n = cfg->table_n[m];
        S->cum[m] = (double *)malloc((size_t)(n + 1) * sizeof(double));
        S->cum[m][0] = 0.0;
        for (int j = 0; j < n; j++) S->cum[m][j + 1] = S->cum[m][j] + cfg->table[m][j];
        S->dq[m] = (cfg->table_qhi[m] - cfg->table_qlo[m]) / (double)n;
        S->xi_table[m] = ((2.0 * S->cum[m][n]) * S->dq[m]) / (PI_D * cfg->hbar);
    }
    S->I = (inst_t *)calloc((size_t)cfg->B, sizeof(inst_t));
    for (int b = 0; b < cfg->B; b++) {
        setup_instance(S, b);
        /* The sp1 box reads xi_m |sin| / (2 gamma0) as a probability and the
         * wp box uses it as a weight factor; both need it <= 1 (Remark 3,
         * gamma0 >= xi/2).  A configuration that breaks this is refused. */
        const inst_t *I = &S->I[b];
        int bad = !(I->gamma0 > 0.0);
        for (int m = 0; m < cfg->M; m++) {
            if (!(I->c[m] <= 1.0)) bad = 1;
            if (cfg->time_dependent && cfg->comp_kind[m] == KIND_GAUSS) {
                double xmax = (2.0 * (fabs(I->H[m]) * (fabs(cfg->mod_a[m]) + fabs(cfg->mod_b[m])))) / cfg->hbar;
                if (xmax > 2.0 * I->gamma0 * (1.0 + 1e-12)) bad = 1;
            }
        }
        if (bad) {
            S->cfg.B = b + 1;
            orc_destroy(S);
            return NULL;
        }
    }
    for (int b = 0; b < cfg->B; b++) {
        if (cfg->init_kind == 1) init_from_histogram(S, b);
        else init_instance(S, b);
    }
    return S;
}

void orc_destroy(orc_sim *S)
{
    if (!S) return;
    for (int b = 0; b < S->cfg.B; b++) {
        ens_free(&S->I[b].real);
        ens_free(&S->I[b].ghost);
        for (int m = 0; m < ORC_MAXM; m++) free(S->I[b].xi_tab[m]);
    }
    for (int m = 0; m < ORC_MAXM; m++) free(S->cum[m]);
    for (int c = 0; c < 3; c++) free(S->kept[c]);
    free(S->I);
    free(S);
}

/* ------------------------------------------------------------------------ */
/* Kick sampling for component m (Remark 3, Eq. majorant): q from G_m/xi_m.  */
/* Gaussian kind: q = Z/(2w) with Z standard normal (Box-Muller).            */
/* Table kind: piecewise-constant density proportional to the table,         */
/* inverse CDF, uniform within the chosen bin.                               */
/* ------------------------------------------------------------------------ */
static double sample_kick(const orc_sim *S, const inst_t *I, int m, double u1, double u2)
{
    if (S->cfg.comp_kind[m] == KIND_GAUSS) {
        double R = sqrt(-2.0 * orc_dlog(1.0 - u1));
        double z = R * orc_dcos(TWO_PI * u2);
        return z * I->sq[m];
    }
    int n = S->cfg.table_n[m];
    const double *cum = S->cum[m];
    double target = u1 * cum[n];
    /* largest j in [0, n-1] with cum[j] <= target */
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) / 2;
        if (cum[mid] <= target) lo = mid; else hi = mid - 1;
    }
    return S->cfg.table_qlo[m] + ((double)lo + u2) * S->dq[m];
}

/* r_m(x): the argument of the sine for component m. */
static double comp_arg(const orc_sim *S, int m, const double *x, double center)
{
    switch (S->cfg.comp_axis[m]) {
    case 0: return x[0] - center;
    case 1: return x[1] - center;
    default: return (x[0] - x[1]) - center;
    }
}

/* One jump of component m at event position xe (Remark 3, Eq. majorant):
 * the kick q from G_m/xi_m, the sine of the kernel's phase, the direction
 * sigma = sgn(F[V_m]) sgn(sin) of the "+" offspring, and the acceptance
 * uniform (component 0 shares the draw that produced the life-length). */
typedef struct { double q, arg, sn, sigma, u_acc, c; } jump_t;

/* Pair probability per unit |sin| and sign of F[V_m] at absolute time t:
 * Remark 1 evaluates the kernel of a time-varying potential at the jump. */
static void kernel_at(const orc_sim *S, const inst_t *I, int m, double t, double *c, double *sgnV)
{
    const orc_config *C = &S->cfg;
    if (C->comp_kind[m] != KIND_GAUSS) { *c = I->c[m]; *sgnV = C->comp_sgn[m]; return; }
    if (!C->time_dependent) { *c = I->c[m]; *sgnV = I->H[m] >= 0.0 ? 1.0 : -1.0; return; }
    double f = C->mod_a[m] + C->mod_b[m] * orc_dcos(C->mod_omega[m] * t + C->mod_phase[m]);
    double He = I->H[m] * f;
    double xi = (2.0 * fabs(He)) / C->hbar;
    *c = xi / (2.0 * I->gamma0);
    *sgnV = He >= 0.0 ? 1.0 : -1.0;
}

static void draw_jump(const orc_sim *S, const inst_t *I, uint64_t id, uint32_t e, int m,
                      const double *xe, double u_acc0, double t_abs, jump_t *J)
{
    const orc_config *C = &S->cfg;
    uint32_t rq[4];
    rng4(C->seed, I->key_inst, id, S->step, TAG_STEP, e, (uint32_t)(1 + m), rq);
    J->q = sample_kick(S, I, m, orc_u01(rq[0], rq[1]), orc_u01(rq[2], rq[3]));
    J->arg = (2.0 * J->q) * comp_arg(S, m, xe, I->center[m]);
    J->sn = orc_dsin(J->arg);
    double sgnV;
    kernel_at(S, I, m, t_abs, &J->c, &sgnV);
    J->sigma = (J->sn > 0.0) ? sgnV : -sgnV;
    J->u_acc = u_acc0;
    if (m > 0) {
        uint32_t ra[4];
        rng4(C->seed, I->key_inst, id, S->step, TAG_STEP, e, (uint32_t)(8 + m), ra);
        J->u_acc = orc_u01(ra[0], ra[1]);
    }
}

static int in_kbox(const orc_sim *S, const double *k)
{
    for (int d = 0; d < S->cfg.dim; d++)
        if (!(k[d] >= S->cfg.k_lo && k[d] < S->cfg.k_hi)) return 0;
    return 1;
}

/* Alg. 4: a kick from V_W^+(x, .)/xi(x) by rejection.  Proposal q from the
 * Gaussian g = G/xi_hat (Box-Muller), accepted iff u < [sgnV sin(2 q r)]^+.
 * Proposal i of (particle, event e, component m) draws from tag 8 with event
 * field e + 4096 i.  Returns 0 if ORC_REJECT_MAX proposals were rejected. */
static int reject_kick(const orc_sim *S, const inst_t *I, uint64_t id, uint32_t e, int m,
                       double r, double *q_out)
{
    const orc_config *C = &S->cfg;
    double sgnV = I->H[m] >= 0.0 ? 1.0 : -1.0;
    for (uint32_t i = 0; i < ORC_REJECT_MAX; i++) {
        uint32_t ra[4], rb[4];
        uint32_t ev = e + (i << 12);
        rng4(C->seed, I->key_inst, id, S->step, TAG_REJECT, ev, (uint32_t)m, ra);
        rng4(C->seed, I->key_inst, id, S->step, TAG_REJECT, ev, (uint32_t)(4 + m), rb);
        double R = sqrt(-2.0 * orc_dlog(1.0 - orc_u01(ra[0], ra[1])));
        double q = (R * orc_dcos(TWO_PI * orc_u01(ra[2], ra[3]))) * I->sq[m];
        double p = sgnV * orc_dsin((2.0 * q) * r);
        if (orc_u01(rb[0], rb[1]) < p) { *q_out = q; return 1; }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Alg. 1 for one particle over the rest of the current step, emitting its   */
/* offspring (and theirs) in depth-first preorder: for each jump in time      */
/* order, for each component in order, the "+" child, its own family, then    */
/* the "-" child and its family.  The particle itself keeps k after a jump   */
/* (offspring 2M+1), so its end-of-step position does not depend on jumps.    */
/* Pinned by tests/test_oracle_physics.py and tests/test_oracle_invariants.py */
/* ------------------------------------------------------------------------ */
static void walk(orc_sim *S, inst_t *I, ens_t *out, const part_t *P, int depth);

/* ------------------------------------------------------------------------ */
/* Derivative ghost pairs: the x0 tangent without the likelihood-ratio score. */
/* The pair intensity of component m at a jump is c sin(2 q (x - x0)) per     */
/* unit of the kick density (Alg. 1, pair box, with the majorant of Remark 3) */
/* and depends on x0 only through the sine; its x0-derivative is              */
/* -2 q c cos(2 q (x - x0)).  With probability c |cos| (an independent        */
/* uniform) and the same kick q, a pair of ghosts (sign 0) is placed at       */
/* k +/- sigma' q, sigma' = sgn(F[V]) sgn(cos), carrying x0-tangents          */
/* -/+ 2 q s (s the parent's sign) and zero (H, w) tangents.  Its expectation */
/* is the x0-derivative of the signed pair measure, and the tangent is        */
/* bounded by 2|q|, so it has finite variance where the score -2q cot does    */
/* not.  Only signed particles spawn them; the ghosts then walk like any      */
/* particle and join the real ensemble until the next annihilation folds      */
/* their tangents into the cell sums.  Order: after the jump's real pairs, per */
/* component, "+" ghost and its family, then "-" ghost and its family.        */
/* Pinned by tests/test_oracle_gradient.py (finite differences under common  */
/* random numbers; variance below the score's).                               */
/* ------------------------------------------------------------------------ */
static void deriv_pairs(orc_sim *S, inst_t *I, ens_t *out, const part_t *P, int depth,
                        uint32_t e, const double *xe, double te)
{
    const orc_config *C = &S->cfg;
    const double dt = C->dt;
    for (int m = 0; m < C->M; m++) {
        jump_t J;
        double sgnV;
        draw_jump(S, I, P->id, e, m, xe, 0.0, (double)S->step * dt + te, &J);
        kernel_at(S, I, m, (double)S->step * dt + te, &J.c, &sgnV);
        double cs = orc_dcos(J.arg);
        uint32_t ru[4], rc[4];
        rng4(C->seed, I->key_inst, P->id, S->step, TAG_DERIV, e, (uint32_t)m, ru);
        if (!(orc_u01(ru[0], ru[1]) < J.c * fabs(cs))) continue;
        rng4(C->seed, I->key_inst, P->id, S->step, TAG_DERIV, e, (uint32_t)(8 + m), rc);
        uint64_t cid[2] = {
            (3ull << 62) | ((uint64_t)(rc[1] & 0x3FFFFFFFu) << 32) | rc[0],
            (3ull << 62) | ((uint64_t)(rc[3] & 0x3FFFFFFFu) << 32) | rc[2] };
        double kick = (cs > 0.0 ? sgnV : -sgnV) * J.q;
        double dx0 = (2.0 * J.q) * (double)P->sgn;
        for (int side = 0; side < 2; side++) {
            part_t ch;
            memset(&ch, 0, sizeof(ch));
            ch.k[0] = P->k[0]; ch.k[1] = P->k[1];
            switch (C->comp_axis[m]) {
            case 0: ch.k[0] = side == 0 ? P->k[0] + kick : P->k[0] - kick; break;
            case 1: ch.k[1] = side == 0 ? P->k[1] + kick : P->k[1] - kick; break;
            default:
                ch.k[0] = side == 0 ? P->k[0] + kick : P->k[0] - kick;
                ch.k[1] = side == 0 ? P->k[1] - kick : P->k[1] + kick;
                break;
            }
            ch.sgn = 0;
            ch.w = 0.0;
            ch.id = cid[side];
            ch.D[2] = side == 0 ? -dx0 : dx0;
            if (!in_kbox(S, ch.k)) continue;   /* nullified outside K, like any offspring */
            ch.t0 = te;
            part_t rec = ch;
            for (int d = 0; d < C->dim; d++) {
                ch.x[d] = xe[d];
                rec.x[d] = xe[d] + (S->vfac * ch.k[d]) * (dt - te);
            }
            ens_push(out, &rec);
            walk(S, I, out, &ch, depth + 1);
        }
    }
}

static void walk(orc_sim *S, inst_t *I, ens_t *out, const part_t *P, int depth)
{
    const orc_config *C = &S->cfg;
    const double dt = C->dt;
    /* ghosts (weight 0) branch by the sp1 rule in either strategy: a pair
     * with probability c|sin| carries the parent's tangent, which has the
     * expectation of wp's always-emitted pair with tangent factor c|sin| */
    const int sp2 = (C->strategy == STRAT_SP2) && !S->ghost_pass;
    if (depth > I->st.max_depth) I->st.max_depth = depth;
    double t = P->t0;
    for (uint32_t e = 0;; e++) {
        if (e >= ORC_EMAX) { I->st.event_cap_hits++; break; }
        uint32_t r[4];
        rng4(C->seed, I->key_inst, P->id, S->step, TAG_STEP, e, 0, r);
        double u_tau = orc_u01(r[0], r[1]);
        double u_acc0 = orc_u01(r[2], r[3]);
        /* exact life-length for constant gamma0 (Sec. 3.2.1) */
        double tau = -orc_dlog(1.0 - u_tau) / I->gamma0;
        double te = t + tau;
        if (!(te <= dt)) break;           /* rule 2: frozen at the end of the step */
        I->st.events++;
        double xe[2] = { 0.0, 0.0 };
        for (int d = 0; d < C->dim; d++)
            xe[d] = P->x[d] + (S->vfac * P->k[d]) * (te - P->t0);
        for (int m = 0; m < C->M; m++) {
            jump_t J;
            double t_abs = (double)S->step * dt + te;
            double amp = 0.0;
            if (C->sampler[m] == 1) {
                /* Alg. 1 sp1 box with Pr = xi(x)/gamma0 and Alg. 4 for the kick */
                double r = comp_arg(S, m, xe, I->center[m]);
                double u_acc = u_acc0;
                if (m > 0) {
                    uint32_t ra[4];
                    rng4(C->seed, I->key_inst, P->id, S->step, TAG_STEP, e, (uint32_t)(8 + m), ra);
                    u_acc = orc_u01(ra[0], ra[1]);
                }
                if (!(u_acc < xi_interp(I, m, r) / I->gamma0)) continue;
                double qk;
                if (!reject_kick(S, I, P->id, e, m, r, &qk)) continue;
                J.q = qk;
                J.arg = (2.0 * qk) * r;
                J.sn = 1.0;
                J.sigma = 1.0;
                J.c = I->c[m];
            } else {
                draw_jump(S, I, P->id, e, m, xe, u_acc0, t_abs, &J);
                if (!sp2) {
                    if (!(J.u_acc < J.c * fabs(J.sn))) continue; /* sp1 box of Alg. 1 */
                } else {
                    amp = P->w * (J.c * fabs(J.sn));             /* wp/sp2 box of Alg. 1 */
                }
            }
            double q = J.q, arg = J.arg, sn = J.sn, sigma = J.sigma;
            I->st.pairs++;
            uint32_t rc[4];
            rng4(C->seed, I->key_inst, P->id, S->step, TAG_CHILD, e, (uint32_t)m, rc);
            uint64_t cls = ((P->id >> 62) & 1u) ? 3u : 2u; /* ghost lineage keeps bit 62 */
            uint64_t cid[2] = {
                (cls << 62) | ((uint64_t)(rc[1] & 0x3FFFFFFFu) << 32) | rc[0],
                (cls << 62) | ((uint64_t)(rc[3] & 0x3FFFFFFFu) << 32) | rc[2] };
            double kick = sigma * q;
            /* LR score of (kick density, acceptance) w.r.t. (H, w, x0) */
            double score[3] = { 0.0, 0.0, 0.0 };
            /* sp2: the "+" child's tangent X, the "-" child's -X (see below) */
            double X[3] = { 0.0, 0.0, 0.0 };
            if (C->track_tangent) {
                double wdt = I->width[m];
                score[0] = 1.0 / I->H[m];
                score[1] = 1.0 / wdt - ((4.0 * wdt) * q) * q;
                if (sp2) {
                    /* The pair adds w c sgn(V) sin(2qr) [f(k+q) - f(k-q)] with q from
                     * G/xi_hat (wp box of Alg. 1, Remark 3).  Differentiating its
                     * expectation: the kick density times c is G/(2 gamma0), whose
                     * log-derivative is score[0..1] (zero for x0), the parent's weight
                     * carries D, and sin(2q(x - x0)) has x0-derivative -2q cos.  In
                     * the children's frame (k +/- sigma q, weights +/- w c|sin|):
                     * X = c|sin| (D + w score) + w c sgn(sin) d(sin)/d(theta). */
                    double a = J.c * fabs(sn);
                    double g = P->w * (J.c * (sn > 0.0 ? 1.0 : -1.0));
                    X[0] = a * (P->D[0] + P->w * score[0]);
                    X[1] = a * (P->D[1] + P->w * score[1]);
                    X[2] = a * P->D[2] + g * (-(2.0 * q) * orc_dcos(arg));
                } else {
                    score[2] = C->track_tangent == 2 ? 0.0 : -(2.0 * q) * (orc_dcos(arg) / sn);
                }
            }
            for (int side = 0; side < 2; side++) {
                double sdir = side == 0 ? 1.0 : -1.0;
                part_t ch;
                memset(&ch, 0, sizeof(ch));
                ch.k[0] = P->k[0]; ch.k[1] = P->k[1];
                switch (C->comp_axis[m]) {
                case 0: ch.k[0] = side == 0 ? P->k[0] + kick : P->k[0] - kick; break;
                case 1: ch.k[1] = side == 0 ? P->k[1] + kick : P->k[1] - kick; break;
                default:
                    ch.k[0] = side == 0 ? P->k[0] + kick : P->k[0] - kick;
                    ch.k[1] = side == 0 ? P->k[1] - kick : P->k[1] + kick;
                    break;
                }
                ch.sgn = side == 0 ? P->sgn : -P->sgn;
                ch.w = side == 0 ? amp : -amp;
                ch.id = cid[side];
                if (C->track_tangent) {
                    for (int c = 0; c < 3; c++)
                        ch.D[c] = sp2 ? sdir * X[c] : sdir * P->D[c] + (double)ch.sgn * score[c];
                }
                if (!in_kbox(S, ch.k)) {   /* k-truncation: nullified outside K */
                    if (sp2) {
                        double a = fabs(ch.w) * 4294967296.0;
                        int64_t q32 = (int64_t)floor(a);
                        I->st.killed += ch.w < 0.0 ? -q32 : q32;
                    } else {
                        I->st.killed += ch.sgn;
                    }
                    continue;
                }
                ch.t0 = te;
                part_t rec = ch;
                for (int d = 0; d < C->dim; d++) {
                    ch.x[d] = xe[d];
                    rec.x[d] = xe[d] + (S->vfac * ch.k[d]) * (dt - te);
                }
                ens_push(out, &rec);
                walk(S, I, out, &ch, depth + 1);
            }
        }
        if (C->track_tangent == 2 && P->sgn != 0) deriv_pairs(S, I, out, P, depth, e, xe, te);
        t = te;
    }
}

static void step_ensemble(orc_sim *S, inst_t *I, ens_t *E)
{
    const orc_config *C = &S->cfg;
    int64_t n0 = E->n;
    ens_t kids;
    memset(&kids, 0, sizeof(kids));
    for (int64_t i = 0; i < n0; i++) {
        part_t p;
        ens_load(E, i, &p);
        walk(S, I, &kids, &p, 0);
        for (int d = 0; d < C->dim; d++)
            E->x[d][i] = p.x[d] + (S->vfac * p.k[d]) * (C->dt - 0.0);
    }
    ens_reserve(E, n0 + kids.n);
    for (int64_t j = 0; j < kids.n; j++) {
        part_t p;
        ens_load(&kids, j, &p);
        ens_push(E, &p);
    }
    ens_free(&kids);
}

void orc_step(orc_sim *S, int nsteps)
{
    for (int s = 0; s < nsteps; s++) {
        for (int b = 0; b < S->cfg.B; b++) {
            inst_t *I = &S->I[b];
            step_ensemble(S, I, &I->real);
            if (S->cfg.track_tangent) {
                S->ghost_pass = 1;
                step_ensemble(S, I, &I->ghost);
                S->ghost_pass = 0;
            }
        }
        S->step++;
    }
}

/* ------------------------------------------------------------------------ */
/* Cells of the uniform grid D_nu = X_nu1 x K_nu2 (Sec. 4.3).               */
/* ------------------------------------------------------------------------ */
static int64_t cell_of(const orc_sim *S, const double *x, const double *k)
{
    const orc_config *C = &S->cfg;
    double dx = (C->x_hi - C->x_lo) / (double)C->nx;
    double dk = (C->k_hi - C->k_lo) / (double)C->nk;
    int64_t ix[2] = { 0, 0 }, ik[2] = { 0, 0 };
    for (int d = 0; d < C->dim; d++) {
        double qx = (x[d] - C->x_lo) / dx;
        double qk = (k[d] - C->k_lo) / dk;
        if (!(qx >= 0.0 && qx < (double)C->nx)) return -1;
        if (!(qk >= 0.0 && qk < (double)C->nk)) return -1;
        ix[d] = (int64_t)qx;
        ik[d] = (int64_t)qk;
    }
    if (C->dim == 1) return ix[0] + (int64_t)C->nx * ik[0];
    return ((ik[1] * C->nk + ik[0]) * C->nx + ix[1]) * C->nx + ix[0];
}

static int64_t n_cells(const orc_sim *S)
{
    const orc_config *C = &S->cfg;
    if (C->dim == 1) return (int64_t)C->nx * C->nk;
    return (int64_t)C->nx * C->nx * C->nk * C->nk;
}

/* Uniform position in cell nu (Alg. 3 step 3) from uniforms u[2*dim]. */
static void place_in_cell(const orc_sim *S, int64_t nu, const double *ux, const double *uk,
                          double *x, double *k)
{
    const orc_config *C = &S->cfg;
    double dx = (C->x_hi - C->x_lo) / (double)C->nx;
    double dk = (C->k_hi - C->k_lo) / (double)C->nk;
    int64_t ix[2], ik[2];
    if (C->dim == 1) {
        ix[0] = nu % C->nx; ik[0] = nu / C->nx;
    } else {
        int64_t r = nu;
        ix[0] = r % C->nx; r /= C->nx;
        ix[1] = r % C->nx; r /= C->nx;
        ik[0] = r % C->nk; r /= C->nk;
        ik[1] = r;
    }
    for (int d = 0; d < C->dim; d++) {
        x[d] = C->x_lo + ((double)ix[d] + ux[d]) * dx;
        k[d] = C->k_lo + ((double)ik[d] + uk[d]) * dk;
    }
}

static void regen_draws(const orc_sim *S, const inst_t *I, uint64_t id, uint32_t tag,
                        double *ux, double *uk)
{
    for (int d = 0; d < S->cfg.dim; d++) {
        uint32_t r[4];
        rng4(S->cfg.seed, I->key_inst, id, S->step, tag, 0, (uint32_t)d, r);
        ux[d] = orc_u01(r[0], r[1]);
        uk[d] = orc_u01(r[2], r[3]);
    }
}

/* Regenerate |n_nu| particles of sign sgn(n_nu) per cell in ascending nu,
 * id = (nu << 32) | j.  With tangents, each regenerated particle carries
 * T_nu/|n_nu|; a cell that was occupied but nets to zero gets one ghost
 * (sign 0) carrying T_nu. */
static void regenerate(orc_sim *S, inst_t *I, const int64_t *cnt, const int64_t *occ,
                       const double *T)
{
    int64_t nc = n_cells(S);
    ens_t out, gout;
    memset(&out, 0, sizeof(out));
    memset(&gout, 0, sizeof(gout));
    for (int64_t nu = 0; nu < nc; nu++) {
        int64_t n = cnt[nu];
        int64_t an = n < 0 ? -n : n;
        for (int64_t j = 0; j < an; j++) {
            part_t p;
            memset(&p, 0, sizeof(p));
            p.id = ((uint64_t)nu << 32) | (uint64_t)j;
            double ux[2], uk[2];
            regen_draws(S, I, p.id, TAG_REGEN, ux, uk);
            place_in_cell(S, nu, ux, uk, p.x, p.k);
            p.sgn = n > 0 ? 1 : -1;
            p.w = n > 0 ? 1.0 : -1.0;
            if (T)
                for (int c = 0; c < 3; c++) p.D[c] = T[3 * nu + c] / (double)an;
            ens_push(&out, &p);
        }
        if (T && n == 0 && occ[nu] > 0) {
            part_t g;
            memset(&g, 0, sizeof(g));
            g.id = ((uint64_t)1 << 62) | ((uint64_t)nu << 32);
            double ux[2], uk[2];
            regen_draws(S, I, g.id, TAG_GHOST, ux, uk);
            place_in_cell(S, nu, ux, uk, g.x, g.k);
            g.sgn = 0;
            g.w = 0.0;
            for (int c = 0; c < 3; c++) g.D[c] = T[3 * nu + c];
            ens_push(&gout, &g);
        }
    }
    ens_free(&I->real);
    I->real = out;
    ens_free(&I->ghost);
    I->ghost = gout;
}

/* Alg. 3 (Sec. 4.1): importance sampling from a signed histogram d_nu.
 * Step 1 (rounding): m = N_alpha mu(D_nu) |d_nu|, n = [m] + p with p = 1 iff
 * u < m - [m] (one uniform per cell, tag 7 at step 0); step 2: sign
 * sgn(d_nu); step 3: uniform in the cell (the same placement, ids and order as
 * a regeneration). */
static void init_from_histogram(orc_sim *S, int b)
{
    const orc_config *C = &S->cfg;
    inst_t *I = &S->I[b];
    int64_t nc = n_cells(S);
    double dx = (C->x_hi - C->x_lo) / (double)C->nx;
    double dk = (C->k_hi - C->k_lo) / (double)C->nk;
    double mu = C->dim == 1 ? dx * dk : ((dx * dx) * dk) * dk;
    int64_t *cnt = (int64_t *)calloc((size_t)nc, sizeof(int64_t));
    for (int64_t nu = 0; nu < nc; nu++) {
        double dv = C->init_hist[(int64_t)b * nc + nu];
        if (dv == 0.0) continue;
        double m = ((double)I->N0 * mu) * fabs(dv);
        double fl = floor(m);
        uint32_t r[4];
        rng4(C->seed, I->key_inst, (uint64_t)nu, 0, TAG_HIST, 0, 0, r);
        int64_t n = (int64_t)fl + (orc_u01(r[0], r[1]) < m - fl ? 1 : 0);
        cnt[nu] = dv > 0.0 ? n : -n;
    }
    regenerate(S, I, cnt, NULL, NULL);
    free(cnt);
}

/* Sums of tangents over the particles of a cell or a density bin (the
 * differentiation form; the paper defines no such sums): each component D of
 * a particle enters as the integer trunc(D 2^32) (32.32 fixed point, which
 * needs |D| < 2^31), the integer sums are exact, so no summation order is
 * singled out, and a sum Q has the value (double)floor(Q / 2^32) +
 * (double)(Q mod 2^32) 2^-32.  A component outside the range, or not a
 * number, adds nothing and is counted in range_errors. */
static void fx_add(inst_t *I, i128 *Q, const double *D)
{
    for (int c = 0; c < 3; c++) {
        if (!(fabs(D[c]) < 2147483648.0)) { I->st.range_errors++; continue; }
        Q[c] += (i128)(int64_t)(D[c] * 4294967296.0);
    }
}

static double fx_value(i128 Q)
{
    i128 h = Q >> 32;                                  /* floor(Q / 2^32) */
    uint64_t lo = (uint64_t)(Q - h * ((i128)1 << 32)); /* Q mod 2^32 */
    return (double)(int64_t)h + (double)lo * 0x1p-32;
}

/* sp1 annihilation: Eq. signed_histogram, n_nu = n_nu^+ - n_nu^- exactly,
 * then Alg. 3 without its rounding step (m is already an integer). */
static void annihilate_sp1(orc_sim *S, inst_t *I)
{
    const orc_config *C = &S->cfg;
    int64_t nc = n_cells(S);
    int64_t *cnt = (int64_t *)calloc((size_t)nc, sizeof(int64_t));
    int64_t *occ = (int64_t *)calloc((size_t)nc, sizeof(int64_t));
    i128 *Q = C->track_tangent ? (i128 *)calloc((size_t)nc * 3, sizeof(i128)) : NULL;
    for (int64_t i = 0; i < I->real.n; i++) {
        double x[2] = { I->real.x[0][i], I->real.x[1][i] };
        double k[2] = { I->real.k[0][i], I->real.k[1][i] };
        int64_t nu = cell_of(S, x, k);
        if (nu < 0) { I->st.escaped += I->real.sgn[i]; continue; }
        cnt[nu] += I->real.sgn[i];
        occ[nu] += 1;
        if (Q) fx_add(I, Q + 3 * nu, I->real.D + 3 * i);
    }
    double *T = NULL;
    if (Q) {
        for (int64_t i = 0; i < I->ghost.n; i++) {
            double x[2] = { I->ghost.x[0][i], I->ghost.x[1][i] };
            double k[2] = { I->ghost.k[0][i], I->ghost.k[1][i] };
            int64_t nu = cell_of(S, x, k);
            if (nu < 0) continue;
            occ[nu] += 1;
            fx_add(I, Q + 3 * nu, I->ghost.D + 3 * i);
        }
        T = (double *)malloc((size_t)nc * 3 * sizeof(double));
        for (int64_t j = 0; j < 3 * nc; j++) T[j] = fx_value(Q[j]);
    }
    regenerate(S, I, cnt, occ, T);
    free(cnt); free(occ); free(Q); free(T);
}

/* ------------------------------------------------------------------------ */
/* sp2 annihilation.                                                          */
/* Alg. 2 (residual bootstrap) per sign class with the weights quantised once */
/* to A_i = floor(|w_i| 2^32), then Eq. boostrap_histogram cell values        */
/* m_nu = N_alpha |lambda^+ n~^+/N^+ + lambda^- n~^-/N^-|, with              */
/* lambda^pm N_alpha = +-S^pm/2^32 (Eq. lambda), as the exact rational        */
/* |S^+ n^+ N^- - S^- n^- N^+| / (2^32 N^+ N^-), and the rounding step of    */
/* Alg. 3 with one uniform per cell.                                          */
/* ------------------------------------------------------------------------ */

/* floor(r * R / 2^64) for r < 2^64, R < 2^127: a uniform integer in [0, R). */
static u128 scale_u64(uint64_t r, u128 R)
{
    uint64_t Rlo = (uint64_t)R;
    u128 Rhi = R >> 64;
    return (u128)r * Rhi + (((u128)r * (u128)Rlo) >> 64);
}

/* Residual bootstrap of one class (Alg. 2).  A[0..n-1] are the quantised
 * weights in canonical order; copies[i] receives k_i + hits_i. */
void orc_bootstrap_class(int64_t n, const uint64_t *A, uint32_t seed, uint32_t inst,
                         uint32_t step, uint32_t cls, int64_t *copies)
{
    u128 S = 0;
    for (int64_t i = 0; i < n; i++) S += A[i];
    for (int64_t i = 0; i < n; i++) copies[i] = 0;
    if (n == 0 || S == 0) return;
    int64_t sumk = 0;
    u128 *P = (u128 *)malloc((size_t)(n + 1) * sizeof(u128));
    P[0] = 0;
    for (int64_t i = 0; i < n; i++) {
        u128 num = (u128)(uint64_t)n * (u128)A[i];
        u128 ki = num / S;                   /* step 1: floor of n w~_i */
        u128 ri = num - ki * S;              /* residual, scaled by S */
        copies[i] = (int64_t)ki;
        sumk += (int64_t)ki;
        P[i + 1] = P[i] + ri;
    }
    int64_t Nr = n - sumk;                   /* remaining draws */
    u128 R = S * (u128)(uint64_t)Nr;         /* == P[n] */
    for (int64_t d = 0; d < Nr; d++) {       /* step 2: N_r i.i.d. draws */
        uint32_t r[4];
        rng4(seed, inst, (uint64_t)d, step, TAG_BOOT, 0, cls, r);
        uint64_t bits = ((uint64_t)r[1] << 32) | r[0];
        u128 U = scale_u64(bits, R);
        /* the i with P[i] <= U < P[i+1] */
        int64_t lo = 0, hi = n - 1;
        while (lo < hi) {
            int64_t mid = (lo + hi + 1) / 2;
            if (P[mid] <= U) lo = mid; else hi = mid - 1;
        }
        copies[lo] += 1;
    }
    free(P);
}

/* Rounding step of Alg. 3 for one cell value |num|/den:
 * floor(|num|/den) + [U < |num| mod den], U uniform in [0, den). */
int64_t orc_round_cell(u128 num, u128 den, uint32_t seed, uint32_t inst, uint32_t step,
                       uint64_t cell)
{
    u128 q = num / den;
    u128 rem = num - q * den;
    uint32_t r[4];
    rng4(seed, inst, cell, step, TAG_ROUND, 0, 0, r);
    uint64_t bits = ((uint64_t)r[1] << 32) | r[0];
    u128 U = scale_u64(bits, den);
    return (int64_t)q + (U < rem ? 1 : 0);
}

/* ctypes-friendly wrapper: num and den split into 64-bit halves. */
int64_t orc_round_cell64(uint64_t num_hi, uint64_t num_lo, uint64_t den_hi, uint64_t den_lo,
                         uint32_t seed, uint32_t inst, uint32_t step, uint64_t cell)
{
    u128 num = ((u128)num_hi << 64) | num_lo;
    u128 den = ((u128)den_hi << 64) | den_lo;
    return orc_round_cell(num, den, seed, inst, step, cell);
}

static void annihilate_sp2(orc_sim *S, inst_t *I)
{
    int64_t nc = n_cells(S);
    int64_t n = I->real.n;
    int64_t *cell = (int64_t *)malloc((size_t)(n ? n : 1) * sizeof(int64_t));
    uint64_t *A[2];
    int64_t *idx[2], cn[2] = { 0, 0 };
    for (int c = 0; c < 2; c++) {
        A[c] = (uint64_t *)malloc((size_t)(n ? n : 1) * sizeof(uint64_t));
        idx[c] = (int64_t *)malloc((size_t)(n ? n : 1) * sizeof(int64_t));
    }
    /* classes in canonical order; out-of-box weight is tallied in Q32 */
    for (int64_t i = 0; i < n; i++) {
        double x[2] = { I->real.x[0][i], I->real.x[1][i] };
        double k[2] = { I->real.k[0][i], I->real.k[1][i] };
        double w = I->real.w[i];
        uint64_t a = (uint64_t)floor(fabs(w) * 4294967296.0);
        cell[i] = cell_of(S, x, k);
        if (cell[i] < 0) {
            I->st.escaped += w < 0.0 ? -(int64_t)a : (int64_t)a;
            continue;
        }
        if (w > 0.0) { A[0][cn[0]] = a; idx[0][cn[0]++] = i; }
        else if (w < 0.0) { A[1][cn[1]] = a; idx[1][cn[1]++] = i; }
    }
    int64_t *ntil[2];
    uint64_t Ssum[2] = { 0, 0 };
    for (int c = 0; c < 2; c++) {
        ntil[c] = (int64_t *)calloc((size_t)nc, sizeof(int64_t));
        int64_t *copies = (int64_t *)malloc((size_t)(cn[c] ? cn[c] : 1) * sizeof(int64_t));
        orc_bootstrap_class(cn[c], A[c], S->cfg.seed, I->key_inst, S->step, (uint32_t)c, copies);
        for (int64_t j = 0; j < cn[c]; j++) {
            Ssum[c] += A[c][j];
            ntil[c][cell[idx[c][j]]] += copies[j];
        }
        free(copies);
    }
    I->st.S_plus = (int64_t)Ssum[0]; I->st.S_minus = (int64_t)Ssum[1];
    I->st.N_plus = cn[0]; I->st.N_minus = cn[1];
    int64_t *cnt = (int64_t *)calloc((size_t)nc, sizeof(int64_t));
    for (int64_t nu = 0; nu < nc; nu++) {
        i128 num;
        u128 den;
        if (cn[0] > 0 && cn[1] > 0) {
            num = (i128)((u128)Ssum[0] * (u128)ntil[0][nu] * (u128)cn[1])
                - (i128)((u128)Ssum[1] * (u128)ntil[1][nu] * (u128)cn[0]);
            den = ((u128)cn[0] * (u128)cn[1]) << 32;
        } else if (cn[0] > 0) {
            num = (i128)((u128)Ssum[0] * (u128)ntil[0][nu]);
            den = (u128)cn[0] << 32;
        } else if (cn[1] > 0) {
            num = -(i128)((u128)Ssum[1] * (u128)ntil[1][nu]);
            den = (u128)cn[1] << 32;
        } else {
            continue;
        }
        if (num == 0) continue;
        u128 an = num < 0 ? (u128)(-num) : (u128)num;
        int64_t m = orc_round_cell(an, den, S->cfg.seed, I->key_inst, S->step, (uint64_t)nu);
        cnt[nu] = num < 0 ? -m : m;
    }
    if (S->keep_cells) {   /* test hook: the bootstrap counts and the rounded cell values */
        int64_t off = (int64_t)(I - S->I) * nc;
        for (int64_t nu = 0; nu < nc; nu++) {
            S->kept[0][off + nu] = ntil[0][nu];
            S->kept[1][off + nu] = ntil[1][nu];
            S->kept[2][off + nu] = cnt[nu];
        }
    }
    /* tangents: the cell sums of Eq. boostrap_histogram's expectation,
     * sum of w_i, are differentiated directly: T_nu = sum of D_i over the
     * particles and ghosts in the cell, as in sp1 */
    int64_t *occ = NULL;
    double *T = NULL;
    if (S->cfg.track_tangent) {
        occ = (int64_t *)calloc((size_t)nc, sizeof(int64_t));
        i128 *Q = (i128 *)calloc((size_t)nc * 3, sizeof(i128));
        for (int64_t i = 0; i < n; i++) {
            if (cell[i] < 0) continue;
            occ[cell[i]] += 1;
            fx_add(I, Q + 3 * cell[i], I->real.D + 3 * i);
        }
        for (int64_t i = 0; i < I->ghost.n; i++) {
            double x[2] = { I->ghost.x[0][i], I->ghost.x[1][i] };
            double k[2] = { I->ghost.k[0][i], I->ghost.k[1][i] };
            int64_t nu = cell_of(S, x, k);
            if (nu < 0) continue;
            occ[nu] += 1;
            fx_add(I, Q + 3 * nu, I->ghost.D + 3 * i);
        }
        T = (double *)malloc((size_t)nc * 3 * sizeof(double));
        for (int64_t j = 0; j < 3 * nc; j++) T[j] = fx_value(Q[j]);
        free(Q);
    }
    regenerate(S, I, cnt, occ, T);
    for (int c = 0; c < 2; c++) { free(A[c]); free(idx[c]); free(ntil[c]); }
    free(cell);
    free(cnt);
    free(occ);
    free(T);
}

void orc_annihilate(orc_sim *S)
{
    for (int b = 0; b < S->cfg.B; b++) {
        if (S->cfg.strategy == STRAT_SP2) annihilate_sp2(S, &S->I[b]);
        else annihilate_sp1(S, &S->I[b]);
    }
}

/* Steps with resampling at the scheduled instants and whenever the particle
 * number is about to exceed a threshold (Sec. 5, the resampling instants):
 * after each step, the ensemble is annihilated if the number of steps done
 * is a multiple of `every` (every > 0), or if some instance holds more than
 * `limit` particles (limit > 0). */
void orc_run_adaptive(orc_sim *S, int nsteps, int every, int64_t limit)
{
    for (int s = 0; s < nsteps; s++) {
        orc_step(S, 1);
        int sched = every > 0 && S->step % (uint32_t)every == 0;
        int over = 0;
        for (int b = 0; b < S->cfg.B; b++)
            if (limit > 0 && S->I[b].real.n > limit) over = 1;
        if (!sched && !over) continue;
        orc_annihilate(S);
        for (int b = 0; b < S->cfg.B; b++) {
            S->I[b].st.annihilations++;
            if (!sched) S->I[b].st.triggered++;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Density (Eq. estimator with A = indicator of a position bin):             */
/* rho_b = sum_{i in b} w_i / (N_alpha dx_b).  sp1 sums signs exactly; sp2    */
/* sums weights in Q32 fixed point, exact for the +-1 weights left by the     */
/* bootstrap.  out[b * nbins + j].                                            */
/* ------------------------------------------------------------------------ */
void orc_density(orc_sim *S, int axis, int nbins, double lo, double hi, double *out)
{
    double dxb = (hi - lo) / (double)nbins;
    int64_t *acc = (int64_t *)malloc((size_t)nbins * sizeof(int64_t));
    for (int b = 0; b < S->cfg.B; b++) {
        inst_t *I = &S->I[b];
        memset(acc, 0, (size_t)nbins * sizeof(int64_t));
        for (int64_t i = 0; i < I->real.n; i++) {
            double q = (I->real.x[axis][i] - lo) / dxb;
            if (!(q >= 0.0 && q < (double)nbins)) continue;
            int j = (int)q;
            if (S->cfg.strategy == STRAT_SP2) {
                double w = I->real.w[i];
                acc[j] += (int64_t)(w * 4294967296.0);
            } else {
                acc[j] += I->real.sgn[i];
            }
        }
        double denom = (double)I->N0 * dxb;
        for (int j = 0; j < nbins; j++) {
            double v = (double)acc[j];
            if (S->cfg.strategy == STRAT_SP2) v = v * 0x1p-32;
            out[(int64_t)b * nbins + j] = v / denom;
        }
    }
    free(acc);
}

/* Bin sums of the tangents of instance b's real particles and ghosts in
 * fixed point (fx_add): T[c * nbins + j] = value of sum_{i in bin j} D_i[c]. */
static void tangent_bins(orc_sim *S, int b, int axis, int nbins, double lo, double dxb, double *T)
{
    inst_t *I = &S->I[b];
    i128 *Q = (i128 *)calloc((size_t)nbins * 3, sizeof(i128));
    ens_t *E2[2] = { &I->real, &I->ghost };
    for (int e = 0; e < 2; e++) {
        ens_t *E = E2[e];
        for (int64_t i = 0; i < E->n; i++) {
            double q = (E->x[axis][i] - lo) / dxb;
            if (!(q >= 0.0 && q < (double)nbins)) continue;
            i128 acc[3] = { 0, 0, 0 };
            fx_add(I, acc, E->D + 3 * i);
            for (int c = 0; c < 3; c++) Q[(int64_t)c * nbins + (int)q] += acc[c];
        }
    }
    for (int64_t j = 0; j < 3 * (int64_t)nbins; j++) T[j] = fx_value(Q[j]);
    free(Q);
}

/* Tangent density J[b][c][j] = sum_{i in j} D_i[c] / (N_alpha dx_b), the bin
 * sums taken over real particles and ghosts in fixed point (fx_add). */
void orc_density_tangent(orc_sim *S, int axis, int nbins, double lo, double hi, double *out)
{
    double dxb = (hi - lo) / (double)nbins;
    for (int b = 0; b < S->cfg.B; b++) {
        double *o = out + (int64_t)b * 3 * nbins;
        tangent_bins(S, b, axis, nbins, lo, dxb, o);
        double denom = (double)S->I[b].N0 * dxb;
        for (int j = 0; j < 3 * nbins; j++) o[j] = o[j] / denom;
    }
}

/* Backward pass of the density: out[b * 3 + c] = (sum_j g[b * nbins + j]
 * T[c][j]) / (N_alpha dx_b), with the fixed-point bin sums T of
 * tangent_bins and the contraction taken over the bins in ascending order. */
void orc_density_vjp(orc_sim *S, int axis, int nbins, double lo, double hi, const double *g, double *out)
{
    double dxb = (hi - lo) / (double)nbins;
    double *T = (double *)malloc((size_t)nbins * 3 * sizeof(double));
    for (int b = 0; b < S->cfg.B; b++) {
        tangent_bins(S, b, axis, nbins, lo, dxb, T);
        double denom = (double)S->I[b].N0 * dxb;
        for (int c = 0; c < 3; c++) {
            double acc = 0.0;
            for (int j = 0; j < nbins; j++) acc = acc + g[(int64_t)b * nbins + j] * T[(int64_t)c * nbins + j];
            out[b * 3 + c] = acc / denom;
        }
    }
    free(T);
}

/* ------------------------------------------------------------------------ */
/* Accessors.                                                                */
/* ------------------------------------------------------------------------ */
int64_t orc_count(const orc_sim *S, int b, int ghost)
{
    return ghost ? S->I[b].ghost.n : S->I[b].real.n;
}

/* Copy instance b's ensemble out (any pointer may be NULL). */
void orc_get(const orc_sim *S, int b, int ghost, double *x, double *k, int8_t *sgn,
             double *w, uint64_t *id, double *D)
{
    const ens_t *E = ghost ? &S->I[b].ghost : &S->I[b].real;
    int dim = S->cfg.dim;
    for (int64_t i = 0; i < E->n; i++) {
        for (int d = 0; d < dim; d++) {
            if (x) x[d * E->n + i] = E->x[d][i];
            if (k) k[d * E->n + i] = E->k[d][i];
        }
        if (sgn) sgn[i] = E->sgn[i];
        if (w) w[i] = E->w[i];
        if (id) id[i] = E->id[i];
        if (D) { D[3 * i] = E->D[3 * i]; D[3 * i + 1] = E->D[3 * i + 1]; D[3 * i + 2] = E->D[3 * i + 2]; }
    }
}

/* Replace instance b's ensemble (test hook for building special states). */
void orc_set(orc_sim *S, int b, int64_t n, const double *x, const double *k, const int8_t *sgn,
             const double *w, const uint64_t *id)
{
    inst_t *I = &S->I[b];
    ens_free(&I->real);
    ens_reserve(&I->real, n);
    int dim = S->cfg.dim;
    for (int64_t i = 0; i < n; i++) {
        part_t p;
        memset(&p, 0, sizeof(p));
        for (int d = 0; d < dim; d++) { p.x[d] = x[d * n + i]; p.k[d] = k[d * n + i]; }
        p.sgn = sgn ? sgn[i] : 1;
        p.w = w ? w[i] : (double)p.sgn;
        p.id = id ? id[i] : (uint64_t)i;
        ens_push(&I->real, &p);
    }
}

void orc_get_stats(const orc_sim *S, int b, orc_stats *out)
{
    const inst_t *I = &S->I[b];
    orc_stats st = I->st;
    st.n = I->real.n;
    st.n_ghost = I->ghost.n;
    st.n_plus = st.n_minus = st.net = 0;
    for (int64_t i = 0; i < I->real.n; i++) {
        int s = S->cfg.strategy == STRAT_SP2 ? (I->real.w[i] > 0.0 ? 1 : (I->real.w[i] < 0.0 ? -1 : 0))
                                              : I->real.sgn[i];
        if (s > 0) st.n_plus++; else if (s < 0) st.n_minus++;
        st.net += s;
    }
    st.step = S->step;
    *out = st;
}

/* Test hook: keep, from now on, each sp2 annihilation's per-cell bootstrap
 * counts n~+_nu, n~-_nu and rounded signed cell counts n_nu, readable with
 * orc_get_cells ([N_h] int64 each for instance b). */
void orc_keep_cells(orc_sim *S, int on)
{
    S->keep_cells = on;
    if (on && !S->kept[0]) {
        size_t n = (size_t)S->cfg.B * (size_t)n_cells(S);
        for (int c = 0; c < 3; c++) S->kept[c] = (int64_t *)calloc(n, sizeof(int64_t));
    }
}

void orc_get_cells(const orc_sim *S, int b, int64_t *nplus, int64_t *nminus, int64_t *cnt)
{
    int64_t nc = n_cells(S);
    for (int64_t nu = 0; nu < nc; nu++) {
        nplus[nu] = S->kept[0] ? S->kept[0][(int64_t)b * nc + nu] : 0;
        nminus[nu] = S->kept[1] ? S->kept[1][(int64_t)b * nc + nu] : 0;
        cnt[nu] = S->kept[2] ? S->kept[2][(int64_t)b * nc + nu] : 0;
    }
}

uint32_t orc_get_step(const orc_sim *S) { return S->step; }
double orc_get_gamma0(const orc_sim *S, int b) { return S->I[b].gamma0; }
double orc_get_xi(const orc_sim *S, int b, int m) { return S->I[b].xi[m]; }

/* Test hook: one jump of component m for a particle at x with the acceptance
 * and kick of the sp1 box, for lineage id and event e at the current step.
 * Writes accepted (0/1), signed kick sigma*q, and sin value. */
void orc_probe_jump(orc_sim *S, int b, int m, const double *x, uint64_t id, uint32_t e,
                    int32_t *accepted, double *kick, double *sn_out)
{
    inst_t *I = &S->I[b];
    uint32_t r[4];
    rng4(S->cfg.seed, I->key_inst, id, S->step, TAG_STEP, e, 0, r);
    jump_t J;
    draw_jump(S, I, id, e, m, x, orc_u01(r[2], r[3]), (double)S->step * S->cfg.dt, &J);
    *accepted = (J.u_acc < J.c * fabs(J.sn)) ? 1 : 0;
    *kick = J.sigma * J.q;
    *sn_out = J.sn;
}
