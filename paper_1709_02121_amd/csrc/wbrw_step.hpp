// One time step of the Wigner branching random walk (Alg. 1, Sec. 2), after
// the streaming pass (wbrw_stream.hpp):
//
// k_events: every tile turns its wavefront ballots into the ordered list of
// event parents (instance by instance, in particle order), at an offset
// taken from group sums of the tiles' event counts.
//
// k_family (latency-bound, ~3% of particles): one thread per event parent
// walks the parent's whole family within the step, depth first: for each
// jump in time order, each component in order, the "+" offspring, its own
// family, then the "-" offspring and its family.  Offspring are new particles
// of the system with their own lineage ids and exponential clocks (Alg. 1
// rule 3).  The common family (one jump, offspring that do not jump again
// before the end of the step) is evaluated for all parents in lockstep; the
// others take the general walk, spread over the block.  Records hold the
// end-of-step state, so no generation is revisited in a later launch.  Each
// tile stages its records contiguously in the inactive buffer set and adds
// its record count to the sum of its group of kSupGroup tiles;
// k_place_records finds each tile's place from those sums and copies the
// records there, after the instance's particles.
#pragma once
#include <type_traits>

#include "wbrw_dev.hpp"
#include "wbrw_math.hpp"
#include "wbrw_stream.hpp"

namespace wbrw {

// ---------------------------------------------------------------------------
// Kernel phase and kick sampling (Sec. 4.2, Remark 3 / Eq. majorant_approach)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double phase_offset(const Dev &d, int m, const double *xe, double c)
{
    const int a = d.axis[m];
    if (a == 0) return xe[0] - c;
    if (a == 1) return xe[1] - c;
    return (xe[0] - xe[1]) - c;
}

// q from G_m / xi_m: Gaussian (Box-Muller, std 1/(2w)) or inverse CDF of the
// piecewise-constant table with a uniform offset inside the chosen bin.  The
// bin is the last j < n with cum[j] <= u1 cum[n].  A guide table (Chen and
// Asau's method) gives the answer's range: for u1 in bucket i = floor(u1 kg)
// the target u1 cum[n] lies between the rounded bucket ends, so the bin lies
// in [guide[i], guide[i + 1]], nearly always one or two bins wide, where a
// binary search over the whole table took 12 dependent loads.  The bin found
// is the same.
__device__ __forceinline__ double kick_sample(const Dev &d, const InstParam &P, int m, double u1,
                                              double u2)
{
    if (d.kind[m] == 0) {
        const double R = sqrt(-2.0 * ln_series(1.0 - u1));
        const double z = R * cos_det(kTwoPi * u2);
        return z * P.sq[m];
    }
    const Table T = d.tab[m];
    const double target = u1 * T.cum[T.n];
    const int i = (int)(u1 * (double)T.kg);
    int lo = T.guide[i], hi = T.guide[i + 1];
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (T.cum[mid] <= target) lo = mid; else hi = mid - 1;
    }
    return T.q_lo + ((double)lo + u2) * T.dq;
}

// Alg. 4: xi(|r|) by linear interpolation on its grid (constant beyond it)
__device__ __forceinline__ double xi_lerp(const double *tab, double h, double r)
{
    const double a = fabs(r) / h;
    if (!(a < (double)kXiN)) return tab[kXiN];
    const int j = (int)a;
    const double t = a - (double)j;
    return tab[j] + t * (tab[j + 1] - tab[j]);
}

// Alg. 4: kick from V_W^+(x, .)/xi(x) by rejection (proposal from the Gaussian
// majorant, accept iff u < [sgnV sin(2 q r)]^+); false if every proposal failed.
__device__ __forceinline__ bool reject_kick(const Dev &d, const InstParam &P, uint64_t id,
                                            uint32_t step, uint32_t e, int m, double r, double &q_out)
{
    const double sgv = P.H[m] >= 0.0 ? 1.0 : -1.0;
    for (uint32_t i = 0; i < kRejectMax; ++i) {
        const uint32_t ev = e + (i << 12);
        const W4 a = draw(id, step, kTagReject, ev, (uint32_t)m, d.seed, P.key);
        const W4 b = draw(id, step, kTagReject, ev, (uint32_t)(4 + m), d.seed, P.key);
        const double R = sqrt(-2.0 * ln_series(1.0 - unit53(a.a, a.b)));
        const double q = (R * cos_det(kTwoPi * unit53(a.c, a.d))) * P.sq[m];
        const double p = sgv * sin_det((2.0 * q) * r);
        if (unit53(b.a, b.b) < p) { q_out = q; return true; }
    }
    return false;
}

template <int DIM>
__device__ __forceinline__ bool in_kbox(const Dev &d, const double *k)
{
    if (!(k[0] >= d.k_lo && k[0] < d.k_hi)) return false;
    if (DIM == 2 && !(k[1] >= d.k_lo && k[1] < d.k_hi)) return false;
    return true;
}


// After k_stream: the ordered event list.  Every streaming tile turns its
// ballots into the within-instance indices of its event parents, at the
// tile's offset in its instance's list (order: particle slot, wavefront,
// lane, as in the particle array); the offset is the sum of the event counts
// of the instance's earlier tiles, taken from the 64-tile group sums.  Block
// 0 (dispatched first) instead adds up the streaming blocks' per-instance
// event counts and lays out the family tiles.  Before that it clears the
// previous step's family-tile group sums (read by the previous placement
// launch, so its closing block could not) and keeps the particle counts,
// after which the step's records go (the placement launch's closing block
// updates them).
__global__ __launch_bounds__(kThreads) void k_events(Dev d, int ghost, int sgrid)
{
    const int B = d.B;
    const int tid = threadIdx.x;
    if (blockIdx.x == 0) {
        constexpr int kLdsB = 512;
        __shared__ int64_t s_ev[kLdsB];
        int64_t *evc = d.evc + (int64_t)ghost * B;
        const bool lds = B <= kLdsB;
        if (lds)
            for (int b = tid; b < B; b += kThreads) s_ev[b] = 0;
        {
            uint64_t *supB = ghost ? d.supBg : d.supB;
            const int64_t nb = (d.tileB[(int64_t)ghost * (B + 1) + B] + kSupGroup - 1) / kSupGroup;
            for (int64_t g = tid; g < nb; g += kThreads) supB[g * kSupStride] = 0;
            const int64_t *Ncur = ghost ? d.NG : d.N;
            for (int b = tid; b < B; b += kThreads) d.Nbase[(int64_t)ghost * B + b] = Ncur[b];
        }
        __syncthreads();
        for (int g = tid; g < sgrid; g += kThreads) {
            const int64_t cb = d.spart[2 * g], c = d.spart[2 * g + 1];
            if (cb < 0 || c == 0) continue;
            if (lds) atomicAdd((unsigned long long *)&s_ev[cb], (unsigned long long)c);
            else atomicAdd((unsigned long long *)&evc[cb], (unsigned long long)c);
        }
        __syncthreads();
        // evc already holds what k_stream's blocks added on changing instance
        if (lds)
            for (int b = tid; b < B; b += kThreads)
                if (s_ev[b]) atomicAdd((unsigned long long *)&evc[b], (unsigned long long)s_ev[b]);
        __syncthreads();
        const int64_t ftile = ghost ? kTileB : fam_tile(d.dim, d.tangent != 0);
        block_prefix(d.tileB + (int64_t)ghost * (B + 1), B, [&](int b) {
            const int64_t e = (int64_t)__hip_atomic_load((unsigned long long *)&evc[b], __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT);
            return (e + ftile - 1) / ftile;
        });
        return;
    }
    // One wavefront per streaming tile, so that every tile's loads are in
    // flight at once (the grid holds about as many wavefronts as tiles).
    const int64_t *plan = d.tileA + (int64_t)ghost * (B + 1);
    const int64_t ntiles = plan[B];
    const uint64_t *tc = ghost ? d.tcAg : d.tcA;
    const uint64_t *sup = ghost ? d.supAg : d.supA;
    const uint64_t *emask = ghost ? d.emAg : d.emA;
    uint32_t *evi = ghost ? d.gev_idx : d.ev_idx;
    const int lane = tid & 63, wv = tid >> 6;
    constexpr int kWaves = kThreads / 64;
    static_assert(kTileA / 64 <= 64, "one lane per ballot of a tile");
    for (int64_t t = (int64_t)(blockIdx.x - 1) * kWaves + wv; t < ntiles; t += (int64_t)(gridDim.x - 1) * kWaves) {
        const int b = segment_of(plan, B, t);
        const int64_t tl = t - plan[b];
        const InstParam &P = d.ip[b];
        const int64_t base = ghost ? P.gbase : P.base;
        // ballot q holds the tile's particles [64 q, 64 q + 64), whatever the
        // streaming kernel's block shape (loaded before the offset sum, to
        // overlap it); exclusive scan of their popcounts in q order
        const uint64_t *em = emask + t * (kTileA / 64);
        const uint64_t mine = lane < kTileA / 64 ? em[lane] : 0ull;
        const uint64_t rel = wave_range_sum(TileRange(tc, sup, plan[b], t));
        const uint32_t c = (uint32_t)__popcll(mine);
        uint32_t inc = c;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t v = __shfl_up(inc, o, 64);
            if (lane >= o) inc += v;
        }
        const uint32_t exc = inc - c;
        const uint32_t mlo = (uint32_t)mine, mhi = (uint32_t)(mine >> 32);
#pragma unroll 4
        for (int q = 0; q < kTileA / 64; ++q) {
            const uint64_t m = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)mhi, q) << 32) |
                               (uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)mlo, q);
            if (m == 0ull) continue;
            const uint32_t off = (uint32_t)__builtin_amdgcn_readlane((int)exc, q);
            if ((m >> lane) & 1ull) {
                const int64_t pos = base + (int64_t)rel + off + lane_rank(m);
                evi[pos] = (uint32_t)(tl * kTileA + (int64_t)q * 64 + lane);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Pass 2: family trees of event parents
// ---------------------------------------------------------------------------
// Kick and weight of a created pair (see draw_pair).
struct PairDraw {
    double q, arg, sn, sigma, amp;
};

struct Node {
    double x[2], k[2];   // position at t0, wave vector
    double t0;           // start of this particle's walk within the step
    double w;            // sp2 weight
    double D[3];         // tangent
    uint64_t id;
    int32_t sg;          // sp1 sign, 0 for a ghost
    int32_t depth;
    double t;            // time of its latest jump (t0 before the first)
    double te;           // time of the jump being expanded
    double xe[2];        // position at te
    double ua0;          // acceptance uniform of component 0
    uint32_t e;          // jump index
    int32_t m, side, in_ev;
};

// True if the clock draw u certainly gives no jump before the end of the
// step for a clock running from t, i.e. t - ln(1-u)/gamma0 > dt as the exact
// test evaluates it.  -ln(1-u) >= u makes u > gamma0 (dt - t) sufficient in
// exact arithmetic; the relative 2^-30 and absolute dt 2^-40 margins cover
// the rounding of the exact test (the logarithm within a few ulp, the
// division, the sum compared with dt).  Only draws below the bound (a few
// percent) pay for the logarithm.
__device__ __forceinline__ bool surely_no_jump(double u, double t, double dt, double g0)
{
    return u > g0 * ((dt - t) * (1.0 + 0x1p-30) + dt * 0x1p-40);
}

struct Tally {
    int64_t events, pairs, killed, cap;
    int32_t maxdepth;
};

// The records of a family found by fast_family (at most R: nearly always
// one pair in 1D; in 4D, where each of the three components may add a pair,
// up to two; with derivative pairs at most one of each), kept in LDS until
// the ordered scan has placed them.  All of them are born at the family's
// one jump, so that jump's position and time are kept once per slot and the
// end-of-step positions are formed when the records are written.
template <int DIM, bool SP2, bool TAN>
struct Stash {
    static constexpr int R = (!SP2 && (TAN || DIM == 2)) ? 4 : 2;
    static constexpr int F = fam_tile(DIM, TAN);   // event parents per tile
    double xe0[F], te[F];
    double xe1[DIM == 2 ? F : 1];
    double k0[R][F];
    double k1[DIM == 2 ? R : 1][DIM == 2 ? F : 1];
    double w[SP2 ? R : 1][SP2 ? F : 1];
    double D[TAN ? 3 * R : 1][TAN ? F : 1];
    uint64_t id[R][F];
    int8_t sg[R][F];
};

// The families of a tile that are not of the lockstep kind, expanded level
// by level: every node (a family root, or a kept offspring, which is a
// record) of one level is expanded by one lane, which walks its jumps in time
// order and appends its kept offspring with their parent, rank among the
// parent's offspring and depth; offspring that jump again within the step
// form the next level.  Subtree sizes and depth-first positions then give
// every record its place in the canonical order.  The tallies are kept per
// node, so that a family whose nodes do not all fit can be dropped and
// walked again depth first.
template <int DIM, bool SP2, bool TAN>
struct Tree {
    static constexpr int kNodes = 256;
    double x0[kNodes], k0[kNodes];   // position at birth (t0), wave vector
    double x1[DIM == 2 ? kNodes : 1], k1[DIM == 2 ? kNodes : 1];
    double t0[kNodes];
    double w[SP2 ? kNodes : 1];
    double D[TAN ? 3 : 1][TAN ? kNodes : 1];
    uint64_t id[kNodes];
    int64_t killed[kNodes];          // k-truncation tally of the node's jumps
    uint32_t size[kNodes];           // records in the subtree (a root: its family's)
    uint16_t par[kNodes];            // parent node (roots: none)
    uint16_t rank[kNodes];           // among the parent's kept offspring
    uint16_t slot[kNodes];           // tile slot of the family
    uint16_t nch[kNodes];            // kept offspring
    uint16_t cst[kNodes];            // first of its offspring in `child`
    uint16_t child[kNodes];          // offspring grouped by parent, in rank order
    uint16_t front[2][kNodes];       // the levels being expanded / collected
    uint16_t events[kNodes], pairs[kNodes];
    int16_t pos[kNodes];             // depth-first position within the family
    int8_t sg[kNodes];
    uint8_t depth[kNodes], capped[kNodes];
    uint32_t n, nf[2], maxd;
};

// 4D kernels: the records of the families that took the general walk, in
// order of creation across the tile, each tagged with its family's slot and
// its rank within the family; past kPool they go on in the block's overflow
// area in HBM.  A family whose records do not all fit there either is walked
// again when the records are written.  (In 4D about a fifth of
// the families of a tile are not of the lockstep kind, with some ten records
// each: too many nodes for a Tree in an LDS budget that keeps three blocks
// per CU.)  384 records fill the LDS that three blocks per CU leave; a record
// kept in LDS is cheaper than one stored to HBM, since a later load of the
// walk waits on the same counter as every store before it.
constexpr int kPool = 384;
template <int DIM, bool SP2, bool TAN>
struct Pool {
    double x0[kPool], k0[kPool];
    double x1[DIM == 2 ? kPool : 1], k1[DIM == 2 ? kPool : 1];
    double w[SP2 ? kPool : 1];
    double D[TAN ? 3 : 1][TAN ? kPool : 1];
    uint64_t id[kPool];
    uint16_t slot[kPool], rank[kPool];
    int8_t sg[kPool];
    uint32_t n;
};

// Pair decision and kick of component m at jump e of particle `id`
// (Alg. 1 rules 3-5 with the majorant sampler of Remark 3, or Alg. 4):
// returns false if no pair is created.

template <bool SP2>
__device__ __forceinline__ bool draw_pair(const Dev &d, const InstParam &P, uint64_t id, uint32_t step,
                                          uint32_t e, int m, const double *xe, double te, double ua0,
                                          double w, PairDraw &J, const W4 *kick_draw = nullptr)
{
    const uint32_t seed = d.seed, key = P.key;
    double cm = P.c[m], sgv = P.sgnV[m];
    bool alg4 = false;
    if (d.sampler[m] == 1) {
        // Alg. 1 sp1 box with Pr = xi(x)/gamma0, kick by Alg. 4
        const double r = phase_offset(d, m, xe, P.center[m]);
        double ua = ua0;
        if (m > 0) {
            const W4 ra = draw(id, step, kTagStep, e, (uint32_t)(8 + m), seed, key);
            ua = unit53(ra.a, ra.b);
        }
        const double *tab = d.xi_tab + ((int64_t)(&P - d.ip) * d.M + m) * (kXiN + 1);
        double qk = 0.0;
        if (!(ua < xi_lerp(tab, P.xi_h[m], r) / P.gamma0) || !reject_kick(d, P, id, step, e, m, r, qk))
            return false;
        J.q = qk;
        J.arg = (2.0 * qk) * r;
        J.sn = 1.0;
        sgv = 1.0;
        alg4 = true;
    } else {
        const W4 rq = kick_draw ? *kick_draw : draw(id, step, kTagStep, e, (uint32_t)(1 + m), seed, key);
        J.q = kick_sample(d, P, m, unit53(rq.a, rq.b), unit53(rq.c, rq.d));
        J.arg = (2.0 * J.q) * phase_offset(d, m, xe, P.center[m]);
        J.sn = sin_det(J.arg);
    }
    if (d.tdep && d.kind[m] == 0 && !alg4) {   // Remark 1: kernel at the absolute jump time
        const double tabs = (double)step * d.dt + te;
        const double f = P.ma[m] + P.mb[m] * cos_det(P.mw[m] * tabs + P.mp[m]);
        const double He = P.H[m] * f;
        cm = ((2.0 * fabs(He)) / d.hbar) / (2.0 * P.gamma0);
        sgv = He >= 0.0 ? 1.0 : -1.0;
    }
    J.sigma = (J.sn > 0.0) ? sgv : -sgv;
    J.amp = 0.0;
    if (!SP2 && !alg4) {
        double ua = ua0;
        if (m > 0) {
            const W4 ra = draw(id, step, kTagStep, e, (uint32_t)(8 + m), seed, key);
            ua = unit53(ra.a, ra.b);
        }
        if (!(ua < cm * fabs(J.sn))) return false;   // no pair: only the survivor continues
    } else if (SP2) {
        J.amp = w * (cm * fabs(J.sn));
    }
    return true;
}

// Offspring `side` (0: "+", 1: "-") of the pair J of component m at jump e;
// rc is the child-id draw of (parent, e, m).  Sets k, sign, weight, id and
// tangent of ch.
__device__ __forceinline__ void child_id_k(const Dev &d, const Node &par, uint64_t cls, int m, int side,
                                           const PairDraw &J, const W4 &rc, Node &ch)
{
    ch.id = side == 0 ? ((cls << 62) | ((uint64_t)(rc.b & 0x3FFFFFFFu) << 32) | (uint64_t)rc.a)
                      : ((cls << 62) | ((uint64_t)(rc.d & 0x3FFFFFFFu) << 32) | (uint64_t)rc.c);
    const double kick = J.sigma * J.q;
    ch.k[0] = par.k[0];
    ch.k[1] = par.k[1];
    const int ax = d.axis[m];
    if (ax == 0) {
        ch.k[0] = side == 0 ? par.k[0] + kick : par.k[0] - kick;
    } else if (ax == 1) {
        ch.k[1] = side == 0 ? par.k[1] + kick : par.k[1] - kick;
    } else {
        ch.k[0] = side == 0 ? par.k[0] + kick : par.k[0] - kick;
        ch.k[1] = side == 0 ? par.k[1] - kick : par.k[1] + kick;
    }
}

template <bool SP2, bool TAN>
__device__ __forceinline__ void make_child(const Dev &d, const InstParam &P, const Node &par, int m, int side,
                                           const PairDraw &J, const W4 &rc, Node &ch)
{
    const uint64_t cls = ((par.id >> 62) & 1ull) ? 3ull : 2ull;   // ghost lineages keep bit 62
    child_id_k(d, par, cls, m, side, J, rc, ch);
    ch.sg = side == 0 ? par.sg : -par.sg;
    ch.w = side == 0 ? J.amp : -J.amp;
    if constexpr (TAN && SP2) {
        // The wp pair adds w c sgn(V) sin(2qr) [f(k+q) - f(k-q)] with q drawn
        // from G/xi_hat.  Differentiating its expectation: c times the kick
        // density is G/(2 gamma0), whose log-derivative is (1/H, 1/w - 4wq^2, 0);
        // the parent's weight carries D; sin(2q(x - x0)) has x0-derivative
        // -2q cos.  In the children's frame (k +/- sigma q, weights
        // +/- w c|sin|) the "+" child carries
        // X = c|sin| (D + w dlogG) + w c sgn(sin) dsin, the "-" child -X.
        const double wd = P.width[m];
        const double s0 = 1.0 / P.H[m];
        const double s1 = 1.0 / wd - ((4.0 * wd) * J.q) * J.q;
        // tangents require a static kernel, so c is the instance's constant
        const double cm = P.c[m];
        const double a = cm * fabs(J.sn);
        const double g = par.w * (cm * (J.sn > 0.0 ? 1.0 : -1.0));
        const double x0 = a * (par.D[0] + par.w * s0);
        const double x1 = a * (par.D[1] + par.w * s1);
        const double x2 = a * par.D[2] + g * (-(2.0 * J.q) * cos_det(J.arg));
        const double sdir = side == 0 ? 1.0 : -1.0;
        ch.D[0] = sdir * x0;
        ch.D[1] = sdir * x1;
        ch.D[2] = sdir * x2;
    } else if constexpr (TAN) {
        const double wd = P.width[m];
        const double s0 = 1.0 / P.H[m];
        const double s1 = 1.0 / wd - ((4.0 * wd) * J.q) * J.q;
        // tangent mode 2 carries the x0 derivative by derivative pairs instead
        const double s2 = d.tangent == 2 ? 0.0 : -(2.0 * J.q) * (cos_det(J.arg) / J.sn);
        const double sdir = side == 0 ? 1.0 : -1.0;
        const double sgd = (double)ch.sg;
        ch.D[0] = sdir * par.D[0] + sgd * s0;
        ch.D[1] = sdir * par.D[1] + sgd * s1;
        ch.D[2] = sdir * par.D[2] + sgd * s2;
    } else {
        ch.D[0] = ch.D[1] = ch.D[2] = 0.0;
    }
}

// Derivative pair of component m at jump e (tangent mode 2).  The pair
// intensity per unit kick density, c sin(2 q (x - x0)), depends on x0 only
// through the sine, whose x0-derivative gives -2 q c cos(2 q (x - x0)).
// With the jump's own kick q and an independent uniform, a pair of ghosts
// is created with probability c |cos|, directed by sgn(F[V]) sgn(cos); the
// "+" ghost carries the x0-tangent -2 q s and the "-" ghost +2 q s (s the
// parent's sign).  Its expectation is the x0-derivative of the signed pair
// measure with a tangent bounded by 2|q|, where the score -2q cot(2 q r) has
// infinite variance.  Returns false if no pair is created.
__device__ __forceinline__ bool draw_deriv(const Dev &d, const InstParam &P, uint64_t id, uint32_t step,
                                           uint32_t e, int m, const double *xe, PairDraw &J,
                                           const W4 *kick_draw = nullptr)
{
    const W4 rq = kick_draw ? *kick_draw : draw(id, step, kTagStep, e, (uint32_t)(1 + m), d.seed, P.key);
    const W4 ru = draw(id, step, kTagDeriv, e, (uint32_t)m, d.seed, P.key);
    J.q = kick_sample(d, P, m, unit53(rq.a, rq.b), unit53(rq.c, rq.d));
    J.arg = (2.0 * J.q) * phase_offset(d, m, xe, P.center[m]);
    const double cs = cos_det(J.arg);
    if (!(unit53(ru.a, ru.b) < P.c[m] * fabs(cs))) return false;
    J.sn = cs;
    J.sigma = (cs > 0.0) ? P.sgnV[m] : -P.sgnV[m];
    J.amp = 0.0;
    return true;
}

// Ghost `side` of the derivative pair J (rc: its id draw); ghost lineage ids.
__device__ __forceinline__ void make_deriv_child(const Dev &d, const Node &par, int m, int side,
                                                 const PairDraw &J, const W4 &rc, Node &ch)
{
    child_id_k(d, par, 3ull, m, side, J, rc, ch);
    ch.sg = 0;
    ch.w = 0.0;
    const double dx0 = (2.0 * J.q) * (double)par.sg;
    ch.D[0] = 0.0;
    ch.D[1] = 0.0;
    ch.D[2] = side == 0 ? -dx0 : dx0;
}

// k-truncation tally of a child that left the k-box (Sec. 2)
template <bool SP2>
__device__ __forceinline__ int64_t killed_amount(const Node &ch)
{
    if (SP2) {
        const int64_t q32 = (int64_t)floor(fabs(ch.w) * 4294967296.0);
        return ch.w < 0.0 ? -q32 : q32;
    }
    return ch.sg;
}

// Child ch of the family in `slot`, kept in stash row r (the family's jump
// is kept in the slot's xe0, xe1, te).
template <int DIM, bool SP2, bool TAN>
__device__ __forceinline__ void stash_record(Stash<DIM, SP2, TAN> *sh, int r, int slot, const Node &ch)
{
    sh->k0[r][slot] = ch.k[0];
    if (DIM == 2) sh->k1[r][slot] = ch.k[1];
    if (SP2) sh->w[r][slot] = ch.w; else sh->sg[r][slot] = (int8_t)ch.sg;
    sh->id[r][slot] = ch.id;
    if (TAN) {
        sh->D[3 * r][slot] = ch.D[0];
        sh->D[3 * r + 1][slot] = ch.D[1];
        sh->D[3 * r + 2][slot] = ch.D[2];
    }
}

// The block's overflow area of the pool (see kGPool): field f of record g
// is at f * kGPool + g of the doubles.
struct GPoolView {
    double *f;
    uint64_t *id;
    uint32_t *sr;    // slot | rank << 16
    int8_t *sg;
};
__device__ __forceinline__ GPoolView gpool_view(const Dev &d)
{
    char *b = d.gpool + (size_t)blockIdx.x * kGPoolBytes;
    return {(double *)b, (uint64_t *)(b + (size_t)8 * 8 * kGPool), (uint32_t *)(b + (size_t)9 * 8 * kGPool),
            (int8_t *)(b + (size_t)(9 * 8 + 4) * kGPool)};
}
__device__ __forceinline__ uint32_t gpool_cap(const Dev &d)
{
    return (int)blockIdx.x < d.gpool_blocks ? (uint32_t)kGPool : 0u;
}

template <int DIM, bool SP2, bool TAN>
__device__ __forceinline__ bool pool_record(const Dev &d, Pool<DIM, SP2, TAN> *pl, int rank, int slot,
                                            const double *xe, double te, const Node &ch)
{
    const uint32_t r = atomicAdd(&pl->n, 1u);
    const double x0 = xe[0] + (d.vfac * ch.k[0]) * (d.dt - te);
    const double x1 = DIM == 2 ? xe[1] + (d.vfac * ch.k[1]) * (d.dt - te) : 0.0;
    if (r < (uint32_t)kPool) {
        pl->x0[r] = x0;
        pl->k0[r] = ch.k[0];
        if (DIM == 2) {
            pl->x1[r] = x1;
            pl->k1[r] = ch.k[1];
        }
        if (SP2) pl->w[r] = ch.w; else pl->sg[r] = (int8_t)ch.sg;
        pl->id[r] = ch.id;
        if (TAN) {
            pl->D[0][r] = ch.D[0];
            pl->D[1][r] = ch.D[1];
            pl->D[2][r] = ch.D[2];
        }
        pl->slot[r] = (uint16_t)slot;
        pl->rank[r] = (uint16_t)rank;
        return true;
    }
    const uint32_t g = r - (uint32_t)kPool;
    if (g >= gpool_cap(d)) return false;
    const GPoolView v = gpool_view(d);
    v.f[g] = x0;
    v.f[kGPool + g] = ch.k[0];
    if (DIM == 2) {
        v.f[2 * kGPool + g] = x1;
        v.f[3 * kGPool + g] = ch.k[1];
    }
    if (SP2) v.f[4 * kGPool + g] = ch.w; else v.sg[g] = (int8_t)ch.sg;
    if (TAN) {
        v.f[5 * kGPool + g] = ch.D[0];
        v.f[6 * kGPool + g] = ch.D[1];
        v.f[7 * kGPool + g] = ch.D[2];
    }
    v.id[g] = ch.id;
    v.sr[g] = (uint32_t)slot | ((uint32_t)rank << 16);
    return true;
}

// A pair created at time te, as fast_family keeps it: both children into
// the stash (clearing `fast` if it is full) unless the k-box removes them,
// and `fast` cleared if either child jumps again within the step.
template <int DIM, bool SP2, bool TAN>
__device__ __forceinline__ void leaf_pair(const Dev &d, const InstParam &P, uint32_t step, const Node (&ch)[2],
                                          double te, Stash<DIM, SP2, TAN> *sh, int slot,
                                          uint32_t &cnt, Tally &tl, bool &fast)
{
    // both offspring's first clock draws, together
    const W4 l0 = draw(ch[0].id, step, kTagStep, 0u, 0u, d.seed, P.key);
    const W4 l1 = draw(ch[1].id, step, kTagStep, 0u, 0u, d.seed, P.key);
#pragma unroll
    for (int side = 0; side < 2; ++side) {
        if (!in_kbox<DIM>(d, ch[side].k)) {
            tl.killed += killed_amount<SP2>(ch[side]);
            continue;
        }
        if (cnt < (uint32_t)Stash<DIM, SP2, TAN>::R)
            stash_record<DIM, SP2, TAN>(sh, (int)cnt, slot, ch[side]);
        else fast = false;
        cnt++;
        if (tl.maxdepth < 1) tl.maxdepth = 1;
        const double u0 = side == 0 ? unit53(l0.a, l0.b) : unit53(l1.a, l1.b);
        if (!surely_no_jump(u0, te, d.dt, P.gamma0) && te + (-ln_series(1.0 - u0) / P.gamma0) <= d.dt)
            fast = false;
    }
}

// The common family in lockstep: the parent jumps once in the step, and
// every kept child is a leaf (its first clock draw falls past the end of
// the step).  Produces the same records, in the same order, and the same
// tallies as walk_family would, with no per-lane state machine.  Returns
// false if the family is not of this kind (a second jump of the parent, a
// child that jumps again, or more than kStash records); cnt and tl are then
// to be discarded.
template <int DIM, bool SP2, bool TAN>
__device__ __forceinline__ bool fast_family(const Dev &d, const InstParam &P, uint32_t step,
                                            const Node &root, Stash<DIM, SP2, TAN> *sh, int slot,
                                            uint32_t &cnt, Tally &tl)
{
    const uint32_t seed = d.seed, key = P.key;
    cnt = 0;
    // The draws that do not depend on each other are taken together, so
    // their Philox chains interleave: the first and second clock draws, and
    // the kick and child-id draws of component 0.
    const W4 r = draw(root.id, step, kTagStep, 0u, 0u, seed, key);
    const W4 r1 = draw(root.id, step, kTagStep, 1u, 0u, seed, key);
    const W4 rq0 = draw(root.id, step, kTagStep, 0u, 1u, seed, key);
    const W4 rc0 = draw(root.id, step, kTagChild, 0u, 0u, seed, key);
    const double te = root.t0 + (-ln_series(1.0 - unit53(r.a, r.b)) / P.gamma0);
    if (!(te <= d.dt)) return true;
    tl.events++;
    const double ua0 = unit53(r.c, r.d);
    double xe[2];
    xe[0] = root.x[0] + (d.vfac * root.k[0]) * (te - root.t0);
    xe[1] = DIM == 2 ? root.x[1] + (d.vfac * root.k[1]) * (te - root.t0) : 0.0;
    sh->xe0[slot] = xe[0];
    if (DIM == 2) sh->xe1[slot] = xe[1];
    sh->te[slot] = te;
    bool fast = true;
    for (int m = 0; m < d.M; ++m) {
        PairDraw J;
        if (!draw_pair<SP2>(d, P, root.id, step, 0u, m, xe, te, ua0, root.w, J, m == 0 ? &rq0 : nullptr))
            continue;
        tl.pairs++;
        const W4 rc = m == 0 ? rc0 : draw(root.id, step, kTagChild, 0u, (uint32_t)m, seed, key);
        Node ch[2];
        make_child<SP2, TAN>(d, P, root, m, 0, J, rc, ch[0]);
        make_child<SP2, TAN>(d, P, root, m, 1, J, rc, ch[1]);
        leaf_pair<DIM, SP2, TAN>(d, P, step, ch, te, sh, slot, cnt, tl, fast);
    }
    if constexpr (TAN) {
        if (d.tangent == 2 && root.sg != 0) {
            for (int m = 0; m < d.M; ++m) {    // derivative pairs, after the jump's real pairs
                PairDraw J;
                if (!draw_deriv(d, P, root.id, step, 0u, m, xe, J, m == 0 ? &rq0 : nullptr)) continue;
                const W4 rc = draw(root.id, step, kTagDeriv, 0u, (uint32_t)(8 + m), seed, key);
                Node ch[2];
                make_deriv_child(d, root, m, 0, J, rc, ch[0]);
                make_deriv_child(d, root, m, 1, J, rc, ch[1]);
                leaf_pair<DIM, SP2, TAN>(d, P, step, ch, te, sh, slot, cnt, tl, fast);
            }
        }
    }
    const double u1 = unit53(r1.a, r1.b);
    if (!surely_no_jump(u1, te, d.dt, P.gamma0) && te + (-ln_series(1.0 - u1) / P.gamma0) <= d.dt)
        fast = false;
    return fast;
}

// Pair slots of a jump in walk_family: components 0..M-1, then (tangent
// mode 2, signed particles) their derivative pairs as slots M..2M-1.  Without
// tangents these are exactly the pair draw and make_child.
template <bool TAN>
__device__ __forceinline__ int slot_end(const Dev &d, const Node &cur, int M)
{
    if constexpr (TAN) return (d.tangent == 2 && cur.sg != 0) ? 2 * M : M;
    else return M;
}

template <bool SP2, bool TAN>
__device__ __forceinline__ bool slot_draw(const Dev &d, const InstParam &P, const Node &cur, uint32_t step,
                                          int slot, int M, PairDraw &J, W4 &rc)
{
    if constexpr (TAN) {
        if (slot >= M) {
            if (!draw_deriv(d, P, cur.id, step, cur.e, slot - M, cur.xe, J)) return false;
            rc = draw(cur.id, step, kTagDeriv, cur.e, (uint32_t)(8 + slot - M), d.seed, P.key);
            return true;
        }
    }
    if (!draw_pair<SP2>(d, P, cur.id, step, cur.e, slot, cur.xe, cur.te, cur.ua0, cur.w, J)) return false;
    rc = draw(cur.id, step, kTagChild, cur.e, (uint32_t)slot, d.seed, P.key);
    return true;
}

template <bool SP2, bool TAN>
__device__ __forceinline__ void slot_child(const Dev &d, const InstParam &P, const Node &cur, int slot, int M,
                                           int side, const PairDraw &J, const W4 &rc, Node &ch)
{
    if constexpr (TAN) {
        if (slot >= M) {
            make_deriv_child(d, cur, slot - M, side, J, rc, ch);
            return;
        }
    }
    make_child<SP2, TAN>(d, P, cur, slot, side, J, rc, ch);
}

// General depth-first walk of one family (any number of jumps and levels):
// in the 4D and tangent kernels for every family that is not of the lockstep
// kind, in the others for those whose nodes do not fit the tile's Tree.  Counting mode (EMIT false)
// tallies, counts the records and puts them into the tile's pool if one is
// given (clearing `pooled` if one did not fit); emitting mode writes every
// record from first_rec on.
template <int DIM, bool SP2, bool TAN, bool EMIT>
__device__ uint32_t walk_family(const Dev &d, const InstParam &P, uint32_t step, Node cur,
                                const Ens &out, int64_t base, int64_t first_rec, int64_t cap,
                                int64_t dstride, Tally &tl, uint32_t &err,
                                Pool<DIM, SP2, TAN> *pl, int slot, bool &pooled)
{
    Node stack[kMaxDepth];
    PairDraw stackJ[kMaxDepth];
    W4 stackR[kMaxDepth];
    int sp = 0;
    uint32_t nrec = 0;
    const uint32_t seed = d.seed, key = P.key;
    const int M = d.M;
    cur.t = cur.t0;
    cur.e = 0;
    cur.in_ev = 0;
    cur.depth = 0;
    for (;;) {
        if (!cur.in_ev) {
            bool done = false;
            if (cur.e >= kEventCap) {
                if (!EMIT) tl.cap++;
                done = true;
            } else {
                const W4 r = draw(cur.id, step, kTagStep, cur.e, 0u, seed, key);
                const double u = unit53(r.a, r.b);
                const double te = surely_no_jump(u, cur.t, d.dt, P.gamma0)
                                      ? d.dt + 1.0 : cur.t + (-ln_series(1.0 - u) / P.gamma0);
                if (!(te <= d.dt)) {
                    done = true;
                } else {
                    if (!EMIT) tl.events++;
                    cur.te = te;
                    cur.ua0 = unit53(r.c, r.d);
                    cur.xe[0] = cur.x[0] + (d.vfac * cur.k[0]) * (te - cur.t0);
                    if (DIM == 2) cur.xe[1] = cur.x[1] + (d.vfac * cur.k[1]) * (te - cur.t0);
                    else cur.xe[1] = 0.0;
                    cur.in_ev = 1;
                    cur.m = 0;
                    cur.side = 0;
                }
            }
            if (done) {
                if (sp == 0) break;
                cur = stack[--sp];
                continue;
            }
        }
        if (cur.m >= slot_end<TAN>(d, cur, M)) {
            cur.t = cur.te;
            cur.e += 1u;
            cur.in_ev = 0;
            continue;
        }
        const int m = cur.m;
        PairDraw J;
        W4 rc;
        if (cur.side == 0) {
            if (!slot_draw<SP2, TAN>(d, P, cur, step, m, M, J, rc)) {
                cur.m += 1;
                continue;
            }
            if (!EMIT && (!TAN || m < M)) tl.pairs++;
        } else {
            J = stackJ[sp];        // saved when this frame descended into its "+" offspring
            rc = stackR[sp];
        }
        bool descend = false;
        Node ch;
        for (int side = cur.side; side < 2 && !descend; ++side) {
            slot_child<SP2, TAN>(d, P, cur, m, M, side, J, rc, ch);
            if (!in_kbox<DIM>(d, ch.k)) {          // k-truncation (Sec. 2)
                if (!EMIT) tl.killed += killed_amount<SP2>(ch);
                continue;
            }
            if (EMIT) {
                const int64_t li = first_rec + nrec;
                if (li < cap) {
                    const int64_t o = base + li;
                    out.x0[o] = cur.xe[0] + (d.vfac * ch.k[0]) * (d.dt - cur.te);
                    out.k0[o] = ch.k[0];
                    if (DIM == 2) {
                        out.x1[o] = cur.xe[1] + (d.vfac * ch.k[1]) * (d.dt - cur.te);
                        out.k1[o] = ch.k[1];
                    }
                    if (SP2) out.w[o] = ch.w; else out.sg[o] = (int8_t)ch.sg;
                    out.id[o] = ch.id;
                    if (TAN) {
                        out.D[o] = ch.D[0];
                        out.D[dstride + o] = ch.D[1];
                        out.D[2 * dstride + o] = ch.D[2];
                    }
                } else {
                    err |= kErrCapacity;
                }
            } else if (pooled) {
                pooled = pool_record<DIM, SP2, TAN>(d, pl, (int)nrec, slot, cur.xe, cur.te, ch);
            }
            nrec++;
            ch.depth = cur.depth + 1;
            if (!EMIT && ch.depth > tl.maxdepth) tl.maxdepth = ch.depth;
            // The child's first clock draw, exactly as its own walk would take
            // it: most children do not jump before the end of the step, and
            // then there is nothing to walk and the parent stays off the stack.
            const W4 r0 = draw(ch.id, step, kTagStep, 0u, 0u, seed, key);
            const double u0 = unit53(r0.a, r0.b);
            if (surely_no_jump(u0, cur.te, d.dt, P.gamma0) ||
                !(cur.te + (-ln_series(1.0 - u0) / P.gamma0) <= d.dt))
                continue;
            if (sp >= kMaxDepth) {
                err |= kErrDepth;
                continue;
            }
            // descend into the child; the parent resumes with its "-"
            // offspring (pair kept with the frame) or its next component
            if (side == 0) {
                stackJ[sp] = J;
                stackR[sp] = rc;
                cur.side = 1;
            } else {
                cur.side = 0;
                cur.m += 1;
            }
            descend = true;
        }
        if (!descend) {
            cur.side = 0;
            cur.m += 1;
            continue;
        }
        ch.x[0] = cur.xe[0];
        ch.x[1] = cur.xe[1];
        ch.t0 = cur.te;
        ch.t = ch.t0;
        ch.e = 0;
        ch.in_ev = 0;
        ch.m = 0;
        ch.side = 0;
        stack[sp++] = cur;
        cur = ch;
    }
    return nrec;
}

// Expands node n of the tile's Tree (see Tree): walks its jumps from its
// birth time to the end of the step and appends every kept offspring, and
// the offspring that jump again to the next level.  The draws and the
// arithmetic are walk_family's, so the records are the same.  A family
// whose nodes overflow the Tree is marked in `in_tree` and left to
// walk_family.
template <int DIM, bool SP2, bool TAN>
__device__ void expand_node(const Dev &d, const InstParam &P, uint32_t step, Tree<DIM, SP2, TAN> *tr, int n,
                            int next, uint8_t *in_tree)
{
    const uint32_t seed = d.seed, key = P.key;
    const int M = d.M;
    const int fam = tr->slot[n];
    Node cur;
    cur.x[0] = tr->x0[n];
    cur.k[0] = tr->k0[n];
    cur.x[1] = DIM == 2 ? tr->x1[n] : 0.0;
    cur.k[1] = DIM == 2 ? tr->k1[n] : 0.0;
    cur.t0 = tr->t0[n];
    cur.w = SP2 ? tr->w[n] : 0.0;
    if (TAN) {
        cur.D[0] = tr->D[0][n];
        cur.D[1] = tr->D[1][n];
        cur.D[2] = tr->D[2][n];
    } else {
        cur.D[0] = cur.D[1] = cur.D[2] = 0.0;
    }
    cur.id = tr->id[n];
    cur.sg = SP2 ? 0 : (int32_t)tr->sg[n];
    cur.depth = tr->depth[n];
    uint32_t nkept = 0, nev = 0, npairs = 0;
    int64_t killed = 0;
    uint8_t capped = 0;
    double t = cur.t0;
    for (uint32_t e = 0;; ++e) {
        if (e >= kEventCap) {
            capped = 1;
            break;
        }
        const W4 r = draw(cur.id, step, kTagStep, e, 0u, seed, key);
        const double u = unit53(r.a, r.b);
        const double te = surely_no_jump(u, t, d.dt, P.gamma0) ? d.dt + 1.0 : t + (-ln_series(1.0 - u) / P.gamma0);
        if (!(te <= d.dt)) break;
        nev++;
        cur.e = e;
        cur.te = te;
        cur.ua0 = unit53(r.c, r.d);
        cur.xe[0] = cur.x[0] + (d.vfac * cur.k[0]) * (te - cur.t0);
        cur.xe[1] = DIM == 2 ? cur.x[1] + (d.vfac * cur.k[1]) * (te - cur.t0) : 0.0;
        const int mend = slot_end<TAN>(d, cur, M);
        for (int m = 0; m < mend; ++m) {
            PairDraw J;
            W4 rc;
            if (!slot_draw<SP2, TAN>(d, P, cur, step, m, M, J, rc)) continue;
            if (!TAN || m < M) npairs++;
            for (int side = 0; side < 2; ++side) {
                Node ch;
                slot_child<SP2, TAN>(d, P, cur, m, M, side, J, rc, ch);
                if (!in_kbox<DIM>(d, ch.k)) {          // k-truncation (Sec. 2)
                    killed += killed_amount<SP2>(ch);
                    continue;
                }
                const uint32_t c = atomicAdd(&tr->n, 1u);
                if (c >= (uint32_t)Tree<DIM, SP2, TAN>::kNodes) {
                    in_tree[fam] = 0;
                    continue;
                }
                tr->x0[c] = cur.xe[0];
                tr->k0[c] = ch.k[0];
                if (DIM == 2) {
                    tr->x1[c] = cur.xe[1];
                    tr->k1[c] = ch.k[1];
                }
                tr->t0[c] = te;
                if (SP2) tr->w[c] = ch.w; else tr->sg[c] = (int8_t)ch.sg;
                if (TAN) {
                    tr->D[0][c] = ch.D[0];
                    tr->D[1][c] = ch.D[1];
                    tr->D[2][c] = ch.D[2];
                }
                tr->id[c] = ch.id;
                tr->par[c] = (uint16_t)n;
                tr->rank[c] = (uint16_t)nkept;
                tr->slot[c] = (uint16_t)fam;
                tr->depth[c] = (uint8_t)(cur.depth + 1);
                atomicMax(&tr->maxd, (uint32_t)(cur.depth + 1));
                tr->nch[c] = 0;
                tr->size[c] = 0;
                tr->events[c] = 0;
                tr->pairs[c] = 0;
                tr->killed[c] = 0;
                tr->capped[c] = 0;
                nkept++;
                // the offspring's first clock draw, as its own walk takes it
                const W4 r0 = draw(ch.id, step, kTagStep, 0u, 0u, seed, key);
                const double u0 = unit53(r0.a, r0.b);
                if (!surely_no_jump(u0, te, d.dt, P.gamma0) && te + (-ln_series(1.0 - u0) / P.gamma0) <= d.dt) {
                    tr->front[next][atomicAdd(&tr->nf[next], 1u)] = (uint16_t)c;
                }
            }
        }
        t = te;
    }
    tr->nch[n] = (uint16_t)nkept;
    tr->events[n] = (uint16_t)nev;
    tr->pairs[n] = (uint16_t)npairs;
    tr->killed[n] = killed;
    tr->capped[n] = capped;
}

template <int DIM, bool SP2, bool TAN>
__global__ __launch_bounds__(kThreads, 3) void k_family(Dev d, int ghost)
{
    // A tile holds FS event parents, slot = tid + h * kThreads for h < SPT.
    constexpr int FS = Stash<DIM, SP2, TAN>::F;
    constexpr int SPT = FS / kThreads;
    constexpr int NN = Tree<DIM, SP2, TAN>::kNodes;
    // level-by-level expansion for the 1D kernels (with tangents the table
    // needs 78 KB of LDS, two blocks per CU, which their registers allow
    // anyway); the 4D ones (about half the families of a tile are slow) keep
    // the pool and one depth-first walk per lane
    constexpr bool kTree = DIM == 1;
    __shared__ int64_t s_t;
    __shared__ uint32_t s_wsum[4];
    __shared__ int64_t s_excl;
    __shared__ int64_t s_tal[5];
    __shared__ uint32_t s_nslow;
    __shared__ uint16_t s_slow[FS];          // slots whose family needs the general walk
    __shared__ uint32_t s_cnt[FS];           // record count of every slot
    __shared__ int64_t s_first[FS];          // output offset of every slot's first record
    __shared__ uint8_t s_tree[FS];           // the slot's family is in the Tree (or the pool)
    __shared__ uint8_t s_fast[FS];           // the slot's records are in the stash
    __shared__ Stash<DIM, SP2, TAN> s_stash;
    __shared__ typename std::conditional<kTree, Tree<DIM, SP2, TAN>, Pool<DIM, SP2, TAN>>::type s_walk;

    Ctl *ctl = d.ctl;
    const uint32_t step = ctl->step;
    const int B = d.B;
    const int64_t *plan = d.tileB + (int64_t)ghost * (B + 1);
    const int64_t ntiles = plan[B];
    const uint32_t set = ghost ? ctl->gcur : ctl->cur;
    const Ens E = pick_set(d, ghost, set);
    // records are staged in the inactive buffer set, tile by tile, and
    // placed after the ordered scan by k_place_records
    const Ens S = pick_set(d, ghost, set ^ 1u);
    uint64_t *tcnt = ghost ? d.tcBg : d.tcB;
    uint64_t *tsup = ghost ? d.supBg : d.supB;
    int64_t *tstg = ghost ? d.tsBg : d.tsB;
    const uint32_t *evi = ghost ? d.gev_idx : d.ev_idx;
    const int pass = ghost ? kPassFamilyG : kPassFamily;
    const int64_t dstride = ghost ? d.gcap_total : d.cap_total;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    uint32_t err = 0;

    // the event parent at index i of the particle set, at the start of the
    // step, and that of tile position `slot`
    auto load_root_at = [&](int64_t i) {
        Node root;
        root.x[0] = E.x0[i];
        root.x[1] = DIM == 2 ? E.x1[i] : 0.0;
        root.k[0] = E.k0[i];
        root.k[1] = DIM == 2 ? E.k1[i] : 0.0;
        root.t0 = 0.0;
        root.id = E.id[i];
        root.w = SP2 ? E.w[i] : 0.0;
        root.sg = SP2 ? 0 : (int32_t)E.sg[i];
        if (TAN) {
            root.D[0] = E.D[i];
            root.D[1] = E.D[dstride + i];
            root.D[2] = E.D[2 * dstride + i];
        } else {
            root.D[0] = root.D[1] = root.D[2] = 0.0;
        }
        return root;
    };
    auto load_root = [&](int64_t base, int64_t j0, int slot) {
        return load_root_at(base + (int64_t)evi[base + j0 + slot]);
    };

    // Tallies stay in LDS while the block works on one instance; they go to
    // the instance's counters when the block moves on to another one, and the
    // last instance's share is left in the block's slot of fpart for the
    // closing block of the placement launch.  Per-tile atomics on one cache line would serialise
    // the whole grid.
    int cb = -1;
    bool first = true;
    if (tid < 5) s_tal[tid] = 0;
    for (;;) {
        if (tid == 0) {
            s_t = next_tile_static_first(&ctl->ticket[pass], ntiles, first);
            s_nslow = 0;
            if constexpr (!kTree) s_walk.n = 0;
        }
        __syncthreads();
        const int64_t t = s_t;
        if (t >= ntiles) break;
        const int b = segment_of(plan, B, t);
        if (b != cb) {
            if (tid == 0 && cb >= 0) {
                int64_t *T = d.tally + (int64_t)cb * kTalCount;
                if (s_tal[0]) atomicAdd((unsigned long long *)&T[kTalEvents], (unsigned long long)s_tal[0]);
                if (s_tal[1]) atomicAdd((unsigned long long *)&T[kTalPairs], (unsigned long long)s_tal[1]);
                if (s_tal[2]) atomicAdd((unsigned long long *)&T[kTalKilled], (unsigned long long)s_tal[2]);
                if (s_tal[3]) atomicAdd((unsigned long long *)&T[kTalEventCap], (unsigned long long)s_tal[3]);
                if (s_tal[4]) atomicMax((unsigned long long *)&T[kTalMaxDepth], (unsigned long long)s_tal[4]);
                for (int q = 0; q < 5; ++q) s_tal[q] = 0;
            }
            cb = b;
        }
        const int64_t tl_i = t - plan[b];
        const InstParam &P = d.ip[b];
        const int64_t base = ghost ? P.gbase : P.base;
        const int64_t cap = ghost ? P.gcap : P.cap;
        const int64_t nev = d.evc[(int64_t)ghost * B + b];
        const int64_t j0 = tl_i * FS;

        // 1. every family in lockstep on the common path; a slow family's
        //    partial tallies are dropped (its general walk counts them)
        Tally tal{0, 0, 0, 0, 0};
#pragma unroll
        for (int h = 0; h < SPT; ++h) {
            const int slot = tid + h * kThreads;
            uint32_t cnt = 0;
            bool fast = false;
            if (j0 + slot < nev) {
                const int64_t pi = base + (int64_t)evi[base + j0 + slot];
                const Node root = load_root_at(pi);
                // the parent's position at the end of the step (k_stream left
                // it at the start)
                const double xend0 = root.x[0] + (d.vfac * root.k[0]) * d.dt;
                const double xend1 = DIM == 2 ? root.x[1] + (d.vfac * root.k[1]) * d.dt : 0.0;
                Tally th{0, 0, 0, 0, 0};
                fast = fast_family<DIM, SP2, TAN>(d, P, step, root, &s_stash, slot, cnt, th);
                if (fast) {
                    tal.events += th.events;
                    tal.pairs += th.pairs;
                    tal.killed += th.killed;
                    tal.cap += th.cap;
                    tal.maxdepth = max(tal.maxdepth, th.maxdepth);
                    // nothing in this launch reads a lockstep family's parent
                    // again: it moves now, with no second gather
                    E.x0[pi] = xend0;
                    if (DIM == 2) E.x1[pi] = xend1;
                } else {
                    s_slow[atomicAdd(&s_nslow, 1u)] = (uint16_t)slot;
                }
            }
            s_cnt[slot] = fast ? cnt : 0u;
            s_fast[slot] = fast ? 1 : 0;
        }
        __syncthreads();
        // 2. the other families: level by level in the Tree, or walked depth
        //    first, one family per lane, with their records pooled
        const int nslow = (int)s_nslow;
        const int kme = lane * 4 + wv;
        int nn = 0;                          // Tree nodes
        if constexpr (kTree) {
            auto &tree = s_walk;
            // root k of the slow list is node k; nodes are spread over the
            // block's threads with consecutive ones in different wavefronts
            for (int k = tid; k < nslow; k += kThreads) {
                const int slot = s_slow[k];
                s_tree[slot] = k < NN ? 1 : 0;
                if (k >= NN) continue;
                const Node root = load_root(base, j0, slot);
                tree.x0[k] = root.x[0];
                tree.k0[k] = root.k[0];
                if (DIM == 2) {
                    tree.x1[k] = root.x[1];
                    tree.k1[k] = root.k[1];
                }
                tree.t0[k] = 0.0;
                if (SP2) tree.w[k] = root.w; else tree.sg[k] = (int8_t)root.sg;
                if (TAN) {
                    tree.D[0][k] = root.D[0];
                    tree.D[1][k] = root.D[1];
                    tree.D[2][k] = root.D[2];
                }
                tree.id[k] = root.id;
                tree.slot[k] = (uint16_t)slot;
                tree.depth[k] = 0;
                tree.size[k] = 0;
                tree.nch[k] = 0;
                tree.events[k] = 0;
                tree.pairs[k] = 0;
                tree.killed[k] = 0;
                tree.capped[k] = 0;
                tree.front[0][k] = (uint16_t)k;
            }
            if (tid == 0) {
                const uint32_t nr = (uint32_t)min(nslow, NN);
                tree.n = nr;
                tree.nf[0] = nr;
                tree.nf[1] = 0;
                tree.maxd = 0;
            }
            __syncthreads();
            for (int lv = 0;; lv ^= 1) {
                const uint32_t nf = tree.nf[lv];
                if (nf == 0) break;
                for (uint32_t k = kme; k < nf; k += kThreads) {
                    const int n = tree.front[lv][k];
                    if (s_tree[tree.slot[n]]) expand_node<DIM, SP2, TAN>(d, P, step, &tree, n, lv ^ 1, s_tree);
                }
                __syncthreads();
                if (tid == 0) tree.nf[lv] = 0;
                __syncthreads();
            }
            nn = (int)min(tree.n, (uint32_t)NN);
            const int maxd = (int)tree.maxd;
            // subtree sizes, deepest level first (a root gets its family's count)
            for (int dd = maxd; dd >= 1; --dd) {
                for (int k = tid; k < nn; k += kThreads)
                    if (tree.depth[k] == dd) {
                        const uint32_t sz = tree.size[k] + 1u;
                        tree.size[k] = sz;
                        atomicAdd(&tree.size[tree.par[k]], sz);
                    }
                __syncthreads();
            }
            // offspring grouped by parent (exclusive scan of the offspring counts
            // in node order), then depth-first positions, top level first
            {
                constexpr int NPT = NN / kThreads;    // nodes tid * NPT + q, q < NPT
                uint32_t c[NPT], csum = 0;
    #pragma unroll
                for (int q = 0; q < NPT; ++q) {
                    const int k = tid * NPT + q;
                    c[q] = k < nn ? (uint32_t)tree.nch[k] : 0u;
                    csum += c[q];
                }
                uint32_t incl = csum;
    #pragma unroll
                for (int o = 1; o < 64; o <<= 1) {
                    const uint32_t v = __shfl_up(incl, o, 64);
                    if (lane >= o) incl += v;
                }
                if (lane == 63) s_wsum[wv] = incl;
                __syncthreads();
                uint32_t run = incl - csum;
                for (int q = 0; q < wv; ++q) run += s_wsum[q];
    #pragma unroll
                for (int q = 0; q < NPT; ++q) {
                    const int k = tid * NPT + q;
                    if (k < nn) {
                        tree.cst[k] = (uint16_t)run;
                        if (tree.depth[k] == 0) tree.pos[k] = -1;
                    }
                    run += c[q];
                }
                __syncthreads();
            }
            for (int k = tid; k < nn; k += kThreads)
                if (tree.depth[k] > 0) tree.child[tree.cst[tree.par[k]] + tree.rank[k]] = (uint16_t)k;
            __syncthreads();
            for (int dd = 0; dd < maxd; ++dd) {
                for (int k = tid; k < nn; k += kThreads)
                    if (tree.depth[k] == dd) {
                        int run = tree.pos[k] + 1;
                        const int c0 = tree.cst[k], nc = tree.nch[k];
                        for (int j = 0; j < nc; ++j) {
                            const int c = tree.child[c0 + j];
                            tree.pos[c] = (int16_t)run;
                            run += (int)tree.size[c];
                        }
                    }
                __syncthreads();
            }
            // record counts, tallies (from the Tree, or by a counting walk for the
            // families that did not fit)
            for (int k = tid; k < nn; k += kThreads) {
                if (!s_tree[tree.slot[k]]) continue;
                tal.events += tree.events[k];
                tal.pairs += tree.pairs[k];
                tal.killed += tree.killed[k];
                tal.cap += tree.capped[k];
                tal.maxdepth = max(tal.maxdepth, (int32_t)tree.depth[k]);
            }
            for (int k = kme; k < nslow; k += kThreads) {
                const int slot = s_slow[k];
                if (s_tree[slot]) {
                    s_cnt[slot] = tree.size[k];
                    continue;
                }
                const Node root = load_root(base, j0, slot);
                bool unused = false;
                s_cnt[slot] = walk_family<DIM, SP2, TAN, false>(d, P, step, root, E, base, 0, cap, dstride, tal, err,
                                                                nullptr, slot, unused);
            }
            __syncthreads();

        } else {
            auto &s_pool = s_walk;
            for (int k = kme; k < nslow; k += kThreads) {
                const int slot = s_slow[k];
                const Node root = load_root(base, j0, slot);
                bool pooled = true;
                s_cnt[slot] = walk_family<DIM, SP2, TAN, false>(d, P, step, root, E, base, 0, cap, dstride, tal,
                                                                err, &s_pool, slot, pooled);
                s_tree[slot] = pooled ? 1 : 0;
            }
            __syncthreads();
        }

        // 3. ordered exclusive scan of the record counts over the tile, in
        //    slot order (h, then tid)
        uint32_t excl[SPT];
        uint32_t agg = 0;
#pragma unroll
        for (int h = 0; h < SPT; ++h) {
            const uint32_t c = s_cnt[tid + h * kThreads];
            uint32_t incl = c;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const uint32_t v = __shfl_up(incl, o, 64);
                if (lane >= o) incl += v;
            }
            if (lane == 63) s_wsum[wv] = incl;
            __syncthreads();
            uint32_t woff = 0, part = 0;
            for (int q = 0; q < 4; ++q) {
                if (q < wv) woff += s_wsum[q];
                part += s_wsum[q];
            }
            excl[h] = agg + woff + incl - c;
            agg += part;
            __syncthreads();
        }
        if (tid == 0) {
            // the tile's records take a contiguous stretch of the staging
            // area; no tile waits for another
            const int64_t sb = (int64_t)atomicAdd((unsigned long long *)&d.stg[(int64_t)ghost * B + b],
                                                  (unsigned long long)agg);
            s_excl = sb;
            tcnt[t] = agg;
            tstg[t] = sb;
            if (agg)
                atomicAdd((unsigned long long *)&tsup[(t / kSupGroup) * kSupStride], (unsigned long long)agg);
        }
        __syncthreads();
#pragma unroll
        for (int h = 0; h < SPT; ++h) s_first[tid + h * kThreads] = s_excl + (int64_t)excl[h];

        // 4. records into the staging area: from the stash and the Tree (or
        //    the pool), or by a second full walk for a family that did not fit
#pragma unroll
        for (int h = 0; h < SPT; ++h) {
            const int slot = tid + h * kThreads;
            if (!s_fast[slot]) continue;
            const uint32_t cnt = s_cnt[slot];
            const int64_t my_first = s_excl + (int64_t)excl[h];
            const double xe0 = s_stash.xe0[slot], xe1 = DIM == 2 ? s_stash.xe1[slot] : 0.0;
            const double rest = d.dt - s_stash.te[slot];
            for (uint32_t r = 0; r < cnt; ++r) {
                const int64_t li = my_first + r;
                if (li >= cap) { err |= kErrCapacity; continue; }
                const int64_t o = base + li;
                const double k0 = s_stash.k0[r][slot];
                S.x0[o] = xe0 + (d.vfac * k0) * rest;
                S.k0[o] = k0;
                if (DIM == 2) {
                    const double k1 = s_stash.k1[r][slot];
                    S.x1[o] = xe1 + (d.vfac * k1) * rest;
                    S.k1[o] = k1;
                }
                if (SP2) S.w[o] = s_stash.w[r][slot]; else S.sg[o] = s_stash.sg[r][slot];
                S.id[o] = s_stash.id[r][slot];
                if (TAN) {
                    S.D[o] = s_stash.D[3 * r][slot];
                    S.D[dstride + o] = s_stash.D[3 * r + 1][slot];
                    S.D[2 * dstride + o] = s_stash.D[3 * r + 2][slot];
                }
            }
        }
        __syncthreads();
        if constexpr (kTree) {
            auto &tree = s_walk;
            for (int k = tid; k < nn; k += kThreads) {
                if (tree.depth[k] == 0 || !s_tree[tree.slot[k]]) continue;
                const int64_t li = s_first[tree.slot[k]] + tree.pos[k];
                if (li >= cap) { err |= kErrCapacity; continue; }
                const int64_t o = base + li;
                const double t0 = tree.t0[k];
                S.x0[o] = tree.x0[k] + (d.vfac * tree.k0[k]) * (d.dt - t0);
                S.k0[o] = tree.k0[k];
                if (DIM == 2) {
                    S.x1[o] = tree.x1[k] + (d.vfac * tree.k1[k]) * (d.dt - t0);
                    S.k1[o] = tree.k1[k];
                }
                if (SP2) S.w[o] = tree.w[k]; else S.sg[o] = tree.sg[k];
                S.id[o] = tree.id[k];
                if (TAN) {
                    S.D[o] = tree.D[0][k];
                    S.D[dstride + o] = tree.D[1][k];
                    S.D[2 * dstride + o] = tree.D[2][k];
                }
            }
            for (int k = kme; k < nslow; k += kThreads) {
                const int slot = s_slow[k];
                if (s_tree[slot]) continue;
                const Node root = load_root(base, j0, slot);
                Tally none{0, 0, 0, 0, 0};
                bool unused = false;
                walk_family<DIM, SP2, TAN, true>(d, P, step, root, S, base, s_first[slot], cap, dstride, none, err,
                                                 nullptr, slot, unused);
            }
        } else {
            auto &s_pool = s_walk;
            const int npool = (int)min(s_pool.n, (uint32_t)kPool);
            for (int r = tid; r < npool; r += kThreads) {
                const int slot = s_pool.slot[r];
                if (!s_tree[slot]) continue;
                const int64_t li = s_first[slot] + s_pool.rank[r];
                if (li >= cap) { err |= kErrCapacity; continue; }
                const int64_t o = base + li;
                S.x0[o] = s_pool.x0[r];
                S.k0[o] = s_pool.k0[r];
                if (DIM == 2) {
                    S.x1[o] = s_pool.x1[r];
                    S.k1[o] = s_pool.k1[r];
                }
                if (SP2) S.w[o] = s_pool.w[r]; else S.sg[o] = s_pool.sg[r];
                S.id[o] = s_pool.id[r];
                if (TAN) {
                    S.D[o] = s_pool.D[0][r];
                    S.D[dstride + o] = s_pool.D[1][r];
                    S.D[2 * dstride + o] = s_pool.D[2][r];
                }
            }
            // the overflow area (written by this block's threads before the
            // last barrier)
            const int ngp = (int)min(s_pool.n - min(s_pool.n, (uint32_t)kPool), gpool_cap(d));
            if (ngp) {
                const GPoolView v = gpool_view(d);
                for (int g = tid; g < ngp; g += kThreads) {
                    const uint32_t sr = v.sr[g];
                    const int slot = (int)(sr & 0xFFFFu);
                    if (!s_tree[slot]) continue;
                    const int64_t li = s_first[slot] + (int64_t)(sr >> 16);
                    if (li >= cap) { err |= kErrCapacity; continue; }
                    const int64_t o = base + li;
                    S.x0[o] = v.f[g];
                    S.k0[o] = v.f[kGPool + g];
                    if (DIM == 2) {
                        S.x1[o] = v.f[2 * kGPool + g];
                        S.k1[o] = v.f[3 * kGPool + g];
                    }
                    if (SP2) S.w[o] = v.f[4 * kGPool + g]; else S.sg[o] = v.sg[g];
                    S.id[o] = v.id[g];
                    if (TAN) {
                        S.D[o] = v.f[5 * kGPool + g];
                        S.D[dstride + o] = v.f[6 * kGPool + g];
                        S.D[2 * dstride + o] = v.f[7 * kGPool + g];
                    }
                }
            }
            for (int k = kme; k < nslow; k += kThreads) {
                const int slot = s_slow[k];
                if (s_tree[slot]) continue;
                const Node root = load_root(base, j0, slot);
                Tally none{0, 0, 0, 0, 0};
                bool unused = false;
                walk_family<DIM, SP2, TAN, true>(d, P, step, root, S, base, s_first[slot], cap, dstride, none, err,
                                                 &s_pool, slot, unused);
            }
        }

        // per-instance tallies, summed over the wavefront first
        int64_t tv[4] = {tal.events, tal.pairs, tal.killed, tal.cap};
        int64_t tm = tal.maxdepth;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
            for (int q = 0; q < 4; ++q) tv[q] += __shfl_xor(tv[q], o, 64);
            tm = max(tm, __shfl_xor(tm, o, 64));
        }
        if (lane == 0) {
            for (int q = 0; q < 4; ++q)
                if (tv[q]) atomicAdd((unsigned long long *)&s_tal[q], (unsigned long long)tv[q]);
            if (tm) atomicMax((unsigned long long *)&s_tal[4], (unsigned long long)tm);
        }
        __syncthreads();
        // every walk of this tile is done: the other parents move to the end
        // of the step
#pragma unroll
        for (int h = 0; h < SPT; ++h) {
            const int slot = tid + h * kThreads;
            if (j0 + slot < nev && !s_fast[slot]) {
                const int64_t pi = base + (int64_t)evi[base + j0 + slot];
                E.x0[pi] = E.x0[pi] + (d.vfac * E.k0[pi]) * d.dt;
                if (DIM == 2) E.x1[pi] = E.x1[pi] + (d.vfac * E.k1[pi]) * d.dt;
            }
        }
    }
    if (tid == 0) {
        int64_t *F = d.fpart + (int64_t)blockIdx.x * 8;
        F[0] = cb;
        for (int q = 0; q < 5; ++q) F[1 + q] = s_tal[q];
    }
    if (err) atomicOr(&ctl->err, err);
}

__device__ void close_family(const Dev &d, int ghost, int advance, int fgrid);

// Every family tile's staged records (contiguous in the inactive buffer set)
// go to their place after the instance's particles: tile order, then the
// order of the family walks within the tile.  Block 0 (dispatched first)
// closes the step (close_family).
template <int DIM, bool SP2, bool TAN>
__global__ __launch_bounds__(kThreads) void k_place_records(Dev d, int ghost, int advance, int fgrid)
{
    if (blockIdx.x == 0) {
        close_family(d, ghost, advance, fgrid);
        return;
    }
    Ctl *ctl = d.ctl;
    const int B = d.B;
    const int64_t *plan = d.tileB + (int64_t)ghost * (B + 1);
    const int64_t ntiles = plan[B];
    const int64_t *Nb = d.Nbase + (int64_t)ghost * B;   // counts at the start of the step
    const uint32_t set = ghost ? ctl->gcur : ctl->cur;
    const Ens E = pick_set(d, ghost, set);
    const Ens S = pick_set(d, ghost, set ^ 1u);
    const uint64_t *tc = ghost ? d.tcBg : d.tcB;
    const uint64_t *sup = ghost ? d.supBg : d.supB;
    const int64_t *ts = ghost ? d.tsBg : d.tsB;
    __shared__ uint64_t s_w[kThreads / 64];
    const int64_t dstride = ghost ? d.gcap_total : d.cap_total;
    uint32_t err = 0;
    for (int64_t t = blockIdx.x - 1; t < ntiles; t += gridDim.x - 1) {
        const int b = segment_of(plan, B, t);
        const InstParam &P = d.ip[b];
        const int64_t base = ghost ? P.gbase : P.base;
        const int64_t cap = ghost ? P.gcap : P.cap;
        const int64_t n = (int64_t)tc[t], src = ts[t];
        // a record staged past the capacity was never written (k_family
        // flagged it); one whose place is past the capacity is an overflow
        struct Rec { double x0, x1, k0, k1, w, D[3]; uint64_t id; int8_t sg; };
        auto load = [&](int64_t r) {
            Rec q;
            const int64_t i = base + src + r;
            q.x0 = S.x0[i];
            q.k0 = S.k0[i];
            q.x1 = DIM == 2 ? S.x1[i] : 0.0;
            q.k1 = DIM == 2 ? S.k1[i] : 0.0;
            q.w = SP2 ? S.w[i] : 0.0;
            q.sg = SP2 ? (int8_t)0 : S.sg[i];
            q.id = S.id[i];
            for (int c = 0; c < 3; ++c) q.D[c] = TAN ? S.D[c * dstride + i] : 0.0;
            return q;
        };
        auto store = [&](int64_t r, const Rec &q, int64_t dst) {
            if (dst + r >= cap) { err |= kErrCapacity; return; }
            const int64_t o = base + dst + r;
            E.x0[o] = q.x0;
            E.k0[o] = q.k0;
            if (DIM == 2) {
                E.x1[o] = q.x1;
                E.k1[o] = q.k1;
            }
            if (SP2) E.w[o] = q.w; else E.sg[o] = q.sg;
            E.id[o] = q.id;
            if (TAN)
                for (int c = 0; c < 3; ++c) E.D[c * dstride + o] = q.D[c];
        };
        // the first records of the tile are loaded before the tile's place
        // is summed, so that the two overlap
        constexpr int kPre = 4;
        Rec pre[kPre];
#pragma unroll
        for (int h = 0; h < kPre; ++h) {
            const int64_t r = threadIdx.x + (int64_t)h * kThreads;
            if (r < n && src + r < cap) pre[h] = load(r);
        }
        const int64_t dst = Nb[b] + (int64_t)block_range_sum(TileRange(tc, sup, plan[b], t), s_w);
#pragma unroll
        for (int h = 0; h < kPre; ++h) {
            const int64_t r = threadIdx.x + (int64_t)h * kThreads;
            if (r < n && src + r < cap) store(r, pre[h], dst);
        }
        for (int64_t r = threadIdx.x + (int64_t)kPre * kThreads; r < n && src + r < cap; r += kThreads)
            store(r, load(r), dst);
    }
    if (err) atomicOr(&ctl->err, err);
}

// After k_family, in the first block of the placement launch: the family
// blocks' tallies, the new particle counts with the capacity clamp, cleared
// event and record counts, the streaming-tile plan of the next step, and the
// step counter.  Nothing here is read by the placing blocks: they take the
// particle counts kept by k_events, and the family-tile group sums are
// cleared by the next k_events.
__device__ void close_family(const Dev &d, int ghost, int advance, int fgrid)
{
    Ctl *ctl = d.ctl;
    const int B = d.B;
    int64_t *Ncur = ghost ? d.NG : d.N;
    int64_t *rec = d.stg + (int64_t)ghost * B;   // records of the step (staging fill)
    int64_t *evc = d.evc + (int64_t)ghost * B;
    const int tid = threadIdx.x;
    // Loads that do not depend on the family blocks' tallies go first, so
    // that their latency overlaps the reduction below; thread b < kThreads
    // keeps instance b's values in registers.
    const uint32_t step = ctl->step;
    const int64_t tilesA = d.tileA[(int64_t)ghost * (B + 1) + B];
    const bool own = tid < B;
    int64_t n_own = 0, rec_own = 0, cap_own = 0, tal_own[kTalCount] = {};
    if (own) {
        n_own = Ncur[tid];
        rec_own = rec[tid];
        cap_own = ghost ? d.ip[tid].gcap : d.ip[tid].cap;
#pragma unroll
        for (int q = 0; q < kTalCount; ++q) tal_own[q] = d.tally[(int64_t)tid * kTalCount + q];
    }
    // the family blocks' last tallies, summed per instance in LDS when the
    // instances fit (global atomics from one block on one line serialise)
    constexpr int kLdsB = 256;
    __shared__ int64_t s_acc[5][kLdsB];
    const bool lds = B <= kLdsB;
    if (lds)
        for (int b = tid; b < B; b += kThreads)
            for (int q = 0; q < 5; ++q) s_acc[q][b] = 0;
    __syncthreads();
    for (int g = tid; g < fgrid; g += kThreads) {
        const int64_t *F = d.fpart + (int64_t)g * 8;
        if (F[0] < 0) continue;
        if (lds) {
            const int b = (int)F[0];
            for (int q = 0; q < 4; ++q)
                if (F[1 + q]) atomicAdd((unsigned long long *)&s_acc[q][b], (unsigned long long)F[1 + q]);
            if (F[5]) atomicMax((unsigned long long *)&s_acc[4][b], (unsigned long long)F[5]);
        } else {
            int64_t *T = d.tally + F[0] * kTalCount;
            if (F[1]) atomicAdd((unsigned long long *)&T[kTalEvents], (unsigned long long)F[1]);
            if (F[2]) atomicAdd((unsigned long long *)&T[kTalPairs], (unsigned long long)F[2]);
            if (F[3]) atomicAdd((unsigned long long *)&T[kTalKilled], (unsigned long long)F[3]);
            if (F[4]) atomicAdd((unsigned long long *)&T[kTalEventCap], (unsigned long long)F[4]);
            if (F[5]) atomicMax((unsigned long long *)&T[kTalMaxDepth], (unsigned long long)F[5]);
        }
    }
    __syncthreads();
    int64_t n_next = 0;   // instance tid's count for the next step
    int over = 0;         // an instance of this thread holds more than ann_limit
    for (int b = tid; b < B; b += kThreads) {
        const bool mine = b == tid;
        int64_t *T = d.tally + (int64_t)b * kTalCount;
        if (lds) {   // (the global path above already added its atomics)
            const int64_t ev = mine ? tal_own[kTalEvents] : T[kTalEvents];
            const int64_t pr = mine ? tal_own[kTalPairs] : T[kTalPairs];
            const int64_t kl = mine ? tal_own[kTalKilled] : T[kTalKilled];
            const int64_t ec = mine ? tal_own[kTalEventCap] : T[kTalEventCap];
            const int64_t md = mine ? tal_own[kTalMaxDepth] : T[kTalMaxDepth];
            T[kTalEvents] = ev + s_acc[0][b];
            T[kTalPairs] = pr + s_acc[1][b];
            T[kTalKilled] = kl + s_acc[2][b];
            T[kTalEventCap] = ec + s_acc[3][b];
            if (s_acc[4][b] > md) T[kTalMaxDepth] = s_acc[4][b];
        }
        const int64_t n0 = mine ? n_own : Ncur[b];
        const int64_t cap = mine ? cap_own : (ghost ? d.ip[b].gcap : d.ip[b].cap);
        if (!ghost) T[kTalPSteps] = (mine ? tal_own[kTalPSteps] : T[kTalPSteps]) + n0;
        int64_t n = n0 + (mine ? rec_own : rec[b]);
        rec[b] = 0;
        if (n > cap) {
            atomicOr(&ctl->err, kErrCapacity);
            n = cap;
        }
        Ncur[b] = n;
        if (mine) n_next = n;
        evc[b] = 0;
        if (d.ann_limit > 0 && n > d.ann_limit) over = 1;
    }
    // conditional annihilation after this step: scheduled, or an instance
    // about to outgrow the threshold (the real ensemble's closing block)
    const int any_over = __syncthreads_or(over);
    if (d.cond_ann && !ghost && tid == 0) {
        const bool sched = d.ann_every > 0 && (step + 1u) % (uint32_t)d.ann_every == 0u;
        ctl->ann_now = (sched || any_over) ? 1u : 0u;
        if (any_over && !sched)
            for (int b = 0; b < B; ++b) d.tally[(int64_t)b * kTalCount + kTalTrig] += 1;
    }
    {   // clear the group sums of this step's streaming tiles
        uint64_t *supA = ghost ? d.supAg : d.supA;
        const int64_t na = (tilesA + kSupGroup - 1) / kSupGroup;
        for (int64_t g = tid; g < na; g += kThreads) supA[g * kSupStride] = 0;
    }
    __syncthreads();
    // the next step's tile plan (block_prefix evaluates instance b on thread
    // b mod kThreads, which wrote Ncur[b] above)
    block_prefix(d.tileA + (int64_t)ghost * (B + 1), B, [&](int b) {
        const int64_t n = b == tid ? n_next : Ncur[b];
        return (n + kTileA - 1) / kTileA;
    });
    if (tid == 0 && advance) ctl->step = step + 1u;
}

}  // namespace wbrw
