// One time step of the Wigner branching random walk (Alg. 1, Sec. 2) as two
// persistent kernels.
//
// Pass 1, k_stream (HBM-bound): every particle draws its first life-length
// (exact for a constant gamma0, Sec. 3.2.1), moves freely to the end of the
// step (a particle keeps its k after a jump: offspring 2M+1 of Alg. 1, so its
// end position does not depend on its jumps) and, if its first jump falls
// inside the step, is appended to an ordered per-instance event list together
// with its start position.  Ordering uses a wavefront ballot, an LDS scan over
// the block and a decoupled look-back across tiles.  Only the first of the
// two uniforms decides, and only a 1e-9-wide band around the threshold
// evaluates the logarithm.
//
// Pass 2, k_family (latency-bound, ~3% of particles): one thread per event
// parent walks the parent's whole family within the step, depth first: for
// each jump in time order, each component in order, the "+" offspring, its own
// family, then the "-" offspring and its family.  Offspring are new particles
// of the system with their own lineage ids and exponential clocks (Alg. 1
// rule 3).  A first walk counts the records and keeps the first two in LDS;
// after an ordered scan with look-back fixes the output offset, families of
// at most two records (nearly all) are copied out and only larger ones are
// walked again to write them.  A child whose first clock draw falls past the
// end of the step is a leaf and never enters the walk's stack.  Records hold
// the end-of-step state, so no generation is revisited in a later launch.
#pragma once
#include "wbrw_dev.hpp"
#include "wbrw_math.hpp"

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
// piecewise-constant table with a uniform offset inside the chosen bin.
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
    int lo = 0, hi = T.n - 1;
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

// ---------------------------------------------------------------------------
// Pass 1: streaming clock test + free flight + ordered event compaction
// ---------------------------------------------------------------------------
template <int DIM>
__global__ __launch_bounds__(kThreads) void k_stream(Dev d, int ghost)
{
    __shared__ int64_t s_t;
    __shared__ uint32_t s_wcnt[kPPT * 4];
    __shared__ uint32_t s_woff[kPPT * 4];
    __shared__ uint32_t s_excl;

    Ctl *ctl = d.ctl;
    const uint32_t step = ctl->step;
    const uint32_t epoch = 2u * step + (uint32_t)ghost + 1u;
    const int B = d.B;
    const int64_t *plan = d.tileA + (int64_t)ghost * (B + 1);
    const int64_t ntiles = plan[B];
    const int64_t *Ncur = ghost ? d.NG : d.N;
    const Ens E = pick_set(d, ghost, ghost ? ctl->gcur : ctl->cur);
    uint64_t *st = ghost ? d.stAg : d.stA;
    uint32_t *evi = ghost ? d.gev_idx : d.ev_idx;
    double *evx0 = ghost ? d.gev_x0 : d.ev_x0;
    double *evx1 = ghost ? d.gev_x1 : d.ev_x1;
    const int pass = ghost ? kPassStreamG : kPassStream;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;

    for (;;) {
        if (tid == 0) s_t = next_tile(&ctl->ticket[pass], ntiles);
        __syncthreads();
        const int64_t t = s_t;
        if (t >= ntiles) break;
        const int b = segment_of(plan, B, t);
        const int64_t first = plan[b];
        const int64_t tl = t - first;
        const int64_t last = plan[b + 1] - 1;
        const InstParam &P = d.ip[b];
        const int64_t base = ghost ? P.gbase : P.base;
        const int64_t n = Ncur[b];
        const double thr_lo = P.thr_lo, thr_hi = P.thr_hi, g0 = P.gamma0;
        const uint32_t key = P.key;

        // All loads of the thread's kPPT particles are issued before any
        // compute or store, so every wave keeps 3*kPPT (4D: 5*kPPT) loads in
        // flight; full tiles need no bounds checks.
        const int64_t li0 = tl * kTileA + tid;
        const bool full = (tl + 1) * kTileA <= n;
        double xs0[kPPT], xs1[kPPT], kv0[kPPT], kv1[kPPT];
        uint64_t idv[kPPT];
        if (full) {
#pragma unroll
            for (int j = 0; j < kPPT; ++j) {
                const int64_t i = base + li0 + (int64_t)j * kThreads;
                xs0[j] = E.x0[i];
                kv0[j] = E.k0[i];
                idv[j] = E.id[i];
                if (DIM == 2) { xs1[j] = E.x1[i]; kv1[j] = E.k1[i]; }
            }
        } else {
#pragma unroll
            for (int j = 0; j < kPPT; ++j) {
                const int64_t li = li0 + (int64_t)j * kThreads;
                const int64_t i = base + (li < n ? li : 0);
                xs0[j] = E.x0[i];
                kv0[j] = E.k0[i];
                idv[j] = E.id[i];
                if (DIM == 2) { xs1[j] = E.x1[i]; kv1[j] = E.k1[i]; }
            }
        }
        uint32_t rank[kPPT];
        uint32_t evbits = 0;
#pragma unroll
        for (int j = 0; j < kPPT; ++j) {
            const bool valid = full || (li0 + (int64_t)j * kThreads < n);
            bool ev = false;
            const W4 r = draw(idv[j], step, kTagStep, 0u, 0u, d.seed, key);
            const double u = unit53(r.a, r.b);
            if (u < thr_lo) {
                ev = true;
            } else if (u <= thr_hi) {
                const double tau = -ln_series(1.0 - u) / g0;
                const double te = 0.0 + tau;
                ev = (te <= d.dt);
            }
            ev = ev && valid;
            const uint64_t m = __ballot(ev);
            rank[j] = lane_rank(m);
            if (lane == 0) s_wcnt[j * 4 + wv] = (uint32_t)__popcll(m);
            evbits |= (ev ? 1u : 0u) << j;
        }
        // free flight to the end of the step
#pragma unroll
        for (int j = 0; j < kPPT; ++j) {
            const int64_t li = li0 + (int64_t)j * kThreads;
            if (full || li < n) {
                const int64_t i = base + li;
                E.x0[i] = xs0[j] + (d.vfac * kv0[j]) * d.dt;
                if (DIM == 2) E.x1[i] = xs1[j] + (d.vfac * kv1[j]) * d.dt;
            }
        }
        __syncthreads();
        if (wv == 0) {
            // exclusive scan of the kPPT x 4 wave counts, in (j, wave) order
            static_assert(kPPT * 4 <= 64, "one lane per (particle slot, wave)");
            const uint32_t c = lane < kPPT * 4 ? s_wcnt[lane] : 0u;
            uint32_t inc = c;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const uint32_t v = __shfl_up(inc, o, 64);
                if (lane >= o) inc += v;
            }
            if (lane < kPPT * 4) s_woff[lane] = inc - c;
            const uint32_t acc = __shfl(inc, 63, 64);
            const uint32_t excl = tile_prefix(st, t, first, epoch, acc);
            if (lane == 0) {
                if (t == last) d.evc[(int64_t)ghost * B + b] = (int64_t)(excl + acc);
                s_excl = excl;
            }
        }
        __syncthreads();
        const uint32_t ex = s_excl;
#pragma unroll
        for (int j = 0; j < kPPT; ++j) {
            if ((evbits >> j) & 1u) {
                const int64_t pos = base + ex + s_woff[j * 4 + wv] + rank[j];
                evi[pos] = (uint32_t)(tl * kTileA + (int64_t)j * kThreads + tid);
                evx0[pos] = xs0[j];
                if (DIM == 2) evx1[pos] = xs1[j];
            }
        }
        __syncthreads();
    }

}

// After k_stream (one block): the family-tile plan from the event counts,
// cleared record counts, and the particle-step tally.
__global__ __launch_bounds__(kThreads) void k_close_stream(Dev d, int ghost)
{
    const int B = d.B;
    const int64_t *Ncur = ghost ? d.NG : d.N;
    block_plan(d.tileB + (int64_t)ghost * (B + 1), d.evc + (int64_t)ghost * B, B, kTileB);
    for (int b = threadIdx.x; b < B; b += kThreads) {
        d.chc[(int64_t)ghost * B + b] = 0;
        if (!ghost) d.tally[(int64_t)b * kTalCount + kTalPSteps] += Ncur[b];
    }
}

// ---------------------------------------------------------------------------
// Pass 2: family trees of event parents
// ---------------------------------------------------------------------------
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

struct Tally {
    int64_t events, pairs, killed, cap;
    int32_t maxdepth;
};

// The first kStash records of each thread's family, kept in LDS by the
// counting walk: a family with at most kStash records (most of them: one
// pair) is copied out after the scan instead of being walked a second time.
constexpr int kStash = 2;
template <int DIM, bool SP2, bool TAN>
struct Stash {
    double x0[kStash][kTileB], k0[kStash][kTileB];
    double x1[DIM == 2 ? kStash : 1][DIM == 2 ? kTileB : 1];
    double k1[DIM == 2 ? kStash : 1][DIM == 2 ? kTileB : 1];
    double w[SP2 ? kStash : 1][SP2 ? kTileB : 1];
    double D[TAN ? 3 * kStash : 1][TAN ? kTileB : 1];
    uint64_t id[kStash][kTileB];
    int8_t sg[kStash][kTileB];
};

template <int DIM, bool SP2, bool TAN, bool EMIT>
__device__ uint32_t walk_family(const Dev &d, const InstParam &P, uint32_t step, Node cur,
                                const Ens &out, int64_t base, int64_t first_rec, int64_t cap,
                                int64_t dstride, Tally &tl, uint32_t &err,
                                Stash<DIM, SP2, TAN> *sh)
{
    Node stack[kMaxDepth];
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
                const double tau = -ln_series(1.0 - u) / P.gamma0;
                const double te = cur.t + tau;
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
        if (cur.m >= M) {
            cur.t = cur.te;
            cur.e += 1u;
            cur.in_ev = 0;
            continue;
        }
        const int m = cur.m;
        double q, arg, sn, cm = P.c[m], sgv = P.sgnV[m];
        bool alg4 = false;
        if (d.sampler[m] == 1) {
            // Alg. 1 sp1 box with Pr = xi(x)/gamma0, kick by Alg. 4
            const double r = phase_offset(d, m, cur.xe, P.center[m]);
            double ua = cur.ua0;
            if (m > 0) {
                const W4 ra = draw(cur.id, step, kTagStep, cur.e, (uint32_t)(8 + m), seed, key);
                ua = unit53(ra.a, ra.b);
            }
            const double *tab = d.xi_tab + ((int64_t)(&P - d.ip) * d.M + m) * (kXiN + 1);
            double qk = 0.0;
            if (!(ua < xi_lerp(tab, P.xi_h[m], r) / P.gamma0) || !reject_kick(d, P, cur.id, step, cur.e, m, r, qk)) {
                cur.m += 1;
                cur.side = 0;
                continue;
            }
            q = qk;
            arg = (2.0 * qk) * r;
            sn = 1.0;
            sgv = 1.0;
            alg4 = true;
        } else {
            const W4 rq = draw(cur.id, step, kTagStep, cur.e, (uint32_t)(1 + m), seed, key);
            q = kick_sample(d, P, m, unit53(rq.a, rq.b), unit53(rq.c, rq.d));
            arg = (2.0 * q) * phase_offset(d, m, cur.xe, P.center[m]);
            sn = sin_det(arg);
        }
        if (d.tdep && d.kind[m] == 0 && !alg4) {   // Remark 1: kernel at the absolute jump time
            const double tabs = (double)step * d.dt + cur.te;
            const double f = P.ma[m] + P.mb[m] * cos_det(P.mw[m] * tabs + P.mp[m]);
            const double He = P.H[m] * f;
            cm = ((2.0 * fabs(He)) / d.hbar) / (2.0 * P.gamma0);
            sgv = He >= 0.0 ? 1.0 : -1.0;
        }
        const double sigma = (sn > 0.0) ? sgv : -sgv;
        double amp = 0.0;
        if (!SP2 && !alg4) {
            double ua = cur.ua0;
            if (m > 0) {
                const W4 ra = draw(cur.id, step, kTagStep, cur.e, (uint32_t)(8 + m), seed, key);
                ua = unit53(ra.a, ra.b);
            }
            if (!(ua < cm * fabs(sn))) {       // no pair: only the survivor continues
                cur.m += 1;
                cur.side = 0;
                continue;
            }
        } else if (SP2) {
            amp = cur.w * (cm * fabs(sn));
        }
        const int side = cur.side;
        if (!EMIT && side == 0) tl.pairs++;
        if (side == 0) { cur.side = 1; } else { cur.side = 0; cur.m += 1; }

        const W4 rc = draw(cur.id, step, kTagChild, cur.e, (uint32_t)m, seed, key);
        const uint64_t cls = ((cur.id >> 62) & 1ull) ? 3ull : 2ull;
        const uint64_t cid = side == 0
            ? ((cls << 62) | ((uint64_t)(rc.b & 0x3FFFFFFFu) << 32) | (uint64_t)rc.a)
            : ((cls << 62) | ((uint64_t)(rc.d & 0x3FFFFFFFu) << 32) | (uint64_t)rc.c);
        const double kick = sigma * q;
        Node ch;
        ch.k[0] = cur.k[0];
        ch.k[1] = cur.k[1];
        const int ax = d.axis[m];
        if (ax == 0) {
            ch.k[0] = side == 0 ? cur.k[0] + kick : cur.k[0] - kick;
        } else if (ax == 1) {
            ch.k[1] = side == 0 ? cur.k[1] + kick : cur.k[1] - kick;
        } else {
            ch.k[0] = side == 0 ? cur.k[0] + kick : cur.k[0] - kick;
            ch.k[1] = side == 0 ? cur.k[1] - kick : cur.k[1] + kick;
        }
        ch.sg = side == 0 ? cur.sg : -cur.sg;
        ch.w = side == 0 ? amp : -amp;
        ch.id = cid;
        if (TAN) {
            const double wd = P.width[m];
            const double s0 = 1.0 / P.H[m];
            const double s1 = 1.0 / wd - ((4.0 * wd) * q) * q;
            const double s2 = -(2.0 * q) * (cos_det(arg) / sn);
            const double sdir = side == 0 ? 1.0 : -1.0;
            const double sgd = (double)ch.sg;
            ch.D[0] = sdir * cur.D[0] + sgd * s0;
            ch.D[1] = sdir * cur.D[1] + sgd * s1;
            ch.D[2] = sdir * cur.D[2] + sgd * s2;
        } else {
            ch.D[0] = ch.D[1] = ch.D[2] = 0.0;
        }
        if (!in_kbox<DIM>(d, ch.k)) {          // k-truncation (Sec. 2)
            if (!EMIT) {
                if (SP2) {
                    const int64_t q32 = (int64_t)floor(fabs(ch.w) * 4294967296.0);
                    tl.killed += ch.w < 0.0 ? -q32 : q32;
                } else {
                    tl.killed += ch.sg;
                }
            }
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
        } else if (nrec < (uint32_t)kStash) {
            const int r = (int)nrec, l = threadIdx.x;
            sh->x0[r][l] = cur.xe[0] + (d.vfac * ch.k[0]) * (d.dt - cur.te);
            sh->k0[r][l] = ch.k[0];
            if (DIM == 2) {
                sh->x1[r][l] = cur.xe[1] + (d.vfac * ch.k[1]) * (d.dt - cur.te);
                sh->k1[r][l] = ch.k[1];
            }
            if (SP2) sh->w[r][l] = ch.w; else sh->sg[r][l] = (int8_t)ch.sg;
            sh->id[r][l] = ch.id;
            if (TAN) {
                sh->D[3 * r][l] = ch.D[0];
                sh->D[3 * r + 1][l] = ch.D[1];
                sh->D[3 * r + 2][l] = ch.D[2];
            }
        }
        nrec++;
        ch.depth = cur.depth + 1;
        if (!EMIT && ch.depth > tl.maxdepth) tl.maxdepth = ch.depth;
        {
            // The child's first clock draw, exactly as its own walk would take
            // it: most children do not jump before the end of the step, and
            // then there is nothing to walk and the parent stays off the stack.
            const W4 r0 = draw(ch.id, step, kTagStep, 0u, 0u, seed, key);
            const double tau0 = -ln_series(1.0 - unit53(r0.a, r0.b)) / P.gamma0;
            if (!(cur.te + tau0 <= d.dt)) continue;
        }
        if (sp >= kMaxDepth) {
            err |= kErrDepth;
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

template <int DIM, bool SP2, bool TAN>
__global__ __launch_bounds__(kThreads) void k_family(Dev d, int ghost)
{
    __shared__ int64_t s_t;
    __shared__ uint32_t s_wsum[4];
    __shared__ uint32_t s_excl;
    __shared__ int64_t s_tal[5];
    __shared__ Stash<DIM, SP2, TAN> s_stash;

    Ctl *ctl = d.ctl;
    const uint32_t step = ctl->step;
    const uint32_t epoch = 2u * step + (uint32_t)ghost + 1u;
    const int B = d.B;
    const int64_t *plan = d.tileB + (int64_t)ghost * (B + 1);
    const int64_t ntiles = plan[B];
    int64_t *Ncur = ghost ? d.NG : d.N;
    const Ens E = pick_set(d, ghost, ghost ? ctl->gcur : ctl->cur);
    uint64_t *st = ghost ? d.stBg : d.stB;
    const uint32_t *evi = ghost ? d.gev_idx : d.ev_idx;
    const double *evx0 = ghost ? d.gev_x0 : d.ev_x0;
    const double *evx1 = ghost ? d.gev_x1 : d.ev_x1;
    const int pass = ghost ? kPassFamilyG : kPassFamily;
    const int64_t dstride = ghost ? d.gcap_total : d.cap_total;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    uint32_t err = 0;

    for (;;) {
        if (tid == 0) s_t = next_tile(&ctl->ticket[pass], ntiles);
        if (tid < 5) s_tal[tid] = 0;
        __syncthreads();
        const int64_t t = s_t;
        if (t >= ntiles) break;
        const int b = segment_of(plan, B, t);
        const int64_t first = plan[b];
        const int64_t tl_i = t - first;
        const int64_t last = plan[b + 1] - 1;
        const InstParam &P = d.ip[b];
        const int64_t base = ghost ? P.gbase : P.base;
        const int64_t cap = ghost ? P.gcap : P.cap;
        const int64_t nev = d.evc[(int64_t)ghost * B + b];
        const int64_t n_before = Ncur[b];
        const int64_t j = tl_i * kTileB + tid;
        const bool ok = j < nev;

        Node root;
        root.x[0] = root.x[1] = root.k[0] = root.k[1] = 0.0;
        root.t0 = 0.0;
        root.w = 0.0;
        root.D[0] = root.D[1] = root.D[2] = 0.0;
        root.id = 0;
        root.sg = 0;
        if (ok) {
            const int64_t pos = base + j;
            const int64_t i = base + (int64_t)evi[pos];
            root.x[0] = evx0[pos];
            root.k[0] = E.k0[i];
            if (DIM == 2) { root.x[1] = evx1[pos]; root.k[1] = E.k1[i]; }
            root.id = E.id[i];
            if (SP2) root.w = E.w[i]; else root.sg = (int32_t)E.sg[i];
            if (TAN) {
                root.D[0] = E.D[i];
                root.D[1] = E.D[dstride + i];
                root.D[2] = E.D[2 * dstride + i];
            }
        }
        Tally tal{0, 0, 0, 0, 0};
        uint32_t cnt = 0;
        if (ok) cnt = walk_family<DIM, SP2, TAN, false>(d, P, step, root, E, base, 0, cap, dstride, tal, err,
                                                        &s_stash);

        // ordered exclusive scan of the record counts over the tile
        uint32_t incl = cnt;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t v = __shfl_up(incl, o, 64);
            if (lane >= o) incl += v;
        }
        if (lane == 63) s_wsum[wv] = incl;
        __syncthreads();
        uint32_t woff = 0, agg = 0;
        for (int q = 0; q < 4; ++q) {
            if (q < wv) woff += s_wsum[q];
            agg += s_wsum[q];
        }
        if (wv == 0) {
            const uint32_t excl = tile_prefix(st, t, first, epoch, agg);
            if (lane == 0) {
                if (t == last) d.chc[(int64_t)ghost * B + b] = (int64_t)(excl + agg);
                s_excl = excl;
            }
        }
        __syncthreads();
        const int64_t my_first = n_before + (int64_t)s_excl + (int64_t)(woff + incl - cnt);
        if (ok && cnt > (uint32_t)kStash) {
            walk_family<DIM, SP2, TAN, true>(d, P, step, root, E, base, my_first, cap, dstride, tal, err,
                                             &s_stash);
        } else if (ok) {
            for (uint32_t r = 0; r < cnt; ++r) {
                const int64_t li = my_first + r;
                if (li >= cap) { err |= kErrCapacity; continue; }
                const int64_t o = base + li;
                E.x0[o] = s_stash.x0[r][tid];
                E.k0[o] = s_stash.k0[r][tid];
                if (DIM == 2) {
                    E.x1[o] = s_stash.x1[r][tid];
                    E.k1[o] = s_stash.k1[r][tid];
                }
                if (SP2) E.w[o] = s_stash.w[r][tid]; else E.sg[o] = s_stash.sg[r][tid];
                E.id[o] = s_stash.id[r][tid];
                if (TAN) {
                    E.D[o] = s_stash.D[3 * r][tid];
                    E.D[dstride + o] = s_stash.D[3 * r + 1][tid];
                    E.D[2 * dstride + o] = s_stash.D[3 * r + 2][tid];
                }
            }
        }

        // per-instance tallies
        if (tal.events) atomicAdd((unsigned long long *)&s_tal[0], (unsigned long long)tal.events);
        if (tal.pairs) atomicAdd((unsigned long long *)&s_tal[1], (unsigned long long)tal.pairs);
        if (tal.killed) atomicAdd((unsigned long long *)&s_tal[2], (unsigned long long)tal.killed);
        if (tal.cap) atomicAdd((unsigned long long *)&s_tal[3], (unsigned long long)tal.cap);
        if (tal.maxdepth) atomicMax((unsigned long long *)&s_tal[4], (unsigned long long)tal.maxdepth);
        __syncthreads();
        if (tid == 0) {
            int64_t *T = d.tally + (int64_t)b * kTalCount;
            if (s_tal[0]) atomicAdd((unsigned long long *)&T[kTalEvents], (unsigned long long)s_tal[0]);
            if (s_tal[1]) atomicAdd((unsigned long long *)&T[kTalPairs], (unsigned long long)s_tal[1]);
            if (s_tal[2]) atomicAdd((unsigned long long *)&T[kTalKilled], (unsigned long long)s_tal[2]);
            if (s_tal[3]) atomicAdd((unsigned long long *)&T[kTalEventCap], (unsigned long long)s_tal[3]);
            if (s_tal[4]) atomicMax((unsigned long long *)&T[kTalMaxDepth], (unsigned long long)s_tal[4]);
        }
        __syncthreads();
    }
    if (err) atomicOr(&ctl->err, err);

}

// After k_family (one block): the new particle counts with the capacity
// clamp, cleared event and record counts, the streaming-tile plan of the
// next step, and the step counter.
__global__ __launch_bounds__(kThreads) void k_close_family(Dev d, int ghost, int advance)
{
    Ctl *ctl = d.ctl;
    const int B = d.B;
    const uint32_t step = ctl->step;
    int64_t *Ncur = ghost ? d.NG : d.N;
    const int tid = threadIdx.x;
    int64_t *chc = d.chc + (int64_t)ghost * B;
    int64_t *evc = d.evc + (int64_t)ghost * B;
    for (int b = tid; b < B; b += kThreads) {
        const InstParam &P = d.ip[b];
        const int64_t cap = ghost ? P.gcap : P.cap;
        int64_t n = Ncur[b] + chc[b];
        if (n > cap) {
            atomicOr(&ctl->err, kErrCapacity);
            n = cap;
        }
        Ncur[b] = n;
        chc[b] = 0;
        evc[b] = 0;
    }
    __syncthreads();
    block_plan(d.tileA + (int64_t)ghost * (B + 1), Ncur, B, kTileA);
    if (tid == 0 && advance) ctl->step = step + 1u;
}

}  // namespace wbrw
