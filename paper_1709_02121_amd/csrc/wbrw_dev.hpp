// Device-side data layout of the WBRW library.
//
// Particles of all instances live in one structure of arrays; instance b owns
// the segment [base_b, base_b + cap_b).  Two such sets exist and annihilation
// writes the regenerated ensemble into the inactive one ("cur" flips).  All
// mutable bookkeeping (counts, tile plans, tickets, look-back status words,
// tallies, the step counter) is device resident, so a step or an epoch can be
// enqueued, or captured into a hipGraph, without host round trips.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wbrw {

constexpr int kMaxM = 4;
constexpr int kThreads = 256;           // threads per block in every kernel
constexpr int kPPT = 8;                 // particles (or cells) per thread in streaming passes
constexpr int kTileA = kThreads * kPPT; // particles per streaming tile
constexpr int kTileB = kThreads;        // event-parents per family tile (the smallest; see fam_tile)
constexpr int kTileS = kThreads * kPPT; // cells per scan tile
constexpr int kSupGroup = 64;           // tiles per group sum of per-tile counts
constexpr int kSupStride = 16;          // u64 slots between group sums (one per 128 B line)
constexpr int kXcd = 8;                 // accelerator complexes (XCDs), each with its own L2
constexpr int kTileR = kThreads * 4;    // regenerated particles per tile
constexpr int kMaxDepth = 16;           // deepest family tree walked within one step
constexpr uint32_t kEventCap = 4096u;   // jumps per particle-step
constexpr int kXiN = 4096;              // xi(r) grid intervals (Alg. 4 sampler)
constexpr int kXiQ = 8192;              // quadrature nodes for xi(r)
constexpr uint32_t kRejectMax = 256u;   // rejection proposals per kick
constexpr int kMaxGrid = 8192;          // blocks of a persistent launch (per-block partials)
// 4D family kernels: records of the general walks beyond the block's LDS pool
// go to a per-block overflow area in HBM (kGPool records for each of the
// first kGPoolBlocks blocks), so that they need not be walked a second time
// when they are written.  Per record: eight doubles (x0, k0, x1, k1, w and
// three tangents), the id, slot and rank, and the sign.
constexpr int kGPool = 1024;
constexpr int kGPoolBlocks = 1024;
constexpr size_t kGPoolBytes = (size_t)kGPool * (8 * 8 + 8 + 4 + 1);

// Event parents per family tile of the particle pass.  A tile's slow family
// walks run concurrently, so larger tiles shorten the walk-bound critical
// path; the 1D plain and sp2 kernels have the LDS for two parents per thread,
// the 4D and tangent ones (larger records, four stash rows) one.  Ghost passes
// use the tangent kernel, hence kTileB.
constexpr int fam_tile(int dim, bool tangent) { return (dim == 1 && !tangent) ? 2 * kThreads : kTileB; }

enum : uint32_t { kErrCapacity = 1u, kErrDepth = 2u, kErrRange = 4u };

// tally slots per instance
enum : int {
    kTalEvents = 0, kTalPairs, kTalKilled, kTalEscaped, kTalMaxDepth, kTalEventCap,
    kTalSplus, kTalSminus, kTalNplus, kTalNminus, kTalPSteps, kTalAnn, kTalTrig, kTalCount = 16
};

// ticket counters of the persistent passes
enum : int {
    kPassFamily = 1, kPassFamilyG = 3, kPassGhost = 7, kPassCount = 8
};

struct InstParam {
    double gamma0;
    double thr_lo, thr_hi;          // certain-jump / certain-no-jump band on the first uniform
    double c[kMaxM];                // xi_m / (2 gamma0)
    double sq[kMaxM];               // Gaussian kick std 1/(2w)
    double H[kMaxM], width[kMaxM];  // Gaussian parameters (tangent scores)
    double center[kMaxM];           // centre of the kernel phase
    double sgnV[kMaxM];             // sign of F[V_m]
    double xi_h[kMaxM];             // Alg. 4 sampler: xi grid spacing in |x - x0|
    double ma[kMaxM], mb[kMaxM];    // time-varying height factor a + b cos(omega t + phase)
    double mw[kMaxM], mp[kMaxM];
    int64_t base, cap;              // particle segment
    int64_t gbase, gcap;            // ghost segment
    int64_t N0;                     // sample size N_alpha
    int64_t rbase, rtiles;          // this instance's slots in Dev::rstart
    uint32_t key;                   // Philox key word 1
    uint32_t pad;
};

struct Table {
    const double *cum;    // n + 1 cumulative sums of |F[V](2q_j)|
    const int32_t *guide; // kg + 1 entries: guide[i] = the last bin j < n with
                          // cum[j] <= (i / kg) cum[n] (as the sampler rounds it)
    int32_t n;
    int32_t kg;           // guide buckets, a power of two >= n
    double q_lo, dq;
};

struct Ens {
    double *x0, *x1, *k0, *k1;
    int8_t *sg;
    double *w;
    uint64_t *id;
    double *D;     // planar [3][cap_total]
};

struct Ctl {
    uint32_t step;             // steps completed (Philox counter word 2)
    uint32_t cur;              // active real buffer set
    uint32_t gcur;             // active ghost buffer set
    uint32_t err;              // sticky error bits
    uint32_t ann_seq;          // annihilations so far (look-back epoch of the scans)
    uint32_t ann_now;          // conditional annihilation: the one after this step runs
    uint32_t pad[2];
    uint32_t ticket[kPassCount];   // zero between launches (see next_tile)
};

struct Dev {
    // sizes and constants
    int32_t B, dim, M, strategy, tangent;
    int32_t tdep;               // some Gaussian height varies in time
    // conditional annihilation (wbrw_run_adaptive): the step's closing kernel
    // sets ctl->ann_now when the step count is a multiple of ann_every or an
    // instance holds more than ann_limit particles, and with cond_ann set the
    // annihilation kernels run only then
    int32_t cond_ann, ann_every;
    int64_t ann_limit;
    double hbar;
    int32_t nx, nk;
    uint32_t seed;
    int64_t Nh;                 // cells per instance
    int64_t cap_total, gcap_total;
    double dt, vfac;
    double x_lo, x_hi, k_lo, k_hi, dx, dk;
    int32_t kind[kMaxM], axis[kMaxM], sampler[kMaxM];
    const double *xi_tab;       // [B][M][kXiN + 1] xi(r) tables of the Alg. 4 sampler
    Table tab[kMaxM];
    // buffers
    Ens ens[2], gens[2];
    const InstParam *ip;
    Ctl *ctl;
    int64_t *N, *NG, *Nnew, *NGnew;
    int64_t *Nbase;             // [2][B] counts at the start of the step (real, ghost): the records go after them
    int64_t *evc;               // [2][B] event counts (real, ghost)
    int64_t *tileA;             // [2][B+1] streaming-tile plan (real, ghost)
    int64_t *tileB;             // [2][B+1] family-tile plan
    int64_t *tileR;             // [B+1] regeneration-tile plan
    int64_t *tileG;             // [B+1] ghost-regeneration plan
    int64_t *tally;             // [B][kTalCount]
    int64_t *fpart;             // [kMaxGrid][8]: instance and tallies of each family block
    char *gpool;                // [gpool_blocks][kGPoolBytes] (4D only, else null)
    int32_t gpool_blocks;
    int64_t *rstart;            // first cell of every regeneration tile (written by k_scan)
    uint32_t *ev_idx;           // [cap_total] event-parent index within its instance
    uint32_t *gev_idx;          // ghosts
    uint64_t *stS;              // scan-tile sums of |n_nu|, then their exclusive prefix
    uint64_t *stG;              // look-back status words of k_ghosts
    uint64_t *tcB, *tcBg;               // per family tile: record count
    uint64_t *supB, *supBg;             // per kSupGroup family tiles: sum of their record
                                        // counts (entries kSupStride apart)
    int64_t *tsB, *tsBg;                // per family tile: where its records were staged
    int64_t *stg;                       // [2][B] staging fill of the inactive buffer sets
    uint64_t *tcA, *tcAg;               // per streaming tile: event count
    uint64_t *supA, *supAg;             // per kSupGroup streaming tiles: sum of their event
                                        // counts (entries kSupStride apart)
    int64_t *spart;                     // [kMaxGrid][2]: each streaming block's last
                                        // instance and its events there
    uint64_t *emA, *emAg;               // per streaming tile: kTileA / 64 wavefront event ballots
    int64_t *Nsrt;              // [B] particles in cell order at the front of each instance
    int64_t *srtS;              // [B+1] prefix of floor(Nsrt[b] / kTileA)
    int32_t *cnt;               // [B][Nh] signed counts (sp1) / rounded counts (sp2)
    int32_t *cntx;              // partial counts of the blocks on the other XCDs (copy 0
                                // is the grid itself): sp1 [kXcd - 1][B][Nh] of cnt, sp2
                                // [kXcd - 1][2][B][Nh] of ntil; null when not used
    int64_t *off;               // [B][Nh] exclusive prefix of |n_nu|, bit 62 = negative cell
    int32_t *occ;               // [B][Nh] occupancy (tangents)
    int64_t *Tq;                // [6][B][Nh] tangent sums per cell in 32.32 fixed point
                                // (see fx_split): plane 2c high words, 2c + 1 low words
    int32_t *occx;              // with tangents: [kXcd - 1][B][Nh] XCD copies of occ,
    int64_t *Tqx;               // and [kXcd - 1][6][B][Nh] of Tq (see cntx); else null
    int32_t *ntil;              // [2][B][Nh] sp2 bootstrap counts per class
    int64_t *dacc;              // [kXcd][B][max_bins] density accumulator, one per XCD
                                // (a block flushes into copy blockIdx mod kXcd)
    int64_t *dTq;               // [B][6][max_bins] tangent density sums (fixed point, as Tq)
    int32_t max_bins;
    // sp2 bootstrap scratch
    uint64_t *bA;               // [cap_total] quantised weight, then the residual
    int32_t *bcopies;           // [cap_total] copies per particle
    int8_t *bcls;               // [cap_total] class (0 +, 1 -, -1 none)
    int64_t *bcell;             // [cap_total] cell or -1
    uint64_t *bP;               // [2][cap_total] 128-bit residual prefix (lo, hi interleaved)
    uint64_t *bTile;            // [2][tiles] 128-bit tile sums
    int32_t *bG;                // [2][4 cap_total] draw guide per class, four
                                // slots per particle slot (sp2_guide_bits)
    int64_t *bcls_stat;         // [B][8]: N+, N-, S+, S-, sumk+, sumk-, Nr+, Nr-
    int64_t *tileD;             // [2][B+1] draw-tile plan (per class)
    int64_t *bscan_tiles;       // [B+1] tiles per instance for the residual scan
    int64_t tstride;            // tiles per class in bTile
};

// An annihilation kernel enqueued after a step of wbrw_run_adaptive does
// nothing unless that step's closing kernel asked for the annihilation.
__device__ __forceinline__ bool ann_skipped(const Dev &d)
{
    return d.cond_ann && d.ctl->ann_now == 0u;
}

__device__ __forceinline__ Ens pick_set(const Dev &d, int ghost, uint32_t which)
{
    if (ghost) return which ? d.gens[1] : d.gens[0];
    return which ? d.ens[1] : d.ens[0];
}

// segment b with plan[b] <= t < plan[b+1]
__device__ __forceinline__ int segment_of(const int64_t *plan, int B, int64_t t)
{
    int lo = 0, hi = B - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (plan[mid] <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Sum over tiles [a, c) of per-tile counts tc, with sup holding the sums of
// whole groups of kSupGroup tiles (kSupStride apart): the tiles before the
// first whole group, the group sums, the tiles after the last whole group.
// Element e < n() of that list is load(e).
struct TileRange {
    const uint64_t *tc, *sup;
    int64_t a, ga, gc, nh, ng, nt;
    __device__ __forceinline__ TileRange(const uint64_t *tc_, const uint64_t *sup_, int64_t a_, int64_t c)
        : tc(tc_), sup(sup_), a(a_)
    {
        ga = (a + kSupGroup - 1) / kSupGroup * kSupGroup;
        gc = c / kSupGroup * kSupGroup;
        const bool groups = ga <= gc;
        nh = c <= a ? 0 : (groups ? ga - a : c - a);
        ng = groups ? (gc - ga) / kSupGroup : 0;
        nt = groups ? c - gc : 0;
    }
    __device__ __forceinline__ int64_t n() const { return nh + ng + nt; }
    __device__ __forceinline__ uint64_t load(int64_t e) const
    {
        if (e < nh) return tc[a + e];
        if (e < nh + ng) return sup[(ga / kSupGroup + (e - nh)) * kSupStride];
        return tc[gc + (e - nh - ng)];
    }
};

// TileRange sum for every lane of the wavefront
__device__ __forceinline__ uint64_t wave_range_sum(const TileRange &R)
{
    const int lane = threadIdx.x & 63;
    uint64_t v = 0;
    for (int64_t e = lane; e < R.n(); e += 64) v += R.load(e);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// TileRange sum for every thread of the block (s_w: kThreads / 64 slots)
__device__ __forceinline__ uint64_t block_range_sum(const TileRange &R, uint64_t *s_w)
{
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    uint64_t v = 0;
    for (int64_t e = tid; e < R.n(); e += kThreads) v += R.load(e);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (lane == 0) s_w[wv] = v;
    __syncthreads();
    uint64_t tot = 0;
#pragma unroll
    for (int q = 0; q < kThreads / 64; ++q) tot += s_w[q];
    __syncthreads();
    return tot;
}

// ---- decoupled look-back (single-pass ordered scans) ----------------------
// status word: [epoch:30 | flag:2 | value:32]; flag 1 = tile aggregate, 2 = inclusive prefix
__device__ __forceinline__ void lb_publish(uint64_t *st, uint32_t epoch, uint32_t flag, uint32_t v)
{
    const uint64_t w = ((uint64_t)((epoch << 2) | flag) << 32) | (uint64_t)v;
    __hip_atomic_store(st, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// exclusive prefix of tile t over the tiles [first, t) of its segment
__device__ __forceinline__ uint32_t lb_lookback(uint64_t *st, int64_t t, int64_t first, uint32_t epoch)
{
    uint32_t excl = 0;
    int64_t p = t - 1;
    while (p >= first) {
        uint64_t w;
        for (;;) {
            w = __hip_atomic_load(st + p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t hi = (uint32_t)(w >> 32);
            if ((hi >> 2) == epoch && (hi & 3u) != 0u) break;
            __builtin_amdgcn_s_sleep(1);
        }
        excl += (uint32_t)w;
        if (((uint32_t)(w >> 32) & 3u) == 2u) break;
        --p;
    }
    return excl;
}

// Wave-parallel look-back: the 64 lanes of one wavefront examine 64
// predecessors per round, wait until each has published, and sum back to the
// nearest inclusive prefix.  Returns the exclusive prefix to every lane.
__device__ __forceinline__ uint32_t lb_lookback_wave(uint64_t *st, int64_t t, int64_t first, uint32_t epoch)
{
    const int lane = threadIdx.x & 63;
    uint32_t excl = 0;
    for (int64_t top = t - 1; top >= first; top -= 64) {
        const int64_t p = top - lane;
        uint32_t flag = 2u, val = 0u;   // lanes past the segment start act as a zero prefix
        if (p >= first) {
            for (;;) {
                const uint64_t w = __hip_atomic_load(st + p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const uint32_t hi = (uint32_t)(w >> 32);
                if ((hi >> 2) == epoch && (hi & 3u) != 0u) {
                    flag = hi & 3u;
                    val = (uint32_t)w;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        const uint64_t incl = __ballot(flag == 2u);
        const int stop = incl ? (__ffsll((unsigned long long)incl) - 1) : 64;
        uint32_t v = lane <= stop ? val : 0u;
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        excl += v;
        if (incl) break;
    }
    return excl;
}

// Publishes tile t's aggregate, looks back over its segment [first, t) and
// publishes its inclusive prefix.  Called by all lanes of wavefront 0.
__device__ __forceinline__ uint32_t tile_prefix(uint64_t *st, int64_t t, int64_t first, uint32_t epoch,
                                                uint32_t agg)
{
    const int lane = threadIdx.x & 63;
    if (t == first) {
        if (lane == 0) lb_publish(st + t, epoch, 2u, agg);
        return 0u;
    }
    if (lane == 0) lb_publish(st + t, epoch, 1u, agg);
    const uint32_t excl = lb_lookback_wave(st, t, first, epoch);
    if (lane == 0) lb_publish(st + t, epoch, 2u, excl + agg);
    return excl;
}

// Next tile of a persistent pass, for thread 0 of a block.  Every block
// draws until it gets a ticket >= ntiles, so one launch hands out exactly
// ntiles + gridDim.x tickets, and the block that draws the last of them
// clears the counter for the next launch (which sees it after the kernel
// boundary).  No block waits for the others at the end, and no device-wide
// fence is needed.  Work that needs every block's results runs in one extra
// block of the next launch.
__device__ __forceinline__ int64_t next_tile(uint32_t *ctr, int64_t ntiles)
{
    const uint32_t t = atomicAdd(ctr, 1u);
    if ((int64_t)t == ntiles + (int64_t)gridDim.x - 1)
        __hip_atomic_store(ctr, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return (int64_t)t;
}

// The same dispenser with every block's first tile given statically (block
// b takes tile b): when the tiles are about as many as the blocks, every
// block starts at once instead of queueing behind one atomic on one line
// (some 11 ns each).  The counter then hands out tiles gridDim.x, ...: each
// of those tickets is drawn once and every block draws one ticket past the
// end, so the block that draws ticket max(0, ntiles - gridDim.x) +
// gridDim.x - 1 clears the counter.  `first` is the caller's flag, true on
// its first call.
__device__ __forceinline__ int64_t next_tile_static_first(uint32_t *ctr, int64_t ntiles, bool &first)
{
    const int64_t G = (int64_t)gridDim.x;
    if (first) {
        first = false;
        if ((int64_t)blockIdx.x < ntiles) return (int64_t)blockIdx.x;
    }
    const int64_t D = ntiles > G ? ntiles - G : 0;
    const uint32_t u = atomicAdd(ctr, 1u);
    if ((int64_t)u == D + G - 1) __hip_atomic_store(ctr, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return G + (int64_t)u;
}

// Exclusive scan of the per-tile counts cnt[0..T) into pre[0..T) by one
// block (pre may be cnt); returns the total to every thread.  Chunks of
// kThreads x P counts are loaded coalesced (all loads in flight together)
// into LDS, padded by one slot per P so that the per-thread runs below fall
// in different banks; every thread scans its own run of P, the run totals are
// scanned within each wavefront and across the four wavefronts, and the
// prefixes leave LDS coalesced.
constexpr int kScanP = 24;
template <int P>
__device__ __forceinline__ uint64_t scan_chunks(const uint64_t *cnt, uint64_t *pre, int64_t T,
                                                uint64_t *s_v, uint64_t *s_w)
{
    constexpr int C = kThreads * P, W = kThreads / 64;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int run0 = tid * (P + 1);
    uint64_t carry = 0;
    for (int64_t c0 = 0; c0 < T; c0 += C) {
        const int n = (int)min((int64_t)C, T - c0);
        __syncthreads();
        uint64_t v[P], acc = 0;
#pragma unroll
        for (int r = 0; r < P; ++r)   // clamped, unconditional: no branch between the loads
            v[r] = cnt[c0 + min(r * kThreads + tid, n - 1)];
#pragma unroll
        for (int r = 0; r < P; ++r) {
            const int i = r * kThreads + tid;
            s_v[i + i / P] = v[r];
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < P; ++r) {
            v[r] = tid * P + r < n ? s_v[run0 + r] : 0ull;
            acc += v[r];
        }
        uint64_t incl = acc;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint64_t y = __shfl_up(incl, o, 64);
            if (lane >= o) incl += y;
        }
        if (lane == 63) s_w[wv] = incl;
        __syncthreads();
        uint64_t below = 0, chunk = 0;
#pragma unroll
        for (int w = 0; w < W; ++w) {
            const uint64_t t = s_w[w];
            below += w < wv ? t : 0ull;
            chunk += t;
        }
        uint64_t run = carry + below + (incl - acc);
#pragma unroll
        for (int r = 0; r < P; ++r) {
            s_v[run0 + r] = run;
            run += v[r];
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < P; ++r) {
            const int i = r * kThreads + tid;
            if (i < n) pre[c0 + i] = s_v[i + i / P];
        }
        carry += chunk;
    }
    __syncthreads();
    return carry;
}

__device__ __forceinline__ uint64_t scan_tile_counts(const uint64_t *cnt, uint64_t *pre, int64_t T)
{
    __shared__ uint64_t s_v[kThreads * (kScanP + 1)];
    __shared__ uint64_t s_w[kThreads / 64];
    // a short list takes one small chunk: fewer loads and LDS passes per thread
    if (T <= kThreads * 4) return scan_chunks<4>(cnt, pre, T, s_v, s_w);
    return scan_chunks<kScanP>(cnt, pre, T, s_v, s_w);
}

// plan[b] = sum_{b' < b} value(b'), plan[B] = total; one block.  Values are
// scanned within each wavefront, then across the four wavefronts.
template <class F>
__device__ __forceinline__ void block_prefix(int64_t *plan, int B, F value)
{
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    if (B == 1) {
        if (tid == 0) {
            plan[1] = value(0);
            plan[0] = 0;
        }
        __syncthreads();
        return;
    }
    __shared__ int64_t s_w[kThreads / 64];
    int64_t carry = 0;
    for (int c0 = 0; c0 < B; c0 += kThreads) {
        const int b = c0 + tid;
        const int64_t v = b < B ? value(b) : 0;
        int64_t incl = v;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int64_t y = __shfl_up(incl, o, 64);
            if (lane >= o) incl += y;
        }
        __syncthreads();
        if (lane == 63) s_w[wv] = incl;
        __syncthreads();
        int64_t below = 0, chunk = 0;
#pragma unroll
        for (int w = 0; w < kThreads / 64; ++w) {
            const int64_t t = s_w[w];
            below += w < wv ? t : 0;
            chunk += t;
        }
        if (b < B) plan[b] = carry + below + incl - v;
        carry += chunk;
    }
    if (tid == 0) plan[B] = carry;
    __syncthreads();
}

// plan[b] = sum_{b' < b} ceil(cnt[b'] / tile), plan[B] = total; one block.
__device__ __forceinline__ void block_plan(int64_t *plan, const int64_t *cnt, int B, int64_t tile)
{
    block_prefix(plan, B, [&](int b) { return (cnt[b] + tile - 1) / tile; });
}

// Cost of binning a streaming tile: kBinSortedCost inside the cell-ordered
// front of its instance (the first Nsrt[b] particles, as the last
// regeneration left them), kBinLateCost after it, where the offspring
// appended since then scatter over many more cells per tile.  With srtS[b] =
// sum_{b' < b} floor(Nsrt[b'] / kTileA), the cost of the tiles before
// instance b is kBinLateCost tileA[b] - (kBinLateCost - kBinSortedCost)
// srtS[b]; it needs N[b] >= Nsrt[b], which holds because steps only append.
constexpr int64_t kBinSortedCost = 1, kBinLateCost = 3;

// Tangent sums over cells and bins are exact integer sums in 32.32 fixed
// point, so that no summation order is singled out: a component D enters as
// q = trunc(D 2^32), which needs |D| < 2^31 (else, or for a NaN, it adds
// nothing and false is returned), split as hi = floor(q / 2^32) and
// lo = q mod 2^32.  Over at most 2^31 particles the high words sum to less
// than 2^62 and the low words to less than 2^63, so two 64-bit sums per
// component are exact without carries.
__device__ __forceinline__ bool fx_split(double D, int64_t &hi, uint64_t &lo)
{
    if (!(fabs(D) < 2147483648.0)) {
        hi = 0;
        lo = 0;
        return false;
    }
    const int64_t q = (int64_t)(D * 4294967296.0);
    hi = q >> 32;
    lo = (uint64_t)q & 0xFFFFFFFFull;
    return true;
}

// value of the sum with high-word sum hs and low-word sum ls:
// (double)floor(Q / 2^32) + (double)(Q mod 2^32) 2^-32, Q = hs 2^32 + ls
__device__ __forceinline__ double fx_value(int64_t hs, uint64_t ls)
{
    const int64_t h = hs + (int64_t)(ls >> 32);
    return (double)h + (double)(ls & 0xFFFFFFFFull) * 0x1p-32;
}

__device__ __forceinline__ uint32_t lane_rank(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

}  // namespace wbrw
