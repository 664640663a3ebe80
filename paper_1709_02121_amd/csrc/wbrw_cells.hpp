// Phase-space cells: initial sampling, sp1 annihilation and the density readout.
//
// Annihilation (Sec. 4.3, Eq. signed_histogram; Alg. 3 step 3):
//   k_bin     one pass over the particles: cell index on the uniform grid
//             D_nu = X_nu1 x K_nu2 (escaped sign tallied), signs summed per
//             cell in an LDS hash per block, then integer atomic adds into the
//             instance's count grid (one copy per XCD): the per-cell sums
//             n_nu^+ - n_nu^- are exact and order independent;
//   k_scan_sums, k_close_scan, k_scan
//             ordered exclusive scan of |n_nu| per instance in three launches
//             (tile sums, their one-block scan, the offsets), which is also
//             the output layout: ascending cell, then index within the cell;
//   k_regen   one thread per output particle: the cell by binary search in the
//             scan, position uniform in the cell, sign sgn(n_nu), lineage id
//             (nu << 32) | j; written to the inactive buffer set, which then
//             becomes active.
// Density (Eq. estimator with an indicator observable): integer (sp1) or
// 2^-32 fixed-point (sp2) atomics per bin, then one division per bin; the
// tangent density and the backward pass sum tangents in 32.32 fixed point.
#pragma once
#include "wbrw_dev.hpp"
#include "wbrw_math.hpp"

namespace wbrw {

// Run aggregation over a wavefront: lanes hold consecutive elements, and a
// run is a maximal group of consecutive lanes with equal key.  On return the
// last lane of each run holds in v the sum of its run and gets true; keys < 0
// never commit.  Must be called by all 64 lanes.
template <typename T>
__device__ __forceinline__ T run_sum(int64_t key, T v, bool &commit)
{
    const int lane = threadIdx.x & 63;
    const int64_t kprev = __shfl_up(key, 1, 64);
    const int64_t knext = __shfl_down(key, 1, 64);
    const bool head = lane == 0 || kprev != key;
    const bool tail = lane == 63 || knext != key;
    const uint64_t heads = __ballot(head);
    const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
    const int start = 63 - __builtin_clzll(heads & upto);
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const T u = __shfl_up(v, o, 64);
        if (lane - o >= start) v += u;
    }
    commit = tail && key >= 0;
    return v;
}

constexpr int64_t kOffMask = (1ll << 62) - 1;
constexpr int64_t kOffNeg = 1ll << 62;

// Cell of a phase-space point or -1 outside the grid.
template <int DIM>
__device__ __forceinline__ int64_t cell_index(const Dev &d, double x0, double x1, double k0, double k1)
{
    const double qx0 = (x0 - d.x_lo) / d.dx;
    const double qk0 = (k0 - d.k_lo) / d.dk;
    if (!(qx0 >= 0.0 && qx0 < (double)d.nx)) return -1;
    if (!(qk0 >= 0.0 && qk0 < (double)d.nk)) return -1;
    const int64_t ix0 = (int64_t)qx0, ik0 = (int64_t)qk0;
    if (DIM == 1) return ix0 + (int64_t)d.nx * ik0;
    const double qx1 = (x1 - d.x_lo) / d.dx;
    const double qk1 = (k1 - d.k_lo) / d.dk;
    if (!(qx1 >= 0.0 && qx1 < (double)d.nx)) return -1;
    if (!(qk1 >= 0.0 && qk1 < (double)d.nk)) return -1;
    const int64_t ix1 = (int64_t)qx1, ik1 = (int64_t)qk1;
    return ((ik1 * d.nk + ik0) * d.nx + ix1) * d.nx + ix0;
}

// Uniform position in cell nu from the uniforms of draw sub 0 (axis 0) and 1.
template <int DIM>
__device__ __forceinline__ void cell_point(const Dev &d, int64_t nu, uint64_t id, uint32_t tag,
                                           uint32_t step, uint32_t key, double *x, double *k)
{
    int64_t ix[2], ik[2];
    if (DIM == 1) {
        ix[0] = nu % d.nx;
        ik[0] = nu / d.nx;
    } else {
        int64_t r = nu;
        ix[0] = r % d.nx; r /= d.nx;
        ix[1] = r % d.nx; r /= d.nx;
        ik[0] = r % d.nk; r /= d.nk;
        ik[1] = r;
    }
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const W4 u = draw(id, step, tag, 0u, (uint32_t)a, d.seed, key);
        x[a] = d.x_lo + ((double)ix[a] + unit53(u.a, u.b)) * d.dx;
        k[a] = d.k_lo + ((double)ik[a] + unit53(u.c, u.d)) * d.dk;
    }
}

// ---------------------------------------------------------------------------
// Initial ensembles: x ~ N(mean_x, sigma_x), k ~ N(mean_k, sigma_k) per axis by
// Box-Muller on draw (id = j, step 0, tag init, sub = axis); sign +1.
// ---------------------------------------------------------------------------
template <int DIM>
__global__ __launch_bounds__(kThreads) void k_init(Dev d, double mx0, double mx1, double sx0,
                                                   double sx1, double mk0, double mk1, double sk0,
                                                   double sk1)
{
    const int B = d.B;
    const int64_t *plan = d.tileA;
    const int64_t ntiles = plan[B];
    const Ens E = d.ens[0];
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int b = segment_of(plan, B, t);
        const InstParam &P = d.ip[b];
        const int64_t n = d.N[b];
        for (int j = 0; j < kPPT; ++j) {
            const int64_t li = (t - plan[b]) * kTileA + (int64_t)j * kThreads + threadIdx.x;
            if (li >= n) continue;
            const int64_t i = P.base + li;
            const double mx[2] = {mx0, mx1}, sx[2] = {sx0, sx1}, mk[2] = {mk0, mk1}, sk[2] = {sk0, sk1};
            double xo[2], ko[2];
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                const W4 r = draw((uint64_t)li, 0u, kTagInit, 0u, (uint32_t)a, d.seed, P.key);
                const double u1 = unit53(r.a, r.b), u2 = unit53(r.c, r.d);
                const double R = sqrt(-2.0 * ln_series(1.0 - u1));
                const double th = kTwoPi * u2;
                const double z1 = R * cos_det(th);
                const double z2 = R * sin_det(th);
                xo[a] = mx[a] + sx[a] * z1;
                ko[a] = mk[a] + sk[a] * z2;
            }
            E.x0[i] = xo[0];
            E.k0[i] = ko[0];
            if (DIM == 2) { E.x1[i] = xo[1]; E.k1[i] = ko[1]; }
            if (d.strategy == 1) E.w[i] = 1.0; else E.sg[i] = 1;
            E.id[i] = (uint64_t)li;
            if (d.tangent) {
                E.D[i] = 0.0;
                E.D[d.cap_total + i] = 0.0;
                E.D[2 * d.cap_total + i] = 0.0;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Alg. 3 (Sec. 4.1), signed initial data: n_nu = [m] + p with
// m = N_alpha mu(D_nu) |d_nu| and p = 1 iff u < m - [m] (one uniform per cell),
// sign sgn(d_nu); k_scan and k_regen then place the particles uniformly.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_hist_round(Dev d, const double *hist, double mu)
{
    const int64_t plane = (int64_t)d.B * d.Nh;
    for (int64_t g = (int64_t)blockIdx.x * kThreads + threadIdx.x; g < plane;
         g += (int64_t)gridDim.x * kThreads) {
        const double dv = hist[g];
        if (dv == 0.0) { d.cnt[g] = 0; continue; }
        const int64_t b = g / d.Nh, nu = g - b * d.Nh;
        const InstParam &P = d.ip[b];
        const double m = ((double)P.N0 * mu) * fabs(dv);
        const double fl = floor(m);
        const W4 u = draw((uint64_t)nu, 0u, kTagHist, 0u, 0u, d.seed, P.key);
        const int64_t n = (int64_t)fl + (unit53(u.a, u.b) < m - fl ? 1 : 0);
        d.cnt[g] = (int32_t)(dv > 0.0 ? n : -n);
    }
}

// ---------------------------------------------------------------------------
// sp1 annihilation, pass 1: binning with exact integer sums per cell.  With
// tangents, also the occupancy and the tangent sums T_nu per cell (for sp2
// only these: its counts come from the bootstrap).
// ---------------------------------------------------------------------------
// Binning cost of the particle tiles before instance b (see kBinLateCost).
__device__ __forceinline__ int64_t bin_cost_before(const Dev &d, const int64_t *plan, int b)
{
    return kBinLateCost * plan[b] - (kBinLateCost - kBinSortedCost) * d.srtS[b];
}

// The first particle tile whose cost prefix reaches c, or the tile count
// when c reaches the total.
__device__ __forceinline__ int64_t tile_at_cost(const Dev &d, const int64_t *plan, int64_t c)
{
    const int B = d.B;
    if (c >= bin_cost_before(d, plan, B)) return plan[B];
    int lo = 0, hi = B - 1;   // the last instance whose cost prefix is <= c
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (bin_cost_before(d, plan, mid) <= c) lo = mid; else hi = mid - 1;
    }
    const int64_t r = c - bin_cost_before(d, plan, lo);
    const int64_t srt = d.srtS[lo + 1] - d.srtS[lo];
    // cost before tile l of the instance: kBinSortedCost l up to srt, then
    // kBinSortedCost srt + kBinLateCost (l - srt)
    const int64_t rs = kBinSortedCost * srt;
    return plan[lo] + (r <= rs ? (r + kBinSortedCost - 1) / kBinSortedCost
                               : srt + (r - rs + kBinLateCost - 1) / kBinLateCost);
}

template <int DIM, bool SP2, bool TAN, int SLOTS = 4096>
__global__ __launch_bounds__(kThreads) void k_bin(Dev d, int ghost)
{
    if (ann_skipped(d)) return;
    // Each block takes a contiguous run of tiles.  Without tangents the
    // signs are summed per cell in an LDS hash table (open addressing on the
    // cell index, 8 probes) that lives across the block's tiles and is added
    // to the count grid when the block moves to another instance, when it is
    // half full, and at the end: a cell-ordered ensemble straddles cell
    // boundaries after a few steps of drift, so equal cells are close in the
    // array but rarely in adjacent lanes, and neighbouring tiles share most
    // of their cells.  A particle whose probes all fail adds directly.  The
    // table's size (SLOTS, a power of two) trades flushes against blocks per
    // CU; the autotuner picks it.
    // With tangents the table's slots hold, per cell, the count, the
    // occupancy and the six 32.32 fixed-point halves of the tangent sums
    // (kTSlots of them), and each run of equal cells in consecutive lanes,
    // summed in registers first, adds to its slot with LDS atomics.
    constexpr int kSlots = TAN ? 512 : SLOTS;
    static_assert((SLOTS & (SLOTS - 1)) == 0, "a power of two");
    constexpr int kHashShift = 32 - (TAN ? 9 : 12);
    __shared__ int64_t s_esc;
    __shared__ uint32_t s_nkeys;
    __shared__ int32_t s_key[kSlots];
    __shared__ int32_t s_val[kSlots];                      // count
    __shared__ int32_t s_occ[TAN ? kSlots : 1];
    __shared__ unsigned long long s_tq[TAN ? 6 : 1][TAN ? kSlots : 1];
    Ctl *ctl = d.ctl;
    const int B = d.B;
    const int64_t *plan = d.tileA + (int64_t)ghost * (B + 1);
    const int64_t ntiles = plan[B];
    const int64_t *Ncur = ghost ? d.NG : d.N;
    const Ens E = pick_set(d, ghost, ghost ? ctl->gcur : ctl->cur);
    const int tid = threadIdx.x;
    // plain sp1: this block's XCD copy of the count grid (blocks are dealt
    // to the XCDs round robin; any other placement is still correct)
    const int xc = (int)(blockIdx.x % kXcd);
    const int64_t ncell = d.Nh * (int64_t)B;
    const bool own = d.cntx == nullptr || xc == 0 || (TAN && d.occx == nullptr);
    int32_t *const cg = own ? d.cnt : d.cntx + (int64_t)(xc - 1) * ncell;
    int32_t *const og = own ? d.occ : d.occx + (int64_t)(xc - 1) * ncell;
    int64_t *const tg = own ? d.Tq : d.Tqx + (int64_t)(xc - 1) * 6 * ncell;
    uint32_t err = 0;
    for (int j = tid; j < kSlots; j += kThreads) {
        s_key[j] = -1;
        s_val[j] = 0;
        if constexpr (TAN) {
            s_occ[j] = 0;
#pragma unroll
            for (int q = 0; q < 6; ++q) s_tq[q][j] = 0ull;
        }
    }
    if (tid == 0) { s_esc = 0; s_nkeys = 0; }
    auto flush = [&](int fb) {
        const int64_t fbase = (int64_t)fb * d.Nh;
        for (int j = tid; j < kSlots; j += kThreads) {
            const int k = s_key[j];
            if (k < 0) continue;
            const int v = s_val[j];
            if (v != 0) atomicAdd(&cg[fbase + k], v);
            s_key[j] = -1;
            s_val[j] = 0;
            if constexpr (TAN) {
                if (s_occ[j] != 0) atomicAdd(&og[fbase + k], s_occ[j]);
                s_occ[j] = 0;
#pragma unroll
                for (int q = 0; q < 6; ++q) {
                    const unsigned long long t = s_tq[q][j];
                    if (t) atomicAdd((unsigned long long *)&tg[(int64_t)q * ncell + fbase + k], t);
                    s_tq[q][j] = 0ull;
                }
            }
        }
        if (tid == 0) {
            if (s_esc)
                atomicAdd((unsigned long long *)&d.tally[(int64_t)fb * kTalCount + kTalEscaped],
                          (unsigned long long)s_esc);
            s_esc = 0;
            s_nkeys = 0;
        }
        __syncthreads();
    };
    // The block's contiguous run of tiles: an equal share of the binning cost
    // for the particles, an equal share of the tiles for the ghosts.
    int64_t t0, t1;
    if (ghost) {
        t0 = ntiles * blockIdx.x / gridDim.x;
        t1 = ntiles * (blockIdx.x + 1) / gridDim.x;
    } else {
        const int64_t W = bin_cost_before(d, plan, B);
        t0 = tile_at_cost(d, plan, (W * blockIdx.x + gridDim.x - 1) / gridDim.x);
        t1 = tile_at_cost(d, plan, (W * (blockIdx.x + 1) + gridDim.x - 1) / gridDim.x);
    }
    int cb = -1;
    for (int64_t t = t0; t < t1; ++t) {
        __syncthreads();
        const int b = segment_of(plan, B, t);
        // every thread reads the fill level before the flush resets it
        const bool full = cb >= 0 && (b != cb || s_nkeys > (uint32_t)(kSlots / 2));
        __syncthreads();
        if (full) flush(cb);
        cb = b;
        const InstParam &P = d.ip[b];
        const int64_t base = ghost ? P.gbase : P.base;
        const int64_t n = Ncur[b];
        const int64_t cbase = (int64_t)b * d.Nh;
        int64_t esc = 0;
        uint32_t ins = 0;      // keys this thread added to the hash
        const int64_t li0 = (t - plan[b]) * kTileA + tid;
        double xa[kPPT], xb[kPPT], ka[kPPT], kb[kPPT];
        int sv[kPPT];
#pragma unroll
        for (int j = 0; j < kPPT; ++j) {      // loads first: kPPT in flight per thread
            const int64_t li = li0 + (int64_t)j * kThreads;
            const int64_t i = base + (li < n ? li : 0);
            xa[j] = E.x0[i];
            ka[j] = E.k0[i];
            xb[j] = DIM == 2 ? E.x1[i] : 0.0;
            kb[j] = DIM == 2 ? E.k1[i] : 0.0;
            sv[j] = (ghost || SP2) ? 0 : (int)E.sg[i];
        }
#pragma unroll
        for (int j = 0; j < kPPT; ++j) {
            const int64_t li = li0 + (int64_t)j * kThreads;
            const bool live = li < n;
            const int64_t i = base + (live ? li : 0);
            const int64_t nu = live ? cell_index<DIM>(d, xa[j], xb[j], ka[j], kb[j]) : -1;
            const int s = live ? sv[j] : 0;
            if (live && nu < 0) {
                esc += s;
                if (!(isfinite(xa[j]) && isfinite(xb[j]) && isfinite(ka[j]) && isfinite(kb[j]))) err |= kErrRange;
            }
            if (!TAN) {
                if (nu < 0 || s == 0) continue;
                const int rs = s;
                const int key = (int)nu;
                const uint32_t h = ((uint32_t)key * 2654435761u) >> kHashShift;
                bool done = false;
                for (int pr = 0; pr < 8 && !done; ++pr) {
                    const int slot = (int)((h + (uint32_t)pr) & (uint32_t)(kSlots - 1));
                    int k = __hip_atomic_load(&s_key[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    if (k == -1) {
                        k = atomicCAS(&s_key[slot], -1, key);
                        if (k == -1) ++ins;
                    }
                    if (k == -1 || k == key) {
                        atomicAdd(&s_val[slot], rs);
                        done = true;
                    }
                }
                if (!done) atomicAdd(&cg[cbase + nu], rs);
            } else {
                // lanes hold consecutive particles: sum equal-cell runs in
                // registers, then the run's last lane adds them to the cell's
                // slot (sp2's cell counts come from the bootstrap)
                bool commit;
                const bool cnt = !ghost && !SP2;
                const int ns = run_sum<int>(nu, (cnt && nu >= 0) ? s : 0, commit);
                const bool in = nu >= 0;
                const int64_t ds = ghost ? d.gcap_total : d.cap_total;
                const int no = run_sum<int>(nu, in ? 1 : 0, commit);
                unsigned long long tq[6];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    int64_t hi = 0;
                    uint64_t lo = 0;
                    if (in && !fx_split(E.D[c * ds + i], hi, lo)) err |= kErrRange;
                    tq[2 * c] = (unsigned long long)run_sum<int64_t>(nu, hi, commit);
                    tq[2 * c + 1] = (unsigned long long)run_sum<uint64_t>(nu, lo, commit);
                }
                if (commit) {
                    const int key = (int)nu;
                    const uint32_t h = ((uint32_t)key * 2654435761u) >> kHashShift;
                    int slot = -1;
                    for (int pr = 0; pr < 8 && slot < 0; ++pr) {
                        const int sl = (int)((h + (uint32_t)pr) & (uint32_t)(kSlots - 1));
                        int k = __hip_atomic_load(&s_key[sl], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                        if (k == -1) {
                            k = atomicCAS(&s_key[sl], -1, key);
                            if (k == -1) ++ins;
                        }
                        if (k == -1 || k == key) slot = sl;
                    }
                    if (slot >= 0) {
                        if (ns) atomicAdd(&s_val[slot], ns);
                        atomicAdd(&s_occ[slot], no);
#pragma unroll
                        for (int q = 0; q < 6; ++q)
                            if (tq[q]) atomicAdd(&s_tq[q][slot], tq[q]);
                    } else {   // every probe taken: straight to the grids
                        if (ns) atomicAdd(&cg[cbase + nu], ns);
                        atomicAdd(&og[cbase + nu], no);
#pragma unroll
                        for (int q = 0; q < 6; ++q)
                            if (tq[q]) atomicAdd((unsigned long long *)&tg[(int64_t)q * ncell + cbase + nu], tq[q]);
                    }
                }
            }
        }
        if (esc) atomicAdd((unsigned long long *)&s_esc, (unsigned long long)esc);
        {   // the tile's new keys, one LDS atomic per wavefront
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) ins += __shfl_xor(ins, o, 64);
            if ((tid & 63) == 0 && ins) atomicAdd(&s_nkeys, ins);
            ins = 0;
        }
    }
    __syncthreads();
    if (cb >= 0) flush(cb);
    if (err) atomicOr(&ctl->err, err);
}

// ---------------------------------------------------------------------------
// sp1 annihilation, pass 2: ordered scan of |n_nu| per instance, in three
// launches with no tile waiting for another: k_scan_sums (the sum of every
// scan tile), k_close_scan (one block: their exclusive scan, the new counts
// Nnew[b] with the capacity clamp, the regeneration-tile plan), k_scan
// (off[nu] = exclusive prefix | (n_nu < 0 ? bit 62 : 0), the first cell of
// every regeneration tile; with zero_counts the count grid is cleared for the
// next annihilation).  A look-back chain over the tiles of an instance cost
// more than the extra launch.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_scan_sums(Dev d)
{
    if (ann_skipped(d)) return;
    __shared__ uint64_t s_w[kThreads / 64];
    const int B = d.B;
    const int64_t tiles_per = (d.Nh + kTileS - 1) / kTileS;
    const int64_t ntiles = tiles_per * B;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int b = (int)(t / tiles_per);
        const int64_t tl = t - (int64_t)b * tiles_per;
        const int64_t cbase = (int64_t)b * d.Nh;
        uint64_t sum = 0;
        if (d.cntx == nullptr || d.strategy == WBRW_SP2) {
#pragma unroll
            for (int j = 0; j < kPPT; ++j) {      // lanes take consecutive cells
                const int64_t c = tl * kTileS + (int64_t)j * kThreads + tid;
                const int32_t v = c < d.Nh ? d.cnt[cbase + c] : 0;
                sum += (uint64_t)(v < 0 ? -v : v);
            }
        } else {
            // fold the XCD copies of the sp1 counts into cnt and clear them;
            // every cell's loads are issued before any is used
            const int64_t nc = d.Nh * B;
            int32_t v[kPPT], part[kPPT][kXcd - 1];
#pragma unroll
            for (int j = 0; j < kPPT; ++j) {
                const int64_t c = min(tl * kTileS + (int64_t)j * kThreads + tid, d.Nh - 1);
                v[j] = d.cnt[cbase + c];
#pragma unroll
                for (int x = 0; x < kXcd - 1; ++x) part[j][x] = d.cntx[(int64_t)x * nc + cbase + c];
            }
#pragma unroll
            for (int j = 0; j < kPPT; ++j) {
                const int64_t c = tl * kTileS + (int64_t)j * kThreads + tid;
                if (c >= d.Nh) continue;
                const int64_t g = cbase + c;
                bool moved = false;
#pragma unroll
                for (int x = 0; x < kXcd - 1; ++x) {
                    v[j] += part[j][x];
                    if (part[j][x] != 0) {
                        d.cntx[(int64_t)x * nc + g] = 0;
                        moved = true;
                    }
                }
                if (moved) d.cnt[g] = v[j];
                sum += (uint64_t)(v[j] < 0 ? -v[j] : v[j]);
            }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
        if (lane == 0) s_w[wv] = sum;
        __syncthreads();
        if (tid == 0) {
            uint64_t tot = 0;
            for (int q = 0; q < kThreads / 64; ++q) tot += s_w[q];
            d.stS[t] = tot;
        }
        __syncthreads();
    }
}

// With tangents: the XCD copies of the occupancy and tangent sums are added
// into occ and Tcell (in copy order) and cleared.
__global__ __launch_bounds__(kThreads) void k_fold_tangents(Dev d)
{
    const int64_t nc = d.Nh * (int64_t)d.B;
    for (int64_t g = (int64_t)blockIdx.x * kThreads + threadIdx.x; g < nc; g += (int64_t)gridDim.x * kThreads) {
        int32_t po[kXcd - 1];
#pragma unroll
        for (int x = 0; x < kXcd - 1; ++x) po[x] = d.occx[(int64_t)x * nc + g];
        int32_t o = d.occ[g];
        int64_t tv[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) tv[q] = d.Tq[q * nc + g];
        bool any = false;
        for (int x = 0; x < kXcd - 1; ++x) {
            if (po[x] == 0) continue;   // a copy that saw no particle here holds no sums
            const int64_t tx = (int64_t)x * 6 * nc + g;
            o += po[x];
            d.occx[(int64_t)x * nc + g] = 0;
#pragma unroll
            for (int q = 0; q < 6; ++q) {   // exact integer sums: any order
                tv[q] += d.Tqx[tx + q * nc];
                d.Tqx[tx + q * nc] = 0;
            }
            any = true;
        }
        if (any) {
            d.occ[g] = o;
#pragma unroll
            for (int q = 0; q < 6; ++q) d.Tq[q * nc + g] = tv[q];
        }
    }
}

// After k_scan_sums (one block): the scan of the tile sums (in place), the
// new counts with the capacity clamp, and the regeneration-tile plan.
__global__ __launch_bounds__(kThreads) void k_close_scan(Dev d)
{
    if (ann_skipped(d)) return;
    Ctl *ctl = d.ctl;
    const int B = d.B;
    const int64_t tiles_per = (d.Nh + kTileS - 1) / kTileS;
    const int64_t T = tiles_per * B;
    const uint64_t total = scan_tile_counts(d.stS, d.stS, T);
    for (int b = threadIdx.x; b < B; b += kThreads) {
        const int64_t f = (int64_t)b * tiles_per, l = f + tiles_per;
        int64_t n = (int64_t)((l < T ? d.stS[l] : total) - d.stS[f]);
        if (n > d.ip[b].cap) {
            atomicOr(&ctl->err, kErrCapacity);
            n = d.ip[b].cap;
        }
        d.Nnew[b] = n;
    }
    __syncthreads();
    block_plan(d.tileR, d.Nnew, B, kTileR);
}

__global__ __launch_bounds__(kThreads) void k_scan(Dev d, int zero_counts)
{
    if (ann_skipped(d)) return;
    // Lanes take consecutive cells (coalesced): cell j * kThreads + tid of the
    // tile.  Each of the kPPT rows is scanned within the wavefront; the
    // (row, wavefront) totals are scanned in that order by one wavefront.
    constexpr int kW = kThreads / 64;
    __shared__ uint32_t s_tot[kPPT * kW];
    const int B = d.B;
    const int64_t tiles_per = (d.Nh + kTileS - 1) / kTileS;
    const int64_t ntiles = tiles_per * B;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int b = (int)(t / tiles_per);
        const int64_t tl = t - (int64_t)b * tiles_per;
        const int64_t cbase = (int64_t)b * d.Nh;
        const int64_t c0 = tl * kTileS + tid;
        int32_t v[kPPT];
        uint32_t ex[kPPT];
#pragma unroll
        for (int j = 0; j < kPPT; ++j) {
            const int64_t c = c0 + (int64_t)j * kThreads;
            v[j] = (c < d.Nh) ? d.cnt[cbase + c] : 0;
        }
#pragma unroll
        for (int j = 0; j < kPPT; ++j) {
            const uint32_t a = (uint32_t)(v[j] < 0 ? -v[j] : v[j]);
            uint32_t incl = a;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const uint32_t y = __shfl_up(incl, o, 64);
                if (lane >= o) incl += y;
            }
            if (lane == 63) s_tot[j * kW + wv] = incl;
            ex[j] = incl - a;
        }
        __syncthreads();
        if (wv == 0) {   // exclusive scan of the kPPT * kW totals, in place
            const uint32_t a = lane < kPPT * kW ? s_tot[lane] : 0u;
            uint32_t incl = a;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const uint32_t y = __shfl_up(incl, o, 64);
                if (lane >= o) incl += y;
            }
            if (lane < kPPT * kW) s_tot[lane] = incl - a;
        }
        __syncthreads();
        const int64_t tbase = (int64_t)(d.stS[t] - d.stS[(int64_t)b * tiles_per]);
        const InstParam &P = d.ip[b];
        int64_t *rst = d.rstart + P.rbase;
#pragma unroll
        for (int j = 0; j < kPPT; ++j) {
            const int64_t c = c0 + (int64_t)j * kThreads;
            if (c >= d.Nh) continue;
            const int64_t run = tbase + (int64_t)s_tot[j * kW + wv] + (int64_t)ex[j];
            const int64_t a = v[j] < 0 ? -v[j] : v[j];
            d.off[cbase + c] = run | (v[j] < 0 ? kOffNeg : 0);
            // this cell holds the first output of every regeneration tile
            // that starts inside [run, run + a)
            for (int64_t q = (run + kTileR - 1) / kTileR; q * kTileR < run + a && q < P.rtiles; ++q)
                rst[q] = c;
            if (zero_counts && v[j] != 0) d.cnt[cbase + c] = 0;
        }
        __syncthreads();
    }
}

// largest cell nu in [lo, hi] with (off[nu] & mask) <= o
__device__ __forceinline__ int64_t cell_of_output(const int64_t *off, int64_t lo, int64_t hi, int64_t o)
{
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if ((off[mid] & kOffMask) <= o) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// ---------------------------------------------------------------------------
// sp1/sp2 annihilation, pass 3: regeneration into the inactive buffer set.
// ---------------------------------------------------------------------------
template <int DIM, bool SP2, bool TAN>
__global__ __launch_bounds__(kThreads) void k_regen(Dev d)
{
    if (ann_skipped(d)) return;
    Ctl *ctl = d.ctl;
    const uint32_t step = ctl->step;
    const int B = d.B;
    const int64_t ntiles = d.tileR[B];
    const Ens O = pick_set(d, 0, ctl->cur ^ 1u);
    const int tid = threadIdx.x;
    // the offsets of a tile's cells, staged in LDS when they fit, so that the
    // searches below cost LDS rather than dependent global loads
    constexpr int kCells = 2048;
    __shared__ int64_t s_off[kCells];
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        __syncthreads();
        const int b = segment_of(d.tileR, B, t);
        const InstParam &P = d.ip[b];
        const int64_t nout = d.Nnew[b];
        const int64_t cbase = (int64_t)b * d.Nh;
        const int64_t *off = d.off + cbase;
        // the tile's outputs lie in cells [first cell of this tile, first
        // cell of the next one] (the scan recorded both), so each search
        // covers a few cells where the ensemble is dense
        const int64_t q = t - d.tileR[b];
        const int64_t nu_lo = d.rstart[P.rbase + q];
        const int64_t nu_hi = (q + 1) * kTileR < nout ? d.rstart[P.rbase + q + 1] : d.Nh - 1;
        const int64_t span = nu_hi - nu_lo + 1;
        const bool staged = span <= kCells;
        if (staged)
            for (int c = tid; c < (int)span; c += kThreads) s_off[c] = off[nu_lo + c];
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kTileR / kThreads; ++j) {
            const int64_t o = q * kTileR + (int64_t)j * kThreads + tid;
            if (o >= nout) continue;
            int64_t nu, onu;
            if (staged) {
                int lo = 0, hi = (int)span - 1;   // the last staged cell with offset <= o
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if ((s_off[mid] & kOffMask) <= o) lo = mid; else hi = mid - 1;
                }
                nu = nu_lo + lo;
                onu = s_off[lo];
            } else {
                nu = cell_of_output(off, nu_lo, nu_hi, o);
                onu = off[nu];
            }
            const int64_t jj = o - (onu & kOffMask);
            const uint64_t id = ((uint64_t)nu << 32) | (uint64_t)jj;
            double x[2] = {0.0, 0.0}, k[2] = {0.0, 0.0};
            cell_point<DIM>(d, nu, id, kTagRegen, step, P.key, x, k);
            // the ensemble is read again only by the next launches: its
            // writes bypass the caches (non-temporal)
            const int64_t i = P.base + o;
            __builtin_nontemporal_store(x[0], &O.x0[i]);
            __builtin_nontemporal_store(k[0], &O.k0[i]);
            if (DIM == 2) {
                __builtin_nontemporal_store(x[1], &O.x1[i]);
                __builtin_nontemporal_store(k[1], &O.k1[i]);
            }
            const bool neg = (onu & kOffNeg) != 0;
            if (SP2) O.w[i] = neg ? -1.0 : 1.0; else O.sg[i] = neg ? (int8_t)-1 : (int8_t)1;
            __builtin_nontemporal_store(id, &O.id[i]);
            if (TAN) {
                const int64_t nxt = (nu + 1 < d.Nh) ? (off[nu + 1] & kOffMask) : nout;
                const double an = (double)(nxt - (onu & kOffMask));
                const int64_t nc = d.Nh * (int64_t)B;
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    O.D[c * d.cap_total + i] = fx_value(d.Tq[(2 * c) * nc + cbase + nu],
                                                        (uint64_t)d.Tq[(2 * c + 1) * nc + cbase + nu]) / an;
            }
        }
    }
}

// After k_regen (one block): the new counts and tile plan; the regenerated
// buffer set becomes the active one.
__global__ __launch_bounds__(kThreads) void k_close_regen(Dev d)
{
    if (ann_skipped(d)) return;
    Ctl *ctl = d.ctl;
    const int B = d.B;
    for (int b = threadIdx.x; b < B; b += kThreads) {
        d.N[b] = d.Nnew[b];
        d.Nsrt[b] = d.Nnew[b];   // the regenerated ensemble is in cell order
        d.tally[(int64_t)b * kTalCount + kTalAnn] += 1;
    }
    __syncthreads();
    block_plan(d.tileA, d.N, B, kTileA);
    block_prefix(d.srtS, B, [&](int b) { return d.Nsrt[b] / kTileA; });
    if (threadIdx.x == 0) {
        ctl->cur ^= 1u;
        ctl->ann_seq += 1u;
    }
}

// ---------------------------------------------------------------------------
// Density: bins of width (hi - lo)/nbins on position axis `axis`.
// ---------------------------------------------------------------------------
template <int DIM, bool SP2, bool TAN>
__global__ __launch_bounds__(kThreads) void k_density_bin(Dev d, int ghost, int axis, int nbins,
                                                          double lo, double dxb)
{
    // Each block keeps a private histogram of the instance it is working on
    // in LDS and adds its non-zero bins to the global accumulator when its
    // tiles move on to the next instance and when it runs out of tiles.
    // Integer weights (signs, 32.32 fixed-point weights) sum exactly in any
    // order.  Histograms wider than the LDS array go straight to HBM.  The
    // tangent histogram (six words per bin) keeps up to 2048 bins in LDS,
    // 96 KB: one block per CU, each flushing once (its own grid).
    constexpr int kLds = TAN ? 12288 : 4096;
    __shared__ uint64_t s_raw[kLds];
    Ctl *ctl = d.ctl;
    const int B = d.B;
    const int64_t *plan = d.tileA + (int64_t)ghost * (B + 1);
    const int64_t ntiles = plan[B];
    const int64_t *Ncur = ghost ? d.NG : d.N;
    const Ens E = pick_set(d, ghost, ghost ? ctl->gcur : ctl->cur);
    const double *X = (axis == 1) ? E.x1 : E.x0;
    const int64_t ds = ghost ? d.gcap_total : d.cap_total;
    const int tid = threadIdx.x, lane = tid & 63;
    // this block's XCD copy of the accumulator (atomics stay in its L2)
    int64_t *const dx = d.dacc + (int64_t)(blockIdx.x % kXcd) * B * d.max_bins;
    // tangents: six fixed-point words per bin (high and low word of each
    // component, see fx_split), exact in any order
    const int width = TAN ? 6 * nbins : nbins;
    const bool priv = width <= kLds;
    uint32_t err = 0;
    if (priv)
        for (int j = tid; j < width; j += kThreads) s_raw[j] = 0ull;
    int cb = -1;
    auto flush = [&](int fb) {
        __syncthreads();
        for (int j = tid; j < width; j += kThreads) {
            const uint64_t v = s_raw[j];
            if (v == 0ull) continue;
            s_raw[j] = 0ull;
            if (TAN) {
                const int w = j / nbins, bin = j - w * nbins;
                atomicAdd((unsigned long long *)(d.dTq + (int64_t)fb * 6 * d.max_bins + (int64_t)w * d.max_bins + bin),
                          (unsigned long long)v);
            } else {
                atomicAdd((unsigned long long *)&dx[(int64_t)fb * d.max_bins + j], (unsigned long long)v);
            }
        }
        __syncthreads();
    };
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        __syncthreads();
        const int b = segment_of(plan, B, t);
        if (priv && b != cb) {
            if (cb >= 0) flush(cb);
            cb = b;
        }
        const InstParam &P = d.ip[b];
        const int64_t base = ghost ? P.gbase : P.base;
        const int64_t n = Ncur[b];
        const int64_t li0 = (t - plan[b]) * kTileA + tid;
        double xv[kPPT], wv[kPPT];
#pragma unroll
        for (int j = 0; j < kPPT; ++j) {      // loads first
            const int64_t li = li0 + (int64_t)j * kThreads;
            const int64_t i = base + (li < n ? li : 0);
            xv[j] = X[i];
            if (!TAN) wv[j] = SP2 ? E.w[i] : (double)E.sg[i];
        }
#pragma unroll
        for (int j = 0; j < kPPT; ++j) {
            const int64_t li = li0 + (int64_t)j * kThreads;
            const bool live = li < n;
            const int64_t i = base + (live ? li : 0);
            const double q = (xv[j] - lo) / dxb;
            const int64_t bin = (live && q >= 0.0 && q < (double)nbins) ? (int64_t)q : -1;
            bool commit;
            if (TAN) {
                const bool in = bin >= 0;
                int64_t *acc = d.dTq + (int64_t)b * 6 * d.max_bins;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    int64_t hi = 0;
                    uint64_t lo = 0;
                    if (in && !fx_split(E.D[c * ds + i], hi, lo)) err |= kErrRange;
                    hi = run_sum<int64_t>(bin, hi, commit);
                    lo = run_sum<uint64_t>(bin, lo, commit);
                    if (!commit) continue;
                    if (priv) {
                        if (hi) atomicAdd((unsigned long long *)&s_raw[(2 * c) * nbins + bin], (unsigned long long)hi);
                        if (lo) atomicAdd((unsigned long long *)&s_raw[(2 * c + 1) * nbins + bin], (unsigned long long)lo);
                    } else {
                        if (hi) atomicAdd((unsigned long long *)&acc[(int64_t)(2 * c) * d.max_bins + bin], (unsigned long long)hi);
                        if (lo) atomicAdd((unsigned long long *)&acc[(int64_t)(2 * c + 1) * d.max_bins + bin], (unsigned long long)lo);
                    }
                }
            } else {
                uint64_t *acc = priv ? s_raw : (uint64_t *)dx + (int64_t)b * d.max_bins;
                if (SP2) {
                    int64_t v = bin >= 0 ? (int64_t)(wv[j] * 4294967296.0) : 0;
                    v = run_sum<int64_t>(bin, v, commit);
                    if (commit && v != 0) atomicAdd((unsigned long long *)&acc[bin], (unsigned long long)v);
                    continue;
                }
                // sp1 signs are +-1: a run of equal bins across the wavefront
                // sums to (# plus) - (# minus) of its lanes.  A wavefront with
                // few runs (the cell-ordered front) commits one atomic per run;
                // one with many (scattered offspring) adds lane by lane.
                const int key = (int)bin;
                const int sgn = bin >= 0 ? (int)wv[j] : 0;
                const uint64_t plus = __ballot(sgn > 0), minus = __ballot(sgn < 0);
                const int prev = __shfl_up(key, 1, 64);
                const uint64_t heads = __ballot(lane == 0 || key != prev);
                if (__popcll(heads) > 8) {
                    if (sgn != 0) atomicAdd((unsigned long long *)&acc[bin], (unsigned long long)(int64_t)sgn);
                    continue;
                }
                for (uint64_t hm = heads; hm != 0ull;) {
                    const int h = __builtin_ctzll(hm);
                    hm &= hm - 1ull;
                    const uint64_t upto = hm ? ((1ull << __builtin_ctzll(hm)) - 1ull) : ~0ull;
                    const uint64_t seg = upto & ~((1ull << h) - 1ull);
                    const int v = __popcll(plus & seg) - __popcll(minus & seg);
                    const int kh = __builtin_amdgcn_readlane(key, h);
                    if (lane == h && kh >= 0 && v != 0)
                        atomicAdd((unsigned long long *)&acc[kh], (unsigned long long)(int64_t)v);
                }
            }
        }
    }
    if (priv && cb >= 0) flush(cb);
    if (err) atomicOr(&ctl->err, err);
}

// out[b][j] = acc / (N0_b dxb); the accumulator is cleared.
template <bool SP2, bool TAN>
__global__ __launch_bounds__(kThreads) void k_density_out(Dev d, int nbins, double dxb, double *out)
{
    const int B = d.B;
    const int comps = TAN ? 3 : 1;
    const int64_t total = (int64_t)B * comps * nbins;
    for (int64_t g = (int64_t)blockIdx.x * kThreads + threadIdx.x; g < total;
         g += (int64_t)gridDim.x * kThreads) {
        const int64_t b = g / ((int64_t)comps * nbins);
        const int64_t r = g - b * comps * nbins;
        const int64_t c = r / nbins, j = r - c * nbins;
        const double denom = (double)d.ip[b].N0 * dxb;
        if (TAN) {
            int64_t *acc = d.dTq + b * 6 * d.max_bins + (2 * c) * d.max_bins + j;
            out[g] = fx_value(acc[0], (uint64_t)acc[d.max_bins]) / denom;
            acc[0] = 0;
            acc[d.max_bins] = 0;
        } else {
            // the XCD copies, summed in copy order (exact integers) and cleared
            int64_t sum = 0;
            for (int x = 0; x < kXcd; ++x) {
                int64_t *acc = d.dacc + ((int64_t)x * B + b) * d.max_bins + j;
                sum += *acc;
                *acc = 0;
            }
            double v = (double)sum;
            if (SP2) v = v * 0x1p-32;
            out[g] = v / denom;
        }
    }
}

// Vector-Jacobian product of the density, after k_density_bin<.., true> has
// summed the tangents of real particles and ghosts per bin:
// grad[b][c] = (sum over bins j in ascending order of g[b][j] T_c[j]) /
// (N0_b dxb), T_c[j] the fixed-point bin sum; one thread per (instance,
// component), which also clears its sums.  This is the backward pass of the
// differentiation form: the likelihood-ratio scores are already carried per
// particle.
__global__ __launch_bounds__(kThreads) void k_vjp_out(Dev d, int nbins, double dxb, const double *g, double *out)
{
    // One wavefront per (instance, component): the lanes load 64 bins at a
    // time and form their products g_j T_j, which are then added in
    // ascending bin order (the order that fixes the result's bits).
    const int lane = threadIdx.x & 63;
    constexpr int kW = kThreads / 64;
    for (int64_t q = (int64_t)blockIdx.x * kW + (threadIdx.x >> 6); q < (int64_t)d.B * 3;
         q += (int64_t)gridDim.x * kW) {
        const int64_t b = q / 3, c = q - b * 3;
        int64_t *hi = d.dTq + b * 6 * d.max_bins + (2 * c) * d.max_bins;
        int64_t *lo = hi + d.max_bins;
        const double *gb = g + b * nbins;
        double acc = 0.0;
        for (int j0 = 0; j0 < nbins; j0 += 64) {
            const int j = j0 + lane;
            double p = 0.0;
            if (j < nbins) {
                p = gb[j] * fx_value(hi[j], (uint64_t)lo[j]);
                hi[j] = 0;
                lo[j] = 0;
            }
            const int m = min(64, nbins - j0);
            const uint64_t pb = (uint64_t)__double_as_longlong(p);
            const int plo = (int)(uint32_t)pb, phi = (int)(uint32_t)(pb >> 32);
            for (int k = 0; k < m; ++k) {   // lane k's product, read as a scalar
                const uint64_t v = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane(phi, k) << 32) |
                                   (uint64_t)(uint32_t)__builtin_amdgcn_readlane(plo, k);
                acc = acc + __longlong_as_double((long long)v);
            }
        }
        if (lane == 0) out[q] = acc / ((double)d.ip[b].N0 * dxb);
    }
}

// Clears `n` 64-bit words (used instead of hipMemsetAsync so that every
// enqueued operation is a kernel).
__global__ __launch_bounds__(kThreads) void k_fill64(uint64_t *p, int64_t n, uint64_t v)
{
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
        p[i] = v;
}

// The same for 32-bit words.
__global__ __launch_bounds__(kThreads) void k_fill32(int32_t *p, int64_t n, int32_t v)
{
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
        p[i] = v;
}

}  // namespace wbrw
