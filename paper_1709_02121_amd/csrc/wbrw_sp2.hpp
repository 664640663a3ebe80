// sp2 annihilation: the signed residual bootstrap (Alg. 2 applied to each sign
// class, Eqs. lambda and double_bootstrap of Sec. 3.3), the histogram of the
// filtered classes (Eq. boostrap_histogram, Sec. 4.3) and the rounding step of
// Alg. 3; plus the tangent ghosts of the differentiation form.
//
// The weights are quantised once, A_i = floor(|w_i| 2^32); everything after
// that is exact integer arithmetic, so the result does not depend on the order
// in which the GPU reduces:
//   N_c, S_c = sum A_i                    per class c (integer atomics)
//   k_i = floor(N_c A_i / S_c), r_i = N_c A_i - k_i S_c   (copies kept, residual)
//   P_c = exclusive prefix of r_i over the class in particle order (128-bit)
//   N_r = N_c - sum k_i draws U_d uniform in [0, S_c N_r), each adding one copy
//         to the i with P_c[i] <= U_d < P_c[i+1]
//   n~_c[nu] = sum of copies per cell
//   m_nu = |S+ n~+ N- - S- n~- N+| / (2^32 N+ N-), rounded up with probability
//          equal to its fractional part (one uniform per cell), sign of the
//          difference; then the sp1 scan / regeneration.
#pragma once
#include "wbrw_cells.hpp"
#include "wbrw_dev.hpp"
#include "wbrw_math.hpp"

namespace wbrw {

typedef unsigned __int128 u128;
typedef __int128 i128;

// bcls_stat slots per instance
enum : int { kBN0 = 0, kBN1, kBS0, kBS1, kBK0, kBK1, kBNr0, kBNr1 };

// floor(r * R / 2^64): an integer uniform on [0, R) from 64 random bits
__device__ __forceinline__ u128 scale64(uint64_t r, u128 R)
{
    const uint64_t lo = (uint64_t)R;
    const u128 hi = R >> 64;
    return (u128)r * hi + (((u128)r * (u128)lo) >> 64);
}

__device__ __forceinline__ void st128(uint64_t *p, u128 v)
{
    p[0] = (uint64_t)v;
    p[1] = (uint64_t)(v >> 64);
}

// st128 past the caches, for data that only a later launch reads
__device__ __forceinline__ void st128_nt(uint64_t *p, u128 v)
{
    __builtin_nontemporal_store((uint64_t)v, p);
    __builtin_nontemporal_store((uint64_t)(v >> 64), p + 1);
}

__device__ __forceinline__ u128 ld128(const uint64_t *p)
{
    return ((u128)p[1] << 64) | (u128)p[0];
}

// Sum of v over the block (all threads call it; the result is in thread 0).
__device__ __forceinline__ unsigned long long block_sum(unsigned long long v, unsigned long long *s_w)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    __syncthreads();
    if (lane == 0) s_w[wv] = v;
    __syncthreads();
    unsigned long long t = 0;
    if (threadIdx.x == 0)
        for (int q = 0; q < kThreads / 64; ++q) t += s_w[q];
    return t;
}

// ---- stage 1: classes, quantised weights, cells; class sizes and sums ------
// Each block takes a contiguous run of tiles and sums N+, N-, S+, S- and the
// escaped weight per instance; a block's last instance is left in its slot
// of fpart for k_sp2_close_classify (others, rare, go to the counters
// directly).  Per-tile atomics on the instance's counters would serialise.
template <int DIM>
__global__ __launch_bounds__(kThreads) void k_sp2_classify(Dev d)
{
    if (ann_skipped(d)) return;
    __shared__ unsigned long long s_w[kThreads / 64];
    Ctl *ctl = d.ctl;
    const int B = d.B;
    const int64_t *plan = d.tileA;
    const int64_t ntiles = plan[B];
    const Ens E = pick_set(d, 0, ctl->cur);
    const int tid = threadIdx.x;
    unsigned long long acc[5] = {0, 0, 0, 0, 0};   // N0, N1, S0, S1, escaped
    auto publish = [&](int fb, bool last) {
        unsigned long long tot[5];
        for (int q = 0; q < 5; ++q) tot[q] = block_sum(acc[q], s_w);
        if (tid == 0) {
            if (last) {
                int64_t *F = d.fpart + (int64_t)blockIdx.x * 8;
                F[0] = fb;
                for (int q = 0; q < 5; ++q) F[1 + q] = (int64_t)tot[q];
            } else {
                unsigned long long *st = (unsigned long long *)(d.bcls_stat + (int64_t)fb * 8);
                for (int q = 0; q < 4; ++q)
                    if (tot[q]) atomicAdd(&st[q], tot[q]);
                if (tot[4])
                    atomicAdd((unsigned long long *)&d.tally[(int64_t)fb * kTalCount + kTalEscaped], tot[4]);
            }
        }
        for (int q = 0; q < 5; ++q) acc[q] = 0;
    };
    const int64_t per = (ntiles + gridDim.x - 1) / gridDim.x;
    const int64_t t0 = min((int64_t)blockIdx.x * per, ntiles), t1 = min(t0 + per, ntiles);
    int cb = -1;
    for (int64_t t = t0; t < t1; ++t) {
        const int b = segment_of(plan, B, t);
        if (b != cb) {
            if (cb >= 0) publish(cb, false);
            cb = b;
        }
        const InstParam &P = d.ip[b];
        const int64_t n = d.N[b];
        const int64_t li0 = (t - plan[b]) * kTileA + tid;
        double wv[kPPT], xa[kPPT], xb[kPPT], ka[kPPT], kb[kPPT];
#pragma unroll
        for (int j = 0; j < kPPT; ++j) {      // loads first: kPPT in flight per thread
            const int64_t li = li0 + (int64_t)j * kThreads;
            const int64_t i = P.base + (li < n ? li : 0);
            wv[j] = E.w[i];
            xa[j] = E.x0[i];
            ka[j] = E.k0[i];
            xb[j] = DIM == 2 ? E.x1[i] : 0.0;
            kb[j] = DIM == 2 ? E.k1[i] : 0.0;
        }
#pragma unroll
        for (int j = 0; j < kPPT; ++j) {
            const int64_t li = li0 + (int64_t)j * kThreads;
            if (li >= n) continue;
            const int64_t i = P.base + li;
            const double w = wv[j];
            const uint64_t A = (uint64_t)floor(fabs(w) * 4294967296.0);
            const int64_t nu = cell_index<DIM>(d, xa[j], xb[j], ka[j], kb[j]);
            int8_t cls = -1;
            if (nu < 0) {
                acc[4] += w < 0.0 ? (unsigned long long)(-(long long)A) : (unsigned long long)A;
            } else if (w > 0.0) {
                cls = 0; acc[0] += 1; acc[2] += A;
            } else if (w < 0.0) {
                cls = 1; acc[1] += 1; acc[3] += A;
            }
            d.bcls[i] = cls;
            d.bA[i] = cls >= 0 ? A : 0ull;
            d.bcell[i] = nu;
        }
    }
    publish(cb, true);
}

// After k_sp2_classify (one block): the blocks' last-instance sums into the
// class counters (summed per instance in LDS when the instances fit).
__global__ __launch_bounds__(kThreads) void k_sp2_close_classify(Dev d, int grid)
{
    if (ann_skipped(d)) return;
    constexpr int kLdsB = 512;
    __shared__ unsigned long long s_acc[5][kLdsB];
    const int B = d.B;
    const int tid = threadIdx.x;
    const bool lds = B <= kLdsB;
    if (lds)
        for (int b = tid; b < B; b += kThreads)
            for (int q = 0; q < 5; ++q) s_acc[q][b] = 0;
    __syncthreads();
    for (int g = tid; g < grid; g += kThreads) {
        const int64_t *F = d.fpart + (int64_t)g * 8;
        if (F[0] < 0) continue;
        const int b = (int)F[0];
        for (int q = 0; q < 5; ++q) {
            if (!F[1 + q]) continue;
            if (lds) {
                atomicAdd(&s_acc[q][b], (unsigned long long)F[1 + q]);
            } else if (q < 4) {
                atomicAdd((unsigned long long *)&d.bcls_stat[(int64_t)b * 8 + q], (unsigned long long)F[1 + q]);
            } else {
                atomicAdd((unsigned long long *)&d.tally[(int64_t)b * kTalCount + kTalEscaped],
                          (unsigned long long)F[5]);
            }
        }
    }
    __syncthreads();
    if (lds)
        for (int b = tid; b < B; b += kThreads) {
            int64_t *st = d.bcls_stat + (int64_t)b * 8;
            for (int q = 0; q < 4; ++q) st[q] += (int64_t)s_acc[q][b];
            d.tally[(int64_t)b * kTalCount + kTalEscaped] += (int64_t)s_acc[4][b];
        }
}

// ---- stage 2: kept copies k_i, residuals r_i, per-tile residual sums --------
// Each block takes a contiguous run of tiles; the kept-copy sums per class
// are summed per instance and left in fpart (instance changes, rare, add to
// the counters) for k_sp2_tilescan.  The 128-bit residual sums are per tile.

// floor(num / den) and the remainder for num < 2^63, 0 < den < 2^63 and a
// quotient below 2^32 (k_i <= N_c here), from rcp = 1/den in double: the
// estimate num * rcp is within one of the quotient, and the remainder,
// exact in 64-bit arithmetic since q den <= num + den < 2^64, corrects it.
__device__ __forceinline__ uint64_t udiv_small(uint64_t num, uint64_t den, double rcp, uint64_t &rem)
{
    uint64_t q = (uint64_t)((double)num * rcp);
    int64_t r = (int64_t)(num - q * den);
    while (r < 0) { --q; r += (int64_t)den; }
    while ((uint64_t)r >= den) { ++q; r -= (int64_t)den; }
    rem = (uint64_t)r;
    return q;
}

__global__ __launch_bounds__(kThreads) void k_sp2_resid(Dev d)
{
    if (ann_skipped(d)) return;
    __shared__ uint64_t s_wlo[2][kThreads / 64], s_whi[2][kThreads / 64];   // wavefront residual sums
    __shared__ unsigned long long s_w[kThreads / 64];
    Ctl *ctl = d.ctl;
    const int B = d.B;
    const int64_t *plan = d.tileA;
    const int64_t ntiles = plan[B];
    const int tid = threadIdx.x;
    const int64_t C = d.cap_total;
    unsigned long long ks[2] = {0, 0};       // this thread's kept copies per class
    auto publish = [&](int fb, bool last) {
        const unsigned long long k0 = block_sum(ks[0], s_w), k1 = block_sum(ks[1], s_w);
        if (tid == 0) {
            if (last) {
                int64_t *F = d.fpart + (int64_t)blockIdx.x * 8;
                F[0] = fb;
                F[1] = (int64_t)k0;
                F[2] = (int64_t)k1;
            } else {
                unsigned long long *bs = (unsigned long long *)(d.bcls_stat + (int64_t)fb * 8);
                if (k0) atomicAdd(&bs[kBK0], k0);
                if (k1) atomicAdd(&bs[kBK1], k1);
            }
        }
        ks[0] = ks[1] = 0;
    };
    const int64_t per = (ntiles + gridDim.x - 1) / gridDim.x;
    const int64_t ta = min((int64_t)blockIdx.x * per, ntiles), tb = min(ta + per, ntiles);
    int cb = -1;
    for (int64_t t = ta; t < tb; ++t) {
        const int b = segment_of(plan, B, t);
        if (b != cb) {
            if (cb >= 0) publish(cb, false);
            cb = b;
        }
        __syncthreads();
        const InstParam &P = d.ip[b];
        const int64_t n = d.N[b];
        const int64_t *st = d.bcls_stat + (int64_t)b * 8;
        const uint64_t Nc[2] = {(uint64_t)st[kBN0], (uint64_t)st[kBN1]};
        const uint64_t Sc[2] = {(uint64_t)st[kBS0], (uint64_t)st[kBS1]};
        const double rcp[2] = {Sc[0] ? 1.0 / (double)Sc[0] : 0.0, Sc[1] ? 1.0 / (double)Sc[1] : 0.0};
        u128 rs[2] = {0, 0};
        const int64_t li0 = (t - plan[b]) * kTileA + tid;
        int8_t cv[kPPT];
        uint64_t av[kPPT];
#pragma unroll
        for (int j = 0; j < kPPT; ++j) {      // loads first: kPPT in flight per thread
            const int64_t li = li0 + (int64_t)j * kThreads;
            const int64_t i = P.base + (li < n ? li : 0);
            cv[j] = d.bcls[i];
            av[j] = d.bA[i];
        }
#pragma unroll
        for (int j = 0; j < kPPT; ++j) {
            const int64_t li = li0 + (int64_t)j * kThreads;
            if (li >= n) continue;
            const int64_t i = P.base + li;
            const int8_t c = cv[j];
            uint64_t k = 0, r = 0;
            if (c >= 0 && Sc[c] > 0) {
                const uint64_t num = Nc[c] * av[j];       // < 2^63
                k = udiv_small(num, Sc[c], rcp[c], r);
                ks[c] += k;
                rs[c] += r;
            }
            d.bcopies[i] = (int32_t)k;
            d.bA[i] = r;               // A_i is no longer needed: the residual
        }
        // tile sums of the 128-bit residuals: within each wavefront (64-bit
        // halves with carry), then the four wavefront sums by one thread
        for (int c = 0; c < 2; ++c) {
            uint64_t lo = (uint64_t)rs[c], hi = (uint64_t)(rs[c] >> 64);
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                const uint64_t plo = __shfl_xor(lo, o, 64), phi = __shfl_xor(hi, o, 64);
                const uint64_t nlo = lo + plo;
                hi = hi + phi + (nlo < lo ? 1ull : 0ull);
                lo = nlo;
            }
            if ((tid & 63) == 0) { s_wlo[c][tid >> 6] = lo; s_whi[c][tid >> 6] = hi; }
        }
        __syncthreads();
        if (tid == 0) {
            for (int c = 0; c < 2; ++c) {
                u128 sum = 0;
                for (int w = 0; w < kThreads / 64; ++w) sum += ((u128)s_whi[c][w] << 64) | s_wlo[c][w];
                st128(d.bTile + 2 * ((int64_t)c * d.tstride + t), sum);
            }
        }
        __syncthreads();
    }
    publish(cb, true);
}

// ---- stage 3: exclusive scan of the tile sums per instance and class; the
// draw counts N_r and the draw-tile plan.  One block per instance. ----------
// Exclusive scan of the 128-bit values v[t0..t1) in place, by one block.
// Chunks of kThreads x 8 values are loaded coalesced (all loads in flight)
// into LDS, padded by one slot per 8 so that the per-thread runs fall in
// different banks; every thread sums its run of 8, the run sums are scanned
// within each wavefront (64-bit halves with carry) and across the four
// wavefronts, and the prefixes leave LDS coalesced.
__device__ __forceinline__ void scan_u128_exclusive(uint64_t *v, int64_t t0, int64_t t1)
{
    constexpr int P = 8, C = kThreads * P, W = kThreads / 64;
    __shared__ uint64_t s_lo[C + C / P], s_hi[C + C / P];
    __shared__ uint64_t s_wlo[W], s_whi[W];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int run0 = tid * (P + 1);
    u128 carry = 0;
    for (int64_t c0 = t0; c0 < t1; c0 += C) {
        const int n = (int)min((int64_t)C, t1 - c0);
        __syncthreads();
        u128 x[P];
#pragma unroll
        for (int r = 0; r < P; ++r)   // clamped, unconditional: no branch between the loads
            x[r] = ld128(v + 2 * (c0 + min(r * kThreads + tid, n - 1)));
#pragma unroll
        for (int r = 0; r < P; ++r) {
            const int i = r * kThreads + tid;
            s_lo[i + i / P] = (uint64_t)x[r];
            s_hi[i + i / P] = (uint64_t)(x[r] >> 64);
        }
        __syncthreads();
        u128 acc = 0;
#pragma unroll
        for (int r = 0; r < P; ++r) {
            x[r] = tid * P + r < n ? (((u128)s_hi[run0 + r] << 64) | s_lo[run0 + r]) : (u128)0;
            acc += x[r];
        }
        uint64_t lo = (uint64_t)acc, hi = (uint64_t)(acc >> 64);
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint64_t plo = __shfl_up(lo, o, 64), phi = __shfl_up(hi, o, 64);
            if (lane >= o) {
                const uint64_t nlo = lo + plo;
                hi = hi + phi + (nlo < lo ? 1ull : 0ull);
                lo = nlo;
            }
        }
        if (lane == 63) { s_wlo[wv] = lo; s_whi[wv] = hi; }
        __syncthreads();
        u128 below = 0, chunk = 0;
#pragma unroll
        for (int w = 0; w < W; ++w) {
            const u128 t = ((u128)s_whi[w] << 64) | s_wlo[w];
            if (w < wv) below += t;
            chunk += t;
        }
        u128 run = carry + below + ((((u128)hi << 64) | lo) - acc);
#pragma unroll
        for (int r = 0; r < P; ++r) {
            s_lo[run0 + r] = (uint64_t)run;
            s_hi[run0 + r] = (uint64_t)(run >> 64);
            run += x[r];
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < P; ++r) {
            const int i = r * kThreads + tid;
            if (i < n) st128(v + 2 * (c0 + i), ((u128)s_hi[i + i / P] << 64) | s_lo[i + i / P]);
        }
        carry += chunk;
    }
    __syncthreads();
}

__global__ __launch_bounds__(kThreads) void k_sp2_tilescan(Dev d, int rgrid)
{
    if (ann_skipped(d)) return;
    __shared__ unsigned long long s_w[kThreads / 64];
    Ctl *ctl = d.ctl;
    const int B = d.B;
    const int tid = threadIdx.x;
    for (int b = blockIdx.x; b < B; b += gridDim.x) {
        // the k_sp2_resid blocks' kept-copy sums of this instance
        unsigned long long k0 = 0, k1 = 0;
        for (int g = tid; g < rgrid; g += kThreads) {
            const int64_t *F = d.fpart + (int64_t)g * 8;
            if (F[0] != b) continue;
            k0 += (unsigned long long)F[1];
            k1 += (unsigned long long)F[2];
        }
        k0 = block_sum(k0, s_w);
        k1 = block_sum(k1, s_w);
        if (tid == 0) {
            d.bcls_stat[(int64_t)b * 8 + kBK0] += (int64_t)k0;
            d.bcls_stat[(int64_t)b * 8 + kBK1] += (int64_t)k1;
        }
        const int64_t t0 = d.tileA[b], t1 = d.tileA[b + 1];
        for (int c = 0; c < 2; ++c)
            scan_u128_exclusive(d.bTile + 2 * ((int64_t)c * d.tstride), t0, t1);
        if (tid == 0) {
            int64_t *st = d.bcls_stat + (int64_t)b * 8;
            st[kBNr0] = st[kBN0] - st[kBK0];
            st[kBNr1] = st[kBN1] - st[kBK1];
            if (st[kBS0] == 0) st[kBNr0] = 0;
            if (st[kBS1] == 0) st[kBNr1] = 0;
            d.Nnew[b] = st[kBNr0];            // staging for the draw plan (class 0)
            d.NGnew[b] = st[kBNr1];           // (class 1)
        }
        __syncthreads();
    }
}

// After k_sp2_tilescan (one block): the draw-tile plans of both classes.
__global__ __launch_bounds__(kThreads) void k_close_sp2_tilescan(Dev d)
{
    if (ann_skipped(d)) return;
    const int B = d.B;
    block_plan(d.tileD, d.Nnew, B, kTileR);
    block_plan(d.tileD + (B + 1), d.NGnew, B, kTileR);
}

// ---- draw guide ------------------------------------------------------------
// A class with N_r draws splits the draws' 64 random bits into K = 2^bits
// buckets by their top bits, K the largest power of two below 4 N_r.  Guide
// entry k < K is the particle whose residual interval [P_i, P_i + r_i) holds
// the bucket's least value B_k = floor(k R / K); entry K is n - 1.  A draw in
// bucket k has B_k <= U <= B_(k+1), so its particle lies between entries k
// and k + 1 and the search over that slice returns what the search over the
// whole prefix does; mostly the slice is one particle, and there is no search.
// Since r_i < S_c, an interval spans less than K / N_r < 4 buckets, so a
// particle writes at most four entries.  The guide of an instance's class
// has 4 slots per particle slot: K + 1 <= 4 N_r <= 4 n entries fit.
__device__ __forceinline__ int sp2_guide_bits(int64_t Nr)
{
    // K < 4 N_r (K <= 2^30)
    return Nr >= 2 ? min(30, 65 - __clzll((unsigned long long)(Nr - 1))) : 0;
}

__device__ __forceinline__ double u128_to_f64(u128 v)
{
    return (double)(uint64_t)(v >> 64) * 0x1p64 + (double)(uint64_t)v;
}

// k R for k < 2^32: two 32 x 64-bit products (R < 2^95 as S_c < 2^64 and
// N_r < 2^31, so k R < 2^128)
__device__ __forceinline__ u128 mul32_128(uint32_t k, u128 R)
{
    return (u128)k * (uint64_t)R + (((u128)k * (uint64_t)(R >> 64)) << 64);
}

// The least k in [0, K] with B_k >= P, B_k = floor(k R / 2^bits) (the value
// scale64(k 2^(64 - bits), R) takes), B_K = R: the least k with
// k R >= P 2^bits.  The estimate e is within one of the exact quotient
// (K <= 2^30 as n < 2^31), so the corrections take a step or two.
__device__ __forceinline__ uint32_t sp2_guide_first(u128 P, int bits, u128 R)
{
    const uint32_t K = 1u << bits;
    const u128 Ps = P << bits;
    const double e = u128_to_f64(P) / u128_to_f64(R) * (double)K;
    uint32_t k = e <= 0.0 ? 0u : (e >= (double)K ? K : (uint32_t)e);
    while (k > 0 && mul32_128(k - 1, R) >= Ps) --k;
    while (k < K && mul32_128(k, R) < Ps) ++k;
    return k;
}

// ---- stage 4: per-particle exclusive prefixes P_0, P_1 (128-bit) -----------
// and the draw guides
__global__ __launch_bounds__(kThreads) void k_sp2_prefix(Dev d)
{
    if (ann_skipped(d)) return;
    // Lanes take consecutive particles (coalesced): particle j * kThreads +
    // tid of the tile.  One class at a time: each of the kPPT rows is scanned
    // within the wavefront (shuffles of the 64-bit halves with carry); the
    // (row, wavefront) totals are then scanned in that order by one
    // wavefront.  A class without draws is skipped (nothing reads its prefix).
    constexpr int kW = kThreads / 64;
    __shared__ uint64_t s_lo[kPPT * kW], s_hi[kPPT * kW];
    const int B = d.B;
    const int64_t *plan = d.tileA;
    const int64_t ntiles = plan[B];
    const int64_t C = d.cap_total;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int b = segment_of(plan, B, t);
        const InstParam &P = d.ip[b];
        const int64_t n = d.N[b];
        const int64_t li0 = (t - plan[b]) * kTileA + tid;
        const int64_t *st = d.bcls_stat + (int64_t)b * 8;
        uint64_t r[kPPT];
        int8_t cl[kPPT];
#pragma unroll
        for (int j = 0; j < kPPT; ++j) {
            const int64_t li = li0 + (int64_t)j * kThreads;
            const int64_t i = P.base + (li < n ? li : 0);
            r[j] = d.bA[i];                   // the residual r_i since stage 3
            cl[j] = li < n ? d.bcls[i] : (int8_t)-1;
        }
        for (int c = 0; c < 2; ++c) {
            const int64_t Nr = st[kBNr0 + c];
            __syncthreads();                  // s_lo, s_hi free again
            if (Nr <= 0) continue;
            const u128 tb = ld128(d.bTile + 2 * ((int64_t)c * d.tstride + t));
            uint64_t elo[kPPT], ehi[kPPT];    // exclusive within (row, wavefront)
#pragma unroll
            for (int j = 0; j < kPPT; ++j) {
                const uint64_t v = cl[j] == c ? r[j] : 0ull;
                uint64_t lo = v, hi = 0;
#pragma unroll
                for (int o = 1; o < 64; o <<= 1) {
                    const uint64_t plo = __shfl_up(lo, o, 64), phi = __shfl_up(hi, o, 64);
                    if (lane >= o) {
                        const uint64_t nlo = lo + plo;
                        hi = hi + phi + (nlo < lo ? 1ull : 0ull);
                        lo = nlo;
                    }
                }
                if (lane == 63) { s_lo[j * kW + wv] = lo; s_hi[j * kW + wv] = hi; }
                elo[j] = lo - v;
                ehi[j] = hi - (lo < v ? 1ull : 0ull);
            }
            __syncthreads();
            if (wv == 0) {   // exclusive scan of the kPPT * kW totals, in place
                const uint64_t v0 = lane < kPPT * kW ? s_lo[lane] : 0ull;
                const uint64_t v1 = lane < kPPT * kW ? s_hi[lane] : 0ull;
                uint64_t lo = v0, hi = v1;
#pragma unroll
                for (int o = 1; o < 64; o <<= 1) {
                    const uint64_t plo = __shfl_up(lo, o, 64), phi = __shfl_up(hi, o, 64);
                    if (lane >= o) {
                        const uint64_t nlo = lo + plo;
                        hi = hi + phi + (nlo < lo ? 1ull : 0ull);
                        lo = nlo;
                    }
                }
                const uint64_t xlo = lo - v0, xhi = hi - v1 - (lo < v0 ? 1ull : 0ull);
                if (lane < kPPT * kW) { s_lo[lane] = xlo; s_hi[lane] = xhi; }
            }
            __syncthreads();
            const int gb = sp2_guide_bits(Nr);
            const u128 R = (u128)(uint64_t)st[kBS0 + c] * (u128)(uint64_t)Nr;
            int32_t *G = d.bG + 4 * ((int64_t)c * C + P.base);
            uint64_t *Pc = d.bP + 2 * (int64_t)c * C;
#pragma unroll
            for (int j = 0; j < kPPT; ++j) {
                const int64_t li = li0 + (int64_t)j * kThreads;
                if (li >= n) continue;
                const int64_t i = P.base + li;
                const u128 pc = tb + (((u128)s_hi[j * kW + wv] << 64) | s_lo[j * kW + wv]) +
                                (((u128)ehi[j] << 64) | elo[j]);
                st128_nt(Pc + 2 * i, pc);
                if (cl[j] == c && r[j] != 0ull) {
                    const u128 end = (pc + (u128)r[j]) << gb;
                    for (uint32_t k = sp2_guide_first(pc, gb, R); k < (1u << gb) && mul32_128(k, R) < end; ++k)
                        G[k] = (int32_t)li;
                }
                if (li == n - 1) G[1u << gb] = (int32_t)li;
            }
        }
    }
}

// ---- stage 5: the N_r i.i.d. draws of each class (Alg. 2 step 2) ------------
// One draw per thread at a time: the searches are short (the guide leaves
// about n / N_r particles), and more searches in flight per thread measured
// slower.
__global__ __launch_bounds__(kThreads) void k_sp2_draw(Dev d)
{
    if (ann_skipped(d)) return;
    Ctl *ctl = d.ctl;
    const int B = d.B;
    const uint32_t step = ctl->step;
    const int64_t n0 = d.tileD[B], ntiles = n0 + d.tileD[2 * B + 1];
    const int64_t C = d.cap_total;
    const int tid = threadIdx.x;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int c = t < n0 ? 0 : 1;
        const int64_t *plan = d.tileD + (int64_t)c * (B + 1);
        const int64_t tc = t - (c ? n0 : 0);
        const int b = segment_of(plan, B, tc);
        const InstParam &P = d.ip[b];
        const int64_t *st = d.bcls_stat + (int64_t)b * 8;
        const int64_t Nr = st[kBNr0 + c];
        const u128 R = (u128)(uint64_t)st[kBS0 + c] * (u128)(uint64_t)Nr;
        const uint64_t *Pc = d.bP + 2 * (int64_t)c * C + 2 * P.base;
        const int32_t *G = d.bG + 4 * ((int64_t)c * C + P.base);
        const int gb = sp2_guide_bits(Nr);
        for (int j = 0; j < kTileR / kThreads; ++j) {
            const int64_t dd = (tc - plan[b]) * kTileR + (int64_t)j * kThreads + tid;
            if (dd >= Nr) break;
            const W4 w = draw((uint64_t)dd, step, kTagBoot, 0u, (uint32_t)c, d.seed, P.key);
            const uint64_t bits = ((uint64_t)w.b << 32) | (uint64_t)w.a;
            const u128 U = scale64(bits, R);
            const uint64_t k = gb ? bits >> (64 - gb) : 0ull;
            int32_t lo = G[k], hi = G[k + 1];
            while (lo < hi) {
                const int32_t mid = lo + ((hi - lo + 1) >> 1);
                if (ld128(Pc + 2 * (int64_t)mid) <= U) lo = mid; else hi = mid - 1;
            }
            atomicAdd(&d.bcopies[P.base + lo], 1);
        }
    }
}

// ---- stage 6: filtered counts per cell and class ---------------------------
// Copies are summed per (cell, class) in an LDS hash table per block (open
// addressing, 8 probes), over a contiguous run of tiles, and added to the
// count grids when the block moves to another instance, when the table is
// half full, and at the end: the ensemble's regenerated part puts thousands
// of particles in each cell, whose device-wide atomics would serialise.  An
// update whose probes all fail adds directly.
__global__ __launch_bounds__(kThreads) void k_sp2_cells(Dev d)
{
    if (ann_skipped(d)) return;
    constexpr int kSlots = 4096;
    __shared__ int32_t s_key[kSlots];
    __shared__ int32_t s_val[kSlots];
    __shared__ uint32_t s_nkeys;
    const int B = d.B;
    const int64_t *plan = d.tileA;
    const int64_t ntiles = plan[B];
    const int tid = threadIdx.x;
    const int64_t plane = (int64_t)B * d.Nh;
    // this block's XCD copy of the two class grids (blocks are dealt to the
    // XCDs round robin; any other placement is still correct)
    const int xc = (int)(blockIdx.x % kXcd);
    int32_t *const tg = (d.cntx == nullptr || xc == 0) ? d.ntil : d.cntx + (int64_t)(xc - 1) * 2 * plane;
    for (int j = tid; j < kSlots; j += kThreads) { s_key[j] = -1; s_val[j] = 0; }
    if (tid == 0) s_nkeys = 0;
    // key = 2 cell + class (N_h < 2^30)
    auto flush = [&](int fb) {
        for (int j = tid; j < kSlots; j += kThreads) {
            const int k = s_key[j];
            if (k < 0) continue;
            const int v = s_val[j];
            if (v != 0) atomicAdd(&tg[(int64_t)(k & 1) * plane + (int64_t)fb * d.Nh + (k >> 1)], v);
            s_key[j] = -1;
            s_val[j] = 0;
        }
        if (tid == 0) s_nkeys = 0;
        __syncthreads();
    };
    // an equal share of the binning cost (see kBinLateCost) per block
    const int64_t W = bin_cost_before(d, plan, B);
    const int64_t t0 = tile_at_cost(d, plan, (W * blockIdx.x + gridDim.x - 1) / gridDim.x);
    const int64_t t1 = tile_at_cost(d, plan, (W * (blockIdx.x + 1) + gridDim.x - 1) / gridDim.x);
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
        const int64_t n = d.N[b];
        const int64_t li0 = (t - plan[b]) * kTileA + tid;
        int8_t cl[kPPT];
        int32_t cp[kPPT];
        int64_t cell[kPPT];
#pragma unroll
        for (int j = 0; j < kPPT; ++j) {      // loads first
            const int64_t li = li0 + (int64_t)j * kThreads;
            const int64_t i = P.base + (li < n ? li : 0);
            cl[j] = li < n ? d.bcls[i] : (int8_t)-1;
            cp[j] = d.bcopies[i];
            cell[j] = d.bcell[i];
        }
#pragma unroll
        for (int j = 0; j < kPPT; ++j) {
            if (cl[j] < 0 || cp[j] == 0) continue;
            const int key = (int)(cell[j] << 1) | (int)cl[j];
            const uint32_t h = ((uint32_t)key * 2654435761u) >> 20;
            bool done = false;
            for (int pr = 0; pr < 8 && !done; ++pr) {
                const int slot = (int)((h + (uint32_t)pr) & (uint32_t)(kSlots - 1));
                int k = __hip_atomic_load(&s_key[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                if (k == -1) {
                    k = atomicCAS(&s_key[slot], -1, key);
                    if (k == -1) atomicAdd(&s_nkeys, 1u);
                }
                if (k == -1 || k == key) {
                    atomicAdd(&s_val[slot], cp[j]);
                    done = true;
                }
            }
            if (!done) atomicAdd(&tg[(int64_t)cl[j] * plane + (int64_t)b * d.Nh + cell[j]], cp[j]);
        }
    }
    __syncthreads();
    if (cb >= 0) flush(cb);
}

// ---- stage 7: exact rational cell values and the rounding step -------------
__global__ __launch_bounds__(kThreads) void k_sp2_round(Dev d)
{
    if (ann_skipped(d)) return;
    Ctl *ctl = d.ctl;
    const int B = d.B;
    const uint32_t step = ctl->step;
    const int64_t plane = (int64_t)B * d.Nh;
    for (int64_t g = (int64_t)blockIdx.x * kThreads + threadIdx.x; g < plane;
         g += (int64_t)gridDim.x * kThreads) {
        const int64_t b = g / d.Nh, nu = g - b * d.Nh;
        int32_t n0 = d.ntil[g], n1 = d.ntil[plane + g];
        if (d.cntx) {   // fold the XCD copies of the class counts and clear them
            int32_t p0[kXcd - 1], p1[kXcd - 1];
#pragma unroll
            for (int x = 0; x < kXcd - 1; ++x) {
                p0[x] = d.cntx[(int64_t)x * 2 * plane + g];
                p1[x] = d.cntx[(int64_t)x * 2 * plane + plane + g];
            }
#pragma unroll
            for (int x = 0; x < kXcd - 1; ++x) {
                n0 += p0[x];
                n1 += p1[x];
                if (p0[x]) d.cntx[(int64_t)x * 2 * plane + g] = 0;
                if (p1[x]) d.cntx[(int64_t)x * 2 * plane + plane + g] = 0;
            }
        }
        if (n0 == 0 && n1 == 0) continue;
        d.ntil[g] = 0;
        d.ntil[plane + g] = 0;
        const int64_t *st = d.bcls_stat + b * 8;
        const uint64_t N0 = (uint64_t)st[kBN0], N1 = (uint64_t)st[kBN1];
        const uint64_t S0 = (uint64_t)st[kBS0], S1 = (uint64_t)st[kBS1];
        i128 num;
        u128 den;
        if (N0 > 0 && N1 > 0) {
            num = (i128)((u128)S0 * (u128)(uint64_t)n0 * (u128)N1) -
                  (i128)((u128)S1 * (u128)(uint64_t)n1 * (u128)N0);
            den = ((u128)N0 * (u128)N1) << 32;
        } else if (N0 > 0) {
            num = (i128)((u128)S0 * (u128)(uint64_t)n0);
            den = (u128)N0 << 32;
        } else {
            num = -(i128)((u128)S1 * (u128)(uint64_t)n1);
            den = (u128)N1 << 32;
        }
        if (num == 0) continue;
        const u128 an = num < 0 ? (u128)(-num) : (u128)num;
        const u128 q = an / den;
        const u128 rem = an - q * den;
        const W4 w = draw((uint64_t)nu, step, kTagRound, 0u, 0u, d.seed, d.ip[b].key);
        const uint64_t bits = ((uint64_t)w.b << 32) | (uint64_t)w.a;
        const u128 U = scale64(bits, den);
        const int64_t m = (int64_t)q + (U < rem ? 1 : 0);
        d.cnt[g] = (int32_t)(num < 0 ? -m : m);
    }
}

// the last bootstrap's class sizes and sums into the tallies; clear the stats
__global__ __launch_bounds__(kThreads) void k_sp2_close(Dev d)
{
    if (ann_skipped(d)) return;
    for (int b = blockIdx.x * kThreads + threadIdx.x; b < d.B; b += gridDim.x * kThreads) {
        int64_t *st = d.bcls_stat + (int64_t)b * 8;
        int64_t *T = d.tally + (int64_t)b * kTalCount;
        T[kTalNplus] = st[kBN0];
        T[kTalNminus] = st[kBN1];
        T[kTalSplus] = st[kBS0];
        T[kTalSminus] = st[kBS1];
        for (int q = 0; q < 8; ++q) st[q] = 0;
    }
}

template <int DIM>
int enqueue_sp2_bootstrap(const Dev &d, hipStream_t s, int grid, int grid_scan, int grid_draw)
{
    hipLaunchKernelGGL(k_sp2_classify<DIM>, dim3(grid), dim3(kThreads), 0, s, d);
    hipLaunchKernelGGL(k_sp2_close_classify, dim3(1), dim3(kThreads), 0, s, d, grid);
    hipLaunchKernelGGL(k_sp2_resid, dim3(grid), dim3(kThreads), 0, s, d);
    hipLaunchKernelGGL(k_sp2_tilescan, dim3(std::min(d.B, grid_scan)), dim3(kThreads), 0, s, d, grid);
    hipLaunchKernelGGL(k_close_sp2_tilescan, dim3(1), dim3(kThreads), 0, s, d);
    hipLaunchKernelGGL(k_sp2_prefix, dim3(grid), dim3(kThreads), 0, s, d);
    hipLaunchKernelGGL(k_sp2_draw, dim3(grid_draw), dim3(kThreads), 0, s, d);
    hipLaunchKernelGGL(k_sp2_cells, dim3(grid), dim3(kThreads), 0, s, d);
    hipLaunchKernelGGL(k_sp2_round, dim3(grid), dim3(kThreads), 0, s, d);
    hipLaunchKernelGGL(k_sp2_close, dim3(1), dim3(kThreads), 0, s, d);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

// ---------------------------------------------------------------------------
// Tangent ghosts: one per cell that was occupied but nets to zero, carrying the
// cell's tangent sum T_nu; positions uniform in the cell (draw tag ghost, id
// (1 << 62) | (nu << 32)); ascending cell order.  Also clears the count,
// occupancy and tangent grids.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_ghosts(Dev d)
{
    __shared__ int64_t s_t;
    __shared__ uint32_t s_wsum[4];
    __shared__ uint32_t s_excl;
    Ctl *ctl = d.ctl;
    const uint32_t epoch = ctl->ann_seq;      // already advanced by the regeneration
    const uint32_t step = ctl->step;
    const int B = d.B;
    const int64_t tiles_per = (d.Nh + kTileS - 1) / kTileS;
    const int64_t ntiles = tiles_per * B;
    const Ens G = pick_set(d, 1, ctl->gcur ^ 1u);
    const int64_t nc = d.Nh * (int64_t)B;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    for (;;) {
        if (tid == 0) s_t = next_tile(&ctl->ticket[kPassGhost], ntiles);
        __syncthreads();
        const int64_t t = s_t;
        if (t >= ntiles) break;
        const int b = (int)(t / tiles_per);
        const int64_t tl = t - (int64_t)b * tiles_per;
        const int64_t cbase = (int64_t)b * d.Nh;
        const InstParam &P = d.ip[b];
        const int64_t c0 = tl * kTileS + (int64_t)tid * kPPT;
        uint32_t flags = 0, sum = 0;
        for (int j = 0; j < kPPT; ++j) {
            const int64_t c = c0 + j;
            if (c < d.Nh && d.cnt[cbase + c] == 0 && d.occ[cbase + c] > 0) { flags |= 1u << j; sum++; }
        }
        uint32_t incl = sum;
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(incl, o, 64);
            if (lane >= o) incl += y;
        }
        if (lane == 63) s_wsum[wv] = incl;
        __syncthreads();
        uint32_t woff = 0, agg = 0;
        for (int q = 0; q < 4; ++q) { if (q < wv) woff += s_wsum[q]; agg += s_wsum[q]; }
        if (wv == 0) {
            const uint32_t excl = tile_prefix(d.stG, t, (int64_t)b * tiles_per, epoch, agg);
            if (lane == 0) {
                if (tl == tiles_per - 1) d.NGnew[b] = (int64_t)(excl + agg);
                s_excl = excl;
            }
        }
        __syncthreads();
        int64_t gi = (int64_t)s_excl + (int64_t)(woff + incl - sum);
        for (int j = 0; j < kPPT; ++j) {
            const int64_t c = c0 + j;
            if (c >= d.Nh) break;
            if ((flags >> j) & 1u) {
                if (gi < P.gcap) {
                    const int64_t o = P.gbase + gi;
                    const uint64_t id = (1ull << 62) | ((uint64_t)c << 32);
                    double x[2], k[2];
                    cell_point<1>(d, c, id, kTagGhost, step, P.key, x, k);
                    G.x0[o] = x[0];
                    G.k0[o] = k[0];
                    G.sg[o] = 0;
                    G.id[o] = id;
#pragma unroll
                    for (int q = 0; q < 3; ++q)
                        G.D[q * d.gcap_total + o] = fx_value(d.Tq[(2 * q) * nc + cbase + c],
                                                             (uint64_t)d.Tq[(2 * q + 1) * nc + cbase + c]);
                }
                gi++;
            }
            d.cnt[cbase + c] = 0;
            d.occ[cbase + c] = 0;
#pragma unroll
            for (int q = 0; q < 6; ++q) d.Tq[q * nc + cbase + c] = 0;
        }
        __syncthreads();
    }
}

// After k_ghosts (one block): ghost counts with the capacity clamp, their tile
// plan, and the ghost buffer flip.
__global__ __launch_bounds__(kThreads) void k_close_ghosts(Dev d)
{
    Ctl *ctl = d.ctl;
    const int B = d.B;
    for (int b = threadIdx.x; b < B; b += kThreads) {
        int64_t n = d.NGnew[b];
        if (n > d.ip[b].gcap) { atomicOr(&ctl->err, kErrCapacity); n = d.ip[b].gcap; }
        d.NG[b] = n;
    }
    __syncthreads();
    block_plan(d.tileA + (B + 1), d.NG, B, kTileA);
    if (threadIdx.x == 0) ctl->gcur ^= 1u;
}

}  // namespace wbrw
