// One time step of the Wigner branching random walk (Alg. 1, Sec. 2),
// pass 1: k_stream (HBM-bound).  Every particle draws its first
// life-length (exact for a constant gamma0, Sec. 3.2.1) and, unless that jump
// falls inside the step, moves freely to the end of the step (a particle
// keeps its k after a jump: offspring 2M+1 of Alg. 1, so its end position
// does not depend on its jumps).  Only the first of the two uniforms decides,
// and only a 1e-9-wide band around the threshold evaluates the logarithm.
// The event flags of each tile are kept as wavefront ballots; the ordered
// event list is built from them by the passes in wbrw_step.hpp.
#pragma once
#include "wbrw_dev.hpp"
#include "wbrw_math.hpp"

namespace wbrw {

// ---------------------------------------------------------------------------
// Pass 1: streaming clock test + free flight; the event flags of every tile
// are kept as wavefront ballots, and the tile's event count is stored and
// added to the sum of its group of kSupGroup tiles.  No tile waits for
// another: tiles are assigned statically, and k_events builds the ordered
// event list from the ballots.  Each block also counts its events per
// instance: added to the instance's count when the block moves on to
// another instance, left in the block's slot of spart at the end.
//
// NT threads per block, PPT particles per thread, NT * PPT = kTileA: thread
// tid takes tile particles j * NT + tid, so ballot q = j * (NT / 64) + w of
// wavefront w covers the tile's particles [64 q, 64 q + 64) whatever the
// shape, and the event list does not depend on it (the autotuner picks it).
// ---------------------------------------------------------------------------
// register budget: as for three 256-thread blocks per CU (the loads of 16
// particles per thread need it at 128 threads)
template <int NT>
constexpr int stream_min_blocks = NT >= 512 ? 1 : 3;

template <int DIM, int NT = kThreads, int PPT = kPPT>
__global__ __launch_bounds__(NT, stream_min_blocks<NT>) void k_stream(Dev d, int ghost)
{
    static_assert(NT * PPT == kTileA, "a streaming tile is kTileA particles");
    static_assert(NT % 64 == 0, "whole wavefronts");
    constexpr int kW = NT / 64;
    __shared__ uint32_t s_wcnt[kW];
    const Ctl *ctl = d.ctl;
    const uint32_t step = ctl->step;
    const int B = d.B;
    const int64_t *plan = d.tileA + (int64_t)ghost * (B + 1);
    const int64_t ntiles = plan[B];
    const int64_t *Ncur = ghost ? d.NG : d.N;
    const Ens E = pick_set(d, ghost, ghost ? ctl->gcur : ctl->cur);
    uint64_t *tcnt = ghost ? d.tcAg : d.tcA;
    uint64_t *tsup = ghost ? d.supAg : d.supA;
    int64_t *evc = d.evc + (int64_t)ghost * B;
    uint64_t *emask = ghost ? d.emAg : d.emA;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    int cb = -1;        // instance of the block's event count acc (thread 0)
    uint64_t acc = 0;

    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int b = segment_of(plan, B, t);
        const int64_t tl = t - plan[b];
        const InstParam &P = d.ip[b];
        const int64_t base = ghost ? P.gbase : P.base;
        const int64_t n = Ncur[b];
        const double thr_lo = P.thr_lo, thr_hi = P.thr_hi, g0 = P.gamma0;
        const uint32_t key = P.key;

        // All loads of the thread's PPT particles are issued before any
        // compute or store, so every wave keeps 3*PPT (4D: 5*PPT) loads in
        // flight; full tiles need no bounds checks.
        const int64_t li0 = tl * kTileA + tid;
        const bool full = (tl + 1) * kTileA <= n;
        double xs0[PPT], xs1[PPT], kv0[PPT], kv1[PPT];
        uint64_t idv[PPT];
        if (full) {
#pragma unroll
            for (int j = 0; j < PPT; ++j) {
                const int64_t i = base + li0 + (int64_t)j * NT;
                xs0[j] = E.x0[i];
                kv0[j] = E.k0[i];
                idv[j] = E.id[i];
                if (DIM == 2) { xs1[j] = E.x1[i]; kv1[j] = E.k1[i]; }
            }
        } else {
#pragma unroll
            for (int j = 0; j < PPT; ++j) {
                const int64_t li = li0 + (int64_t)j * NT;
                const int64_t i = base + (li < n ? li : 0);
                xs0[j] = E.x0[i];
                kv0[j] = E.k0[i];
                idv[j] = E.id[i];
                if (DIM == 2) { xs1[j] = E.x1[i]; kv1[j] = E.k1[i]; }
            }
        }
        uint32_t evbits = 0, nev = 0;
        uint64_t *em = emask + t * (kTileA / 64);
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            const bool valid = full || (li0 + (int64_t)j * NT < n);
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
            if (lane == 0) em[j * kW + wv] = m;
            nev += (uint32_t)__popcll(m);
            evbits |= (ev ? 1u : 0u) << j;
        }
        // free flight to the end of the step; an event parent keeps its
        // start position, which its family walk needs, and k_family moves it.
        // Its start position is written back too, so that every line is
        // written whole (no byte-masked partial writes).  The positions are
        // not read again in this launch: non-temporal stores keep them from
        // displacing cached lines.
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            const int64_t li = li0 + (int64_t)j * NT;
            if (full || li < n) {
                const int64_t i = base + li;
                const bool evj = (evbits >> j) & 1u;
                __builtin_nontemporal_store(evj ? xs0[j] : xs0[j] + (d.vfac * kv0[j]) * d.dt, &E.x0[i]);
                if (DIM == 2) __builtin_nontemporal_store(evj ? xs1[j] : xs1[j] + (d.vfac * kv1[j]) * d.dt, &E.x1[i]);
            }
        }
        if (lane == 0) s_wcnt[wv] = nev;
        __syncthreads();
        if (tid == 0) {
            uint64_t c = 0;
#pragma unroll
            for (int w = 0; w < kW; ++w) c += s_wcnt[w];
            tcnt[t] = c;
            if (c) atomicAdd((unsigned long long *)&tsup[(t / kSupGroup) * kSupStride], (unsigned long long)c);
            if (b != cb) {
                if (cb >= 0 && acc) atomicAdd((unsigned long long *)&evc[cb], (unsigned long long)acc);
                cb = b;
                acc = 0;
            }
            acc += c;
        }
        __syncthreads();
    }
    if (tid == 0) {
        d.spart[2 * (int64_t)blockIdx.x] = cb;
        d.spart[2 * (int64_t)blockIdx.x + 1] = (int64_t)acc;
    }
}

}  // namespace wbrw
