// Host runtime and C ABI of the WBRW library (declared in include/wbrw.h).
//
// The runtime validates the configuration, lays one caller-owned device
// workspace out into the arrays described in wbrw_dev.hpp, derives the
// per-instance constants of the jump process, and enqueues kernels.  It never
// allocates device memory and never synchronises except where the ABI says so.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/wbrw.h"
#include "wbrw_cells.hpp"
#include "wbrw_dev.hpp"
#include "wbrw_math.hpp"
#include "wbrw_sp2.hpp"
#include "wbrw_step.hpp"

using namespace wbrw;

namespace {

constexpr size_t kAlign = 256;

struct Layout {
    size_t total = 0;
    size_t zero_begin = 0, zero_end = 0;   // region cleared at init
    // offsets
    size_t ens[2][8] = {}, gens[2][8] = {};
    size_t ip = 0, tab[kMaxM] = {}, guide[kMaxM] = {}, ctl = 0;
    size_t N = 0, NG = 0, Nnew = 0, NGnew = 0, Nbase = 0, evc = 0, tileA = 0, Nsrt = 0, srtS = 0, tileB = 0, tileR = 0,
           tileG = 0, tally = 0, fpart = 0, rstart = 0, rtiles = 0, ev_idx = 0, gev_idx = 0,
           tcA = 0, tcAg = 0, supA = 0, supAg = 0, spart = 0, emA = 0, emAg = 0, tcB = 0, tcBg = 0, supB = 0, supBg = 0, tsB = 0, tsBg = 0, stg = 0, stS = 0, stG = 0, cnt = 0, cntx = 0, occx = 0, Tqx = 0, off = 0,
           occ = 0, Tq = 0, ntil = 0, dacc = 0, dTq = 0, bA = 0, bcopies = 0, bcls = 0,
           bcell = 0, bP = 0, bTile = 0, bG = 0, bcls_stat = 0, tileD = 0, bscan_tiles = 0, hist = 0, xitab = 0,
           gpool = 0;
    int64_t cap_total = 0, gcap_total = 0, Nh = 0;
    int64_t tilesA = 0, tilesAg = 0, tilesB = 0, tilesBg = 0, tilesS = 0, tilesP = 0;
};

size_t take(size_t &cursor, size_t bytes)
{
    cursor = (cursor + kAlign - 1) / kAlign * kAlign;
    const size_t at = cursor;
    cursor += bytes;
    return at;
}

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// buckets of a table's guide: the least power of two >= n
int32_t guide_buckets(int32_t n)
{
    int32_t k = 1;
    while (k < n) k <<= 1;
    return k;
}

// guide[i] = the last j < n with cum[j] <= t_i, t_i = (i / kg) cum[n] rounded
// as the sampler rounds u1 cum[n] (kg a power of two, so i / kg is exact and
// u1 >= i / kg gives u1 cum[n] >= t_i); cum is non-decreasing
void build_guide(const std::vector<double> &cum, int32_t n, int32_t kg, std::vector<int32_t> &guide)
{
    guide.assign((size_t)kg + 1, 0);
    int32_t j = 0;
    for (int32_t i = 0; i <= kg; ++i) {
        const double t = ((double)i / (double)kg) * cum[n];
        while (j + 1 < n && cum[j + 1] <= t) ++j;
        guide[i] = j;
    }
}

int validate(const wbrw_config *c)
{
    if (!c) return WBRW_EINVAL;
    if (c->dim != 1 && c->dim != 2) return WBRW_EINVAL;
    if (c->strategy != WBRW_SP1 && c->strategy != WBRW_SP2) return WBRW_EINVAL;
    if (c->n_components < 1 || c->n_components > WBRW_MAX_COMPONENTS) return WBRW_EINVAL;
    if (c->n_instances < 1 || c->n_instances > 65536) return WBRW_EINVAL;
    if (!c->N0 || !c->capacity) return WBRW_EINVAL;
    if (!(c->hbar > 0) || !(c->mass > 0) || !(c->dt > 0)) return WBRW_EINVAL;
    if (!(c->x_hi > c->x_lo) || !(c->k_hi > c->k_lo) || c->nx < 1 || c->nk < 1) return WBRW_EINVAL;
    if (c->max_density_bins < 1) return WBRW_EINVAL;
    if (c->track_tangent < 0 || c->track_tangent > 2) return WBRW_EINVAL;
    if (c->track_tangent) {
        // sp2's x0 tangent is pathwise and bounded: derivative pairs are sp1's
        if ((c->strategy == WBRW_SP2 && c->track_tangent != 1) || c->dim != 1 || c->n_components != 1 ||
            c->comp[0].kind != WBRW_KERNEL_GAUSSIAN || c->ghost_capacity < 1 || c->comp[0].modulated)
            return WBRW_EINVAL;
    }
    for (int m = 0; m < c->n_components; ++m) {
        const wbrw_component &q = c->comp[m];
        if (q.sampler != 0 && (q.sampler != 1 || q.kind != WBRW_KERNEL_GAUSSIAN ||
                               c->strategy != WBRW_SP1 || q.modulated || c->track_tangent))
            return WBRW_EINVAL;
        if (!q.modulated) continue;
        if (q.kind != WBRW_KERNEL_GAUSSIAN || !std::isfinite(q.mod_a) || !std::isfinite(q.mod_b) ||
            !std::isfinite(q.mod_omega) || !std::isfinite(q.mod_phase))
            return WBRW_EINVAL;
        // a given gamma0 must keep the pair probability <= 1 at every time
        if (c->gamma0 > 0 && q.H)
            for (int b = 0; b < c->n_instances; ++b)
                if ((2.0 * (std::fabs(q.H[b]) * (std::fabs(q.mod_a) + std::fabs(q.mod_b)))) / c->hbar >
                    2.0 * c->gamma0 * (1.0 + 1e-12))
                    return WBRW_EINVAL;
    }
    if (!(c->gamma0 > 0) && !(c->gamma_scale > 0)) return WBRW_EINVAL;
    for (int m = 0; m < c->n_components; ++m) {
        const wbrw_component &q = c->comp[m];
        if (q.axis < 0 || q.axis > 2 || (c->dim == 1 && q.axis != 0)) return WBRW_EINVAL;
        if (q.kind == WBRW_KERNEL_GAUSSIAN) {
            if (!q.H || !q.width || !q.center_b) return WBRW_EINVAL;
            for (int b = 0; b < c->n_instances; ++b)
                if (!(q.width[b] > 0) || q.H[b] == 0.0 || !std::isfinite(q.H[b])) return WBRW_EINVAL;
        } else if (q.kind == WBRW_KERNEL_TABLE) {
            if (!q.table || q.table_n < 1 || q.table_n > 65536 || !(q.q_hi > q.q_lo)) return WBRW_EINVAL;
            if (q.sign != 1.0 && q.sign != -1.0) return WBRW_EINVAL;
            double s = 0;
            for (int j = 0; j < q.table_n; ++j) {
                if (!(q.table[j] >= 0)) return WBRW_EINVAL;
                s += q.table[j];
            }
            if (!(s > 0)) return WBRW_EINVAL;
        } else {
            return WBRW_EINVAL;
        }
    }
    for (int b = 0; b < c->n_instances; ++b) {
        if (c->N0[b] < 0 || c->capacity[b] < c->N0[b] || c->capacity[b] >= (1ll << 31)) return WBRW_EINVAL;
    }
    // The pair probability xi_m |sin| / (2 gamma0) of the sp1 box (and the wp
    // weight factor) must stay <= 1 (Remark 3: gamma0 >= xi_m / 2).  The
    // normalisers and gamma0 are computed exactly as derive() does.
    {
        double xi_t[kMaxM] = {};
        for (int m = 0; m < c->n_components; ++m) {
            const wbrw_component &q = c->comp[m];
            if (q.kind != WBRW_KERNEL_TABLE) continue;
            double cum = 0.0;
            for (int j = 0; j < q.table_n; ++j) cum = cum + q.table[j];
            const double dq = (q.q_hi - q.q_lo) / (double)q.table_n;
            xi_t[m] = ((2.0 * cum) * dq) / (0x1.921fb54442d18p+1 * c->hbar);
        }
        for (int b = 0; b < c->n_instances; ++b) {
            double g = 0.0, xi[kMaxM] = {};
            for (int m = 0; m < c->n_components; ++m) {
                const wbrw_component &q = c->comp[m];
                if (q.kind == WBRW_KERNEL_GAUSSIAN) {
                    xi[m] = (2.0 * std::fabs(q.H[b])) / c->hbar;
                    if (q.modulated) {
                        const double xmax = (2.0 * (std::fabs(q.H[b]) * (std::fabs(q.mod_a) + std::fabs(q.mod_b)))) / c->hbar;
                        if (xmax > g) g = xmax;
                    }
                } else {
                    xi[m] = xi_t[m];
                }
                if (xi[m] > g) g = xi[m];
            }
            const double g0 = (c->gamma0 > 0.0) ? c->gamma0 : c->gamma_scale * (g / 2.0);
            if (!(g0 > 0.0) || !std::isfinite(g0)) return WBRW_EINVAL;
            for (int m = 0; m < c->n_components; ++m)
                if (!(xi[m] / (2.0 * g0) <= 1.0)) return WBRW_EINVAL;
        }
    }
    const int64_t nh = c->dim == 1 ? (int64_t)c->nx * c->nk
                                   : (int64_t)c->nx * c->nx * (int64_t)c->nk * c->nk;
    if (nh >= (1ll << 31)) return WBRW_EINVAL;
    if (c->strategy == WBRW_SP2 && nh >= (1ll << 30)) return WBRW_EINVAL;   // (cell, class) keys
    return WBRW_OK;
}

// Plain sp1 binning (and the sp2 bootstrap's per-class counting) adds its
// counts into one grid per XCD, so that the atomics of an XCD's blocks stay
// in that XCD's L2; the scan (sp2: the rounding pass) folds the copies
// together.  Worth it while the extra grids (read once per annihilation) are
// small beside the ensemble that is binned.
bool xcd_counts(const wbrw_config *c)
{
    const int64_t nh = c->dim == 1 ? (int64_t)c->nx * c->nk : (int64_t)c->nx * c->nx * (int64_t)c->nk * c->nk;
    int64_t n0 = 0;
    for (int b = 0; b < c->n_instances; ++b) n0 += c->N0[b];
    return (int64_t)(kXcd - 1) * nh * c->n_instances <= n0;
}

Layout make_layout(const wbrw_config *c)
{
    Layout L;
    const int B = c->n_instances;
    const bool sp2 = c->strategy == WBRW_SP2, tan = c->track_tangent != 0;
    for (int b = 0; b < B; ++b) {
        L.cap_total += c->capacity[b];
        L.tilesA += ceil_div(c->capacity[b], kTileA) + 1;
        L.tilesB += ceil_div(c->capacity[b], kTileB) + 1;
        L.tilesP += ceil_div(c->capacity[b], kTileS) + 1;
        L.rtiles += ceil_div(c->capacity[b], kTileR) + 1;
        if (tan) {
            L.gcap_total += c->ghost_capacity;
            L.tilesAg += ceil_div(c->ghost_capacity, kTileA) + 1;
            L.tilesBg += ceil_div(c->ghost_capacity, kTileB) + 1;
        }
    }
    L.Nh = c->dim == 1 ? (int64_t)c->nx * c->nk : (int64_t)c->nx * c->nx * (int64_t)c->nk * c->nk;
    L.tilesS = ceil_div(L.Nh, kTileS) * B;
    const size_t C = (size_t)L.cap_total, G = (size_t)L.gcap_total, Nh = (size_t)L.Nh;
    const size_t BB = (size_t)B, MB = (size_t)c->max_density_bins;
    size_t cur = 0;
    for (int s = 0; s < 2; ++s) {
        L.ens[s][0] = take(cur, C * 8);
        L.ens[s][1] = c->dim == 2 ? take(cur, C * 8) : 0;
        L.ens[s][2] = take(cur, C * 8);
        L.ens[s][3] = c->dim == 2 ? take(cur, C * 8) : 0;
        L.ens[s][4] = sp2 ? 0 : take(cur, C);
        L.ens[s][5] = sp2 ? take(cur, C * 8) : 0;
        L.ens[s][6] = take(cur, C * 8);
        L.ens[s][7] = tan ? take(cur, C * 24) : 0;
        if (tan) {
            L.gens[s][0] = take(cur, G * 8);
            L.gens[s][2] = take(cur, G * 8);
            L.gens[s][4] = take(cur, G);
            L.gens[s][6] = take(cur, G * 8);
            L.gens[s][7] = take(cur, G * 24);
        }
    }
    L.ev_idx = take(cur, C * 4);
    if (tan) L.gev_idx = take(cur, G * 4);
    L.ip = take(cur, BB * sizeof(InstParam));
    for (int m = 0; m < c->n_components; ++m)
        if (c->comp[m].kind == WBRW_KERNEL_TABLE) {
            L.tab[m] = take(cur, ((size_t)c->comp[m].table_n + 1) * 8);
            L.guide[m] = take(cur, ((size_t)guide_buckets(c->comp[m].table_n) + 1) * 4);
        }
    L.off = take(cur, BB * Nh * 8);
    if (c->init_hist) L.hist = take(cur, BB * Nh * 8);
    bool alg4 = false;
    for (int m = 0; m < c->n_components; ++m) alg4 = alg4 || c->comp[m].sampler == 1;
    if (alg4) L.xitab = take(cur, BB * (size_t)c->n_components * (kXiN + 1) * 8);
    if (c->dim == 2) L.gpool = take(cur, (size_t)kGPoolBlocks * kGPoolBytes);
    if (sp2) {
        L.bA = take(cur, C * 8);
        L.bcopies = take(cur, C * 4);
        L.bcls = take(cur, C);
        L.bcell = take(cur, C * 8);
        L.bP = take(cur, 2 * C * 16);
        L.bTile = take(cur, 2 * (size_t)L.tilesP * 16);
        L.bG = take(cur, 2 * 4 * C * 4);
    }
    // everything below starts zeroed
    L.zero_begin = (cur + kAlign - 1) / kAlign * kAlign;
    L.ctl = take(cur, sizeof(Ctl));
    L.N = take(cur, BB * 8);
    L.NG = take(cur, BB * 8);
    L.Nnew = take(cur, BB * 8);
    L.NGnew = take(cur, BB * 8);
    L.Nbase = take(cur, 2 * BB * 8);
    L.evc = take(cur, 2 * BB * 8);
    L.tileA = take(cur, 2 * (BB + 1) * 8);
    L.Nsrt = take(cur, BB * 8);
    L.srtS = take(cur, (BB + 1) * 8);
    L.tileB = take(cur, 2 * (BB + 1) * 8);
    L.tileR = take(cur, (BB + 1) * 8);
    L.tileG = take(cur, (BB + 1) * 8);
    L.tally = take(cur, BB * kTalCount * 8);
    L.fpart = take(cur, (size_t)kMaxGrid * 8 * 8);
    L.rstart = take(cur, (size_t)L.rtiles * 8);
    L.tcA = take(cur, (size_t)L.tilesA * 8);
    L.supA = take(cur, (size_t)(L.tilesA / kSupGroup + 1) * kSupStride * 8);
    L.spart = take(cur, (size_t)kMaxGrid * 2 * 8);
    L.emA = take(cur, (size_t)L.tilesA * (kTileA / 64) * 8);
    L.tcB = take(cur, (size_t)L.tilesB * 8);
    L.supB = take(cur, (size_t)(L.tilesB / kSupGroup + 1) * kSupStride * 8);
    L.tsB = take(cur, (size_t)L.tilesB * 8);
    L.stg = take(cur, 2 * BB * 8);
    if (tan) {
        L.tcAg = take(cur, (size_t)L.tilesAg * 8);
        L.supAg = take(cur, (size_t)(L.tilesAg / kSupGroup + 1) * kSupStride * 8);
        L.emAg = take(cur, (size_t)L.tilesAg * (kTileA / 64) * 8);
        L.tcBg = take(cur, (size_t)L.tilesBg * 8);
        L.supBg = take(cur, (size_t)(L.tilesBg / kSupGroup + 1) * kSupStride * 8);
        L.tsBg = take(cur, (size_t)L.tilesBg * 8);
        L.stG = take(cur, (size_t)L.tilesS * 8);
    }
    L.stS = take(cur, (size_t)L.tilesS * 8);
    L.cnt = take(cur, BB * Nh * 4);
    if (xcd_counts(c)) L.cntx = take(cur, (size_t)(kXcd - 1) * (sp2 ? 2 : 1) * BB * Nh * 4);
    if (tan) {
        L.occ = take(cur, BB * Nh * 4);
        L.Tq = take(cur, 6 * BB * Nh * 8);
        if (L.cntx) {
            L.occx = take(cur, (size_t)(kXcd - 1) * BB * Nh * 4);
            L.Tqx = take(cur, (size_t)(kXcd - 1) * 6 * BB * Nh * 8);
        }
        L.dTq = take(cur, 6 * BB * MB * 8);
    }
    if (sp2) {
        L.ntil = take(cur, 2 * BB * Nh * 4);
        L.bcls_stat = take(cur, BB * 8 * 8);
        L.tileD = take(cur, 2 * (BB + 1) * 8);
        L.bscan_tiles = take(cur, (BB + 1) * 8);
    }
    L.dacc = take(cur, kXcd * BB * MB * 8);   // one accumulator per XCD
    L.zero_end = (cur + kAlign - 1) / kAlign * kAlign;
    L.total = L.zero_end;
    return L;
}

}  // namespace

// Device scratch of wbrw_density_noalloc: its per-XCD density accumulators
// (kXcd x B x nbins int64), for callers that cannot allocate.  Every GPU the
// library runs on holds one copy until the process ends; all calls on that
// GPU share it.  The host-side name is only a stand-in for the symbol: device
// code gets the address that hipGetSymbolAddress returns for each GPU.
constexpr int64_t kNoAllocWords = int64_t(1) << 19;   // 4 MiB
static __device__ __align__(256) int64_t scratch[kNoAllocWords];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
int64_t *g_scratch[kMaxDevices] = {};

// The scratch array's address on the current device, looked up once per
// device (the device must be current).
int scratch_on_current_device(int dev, int64_t **out)
{
    if (dev < 0 || dev >= kMaxDevices) return WBRW_EINVAL;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            std::fprintf(stderr, "wbrw: hipGetSymbolAddress(scratch) failed: %s\n", hipGetErrorString(e));
            return WBRW_EHIP;
        }
        g_scratch[dev] = (int64_t *)p;
    }
    *out = g_scratch[dev];
    return WBRW_OK;
}
}  // namespace

struct wbrw_handle {
    int B = 0, dim = 0, M = 0, strategy = 0, tangent = 0;
    int device = 0;
    int64_t *scratch_ptr = nullptr;   // this device's copy of `scratch`
    hipStream_t stream = nullptr;
    char *ws = nullptr;
    Layout L;
    Dev d{};
    std::vector<InstParam> ip;
    int cus = 0;
    int grid[16] = {};
    hipGraphExec_t gexec = nullptr;
    int graph_every = -1;
    hipGraphExec_t gexec_ad = nullptr;        // one step + conditional annihilation
    int ad_every = -1;
    int64_t ad_limit = -1;
    int sticky = WBRW_OK;
    int64_t host_step = 0;   // steps enqueued so far (mirror of the device counter)
    int prof = 0;   // 1: every stage and step marked; 2: whole steps only
    // launch shapes the autotuner chooses among (results do not depend on
    // them): streaming block shape (kStreamShapes), binning hash size
    int stream_shape = 0;
    int bin_slots = 4096;
    int occ_stream[3] = {};   // blocks per CU of each streaming shape (0: not built)
    int occ_bin[3] = {};      // of each binning hash size (kBinSlots)
    int occ_family = 0;
    struct Mark { int stage; hipEvent_t a, b; };
    std::vector<Mark> marks;
    int open_stage = -1;
    hipEvent_t open_ev = nullptr;
    hipEvent_t step_ev = nullptr;    // start of the step being enqueued (WBRW_STAGE_STEP)
};

namespace {

#define HIPCHK(x)                                        \
    do {                                                 \
        hipError_t e_ = (x);                             \
        if (e_ != hipSuccess) {                          \
            std::fprintf(stderr, "wbrw: %s failed: %s\n", #x, hipGetErrorString(e_)); \
            return WBRW_EHIP;                            \
        }                                                \
    } while (0)

template <typename T>
T *at(char *base, size_t off) { return reinterpret_cast<T *>(base + off); }

enum { G_STREAM = 0, G_FAMILY, G_BIN, G_SCAN, G_REGEN, G_DENS, G_SP2, G_GHOST, G_EVENTS, G_DRAW, G_DENST, G_COUNT };

template <typename K>
int blocks_per_cu(K kernel, int nt = kThreads)
{
    int per = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, nt, 0) != hipSuccess || per < 1) per = 1;
    return per;
}

template <typename K>
int persistent_blocks(K kernel, int cus, int nt = kThreads)
{
    return std::min(blocks_per_cu(kernel, nt) * cus, kMaxGrid);
}

// Streaming block shapes (threads, particles per thread; a tile is always
// kTileA particles) and binning hash sizes the autotuner chooses among.
// The 4D streaming kernel holds five values per particle, too many for 16
// particles per thread, so shape 1 is 1D only.
constexpr int kStreamShapes[3][2] = {{kThreads, kPPT}, {128, 16}, {512, 4}};
constexpr int kBinSlots[3] = {4096, 2048, 8192};

template <int DIM>
void launch_stream(const wbrw_handle *h, hipStream_t s, int ghost)
{
    const Dev &d = h->d;
    const dim3 g(h->grid[G_STREAM]);
    if constexpr (DIM == 1)
        if (h->stream_shape == 1) {
            hipLaunchKernelGGL((k_stream<DIM, 128, 16>), g, dim3(128), 0, s, d, ghost);
            return;
        }
    if (h->stream_shape == 2) {
        hipLaunchKernelGGL((k_stream<DIM, 512, 4>), g, dim3(512), 0, s, d, ghost);
        return;
    }
    hipLaunchKernelGGL((k_stream<DIM>), g, dim3(kThreads), 0, s, d, ghost);
}

template <int DIM>
void launch_bin_plain(const wbrw_handle *h, hipStream_t s)
{
    const Dev &d = h->d;
    const dim3 g(h->grid[G_BIN]);
    if (h->bin_slots == 2048)
        hipLaunchKernelGGL((k_bin<DIM, false, false, 2048>), g, dim3(kThreads), 0, s, d, 0);
    else if (h->bin_slots == 8192)
        hipLaunchKernelGGL((k_bin<DIM, false, false, 8192>), g, dim3(kThreads), 0, s, d, 0);
    else
        hipLaunchKernelGGL((k_bin<DIM, false, false>), g, dim3(kThreads), 0, s, d, 0);
}

// Alg. 4 sampler: xi(r) = (1/2) int |V_W| dq for the Gaussian barrier on
// r_j = j h, h = 8w / kXiN, by the midpoint rule over q in [-8/w, 8/w).
void xi_table(double H, double w, double hbar, double *tab, double &h_out)
{
    const double pi = 0x1.921fb54442d18p+1;
    const double h = (8.0 * w) / (double)kXiN;
    const double qlo = -8.0 / w, dq = (16.0 / w) / (double)kXiQ;
    const double pref = ((std::fabs(H) * w) * std::sqrt(2.0 * pi)) / (pi * hbar);
    for (int j = 0; j <= kXiN; ++j) {
        const double r = (double)j * h;
        double acc = 0.0;
        for (int i = 0; i < kXiQ; ++i) {
            const double q = qlo + ((double)i + 0.5) * dq;
            acc += std::exp(-2.0 * ((w * w) * (q * q))) * std::fabs(std::sin(2.0 * q * r));
        }
        tab[j] = (pref * acc) * dq;
    }
    h_out = h;
}

// derived per-instance constants (Remark 3: xi_m and the pair probability)
void derive(const wbrw_config *c, int b, const std::vector<double> &xi_tab,
            InstParam &P)
{
    std::memset(&P, 0, sizeof(P));
    double g = 0.0;
    for (int m = 0; m < c->n_components; ++m) {
        const wbrw_component &q = c->comp[m];
        double xi;
        if (q.kind == WBRW_KERNEL_GAUSSIAN) {
            P.H[m] = q.H[b];
            P.width[m] = q.width[b];
            P.center[m] = q.center_b[b];
            xi = (2.0 * std::fabs(P.H[m])) / c->hbar;   // (1/(pi hbar)) int |F[V](s)| ds = 2|H|/hbar
            P.sq[m] = 0.5 / P.width[m];
            P.sgnV[m] = P.H[m] >= 0.0 ? 1.0 : -1.0;
            P.ma[m] = q.modulated ? q.mod_a : 1.0;
            P.mb[m] = q.modulated ? q.mod_b : 0.0;
            P.mw[m] = q.modulated ? q.mod_omega : 0.0;
            P.mp[m] = q.modulated ? q.mod_phase : 0.0;
            if (q.modulated) {   // the largest xi_m over time bounds a derived gamma0
                const double xmax = (2.0 * (std::fabs(P.H[m]) * (std::fabs(q.mod_a) + std::fabs(q.mod_b)))) / c->hbar;
                if (xmax > g) g = xmax;
            }
        } else {
            xi = xi_tab[m];
            P.center[m] = q.center;
            P.sgnV[m] = q.sign;
            P.H[m] = 1.0;
            P.width[m] = 1.0;
        }
        P.c[m] = xi;   // temporarily hold xi_m
        if (xi > g) g = xi;
    }
    P.gamma0 = (c->gamma0 > 0.0) ? c->gamma0 : c->gamma_scale * (g / 2.0);
    for (int m = 0; m < c->n_components; ++m) P.c[m] = P.c[m] / (2.0 * P.gamma0);
    // probability of a first jump within dt, and a band around it outside of
    // which the comparison tau <= dt cannot be decided differently by rounding
    const long double pj = -std::expm1l(-(long double)P.gamma0 * (long double)c->dt);
    P.thr_lo = (double)(pj * (1.0L - 1e-9L));
    P.thr_hi = (double)(pj * (1.0L + 1e-9L));
    P.N0 = c->N0[b];
    P.key = (uint32_t)(c->instance_offset + b);
}

void plan_host(std::vector<int64_t> &plan, const int64_t *n, int B, int64_t tile)
{
    plan.assign(B + 1, 0);
    for (int b = 0; b < B; ++b) plan[b + 1] = plan[b] + ceil_div(n[b], tile);
}

int launch_check()
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        std::fprintf(stderr, "wbrw: kernel launch failed: %s\n", hipGetErrorString(e));
        return WBRW_EHIP;
    }
    return WBRW_OK;
}

// per-stage profiling marks (no-ops unless wbrw_profile enabled them)
void stage_begin(wbrw_t h, int stage)
{
    if (h->prof != 1) return;
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return;
    (void)hipEventRecord(e, h->stream);
    h->open_stage = stage;
    h->open_ev = e;
}

void stage_end(wbrw_t h)
{
    if (h->prof != 1 || h->open_stage < 0) return;
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return;
    (void)hipEventRecord(e, h->stream);
    h->marks.push_back({h->open_stage, h->open_ev, e});
    h->open_stage = -1;
    h->open_ev = nullptr;
}

// the outer mark of a whole step (the stage marks above nest inside it)
void step_begin(wbrw_t h)
{
    if (!h->prof) return;
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return;
    (void)hipEventRecord(e, h->stream);
    h->step_ev = e;
}

void step_end(wbrw_t h)
{
    if (!h->prof || !h->step_ev) return;
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return;
    (void)hipEventRecord(e, h->stream);
    h->marks.push_back({WBRW_STAGE_STEP, h->step_ev, e});
    h->step_ev = nullptr;
}

// Ordered scan of |n_nu| (see k_scan_sums): tile sums, their one-block scan
// with the new counts, then the offsets and regeneration-tile starts.
void enqueue_scan(int grid, hipStream_t s, const Dev &d, int zero_counts)
{
    hipLaunchKernelGGL(k_scan_sums, dim3(grid), dim3(kThreads), 0, s, d);
    hipLaunchKernelGGL(k_close_scan, dim3(1), dim3(kThreads), 0, s, d);
    hipLaunchKernelGGL(k_scan, dim3(grid), dim3(kThreads), 0, s, d, zero_counts);
}

template <int DIM>
void enqueue_step_dim(wbrw_t h)
{
    const Dev &d = h->d;
    hipStream_t s = h->stream;
    const bool tan = h->tangent != 0;
    // stage marks bracket the main kernels (the placement launch's last
    // block closes the step)
    stage_begin(h, WBRW_STAGE_STREAM);
    launch_stream<DIM>(h, s, 0);
    stage_end(h);
    stage_begin(h, WBRW_STAGE_EVENTS);
    hipLaunchKernelGGL(k_events, dim3(h->grid[G_EVENTS] + 1), dim3(kThreads), 0, s, d, 0, h->grid[G_STREAM]);
    stage_end(h);
    stage_begin(h, WBRW_STAGE_FAMILY);
    if (h->strategy == WBRW_SP2 && tan)
        hipLaunchKernelGGL((k_family<DIM, true, true>), dim3(h->grid[G_FAMILY]), dim3(kThreads), 0, s, d, 0);
    else if (h->strategy == WBRW_SP2)
        hipLaunchKernelGGL((k_family<DIM, true, false>), dim3(h->grid[G_FAMILY]), dim3(kThreads), 0, s, d, 0);
    else if (tan)
        hipLaunchKernelGGL((k_family<DIM, false, true>), dim3(h->grid[G_FAMILY]), dim3(kThreads), 0, s, d, 0);
    else
        hipLaunchKernelGGL((k_family<DIM, false, false>), dim3(h->grid[G_FAMILY]), dim3(kThreads), 0, s, d, 0);
    stage_end(h);
    stage_begin(h, WBRW_STAGE_PLACE);
    const dim3 pg(h->grid[G_EVENTS] + 1);
    const int adv = tan ? 0 : 1, fg = h->grid[G_FAMILY];
    if (h->strategy == WBRW_SP2 && tan)
        hipLaunchKernelGGL((k_place_records<DIM, true, true>), pg, dim3(kThreads), 0, s, d, 0, adv, fg);
    else if (h->strategy == WBRW_SP2)
        hipLaunchKernelGGL((k_place_records<DIM, true, false>), pg, dim3(kThreads), 0, s, d, 0, adv, fg);
    else if (tan)
        hipLaunchKernelGGL((k_place_records<DIM, false, true>), pg, dim3(kThreads), 0, s, d, 0, adv, fg);
    else
        hipLaunchKernelGGL((k_place_records<DIM, false, false>), pg, dim3(kThreads), 0, s, d, 0, adv, fg);
    stage_end(h);
    if (tan) {
        // ghosts (weight 0) branch by the sp1 rule in either strategy
        stage_begin(h, WBRW_STAGE_GHOST);
        launch_stream<DIM>(h, s, 1);
        hipLaunchKernelGGL(k_events, dim3(h->grid[G_EVENTS] + 1), dim3(kThreads), 0, s, d, 1, h->grid[G_STREAM]);
        hipLaunchKernelGGL((k_family<DIM, false, true>), dim3(h->grid[G_FAMILY]), dim3(kThreads), 0, s, d, 1);
        hipLaunchKernelGGL((k_place_records<DIM, false, true>), pg, dim3(kThreads), 0, s, d, 1, 1, fg);
        stage_end(h);
    }
}

int enqueue_step(wbrw_t h)
{
    step_begin(h);
    if (h->dim == 1) enqueue_step_dim<1>(h); else enqueue_step_dim<2>(h);
    step_end(h);
    h->host_step += 1;
    return launch_check();
}

template <int DIM>
int enqueue_annihilate_dim(wbrw_t h)
{
    const Dev &d = h->d;
    hipStream_t s = h->stream;
    if (h->strategy == WBRW_SP2) {
        const bool tan = h->tangent != 0;
        if (tan) {
            // occupancy and tangent sums per cell, particles and ghosts
            stage_begin(h, WBRW_STAGE_BIN);
            hipLaunchKernelGGL((k_bin<DIM, true, true>), dim3(h->grid[G_BIN]), dim3(kThreads), 0, s, d, 0);
            hipLaunchKernelGGL((k_bin<DIM, true, true>), dim3(h->grid[G_BIN]), dim3(kThreads), 0, s, d, 1);
            if (d.occx) hipLaunchKernelGGL(k_fold_tangents, dim3(h->grid[G_SCAN]), dim3(kThreads), 0, s, d);
            stage_end(h);
        }
        stage_begin(h, WBRW_STAGE_BOOTSTRAP);
        int rc = enqueue_sp2_bootstrap<DIM>(d, s, h->grid[G_SP2], h->grid[G_SCAN], h->grid[G_DRAW]);
        stage_end(h);
        if (rc) return rc;
        stage_begin(h, WBRW_STAGE_SCAN);
        // with tangents the counts stay for the ghost pass, which clears them
        enqueue_scan(h->grid[G_SCAN], s, d, tan ? 0 : 1);
        stage_end(h);
        stage_begin(h, WBRW_STAGE_REGEN);
        if (tan) hipLaunchKernelGGL((k_regen<DIM, true, true>), dim3(h->grid[G_REGEN]), dim3(kThreads), 0, s, d);
        else hipLaunchKernelGGL((k_regen<DIM, true, false>), dim3(h->grid[G_REGEN]), dim3(kThreads), 0, s, d);
        hipLaunchKernelGGL(k_close_regen, dim3(1), dim3(kThreads), 0, s, d);
        stage_end(h);
        if (tan) {
            stage_begin(h, WBRW_STAGE_GHOST);
            hipLaunchKernelGGL(k_ghosts, dim3(h->grid[G_GHOST]), dim3(kThreads), 0, s, d);
            hipLaunchKernelGGL(k_close_ghosts, dim3(1), dim3(kThreads), 0, s, d);
            stage_end(h);
        }
        return launch_check();
    }
    if (h->tangent) {
        stage_begin(h, WBRW_STAGE_BIN);
        hipLaunchKernelGGL((k_bin<DIM, false, true>), dim3(h->grid[G_BIN]), dim3(kThreads), 0, s, d, 0);
        hipLaunchKernelGGL((k_bin<DIM, false, true>), dim3(h->grid[G_BIN]), dim3(kThreads), 0, s, d, 1);
        if (d.occx) hipLaunchKernelGGL(k_fold_tangents, dim3(h->grid[G_SCAN]), dim3(kThreads), 0, s, d);
        stage_end(h);
        stage_begin(h, WBRW_STAGE_SCAN);
        enqueue_scan(h->grid[G_SCAN], s, d, 0);
        stage_end(h);
        stage_begin(h, WBRW_STAGE_REGEN);
        hipLaunchKernelGGL((k_regen<DIM, false, true>), dim3(h->grid[G_REGEN]), dim3(kThreads), 0, s, d);
        hipLaunchKernelGGL(k_close_regen, dim3(1), dim3(kThreads), 0, s, d);
        stage_end(h);
        stage_begin(h, WBRW_STAGE_GHOST);
        hipLaunchKernelGGL(k_ghosts, dim3(h->grid[G_GHOST]), dim3(kThreads), 0, s, d);
        hipLaunchKernelGGL(k_close_ghosts, dim3(1), dim3(kThreads), 0, s, d);
        stage_end(h);
        return launch_check();
    }
    stage_begin(h, WBRW_STAGE_BIN);
    launch_bin_plain<DIM>(h, s);
    stage_end(h);
    stage_begin(h, WBRW_STAGE_SCAN);
    enqueue_scan(h->grid[G_SCAN], s, d, 1);
    stage_end(h);
    stage_begin(h, WBRW_STAGE_REGEN);
    hipLaunchKernelGGL((k_regen<DIM, false, false>), dim3(h->grid[G_REGEN]), dim3(kThreads), 0, s, d);
    hipLaunchKernelGGL(k_close_regen, dim3(1), dim3(kThreads), 0, s, d);
    stage_end(h);
    return launch_check();
}

int enqueue_annihilate(wbrw_t h)
{
    return h->dim == 1 ? enqueue_annihilate_dim<1>(h) : enqueue_annihilate_dim<2>(h);
}

template <int DIM>
void set_grids_dim(wbrw_t h)
{
    const int cus = h->cus;
    h->occ_stream[0] = blocks_per_cu(k_stream<DIM>);
    if constexpr (DIM == 1) h->occ_stream[1] = blocks_per_cu(k_stream<DIM, 128, 16>, 128);
    h->occ_stream[2] = blocks_per_cu(k_stream<DIM, 512, 4>, 512);
    h->occ_bin[0] = blocks_per_cu(k_bin<DIM, false, false>);
    h->occ_bin[1] = blocks_per_cu(k_bin<DIM, false, false, 2048>);
    h->occ_bin[2] = blocks_per_cu(k_bin<DIM, false, false, 8192>);
    h->stream_shape = 0;
    h->bin_slots = kBinSlots[0];
    h->grid[G_STREAM] = std::min(h->occ_stream[0] * cus, kMaxGrid);
    if (h->strategy == WBRW_SP2 && h->tangent)
        h->grid[G_FAMILY] = persistent_blocks(k_family<DIM, true, true>, cus);
    else if (h->strategy == WBRW_SP2)
        h->grid[G_FAMILY] = persistent_blocks(k_family<DIM, true, false>, cus);
    else if (h->tangent)
        h->grid[G_FAMILY] = persistent_blocks(k_family<DIM, false, true>, cus);
    else
        h->grid[G_FAMILY] = persistent_blocks(k_family<DIM, false, false>, cus);
    h->occ_family = std::max(1, h->grid[G_FAMILY] / std::max(1, cus));
    h->grid[G_BIN] = std::min(h->occ_bin[0] * cus, kMaxGrid);
    h->grid[G_SCAN] = persistent_blocks(k_scan, cus);
    h->grid[G_REGEN] = persistent_blocks(k_regen<DIM, false, false>, cus);
    h->grid[G_DENS] = persistent_blocks(k_density_bin<DIM, false, false>, cus);
    h->grid[G_DENST] = persistent_blocks(k_density_bin<1, false, true>, cus);
    h->grid[G_SP2] = persistent_blocks(k_sp2_classify<DIM>, cus);
    h->grid[G_GHOST] = persistent_blocks(k_ghosts, cus);
    h->grid[G_EVENTS] = persistent_blocks(k_events, cus);
    h->grid[G_DRAW] = persistent_blocks(k_sp2_draw, cus);
}

}  // namespace

extern "C" {

const char *wbrw_strerror(int code)
{
    switch (code) {
    case WBRW_OK: return "ok";
    case WBRW_EINVAL: return "invalid argument or configuration";
    case WBRW_ECAPACITY: return "an instance outgrew its particle capacity";
    case WBRW_EHIP: return "HIP runtime error";
    case WBRW_ESTATE: return "invalid state";
    case WBRW_EDEPTH: return "family tree deeper than the per-step limit";
    case WBRW_ERANGE: return "a non-finite position, or a tangent outside the fixed-point range";
    default: return "unknown error";
    }
}

int wbrw_workspace_size(const wbrw_config *cfg, size_t *bytes)
{
    if (!bytes) return WBRW_EINVAL;
    const int v = validate(cfg);
    if (v) return v;
    *bytes = make_layout(cfg).total;
    return WBRW_OK;
}

int wbrw_init(const wbrw_config *cfg, void *workspace, size_t workspace_bytes, void *hip_stream,
              wbrw_t *out)
{
    if (!out || !workspace) return WBRW_EINVAL;
    *out = nullptr;
    const int v = validate(cfg);
    if (v) return v;
    if (((uintptr_t)workspace) % kAlign) return WBRW_EINVAL;
    Layout L = make_layout(cfg);
    if (workspace_bytes < L.total) return WBRW_EINVAL;

    wbrw_handle *h = new (std::nothrow) wbrw_handle();
    if (!h) return WBRW_EINVAL;
    h->B = cfg->n_instances;
    h->dim = cfg->dim;
    h->M = cfg->n_components;
    h->strategy = cfg->strategy;
    h->tangent = cfg->track_tangent;
    h->stream = (hipStream_t)hip_stream;
    h->ws = (char *)workspace;
    h->L = L;
    char *w = h->ws;

    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&h->cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        delete h;
        return WBRW_EHIP;
    }
    h->device = dev;
    {
        const int rc = scratch_on_current_device(dev, &h->scratch_ptr);
        if (rc) { delete h; return rc; }
    }

    Dev &d = h->d;
    d.B = h->B;
    d.dim = h->dim;
    d.M = h->M;
    d.strategy = h->strategy;
    d.tangent = h->tangent;
    d.hbar = cfg->hbar;
    d.tdep = 0;
    for (int m = 0; m < cfg->n_components; ++m) if (cfg->comp[m].modulated) d.tdep = 1;
    d.nx = cfg->nx;
    d.nk = cfg->nk;
    d.seed = cfg->seed;
    d.Nh = L.Nh;
    d.cap_total = L.cap_total;
    d.gcap_total = L.gcap_total;
    d.dt = cfg->dt;
    d.vfac = cfg->hbar / cfg->mass;
    d.x_lo = cfg->x_lo;
    d.x_hi = cfg->x_hi;
    d.k_lo = cfg->k_lo;
    d.k_hi = cfg->k_hi;
    d.dx = (cfg->x_hi - cfg->x_lo) / (double)cfg->nx;
    d.dk = (cfg->k_hi - cfg->k_lo) / (double)cfg->nk;
    d.max_bins = cfg->max_density_bins;

    // kernel tables: cumulative sums and normalisers
    std::vector<double> xi_tab(kMaxM, 0.0);
    std::vector<std::vector<double>> cums(kMaxM);
    for (int m = 0; m < h->M; ++m) {
        const wbrw_component &q = cfg->comp[m];
        d.kind[m] = q.kind;
        d.axis[m] = q.axis;
        d.sampler[m] = q.sampler;
        if (q.kind != WBRW_KERNEL_TABLE) continue;
        std::vector<double> &cm = cums[m];
        cm.resize((size_t)q.table_n + 1);
        cm[0] = 0.0;
        for (int j = 0; j < q.table_n; ++j) cm[j + 1] = cm[j] + q.table[j];
        const double dq = (q.q_hi - q.q_lo) / (double)q.table_n;
        // xi_m = (2/(pi hbar)) sum_j |F[V](2 q_j)| dq
        xi_tab[m] = ((2.0 * cm[q.table_n]) * dq) / (0x1.921fb54442d18p+1 * cfg->hbar);
        d.tab[m].cum = at<double>(w, L.tab[m]);
        d.tab[m].guide = at<int32_t>(w, L.guide[m]);
        d.tab[m].kg = guide_buckets(q.table_n);
        d.tab[m].n = q.table_n;
        d.tab[m].q_lo = q.q_lo;
        d.tab[m].dq = dq;
    }
    h->ip.resize(h->B);
    int64_t base = 0, gbase = 0, rbase = 0;
    for (int b = 0; b < h->B; ++b) {
        derive(cfg, b, xi_tab, h->ip[b]);
        h->ip[b].base = base;
        h->ip[b].cap = cfg->capacity[b];
        base += cfg->capacity[b];
        h->ip[b].rbase = rbase;
        h->ip[b].rtiles = ceil_div(cfg->capacity[b], kTileR) + 1;
        rbase += h->ip[b].rtiles;
        if (h->tangent) {
            h->ip[b].gbase = gbase;
            h->ip[b].gcap = cfg->ghost_capacity;
            gbase += cfg->ghost_capacity;
        }
    }
    for (int s = 0; s < 2; ++s) {
        Ens &E = d.ens[s];
        E.x0 = at<double>(w, L.ens[s][0]);
        E.x1 = cfg->dim == 2 ? at<double>(w, L.ens[s][1]) : nullptr;
        E.k0 = at<double>(w, L.ens[s][2]);
        E.k1 = cfg->dim == 2 ? at<double>(w, L.ens[s][3]) : nullptr;
        E.sg = h->strategy == WBRW_SP2 ? nullptr : at<int8_t>(w, L.ens[s][4]);
        E.w = h->strategy == WBRW_SP2 ? at<double>(w, L.ens[s][5]) : nullptr;
        E.id = at<uint64_t>(w, L.ens[s][6]);
        E.D = h->tangent ? at<double>(w, L.ens[s][7]) : nullptr;
        Ens &G = d.gens[s];
        std::memset(&G, 0, sizeof(G));
        if (h->tangent) {
            G.x0 = at<double>(w, L.gens[s][0]);
            G.k0 = at<double>(w, L.gens[s][2]);
            G.sg = at<int8_t>(w, L.gens[s][4]);
            G.id = at<uint64_t>(w, L.gens[s][6]);
            G.D = at<double>(w, L.gens[s][7]);
        }
    }
    std::vector<double> xitabs;
    if (L.xitab) {
        xitabs.assign((size_t)h->B * h->M * (kXiN + 1), 0.0);
        for (int b = 0; b < h->B; ++b)
            for (int m = 0; m < h->M; ++m)
                if (cfg->comp[m].sampler == 1)
                    xi_table(cfg->comp[m].H[b], cfg->comp[m].width[b], cfg->hbar,
                             &xitabs[((size_t)b * h->M + m) * (kXiN + 1)], h->ip[b].xi_h[m]);
        d.xi_tab = at<double>(w, L.xitab);
    }
    d.ip = at<InstParam>(w, L.ip);
    d.ctl = at<Ctl>(w, L.ctl);
    d.N = at<int64_t>(w, L.N);
    d.NG = at<int64_t>(w, L.NG);
    d.Nnew = at<int64_t>(w, L.Nnew);
    d.NGnew = at<int64_t>(w, L.NGnew);
    d.Nbase = at<int64_t>(w, L.Nbase);
    d.evc = at<int64_t>(w, L.evc);
    d.tileA = at<int64_t>(w, L.tileA);
    d.Nsrt = at<int64_t>(w, L.Nsrt);
    d.srtS = at<int64_t>(w, L.srtS);
    d.tileB = at<int64_t>(w, L.tileB);
    d.tileR = at<int64_t>(w, L.tileR);
    d.tileG = at<int64_t>(w, L.tileG);
    d.tally = at<int64_t>(w, L.tally);
    d.fpart = at<int64_t>(w, L.fpart);
    d.gpool = L.gpool ? at<char>(w, L.gpool) : nullptr;
    d.gpool_blocks = L.gpool ? kGPoolBlocks : 0;
    d.rstart = at<int64_t>(w, L.rstart);
    d.ev_idx = at<uint32_t>(w, L.ev_idx);
    d.gev_idx = h->tangent ? at<uint32_t>(w, L.gev_idx) : nullptr;
    d.tcA = at<uint64_t>(w, L.tcA);
    d.supA = at<uint64_t>(w, L.supA);
    d.spart = at<int64_t>(w, L.spart);
    d.emA = at<uint64_t>(w, L.emA);
    d.tcB = at<uint64_t>(w, L.tcB);
    d.supB = at<uint64_t>(w, L.supB);
    d.tsB = at<int64_t>(w, L.tsB);
    d.stg = at<int64_t>(w, L.stg);
    d.tcAg = h->tangent ? at<uint64_t>(w, L.tcAg) : nullptr;
    d.supAg = h->tangent ? at<uint64_t>(w, L.supAg) : nullptr;
    d.emAg = h->tangent ? at<uint64_t>(w, L.emAg) : nullptr;
    d.tcBg = h->tangent ? at<uint64_t>(w, L.tcBg) : nullptr;
    d.supBg = h->tangent ? at<uint64_t>(w, L.supBg) : nullptr;
    d.tsBg = h->tangent ? at<int64_t>(w, L.tsBg) : nullptr;
    d.stG = h->tangent ? at<uint64_t>(w, L.stG) : nullptr;
    d.stS = at<uint64_t>(w, L.stS);
    d.cnt = at<int32_t>(w, L.cnt);
    d.cntx = L.cntx ? at<int32_t>(w, L.cntx) : nullptr;
    d.off = at<int64_t>(w, L.off);
    d.occ = h->tangent ? at<int32_t>(w, L.occ) : nullptr;
    d.Tq = h->tangent ? at<int64_t>(w, L.Tq) : nullptr;
    d.occx = L.occx ? at<int32_t>(w, L.occx) : nullptr;
    d.Tqx = L.Tqx ? at<int64_t>(w, L.Tqx) : nullptr;
    d.dTq = h->tangent ? at<int64_t>(w, L.dTq) : nullptr;
    d.dacc = at<int64_t>(w, L.dacc);
    if (h->strategy == WBRW_SP2) {
        d.ntil = at<int32_t>(w, L.ntil);
        d.bA = at<uint64_t>(w, L.bA);
        d.bcopies = at<int32_t>(w, L.bcopies);
        d.bcls = at<int8_t>(w, L.bcls);
        d.bcell = at<int64_t>(w, L.bcell);
        d.bP = at<uint64_t>(w, L.bP);
        d.bTile = at<uint64_t>(w, L.bTile);
        d.bG = at<int32_t>(w, L.bG);
        d.bcls_stat = at<int64_t>(w, L.bcls_stat);
        d.tileD = at<int64_t>(w, L.tileD);
        d.bscan_tiles = at<int64_t>(w, L.bscan_tiles);
        d.tstride = L.tilesP;
    }

    if (h->dim == 1) set_grids_dim<1>(h); else set_grids_dim<2>(h);

    hipStream_t s = h->stream;
    auto fail = [&](int rc) { delete h; return rc; };
    // clear the bookkeeping region with a kernel
    const int64_t nz = (int64_t)((L.zero_end - L.zero_begin) / 8);
    hipLaunchKernelGGL(k_fill64, dim3(std::max(1, std::min<int>(h->cus * 8, (int)ceil_div(nz, kThreads)))),
                       dim3(kThreads), 0, s, at<uint64_t>(w, L.zero_begin), nz, 0ull);
    if (launch_check()) return fail(WBRW_EHIP);
    // constants and initial counts / plans
    std::vector<int64_t> N0(cfg->N0, cfg->N0 + h->B), plan;
    plan_host(plan, N0.data(), h->B, kTileA);
    if (hipMemcpyAsync((void *)d.ip, h->ip.data(), sizeof(InstParam) * h->B, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(d.N, N0.data(), 8 * h->B, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(d.tileA, plan.data(), 8 * (h->B + 1), hipMemcpyHostToDevice, s) != hipSuccess)
        return fail(WBRW_EHIP);
    if (h->tangent) {
        std::vector<int64_t> gplan(h->B + 1, 0);
        if (hipMemcpyAsync(d.tileA + h->B + 1, gplan.data(), 8 * (h->B + 1), hipMemcpyHostToDevice, s) != hipSuccess)
            return fail(WBRW_EHIP);
    }
    if (L.xitab &&
        hipMemcpyAsync((void *)d.xi_tab, xitabs.data(), 8 * xitabs.size(), hipMemcpyHostToDevice, s) != hipSuccess)
        return fail(WBRW_EHIP);
    std::vector<std::vector<int32_t>> guides(kMaxM);
    for (int m = 0; m < h->M; ++m) {
        if (cfg->comp[m].kind != WBRW_KERNEL_TABLE) continue;
        build_guide(cums[m], cfg->comp[m].table_n, d.tab[m].kg, guides[m]);
        if (hipMemcpyAsync((void *)d.tab[m].cum, cums[m].data(), 8 * cums[m].size(), hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemcpyAsync((void *)d.tab[m].guide, guides[m].data(), 4 * guides[m].size(), hipMemcpyHostToDevice, s) != hipSuccess)
            return fail(WBRW_EHIP);
    }
    if (cfg->init_hist) {
        // Alg. 3 from the caller's signed histogram: rounding, scan, placement
        double *hd = at<double>(w, L.hist);
        if (hipMemcpyAsync(hd, cfg->init_hist, 8 * (size_t)h->B * L.Nh, hipMemcpyHostToDevice, s) != hipSuccess)
            return fail(WBRW_EHIP);
        const double mu = cfg->dim == 1 ? d.dx * d.dk : ((d.dx * d.dx) * d.dk) * d.dk;
        const int nb = std::max(1, std::min(h->cus * 8, (int)ceil_div((int64_t)h->B * L.Nh, kThreads)));
        hipLaunchKernelGGL(k_hist_round, dim3(nb), dim3(kThreads), 0, s, d, (const double *)hd, mu);
        enqueue_scan(h->grid[G_SCAN], s, d, 1);
        if (h->dim == 1) {
            if (h->strategy == WBRW_SP2 && h->tangent) hipLaunchKernelGGL((k_regen<1, true, true>), dim3(h->grid[G_REGEN]), dim3(kThreads), 0, s, d);
            else if (h->strategy == WBRW_SP2) hipLaunchKernelGGL((k_regen<1, true, false>), dim3(h->grid[G_REGEN]), dim3(kThreads), 0, s, d);
            else if (h->tangent) hipLaunchKernelGGL((k_regen<1, false, true>), dim3(h->grid[G_REGEN]), dim3(kThreads), 0, s, d);
            else hipLaunchKernelGGL((k_regen<1, false, false>), dim3(h->grid[G_REGEN]), dim3(kThreads), 0, s, d);
        } else {
            if (h->strategy == WBRW_SP2) hipLaunchKernelGGL((k_regen<2, true, false>), dim3(h->grid[G_REGEN]), dim3(kThreads), 0, s, d);
            else hipLaunchKernelGGL((k_regen<2, false, false>), dim3(h->grid[G_REGEN]), dim3(kThreads), 0, s, d);
        }
        hipLaunchKernelGGL(k_close_regen, dim3(1), dim3(kThreads), 0, s, d);
        if (launch_check()) return fail(WBRW_EHIP);
        if (hipStreamSynchronize(s) != hipSuccess) return fail(WBRW_EHIP);
        *out = h;
        return WBRW_OK;
    }
    const int init_blocks = std::max<int64_t>(1, std::min<int64_t>(plan[h->B], (int64_t)h->cus * 16));
    if (h->dim == 1)
        hipLaunchKernelGGL(k_init<1>, dim3(init_blocks), dim3(kThreads), 0, s, d,
                           cfg->init_mean_x[0], cfg->init_mean_x[1], cfg->init_sigma_x[0], cfg->init_sigma_x[1],
                           cfg->init_mean_k[0], cfg->init_mean_k[1], cfg->init_sigma_k[0], cfg->init_sigma_k[1]);
    else
        hipLaunchKernelGGL(k_init<2>, dim3(init_blocks), dim3(kThreads), 0, s, d,
                           cfg->init_mean_x[0], cfg->init_mean_x[1], cfg->init_sigma_x[0], cfg->init_sigma_x[1],
                           cfg->init_mean_k[0], cfg->init_mean_k[1], cfg->init_sigma_k[0], cfg->init_sigma_k[1]);
    if (launch_check()) return fail(WBRW_EHIP);
    // host staging buffers above must outlive the copies
    if (hipStreamSynchronize(s) != hipSuccess) return fail(WBRW_EHIP);
    *out = h;
    return WBRW_OK;
}

int wbrw_step(wbrw_t h, int32_t nsteps)
{
    if (!h || nsteps < 0) return WBRW_EINVAL;
    for (int i = 0; i < nsteps; ++i) {
        const int rc = enqueue_step(h);
        if (rc) return rc;
    }
    return WBRW_OK;
}

int wbrw_annihilate(wbrw_t h)
{
    if (!h) return WBRW_EINVAL;
    return enqueue_annihilate(h);
}

int wbrw_run(wbrw_t h, int32_t nsteps, int32_t every, int32_t use_graph)
{
    if (!h || nsteps < 0 || every < 0) return WBRW_EINVAL;
    if (every == 0) return wbrw_step(h, nsteps);
    int left = nsteps;
    // eager steps up to the next multiple of `every` (counted from step 0)
    while (left > 0 && (h->host_step % every) != 0) {
        int rc = enqueue_step(h);
        if (!rc && h->host_step % every == 0) rc = enqueue_annihilate(h);
        if (rc) return rc;
        --left;
    }
    const int epochs = left / every;
    if (use_graph && h->stream != nullptr && epochs > 0) {
        if (h->graph_every != every) {
            if (h->gexec) { (void)hipGraphExecDestroy(h->gexec); h->gexec = nullptr; }
            hipGraph_t g;
            const int prof = h->prof;
            h->prof = 0;
            const int64_t hs = h->host_step;
            HIPCHK(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
            int rc = WBRW_OK;
            for (int i = 0; i < every && !rc; ++i) rc = enqueue_step(h);
            if (!rc) rc = enqueue_annihilate(h);
            hipError_t e = hipStreamEndCapture(h->stream, &g);
            h->prof = prof;
            h->host_step = hs;   // capture enqueued nothing
            if (rc) return rc;
            HIPCHK(e);
            HIPCHK(hipGraphInstantiate(&h->gexec, g, nullptr, nullptr, 0));
            (void)hipGraphDestroy(g);
            h->graph_every = every;
        }
        for (int ep = 0; ep < epochs; ++ep) {
            HIPCHK(hipGraphLaunch(h->gexec, h->stream));
            h->host_step += every;
        }
    } else {
        for (int ep = 0; ep < epochs; ++ep) {
            int rc = wbrw_step(h, every);
            if (!rc) rc = enqueue_annihilate(h);
            if (rc) return rc;
        }
    }
    return wbrw_step(h, left - epochs * every);
}

int wbrw_run_adaptive(wbrw_t h, int32_t nsteps, int32_t every, int64_t limit, int32_t use_graph)
{
    if (!h || nsteps < 0 || every < 0 || limit < 0) return WBRW_EINVAL;
    // the threshold is one instance's; tangents would need the ghost pass
    // conditioned too
    if (h->tangent || (limit > 0 && h->B != 1)) return WBRW_EINVAL;
    Dev &d = h->d;
    const int32_t c0 = d.cond_ann, e0 = d.ann_every;
    const int64_t l0 = d.ann_limit;
    d.cond_ann = 1;
    d.ann_every = every;
    d.ann_limit = limit;
    auto restore = [&]() { d.cond_ann = c0; d.ann_every = e0; d.ann_limit = l0; };
    int rc = WBRW_OK;
    if (use_graph && h->stream != nullptr && nsteps > 0) {
        if (!h->gexec_ad || h->ad_every != every || h->ad_limit != limit) {
            if (h->gexec_ad) { (void)hipGraphExecDestroy(h->gexec_ad); h->gexec_ad = nullptr; }
            hipGraph_t g;
            const int prof = h->prof;
            h->prof = 0;
            const int64_t hs = h->host_step;
            if (hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) { restore(); return WBRW_EHIP; }
            rc = enqueue_step(h);
            if (!rc) rc = enqueue_annihilate(h);
            const hipError_t e = hipStreamEndCapture(h->stream, &g);
            h->prof = prof;
            h->host_step = hs;
            if (!rc && e != hipSuccess) rc = WBRW_EHIP;
            if (!rc && hipGraphInstantiate(&h->gexec_ad, g, nullptr, nullptr, 0) != hipSuccess) rc = WBRW_EHIP;
            if (e == hipSuccess) (void)hipGraphDestroy(g);
            if (rc) { restore(); return rc; }
            h->ad_every = every;
            h->ad_limit = limit;
        }
        for (int i = 0; i < nsteps && !rc; ++i) {
            if (hipGraphLaunch(h->gexec_ad, h->stream) != hipSuccess) rc = WBRW_EHIP;
            h->host_step += 1;
        }
    } else {
        for (int i = 0; i < nsteps && !rc; ++i) {
            rc = enqueue_step(h);
            if (!rc) rc = enqueue_annihilate(h);
        }
    }
    restore();
    return rc;
}

int wbrw_density(wbrw_t h, int32_t axis, int32_t nbins, double lo, double hi, double *d_out)
{
    if (!h || !d_out || nbins < 1 || nbins > h->d.max_bins || !(hi > lo)) return WBRW_EINVAL;
    if (axis < 0 || axis >= h->dim) return WBRW_EINVAL;
    const double dxb = (hi - lo) / (double)nbins;
    const Dev &d = h->d;
    hipStream_t s = h->stream;
    const bool sp2 = h->strategy == WBRW_SP2;
    const int outb = std::max(1, std::min(h->cus * 4, (int)ceil_div((int64_t)h->B * nbins, kThreads)));
    stage_begin(h, WBRW_STAGE_DENSITY);
    if (h->dim == 1) {
        if (sp2) hipLaunchKernelGGL((k_density_bin<1, true, false>), dim3(h->grid[G_DENS]), dim3(kThreads), 0, s, d, 0, axis, nbins, lo, dxb);
        else hipLaunchKernelGGL((k_density_bin<1, false, false>), dim3(h->grid[G_DENS]), dim3(kThreads), 0, s, d, 0, axis, nbins, lo, dxb);
    } else {
        if (sp2) hipLaunchKernelGGL((k_density_bin<2, true, false>), dim3(h->grid[G_DENS]), dim3(kThreads), 0, s, d, 0, axis, nbins, lo, dxb);
        else hipLaunchKernelGGL((k_density_bin<2, false, false>), dim3(h->grid[G_DENS]), dim3(kThreads), 0, s, d, 0, axis, nbins, lo, dxb);
    }
    if (sp2) hipLaunchKernelGGL((k_density_out<true, false>), dim3(outb), dim3(kThreads), 0, s, d, nbins, dxb, d_out);
    else hipLaunchKernelGGL((k_density_out<false, false>), dim3(outb), dim3(kThreads), 0, s, d, nbins, dxb, d_out);
    stage_end(h);
    return launch_check();
}

int wbrw_density_noalloc(wbrw_t h, int32_t axis, int32_t nbins, double lo, double hi, double *d_out)
{
    if (!h || !d_out || nbins < 1 || !(hi > lo)) return WBRW_EINVAL;
    if (axis < 0 || axis >= h->dim) return WBRW_EINVAL;
    const int64_t words = (int64_t)kXcd * h->B * nbins;
    if (words > kNoAllocWords) return WBRW_EINVAL;
    if (!h->scratch_ptr) return WBRW_ESTATE;
    const double dxb = (hi - lo) / (double)nbins;
    // the same kernels as wbrw_density, with the accumulators ([kXcd][B][nbins])
    // in this device's scratch instead of the workspace
    Dev d = h->d;
    d.dacc = h->scratch_ptr;
    d.max_bins = nbins;
    hipStream_t s = h->stream;
    const bool sp2 = h->strategy == WBRW_SP2;
    // the accumulators start at zero (the readout clears what it reads, but a
    // call that failed part way, or the first call, may find anything)
    const int fb = std::max(1, std::min(h->cus * 4, (int)ceil_div(words, kThreads)));
    hipLaunchKernelGGL(k_fill64, dim3(fb), dim3(kThreads), 0, s, (uint64_t *)h->scratch_ptr, words, 0ull);
    const int outb = std::max(1, std::min(h->cus * 4, (int)ceil_div((int64_t)h->B * nbins, kThreads)));
    stage_begin(h, WBRW_STAGE_DENSITY);
    if (h->dim == 1) {
        if (sp2) hipLaunchKernelGGL((k_density_bin<1, true, false>), dim3(h->grid[G_DENS]), dim3(kThreads), 0, s, d, 0, axis, nbins, lo, dxb);
        else hipLaunchKernelGGL((k_density_bin<1, false, false>), dim3(h->grid[G_DENS]), dim3(kThreads), 0, s, d, 0, axis, nbins, lo, dxb);
    } else {
        if (sp2) hipLaunchKernelGGL((k_density_bin<2, true, false>), dim3(h->grid[G_DENS]), dim3(kThreads), 0, s, d, 0, axis, nbins, lo, dxb);
        else hipLaunchKernelGGL((k_density_bin<2, false, false>), dim3(h->grid[G_DENS]), dim3(kThreads), 0, s, d, 0, axis, nbins, lo, dxb);
    }
    if (sp2) hipLaunchKernelGGL((k_density_out<true, false>), dim3(outb), dim3(kThreads), 0, s, d, nbins, dxb, d_out);
    else hipLaunchKernelGGL((k_density_out<false, false>), dim3(outb), dim3(kThreads), 0, s, d, nbins, dxb, d_out);
    stage_end(h);
    return launch_check();
}

int wbrw_density_tangent(wbrw_t h, int32_t axis, int32_t nbins, double lo, double hi, double *d_out)
{
    if (!h || !d_out || !h->tangent || nbins < 1 || nbins > h->d.max_bins || !(hi > lo) || axis != 0)
        return WBRW_EINVAL;
    const double dxb = (hi - lo) / (double)nbins;
    const Dev &d = h->d;
    hipStream_t s = h->stream;
    hipLaunchKernelGGL((k_density_bin<1, false, true>), dim3(h->grid[G_DENST]), dim3(kThreads), 0, s, d, 0, axis, nbins, lo, dxb);
    hipLaunchKernelGGL((k_density_bin<1, false, true>), dim3(h->grid[G_DENST]), dim3(kThreads), 0, s, d, 1, axis, nbins, lo, dxb);
    const int outb = std::max(1, std::min(h->cus * 4, (int)ceil_div((int64_t)h->B * 3 * nbins, kThreads)));
    hipLaunchKernelGGL((k_density_out<false, true>), dim3(outb), dim3(kThreads), 0, s, d, nbins, dxb, d_out);
    return launch_check();
}

int wbrw_density_vjp(wbrw_t h, int32_t axis, int32_t nbins, double lo, double hi, const double *g,
                     double *grad_out)
{
    if (!h || !g || !grad_out || !h->tangent || nbins < 1 || !(hi > lo) || axis != 0) return WBRW_EINVAL;
    const double dxb = (hi - lo) / (double)nbins;
    const Dev &d = h->d;
    hipStream_t s = h->stream;
    if (nbins > h->d.max_bins) return WBRW_EINVAL;
    // the tangent bin sums (fixed point, real particles and ghosts), then the
    // contraction with g in bin order
    stage_begin(h, WBRW_STAGE_DENSITY);
    hipLaunchKernelGGL((k_density_bin<1, false, true>), dim3(h->grid[G_DENST]), dim3(kThreads), 0, s, d, 0, axis, nbins, lo, dxb);
    hipLaunchKernelGGL((k_density_bin<1, false, true>), dim3(h->grid[G_DENST]), dim3(kThreads), 0, s, d, 1, axis, nbins, lo, dxb);
    const int ob = std::max(1, (int)ceil_div((int64_t)h->B * 3, kThreads / 64));   // a wavefront each
    hipLaunchKernelGGL(k_vjp_out, dim3(ob), dim3(kThreads), 0, s, d, nbins, dxb, g, grad_out);
    stage_end(h);
    return launch_check();
}

// ---- snapshots ------------------------------------------------------------
namespace {

struct SnapHeader {
    uint64_t magic, total;
    int32_t B, dim, strategy, tangent;
    Ctl ctl;
};

// bytes per particle of the real / ghost ensembles in a snapshot
size_t real_bytes(const wbrw_handle *h)
{
    return 8 * 2 * h->dim + (h->strategy == WBRW_SP2 ? 8 : 1) + 8 + (h->tangent ? 24 : 0);
}
size_t ghost_bytes(const wbrw_handle *h) { return h->tangent ? 8 * 2 + 1 + 8 + 24 : 0; }

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

int snap_counts(wbrw_t h, std::vector<int64_t> &N, std::vector<int64_t> &NG, Ctl &c, size_t &total)
{
    HIPCHK(hipStreamSynchronize(h->stream));
    N.resize(h->B);
    NG.assign(h->B, 0);
    HIPCHK(hipMemcpy(N.data(), h->d.N, 8 * h->B, hipMemcpyDeviceToHost));
    if (h->tangent) HIPCHK(hipMemcpy(NG.data(), h->d.NG, 8 * h->B, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(&c, h->d.ctl, sizeof(Ctl), hipMemcpyDeviceToHost));
    int64_t nr = 0, ng = 0;
    for (int b = 0; b < h->B; ++b) { nr += N[b]; ng += NG[b]; }
    total = align_up(sizeof(SnapHeader)) + align_up(16 * (size_t)h->B) +
            align_up(8 * (size_t)h->B * kTalCount) + 16 * kAlign +
            (size_t)nr * real_bytes(h) + (size_t)ng * ghost_bytes(h);
    return WBRW_OK;
}

// Copies the fields of one ensemble between the workspace and a packed
// snapshot region: field-major, instances in order.
int copy_fields(wbrw_t h, int ghost, char *packed, const std::vector<int64_t> &N, bool to_snap,
                uint32_t set, size_t &cursor)
{
    const Ens E = ghost ? h->d.gens[set] : h->d.ens[set];
    const int64_t tot = ghost ? h->d.gcap_total : h->d.cap_total;
    struct F { char *base; size_t esz; int64_t stride; };
    std::vector<F> f;
    f.push_back({(char *)E.x0, 8, 0});
    if (!ghost && h->dim == 2) f.push_back({(char *)E.x1, 8, 0});
    f.push_back({(char *)E.k0, 8, 0});
    if (!ghost && h->dim == 2) f.push_back({(char *)E.k1, 8, 0});
    if (E.sg) f.push_back({(char *)E.sg, 1, 0});
    if (E.w) f.push_back({(char *)E.w, 8, 0});
    f.push_back({(char *)E.id, 8, 0});
    if (E.D) for (int c = 0; c < 3; ++c) f.push_back({(char *)(E.D + c * tot), 8, 0});
    for (const F &fld : f) {
        cursor = align_up(cursor);
        for (int b = 0; b < h->B; ++b) {
            const int64_t base = ghost ? h->ip[b].gbase : h->ip[b].base;
            const size_t n = (size_t)N[b] * fld.esz;
            if (n) {
                char *ws = fld.base + (size_t)base * fld.esz;
                if (to_snap) HIPCHK(hipMemcpyAsync(packed + cursor, ws, n, hipMemcpyDeviceToDevice, h->stream));
                else HIPCHK(hipMemcpyAsync(ws, packed + cursor, n, hipMemcpyDeviceToDevice, h->stream));
            }
            cursor += n;
        }
    }
    return WBRW_OK;
}

}  // namespace

int wbrw_snapshot_size(wbrw_t h, size_t *bytes)
{
    if (!h || !bytes) return WBRW_EINVAL;
    std::vector<int64_t> N, NG;
    Ctl c;
    const int rc = snap_counts(h, N, NG, c, *bytes);
    return rc;
}

int wbrw_snapshot(wbrw_t h, void *dst, size_t bytes)
{
    if (!h || !dst) return WBRW_EINVAL;
    std::vector<int64_t> N, NG;
    Ctl c;
    size_t total = 0;
    int rc = snap_counts(h, N, NG, c, total);
    if (rc) return rc;
    if (bytes < total) return WBRW_EINVAL;
    if (c.err) return (c.err & kErrCapacity) ? WBRW_ECAPACITY : (c.err & kErrDepth) ? WBRW_EDEPTH : WBRW_ERANGE;
    SnapHeader hd;
    std::memset(&hd, 0, sizeof(hd));
    hd.magic = 0x5742525753534e50ull;
    hd.total = total;
    hd.B = h->B;
    hd.dim = h->dim;
    hd.strategy = h->strategy;
    hd.tangent = h->tangent;
    hd.ctl = c;
    char *p = (char *)dst;
    size_t cur = 0;
    std::vector<int64_t> counts(2 * h->B);
    for (int b = 0; b < h->B; ++b) { counts[b] = N[b]; counts[h->B + b] = NG[b]; }
    HIPCHK(hipMemcpy(p, &hd, sizeof(hd), hipMemcpyHostToDevice));
    cur = align_up(sizeof(SnapHeader));
    HIPCHK(hipMemcpy(p + cur, counts.data(), 16 * h->B, hipMemcpyHostToDevice));
    cur = align_up(cur + 16 * h->B);
    HIPCHK(hipMemcpyAsync(p + cur, h->d.tally, 8 * (size_t)h->B * kTalCount, hipMemcpyDeviceToDevice, h->stream));
    cur = align_up(cur + 8 * (size_t)h->B * kTalCount);
    rc = copy_fields(h, 0, p, N, true, c.cur, cur);
    if (!rc && h->tangent) rc = copy_fields(h, 1, p, NG, true, c.gcur, cur);
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(h->stream));
    return WBRW_OK;
}

int wbrw_restore(wbrw_t h, const void *src, size_t bytes)
{
    if (!h || !src) return WBRW_EINVAL;
    HIPCHK(hipStreamSynchronize(h->stream));
    SnapHeader hd;
    if (bytes < sizeof(hd)) return WBRW_EINVAL;
    HIPCHK(hipMemcpy(&hd, src, sizeof(hd), hipMemcpyDeviceToHost));
    if (hd.magic != 0x5742525753534e50ull || hd.B != h->B || hd.dim != h->dim ||
        hd.strategy != h->strategy || hd.tangent != h->tangent || hd.total > bytes)
        return WBRW_EINVAL;
    const char *p = (const char *)src;
    size_t cur = align_up(sizeof(SnapHeader));
    std::vector<int64_t> counts(2 * h->B), N(h->B), NG(h->B);
    HIPCHK(hipMemcpy(counts.data(), p + cur, 16 * h->B, hipMemcpyDeviceToHost));
    cur = align_up(cur + 16 * h->B);
    for (int b = 0; b < h->B; ++b) {
        N[b] = counts[b];
        NG[b] = counts[h->B + b];
        if (N[b] > h->ip[b].cap || (h->tangent && NG[b] > h->ip[b].gcap)) return WBRW_EINVAL;
    }
    HIPCHK(hipMemcpyAsync(h->d.tally, p + cur, 8 * (size_t)h->B * kTalCount, hipMemcpyDeviceToDevice, h->stream));
    cur = align_up(cur + 8 * (size_t)h->B * kTalCount);
    // restore into set 0 / ghost set 0 and reset the control block
    int rc = copy_fields(h, 0, (char *)p, N, false, 0u, cur);
    if (!rc && h->tangent) rc = copy_fields(h, 1, (char *)p, NG, false, 0u, cur);
    if (rc) return rc;
    // The look-back status words of k_ghosts carry the annihilation count as
    // their epoch, and words written by this handle before the restore stay
    // in the workspace: the count continues past every epoch the handle has
    // used (never rewound to the snapshot's), so no stale word can match.
    Ctl now;
    HIPCHK(hipMemcpy(&now, h->d.ctl, sizeof(Ctl), hipMemcpyDeviceToHost));
    Ctl c;
    std::memset(&c, 0, sizeof(c));
    c.step = hd.ctl.step;
    c.ann_seq = std::max(now.ann_seq, hd.ctl.ann_seq) + 1u;
    std::vector<int64_t> plan, gplan;
    plan_host(plan, N.data(), h->B, kTileA);
    plan_host(gplan, NG.data(), h->B, kTileA);
    HIPCHK(hipMemcpyAsync(h->d.N, N.data(), 8 * h->B, hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipMemcpyAsync(h->d.tileA, plan.data(), 8 * (h->B + 1), hipMemcpyHostToDevice, h->stream));
    // the restored order is not known to be cell order (Nsrt = 0)
    std::vector<int64_t> zeros(h->B + 1, 0);
    HIPCHK(hipMemcpyAsync(h->d.Nsrt, zeros.data(), 8 * h->B, hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipMemcpyAsync(h->d.srtS, zeros.data(), 8 * (h->B + 1), hipMemcpyHostToDevice, h->stream));
    if (h->tangent) {
        HIPCHK(hipMemcpyAsync(h->d.NG, NG.data(), 8 * h->B, hipMemcpyHostToDevice, h->stream));
        HIPCHK(hipMemcpyAsync(h->d.tileA + h->B + 1, gplan.data(), 8 * (h->B + 1), hipMemcpyHostToDevice, h->stream));
    }
    HIPCHK(hipMemcpyAsync(h->d.ctl, &c, sizeof(Ctl), hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    h->host_step = hd.ctl.step;
    return WBRW_OK;
}

int wbrw_stats(wbrw_t h, int32_t b, wbrw_stats_t *out)
{
    if (!h || !out || b < 0 || b >= h->B) return WBRW_EINVAL;
    HIPCHK(hipStreamSynchronize(h->stream));
    Ctl c;
    int64_t tal[kTalCount], n = 0, ng = 0;
    HIPCHK(hipMemcpy(&c, h->d.ctl, sizeof(Ctl), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(tal, h->d.tally + (int64_t)b * kTalCount, sizeof(tal), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(&n, h->d.N + b, 8, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(&ng, h->d.NG + b, 8, hipMemcpyDeviceToHost));
    std::memset(out, 0, sizeof(*out));
    out->n = n;
    out->n_ghost = ng;
    out->events = tal[kTalEvents];
    out->pairs = tal[kTalPairs];
    out->killed = tal[kTalKilled];
    out->escaped = tal[kTalEscaped];
    out->max_depth = tal[kTalMaxDepth];
    out->event_cap_hits = tal[kTalEventCap];
    out->S_plus = tal[kTalSplus];
    out->S_minus = tal[kTalSminus];
    out->N_plus = tal[kTalNplus];
    out->N_minus = tal[kTalNminus];
    out->step = c.step;
    out->particle_steps = tal[kTalPSteps];
    out->gamma0 = h->ip[b].gamma0;
    out->annihilations = tal[kTalAnn];
    out->triggered = tal[kTalTrig];
    if (c.err & kErrCapacity) return WBRW_ECAPACITY;
    if (c.err & kErrDepth) return WBRW_EDEPTH;
    if (c.err & kErrRange) return WBRW_ERANGE;
    return WBRW_OK;
}

int wbrw_count(wbrw_t h, int32_t b, int32_t ghost, int64_t *n)
{
    if (!h || !n || b < 0 || b >= h->B) return WBRW_EINVAL;
    HIPCHK(hipStreamSynchronize(h->stream));
    HIPCHK(hipMemcpy(n, (ghost ? h->d.NG : h->d.N) + b, 8, hipMemcpyDeviceToHost));
    return WBRW_OK;
}

int wbrw_export(wbrw_t h, int32_t b, int32_t ghost, int64_t n, double *x, double *k, int8_t *sign,
                double *w, uint64_t *id, double *D)
{
    if (!h || b < 0 || b >= h->B || n < 0) return WBRW_EINVAL;
    if (ghost && !h->tangent) return WBRW_EINVAL;
    HIPCHK(hipStreamSynchronize(h->stream));
    Ctl c;
    int64_t cur_n = 0;
    HIPCHK(hipMemcpy(&c, h->d.ctl, sizeof(Ctl), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(&cur_n, (ghost ? h->d.NG : h->d.N) + b, 8, hipMemcpyDeviceToHost));
    if (cur_n != n) return WBRW_EINVAL;
    const Ens E = ghost ? h->d.gens[c.gcur] : h->d.ens[c.cur];
    const InstParam &P = h->ip[b];
    const int64_t base = ghost ? P.gbase : P.base;
    const int64_t tot = ghost ? h->d.gcap_total : h->d.cap_total;
    hipStream_t s = h->stream;
    const hipMemcpyKind kd = hipMemcpyDeviceToDevice;
    if (n == 0) return WBRW_OK;
    if (x) {
        HIPCHK(hipMemcpyAsync(x, E.x0 + base, 8 * n, kd, s));
        if (h->dim == 2) HIPCHK(hipMemcpyAsync(x + n, E.x1 + base, 8 * n, kd, s));
    }
    if (k) {
        HIPCHK(hipMemcpyAsync(k, E.k0 + base, 8 * n, kd, s));
        if (h->dim == 2) HIPCHK(hipMemcpyAsync(k + n, E.k1 + base, 8 * n, kd, s));
    }
    if (sign) {
        if (!E.sg) return WBRW_EINVAL;
        HIPCHK(hipMemcpyAsync(sign, E.sg + base, n, kd, s));
    }
    if (w) {
        if (!E.w) return WBRW_EINVAL;
        HIPCHK(hipMemcpyAsync(w, E.w + base, 8 * n, kd, s));
    }
    if (id) HIPCHK(hipMemcpyAsync(id, E.id + base, 8 * n, kd, s));
    if (D) {
        if (!E.D) return WBRW_EINVAL;
        for (int c3 = 0; c3 < 3; ++c3)
            HIPCHK(hipMemcpy2DAsync(D + c3, 24, E.D + c3 * tot + base, 8, 8, n, kd, s));
    }
    HIPCHK(hipStreamSynchronize(s));
    return WBRW_OK;
}

// A launch configuration: {stream blocks, family blocks, stream threads,
// stream particles per thread, bin blocks, bin hash slots}.
static void read_launch(const wbrw_handle *h, int32_t *c)
{
    c[0] = h->grid[G_STREAM];
    c[1] = h->grid[G_FAMILY];
    c[2] = kStreamShapes[h->stream_shape][0];
    c[3] = kStreamShapes[h->stream_shape][1];
    c[4] = h->grid[G_BIN];
    c[5] = h->bin_slots;
}

static void drop_graphs(wbrw_t h)
{
    if (h->gexec) {   // a captured epoch holds the old launch shapes
        (void)hipGraphExecDestroy(h->gexec);
        h->gexec = nullptr;
        h->graph_every = -1;
    }
    if (h->gexec_ad) {
        (void)hipGraphExecDestroy(h->gexec_ad);
        h->gexec_ad = nullptr;
    }
}

int wbrw_get_launch(wbrw_t h, int32_t *cfg)
{
    if (!h || !cfg) return WBRW_EINVAL;
    read_launch(h, cfg);
    return WBRW_OK;
}

int wbrw_set_launch(wbrw_t h, const int32_t *cfg)
{
    if (!h || !cfg) return WBRW_EINVAL;
    int shape = -1, slots = -1;
    for (int i = 0; i < 3; ++i) {
        if (cfg[2] == kStreamShapes[i][0] && cfg[3] == kStreamShapes[i][1] && h->occ_stream[i] > 0) shape = i;
        if (cfg[5] == kBinSlots[i]) slots = i;
    }
    if (shape < 0 || slots < 0) return WBRW_EINVAL;
    for (int q : {0, 1, 4})
        if (cfg[q] < 1 || cfg[q] > kMaxGrid) return WBRW_EINVAL;
    HIPCHK(hipStreamSynchronize(h->stream));
    h->stream_shape = shape;
    h->bin_slots = kBinSlots[slots];
    h->grid[G_STREAM] = cfg[0];
    h->grid[G_FAMILY] = cfg[1];
    h->grid[G_BIN] = cfg[4];
    drop_graphs(h);
    return WBRW_OK;
}

// Candidates: every streaming shape at 1..(its occupancy) blocks per CU
// (from the list below), the family kernel likewise, and for plain sp1 every
// binning hash size at its full occupancy and half of it.
static const int kPerCu[] = {1, 2, 3, 4, 6, 8, 12, 16};

int wbrw_autotune(wbrw_t h, int32_t steps_per_candidate, int32_t *chosen)
{
    if (!h || steps_per_candidate < 1) return WBRW_EINVAL;
    const int cus = std::max(1, h->cus);
    struct SC { int shape, grid; };
    std::vector<SC> cs;
    std::vector<int> cf;
    for (int sh = 0; sh < 3; ++sh)
        for (int per : kPerCu)
            if (h->occ_stream[sh] > 0 && per <= h->occ_stream[sh]) cs.push_back({sh, std::min(per * cus, kMaxGrid)});
    for (int per : kPerCu)
        if (per <= h->occ_family) cf.push_back(std::min(per * cus, kMaxGrid));
    const int prof = h->prof;
    const std::vector<wbrw_handle::Mark> saved = h->marks;
    h->marks.clear();
    std::vector<double> ts(cs.size(), 0.0), tf(cf.size(), 0.0);   // time per particle-step, summed
    std::vector<int> ns(cs.size(), 0), nf(cf.size(), 0);             // timed runs of each
    const size_t ncand = std::max(cs.size(), cf.size());
    int rc = WBRW_OK;
    auto psteps = [&](int64_t &out) {
        int64_t tal[kTalCount];
        out = 0;
        for (int b = 0; b < h->B; ++b) {
            if (hipMemcpy(tal, h->d.tally + (int64_t)b * kTalCount, sizeof(tal), hipMemcpyDeviceToHost) != hipSuccess)
                return WBRW_EHIP;
            out += tal[kTalPSteps];
        }
        return WBRW_OK;
    };
    // the binning pass of plain sp1, first, on the caller's ensemble (call
    // the autotuner where an annihilation is due, so that this state is a
    // typical one), timed alone: it only adds into the count grids, which
    // are cleared again, and into the escaped tallies, which are restored,
    // so the ensemble is untouched; the best of two timed passes counts
    if (h->strategy == WBRW_SP1 && !h->tangent) {
        std::vector<int64_t> tal((size_t)h->B * kTalCount);
        if (hipStreamSynchronize(h->stream) != hipSuccess ||
            hipMemcpy(tal.data(), h->d.tally, tal.size() * 8, hipMemcpyDeviceToHost) != hipSuccess) {
            h->marks = saved;
            return WBRW_EHIP;
        }
        struct BC { int slots, grid; };
        std::vector<BC> cb;
        for (int i = 0; i < 3; ++i) {
            const int full = std::min(h->occ_bin[i] * cus, kMaxGrid);
            cb.push_back({kBinSlots[i], full});
            if (h->occ_bin[i] > 1) cb.push_back({kBinSlots[i], std::max(cus, full / 2)});
        }
        std::vector<float> tb(cb.size(), 1e30f);
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = WBRW_EHIP;
        const size_t ncell = (size_t)h->d.Nh * (size_t)h->B;
        for (int pass = 0; pass < 3 && !rc; ++pass)
            for (size_t i = 0; i < cb.size() && !rc; ++i) {
                h->bin_slots = cb[i].slots;
                h->grid[G_BIN] = cb[i].grid;
                if (hipEventRecord(e0, h->stream) != hipSuccess) { rc = WBRW_EHIP; break; }
                if (h->dim == 1) launch_bin_plain<1>(h, h->stream); else launch_bin_plain<2>(h, h->stream);
                if (hipEventRecord(e1, h->stream) != hipSuccess) { rc = WBRW_EHIP; break; }
                hipLaunchKernelGGL(k_fill32, dim3(std::max<int64_t>(1, std::min<int64_t>(4096, ((int64_t)ncell + 255) / 256))),
                                   dim3(kThreads), 0, h->stream, h->d.cnt, (int64_t)ncell, 0);
                if (h->d.cntx)
                    hipLaunchKernelGGL(k_fill32, dim3(4096), dim3(kThreads), 0, h->stream, h->d.cntx,
                                       (int64_t)ncell * (kXcd - 1), 0);
                if (hipStreamSynchronize(h->stream) != hipSuccess) { rc = WBRW_EHIP; break; }
                float t = 0.f;
                (void)hipEventElapsedTime(&t, e0, e1);
                if (pass > 0) tb[i] = std::min(tb[i], t);
            }
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (hipMemcpy(h->d.tally, tal.data(), tal.size() * 8, hipMemcpyHostToDevice) != hipSuccess && !rc) rc = WBRW_EHIP;
        if (!rc) {
            size_t bb = 0;
            for (size_t i = 1; i < cb.size(); ++i) if (tb[i] < tb[bb]) bb = i;
            h->bin_slots = cb[bb].slots;
            h->grid[G_BIN] = cb[bb].grid;
        }
    }
    if (rc) { h->prof = prof; h->marks = saved; return rc; }
    // step candidates: step i runs streaming candidate i mod |cs| and family
    // candidate i mod |cf|; the first pass warms caches and code
    for (int pass = 0; pass < 2 && !rc; ++pass) {
        for (size_t i = 0; i < ncand && !rc; ++i) {
            const SC &a = cs[i % cs.size()];
            h->stream_shape = a.shape;
            h->grid[G_STREAM] = a.grid;
            h->grid[G_FAMILY] = cf[i % cf.size()];
            int64_t before = 0, after = 0;
            if (hipStreamSynchronize(h->stream) != hipSuccess || (rc = psteps(before))) { rc = rc ? rc : WBRW_EHIP; break; }
            h->prof = 1;
            for (int k = 0; k < steps_per_candidate && !rc; ++k) rc = enqueue_step(h);
            h->prof = 0;
            if (rc) break;
            if (hipStreamSynchronize(h->stream) != hipSuccess || (rc = psteps(after))) { rc = rc ? rc : WBRW_EHIP; break; }
            double a_s = 0, a_f = 0;
            for (auto &m : h->marks) {
                float t = 0.f;
                (void)hipEventElapsedTime(&t, m.a, m.b);
                if (m.stage == WBRW_STAGE_STREAM) a_s += t;
                if (m.stage == WBRW_STAGE_FAMILY) a_f += t;
                (void)hipEventDestroy(m.a);
                (void)hipEventDestroy(m.b);
            }
            h->marks.clear();
            const double ps = (double)std::max<int64_t>(1, after - before);
            if (pass == 1) {
                ts[i % cs.size()] += a_s / ps;
                ns[i % cs.size()] += 1;
                tf[i % cf.size()] += a_f / ps;
                nf[i % cf.size()] += 1;
            }
        }
    }
    if (rc) { h->prof = prof; h->marks = saved; return rc; }
    size_t bs = 0, bf = 0;   // the least mean time per particle-step
    for (size_t i = 1; i < cs.size(); ++i) if (ts[i] * ns[bs] < ts[bs] * ns[i]) bs = i;
    for (size_t i = 1; i < cf.size(); ++i) if (tf[i] * nf[bf] < tf[bf] * nf[i]) bf = i;
    h->stream_shape = cs[bs].shape;
    h->grid[G_STREAM] = cs[bs].grid;
    h->grid[G_FAMILY] = cf[bf];
    h->marks = saved;
    h->prof = prof;
    drop_graphs(h);
    if (rc) return rc;
    if (chosen) read_launch(h, chosen);
    return WBRW_OK;
}

static void drop_marks(wbrw_t h)
{
    for (auto &m : h->marks) {
        (void)hipEventDestroy(m.a);
        (void)hipEventDestroy(m.b);
    }
    h->marks.clear();
}

int wbrw_profile(wbrw_t h, int32_t enable)
{
    if (!h) return WBRW_EINVAL;
    if (enable) {
        HIPCHK(hipStreamSynchronize(h->stream));
        drop_marks(h);
    }
    h->prof = enable == 2 ? 2 : (enable != 0 ? 1 : 0);
    return WBRW_OK;
}

int wbrw_profile_read(wbrw_t h, double *ms, int64_t *launches)
{
    if (!h || !ms || !launches) return WBRW_EINVAL;
    HIPCHK(hipStreamSynchronize(h->stream));
    for (int s = 0; s < WBRW_STAGE_COUNT; ++s) { ms[s] = 0.0; launches[s] = 0; }
    for (auto &m : h->marks) {
        float t = 0.f;
        HIPCHK(hipEventElapsedTime(&t, m.a, m.b));
        ms[m.stage] += t;
        launches[m.stage] += 1;
    }
    return WBRW_OK;
}

int wbrw_destroy(wbrw_t h)
{
    if (!h) return WBRW_EINVAL;
    drop_marks(h);
    if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
    if (h->gexec_ad) (void)hipGraphExecDestroy(h->gexec_ad);
    delete h;
    return WBRW_OK;
}

}  // extern "C"
