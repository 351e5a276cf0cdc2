// eis_api.cpp -- host runtime behind include/eis.h.
//
// A context owns one HIP stream (default priority), the device prime table
// of the squarefree sieve, and grow-on-demand scratch buffers.  A range
// [a, b) is cut into passes of at most kPassCandidates candidates; each pass
// runs prime offsets -> sieve -> walk -> popcount on the stream.  The serving
// loop and the batched launch are built on the same pass machinery.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "../../include/eis.h"
#include "eis_internal.h"

using namespace eis;

namespace {

constexpr u64 kDefaultMaxSteps = u64(1) << 28;
// mu_1 is the distinguished ideal number window_scale * d^(1/4) / 16, about
// window_scale * d^(1/4) reduction steps from (1).
constexpr double kDefaultWindowScale = 3.5;
// Below this height the plain walk is as fast as the giant steps (AUTO).
constexpr u64 kDefaultInfraMinHeight = 100000000ull;
// d's per infrastructure batch (dictionaries of one batch are resident).
constexpr u64 kInfraBatch = u64(1) << 21;
constexpr u64 kPrimeLimit = 1000000;  // isqrt(EIS_MAX_D - 1) = 999999

// odd primes p <= lim (plain Eratosthenes on the host)
std::vector<u32> odd_primes_upto(u64 lim)
{
    std::vector<uint8_t> comp(lim + 1, 0);
    std::vector<u32> out;
    for (u64 i = 2; i <= lim; i++) {
        if (comp[i]) continue;
        if (i > 2) out.push_back((u32)i);
        for (u64 j = i * i; j <= lim; j += i) comp[j] = 1;
    }
    return out;
}

u64 isqrt_host(u64 n)
{
    u64 r = 0, bit = u64(1) << 62;
    while (bit > n) bit >>= 2;
    while (bit) {
        if (n >= r + bit) {
            n -= r + bit;
            r = (r >> 1) + bit;
        } else {
            r >>= 1;
        }
        bit >>= 2;
    }
    return r;
}

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

}  // namespace

struct eis_ctx {
    eis_config cfg{};
    int device = 0;
    int num_cu = 0;
    int walk_blocks_per_cu = 1;
    hipStream_t stream = nullptr;
    hipEvent_t ev_walk0 = nullptr, ev_walk1 = nullptr, ev_all0 = nullptr, ev_all1 = nullptr;

    // prime table
    std::vector<u32> primes_host;
    PrimeEntry *d_primes = nullptr;
    u32 nsmall = 0;

    // scratch (sized for one pass)
    u64 *d_roff = nullptr;
    u32 *d_sq_words = nullptr;
    u32 *d_eis_words = nullptr;
    u32 *d_list = nullptr;
    PassCounters *d_ctr = nullptr;
    unsigned long long *d_counts = nullptr;  // {n_sqfree, n_eis}
    u64 bytes_held = 0;

    // infrastructure-method scratch
    WindowState *d_state = nullptr;
    unsigned long long *d_lists = nullptr;
    unsigned long long *d_tables = nullptr;
    u32 *d_glist = nullptr;
    u32 *d_q = nullptr;             // per-batch queue heads (3 cache lines)
    u32 *d_fb_list = nullptr;
    PassCounters *d_fb_ctr = nullptr;
    u32 *h_pinned = nullptr;        // pinned host word for the list length
    u64 infra_batch_cap = 0;        // d's per batch the scratch holds
    u64 infra_stride_cap = 0;       // dictionary words per d the scratch holds
    u32 infra_emax_cap = 0;
    u32 infra_tsize_cap = 0;
    int window_blocks_per_cu = 1;
    int giant_blocks_per_cu = 1;

    std::mutex stats_mu;
    eis_stats stats{};
    int async_status = EIS_OK;
};

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------

static int hip_status(hipError_t e)
{
    if (e == hipSuccess) return EIS_OK;
    if (e == hipErrorOutOfMemory) return EIS_ENOMEM;
    return EIS_EDEVICE;
}

#define HIP_TRY(expr)                          \
    do {                                       \
        hipError_t _e = (expr);                \
        if (_e != hipSuccess) return hip_status(_e); \
    } while (0)

extern "C" uint64_t eis_first_candidate(uint64_t a)
{
    return a + ((5 + 8 - (a % 8)) % 8);
}

extern "C" uint64_t eis_num_candidates(uint64_t a, uint64_t b)
{
    if (a >= b) return 0;
    u64 d0 = eis_first_candidate(a);
    if (d0 >= b) return 0;
    return (b - 1 - d0) / 8 + 1;
}

extern "C" const char *eis_strerror(int status)
{
    switch (status) {
    case EIS_OK: return "ok";
    case EIS_EINVAL: return "invalid argument";
    case EIS_ERANGE: return "range exceeds EIS_MAX_D";
    case EIS_ENOMEM: return "out of device memory or memory budget";
    case EIS_EDEVICE: return "no usable gfx950 device or HIP runtime error";
    case EIS_EBUSY: return "serving queue full";
    case EIS_ECANCELED: return "request cancelled";
    case EIS_ETIMEDOUT: return "timed out";
    case EIS_EINTERNAL: return "step budget exceeded or internal check failed";
    default: return "unknown status";
    }
}

extern "C" int eis_abi_version(void) { return EIS_ABI_VERSION; }

extern "C" void eis_config_default(eis_config *cfg)
{
    if (!cfg) return;
    std::memset(cfg, 0, sizeof(*cfg));
    cfg->device = 0;
    cfg->method = EIS_METHOD_AUTO;
}

static void free_infra(eis_ctx *c)
{
    (void)hipFree(c->d_state);
    (void)hipFree(c->d_lists);
    (void)hipFree(c->d_tables);
    (void)hipFree(c->d_glist);
    c->d_state = nullptr;
    c->d_lists = c->d_tables = nullptr;
    c->d_glist = nullptr;
    c->infra_batch_cap = c->infra_stride_cap = 0;
}

static void free_scratch(eis_ctx *c)
{
    free_infra(c);
    (void)hipFree(c->d_roff);
    (void)hipFree(c->d_sq_words);
    (void)hipFree(c->d_eis_words);
    (void)hipFree(c->d_list);
    c->d_roff = nullptr;
    c->d_sq_words = c->d_eis_words = c->d_list = nullptr;
}

extern "C" void eis_destroy(eis_ctx *c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    free_scratch(c);
    (void)hipFree(c->d_primes);
    (void)hipFree(c->d_ctr);
    (void)hipFree(c->d_counts);
    (void)hipFree(c->d_q);
    (void)hipFree(c->d_fb_list);
    (void)hipFree(c->d_fb_ctr);
    if (c->h_pinned) (void)hipHostFree(c->h_pinned);
    if (c->ev_walk0) (void)hipEventDestroy(c->ev_walk0);
    if (c->ev_walk1) (void)hipEventDestroy(c->ev_walk1);
    if (c->ev_all0) (void)hipEventDestroy(c->ev_all0);
    if (c->ev_all1) (void)hipEventDestroy(c->ev_all1);
    if (c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

extern "C" int eis_create(const eis_config *cfg, eis_ctx **out)
{
    if (!out) return EIS_EINVAL;
    eis_config def;
    eis_config_default(&def);
    if (!cfg) cfg = &def;
    if (cfg->flags != 0) return EIS_EINVAL;
    if (cfg->method < EIS_METHOD_BABY || cfg->method > EIS_METHOD_AUTO) return EIS_EINVAL;
    if (cfg->window_scale < 0) return EIS_EINVAL;

    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return EIS_EDEVICE;
    if (cfg->device < 0 || cfg->device >= ndev) return EIS_EDEVICE;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, cfg->device) != hipSuccess) return EIS_EDEVICE;
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return EIS_EDEVICE;

    eis_ctx *c = new (std::nothrow) eis_ctx();
    if (!c) return EIS_ENOMEM;
    c->cfg = *cfg;
    c->cfg.tune_cache_path = nullptr;  // not retained beyond the call
    if (c->cfg.max_steps_per_d == 0) c->cfg.max_steps_per_d = kDefaultMaxSteps;
    if (c->cfg.window_scale == 0.0) c->cfg.window_scale = kDefaultWindowScale;
    if (c->cfg.max_steps_per_d > 0xffff0000ull) c->cfg.max_steps_per_d = 0xffff0000ull;
    c->device = cfg->device;
    c->num_cu = prop.multiProcessorCount;
    int rc = EIS_OK;
    do {
        if (hipSetDevice(c->device) != hipSuccess) { rc = EIS_EDEVICE; break; }
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            rc = EIS_EDEVICE;
            break;
        }
        if (hipEventCreate(&c->ev_walk0) != hipSuccess || hipEventCreate(&c->ev_walk1) != hipSuccess ||
            hipEventCreate(&c->ev_all0) != hipSuccess || hipEventCreate(&c->ev_all1) != hipSuccess) {
            rc = EIS_EDEVICE;
            break;
        }
        // prime table: odd p <= 10^6, m = p^2, 8^{-1} mod m = (7m + 1)/8
        // (p odd => m = 1 mod 8)
        c->primes_host = odd_primes_upto(kPrimeLimit);
        std::vector<PrimeEntry> tab(c->primes_host.size());
        for (size_t k = 0; k < tab.size(); k++) {
            u64 p = c->primes_host[k];
            tab[k].m = p * p;
            tab[k].inv8 = (7 * tab[k].m + 1) / 8;
            if (tab[k].m < 4096) c->nsmall = (u32)(k + 1);
        }
        if (hipMalloc(&c->d_primes, tab.size() * sizeof(PrimeEntry)) != hipSuccess) {
            rc = EIS_ENOMEM;
            break;
        }
        if (hipMemcpy(c->d_primes, tab.data(), tab.size() * sizeof(PrimeEntry),
                      hipMemcpyHostToDevice) != hipSuccess) {
            rc = EIS_EDEVICE;
            break;
        }
        if (hipMalloc(&c->d_ctr, sizeof(PassCounters)) != hipSuccess ||
            hipMalloc(&c->d_counts, 4 * sizeof(unsigned long long)) != hipSuccess) {
            rc = EIS_ENOMEM;
            break;
        }
        if (hipMalloc(&c->d_q, 3 * 64) != hipSuccess ||
            hipMalloc(&c->d_fb_ctr, sizeof(PassCounters)) != hipSuccess ||
            hipMalloc(&c->d_fb_list, kPassCandidates * sizeof(u32)) != hipSuccess) {
            rc = EIS_ENOMEM;
            break;
        }
        if (hipHostMalloc(reinterpret_cast<void **>(&c->h_pinned), 64, hipHostMallocDefault) != hipSuccess) {
            rc = EIS_ENOMEM;
            break;
        }
        c->walk_blocks_per_cu = walk_baby_blocks_per_cu();
        c->window_blocks_per_cu = walk_window_blocks_per_cu();
        c->giant_blocks_per_cu = walk_giant_blocks_per_cu();
    } while (0);
    if (rc != EIS_OK) {
        eis_destroy(c);
        return rc;
    }
    *out = c;
    return EIS_OK;
}

// Make sure the per-pass scratch can hold `ncand` candidates.
static int ensure_scratch(eis_ctx *c)
{
    if (c->d_list) return EIS_OK;
    const u64 ncand = kPassCandidates;
    const u64 nwords = ncand / 32;
    u64 need = c->primes_host.size() * sizeof(u64) + 2 * nwords * sizeof(u32) + ncand * sizeof(u32);
    if (c->cfg.mem_budget_bytes && need > c->cfg.mem_budget_bytes) return EIS_ENOMEM;
    if (hipMalloc(&c->d_roff, c->primes_host.size() * sizeof(u64)) != hipSuccess ||
        hipMalloc(&c->d_sq_words, nwords * sizeof(u32)) != hipSuccess ||
        hipMalloc(&c->d_eis_words, nwords * sizeof(u32)) != hipSuccess ||
        hipMalloc(&c->d_list, ncand * sizeof(u32)) != hipSuccess) {
        free_scratch(c);
        return EIS_ENOMEM;
    }
    c->bytes_held = need;
    return EIS_OK;
}

// number of table primes p with p^2 <= dmax
static u32 primes_needed(const eis_ctx *c, u64 dmax)
{
    u64 r = isqrt_host(dmax);
    return (u32)(std::upper_bound(c->primes_host.begin(), c->primes_host.end(), (u32)std::min<u64>(r, 0xffffffffu)) -
                 c->primes_host.begin());
}

static bool use_infra(const eis_ctx *c, u64 d0)
{
    if (c->cfg.method == EIS_METHOD_INFRA) return true;
    if (c->cfg.method == EIS_METHOD_BABY) return false;
    return d0 >= kDefaultInfraMinHeight;
}

// Dictionary geometry for heights up to dmax.
static void infra_geometry(const eis_ctx *c, u64 dmax, u32 &emax, u32 &tsize)
{
    double n = c->cfg.window_scale * std::pow((double)dmax, 0.25) / 16.0;
    u32 emain = (u32)std::max(2.0, std::floor(n + 1.0));
    emain = std::max<u32>(emain, 16);
    emax = emain + 16;
    if (emax > 496) emax = 496;
    // load factor at most 0.5 for the usual count (mu_1 plus a few)
    tsize = 32;
    while (tsize < 2 * (emain + 4)) tsize <<= 1;
}

// Scratch of one infrastructure batch: `batch` d's (rounded up to whole
// tiles of 64), `emax` list entries and `tsize` table slots each.
static int ensure_infra(eis_ctx *c, u64 batch, u32 emax, u32 tsize)
{
    const u64 tiles = (batch + 63) / 64;
    const u64 stride = (u64)emax + tsize;
    if (c->d_lists && c->infra_batch_cap >= tiles * 64 && c->infra_stride_cap >= stride &&
        c->infra_emax_cap >= emax && c->infra_tsize_cap >= tsize)
        return EIS_OK;
    free_infra(c);
    const u64 bytes = tiles * 64 * (stride * 8 + sizeof(WindowState) + sizeof(u32));
    if (c->cfg.mem_budget_bytes && c->bytes_held + bytes > c->cfg.mem_budget_bytes) return EIS_ENOMEM;
    if (hipMalloc(&c->d_lists, tiles * 64 * emax * 8) != hipSuccess ||
        hipMalloc(&c->d_tables, tiles * 64 * tsize * 8) != hipSuccess ||
        hipMalloc(&c->d_state, tiles * 64 * sizeof(WindowState)) != hipSuccess ||
        hipMalloc(&c->d_glist, tiles * 64 * sizeof(u32)) != hipSuccess) {
        free_infra(c);
        return EIS_ENOMEM;
    }
    c->infra_batch_cap = tiles * 64;
    c->infra_stride_cap = stride;
    c->infra_emax_cap = emax;
    c->infra_tsize_cap = tsize;
    return EIS_OK;
}

// Walk of the compacted list with the plain method (grid sized to n when n
// is known on the host, else to the whole device).
static int enqueue_walk_baby(eis_ctx *c, u64 d0, const u32 *list, PassCounters *ctr, u64 n_hint,
                             hipStream_t st)
{
    WalkParams wp;
    wp.d0 = d0;
    wp.list = list;
    wp.ctr = ctr;
    wp.eis_words = c->d_eis_words;
    wp.max_steps = (u32)c->cfg.max_steps_per_d;
    u64 want_blocks = (n_hint + 255) / 256;
    u64 max_blocks = (u64)c->num_cu * (u64)c->walk_blocks_per_cu;
    u32 grid = (u32)std::max<u64>(1, std::min(want_blocks, max_blocks));
    HIP_TRY(launch_walk_baby(wp, grid, st));
    return EIS_OK;
}

// Enqueue one pass: candidates d0 + 8 i, i < n (n <= kPassCandidates).
// Bitmaps land in c->d_sq_words / c->d_eis_words; counts are added to
// counts[0..1].  The infrastructure method reads the list length back to
// the host once per pass, to size its batches.
static int enqueue_pass(eis_ctx *c, u64 d0, u32 n, unsigned long long *counts, hipStream_t st)
{
    const u64 nwords = (n + 31) / 32;
    const u64 dmax = d0 + 8ull * (n - 1);
    const u32 np = primes_needed(c, dmax);
    HIP_TRY(launch_zero_u32(reinterpret_cast<u32 *>(c->d_ctr), sizeof(PassCounters) / 4, st));
    HIP_TRY(launch_zero_u32(reinterpret_cast<u32 *>(c->d_fb_ctr), sizeof(PassCounters) / 4, st));
    HIP_TRY(launch_zero_u32(c->d_eis_words, nwords, st));
    HIP_TRY(launch_prime_offsets(c->d_primes, np, d0, c->d_roff, st));
    HIP_TRY(launch_sieve(c->d_primes, c->d_roff, np, std::min(c->nsmall, np), n, c->d_sq_words,
                         c->d_list, c->d_ctr, st));
    u64 launches = 6;
    HIP_TRY(hipEventRecord(c->ev_walk0, st));
    if (!use_infra(c, d0)) {
        int rc = enqueue_walk_baby(c, d0, c->d_list, c->d_ctr, n, st);
        if (rc != EIS_OK) return rc;
        launches += 1;
    } else {
        HIP_TRY(hipMemcpyAsync(c->h_pinned, &c->d_ctr->list_len, sizeof(u32), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        const u64 nd = *c->h_pinned;
        u32 emax, tsize;
        infra_geometry(c, dmax, emax, tsize);
        const u64 batch = std::min<u64>(std::max<u64>(nd, 1), kInfraBatch);
        int rc = ensure_infra(c, batch, emax, tsize);
        if (rc != EIS_OK) return rc;
        InfraParams ip;
        ip.d0 = d0;
        ip.list = c->d_list;
        ip.ctr = c->d_ctr;
        ip.win_next = c->d_q;
        ip.giant_len = c->d_q + 16;
        ip.giant_next = c->d_q + 32;
        ip.giant_list = c->d_glist;
        ip.fb_list = c->d_fb_list;
        ip.fb_ctr = c->d_fb_ctr;
        ip.state = c->d_state;
        ip.lists = c->d_lists;
        ip.tables = c->d_tables;
        ip.emax = emax;
        ip.tsize = tsize;
        ip.window_scale = (float)c->cfg.window_scale;
        ip.max_steps = (u32)c->cfg.max_steps_per_d;
        ip.max_giants = 1u << 20;
        ip.eis_words = c->d_eis_words;
        const u64 max_win = (u64)c->num_cu * (u64)c->window_blocks_per_cu;
        const u64 max_giant = (u64)c->num_cu * (u64)c->giant_blocks_per_cu;
        for (u64 k0 = 0; k0 < nd; k0 += batch) {
            const u64 k1 = std::min<u64>(nd, k0 + batch);
            ip.k0 = (u32)k0;
            ip.k1 = (u32)k1;
            const u64 nb = k1 - k0;
            HIP_TRY(launch_zero_u32(c->d_q, 3 * 16, st));
            const u32 gw = (u32)std::max<u64>(1, std::min((nb + 255) / 256, max_win));
            // window waves take tiles of 64 d's
            HIP_TRY(launch_walk_window(ip, gw, st));
            HIP_TRY(launch_build_tables(ip, (u32)nb, st));
            const u32 gg = (u32)std::max<u64>(1, std::min((nb + 255) / 256, max_giant));
            HIP_TRY(launch_walk_giant(ip, gg, st));
            launches += 4;
        }
        // d's that left the giant-step method: the plain walk, exact for all d
        rc = enqueue_walk_baby(c, d0, c->d_fb_list, c->d_fb_ctr, 256ull * (u64)c->num_cu, st);
        if (rc != EIS_OK) return rc;
        launches += 1;
    }
    HIP_TRY(hipEventRecord(c->ev_walk1, st));
    HIP_TRY(launch_popcount_add(c->d_sq_words, nwords, counts + 0, st));
    HIP_TRY(launch_popcount_add(c->d_eis_words, nwords, counts + 1, st));
    std::lock_guard<std::mutex> lk(c->stats_mu);
    c->stats.launches += launches + 2;
    return EIS_OK;
}

// Read the per-pass counters after the stream has finished the pass.
static int collect_pass(eis_ctx *c)
{
    PassCounters h, f;
    if (hipMemcpy(&h, c->d_ctr, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess) return EIS_EDEVICE;
    if (hipMemcpy(&f, c->d_fb_ctr, sizeof(f), hipMemcpyDeviceToHost) != hipSuccess) return EIS_EDEVICE;
    h.baby_steps += f.baby_steps;
    h.refills += f.refills;
    h.err_count += f.err_count;
    float wms = 0.f;
    bool have_ms = hipEventElapsedTime(&wms, c->ev_walk0, c->ev_walk1) == hipSuccess;
    std::lock_guard<std::mutex> lk(c->stats_mu);
    if (have_ms) c->stats.last_walk_ms = wms;
    c->stats.discriminants += h.list_len;
    c->stats.baby_steps += h.baby_steps;
    c->stats.giant_steps += h.giant_steps;
    c->stats.refills += h.refills;
    c->stats.fallbacks += f.list_len;
    return h.err_count ? EIS_EINTERNAL : EIS_OK;
}

static int check_range(uint64_t a, uint64_t b)
{
    if (a >= b) return EIS_OK;
    if (b > EIS_MAX_D) return EIS_ERANGE;
    return EIS_OK;
}

// Core driver: every pass of [a, b); bitmaps go to host (h_*) or device
// (d_*) byte buffers at the pass's byte offset.
static int run_range(eis_ctx *c, uint64_t a, uint64_t b, uint8_t *h_sq, uint8_t *h_eis,
                     uint8_t *d_sq, uint8_t *d_eis, uint64_t *n_sq, uint64_t *n_eis,
                     unsigned long long *d_counts_out, hipStream_t st, bool sync)
{
    if (hipSetDevice(c->device) != hipSuccess) return EIS_EDEVICE;
    int rc = ensure_scratch(c);
    if (rc != EIS_OK) return rc;
    const u64 n = eis_num_candidates(a, b);
    const u64 d0 = eis_first_candidate(a);
    unsigned long long *counts = d_counts_out ? d_counts_out : c->d_counts;
    HIP_TRY(launch_zero_u32(reinterpret_cast<u32 *>(counts), 4, st));
    HIP_TRY(hipEventRecord(c->ev_all0, st));
    int status = EIS_OK;
    for (u64 off = 0; off < n; off += kPassCandidates) {
        const u32 pn = (u32)std::min<u64>(kPassCandidates, n - off);
        rc = enqueue_pass(c, d0 + 8 * off, pn, counts, st);
        if (rc != EIS_OK) return rc;
        const size_t bytes = (pn + 7) / 8;
        const size_t boff = off / 8;
        if (h_sq) HIP_TRY(hipMemcpyAsync(h_sq + boff, c->d_sq_words, bytes, hipMemcpyDeviceToHost, st));
        if (h_eis) HIP_TRY(hipMemcpyAsync(h_eis + boff, c->d_eis_words, bytes, hipMemcpyDeviceToHost, st));
        if (d_sq) HIP_TRY(hipMemcpyAsync(d_sq + boff, c->d_sq_words, bytes, hipMemcpyDeviceToDevice, st));
        if (d_eis) HIP_TRY(hipMemcpyAsync(d_eis + boff, c->d_eis_words, bytes, hipMemcpyDeviceToDevice, st));
        if (sync || off + kPassCandidates < n) {
            // the pass buffers are reused: wait before the next pass
            HIP_TRY(hipStreamSynchronize(st));
            int prc = collect_pass(c);
            if (prc != EIS_OK) status = prc;
        }
    }
    HIP_TRY(hipEventRecord(c->ev_all1, st));
    if (sync) {
        HIP_TRY(hipStreamSynchronize(st));
        unsigned long long hc[2] = {0, 0};
        HIP_TRY(hipMemcpy(hc, counts, sizeof(hc), hipMemcpyDeviceToHost));
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, c->ev_all0, c->ev_all1) == hipSuccess) {
            std::lock_guard<std::mutex> lk(c->stats_mu);
            c->stats.last_total_ms = ms;
        }
        if (status != EIS_OK) return status;
        if (n_sq) *n_sq = hc[0];
        if (n_eis) *n_eis = hc[1];
    }
    return status;
}

extern "C" int eis_count(eis_ctx *c, uint64_t a, uint64_t b, uint64_t *n_sqfree, uint64_t *n_eis)
{
    if (!c) return EIS_EINVAL;
    int rc = check_range(a, b);
    if (rc != EIS_OK) return rc;
    if (a >= b) {
        if (n_sqfree) *n_sqfree = 0;
        if (n_eis) *n_eis = 0;
        return EIS_OK;
    }
    return run_range(c, a, b, nullptr, nullptr, nullptr, nullptr, n_sqfree, n_eis, nullptr,
                     c->stream, true);
}

extern "C" int eis_classify(eis_ctx *c, uint64_t a, uint64_t b, uint8_t *sqfree_bits,
                            uint8_t *eis_bits, size_t len_bytes, uint64_t *n_sqfree,
                            uint64_t *n_eis)
{
    if (!c) return EIS_EINVAL;
    int rc = check_range(a, b);
    if (rc != EIS_OK) return rc;
    const u64 n = eis_num_candidates(a, b);
    if ((sqfree_bits || eis_bits) && len_bytes < (n + 7) / 8) return EIS_EINVAL;
    if (a >= b || n == 0) {
        if (n_sqfree) *n_sqfree = 0;
        if (n_eis) *n_eis = 0;
        return EIS_OK;
    }
    // stage into temporaries so that an error leaves the caller's buffers untouched
    std::vector<uint8_t> tsq(sqfree_bits ? (n + 7) / 8 : 0), teis(eis_bits ? (n + 7) / 8 : 0);
    u64 cs = 0, ce = 0;
    rc = run_range(c, a, b, sqfree_bits ? tsq.data() : nullptr, eis_bits ? teis.data() : nullptr,
                   nullptr, nullptr, &cs, &ce, nullptr, c->stream, true);
    if (rc != EIS_OK) return rc;
    if (sqfree_bits) std::memcpy(sqfree_bits, tsq.data(), tsq.size());
    if (eis_bits) std::memcpy(eis_bits, teis.data(), teis.size());
    if (n_sqfree) *n_sqfree = cs;
    if (n_eis) *n_eis = ce;
    return EIS_OK;
}

extern "C" int eis_classify_async(eis_ctx *c, uint64_t a, uint64_t b, void *d_sqfree_bits,
                                  void *d_eis_bits, uint64_t *d_counts2, void *hip_stream)
{
    if (!c) return EIS_EINVAL;
    int rc = check_range(a, b);
    if (rc != EIS_OK) return rc;
    hipStream_t st = hip_stream ? reinterpret_cast<hipStream_t>(hip_stream) : c->stream;
    const u64 n = eis_num_candidates(a, b);
    if (n == 0) {
        if (d_counts2) {
            if (hipSetDevice(c->device) != hipSuccess) return EIS_EDEVICE;
            HIP_TRY(launch_zero_u32(reinterpret_cast<u32 *>(d_counts2), 4, st));
        }
        return EIS_OK;
    }
    rc = run_range(c, a, b, nullptr, nullptr, reinterpret_cast<uint8_t *>(d_sqfree_bits),
                   reinterpret_cast<uint8_t *>(d_eis_bits), nullptr, nullptr,
                   reinterpret_cast<unsigned long long *>(d_counts2), st, false);
    if (rc == EIS_EINTERNAL) c->async_status = rc;
    return rc;
}

extern "C" int eis_last_error(eis_ctx *c)
{
    if (!c) return EIS_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return EIS_EDEVICE;
    HIP_TRY(hipStreamSynchronize(c->stream));
    int rc = collect_pass(c);
    if (rc == EIS_OK) rc = c->async_status;
    c->async_status = EIS_OK;
    return rc;
}

extern "C" int eis_count_batch(eis_ctx *c, const uint64_t *a, const uint64_t *b, size_t n,
                               uint64_t *n_sqfree, uint64_t *n_eis)
{
    if (!c || (n && (!a || !b))) return EIS_EINVAL;
    for (size_t k = 0; k < n; k++) {
        int rc = check_range(a[k], b[k]);
        if (rc != EIS_OK) return rc;
    }
    std::vector<uint64_t> s(n), e(n);
    for (size_t k = 0; k < n; k++) {
        int rc = eis_count(c, a[k], b[k], &s[k], &e[k]);
        if (rc != EIS_OK) return rc;
    }
    for (size_t k = 0; k < n; k++) {
        if (n_sqfree) n_sqfree[k] = s[k];
        if (n_eis) n_eis[k] = e[k];
    }
    return EIS_OK;
}

extern "C" int eis_submit(eis_ctx *c, uint64_t, uint64_t, uint64_t *)
{
    if (!c) return EIS_EINVAL;
    return EIS_EINVAL;
}

extern "C" int eis_wait(eis_ctx *c, uint64_t, int64_t, uint64_t *, uint64_t *)
{
    if (!c) return EIS_EINVAL;
    return EIS_EINVAL;
}

extern "C" int eis_cancel(eis_ctx *c, uint64_t)
{
    if (!c) return EIS_EINVAL;
    return EIS_EINVAL;
}

extern "C" int eis_get_stats(eis_ctx *c, eis_stats *out)
{
    if (!c || !out) return EIS_EINVAL;
    std::lock_guard<std::mutex> lk(c->stats_mu);
    *out = c->stats;
    return EIS_OK;
}
