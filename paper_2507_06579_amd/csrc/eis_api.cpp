// eis_api.cpp -- host runtime behind include/eis.h.
//
// Everything is organised in passes.  A pass is a set of at most
// kMaxSegments segments (ranges or pieces of ranges) with at most
// kPassCandidates candidates together; one pass is one launch sequence on the
// context's stream:
//
//   zero counters -> prime offsets (all segments) -> sieve (all segments, one
//   launch) -> plain walk (one persistent launch over every item of the
//   plain-walk segments) -> giant-step batches (window, table build, giant
//   walk) over the items of the giant-step segments -> plain walk of the
//   hand-offs -> per-segment popcounts
//
// The segment table lives in device memory, so the launch sequence of a pass
// depends only on its shape; the batched call replays it from a hipGraph.
// The single-range calls, the batched call and the serving loop all run on
// this machinery; a mutex serialises them on the pass buffers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "../../include/eis.h"
#include "eis_internal.h"

using namespace eis;

namespace {

constexpr u64 kDefaultMaxSteps = u64(1) << 28;
// mu_1 is the distinguished ideal number window_scale * d^(1/4) / 16, about
// window_scale * d^(1/4) reduction steps from (1).
constexpr double kDefaultWindowScale = 2.0;
// AUTO method: segments starting at or above this height take giant steps.
constexpr u64 kDefaultInfraMinHeight = 100000000ull;
// Giant-step batches: a batch's dictionaries are resident, so a batch holds
// as many d's as the memory budget allows (a pass at most), rounded down to
// whole 2^16 d's but at least this many.  Large batches matter: every batch
// ends with a tail in which lanes whose queue is drained idle until the
// slowest d of their wave is done.
constexpr u64 kInfraBatchMin = u64(1) << 16;
constexpr u64 kPrimeLimit = 1000000;  // isqrt(EIS_MAX_D - 1) = 999999
constexpr u32 kPassWords = (u32)(kPassCandidates / 32) + kMaxSegments;
// queue heads of the giant-step method (three cache lines) and the task
// counts of its cost buckets (one line each), in 32-bit words
constexpr u32 kQueueWords = (3 + kCostBuckets) * 16;
// counter sets of a pass: plain walk, giant steps, hand-offs, the retry
// round's hand-offs
constexpr u32 kPassCounterSets = 4;
// the retry round takes mu_1 this many distinguished ideals later
constexpr u32 kRetryShift = 4;
constexpr u32 kDefaultServeSlots = 64;
// serving: candidates of one request per pass (a larger request advances a
// chunk per pass, so that requests behind it are not held up)
constexpr u64 kServeChunk = u64(1) << 20;

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

// A segment as the host plans it.
struct HostSeg {
    u64 d0;
    u32 n;
    u32 slot;      // count slot
    u32 method;    // 0 plain walk, 1 giant steps
    float wscale;  // giant steps: window scale of the segment
    u64 dst_bit;   // candidate offset of the segment in the caller's bitmap
    u32 set = kSetSquarefree;  // the candidate set counted and walked
    u32 walk_chunk = kDefaultWalkChunk;  // giant walk: reduction steps per walk phase
};

struct Request {
    u64 ticket = 0;
    u64 d0 = 0, ncand = 0;
    u64 dispatched = 0;  // candidates handed to passes
    u64 completed = 0;   // candidates whose pass has finished
    u64 n_sq = 0, n_eis = 0;
    u64 reserved = 0;    // device bytes admitted for it (see chunk_footprint)
    int status = EIS_OK;
    bool cancelled = false;
    bool finished = false;
};

}  // namespace

// Device buffers one pass runs on: the context's own (allocated on first
// use and kept) or views into the no-allocation scratch.
struct PassBufs {
    SegInfo *segs = nullptr;    // segment table
    SegInfo *h_segs = nullptr;  // pinned staging of the table (null: a kernel stores it)
    u64 *roff = nullptr;        // prime offsets
    u64 roff_cap = 0;
    u32 *sq_words = nullptr, *eis_words = nullptr;  // pass bitmaps
    u32 *list_plain = nullptr, *list_giant = nullptr, *fb_list = nullptr;
    PassCounters *ctrs = nullptr;  // [0] plain walk, [1] giant steps, [2] hand-offs,
                                   // [3] hand-offs of the retry round
    u32 *q = nullptr;              // giant-step queue heads (3 cache lines), then the task
                                   // counts of the cost buckets (one line each)
    unsigned long long *counts = nullptr;  // (pi_D, pi_E) per count slot
    u64 counts_cap = 0;                    // pairs
    // giant-step scratch
    WindowState *state = nullptr;
    GiantTask *tasks = nullptr;  // kCostBuckets buckets of infra_batch_cap tasks
    unsigned long long *lists = nullptr;
    u32 *lres = nullptr;
    u16 *tables = nullptr;
    u64 infra_bytes = 0;
    u64 infra_batch_cap = 0;
    u32 infra_emax_cap = 0;
    u32 infra_tsize_cap = 0;
    bool ready = false;
};

// A pass of the server in flight: its own counters, counts and pinned host
// staging (the host fills the next pass's segment table and reads the last
// pass's counts while this one runs); the rest of the pass buffers is the
// context's, which the passes use in stream order.
struct Flight {
    PassCounters *ctrs = nullptr;
    unsigned long long *counts = nullptr;    // 2 per segment
    SegInfo *h_segs = nullptr;               // pinned
    unsigned long long *h_counts = nullptr;  // pinned
    hipEvent_t done = nullptr;
    std::vector<std::pair<u64, u64>> parts;  // (ticket, candidates) per segment
    bool retry = false;
    bool busy = false;
    u64 seq = 0;
};

// Autotuner height bins: bin b holds 10^(b/2) <= d < 10^((b+1)/2), b < 25.
constexpr int kTuneBins = 25;
constexpr int kTuneFirstBin = 12;  // below 10^6 the plain walk, untimed

struct eis_ctx {
    eis_config cfg{};
    int device = 0;
    int num_cu = 0;
    int walk_blocks_per_cu = 1;
    int window_blocks_per_cu = 1;
    int giant_blocks_per_cu = 1;
    hipStream_t stream = nullptr;
    hipEvent_t ev_walk0 = nullptr, ev_walk1 = nullptr, ev_all0 = nullptr, ev_all1 = nullptr;
    double window_scale = kDefaultWindowScale;
    u64 infra_min_height = kDefaultInfraMinHeight;
    bool use_graphs = true;
    // autotuner choices per height bin (half decades, see bin_of)
    bool tuned = false;
    int tuned_method[kTuneBins] = {};
    double tuned_ws[kTuneBins] = {};
    u32 tuned_chunk[kTuneBins] = {};     // giant walk: reduction steps per walk phase
    u32 tuned_pass_log2[kTuneBins] = {}; // a range's pass size, log2 of candidates
    std::string tune_path;

    // prime table
    std::vector<u32> primes_host;
    PrimeEntry *d_primes = nullptr;
    u32 nsmall = 0;    // primes with p^2 < 4096
    u32 nsmall_p = 0;  // primes with p < 4096

    // pass buffers (the context's own, allocated on first use)
    PassBufs pb;
    unsigned long long *h_counts = nullptr;  // pinned
    u64 h_counts_cap = 0;
    bool uncollected = false;            // a pass whose counters nobody has read yet
    hipStream_t pending_stream = nullptr;  // the stream it runs on
    PassCounters *pending_ctrs = nullptr;  // its counters
    bool pending_retry = false;          // it has the retry round

    // per-kernel timing (EIS_FLAG_KERNEL_TIMES): event pairs of this pass
    bool kernel_times = false;
    std::vector<hipEvent_t> kev;
    std::vector<int> kev_kind;
    u32 kev_used = 0;
    u64 bytes_held = 0;

    // captured pass sequences, by shape
    std::map<std::vector<u64>, hipGraphExec_t> graphs;

    std::mutex gpu_mu;  // pass buffers and the stream
    std::mutex stats_mu;
    eis_stats stats{};
    int async_status = EIS_OK;

    // serving
    std::mutex smu;
    std::condition_variable scv;    // wakes the server loop
    std::condition_variable dcv;    // wakes waiters
    std::deque<u64> order;          // tickets in arrival order (not finished)
    std::map<u64, Request> reqs;
    u64 next_ticket = 1;
    bool stop = false;
    std::thread server;
    Flight flights[2];
    std::atomic<bool> flights_ready{false};
    u64 flight_seq = 0;
    u64 serve_budget = 0;    // device bytes for the requests' giant-step scratch
    u64 serve_reserved = 0;  // of which the admitted requests hold
    hipEvent_t ev_order = nullptr;  // orders other streams after the context's
};

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------

static int hip_status(hipError_t e)
{
    if (e == hipSuccess) return EIS_OK;
    if (e == hipErrorOutOfMemory) return EIS_ENOMEM;
    return EIS_EDEVICE;
}

// With EIS_TRACE_ERRORS set in the environment, every failed HIP call is
// reported on stderr with its source line (the status alone does not say
// which call failed).
static int hip_fail(hipError_t e, const char *what, int line)
{
    static const bool trace = std::getenv("EIS_TRACE_ERRORS") != nullptr;
    if (trace) std::fprintf(stderr, "eis: line %d: %s: %s\n", line, what, hipGetErrorString(e));
    return hip_status(e);
}

// a call whose failure is not acted on (teardown), reported when tracing
#define HIP_IGNORE(expr)                                            \
    do {                                                            \
        hipError_t _e = (expr);                                     \
        if (_e != hipSuccess) (void)hip_fail(_e, #expr, __LINE__);  \
    } while (0)

#define HIP_TRY(expr)                                               \
    do {                                                            \
        hipError_t _e = (expr);                                     \
        if (_e != hipSuccess) return hip_fail(_e, #expr, __LINE__); \
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

// Autotuner cache: a small JSON object written by eis_tune,
//   {"arch": "gfx950", "bins": [{"b": 12, "method": 0, "window_scale": 2.0,
//     "walk_chunk": 16, "pass_log2": 24, ...}, ...]}
// read back by scanning for the keys of every bin (the two shape keys are
// optional: a bin without them keeps the defaults).
static void load_tune_cache(eis_ctx *c)
{
    FILE *f = std::fopen(c->tune_path.c_str(), "r");
    if (!f) return;
    std::string txt;
    char buf[4096];
    size_t got;
    while ((got = std::fread(buf, 1, sizeof(buf), f)) > 0) txt.append(buf, got);
    std::fclose(f);
    if (txt.find("\"gfx950\"") == std::string::npos) return;
    int method[kTuneBins];
    double ws[kTuneBins];
    u32 chunk[kTuneBins], plog[kTuneBins];
    u32 seen = 0;
    size_t at = 0;
    while ((at = txt.find("\"b\":", at)) != std::string::npos) {
        int b = -1, m = -1;
        double w = 0.0;
        if (std::sscanf(txt.c_str() + at, "\"b\": %d, \"method\": %d, \"window_scale\": %lf", &b, &m,
                        &w) == 3 &&
            b >= 0 && b < kTuneBins && (m == 0 || m == 1) && w > 0.0 && w < 100.0) {
            method[b] = m;
            ws[b] = w;
            seen |= 1u << b;
            // optional shape keys within this bin's object
            const size_t end = txt.find('}', at);
            const std::string obj = txt.substr(at, end == std::string::npos ? std::string::npos : end - at);
            int ch = (int)kDefaultWalkChunk, pl2 = 24;
            const size_t kc = obj.find("\"walk_chunk\":");
            if (kc != std::string::npos) std::sscanf(obj.c_str() + kc, "\"walk_chunk\": %d", &ch);
            const size_t kp = obj.find("\"pass_log2\":");
            if (kp != std::string::npos) std::sscanf(obj.c_str() + kp, "\"pass_log2\": %d", &pl2);
            chunk[b] = (u32)std::min(std::max(ch, 1), 64);
            plog[b] = (u32)std::min(std::max(pl2, 22), 24);
        }
        at += 4;
    }
    // every bin must be present
    if (seen != (1u << kTuneBins) - 1) return;
    for (int b = 0; b < kTuneBins; b++) {
        c->tuned_method[b] = method[b];
        c->tuned_ws[b] = ws[b];
        c->tuned_chunk[b] = chunk[b];
        c->tuned_pass_log2[b] = plog[b];
    }
    c->tuned = true;
}

static void free_infra(eis_ctx *c)
{
    HIP_IGNORE(hipFree(c->pb.state));
    HIP_IGNORE(hipFree(c->pb.tasks));
    HIP_IGNORE(hipFree(c->pb.lists));
    HIP_IGNORE(hipFree(c->pb.lres));
    HIP_IGNORE(hipFree(c->pb.tables));
    c->pb.state = nullptr;
    c->pb.tasks = nullptr;
    c->pb.lists = nullptr;
    c->pb.lres = nullptr;
    c->pb.tables = nullptr;
    c->bytes_held -= c->pb.infra_bytes;
    c->pb.infra_bytes = 0;
    c->pb.infra_batch_cap = 0;
    c->pb.infra_emax_cap = c->pb.infra_tsize_cap = 0;
}

static void drop_graphs(eis_ctx *c)
{
    for (auto &kv : c->graphs) HIP_IGNORE(hipGraphExecDestroy(kv.second));
    c->graphs.clear();
}

static void stop_server(eis_ctx *c)
{
    {
        std::lock_guard<std::mutex> lk(c->smu);
        c->stop = true;
    }
    c->scv.notify_all();
    c->dcv.notify_all();
    if (c->server.joinable()) c->server.join();
}

extern "C" void eis_destroy(eis_ctx *c)
{
    if (!c) return;
    stop_server(c);
    HIP_IGNORE(hipSetDevice(c->device));
    if (c->stream) HIP_IGNORE(hipStreamSynchronize(c->stream));
    for (Flight &f : c->flights) {
        HIP_IGNORE(hipFree(f.ctrs));
        HIP_IGNORE(hipFree(f.counts));
        if (f.h_segs) HIP_IGNORE(hipHostFree(f.h_segs));
        if (f.h_counts) HIP_IGNORE(hipHostFree(f.h_counts));
        if (f.done) HIP_IGNORE(hipEventDestroy(f.done));
    }
    if (c->ev_order) HIP_IGNORE(hipEventDestroy(c->ev_order));
    c->ev_order = nullptr;

    drop_graphs(c);
    free_infra(c);
    HIP_IGNORE(hipFree(c->d_primes));
    HIP_IGNORE(hipFree(c->pb.segs));
    HIP_IGNORE(hipFree(c->pb.roff));
    HIP_IGNORE(hipFree(c->pb.sq_words));
    HIP_IGNORE(hipFree(c->pb.eis_words));
    HIP_IGNORE(hipFree(c->pb.list_plain));
    HIP_IGNORE(hipFree(c->pb.list_giant));
    HIP_IGNORE(hipFree(c->pb.fb_list));
    HIP_IGNORE(hipFree(c->pb.ctrs));
    HIP_IGNORE(hipFree(c->pb.counts));
    HIP_IGNORE(hipFree(c->pb.q));
    if (c->pb.h_segs) HIP_IGNORE(hipHostFree(c->pb.h_segs));
    if (c->h_counts) HIP_IGNORE(hipHostFree(c->h_counts));
    if (c->ev_walk0) HIP_IGNORE(hipEventDestroy(c->ev_walk0));
    if (c->ev_walk1) HIP_IGNORE(hipEventDestroy(c->ev_walk1));
    for (hipEvent_t e : c->kev) HIP_IGNORE(hipEventDestroy(e));
    if (c->ev_all0) HIP_IGNORE(hipEventDestroy(c->ev_all0));
    if (c->ev_all1) HIP_IGNORE(hipEventDestroy(c->ev_all1));
    if (c->stream) HIP_IGNORE(hipStreamDestroy(c->stream));
    // teardown leaves no error pending in this thread for later calls
    (void)hipGetLastError();
    delete c;
}

extern "C" int eis_create(const eis_config *cfg, eis_ctx **out)
{
    if (!out) return EIS_EINVAL;
    eis_config def;
    eis_config_default(&def);
    if (!cfg) cfg = &def;
    if ((cfg->flags & ~(uint32_t)(EIS_FLAG_NO_GRAPHS | EIS_FLAG_KERNEL_TIMES |
                                  EIS_FLAG_NO_CONJUGATE_LOOKUPS | EIS_FLAG_NO_SMALL_NORM_PRODUCT)) != 0)
        return EIS_EINVAL;
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
    if (cfg->tune_cache_path) c->tune_path = cfg->tune_cache_path;
    c->cfg.tune_cache_path = nullptr;  // the context keeps its own copy
    if (c->cfg.max_steps_per_d == 0) c->cfg.max_steps_per_d = kDefaultMaxSteps;
    if (c->cfg.max_steps_per_d > 0xffff0000ull) c->cfg.max_steps_per_d = 0xffff0000ull;
    if (c->cfg.serve_slots == 0) c->cfg.serve_slots = kDefaultServeSlots;
    c->window_scale = cfg->window_scale > 0 ? cfg->window_scale : kDefaultWindowScale;
    c->use_graphs = (cfg->flags & EIS_FLAG_NO_GRAPHS) == 0;
    c->kernel_times = (cfg->flags & EIS_FLAG_KERNEL_TIMES) != 0;
    c->device = cfg->device;
    c->num_cu = prop.multiProcessorCount;
    int rc = EIS_OK;
    do {
        if (hipSetDevice(c->device) != hipSuccess) { rc = EIS_EDEVICE; break; }
        if (c->cfg.mem_budget_bytes == 0) {
            size_t free_b = 0, total_b = 0;
            if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) { rc = EIS_EDEVICE; break; }
            c->cfg.mem_budget_bytes = free_b / 4;
        }
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
            tab[k].p = (u32)p;
            // 8^{-1} mod p = 8^(p-2) mod p (Fermat)
            u64 inv = 1, base = 8 % p;
            for (u64 e = p - 2; e; e >>= 1) {
                if (e & 1) inv = inv * base % p;
                base = base * base % p;
            }
            tab[k].inv8p = (u32)inv;
            if (tab[k].m < 4096) c->nsmall = (u32)(k + 1);
            if (p < 4096) c->nsmall_p = (u32)(k + 1);
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
        c->walk_blocks_per_cu = walk_baby_blocks_per_cu();
        c->window_blocks_per_cu = walk_window_blocks_per_cu();
        c->giant_blocks_per_cu = walk_giant_blocks_per_cu();
        // the no-allocation scratch of this device: its address is looked
        // up here, once per device (a failure shows in that entry point)
        (void)noalloc_scratch_init(c->device);
        if (!c->tune_path.empty()) load_tune_cache(c);
    } while (0);
    if (rc != EIS_OK) {
        eis_destroy(c);
        return rc;
    }
    *out = c;
    return EIS_OK;
}

// ---------------------------------------------------------------------------
// buffers
// ---------------------------------------------------------------------------

static int ensure_pass_buffers(eis_ctx *c)
{
    if (c->pb.ready) return EIS_OK;
    const u64 need = kMaxSegments * sizeof(SegInfo) + 2ull * kPassWords * 4 +
                     3ull * kPassCandidates * 4 + kPassCounterSets * sizeof(PassCounters) + kQueueWords * 4;
    if (c->bytes_held + need > c->cfg.mem_budget_bytes) return EIS_ENOMEM;
    if (hipMalloc(&c->pb.segs, kMaxSegments * sizeof(SegInfo)) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void **>(&c->pb.h_segs), kMaxSegments * sizeof(SegInfo),
                      hipHostMallocDefault) != hipSuccess ||
        hipMalloc(&c->pb.sq_words, (u64)kPassWords * 4) != hipSuccess ||
        hipMalloc(&c->pb.eis_words, (u64)kPassWords * 4) != hipSuccess ||
        hipMalloc(&c->pb.list_plain, kPassCandidates * 4) != hipSuccess ||
        hipMalloc(&c->pb.list_giant, kPassCandidates * 4) != hipSuccess ||
        hipMalloc(&c->pb.fb_list, kPassCandidates * 4) != hipSuccess ||
        hipMalloc(&c->pb.ctrs, kPassCounterSets * sizeof(PassCounters)) != hipSuccess ||
        hipMalloc(&c->pb.q, kQueueWords * 4) != hipSuccess)
        return EIS_ENOMEM;
    c->bytes_held += need;
    c->pb.ready = true;
    return EIS_OK;
}

// Before a shared pass buffer is freed or replaced: let every pass already
// enqueued on the context's stream (the server keeps up to two in flight)
// finish with it.
static int quiesce(eis_ctx *c)
{
    HIP_TRY(hipStreamSynchronize(c->stream));
    return EIS_OK;
}

// The prime offsets of a pass's segments; grows by half again at least, as
// rising heights need slowly more primes (each reallocation also drops the
// captured graphs).
static int ensure_roff(eis_ctx *c, u64 n)
{
    if (c->pb.roff_cap >= n) return EIS_OK;
    int qrc = quiesce(c);
    if (qrc != EIS_OK) return qrc;
    const u64 cap = std::max(n, c->pb.roff_cap + c->pb.roff_cap / 2);
    (void)hipFree(c->pb.roff);
    c->pb.roff = nullptr;
    c->pb.roff_cap = 0;
    if (hipMalloc(&c->pb.roff, cap * sizeof(u64)) != hipSuccess) return EIS_ENOMEM;
    c->pb.roff_cap = cap;
    drop_graphs(c);  // captured sequences hold the old pointer
    return EIS_OK;
}

static int ensure_counts(eis_ctx *c, u64 pairs)
{
    if (c->pb.counts_cap < pairs) {
        int qrc = quiesce(c);
        if (qrc != EIS_OK) return qrc;
        (void)hipFree(c->pb.counts);
        c->pb.counts = nullptr;
        c->pb.counts_cap = 0;
        u64 cap = std::max<u64>(pairs, kMaxSegments);
        if (hipMalloc(&c->pb.counts, cap * 2 * sizeof(unsigned long long)) != hipSuccess)
            return EIS_ENOMEM;
        c->pb.counts_cap = cap;
        drop_graphs(c);
    }
    if (c->h_counts_cap < pairs) {
        if (c->h_counts) (void)hipHostFree(c->h_counts);
        c->h_counts = nullptr;
        c->h_counts_cap = 0;
        u64 cap = std::max<u64>(pairs, kMaxSegments);
        if (hipHostMalloc(reinterpret_cast<void **>(&c->h_counts),
                          cap * 2 * sizeof(unsigned long long), hipHostMallocDefault) != hipSuccess)
            return EIS_ENOMEM;
        c->h_counts_cap = cap;
    }
    return EIS_OK;
}

// Device bytes per d of the giant-step method: the list (8-byte keys and
// 4-byte residue sums), the table, the window record and a task slot in
// every cost bucket.
static u64 infra_bytes_per_d(u32 emax, u32 tsize)
{
    return (u64)emax * 12 + (u64)tsize * 2 + sizeof(WindowState) + kCostBuckets * sizeof(GiantTask);
}

// Scratch of the giant-step method: `batch` d's (whole tiles of 64), `emax`
// list entries and `tsize` table slots each.  A reallocation keeps room for
// the d's held before and adds an eighth more entries and slots than asked
// for, when the budget allows, so that a sweep of rising heights, whose lists
// and tables grow slowly, does not free and allocate its scratch (gigabytes,
// and at times hundreds of milliseconds each way) at almost every call.  The
// d's themselves get no room beyond the need: serving measured worse with it
// (a larger allocation is a longer stall when a burst outgrows the scratch).
constexpr u32 kEmaxMax = 496;  // list entries per d at most (9-bit slot indices)

static u32 round8_up(u64 x) { return (u32)((x + 7) / 8 * 8); }

static int ensure_infra(eis_ctx *c, u64 batch, u32 emax, u32 tsize)
{
    const u64 need = (batch + 63) / 64 * 64;
    if (c->pb.lists && c->pb.infra_batch_cap >= need && c->pb.infra_emax_cap >= emax &&
        c->pb.infra_tsize_cap >= tsize)
        return EIS_OK;
    const u64 old_cap = c->pb.lists ? c->pb.infra_batch_cap : 0;
    int qrc = quiesce(c);
    if (qrc != EIS_OK) return qrc;
    free_infra(c);
    drop_graphs(c);
    u64 cap = std::max(need, old_cap);
    u32 ecap = std::max(emax, std::min(round8_up(emax + emax / 8), kEmaxMax));
    u32 tcap = std::max(tsize, std::min(round8_up(tsize + tsize / 8), kTableSlotsMax));
    if (c->bytes_held + cap * infra_bytes_per_d(ecap, tcap) > c->cfg.mem_budget_bytes) {
        cap = need;
        ecap = emax;
        tcap = tsize;
    }
    const u64 bytes = cap * infra_bytes_per_d(ecap, tcap);
    if (c->bytes_held + bytes > c->cfg.mem_budget_bytes) return EIS_ENOMEM;
    if (hipMalloc(&c->pb.lists, cap * ecap * 8) != hipSuccess ||
        hipMalloc(&c->pb.lres, cap * ecap * 4) != hipSuccess ||
        hipMalloc(&c->pb.tables, cap * tcap * 2) != hipSuccess ||
        hipMalloc(&c->pb.state, cap * sizeof(WindowState)) != hipSuccess ||
        hipMalloc(&c->pb.tasks, cap * kCostBuckets * sizeof(GiantTask)) != hipSuccess) {
        free_infra(c);
        return EIS_ENOMEM;
    }
    c->pb.infra_bytes = bytes;
    c->bytes_held += bytes;
    c->pb.infra_batch_cap = cap;
    c->pb.infra_emax_cap = ecap;
    c->pb.infra_tsize_cap = tcap;
    return EIS_OK;
}

// number of table primes p with p^2 <= dmax
static u32 primes_needed(const eis_ctx *c, u64 dmax)
{
    u64 r = isqrt_host(dmax);
    return (u32)(std::upper_bound(c->primes_host.begin(), c->primes_host.end(),
                                  (u32)std::min<u64>(r, 0xffffffffu)) -
                 c->primes_host.begin());
}

// Dictionary geometry for heights up to dmax: mu_1 is entry scaled_root/16
// (at least the 16th), and the window runs a few entries past it, or (the
// variant with the paper's stride) to 1.5 times its step count.
static void infra_geometry(double scaled_root, u32 variant, u32 &emax, u32 &tsize)
{
    double n = scaled_root / 16.0;
    u32 emain = (u32)std::max(2.0, std::floor(n + 1.0));
    emain = std::max<u32>(emain, 16);
    const u32 want = (variant & kVariantNoConjugate) ? emain + (3 * emain) / 4 + 16 : emain + 16;
    emax = (want + 7) / 8 * 8;  // whole 4-entry chunks of the window walk's write-outs
    if (emax > kEmaxMax) emax = kEmaxMax;
    // whole 8-slot groups (one 16-byte load each) at a load of at most 0.3
    // for the usual count: a lookup then reads a second group for fewer than
    // one key in 300; at most kTableSlotsMax slots
    const u32 count = (variant & kVariantNoConjugate) ? emain + emain / 2 + 4 : emain + 4;
    const u32 groups = (10 * std::min(count, emax) + 23) / 24;
    tsize = 8 * std::min(std::max(groups, 4u), kTableSlotsMax / 8);
}

// the method variant bits of a context's flags
static u32 variant_of(const eis_ctx *c)
{
    return ((c->cfg.flags & EIS_FLAG_NO_CONJUGATE_LOOKUPS) ? kVariantNoConjugate : 0u) |
           ((c->cfg.flags & EIS_FLAG_NO_SMALL_NORM_PRODUCT) ? kVariantNoSmallNorm : 0u);
}

// lower end of tuner bin b: 10^(b/2), rounded up for odd b
static u64 bin_start(int b)
{
    u64 p = 1;
    for (int t = 0; t < b / 2; t++) p *= 10;
    if (b % 2) p = (u64)std::ceil((double)p * 3.1622776601683795);
    return p;
}

// b with bin_start(b) <= d < bin_start(b + 1), at most kTuneBins - 1
static int bin_of(u64 d)
{
    int b = 0;
    while (b < kTuneBins - 1 && d >= bin_start(b + 1)) b++;
    return b;
}

static u32 method_for(const eis_ctx *c, u64 d0)
{
    if (c->cfg.method == EIS_METHOD_INFRA) return 1;
    if (c->cfg.method == EIS_METHOD_BABY) return 0;
    if (c->tuned) return (u32)c->tuned_method[bin_of(d0)];
    return d0 >= c->infra_min_height ? 1 : 0;
}

static double scale_for(const eis_ctx *c, u64 d0)
{
    if (c->cfg.window_scale > 0) return c->cfg.window_scale;
    if (c->tuned) return c->tuned_ws[bin_of(d0)];
    return c->window_scale;
}

static u32 chunk_for(const eis_ctx *c, u64 d0)
{
    if (c->tuned) return c->tuned_chunk[bin_of(d0)];
    return kDefaultWalkChunk;
}

// candidates per pass when a range starting at d0 is cut into passes
static u64 pass_for(const eis_ctx *c, u64 d0)
{
    if (c->tuned) return u64(1) << c->tuned_pass_log2[bin_of(d0)];
    return kPassCandidates;
}

// ---------------------------------------------------------------------------
// one pass
// ---------------------------------------------------------------------------

struct PassPlan {
    u32 nseg = 0, nblocks = 0, np_max = 0, words = 0;
    u64 plain_cand = 0, giant_cand = 0;
    u32 emax = 0, tsize = 0;
    u64 batch = 0;
    u32 nbatches = 0;
    u32 grid_plain = 0, grid_win = 0, grid_giant = 0, grid_fb = 0, grid_tables = 0;
    u64 roff_total = 0;
    u32 walk_chunk = kDefaultWalkChunk;  // that of the highest giant-step segment
    u64 dmax = 0;                        // the largest candidate d of the pass
};

// Whether the walks of the pass may leave the quotient's overshoot test out.
static bool exact_quot(const PassPlan &pl) { return pl.dmax <= kExactQuotMaxD; }

// Fill the pinned segment table and the plan of a pass.
static void plan_pass(eis_ctx *c, const HostSeg *segs, u32 nseg, SegInfo *hs, u64 infra_avail,
                      u64 batch_min, PassPlan &pl)
{
    pl = PassPlan();
    pl.nseg = nseg;
    u32 word = 0, block = 0;
    u64 roff = 0;
    double nmax_giant = 0.0;  // largest wscale * d^(1/4) of the giant-step segments
    u64 dmax_giant = 0;       // start of the highest giant-step segment
    for (u32 s = 0; s < pl.nseg; s++) {
        const HostSeg &h = segs[s];
        SegInfo &g = hs[s];
        g.d0 = h.d0;
        g.n = h.n;
        g.word_off = word;
        g.block_off = block;
        const u64 dlast = h.d0 + 8ull * (h.n - 1);
        if (h.n) pl.dmax = std::max(pl.dmax, dlast);
        g.np = primes_needed(c, dlast);
        g.roff_off = (u32)roff;
        g.method = h.method;
        g.count_slot = h.slot;
        g.wscale = h.wscale;
        g.set = h.set;
        word += (h.n + 31) / 32;
        block += (h.n + kSegCandidates - 1) / kSegCandidates;
        roff += g.np;
        pl.np_max = std::max(pl.np_max, g.np);
        if (h.method) {
            if (pl.giant_cand == 0 || h.d0 > dmax_giant) {
                dmax_giant = h.d0;
                pl.walk_chunk = h.walk_chunk;
            }
            pl.giant_cand += h.n;
            nmax_giant = std::max(nmax_giant, (double)g.wscale * std::pow((double)dlast, 0.25));
        } else {
            pl.plain_cand += h.n;
        }
    }
    pl.words = word;
    pl.nblocks = block;
    pl.roff_total = roff;
    const u64 max_plain = (u64)c->num_cu * c->walk_blocks_per_cu;
    pl.grid_plain = (u32)std::min<u64>((pl.plain_cand + 255) / 256, max_plain);
    pl.grid_fb = (u32)c->num_cu;
    if (pl.giant_cand) {
        infra_geometry(nmax_giant, variant_of(c), pl.emax, pl.tsize);
        const u64 per_d = infra_bytes_per_d(pl.emax, pl.tsize);
        const u64 fit = std::max<u64>(infra_avail / per_d / batch_min * batch_min, batch_min);
        pl.batch = std::min<u64>(pl.giant_cand, fit);
        pl.nbatches = (u32)((pl.giant_cand + pl.batch - 1) / pl.batch);
        const u64 max_win = (u64)c->num_cu * c->window_blocks_per_cu;
        const u64 max_giant = (u64)c->num_cu * c->giant_blocks_per_cu;
        pl.grid_win = (u32)std::max<u64>(1, std::min((pl.batch + 255) / 256, max_win));
        pl.grid_giant = (u32)std::max<u64>(1, std::min((pl.batch + 255) / 256, max_giant));
        // table build: 8 resident blocks per CU (16 KB of LDS each)
        pl.grid_tables = (u32)std::max<u64>(1, std::min((pl.batch + 3) / 4, (u64)c->num_cu * 8));
    }
}

static int collect_pass(eis_ctx *c);
static int add_counters(eis_ctx *c, const PassCounters *h, bool retry);

// Wait for the pass an asynchronous call left running (it may be on another
// stream) before anything of a new call touches the shared buffers; its
// status goes to eis_last_error.
static int settle_pending(eis_ctx *c)
{
    if (!c->uncollected) return EIS_OK;
    HIP_TRY(hipStreamSynchronize(c->pending_stream));
    int prc = collect_pass(c);
    if (prc != EIS_OK && c->async_status == EIS_OK) c->async_status = prc;
    return EIS_OK;
}

// Per-kernel timing: an event pair around one launch, read by collect_pass.
static int kt_begin(eis_ctx *c, hipStream_t st, int kind)
{
    const u32 i = c->kev_used;
    while (c->kev.size() < 2 * (size_t)(i + 1)) {
        hipEvent_t e = nullptr;
        HIP_TRY(hipEventCreate(&e));
        c->kev.push_back(e);
    }
    if (c->kev_kind.size() <= i) c->kev_kind.resize(i + 1);
    c->kev_kind[i] = kind;
    HIP_TRY(hipEventRecord(c->kev[2 * i], st));
    return EIS_OK;
}

static int kt_end(eis_ctx *c, hipStream_t st)
{
    HIP_TRY(hipEventRecord(c->kev[2 * c->kev_used + 1], st));
    c->kev_used++;
    return EIS_OK;
}

// one launch, timed when kt
#define KLAUNCH(kind, expr)                        \
    do {                                           \
        if (kt) {                                  \
            int _r = kt_begin(c, st, (kind));      \
            if (_r != EIS_OK) return _r;           \
        }                                          \
        HIP_TRY(expr);                             \
        if (kt) {                                  \
            int _r = kt_end(c, st);                \
            if (_r != EIS_OK) return _r;           \
        }                                          \
    } while (0)

// Enqueue the launch sequence of a planned pass (after the segment table
// upload).  Captured into graphs by shape.
static int enqueue_pass_body(eis_ctx *c, const PassPlan &pl, const PassBufs &B, hipStream_t st,
                             bool timed)
{
    PassCounters *ctr_plain = B.ctrs, *ctr_giant = B.ctrs + 1, *ctr_fb = B.ctrs + 2,
                 *ctr_fb2 = B.ctrs + 3;
    const bool kt = timed && c->kernel_times;
    HIP_TRY(launch_zero_u32(reinterpret_cast<u32 *>(B.ctrs),
                            kPassCounterSets * sizeof(PassCounters) / 4, st));
    HIP_TRY(launch_zero_u32(B.eis_words, pl.words, st));
    KLAUNCH(EIS_K_PRIME_OFFSETS,
            launch_prime_offsets(c->d_primes, B.segs, pl.nseg, pl.np_max, B.roff, st));
    KLAUNCH(EIS_K_SIEVE, launch_sieve(c->d_primes, B.roff, B.segs, pl.nseg, pl.nblocks,
                                      c->nsmall, c->nsmall_p, B.sq_words, B.list_plain,
                                      ctr_plain,
                                      B.list_giant, ctr_giant, st));
    if (timed) HIP_TRY(hipEventRecord(c->ev_walk0, st));
    WalkParams wp;
    wp.segs = B.segs;
    wp.nseg = pl.nseg;
    wp.eis_words = B.eis_words;
    wp.max_steps = (u32)c->cfg.max_steps_per_d;
    wp.exact_quot = exact_quot(pl) ? 1u : 0u;
    if (pl.plain_cand) {
        wp.list = B.list_plain;
        wp.ctr = ctr_plain;
        KLAUNCH(EIS_K_WALK_PLAIN, launch_walk_baby(wp, pl.grid_plain, st));
    }
    if (pl.giant_cand) {
        InfraParams ip;
        ip.segs = B.segs;
        ip.nseg = pl.nseg;
        ip.list = B.list_giant;
        ip.list_ctr = ctr_giant;
        ip.batch = (u32)pl.batch;
        ip.ctr = ctr_giant;
        ip.win_next = B.q;
        ip.giant_next = B.q + 16;
        ip.fb_list = B.fb_list;
        ip.fb_ctr = ctr_fb;
        ip.state = B.state;
        ip.tasks = B.tasks;
        ip.task_cap = (u32)B.infra_batch_cap;
        ip.gbuckets = B.q + 3 * 16;
        ip.lists = B.lists;
        ip.lres = B.lres;
        ip.tables = B.tables;
        ip.emax = pl.emax;
        ip.tsize = pl.tsize;
        ip.max_steps = (u32)c->cfg.max_steps_per_d;
        ip.max_giants = 1u << 20;
        ip.emain_shift = 0;
        ip.variant = variant_of(c);
        ip.walk_chunk = pl.walk_chunk;
        ip.exact_quot = wp.exact_quot;
        ip.eis_words = B.eis_words;
        for (u32 bi = 0; bi < pl.nbatches; bi++) {
            ip.k0 = (u32)(bi * pl.batch);
            HIP_TRY(launch_zero_u32(B.q, kQueueWords, st));
            KLAUNCH(EIS_K_WALK_WINDOW, launch_walk_window(ip, pl.grid_win, false, st));
            KLAUNCH(EIS_K_BUILD_TABLES, launch_build_tables(ip, pl.grid_tables, false, st));
            KLAUNCH(EIS_K_GIANT_SQUARE, launch_giant_square(ip, false, st));
            KLAUNCH(EIS_K_WALK_GIANT, launch_walk_giant(ip, pl.grid_giant, false, st));
        }
        // The d's handed off, once more with mu_1 kRetryShift distinguished
        // ideals later: a hand-off comes from a composition whose magnitudes
        // pass 2^52 (one of the ideals has a small norm, at heights near
        // 10^12) or from another check, and a different mu_1 gives other
        // giant ideals.  With one batch per pass the hand-offs fit the batch
        // buffers; the plain walk then takes what the retry hands off.  Its
        // kernels exit at once when there is nothing to retry.
        wp.list = B.fb_list;
        wp.ctr = ctr_fb;
        if (pl.nbatches == 1) {
            InfraParams rp = ip;
            rp.list = B.fb_list;
            rp.list_ctr = ctr_fb;
            rp.k0 = 0;
            // its hand-offs go to the plain walk's list, which that walk,
            // earlier on the stream, no longer needs
            rp.fb_list = B.list_plain;
            rp.fb_ctr = ctr_fb2;
            rp.emain_shift = kRetryShift;
            if (kt) {
                int r = kt_begin(c, st, EIS_K_GIANT_RETRY);
                if (r != EIS_OK) return r;
            }
            HIP_TRY(launch_zero_u32(B.q, kQueueWords, st));
            HIP_TRY(launch_walk_window(rp, c->num_cu, true, st));
            HIP_TRY(launch_build_tables(rp, c->num_cu, true, st));
            HIP_TRY(launch_giant_square(rp, true, st));
            HIP_TRY(launch_walk_giant(rp, c->num_cu, true, st));
            if (kt) {
                int r = kt_end(c, st);
                if (r != EIS_OK) return r;
            }
            wp.list = B.list_plain;
            wp.ctr = ctr_fb2;
        }
        // the rest: the plain walk, exact for all d
        KLAUNCH(EIS_K_WALK_HANDOFF, launch_walk_baby(wp, pl.grid_fb, st));
    }
    if (timed) HIP_TRY(hipEventRecord(c->ev_walk1, st));
    KLAUNCH(EIS_K_POPCOUNT,
            launch_popcount_segs(B.sq_words, B.eis_words, B.segs, pl.nseg,
                                 (u32)((kPassCandidates + 31) / 32), B.counts, st));
    return EIS_OK;
}

static std::vector<u64> plan_key(const eis_ctx *c, const PassPlan &pl)
{
    return {pl.nseg, pl.nblocks, pl.np_max, pl.words, pl.plain_cand ? 1ull : 0ull,
            pl.giant_cand ? 1ull : 0ull, pl.emax, pl.tsize, pl.batch, pl.nbatches, pl.grid_plain,
            pl.grid_win, pl.grid_giant, pl.grid_fb, c->cfg.max_steps_per_d, pl.walk_chunk,
            exact_quot(pl) ? 1ull : 0ull};
}

// Enqueue a planned pass on buffer set B, whose segment table is in place:
// a graph replay when `graph` (captured on first use, keyed by the pass
// shape and the buffer set), else launch by launch (with the per-kernel
// events when `timed`).
static int launch_pass(eis_ctx *c, const PassPlan &pl, const PassBufs &B, hipStream_t st,
                       bool graph, bool timed)
{
    if (graph && c->use_graphs && st == c->stream) {
        std::vector<u64> key = plan_key(c, pl);
        key.push_back((u64)reinterpret_cast<uintptr_t>(B.ctrs));
        auto it = c->graphs.find(key);
        if (it == c->graphs.end()) {
            // capture on an idle stream (a server pass may still be in flight)
            HIP_TRY(hipStreamSynchronize(st));
            hipGraph_t g = nullptr;
            HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
            int brc = enqueue_pass_body(c, pl, B, st, false);
            hipError_t e = hipStreamEndCapture(st, &g);
            if (brc != EIS_OK) {
                if (g) (void)hipGraphDestroy(g);
                return brc;
            }
            if (e != hipSuccess) return hip_status(e);
            hipGraphExec_t ge = nullptr;
            e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) return hip_status(e);
            it = c->graphs.emplace(key, ge).first;
        }
        // a replay is timed as a whole (the walk events are not in the graph)
        HIP_TRY(hipEventRecord(c->ev_walk0, st));
        HIP_TRY(hipGraphLaunch(it->second, st));
        HIP_TRY(hipEventRecord(c->ev_walk1, st));
        return EIS_OK;
    }
    return enqueue_pass_body(c, pl, B, st, timed);
}

// Record that a pass is in flight on `st` with counters `ctrs`.
static void mark_pending(eis_ctx *c, const PassPlan &pl, PassCounters *ctrs, hipStream_t st)
{
    c->uncollected = true;
    c->pending_stream = st;
    c->pending_ctrs = ctrs;
    c->pending_retry = pl.giant_cand && pl.nbatches == 1;
    const u64 launches = 7 + (pl.giant_cand ? 1 + 5ull * pl.nbatches + (pl.nbatches == 1 ? 5 : 0) : 0);
    std::lock_guard<std::mutex> lk(c->stats_mu);
    c->stats.launches += launches;
}

// Run one pass of segments on the context's buffers (counts are accumulated
// into c->pb.counts, which the caller zeroes).  Asynchronous: the counters
// are read by collect_pass once the stream has finished.
// Plan a pass on the context's buffers and allocate what it needs (done by
// run_pass; the tuner calls it ahead, so that no allocation falls inside a
// timed region).
static int prepare_pass(eis_ctx *c, const std::vector<HostSeg> &segs, PassPlan &pl)
{
    int rc = settle_pending(c);
    if (rc != EIS_OK) return rc;
    rc = ensure_pass_buffers(c);
    if (rc != EIS_OK) return rc;
    const u64 held = c->bytes_held - c->pb.infra_bytes;  // other buffers of the context
    const u64 avail = c->cfg.mem_budget_bytes > held ? c->cfg.mem_budget_bytes - held : 0;
    plan_pass(c, segs.data(), (u32)segs.size(), c->pb.h_segs, avail, kInfraBatchMin, pl);
    rc = ensure_roff(c, std::max<u64>(pl.roff_total, 1));
    if (rc != EIS_OK) return rc;
    if (pl.giant_cand) {
        rc = ensure_infra(c, pl.batch, pl.emax, pl.tsize);
        if (rc != EIS_OK) return rc;
    }
    return EIS_OK;
}

static int run_pass(eis_ctx *c, const std::vector<HostSeg> &segs, hipStream_t st, bool graph,
                    PassPlan &pl)
{
    (void)hipGetLastError();  // launch checks below must not see an older error
    c->kev_used = 0;
    int rc = prepare_pass(c, segs, pl);
    if (rc != EIS_OK) return rc;
    HIP_TRY(hipMemcpyAsync(c->pb.segs, c->pb.h_segs, pl.nseg * sizeof(SegInfo), hipMemcpyHostToDevice, st));
    rc = launch_pass(c, pl, c->pb, st, graph, true);
    if (rc != EIS_OK) return rc;
    mark_pending(c, pl, c->pb.ctrs, st);
    return EIS_OK;
}

// Read the pass counters after the stream has finished the pass.
// Add the counters of a finished pass (at `ctrs`; `retry`: it had the retry
// round) to the statistics; EIS_EINTERNAL if a walk of it overran its step
// budget.  With `timed`, the pass's event pairs are read too.
static int collect_counters(eis_ctx *c, PassCounters *ctrs, bool retry, bool timed)
{
    PassCounters h[kPassCounterSets];
    if (hipMemcpy(h, ctrs, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess) return EIS_EDEVICE;
    if (!timed) {
        std::lock_guard<std::mutex> lk(c->stats_mu);
        return add_counters(c, h, retry);
    }
    float wms = 0.f;
    bool have_ms = hipEventElapsedTime(&wms, c->ev_walk0, c->ev_walk1) == hipSuccess;
    if (!have_ms) (void)hipGetLastError();
    std::vector<float> kms(c->kev_used, 0.f);
    bool have_kms = true;
    for (u32 i = 0; i < c->kev_used && have_kms; i++)
        have_kms = hipEventElapsedTime(&kms[i], c->kev[2 * i], c->kev[2 * i + 1]) == hipSuccess;
    if (!have_kms) (void)hipGetLastError();
    std::lock_guard<std::mutex> lk(c->stats_mu);
    if (have_ms) c->stats.last_walk_ms = wms;
    if (have_kms) {
        for (u32 i = 0; i < c->kev_used; i++) {
            c->stats.kernel_launches[c->kev_kind[i]]++;
            c->stats.kernel_ms[c->kev_kind[i]] += kms[i];
        }
    }
    c->kev_used = 0;
    return add_counters(c, h, retry);
}

// Read the pass counters after the stream has finished the pass.
static int collect_pass(eis_ctx *c)
{
    c->uncollected = false;
    return collect_counters(c, c->pending_ctrs, c->pending_retry, true);
}

// The counter sets of one pass into the statistics (stats_mu held).
static int add_counters(eis_ctx *c, const PassCounters *h, bool retry)
{
    c->stats.discriminants += (u64)h[0].list_len + h[1].list_len;
    // the hand-off walk ran on the retry round's list when there was one
    const PassCounters &hf = retry ? h[3] : h[2];
    c->stats.baby_steps += h[0].baby_steps + h[1].baby_steps + h[1].chunk_steps + hf.baby_steps;
    c->stats.kernel_steps[EIS_K_WALK_PLAIN] += h[0].baby_steps;
    c->stats.kernel_steps[EIS_K_WALK_WINDOW] += h[1].baby_steps;
    c->stats.kernel_steps[EIS_K_WALK_GIANT] += h[1].chunk_steps;
    c->stats.kernel_steps[EIS_K_WALK_HANDOFF] += hf.baby_steps;
    c->stats.giant_steps += h[1].giant_steps;
    c->stats.giant_compositions += h[1].giant_comps;
    c->stats.giant_euclid_steps += h[1].giant_euclid;
    c->stats.giant_xgcd_steps += h[1].giant_xgcd;
    c->stats.giant_reduce_steps += h[1].giant_reduce;
    c->stats.giant_gcd_branches += h[1].giant_gcd_branch;
    c->stats.giant_lookups += h[1].giant_lookups;
    c->stats.window_entries += h[1].window_entries;
    c->stats.giant_compose_phases += h[1].giant_phases[0];
    c->stats.giant_compose_lanes += h[1].giant_lanes[0];
    c->stats.giant_walk_phases += h[1].giant_phases[1];
    c->stats.giant_walk_lanes += h[1].giant_lanes[1];
    c->stats.refills += h[0].refills + h[1].refills + hf.refills;
    c->stats.fallbacks += hf.list_len;
    if (retry) c->stats.giant_retries += h[2].list_len;
    return (h[0].err_count | h[1].err_count | hf.err_count) ? EIS_EINTERNAL : EIS_OK;
}

static int check_range(uint64_t a, uint64_t b)
{
    if (a >= b) return EIS_OK;
    if (b > EIS_MAX_D) return EIS_ERANGE;
    return EIS_OK;
}

// Core driver of one range: one pass per piece of at most kPassCandidates
// candidates; bitmaps go to host (h_*) or device (d_*) byte buffers.
static int run_range(eis_ctx *c, uint64_t a, uint64_t b, uint8_t *h_sq, uint8_t *h_eis,
                     uint8_t *d_sq, uint8_t *d_eis, uint64_t *n_sq, uint64_t *n_eis,
                     unsigned long long *d_counts_out, hipStream_t st, bool sync,
                     u32 set = kSetSquarefree)
{
    if (hipSetDevice(c->device) != hipSuccess) return EIS_EDEVICE;
    int rc = settle_pending(c);
    if (rc == EIS_OK) rc = ensure_counts(c, 1);
    if (rc != EIS_OK) return rc;
    if (st != c->stream) {
        // the shared pass buffers may still be in use by passes on the
        // context's own stream (the server's): order this stream after them
        if (!c->ev_order) HIP_TRY(hipEventCreate(&c->ev_order));
        HIP_TRY(hipEventRecord(c->ev_order, c->stream));
        HIP_TRY(hipStreamWaitEvent(st, c->ev_order, 0));
    }
    const u64 n = eis_num_candidates(a, b);
    const u64 d0 = eis_first_candidate(a);
    HIP_TRY(launch_zero_u32(reinterpret_cast<u32 *>(c->pb.counts), 4, st));
    HIP_TRY(hipEventRecord(c->ev_all0, st));
    int status = EIS_OK;
    // passes of the tuned size for the range's height (a multiple of 2^22
    // candidates, so that every pass starts on a bitmap byte)
    const u64 ps = std::min<u64>(std::max<u64>(pass_for(c, d0), u64(1) << 22), kPassCandidates);
    for (u64 off = 0; off < n; off += ps) {
        const u32 pn = (u32)std::min<u64>(ps, n - off);
        std::vector<HostSeg> segs(1);
        segs[0].d0 = d0 + 8 * off;
        segs[0].n = pn;
        segs[0].slot = 0;
        segs[0].method = method_for(c, segs[0].d0);
        segs[0].wscale = (float)scale_for(c, segs[0].d0);
        segs[0].walk_chunk = chunk_for(c, segs[0].d0);
        segs[0].dst_bit = off;
        segs[0].set = set;
        PassPlan pl;
        rc = run_pass(c, segs, st, false, pl);
        if (rc != EIS_OK) return rc;
        const size_t bytes = (pn + 7) / 8;
        const size_t boff = off / 8;
        if (h_sq) HIP_TRY(hipMemcpyAsync(h_sq + boff, c->pb.sq_words, bytes, hipMemcpyDeviceToHost, st));
        if (h_eis) HIP_TRY(hipMemcpyAsync(h_eis + boff, c->pb.eis_words, bytes, hipMemcpyDeviceToHost, st));
        if (d_sq) HIP_TRY(hipMemcpyAsync(d_sq + boff, c->pb.sq_words, bytes, hipMemcpyDeviceToDevice, st));
        if (d_eis) HIP_TRY(hipMemcpyAsync(d_eis + boff, c->pb.eis_words, bytes, hipMemcpyDeviceToDevice, st));
        if (sync || off + ps < n) {
            // the pass buffers are reused: wait before the next pass
            HIP_TRY(hipStreamSynchronize(st));
            int prc = collect_pass(c);
            if (prc != EIS_OK) status = prc;
        }
    }
    if (d_counts_out) {
        HIP_TRY(hipMemcpyAsync(d_counts_out, c->pb.counts, 2 * sizeof(unsigned long long),
                               hipMemcpyDeviceToDevice, st));
    }
    HIP_TRY(hipEventRecord(c->ev_all1, st));
    if (sync) {
        HIP_TRY(hipStreamSynchronize(st));
        unsigned long long hc[2] = {0, 0};
        HIP_TRY(hipMemcpy(hc, c->pb.counts, sizeof(hc), hipMemcpyDeviceToHost));
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, c->ev_all0, c->ev_all1) == hipSuccess) {
            std::lock_guard<std::mutex> lk(c->stats_mu);
            c->stats.last_total_ms = ms;
        } else {
            (void)hipGetLastError();
        }
        if (status != EIS_OK) return status;
        if (n_sq) *n_sq = hc[0];
        if (n_eis) *n_eis = hc[1];
    }
    return status;
}

extern "C" int eis_count_set(eis_ctx *c, int set, uint64_t a, uint64_t b, uint64_t *n_set,
                             uint64_t *n_eis)
{
    if (!c || (set != EIS_SET_SQUAREFREE && set != EIS_SET_PRIME)) return EIS_EINVAL;
    int rc = check_range(a, b);
    if (rc != EIS_OK) return rc;
    if (eis_num_candidates(a, b) == 0) {
        if (n_set) *n_set = 0;
        if (n_eis) *n_eis = 0;
        return EIS_OK;
    }
    std::lock_guard<std::mutex> g(c->gpu_mu);
    return run_range(c, a, b, nullptr, nullptr, nullptr, nullptr, n_set, n_eis, nullptr,
                     c->stream, true, (u32)set);
}

extern "C" int eis_count(eis_ctx *c, uint64_t a, uint64_t b, uint64_t *n_sqfree, uint64_t *n_eis)
{
    return eis_count_set(c, EIS_SET_SQUAREFREE, a, b, n_sqfree, n_eis);
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
    if (n == 0) {
        if (n_sqfree) *n_sqfree = 0;
        if (n_eis) *n_eis = 0;
        return EIS_OK;
    }
    // stage into temporaries so that an error leaves the caller's buffers untouched
    std::vector<uint8_t> tsq(sqfree_bits ? (n + 7) / 8 : 0), teis(eis_bits ? (n + 7) / 8 : 0);
    u64 cs = 0, ce = 0;
    {
        std::lock_guard<std::mutex> g(c->gpu_mu);
        rc = run_range(c, a, b, sqfree_bits ? tsq.data() : nullptr,
                       eis_bits ? teis.data() : nullptr, nullptr, nullptr, &cs, &ce, nullptr,
                       c->stream, true);
    }
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
    std::lock_guard<std::mutex> g(c->gpu_mu);
    if (hipSetDevice(c->device) != hipSuccess) return EIS_EDEVICE;
    if (n == 0) {
        if (d_counts2) HIP_TRY(launch_zero_u32(reinterpret_cast<u32 *>(d_counts2), 4, st));
        return EIS_OK;
    }
    rc = run_range(c, a, b, nullptr, nullptr, reinterpret_cast<uint8_t *>(d_sqfree_bits),
                   reinterpret_cast<uint8_t *>(d_eis_bits), nullptr, nullptr,
                   reinterpret_cast<unsigned long long *>(d_counts2), st, false);
    if (rc == EIS_EINTERNAL) c->async_status = rc;
    return rc;
}

// Buffers of one pass carved out of the no-allocation scratch at `base`:
// the fixed part for a single segment of at most kNoAllocMaxCandidates
// candidates, then the giant-step scratch of the planned batch.  Returns the
// offset of the giant-step part, or the first byte past the end.
static u64 carve_fixed(eis_ctx *c, unsigned char *base, PassBufs &B)
{
    u64 off = 0;
    auto take = [&](u64 bytes) {
        unsigned char *p = base + off;
        off = (off + bytes + 255) / 256 * 256;
        return p;
    };
    const u64 words = kNoAllocMaxCandidates / 32 + 1;
    B = PassBufs();
    B.segs = reinterpret_cast<SegInfo *>(take(sizeof(SegInfo)));
    B.ctrs = reinterpret_cast<PassCounters *>(take(kPassCounterSets * sizeof(PassCounters)));
    B.q = reinterpret_cast<u32 *>(take(kQueueWords * 4));
    B.counts = reinterpret_cast<unsigned long long *>(take(2 * sizeof(unsigned long long)));
    B.counts_cap = 1;
    B.roff_cap = c->primes_host.size();
    B.roff = reinterpret_cast<u64 *>(take(B.roff_cap * sizeof(u64)));
    B.sq_words = reinterpret_cast<u32 *>(take(words * 4));
    B.eis_words = reinterpret_cast<u32 *>(take(words * 4));
    B.list_plain = reinterpret_cast<u32 *>(take(kNoAllocMaxCandidates * 4));
    B.list_giant = reinterpret_cast<u32 *>(take(kNoAllocMaxCandidates * 4));
    B.fb_list = reinterpret_cast<u32 *>(take(kNoAllocMaxCandidates * 4));
    B.ready = true;
    return off;
}

static bool carve_infra(unsigned char *base, u64 off, const PassPlan &pl, PassBufs &B)
{
    const u64 cap = (pl.batch + 63) / 64 * 64;
    const u64 sizes[5] = {cap * pl.emax * 8, cap * pl.emax * 4, cap * pl.tsize * 2,
                          cap * sizeof(WindowState), cap * kCostBuckets * sizeof(GiantTask)};
    unsigned char *p[5];
    for (int k = 0; k < 5; k++) {
        p[k] = base + off;
        off = (off + sizes[k] + 255) / 256 * 256;
    }
    if (off > kNoAllocScratchBytes) return false;
    B.lists = reinterpret_cast<unsigned long long *>(p[0]);
    B.lres = reinterpret_cast<u32 *>(p[1]);
    B.tables = reinterpret_cast<u16 *>(p[2]);
    B.state = reinterpret_cast<WindowState *>(p[3]);
    B.tasks = reinterpret_cast<GiantTask *>(p[4]);
    B.infra_batch_cap = cap;
    B.infra_emax_cap = pl.emax;
    B.infra_tsize_cap = pl.tsize;
    return true;
}

extern "C" int eis_classify_async_noalloc(eis_ctx *c, uint64_t a, uint64_t b,
                                          void *d_sqfree_bits, void *d_eis_bits,
                                          uint64_t *d_counts2, void *hip_stream)
{
    if (!c) return EIS_EINVAL;
    int rc = check_range(a, b);
    if (rc != EIS_OK) return rc;
    const u64 n = eis_num_candidates(a, b);
    if (n > kNoAllocMaxCandidates) return EIS_ENOMEM;
    hipStream_t st = hip_stream ? reinterpret_cast<hipStream_t>(hip_stream) : c->stream;
    std::lock_guard<std::mutex> g(c->gpu_mu);
    if (hipSetDevice(c->device) != hipSuccess) return EIS_EDEVICE;
    if (n == 0) {
        if (d_counts2) HIP_TRY(launch_zero_u32(reinterpret_cast<u32 *>(d_counts2), 4, st));
        return EIS_OK;
    }
    unsigned char *base = static_cast<unsigned char *>(noalloc_scratch(c->device));
    if (!base) return EIS_EDEVICE;
    (void)hipGetLastError();  // launch checks below must not see an older error
    rc = settle_pending(c);
    if (rc != EIS_OK) return rc;
    c->kev_used = 0;
    PassBufs B;
    const u64 infra_off = carve_fixed(c, base, B);
    HostSeg h;
    h.d0 = eis_first_candidate(a);
    h.n = (u32)n;
    h.slot = 0;
    h.method = method_for(c, h.d0);
    h.wscale = (float)scale_for(c, h.d0);
    h.walk_chunk = chunk_for(c, h.d0);
    h.dst_bit = 0;
    SegInfo hs;
    PassPlan pl;
    // the giant-step part: five arrays, each rounded up to 256 bytes
    plan_pass(c, &h, 1, &hs, kNoAllocScratchBytes - infra_off - 5 * 256, 64, pl);
    if (pl.roff_total > B.roff_cap) return EIS_EINTERNAL;
    if (pl.giant_cand && !carve_infra(base, infra_off, pl, B)) return EIS_ENOMEM;
    HIP_TRY(launch_store_seg(hs, B.segs, st));
    HIP_TRY(launch_zero_u32(reinterpret_cast<u32 *>(B.counts), 4, st));
    rc = launch_pass(c, pl, B, st, false, false);
    if (rc != EIS_OK) return rc;
    const size_t bytes = (n + 7) / 8;
    if (d_sqfree_bits)
        HIP_TRY(hipMemcpyAsync(d_sqfree_bits, B.sq_words, bytes, hipMemcpyDeviceToDevice, st));
    if (d_eis_bits)
        HIP_TRY(hipMemcpyAsync(d_eis_bits, B.eis_words, bytes, hipMemcpyDeviceToDevice, st));
    if (d_counts2)
        HIP_TRY(hipMemcpyAsync(d_counts2, B.counts, 2 * sizeof(unsigned long long),
                               hipMemcpyDeviceToDevice, st));
    mark_pending(c, pl, B.ctrs, st);
    return EIS_OK;
}

extern "C" int eis_last_error(eis_ctx *c)
{
    if (!c) return EIS_EINVAL;
    std::lock_guard<std::mutex> g(c->gpu_mu);
    if (hipSetDevice(c->device) != hipSuccess) return EIS_EDEVICE;
    int rc = EIS_OK;
    if (c->uncollected) {
        HIP_TRY(hipStreamSynchronize(c->pending_stream));
        rc = collect_pass(c);
    }
    if (rc == EIS_OK) rc = c->async_status;
    c->async_status = EIS_OK;
    return rc;
}

// ---------------------------------------------------------------------------
// batched counts
// ---------------------------------------------------------------------------

// Cut ranges into pieces of at most kPassCandidates candidates, order them
// by estimated cost (height first: the walks of high d are the long ones, so
// they start first and the tail of the persistent launch is short), and pack
// them into passes of at most kMaxSegments pieces and kPassCandidates
// candidates.
static void pack_passes(eis_ctx *c, const std::vector<std::tuple<u64, u64, u32>> &ranges,
                        std::vector<std::vector<HostSeg>> &passes, u32 set = kSetSquarefree)
{
    std::vector<HostSeg> pieces;
    for (const auto &r : ranges) {
        const u64 a = std::get<0>(r), b = std::get<1>(r);
        const u32 slot = std::get<2>(r);
        const u64 n = eis_num_candidates(a, b);
        const u64 d0 = eis_first_candidate(a);
        for (u64 off = 0; off < n; off += kPassCandidates) {
            HostSeg h;
            h.d0 = d0 + 8 * off;
            h.n = (u32)std::min<u64>(kPassCandidates, n - off);
            h.slot = slot;
            h.method = method_for(c, h.d0);
            h.wscale = (float)scale_for(c, h.d0);
            h.walk_chunk = chunk_for(c, h.d0);
            h.dst_bit = off;
            h.set = set;
            pieces.push_back(h);
        }
    }
    std::sort(pieces.begin(), pieces.end(), [](const HostSeg &x, const HostSeg &y) {
        return x.d0 > y.d0;
    });
    std::vector<HostSeg> cur;
    u64 cand = 0;
    for (const HostSeg &h : pieces) {
        // a segment's bitmap starts on a word: count its padding too
        const u64 cost = (h.n + 31) / 32 * 32;
        if (!cur.empty() && (cur.size() == kMaxSegments || cand + cost > kPassCandidates)) {
            passes.push_back(cur);
            cur.clear();
            cand = 0;
        }
        cur.push_back(h);
        cand += cost;
    }
    if (!cur.empty()) passes.push_back(cur);
}

extern "C" int eis_count_batch_set(eis_ctx *c, int set, const uint64_t *a, const uint64_t *b,
                                   size_t n, uint64_t *n_set, uint64_t *n_eis)
{
    if (!c || (n && (!a || !b))) return EIS_EINVAL;
    if (set != EIS_SET_SQUAREFREE && set != EIS_SET_PRIME) return EIS_EINVAL;
    for (size_t k = 0; k < n; k++) {
        int rc = check_range(a[k], b[k]);
        if (rc != EIS_OK) return rc;
    }
    std::vector<std::tuple<u64, u64, u32>> ranges;
    for (size_t k = 0; k < n; k++)
        if (eis_num_candidates(a[k], b[k])) ranges.emplace_back(a[k], b[k], (u32)k);
    std::vector<std::vector<HostSeg>> passes;
    std::lock_guard<std::mutex> g(c->gpu_mu);
    if (hipSetDevice(c->device) != hipSuccess) return EIS_EDEVICE;
    pack_passes(c, ranges, passes, (u32)set);
    int rc = settle_pending(c);
    if (rc == EIS_OK) rc = ensure_counts(c, std::max<u64>(n, 1));
    if (rc != EIS_OK) return rc;
    hipStream_t st = c->stream;
    HIP_TRY(launch_zero_u32(reinterpret_cast<u32 *>(c->pb.counts), 4 * std::max<u64>(n, 1), st));
    HIP_TRY(hipEventRecord(c->ev_all0, st));
    int status = EIS_OK;
    for (const auto &segs : passes) {
        PassPlan pl;
        rc = run_pass(c, segs, st, true, pl);
        if (rc != EIS_OK) return rc;
        HIP_TRY(hipStreamSynchronize(st));
        int prc = collect_pass(c);
        if (prc != EIS_OK) status = prc;
    }
    HIP_TRY(hipEventRecord(c->ev_all1, st));
    if (n) {
        HIP_TRY(hipMemcpyAsync(c->h_counts, c->pb.counts, 2 * n * sizeof(unsigned long long),
                               hipMemcpyDeviceToHost, st));
    }
    HIP_TRY(hipStreamSynchronize(st));
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->ev_all0, c->ev_all1) == hipSuccess) {
        std::lock_guard<std::mutex> lk(c->stats_mu);
        c->stats.last_total_ms = ms;
    } else {
        (void)hipGetLastError();
    }
    if (status != EIS_OK) return status;
    for (size_t k = 0; k < n; k++) {
        if (n_set) n_set[k] = c->h_counts[2 * k];
        if (n_eis) n_eis[k] = c->h_counts[2 * k + 1];
    }
    return EIS_OK;
}

extern "C" int eis_count_batch(eis_ctx *c, const uint64_t *a, const uint64_t *b, size_t n,
                               uint64_t *n_sqfree, uint64_t *n_eis)
{
    return eis_count_batch_set(c, EIS_SET_SQUAREFREE, a, b, n, n_sqfree, n_eis);
}

// ---------------------------------------------------------------------------
// serving: continuous batching of range-count requests
// ---------------------------------------------------------------------------
//
// A server thread runs passes back to back.  Each pass takes, in arrival
// order, the next chunk (at most kServeChunk candidates) of every admitted
// request, up to the pass's capacity; a request finishes when its last chunk
// has been through a pass.  Requests that arrive while a pass runs join the
// next one, next to the remaining chunks of the earlier ones.  Two passes
// are in flight at a time (each with its own counters and host staging):
// the server enqueues pass k+1 before it waits for pass k, so the device
// does not idle while the host plans.
//
// Admission is by slots and by device memory.  The plain walk keeps no
// per-d state beyond the fixed pass buffers; a chunk at a height that takes
// giant steps needs the lists, tables, window records and tasks of its
// candidates (chunk_footprint).  A request reserves its first chunk's
// footprint against the serving budget (the context's budget less the fixed
// buffers) while it is in the arrival order: eis_submit refuses it with
// EIS_EBUSY while the admitted requests hold too much of the budget, and
// with EIS_ENOMEM if it could not fit even alone.

// Device bytes of giant-step scratch that n candidates from d0 hold while
// their pass runs (0 at heights the plain walk takes).
static u64 chunk_footprint(const eis_ctx *c, u64 d0, u64 n)
{
    if (n == 0 || !method_for(c, d0)) return 0;
    const u64 dlast = d0 + 8 * (n - 1);
    u32 emax = 0, tsize = 0;
    infra_geometry((double)(float)scale_for(c, d0) * std::pow((double)dlast, 0.25), variant_of(c), emax,
                   tsize);
    return n * infra_bytes_per_d(emax, tsize);
}

// The fixed buffers of serving and the two flights (gpu_mu held).
static int ensure_flights(eis_ctx *c)
{
    if (c->flights_ready) return EIS_OK;
    int rc = ensure_pass_buffers(c);
    if (rc == EIS_OK) rc = ensure_roff(c, std::max<u64>(c->primes_host.size(), 1));
    if (rc != EIS_OK) return rc;
    const u64 per = kPassCounterSets * sizeof(PassCounters) + 2ull * kMaxSegments * 8;
    if (c->bytes_held + 2 * per > c->cfg.mem_budget_bytes) return EIS_ENOMEM;
    for (Flight &f : c->flights) {
        if (hipMalloc(&f.ctrs, kPassCounterSets * sizeof(PassCounters)) != hipSuccess ||
            hipMalloc(&f.counts, 2ull * kMaxSegments * 8) != hipSuccess ||
            hipHostMalloc(reinterpret_cast<void **>(&f.h_segs), kMaxSegments * sizeof(SegInfo),
                          hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc(reinterpret_cast<void **>(&f.h_counts), 2ull * kMaxSegments * 8,
                          hipHostMallocDefault) != hipSuccess)
            return EIS_ENOMEM;
        if (hipEventCreate(&f.done) != hipSuccess) return EIS_EDEVICE;
    }
    c->bytes_held += 2 * per;
    const u64 fixed = c->bytes_held - c->pb.infra_bytes;
    c->serve_budget = c->cfg.mem_budget_bytes > fixed ? c->cfg.mem_budget_bytes - fixed : 0;
    c->flights_ready = true;
    std::lock_guard<std::mutex> lk(c->stats_mu);
    c->stats.serve_bytes_budget = c->serve_budget;
    return EIS_OK;
}

// Enqueue one pass of the server on flight f (gpu_mu held).
static int enqueue_flight(eis_ctx *c, Flight &f, const std::vector<HostSeg> &segs)
{
    (void)hipGetLastError();  // launch checks below must not see an older error
    int rc = settle_pending(c);
    if (rc != EIS_OK) return rc;
    hipStream_t st = c->stream;
    const u64 held = c->bytes_held - c->pb.infra_bytes;
    const u64 avail = c->cfg.mem_budget_bytes > held ? c->cfg.mem_budget_bytes - held : 0;
    PassPlan pl;
    plan_pass(c, segs.data(), (u32)segs.size(), f.h_segs, avail, kInfraBatchMin, pl);
    rc = ensure_roff(c, std::max<u64>(pl.roff_total, 1));
    if (rc == EIS_OK && pl.giant_cand) rc = ensure_infra(c, pl.batch, pl.emax, pl.tsize);
    if (rc != EIS_OK) return rc;
    PassBufs B = c->pb;
    B.ctrs = f.ctrs;
    B.counts = f.counts;
    B.counts_cap = kMaxSegments;
    HIP_TRY(hipMemcpyAsync(B.segs, f.h_segs, pl.nseg * sizeof(SegInfo), hipMemcpyHostToDevice, st));
    HIP_TRY(launch_zero_u32(reinterpret_cast<u32 *>(f.counts), 4ull * pl.nseg, st));
    rc = launch_pass(c, pl, B, st, true, false);
    if (rc != EIS_OK) return rc;
    HIP_TRY(hipMemcpyAsync(f.h_counts, f.counts, 2ull * pl.nseg * 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipEventRecord(f.done, st));
    f.retry = pl.giant_cand && pl.nbatches == 1;
    f.busy = true;
    f.seq = ++c->flight_seq;
    const u64 launches = 7 + (pl.giant_cand ? 1 + 5ull * pl.nbatches + (pl.nbatches == 1 ? 5 : 0) : 0);
    std::lock_guard<std::mutex> lk(c->stats_mu);
    c->stats.launches += launches;
    return EIS_OK;
}

// Hand the counts of a finished pass (or its error) to its requests and
// retire what is finished or cancelled (smu taken here).
static void finish_parts(eis_ctx *c, const std::vector<std::pair<u64, u64>> &parts,
                         const unsigned long long *h_counts, int rc)
{
    {
        std::lock_guard<std::mutex> lk(c->smu);
        for (size_t s = 0; s < parts.size(); s++) {
            auto it = c->reqs.find(parts[s].first);
            if (it == c->reqs.end()) continue;
            Request &r = it->second;
            if (rc != EIS_OK) {
                r.status = rc;
                r.finished = true;
                continue;
            }
            r.n_sq += h_counts[2 * s];
            r.n_eis += h_counts[2 * s + 1];
            r.completed += parts[s].second;
            if (r.completed >= r.ncand) r.finished = true;
        }
        // retire finished and cancelled requests from the arrival order, and
        // release their device-memory reservations
        std::deque<u64> keep;
        for (u64 t : c->order) {
            Request &r = c->reqs[t];
            if (r.finished || (r.cancelled && r.completed >= r.dispatched)) {
                if (!r.finished) r.finished = true;
                c->serve_reserved -= r.reserved;
                r.reserved = 0;
                std::lock_guard<std::mutex> sl(c->stats_mu);
                if (r.status == EIS_OK && !r.cancelled) c->stats.requests_done++;
                c->stats.serve_bytes_reserved = c->serve_reserved;
            } else {
                keep.push_back(t);
            }
        }
        c->order.swap(keep);
    }
    c->dcv.notify_all();
}

// Wait for flight f's pass and hand out its results.
static void collect_flight(eis_ctx *c, Flight &f)
{
    int rc = (hipEventSynchronize(f.done) == hipSuccess) ? EIS_OK : EIS_EDEVICE;
    if (rc == EIS_OK) rc = collect_counters(c, f.ctrs, f.retry, false);
    f.busy = false;
    finish_parts(c, f.parts, f.h_counts, rc);
    f.parts.clear();
}

static void server_loop(eis_ctx *c)
{
    (void)hipSetDevice(c->device);
    int cur = 0;  // the flight the next pass goes to
    for (;;) {
        std::vector<HostSeg> segs;
        std::vector<std::pair<u64, u64>> parts;  // (ticket, candidates) per segment
        bool stop = false;
        {
            std::unique_lock<std::mutex> lk(c->smu);
            auto has_work = [&] {
                for (u64 t : c->order) {
                    const Request &r = c->reqs[t];
                    if (!r.cancelled && r.dispatched < r.ncand) return true;
                }
                return false;
            };
            const bool in_flight = c->flights[0].busy || c->flights[1].busy;
            if (!in_flight) c->scv.wait(lk, [&] { return c->stop || has_work(); });
            stop = c->stop;
            // With a pass in flight, the next one is planned at once only
            // when at least half a pass of work is waiting: a small pass
            // queued behind a running one would hold up the requests that
            // arrive meanwhile (they would wait for both), and under light
            // load the device has no backlog to keep it busy anyway.
            bool plan = !stop;
            if (plan && in_flight) {
                u64 waiting = 0;
                for (u64 t : c->order) {
                    const Request &r = c->reqs[t];
                    if (!r.cancelled) waiting += r.ncand - r.dispatched;
                }
                plan = waiting >= kPassCandidates / 2;
            }
            u64 cand = 0;
            for (u64 t : plan ? c->order : std::deque<u64>()) {
                Request &r = c->reqs[t];
                if (r.cancelled || r.dispatched >= r.ncand) continue;
                if (segs.size() == kMaxSegments) break;
                u64 take = std::min<u64>(r.ncand - r.dispatched, kServeChunk);
                const u64 room = kPassCandidates - cand;
                if (room < 64) break;
                take = std::min<u64>(take, room / 32 * 32);
                HostSeg h;
                h.d0 = r.d0 + 8 * r.dispatched;
                h.n = (u32)take;
                h.slot = (u32)segs.size();
                h.method = method_for(c, h.d0);
                h.wscale = (float)scale_for(c, h.d0);
                h.walk_chunk = chunk_for(c, h.d0);
                h.dst_bit = 0;
                segs.push_back(h);
                parts.emplace_back(t, take);
                r.dispatched += take;
                cand += (take + 31) / 32 * 32;
            }
        }
        if (stop) {
            for (Flight &f : c->flights)
                if (f.busy) {
                    (void)hipEventSynchronize(f.done);
                    f.busy = false;
                }
            return;
        }
        bool enqueued = false;
        if (!segs.empty()) {
            Flight &f = c->flights[cur];
            if (f.busy) collect_flight(c, f);
            int rc;
            {
                std::lock_guard<std::mutex> g(c->gpu_mu);
                rc = enqueue_flight(c, f, segs);
            }
            f.parts = parts;
            if (rc != EIS_OK) {
                f.busy = false;
                finish_parts(c, f.parts, nullptr, rc);
                f.parts.clear();
            } else {
                enqueued = true;
                cur ^= 1;
            }
        }
        // Wait for the older pass in flight; the newer one keeps the device
        // busy meanwhile.  A pass just enqueued alone is not waited for:
        // the next round plans the pass behind it first.
        Flight &f0 = c->flights[0], &f1 = c->flights[1];
        Flight *older = nullptr;
        if (f0.busy && f1.busy)
            older = (f0.seq < f1.seq) ? &f0 : &f1;
        else if (!enqueued)
            older = f0.busy ? &f0 : (f1.busy ? &f1 : nullptr);
        if (older) collect_flight(c, *older);
    }
}

extern "C" int eis_submit(eis_ctx *c, uint64_t a, uint64_t b, uint64_t *ticket)
{
    if (!c || !ticket) return EIS_EINVAL;
    int rc = check_range(a, b);
    if (rc != EIS_OK) return rc;
    {
        std::lock_guard<std::mutex> lk(c->smu);
        if (c->stop) return EIS_EINVAL;
        if (c->order.size() >= c->cfg.serve_slots) return EIS_EBUSY;
    }
    if (!c->flights_ready) {
        std::lock_guard<std::mutex> g(c->gpu_mu);
        if (hipSetDevice(c->device) != hipSuccess) return EIS_EDEVICE;
        rc = ensure_flights(c);
        if (rc != EIS_OK) return rc;
    }
    {
        std::lock_guard<std::mutex> lk(c->smu);
        if (c->stop) return EIS_EINVAL;
        if (c->order.size() >= c->cfg.serve_slots) return EIS_EBUSY;
        Request r;
        r.d0 = eis_first_candidate(a);
        r.ncand = eis_num_candidates(a, b);
        r.reserved = chunk_footprint(c, r.d0, std::min<u64>(r.ncand, kServeChunk));
        if (r.reserved > c->serve_budget) return EIS_ENOMEM;
        if (c->serve_reserved + r.reserved > c->serve_budget) return EIS_EBUSY;
        if (!c->server.joinable()) c->server = std::thread(server_loop, c);
        r.ticket = c->next_ticket++;
        if (r.ncand == 0) {
            r.finished = true;
            r.reserved = 0;
        }
        c->serve_reserved += r.reserved;
        {
            std::lock_guard<std::mutex> sl(c->stats_mu);
            c->stats.serve_bytes_reserved = c->serve_reserved;
        }
        c->reqs[r.ticket] = r;
        if (!r.finished) c->order.push_back(r.ticket);
        *ticket = r.ticket;
    }
    c->scv.notify_all();
    return EIS_OK;
}

extern "C" int eis_wait(eis_ctx *c, uint64_t ticket, int64_t timeout_us, uint64_t *n_sqfree,
                        uint64_t *n_eis)
{
    if (!c) return EIS_EINVAL;
    std::unique_lock<std::mutex> lk(c->smu);
    if (c->reqs.find(ticket) == c->reqs.end()) return EIS_EINVAL;
    // A ticket that disappears while we wait was retired by another waiter:
    // stop waiting (it is reported as unknown below), never re-create it.
    auto ready = [&] {
        auto f = c->reqs.find(ticket);
        return f == c->reqs.end() || f->second.finished || c->stop;
    };
    if (timeout_us < 0) {
        c->dcv.wait(lk, ready);
    } else if (!c->dcv.wait_for(lk, std::chrono::microseconds(timeout_us), ready)) {
        return EIS_ETIMEDOUT;
    }
    auto it = c->reqs.find(ticket);
    if (it == c->reqs.end()) return EIS_EINVAL;
    Request r = it->second;
    if (!r.finished) return EIS_ETIMEDOUT;
    c->reqs.erase(it);
    if (r.cancelled) return EIS_ECANCELED;
    if (r.status != EIS_OK) return r.status;
    if (n_sqfree) *n_sqfree = r.n_sq;
    if (n_eis) *n_eis = r.n_eis;
    return EIS_OK;
}

extern "C" int eis_cancel(eis_ctx *c, uint64_t ticket)
{
    if (!c) return EIS_EINVAL;
    {
        std::lock_guard<std::mutex> lk(c->smu);
        auto it = c->reqs.find(ticket);
        if (it == c->reqs.end()) return EIS_EINVAL;
        Request &r = it->second;
        if (!r.finished) {
            r.cancelled = true;
            if (r.completed >= r.dispatched) {
                // nothing of it is on the device: retire it now
                r.finished = true;
                c->serve_reserved -= r.reserved;
                r.reserved = 0;
                {
                    std::lock_guard<std::mutex> sl(c->stats_mu);
                    c->stats.serve_bytes_reserved = c->serve_reserved;
                }
                std::deque<u64> keep;
                for (u64 t : c->order)
                    if (t != ticket) keep.push_back(t);
                c->order.swap(keep);
            }
        }
    }
    c->dcv.notify_all();
    c->scv.notify_all();
    return EIS_OK;
}

// ---------------------------------------------------------------------------
// autotuner
// ---------------------------------------------------------------------------

// Device time of the candidates [d0, d0 + 8 n) cut into passes of ps
// candidates, with a given method, window scale and walk chunk.
static int time_range(eis_ctx *c, u64 d0, u64 n, u64 ps, u32 method, double ws, u32 chunk,
                      float &ms)
{
    hipStream_t st = c->stream;
    int rc = settle_pending(c);
    if (rc == EIS_OK) rc = ensure_counts(c, 1);
    if (rc == EIS_OK && n) {
        // allocate for the first (largest) pass before the timed region
        std::vector<HostSeg> segs(1);
        segs[0].d0 = d0;
        segs[0].n = (u32)std::min<u64>(ps, n);
        segs[0].slot = 0;
        segs[0].method = method;
        segs[0].wscale = (float)ws;
        segs[0].walk_chunk = chunk;
        segs[0].dst_bit = 0;
        PassPlan pl;
        rc = prepare_pass(c, segs, pl);
    }
    if (rc == EIS_OK && launch_zero_u32(reinterpret_cast<u32 *>(c->pb.counts), 4, st) != hipSuccess)
        rc = EIS_EDEVICE;
    if (rc == EIS_OK && hipEventRecord(c->ev_all0, st) != hipSuccess) rc = EIS_EDEVICE;
    for (u64 off = 0; rc == EIS_OK && off < n; off += ps) {
        std::vector<HostSeg> segs(1);
        segs[0].d0 = d0 + 8 * off;
        segs[0].n = (u32)std::min<u64>(ps, n - off);
        segs[0].slot = 0;
        segs[0].method = method;
        segs[0].wscale = (float)ws;
        segs[0].walk_chunk = chunk;
        segs[0].dst_bit = 0;
        PassPlan pl;
        rc = run_pass(c, segs, st, false, pl);
        if (rc == EIS_OK && hipStreamSynchronize(st) != hipSuccess) rc = EIS_EDEVICE;
        if (rc == EIS_OK) rc = collect_pass(c);
    }
    if (rc == EIS_OK && hipEventRecord(c->ev_all1, st) != hipSuccess) rc = EIS_EDEVICE;
    if (rc == EIS_OK && hipStreamSynchronize(st) != hipSuccess) rc = EIS_EDEVICE;
    if (rc == EIS_OK && hipEventElapsedTime(&ms, c->ev_all0, c->ev_all1) != hipSuccess) rc = EIS_EDEVICE;
    return rc;
}

// Autotuner.  Per half-decade bin from 10^6: the plain walk against the
// giant-step method at eight window scales, each timed on 2^22 candidates at
// the bin's lower and upper quarter points (plain_ms, giant_ms and scale_ms
// are these sums); then, at the bin's geometric middle, for the giant-step
// method the walk chunk (8, 16, 32 reduction steps per walk phase) at the
// chosen scale on a full pass of candidates (on half a pass the giant walk
// has half the d's per wave and its walk phases run less full, which made
// 32 look best where it is 2-5 % slower on full passes), and the pass size
// (2^24, 2^23, 2^22 candidates; a smaller pass must be 2 % faster to be
// kept) on a full pass of candidates.  The cache records every timing beside the choices.
extern "C" int eis_tune(eis_ctx *c)
{
    if (!c) return EIS_EINVAL;
    std::lock_guard<std::mutex> g(c->gpu_mu);
    if (hipSetDevice(c->device) != hipSuccess) return EIS_EDEVICE;
    constexpr int kScales = 8;
    const double scales[kScales] = {1.0, 1.5, 1.75, 2.0, 2.25, 2.5, 3.5, 5.0};
    const u32 chunks[] = {8, 16, 32};
    const u32 plogs[] = {24, 23, 22};  // the largest first: a smaller one must win by 2 %
    const u32 n = 1u << 23;  // candidates per sample: half a full pass
    int method[kTuneBins];
    double wsc[kTuneBins], plain_ms[kTuneBins], giant_ms[kTuneBins];
    u32 chunk[kTuneBins], plog[kTuneBins];
    double chunk_ms[kTuneBins][3], pass_ms[kTuneBins][3], scale_ms[kTuneBins][kScales];
    for (int b = 0; b < kTuneBins; b++) {
        method[b] = 0;
        wsc[b] = kDefaultWindowScale;
        plain_ms[b] = giant_ms[b] = 0.0;
        chunk[b] = kDefaultWalkChunk;
        plog[b] = 24;
        for (int k = 0; k < 3; k++) chunk_ms[b][k] = pass_ms[b][k] = 0.0;
        for (int k = 0; k < kScales; k++) scale_ms[b][k] = 0.0;
    }
    float ms = 0.f;
    // one untimed pass of each method allocates every buffer
    int rc = time_range(c, 1000000005ull, n, n, 0, kDefaultWindowScale, kDefaultWalkChunk, ms);
    if (rc == EIS_OK) rc = time_range(c, 1000000005ull, n, n, 1, 5.0, kDefaultWalkChunk, ms);
    if (rc != EIS_OK) return rc;
    // bins from 10^6 up.  The method and the window scale are timed at two
    // heights of the bin (its lower and upper quarter points, half a sample
    // each) and chosen by the sum, so that a choice fits the whole bin and
    // two nearly equal scales are not told apart by one sample's noise; the
    // walk chunk and the pass size at its geometric middle.  The last
    // sample, from 10^11.875, ends below 10^12.
    for (int b = kTuneFirstBin; b < kTuneBins - 1; b++) {
        const u64 d0 = eis_first_candidate((u64)std::llround(std::pow(10.0, (b + 0.5) / 2.0)));
        const u64 dq[2] = {eis_first_candidate((u64)std::llround(std::pow(10.0, (b + 0.25) / 2.0))),
                           eis_first_candidate((u64)std::llround(std::pow(10.0, (b + 0.75) / 2.0)))};
        auto two_heights = [&](u32 m, double ws, double &sum) {
            sum = 0.0;
            for (int q = 0; q < 2; q++) {
                const int r = time_range(c, dq[q], n / 2, n / 2, m, ws, kDefaultWalkChunk, ms);
                if (r != EIS_OK) return r;
                sum += ms;
            }
            return (int)EIS_OK;
        };
        rc = two_heights(0, kDefaultWindowScale, plain_ms[b]);
        if (rc != EIS_OK) return rc;
        double best = 1e30, best_ws = kDefaultWindowScale;
        for (int k = 0; k < kScales; k++) {
            rc = two_heights(1, scales[k], scale_ms[b][k]);
            if (rc != EIS_OK) return rc;
            if (scale_ms[b][k] < best) {
                best = scale_ms[b][k];
                best_ws = scales[k];
            }
        }
        method[b] = best < plain_ms[b] ? 1 : 0;
        wsc[b] = best_ws;
        giant_ms[b] = best;
        if (method[b]) {
            double cbest = 1e30;
            for (int k = 0; k < 3; k++) {
                rc = time_range(c, d0, kPassCandidates, kPassCandidates, 1, best_ws, chunks[k], ms);
                if (rc != EIS_OK) return rc;
                chunk_ms[b][k] = ms;
                if (ms < cbest) {
                    cbest = ms;
                    chunk[b] = chunks[k];
                }
            }
        }
        double pbest = 1e30;
        for (int k = 0; k < 3; k++) {
            rc = time_range(c, d0, kPassCandidates, u64(1) << plogs[k], (u32)method[b], wsc[b],
                            chunk[b], ms);
            if (rc != EIS_OK) return rc;
            pass_ms[b][k] = ms;
            if (ms < pbest * (k ? 0.98 : 1.0)) {
                pbest = ms;
                plog[b] = plogs[k];
            }
        }
    }
    // below 10^6 the plain walk; the last bin holds d = 10^12 only
    for (int b = 0; b < kTuneFirstBin; b++) wsc[b] = wsc[kTuneFirstBin];
    method[kTuneBins - 1] = method[kTuneBins - 2];
    wsc[kTuneBins - 1] = wsc[kTuneBins - 2];
    chunk[kTuneBins - 1] = chunk[kTuneBins - 2];
    plog[kTuneBins - 1] = plog[kTuneBins - 2];
    {
        std::lock_guard<std::mutex> lk(c->smu);
        for (int b = 0; b < kTuneBins; b++) {
            c->tuned_method[b] = method[b];
            c->tuned_ws[b] = wsc[b];
            c->tuned_chunk[b] = chunk[b];
            c->tuned_pass_log2[b] = plog[b];
        }
        c->tuned = true;
    }
    if (!c->tune_path.empty()) {
        FILE *f = std::fopen(c->tune_path.c_str(), "w");
        if (!f) return EIS_EINVAL;
        std::fprintf(f, "{\"arch\": \"gfx950\", \"sample_candidates\": %u, \"scales\": [", n);
        for (int k = 0; k < kScales; k++) std::fprintf(f, "%s%.2f", k ? ", " : "", scales[k]);
        std::fprintf(f, "], \"bins\": [\n");
        for (int b = 0; b < kTuneBins; b++) {
            std::fprintf(f,
                         "  {\"b\": %d, \"method\": %d, \"window_scale\": %.3f, \"walk_chunk\": %u, "
                         "\"pass_log2\": %u, \"from\": %llu, \"plain_ms\": %.3f, \"giant_ms\": %.3f, "
                         "\"chunk_ms_8_16_32\": [%.3f, %.3f, %.3f], \"pass_ms_24_23_22\": [%.3f, %.3f, %.3f], "
                         "\"scale_ms\": [",
                         b, method[b], wsc[b], chunk[b], plog[b], (unsigned long long)bin_start(b),
                         plain_ms[b], giant_ms[b], chunk_ms[b][0], chunk_ms[b][1], chunk_ms[b][2],
                         pass_ms[b][0], pass_ms[b][1], pass_ms[b][2]);
            for (int k = 0; k < kScales; k++) std::fprintf(f, "%s%.3f", k ? ", " : "", scale_ms[b][k]);
            std::fprintf(f, "]}%s\n", b < kTuneBins - 1 ? "," : "");
        }
        std::fprintf(f, "]}\n");
        if (std::fclose(f) != 0) return EIS_EINVAL;
    }
    return EIS_OK;
}

extern "C" int eis_tuned_shape(eis_ctx *c, uint64_t d, uint32_t *walk_chunk,
                               uint64_t *pass_candidates)
{
    if (!c) return EIS_EINVAL;
    std::lock_guard<std::mutex> lk(c->smu);
    if (walk_chunk) *walk_chunk = chunk_for(c, d);
    if (pass_candidates)
        *pass_candidates = std::min<u64>(std::max<u64>(pass_for(c, d), u64(1) << 22), kPassCandidates);
    return EIS_OK;
}

extern "C" int eis_tuned_choice(eis_ctx *c, uint64_t d, int *method, double *window_scale)
{
    if (!c) return EIS_EINVAL;
    std::lock_guard<std::mutex> lk(c->smu);
    if (method) *method = (int)method_for(c, d) ? EIS_METHOD_INFRA : EIS_METHOD_BABY;
    if (window_scale) *window_scale = scale_for(c, d);
    return EIS_OK;
}

extern "C" int eis_get_stats(eis_ctx *c, eis_stats *out)
{
    if (!c || !out) return EIS_EINVAL;
    std::lock_guard<std::mutex> lk(c->stats_mu);
    *out = c->stats;
    return EIS_OK;
}
