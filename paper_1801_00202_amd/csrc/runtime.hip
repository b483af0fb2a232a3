// runtime.hip -- host side of libmce.so: the C ABI of include/mce.h.
//
// Responsibilities: input validation (before any HIP call), device buffers of
// a handle, launch configuration of the persistent search, result copy-out,
// the per-handle hipGraph of the solve sequence, and the serving scheduler.
#include "mce.h"
#include "mce_internal.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

using namespace mce;

namespace {

// ------------------------------------------------------------ options ----

struct Options {
    int64_t waves_per_block = 0; // 0: auto
    int64_t blocks = 0;          // 0: fill the device
    int64_t lds_depth = -1;      // -1: auto
    int64_t split_threshold = 0; // 0: auto
    int64_t check_interval = 0;  // 0: auto
    int64_t queue_cap = 0;       // 0: auto
    int64_t watchdog_ms = 0;     // 0: none
    int64_t graph = 1;           // hipGraph replay: 0 never, 1 batches, 2 always
    int64_t refresh_children = 0; // 0: auto
    int64_t pivot = 0;            // kPivot*
    int64_t local_graphs = 1;     // sparse graphs of more than 4096 vertices on local graphs: 0 never, 1 when they fit
};

std::mutex g_opt_mu;
Options g_opt;

Options options()
{
    std::lock_guard<std::mutex> lk(g_opt_mu);
    return g_opt;
}

thread_local mce_stats_t t_stats;

// ------------------------------------------------------------- device ----

struct DeviceInfo {
    int ok = 0;
    int device = -1;
    int cus = 0;
    size_t lds_per_block = 0;
    size_t lds_per_cu = 0;
    int wall_khz = 0;
};

std::mutex g_dev_mu;
DeviceInfo g_dev;
bool g_dev_probed = false;

// The library runs on the current HIP device, which must be a gfx950.
int device_info(DeviceInfo* out)
{
    std::lock_guard<std::mutex> lk(g_dev_mu);
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return MCE_E_DEVICE;
    if (!g_dev_probed || g_dev.device != dev) {
        g_dev_probed = true;
        g_dev = DeviceInfo();
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return MCE_E_DEVICE;
        if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return MCE_E_DEVICE;
        g_dev.device = dev;
        g_dev.cus = prop.multiProcessorCount;
        g_dev.lds_per_block = prop.sharedMemPerBlock;
        g_dev.lds_per_cu = prop.maxSharedMemoryPerMultiProcessor ? prop.maxSharedMemoryPerMultiProcessor
                                                                 : prop.sharedMemPerBlock;
        if (hipDeviceGetAttribute(&g_dev.wall_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess)
            g_dev.wall_khz = 0;
        g_dev.ok = 1;
    }
    if (!g_dev.ok) return MCE_E_DEVICE;
    *out = g_dev;
    return MCE_OK;
}

#define HIP_TRY(expr)                                   \
    do {                                                \
        hipError_t _e = (expr);                         \
        if (_e != hipSuccess) return hip_status(_e);    \
    } while (0)

int hip_status(hipError_t e)
{
    if (e == hipSuccess) return MCE_OK;
    if (e == hipErrorOutOfMemory) return MCE_E_NOMEM;
    return MCE_E_DEVICE;
}

// Caching device allocator: freed blocks stay with the library and are handed
// out again, so handles created per request do not pay for hipMalloc.  Sizes
// are rounded up to a power of two (at least 4 KiB).  Blocks are returned only
// when the device has finished with them (callers synchronise first).
struct Pool {
    std::mutex mu;
    std::multimap<size_t, void*> free_blocks;
    size_t cached = 0;
};

Pool& pool()
{
    static Pool* p = new Pool(); // never destroyed: HIP may be torn down first at exit
    return *p;
}

size_t pool_round(size_t want)
{
    size_t r = 4096;
    while (r < want) r <<= 1;
    return r;
}

void* pool_alloc(size_t want, size_t* got)
{
    const size_t sz = pool_round(want);
    Pool& pl = pool();
    {
        std::lock_guard<std::mutex> lk(pl.mu);
        auto it = pl.free_blocks.find(sz);
        if (it != pl.free_blocks.end()) {
            void* p = it->second;
            pl.free_blocks.erase(it);
            pl.cached -= sz;
            *got = sz;
            return p;
        }
    }
    void* p = nullptr;
    if (hipMalloc(&p, sz) != hipSuccess) {
        (void)hipGetLastError();
        // give the cached blocks back to HIP and retry once
        std::lock_guard<std::mutex> lk(pl.mu);
        for (auto& kv : pl.free_blocks) (void)hipFree(kv.second);
        pl.free_blocks.clear();
        pl.cached = 0;
        if (hipMalloc(&p, sz) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
    }
    *got = sz;
    return p;
}

void pool_free(void* p, size_t sz)
{
    if (!p) return;
    Pool& pl = pool();
    std::lock_guard<std::mutex> lk(pl.mu);
    pl.free_blocks.emplace(sz, p);
    pl.cached += sz;
}

// Grow-only device buffer on the caching allocator, or a borrowed view of
// fixed size (a slice of the allocation-free entry point's scratch area),
// which is never reallocated or freed: asking it for more is MCE_E_NOMEM.
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    bool borrowed = false;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { reset(); }
    void borrow(void* q, size_t n)
    {
        reset();
        p = q;
        bytes = n;
        borrowed = true;
    }
    void reset()
    {
        if (!borrowed) pool_free(p, bytes);
        p = nullptr;
        bytes = 0;
        borrowed = false;
    }
    int ensure(size_t want)
    {
        if (want <= bytes && p) return MCE_OK;
        if (borrowed) return MCE_E_NOMEM;
        reset();
        p = pool_alloc(want ? want : 8, &bytes);
        if (!p) {
            bytes = 0;
            return MCE_E_NOMEM;
        }
        return MCE_OK;
    }
    template <class T> T* as() const { return static_cast<T*>(p); }
};

// Pinned host blocks, cached by power-of-two size like the device blocks
// (handles are made and released per solve; hipHostMalloc and hipHostFree
// cost tens of microseconds each).  At most kPinnedCacheBytes stay cached.
constexpr size_t kPinnedCacheBytes = 256ull << 20;

struct PinnedPool {
    std::mutex mu;
    std::multimap<size_t, void*> free_blocks;
    size_t cached = 0;
};

PinnedPool& pinned_pool()
{
    static PinnedPool* p = new PinnedPool(); // never destroyed: HIP may be torn down first at exit
    return *p;
}

void* pinned_alloc(size_t want, size_t* got)
{
    const size_t sz = pool_round(want);
    PinnedPool& pl = pinned_pool();
    {
        std::lock_guard<std::mutex> lk(pl.mu);
        auto it = pl.free_blocks.find(sz);
        if (it != pl.free_blocks.end()) {
            void* p = it->second;
            pl.free_blocks.erase(it);
            pl.cached -= sz;
            *got = sz;
            return p;
        }
    }
    void* p = nullptr;
    if (hipHostMalloc(&p, sz, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    *got = sz;
    return p;
}

void pinned_free(void* p, size_t sz)
{
    if (!p) return;
    PinnedPool& pl = pinned_pool();
    {
        std::lock_guard<std::mutex> lk(pl.mu);
        if (pl.cached + sz <= kPinnedCacheBytes) {
            pl.free_blocks.emplace(sz, p);
            pl.cached += sz;
            return;
        }
    }
    (void)hipHostFree(p);
}

struct HostPinned {
    void* p = nullptr;
    size_t bytes = 0;
    bool borrowed = false; // a fixed host block owned elsewhere (not pinned)
    HostPinned() = default;
    HostPinned(const HostPinned&) = delete;
    HostPinned& operator=(const HostPinned&) = delete;
    ~HostPinned() { reset(); }
    void borrow(void* q, size_t n)
    {
        reset();
        p = q;
        bytes = n;
        borrowed = true;
    }
    void reset()
    {
        if (!borrowed) pinned_free(p, bytes);
        p = nullptr;
        bytes = 0;
        borrowed = false;
    }
    int ensure(size_t want)
    {
        if (want <= bytes && p) return MCE_OK;
        if (borrowed) return MCE_E_NOMEM;
        reset();
        p = pinned_alloc(want ? want : 8, &bytes);
        if (!p) {
            bytes = 0;
            return MCE_E_NOMEM;
        }
        return MCE_OK;
    }
    template <class T> T* as() const { return static_cast<T*>(p); }
};

uint32_t next_pow2(uint64_t x)
{
    uint32_t r = 1;
    while (r < x && r < (1u << 30)) r <<= 1;
    return r;
}

// ----------------------------------------------------------- validation --

// A simple graph: zero diagonal, no bit at a column >= n, symmetric.
int validate_host(uint32_t n, const uint64_t* rows, uint64_t rs)
{
    if (n > MCE_MAX_N) return MCE_E_INVAL;
    if (n == 0) return MCE_OK;
    if (!rows) return MCE_E_INVAL;
    if (rs * 64u < n) return MCE_E_INVAL;
    for (uint32_t i = 0; i < n; i++) {
        const uint64_t* r = rows + (uint64_t)i * rs;
        for (uint64_t w = 0; w < rs; w++) {
            uint64_t x = r[w];
            const uint64_t lo = w * 64u;
            if (lo + 64u > n) {
                const uint64_t valid = (lo >= n) ? 0ull : ((1ull << (n - lo)) - 1ull);
                if (x & ~valid) return MCE_E_INVAL;
            }
            while (x) {
                const uint32_t b = (uint32_t)__builtin_ctzll(x);
                x &= x - 1;
                const uint32_t j = (uint32_t)(lo + b);
                if (j == i) return MCE_E_INVAL;
                if (!((rows[(uint64_t)j * rs + (i >> 6)] >> (i & 63)) & 1u)) return MCE_E_INVAL;
            }
        }
    }
    return MCE_OK;
}

// ------------------------------------------------------ launch config ----

struct LaunchCfg {
    uint32_t wpb = 4;
    uint32_t blocks = 0;
    uint32_t lds_depth = 16;
    uint32_t split_threshold = 0;
    uint32_t check_interval = 32;
    uint32_t cap = 0;
    uint32_t wave_lds_words = 0;
    uint32_t slot_words = 0;
    uint32_t w32cap = 0;
    uint32_t spill_levels = 0;
    uint32_t spill_chunks = 0;
    uint32_t rule = 0; // pivot rule (kPivot*)
    bool operator==(const LaunchCfg& o) const
    {
        return rule == o.rule && wpb == o.wpb && blocks == o.blocks && lds_depth == o.lds_depth &&
               split_threshold == o.split_threshold && check_interval == o.check_interval &&
               cap == o.cap && wave_lds_words == o.wave_lds_words && slot_words == o.slot_words &&
               w32cap == o.w32cap && spill_levels == o.spill_levels && spill_chunks == o.spill_chunks;
    }
};

} // namespace

// ------------------------------------------------------------- handle ----

struct mce_graph_s {
    std::mutex mu;
    int device = -1;
    uint32_t num_graphs = 0;
    std::vector<GraphDesc> desc;
    uint32_t max_n = 0, max_w32 = 0;
    uint64_t in_words = 0, adj_words = 0, ord_words = 0, hist_total = 0;
    DevBuf d_desc, d_in, d_adj, d_order, d_nbr;
    // workspace of the solve
    DevBuf d_results, d_hist, d_ctl, d_rec, d_mail, d_mail_rec, d_spill, d_state, d_exit, d_params, d_sub;
    // ctl | results | hist in one block, the layout of h_out, so that one copy
    // brings them back (d_ctl, d_results and d_hist are views into it)
    DevBuf d_out;
    // parameter block of the captured graph: written once, before the capture,
    // and read by every replay; no other solve touches it
    DevBuf d_params_graph;
    // bumped whenever a workspace buffer is reallocated: a captured graph holds
    // the buffer addresses of its capture and is replayed only while they stand
    uint64_t ws_gen = 0;
    HostPinned h_out;  // ctl | results | hist, copied back in one go
    HostPinned h_flag; // the validation flag of rows given in device memory, read back
    HostPinned h_desc; // staging of d_desc's copy, kept while it may be in flight
    // chunk buffers of mce_enumerate_stream
    DevBuf d_sv, d_so;
    HostPinned h_sv, h_so;
    // launch choices fixed for this handle by mce_autotune (0: automatic)
    struct Tune {
        uint32_t wpb = 0, wgs_per_cu = 0, split_threshold = 0, check_interval = 0;
    } tune;
    hipGraphExec_t graph_exec = nullptr;
    LaunchCfg graph_cfg;
    uint64_t graph_gen = 0;
    // serving jobs submitted for this handle and not yet finished, and
    // whether one of them runs (jobs of one handle run one at a time: they
    // share its workspace)
    std::atomic<uint32_t> jobs_in_flight{0};
    bool job_running = false; // guarded by the server's lock
    // workspace of fixed size (the allocation-free entry point): launch
    // shapes are cut down to what it holds instead of growing it
    bool fixed_ws = false;
    // Local graphs of the root children (a single graph of more than 4096
    // vertices whose root children all have at most kLocalMaxN - 1
    // neighbours): built at the first solve that can use them and kept.
    // local_state: 0 not looked at, 1 built, -1 not used for this handle.
    int local_state = 0;
    uint32_t lcount = 0, lmax_w32 = 0, lmax_n = 0;
    DevBuf d_ldesc, d_ladj, d_lord, d_lidmap, d_lpx;
    // pinned host blocks of the build: the plan read back, and the layout
    // (source of d_ldesc's copy, kept while it may be in flight)
    HostPinned h_lplan, h_ldesc;
    hipEvent_t ev_local = nullptr;     // recorded after the local graphs' build
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    float prepare_ms = 0.f;
    bool prepared_timed = false;
    // learned from reruns, kept for the next solves of this handle: spill
    // chunks for every wavefront, and chunks of the full stack depth
    uint32_t spill_floor = 0;
    bool spill_full_depth = false;
    ~mce_graph_s()
    {
        if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
        for (auto& e : ev)
            if (e) (void)hipEventDestroy(e);
        if (ev_local) (void)hipEventDestroy(ev_local);
    }
};

namespace {

size_t out_bytes(const mce_graph_s* h)
{
    return sizeof(QueueCtl) + sizeof(DevResult) * h->num_graphs + 8 * h->hist_total;
}

// Stack levels a spill chunk holds at first: enough for every search of
// these workloads; a deeper one stops with kErrDepth and reruns with chunks of
// the full depth n - lds_depth.
constexpr uint32_t kSpillLevelsFirst = 64;
// Bounds of the LDS stack window chosen when the caller sets none.
constexpr uint32_t kAutoDepth = 12, kMinAutoDepth = 4;

// local: the solve runs on the handle's local graphs (their widths, depths
// and number of root units) instead of its own graphs.
int make_cfg(mce_graph_s* h, LaunchCfg* cfg, uint32_t spill_chunks_floor, uint32_t blocks_cap = 0,
             bool full_depth = false, bool local = false)
{
    DeviceInfo di;
    int rc = device_info(&di);
    if (rc != MCE_OK) return rc;
    const Options o = options();
    const uint32_t mw32 = local ? h->lmax_w32 : h->max_w32;
    const uint32_t mn = local ? h->lmax_n : h->max_n;
    const uint64_t units = local ? h->lcount : h->num_graphs;
    LaunchCfg c;
    // Searches on local graphs default to workgroups of two wavefronts, four
    // a CU: every wavefront searches a local graph of its own, and with half
    // as many in flight their rows stay in L2 more often (G(10^4, 0.03):
    // 1.84 ms against 2.16 ms with eight-wavefront workgroups, two a CU).
    const bool local_auto = local && o.waves_per_block <= 0 && o.blocks <= 0 && !h->tune.wpb;
    constexpr uint32_t kLocalWpb = 2, kLocalWgsPerCu = 4;
    // an explicit option wins, then the handle's tuned choice, then the default
    c.wpb = o.waves_per_block > 0 ? (uint32_t)std::min<int64_t>(o.waves_per_block, 16)
                                  : (h->tune.wpb ? h->tune.wpb : (local_auto ? kLocalWpb : 8u));
    c.wpb = std::min<uint32_t>(c.wpb, max_search_wpb(search_chunks(mw32)));
    c.w32cap = std::max<uint32_t>(mw32, 1u);
    c.rule = (uint32_t)o.pivot;
    c.slot_words = lds_frame_words(c.w32cap);
    const uint32_t slack = lds_slack_words(c.w32cap);
    const uint32_t rec_words = kRecHeader + 4 * c.w32cap;
    auto wave_words = [&](uint32_t dep) {
        const uint32_t wl = kWaveFixedWords + (dep + 1) * c.slot_words + slack;
        return (wl + 3u) & ~3u; // frames on 16-byte boundaries
    };
    uint32_t depth;
    if (o.lds_depth >= 0) {
        depth = (uint32_t)std::min<int64_t>(o.lds_depth, 64);
    } else {
        // The deepest window, up to kAutoDepth levels, with which the
        // workgroups that the registers allow on a CU also fit in its LDS;
        // frames below it go to the spill pool.
        int by_regs = 0;
        HIP_TRY(search_occupancy(mw32, c.rule, c.wpb, 0, &by_regs));
        uint32_t wgs = (uint32_t)std::max(by_regs, 1);
        if (o.blocks <= 0 && h->tune.wgs_per_cu) wgs = std::min(wgs, h->tune.wgs_per_cu);
        if (local_auto) wgs = std::min(wgs, kLocalWgsPerCu);
        depth = kAutoDepth;
        while (depth > kMinAutoDepth &&
               (uint64_t)search_lds_bytes(wave_words(depth), rec_words, c.wpb) * wgs > di.lds_per_cu)
            depth--;
    }
    // keep a workgroup within the LDS limit
    for (;;) {
        const uint32_t wl = wave_words(depth);
        if (search_lds_bytes(wl, rec_words, c.wpb) <= di.lds_per_block || (depth == 0 && c.wpb == 1)) {
            c.wave_lds_words = wl;
            break;
        }
        if (depth > 0) depth--;
        else c.wpb--;
    }
    c.lds_depth = depth;
    // Sixteen wavefronts a workgroup with a stack window of two levels or
    // less once ran past its time limit under an earlier work distribution,
    // and no cause was shown; the shape is refused until one is.
    if (c.wpb >= 16 && c.lds_depth <= 2) return MCE_E_INVAL;
    const uint32_t lds_bytes = search_lds_bytes(c.wave_lds_words, rec_words, c.wpb);
    if (o.blocks > 0) {
        c.blocks = (uint32_t)o.blocks;
    } else {
        int bpc = 0;
        HIP_TRY(search_occupancy(mw32, c.rule, c.wpb, lds_bytes, &bpc));
        if (bpc < 1) bpc = 1;
        if (h->tune.wgs_per_cu) bpc = std::min<int>(bpc, (int)h->tune.wgs_per_cu);
        if (local_auto) bpc = std::min<int>(bpc, (int)kLocalWgsPerCu);
        c.blocks = (uint32_t)di.cus * (uint32_t)bpc;
    }
    if (blocks_cap && c.blocks > blocks_cap) c.blocks = blocks_cap;
    const uint32_t waves = c.blocks * c.wpb;
    c.split_threshold = o.split_threshold > 0 ? (uint32_t)o.split_threshold
                                              : (h->tune.split_threshold ? h->tune.split_threshold : 12u);
    // single graphs of up to 512 vertices look at their workgroup twice as
    // often by default: their searches are short, and their work has to
    // spread fast (the served mix: 6% more capacity, 8% lower p50 and p99)
    const uint32_t ci_auto = (h->num_graphs == 1 && h->max_n <= 512u) ? 16u : 32u;
    c.check_interval = next_pow2(o.check_interval > 0 ? (uint64_t)o.check_interval
                                                      : (h->tune.check_interval ? h->tune.check_interval : ci_auto));
    uint64_t cap = o.queue_cap > 0 ? (uint64_t)o.queue_cap
                                   : std::max<uint64_t>({(uint64_t)waves * 2u, units * 2u, 1024u});
    cap = std::max<uint64_t>(cap, units + 1u);
    c.cap = next_pow2(cap);
    c.spill_levels = mn > c.lds_depth ? mn - c.lds_depth : 1u;
    if (!full_depth) c.spill_levels = std::min(c.spill_levels, kSpillLevelsFirst);
    c.spill_chunks = std::max<uint32_t>(std::min<uint32_t>(waves, 64u), spill_chunks_floor);
    c.spill_chunks = std::min<uint32_t>(c.spill_chunks, waves);
    *cfg = c;
    return MCE_OK;
}

int ensure_workspace_bufs(mce_graph_s* h, const LaunchCfg& c);

// The workspace of a solve; a reallocated buffer makes any captured graph of
// the handle stale (see ws_gen).
int ensure_workspace(mce_graph_s* h, const LaunchCfg& c)
{
    const void* before[] = {h->d_out.p, h->d_rec.p, h->d_mail.p, h->d_mail_rec.p,
                            h->d_spill.p, h->d_state.p, h->d_exit.p, h->h_out.p};
    const int rc = ensure_workspace_bufs(h, c);
    const void* after[] = {h->d_out.p, h->d_rec.p, h->d_mail.p, h->d_mail_rec.p,
                           h->d_spill.p, h->d_state.p, h->d_exit.p, h->h_out.p};
    if (std::memcmp(before, after, sizeof(before)) != 0) h->ws_gen++;
    return rc;
}

int ensure_workspace_bufs(mce_graph_s* h, const LaunchCfg& c)
{
    int rc;
    const size_t res_bytes = sizeof(DevResult) * h->num_graphs;
    const size_t hist_bytes = 8 * std::max<uint64_t>(h->hist_total, 1);
    if ((rc = h->d_out.ensure(sizeof(QueueCtl) + res_bytes + hist_bytes)) != MCE_OK) return rc;
    char* o = h->d_out.as<char>();
    h->d_ctl.borrow(o, sizeof(QueueCtl));
    h->d_results.borrow(o + sizeof(QueueCtl), res_bytes);
    h->d_hist.borrow(o + sizeof(QueueCtl) + res_bytes, hist_bytes);
    const uint64_t rec_words = kRecHeader + 4ull * c.w32cap;
    if ((rc = h->d_rec.ensure(4ull * rec_words * c.cap)) != MCE_OK) return rc;
    if ((rc = h->d_mail.ensure(sizeof(Mailbox) * (uint64_t)c.blocks)) != MCE_OK) return rc;
    if ((rc = h->d_mail_rec.ensure(4ull * rec_words * c.blocks)) != MCE_OK) return rc;
    const uint64_t spill = 4ull * spill_frame_words(c.w32cap) * c.spill_levels * c.spill_chunks;
    if ((rc = h->d_spill.ensure(spill)) != MCE_OK) return rc;
    if ((rc = h->d_state.ensure(4ull * c.blocks * c.wpb)) != MCE_OK) return rc;
    if ((rc = h->d_exit.ensure(sizeof(WaveExit) * c.blocks * c.wpb)) != MCE_OK) return rc;
    if ((rc = h->d_params.ensure(sizeof(SearchParams))) != MCE_OK) return rc;
    if ((rc = h->h_out.ensure(out_bytes(h))) != MCE_OK) return rc;
    return MCE_OK;
}

SearchParams make_params(mce_graph_s* h, const LaunchCfg& c, bool local = false)
{
    SearchParams sp;
    std::memset(&sp, 0, sizeof(sp));
    sp.graphs = local ? h->d_ldesc.as<GraphDesc>() : h->d_desc.as<GraphDesc>();
    sp.adj = local ? h->d_ladj.as<uint32_t>() : h->d_adj.as<uint32_t>();
    sp.order = local ? h->d_lord.as<uint32_t>() : h->d_order.as<uint32_t>();
    sp.idmap = local ? h->d_lidmap.as<uint32_t>() : nullptr;
    sp.results = h->d_results.as<DevResult>();
    sp.hist = h->d_hist.as<unsigned long long>();
    sp.ctl = h->d_ctl.as<QueueCtl>();
    sp.rec = h->d_rec.as<uint32_t>();
    sp.mail = h->d_mail.as<Mailbox>();
    sp.mail_rec = h->d_mail_rec.as<uint32_t>();
    sp.num_wg = c.blocks;
    sp.spill = h->d_spill.as<uint32_t>();
    sp.wave_state = h->d_state.as<uint32_t>();
    sp.exits = h->d_exit.as<WaveExit>();
    sp.rec_words = kRecHeader + 4 * c.w32cap;
    sp.w32cap = c.w32cap;
    sp.slot_words = c.slot_words;
    sp.spill_words = spill_frame_words(c.w32cap);
    sp.lds_depth = c.lds_depth;
    sp.spill_levels = c.spill_levels;
    sp.spill_chunks = c.spill_chunks;
    sp.wave_lds_words = c.wave_lds_words;
    sp.split_threshold = c.split_threshold;
    sp.check_interval = c.check_interval;
    sp.pivot_rule = c.rule;
    const Options o = options();
    DeviceInfo di;
    const bool have_clock = device_info(&di) == MCE_OK && di.wall_khz > 0;
    if (o.watchdog_ms > 0 && have_clock) sp.watchdog_ticks = (uint64_t)o.watchdog_ms * (uint64_t)di.wall_khz;
    // a busy workgroup looks at its mailbox every refresh_children children
    sp.refresh_children = o.refresh_children > 0 ? (uint32_t)o.refresh_children : sp.check_interval;
    if (sp.refresh_children < sp.check_interval) sp.refresh_children = sp.check_interval;
    // an idle workgroup reads the end-of-search counter every poll_iters looks
    sp.poll_iters = 4;
    return sp;
}

// The solve sequence on a stream: reset, root, search, copy-out.
// d_sp: device copy of sp already written by the caller (a graph capture), or
// null: the reset kernel writes sp (its own argument) into d_params.
int enqueue_solve(mce_graph_s* h, const LaunchCfg& c, const SearchParams& sp, uint64_t first,
                  uint64_t last, hipStream_t s, bool timed, const uint32_t* sub_bits = nullptr,
                  const SearchParams* d_sp = nullptr, bool local = false)
{
    HIP_TRY(launch_reset(sp, h->num_graphs, h->hist_total, c.blocks, d_sp ? nullptr : h->d_params.as<SearchParams>(),
                         s));
    if (local) {
        // the root children [first, last) of the local graphs
        HIP_TRY(launch_local_units(sp, h->d_lpx.as<uint32_t>(), h->lcount, h->lmax_w32, first, last, s));
    } else if (sub_bits) {
        // one given node of graph 0 instead of the root
        HIP_TRY(launch_subproblem(sp, h->max_w32, sub_bits, s));
    } else {
        // the root children of all graphs fill at most the pool
        const uint32_t max_units = std::max<uint32_t>(1u, c.cap / h->num_graphs);
        HIP_TRY(launch_root(sp, h->num_graphs, h->max_w32, first, last, max_units, s));
    }
    if (!d_sp) d_sp = h->d_params.as<SearchParams>();
    if (timed) HIP_TRY(hipEventRecord(h->ev[2], s));
    HIP_TRY(launch_search(sp, d_sp, local ? h->lmax_w32 : h->max_w32, c.blocks, c.wpb, s));
    if (timed) HIP_TRY(hipEventRecord(h->ev[3], s));
    HIP_TRY(launch_exit_fold(sp, c.blocks * c.wpb, s));
    // control block, results and histogram are one block (d_out), laid out as h_out
    HIP_TRY(hipMemcpyAsync(h->h_out.p, sp.ctl, out_bytes(h), hipMemcpyDeviceToHost, s));
    return MCE_OK;
}

void fill_result(const mce_graph_s* h, uint32_t gi, const DevResult& r, const uint64_t* hist,
                 bool root_counted, mce_result_t* out)
{
    const GraphDesc& gd = h->desc[gi];
    out->count = r.count;
    out->nodes = r.nodes;
    out->children = r.children;
    // every child is a new node, a maximal clique or a dead end; the root is a
    // node but no child
    out->dead_ends = r.children - (r.nodes - (root_counted ? 1u : 0u)) - r.count;
    out->hash_xor = r.hash_xor;
    out->hash_sum = r.hash_sum;
    out->omega = r.omega;
    out->status = MCE_OK;
    if (out->hist && out->hist_len) {
        const uint32_t len = out->hist_len;
        for (uint32_t k = 0; k < len; k++) out->hist[k] = (k <= gd.n) ? hist[gd.hist_off + k] : 0ull;
    }
}

// n = 0: the empty clique only.
void fill_empty_graph(uint64_t first, uint64_t last, mce_result_t* out)
{
    const bool root = first == 0 && last > 0;
    out->count = root ? 1 : 0;
    out->nodes = out->children = out->dead_ends = 0;
    out->hash_xor = out->hash_sum = 0; // h({}) = mix64(0) = 0
    out->omega = 0;
    out->status = MCE_OK;
    if (out->hist && out->hist_len) {
        std::memset(out->hist, 0, 8ull * out->hist_len);
        out->hist[0] = root ? 1 : 0;
    }
}

int read_results(mce_graph_s* h, uint64_t first, uint64_t last, mce_result_t* res, QueueCtl* ctl_out)
{
    const char* out = static_cast<const char*>(h->h_out.p);
    const QueueCtl* ctl = reinterpret_cast<const QueueCtl*>(out);
    const DevResult* r = reinterpret_cast<const DevResult*>(out + sizeof(QueueCtl));
    const uint64_t* hist = reinterpret_cast<const uint64_t*>(out + sizeof(QueueCtl) + sizeof(DevResult) * h->num_graphs);
    if (ctl_out) *ctl_out = *ctl;
    for (uint32_t i = 0; i < h->num_graphs; i++) {
        if (h->desc[i].n == 0) fill_empty_graph(first, last, &res[i]);
        else fill_result(h, i, r[i], hist, first == 0 && last > 0, &res[i]);
    }
    return MCE_OK;
}

int ensure_events(mce_graph_s* h)
{
    for (auto& e : h->ev)
        if (!e) HIP_TRY(hipEventCreate(&e));
    return MCE_OK;
}

// The local graphs of a single graph of more than 4096 vertices, built once
// on stream s: the degrees and root-child flags of its positions come to the
// host (a wait), which lays the local graphs out (each root child l:
// |N(l)| + 1 vertices) and gives up if one would be wider than the one-chunk
// layout; the device then builds them, and ev_local marks the end of the
// build (solves on other streams wait for it).
int ensure_local(mce_graph_s* h, hipStream_t s)
{
    if (h->local_state != 0) return MCE_OK;
    h->local_state = -1;
    if (h->fixed_ws || h->num_graphs != 1 || h->desc[0].n <= 4096u || options().local_graphs == 0) return MCE_OK;
    const uint32_t n = h->desc[0].n;
    DevBuf plan;
    int rc;
    // pinned host memory on both copies: a pageable one is staged by the
    // runtime and costs tens of microseconds more on every job
    if ((rc = plan.ensure(4ull * n)) != MCE_OK) return rc;
    if ((rc = h->h_lplan.ensure(4ull * n)) != MCE_OK) return rc;
    if ((rc = h->h_ldesc.ensure(sizeof(GraphDesc) * n)) != MCE_OK) return rc;
    const uint32_t* hp = h->h_lplan.as<uint32_t>();
    GraphDesc* ld = h->h_ldesc.as<GraphDesc>();
    HIP_TRY(launch_local_plan(h->d_desc.as<GraphDesc>(), h->d_adj.as<uint32_t>(), n, plan.as<uint32_t>(), s));
    HIP_TRY(hipMemcpyAsync(h->h_lplan.p, plan.p, 4ull * n, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    uint32_t count = 0;
    uint64_t adj = 0, ord = 0, px = 0;
    uint32_t mw = 0, mn = 0;
    for (uint32_t v = 0; v < n; v++) {
        if (!(hp[v] & 0x80000000u)) continue;
        const uint32_t k = (hp[v] & 0x7fffffffu) + 1u;
        if (k > kLocalMaxN) return MCE_OK; // a wide neighbourhood: the whole graph's layout instead
        GraphDesc& gd = ld[count++];
        std::memset(&gd, 0, sizeof(gd));
        gd.n = k;
        gd.w32 = (k + 31u) / 32u;
        gd.rstride = gd.w32 + 1u;
        gd.rw64 = v;     // the root child's position
        gd.in_off = px;  // its node's P, X and own local id in lpx
        gd.adj_off = adj;
        gd.ord_off = ord;
        gd.idmap_off = ord;
        gd.hist_off = h->desc[0].hist_off;
        gd.res = 0;
        adj += (uint64_t)k * gd.rstride;
        ord += k;
        px += 2ull * gd.w32 + 1u;
        mw = std::max(mw, gd.w32);
        mn = std::max(mn, k);
    }
    if (count == 0) return MCE_OK;
    if ((rc = h->d_ldesc.ensure(sizeof(GraphDesc) * count)) != MCE_OK) return rc;
    // 128 words of padding: a row load reads up to 64 words from the row start
    if ((rc = h->d_ladj.ensure(4 * (adj + 128))) != MCE_OK) return rc;
    if ((rc = h->d_lord.ensure(4 * ord)) != MCE_OK) return rc;
    if ((rc = h->d_lidmap.ensure(4 * ord)) != MCE_OK) return rc;
    if ((rc = h->d_lpx.ensure(4 * px)) != MCE_OK) return rc;
    HIP_TRY(hipMemcpyAsync(h->d_ldesc.p, ld, sizeof(GraphDesc) * count, hipMemcpyHostToDevice, s));
    HIP_TRY(launch_local_build(h->d_desc.as<GraphDesc>(), h->d_adj.as<uint32_t>(), h->d_order.as<uint32_t>(), n,
                               h->d_ldesc.as<GraphDesc>(), count, h->d_ladj.as<uint32_t>(),
                               h->d_lord.as<uint32_t>(), h->d_lidmap.as<uint32_t>(), h->d_lpx.as<uint32_t>(), s));
    // no wait here: the build's end is an event that solves wait for (on
    // this stream, a no-op), and the host layout stays with the handle
    if (!h->ev_local) HIP_TRY(hipEventCreateWithFlags(&h->ev_local, hipEventDisableTiming));
    HIP_TRY(hipEventRecord(h->ev_local, s));
    h->lcount = count;
    h->lmax_w32 = mw;
    h->lmax_n = mn;
    h->local_state = 1;
    return MCE_OK;
}

// Cut a launch configuration down to a workspace of fixed size: the pool of
// root units, the mailboxes and wavefront states, and the spill pool.  A
// rerun that needs a spill chunk for every wavefront (floor) runs with as
// many wavefronts as chunks fit.  MCE_E_NOMEM if not even one chunk fits.
int fit_fixed_workspace(mce_graph_s* h, LaunchCfg* c, uint32_t floor)
{
    const uint64_t rec_bytes = 4ull * (kRecHeader + 4ull * c->w32cap);
    const uint64_t recs = h->d_rec.bytes / rec_bytes;
    if (recs < 2) return MCE_E_NOMEM;
    uint32_t cap = 1;
    while (2ull * cap <= recs && 2ull * cap <= c->cap) cap *= 2;
    c->cap = cap;
    const uint64_t wg_max = std::min<uint64_t>(h->d_mail.bytes / sizeof(Mailbox), h->d_mail_rec.bytes / rec_bytes);
    const uint64_t waves_max = std::min<uint64_t>(h->d_state.bytes / 4, h->d_exit.bytes / sizeof(WaveExit));
    const uint64_t chunk_bytes = 4ull * spill_frame_words(c->w32cap) * c->spill_levels;
    const uint64_t chunks_fit = h->d_spill.bytes / chunk_bytes;
    if (chunks_fit == 0 || wg_max == 0) return MCE_E_NOMEM;
    uint64_t blocks = std::min<uint64_t>(c->blocks, wg_max);
    uint32_t wpb = c->wpb;
    while (blocks * wpb > waves_max) blocks--;
    // every wavefront needs a chunk (a rerun after the pool ran out)
    if (floor != 0 && blocks * wpb > chunks_fit) {
        if (chunks_fit >= wpb) {
            blocks = chunks_fit / wpb;
        } else {
            blocks = 1;
            wpb = (uint32_t)chunks_fit;
        }
    }
    c->blocks = (uint32_t)std::max<uint64_t>(blocks, 1);
    c->wpb = wpb;
    const uint64_t waves = (uint64_t)c->blocks * c->wpb;
    c->spill_chunks = (uint32_t)std::min<uint64_t>({(uint64_t)std::max(c->spill_chunks, std::min<uint32_t>(floor, (uint32_t)waves)), waves, chunks_fit});
    return MCE_OK;
}

// Run one solve (count, count_range or enumerate) synchronously.
int run_solve(mce_graph_t g, uint64_t first, uint64_t last, mce_result_t* res, hipStream_t s,
              uint32_t* verts, uint64_t verts_cap, uint64_t* offs, uint64_t offs_cap,
              QueueCtl* ctl_out, bool use_graph, uint32_t blocks_cap = 0, const uint32_t* sub_bits = nullptr,
              const uint32_t* cancel = nullptr, uint32_t* lds_bytes_out = nullptr)
{
    int rc = ensure_events(g);
    if (rc != MCE_OK) return rc;
    // a whole-graph or root-range solve of a sparse wide graph runs on the
    // local graphs of its root children
    if (!sub_bits && (rc = ensure_local(g, s)) != MCE_OK) return rc;
    const bool local = !sub_bits && g->local_state == 1;
    if (local) HIP_TRY(hipStreamWaitEvent(s, g->ev_local, 0));
    if (local) use_graph = false;
    uint32_t floor = g->spill_floor;
    bool full_depth = g->spill_full_depth;
    for (int attempt = 0; attempt < 4; attempt++) {
        LaunchCfg c;
        if ((rc = make_cfg(g, &c, floor, blocks_cap, full_depth, local)) != MCE_OK) return rc;
        if (g->fixed_ws && (rc = fit_fixed_workspace(g, &c, floor)) != MCE_OK) return rc;
        if ((rc = ensure_workspace(g, c)) != MCE_OK) return rc;
        SearchParams sp = make_params(g, c, local);
        sp.cancel = cancel;
        if (lds_bytes_out) *lds_bytes_out = search_lds_bytes(c.wave_lds_words, kRecHeader + 4 * c.w32cap, c.wpb) * c.blocks;
        const bool enumerate = verts != nullptr || offs != nullptr;
        if (enumerate) {
            sp.enumerate = 1;
            sp.verts = verts;
            sp.verts_cap = verts ? verts_cap : 0;
            sp.offs = reinterpret_cast<unsigned long long*>(offs);
            sp.offs_cap = offs ? offs_cap : 0;
        }
        auto t0 = std::chrono::steady_clock::now();
        (void)t0;
        HIP_TRY(hipEventRecord(g->ev[0], s));
        if (use_graph && !enumerate && first == 0 && last == UINT64_MAX) {
            // A captured graph is replayed only with the launch configuration
            // and the workspace buffers it was captured with; its parameter
            // block is its own (the solves outside the graph stage theirs
            // elsewhere), so a replay reads exactly what its capture wrote.
            if (!g->graph_exec || !(g->graph_cfg == c) || g->graph_gen != g->ws_gen) {
                if (g->graph_exec) {
                    (void)hipGraphExecDestroy(g->graph_exec);
                    g->graph_exec = nullptr;
                }
                if ((rc = g->d_params_graph.ensure(sizeof(SearchParams))) != MCE_OK) return rc;
                HIP_TRY(hipStreamSynchronize(s));
                HIP_TRY(hipMemcpy(g->d_params_graph.p, &sp, sizeof(sp), hipMemcpyHostToDevice));
                hipStream_t cs;
                HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
                hipGraph_t graph = nullptr;
                hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
                if (e == hipSuccess) {
                    rc = enqueue_solve(g, c, sp, first, last, cs, false, nullptr,
                                       g->d_params_graph.as<SearchParams>());
                    e = hipStreamEndCapture(cs, &graph);
                }
                (void)hipStreamDestroy(cs);
                if (e != hipSuccess || rc != MCE_OK) {
                    if (graph) (void)hipGraphDestroy(graph);
                    return rc != MCE_OK ? rc : hip_status(e);
                }
                e = hipGraphInstantiate(&g->graph_exec, graph, nullptr, nullptr, 0);
                (void)hipGraphDestroy(graph);
                if (e != hipSuccess) {
                    g->graph_exec = nullptr;
                    return hip_status(e);
                }
                g->graph_cfg = c;
                g->graph_gen = g->ws_gen;
            }
            HIP_TRY(hipGraphLaunch(g->graph_exec, s));
        } else {
            if ((rc = enqueue_solve(g, c, sp, first, last, s, true, sub_bits, nullptr, local)) != MCE_OK) return rc;
        }
        HIP_TRY(hipEventRecord(g->ev[1], s));
        HIP_TRY(hipStreamSynchronize(s));
        QueueCtl ctl;
        read_results(g, first, last, res, &ctl);
        if (ctl.error & kErrWatchdog) {
            // report where the wavefronts were when the deadline passed
            std::vector<uint32_t> st(c.blocks * c.wpb);
            uint32_t n[5] = {0, 0, 0, 0, 0};
            if (hipMemcpy(st.data(), g->d_state.p, 4ull * st.size(), hipMemcpyDeviceToHost) == hipSuccess)
                for (uint32_t x : st) n[x < 5 ? x : 0]++;
            std::fprintf(stderr,
                         "libmce: search stopped by the watchdog (error bits %u); wavefronts: %u idle, "
                         "%u fetching, %u busy, %u exited, %u never started; work %u, root units %u of %u taken\n",
                         ctl.error, n[kWaveIdle], n[kWaveFetch], n[kWaveBusy], n[kWaveExited], n[0], ctl.work,
                         std::min(ctl.pool_next, ctl.pool_size), ctl.pool_size);
            return MCE_E_DEVICE;
        }
        if (ctl.error & (kErrSpill | kErrDepth)) {
            if (ctl.error & kErrSpill) floor = c.blocks * c.wpb; // one chunk for every wavefront
            if (ctl.error & kErrDepth) full_depth = true;
            g->spill_floor = floor;
            g->spill_full_depth = full_depth;
            continue;
        }
        if (ctl.error & kErrCancel) return MCE_E_CANCELLED;
        if (ctl.error & kErrClique) return MCE_E_NOMEM;
        if (ctl.error) return MCE_E_DEVICE;
        if (ctl_out) *ctl_out = ctl;
        float ms = 0.f;
        mce_stats_t st;
        std::memset(&st, 0, sizeof(st));
        if (hipEventElapsedTime(&ms, g->ev[0], g->ev[1]) == hipSuccess) st.search_us = ms * 1000.0;
        // a replayed graph carries no events around the search kernel
        const bool replayed = use_graph && !enumerate && first == 0 && last == UINT64_MAX;
        st.local_graphs = local ? g->lcount : 0;
        if (!replayed && hipEventElapsedTime(&ms, g->ev[2], g->ev[3]) == hipSuccess)
            st.search_kernel_us = ms * 1000.0;
        (void)hipGetLastError(); // a failed timing query must not surface in a later launch check
        st.prepare_us = g->prepare_ms * 1000.0;
        st.blocks = c.blocks;
        st.waves_per_block = c.wpb;
        st.lds_depth = c.lds_depth;
        st.lds_bytes_per_block = search_lds_bytes(c.wave_lds_words, kRecHeader + 4 * c.w32cap, c.wpb);
        st.donations = ctl.donations;
        st.units = ctl.units;
        st.spills = ctl.spill_levels_written;
        st.checks = ctl.checks;
        st.flushes = ctl.flushes;
        st.attempts = (uint32_t)attempt + 1u;
        st.busy_frac = ctl.run_ticks ? (double)ctl.busy_ticks / (double)ctl.run_ticks : 0.0;
        st.ramp_frac = ctl.run_ticks ? (double)ctl.ramp_ticks / (double)ctl.run_ticks : 0.0;
        st.tail_frac = ctl.run_ticks ? (double)ctl.tail_ticks / (double)ctl.run_ticks : 0.0;
        t_stats = st;
        return MCE_OK;
    }
    return MCE_E_NOMEM;
}

} // namespace

// ================================================================ C ABI ==

static int finish_prepare_timing_locked(mce_graph_t g)
{
    if (g->prepared_timed) return MCE_OK;
    HIP_TRY(hipEventSynchronize(g->ev[1]));
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, g->ev[0], g->ev[1]) == hipSuccess) g->prepare_ms = ms;
    g->prepared_timed = true;
    return MCE_OK;
}

extern "C" {

const char* mce_strerror(int code)
{
    switch (code) {
    case MCE_OK: return "ok";
    case MCE_PENDING: return "pending";
    case MCE_E_INVAL: return "invalid argument or non-simple graph";
    case MCE_E_NOMEM: return "out of memory";
    case MCE_E_TRUNCATED: return "output buffer too small";
    case MCE_E_DEVICE: return "HIP error or no gfx950 device";
    case MCE_E_BUSY: return "busy";
    case MCE_E_CANCELLED: return "cancelled";
    default: return "unknown status";
    }
}

int mce_set_option(int key, int64_t value)
{
    std::lock_guard<std::mutex> lk(g_opt_mu);
    switch (key) {
    case MCE_OPT_WAVES_PER_BLOCK:
        if (value < 0 || value > 16) return MCE_E_INVAL;
        g_opt.waves_per_block = value;
        return MCE_OK;
    case MCE_OPT_BLOCKS:
        if (value < 0 || value > (1 << 20)) return MCE_E_INVAL;
        g_opt.blocks = value;
        return MCE_OK;
    case MCE_OPT_LDS_DEPTH:
        if (value < -1 || value > 64) return MCE_E_INVAL;
        g_opt.lds_depth = value;
        return MCE_OK;
    case MCE_OPT_SPLIT_THRESHOLD:
        if (value < 0 || value > (1 << 30)) return MCE_E_INVAL;
        g_opt.split_threshold = value;
        return MCE_OK;
    case MCE_OPT_CHECK_INTERVAL:
        if (value < 0 || value > (1 << 30)) return MCE_E_INVAL;
        g_opt.check_interval = value;
        return MCE_OK;
    case MCE_OPT_QUEUE_CAP:
        if (value < 0 || value > (1 << 26) || (value & (value - 1))) return MCE_E_INVAL;
        g_opt.queue_cap = value;
        return MCE_OK;
    case MCE_OPT_WATCHDOG_MS:
        if (value < 0) return MCE_E_INVAL;
        g_opt.watchdog_ms = value;
        return MCE_OK;
    case MCE_OPT_GRAPH:
        if (value < 0 || value > 2) return MCE_E_INVAL;
        g_opt.graph = value;
        return MCE_OK;
    case MCE_OPT_REFRESH_CHILDREN:
        if (value < 0 || value > (1 << 30)) return MCE_E_INVAL;
        g_opt.refresh_children = value;
        return MCE_OK;
    case MCE_OPT_PIVOT:
        if (value < 0 || value > 2) return MCE_E_INVAL;
        g_opt.pivot = value;
        return MCE_OK;
    case MCE_OPT_LOCAL_GRAPHS:
        if (value < 0 || value > 1) return MCE_E_INVAL;
        g_opt.local_graphs = value;
        return MCE_OK;
    default: return MCE_E_INVAL;
    }
}

int mce_get_option(int key, int64_t* value)
{
    if (!value) return MCE_E_INVAL;
    std::lock_guard<std::mutex> lk(g_opt_mu);
    switch (key) {
    case MCE_OPT_WAVES_PER_BLOCK: *value = g_opt.waves_per_block; return MCE_OK;
    case MCE_OPT_BLOCKS: *value = g_opt.blocks; return MCE_OK;
    case MCE_OPT_LDS_DEPTH: *value = g_opt.lds_depth; return MCE_OK;
    case MCE_OPT_SPLIT_THRESHOLD: *value = g_opt.split_threshold; return MCE_OK;
    case MCE_OPT_CHECK_INTERVAL: *value = g_opt.check_interval; return MCE_OK;
    case MCE_OPT_QUEUE_CAP: *value = g_opt.queue_cap; return MCE_OK;
    case MCE_OPT_WATCHDOG_MS: *value = g_opt.watchdog_ms; return MCE_OK;
    case MCE_OPT_GRAPH: *value = g_opt.graph; return MCE_OK;
    case MCE_OPT_REFRESH_CHILDREN: *value = g_opt.refresh_children; return MCE_OK;
    case MCE_OPT_PIVOT: *value = g_opt.pivot; return MCE_OK;
    case MCE_OPT_LOCAL_GRAPHS: *value = g_opt.local_graphs; return MCE_OK;
    default: return MCE_E_INVAL;
    }
}

int mce_last_stats(mce_stats_t* out)
{
    if (!out) return MCE_E_INVAL;
    *out = t_stats;
    return MCE_OK;
}

int mce_prepare(uint32_t n, const uint64_t* rows, uint32_t row_words, const mce_batch_t* batch,
                uint32_t flags, void* hip_stream, mce_graph_t* out)
{
    if (!out) return MCE_E_INVAL;
    *out = nullptr;
    if (flags & ~MCE_F_DEVICE_PTR) return MCE_E_INVAL;
    const bool dev_ptr = (flags & MCE_F_DEVICE_PTR) != 0;
    std::vector<GraphDesc> desc;
    uint64_t in_words = 0;
    // ---- shape checks and host validation (no HIP call before this) ----
    if (!batch) {
        if (n > MCE_MAX_N) return MCE_E_INVAL;
        if (n > 0 && (!rows || (uint64_t)row_words * 64u < n)) return MCE_E_INVAL;
        GraphDesc gd;
        std::memset(&gd, 0, sizeof(gd));
        gd.idmap_off = kNoMap;
        gd.n = n;
        gd.w32 = (n + 31) / 32;
        gd.rstride = gd.w32 + 1;
        gd.rw64 = n ? row_words : 0;
        gd.in_off = 0;
        desc.push_back(gd);
        in_words = (uint64_t)n * (n ? row_words : 0);
        if (!dev_ptr && n) {
            int rc = validate_host(n, rows, row_words);
            if (rc != MCE_OK) return rc;
        }
    } else {
        if (batch->num_graphs == 0 || !batch->n || !batch->row_offset_words) return MCE_E_INVAL;
        in_words = row_words;
        bool any = false;
        for (uint32_t i = 0; i < batch->num_graphs; i++) {
            const uint32_t ni = batch->n[i];
            if (ni > MCE_MAX_N) return MCE_E_INVAL;
            GraphDesc gd;
            std::memset(&gd, 0, sizeof(gd));
            gd.idmap_off = kNoMap;
            gd.res = (uint32_t)i;
            gd.n = ni;
            gd.w32 = (ni + 31) / 32;
            gd.rstride = gd.w32 + 1;
            gd.rw64 = (ni + 63) / 64;
            gd.in_off = batch->row_offset_words[i];
            if (ni && gd.in_off + (uint64_t)ni * gd.rw64 > (uint64_t)row_words) return MCE_E_INVAL;
            any = any || ni > 0;
            desc.push_back(gd);
        }
        if (any && !rows) return MCE_E_INVAL;
        if (!dev_ptr)
            for (const GraphDesc& gd : desc) {
                int rc = validate_host(gd.n, rows + gd.in_off, gd.rw64);
                if (rc != MCE_OK) return rc;
            }
    }
    // ---- device part ----
    DeviceInfo di;
    int rc = device_info(&di);
    if (rc != MCE_OK) return rc;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    std::unique_ptr<mce_graph_s> h(new mce_graph_s());
    h->device = di.device;
    h->num_graphs = (uint32_t)desc.size();
    uint64_t adj = 0, ord = 0, hist = 0;
    for (GraphDesc& gd : desc) {
        gd.adj_off = adj;
        gd.ord_off = ord;
        gd.hist_off = hist;
        adj += (uint64_t)gd.n * gd.rstride;
        ord += gd.n;
        hist += gd.n + 1;
        h->max_n = std::max(h->max_n, gd.n);
        h->max_w32 = std::max(h->max_w32, gd.w32);
    }
    h->desc = desc;
    h->in_words = in_words;
    h->adj_words = adj;
    h->ord_words = ord;
    h->hist_total = hist;
    if ((rc = h->d_desc.ensure(sizeof(GraphDesc) * desc.size())) != MCE_OK) return rc;
    if ((rc = h->d_in.ensure(8 * std::max<uint64_t>(in_words, 1))) != MCE_OK) return rc;
    // 128 words of padding: a row load reads up to 128 words from the row start
    if ((rc = h->d_adj.ensure(4 * (adj + 128))) != MCE_OK) return rc;
    if ((rc = h->d_order.ensure(4 * std::max<uint64_t>(ord, 1))) != MCE_OK) return rc;
    if ((rc = ensure_events(h.get())) != MCE_OK) return rc;
    if ((rc = h->h_desc.ensure(sizeof(GraphDesc) * desc.size())) != MCE_OK) return rc;
    std::memcpy(h->h_desc.p, desc.data(), sizeof(GraphDesc) * desc.size());
    HIP_TRY(hipEventRecord(h->ev[0], s));
    HIP_TRY(hipMemcpyAsync(h->d_desc.p, h->h_desc.p, sizeof(GraphDesc) * desc.size(), hipMemcpyHostToDevice, s));
    if (in_words)
        HIP_TRY(hipMemcpyAsync(h->d_in.p, rows, 8 * in_words,
                               dev_ptr ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
    if (dev_ptr) {
        // validate on the device, then wait for the flag
        DevBuf flag;
        if ((rc = flag.ensure(4)) != MCE_OK) return rc;
        HIP_TRY(hipMemsetAsync(flag.p, 0, 4, s));
        for (const GraphDesc& gd : desc)
            if (gd.n) HIP_TRY(launch_validate(h->d_in.as<uint64_t>() + gd.in_off, gd.n, gd.rw64, flag.as<unsigned int>(), s));
        if ((rc = h->h_flag.ensure(4)) != MCE_OK) return rc;
        HIP_TRY(hipMemcpyAsync(h->h_flag.p, flag.p, 4, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (*h->h_flag.as<unsigned int>()) return MCE_E_INVAL;
    }
    uint64_t max_words = 0;
    for (const GraphDesc& gd : desc) max_words = std::max<uint64_t>(max_words, (uint64_t)gd.n * gd.rw64);
    // neighbour lists for the degree-bucket ordering of graphs of more than
    // 4096 vertices and a word a graph after them (kept with the handle: the
    // ordering runs asynchronously)
    const uint32_t cap = order_list_cap(h->max_n);
    const uint64_t lbytes = (2ull * cap * ord + 3u) & ~3ull;
    if (cap != 0u && (rc = h->d_nbr.ensure(lbytes + 4ull * h->num_graphs)) != MCE_OK) return rc;
    HIP_TRY(launch_order(h->d_desc.as<GraphDesc>(), h->num_graphs, h->max_n, max_words, h->d_in.as<uint64_t>(),
                         h->d_order.as<uint32_t>(), cap != 0u ? h->d_nbr.as<uint16_t>() : nullptr, cap,
                         cap != 0u ? reinterpret_cast<uint32_t*>(h->d_nbr.as<char>() + lbytes) : nullptr, s));
    HIP_TRY(launch_relabel(h->d_desc.as<GraphDesc>(), h->num_graphs, h->max_n, h->d_in.as<uint64_t>(),
                           h->d_order.as<uint32_t>(), h->d_adj.as<uint32_t>(), s));
    HIP_TRY(hipEventRecord(h->ev[1], s));
    *out = h.release();
    return MCE_OK;
}

int mce_num_graphs(mce_graph_t g, uint32_t* num_graphs)
{
    if (!g || !num_graphs) return MCE_E_INVAL;
    *num_graphs = g->num_graphs;
    return MCE_OK;
}


int mce_get_order(mce_graph_t g, uint32_t graph_index, uint32_t* order, uint32_t cap)
{
    if (!g || graph_index >= g->num_graphs) return MCE_E_INVAL;
    std::lock_guard<std::mutex> lk(g->mu);
    const GraphDesc& gd = g->desc[graph_index];
    if (gd.n && (!order || cap < gd.n)) return MCE_E_INVAL;
    if (gd.n == 0) return MCE_OK;
    int rc = finish_prepare_timing_locked(g);
    if (rc != MCE_OK) return rc;
    HIP_TRY(hipMemcpy(order, g->d_order.as<uint32_t>() + gd.ord_off, 4ull * gd.n, hipMemcpyDeviceToHost));
    return MCE_OK;
}

int mce_root_branches(mce_graph_t g, uint32_t graph_index, uint64_t* out)
{
    if (!g || !out || graph_index >= g->num_graphs) return MCE_E_INVAL;
    std::lock_guard<std::mutex> lk(g->mu);
    const GraphDesc& gd = g->desc[graph_index];
    if (gd.n == 0) {
        *out = 0;
        return MCE_OK;
    }
    int rc = finish_prepare_timing_locked(g);
    if (rc != MCE_OK) return rc;
    std::vector<uint32_t> row0(gd.w32);
    HIP_TRY(hipMemcpy(row0.data(), g->d_adj.as<uint32_t>() + gd.adj_off, 4ull * gd.w32, hipMemcpyDeviceToHost));
    uint64_t nb = 0;
    for (uint32_t w = 0; w < gd.w32; w++) nb += (uint32_t)__builtin_popcount(row0[w]);
    *out = gd.n - nb; // position 0 and its non-neighbours
    return MCE_OK;
}

int mce_count(mce_graph_t g, mce_result_t* res, void* hip_stream)
{
    if (!g || !res) return MCE_E_INVAL;
    std::lock_guard<std::mutex> lk(g->mu);
    int rc = finish_prepare_timing_locked(g);
    if (rc != MCE_OK) return rc;
    const int64_t gm = options().graph;
    const bool use_graph = gm == 2 || (gm == 1 && g->num_graphs > 1);
    rc = run_solve(g, 0, UINT64_MAX, res, static_cast<hipStream_t>(hip_stream), nullptr, 0, nullptr, 0,
                   nullptr, use_graph);
    if (rc != MCE_OK)
        for (uint32_t i = 0; i < g->num_graphs; i++) res[i].status = rc;
    return rc;
}

int mce_count_range(mce_graph_t g, uint64_t first, uint64_t last, mce_result_t* res, void* hip_stream)
{
    if (!g || !res || g->num_graphs != 1) return MCE_E_INVAL;
    std::lock_guard<std::mutex> lk(g->mu);
    int rc = finish_prepare_timing_locked(g);
    if (rc != MCE_OK) return rc;
    rc = run_solve(g, first, last, res, static_cast<hipStream_t>(hip_stream), nullptr, 0, nullptr, 0,
                   nullptr, false);
    if (rc != MCE_OK) res->status = rc;
    return rc;
}

int mce_count_subproblem(mce_graph_t g, const uint32_t* R, uint32_t nr, const uint32_t* P, uint32_t np,
                         const uint32_t* X, uint32_t nx, mce_result_t* res, void* hip_stream)
{
    if (!g || !res || g->num_graphs != 1 || np == 0 || !P || (nr && !R) || (nx && !X)) return MCE_E_INVAL;
    const uint32_t n = g->desc[0].n, w32 = g->desc[0].w32;
    // position bitsets R, P, X; the three sets must be disjoint
    std::vector<uint32_t> bits(3ull * w32, 0u);
    auto add = [&](const uint32_t* list, uint32_t len, uint32_t which) -> bool {
        for (uint32_t i = 0; i < len; i++) {
            const uint32_t v = list[i];
            if (v >= n) return false;
            for (uint32_t t = 0; t < 3; t++)
                if (bits[(size_t)t * w32 + v / 32] >> (v % 32) & 1u) return false;
            bits[(size_t)which * w32 + v / 32] |= 1u << (v % 32);
        }
        return true;
    };
    if (!add(R, nr, 0) || !add(P, np, 1) || !add(X, nx, 2)) return MCE_E_INVAL;
    std::lock_guard<std::mutex> lk(g->mu);
    int rc = finish_prepare_timing_locked(g);
    if (rc != MCE_OK) return rc;
    if ((rc = g->d_sub.ensure(4ull * bits.size())) != MCE_OK) return rc;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    HIP_TRY(hipMemcpyAsync(g->d_sub.p, bits.data(), 4ull * bits.size(), hipMemcpyHostToDevice, s));
    rc = run_solve(g, 0, UINT64_MAX, res, s, nullptr, 0, nullptr, 0, nullptr, false, 0, g->d_sub.as<uint32_t>());
    if (rc != MCE_OK) res->status = rc;
    return rc;
}

int mce_enumerate(mce_graph_t g, uint32_t* verts, uint64_t verts_cap, uint64_t* offsets,
                  uint64_t offsets_cap, uint64_t* verts_needed, uint64_t* offsets_needed,
                  mce_result_t* res, void* hip_stream)
{
    if (!g || !res || g->num_graphs != 1) return MCE_E_INVAL;
    if ((!verts && verts_cap) || (!offsets && offsets_cap)) return MCE_E_INVAL;
    std::lock_guard<std::mutex> lk(g->mu);
    int rc = finish_prepare_timing_locked(g);
    if (rc != MCE_OK) return rc;
    if (g->desc[0].n == 0) {
        fill_empty_graph(0, UINT64_MAX, res);
        if (verts_needed) *verts_needed = 0;
        if (offsets_needed) *offsets_needed = 2;
        if (offsets_cap < 2) return MCE_E_TRUNCATED;
        const uint64_t z[2] = {0, 0};
        HIP_TRY(hipMemcpy(offsets, z, sizeof(z), hipMemcpyHostToDevice));
        return MCE_OK;
    }
    // a non-null pointer marks enumerate mode even with zero capacity
    static uint32_t dummy_v;
    static uint64_t dummy_o;
    uint32_t* v = verts ? verts : &dummy_v;
    uint64_t* o = offsets ? offsets : &dummy_o;
    QueueCtl ctl;
    rc = run_solve(g, 0, UINT64_MAX, res, static_cast<hipStream_t>(hip_stream), v, verts ? verts_cap : 0,
                   o, offsets ? offsets_cap : 0, &ctl, false);
    if (rc != MCE_OK) {
        res->status = rc;
        return rc;
    }
    if (verts_needed) *verts_needed = ctl.vcursor;
    if (offsets_needed) *offsets_needed = ctl.ocursor;
    if (ctl.vcursor > verts_cap || ctl.ocursor > offsets_cap) {
        res->status = MCE_E_TRUNCATED;
        return MCE_E_TRUNCATED;
    }
    return MCE_OK;
}

int mce_enumerate_stream(mce_graph_t g, uint64_t chunk_verts, mce_clique_sink_t sink, void* user,
                         mce_result_t* res, void* hip_stream)
{
    if (!g || !res || !sink || g->num_graphs != 1) return MCE_E_INVAL;
    std::lock_guard<std::mutex> lk(g->mu);
    int rc = finish_prepare_timing_locked(g);
    if (rc != MCE_OK) return rc;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const GraphDesc& gd = g->desc[0];
    uint64_t* user_hist = res->hist;
    const uint32_t user_len = res->hist_len;
    if (gd.n == 0) {
        fill_empty_graph(0, UINT64_MAX, res);
        const uint64_t z[2] = {0, 0};
        const uint32_t none = 0;
        return sink(user, &none, z, 1) ? MCE_E_CANCELLED : MCE_OK;
    }
    if (chunk_verts == 0) chunk_verts = 1ull << 24;
    // children of the root: position 0 and its non-neighbours
    std::vector<uint32_t> row0(gd.w32);
    HIP_TRY(hipMemcpy(row0.data(), g->d_adj.as<uint32_t>() + gd.adj_off, 4ull * gd.w32, hipMemcpyDeviceToHost));
    uint64_t nb = 0;
    for (uint32_t w = 0; w < gd.w32; w++) nb += (uint32_t)__builtin_popcount(row0[w]);
    const uint64_t total = gd.n - nb;
    // running totals
    mce_result_t acc;
    std::memset(&acc, 0, sizeof(acc));
    std::vector<uint64_t> hist_acc(gd.n + 1, 0), hist_r(gd.n + 1, 0);
    uint64_t cap_v = chunk_verts, cap_o = 2 * chunk_verts;
    uint64_t a = 0, span = total; // the first try covers everything
    while (a < total) {
        if (span > total - a) span = total - a;
        if ((rc = g->d_sv.ensure(4 * cap_v)) != MCE_OK) return rc;
        if ((rc = g->d_so.ensure(8 * cap_o)) != MCE_OK) return rc;
        mce_result_t r;
        std::memset(&r, 0, sizeof(r));
        r.hist = hist_r.data();
        r.hist_len = (uint32_t)hist_r.size();
        QueueCtl ctl;
        rc = run_solve(g, a, a + span, &r, s, g->d_sv.as<uint32_t>(), cap_v, g->d_so.as<uint64_t>(), cap_o, &ctl,
                       false);
        if (rc != MCE_OK) return rc;
        if (ctl.vcursor > cap_v || ctl.ocursor > cap_o) {
            // too much output for the chunk: split the range, or (one child)
            // give it the buffer it needs
            if (span > 1) {
                const double f = std::min((double)cap_v / (double)std::max<uint64_t>(ctl.vcursor, 1),
                                          (double)cap_o / (double)std::max<uint64_t>(ctl.ocursor, 1));
                span = std::max<uint64_t>(1, std::min<uint64_t>(span / 2, (uint64_t)((double)span * f * 0.8)));
            } else {
                cap_v = std::max<uint64_t>(cap_v, ctl.vcursor);
                cap_o = std::max<uint64_t>(cap_o, ctl.ocursor);
            }
            continue;
        }
        // deliver the chunk
        if ((rc = g->h_sv.ensure(4 * std::max<uint64_t>(ctl.vcursor, 1))) != MCE_OK) return rc;
        if ((rc = g->h_so.ensure(8 * std::max<uint64_t>(ctl.ocursor, 1))) != MCE_OK) return rc;
        if (ctl.vcursor)
            HIP_TRY(hipMemcpyAsync(g->h_sv.p, g->d_sv.p, 4 * ctl.vcursor, hipMemcpyDeviceToHost, s));
        if (ctl.ocursor)
            HIP_TRY(hipMemcpyAsync(g->h_so.p, g->d_so.p, 8 * ctl.ocursor, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        acc.count += r.count;
        acc.nodes += r.nodes;
        acc.children += r.children;
        acc.dead_ends += r.dead_ends;
        acc.hash_xor ^= r.hash_xor;
        acc.hash_sum += r.hash_sum;
        acc.omega = std::max(acc.omega, r.omega);
        for (size_t k = 0; k < hist_r.size(); k++) hist_acc[k] += hist_r[k];
        a += span;
        const bool stop = r.count && sink(user, static_cast<const uint32_t*>(g->h_sv.p),
                                          static_cast<const uint64_t*>(g->h_so.p), r.count) != 0;
        if (stop || a >= total) {
            *res = acc;
            res->hist = user_hist;
            res->hist_len = user_len;
            res->status = stop ? MCE_E_CANCELLED : MCE_OK;
            if (user_hist)
                for (uint32_t k = 0; k < user_len; k++) user_hist[k] = k < hist_acc.size() ? hist_acc[k] : 0;
            return stop ? MCE_E_CANCELLED : MCE_OK;
        }
        // a range that used little of the chunk doubles for the next one
        if (ctl.vcursor < cap_v / 4 && ctl.ocursor < cap_o / 4) span *= 2;
    }
    *res = acc;
    res->hist = user_hist;
    res->hist_len = user_len;
    res->status = MCE_OK;
    if (user_hist)
        for (uint32_t k = 0; k < user_len; k++) user_hist[k] = k < hist_acc.size() ? hist_acc[k] : 0;
    return MCE_OK;
}

int mce_autotune(mce_graph_t g, uint32_t max_trials, mce_tune_t* out, void* hip_stream)
{
    if (!g) return MCE_E_INVAL;
    std::lock_guard<std::mutex> lk(g->mu);
    int rc = finish_prepare_timing_locked(g);
    if (rc != MCE_OK) return rc;
    if (max_trials == 0) max_trials = 32;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const uint32_t ng = g->num_graphs;
    std::vector<mce_result_t> ref(ng), cur(ng);
    bool have_ref = false;
    uint32_t trials = 0;
    // One candidate: the best of two timed solves (HIP events around the
    // whole solve); every solve must give exactly the results of the first.
    auto trial = [&](const mce_graph_s::Tune& t, double* us) -> int {
        g->tune = t;
        double best = 1e300;
        for (int r = 0; r < 2; r++) {
            for (auto& x : cur) std::memset(&x, 0, sizeof(x));
            const int e = run_solve(g, 0, UINT64_MAX, cur.data(), s, nullptr, 0, nullptr, 0, nullptr, false);
            if (e != MCE_OK) return e;
            best = std::min(best, t_stats.search_us);
            if (!have_ref) {
                ref = cur;
                have_ref = true;
            }
            for (uint32_t i = 0; i < ng; i++) {
                const mce_result_t &a = ref[i], &b = cur[i];
                if (a.count != b.count || a.nodes != b.nodes || a.children != b.children ||
                    a.dead_ends != b.dead_ends || a.hash_xor != b.hash_xor || a.hash_sum != b.hash_sum ||
                    a.omega != b.omega)
                    return MCE_E_DEVICE; // a schedule changed a result: a bug, not a tuning choice
            }
        }
        trials++;
        *us = best;
        return MCE_OK;
    };
    // The automatic choice first, written out as a tuned one.
    mce_graph_s::Tune best_t;
    double best_us = 0, auto_us = 0;
    if ((rc = trial(best_t, &auto_us)) != MCE_OK) return rc;
    {
        LaunchCfg c;
        if ((rc = make_cfg(g, &c, g->spill_floor, 0, g->spill_full_depth, g->local_state == 1)) != MCE_OK) return rc;
        DeviceInfo di;
        if ((rc = device_info(&di)) != MCE_OK) return rc;
        best_t.wpb = c.wpb;
        best_t.wgs_per_cu = std::max<uint32_t>(c.blocks / (uint32_t)std::max(di.cus, 1), 1u);
        best_t.split_threshold = c.split_threshold;
        best_t.check_interval = c.check_interval;
    }
    best_us = auto_us;
    auto consider = [&](mce_graph_s::Tune t) -> int {
        if (trials >= max_trials) return MCE_OK;
        double us = 0;
        const int e = trial(t, &us);
        if (e != MCE_OK) return e;
        if (us < best_us) {
            best_us = us;
            best_t = t;
        }
        return MCE_OK;
    };
    // 1. Launch shape: wavefronts per workgroup and workgroups per CU (the
    //    LDS stack window is then the deepest that fits).
    const mce_graph_s::Tune shape0 = best_t;
    for (uint32_t wpb : {4u, 8u, 16u}) {
        int by_regs = 0;
        HIP_TRY(search_occupancy(g->local_state == 1 ? g->lmax_w32 : g->max_w32, (uint32_t)options().pivot, wpb, 0,
                             &by_regs));
        for (uint32_t k = 1; k <= (uint32_t)std::min(by_regs, 4); k++) {
            if (wpb == shape0.wpb && k == shape0.wgs_per_cu) continue;
            mce_graph_s::Tune t = shape0;
            t.wpb = wpb;
            t.wgs_per_cu = k;
            g->tune = t;
            LaunchCfg c;
            if (make_cfg(g, &c, g->spill_floor, 0, g->spill_full_depth, g->local_state == 1) != MCE_OK ||
                c.lds_depth < 2 ||
                c.wpb != wpb)
                continue; // too little LDS for a useful stack window
            if ((rc = consider(t)) != MCE_OK) return rc;
        }
    }
    // 2. Split threshold, 3. check interval, each around the best so far.
    const mce_graph_s::Tune split0 = best_t;
    for (uint32_t st : {6u, 12u, 20u, 32u}) {
        if (st == split0.split_threshold) continue;
        mce_graph_s::Tune t = split0;
        t.split_threshold = st;
        if ((rc = consider(t)) != MCE_OK) return rc;
    }
    const mce_graph_s::Tune ci0 = best_t;
    for (uint32_t ci : {16u, 32u, 64u}) {
        if (ci == ci0.check_interval) continue;
        mce_graph_s::Tune t = ci0;
        t.check_interval = ci;
        if ((rc = consider(t)) != MCE_OK) return rc;
    }
    g->tune = best_t;
    if (out) {
        LaunchCfg c;
        if ((rc = make_cfg(g, &c, g->spill_floor, 0, g->spill_full_depth, g->local_state == 1)) != MCE_OK) return rc;
        out->waves_per_block = c.wpb;
        out->blocks = c.blocks;
        out->lds_depth = c.lds_depth;
        out->split_threshold = c.split_threshold;
        out->check_interval = c.check_interval;
        out->trials = trials;
        out->auto_us = auto_us;
        out->best_us = best_us;
    }
    return MCE_OK;
}

int mce_clear_tuning(mce_graph_t g)
{
    if (!g) return MCE_E_INVAL;
    std::lock_guard<std::mutex> lk(g->mu);
    g->tune = mce_graph_s::Tune();
    return MCE_OK;
}

int mce_release(mce_graph_t g)
{
    if (!g) return MCE_OK;
    // a served job still queued or running holds the handle (checked before
    // the handle's lock, which a running job holds)
    if (g->jobs_in_flight.load() != 0) return MCE_E_BUSY;
    {
        std::lock_guard<std::mutex> lk(g->mu);
        if (g->jobs_in_flight.load() != 0) return MCE_E_BUSY;
        // every solve waits for its own stream before it returns; only the
        // prepare work (ordering, renumbering) and, after a solve that failed
        // before its launch, the build of the local graphs may still be in
        // flight
        if (g->ev[1] && !g->prepared_timed) (void)hipEventSynchronize(g->ev[1]);
        if (g->ev_local) (void)hipEventSynchronize(g->ev_local);
    }
    delete g;
    return MCE_OK;
}

} // extern "C"

// ------------------------------------------------- allocation-free entry --
//
// mce_count_noalloc runs the whole path of one graph (validation, ordering,
// renumbering, root units, search, reduction) on buffers carved out of a
// fixed device scratch area instead of allocated ones.  The area is the
// file-scope device array below; each device the library runs on holds its
// own copy until the process ends.  In host code the array's name is a
// host-side stand-in, not a device address: its device address is taken
// once per device (with that device current) by hipGetSymbolAddress, and only
// that address is ever handed to kernels and copies.

static __device__ __align__(256) unsigned char scratch[MCE_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kNoAllocDevices = 64;
// Fixed parts of the scratch area (the rest is the spill pool): a pool of
// root units, mailboxes and record slots for up to kNoAllocWorkgroups search
// workgroups, and states and exit records for up to kNoAllocWaves wavefronts
// (10 MiB of the area).  Unit records are sized for the widest layout the
// entry point takes (w32 = 64).
constexpr uint32_t kNoAllocW32 = (MCE_NOALLOC_MAX_N + 31u) / 32u;
constexpr uint32_t kNoAllocRecords = 8192, kNoAllocWorkgroups = 1024, kNoAllocWaves = 16384;

struct NoAllocCtx {
    std::mutex mu;
    bool ready = false;
    char* base = nullptr;          // device address of this device's scratch
    mce_graph_s* h = nullptr;      // a handle whose buffers are views of the scratch
    std::vector<unsigned char> host_out; // fixed host block
};

NoAllocCtx g_noalloc[kNoAllocDevices];

// Set-up, once per device, with the device current: the scratch's device
// address and the views of it.  The only allocations are host objects and
// HIP events made here, before the first solve.
int noalloc_setup(NoAllocCtx& x, int dev)
{
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
        (void)hipGetLastError();
        return MCE_E_DEVICE;
    }
    x.base = static_cast<char*>(ptr);
    std::unique_ptr<mce_graph_s> h(new mce_graph_s());
    h->device = dev;
    h->num_graphs = 1;
    h->desc.resize(1);
    h->fixed_ws = true;
    size_t off = 0;
    auto take = [&](DevBuf& b, size_t bytes) {
        bytes = (bytes + 255) & ~(size_t)255;
        b.borrow(x.base + off, bytes);
        off += bytes;
    };
    const size_t rec_bytes = 4ull * (kRecHeader + 4ull * kNoAllocW32);
    take(h->d_desc, sizeof(GraphDesc));
    take(h->d_order, 4ull * MCE_NOALLOC_MAX_N);
    take(h->d_adj, 4ull * ((uint64_t)MCE_NOALLOC_MAX_N * (kNoAllocW32 + 1) + 128));
    take(h->d_out, sizeof(QueueCtl) + sizeof(DevResult) + 8ull * (MCE_NOALLOC_MAX_N + 1));
    take(h->d_params, sizeof(SearchParams));
    take(h->d_sub, 256); // the validation flag
    take(h->d_rec, rec_bytes * kNoAllocRecords);
    take(h->d_mail, sizeof(Mailbox) * kNoAllocWorkgroups);
    take(h->d_mail_rec, rec_bytes * kNoAllocWorkgroups);
    take(h->d_state, 4ull * kNoAllocWaves);
    take(h->d_exit, sizeof(WaveExit) * kNoAllocWaves);
    if (off >= MCE_NOALLOC_SCRATCH_BYTES) return MCE_E_NOMEM;
    h->d_spill.borrow(x.base + off, MCE_NOALLOC_SCRATCH_BYTES - off);
    x.host_out.assign(sizeof(DevResult) + sizeof(QueueCtl) + 8ull * (MCE_NOALLOC_MAX_N + 1), 0);
    h->h_out.borrow(x.host_out.data(), x.host_out.size());
    int rc = ensure_events(h.get());
    if (rc != MCE_OK) return rc;
    x.h = h.release();
    x.ready = true;
    return MCE_OK;
}

} // namespace

extern "C" int mce_count_noalloc(uint32_t n, const uint64_t* rows, uint32_t row_words, mce_result_t* res,
                                 void* hip_stream)
{
    if (!res || n > MCE_NOALLOC_MAX_N) return MCE_E_INVAL;
    if (n > 0 && (!rows || (uint64_t)row_words * 64u < n)) return MCE_E_INVAL;
    if (n == 0) {
        fill_empty_graph(0, UINT64_MAX, res);
        return MCE_OK;
    }
    DeviceInfo di;
    int rc = device_info(&di);
    if (rc != MCE_OK) return rc;
    if (di.device < 0 || di.device >= kNoAllocDevices) return MCE_E_DEVICE;
    NoAllocCtx& x = g_noalloc[di.device];
    std::lock_guard<std::mutex> lk(x.mu);
    if (!x.ready && (rc = noalloc_setup(x, di.device)) != MCE_OK) return rc;
    mce_graph_s* h = x.h;
    std::lock_guard<std::mutex> hl(h->mu);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    // this call's graph: the caller's rows are read in place
    GraphDesc& gd = h->desc[0];
    std::memset(&gd, 0, sizeof(gd));
    gd.idmap_off = kNoMap;
    gd.n = n;
    gd.w32 = (n + 31) / 32;
    gd.rstride = gd.w32 + 1;
    gd.rw64 = row_words;
    h->max_n = n;
    h->max_w32 = gd.w32;
    h->in_words = (uint64_t)n * row_words;
    h->adj_words = (uint64_t)n * gd.rstride;
    h->ord_words = n;
    h->hist_total = n + 1;
    h->tune = mce_graph_s::Tune();
    h->spill_floor = 0;
    h->spill_full_depth = false;
    h->prepared_timed = false;
    HIP_TRY(hipEventRecord(h->ev[0], s));
    HIP_TRY(hipMemcpyAsync(h->d_desc.p, &gd, sizeof(GraphDesc), hipMemcpyHostToDevice, s));
    // validation on the device (zero diagonal, symmetry, no padding bits)
    unsigned int* flag = h->d_sub.as<unsigned int>();
    HIP_TRY(launch_fill_u32(flag, 1, 0u, s));
    HIP_TRY(launch_validate(rows, n, row_words, flag, s));
    unsigned int bad = 0;
    HIP_TRY(hipMemcpyAsync(&bad, flag, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (bad) return MCE_E_INVAL;
    HIP_TRY(launch_order(h->d_desc.as<GraphDesc>(), 1, n, (uint64_t)n * row_words, rows, h->d_order.as<uint32_t>(),
                         nullptr, 0, nullptr, s));
    HIP_TRY(launch_relabel(h->d_desc.as<GraphDesc>(), 1, n, rows, h->d_order.as<uint32_t>(), h->d_adj.as<uint32_t>(), s));
    HIP_TRY(hipEventRecord(h->ev[1], s));
    if ((rc = finish_prepare_timing_locked(h)) != MCE_OK) return rc;
    rc = run_solve(h, 0, UINT64_MAX, res, s, nullptr, 0, nullptr, 0, nullptr, false);
    if (rc != MCE_OK) res->status = rc;
    return rc;
}

// ------------------------------------------------------------ serving ----
//
// Jobs wait in a host FIFO and run on up to kSlots worker threads, each with a
// stream of its own.  A job is admitted when its workspace fits the HBM
// budget and its workgroups' LDS fits what the running jobs leave of the
// device's LDS; its share of the device follows the load at admission: a job
// that starts with nothing else running or waiting gets the share a lone job
// is given (the whole device by default), one that starts while others run
// or wait gets an equal part (at least 1 / kSlots), cut down to the LDS left.
// A running job can be cancelled: its slot's word in coherent pinned host
// memory is set, and the search stops at its next look at its error bits.

namespace {

struct Job {
    uint64_t ticket = 0;
    mce_graph_t g = nullptr;
    int state = 0; // 0 queued, 1 running, 2 done, 3 cancelled before it ran
    int status = MCE_OK;
    uint32_t slot = 0;
    mce_result_t res;
    std::vector<uint64_t> hist;
    uint64_t hbm = 0;             // device memory of the job's workspace (all its workgroups)
    uint32_t blocks_full = 0;     // workgroups of the job's solve on an idle device
    uint64_t lds_per_block = 0;   // LDS bytes one of its workgroups holds
    uint32_t blocks = 0;          // workgroups it was given
};

constexpr uint32_t kSlots = 4;
constexpr size_t kMaxQueued = 1u << 16;

struct Server {
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::shared_ptr<Job>> fifo;
    std::unordered_map<uint64_t, std::shared_ptr<Job>> jobs;
    std::vector<std::thread> workers;
    uint64_t next_ticket = 1;
    uint64_t hbm_budget = 0, hbm_used = 0;
    uint64_t lds_total = 0, lds_used = 0;
    uint32_t running = 0;
    uint32_t alone_pct = 50;  // share of the device's workgroups a job gets when it is alone
    uint32_t wg_per_100v = 0; // at most this many workgroups per 100 vertices of the job's graph (0: no cap)
    uint32_t* cancel = nullptr; // kSlots words, coherent pinned host memory
    bool started = false, stop = false;
    int device = -1;
    ~Server()
    {
        {
            std::lock_guard<std::mutex> lk(mu);
            stop = true;
        }
        cv_work.notify_all();
        for (auto& t : workers)
            if (t.joinable()) t.join();
    }
};

Server& server()
{
    static Server s;
    return s;
}

// The job's demands on an idle device: workgroups, LDS per workgroup, and
// device memory of its workspace.
int job_demand(mce_graph_s* h, Job* job)
{
    LaunchCfg c;
    int rc = make_cfg(h, &c, 0, 0, false, h->local_state == 1);
    if (rc != MCE_OK) return rc;
    const uint64_t rec_words = kRecHeader + 4ull * c.w32cap;
    job->blocks_full = c.blocks;
    job->lds_per_block = search_lds_bytes(c.wave_lds_words, (uint32_t)rec_words, c.wpb);
    job->hbm = sizeof(DevResult) * h->num_graphs + 8ull * h->hist_total + 4ull * c.cap * rec_words +
               (sizeof(Mailbox) + 4ull * rec_words) * c.blocks +
               4ull * spill_frame_words(c.w32cap) * c.spill_levels * c.spill_chunks;
    return MCE_OK;
}

// Workgroups for a queued job now (0: it does not fit yet).  Called with the
// server lock held; waiting = queued jobs, this one included.
uint32_t admit_blocks(const Server& sv, const Job& j, size_t waiting)
{
    if (sv.running != 0 && sv.hbm_used + j.hbm > sv.hbm_budget) return 0;
    uint64_t full = std::max<uint32_t>(j.blocks_full, 1u);
    // a small graph cannot keep many workgroups busy: each one only adds to
    // the launch and to the end of the search
    if (sv.wg_per_100v != 0)
        full = std::min<uint64_t>(full, std::max<uint64_t>(16u, (uint64_t)j.g->desc[0].n * sv.wg_per_100v / 100u));
    uint64_t want;
    if (sv.running == 0 && waiting <= 1) {
        want = std::max<uint64_t>(full * sv.alone_pct / 100, 1);
    } else {
        // as many jobs run at once as there are slots: each gets an equal part
        want = std::max<uint64_t>(full / kSlots, 1);
    }
    const uint64_t lds_free = sv.lds_total > sv.lds_used ? sv.lds_total - sv.lds_used : 0;
    const uint64_t fit = j.lds_per_block ? lds_free / j.lds_per_block : want;
    // a job that would get less than an eighth of its own width waits for
    // more room, unless nothing runs (then it takes what it asked for)
    if (sv.running != 0) {
        want = std::min(want, fit);
        if (want < std::max<uint64_t>(full / 8, 1)) return 0;
    }
    return (uint32_t)want;
}

void worker_loop(uint32_t slot)
{
    Server& sv = server();
    (void)hipSetDevice(sv.device);
    hipStream_t s = nullptr;
    (void)hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    for (;;) {
        std::shared_ptr<Job> job;
        {
            std::unique_lock<std::mutex> lk(sv.mu);
            for (;;) {
                if (sv.stop) break;
                // drop entries cancelled before they ran
                while (!sv.fifo.empty() && sv.fifo.front()->state == 3) sv.fifo.pop_front();
                // the first queued job that fits (FIFO otherwise)
                size_t waiting = 0;
                for (auto& q : sv.fifo) waiting += q->state == 0;
                for (auto it = sv.fifo.begin(); it != sv.fifo.end(); ++it) {
                    if ((*it)->state != 0 || (*it)->g->job_running) continue;
                    const uint32_t b = admit_blocks(sv, **it, waiting);
                    if (b != 0) {
                        job = *it;
                        job->blocks = b;
                        sv.fifo.erase(it);
                        break;
                    }
                }
                if (job) break;
                sv.cv_work.wait(lk);
            }
            if (!job) break;
            job->state = 1;
            job->slot = slot;
            job->g->job_running = true;
            sv.running++;
            sv.hbm_used += job->hbm;
            sv.lds_used += job->lds_per_block * job->blocks;
            __atomic_store_n(&sv.cancel[slot], 0u, __ATOMIC_RELEASE);
        }
        int rc;
        {
            std::lock_guard<std::mutex> hl(job->g->mu);
            rc = finish_prepare_timing_locked(job->g);
            if (rc == MCE_OK)
                rc = run_solve(job->g, 0, UINT64_MAX, &job->res, s, nullptr, 0, nullptr, 0, nullptr, false,
                               job->blocks, nullptr, &sv.cancel[slot]);
        }
        {
            std::lock_guard<std::mutex> lk(sv.mu);
            job->g->job_running = false;
            job->g->jobs_in_flight.fetch_sub(1);
            job->status = rc;
            job->res.status = rc;
            job->state = 2;
            sv.running--;
            sv.hbm_used -= job->hbm;
            sv.lds_used -= job->lds_per_block * job->blocks;
        }
        sv.cv_done.notify_all();
        sv.cv_work.notify_all();
    }
    if (s) (void)hipStreamDestroy(s);
}

int server_start()
{
    Server& sv = server();
    if (sv.started) return MCE_OK;
    DeviceInfo di;
    int rc = device_info(&di);
    if (rc != MCE_OK) return rc;
    size_t free_b = 0, total_b = 0;
    HIP_TRY(hipMemGetInfo(&free_b, &total_b));
    void* flags = nullptr;
    HIP_TRY(hipHostMalloc(&flags, 4 * kSlots, hipHostMallocMapped | hipHostMallocCoherent));
    std::memset(flags, 0, 4 * kSlots);
    sv.cancel = static_cast<uint32_t*>(flags);
    sv.device = di.device;
    sv.hbm_budget = free_b / 2;
    sv.lds_total = (uint64_t)di.cus * di.lds_per_cu;
    if (const char* e = std::getenv("MCE_SERVE_ALONE_PCT")) {
        const long v = std::strtol(e, nullptr, 10);
        if (v >= 1 && v <= 100) sv.alone_pct = (uint32_t)v;
    }
    if (const char* e = std::getenv("MCE_SERVE_WG_PER_100V")) {
        const long v = std::strtol(e, nullptr, 10);
        if (v >= 0 && v <= 100000) sv.wg_per_100v = (uint32_t)v;
    }
    // the LDS the admitted jobs' workgroups may hold together, in percent of
    // the device's (above 100: workgroups of later jobs queue in hardware
    // for LDS that earlier jobs release)
    if (const char* e = std::getenv("MCE_SERVE_LDS_PCT")) {
        const long v = std::strtol(e, nullptr, 10);
        if (v >= 10 && v <= 1000) sv.lds_total = sv.lds_total * (uint64_t)v / 100u;
    }
    for (uint32_t i = 0; i < kSlots; i++) sv.workers.emplace_back(worker_loop, i);
    sv.started = true;
    return MCE_OK;
}

} // namespace

extern "C" {

int mce_submit(mce_graph_t g, uint32_t flags, uint64_t* ticket)
{
    if (!g || !ticket || flags != 0 || g->num_graphs != 1) return MCE_E_INVAL;
    Server& sv = server();
    auto job = std::make_shared<Job>();
    job->g = g;
    std::memset(&job->res, 0, sizeof(job->res));
    job->hist.assign(g->desc[0].n + 1, 0);
    job->res.hist = job->hist.data();
    job->res.hist_len = (uint32_t)job->hist.size();
    {
        std::lock_guard<std::mutex> hl(g->mu);
        int rc = job_demand(g, job.get());
        if (rc != MCE_OK) return rc;
    }
    {
        std::lock_guard<std::mutex> lk(sv.mu);
        int rc = server_start();
        if (rc != MCE_OK) return rc;
        if (sv.fifo.size() >= kMaxQueued) return MCE_E_BUSY;
        job->ticket = sv.next_ticket++;
        g->jobs_in_flight.fetch_add(1);
        sv.jobs[job->ticket] = job;
        sv.fifo.push_back(job);
        *ticket = job->ticket;
    }
    sv.cv_work.notify_one();
    return MCE_OK;
}

int mce_poll(uint64_t ticket, mce_result_t* res, int32_t timeout_us)
{
    if (!res) return MCE_E_INVAL;
    Server& sv = server();
    std::unique_lock<std::mutex> lk(sv.mu);
    auto it = sv.jobs.find(ticket);
    if (it == sv.jobs.end()) return MCE_E_INVAL;
    std::shared_ptr<Job> job = it->second;
    auto done = [&] { return job->state >= 2; };
    if (!done()) {
        if (timeout_us == 0) return MCE_PENDING;
        if (timeout_us < 0) sv.cv_done.wait(lk, done);
        else if (!sv.cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), done)) return MCE_PENDING;
        it = sv.jobs.find(ticket); // another thread may have polled it meanwhile
        if (it == sv.jobs.end()) return MCE_E_INVAL;
    }
    sv.jobs.erase(it);
    if (job->state == 3) return MCE_E_CANCELLED;
    if (job->status != MCE_OK) return job->status;
    uint64_t* user_hist = res->hist;
    const uint32_t user_len = res->hist_len;
    *res = job->res;
    res->hist = user_hist;
    res->hist_len = user_len;
    if (user_hist)
        for (uint32_t k = 0; k < user_len; k++) user_hist[k] = k < job->hist.size() ? job->hist[k] : 0;
    return MCE_OK;
}

int mce_cancel(uint64_t ticket)
{
    Server& sv = server();
    std::lock_guard<std::mutex> lk(sv.mu);
    auto it = sv.jobs.find(ticket);
    if (it == sv.jobs.end()) return MCE_E_INVAL;
    Job& j = *it->second;
    if (j.state == 0) {
        j.state = 3;
        j.g->jobs_in_flight.fetch_sub(1);
        sv.cv_done.notify_all();
        sv.cv_work.notify_all();
        return MCE_OK;
    }
    if (j.state == 1) {
        // the search reads the word at its next look at its error bits
        __atomic_store_n(&sv.cancel[j.slot], 1u, __ATOMIC_RELEASE);
        return MCE_OK;
    }
    return MCE_E_BUSY; // finished (or cancelled) already
}

} // extern "C"
