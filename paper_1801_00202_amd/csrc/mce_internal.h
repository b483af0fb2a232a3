// mce_internal.h -- types shared by the device kernels and the host runtime of
// libmce.so.  Not part of the public ABI (include/mce.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mce {

constexpr uint32_t kMaxN = 16384;
// Per-wavefront clique buffer in LDS: each buffered clique is the list of the
// non-empty 16-bit halves of its input-id bitset, one word per half
// (half index << 16 | bits), in increasing order; at most 64 cliques.
constexpr uint32_t kCliqueSlots = 512;
// Per-wavefront LDS histogram; larger clique sizes go straight to HBM.
constexpr uint32_t kHistLds = 64;
// Words at the head of a queue record (graph index, spare).
constexpr uint32_t kRecHeader = 2;
// Per-workgroup LDS: a header and a LIFO of units shared by its wavefronts.
constexpr uint32_t kWgHdrWords = 16;
constexpr uint32_t kLocalSlots = 8;
// LDS words of a wavefront before its frames: histogram (kHistLds u64), the
// clique buffer (kCliqueSlots words), 64 words that absorb the stores of lanes
// with nothing to store, a 32-word context block and a 128-word save area for
// the search loop's lane registers.  Then come the stack window, the slot of
// the current frame and some slack (lds_frame_words).
constexpr uint32_t kWaveFixedWords = kHistLds * 2 + kCliqueSlots + 64 + 32 + 128;

// Wavefront-lane layout of the search: one 32-bit word per lane and chunk.
// A graph with w32 + 1 <= 64 row words (n <= 2016) uses one chunk, larger ones
// two (the +1 is the input-id word of a row, read while w32 < 128), then four
// (n <= 8160) and eight (n <= kMaxN).
constexpr uint32_t kOneChunkMaxW32 = 63;
inline uint32_t search_chunks(uint32_t max_w32)
{
    return max_w32 <= kOneChunkMaxW32 ? 1u : max_w32 <= 127u ? 2u : max_w32 <= 255u ? 4u : 8u;
}

// Wavefronts per search workgroup at most: four for the wide layouts, whose
// registers per lane would not fit four wavefronts per SIMD.
constexpr uint32_t max_search_wpb(uint32_t chunks) { return chunks >= 4u ? 4u : 16u; }

// LDS stack frame (P, X, L and the row of the frame's next candidate,
// interleaved per lane, 16 bytes a lane): words per frame, and the slack after
// the last frame that absorbs the accesses of lanes past the row.  With one
// chunk a frame spans lanes 0..max_w32, so that the row's input-id word (lane
// w32) is kept.
inline uint32_t lds_frame_words(uint32_t max_w32)
{
    return search_chunks(max_w32) == 1 ? 4u * (max_w32 + 1u) : 256u * search_chunks(max_w32);
}
inline uint32_t lds_slack_words(uint32_t max_w32)
{
    return search_chunks(max_w32) == 1 ? 4u * (63u - max_w32) : 0u;
}
// Spill frame in HBM: (P, X, L, child id) per lane, 16 bytes a lane, all lanes.
inline uint32_t spill_frame_words(uint32_t max_w32) { return 256u * search_chunks(max_w32); }

// One graph of a handle, in device memory.
struct GraphDesc {
    uint32_t n;        // vertices
    uint32_t w32;      // 32-bit words of a bitset, ceil(n/32)
    uint32_t rw64;     // uint64 words of an input row, ceil(n/64)
    uint32_t rstride;  // uint32 words between renumbered rows: w32 + 1 (the last word of a
                       // row holds the vertex's input id)
    uint64_t in_off;   // first uint64 word of the input rows
    uint64_t adj_off;  // first uint32 word of the renumbered rows (row stride rstride)
    uint64_t ord_off;  // first entry of order[] (position -> input id)
    uint64_t hist_off; // first entry of the graph's histogram (n + 1 entries)
    // Local graphs (the root children of a sparse graph of more than 4096
    // vertices, each solved on the subgraph its neighbourhood induces): the
    // ids of a local graph are local ranks, reported through idmap; an
    // ordinary graph has idmap_off = kNoMap.
    uint64_t idmap_off; // first entry of the id map (local id -> input id), or kNoMap
    uint32_t res;       // the DevResult (and histogram) the graph's totals go to
    uint32_t pad;
};
// For a local graph, rw64 holds the root child's position in the whole graph
// and in_off the first word of its node's P and X bitsets (w32 words each,
// local positions) followed by the root child's own local id, in lpx.
constexpr uint64_t kNoMap = ~0ull;
// Vertices of a local graph at most (one-chunk layout: w32 + 1 <= 64).
constexpr uint32_t kLocalMaxN = 2016;
static_assert(sizeof(GraphDesc) == 64, "GraphDesc layout");

// Per-graph totals, accumulated with device atomics.
struct DevResult {
    unsigned long long count, nodes, children, dead_ends, hash_xor, hash_sum;
    unsigned long long root_branches;
    unsigned int omega, status;
    unsigned int unit_base, unit_count; // queue slots of the graph's root units
};

// Control block of one search launch.  Words written by many workgroups sit
// on cache lines of their own.
struct QueueCtl {
    unsigned int pool_next, pad_h[31]; // next root unit to hand out
    unsigned int pool_size, pad_t[31]; // root units written by the root kernels
    unsigned int work, pad_w[31];      // root units not handed out + units in transit
                                       // + workgroups holding work; the search ends at 0
    unsigned int error, pad_e[31];
    unsigned long long donations, units;
    unsigned long long spill_next;           // next free chunk of the spill pool
    unsigned long long spill_levels_written; // stack levels stored in HBM
    unsigned long long vcursor, ocursor;     // enumerate output cursors
    unsigned long long checks, flushes;      // suspensions of the search loop, by reason
    unsigned long long busy_ticks, run_ticks; // wall-clock ticks on units / from start to exit, all wavefronts
    unsigned long long ramp_ticks, tail_ticks; // before the first unit / after the last one
};

// Mailbox of one search workgroup in HBM.  A workgroup out of work asks one
// other workgroup at a time: it writes its id + 1 into that workgroup's req
// word (compare-and-swap from 0), and the asked workgroup answers in the
// asker's state word: a unit (copied to the asker's record slot first) or a
// refusal.  The hint word says how many of the workgroup's wavefronts were
// busy when it last looked (0 when it holds no work), so that askers can
// prefer busy workgroups.  Each word has a cache line of its own.
struct Mailbox {
    unsigned int req, pad_r[31];   // asking workgroup + 1, 0: none
    unsigned int state, pad_s[31]; // answer to this workgroup's own question
    unsigned int hint, pad_b[31];  // busy wavefronts (a hint, written by the owner only)
};
constexpr unsigned int kMailNone = 0u, kMailUnit = 1u, kMailRefused = 2u;

// Exit record of one search wavefront: its totals of the graph it worked on
// last (not yet added to that graph's result slot) and its counters.  The
// exit-fold kernel that runs after the search adds the records up, so that the
// wavefronts, which leave within microseconds of each other, issue no atomics
// on the same few words at once.
constexpr unsigned int kNoSlot = 0xffffffffu;
struct WaveExit {
    unsigned int res, omega; // result slot (kNoSlot: the wavefront held no graph), largest clique
    unsigned long long hist_off; // where hist adds into SearchParams.hist
    unsigned long long count, nodes, children, hash_xor, hash_sum;
    unsigned long long units, donations, spills, checks, flushes; // QueueCtl counters
    unsigned long long busy, run, ramp, tail;                     // wall-clock ticks (QueueCtl *_ticks)
    unsigned long long hist[kHistLds];
};
static_assert(sizeof(WaveExit) == 8 * (16 + kHistLds), "WaveExit layout");

// QueueCtl.error bits
constexpr unsigned int kErrSpill = 1u; // spill pool exhausted: rerun with a larger pool
constexpr unsigned int kErrDepth = 2u; // stack deeper than a spill chunk: rerun with chunks of full depth
constexpr unsigned int kErrWatchdog = 4u; // the search ran past its deadline
constexpr unsigned int kErrCancel = 16u;  // the host asked the search to stop (SearchParams.cancel)
constexpr unsigned int kErrClique = 8u;   // a clique with more non-empty 16-bit id groups than the
                                          // clique buffer's slots (only possible for n > 8192)

struct SearchParams {
    const GraphDesc* graphs;
    const uint32_t* adj;
    const uint32_t* order;
    DevResult* results;
    unsigned long long* hist;
    QueueCtl* ctl;
    uint32_t* rec;            // root units, cap * rec_words
    Mailbox* mail;            // one per workgroup
    uint32_t* mail_rec;       // one record slot per workgroup, rec_words each
    uint32_t* spill;          // per wavefront: spill_levels * slot_words
    uint32_t* verts;          // enumerate output (device) or nullptr
    unsigned long long* offs;
    unsigned long long verts_cap, offs_cap;
    uint32_t num_wg;          // search workgroups
    uint32_t rec_words;       // kRecHeader + 4 * w32cap
    uint32_t w32cap;          // bitset stride in LDS slots and records
    uint32_t slot_words;      // LDS frame stride (lds_frame_words)
    uint32_t spill_words;     // spill frame stride (spill_frame_words)
    uint32_t lds_depth;       // stack levels in LDS
    uint32_t spill_levels;    // stack levels in one spill chunk
    uint32_t spill_chunks;    // chunks in the spill pool
    uint32_t wave_lds_words;  // LDS words per wavefront
    uint32_t split_threshold;
    uint32_t check_interval;
    uint32_t enumerate;
    uint64_t watchdog_ticks;  // wall-clock ticks a wavefront may run (0 = no limit)
    uint32_t refresh_children; // children a workgroup processes between two looks at its mailbox
    uint32_t poll_iters;       // idle iterations between two looks at the end-of-search counter
    uint32_t* wave_state;     // per wavefront: kWave* phase (for deadline reports), or null
    WaveExit* exits;          // per wavefront (blockIdx.x * waves per workgroup + wavefront)
    uint32_t pivot_rule;      // kPivot*
    uint32_t pad0;
    // host-written word in coherent pinned host memory, or null: non-zero asks
    // the search to stop (a served job cancelled while it runs)
    const uint32_t* cancel;
    const uint32_t* idmap;    // id maps of local graphs (GraphDesc.idmap_off), or null
};
// Pivot rules (SearchParams.pivot_rule, MCE_OPT_PIVOT).
constexpr uint32_t kPivotGreedy = 0, kPivotTomita = 1, kPivotTX = 2;

// Phases recorded in SearchParams.wave_state.
constexpr uint32_t kWaveIdle = 1, kWaveFetch = 2, kWaveBusy = 3, kWaveExited = 4;

// Dynamic LDS of one search workgroup.
inline uint32_t search_lds_bytes(uint32_t wave_lds_words, uint32_t rec_words, uint32_t waves)
{
    return 4u * (kWgHdrWords + kLocalSlots * rec_words + wave_lds_words * waves);
}

// Host-side launchers (kernels.hip).
hipError_t launch_validate(const uint64_t* rows, uint32_t n, uint32_t rw, unsigned int* flag,
                           hipStream_t s);
// max_words: the largest n * rw64 of the graphs (their input rows' words).
// nbr: for graphs of more than 4096 vertices, room for cap 16-bit entries
// a vertex (indexed like order), cap = order_list_cap(max_n), used for
// neighbour lists during the ordering, and done: a word a graph; nullptr
// (or cap 0): none.
uint32_t order_list_cap(uint32_t max_n);
hipError_t launch_order(const GraphDesc* graphs, uint32_t num_graphs, uint32_t max_n, uint64_t max_words,
                        const uint64_t* rows_in, uint32_t* order, uint16_t* nbr, uint32_t cap, uint32_t* done,
                        hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, uint32_t count, uint32_t value, hipStream_t s);
hipError_t launch_relabel(const GraphDesc* graphs, uint32_t num_graphs, uint32_t max_n,
                          const uint64_t* rows_in, const uint32_t* order, uint32_t* adj,
                          hipStream_t s);
// Zeroes the results, histogram, mailboxes and control block of a solve, and
// writes sp to params_out when that is not null.
hipError_t launch_reset(const SearchParams& sp, uint32_t num_graphs, uint64_t hist_total,
                        uint32_t workgroups, SearchParams* params_out, hipStream_t s);
hipError_t launch_root(const SearchParams& sp, uint32_t num_graphs, uint32_t max_w32,
                       uint64_t first, uint64_t last, uint32_t max_units, hipStream_t s);
hipError_t launch_subproblem(const SearchParams& sp, uint32_t max_w32, const uint32_t* bits, hipStream_t s);
// Local graphs of the root children of graph gparent (a single graph):
// per position, its degree with bit 31 set when it is a root child; then the
// local graphs themselves (rows, orders, id maps, the P and X bitsets of the
// root child's node at lpx + in_off); then, per solve, the root children with
// branch index in [first, last) as units (or leaves counted at once).
hipError_t launch_local_plan(const GraphDesc* gparent, const uint32_t* adj, uint32_t n, uint32_t* out, hipStream_t s);
hipError_t launch_local_build(const GraphDesc* gparent, const uint32_t* adj, const uint32_t* order, uint32_t n,
                              const GraphDesc* lgraphs, uint32_t count, uint32_t* ladj, uint32_t* lord,
                              uint32_t* lidmap, uint32_t* lpx, hipStream_t s);
hipError_t launch_local_units(const SearchParams& sp, const uint32_t* lpx, uint32_t count, uint32_t max_w32,
                              uint64_t first, uint64_t last, hipStream_t s);
hipError_t launch_search(const SearchParams& sp, const SearchParams* d_sp, uint32_t max_w32, uint32_t blocks,
                         uint32_t waves_per_block, hipStream_t s);
// Adds the exit records of the last search launch's `waves` wavefronts into
// the result slots, the histogram and the control block's counters.
hipError_t launch_exit_fold(const SearchParams& sp, uint32_t waves, hipStream_t s);
hipError_t search_occupancy(uint32_t max_w32, uint32_t rule, uint32_t waves_per_block, uint32_t lds_bytes,
                            int* blocks_per_cu);

} // namespace mce
