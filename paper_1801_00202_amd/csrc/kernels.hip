// kernels.hip -- gfx950 device code of libmce.so.
//
// The search follows Alg. 4 of San Segundo, Artieda & Strash (BKPivotOrdered
// with ChoosePivotOrdered) under the GreedyBB pivot rule of Sec. 4.3, on the
// bitset encoding of Sec. 4.1, after the maximum-degree-first ordering and
// renumbering of Sec. 4.2.
//
// Execution model (gfx950, wave64):
//   * One wavefront owns one subproblem.  A bitset over n vertices is spread
//     over the lanes as 32-bit words: word w lives in lane (w mod 64), register
//     chunk (w div 64); WPL = chunks per lane (1 for n <= 2048, 2 up to 4096).
//     Lanes holding no word keep zeros, so AND/ANDN leave them zero.
//   * Empty tests and "first vertex" scans are a ballot of the non-zero words,
//     a find-first on the scalar mask and a readlane of that word: the pivot
//     and branch choice run on the scalar unit, the set algebra on the vector
//     unit.
//   * The DFS stack keeps the current node (P, X, L) in registers and its
//     ancestors in an LDS window of lds_depth levels per wavefront; deeper
//     levels go to a per-wavefront chunk of an HBM spill pool.
//   * R is kept as a bitset over *input* ids, so a reported clique is already
//     sorted: its ids are written to an LDS buffer by a prefix sum over the
//     lanes and hashed later, one clique per lane.
//   * Work moves between wavefronts through a bounded MPMC queue in HBM.  A
//     busy wavefront that sees the queue short hands over the later half of
//     the candidate set of its shallowest frame: it keeps (P, X, L1) and
//     publishes (R, P \ L1, X u L1, L2), which is exactly what the sequential
//     loop would reach after branching on L1 (steps 12-13 of Alg. 4).
#include "mce_internal.h"

#include <mutex>

namespace mce {
namespace {

constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;

__device__ __forceinline__ uint32_t lane_id()
{
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

__device__ __forceinline__ uint32_t rdlane(uint32_t x, uint32_t l)
{
    return (uint32_t)__builtin_amdgcn_readlane((int)x, (int)l);
}

__device__ __forceinline__ uint32_t bcast0(uint32_t x)
{
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)x);
}

__device__ __forceinline__ uint32_t umax_early(uint32_t a, uint32_t b) { return a > b ? a : b; }

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint32_t dpp(uint32_t x)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, ROW_MASK, 0xf, false);
}

// Inclusive prefix sum over the 64 lanes: shifts by 1, 2, 4, 8 inside each row
// of 16 lanes, then lane 15 of a row is added to the next row and lane 31 to
// the upper half.
__device__ __forceinline__ uint32_t wave_scan_incl(uint32_t x)
{
    x += dpp<0x111, 0xf>(x);
    x += dpp<0x112, 0xf>(x);
    x += dpp<0x114, 0xf>(x);
    x += dpp<0x118, 0xf>(x);
    x += dpp<0x142, 0xa>(x);
    x += dpp<0x143, 0xc>(x);
    return x;
}

// Maximum over the 64 lanes (same pattern; zero is the identity for keys).
__device__ __forceinline__ uint32_t wave_max(uint32_t x)
{
    x = umax_early(x, dpp<0x111, 0xf>(x));
    x = umax_early(x, dpp<0x112, 0xf>(x));
    x = umax_early(x, dpp<0x114, 0xf>(x));
    x = umax_early(x, dpp<0x118, 0xf>(x));
    x = umax_early(x, dpp<0x142, 0xa>(x));
    x = umax_early(x, dpp<0x143, 0xc>(x));
    return rdlane(x, 63);
}

// SplitMix64 output function (Steele, Lea & Flood 2014), modulo 2^64.
__device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// max(a - b, 0) without a branch on the operands.
__device__ __forceinline__ uint32_t sat_sub(uint32_t a, uint32_t b)
{
    const uint32_t m = a > b ? a : b;
    return m - b;
}

__device__ __forceinline__ uint32_t umin32(uint32_t a, uint32_t b) { return a < b ? a : b; }
__device__ __forceinline__ uint32_t umax32(uint32_t a, uint32_t b) { return a > b ? a : b; }

// How many set bits of a word rank below m in a bitset, given the number of
// set bits in earlier words (before) and in this word (cnt).
__device__ __forceinline__ uint32_t rank_take(uint32_t m, uint32_t before, uint32_t cnt)
{
    return umin32(sat_sub(m, before), cnt);
}

// The lowest m set bits of x.
__device__ __forceinline__ uint32_t low_bits(uint32_t x, uint32_t m)
{
    uint32_t r = 0;
    while (m && x) {
        uint32_t b = x & (0u - x);
        r |= b;
        x ^= b;
        m--;
    }
    return r;
}

// ------------------------------------------------------ lane bitsets -----

template <int WPL>
__device__ __forceinline__ bool any_set(const uint32_t (&s)[WPL])
{
    uint32_t o = s[0];
#pragma unroll
    for (int c = 1; c < WPL; c++) o |= s[c];
    return ballot(o != 0) != 0;
}

// Position of the lowest set bit, or -1 if the set is empty.
template <int WPL>
__device__ __forceinline__ int first_bit(const uint32_t (&s)[WPL])
{
#pragma unroll
    for (int c = 0; c < WPL; c++) {
        uint64_t m = ballot(s[c] != 0);
        if (m) {
            uint32_t l = (uint32_t)__builtin_ctzll(m);
            uint32_t w = rdlane(s[c], l);
            return (int)((((uint32_t)c * 64u + l) << 5) | (uint32_t)__builtin_ctz(w));
        }
    }
    return -1;
}

template <int WPL>
__device__ __forceinline__ void clear_bit(uint32_t (&s)[WPL], uint32_t v, uint32_t lane)
{
    const uint32_t wi = v >> 5, m = 1u << (v & 31);
#pragma unroll
    for (int c = 0; c < WPL; c++)
        if ((wi >> 6) == (uint32_t)c) s[c] = (lane == (wi & 63)) ? (s[c] & ~m) : s[c];
}

template <int WPL>
__device__ __forceinline__ void set_bit(uint32_t (&s)[WPL], uint32_t v, uint32_t lane)
{
    const uint32_t wi = v >> 5, m = 1u << (v & 31);
#pragma unroll
    for (int c = 0; c < WPL; c++)
        if ((wi >> 6) == (uint32_t)c) s[c] = (lane == (wi & 63)) ? (s[c] | m) : s[c];
}

// Inclusive prefix of popcounts over all words (chunk-major), and the total.
template <int WPL>
__device__ __forceinline__ uint32_t popc_scan(const uint32_t (&s)[WPL], uint32_t (&cnt)[WPL],
                                              uint32_t (&incl)[WPL])
{
    uint32_t base = 0;
#pragma unroll
    for (int c = 0; c < WPL; c++) {
        cnt[c] = (uint32_t)__builtin_popcount(s[c]);
        incl[c] = wave_scan_incl(cnt[c]) + base;
        base = rdlane(incl[c], 63);
    }
    return base;
}

// ---------------------------------------------------------------- queue ---

// Bounded MPMC queue (sequence number per slot; D. Vyukov's design).  Slot
// seq == pos: free for the producer of ticket pos; seq == pos + 1: holds the
// unit of ticket pos.  Lane 0 runs the protocol; the wavefront moves the data.
__device__ __forceinline__ bool q_pop(const SearchParams& sp, uint32_t lane, uint32_t* out)
{
    uint32_t pos = 0, ok = 0;
    if (lane == 0) {
        unsigned int* head = &sp.ctl->head;
        pos = __hip_atomic_load(head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        for (;;) {
            uint32_t seq = __hip_atomic_load(&sp.seq[pos & sp.cap_mask], __ATOMIC_ACQUIRE,
                                             __HIP_MEMORY_SCOPE_AGENT);
            int32_t dif = (int32_t)(seq - (pos + 1u));
            if (dif == 0) {
                if (__hip_atomic_compare_exchange_weak(head, &pos, pos + 1u, __ATOMIC_RELAXED,
                                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                    ok = 1;
                    break;
                }
            } else if (dif < 0) {
                break; // empty
            } else {
                pos = __hip_atomic_load(head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
    ok = bcast0(ok);
    *out = bcast0(pos);
    return ok != 0;
}

template <int WPL>
__device__ bool q_push(const SearchParams& sp, uint32_t lane, uint32_t g, uint32_t W,
                       const uint32_t (&Rb)[WPL], const uint32_t (&P)[WPL],
                       const uint32_t (&X)[WPL], const uint32_t (&L)[WPL])
{
    uint32_t pos = 0, ok = 0;
    if (lane == 0) {
        unsigned int* tail = &sp.ctl->tail;
        pos = __hip_atomic_load(tail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        for (;;) {
            uint32_t seq = __hip_atomic_load(&sp.seq[pos & sp.cap_mask], __ATOMIC_ACQUIRE,
                                             __HIP_MEMORY_SCOPE_AGENT);
            int32_t dif = (int32_t)(seq - pos);
            if (dif == 0) {
                if (__hip_atomic_compare_exchange_weak(tail, &pos, pos + 1u, __ATOMIC_RELAXED,
                                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                    ok = 1;
                    break;
                }
            } else if (dif < 0) {
                break; // full
            } else {
                pos = __hip_atomic_load(tail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        if (ok) __hip_atomic_fetch_add(&sp.ctl->pending, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    ok = bcast0(ok);
    pos = bcast0(pos);
    if (!ok) return false;
    uint32_t* r = sp.rec + (size_t)(pos & sp.cap_mask) * sp.rec_words;
    const uint32_t cs = sp.w32cap;
    if (lane == 0) r[0] = g;
#pragma unroll
    for (int c = 0; c < WPL; c++) {
        const uint32_t w = (uint32_t)c * 64u + lane;
        if (w < W) {
            r[kRecHeader + w] = Rb[c];
            r[kRecHeader + cs + w] = P[c];
            r[kRecHeader + 2 * cs + w] = X[c];
            r[kRecHeader + 3 * cs + w] = L[c];
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if (lane == 0)
        __hip_atomic_store(&sp.seq[pos & sp.cap_mask], pos + 1u, __ATOMIC_RELEASE,
                           __HIP_MEMORY_SCOPE_AGENT);
    return true;
}

// ------------------------------------------------------------ kernels ----

// Device-side validation of rows given by device pointer: zero diagonal, no
// bit at a column >= n, symmetry.  Any violation sets *flag.
__global__ void validate_kernel(const uint64_t* rows, uint32_t n, uint32_t rw, unsigned int* flag)
{
    const uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (uint64_t)n * rw) return;
    const uint32_t i = (uint32_t)(idx / rw), w = (uint32_t)(idx % rw);
    uint64_t x = rows[idx];
    bool bad = false;
    if (w == (i >> 6) && ((x >> (i & 63)) & 1u)) bad = true;
    const uint64_t lo = (uint64_t)w * 64u;
    if (lo + 64u > n) {
        uint64_t valid = (lo >= n) ? 0ull : ((1ull << (n - lo)) - 1ull);
        if (x & ~valid) bad = true;
        x &= valid;
    }
    while (x) {
        const uint32_t b = (uint32_t)__builtin_ctzll(x);
        x &= x - 1;
        const uint32_t j = (uint32_t)lo + b;
        if (!((rows[(uint64_t)j * rw + (i >> 6)] >> (i & 63)) & 1u)) bad = true;
    }
    if (bad) atomicOr(flag, 1u);
}

// Maximum-degree-first ordering (Sec. 4.2), one wavefront per graph.  Vertex v
// belongs to lane v / KPL, slot v % KPL, and holds the key
// (deg + 1) << 12 | (4095 - v): the wave maximum of the keys is the vertex of
// largest remaining degree, ties to the smaller id.  Taken vertices hold 0.
template <int KPL>
__global__ void __launch_bounds__(64) order_kernel(const GraphDesc* graphs, const uint64_t* rows_in,
                                                   uint32_t* order)
{
    const GraphDesc gd = graphs[blockIdx.x];
    const uint32_t n = gd.n;
    if (n == 0) return;
    const uint32_t lane = lane_id();
    const uint64_t* in = rows_in + gd.in_off;
    const uint32_t rs = gd.rw64;
    const uint32_t v0 = lane * KPL;
    const uint32_t cw = v0 >> 6, csh = v0 & 63; // word and shift of this lane's row chunk
    const uint64_t cmask = ~0ull >> (64 - KPL);
    uint32_t key[KPL];
#pragma unroll
    for (int j = 0; j < KPL; j++) {
        const uint32_t v = v0 + (uint32_t)j;
        uint32_t deg = 0;
        if (v < n)
            for (uint32_t t = 0; t < rs; t++) deg += (uint32_t)__builtin_popcountll(in[(uint64_t)v * rs + t]);
        key[j] = (v < n) ? (((deg + 1u) << 12) | (4095u - v)) : 0u;
    }
    uint32_t* ord = order + gd.ord_off;
    for (uint32_t i = 0; i < n; i++) {
        uint32_t m = 0;
#pragma unroll
        for (int j = 0; j < KPL; j++) m = umax32(m, key[j]);
        m = wave_max(m);
        const uint32_t v = 4095u - (m & 4095u);
        if (lane == 0) ord[i] = v;
        const uint64_t chunk = (v0 < n) ? ((in[(uint64_t)v * rs + cw] >> csh) & cmask) : 0ull;
        const uint64_t vm = ((v / KPL) == lane) ? (1ull << (v % KPL)) : 0ull;
#pragma unroll
        for (int j = 0; j < KPL; j++) {
            const bool nb = ((chunk >> j) & 1ull) && key[j] != 0u;
            key[j] = ((vm >> j) & 1ull) ? 0u : (key[j] - (nb ? 4096u : 0u));
        }
    }
}

// Renumbering (Sec. 4.2): row i of the new matrix is row order[i] of the input
// with column j taken from column order[j].  Block (i, g), one word per thread.
__global__ void __launch_bounds__(64) relabel_kernel(const GraphDesc* graphs, const uint64_t* rows_in,
                                                     const uint32_t* order, uint32_t* adj)
{
    const GraphDesc gd = graphs[blockIdx.y];
    const uint32_t i = blockIdx.x;
    if (i >= gd.n) return;
    const uint32_t n = gd.n;
    const uint32_t* ord = order + gd.ord_off;
    const uint64_t* src = rows_in + gd.in_off + (uint64_t)ord[i] * gd.rw64;
    uint32_t* dst = adj + gd.adj_off + (uint64_t)i * gd.w32;
    for (uint32_t w = threadIdx.x; w < gd.w32; w += blockDim.x) {
        uint32_t val = 0;
        for (uint32_t b = 0; b < 32; b++) {
            const uint32_t j = w * 32u + b;
            if (j >= n) break;
            const uint32_t o = ord[j];
            val |= (uint32_t)((src[o >> 6] >> (o & 63)) & 1ull) << b;
        }
        dst[w] = val;
    }
}

// Zero the per-graph results and the control block; seq[i] = i (all slots free).
__global__ void reset_kernel(SearchParams sp, uint32_t num_graphs, uint64_t hist_total, uint32_t cap)
{
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    unsigned long long* res = reinterpret_cast<unsigned long long*>(sp.results);
    const uint64_t res_words = (uint64_t)num_graphs * (sizeof(DevResult) / 8);
    for (uint64_t i = tid; i < res_words; i += stride) res[i] = 0ull;
    for (uint64_t i = tid; i < hist_total; i += stride) sp.hist[i] = 0ull;
    for (uint64_t i = tid; i < cap; i += stride) sp.seq[i] = (unsigned int)i;
    if (tid < sizeof(QueueCtl) / 8) reinterpret_cast<unsigned long long*>(sp.ctl)[tid] = 0ull;
}

// Root of each graph (R = {}, P = V, X = {}): its pivot is the first vertex
// of P (position 0), so L0 = {0} u (V \ N(0)).  The children with branch index
// in [first, last) become one unit: P = V minus the earlier children, X = the
// earlier children, L = the selected children.  The root node counts iff
// first == 0.  One wavefront per graph.
template <int WPL>
__global__ void __launch_bounds__(64) root_kernel(SearchParams sp, uint64_t first, uint64_t last)
{
    const uint32_t g = blockIdx.x;
    const GraphDesc gd = sp.graphs[g];
    const uint32_t n = gd.n;
    if (n == 0) return;
    const uint32_t lane = lane_id();
    const uint32_t W = gd.w32;
    const uint32_t* row0 = sp.adj + gd.adj_off;
    uint32_t V[WPL], L0[WPL], cnt[WPL], incl[WPL];
#pragma unroll
    for (int c = 0; c < WPL; c++) {
        const uint32_t w = (uint32_t)c * 64u + lane;
        uint32_t full = 0;
        if (w < W) full = (w == W - 1 && (n & 31)) ? ((1u << (n & 31)) - 1u) : 0xffffffffu;
        V[c] = full;
        L0[c] = full & ~((w < W) ? row0[w] : 0u);
    }
    const uint32_t total = popc_scan<WPL>(L0, cnt, incl);
    if (lane == 0) {
        sp.results[g].root_branches = total;
        if (first == 0) atomicAdd(&sp.results[g].nodes, 1ull);
    }
    const uint32_t lo = first < (uint64_t)total ? (uint32_t)first : total;
    const uint32_t hi = last < (uint64_t)total ? (uint32_t)last : total;
    if (lo >= hi) return;
    uint32_t Rb[WPL], P[WPL], X[WPL], L[WPL];
#pragma unroll
    for (int c = 0; c < WPL; c++) {
        const uint32_t before = incl[c] - cnt[c];
        const uint32_t nb = rank_take(lo, before, cnt[c]);
        const uint32_t nh = rank_take(hi, before, cnt[c]);
        const uint32_t lb = low_bits(L0[c], nb);
        const uint32_t lh = low_bits(L0[c], nh);
        Rb[c] = 0;
        X[c] = lb;
        P[c] = V[c] & ~lb;
        L[c] = lh & ~lb;
    }
    q_push<WPL>(sp, lane, g, W, Rb, P, X, L);
}

// The persistent search.  See the header comment for the layout.
template <int WPL>
__global__ void __launch_bounds__(1024) search_kernel(SearchParams sp)
{
    extern __shared__ uint32_t smem[];
    const uint32_t lane = lane_id();
    const uint32_t wv = threadIdx.x >> 6;
    uint32_t* wl = smem + (size_t)wv * sp.wave_lds_words;
    unsigned long long* hist_l = reinterpret_cast<unsigned long long*>(wl);
    uint32_t* cent = wl + kHistLds * 2;
    uint16_t* cids = reinterpret_cast<uint16_t*>(cent + kCliqueEntries);
    uint32_t* stk = cent + kCliqueEntries + kCliqueIds / 2;
    const uint32_t SW = sp.slot_words, CS = sp.w32cap;
    uint32_t* spill = nullptr;  // this wavefront's chunk of the spill pool, taken on first use

    for (uint32_t i = lane; i < kHistLds; i += 64) hist_l[i] = 0ull;

    const uint64_t t_start = wall_clock64();
    auto overdue = [&]() -> bool {
        return sp.watchdog_ticks != 0 && wall_clock64() - t_start > sp.watchdog_ticks;
    };
    uint64_t acc_x = 0, acc_s = 0;                 // per lane: hashes of flushed cliques
    uint32_t nent = 0, used = 0;                   // clique buffer fill (uniform)
    uint64_t c_nodes = 0, c_children = 0, c_dead = 0, c_count = 0;
    uint32_t c_omega = 0;
    uint64_t n_units = 0, n_don = 0, n_spill = 0;

    for (;;) {
        uint32_t pos;
        if (!q_pop(sp, lane, &pos)) {
            uint32_t pend = 0, err = 0;
            if (lane == 0) {
                pend = __hip_atomic_load(&sp.ctl->pending, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                err = __hip_atomic_load(&sp.ctl->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            pend = bcast0(pend);
            err = bcast0(err);
            if (pend == 0 || err != 0) break;
            if (overdue()) {
                if (lane == 0) atomicOr(&sp.ctl->error, kErrWatchdog);
                break;
            }
            __builtin_amdgcn_s_sleep(8);
            continue;
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        const uint32_t* rec = sp.rec + (size_t)(pos & sp.cap_mask) * sp.rec_words;
        const uint32_t g = bcast0(rec[0]);
        const GraphDesc gd = sp.graphs[g];
        const uint32_t W = gd.w32;
        uint32_t Rb[WPL], P[WPL], X[WPL], L[WPL], roff[WPL];
#pragma unroll
        for (int c = 0; c < WPL; c++) {
            const uint32_t w = (uint32_t)c * 64u + lane;
            const bool in = w < W;
            Rb[c] = in ? rec[kRecHeader + w] : 0u;
            P[c] = in ? rec[kRecHeader + CS + w] : 0u;
            X[c] = in ? rec[kRecHeader + 2 * CS + w] : 0u;
            L[c] = in ? rec[kRecHeader + 3 * CS + w] : 0u;
            roff[c] = in ? w : (W - 1u);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        if (lane == 0)
            __hip_atomic_store(&sp.seq[pos & sp.cap_mask], pos + sp.cap_mask + 1u, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        n_units++;

        const uint32_t* adj = sp.adj + gd.adj_off;
        const uint32_t* ord = sp.order + gd.ord_off;
        unsigned long long* ghist = sp.hist + gd.hist_off;
        uint32_t d = 0;               // frames of this unit on the stack
        uint32_t since = sp.check_interval; // look at the queue right away
        bool abort = false;

        // ---- clique buffer: hash, histogram and (enumerate) output ----
        auto hist_add = [&](uint32_t k, uint32_t c) {
            if (k < kHistLds) {
                if (lane == 0) hist_l[k] += c;
            } else if (lane == 0) {
                atomicAdd(&ghist[k], (unsigned long long)c);
            }
        };
        auto flush = [&]() {
            if (nent == 0) return;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            const bool mine = lane < nent;
            const uint32_t e = mine ? cent[lane] : 0u;
            const uint32_t st = e & 0xffffu, k = e >> 16;
            if (mine) {
                uint64_t h = mix64((uint64_t)k);
                for (uint32_t j = 0; j < k; j++) h = mix64(h + kGolden + (uint64_t)cids[st + j]);
                acc_x ^= h;
                acc_s += h;
            }
            uint64_t rem = ballot(mine);
            while (rem) {
                const uint32_t l0 = (uint32_t)__builtin_ctzll(rem);
                const uint32_t k0 = rdlane(k, l0);
                const uint64_t m = ballot(mine && k == k0);
                hist_add(k0, (uint32_t)__builtin_popcountll(m));
                rem &= ~m;
            }
            if (sp.enumerate) {
                unsigned long long vb = 0, ob = 0;
                if (lane == 0) {
                    vb = atomicAdd(&sp.ctl->vcursor, (unsigned long long)used);
                    ob = atomicAdd(&sp.ctl->ocursor, 2ull * nent);
                }
                vb = ((unsigned long long)bcast0((uint32_t)(vb >> 32)) << 32) | bcast0((uint32_t)vb);
                ob = ((unsigned long long)bcast0((uint32_t)(ob >> 32)) << 32) | bcast0((uint32_t)ob);
                if (vb + used <= sp.verts_cap && ob + 2ull * nent <= sp.offs_cap) {
                    for (uint32_t i = lane; i < used; i += 64) sp.verts[vb + i] = cids[i];
                    if (mine) {
                        sp.offs[ob + 2ull * lane] = vb + st;
                        sp.offs[ob + 2ull * lane + 1ull] = vb + st + k;
                    }
                }
            }
            c_count += nent;
            nent = 0;
            used = 0;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        };
        // Report R u {v} (idv = input id of v): R is the bitset Rb over input
        // ids, so the clique's sorted ids are the set bits in lane order.
        auto report = [&](uint32_t idv) {
            uint32_t cw[WPL], cnt[WPL], incl[WPL];
            const uint32_t iw = idv >> 5, im = 1u << (idv & 31);
#pragma unroll
            for (int c = 0; c < WPL; c++)
                cw[c] = Rb[c] | (((uint32_t)c * 64u + lane == iw) ? im : 0u);
            const uint32_t k = popc_scan<WPL>(cw, cnt, incl);
            c_omega = umax32(c_omega, k);
            if (k > kCliqueIds) {
                // Very large clique: hash it in place on the scalar unit.
                uint64_t h = mix64((uint64_t)k);
#pragma unroll
                for (int c = 0; c < WPL; c++) {
                    uint64_t m = ballot(cw[c] != 0);
                    while (m) {
                        const uint32_t l = (uint32_t)__builtin_ctzll(m);
                        m &= m - 1;
                        uint32_t w = rdlane(cw[c], l);
                        while (w) {
                            const uint32_t b = (uint32_t)__builtin_ctz(w);
                            w &= w - 1;
                            h = mix64(h + kGolden + (uint64_t)((((uint32_t)c * 64u + l) << 5) | b));
                        }
                    }
                }
                if (lane == 0) {
                    acc_x ^= h;
                    acc_s += h;
                }
                hist_add(k, 1);
                c_count += 1;
                if (sp.enumerate) {
                    unsigned long long vb = 0, ob = 0;
                    if (lane == 0) {
                        vb = atomicAdd(&sp.ctl->vcursor, (unsigned long long)k);
                        ob = atomicAdd(&sp.ctl->ocursor, 2ull);
                    }
                    vb = ((unsigned long long)bcast0((uint32_t)(vb >> 32)) << 32) | bcast0((uint32_t)vb);
                    ob = ((unsigned long long)bcast0((uint32_t)(ob >> 32)) << 32) | bcast0((uint32_t)ob);
                    if (vb + k <= sp.verts_cap && ob + 2ull <= sp.offs_cap) {
#pragma unroll
                        for (int c = 0; c < WPL; c++) {
                            uint64_t p = vb + incl[c] - cnt[c];
                            uint32_t x = cw[c];
                            const uint32_t wb = ((uint32_t)c * 64u + lane) << 5;
                            while (x) {
                                sp.verts[p++] = wb | (uint32_t)__builtin_ctz(x);
                                x &= x - 1;
                            }
                        }
                        if (lane == 0) {
                            sp.offs[ob] = vb;
                            sp.offs[ob + 1] = vb + k;
                        }
                    }
                }
                return;
            }
            if (nent == kCliqueEntries || used + k > kCliqueIds) flush();
            const uint32_t base = used;
#pragma unroll
            for (int c = 0; c < WPL; c++) {
                uint32_t p = base + incl[c] - cnt[c];
                uint32_t x = cw[c];
                const uint32_t wb = ((uint32_t)c * 64u + lane) << 5;
                while (x) {
                    cids[p++] = (uint16_t)(wb | (uint32_t)__builtin_ctz(x));
                    x &= x - 1;
                }
            }
            if (lane == 0) cent[nent] = base | (k << 16);
            used += k;
            nent++;
        };

        // ---- stack frames ----
        // frame s: P, X, L of the node at depth s of this unit, after steps
        // 12-13 for the child being explored, and the input id of that child.
        auto spill_base = [&]() -> bool {
            if (spill) return true;
            uint32_t chunk = 0;
            if (lane == 0) chunk = (uint32_t)atomicAdd(&sp.ctl->spill_next, 1ull);
            chunk = bcast0(chunk);
            if (chunk >= sp.spill_chunks) {
                if (lane == 0) atomicOr(&sp.ctl->error, kErrSpill);
                return false;
            }
            spill = sp.spill + (size_t)chunk * sp.spill_levels * SW;
            return true;
        };
        (void)spill_base;

        for (;;) {
            int vi = first_bit<WPL>(L);
            if (vi < 0) {
                // node finished: return to the parent frame
                if (d == 0) break;
                d--;
                uint32_t idv;
                if (d < sp.lds_depth) {
                    const uint32_t* f = stk + (size_t)d * SW;
#pragma unroll
                    for (int c = 0; c < WPL; c++) {
                        const uint32_t w = (uint32_t)c * 64u + lane;
                        const bool in = w < W;
                        P[c] = in ? f[w] : 0u;
                        X[c] = in ? f[CS + w] : 0u;
                        L[c] = in ? f[2 * CS + w] : 0u;
                    }
                    idv = bcast0(f[3 * CS]);
                } else {
                    const uint32_t* f = spill + (size_t)(d - sp.lds_depth) * SW;
#pragma unroll
                    for (int c = 0; c < WPL; c++) {
                        const uint32_t w = (uint32_t)c * 64u + lane;
                        const bool in = w < W;
                        P[c] = in ? f[w] : 0u;
                        X[c] = in ? f[CS + w] : 0u;
                        L[c] = in ? f[2 * CS + w] : 0u;
                    }
                    idv = bcast0(f[3 * CS]);
                }
                clear_bit<WPL>(Rb, idv, lane);
                continue;
            }
            const uint32_t v = (uint32_t)vi;
            // step 11: P' = P n N(v), X' = X n N(v)
            const uint32_t* rv = adj + (size_t)v * W;
            uint32_t row[WPL];
#pragma unroll
            for (int c = 0; c < WPL; c++) row[c] = rv[roff[c]];
            const uint32_t idv = ord[v];
            clear_bit<WPL>(L, v, lane);
            uint32_t P2[WPL], X2[WPL];
#pragma unroll
            for (int c = 0; c < WPL; c++) {
                P2[c] = P[c] & row[c];
                X2[c] = X[c] & row[c];
            }
            // steps 12-13 for the current node
            clear_bit<WPL>(P, v, lane);
            set_bit<WPL>(X, v, lane);
            c_children++;
            if (any_set<WPL>(P2)) {
                // the child is a node: push the current frame, descend
                c_nodes++;
                if (d < sp.lds_depth) {
                    uint32_t* f = stk + (size_t)d * SW;
#pragma unroll
                    for (int c = 0; c < WPL; c++) {
                        const uint32_t w = (uint32_t)c * 64u + lane;
                        if (w < W) {
                            f[w] = P[c];
                            f[CS + w] = X[c];
                            f[2 * CS + w] = L[c];
                        }
                    }
                    if (lane == 0) f[3 * CS] = idv;
                } else {
                    if (d - sp.lds_depth >= sp.spill_levels) {
                        if (lane == 0) atomicOr(&sp.ctl->error, kErrDepth);
                        abort = true;
                        break;
                    }
                    if (!spill_base()) {
                        abort = true;
                        break;
                    }
                    uint32_t* f = spill + (size_t)(d - sp.lds_depth) * SW;
#pragma unroll
                    for (int c = 0; c < WPL; c++) {
                        const uint32_t w = (uint32_t)c * 64u + lane;
                        if (w < W) {
                            f[w] = P[c];
                            f[CS + w] = X[c];
                            f[2 * CS + w] = L[c];
                        }
                    }
                    if (lane == 0) f[3 * CS] = idv;
                    n_spill++;
                }
                d++;
                set_bit<WPL>(Rb, idv, lane);
#pragma unroll
                for (int c = 0; c < WPL; c++) {
                    P[c] = P2[c];
                    X[c] = X2[c];
                }
                // step 9: pivot = first of X if X is non-empty, else first of P
                int pi = first_bit<WPL>(X);
                if (pi < 0) pi = first_bit<WPL>(P);
                // step 10: L = P \ N(p)
                const uint32_t* rp = adj + (size_t)(uint32_t)pi * W;
#pragma unroll
                for (int c = 0; c < WPL; c++) L[c] = P[c] & ~rp[roff[c]];
            } else if (!any_set<WPL>(X2)) {
                report(idv); // P' and X' empty: R u {v} is maximal
            } else {
                c_dead++;
            }

            // ---- work donation ----
            if (++since >= sp.check_interval) {
                since = 0;
                uint32_t qs = 0, err = 0;
                if (lane == 0) {
                    const uint32_t t = __hip_atomic_load(&sp.ctl->tail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    const uint32_t h = __hip_atomic_load(&sp.ctl->head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    err = __hip_atomic_load(&sp.ctl->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    qs = t - h;
                }
                qs = bcast0(qs);
                if (bcast0(err) != 0) {
                    abort = true;
                    break;
                }
                if (overdue()) {
                    if (lane == 0) atomicOr(&sp.ctl->error, kErrWatchdog);
                    abort = true;
                    break;
                }
                if (qs < sp.split_threshold) {
                    // shallowest frame with at least two candidates left
                    for (uint32_t s = 0; s <= d; s++) {
                        uint32_t Ls[WPL], Ps[WPL], Xs[WPL];
                        const uint32_t* f = nullptr;
                        bool in_lds = s < sp.lds_depth;
                        if (s == d) {
#pragma unroll
                            for (int c = 0; c < WPL; c++) {
                                Ls[c] = L[c];
                                Ps[c] = P[c];
                                Xs[c] = X[c];
                            }
                        } else {
                            f = in_lds ? (stk + (size_t)s * SW) : (spill + (size_t)(s - sp.lds_depth) * SW);
#pragma unroll
                            for (int c = 0; c < WPL; c++) {
                                const uint32_t w = (uint32_t)c * 64u + lane;
                                Ls[c] = (w < W) ? f[2 * CS + w] : 0u;
                            }
                        }
                        uint32_t cnt[WPL], incl[WPL];
                        const uint32_t tot = popc_scan<WPL>(Ls, cnt, incl);
                        if (tot < 2) continue;
                        if (s != d) {
#pragma unroll
                            for (int c = 0; c < WPL; c++) {
                                const uint32_t w = (uint32_t)c * 64u + lane;
                                Ps[c] = (w < W) ? f[w] : 0u;
                                Xs[c] = (w < W) ? f[CS + w] : 0u;
                            }
                        }
                        const uint32_t keep = (tot + 1u) / 2u;
                        uint32_t L1[WPL], L2[WPL], Pd[WPL], Xd[WPL], Rs[WPL];
#pragma unroll
                        for (int c = 0; c < WPL; c++) {
                            const uint32_t before = incl[c] - cnt[c];
                            const uint32_t nk = rank_take(keep, before, cnt[c]);
                            L1[c] = low_bits(Ls[c], nk);
                            L2[c] = Ls[c] & ~L1[c];
                            Pd[c] = Ps[c] & ~L1[c];
                            Xd[c] = Xs[c] | L1[c];
                            Rs[c] = Rb[c];
                        }
                        // R of frame s: drop the children pushed from frames s..d-1
                        for (uint32_t j = s; j < d; j++) {
                            const uint32_t* fj = (j < sp.lds_depth) ? (stk + (size_t)j * SW)
                                                                    : (spill + (size_t)(j - sp.lds_depth) * SW);
                            clear_bit<WPL>(Rs, bcast0(fj[3 * CS]), lane);
                        }
                        if (q_push<WPL>(sp, lane, g, W, Rs, Pd, Xd, L2)) {
                            n_don++;
                            if (s == d) {
#pragma unroll
                                for (int c = 0; c < WPL; c++) L[c] = L1[c];
                            } else {
                                uint32_t* fw = in_lds ? (stk + (size_t)s * SW)
                                                      : (spill + (size_t)(s - sp.lds_depth) * SW);
#pragma unroll
                                for (int c = 0; c < WPL; c++) {
                                    const uint32_t w = (uint32_t)c * 64u + lane;
                                    if (w < W) fw[2 * CS + w] = L1[c];
                                }
                            }
                        }
                        break;
                    }
                }
            }
        }

        // ---- unit finished: fold its totals into graph g ----
        flush();
        {
            uint64_t x = acc_x, s = acc_s;
            for (int off = 32; off > 0; off >>= 1) {
                x ^= __shfl_xor(x, off);
                s += __shfl_xor(s, off);
            }
            if (lane == 0) {
                DevResult* r = sp.results + g;
                if (c_count) atomicAdd(&r->count, (unsigned long long)c_count);
                if (c_nodes) atomicAdd(&r->nodes, (unsigned long long)c_nodes);
                if (c_children) atomicAdd(&r->children, (unsigned long long)c_children);
                if (c_dead) atomicAdd(&r->dead_ends, (unsigned long long)c_dead);
                if (x) atomicXor(&r->hash_xor, (unsigned long long)x);
                if (s) atomicAdd(&r->hash_sum, (unsigned long long)s);
                if (c_omega) atomicMax(&r->omega, c_omega);
            }
            for (uint32_t i = lane; i < kHistLds; i += 64) {
                const unsigned long long hv = hist_l[i];
                if (hv) {
                    atomicAdd(&ghist[i], hv);
                    hist_l[i] = 0ull;
                }
            }
            acc_x = acc_s = 0;
            c_count = c_nodes = c_children = c_dead = 0;
            c_omega = 0;
        }
        if (lane == 0) __hip_atomic_fetch_sub(&sp.ctl->pending, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        if (abort) break;
    }
    if (lane == 0) {
        if (n_units) atomicAdd(&sp.ctl->units, (unsigned long long)n_units);
        if (n_don) atomicAdd(&sp.ctl->donations, (unsigned long long)n_don);
        if (n_spill) atomicAdd(&sp.ctl->spill_levels_written, (unsigned long long)n_spill);
    }
}

} // namespace

// ---------------------------------------------------------- launchers ----

hipError_t launch_validate(const uint64_t* rows, uint32_t n, uint32_t rw, unsigned int* flag,
                           hipStream_t s)
{
    const uint64_t total = (uint64_t)n * rw;
    if (total == 0) return hipSuccess;
    const uint32_t blocks = (uint32_t)((total + 255) / 256);
    hipLaunchKernelGGL(validate_kernel, dim3(blocks), dim3(256), 0, s, rows, n, rw, flag);
    return hipGetLastError();
}

hipError_t launch_order(const GraphDesc* graphs, uint32_t num_graphs, uint32_t max_n,
                        const uint64_t* rows_in, uint32_t* order, hipStream_t s)
{
    if (max_n <= 512)
        hipLaunchKernelGGL(order_kernel<8>, dim3(num_graphs), dim3(64), 0, s, graphs, rows_in, order);
    else if (max_n <= 1024)
        hipLaunchKernelGGL(order_kernel<16>, dim3(num_graphs), dim3(64), 0, s, graphs, rows_in, order);
    else if (max_n <= 2048)
        hipLaunchKernelGGL(order_kernel<32>, dim3(num_graphs), dim3(64), 0, s, graphs, rows_in, order);
    else
        hipLaunchKernelGGL(order_kernel<64>, dim3(num_graphs), dim3(64), 0, s, graphs, rows_in, order);
    return hipGetLastError();
}

hipError_t launch_relabel(const GraphDesc* graphs, uint32_t num_graphs, uint32_t max_n,
                          const uint64_t* rows_in, const uint32_t* order, uint32_t* adj,
                          hipStream_t s)
{
    if (max_n == 0) return hipSuccess;
    hipLaunchKernelGGL(relabel_kernel, dim3(max_n, num_graphs), dim3(64), 0, s, graphs, rows_in,
                       order, adj);
    return hipGetLastError();
}

hipError_t launch_reset(const SearchParams& sp, uint32_t num_graphs, uint64_t hist_total,
                        uint32_t cap, hipStream_t s)
{
    uint64_t work = hist_total;
    if (work < cap) work = cap;
    if (work < (uint64_t)num_graphs * 8) work = (uint64_t)num_graphs * 8;
    uint32_t blocks = (uint32_t)((work + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    if (blocks == 0) blocks = 1;
    hipLaunchKernelGGL(reset_kernel, dim3(blocks), dim3(256), 0, s, sp, num_graphs, hist_total, cap);
    return hipGetLastError();
}

hipError_t launch_root(const SearchParams& sp, uint32_t num_graphs, uint32_t max_w32,
                       uint64_t first, uint64_t last, hipStream_t s)
{
    if (max_w32 <= 64)
        hipLaunchKernelGGL(root_kernel<1>, dim3(num_graphs), dim3(64), 0, s, sp, first, last);
    else
        hipLaunchKernelGGL(root_kernel<2>, dim3(num_graphs), dim3(64), 0, s, sp, first, last);
    return hipGetLastError();
}

static hipError_t ensure_search_attr()
{
    // Allow the search kernels the full LDS of a workgroup once per process.
    static std::once_flag once;
    static hipError_t err = hipSuccess;
    std::call_once(once, [] {
        int dev = 0, lds = 0;
        err = hipGetDevice(&dev);
        if (err == hipSuccess) err = hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
        if (err == hipSuccess)
            err = hipFuncSetAttribute((const void*)search_kernel<1>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        if (err == hipSuccess)
            err = hipFuncSetAttribute((const void*)search_kernel<2>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    });
    return err;
}

hipError_t launch_search(const SearchParams& sp, uint32_t max_w32, uint32_t blocks,
                         uint32_t waves_per_block, hipStream_t s)
{
    const uint32_t lds = sp.wave_lds_words * 4u * waves_per_block;
    hipError_t e = ensure_search_attr();
    if (e != hipSuccess) return e;
    if (max_w32 <= 64)
        hipLaunchKernelGGL(search_kernel<1>, dim3(blocks), dim3(64 * waves_per_block), lds, s, sp);
    else
        hipLaunchKernelGGL(search_kernel<2>, dim3(blocks), dim3(64 * waves_per_block), lds, s, sp);
    return hipGetLastError();
}

hipError_t search_occupancy(uint32_t max_w32, uint32_t waves_per_block, uint32_t lds_bytes,
                            int* blocks_per_cu)
{
    const void* k = (max_w32 <= 64) ? (const void*)search_kernel<1> : (const void*)search_kernel<2>;
    hipError_t e = ensure_search_attr();
    if (e != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k, (int)(64 * waves_per_block),
                                                        lds_bytes);
}

} // namespace mce
