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

// The write-lane operation (no clang builtin for it here): the compiler puts
// the lane number in M0, as the instruction's operand rules require.
__device__ int amdgcn_writelane(int src, int lane, int old) __asm("llvm.amdgcn.writelane.i32");

namespace mce {
namespace {

constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;

__device__ __forceinline__ uint32_t lane_id()
{
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// Lanes whose x is non-zero, as a 64-bit mask (a compare into a scalar pair:
// repeated tests of one word share it).
__device__ __forceinline__ uint64_t nz_mask(uint32_t x) { return __builtin_amdgcn_uicmp(x, 0u, 33 /* ne */); }

__device__ __forceinline__ uint32_t rdlane(uint32_t x, uint32_t l)
{
    return (uint32_t)__builtin_amdgcn_readlane((int)x, (int)l);
}

// x with lane l (uniform, below 64) replaced by the uniform value v.
__device__ __forceinline__ uint32_t wrlane(uint32_t x, uint32_t v, uint32_t l)
{
    return (uint32_t)amdgcn_writelane((int)v, (int)l, (int)x);
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

// Sum over the 64 lanes.
__device__ __forceinline__ uint32_t wave_sum(uint32_t x) { return rdlane(wave_scan_incl(x), 63); }

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
    return nz_mask(o) != 0;
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

// Position of the lowest set bit, or -1: the lane's candidate position is
// formed on the vector side and one lane is read, so the scalar side does a
// single find-first.  lane_lo[c] = 32 * (64 c + lane).
template <int WPL>
__device__ __forceinline__ int first_pos(const uint32_t (&s)[WPL], const uint32_t (&lane_lo)[WPL])
{
#pragma unroll
    for (int c = 0; c < WPL; c++) {
        const uint64_t m = nz_mask(s[c]);
        if (m) {
            // only a lane with a set bit is read: no guard for an empty word
            const uint32_t pos = lane_lo[c] | (uint32_t)__builtin_ctz(s[c]);
            return (int)rdlane(pos, (uint32_t)__builtin_ctzll(m));
        }
    }
    return -1;
}

// Position of the lowest set bit of a set known to be non-empty.
template <int WPL>
__device__ __forceinline__ int first_pos_nz(const uint32_t (&s)[WPL], const uint32_t (&lane_lo)[WPL])
{
    if (WPL == 1) {
        const uint64_t m = nz_mask(s[0]);
        const uint32_t pos = lane_lo[0] | (uint32_t)__builtin_ctz(s[0]);
        return (int)rdlane(pos, (uint32_t)__builtin_ctzll(m));
    }
    return first_pos<WPL>(s, lane_lo);
}

// The one-bit mask of position v (uniform) in this lane's words: the word
// index and the bit are scalars, one compare and one select per word.
// lane_w[c] = 64 c + lane.
template <int WPL>
__device__ __forceinline__ void bit_mask(uint32_t v, const uint32_t (&lane_w)[WPL], uint32_t (&m)[WPL])
{
    const uint32_t wi = v >> 5, b = 1u << (v & 31u);
    if (WPL == 1) {
        // one word per lane: the bit written into lane wi of a zero word (v
        // is wave-uniform, so its lane is a scalar)
        m[0] = wrlane(0u, b, wi);
        return;
    }
#pragma unroll
    for (int c = 0; c < WPL; c++) m[c] = lane_w[c] == wi ? b : 0u;
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

// ------------------------------------------------ words shared in HBM ---
//
// Coherence across the XCDs' separate L2 caches: every word that crosses
// workgroups (records, mailboxes, counters) is read and written with
// device-scope accesses (sc1), which bypass the non-coherent cache levels, and
// a wait for all outstanding vector memory operations (vmcnt(0)) separates a
// record from the word that publishes it.  No L2 write-back or invalidate is
// ever issued, so the adjacency rows cached in L2 stay put.

__device__ __forceinline__ uint32_t ld_dev(const uint32_t* p)
{
    return __hip_atomic_load(const_cast<uint32_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void st_dev(uint32_t* p, uint32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The launch's error bits, with a cancellation asked by the host folded in
// when `look` (read from coherent host memory at system scope: a round trip
// over the host link, so callers look only now and then).  Lane 0 only.
__device__ __forceinline__ uint32_t error_or_cancel(const SearchParams& sp, bool look)
{
    uint32_t e = ld_dev(&sp.ctl->error);
    if (e == 0u && look && sp.cancel &&
        __hip_atomic_load(const_cast<uint32_t*>(sp.cancel), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) != 0u) {
        atomicOr(&sp.ctl->error, kErrCancel);
        e = kErrCancel;
    }
    return e;
}

// Wait until every vector memory access issued so far has completed.
__device__ __forceinline__ void vm_drain()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup"); // no compiler motion across
    __builtin_amdgcn_s_waitcnt(0x0F70);                     // vmcnt(0)
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Copy a unit (R, P, X, L of graph g) into a record in HBM.
template <int WPL>
__device__ __forceinline__ void store_record(uint32_t* r, uint32_t cs, uint32_t lane, uint32_t g, uint32_t W,
                                             const uint32_t (&Rb)[WPL], const uint32_t (&P)[WPL],
                                             const uint32_t (&X)[WPL], const uint32_t (&L)[WPL])
{
    if (lane == 0) st_dev(&r[0], g);
#pragma unroll
    for (int c = 0; c < WPL; c++) {
        const uint32_t w = (uint32_t)c * 64u + lane;
        if (w < W) {
            st_dev(&r[kRecHeader + w], Rb[c]);
            st_dev(&r[kRecHeader + cs + w], P[c]);
            st_dev(&r[kRecHeader + 2 * cs + w], X[c]);
            st_dev(&r[kRecHeader + 3 * cs + w], L[c]);
        }
    }
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
// largest remaining degree, ties to the smaller id.  Taken vertices hold 0 and
// are out of the lane's mask of remaining vertices, so that a round costs one
// maximum, one read of the chosen vertex's row chunk and one decrement per
// slot.  The order is written 64 entries at a time from one register.  rows
// is the graph's input rows (rw64 64-bit words each), in LDS or global memory.
template <int KPL>
__device__ __forceinline__ void order_rounds(const GraphDesc& gd, const uint64_t* rows, uint32_t* ord)
{
    using CT = typename std::conditional<KPL == 64, uint64_t, uint32_t>::type;
    const uint32_t n = gd.n;
    const uint32_t lane = lane_id();
    const uint32_t rs = gd.rw64;
    const uint32_t v0 = lane * KPL;
    const CT cmask = (CT)(~0ull >> (64 - KPL));
    // this lane's chunk of a row: word cw (of CT) at shift csh; a lane past n
    // reads the row's last word (its slots are not in the mask)
    const uint32_t rsw = KPL == 64 ? rs : 2u * rs;
    const uint32_t cw = umin32(KPL == 64 ? lane : (v0 >> 5), rsw - 1u);
    const uint32_t csh = KPL == 64 ? 0u : (v0 & 31u);
    const CT* rw = reinterpret_cast<const CT*>(rows);
    uint32_t key[KPL];
    CT alive = 0;
#pragma unroll
    for (int j = 0; j < KPL; j++) {
        const uint32_t v = v0 + (uint32_t)j;
        uint32_t deg = 0;
        if (v < n)
            for (uint32_t t = 0; t < rs; t++) deg += (uint32_t)__builtin_popcountll(rows[(uint64_t)v * rs + t]);
        key[j] = (v < n) ? (((deg + 1u) << 12) | (4095u - v)) : 0u;
        alive |= (v < n) ? ((CT)1 << j) : (CT)0;
    }
    uint32_t obuf = 0;
    for (uint32_t i = 0; i < n; i++) {
        uint32_t m = 0;
#pragma unroll
        for (int j = 0; j < KPL; j++) m = umax32(m, key[j]);
        m = wave_max(m);
        const uint32_t v = 4095u - (m & 4095u);
        obuf = wrlane(obuf, v, i & 63u);
        if ((i & 63u) == 63u || i + 1u == n) {
            if (lane <= (i & 63u)) ord[(i & ~63u) + lane] = obuf;
        }
        const uint32_t lv = v / KPL, jv = v % KPL;
        const CT nb = (CT)(rw[(uint64_t)v * rsw + cw] >> csh) & cmask & alive;
        alive &= ~(lane == lv ? ((CT)1 << jv) : (CT)0);
#pragma unroll
        for (int j = 0; j < KPL; j++) {
            const int t = (int)__builtin_amdgcn_ubfe((uint32_t)(nb >> (j & ~31)), (uint32_t)(j & 31), 1u);
            key[j] = (uint32_t)((int)key[j] + t * -4096);
        }
        key[jv] = lane == lv ? 0u : key[jv];
    }
}

template <int KPL>
__global__ void __launch_bounds__(64) order_kernel(const GraphDesc* graphs, const uint64_t* rows_in,
                                                   uint32_t* order)
{
    const GraphDesc gd = graphs[blockIdx.x];
    if (gd.n == 0) return;
    order_rounds<KPL>(gd, rows_in + gd.in_off, order + gd.ord_off);
}

// The same ordering with the graph's input rows staged in LDS first (when
// they fit), so that each of the n dependent rounds reads the chosen vertex's
// row chunk from LDS instead of waiting for a global load.
template <int KPL>
__global__ void __launch_bounds__(64) order_lds_kernel(const GraphDesc* graphs, const uint64_t* rows_in,
                                                       uint32_t* order)
{
    extern __shared__ uint64_t rows_l[];
    const GraphDesc gd = graphs[blockIdx.x];
    const uint32_t n = gd.n;
    if (n == 0) return;
    const uint64_t* in = rows_in + gd.in_off;
    const uint64_t words = (uint64_t)n * gd.rw64;
    // sixteen loads in flight a lane before their stores (one at a time, the
    // copy of a 1000-vertex graph's rows took longer than its rounds)
    constexpr uint32_t kStageBatch = 16;
    for (uint64_t i0 = lane_id(); i0 < words; i0 += 64u * kStageBatch) {
        uint64_t w[kStageBatch];
#pragma unroll
        for (uint32_t k = 0; k < kStageBatch; k++) {
            const uint64_t i = i0 + 64u * k;
            w[k] = i < words ? in[i] : 0ull;
        }
#pragma unroll
        for (uint32_t k = 0; k < kStageBatch; k++) {
            const uint64_t i = i0 + 64u * k;
            if (i < words) rows_l[i] = w[k];
        }
    }
    __syncthreads();
    order_rounds<KPL>(gd, rows_l, order + gd.ord_off);
}

// The same ordering for graphs of up to kMaxN vertices: a workgroup of 16
// wavefronts, 16 vertices a lane, keys (deg + 1) << 14 | (16383 - v).  Each
// round the wavefronts' maxima meet in LDS (two slot rows in turn, so one
// barrier a round suffices: a row is written again only after every
// wavefront has passed the barrier that follows its last read) and every
// wavefront takes the maximum of the 16.  The row chunk of the runner-up
// (the largest of the other 15 wavefront maxima, the next round's choice
// unless it is a neighbour of this round's or its wavefront's next maximum
// is larger) is requested one round ahead.
__global__ void __launch_bounds__(1024) order_wide_kernel(const GraphDesc* graphs, const uint64_t* rows_in,
                                                          uint32_t* order)
{
    constexpr int KPL = 16;
    __shared__ uint32_t red[2][16];
    const GraphDesc gd = graphs[blockIdx.x];
    const uint32_t n = gd.n;
    if (n == 0) return;
    const uint32_t t = threadIdx.x, lane = lane_id(), wave = bcast0(t >> 6);
    const uint64_t* rows = rows_in + gd.in_off;
    const uint32_t rs = gd.rw64, rsw = 2u * rs;
    const uint32_t v0 = t * KPL;
    // this thread's 16 bits of a row: 32-bit word cw at shift csh (a thread
    // past n reads the row's last word; its slots are not in the mask)
    const uint32_t cw = umin32(v0 >> 5, rsw - 1u), csh = v0 & 31u;
    const uint32_t* rw = reinterpret_cast<const uint32_t*>(rows);
    uint32_t key[KPL];
    uint32_t alive = 0;
#pragma unroll
    for (int j = 0; j < KPL; j++) {
        const uint32_t v = v0 + (uint32_t)j;
        uint32_t deg = 0;
        if (v < n)
            for (uint32_t q = 0; q < rs; q++) deg += (uint32_t)__builtin_popcountll(rows[(uint64_t)v * rs + q]);
        key[j] = (v < n) ? (((deg + 1u) << 14) | (16383u - v)) : 0u;
        alive |= (v < n) ? (1u << j) : 0u;
    }
    uint32_t* ord = order + gd.ord_off;
    uint32_t obuf = 0;
    uint32_t pre_v = 0xffffffffu, pre_w = 0;
    // a wavefront none of whose vertices lost a neighbour or was taken keeps
    // its maximum from the previous round (most of them, on sparse graphs)
    uint32_t wmax = 0;
#pragma unroll
    for (int j = 0; j < KPL; j++) wmax = umax32(wmax, key[j]);
    wmax = wave_max(wmax);
    for (uint32_t i = 0; i < n; i++) {
        if (lane == 0) red[i & 1u][wave] = wmax;
        __syncthreads();
        const uint32_t wm = red[i & 1u][lane & 15u];
        const uint32_t m = wave_max(wm);
        const uint32_t v = 16383u - (m & 16383u);
        const uint32_t m2 = wave_max(wm == m ? 0u : wm);
        const uint32_t word = v == pre_v ? pre_w : rw[(uint64_t)v * rsw + cw];
        if (m2 != 0u) {
            pre_v = 16383u - (m2 & 16383u);
            pre_w = rw[(uint64_t)pre_v * rsw + cw];
        } else {
            pre_v = 0xffffffffu;
        }
        if (wave == 0u) {
            obuf = wrlane(obuf, v, i & 63u);
            if (((i & 63u) == 63u || i + 1u == n) && lane <= (i & 63u)) ord[(i & ~63u) + lane] = obuf;
        }
        const uint32_t owner = v / KPL, jv = v % KPL;
        const uint32_t nb = (word >> csh) & 0xffffu & alive;
        if (ballot(nb != 0u || t == owner) != 0u) {
            alive &= ~(t == owner ? (1u << jv) : 0u);
#pragma unroll
            for (int j = 0; j < KPL; j++) key[j] -= ((nb >> j) & 1u) << 14;
            key[jv] = t == owner ? 0u : key[jv];
            uint32_t lm = 0;
#pragma unroll
            for (int j = 0; j < KPL; j++) lm = umax32(lm, key[j]);
            wmax = wave_max(lm);
        }
    }
}

// Degree of every vertex (the popcount of its input row), one wavefront per
// row, into deg (indexed like order): the first pass of the bucket ordering.
// With nbr, also the vertex's neighbour list if its degree is at most cap:
// cap 16-bit slots a vertex (indexed like order), the neighbours in
// increasing id, then 0xffff in the slots left (the bucket kernel reads the
// lists only when every vertex has one).
__global__ void __launch_bounds__(256) degree_kernel(const GraphDesc* graphs, const uint64_t* rows_in, uint32_t* deg,
                                                     uint16_t* nbr, uint32_t cap)
{
    const GraphDesc gd = graphs[blockIdx.y];
    const uint32_t row = blockIdx.x * 4u + (threadIdx.x >> 6);
    if (row >= gd.n) return;
    const uint32_t lane = lane_id();
    const uint64_t* r = rows_in + gd.in_off + (uint64_t)row * gd.rw64;
    uint32_t c = 0;
    for (uint32_t w = lane; w < gd.rw64; w += 64) c += (uint32_t)__builtin_popcountll(r[w]);
    c = wave_sum(c);
    if (lane == 0) deg[gd.ord_off + row] = c;
    if (nbr == nullptr || c > cap) return;
    // the list (the row's words read again, from the cache)
    uint16_t* lst = nbr + (size_t)(gd.ord_off + row) * cap;
    for (uint32_t e = c + lane; e < cap; e += 64) lst[e] = 0xffffu;
    uint32_t b = 0; // entries before this lane's word of the current group
    for (uint32_t w0 = 0; w0 < gd.rw64; w0 += 64) {
        const uint32_t w = w0 + lane;
        uint64_t x = w < gd.rw64 ? r[w] : 0ull;
        const uint32_t pc = (uint32_t)__builtin_popcountll(x);
        const uint32_t incl = wave_scan_incl(pc);
        for (uint32_t e = b + incl - pc; x; e++, x &= x - 1ull) lst[e] = (uint16_t)((w << 6) | (uint32_t)__builtin_ctzll(x));
        b += rdlane(incl, 63);
    }
}

// Maximum-degree-first ordering by degree buckets (Sec. 4.2), one workgroup
// of 16 wavefronts per graph.  The vertices of the largest remaining degree d,
// taken in increasing id, are exactly the next picks of the one-at-a-time rule
// as long as each is adjacent to none of those picked before it in the same
// round: picking a vertex lowers only its neighbours' degrees, so a bucket
// member that is not a neighbour keeps degree d and is then the largest key
// left (ties go to the smaller id); a member that is a neighbour drops below d
// and waits for a later round.  So a round takes d = the largest degree and
// scans the bucket in id order, and the number of rounds is far below n on
// sparse graphs.  The scan goes by chunks of up to 64 members still at degree
// d: all wavefronts copy the chunk's input rows to LDS (direct-to-LDS loads)
// and form, for each member, the mask of earlier chunk members adjacent to it
// (one ballot a member: lane i tests member i's bit in the member's row);
// wavefront 0 takes the members with an empty mask at once and decides the
// others one by one in member order (a pick iff no earlier pick is in its
// mask); then all wavefronts lower the degrees of the picks' neighbours (LDS
// atomics on the neighbours still in the graph, found by ANDing each row word
// with a bitset of the remaining vertices).  LDS: the remaining degree + 1 of
// every vertex (0: taken), the bitset of remaining vertices, the round's
// bucket (16-bit ids, up to kBucketCand), and the chunk's rows (KW x 64 words
// each, plus one word of padding, so that lane j's row starts in bank j).
// The list variant (LS = 2: graphs whose largest degree is at most 128)
// stages each member's neighbour list (128 16-bit slots from degree_kernel)
// instead of its row: a member's mask is gathered by LDS atomic ORs from the
// chunk positions of its neighbours (a byte a vertex in LDS), and the
// decrements go through the slots, two a lane, with all the reads of a
// wavefront's four members in flight together (on G(10^4, p <= 0.005) a
// quarter less time than the rows' word-wise work).
// order holds the degrees from degree_kernel on entry and the order on exit.
constexpr uint32_t kBucketCand = 2048;
// vertices a thread scans per round: ceil(n / 1024), made odd
constexpr uint32_t kBucketKpt = ((kMaxN + 1023u) >> 10) | 1u;

struct BucketShared {
    uint64_t conf[64];  // the chunk: earlier members adjacent to each member
    uint32_t red[16], red2[16];
    uint32_t chk[64];   // the chunk: member ids
    uint32_t cnum, cursor, pos, pad;
    uint64_t pick;
};
// LDS the bucket kernels hold besides their dynamic part (BucketShared, rounded up)
constexpr uint32_t kBucketStaticLds = 1024;
static_assert(sizeof(BucketShared) <= kBucketStaticLds, "static LDS of the bucket kernels");

// Dynamic LDS words of a bucket kernel for graphs of up to n vertices, before
// the staged rows: degrees, the bitset of remaining vertices, the bucket.
__host__ __device__ constexpr uint32_t bucket_fixed_words(uint32_t n)
{
    return ((n + 63u) & ~63u) + ((((n + 31u) >> 5) + 63u) & ~63u) + kBucketCand / 2;
}

template <int KW, int LS>
__global__ void __launch_bounds__(1024) order_bucket_kernel(const GraphDesc* graphs, const uint64_t* rows_in,
                                                            uint32_t* order, uint32_t ch, const uint16_t* nbr,
                                                            uint32_t cap, uint32_t* done)
{
    extern __shared__ uint32_t lds[];
    __shared__ BucketShared sh;
    const GraphDesc gd = graphs[blockIdx.x];
    const uint32_t n = gd.n;
    static_assert(LS == 0 || LS == 2, "rows, or lists of 128 slots");
    constexpr bool LISTS = LS > 0;
    constexpr uint32_t LSX = LS > 0 ? (uint32_t)LS : 1u; // slots a lane of a member's list
    // the row kernel leaves the graphs that the list kernel ordered
    if (!LISTS && done != nullptr && done[blockIdx.x] != 0u) return;
    if (n == 0) return;
    const uint32_t t = threadIdx.x, lane = lane_id(), wave = bcast0(t >> 6);
    constexpr uint32_t NWV = 16;
    const uint32_t nw = (n + 31u) >> 5;                                      // words that hold vertex bits
    uint32_t* vw = lds;                                                      // n words
    uint32_t* alive = lds + ((n + 63u) & ~63u);                              // nw words
    uint16_t* cand = reinterpret_cast<uint16_t*>(alive + ((nw + 63u) & ~63u)); // kBucketCand
    uint32_t* rowbuf = lds + bucket_fixed_words(n);
    constexpr uint32_t RS = KW * 64u + 1u; // LDS words between staged rows
    uint32_t* ord = order + gd.ord_off;
    const uint32_t* rw = reinterpret_cast<const uint32_t*>(rows_in + gd.in_off);
    const uint32_t rs32 = 2u * gd.rw64; // 32-bit words of an input row
    for (uint32_t v = t; v < n; v += 1024) vw[v] = ord[v] + 1u;
    for (uint32_t w = t; w < nw; w += 1024) alive[w] = (w + 1u < nw || (n & 31u) == 0u) ? ~0u : ((1u << (n & 31u)) - 1u);
    if (t == 0) sh.pos = 0;
    __syncthreads();
    // vertices of this thread for the per-round scans: [v0, v1) (an odd
    // count a thread, so that a wavefront's words of a scan step sit in
    // distinct LDS banks)
    const uint32_t kpt = ((n + 1023u) >> 10) | 1u;
    const uint32_t v0 = umin32(t * kpt, n), v1 = umin32(v0 + kpt, n);
    // LS > 0: the chunk's neighbour lists are staged instead of its rows,
    // 64 LS slots a member (LS per lane), followed in LDS by cpos, the chunk
    // position of every vertex (0xff: not in the chunk).  The list kernel
    // orders a graph only if its largest degree is at most 64 LS (every
    // vertex has a list), and flags in done which graphs it ordered.
    bool first = LISTS;
    uint8_t* cpos = reinterpret_cast<uint8_t*>(rowbuf + 64u * 32u * (uint32_t)LS);
    // the round's choice among the members base .. base + pn - 1 of the
    // chunk, from their masks of adjacent earlier members (wavefront 0):
    // members adjacent to no earlier member are picks; the others in member
    // order, against the picks before them
    auto choose = [&](uint64_t& pick, uint32_t base, uint32_t pn) {
        const bool inpass = lane >= base && lane < base + pn;
        const uint64_t cme = inpass ? sh.conf[lane] : 0ull;
        pick |= ballot(inpass && cme == 0ull);
        uint64_t rest = ballot(inpass && cme != 0ull);
        while (rest) {
            const uint32_t j = (uint32_t)__builtin_ctzll(rest);
            rest &= rest - 1ull;
            const uint64_t cj = ((uint64_t)rdlane((uint32_t)(cme >> 32), j) << 32) | rdlane((uint32_t)cme, j);
            if ((cj & pick) == 0ull) pick |= 1ull << j;
        }
        if (lane == 0) sh.pick = pick;
    };
    for (;;) {
        // this thread's remaining degrees + 1, read once a round
        uint32_t val[kBucketKpt];
#pragma unroll
        for (uint32_t k = 0; k < kBucketKpt; k++) {
            const uint32_t v = v0 + k;
            const uint32_t x = vw[umin32(v, n - 1u)];
            val[k] = (k < kpt && v < v1) ? x : 0u;
        }
        // the largest remaining degree + 1
        uint32_t mx = 0;
#pragma unroll
        for (uint32_t k = 0; k < kBucketKpt; k++) mx = umax32(mx, val[k]);
        mx = wave_max(mx);
        if (lane == 0) sh.red[wave] = mx;
        __syncthreads();
        mx = wave_max(lane < NWV ? sh.red[lane] : 0u);
        if (mx == 0u) break;
        if (first) {
            // the first round's maximum is the largest degree + 1
            first = false;
            if (mx > 64u * LS + 1u) {
                if (t == 0) done[blockIdx.x] = 0u;
                return;
            }
            for (uint32_t v = t; v < n; v += 1024) cpos[v] = 0xffu;
        }
        // its bucket, in increasing id (threads hold consecutive id ranges)
        uint32_t cnt = 0;
#pragma unroll
        for (uint32_t k = 0; k < kBucketKpt; k++) cnt += val[k] == mx ? 1u : 0u;
        const uint32_t incl = wave_scan_incl(cnt);
        if (lane == 63) sh.red2[wave] = incl;
        __syncthreads();
        const uint32_t wtot = lane < NWV ? sh.red2[lane] : 0u;
        const uint32_t wincl = wave_scan_incl(wtot);
        const uint32_t total = rdlane(wincl, NWV - 1);
        uint32_t k0 = rdlane(wincl - wtot, wave) + incl - cnt;
#pragma unroll
        for (uint32_t k = 0; k < kBucketKpt; k++) {
            if (val[k] == mx) {
                if (k0 < kBucketCand) cand[k0] = (uint16_t)(v0 + k);
                k0++;
            }
        }
        const uint32_t T = umin32(total, kBucketCand);
        if (t == 0) sh.cursor = 0;
        __syncthreads();
        for (;;) {
            // the next chunk: up to 64 members still at the round's degree
            if (wave == 0) {
                uint32_t i = sh.cursor, cn = 0;
                while (i < T && cn < 64u) {
                    const uint32_t c = i + lane < T ? (uint32_t)cand[i + lane] : 0u;
                    const bool live = i + lane < T && vw[c] == mx;
                    const uint64_t lv = ballot(live);
                    const uint32_t room = 64u - cn;
                    const uint32_t rk = __builtin_amdgcn_mbcnt_hi((uint32_t)(lv >> 32),
                                                                  __builtin_amdgcn_mbcnt_lo((uint32_t)lv, 0u));
                    if (live && rk < room) sh.chk[cn + rk] = c;
                    const uint32_t nl = (uint32_t)__builtin_popcountll(lv);
                    if (nl <= room) {
                        cn += nl;
                        i += 64u;
                    } else {
                        // the chunk fills up inside this group: resume after its
                        // last member taken
                        uint64_t m = lv;
                        for (uint32_t q = 0; q < room; q++) m &= m - 1ull;
                        i += (uint32_t)__builtin_ctzll(m);
                        cn = 64u;
                    }
                }
                if (lane == 0) {
                    sh.cursor = i;
                    sh.cnum = cn;
                }
                if (LISTS) {
                    sh.conf[lane] = 0ull;
                    if (lane < cn) cpos[sh.chk[lane]] = (uint8_t)lane;
                }
            }
            __syncthreads();
            const uint32_t cnum = sh.cnum;
            if (cnum == 0u) break;
            // member ids, one per lane (lanes past the chunk: member 0)
            const uint32_t cl = lane < cnum ? sh.chk[lane] : sh.chk[0];
            // rows of the chunk into LDS: row j's words [64 q, 64 q + 64) by
            // one load of a wavefront (words past the row's end read the
            // row's first word and are never looked at); chunks of more than
            // ch members take several passes
            uint64_t pick = 0;
            if (LISTS) {
                // the members' lists into LDS, 64 LS slots (32 LS words)
                // each; wavefront w takes members w, w + 16, w + 32, w + 48
                // and alone reads their lists, LS slots a lane, all 4 LS
                // reads of a step in flight together
                constexpr uint32_t NU = 4u * LSX, MW = 32u * LSX;
                const uint16_t* lg = nbr + (size_t)gd.ord_off * cap;
                for (uint32_t j = wave; j < cnum; j += NWV) {
                    const uint32_t* src = reinterpret_cast<const uint32_t*>(lg + (size_t)sh.chk[j] * cap);
#pragma unroll
                    for (uint32_t h = 0; h < MW / 64u; h++)
                        __builtin_amdgcn_global_load_lds(src + h * 64u + lane, rowbuf + j * MW + h * 64u, 4, 0, 0);
                }
                __builtin_amdgcn_s_waitcnt(0x0F70); // vmcnt(0): this wavefront's lists are in LDS
                const uint16_t* l16 = reinterpret_cast<const uint16_t*>(rowbuf);
                uint32_t u[NU];
#pragma unroll
                for (uint32_t k = 0; k < NU; k++) {
                    const uint32_t j = wave + NWV * (k / LSX);
                    u[k] = j < cnum ? (uint32_t)l16[j * 2u * MW + (k % LSX) * 64u + lane] : 0xffffu;
                }
                // member j: the earlier members among its neighbours
                uint32_t q[NU];
#pragma unroll
                for (uint32_t k = 0; k < NU; k++) q[k] = u[k] != 0xffffu ? (uint32_t)cpos[u[k]] : 0xffu;
#pragma unroll
                for (uint32_t k = 0; k < NU; k++) {
                    const uint32_t j = wave + NWV * (k / LSX);
                    if (q[k] < j) atomicOr(reinterpret_cast<unsigned long long*>(&sh.conf[j]), 1ull << q[k]);
                }
                __syncthreads();
                if (wave == 0) choose(pick, 0u, cnum);
                __syncthreads();
                pick = sh.pick;
                // the picks' neighbours still in the graph lose one degree
                uint32_t a[NU];
#pragma unroll
                for (uint32_t k = 0; k < NU; k++) {
                    const uint32_t j = wave + NWV * (k / LSX);
                    if (j >= cnum || !((pick >> j) & 1ull)) u[k] = 0xffffu;
                    a[k] = u[k] != 0xffffu ? alive[u[k] >> 5] : 0u;
                }
#pragma unroll
                for (uint32_t k = 0; k < NU; k++)
                    if ((a[k] >> (u[k] & 31u)) & 1u) atomicSub(&vw[u[k]], 1u);
                __syncthreads();
            }
            for (uint32_t base = 0; !LISTS && base < cnum; base += ch) {
                const uint32_t pn = umin32(ch, cnum - base);
                for (uint32_t j = wave; j < pn; j += NWV) {
                    const uint32_t* src = rw + (size_t)sh.chk[base + j] * rs32;
#pragma unroll
                    for (int q = 0; q < KW; q++) {
                        const uint32_t wi = (uint32_t)q * 64u + lane;
                        __builtin_amdgcn_global_load_lds(src + (wi < rs32 ? wi : 0u),
                                                         rowbuf + j * RS + (uint32_t)q * 64u, 4, 0, 0);
                    }
                }
                __builtin_amdgcn_s_waitcnt(0x0F70); // vmcnt(0): this wavefront's rows are in LDS
                __syncthreads();
                // member base + j: which earlier members its row holds
                for (uint32_t j = wave; j < pn; j += NWV) {
                    const uint32_t w = rowbuf[j * RS + (cl >> 5)];
                    const uint64_t cj = ballot((((w >> (cl & 31u)) & 1u) != 0u) & (lane < base + j));
                    if (lane == 0) sh.conf[base + j] = cj;
                }
                __syncthreads();
                if (wave == 0) choose(pick, base, pn);
                __syncthreads();
                pick = sh.pick;
                // the picks' neighbours still in the graph lose one degree
                // (picks are pairwise non-adjacent and no neighbour of an
                // earlier pick of the round, so none of them is touched)
                for (uint32_t j = wave; j < pn; j += NWV) {
                    if (!((pick >> (base + j)) & 1ull)) continue;
                    const uint32_t* r = rowbuf + j * RS;
                    uint32_t bits[KW];
#pragma unroll
                    for (int q = 0; q < KW; q++) {
                        // (every staged word and alive word is read; the
                        // words past the row's vertex bits are masked)
                        const uint32_t wi = (uint32_t)q * 64u + lane;
                        const uint32_t x = r[wi] & alive[umin32(wi, nw - 1u)];
                        bits[q] = wi < nw ? x : 0u;
                    }
#pragma unroll
                    for (int q = 0; q < KW; q++) {
                        const uint32_t wb = ((uint32_t)q * 64u + lane) << 5;
                        uint32_t b = bits[q];
                        while (b) {
                            const uint32_t u = wb | (uint32_t)__builtin_ctz(b);
                            b &= b - 1u;
                            atomicSub(&vw[u], 1u);
                        }
                    }
                }
                __syncthreads();
            }
            // the picks, in member order, are the next entries of the order;
            // they leave the graph
            if (wave == 0) {
                const uint32_t pos = sh.pos;
                if ((pick >> lane) & 1ull) {
                    const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(pick >> 32),
                                                                    __builtin_amdgcn_mbcnt_lo((uint32_t)pick, 0u));
                    ord[pos + rank] = cl;
                    vw[cl] = 0u;
                    atomicAnd(&alive[cl >> 5], ~(1u << (cl & 31u)));
                }
                if (LISTS && lane < cnum) cpos[cl] = 0xffu;
                if (lane == 0) sh.pos = pos + (uint32_t)__builtin_popcountll(pick);
            }
            __syncthreads();
        }
    }
    if (LISTS && t == 0) done[blockIdx.x] = 1u;
}

// Renumbering (Sec. 4.2): row i of the new matrix is row order[i] of the input
// with column j taken from column order[j].  A workgroup of four wavefronts
// renumbers kRelabelRows rows of one graph (blockIdx.y): it inverts the order
// into LDS (pos[order[j]] = j), then each wavefront takes a row at a time,
// scatters the row's set bits to their positions in an LDS row (one LDS atomic
// OR a neighbour: work in the row's degree, not in n) and writes the row out.
// LDS: ceil64(max n) words of pos, then a row of ceil64(max w32) words per
// wavefront.
constexpr uint32_t kRelabelRows = 16;

__host__ __device__ constexpr uint32_t relabel_lds_words(uint32_t max_n)
{
    return ((max_n + 63u) & ~63u) + 4u * ((((max_n + 31u) >> 5) + 63u) & ~63u);
}

__global__ void __launch_bounds__(256) relabel_kernel(const GraphDesc* graphs, const uint64_t* rows_in,
                                                      const uint32_t* order, uint32_t* adj, uint32_t max_n)
{
    extern __shared__ uint32_t lds[];
    const GraphDesc gd = graphs[blockIdx.y];
    const uint32_t n = gd.n;
    const uint32_t i0 = blockIdx.x * kRelabelRows;
    if (i0 >= n) return;
    const uint32_t t = threadIdx.x, lane = lane_id(), wave = bcast0(t >> 6);
    const uint32_t* ord = order + gd.ord_off;
    uint32_t* pos = lds;
    // eight loads in flight a thread before their stores
    for (uint32_t j0 = t; j0 < n; j0 += 256u * 8u) {
        uint32_t o[8];
#pragma unroll
        for (uint32_t k = 0; k < 8; k++) {
            const uint32_t j = j0 + 256u * k;
            o[k] = j < n ? ord[j] : 0u;
        }
#pragma unroll
        for (uint32_t k = 0; k < 8; k++) {
            const uint32_t j = j0 + 256u * k;
            if (j < n) pos[o[k]] = j;
        }
    }
    uint32_t* rowl = lds + ((max_n + 63u) & ~63u) + wave * ((((max_n + 31u) >> 5) + 63u) & ~63u);
    __syncthreads();
    const uint32_t W = gd.w32, nw64 = (n + 63u) >> 6;
    for (uint32_t k = wave; k < kRelabelRows; k += 4) {
        const uint32_t i = i0 + k;
        if (i >= n) break;
        for (uint32_t w = lane; w < W; w += 64) rowl[w] = 0u;
        // (a wavefront's LDS operations take effect in issue order: the
        // clearing above precedes every OR below)
        const uint64_t* src = rows_in + gd.in_off + (uint64_t)ord[i] * gd.rw64;
        for (uint32_t w = lane; w < nw64; w += 64) {
            uint64_t x = src[w];
            while (x) {
                const uint32_t p = pos[(w << 6) | (uint32_t)__builtin_ctzll(x)];
                x &= x - 1ull;
                atomicOr(&rowl[p >> 5], 1u << (p & 31u));
            }
        }
        uint32_t* dst = adj + gd.adj_off + (uint64_t)i * gd.rstride;
        for (uint32_t w = lane; w < W; w += 64) dst[w] = rowl[w];
        // the word after the row holds the vertex's input id, so that the
        // search gets it with the row
        if (lane == 0 && gd.rstride > W) dst[W] = ord[i];
    }
}

// Zero the per-graph results, the histograms, the control block and the
// mailboxes.
static_assert(sizeof(SearchParams) % 4 == 0 && sizeof(SearchParams) <= 4 * 256,
              "SearchParams copied as words by the first workgroup of 256 threads");
__global__ void reset_kernel(SearchParams sp, uint32_t num_graphs, uint64_t hist_total, uint32_t workgroups,
                             SearchParams* params_out)
{
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    // the search's copy of its parameters in HBM (read by the out-of-line
    // helpers), written from this launch's own argument: no host copy
    if (params_out && tid < sizeof(SearchParams) / 4)
        reinterpret_cast<uint32_t*>(params_out)[tid] = reinterpret_cast<const uint32_t*>(&sp)[tid];
    unsigned long long* res = reinterpret_cast<unsigned long long*>(sp.results);
    const uint64_t res_words = (uint64_t)num_graphs * (sizeof(DevResult) / 8);
    for (uint64_t i = tid; i < res_words; i += stride) res[i] = 0ull;
    for (uint64_t i = tid; i < hist_total; i += stride) sp.hist[i] = 0ull;
    uint32_t* mail = reinterpret_cast<uint32_t*>(sp.mail);
    const uint64_t mail_words = (uint64_t)workgroups * (sizeof(Mailbox) / 4);
    for (uint64_t i = tid; i < mail_words; i += stride) mail[i] = 0u;
    if (tid < sizeof(QueueCtl) / 8) reinterpret_cast<unsigned long long*>(sp.ctl)[tid] = 0ull;
}

// Root of each graph (R = {}, P = V, X = {}): its pivot is the first vertex
// of P (position 0), so L0 = {0} u (V \ N(0)).  The root children with branch
// index in [first, last) are dealt out as units of consecutive children: a
// unit covering the children of index [a, b) has P = V minus the children
// before a, X = the children before a, L = the children in [a, b).  The root
// node counts iff first == 0.

// L0 of graph g, its size, and per-lane ranks (one wavefront).
template <int WPL>
__device__ __forceinline__ uint32_t root_candidates(const SearchParams& sp, const GraphDesc& gd, uint32_t lane,
                                                    uint32_t (&V)[WPL], uint32_t (&L0)[WPL],
                                                    uint32_t (&cnt)[WPL], uint32_t (&incl)[WPL])
{
    const uint32_t n = gd.n, W = gd.w32;
    const uint32_t* row0 = sp.adj + gd.adj_off;
#pragma unroll
    for (int c = 0; c < WPL; c++) {
        const uint32_t w = (uint32_t)c * 64u + lane;
        uint32_t full = 0;
        if (w < W) full = (w == W - 1 && (n & 31)) ? ((1u << (n & 31)) - 1u) : 0xffffffffu;
        V[c] = full;
        L0[c] = full & ~((w < W) ? row0[w] : 0u);
    }
    return popc_scan<WPL>(L0, cnt, incl);
}

// One wavefront per graph: count the root's children, record the root node,
// and reserve pool slots for the graph's units (at most max_units).
template <int WPL>
__global__ void __launch_bounds__(64) root_plan_kernel(SearchParams sp, uint64_t first, uint64_t last,
                                                       uint32_t max_units)
{
    const uint32_t g = blockIdx.x;
    const GraphDesc gd = sp.graphs[g];
    const uint32_t lane = lane_id();
    uint32_t total = 0;
    if (gd.n != 0) {
        uint32_t V[WPL], L0[WPL], cnt[WPL], incl[WPL];
        total = root_candidates<WPL>(sp, gd, lane, V, L0, cnt, incl);
    }
    if (lane != 0) return;
    DevResult* r = sp.results + g;
    r->root_branches = total;
    if (gd.n != 0 && first == 0 && last > 0) atomicAdd(&r->nodes, 1ull);
    const uint32_t lo = first < (uint64_t)total ? (uint32_t)first : total;
    const uint32_t hi = last < (uint64_t)total ? (uint32_t)last : total;
    uint32_t units = hi > lo ? hi - lo : 0u;
    if (units > max_units) units = max_units;
    uint32_t base = 0;
    if (units != 0) {
        base = atomicAdd(&sp.ctl->pool_size, units);
        atomicAdd(&sp.ctl->work, units);
    }
    r->unit_base = base;
    r->unit_count = units;
}

// Grid (graphs, k): wavefront y of graph g writes units y, y + k, ... of the
// graph into the pool slots reserved by root_plan_kernel.  The search kernel
// runs after this one, so plain stores suffice.
template <int WPL>
__global__ void __launch_bounds__(64) root_units_kernel(SearchParams sp, uint64_t first, uint64_t last)
{
    const uint32_t g = blockIdx.x;
    const uint32_t units = sp.results[g].unit_count;
    if (blockIdx.y >= units) return;
    const uint32_t base = sp.results[g].unit_base;
    const GraphDesc gd = sp.graphs[g];
    const uint32_t lane = lane_id();
    const uint32_t W = gd.w32, cs = sp.w32cap;
    uint32_t V[WPL], L0[WPL], cnt[WPL], incl[WPL];
    const uint32_t total = root_candidates<WPL>(sp, gd, lane, V, L0, cnt, incl);
    const uint32_t lo = first < (uint64_t)total ? (uint32_t)first : total;
    const uint32_t hi = last < (uint64_t)total ? (uint32_t)last : total;
    const uint64_t m = hi - lo;
    for (uint32_t j = blockIdx.y; j < units; j += gridDim.y) {
        const uint32_t a = lo + (uint32_t)(m * j / units);
        const uint32_t b = lo + (uint32_t)(m * (j + 1) / units);
        const uint32_t pos = base + j;
        uint32_t* rec = sp.rec + (size_t)pos * sp.rec_words;
        if (lane == 0) rec[0] = g;
#pragma unroll
        for (int c = 0; c < WPL; c++) {
            const uint32_t before = incl[c] - cnt[c];
            const uint32_t la = low_bits(L0[c], rank_take(a, before, cnt[c]));
            const uint32_t lb = low_bits(L0[c], rank_take(b, before, cnt[c]));
            const uint32_t w = (uint32_t)c * 64u + lane;
            if (w < W) {
                rec[kRecHeader + w] = 0u;               // R
                rec[kRecHeader + cs + w] = V[c] & ~la;  // P
                rec[kRecHeader + 2 * cs + w] = la;      // X
                rec[kRecHeader + 3 * cs + w] = lb & ~la; // L
            }
        }
    }
}

// The pivot of a node (P, X) of graph gd by the launch's pivot rule (Alg. 4
// step 9; Sec. 4.3): GreedyBB, the first vertex of X if X is non-empty, else
// the first of P; GreedyBBTX, the vertex of X maximising |P n N(u)| if X is
// non-empty, else the first of P; TomitaBB, the vertex of P u X maximising
// |P n N(u)|; ties to the earlier position.  -1 if P and X are empty.  One
// wavefront.
template <int WPL>
__device__ int node_pivot(const SearchParams& sp, const GraphDesc& gd, const uint32_t (&P)[WPL],
                          const uint32_t (&X)[WPL], uint32_t lane)
{
    const uint32_t W = gd.w32;
    const uint32_t* adj = sp.adj + gd.adj_off;
    int p = first_bit<WPL>(X);
    if (sp.pivot_rule == kPivotTomita || (sp.pivot_rule == kPivotTX && p >= 0)) {
        // the candidate maximising |P n N(u)|, the earliest on ties
        uint32_t C[WPL];
#pragma unroll
        for (int c = 0; c < WPL; c++) C[c] = (sp.pivot_rule == kPivotTomita) ? (P[c] | X[c]) : X[c];
        uint32_t bestc = 0;
        p = -1;
        for (int u = first_bit<WPL>(C); u >= 0; u = first_bit<WPL>(C)) {
            clear_bit<WPL>(C, (uint32_t)u, lane);
            const uint32_t* ru = adj + (size_t)(uint32_t)u * gd.rstride;
            uint32_t cnt = 0;
#pragma unroll
            for (int c = 0; c < WPL; c++) {
                const uint32_t w = (uint32_t)c * 64u + lane;
                cnt += (w < W) ? (uint32_t)__builtin_popcount(P[c] & ru[w]) : 0u;
            }
            cnt = wave_sum(cnt);
            if (p < 0 || cnt > bestc) {
                p = u;
                bestc = cnt;
            }
        }
    }
    if (p < 0) p = first_bit<WPL>(P);
    return p;
}

// One node (R, P, X) of graph 0, given as position bitsets (w32 words each,
// R then P then X), as the only unit of the pool: R is mapped to input ids,
// the node's pivot (by the launch's pivot rule) and L = P \ N(p) are taken
// as in Alg. 4, and the node itself is counted.  One wavefront.  P must not be
// empty (the host checks).
template <int WPL>
__global__ void __launch_bounds__(64) subproblem_kernel(SearchParams sp, const uint32_t* bits)
{
    const GraphDesc gd = sp.graphs[0];
    const uint32_t W = gd.w32, lane = lane_id(), cs = sp.w32cap;
    const uint32_t* ord = sp.order + gd.ord_off;
    const uint32_t* adj = sp.adj + gd.adj_off;
    uint32_t Rp[WPL], P[WPL], X[WPL], Rb[WPL], L[WPL], cnt[WPL], incl[WPL];
#pragma unroll
    for (int c = 0; c < WPL; c++) {
        const uint32_t w = (uint32_t)c * 64u + lane;
        const bool in = w < W;
        Rp[c] = in ? bits[w] : 0u;
        P[c] = in ? bits[W + w] : 0u;
        X[c] = in ? bits[2 * W + w] : 0u;
        Rb[c] = 0u;
    }
    for (int q = first_bit<WPL>(Rp); q >= 0; q = first_bit<WPL>(Rp)) {
        clear_bit<WPL>(Rp, (uint32_t)q, lane);
        set_bit<WPL>(Rb, bcast0(ord[q]), lane);
    }
    const int p = node_pivot<WPL>(sp, gd, P, X, lane);
    if (p < 0) return;
    const uint32_t* rp = adj + (size_t)(uint32_t)p * gd.rstride;
#pragma unroll
    for (int c = 0; c < WPL; c++) {
        const uint32_t w = (uint32_t)c * 64u + lane;
        L[c] = (w < W) ? (P[c] & ~rp[w]) : 0u;
    }
    const uint32_t total = popc_scan<WPL>(L, cnt, incl);
    uint32_t* rec = sp.rec;
    if (lane == 0) {
        rec[0] = 0u;
        sp.results[0].root_branches = total;
        sp.results[0].nodes += 1ull;
        sp.ctl->pool_size = 1u;
        sp.ctl->work = 1u;
    }
#pragma unroll
    for (int c = 0; c < WPL; c++) {
        const uint32_t w = (uint32_t)c * 64u + lane;
        if (w < W) {
            rec[kRecHeader + w] = Rb[c];
            rec[kRecHeader + cs + w] = P[c];
            rec[kRecHeader + 2 * cs + w] = X[c];
            rec[kRecHeader + 3 * cs + w] = L[c];
        }
    }
}

// ------------------------------------------------------- local graphs ----
//
// A sparse graph of more than 4096 vertices is solved root child by root
// child, each on the subgraph induced by S = N(l) u {l} (Alg. 4 at the
// root: the pivot is position 0, the children are L0 = {0} u (V \ N(0)) in
// increasing position, and below child l every set the search forms lies in
// N(l)).  S is numbered by increasing position, so the first vertex of a set
// is the same vertex as in the whole graph and the search tree is the same
// (same pivots, same branch orders, same node count); its members' ids are
// ranked by increasing input id, so that a clique's local-id bitset lists it
// in increasing input id, and a map turns the ranks back into input ids.
// The local bitsets have ceil(|S| / 32) words instead of ceil(n / 32).

// Per position v of the whole graph (renumbered rows, w32 words, stride
// rstride): its degree, with bit 31 set if v is a root child (v = 0 or v not
// adjacent to 0).  One wavefront per position.
__global__ void __launch_bounds__(256) local_plan_kernel(const GraphDesc* gparent, const uint32_t* adj, uint32_t* out)
{
    const GraphDesc G = *gparent;
    const uint32_t v = blockIdx.x * 4u + (threadIdx.x >> 6);
    if (v >= G.n) return;
    const uint32_t lane = lane_id();
    const uint32_t* row = adj + G.adj_off + (size_t)v * G.rstride;
    uint32_t c = 0;
    for (uint32_t w = lane; w < G.w32; w += 64) c += (uint32_t)__builtin_popcount(row[w]);
    c = wave_sum(c);
    if (lane == 0) {
        const uint32_t* row0 = adj + G.adj_off;
        const bool root_child = v == 0u || ((row0[v >> 5] >> (v & 31u)) & 1u) == 0u;
        out[v] = c | (root_child ? 0x80000000u : 0u);
    }
}

// Exclusive prefix popcounts of words[0, W) into pref (one wavefront, eight
// words a lane, W <= 512).
__device__ __forceinline__ void word_prefix(const uint32_t* words, uint32_t* pref, uint32_t W, uint32_t lane)
{
    const uint32_t w0 = lane * 8u;
    uint32_t loc[8], sum = 0;
#pragma unroll
    for (int i = 0; i < 8; i++) {
        loc[i] = (w0 + (uint32_t)i < W) ? (uint32_t)__builtin_popcount(words[w0 + i]) : 0u;
        sum += loc[i];
    }
    uint32_t run = wave_scan_incl(sum) - sum;
#pragma unroll
    for (int i = 0; i < 8; i++) {
        if (w0 + (uint32_t)i < W) pref[w0 + i] = run;
        run += loc[i];
    }
}

// Rank of bit b (< 32) of word w among the set bits of a bitset, given the
// exclusive prefix popcounts of its words.
__device__ __forceinline__ uint32_t bit_rank(const uint32_t* words, const uint32_t* pref, uint32_t w, uint32_t b)
{
    return pref[w] + (uint32_t)__builtin_popcount(words[w] & ((1u << b) - 1u));
}

// One workgroup of 256 per local graph (lgraphs[blockIdx.x]): its member
// list, local order (local position -> local id), id map, rows (with the
// local id after each row) and the P and X bitsets of the root child's node
// (P = N(l) minus the earlier root children, X = N(l) and the earlier root
// children), followed by the root child's own local id.
__global__ void __launch_bounds__(256) local_build_kernel(const GraphDesc* gparent, const uint32_t* adj,
                                                          const uint32_t* order, const GraphDesc* lgraphs,
                                                          uint32_t* ladj, uint32_t* lord, uint32_t* lidmap,
                                                          uint32_t* lpx)
{
    __shared__ uint32_t Sw[512], prefS[512], idw[512], prefI[512];
    __shared__ uint32_t stage[4][64], pxw[2][64];
    __shared__ uint16_t mem[kLocalMaxN];
    const GraphDesc G = *gparent;
    const GraphDesc L = lgraphs[blockIdx.x];
    const uint32_t t = threadIdx.x, lane = lane_id(), wave = t >> 6;
    const uint32_t W = G.w32, p = L.rw64;
    const uint32_t* grow = adj + G.adj_off;
    const uint32_t* gord = order + G.ord_off;
    // S = N(p) u {p}
    for (uint32_t w = t; w < W; w += 256) {
        Sw[w] = grow[(size_t)p * G.rstride + w] | (w == (p >> 5) ? (1u << (p & 31u)) : 0u);
        idw[w] = 0u;
    }
    if (t < 128) pxw[t >> 6][t & 63u] = 0u;
    __syncthreads();
    if (wave == 0) word_prefix(Sw, prefS, W, lane);
    // the members' input ids as a bitset over ids (ids are below n)
    for (uint32_t w = t; w < W; w += 256) {
        uint32_t bits = Sw[w];
        while (bits) {
            const uint32_t q = (w << 5) | (uint32_t)__builtin_ctz(bits);
            bits &= bits - 1u;
            const uint32_t id = gord[q];
            atomicOr(&idw[id >> 5], 1u << (id & 31u));
        }
    }
    __syncthreads();
    if (wave == 0) word_prefix(idw, prefI, W, lane);
    __syncthreads();
    // local position a of member q, its local id, the map, the member list,
    // and the node's P and X (q != p; X: a root child earlier than p)
    const uint32_t* row0 = grow;
    for (uint32_t w = t; w < W; w += 256) {
        uint32_t bits = Sw[w];
        while (bits) {
            const uint32_t b = (uint32_t)__builtin_ctz(bits);
            bits &= bits - 1u;
            const uint32_t q = (w << 5) | b;
            const uint32_t a = bit_rank(Sw, prefS, w, b);
            const uint32_t id = gord[q];
            const uint32_t lid = bit_rank(idw, prefI, id >> 5, id & 31u);
            lord[L.ord_off + a] = lid;
            lidmap[L.idmap_off + lid] = id;
            mem[a] = (uint16_t)q;
            if (q == p) {
                lpx[L.in_off + 2u * L.w32] = lid;
            } else {
                const bool root_child = q == 0u || ((row0[q >> 5] >> (q & 31u)) & 1u) == 0u;
                atomicOr(&pxw[(root_child && q < p) ? 1 : 0][a >> 5], 1u << (a & 31u));
            }
        }
    }
    __syncthreads();
    if (t < L.w32) {
        lpx[L.in_off + t] = pxw[0][t];
        lpx[L.in_off + L.w32 + t] = pxw[1][t];
    }
    // rows: member a's row restricted to S, in local positions, then its id
    for (uint32_t a = wave; a < L.n; a += 4) {
        const uint32_t q = mem[a];
        stage[wave][lane] = 0u;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // the lane's words of the row (at most 512 words, eight a lane) are
        // requested together (words past the row's end read its first word
        // and are dropped), then their bits ranked.  (Requesting the next
        // member's words before ranking these gained nothing more.)
        static_assert(kMaxN / 32u <= 8u * 64u, "a whole-graph row in eight words a lane");
        const uint32_t* rq = grow + (size_t)q * G.rstride;
        uint32_t xs[8];
#pragma unroll
        for (uint32_t k = 0; k < 8; k++) {
            const uint32_t w = lane + 64u * k, wc = w < W ? w : 0u;
            xs[k] = rq[wc];
        }
#pragma unroll
        for (uint32_t k = 0; k < 8; k++) {
            const uint32_t w = lane + 64u * k;
            xs[k] = w < W ? xs[k] & Sw[w] : 0u;
        }
#pragma unroll
        for (uint32_t k = 0; k < 8; k++) {
            const uint32_t w = lane + 64u * k;
            uint32_t x = xs[k];
            while (x) {
                const uint32_t b = (uint32_t)__builtin_ctz(x);
                x &= x - 1u;
                const uint32_t la = bit_rank(Sw, prefS, w, b);
                atomicOr(&stage[wave][la >> 5], 1u << (la & 31u));
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        uint32_t* dst = ladj + L.adj_off + (size_t)a * L.rstride;
        if (lane < L.w32) dst[lane] = stage[wave][lane];
        if (lane == 0) {
            const uint32_t id = gord[q];
            dst[L.w32] = bit_rank(idw, prefI, id >> 5, id & 31u);
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// The root children of branch index [first, last) (local graph i is child i):
// a child whose P is empty is a leaf, counted here (a maximal clique {l} if
// X is also empty, else a dead end); any other becomes a node, counted, with
// its pivot and L = P \ N(p), as a unit of the pool.  The root node counts
// iff first == 0.  A workgroup of kLocalUnitsWaves wavefronts takes as many
// consecutive local graphs, one a wavefront; its counts, hash totals and
// pool slots are gathered in LDS and added to the global counters once (one
// atomic a counter per workgroup instead of one per child: ten thousand
// children on the same words would queue at L2).
constexpr uint32_t kLocalUnitsWaves = 16;

template <int WPL>
__global__ void __launch_bounds__(64 * kLocalUnitsWaves) local_units_kernel(SearchParams sp, const uint32_t* lpx,
                                                                           uint32_t count, uint64_t first,
                                                                           uint64_t last)
{
    __shared__ unsigned long long s_hx, s_hs;
    __shared__ uint32_t s_children, s_nodes, s_count, s_omega, s_units, s_base;
    const uint32_t lane = lane_id(), wave = bcast0(threadIdx.x >> 6);
    const uint32_t i = blockIdx.x * kLocalUnitsWaves + wave;
    DevResult* r = sp.results; // every local graph reports to result 0
    if (threadIdx.x == 0) {
        s_hx = s_hs = 0ull;
        s_children = s_count = s_omega = s_units = 0u;
        s_nodes = (blockIdx.x == 0 && first == 0 && last > 0) ? 1u : 0u; // the root node
    }
    __syncthreads();
    const bool mine = i >= first && i < last && i < count;
    GraphDesc gd;
    uint32_t P[WPL], X[WPL], L[WPL];
    uint32_t rootlid = 0, slot = 0xffffffffu;
    if (mine) {
        gd = sp.graphs[i];
        const uint32_t W = gd.w32;
        const uint32_t* px = lpx + gd.in_off;
#pragma unroll
        for (int c = 0; c < WPL; c++) {
            const uint32_t w = (uint32_t)c * 64u + lane;
            P[c] = w < W ? px[w] : 0u;
            X[c] = w < W ? px[W + w] : 0u;
        }
        rootlid = px[2u * W];
        if (lane == 0) atomicAdd(&s_children, 1u);
        if (!any_set<WPL>(P)) {
            if (!any_set<WPL>(X) && lane == 0) {
                // the clique {l}
                const uint32_t id = sp.idmap[gd.idmap_off + rootlid];
                const uint64_t h = mix64(mix64(1ull) + kGolden + (uint64_t)id);
                atomicAdd(&s_count, 1u);
                atomicXor(&s_hx, (unsigned long long)h);
                atomicAdd(&s_hs, (unsigned long long)h);
                atomicMax(&s_omega, 1u);
            }
        } else {
            const int p = node_pivot<WPL>(sp, gd, P, X, lane);
            const uint32_t* rp = sp.adj + gd.adj_off + (size_t)(uint32_t)p * gd.rstride;
#pragma unroll
            for (int c = 0; c < WPL; c++) {
                const uint32_t w = (uint32_t)c * 64u + lane;
                L[c] = (w < W) ? (P[c] & ~rp[w]) : 0u;
            }
            uint32_t sl = 0;
            if (lane == 0) {
                atomicAdd(&s_nodes, 1u);
                sl = atomicAdd(&s_units, 1u);
            }
            slot = bcast0(sl);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (s_units) {
            s_base = atomicAdd(&sp.ctl->pool_size, s_units);
            atomicAdd(&sp.ctl->work, s_units);
        }
        if (s_children) atomicAdd(&r->children, (unsigned long long)s_children);
        if (s_nodes) atomicAdd(&r->nodes, (unsigned long long)s_nodes);
        if (s_count) {
            atomicAdd(&r->count, (unsigned long long)s_count);
            atomicXor(&r->hash_xor, s_hx);
            atomicAdd(&r->hash_sum, s_hs);
            atomicMax(&r->omega, s_omega);
            atomicAdd(&sp.hist[sp.graphs[0].hist_off + 1], (unsigned long long)s_count);
        }
    }
    __syncthreads();
    if (slot != 0xffffffffu) {
        const uint32_t W = gd.w32, cs = sp.w32cap;
        uint32_t* rec = sp.rec + (size_t)(s_base + slot) * sp.rec_words;
        if (lane == 0) rec[0] = i;
#pragma unroll
        for (int c = 0; c < WPL; c++) {
            const uint32_t w = (uint32_t)c * 64u + lane;
            if (w < W) {
                rec[kRecHeader + w] = (w == (rootlid >> 5)) ? (1u << (rootlid & 31u)) : 0u; // R = {l}
                rec[kRecHeader + cs + w] = P[c];
                rec[kRecHeader + 2 * cs + w] = X[c];
                rec[kRecHeader + 3 * cs + w] = L[c];
            }
        }
    }
}

// ------------------------------------------------------ the search -------
//
// Scheduling is two-level, so that no HBM word is polled by every workgroup:
//   * inside a workgroup, wavefronts share a small LIFO of units in LDS.  A
//     busy wavefront looks at a few LDS counters every check_interval
//     children and, while siblings wait and the LIFO is short (or the LIFO is
//     empty), hands over the later half of the candidates of its shallowest
//     big-enough frame;
//   * between workgroups, a workgroup whose wavefronts are out of work first
//     takes root units from the pool (one atomic counter), then asks other
//     workgroups, one at a time and chosen at random, through their
//     mailboxes.  A busy workgroup looks at its own mailbox every
//     refresh_children children of the workgroup and answers with a unit split
//     off in the same way, or with a refusal.
// Termination: ctl->work counts the root units not handed out, the units in
// transit to a mailbox and the workgroups that hold work (running or in their
// LIFO); the search is over when it reaches zero.

struct WgHdr {
    uint32_t lock;      // LDS spin lock over the LIFO and the counters below
    uint32_t busy;      // wavefronts holding a unit
    uint32_t lq_n;      // units in the LIFO
    uint32_t active;    // this workgroup is counted in ctl->work
    uint32_t fetcher;   // a wavefront is looking for work outside the workgroup
    uint32_t done;      // stop: search over or aborted
    uint32_t req;       // asking workgroup + 1, taken from the mailbox and not answered yet
    uint32_t ticks;     // children processed by the workgroup, in steps of check_interval
    uint32_t out;       // workgroup + 1 that this workgroup has asked (0: none,
                        // kOutReading: the answer is a unit being read)
    uint32_t pool_left; // root units may be left in the pool
    uint32_t pool_size; // root units in the pool
    uint32_t rng;       // xorshift state for choosing whom to ask
    uint32_t hint;      // busy count last written to this workgroup's mailbox hint
    uint32_t pad[3];
};
static_assert(sizeof(WgHdr) == kWgHdrWords * 4, "header size");
constexpr uint32_t kOutReading = 0xffffffffu;
// Workgroups whose busy hints an idle workgroup compares before asking one.
constexpr uint32_t kAskSamples = 8;

__device__ __forceinline__ uint32_t lds_ld(uint32_t* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ void lds_st(uint32_t* p, uint32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Take the workgroup lock.  Returns false only if the search deadline passed
// while waiting; the caller then abandons the search.
__device__ __forceinline__ bool wg_lock(WgHdr* h, uint32_t lane, uint64_t t_start, uint64_t limit)
{
    uint32_t ok = 1;
    if (lane == 0) {
        uint32_t spins = 0;
        while (__hip_atomic_exchange(&h->lock, 1u, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) != 0u) {
            __builtin_amdgcn_s_sleep(1);
            if (limit != 0 && (++spins & 1023u) == 0 && (uint64_t)wall_clock64() - t_start > limit) {
                ok = 0;
                break;
            }
        }
    }
    ok = bcast0(ok);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    return ok != 0;
}

__device__ __forceinline__ void wg_unlock(WgHdr* h, uint32_t lane)
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    if (lane == 0) __hip_atomic_store(&h->lock, 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Per-wavefront LDS layout (32-bit words):
//   [kOffHist, +128)   histogram of clique sizes < kHistLds (u64)
//   [kOffBuf, +kCliqueSlots)  clique buffer (path-id lists or 16-bit halves
//                      of input-id bitsets)
//   [kOffTrash, +64)   one word per lane for stores that must go nowhere (and
//                      the unit's R as ids while the buffer is emptied)
//   [kOffCtx, +32)     WaveCtx: totals and bookkeeping used off the hot path
//   [kOffSave, +128)   the search loop's lane registers while it is suspended:
//                      idstk (64 words), then cent (64 words)
//   [kWaveFixedWords, ...)  lds_depth stack frames, then the slot of the
//                      current frame (written before a check), then slack
// A frame holds P, X, L and the row of the frame's next candidate,
// interleaved per lane: lane w's words of chunk c sit at 4 (64 c + w) .. +3.
constexpr uint32_t kOffHist = 0, kOffBuf = kHistLds * 2, kOffTrash = kOffBuf + kCliqueSlots,
                   kOffCtx = kOffTrash + 64, kOffSave = kOffCtx + 32;
static_assert(kOffSave + 128 == kWaveFixedWords, "layout");

// Clique buffer entries: cent (one word a clique) = start << 16 | flags and
// length.  A list entry (one word a lane layouts, a clique of at most
// kCliqueListMax vertices whose path is in the LDS window) holds the input ids
// pushed on the way down from the unit's node and the last vertex's, one a
// word, in path order; the unit's own R is the fourth word of the current
// frame slot.  Any other entry holds the non-empty 16-bit halves of the
// clique's input-id bitset, in lane order.
constexpr uint32_t kEntryList = 0x8000u, kEntryLen = 0x7fffu;
constexpr uint32_t kCliqueListMax = 16;

struct WaveCtx {
    unsigned long long count, nodes, children; // totals of graph g not yet folded into HBM
    unsigned long long units, donations, spills;
    uint32_t omega, g, spill_chunk, refreshes;
    unsigned long long hx, hs;                 // XOR and sum of the clique hashes of graph g
    // the search loop's scalars while it is suspended (search_unit)
    uint32_t d, budget, nent, used, rcount, refresh;
    uint32_t checks, flushes; // suspensions of the search loop, by reason
    unsigned long long busy;  // wall-clock ticks spent on units
    uint32_t pad[2];
};
// Wall-clock ticks of a wavefront's first unit start and last unit end.
struct WaveTimes {
    unsigned long long first, last;
};
static_assert(sizeof(WaveCtx) == 32 * 4, "ctx size");

__device__ __forceinline__ WaveCtx* wave_ctx(uint32_t* wl) { return reinterpret_cast<WaveCtx*>(wl + kOffCtx); }

// A lane bitset passed by value to the out-of-line helpers (an array reference
// would force it into scratch memory).
template <int WPL> struct LaneBits {
    uint32_t w[WPL];
};

// Hash, histogram and (enumerate) write-out of the nent buffered cliques, one
// clique per lane: lane i's clique is the list of halves at buffer words
// [start, start + cnt), with cent (lane i's saved word) = start << 16 | cnt.
// Empties the buffer.  Off the hot path.
__device__ __attribute__((noinline)) void cold_flush(const SearchParams* __restrict__ spp, uint32_t* wl,
                                                     uint32_t g_v)
{
    const SearchParams& sp = *spp;
    const GraphDesc& gd = sp.graphs[bcast0(g_v)];
    const uint64_t hoff = gd.hist_off;
    // a local graph reports its ids through its map (increasing: the order of
    // a clique's ids is kept)
    const uint32_t* idm = gd.idmap_off != kNoMap ? sp.idmap + gd.idmap_off : nullptr;
    const uint32_t lane = lane_id();
    const uint32_t nent = bcast0(wave_ctx(wl)->nent);
    const uint32_t cent = wl[kOffSave + 64 + lane];
    unsigned long long* ghist = sp.hist + hoff;
    unsigned long long* hist_l = reinterpret_cast<unsigned long long*>(wl + kOffHist);
    const uint32_t* buf = wl + kOffBuf;
    WaveCtx* ctx = wave_ctx(wl);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    const bool mine = lane < nent;
    const bool lst = mine && (cent & kEntryList) != 0u;
    const uint32_t st = mine ? (cent >> 16) : 0u, cnt = mine ? (cent & kEntryLen) : 0u;
    // List entries: the unit's R (the fourth word of the current frame slot,
    // one word a lane, written when the search loop returned) in increasing
    // order into the sink words; then each list lane sorts its path's ids
    // with those (at most kCliqueListMax in all) by a bitonic network.
    uint32_t r = 0;
    uint32_t* sink = wl + kOffTrash;
    if (ballot(lst) != 0ull) {
        const uint32_t* cur = wl + kWaveFixedWords + (size_t)sp.lds_depth * sp.slot_words;
        const uint32_t bw = lane < gd.w32 ? cur[4u * lane + 3u] : 0u;
        uint64_t nz = ballot(bw != 0u);
        uint32_t bl = 0;
        while (nz) {
            const uint32_t l = (uint32_t)__builtin_ctzll(nz);
            nz &= nz - 1ull;
            uint32_t word = rdlane(bw, l);
            while (word) {
                bl = wrlane(bl, (l << 5) | (uint32_t)__builtin_ctz(word), r);
                word &= word - 1u;
                r++;
            }
        }
        sink[lane] = bl;
    }
    uint32_t srt[kCliqueListMax];
    if (lst) {
#pragma unroll
        for (uint32_t j = 0; j < kCliqueListMax; j++) {
            const uint32_t x = j < cnt ? buf[st + j] : sink[umin32(j - cnt, 63u)];
            srt[j] = j < cnt + r ? x : 0xffffffffu;
        }
#pragma unroll
        for (uint32_t kk = 2; kk <= kCliqueListMax; kk <<= 1) {
#pragma unroll
            for (uint32_t jj = kk >> 1; jj > 0; jj >>= 1) {
#pragma unroll
                for (uint32_t i = 0; i < kCliqueListMax; i++) {
                    const uint32_t l = i ^ jj;
                    if (l > i) {
                        const uint32_t x = srt[i], y = srt[l];
                        const bool up = (i & kk) == 0u;
                        srt[i] = up ? umin32(x, y) : umax32(x, y);
                        srt[l] = up ? umax32(x, y) : umin32(x, y);
                    }
                }
            }
        }
    }
    // clique size, then the hash chain over the ids in increasing order
    uint32_t k = 0;
    if (lst) {
        k = cnt + r;
    } else {
        for (uint32_t i = 0; i < cnt; i++) k += (uint32_t)__builtin_popcount(buf[st + i] & 0xffffu);
    }
    uint64_t h = 0;
    if (mine) {
        h = mix64((uint64_t)k);
        if (lst) {
#pragma unroll
            for (uint32_t j = 0; j < kCliqueListMax; j++)
                if (j < k) h = mix64(h + kGolden + (uint64_t)(idm ? idm[srt[j]] : srt[j]));
        } else {
            for (uint32_t i = 0; i < cnt; i++) {
                const uint32_t e = buf[st + i];
                const uint32_t base = (e >> 16) << 4;
                uint32_t bits = e & 0xffffu;
                while (bits) {
                    const uint32_t id = base + (uint32_t)__builtin_ctz(bits);
                    h = mix64(h + kGolden + (uint64_t)(idm ? idm[id] : id));
                    bits &= bits - 1u;
                }
            }
        }
    }
    // XOR and sum over the lanes (lanes without a clique hold 0)
    uint64_t hx = h, hs = h;
    for (int off = 32; off > 0; off >>= 1) {
        hx ^= __shfl_xor(hx, off);
        hs += __shfl_xor(hs, off);
    }
    uint64_t rem = ballot(mine);
    uint32_t kmax = 0;
    while (rem) {
        const uint32_t l0 = (uint32_t)__builtin_ctzll(rem);
        const uint32_t k0 = rdlane(k, l0);
        const uint64_t m = ballot(mine && k == k0);
        const uint32_t c = (uint32_t)__builtin_popcountll(m);
        // counted in LDS (all waves share few sizes: HBM atomics would queue
        // on the same words); sizes past the LDS histogram go to HBM
        if (lane == 0) {
            if (k0 < kHistLds) hist_l[k0] += c;
            else atomicAdd(&ghist[k0], (unsigned long long)c);
        }
        kmax = umax32(kmax, k0);
        rem &= ~m;
    }
    if (lane == 0) {
        ctx->count += nent;
        ctx->omega = umax32(ctx->omega, kmax);
        ctx->hx ^= hx;
        ctx->hs += hs;
        ctx->nent = 0;
        ctx->used = 0;
    }
    if (sp.enumerate) {
        // ids of clique i at verts[vb + (sizes of cliques before i)], and its
        // [begin, end) pair at offs[ob + 2 i]
        const uint32_t kincl = wave_scan_incl(mine ? k : 0u);
        const uint32_t used = rdlane(kincl, 63);
        unsigned long long vb = 0, ob = 0;
        if (lane == 0) {
            vb = atomicAdd(&sp.ctl->vcursor, (unsigned long long)used);
            ob = atomicAdd(&sp.ctl->ocursor, 2ull * nent);
        }
        vb = ((unsigned long long)bcast0((uint32_t)(vb >> 32)) << 32) | bcast0((uint32_t)vb);
        ob = ((unsigned long long)bcast0((uint32_t)(ob >> 32)) << 32) | bcast0((uint32_t)ob);
        if (vb + used <= sp.verts_cap && ob + 2ull * nent <= sp.offs_cap && mine) {
            unsigned long long q = vb + kincl - k;
            sp.offs[ob + 2ull * lane] = q;
            sp.offs[ob + 2ull * lane + 1ull] = q + k;
            if (lst) {
#pragma unroll
                for (uint32_t j = 0; j < kCliqueListMax; j++)
                    if (j < k) sp.verts[q + j] = idm ? idm[srt[j]] : srt[j];
            } else {
                for (uint32_t i = 0; i < cnt; i++) {
                    const uint32_t e = buf[st + i];
                    const uint32_t base = (e >> 16) << 4;
                    uint32_t bits = e & 0xffffu;
                    while (bits) {
                        const uint32_t id = base + (uint32_t)__builtin_ctz(bits);
                        sp.verts[q++] = idm ? idm[id] : id;
                        bits &= bits - 1u;
                    }
                }
            }
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
}

// Fold the wavefront's totals of graph ctx->g (counts, hash totals, omega,
// histogram) into HBM and clear them.  Every value is read before the first
// atomic is issued, so that the atomics leave back to back and the wavefront
// waits for them once: a read issued after an atomic would wait for it, and
// when a search ends every wavefront folds into the same result slot at once,
// where each such wait is a pass through the queue on that slot's cache line.
__device__ __attribute__((noinline)) void cold_fold(const SearchParams* __restrict__ spp, uint32_t* wl)
{
    static_assert(kHistLds == 64, "one histogram entry per lane");
    const SearchParams& sp = *spp;
    const uint32_t lane = lane_id();
    WaveCtx* ctx = wave_ctx(wl);
    const uint32_t g = bcast0(ctx->g);
    if (g == 0xffffffffu) return;
    unsigned long long* hist_l = reinterpret_cast<unsigned long long*>(wl + kOffHist);
    const unsigned long long hv = hist_l[lane];
    const unsigned long long count = ctx->count, nodes = ctx->nodes, children = ctx->children;
    const unsigned long long x = ctx->hx, s = ctx->hs;
    const uint32_t omega = ctx->omega;
    unsigned long long* hp = sp.hist + sp.graphs[g].hist_off + lane;
    DevResult* r = sp.results + sp.graphs[g].res;
    asm volatile("" : : "v"(hp), "v"(r)); // both addresses are formed before the first atomic
    if (lane == 0) {
        if (count) atomicAdd(&r->count, count);
        if (nodes) atomicAdd(&r->nodes, nodes);
        if (children) atomicAdd(&r->children, children);
        if (x) atomicXor(&r->hash_xor, x);
        if (s) atomicAdd(&r->hash_sum, s);
        if (omega) atomicMax(&r->omega, omega);
    }
    if (hv) atomicAdd(hp, hv);
    if (lane == 0) {
        ctx->count = ctx->nodes = ctx->children = 0;
        ctx->hx = ctx->hs = 0;
        ctx->omega = 0;
    }
    hist_l[lane] = 0ull;
}

// The wavefront's exit record (WaveExit): its unfolded totals of graph ctx->g
// and its counters, written with plain stores; exit_fold_kernel adds the
// records up after the launch.  `first` and `last` are lane 0's wall-clock
// ticks of its first unit start and last unit end (0: no unit).
__device__ __attribute__((noinline)) void cold_exit(const SearchParams* __restrict__ spp, uint32_t* wl,
                                                    uint32_t gwave, uint64_t t_start, uint64_t first, uint64_t last)
{
    const SearchParams& sp = *spp;
    const uint32_t lane = lane_id();
    const WaveCtx* ctx = wave_ctx(wl);
    WaveExit* e = sp.exits + gwave;
    const uint32_t g = bcast0(ctx->g);
    e->hist[lane] = reinterpret_cast<const unsigned long long*>(wl + kOffHist)[lane];
    if (lane == 0) {
        const bool none = g == 0xffffffffu;
        e->res = none ? kNoSlot : sp.graphs[g].res;
        e->omega = ctx->omega;
        e->hist_off = none ? 0ull : sp.graphs[g].hist_off;
        e->count = ctx->count;
        e->nodes = ctx->nodes;
        e->children = ctx->children;
        e->hash_xor = ctx->hx;
        e->hash_sum = ctx->hs;
        e->units = ctx->units;
        e->donations = ctx->donations;
        e->spills = ctx->spills;
        e->checks = ctx->checks;
        e->flushes = ctx->flushes;
        e->busy = ctx->busy;
        const uint64_t t_exit = wall_clock64();
        e->run = t_exit - t_start;
        e->ramp = (first ? first : t_exit) - t_start;
        e->tail = first ? t_exit - last : 0ull;
    }
}

// The look at siblings and at the mailbox, when the periodic check of the
// search loop finds something to do.  The loop is suspended: the current
// frame (P, X, L, R) is in its LDS slot, frames 0..d-1 are on the stack, d and
// the ids of the pushed children are in the save area.  May hand the later
// half of the candidates of the shallowest big-enough frame to the LDS LIFO
// or to the workgroup that asked (the current frame's L in its slot is updated
// then).  Returns 1 if the search must stop.
template <int WPL>
__device__ __attribute__((noinline)) uint32_t cold_check(const SearchParams* __restrict__ spp, uint32_t* smem,
                                                         uint32_t* wl, uint32_t W_v, uint32_t g_v, uint64_t t_start)
{
    const SearchParams& sp = *spp;
    const uint32_t lane = lane_id();
    const uint32_t W = bcast0(W_v), g = bcast0(g_v);
    const uint32_t NW = blockDim.x >> 6;
    WgHdr* hdr = reinterpret_cast<WgHdr*>(smem);
    uint32_t* lq = smem + kWgHdrWords;
    WaveCtx* ctx = wave_ctx(wl);
    const uint32_t SW = sp.slot_words, CS = sp.w32cap, RW = sp.rec_words, SPW = sp.spill_words;
    uint32_t* stk = wl + kWaveFixedWords;
    uint32_t* cur = stk + (size_t)sp.lds_depth * SW;
    const uint32_t chunk = bcast0(ctx->spill_chunk);
    const uint32_t d = bcast0(ctx->d);
    const uint32_t refresh_v = bcast0(ctx->refresh);
    const uint32_t idstk = wl[kOffSave + lane];
    uint32_t Rb[WPL];
#pragma unroll
    for (int c = 0; c < WPL; c++) Rb[c] = cur[4u * ((uint32_t)c * 64u + lane) + 3u];
    // word t (0: P, 1: X, 2: L) of chunk c of frame s, for this lane
    auto fword = [&](uint32_t s, int c, uint32_t t) -> uint32_t* {
        const uint32_t li = (uint32_t)c * 64u + lane;
        if (s == d) return cur + 4u * li + t;
        if (s < sp.lds_depth) return stk + (size_t)s * SW + 4u * li + t;
        return sp.spill + ((size_t)chunk * sp.spill_levels + (s - sp.lds_depth)) * SPW + 4u * li + t;
    };
    // input id of the child pushed from frame j (j < d)
    auto child_id = [&](uint32_t j) -> uint32_t {
        if (j < sp.lds_depth) return rdlane(idstk, j);
        return bcast0(sp.spill[((size_t)chunk * sp.spill_levels + (j - sp.lds_depth)) * SPW + 3u]);
    };
    if (bcast0(lds_ld(&hdr->done))) return 1;
    const uint32_t busy = bcast0(lds_ld(&hdr->busy));
    const uint32_t lqn = bcast0(lds_ld(&hdr->lq_n));
    // Where to hand work: first to siblings that wait for it, then to a
    // workgroup that asked through the mailbox, and otherwise keep one unit in
    // stock in the LIFO so that a wavefront that finishes finds work at once.
    const bool siblings_wait = lqn < kLocalSlots && NW - busy > lqn;
    bool to_local = siblings_wait;
    uint32_t asker = 0;
    if (bcast0(lds_ld(&hdr->req)) != 0u) {
        uint32_t a = 0;
        if (lane == 0) {
            a = __hip_atomic_exchange(&hdr->req, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            // a workgroup whose own wavefronts wait has nothing to spare
            if (a != 0u && siblings_wait) {
                st_dev(&sp.mail[a - 1u].state, kMailRefused);
                a = 0u;
            }
        }
        asker = bcast0(a);
    }
    // Units to hand out now: one to the asker; to the LIFO one per waiting
    // sibling (or one to keep in stock).  Each comes from the shallowest frame
    // that can still be split, so a frame may give several in turn.
    uint32_t n_local = 0;
    if (to_local) n_local = umin32(NW - busy - lqn, kLocalSlots - lqn);
    else if (asker == 0u && lqn == 0u) n_local = 1;
    const uint32_t rounds = n_local + (asker != 0u ? 1u : 0u);
    bool gave = false;
    uint32_t given = 0;
    if (rounds != 0u) {
        for (uint32_t s = 0; s <= d && given < rounds;) {
            uint32_t Ls[WPL], Ps[WPL], Xs[WPL], cnt[WPL], incl[WPL];
#pragma unroll
            for (int c = 0; c < WPL; c++) {
                const uint32_t w = (uint32_t)c * 64u + lane;
                Ls[c] = (w < W) ? *fword(s, c, 2) : 0u;
            }
            const uint32_t tot = popc_scan<WPL>(Ls, cnt, incl);
            // an ancestor frame gives even its last candidate (the owner keeps
            // the subtree it is in); the current frame keeps half of its own
            if (tot < (s == d ? 2u : 1u)) {
                s++;
                continue;
            }
            uint32_t pc = 0;
#pragma unroll
            for (int c = 0; c < WPL; c++) {
                const uint32_t w = (uint32_t)c * 64u + lane;
                Ps[c] = (w < W) ? *fword(s, c, 0) : 0u;
                Xs[c] = (w < W) ? *fword(s, c, 1) : 0u;
                pc += (uint32_t)__builtin_popcount(Ps[c]);
            }
            // frames below are smaller still
            if (wave_sum(pc) < sp.split_threshold) break;
            const uint32_t keep = s == d ? (tot + 1u) / 2u : tot / 2u;
            uint32_t L1[WPL], L2[WPL], Pd[WPL], Xd[WPL], Rs[WPL];
#pragma unroll
            for (int c = 0; c < WPL; c++) {
                const uint32_t before = incl[c] - cnt[c];
                L1[c] = low_bits(Ls[c], rank_take(keep, before, cnt[c]));
                L2[c] = Ls[c] & ~L1[c];
                Pd[c] = Ps[c] & ~L1[c];
                Xd[c] = Xs[c] | L1[c];
                Rs[c] = Rb[c];
            }
            // R of frame s: one word a lane, the unit's R with the children
            // pushed from frames 0..s-1; else the current R without the
            // children pushed from frames s..d-1
            if (WPL == 1) {
                for (uint32_t j = 0; j < s; j++) set_bit<WPL>(Rs, child_id(j), lane);
            } else {
                for (uint32_t j = s; j < d; j++) clear_bit<WPL>(Rs, child_id(j), lane);
            }
            bool ok;
            if (asker != 0u && !gave) {
                // the unit is in transit until the asker takes it: count it
                // before it becomes visible
                store_record<WPL>(sp.mail_rec + (size_t)(asker - 1u) * RW, CS, lane, g, W, Rs, Pd, Xd, L2);
                if (lane == 0) __hip_atomic_fetch_add(&sp.ctl->work, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                vm_drain();
                if (lane == 0) st_dev(&sp.mail[asker - 1u].state, kMailUnit);
                ok = true;
            } else {
                if (!wg_lock(hdr, lane, t_start, sp.watchdog_ticks)) return 1;
                const uint32_t n = bcast0(lds_ld(&hdr->lq_n));
                ok = n < kLocalSlots;
                if (ok) {
                    uint32_t* r = lq + (size_t)n * RW;
                    if (lane == 0) r[0] = g;
#pragma unroll
                    for (int c = 0; c < WPL; c++) {
                        const uint32_t w = (uint32_t)c * 64u + lane;
                        if (w < W) {
                            r[kRecHeader + w] = Rs[c];
                            r[kRecHeader + CS + w] = Pd[c];
                            r[kRecHeader + 2 * CS + w] = Xd[c];
                            r[kRecHeader + 3 * CS + w] = L2[c];
                        }
                    }
                    if (lane == 0) lds_st(&hdr->lq_n, n + 1);
                }
                wg_unlock(hdr, lane);
            }
            if (ok) {
#pragma unroll
                for (int c = 0; c < WPL; c++) {
                    const uint32_t w = (uint32_t)c * 64u + lane;
                    if (w < W) *fword(s, c, 2) = L1[c];
                }
                if (lane == 0) ctx->donations += 1;
                gave = gave || asker != 0u;
                given++;
            } else {
                break; // the LIFO is full
            }
        }
    }
    if (asker != 0u && !gave && lane == 0) st_dev(&sp.mail[asker - 1u].state, kMailRefused);
    // Look at this workgroup's mailbox (the caller decides when: once per
    // refresh_children children of the workgroup; paced by work done, not by
    // a clock, because the real-time counter is slow to read from thousands of
    // wavefronts).  Only this workgroup and its askers touch that line.
    if (bcast0(refresh_v)) {
        uint32_t e = 0, rf = 0;
        if (lane == 0) {
            // the busy count other workgroups see, written when it changed
            if (lds_ld(&hdr->hint) != busy) {
                st_dev(&sp.mail[blockIdx.x].hint, busy);
                lds_st(&hdr->hint, busy);
            }
            if (lds_ld(&hdr->req) == 0u) {
                unsigned int* mreq = &sp.mail[blockIdx.x].req;
                if (ld_dev(mreq) != 0u) {
                    const uint32_t a = __hip_atomic_exchange(mreq, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    uint32_t zero = 0u;
                    // a sibling may have taken an earlier question meanwhile:
                    // then this one is refused rather than lost
                    if (a != 0u && !__hip_atomic_compare_exchange_strong(&hdr->req, &zero, a, __ATOMIC_RELAXED,
                                                                         __ATOMIC_RELAXED,
                                                                         __HIP_MEMORY_SCOPE_WORKGROUP))
                        st_dev(&sp.mail[a - 1u].state, kMailRefused);
                }
            }
            rf = ++ctx->refreshes;
            if ((rf & 7u) == 0u) e = error_or_cancel(sp, (rf & 63u) == 0u);
        }
        rf = bcast0(rf);
        const bool late = (rf & 63u) == 0u && sp.watchdog_ticks != 0 &&
                          (uint64_t)wall_clock64() - t_start > sp.watchdog_ticks;
        if (late && lane == 0) atomicOr(&sp.ctl->error, kErrWatchdog);
        if (bcast0(e) != 0u || late) {
            if (lane == 0) lds_st(&hdr->done, 1u);
            return 1;
        }
    }
    return 0;
}

// Spill chunk of this wavefront, for stack levels below its LDS window: taken
// from the pool on first use.  Returns 0xffffffff (and flags the launch for a
// rerun with a larger pool) when the pool is exhausted.
__device__ __attribute__((noinline)) uint32_t cold_spill_chunk(const SearchParams* __restrict__ spp, uint32_t* wl)
{
    const SearchParams& sp = *spp;
    const uint32_t lane = lane_id();
    uint32_t ch = 0;
    if (lane == 0) ch = (uint32_t)atomicAdd(&sp.ctl->spill_next, 1ull);
    ch = bcast0(ch);
    if (ch >= sp.spill_chunks) {
        if (lane == 0) atomicOr(&sp.ctl->error, kErrSpill);
        return 0xffffffffu;
    }
    if (lane == 0) wave_ctx(wl)->spill_chunk = ch;
    return ch;
}

// Flag the launch with error bits (QueueCtl.error).
__device__ __attribute__((noinline)) void cold_error(const SearchParams* __restrict__ spp, uint32_t bits_v)
{
    const uint32_t bits = bcast0(bits_v);
    if (lane_id() == 0) atomicOr(&spp->ctl->error, bits);
}

// Address-space views used by search_unit: constant (read-only during a
// launch: scalar loads) and global.
typedef const __attribute__((address_space(4))) SearchParams CParams;
typedef const __attribute__((address_space(4))) GraphDesc CGraphDesc;
typedef __attribute__((address_space(1))) uint32_t GU32;

// Why search_unit returned.
constexpr uint32_t kUnitDone = 0, kUnitAbort = 1, kUnitCheck = 2, kUnitFlush = 3, kUnitChunk = 4, kUnitDepth = 5,
                   kUnitBig = 6;

// The search of one unit (R, P, X, L) of graph g by one wavefront: Alg. 4
// from that node, branching only on the candidates in L.  The loop calls no
// function and has no lane-dependent branch, so that its registers stay few:
// whenever something must be done off the hot path (look at the siblings and
// the mailbox, hash a full clique buffer, take a spill chunk) it stores its
// state in LDS and returns why (kUnit*); the caller does it and calls again
// with resume = 1.  Counters since the last return are added to the
// wavefront's totals before every return.  wl_off: word offset of the
// wavefront's LDS block.
template <int WPL, int RULE>
__device__ __attribute__((noinline)) uint32_t search_unit(const SearchParams* __restrict__ spp_v, uint32_t wl_off,
                                                          LaneBits<WPL> Rbb, LaneBits<WPL> Pb, LaneBits<WPL> Xb,
                                                          LaneBits<WPL> Lb, uint32_t g_v, uint32_t resume_v)
{
    extern __shared__ uint32_t smem[];
    // The parameter block and the graph descriptors do not change during a
    // launch: read through a wave-uniform pointer in the constant address
    // space they are scalar loads into scalar registers.  The spill pool is addressed as global memory
    // (a generic access would be a FLAT one, after which every wait for a
    // row load must wait for all loads).
    const uint64_t spa = reinterpret_cast<uint64_t>(spp_v);
    const CParams& sp = *(const CParams*)(((uint64_t)bcast0((uint32_t)(spa >> 32)) << 32) | bcast0((uint32_t)spa));
    const uint32_t lane = lane_id();
    const uint32_t NW = blockDim.x >> 6;
    WgHdr* hdr = reinterpret_cast<WgHdr*>(smem);
    uint32_t* wl = smem + bcast0(wl_off);
    WaveCtx* ctx = wave_ctx(wl);
    const uint32_t g = bcast0(g_v);
    const bool resume = bcast0(resume_v) != 0u;
    const CGraphDesc& gd = ((const CGraphDesc*)(sp.graphs))[g];
    const uint64_t adj_off = gd.adj_off;
    const uint32_t W = gd.w32;
    const uint32_t rs4 = 4u * gd.rstride;
    // renumbered rows through a buffer resource: a row is addressed by a
    // scalar offset (v * row stride) plus this lane's word offset
    const uint64_t abase = reinterpret_cast<uint64_t>(sp.adj) + 4ull * adj_off;
    const __amdgpu_buffer_rsrc_t rows = __builtin_amdgcn_make_buffer_rsrc(
        reinterpret_cast<void*>(abase), (short)0, (int)(gd.n * rs4), 0x00020000);
    const uint32_t* ord = sp.order + gd.ord_off;
    uint32_t lane_lo[WPL], lane_w[WPL], voff[WPL];
    bool live[WPL];
#pragma unroll
    for (int c = 0; c < WPL; c++) {
        const uint32_t li = (uint32_t)c * 64u + lane;
        lane_lo[c] = li << 5;
        lane_w[c] = li;
        voff[c] = li << 2;
        live[c] = li < W;
    }
    // input id of the vertex whose row is in r: the word after the row
    auto row_id = [&](const uint32_t (&r)[WPL], uint32_t v) -> uint32_t {
        if (WPL == 1) return rdlane(r[0], W);
        if (W < 64u) return rdlane(r[0], W);
        if (W < 128u) return rdlane(r[1], W - 64u);
        return bcast0(ord[v]);
    };
    (void)ord;
    const uint32_t lds_depth = sp.lds_depth;
    const uint32_t ci = sp.check_interval;
    const uint32_t ci_fast = umax32(ci >> 2, 1u);
    const uint32_t SW = sp.slot_words, SPW = sp.spill_words;
    const uint32_t spill_levels = sp.spill_levels;
    GU32* const spill = (GU32*)(sp.spill);
    // the frame area's offset is hidden from the compiler, so that the frame
    // address stays one vector register (not a register plus a constant that
    // the paired LDS stores cannot encode)
    uint32_t fixed = kWaveFixedWords;
    asm volatile("" : "+s"(fixed));
    uint32_t* stk = wl + fixed;
    uint32_t* cur = stk + (size_t)lds_depth * SW;
    // this lane's words of frame 0 (frame s: + s * SW, chunk c: + 256 c)
    uint32_t* const fl = stk + 4u * lane;
    uint32_t* buf = wl + kOffBuf;
    uint32_t* trash = wl + kOffTrash;
    uint32_t* save = wl + kOffSave;
    // A workgroup looks at its mailbox about once per refresh_children of its
    // children: each of its busy wavefronts every busy * (refresh_children /
    // ci) of its own checks (busy as seen at its last look), at staggered
    // phases, so that a workgroup with one busy wavefront still answers as
    // often as a full one.
    const uint32_t rstep = umax32(sp.refresh_children / ci, 1u);
    uint32_t Rb[WPL], P[WPL], X[WPL], L[WPL];
    uint32_t d, budget, nent, used, rcount, idstk, cent;
    if (!resume) {
#pragma unroll
        for (int c = 0; c < WPL; c++) {
            Rb[c] = Rbb.w[c];
            P[c] = Pb.w[c];
            X[c] = Xb.w[c];
            L[c] = Lb.w[c];
        }
        d = 0;
        budget = ci;
        nent = bcast0(ctx->nent);
        used = bcast0(ctx->used);
        rcount = (bcast0(threadIdx.x >> 6) * rstep) % (umax32(bcast0(lds_ld(&hdr->busy)), 1u) * rstep) + 1u;
        idstk = 0;
        cent = save[64 + lane];
    } else {
#pragma unroll
        for (int c = 0; c < WPL; c++) {
            const uint32_t li = (uint32_t)c * 64u + lane;
            const uint4 q = *reinterpret_cast<const uint4*>(cur + 4u * li);
            P[c] = live[c] ? q.x : 0u;
            X[c] = live[c] ? q.y : 0u;
            L[c] = live[c] ? q.z : 0u;
            Rb[c] = live[c] ? q.w : 0u;
        }
        d = bcast0(ctx->d);
        budget = bcast0(ctx->budget);
        nent = bcast0(ctx->nent);
        used = bcast0(ctx->used);
        rcount = bcast0(ctx->rcount);
        idstk = save[lane];
        cent = save[64 + lane];
    }
    uint32_t chunk = bcast0(ctx->spill_chunk);
    // one word a lane: Rb is the unit's own R throughout (a clique's path
    // ids go to its buffer entry; donations add a frame's path ids), and rsz
    // its size.  Wider layouts keep Rb = the current node's R.
    const uint32_t rsz = WPL == 1 ? wave_sum((uint32_t)__builtin_popcount(Rb[0])) : 0u;
    uint32_t kids = 0;   // children examined since the last return
    uint32_t nodes = 0;  // nodes created since then
    uint32_t spills = 0; // frames written to the spill pool since then
    uint32_t why = kUnitDone;
    // Row v into r (one word per lane); the load is only issued here, and
    // the first use of r waits for it.
    auto load_row = [&](uint32_t v, uint32_t (&r)[WPL]) {
        const uint32_t so = v * rs4;
#pragma unroll
        for (int c = 0; c < WPL; c++)
            r[c] = (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(rows, (int)voff[c], (int)so, 0);
    };
    // cv: the first candidate left in L (-1: none); crow: its row.  The row
    // of the candidate after it is requested before the child cv is
    // examined, and an LDS frame keeps the row of its next candidate, so that
    // returning to a parent costs no row load.
    uint32_t crow[WPL];
    int cv = first_pos<WPL>(L, lane_lo);
    load_row(cv >= 0 ? (uint32_t)cv : 0u, crow);

    for (;;) {
        if (cv < 0) {
            // node finished: return to the parent frame
            if (d == 0) break;
            d--;
            uint32_t idp;
            if (d < lds_depth) {
                const uint32_t* f = fl + d * SW;
#pragma unroll
                for (int c = 0; c < WPL; c++) {
                    const uint4 q = *reinterpret_cast<const uint4*>(f + 256u * c);
                    P[c] = live[c] ? q.x : 0u;
                    X[c] = live[c] ? q.y : 0u;
                    L[c] = live[c] ? q.z : 0u;
                    crow[c] = q.w;
                }
                idp = rdlane(idstk, d);
                cv = first_pos<WPL>(L, lane_lo);
            } else {
                const GU32* f = spill + ((size_t)chunk * spill_levels + (d - lds_depth)) * SPW;
#pragma unroll
                for (int c = 0; c < WPL; c++) {
                    const uint32_t li = (uint32_t)c * 64u + lane;
                    P[c] = f[4 * li];
                    X[c] = f[4 * li + 1];
                    L[c] = f[4 * li + 2];
                }
                idp = bcast0(f[3]);
                cv = first_pos<WPL>(L, lane_lo);
                load_row(cv >= 0 ? (uint32_t)cv : 0u, crow);
            }
            if (WPL > 1) {
                uint32_t m[WPL];
                bit_mask<WPL>(idp, lane_w, m);
#pragma unroll
                for (int c = 0; c < WPL; c++) Rb[c] &= ~m[c];
            }
            (void)idp;
            continue;
        }
        // v is in L, L is a subset of P, and X is disjoint from P: taking v
        // out of L and P and into X flips one bit in each
        const uint32_t v = (uint32_t)cv;
        uint32_t m[WPL];
        bit_mask<WPL>(v, lane_w, m);
#pragma unroll
        for (int c = 0; c < WPL; c++) L[c] ^= m[c];
        // the next candidate's row is on its way while v is examined (with
        // no candidate left, row v again: a load on every path lets the wait
        // for crow below leave this one in flight)
        const int nv = first_pos<WPL>(L, lane_lo);
        uint32_t nrow[WPL];
        load_row(nv >= 0 ? (uint32_t)nv : v, nrow);
        // step 11: P' = P n N(v), X' = X n N(v)
        uint32_t P2[WPL], X2[WPL];
#pragma unroll
        for (int c = 0; c < WPL; c++) {
            P2[c] = P[c] & crow[c];
            X2[c] = X[c] & crow[c];
            // steps 12-13 for the current node
            P[c] ^= m[c];
            X[c] ^= m[c];
        }
        kids++;
        if (any_set<WPL>(P2)) {
            // the child is a node: push the current frame, descend.  A push
            // below the LDS window needs a spill chunk and room in it; without
            // them the child is put back (v into L and P, out of X) and
            // examined again once the caller has made room.
            if (d >= lds_depth && (chunk == 0xffffffffu || d - lds_depth >= spill_levels)) {
#pragma unroll
                for (int c = 0; c < WPL; c++) {
                    L[c] ^= m[c];
                    P[c] ^= m[c];
                    X[c] ^= m[c];
                }
                kids--;
                why = chunk == 0xffffffffu ? kUnitChunk : kUnitDepth;
                break;
            }
            const uint32_t idv = row_id(crow, v);
            nodes++;
            const uint32_t dp = d;
            // the parent's sets; an LDS frame is written below in one store,
            // with the parent's next row (a frame is 16 bytes a lane: one
            // 128-bit store instead of three 32-bit ones that would meet in
            // the same LDS banks)
            uint32_t Pp[WPL], Xp[WPL], Lp[WPL];
#pragma unroll
            for (int c = 0; c < WPL; c++) {
                Pp[c] = P[c];
                Xp[c] = X[c];
                Lp[c] = L[c];
            }
            if (d < lds_depth) {
                idstk = wrlane(idstk, idv, d);
            } else {
                GU32* fs = spill + ((size_t)chunk * spill_levels + (d - lds_depth)) * SPW;
#pragma unroll
                for (int c = 0; c < WPL; c++) {
                    const uint32_t li = (uint32_t)c * 64u + lane;
                    fs[4 * li] = P[c];
                    fs[4 * li + 1] = X[c];
                    fs[4 * li + 2] = L[c];
                    fs[4 * li + 3] = idv;
                }
                spills++;
            }
            d++;
            if (WPL > 1) {
                uint32_t mi[WPL];
                bit_mask<WPL>(idv, lane_w, mi);
#pragma unroll
                for (int c = 0; c < WPL; c++) Rb[c] |= mi[c];
            }
#pragma unroll
            for (int c = 0; c < WPL; c++) {
                P[c] = P2[c];
                X[c] = X2[c];
            }
            // step 9: the pivot.  GreedyBB: the first of X if X is non-empty,
            // else the first of P.  The row of the first of P is requested
            // with the pivot's: it is the first candidate whenever it is not
            // adjacent to the pivot (always when the pivot is that vertex).
            const int px = first_pos<WPL>(X, lane_lo);
            const int pp = first_pos_nz<WPL>(P, lane_lo);
            uint32_t prow[WPL], frow[WPL];
            if (RULE == (int)kPivotGreedy || (RULE == (int)kPivotTX && px < 0)) {
                const uint32_t piv = px >= 0 ? (uint32_t)px : (uint32_t)pp;
                load_row(piv, prow);
                load_row((uint32_t)pp, frow);
            } else {
                // TomitaBB (candidates P u X) and GreedyBBTX (candidates X):
                // the candidate u maximising |P n N(u)|, the earliest on ties.
                // Candidates are taken in order, the next one's row on its way
                // while the current one is counted; no candidate can beat
                // |P| (only a vertex of X reaches it), so the scan stops there.
                load_row((uint32_t)pp, frow);
                uint32_t C[WPL];
                uint32_t pc = 0;
#pragma unroll
                for (int c = 0; c < WPL; c++) {
                    C[c] = (RULE == (int)kPivotTomita) ? (P[c] | X[c]) : X[c];
                    pc += (uint32_t)__builtin_popcount(P[c]);
                }
                const uint32_t psize = wave_sum(pc);
                int u = first_pos<WPL>(C, lane_lo);
                uint32_t urow[WPL];
                load_row((uint32_t)u, urow);
                uint32_t bestc = 0;
                bool have = false;
                for (;;) {
                    uint32_t mu[WPL];
                    bit_mask<WPL>((uint32_t)u, lane_w, mu);
#pragma unroll
                    for (int c = 0; c < WPL; c++) C[c] &= ~mu[c];
                    const int nu = first_pos<WPL>(C, lane_lo);
                    uint32_t urow2[WPL];
                    load_row(nu >= 0 ? (uint32_t)nu : (uint32_t)u, urow2);
                    uint32_t cnt = 0;
#pragma unroll
                    for (int c = 0; c < WPL; c++) cnt += (uint32_t)__builtin_popcount(P[c] & urow[c]);
                    cnt = wave_sum(cnt);
                    if (!have || cnt > bestc) {
                        have = true;
                        bestc = cnt;
#pragma unroll
                        for (int c = 0; c < WPL; c++) prow[c] = urow[c];
                        if (cnt == psize) break;
                    }
                    if (nu < 0) break;
                    u = nu;
#pragma unroll
                    for (int c = 0; c < WPL; c++) urow[c] = urow2[c];
                }
            }
            // step 10: L = P \ N(p)
#pragma unroll
            for (int c = 0; c < WPL; c++) L[c] = P[c] & ~prow[c];
            // the parent's next row, requested before the pivot's, is in:
            // the parent's LDS frame is written now, sets and row together
            // (with no next candidate the row is never read).  A frame in
            // the spill pool keeps no row: the store then goes to the slot of
            // the current frame, which the loop writes whenever it returns,
            // before anything reads it.
            {
                uint32_t* f = fl + (dp < lds_depth ? dp : lds_depth) * SW;
#pragma unroll
                for (int c = 0; c < WPL; c++)
                    *reinterpret_cast<uint4*>(f + 256u * c) = make_uint4(Pp[c], Xp[c], Lp[c], nrow[c]);
            }
            cv = first_pos<WPL>(L, lane_lo);
            if (cv == pp) {
#pragma unroll
                for (int c = 0; c < WPL; c++) crow[c] = frow[c];
            } else if (cv >= 0) {
                load_row((uint32_t)cv, crow);
            }
        } else {
            if (!any_set<WPL>(X2)) {
                // P' and X' empty: R u {v} is maximal.  One word a lane: a
                // clique of at most kCliqueListMax vertices whose path is in
                // the LDS window is written as a list entry (the path's ids,
                // lanes 0..d-1 of the id stack, then v's; lane j writes word
                // j).  Otherwise the entry holds the non-empty 16-bit halves
                // of the clique's bitset over input ids, in lane order (the
                // clique's sorted ids); one word a lane rebuilds R first from
                // the unit's R and the path.  A clique has at most 2 W halves:
                // up to four chunks the buffer is emptied whenever fewer than
                // the longest entry's slots are left; wider graphs count the
                // clique's halves first and, when they do not fit, put the
                // child back and empty the buffer (a clique larger than the
                // whole buffer is an error).
                const uint32_t idv = row_id(crow, v);
                bool listed = false;
                if (WPL == 1 && d < lds_depth && rsz + d + 1u <= kCliqueListMax) {
                    *(lane <= d ? buf + used + lane : trash + lane) = lane < d ? idstk : idv;
                    cent = wrlane(cent, (used << 16) | kEntryList | (d + 1u), nent);
                    used += d + 1u;
                    listed = true;
                }
                if (!listed) {
                    uint32_t mi[WPL], cwd[WPL];
                    uint64_t blo[WPL], bhi[WPL];
                    uint32_t halves = 0;
                    bit_mask<WPL>(idv, lane_w, mi);
#pragma unroll
                    for (int c = 0; c < WPL; c++) cwd[c] = Rb[c] | mi[c];
                    if (WPL == 1) {
                        for (uint32_t j = 0; j < d; j++) {
                            const uint32_t id = j < lds_depth
                                                    ? rdlane(idstk, j)
                                                    : bcast0(spill[((size_t)chunk * spill_levels + (j - lds_depth)) * SPW + 3u]);
                            uint32_t mj[WPL];
                            bit_mask<WPL>(id, lane_w, mj);
                            cwd[0] |= mj[0];
                        }
                    }
#pragma unroll
                    for (int c = 0; c < WPL; c++) {
                        blo[c] = ballot((cwd[c] & 0xffffu) != 0u);
                        bhi[c] = ballot((cwd[c] >> 16) != 0u);
                        halves += (uint32_t)__builtin_popcountll(blo[c]) + (uint32_t)__builtin_popcountll(bhi[c]);
                    }
                    if (WPL >= 4 && used + halves > kCliqueSlots) {
#pragma unroll
                        for (int c = 0; c < WPL; c++) {
                            L[c] ^= m[c];
                            P[c] ^= m[c];
                            X[c] ^= m[c];
                        }
                        kids--;
                        why = used == 0u ? kUnitBig : kUnitFlush;
                        break;
                    }
                    const uint32_t start = used;
#pragma unroll
                    for (int c = 0; c < WPL; c++) {
                        const uint32_t lo = cwd[c] & 0xffffu, hi = cwd[c] >> 16;
                        const uint32_t below =
                            __builtin_amdgcn_mbcnt_hi((uint32_t)(blo[c] >> 32),
                                                      __builtin_amdgcn_mbcnt_lo((uint32_t)blo[c], 0u)) +
                            __builtin_amdgcn_mbcnt_hi((uint32_t)(bhi[c] >> 32),
                                                      __builtin_amdgcn_mbcnt_lo((uint32_t)bhi[c], 0u));
                        const uint32_t plo = used + below;
                        const uint32_t phi = plo + (lo != 0u ? 1u : 0u);
                        const uint32_t hw = (((uint32_t)c * 64u + lane) << 1);
                        *(lo != 0u ? buf + plo : trash + lane) = (hw << 16) | lo;
                        *(hi != 0u ? buf + phi : trash + lane) = ((hw + 1u) << 16) | hi;
                        used += (uint32_t)__builtin_popcountll(blo[c]) + (uint32_t)__builtin_popcountll(bhi[c]);
                    }
                    cent = wrlane(cent, (start << 16) | (used - start), nent);
                }
                nent++;
                cv = nv;
#pragma unroll
                for (int c = 0; c < WPL; c++) crow[c] = nrow[c];
                // a full clique buffer is emptied at once
                if (nent == 64u || (WPL < 4 && used + umax32(2u * W, WPL == 1 ? kCliqueListMax : 0u) > kCliqueSlots)) {
                    why = kUnitFlush;
                    break;
                }
            } else {
                cv = nv;
#pragma unroll
                for (int c = 0; c < WPL; c++) crow[c] = nrow[c];
            }
        }
        if (--budget == 0u) {
            // Look at the siblings and the workgroup's flags (LDS only);
            // suspend for the out-of-line look only when there is something
            // to do.  While siblings wait, look four times as often.
            const uint32_t busy = bcast0(lds_ld(&hdr->busy));
            const uint32_t lqn = bcast0(lds_ld(&hdr->lq_n));
            const uint32_t dn = bcast0(lds_ld(&hdr->done));
            const uint32_t asked = bcast0(lds_ld(&hdr->req));
            const bool waiting = lqn < kLocalSlots && NW - busy > lqn;
            budget = waiting ? ci_fast : ci;
            const uint32_t refresh = --rcount == 0u;
            if (refresh) rcount = umax32(busy, 1u) * rstep;
            if (dn) {
                why = kUnitAbort;
                break;
            }
            if (refresh || asked || lqn == 0u || waiting) {
                // every lane stores the same value: no lane-dependent branch
                ctx->refresh = refresh;
                why = kUnitCheck;
                break;
            }
        }
    }
    // Suspend (or finish): the loop's state to LDS, the counters to the totals.
    if (why != kUnitDone && why != kUnitAbort) {
#pragma unroll
        for (int c = 0; c < WPL; c++) {
            const uint32_t li = (uint32_t)c * 64u + lane;
            *reinterpret_cast<uint4*>(cur + 4u * li) = make_uint4(P[c], X[c], L[c], Rb[c]);
        }
        save[lane] = idstk;
        ctx->d = d;
        ctx->budget = budget;
        ctx->rcount = rcount;
    } else if (WPL == 1) {
        // the unit's R, for the flush of the clique buffer that follows
        cur[4u * lane + 3u] = Rb[0];
    }
    save[64 + lane] = cent;
    ctx->nent = nent;
    ctx->used = used;
    ctx->nodes = ctx->nodes + nodes;
    ctx->children = ctx->children + kids;
    ctx->spills = ctx->spills + spills;
    return why;
}

template <int WPL, int RULE>
__global__ void __launch_bounds__(64 * max_search_wpb(WPL)) search_kernel(SearchParams sp,
                                                                         const SearchParams* __restrict__ spp)
{
    // sp (by value) serves the hot path, where its pointers are known to be
    // global; spp, the same block in HBM, is handed to the out-of-line helpers.
    extern __shared__ uint32_t smem[];
    const uint32_t lane = lane_id();
    const uint32_t wv = threadIdx.x >> 6;
    const uint32_t NW = blockDim.x >> 6;
    WgHdr* hdr = reinterpret_cast<WgHdr*>(smem);
    uint32_t* lq = smem + kWgHdrWords;
    const uint32_t RW = sp.rec_words;
    uint32_t* wl = lq + kLocalSlots * RW + (size_t)wv * sp.wave_lds_words;
    WaveCtx* ctx = wave_ctx(wl);

    if (threadIdx.x < kWgHdrWords) smem[threadIdx.x] = 0u;
    for (uint32_t i = lane; i < kWaveFixedWords; i += 64) wl[i] = 0u;
    if (lane == 0) {
        ctx->g = 0xffffffffu;
        ctx->spill_chunk = 0xffffffffu;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        // written by the root kernels, which ran before this one
        const uint32_t ps = sp.ctl->pool_size;
        hdr->pool_size = ps;
        hdr->pool_left = ps != 0u;
        hdr->rng = (blockIdx.x + 1u) * 0x9E3779B9u;
    }
    __syncthreads();

    const uint64_t t_start = wall_clock64();
    auto overdue = [&]() -> bool {
        return sp.watchdog_ticks != 0 && wall_clock64() - t_start > sp.watchdog_ticks;
    };
    auto give_up = [&]() {
        if (lane == 0) {
            atomicOr(&sp.ctl->error, kErrWatchdog);
            lds_st(&hdr->done, 1u);
        }
    };
    const uint32_t gwave = blockIdx.x * NW + wv;
    auto set_state = [&](uint32_t st) {
        if (lane == 0 && sp.wave_state) sp.wave_state[gwave] = st;
    };
    set_state(kWaveIdle);

    const uint32_t me = blockIdx.x;
    uint32_t backoff = 1, idle_iters = 0, polls = 0;
    WaveTimes times{0, 0}; // lane 0 only
    for (;;) {
        // ================= obtain a unit =================
        // src 1: the LDS LIFO (slot lsl), 2: the pool of root units (index
        // pos), 3: this workgroup's mailbox
        uint32_t src = 0, lsl = 0, pos = 0;
        bool stop = false;
        for (;;) {
            // Look without the lock first; take it only when there is something to do.
            {
                const uint32_t n0 = bcast0(lds_ld(&hdr->lq_n));
                const uint32_t dn0 = bcast0(lds_ld(&hdr->done));
                const uint32_t f0 = bcast0(lds_ld(&hdr->fetcher));
                if (n0 == 0u && dn0 == 0u && f0 != 0u) { // a sibling looks for work
                    if ((++idle_iters & 255u) == 0u && overdue()) {
                        give_up();
                        stop = true;
                        break;
                    }
                    // While siblings are busy, a waiting wavefront takes
                    // questions from other workgroups out of the mailbox, so
                    // that a busy sibling answers at its next check (LDS
                    // only) instead of reading the mailbox itself.
                    if ((idle_iters & 3u) == 0u && lane == 0 && lds_ld(&hdr->busy) != 0u &&
                        lds_ld(&hdr->req) == 0u) {
                        unsigned int* mreq = &sp.mail[me].req;
                        if (ld_dev(mreq) != 0u) {
                            const uint32_t a =
                                __hip_atomic_exchange(mreq, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            uint32_t zero = 0u;
                            if (a != 0u && !__hip_atomic_compare_exchange_strong(&hdr->req, &zero, a,
                                                                                 __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                                                 __HIP_MEMORY_SCOPE_WORKGROUP))
                                st_dev(&sp.mail[a - 1u].state, kMailRefused);
                        }
                    }
                    __builtin_amdgcn_s_sleep(16);
                    continue;
                }
            }
            if (((++idle_iters & 255u) == 0u && overdue()) || !wg_lock(hdr, lane, t_start, sp.watchdog_ticks)) {
                give_up();
                stop = true;
                break;
            }
            const uint32_t n = bcast0(lds_ld(&hdr->lq_n));
            if (n > 0) {
                lsl = n - 1;
                if (lane == 0) {
                    lds_st(&hdr->lq_n, n - 1);
                    lds_st(&hdr->busy, lds_ld(&hdr->busy) + 1);
                }
                src = 1;
                break; // still holding the lock: the record is copied below
            }
            if (bcast0(lds_ld(&hdr->done))) {
                wg_unlock(hdr, lane);
                stop = true;
                break;
            }
            // This wavefront is idle and the LIFO is empty: it looks for work
            // outside the workgroup unless a sibling already does.  The
            // workgroup leaves ctl->work if none of its wavefronts holds a
            // unit any more.
            uint32_t fetch = 0, went_inactive = 0, inactive = 0;
            if (lane == 0 && lds_ld(&hdr->fetcher) == 0u) {
                lds_st(&hdr->fetcher, 1u);
                fetch = 1;
                if (lds_ld(&hdr->busy) == 0u && lds_ld(&hdr->active) != 0u) {
                    lds_st(&hdr->active, 0u);
                    went_inactive = 1;
                }
                inactive = lds_ld(&hdr->active) == 0u;
            }
            wg_unlock(hdr, lane);
            fetch = bcast0(fetch);
            inactive = bcast0(inactive);
            if (lane == 0 && went_inactive) {
                __hip_atomic_fetch_sub(&sp.ctl->work, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                st_dev(&sp.mail[me].hint, 0u);
                lds_st(&hdr->hint, 0u);
            }
            if (fetch) {
                set_state(kWaveFetch);
                uint32_t kind = 0, p = 0, stop_now = 0;
                if (lane == 0) {
                    // (a) the answer to this workgroup's question.  A unit is
                    // marked as being read, so that no later fetcher takes it
                    // again or asks anew before the record slot is free.
                    const uint32_t o = lds_ld(&hdr->out);
                    if (o != 0u && o != kOutReading) {
                        const uint32_t st = ld_dev(&sp.mail[me].state);
                        if (st == kMailUnit) {
                            kind = 3;
                            lds_st(&hdr->out, kOutReading);
                        } else if (st == kMailRefused) {
                            // the cleared answer word must land before a new
                            // question can be answered, or it could wipe that
                            // answer out
                            st_dev(&sp.mail[me].state, kMailNone);
                            vm_drain();
                            lds_st(&hdr->out, 0u);
                        }
                    }
                    // (b) a root unit from the pool
                    if (kind == 0 && lds_ld(&hdr->pool_left) != 0u) {
                        const uint32_t t = __hip_atomic_fetch_add(&sp.ctl->pool_next, 1u, __ATOMIC_RELAXED,
                                                                  __HIP_MEMORY_SCOPE_AGENT);
                        if (t < lds_ld(&hdr->pool_size)) {
                            kind = 2;
                            p = t;
                        } else {
                            lds_st(&hdr->pool_left, 0u);
                        }
                    }
                    // (c) a question to this workgroup while it holds no work:
                    // refuse it (a busy workgroup answers from its checks)
                    if (inactive) {
                        uint32_t a = __hip_atomic_exchange(&hdr->req, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                        unsigned int* mreq = &sp.mail[me].req;
                        if (a == 0u && ld_dev(mreq) != 0u)
                            a = __hip_atomic_exchange(mreq, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        if (a != 0u) st_dev(&sp.mail[a - 1u].state, kMailRefused);
                    }
                    // (d) ask a workgroup: of a few chosen at random, the one
                    // whose hint shows the most busy wavefronts
                    if (kind == 0 && lds_ld(&hdr->out) == 0u && lds_ld(&hdr->pool_left) == 0u && sp.num_wg > 1u) {
                        uint32_t x = lds_ld(&hdr->rng);
                        uint32_t cand[kAskSamples], hint[kAskSamples];
#pragma unroll
                        for (uint32_t t = 0; t < kAskSamples; t++) {
                            x ^= x << 13;
                            x ^= x >> 17;
                            x ^= x << 5;
                            uint32_t c = (uint32_t)(((uint64_t)x * (sp.num_wg - 1u)) >> 32);
                            cand[t] = c >= me ? c + 1u : c;
                        }
#pragma unroll
                        for (uint32_t t = 0; t < kAskSamples; t++) hint[t] = ld_dev(&sp.mail[cand[t]].hint);
                        lds_st(&hdr->rng, x);
                        uint32_t v = cand[0], vb = hint[0];
#pragma unroll
                        for (uint32_t t = 1; t < kAskSamples; t++)
                            if (hint[t] > vb) {
                                v = cand[t];
                                vb = hint[t];
                            }
                        uint32_t zero = 0u;
                        if (__hip_atomic_compare_exchange_strong(&sp.mail[v].req, &zero, me + 1u, __ATOMIC_RELAXED,
                                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                            lds_st(&hdr->out, v + 1u);
                    }
                    // (e) the end of the search, seen by a workgroup that holds no work
                    if (kind == 0 && inactive && (++polls % sp.poll_iters) == 0u) {
                        const uint32_t w = ld_dev(&sp.ctl->work);
                        const uint32_t e = error_or_cancel(sp, (polls & 63u) == 0u);
                        const bool late = (polls & 63u) == 0u && overdue();
                        if (late) atomicOr(&sp.ctl->error, kErrWatchdog);
                        if (w == 0u || e != 0u || late) stop_now = 1;
                    }
                }
                kind = bcast0(kind);
                p = bcast0(p);
                if (bcast0(stop_now)) {
                    if (lane == 0) {
                        lds_st(&hdr->done, 1u);
                        lds_st(&hdr->fetcher, 0u);
                    }
                    stop = true;
                    break;
                }
                if (kind != 0u) {
                    uint32_t was_active = 0;
                    if (!wg_lock(hdr, lane, t_start, sp.watchdog_ticks)) {
                        give_up();
                        stop = true;
                        break;
                    }
                    if (lane == 0) {
                        was_active = lds_ld(&hdr->active);
                        lds_st(&hdr->active, 1u);
                        lds_st(&hdr->busy, lds_ld(&hdr->busy) + 1);
                        lds_st(&hdr->fetcher, 0u);
                    }
                    wg_unlock(hdr, lane);
                    // the unit's count is already covered by this workgroup
                    if (lane == 0 && was_active)
                        __hip_atomic_fetch_sub(&sp.ctl->work, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if (lane == 0 && !was_active) {
                        st_dev(&sp.mail[me].hint, 1u);
                        lds_st(&hdr->hint, 1u);
                    }
                    src = kind;
                    pos = p;
                    break;
                }
                if (lane == 0) lds_st(&hdr->fetcher, 0u);
            }
            for (uint32_t i = 0; i < backoff; i++) __builtin_amdgcn_s_sleep(8);
            if (backoff < 8) backoff <<= 1;
        }
        if (stop) break;
        backoff = 1;
        set_state(kWaveBusy);

        // ================= load the unit =================
        const uint32_t CS = sp.w32cap;
        uint32_t Rb[WPL], P[WPL], X[WPL], L[WPL];
        uint32_t g;
        if (src == 1) {
            const uint32_t* rec = lq + (size_t)lsl * RW;
            g = bcast0(rec[0]);
            const uint32_t W0 = bcast0(sp.graphs[g].w32);
#pragma unroll
            for (int c = 0; c < WPL; c++) {
                const uint32_t w = (uint32_t)c * 64u + lane;
                const bool in = w < W0;
                Rb[c] = in ? rec[kRecHeader + w] : 0u;
                P[c] = in ? rec[kRecHeader + CS + w] : 0u;
                X[c] = in ? rec[kRecHeader + 2 * CS + w] : 0u;
                L[c] = in ? rec[kRecHeader + 3 * CS + w] : 0u;
            }
            wg_unlock(hdr, lane);
        } else {
            const uint32_t* rec = (src == 2) ? (sp.rec + (size_t)pos * RW) : (sp.mail_rec + (size_t)me * RW);
            g = bcast0(ld_dev(&rec[0]));
            const uint32_t W0 = bcast0(sp.graphs[g].w32);
#pragma unroll
            for (int c = 0; c < WPL; c++) {
                const uint32_t w = (uint32_t)c * 64u + lane;
                const bool in = w < W0;
                Rb[c] = in ? ld_dev(&rec[kRecHeader + w]) : 0u;
                P[c] = in ? ld_dev(&rec[kRecHeader + CS + w]) : 0u;
                X[c] = in ? ld_dev(&rec[kRecHeader + 2 * CS + w]) : 0u;
                L[c] = in ? ld_dev(&rec[kRecHeader + 3 * CS + w]) : 0u;
            }
            if (src == 3) {
                // the record is read: the mailbox may take the next answer,
                // once the cleared answer word has landed (else it could
                // wipe out that next answer)
                vm_drain();
                if (lane == 0) st_dev(&sp.mail[me].state, kMailNone);
                vm_drain();
                if (lane == 0) lds_st(&hdr->out, 0u);
            }
        }
        const uint32_t gprev = bcast0(ctx->g);
        if (g != gprev) {
            // the totals are folded into HBM only when the result slot
            // changes: the local graphs of a graph all report into its slot,
            // and a fold a unit would queue their atomics on the same words
            if (gprev != 0xffffffffu && sp.graphs[g].res != sp.graphs[gprev].res) cold_fold(spp, wl);
            if (lane == 0) ctx->g = g;
        }
        if (lane == 0) ctx->units += 1;

        // ================= the search of the unit (Alg. 4) =================
        const uint64_t t_unit = wall_clock64();
        LaneBits<WPL> ub[4];
#pragma unroll
        for (int c = 0; c < WPL; c++) {
            ub[0].w[c] = Rb[c];
            ub[1].w[c] = P[c];
            ub[2].w[c] = X[c];
            ub[3].w[c] = L[c];
        }
        const uint32_t wl_off = (uint32_t)(wl - smem);
        const uint32_t W = bcast0(sp.graphs[g].w32);
        bool abort = false;
        for (uint32_t resume = 0;; resume = 1) {
            const uint32_t why = bcast0(search_unit<WPL, RULE>(spp, wl_off, ub[0], ub[1], ub[2], ub[3], g, resume));
            if (why == kUnitDone) break;
            if (why == kUnitCheck) {
                if (lane == 0) ctx->checks += 1;
                abort = bcast0(cold_check<WPL>(spp, smem, wl, W, g, t_start)) != 0u;
            } else if (why == kUnitFlush) {
                if (lane == 0) ctx->flushes += 1;
                cold_flush(spp, wl, g);
            } else if (why == kUnitChunk) {
                abort = bcast0(cold_spill_chunk(spp, wl)) == 0xffffffffu;
            } else {
                if (why == kUnitDepth) cold_error(spp, kErrDepth);
                if (why == kUnitBig) cold_error(spp, kErrClique);
                abort = true;
            }
            if (abort) break;
        }
        if (bcast0(ctx->nent) != 0u) cold_flush(spp, wl, g);
        if (lane == 0) {
            const uint64_t t_end = wall_clock64();
            ctx->busy += t_end - t_unit;
            if (times.first == 0) times.first = t_unit;
            times.last = t_end;
        }

        // ---- unit finished ----
        set_state(kWaveIdle);
        if (!wg_lock(hdr, lane, t_start, sp.watchdog_ticks)) {
            give_up();
            break;
        }
        if (lane == 0) lds_st(&hdr->busy, lds_ld(&hdr->busy) - 1);
        if (abort && lane == 0) lds_st(&hdr->done, 1u);
        wg_unlock(hdr, lane);
        if (abort) break;
    }
    cold_exit(spp, wl, gwave, t_start, times.first, times.last);
    set_state(kWaveExited);
}

// One wavefront a workgroup, no LDS (so that a fold can start beside other
// work that holds most of a compute unit), kFoldRecs exit records a
// wavefront: lane r < kFoldRecs takes record r's totals and counters, lane i
// adds histogram entry i of all of them.  The counters are summed over the
// wavefront and added to the control block once; when all records that hold
// totals report to the same result slot and histogram (one graph, as in
// every search of local graphs), so are the totals, else each record adds
// its own.  Record indices are clamped instead of branched on, so that a
// lane's loads are independent and leave back to back.
constexpr uint32_t kFoldRecs = 32;
__device__ __forceinline__ unsigned long long wave_sum64(unsigned long long v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ unsigned long long wave_xor64(unsigned long long v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v ^= __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ uint32_t wave_max32(uint32_t v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = umax32(v, (uint32_t)__shfl_xor((int)v, o, 64));
    return v;
}
__device__ __forceinline__ uint32_t wave_min32(uint32_t v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = umin32(v, (uint32_t)__shfl_xor((int)v, o, 64));
    return v;
}
__device__ __forceinline__ unsigned long long wave_min64(unsigned long long v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long a = __shfl_xor(v, o, 64);
        v = a < v ? a : v;
    }
    return v;
}
__device__ __forceinline__ unsigned long long wave_max64(unsigned long long v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long a = __shfl_xor(v, o, 64);
        v = a > v ? a : v;
    }
    return v;
}

__global__ void __launch_bounds__(64) exit_fold_kernel(SearchParams sp, uint32_t waves)
{
    const uint32_t lane = threadIdx.x;
    const uint32_t base = blockIdx.x * kFoldRecs;
    const uint32_t last = waves - 1u;
    // histogram entries first: they are independent of the rest
    unsigned long long x[kFoldRecs], h = 0ull;
#pragma unroll
    for (uint32_t k = 0; k < kFoldRecs; k++) x[k] = sp.exits[umin32(base + k, last)].hist[lane];
#pragma unroll
    for (uint32_t k = 0; k < kFoldRecs; k++) h += base + k <= last ? x[k] : 0ull;
    const uint32_t r = base + lane;
    const bool have = lane < kFoldRecs && r <= last;
    const WaveExit* e = sp.exits + umin32(r, last);
    const uint32_t er = e->res;
    const uint32_t res = have ? er : kNoSlot;
    const bool holds = res != kNoSlot;
    const unsigned long long hoff = e->hist_off, hx = e->hash_xor;
    const uint32_t om = e->omega;
    unsigned long long v[14];
    v[0] = e->units;
    v[1] = e->donations;
    v[2] = e->spills;
    v[3] = e->checks;
    v[4] = e->flushes;
    v[5] = e->busy;
    v[6] = e->run;
    v[7] = e->ramp;
    v[8] = e->tail;
    v[9] = 0ull;
    v[10] = e->count;
    v[11] = e->nodes;
    v[12] = e->children;
    v[13] = e->hash_sum;
    const uint32_t rmin = wave_min32(res), rmax = wave_max32(holds ? res : 0u);
    const unsigned long long omin = wave_min64(holds ? hoff : ~0ull), omax = wave_max64(holds ? hoff : 0ull);
    const bool one_slot = rmin != kNoSlot && rmin == rmax && omin == omax;
    // lane k ends with sum k (k < 14), the XOR (14) or the maximum (15)
    unsigned long long mine = 0ull;
#pragma unroll
    for (uint32_t k = 0; k < 14u; k++) {
        const bool counter = k < 10u;
        if (counter || one_slot) {
            const unsigned long long w = wave_sum64(counter ? (have ? v[k] : 0ull) : (holds ? v[k] : 0ull));
            if (lane == k) mine = w;
        }
    }
    if (one_slot) {
        const unsigned long long wx = wave_xor64(holds ? hx : 0ull);
        const uint32_t wm = wave_max32(holds ? om : 0u);
        if (lane == 14u) mine = wx;
        if (lane == 15u) mine = wm;
    } else {
        // each record adds its own: lane r its totals, lane i entry i of
        // every record's histogram (the entries loaded above)
        if (holds) {
            DevResult* d = sp.results + res;
            if (v[10]) atomicAdd(&d->count, v[10]);
            if (v[11]) atomicAdd(&d->nodes, v[11]);
            if (v[12]) atomicAdd(&d->children, v[12]);
            if (v[13]) atomicAdd(&d->hash_sum, v[13]);
            if (hx) atomicXor(&d->hash_xor, hx);
            if (om) atomicMax(&d->omega, om);
        }
#pragma unroll
        for (uint32_t k = 0; k < kFoldRecs; k++) {
            const uint32_t rk = (uint32_t)__shfl((int)res, (int)k, 64);
            const unsigned long long ok = __shfl(hoff, (int)k, 64);
            if (rk != kNoSlot && x[k] != 0ull) atomicAdd(&sp.hist[ok + lane], x[k]);
        }
    }
    if (mine != 0ull) {
        QueueCtl* c = sp.ctl;
        DevResult* d = sp.results + (one_slot ? rmin : 0u);
        switch (lane) {
        case 0: atomicAdd(&c->units, mine); break;
        case 1: atomicAdd(&c->donations, mine); break;
        case 2: atomicAdd(&c->spill_levels_written, mine); break;
        case 3: atomicAdd(&c->checks, mine); break;
        case 4: atomicAdd(&c->flushes, mine); break;
        case 5: atomicAdd(&c->busy_ticks, mine); break;
        case 6: atomicAdd(&c->run_ticks, mine); break;
        case 7: atomicAdd(&c->ramp_ticks, mine); break;
        case 8: atomicAdd(&c->tail_ticks, mine); break;
        case 10: atomicAdd(&d->count, mine); break;
        case 11: atomicAdd(&d->nodes, mine); break;
        case 12: atomicAdd(&d->children, mine); break;
        case 13: atomicAdd(&d->hash_sum, mine); break;
        case 14: atomicXor(&d->hash_xor, mine); break;
        case 15: atomicMax(&d->omega, (uint32_t)mine); break;
        default: break;
        }
    }
    if (one_slot && h) atomicAdd(&sp.hist[omin + lane], h);
}

} // namespace

// ---------------------------------------------------------- launchers ----

hipError_t launch_validate(const uint64_t* rows, uint32_t n, uint32_t rw, unsigned int* flag,
                           hipStream_t s)
{
    (void)hipGetLastError(); // report only this call's launch errors
    const uint64_t total = (uint64_t)n * rw;
    if (total == 0) return hipSuccess;
    const uint32_t blocks = (uint32_t)((total + 255) / 256);
    hipLaunchKernelGGL(validate_kernel, dim3(blocks), dim3(256), 0, s, rows, n, rw, flag);
    return hipGetLastError();
}

static hipError_t ensure_order_attr()
{
    // Allow the staged ordering kernels the full LDS of a workgroup once per process.
    static std::once_flag once;
    static hipError_t err = hipSuccess;
    std::call_once(once, [] {
        int dev = 0, lds = 0;
        err = hipGetDevice(&dev);
        if (err == hipSuccess) err = hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
        const void* ks[] = {(const void*)order_lds_kernel<8>, (const void*)order_lds_kernel<16>,
                            (const void*)order_lds_kernel<32>};
        for (const void* k : ks)
            if (err == hipSuccess) err = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    });
    return err;
}

static hipError_t ensure_bucket_attr()
{
    // Allow the bucket ordering kernels the full LDS of a workgroup once per process.
    static std::once_flag once;
    static hipError_t err = hipSuccess;
    std::call_once(once, [] {
        int dev = 0, lds = 0;
        err = hipGetDevice(&dev);
        if (err == hipSuccess) err = hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
        // the kernels' static LDS (their shared scalars) comes on top
        const void* ks[] = {(const void*)order_bucket_kernel<4, 0>, (const void*)order_bucket_kernel<6, 0>,
                            (const void*)order_bucket_kernel<8, 0>, (const void*)order_bucket_kernel<4, 2>};
        for (const void* k : ks)
            if (err == hipSuccess)
                err = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, lds - (int)kBucketStaticLds);
    });
    return err;
}

// The bucket ordering's LDS for graphs of up to max_n vertices: kw (64-word
// groups of a row), ch (rows staged at once) and the LDS bytes of a launch;
// ch = 0 when fewer than eight rows fit (the ordering then runs on
// order_wide_kernel).
static hipError_t bucket_shape(uint32_t max_n, uint32_t* kw, uint64_t* ch, uint32_t* lds)
{
    const uint32_t kneed = (((max_n + 31u) / 32u) + 63u) / 64u; // words a lane of a row
    *kw = kneed <= 4u ? 4u : kneed <= 6u ? 6u : 8u;
    const uint64_t fixed = 4ull * bucket_fixed_words(max_n);
    int dev = 0, lds_max = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e != hipSuccess) return e;
    const uint64_t row_bytes = 4ull * (*kw * 64u + 1u);
    const uint64_t stat = kBucketStaticLds;
    uint64_t c = ((uint64_t)lds_max > fixed + stat) ? ((uint64_t)lds_max - fixed - stat) / row_bytes : 0;
    if (c > 64) c = 64;
    *ch = c < 8 ? 0 : c;
    *lds = (uint32_t)(fixed + *ch * row_bytes);
    return hipSuccess;
}

uint32_t order_list_cap(uint32_t max_n)
{
    if (max_n <= 4096) return 0;
    uint32_t kw = 0, lds = 0;
    uint64_t ch = 0;
    if (bucket_shape(max_n, &kw, &ch, &lds) != hipSuccess || ch == 0) return 0;
    // 64 members' lists of 128 slots (2 bytes each) and the chunk
    // positions (a byte a vertex) fit in the LDS of the row kernel
    const uint64_t area = ch * 4ull * (kw * 64u + 1u);
    return area >= 64u * 256u + ((max_n + 3u) & ~3u) ? 128u : 0u;
}

hipError_t launch_order(const GraphDesc* graphs, uint32_t num_graphs, uint32_t max_n, uint64_t max_words,
                        const uint64_t* rows_in, uint32_t* order, uint16_t* nbr, uint32_t cap, uint32_t* done,
                        hipStream_t s)
{
    (void)hipGetLastError(); // report only this call's launch errors
    // rows staged in LDS when the largest graph's (n rows of rw64 words, as
    // given: a single graph's rows may be wider than ceil(n/64) words) fit in
    // a workgroup's LDS
    const uint64_t lds = max_words * 8u;
    int dev = 0, lds_max = 0;
    if (max_n <= 2048 && hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
        lds <= (uint64_t)lds_max) {
        hipError_t e = ensure_order_attr();
        if (e != hipSuccess) return e;
        if (max_n <= 512)
            hipLaunchKernelGGL(order_lds_kernel<8>, dim3(num_graphs), dim3(64), lds, s, graphs, rows_in, order);
        else if (max_n <= 1024)
            hipLaunchKernelGGL(order_lds_kernel<16>, dim3(num_graphs), dim3(64), lds, s, graphs, rows_in, order);
        else
            hipLaunchKernelGGL(order_lds_kernel<32>, dim3(num_graphs), dim3(64), lds, s, graphs, rows_in, order);
        return hipGetLastError();
    }
    if (max_n > 4096) {
        // degrees (and, with nbr, neighbour lists) over the whole device,
        // then the bucket rounds (one workgroup per graph) with as many
        // staged rows per chunk as fit
        uint32_t kw = 0, lds = 0;
        uint64_t ch = 0;
        hipError_t e = bucket_shape(max_n, &kw, &ch, &lds);
        if (e != hipSuccess) return e;
        if (ch == 0) {
            hipLaunchKernelGGL(order_wide_kernel, dim3(num_graphs), dim3(1024), 0, s, graphs, rows_in, order);
            return hipGetLastError();
        }
        if (nbr == nullptr || done == nullptr || cap == 0u || cap != order_list_cap(max_n)) {
            nbr = nullptr;
            cap = 0;
            done = nullptr;
        }
        if ((e = ensure_bucket_attr()) != hipSuccess) return e;
        hipLaunchKernelGGL(degree_kernel, dim3((max_n + 3u) / 4u, num_graphs), dim3(256), 0, s, graphs, rows_in, order,
                           nbr, cap);
        // a graph whose largest degree is at most 128 is ordered on its
        // neighbour lists (the list kernel sets done for every graph), the
        // others on the rows.  Lists of 256 slots for larger degrees were
        // measured too: 2% faster than the rows at G(10^4, 0.01), less than
        // the launch they add elsewhere.
        if (nbr != nullptr) {
            const uint32_t cp = (max_n + 3u) & ~3u, fixed = 4u * bucket_fixed_words(max_n);
            hipLaunchKernelGGL((order_bucket_kernel<4, 2>), dim3(num_graphs), dim3(1024), fixed + 64u * 256u + cp, s,
                               graphs, rows_in, order, 0u, (const uint16_t*)nbr, cap, done);
        }
        if (kw == 4)
            hipLaunchKernelGGL((order_bucket_kernel<4, 0>), dim3(num_graphs), dim3(1024), lds, s, graphs, rows_in,
                               order, (uint32_t)ch, (const uint16_t*)nullptr, 0u, done);
        else if (kw == 6)
            hipLaunchKernelGGL((order_bucket_kernel<6, 0>), dim3(num_graphs), dim3(1024), lds, s, graphs, rows_in,
                               order, (uint32_t)ch, (const uint16_t*)nullptr, 0u, done);
        else
            hipLaunchKernelGGL((order_bucket_kernel<8, 0>), dim3(num_graphs), dim3(1024), lds, s, graphs, rows_in,
                               order, (uint32_t)ch, (const uint16_t*)nullptr, 0u, done);
    } else if (max_n <= 512)
        hipLaunchKernelGGL(order_kernel<8>, dim3(num_graphs), dim3(64), 0, s, graphs, rows_in, order);
    else if (max_n <= 1024)
        hipLaunchKernelGGL(order_kernel<16>, dim3(num_graphs), dim3(64), 0, s, graphs, rows_in, order);
    else if (max_n <= 2048)
        hipLaunchKernelGGL(order_kernel<32>, dim3(num_graphs), dim3(64), 0, s, graphs, rows_in, order);
    else
        hipLaunchKernelGGL(order_kernel<64>, dim3(num_graphs), dim3(64), 0, s, graphs, rows_in, order);
    return hipGetLastError();
}

// Fill count 32-bit words with value (a kernel, not a memset node: callers may
// capture the stream).
__global__ void fill_u32_kernel(uint32_t* p, uint32_t count, uint32_t value)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = value;
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t count, uint32_t value, hipStream_t s)
{
    (void)hipGetLastError(); // report only this call's launch errors
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(fill_u32_kernel, dim3((count + 255) / 256), dim3(256), 0, s, p, count, value);
    return hipGetLastError();
}

hipError_t launch_relabel(const GraphDesc* graphs, uint32_t num_graphs, uint32_t max_n,
                          const uint64_t* rows_in, const uint32_t* order, uint32_t* adj,
                          hipStream_t s)
{
    (void)hipGetLastError(); // report only this call's launch errors
    if (max_n == 0) return hipSuccess;
    const uint32_t lds = 4u * relabel_lds_words(max_n);
    if (lds > 65536u) {
        // more than the default dynamic LDS: allowed once per process
        static std::once_flag once;
        static hipError_t err = hipSuccess;
        std::call_once(once, [] {
            err = hipFuncSetAttribute((const void*)relabel_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)(4u * relabel_lds_words(kMaxN)));
        });
        if (err != hipSuccess) return err;
    }
    hipLaunchKernelGGL(relabel_kernel, dim3((max_n + kRelabelRows - 1u) / kRelabelRows, num_graphs), dim3(256), lds,
                       s, graphs, rows_in, order, adj, max_n);
    return hipGetLastError();
}

hipError_t launch_reset(const SearchParams& sp, uint32_t num_graphs, uint64_t hist_total,
                        uint32_t workgroups, SearchParams* params_out, hipStream_t s)
{
    (void)hipGetLastError(); // report only this call's launch errors
    uint64_t work = hist_total;
    if (work < (uint64_t)workgroups * (sizeof(Mailbox) / 4)) work = (uint64_t)workgroups * (sizeof(Mailbox) / 4);
    if (work < (uint64_t)num_graphs * 8) work = (uint64_t)num_graphs * 8;
    uint32_t blocks = (uint32_t)((work + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    if (blocks == 0) blocks = 1;
    hipLaunchKernelGGL(reset_kernel, dim3(blocks), dim3(256), 0, s, sp, num_graphs, hist_total, workgroups,
                       params_out);
    return hipGetLastError();
}

hipError_t launch_root(const SearchParams& sp, uint32_t num_graphs, uint32_t max_w32,
                       uint64_t first, uint64_t last, uint32_t max_units, hipStream_t s)
{
    (void)hipGetLastError(); // report only this call's launch errors
    // writers per graph: about a unit each for a single graph (a writer
    // takes a few microseconds a unit), few per graph in a batch
    uint32_t k = 1;
    while (k < 1024 && k < max_units && (uint64_t)num_graphs * k < 4096) k <<= 1;
    switch (search_chunks(max_w32)) {
    case 1:
        hipLaunchKernelGGL(root_plan_kernel<1>, dim3(num_graphs), dim3(64), 0, s, sp, first, last, max_units);
        hipLaunchKernelGGL(root_units_kernel<1>, dim3(num_graphs, k), dim3(64), 0, s, sp, first, last);
        break;
    case 2:
        hipLaunchKernelGGL(root_plan_kernel<2>, dim3(num_graphs), dim3(64), 0, s, sp, first, last, max_units);
        hipLaunchKernelGGL(root_units_kernel<2>, dim3(num_graphs, k), dim3(64), 0, s, sp, first, last);
        break;
    case 4:
        hipLaunchKernelGGL(root_plan_kernel<4>, dim3(num_graphs), dim3(64), 0, s, sp, first, last, max_units);
        hipLaunchKernelGGL(root_units_kernel<4>, dim3(num_graphs, k), dim3(64), 0, s, sp, first, last);
        break;
    default:
        hipLaunchKernelGGL(root_plan_kernel<8>, dim3(num_graphs), dim3(64), 0, s, sp, first, last, max_units);
        hipLaunchKernelGGL(root_units_kernel<8>, dim3(num_graphs, k), dim3(64), 0, s, sp, first, last);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_subproblem(const SearchParams& sp, uint32_t max_w32, const uint32_t* bits, hipStream_t s)
{
    (void)hipGetLastError(); // report only this call's launch errors
    switch (search_chunks(max_w32)) {
    case 1: hipLaunchKernelGGL(subproblem_kernel<1>, dim3(1), dim3(64), 0, s, sp, bits); break;
    case 2: hipLaunchKernelGGL(subproblem_kernel<2>, dim3(1), dim3(64), 0, s, sp, bits); break;
    case 4: hipLaunchKernelGGL(subproblem_kernel<4>, dim3(1), dim3(64), 0, s, sp, bits); break;
    default: hipLaunchKernelGGL(subproblem_kernel<8>, dim3(1), dim3(64), 0, s, sp, bits); break;
    }
    return hipGetLastError();
}

hipError_t launch_local_plan(const GraphDesc* gparent, const uint32_t* adj, uint32_t n, uint32_t* out, hipStream_t s)
{
    (void)hipGetLastError(); // report only this call's launch errors
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(local_plan_kernel, dim3((n + 3u) / 4u), dim3(256), 0, s, gparent, adj, out);
    return hipGetLastError();
}

hipError_t launch_local_build(const GraphDesc* gparent, const uint32_t* adj, const uint32_t* order, uint32_t n,
                              const GraphDesc* lgraphs, uint32_t count, uint32_t* ladj, uint32_t* lord,
                              uint32_t* lidmap, uint32_t* lpx, hipStream_t s)
{
    (void)hipGetLastError(); // report only this call's launch errors
    if (count == 0 || n > kMaxN) return n > kMaxN ? hipErrorInvalidValue : hipSuccess;
    hipLaunchKernelGGL(local_build_kernel, dim3(count), dim3(256), 0, s, gparent, adj, order, lgraphs, ladj, lord,
                       lidmap, lpx);
    return hipGetLastError();
}

hipError_t launch_local_units(const SearchParams& sp, const uint32_t* lpx, uint32_t count, uint32_t max_w32,
                              uint64_t first, uint64_t last, hipStream_t s)
{
    (void)hipGetLastError(); // report only this call's launch errors
    if (count == 0) return hipSuccess;
    if (search_chunks(max_w32) != 1) return hipErrorInvalidValue; // local graphs have one-chunk layouts
    hipLaunchKernelGGL(local_units_kernel<1>, dim3((count + kLocalUnitsWaves - 1u) / kLocalUnitsWaves),
                       dim3(64 * kLocalUnitsWaves), 0, s, sp, lpx, count, first, last);
    return hipGetLastError();
}

typedef void (*SearchFn)(SearchParams, const SearchParams*);

template <int RULE>
static SearchFn search_fn_rule(uint32_t chunks)
{
    switch (chunks) {
    case 1: return search_kernel<1, RULE>;
    case 2: return search_kernel<2, RULE>;
    case 4: return search_kernel<4, RULE>;
    default: return search_kernel<8, RULE>;
    }
}

// The search kernel for a bitset width (chunks per lane) and a pivot rule.
static SearchFn search_fn(uint32_t max_w32, uint32_t rule)
{
    const uint32_t chunks = search_chunks(max_w32);
    switch (rule) {
    case kPivotTomita: return search_fn_rule<kPivotTomita>(chunks);
    case kPivotTX: return search_fn_rule<kPivotTX>(chunks);
    default: return search_fn_rule<kPivotGreedy>(chunks);
    }
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
        for (uint32_t w32 : {1u, 127u, 255u, kMaxN / 32u})
            for (uint32_t rule : {kPivotGreedy, kPivotTomita, kPivotTX})
                if (err == hipSuccess)
                    err = hipFuncSetAttribute((const void*)search_fn(w32, rule),
                                              hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    });
    return err;
}

hipError_t launch_search(const SearchParams& sp, const SearchParams* d_sp, uint32_t max_w32, uint32_t blocks,
                         uint32_t waves_per_block, hipStream_t s)
{
    (void)hipGetLastError(); // report only this call's launch errors
    const uint32_t lds = search_lds_bytes(sp.wave_lds_words, sp.rec_words, waves_per_block);
    hipError_t e = ensure_search_attr();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(search_fn(max_w32, sp.pivot_rule), dim3(blocks), dim3(64 * waves_per_block), lds, s, sp,
                       d_sp);
    return hipGetLastError();
}

hipError_t launch_exit_fold(const SearchParams& sp, uint32_t waves, hipStream_t s)
{
    (void)hipGetLastError(); // report only this call's launch errors
    if (waves == 0) return hipSuccess;
    hipLaunchKernelGGL(exit_fold_kernel, dim3((waves + kFoldRecs - 1u) / kFoldRecs), dim3(64), 0, s, sp, waves);
    return hipGetLastError();
}

hipError_t search_occupancy(uint32_t max_w32, uint32_t rule, uint32_t waves_per_block, uint32_t lds_bytes,
                            int* blocks_per_cu)
{
    const void* k = (const void*)search_fn(max_w32, rule);
    hipError_t e = ensure_search_attr();
    if (e != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k, (int)(64 * waves_per_block),
                                                        lds_bytes);
}

} // namespace mce
