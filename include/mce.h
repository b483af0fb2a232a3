/*
 * mce.h -- C ABI of the MI355X maximal clique enumeration library (libmce.so).
 *
 * The library enumerates all maximal cliques of undirected simple graphs
 * (Sec. 2 of San Segundo, Artieda & Strash, "Efficiently Enumerating all
 * Maximal Cliques with Bit-Parallelism") with the paper's GreedyBB method:
 *   - the maximum-degree-first vertex ordering and renumbering of Sec. 4.2,
 *   - Alg. 4 (BKPivotOrdered) with the GreedyBB pivot of Sec. 4.3: the first
 *     vertex of X in the ordering if X is non-empty, else the first of P,
 *   - the bitset encoding of Sec. 4.1 (P, X, L = P \ N(p) as bitstrings).
 * The search runs on one AMD Instinct MI355X (gfx950) as a persistent HIP
 * kernel, one wavefront per subproblem, with on-device work distribution.
 *
 * Graph input format (all entry points): adjacency bitset rows of uint64
 * words, least significant bit first.  Bit j of row i is set iff {i, j} is an
 * edge.  Row i of a graph with n vertices has at least ceil(n/64) words.  The
 * graph must be simple: zero diagonal, symmetric, and no bit set at a column
 * >= n.  0 <= n <= MCE_MAX_N; n = 0 is allowed and has the single maximal
 * clique {} (count 1, hist[0] = 1, no search nodes).  Graphs of more than
 * 4096 vertices (up to 16384, the sizes of the paper's Table 1 rows with
 * n = 10^4) take the same method with bitsets of up to eight 32-bit words a
 * lane; there a maximal clique whose ids fill more than 512 distinct groups
 * of 16 consecutive ids (possible only for n > 8192) does not fit the
 * per-wavefront clique buffer and the call returns MCE_E_NOMEM.
 *
 * Results (per graph): number of maximal cliques, a size histogram, the
 * number of search nodes ("steps" of the paper's tables: calls of Alg. 4 with
 * P non-empty, the root included), children examined, dead ends (children with
 * P' empty and X' non-empty), the size of the largest clique and two 64-bit
 * hashes of the clique set.  A clique K with sorted input ids c_1 < ... < c_k
 * hashes to h(K): h = mix64(k), then h = mix64(h + 0x9E3779B97F4A7C15 + c_i)
 * for i = 1..k, where mix64 is the SplitMix64 output function;
 * hash_xor = XOR of h(K) and hash_sum = sum of h(K) mod 2^64 over all K.
 *
 * Threading: every function may be called from any host thread.  Calls on
 * the same handle are serialised by the library.
 * Errors: functions return a status code (MCE_OK or a negative MCE_E_*);
 * no exception crosses the ABI.  Input validation of host buffers runs before
 * any HIP call, so invalid input is reported even on a machine without a GPU.
 */
#ifndef MCE_H
#define MCE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MCE_MAX_N 16384u

/* Status codes. */
#define MCE_OK 0
#define MCE_PENDING 1          /* mce_poll: the job has not finished yet */
#define MCE_E_INVAL (-1)       /* bad argument or non-simple graph */
#define MCE_E_NOMEM (-2)       /* device or host allocation failed, or a clique too large for the
                                  clique buffer (see above) */
#define MCE_E_TRUNCATED (-3)   /* mce_enumerate: output buffer too small */
#define MCE_E_DEVICE (-4)      /* HIP error, or no usable gfx950 device */
#define MCE_E_BUSY (-5)        /* mce_submit: admission refused */
#define MCE_E_CANCELLED (-6)   /* mce_poll: the job was cancelled */

/* mce_prepare flags. */
#define MCE_F_DEVICE_PTR 0x1u  /* rows (and nothing else) is device memory */

/* Tuning options (mce_set_option / mce_get_option).  Values apply to calls
 * made after the change; 0 restores the automatic choice where noted. */
#define MCE_OPT_WAVES_PER_BLOCK 1  /* search wavefronts per workgroup, 1..16 (0 = auto: 8, or 2 for
                                      searches on local graphs) */
#define MCE_OPT_BLOCKS 2           /* persistent search workgroups (0 = fill the device; searches
                                      on local graphs: four workgroups a CU) */
#define MCE_OPT_LDS_DEPTH 3        /* stack levels kept in LDS per wavefront, 0..64 (rest spill to HBM);
                                      with 16 wavefronts a workgroup a window of 2 levels or less
                                      is refused (the solve returns MCE_E_INVAL) */
#define MCE_OPT_SPLIT_THRESHOLD 4  /* hand over only frames whose P holds at least this many
                                      vertices (0 = auto) */
#define MCE_OPT_CHECK_INTERVAL 5   /* children a wavefront examines between two looks at its
                                      siblings and the mailbox, >= 1 (rounded up to a power of two) */
#define MCE_OPT_QUEUE_CAP 6        /* capacity of the pool of root units (power of two, 0 = auto) */
#define MCE_OPT_WATCHDOG_MS 7      /* stop a search after this many ms and fail with
                                      MCE_E_DEVICE (0 = no limit, the default) */
#define MCE_OPT_GRAPH 8            /* mce_count replays a captured hipGraph of the solve:
                                      0 never, 1 for batch handles (default), 2 always */
#define MCE_OPT_REFRESH_CHILDREN 9 /* children a busy workgroup processes between two looks
                                      at its mailbox for workgroups asking for work (0 = auto:
                                      the check interval, i.e. at every check) */
#define MCE_OPT_PIVOT 10           /* pivot rule of the search (Sec. 4.3; the maximal cliques
                                      are the same under every rule, the tree and its node
                                      count are not):
                                        0 GreedyBB (default): the first vertex of X in the
                                          ordering, else the first of P;
                                        1 TomitaBB: a vertex of P u X maximising |P n N(p)|;
                                        2 GreedyBBTX: a vertex of X maximising |P n N(p)|, else
                                          the first of P (GreedyBBNX picks the same pivot).
                                      Ties go to the earlier vertex of the ordering. */
#define MCE_OPT_LOCAL_GRAPHS 11    /* single graphs of more than 4096 vertices: 1 (default) solves
                                      each root child on the subgraph its neighbourhood induces
                                      (same search tree, bitsets of |N(v)| + 1 bits) when every
                                      root child has at most 2015 neighbours; 0 always uses
                                      bitsets over all n vertices */

typedef struct mce_graph_s *mce_graph_t; /* opaque; owns the device copy, order and rows */

typedef struct {
    uint64_t count;     /* maximal cliques */
    uint64_t nodes;     /* search nodes (calls with P non-empty, root included) */
    uint64_t children;  /* vertices branched on */
    uint64_t dead_ends; /* children with P' empty and X' non-empty */
    uint64_t hash_xor;  /* XOR of h(K) */
    uint64_t hash_sum;  /* sum of h(K) mod 2^64 */
    uint32_t omega;     /* size of the largest maximal clique */
    uint32_t hist_len;  /* in: entries available in hist (0 with hist = NULL) */
    uint64_t *hist;     /* in: caller-owned host array or NULL; out: hist[k] = cliques of size k
                           for k < hist_len */
    int32_t status;     /* MCE_OK, or the error of this graph */
    uint32_t reserved;
} mce_result_t;

typedef struct {
    uint32_t num_graphs;                /* >= 1 */
    const uint32_t *n;                  /* host array: vertex count of graph i */
    const uint64_t *row_offset_words;   /* host array: first word of graph i in rows */
} mce_batch_t;

/*
 * mce_prepare -- copy graph(s) to the device, compute the maximum-degree-first
 * ordering (Sec. 4.2: repeatedly take a vertex of largest degree in the graph
 * of the vertices not yet taken; ties go to the smaller input id), renumber
 * the vertices by position and rebuild the adjacency rows in that numbering.
 *
 *   n, rows, row_words: single graph (batch == NULL): rows holds n rows of
 *       row_words uint64 words each (row_words >= ceil(n/64)).
 *   batch: several graphs in one handle.  Graph i has batch->n[i] vertices and
 *       its rows (ceil(n_i/64) words each, packed) start at word
 *       batch->row_offset_words[i] of rows; row_words is then the total length
 *       of rows in words and n is ignored.
 *   flags: MCE_F_DEVICE_PTR if rows points to device memory (validated on the
 *       device; the call then waits for the stream).
 *   hip_stream: hipStream_t to run on, or NULL for the default stream.
 *   out: receives the handle.
 * Ownership: rows is copied and may be freed when the call returns.
 * Errors: MCE_E_INVAL for NULL pointers, n > MCE_MAX_N, short rows, a set
 * diagonal bit, an asymmetric pair, a bit at a column >= n, or an empty batch;
 * MCE_E_NOMEM; MCE_E_DEVICE.
 */
int mce_prepare(uint32_t n, const uint64_t *rows, uint32_t row_words, const mce_batch_t *batch,
                uint32_t flags, void *hip_stream, mce_graph_t *out);

/* Number of graphs in a handle. */
int mce_num_graphs(mce_graph_t g, uint32_t *num_graphs);

/* The ordering of graph `graph_index`: order[i] = input id at position i
 * (host array of at least n entries).  Waits for the prepare work. */
int mce_get_order(mce_graph_t g, uint32_t graph_index, uint32_t *order, uint32_t cap);

/* Number of children of the root of graph `graph_index` (|L| at the root: the
 * first vertex of the ordering and its non-neighbours, Alg. 4 at R = {}). */
int mce_root_branches(mce_graph_t g, uint32_t graph_index, uint64_t *out);

/*
 * mce_count -- enumerate all maximal cliques of every graph of the handle and
 * fold them into res (an array of num_graphs results; hist/hist_len are read
 * from it).  Blocks until the results are on the host.
 * Errors: MCE_E_INVAL (NULL), MCE_E_NOMEM, MCE_E_DEVICE; res[i].status is set.
 */
int mce_count(mce_graph_t g, mce_result_t *res, void *hip_stream);

/*
 * mce_count_range -- single-graph handles only: the part of the search below
 * the root's children with index in [first, last) of the root's branch order
 * (Alg. 4 at the root; the state before child i has P = V minus the earlier
 * children and X = the earlier children).  The root node is counted iff
 * first == 0.  Summing the results of disjoint ranges that cover
 * [0, mce_root_branches) gives mce_count's result (XOR for hash_xor).
 */
int mce_count_range(mce_graph_t g, uint64_t first, uint64_t last, mce_result_t *res,
                    void *hip_stream);

/*
 * mce_count_subproblem -- single-graph handles only: the search below one node
 * of Alg. 4, (R, P, X), given as lists of positions of the ordering
 * (mce_get_order: position i is input id order[i]).  R is the clique so far,
 * P the candidates, X the excluded vertices; the three lists must be disjoint
 * and P non-empty.  The node's pivot and branch set follow Alg. 4 (pivot: the
 * first vertex of X, else of P; L = P \ N(p)), the node counts as one search
 * node, and the results cover the maximal cliques R u K found below it, hashed
 * on input ids like every result.  Host arrays, copied before the call
 * returns.  Errors: MCE_E_INVAL (NULL, empty P, a position >= n, overlapping
 * lists, a batch handle), MCE_E_NOMEM, MCE_E_DEVICE.
 */
int mce_count_subproblem(mce_graph_t g, const uint32_t *R, uint32_t nr, const uint32_t *P, uint32_t np,
                         const uint32_t *X, uint32_t nx, mce_result_t *res, void *hip_stream);

/*
 * mce_enumerate -- single-graph handles only: like mce_count, and also writes
 * every maximal clique as its sorted input ids.
 *   verts: device array of verts_cap uint32; offsets: device array of
 *   offsets_cap uint64.  Clique j occupies verts[offsets[2j] .. offsets[2j+1]).
 *   The order of the cliques is unspecified.
 *   verts_needed / offsets_needed (host, may be NULL) receive the sizes a
 *   complete output needs: sum of clique sizes, and 2 * count.
 * Returns MCE_E_TRUNCATED when a buffer is too small: the totals in res are
 * still complete, but the contents of verts/offsets are then unspecified.
 */
int mce_enumerate(mce_graph_t g, uint32_t *verts, uint64_t verts_cap, uint64_t *offsets,
                  uint64_t offsets_cap, uint64_t *verts_needed, uint64_t *offsets_needed,
                  mce_result_t *res, void *hip_stream);

/*
 * mce_enumerate_stream -- single-graph handles only: every maximal clique as
 * its sorted input ids, delivered in chunks to a caller function, with device
 * and host memory bounded by the chunk size instead of the whole output.
 *
 * The root's children partition the search (each maximal clique lies in
 * exactly one child's subtree, Alg. 4), so the library enumerates ranges of
 * root children one after the other into a device buffer of chunk_verts ids
 * (offsets: 2 * chunk_verts), copies each range's output to pinned host
 * memory and calls
 *     sink(user, verts, offsets, ncliques)
 * where clique j of the chunk is verts[offsets[2j] .. offsets[2j+1]) (offsets
 * relative to this chunk's verts; host pointers valid only during the call).
 * Ranges grow and shrink with the output they produce; a range that overflows
 * the chunk is enumerated again in smaller pieces, and a single child whose
 * output alone exceeds the chunk gets a buffer of the size it needs.  The
 * order of cliques is unspecified.  A sink returning non-zero stops the
 * enumeration: MCE_E_CANCELLED, res then covers the ranges delivered so far.
 *   chunk_verts  ids per chunk (0: 1 << 24)
 *   res          totals of the whole graph (as mce_count; hist if given)
 * Errors as mce_count; MCE_E_INVAL for a batch handle or a NULL sink/res.
 */
typedef int (*mce_clique_sink_t)(void *user, const uint32_t *verts, const uint64_t *offsets,
                                 uint64_t ncliques);
int mce_enumerate_stream(mce_graph_t g, uint64_t chunk_verts, mce_clique_sink_t sink, void *user,
                         mce_result_t *res, void *hip_stream);

/*
 * Serving.  mce_submit queues a count job for a prepared single-graph handle
 * and returns at once with a ticket.  Up to four jobs run concurrently on the
 * device; a queued job is admitted when its workspace fits the HBM budget
 * (half the device memory free when serving starts) and its workgroups' LDS
 * fits what the running jobs leave.  A job that starts alone spreads over
 * every CU of the device with half of its full workgroup count, one
 * workgroup per CU (environment MCE_SERVE_ALONE_PCT, 1..100, sets another
 * share: the whole count, 100, measured slower on small graphs); one that
 * starts while others run or wait gets a quarter, cut down to the LDS left,
 * and waits while that is under an eighth of its width.
 * MCE_E_BUSY when the host queue is full.  The handle must stay alive until
 * the job has been polled (mce_release refuses it with MCE_E_BUSY before).
 */
int mce_submit(mce_graph_t g, uint32_t flags, uint64_t *ticket);

/* Wait up to timeout_us (0: do not wait, < 0: forever) for a job.  Returns
 * MCE_OK with *res filled (hist as in mce_count), MCE_PENDING, MCE_E_CANCELLED,
 * MCE_E_INVAL for an unknown ticket, or the job's error.  A ticket is
 * forgotten after it has returned anything but MCE_PENDING. */
int mce_poll(uint64_t ticket, mce_result_t *res, int32_t timeout_us);

/* Cancel a job.  A queued job is dropped; a running one stops at the
 * search's next look at its error bits (its workgroups read a word of
 * coherent host memory that this call sets), and mce_poll then returns
 * MCE_E_CANCELLED, or the results if it finished first.  MCE_E_BUSY if the
 * job has already finished, MCE_E_INVAL if the ticket is unknown. */
int mce_cancel(uint64_t ticket);

/* mce_autotune -- choose this handle's launch schedule by timing it.
 *
 * Times complete solves of the handle (mce_count) under candidate schedules
 * and keeps the fastest for later calls on the handle: first the launch shape
 * (search wavefronts per workgroup in {4, 8, 16} and workgroups per CU, each
 * with the deepest LDS stack window that fits), then the split threshold, then
 * the check interval, each around the best choice so far.  Every solve must
 * reproduce the first one's count, nodes, children, dead ends, hashes and
 * omega exactly (the schedule decides only who explores which subtree);
 * otherwise MCE_E_DEVICE.  Options set with mce_set_option still take
 * precedence over the tuned values.
 *   max_trials  candidate schedules to time at most (0: 32); each is solved twice
 *   out         optional: the kept schedule and the solve times of the
 *               automatic and kept schedules (best of two, microseconds)
 *   hip_stream  stream of the solves (NULL: default stream)
 * Thread-safe per handle (takes the handle's lock).  Not an operation of the
 * paper: a runtime aid, like the work distribution it tunes. */
typedef struct {
    uint32_t waves_per_block, blocks, lds_depth, split_threshold, check_interval;
    uint32_t trials;     /* schedules timed */
    double auto_us;      /* solve time with the automatic schedule */
    double best_us;      /* solve time with the kept schedule */
} mce_tune_t;

int mce_autotune(mce_graph_t g, uint32_t max_trials, mce_tune_t *out, void *hip_stream);

/* Forget the tuned schedule of a handle (back to the automatic one). */
int mce_clear_tuning(mce_graph_t g);

/*
 * mce_count_noalloc -- for callers that cannot allocate memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * mce_prepare + mce_count + mce_release of one graph in a single call that
 * allocates nothing.  Every intermediate (ordering, renumbered rows, pool of
 * root units, mailboxes, spill stack, totals) lives in a fixed device scratch
 * area of MCE_NOALLOC_SCRATCH_BYTES that the library holds on each device it
 * runs on until the process ends; a search whose stack outgrows the scratch
 * runs again with fewer wavefronts, and fails with MCE_E_NOMEM only if not
 * even one wavefront's stack fits.
 *   n          vertices, 0 <= n <= MCE_NOALLOC_MAX_N
 *   rows       DEVICE pointer to n rows of row_words uint64 words (format as
 *              mce_prepare); read in place, validated on the device
 *   res        as mce_count (hist/hist_len read from it, host memory)
 *   hip_stream stream to run on (NULL: default); the call waits for it
 * Results are those of mce_prepare + mce_count with the same options.  Calls
 * on one device share its scratch area and are serialised by the library
 * (the area keeps the last call's contents); two processes each have their
 * own copy.
 * Errors: MCE_E_INVAL (NULL, n > MCE_NOALLOC_MAX_N, short rows, non-simple
 * graph), MCE_E_NOMEM, MCE_E_DEVICE.
 */
#define MCE_NOALLOC_MAX_N 2048u
#define MCE_NOALLOC_SCRATCH_BYTES 50331648u /* 48 MiB */
int mce_count_noalloc(uint32_t n, const uint64_t *rows, uint32_t row_words, mce_result_t *res,
                      void *hip_stream);

/* Free the handle and its device memory.  NULL is accepted.  MCE_E_BUSY if a
 * job submitted with mce_submit for it has not finished. */
int mce_release(mce_graph_t g);

/* Static string for a status code. */
const char *mce_strerror(int code);

int mce_set_option(int key, int64_t value);
int mce_get_option(int key, int64_t *value);

/* Timings (microseconds, device clock via HIP events) of the last completed
 * mce_count / mce_count_range / mce_enumerate call of this host thread. */
typedef struct {
    double prepare_us;     /* ordering + renumbering of the handle */
    double search_us;      /* root + persistent search + result copy-out */
    double search_kernel_us; /* the persistent search kernel alone */
    uint32_t blocks;       /* workgroups of the search launch */
    uint32_t waves_per_block;
    uint32_t lds_depth;
    uint32_t lds_bytes_per_block;
    uint64_t donations;    /* units handed to the queue by busy wavefronts */
    uint64_t units;        /* units processed */
    uint64_t spills;       /* stack levels written beyond the LDS window */
    uint64_t checks;       /* times the search loop stopped to look at siblings and mailboxes */
    uint64_t flushes;      /* times it stopped to hash a full clique buffer */
    uint32_t attempts;     /* launches of the last call (a rerun follows an exhausted spill pool) */
    uint32_t local_graphs; /* local graphs the search ran on (0: the whole graph's bitsets) */
    double busy_frac;      /* share of the search kernel's wavefront time spent on units */
    double ramp_frac;      /* share spent before a wavefront's first unit */
    double tail_frac;      /* share spent after its last unit (the rest of the idle time is
                              spent between units, looking for work) */
} mce_stats_t;

int mce_last_stats(mce_stats_t *out);

#ifdef __cplusplus
}
#endif

#endif /* MCE_H */
