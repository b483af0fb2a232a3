/*
 * mce_oracle.c -- plain CPU oracle for maximal clique enumeration.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this file's library.  The product
 * path (the HIP library) shares no code, header, table or helper with it.
 *
 * What is computed (San Segundo, Artieda & Strash, "Efficiently Enumerating
 * all Maximal Cliques with Bit-Parallelism"):
 *   - Sec. 2 (Preliminaries): simple undirected graph, N(v), clique, maximal
 *     clique.  The result set M(G) is unique, so brute force over all vertex
 *     subsets (orc_brute) is the plain definition written out.
 *   - Alg. 2 (Bron-Kerbosch with pivoting) with the Tomita et al. pivot
 *     (p maximises |P cap N(p)| over P cup X, Sec. 3.2): orc_tomita.
 *   - Alg. 4 (BKPivotOrdered / ChoosePivotOrdered, Sec. 4) with the
 *     maximum-degree-first ordering of Sec. 4.2 and the GreedyBB pivot rule of
 *     Sec. 4.3: orc_greedy.  This also fixes the node ("step") count, which
 *     depends on the search tree.
 *   - The same search with the other pivot rules of Sec. 4.3 and Sec. 5:
 *     GreedyBBTX (pivot from X maximising |P cap N(p)|, else the first of P;
 *     GreedyBBNX finds the same pivot with Naude's early exit, so its tree is
 *     the same) and TomitaBB (the Tomita pivot over P cup X, on the
 *     maximum-degree-first ordering): orc_solve_rule.
 *
 * Readings taken where the paper is silent or garbled (each one is listed in
 * the design notes of the repository):
 *   R1  the loop of Alg. 4 runs over every w in L = P \ N(p), in increasing
 *       position, with L fixed when the node is entered;
 *   R3  ties in the ordering go to the smaller input id;
 *   R4  positions are used as labels left to right ("first" = smallest
 *       position);
 *   R5  a node ("step") is a call with P non-empty; the root counts; a child
 *       with P' empty is resolved inline (clique if X' is empty, else a dead
 *       end);
 *   R6  L = P minus N(p); p is in L iff p is in P (zero diagonal);
 *   R8  degrees in the ordering are taken in the remaining graph;
 *   R9  the root pivots (no per-vertex top-level loop);
 *   R10 n = 0 gives the single empty clique, zero nodes.
 *
 * Data representation: an n*n byte matrix for adjacency tests and sorted
 * arrays of vertex labels for P, X, L and R.  No bitsets.
 *
 * Report fold (not in the paper; a fixed definition so results can be compared
 * exactly): every clique K is mapped to input ids, sorted ascending
 * c_1 < ... < c_k, and hashed as
 *   h = mix64(k);  h = mix64(h + 0x9E3779B97F4A7C15 + c_i) for i = 1..k,
 * where mix64 is the SplitMix64 output function (Steele, Lea & Flood, 2014).
 * count, hist[k], XOR and sum (mod 2^64) of h and omega = max k are folded.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

#define ORC_OK 0
#define ORC_E_INVAL (-1)
#define ORC_E_NOMEM (-2)
#define ORC_E_TRUNCATED (-3)
#define ORC_MAX_N 16384u

typedef struct {
    uint64_t count;     /* number of maximal cliques */
    uint64_t nodes;     /* search nodes (calls with P non-empty), R5 */
    uint64_t children;  /* vertices branched on (every v taken from some L) */
    uint64_t dead_ends; /* children with P' empty and X' non-empty */
    uint64_t hash_xor;
    uint64_t hash_sum;
    uint32_t omega;     /* size of the largest maximal clique */
    uint32_t hist_len;  /* entries available in hist */
    uint64_t *hist;     /* caller-owned; hist[k] = number of cliques of size k */
} orc_result;

/* ------------------------------------------------------------------ hash -- */

/* SplitMix64 output function: two xor-shift-multiply rounds and a final
 * xor-shift, all modulo 2^64. */
uint64_t orc_mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* Hash of one clique given as sorted input ids. */
uint64_t orc_clique_hash(const uint32_t *sorted_ids, uint32_t k)
{
    uint64_t h = orc_mix64((uint64_t)k);
    for (uint32_t i = 0; i < k; i++)
        h = orc_mix64(h + 0x9E3779B97F4A7C15ull + (uint64_t)sorted_ids[i]);
    return h;
}

/* ---------------------------------------------------------------- graph -- */

typedef struct {
    uint32_t n;
    unsigned char *adj; /* adj[u*n+v] = 1 iff {u,v} is an edge */
} graph;

/* Rows are uint64 words, least significant bit first: bit j of row i is the
 * pair {i,j}.  A simple graph needs a zero diagonal, symmetry and zero bits at
 * positions >= n.  Returns ORC_E_INVAL otherwise. */
static int graph_from_rows(graph *g, uint32_t n, const uint64_t *rows, uint32_t row_words)
{
    g->n = n;
    g->adj = NULL;
    if (n > ORC_MAX_N) return ORC_E_INVAL;
    if (n == 0) return ORC_OK;
    if (!rows) return ORC_E_INVAL;
    if ((uint64_t)row_words * 64u < n) return ORC_E_INVAL;
    g->adj = (unsigned char *)calloc((size_t)n * n, 1);
    if (!g->adj) return ORC_E_NOMEM;
    for (uint32_t i = 0; i < n; i++) {
        const uint64_t *r = rows + (size_t)i * row_words;
        for (uint32_t w = 0; w < row_words; w++) {
            uint64_t word = r[w];
            for (uint32_t b = 0; b < 64; b++) {
                if (!((word >> b) & 1u)) continue;
                uint64_t j = (uint64_t)w * 64u + b;
                if (j >= n || j == i) { free(g->adj); g->adj = NULL; return ORC_E_INVAL; }
                g->adj[(size_t)i * n + j] = 1;
            }
        }
    }
    for (uint32_t i = 0; i < n; i++)
        for (uint32_t j = i + 1; j < n; j++)
            if (g->adj[(size_t)i * n + j] != g->adj[(size_t)j * n + i]) {
                free(g->adj); g->adj = NULL; return ORC_E_INVAL;
            }
    return ORC_OK;
}

static void graph_free(graph *g) { free(g->adj); g->adj = NULL; }

static inline int is_edge(const graph *g, uint32_t u, uint32_t v)
{
    return g->adj[(size_t)u * g->n + v] != 0;
}

/* ------------------------------------------------------------- ordering -- */

/* Maximum-degree-first ordering (Sec. 4.2): v_1 has maximum degree in G,
 * v_{i+1} has maximum degree in the graph induced by the vertices not yet
 * taken.  Ties go to the smaller input id (reading R3).  order[i] is the input
 * id placed at position i. */
static void max_degree_first(const graph *g, uint32_t *order)
{
    uint32_t n = g->n;
    uint32_t *deg = (uint32_t *)malloc(sizeof(uint32_t) * (n ? n : 1));
    unsigned char *taken = (unsigned char *)calloc(n ? n : 1, 1);
    for (uint32_t v = 0; v < n; v++) {
        uint32_t d = 0;
        for (uint32_t u = 0; u < n; u++) d += is_edge(g, v, u);
        deg[v] = d;
    }
    for (uint32_t i = 0; i < n; i++) {
        uint32_t best = UINT32_MAX;
        for (uint32_t v = 0; v < n; v++) {
            if (taken[v]) continue;
            if (best == UINT32_MAX || deg[v] > deg[best]) best = v;
        }
        order[i] = best;
        taken[best] = 1;
        for (uint32_t u = 0; u < n; u++)
            if (!taken[u] && is_edge(g, best, u)) deg[u]--;
    }
    free(deg);
    free(taken);
}

int orc_order(uint32_t n, const uint64_t *rows, uint32_t row_words, uint32_t *order_out)
{
    graph g;
    int rc = graph_from_rows(&g, n, rows, row_words);
    if (rc != ORC_OK) return rc;
    if (n && !order_out) { graph_free(&g); return ORC_E_INVAL; }
    if (n) max_degree_first(&g, order_out);
    graph_free(&g);
    return ORC_OK;
}

/* ------------------------------------------------------- report folding -- */

typedef struct {
    orc_result *res;
    /* optional clique list, CSR: clique i = ids[off[i] .. off[i+1]) */
    uint32_t *ids;
    uint64_t ids_cap, ids_len;
    uint64_t *off;
    uint64_t off_cap, off_len; /* off_len counts written starts (cliques) */
    uint64_t ids_total;        /* ids of every reported clique, written or not */
    int truncated;
} sink;

static void sink_init(sink *s, orc_result *res)
{
    memset(s, 0, sizeof(*s));
    s->res = res;
}

static void result_clear(orc_result *r)
{
    r->count = r->nodes = r->children = r->dead_ends = 0;
    r->hash_xor = r->hash_sum = 0;
    r->omega = 0;
    if (r->hist) memset(r->hist, 0, sizeof(uint64_t) * r->hist_len);
}

static int cmp_u32(const void *a, const void *b)
{
    uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    return (x > y) - (x < y);
}

/* Fold one maximal clique given as input ids in any order; ids is scratch and
 * gets sorted in place. */
static void sink_report(sink *s, uint32_t *ids, uint32_t k)
{
    qsort(ids, k, sizeof(uint32_t), cmp_u32);
    uint64_t h = orc_clique_hash(ids, k);
    orc_result *r = s->res;
    r->count++;
    r->hash_xor ^= h;
    r->hash_sum += h;
    if (k > r->omega) r->omega = k;
    if (r->hist && k < r->hist_len) r->hist[k]++;
    s->ids_total += k;
    if (s->off && !s->truncated) {
        if (s->off_len + 2 > s->off_cap || s->ids_len + k > s->ids_cap) {
            s->truncated = 1;
        } else {
            s->off[s->off_len] = s->ids_len;
            memcpy(s->ids + s->ids_len, ids, sizeof(uint32_t) * k);
            s->ids_len += k;
            s->off_len++;
            s->off[s->off_len] = s->ids_len;
        }
    }
}

/* ------------------------------------------------------------ GreedyBB --- */

/* Scratch for one depth of the recursion: L, P', X' of a node.  Allocated on
 * first use of each depth, capacity n each. */
typedef struct {
    uint32_t n;
    uint32_t depth_cap;
    uint32_t **bufs; /* 3 buffers per depth */
} arena;

static int arena_init(arena *a, uint32_t n)
{
    a->n = n;
    a->depth_cap = n + 2;
    a->bufs = (uint32_t **)calloc((size_t)a->depth_cap * 3, sizeof(uint32_t *));
    return a->bufs ? ORC_OK : ORC_E_NOMEM;
}

static uint32_t *arena_get(arena *a, uint32_t depth, int which)
{
    uint32_t **slot = &a->bufs[(size_t)depth * 3 + which];
    if (!*slot) *slot = (uint32_t *)malloc(sizeof(uint32_t) * (a->n + 1));
    return *slot;
}

static void arena_free(arena *a)
{
    if (!a->bufs) return;
    for (size_t i = 0; i < (size_t)a->depth_cap * 3; i++) free(a->bufs[i]);
    free(a->bufs);
    a->bufs = NULL;
}

typedef struct {
    const graph *pg;       /* graph relabelled by position (Sec. 4.2, renumbering) */
    const uint32_t *order; /* position -> input id */
    uint32_t *R;           /* current clique, positions, in depth order */
    uint32_t depth;
    uint32_t *report_buf;  /* scratch for input ids of a reported clique */
    arena ar;
    sink *out;
    int tomita;            /* pivot rule: 0 GreedyBB, 1 Tomita, 2 GreedyBBTX */
} search;

static void report_R_plus(search *s, uint32_t v)
{
    for (uint32_t i = 0; i < s->depth; i++) s->report_buf[i] = s->order[s->R[i]];
    s->report_buf[s->depth] = s->order[v];
    sink_report(s->out, s->report_buf, s->depth + 1);
}

/* remove v from the sorted array a[0..*na) */
static void sorted_remove(uint32_t *a, uint32_t *na, uint32_t v)
{
    uint32_t i = 0;
    while (i < *na && a[i] != v) i++;
    if (i == *na) return;
    memmove(a + i, a + i + 1, sizeof(uint32_t) * (*na - i - 1));
    (*na)--;
}

/* insert v into the sorted array a[0..*na) */
static void sorted_insert(uint32_t *a, uint32_t *na, uint32_t v)
{
    uint32_t i = *na;
    while (i > 0 && a[i - 1] > v) { a[i] = a[i - 1]; i--; }
    a[i] = v;
    (*na)++;
}

/* Pivot choice.
 * GreedyBB (ChoosePivotOrdered, Alg. 4; Sec. 4.3): the first vertex of X in
 * the ordering if X is non-empty, else the first vertex of P.  P and X are
 * sorted by position, so "first" is element 0.
 * Tomita (Sec. 3.2): a vertex u of P cup X maximising |P cap N(u)|; ties go to
 * the smaller label.
 * GreedyBBTX (Sec. 4.3): if X is non-empty, a vertex u of X maximising
 * |P cap N(u)| (ties to the smaller label, as for all rules of Sec. 4.3);
 * else the first vertex of P. */
static uint32_t choose_pivot(const search *s, const uint32_t *P, uint32_t np,
                             const uint32_t *X, uint32_t nx)
{
    if (s->tomita == 0) return nx ? X[0] : P[0];
    if (s->tomita == 2 && nx == 0) return P[0];
    const graph *g = s->pg;
    uint32_t best = UINT32_MAX;
    uint32_t best_score = 0;
    for (int side = (s->tomita == 2 ? 1 : 0); side < 2; side++) {
        const uint32_t *S = side ? X : P;
        uint32_t ns = side ? nx : np;
        for (uint32_t i = 0; i < ns; i++) {
            uint32_t u = S[i], score = 0;
            for (uint32_t j = 0; j < np; j++) score += is_edge(g, u, P[j]);
            if (best == UINT32_MAX || score > best_score ||
                (score == best_score && u < best)) {
                best = u;
                best_score = score;
            }
        }
    }
    return best;
}

/* One node of the search: (R, P, X) with P non-empty; the node has already been
 * counted by its parent.  P and X are owned by the caller's scratch and are
 * updated in place (steps 12-13 of Alg. 4); X must have room for |P|+|X|. */
static void node(search *s, uint32_t *P, uint32_t np, uint32_t *X, uint32_t nx)
{
    const graph *g = s->pg;
    orc_result *r = s->out->res;
    uint32_t d = s->depth;
    uint32_t *L = arena_get(&s->ar, d, 0);
    uint32_t *P2 = arena_get(&s->ar, d, 1);
    uint32_t *X2 = arena_get(&s->ar, d, 2);

    /* step 9: pivot; step 10: L = P \ N(p), fixed at node entry (R1, R6) */
    uint32_t p = choose_pivot(s, P, np, X, nx);
    uint32_t nl = 0;
    for (uint32_t i = 0; i < np; i++)
        if (!is_edge(g, p, P[i])) L[nl++] = P[i];

    /* the branch loop: every v of L in increasing position */
    for (uint32_t li = 0; li < nl; li++) {
        uint32_t v = L[li];
        uint32_t np2 = 0, nx2 = 0;
        for (uint32_t i = 0; i < np; i++)
            if (is_edge(g, v, P[i])) P2[np2++] = P[i];
        for (uint32_t i = 0; i < nx; i++)
            if (is_edge(g, v, X[i])) X2[nx2++] = X[i];
        r->children++;
        if (np2) {
            r->nodes++;
            s->R[s->depth++] = v;
            node(s, P2, np2, X2, nx2);
            s->depth--;
        } else if (!nx2) {
            report_R_plus(s, v); /* step 6 of the child: P' and X' empty */
        } else {
            r->dead_ends++;
        }
        /* steps 12-13: P <- P \ {v}, X <- X cup {v} */
        sorted_remove(P, &np, v);
        sorted_insert(X, &nx, v);
    }
}

/* Root state and its branch set.  The root is (R = {}, P = V, X = {}); with X
 * empty its pivot is the first vertex of P.  L0 lists the root's children in
 * branch order. */
typedef struct {
    graph pg;
    uint32_t *order;
    uint32_t *L0;
    uint32_t nl0;
} prepared;

static void prepared_free(prepared *pp)
{
    graph_free(&pp->pg);
    free(pp->order);
    free(pp->L0);
}

static int prepare(prepared *pp, uint32_t n, const uint64_t *rows, uint32_t row_words, int tomita,
                   int use_given_order)
{
    memset(pp, 0, sizeof(*pp));
    graph g;
    int rc = graph_from_rows(&g, n, rows, row_words);
    if (rc != ORC_OK) return rc;
    pp->order = (uint32_t *)malloc(sizeof(uint32_t) * (n + 1));
    pp->L0 = (uint32_t *)malloc(sizeof(uint32_t) * (n + 1));
    if (!pp->order || !pp->L0) { graph_free(&g); prepared_free(pp); return ORC_E_NOMEM; }
    if (n == 0) { pp->pg = g; return ORC_OK; }
    if (use_given_order) {
        for (uint32_t i = 0; i < n; i++) pp->order[i] = i;
    } else {
        max_degree_first(&g, pp->order);
    }
    /* Renumber by position and rebuild the adjacency (Sec. 4.2). */
    pp->pg.n = n;
    pp->pg.adj = (unsigned char *)malloc((size_t)n * n);
    if (!pp->pg.adj) { graph_free(&g); prepared_free(pp); return ORC_E_NOMEM; }
    for (uint32_t i = 0; i < n; i++)
        for (uint32_t j = 0; j < n; j++)
            pp->pg.adj[(size_t)i * n + j] = g.adj[(size_t)pp->order[i] * n + pp->order[j]];
    graph_free(&g);

    /* Root pivot and L0. */
    uint32_t *P = (uint32_t *)malloc(sizeof(uint32_t) * n);
    for (uint32_t i = 0; i < n; i++) P[i] = i;
    search tmp;
    memset(&tmp, 0, sizeof(tmp));
    tmp.pg = &pp->pg;
    tmp.tomita = tomita;
    uint32_t p = choose_pivot(&tmp, P, n, NULL, 0);
    pp->nl0 = 0;
    for (uint32_t i = 0; i < n; i++)
        if (!is_edge(&pp->pg, p, i)) pp->L0[pp->nl0++] = i;
    free(P);
    return ORC_OK;
}

static int search_init(search *s, const prepared *pp, sink *out, int tomita)
{
    memset(s, 0, sizeof(*s));
    uint32_t n = pp->pg.n;
    s->pg = &pp->pg;
    s->order = pp->order;
    s->out = out;
    s->tomita = tomita;
    s->R = (uint32_t *)malloc(sizeof(uint32_t) * (n + 2));
    s->report_buf = (uint32_t *)malloc(sizeof(uint32_t) * (n + 2));
    if (!s->R || !s->report_buf) return ORC_E_NOMEM;
    return arena_init(&s->ar, n);
}

static void search_free(search *s)
{
    free(s->R);
    free(s->report_buf);
    arena_free(&s->ar);
}

/* Root child number ci (0-based, in branch order).  Its parent state is the
 * root after steps 12-13 have run for the earlier children: P = V minus
 * L0[0..ci), X = L0[0..ci). */
static void root_child(search *s, const prepared *pp, uint32_t ci, uint32_t *P, uint32_t *X)
{
    const graph *g = &pp->pg;
    orc_result *r = s->out->res;
    uint32_t n = g->n;
    uint32_t v = pp->L0[ci];
    uint32_t np = 0, nx = 0;
    /* L0 is sorted; walk V and L0 together to split into earlier / not earlier */
    uint32_t li = 0;
    for (uint32_t u = 0; u < n; u++) {
        int earlier = (li < ci && pp->L0[li] == u);
        if (earlier) li++;
        if (!is_edge(g, v, u)) continue;
        if (earlier) X[nx++] = u;
        else P[np++] = u;
    }
    r->children++;
    s->depth = 0;
    if (np) {
        r->nodes++;
        s->R[s->depth++] = v;
        node(s, P, np, X, nx);
        s->depth = 0;
    } else if (!nx) {
        report_R_plus(s, v);
    } else {
        r->dead_ends++;
    }
}

static void fold_empty_graph(sink *out)
{
    /* n = 0: the only maximal clique is the empty set (reading R10) */
    uint32_t dummy = 0;
    sink_report(out, &dummy, 0);
}

/* Solve the root's children with index in [first, last) (all of them when
 * last > |L0|).  The root node itself is counted when first == 0. */
static int solve_range(uint32_t n, const uint64_t *rows, uint32_t row_words, int tomita,
                       int use_given_order, uint64_t first, uint64_t last, sink *out)
{
    prepared pp;
    int rc = prepare(&pp, n, rows, row_words, tomita, use_given_order);
    if (rc != ORC_OK) return rc;
    if (n == 0) {
        if (first == 0 && last > 0) fold_empty_graph(out);
        prepared_free(&pp);
        return ORC_OK;
    }
    search s;
    rc = search_init(&s, &pp, out, tomita);
    uint32_t *P = (uint32_t *)malloc(sizeof(uint32_t) * (n + 1));
    uint32_t *X = (uint32_t *)malloc(sizeof(uint32_t) * (n + 1));
    if (rc != ORC_OK || !P || !X) {
        free(P); free(X); search_free(&s); prepared_free(&pp);
        return ORC_E_NOMEM;
    }
    if (first == 0 && last > 0) out->res->nodes++; /* the root: P = V is non-empty */
    if (last > pp.nl0) last = pp.nl0;
    for (uint64_t ci = first; ci < last; ci++) root_child(&s, &pp, (uint32_t)ci, P, X);
    free(P);
    free(X);
    search_free(&s);
    prepared_free(&pp);
    return ORC_OK;
}

/* ------------------------------------------------------------ public API - */

/* GreedyBB (Alg. 4 + Sec. 4.2 ordering + Sec. 4.3 GreedyBB pivot). */
int orc_greedy(uint32_t n, const uint64_t *rows, uint32_t row_words, orc_result *res)
{
    if (!res) return ORC_E_INVAL;
    result_clear(res);
    sink out;
    sink_init(&out, res);
    return solve_range(n, rows, row_words, 0, 0, 0, UINT64_MAX, &out);
}

/* GreedyBB restricted to root children [first, last). */
int orc_greedy_range(uint32_t n, const uint64_t *rows, uint32_t row_words, uint64_t first,
                     uint64_t last, orc_result *res)
{
    if (!res) return ORC_E_INVAL;
    result_clear(res);
    sink out;
    sink_init(&out, res);
    return solve_range(n, rows, row_words, 0, 0, first, last, &out);
}

/* The search of Alg. 4 on the maximum-degree-first ordering under a pivot
 * rule: 0 GreedyBB (same as orc_greedy), 1 TomitaBB, 2 GreedyBBTX. */
int orc_solve_rule(uint32_t n, const uint64_t *rows, uint32_t row_words, int rule, orc_result *res)
{
    if (!res || rule < 0 || rule > 2) return ORC_E_INVAL;
    result_clear(res);
    sink out;
    sink_init(&out, res);
    return solve_range(n, rows, row_words, rule, 0, 0, UINT64_MAX, &out);
}

/* Number of children of the GreedyBB root, |L0|. */
int orc_root_branches(uint32_t n, const uint64_t *rows, uint32_t row_words, uint64_t *out)
{
    prepared pp;
    int rc = prepare(&pp, n, rows, row_words, 0, 0);
    if (rc != ORC_OK) return rc;
    *out = pp.nl0;
    prepared_free(&pp);
    return ORC_OK;
}

/* GreedyBB with a clique list in CSR form: clique i is ids[off[i]..off[i+1]),
 * sorted ascending, in the order the search reports them.  off needs
 * count+1 entries.  Returns ORC_E_TRUNCATED (totals still valid) when a
 * buffer is too small. */
int orc_greedy_list(uint32_t n, const uint64_t *rows, uint32_t row_words, orc_result *res,
                    uint32_t *ids, uint64_t ids_cap, uint64_t *off, uint64_t off_cap,
                    uint64_t *ids_needed, uint64_t *off_needed)
{
    if (!res || !off || off_cap < 1) return ORC_E_INVAL;
    result_clear(res);
    sink out;
    sink_init(&out, res);
    out.ids = ids;
    out.ids_cap = ids ? ids_cap : 0;
    out.off = off;
    out.off_cap = off_cap;
    off[0] = 0;
    int rc = solve_range(n, rows, row_words, 0, 0, 0, UINT64_MAX, &out);
    if (rc != ORC_OK) return rc;
    if (ids_needed) *ids_needed = out.ids_total;
    if (off_needed) *off_needed = res->count + 1;
    return out.truncated ? ORC_E_TRUNCATED : ORC_OK;
}

/* Alg. 2 with the Tomita pivot, over the input labels (no reordering). */
int orc_tomita(uint32_t n, const uint64_t *rows, uint32_t row_words, orc_result *res)
{
    if (!res) return ORC_E_INVAL;
    result_clear(res);
    sink out;
    sink_init(&out, res);
    return solve_range(n, rows, row_words, 1, 1, 0, UINT64_MAX, &out);
}

/* One subproblem (R, P, X) of a graph whose labels are taken as the positions
 * of the ordering (no reordering).  R, P, X are lists of labels; P and X need
 * not be sorted.  The subproblem root is counted as a node when P is
 * non-empty.  mode 0: GreedyBB pivot, 1: Tomita pivot, 2: GreedyBBTX pivot.  ids (may be NULL: the
 * labels themselves) gives the id reported for each label: cliques are mapped
 * through it and sorted before they are hashed. */
int orc_subproblem(uint32_t n, const uint64_t *rows, uint32_t row_words, int mode, const uint32_t *ids,
                   const uint32_t *R, uint32_t nr, const uint32_t *P, uint32_t np,
                   const uint32_t *X, uint32_t nx, orc_result *res)
{
    if (!res || mode < 0 || mode > 2) return ORC_E_INVAL;
    result_clear(res);
    graph g;
    int rc = graph_from_rows(&g, n, rows, row_words);
    if (rc != ORC_OK) return rc;
    for (uint32_t i = 0; i < nr; i++) if (R[i] >= n) { graph_free(&g); return ORC_E_INVAL; }
    for (uint32_t i = 0; i < np; i++) if (P[i] >= n) { graph_free(&g); return ORC_E_INVAL; }
    for (uint32_t i = 0; i < nx; i++) if (X[i] >= n) { graph_free(&g); return ORC_E_INVAL; }
    if ((uint64_t)nr + np > n || (uint64_t)np + nx > n) { graph_free(&g); return ORC_E_INVAL; }
    prepared pp;
    memset(&pp, 0, sizeof(pp));
    pp.pg = g;
    pp.order = (uint32_t *)malloc(sizeof(uint32_t) * (n + 1));
    for (uint32_t i = 0; i < n; i++) pp.order[i] = ids ? ids[i] : i;
    sink out;
    sink_init(&out, res);
    search s;
    rc = search_init(&s, &pp, &out, mode);
    uint32_t *Pw = (uint32_t *)malloc(sizeof(uint32_t) * (n + 1));
    uint32_t *Xw = (uint32_t *)malloc(sizeof(uint32_t) * (n + 1));
    if (rc == ORC_OK && Pw && Xw) {
        uint32_t npw = 0, nxw = 0;
        for (uint32_t i = 0; i < np; i++) sorted_insert(Pw, &npw, P[i]);
        for (uint32_t i = 0; i < nx; i++) sorted_insert(Xw, &nxw, X[i]);
        for (uint32_t i = 0; i < nr; i++) s.R[i] = R[i];
        s.depth = nr;
        if (npw) {
            res->nodes++;
            node(&s, Pw, npw, Xw, nxw);
        } else if (!nxw) {
            /* R itself is maximal */
            for (uint32_t i = 0; i < nr; i++) s.report_buf[i] = pp.order[R[i]];
            sink_report(&out, s.report_buf, nr);
        }
    } else {
        rc = ORC_E_NOMEM;
    }
    free(Pw);
    free(Xw);
    search_free(&s);
    free(pp.order);
    graph_free(&g);
    return rc;
}

/* Brute force over all 2^n vertex subsets (n <= 24): the definition of a
 * maximal clique (Sec. 2) written out.  Fills count, hist, hashes and omega;
 * node counters stay zero. */
int orc_brute(uint32_t n, const uint64_t *rows, uint32_t row_words, orc_result *res)
{
    if (!res || n > 24) return ORC_E_INVAL;
    result_clear(res);
    graph g;
    int rc = graph_from_rows(&g, n, rows, row_words);
    if (rc != ORC_OK) return rc;
    sink out;
    sink_init(&out, res);
    uint32_t ids[32];
    for (uint64_t mask = 0; mask < (1ull << n); mask++) {
        int clique = 1;
        for (uint32_t u = 0; u < n && clique; u++) {
            if (!((mask >> u) & 1u)) continue;
            for (uint32_t v = u + 1; v < n; v++)
                if (((mask >> v) & 1u) && !is_edge(&g, u, v)) { clique = 0; break; }
        }
        if (!clique) continue;
        int maximal = 1;
        for (uint32_t w = 0; w < n && maximal; w++) {
            if ((mask >> w) & 1u) continue;
            int all = 1;
            for (uint32_t u = 0; u < n; u++)
                if (((mask >> u) & 1u) && !is_edge(&g, w, u)) { all = 0; break; }
            if (all) maximal = 0; /* w extends the clique */
        }
        if (!maximal) continue;
        uint32_t k = 0;
        for (uint32_t u = 0; u < n; u++) if ((mask >> u) & 1u) ids[k++] = u;
        sink_report(&out, ids, k);
    }
    graph_free(&g);
    return ORC_OK;
}

/* ------------------------------------------------------- threaded driver - */

/* GreedyBB with the root's children shared among threads.  Once the root's L0
 * is known, child ci's parent state (P = V minus L0[0..ci), X = L0[0..ci)) is
 * fixed, so the children's subtrees are independent; the totals are sums (and
 * an XOR), which do not depend on the order they are folded in. */
typedef struct {
    const prepared *pp;
    uint64_t next;
    uint64_t last;
    pthread_mutex_t mu;
    orc_result *total;
    int rc;
} mt_shared;

static void result_add(orc_result *dst, const orc_result *src)
{
    dst->count += src->count;
    dst->nodes += src->nodes;
    dst->children += src->children;
    dst->dead_ends += src->dead_ends;
    dst->hash_xor ^= src->hash_xor;
    dst->hash_sum += src->hash_sum;
    if (src->omega > dst->omega) dst->omega = src->omega;
    if (dst->hist && src->hist)
        for (uint32_t k = 0; k < dst->hist_len && k < src->hist_len; k++) dst->hist[k] += src->hist[k];
}

static void *mt_worker(void *arg)
{
    mt_shared *sh = (mt_shared *)arg;
    const prepared *pp = sh->pp;
    uint32_t n = pp->pg.n;
    orc_result local;
    memset(&local, 0, sizeof(local));
    local.hist_len = n + 2;
    local.hist = (uint64_t *)calloc(local.hist_len, sizeof(uint64_t));
    sink out;
    sink_init(&out, &local);
    search s;
    int rc = search_init(&s, pp, &out, 0);
    uint32_t *P = (uint32_t *)malloc(sizeof(uint32_t) * (n + 1));
    uint32_t *X = (uint32_t *)malloc(sizeof(uint32_t) * (n + 1));
    if (rc != ORC_OK || !local.hist || !P || !X) {
        pthread_mutex_lock(&sh->mu);
        sh->rc = ORC_E_NOMEM;
        pthread_mutex_unlock(&sh->mu);
    } else {
        for (;;) {
            uint64_t ci = __atomic_fetch_add(&sh->next, 1, __ATOMIC_RELAXED);
            if (ci >= sh->last) break;
            root_child(&s, pp, (uint32_t)ci, P, X);
        }
        pthread_mutex_lock(&sh->mu);
        result_add(sh->total, &local);
        pthread_mutex_unlock(&sh->mu);
    }
    free(P);
    free(X);
    search_free(&s);
    free(local.hist);
    return NULL;
}

int orc_greedy_range_mt(uint32_t n, const uint64_t *rows, uint32_t row_words, uint64_t first,
                        uint64_t last, int threads, orc_result *res)
{
    if (!res || threads < 1 || threads > 1024) return ORC_E_INVAL;
    result_clear(res);
    prepared pp;
    int rc = prepare(&pp, n, rows, row_words, 0, 0);
    if (rc != ORC_OK) return rc;
    if (n == 0) {
        sink out;
        sink_init(&out, res);
        if (first == 0 && last > 0) fold_empty_graph(&out);
        prepared_free(&pp);
        return ORC_OK;
    }
    if (first == 0 && last > 0) res->nodes++;
    if (last > pp.nl0) last = pp.nl0;
    mt_shared sh;
    sh.pp = &pp;
    sh.next = first;
    sh.last = last;
    sh.total = res;
    sh.rc = ORC_OK;
    pthread_mutex_init(&sh.mu, NULL);
    pthread_t *tid = (pthread_t *)malloc(sizeof(pthread_t) * threads);
    int started = 0;
    for (int t = 0; t < threads; t++) {
        if (pthread_create(&tid[t], NULL, mt_worker, &sh) != 0) break;
        started++;
    }
    if (started == 0) mt_worker(&sh);
    for (int t = 0; t < started; t++) pthread_join(tid[t], NULL);
    free(tid);
    pthread_mutex_destroy(&sh.mu);
    prepared_free(&pp);
    return sh.rc;
}

int orc_greedy_mt(uint32_t n, const uint64_t *rows, uint32_t row_words, int threads, orc_result *res)
{
    return orc_greedy_range_mt(n, rows, row_words, 0, UINT64_MAX, threads, res);
}
