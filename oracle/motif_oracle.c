/*
 * motif_oracle.c -- reference implementation of higher-order motif counting.
 *
 * TEST INFRASTRUCTURE ONLY.  Plain, slow C written from the paper's
 * definitions and algorithms; only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg load it.  It shares no code with the HIP
 * library.
 *
 * Inputs are already normalised by the Python side (oracle/core.py): for each
 * size j in 2..k a flat array of unique hyperedges, each an ascending j-tuple
 * of node ids.  Hyperedges of other sizes cannot lie inside a k-node set
 * (Definition of the vertex-induced sub-hypergraph, Section 3) and are not
 * passed.
 *
 * Contents
 *   - tuple sets: the hyperedge hash set of Section 4.3 (Fig. 3b) and the
 *     "visited" set of Algorithms 2 and 3
 *   - fill-in of a node set and its isomorphism class (Section 4.3)
 *   - ESU (Wernicke 2006), used by Algorithms 2 and 3 on the pairwise graph
 *     and by Algorithm 1 on the clique projection
 *   - Algorithm 2 (order 3) and Algorithm 3 (order 4), exact, on one thread
 *     and spread over host threads
 *   - Algorithm 1 (the baseline of Section 4.1), exact
 *   - Algorithm 4, sampled, on an explicit list of sampled hyperedges
 */
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NONE 0xFFFFFFFFu

/* ------------------------------------------------------------------ */
/* Sets of node tuples (ascending ids, unused slots NONE).             */
/* ------------------------------------------------------------------ */
typedef struct { uint32_t v[4]; } tup;

typedef struct {
    tup *key;
    unsigned char *full;
    size_t cap, n;
} tupset;

static uint64_t mix64(uint64_t x)
{
    x ^= x >> 33; x *= 0xff51afd7ed558ccdULL;
    x ^= x >> 33; x *= 0xc4ceb9fe1a85ec53ULL;
    x ^= x >> 33;
    return x;
}

static uint64_t tup_hash(const tup *t)
{
    uint64_t h = 0x243f6a8885a308d3ULL;
    for (int i = 0; i < 4; i++) h = mix64(h ^ ((uint64_t)t->v[i] + 0x9e3779b97f4a7c15ULL * (uint64_t)(i + 1)));
    return h;
}

static int tup_eq(const tup *a, const tup *b)
{
    return a->v[0] == b->v[0] && a->v[1] == b->v[1] && a->v[2] == b->v[2] && a->v[3] == b->v[3];
}

static int tupset_init(tupset *s, size_t expect)
{
    size_t cap = 16;
    while (cap < 2 * expect + 16) cap <<= 1;
    s->key = (tup *)malloc(cap * sizeof(tup));
    s->full = (unsigned char *)calloc(cap, 1);
    s->cap = cap;
    s->n = 0;
    return (s->key && s->full) ? 0 : -1;
}

static void tupset_free(tupset *s)
{
    free(s->key);
    free(s->full);
    s->key = NULL; s->full = NULL; s->cap = s->n = 0;
}

static int tupset_has(const tupset *s, const tup *t)
{
    size_t mask = s->cap - 1, i = (size_t)tup_hash(t) & mask;
    while (s->full[i]) {
        if (tup_eq(&s->key[i], t)) return 1;
        i = (i + 1) & mask;
    }
    return 0;
}

static int tupset_add(tupset *s, const tup *t);

static int tupset_grow(tupset *s)
{
    tupset bigger;
    if (tupset_init(&bigger, s->cap) != 0) return -1;
    for (size_t i = 0; i < s->cap; i++)
        if (s->full[i] && tupset_add(&bigger, &s->key[i]) < 0) return -1;
    tupset_free(s);
    *s = bigger;
    return 0;
}

/* 1 if added, 0 if already present, -1 on allocation failure */
static int tupset_add(tupset *s, const tup *t)
{
    if (2 * (s->n + 1) > s->cap && tupset_grow(s) != 0) return -1;
    size_t mask = s->cap - 1, i = (size_t)tup_hash(t) & mask;
    while (s->full[i]) {
        if (tup_eq(&s->key[i], t)) return 0;
        i = (i + 1) & mask;
    }
    s->full[i] = 1;
    s->key[i] = *t;
    s->n++;
    return 1;
}

static tup make_tup(const uint32_t *nodes, int n)
{
    tup t;
    for (int i = 0; i < 4; i++) t.v[i] = i < n ? nodes[i] : NONE;
    for (int i = 1; i < n; i++) {                      /* insertion sort, n <= 4 */
        uint32_t x = t.v[i];
        int j = i - 1;
        while (j >= 0 && t.v[j] > x) { t.v[j + 1] = t.v[j]; j--; }
        t.v[j + 1] = x;
    }
    return t;
}

/* ------------------------------------------------------------------ */
/* Patterns and isomorphism classes (Section 4.3, Fig. 3a).            */
/* Local positions 0..k-1 follow ascending node id; pattern bit i is    */
/* the i-th subset of {0..k-1} of size >= 2 in ascending mask order.    */
/* ------------------------------------------------------------------ */
static int n_sub[5];
static int sub_mask[5][11];
static int n_class[5];
static uint32_t class_canon[5][256];
static int tables_ready = 0;

static int popcount(unsigned x) { int c = 0; while (x) { c += x & 1; x >>= 1; } return c; }

static int pattern_connected(uint32_t p, int k)
{
    int parent[4];
    unsigned covered = 0;
    for (int i = 0; i < k; i++) parent[i] = i;
    for (int b = 0; b < n_sub[k]; b++) {
        if (!((p >> b) & 1)) continue;
        int m = sub_mask[k][b], first = -1;
        covered |= (unsigned)m;
        for (int i = 0; i < k; i++) {
            if (!((m >> i) & 1)) continue;
            if (first < 0) { first = i; continue; }
            int a = first, c = i;
            while (parent[a] != a) a = parent[a];
            while (parent[c] != c) c = parent[c];
            if (a != c) parent[a] = c;
        }
    }
    if (covered != (1u << k) - 1) return 0;
    int root = 0;
    while (parent[root] != root) root = parent[root];
    for (int i = 1; i < k; i++) {
        int r = i;
        while (parent[r] != r) r = parent[r];
        if (r != root) return 0;
    }
    return 1;
}

static uint32_t pattern_relabel(uint32_t p, const int *perm, int k)
{
    uint32_t out = 0;
    for (int b = 0; b < n_sub[k]; b++) {
        if (!((p >> b) & 1)) continue;
        int m = sub_mask[k][b], img = 0;
        for (int i = 0; i < k; i++)
            if ((m >> i) & 1) img |= 1 << perm[i];
        for (int c = 0; c < n_sub[k]; c++)
            if (sub_mask[k][c] == img) { out |= 1u << c; break; }
    }
    return out;
}

/* smallest pattern value over all k! relabellings */
static uint32_t pattern_canonical(uint32_t p, int k)
{
    uint32_t best = 0xFFFFFFFFu;
    int perm[4];
    for (int a = 0; a < k; a++)
        for (int b = 0; b < k; b++)
            for (int c = 0; c < k; c++)
                for (int d = 0; d < (k == 4 ? k : 1); d++) {
                    perm[0] = a; perm[1] = b; perm[2] = c; perm[3] = d;
                    int seen = 0, ok = 1;
                    for (int i = 0; i < k; i++) {
                        if (seen & (1 << perm[i])) ok = 0;
                        seen |= 1 << perm[i];
                    }
                    if (!ok) continue;
                    uint32_t q = pattern_relabel(p, perm, k);
                    if (q < best) best = q;
                }
    return best;
}

static int cmp_u32(const void *a, const void *b)
{
    uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    return (x > y) - (x < y);
}

/* pattern -> class id for every labelled pattern, -1 when not connected:
 * the hash map of Section 4.3 (Fig. 3a), built by relabelling every class's
 * canonical pattern under all k! permutations */
static int16_t pattern_to_class[5][2048];

static void build_tables(void)
{
    if (tables_ready) return;
    for (int k = 3; k <= 4; k++) {
        n_sub[k] = 0;
        for (int m = 0; m < (1 << k); m++)
            if (popcount((unsigned)m) >= 2) sub_mask[k][n_sub[k]++] = m;
        int nc = 0;
        for (uint32_t p = 0; p < (1u << n_sub[k]); p++) {
            if (!pattern_connected(p, k)) continue;
            uint32_t c = pattern_canonical(p, k);
            int dup = 0;
            for (int i = 0; i < nc; i++)
                if (class_canon[k][i] == c) { dup = 1; break; }
            if (!dup) class_canon[k][nc++] = c;
        }
        qsort(class_canon[k], (size_t)nc, sizeof(uint32_t), cmp_u32);
        n_class[k] = nc;
        for (uint32_t p = 0; p < (1u << n_sub[k]); p++) pattern_to_class[k][p] = -1;
        int perm[4];
        for (int cls = 0; cls < nc; cls++)
            for (int a = 0; a < k; a++)
                for (int b = 0; b < k; b++)
                    for (int c = 0; c < k; c++)
                        for (int d = 0; d < (k == 4 ? k : 1); d++) {
                            perm[0] = a; perm[1] = b; perm[2] = c; perm[3] = d;
                            int seen = 0, ok = 1;
                            for (int i = 0; i < k; i++) {
                                if (seen & (1 << perm[i])) ok = 0;
                                seen |= 1 << perm[i];
                            }
                            if (ok) pattern_to_class[k][pattern_relabel(class_canon[k][cls], perm, k)] = (int16_t)cls;
                        }
    }
    tables_ready = 1;
}

/* class id of a pattern, -1 when it is not connected */
static int pattern_class(uint32_t p, int k)
{
    return pattern_to_class[k][p];
}

static int pattern_maxcard(uint32_t p, int k)
{
    int mc = 0;
    for (int b = 0; b < n_sub[k]; b++)
        if ((p >> b) & 1) { int s = popcount((unsigned)sub_mask[k][b]); if (s > mc) mc = s; }
    return mc;
}

/* ------------------------------------------------------------------ */
/* Hypergraph view.                                                    */
/* ------------------------------------------------------------------ */
typedef struct {
    int k;
    uint32_t n_nodes;
    const uint32_t *e[5];   /* e[j]: ne[j] ascending j-tuples */
    int64_t ne[5];
    tupset edges;           /* every hyperedge of size 2..k */
    int64_t *inc_off;       /* node -> incident hyperedges (size 2..k) */
    int32_t *inc_size;
    int64_t *inc_idx;
    int64_t *g2_off;        /* pairwise graph: node -> ascending neighbours */
    uint32_t *g2_adj;
} hgraph;

static void hgraph_free(hgraph *g)
{
    tupset_free(&g->edges);
    free(g->inc_off); free(g->inc_size); free(g->inc_idx);
    free(g->g2_off); free(g->g2_adj);
}

static int hgraph_build(hgraph *g, int k, uint32_t n_nodes,
                        const uint32_t *e2, int64_t n2, const uint32_t *e3, int64_t n3,
                        const uint32_t *e4, int64_t n4)
{
    memset(g, 0, sizeof(*g));
    g->k = k;
    g->n_nodes = n_nodes;
    g->e[2] = e2; g->ne[2] = n2;
    g->e[3] = e3; g->ne[3] = n3;
    g->e[4] = e4; g->ne[4] = (k == 4) ? n4 : 0;
    if (tupset_init(&g->edges, (size_t)(n2 + n3 + g->ne[4])) != 0) return -1;
    int64_t total_inc = 0;
    for (int j = 2; j <= k; j++) {
        for (int64_t i = 0; i < g->ne[j]; i++) {
            tup t = make_tup(g->e[j] + (size_t)i * j, j);
            if (tupset_add(&g->edges, &t) < 0) return -1;
        }
        total_inc += g->ne[j] * j;
    }
    g->inc_off = (int64_t *)calloc((size_t)n_nodes + 1, sizeof(int64_t));
    g->inc_size = (int32_t *)malloc((size_t)(total_inc + 1) * sizeof(int32_t));
    g->inc_idx = (int64_t *)malloc((size_t)(total_inc + 1) * sizeof(int64_t));
    g->g2_off = (int64_t *)calloc((size_t)n_nodes + 1, sizeof(int64_t));
    g->g2_adj = (uint32_t *)malloc((size_t)(2 * n2 + 1) * sizeof(uint32_t));
    if (!g->inc_off || !g->inc_size || !g->inc_idx || !g->g2_off || !g->g2_adj) return -1;
    for (int j = 2; j <= k; j++)
        for (int64_t i = 0; i < g->ne[j] * j; i++) g->inc_off[g->e[j][i] + 1]++;
    for (uint32_t v = 0; v < n_nodes; v++) g->inc_off[v + 1] += g->inc_off[v];
    int64_t *fill = (int64_t *)malloc(((size_t)n_nodes + 1) * sizeof(int64_t));
    if (!fill) return -1;
    memcpy(fill, g->inc_off, ((size_t)n_nodes + 1) * sizeof(int64_t));
    for (int j = 2; j <= k; j++)
        for (int64_t i = 0; i < g->ne[j]; i++)
            for (int m = 0; m < j; m++) {
                uint32_t v = g->e[j][i * j + m];
                g->inc_size[fill[v]] = j;
                g->inc_idx[fill[v]] = i;
                fill[v]++;
            }
    for (int64_t i = 0; i < n2; i++) { g->g2_off[e2[2 * i] + 1]++; g->g2_off[e2[2 * i + 1] + 1]++; }
    for (uint32_t v = 0; v < n_nodes; v++) g->g2_off[v + 1] += g->g2_off[v];
    memcpy(fill, g->g2_off, ((size_t)n_nodes + 1) * sizeof(int64_t));
    for (int64_t i = 0; i < n2; i++) {
        uint32_t a = e2[2 * i], b = e2[2 * i + 1];
        g->g2_adj[fill[a]++] = b;
        g->g2_adj[fill[b]++] = a;
    }
    free(fill);
    for (uint32_t v = 0; v < n_nodes; v++)
        qsort(g->g2_adj + g->g2_off[v], (size_t)(g->g2_off[v + 1] - g->g2_off[v]), sizeof(uint32_t), cmp_u32);
    return 0;
}

/* fill-in (Section 4.3, Fig. 3b): test every subset of size >= 2 of the
 * ascending node set V against the hyperedge set */
static uint32_t fill_in(const hgraph *g, const uint32_t *V, int k)
{
    uint32_t p = 0;
    for (int b = 0; b < n_sub[k]; b++) {
        uint32_t nodes[4];
        int n = 0;
        for (int i = 0; i < k; i++)
            if ((sub_mask[k][b] >> i) & 1) nodes[n++] = V[i];
        tup t = make_tup(nodes, n);
        if (tupset_has(&g->edges, &t)) p |= 1u << b;
    }
    return p;
}

/* b in the ascending neighbour row of a (graph given as off/adj) */
static int row_adjacent(const int64_t *off, const uint32_t *adj, uint32_t a, uint32_t b)
{
    const uint32_t *row = adj + off[a];
    size_t n = (size_t)(off[a + 1] - off[a]);
    return bsearch(&b, row, n, sizeof(uint32_t), cmp_u32) != NULL;
}

static void sort_nodes(uint32_t *V, int n)
{
    for (int i = 1; i < n; i++) {
        uint32_t x = V[i];
        int j = i - 1;
        while (j >= 0 && V[j] > x) { V[j + 1] = V[j]; j--; }
        V[j + 1] = x;
    }
}

/* ------------------------------------------------------------------ */
/* ESU (Wernicke 2006) on a graph given as ascending neighbour rows:   */
/* each connected k-node set is produced exactly once, from its        */
/* smallest node.                                                      */
/* ------------------------------------------------------------------ */
typedef struct {
    const int64_t *off;
    const uint32_t *adj;
    int k;
    void (*emit)(void *ctx, const uint32_t *V);
    void *ctx;
    int failed;
} esu_ctx;

static void esu_extend(esu_ctx *c, uint32_t *Vsub, int nsub, const uint32_t *Vext, int64_t next, uint32_t root)
{
    if (nsub == c->k) {
        uint32_t V[4];
        memcpy(V, Vsub, sizeof(uint32_t) * (size_t)c->k);
        sort_nodes(V, c->k);
        c->emit(c->ctx, V);
        return;
    }
    uint32_t *ext = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(next + 1));
    if (!ext) { c->failed = 1; return; }
    memcpy(ext, Vext, sizeof(uint32_t) * (size_t)next);
    while (next > 0) {
        uint32_t w = ext[--next];
        if (nsub + 1 == c->k) {            /* the extended set is complete: its
                                              extension set would never be read */
            Vsub[nsub] = w;
            esu_extend(c, Vsub, nsub + 1, ext, 0, root);
            continue;
        }
        int64_t deg = c->off[w + 1] - c->off[w];
        uint32_t *ext2 = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(next + deg + 1));
        if (!ext2) { c->failed = 1; break; }
        memcpy(ext2, ext, sizeof(uint32_t) * (size_t)next);
        int64_t n2 = next;
        /* exclusive neighbours of w: not in Vsub and not adjacent to Vsub */
        for (int64_t i = 0; i < deg; i++) {
            uint32_t u = c->adj[c->off[w] + i];
            if (u <= root) continue;
            int excl = 1;
            for (int s = 0; s < nsub && excl; s++)
                if (Vsub[s] == u || row_adjacent(c->off, c->adj, Vsub[s], u)) excl = 0;
            if (excl) ext2[n2++] = u;
        }
        Vsub[nsub] = w;
        esu_extend(c, Vsub, nsub + 1, ext2, n2, root);
        free(ext2);
    }
    free(ext);
}

/* the sets whose smallest node is v */
static void esu_root(esu_ctx *c, uint32_t v)
{
    int64_t deg = c->off[v + 1] - c->off[v];
    uint32_t *ext = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(deg + 1));
    if (!ext) { c->failed = 1; return; }
    int64_t n = 0;
    for (int64_t i = 0; i < deg; i++) {
        uint32_t u = c->adj[c->off[v] + i];
        if (u > v) ext[n++] = u;
    }
    uint32_t Vsub[4] = { v, 0, 0, 0 };
    esu_extend(c, Vsub, 1, ext, n, v);
    free(ext);
}

static void esu(const int64_t *off, const uint32_t *adj, uint32_t n_nodes, int k,
                void (*emit)(void *, const uint32_t *), void *ctx, int *failed)
{
    esu_ctx c = { off, adj, k, emit, ctx, 0 };
    for (uint32_t v = 0; v < n_nodes && !c.failed; v++) esu_root(&c, v);
    *failed = c.failed;
}

/* ------------------------------------------------------------------ */
/* Algorithms 2 and 3: exact counts.                                   */
/* ------------------------------------------------------------------ */
typedef struct {
    const hgraph *g;
    int k;
    tupset *visited;
    int64_t *M;
    int failed;
} exact_ctx;

static void exact_emit_unvisited(void *p, const uint32_t *V)
{
    exact_ctx *c = (exact_ctx *)p;
    tup t = make_tup(V, c->k);
    if (tupset_has(c->visited, &t)) return;
    int cls = pattern_class(fill_in(c->g, V, c->k), c->k);
    if (cls < 0) { c->failed = 1; return; }      /* an ESU output is connected */
    c->M[cls]++;
    if (tupset_add(c->visited, &t) < 0) c->failed = 1;
}

/* Count every order-k motif of the normalised hypergraph (k = 3 or 4).
 * Returns 0 on success, -1 on bad arguments or allocation failure. */
int oracle_count_exact(int k, uint32_t n_nodes,
                       const uint32_t *e2, int64_t n2, const uint32_t *e3, int64_t n3,
                       const uint32_t *e4, int64_t n4, int64_t *counts)
{
    if (k != 3 && k != 4) return -1;
    build_tables();
    hgraph g;
    if (hgraph_build(&g, k, n_nodes, e2, n2, e3, n3, e4, n4) != 0) { hgraph_free(&g); return -1; }
    tupset visited;
    if (tupset_init(&visited, 1024) != 0) { hgraph_free(&g); return -1; }
    int64_t M[256];
    memset(M, 0, sizeof(M));
    int failed = 0;

    if (k == 4) {
        /* step 1: every 4-node hyperedge is an occurrence; its node set is visited */
        for (int64_t i = 0; i < g.ne[4] && !failed; i++) {
            const uint32_t *V = g.e[4] + 4 * i;
            int cls = pattern_class(fill_in(&g, V, 4), 4);
            if (cls < 0) { failed = 1; break; }
            M[cls]++;
            tup t = make_tup(V, 4);
            if (tupset_add(&visited, &t) < 0) failed = 1;
        }
        /* step 2: every 3-node hyperedge e with every adjacent hyperedge f
         * (size 2 or 3, sharing a node) such that |e u f| = 4 */
        for (int64_t i = 0; i < g.ne[3] && !failed; i++) {
            const uint32_t *e = g.e[3] + 3 * i;
            for (int m = 0; m < 3 && !failed; m++) {
                uint32_t u = e[m];
                for (int64_t x = g.inc_off[u]; x < g.inc_off[u + 1] && !failed; x++) {
                    int fs = g.inc_size[x];
                    if (fs > 3) continue;
                    const uint32_t *f = g.e[fs] + (size_t)g.inc_idx[x] * fs;
                    uint32_t U[7];
                    int nu = 0;
                    for (int a = 0; a < 3; a++) U[nu++] = e[a];
                    for (int a = 0; a < fs; a++) {
                        int in = 0;
                        for (int b = 0; b < 3; b++) if (e[b] == f[a]) in = 1;
                        if (!in) U[nu++] = f[a];
                    }
                    if (nu != 4) continue;
                    sort_nodes(U, 4);
                    tup t = make_tup(U, 4);
                    if (tupset_has(&visited, &t)) continue;
                    int cls = pattern_class(fill_in(&g, U, 4), 4);
                    if (cls < 0) { failed = 1; break; }
                    M[cls]++;
                    if (tupset_add(&visited, &t) < 0) failed = 1;
                }
            }
        }
    } else {
        /* order 3, step 1: every 3-node hyperedge; its triple is visited */
        for (int64_t i = 0; i < g.ne[3] && !failed; i++) {
            const uint32_t *V = g.e[3] + 3 * i;
            int cls = pattern_class(fill_in(&g, V, 3), 3);
            if (cls < 0) { failed = 1; break; }
            M[cls]++;
            tup t = make_tup(V, 3);
            if (tupset_add(&visited, &t) < 0) failed = 1;
        }
    }
    /* last step: ESU on the pairwise graph; sets not visited are new occurrences */
    if (!failed) {
        exact_ctx c = { &g, k, &visited, M, 0 };
        int esu_failed = 0;
        esu(g.g2_off, g.g2_adj, g.n_nodes, k, exact_emit_unvisited, &c, &esu_failed);
        failed = c.failed || esu_failed;
    }
    tupset_free(&visited);
    hgraph_free(&g);
    if (failed) return -1;
    memcpy(counts, M, sizeof(int64_t) * (size_t)n_class[k]);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Algorithms 2 and 3 on several host threads (OpenMP).                */
/* The same three steps in the same order, each spread over threads;   */
/* `visited` is a set of node sets, so which thread inserts a set      */
/* first does not change which sets are counted: a set is counted by   */
/* the one insertion that finds it absent (steps 1 and 2), and step 3  */
/* only reads the set, which ESU's one-emission-per-set allows.  The   */
/* counts equal the single-thread routine's (tests check it).          */
/* ------------------------------------------------------------------ */
#define N_SHARDS 256

typedef struct {
    tupset s[N_SHARDS];
    omp_lock_t lock[N_SHARDS];
} shardset;

static int shard_of(const tup *t) { return (int)(tup_hash(t) >> 56) & (N_SHARDS - 1); }

/* 1 if added, 0 if present, -1 on allocation failure */
static int shard_add(shardset *ss, const tup *t)
{
    int h = shard_of(t);
    omp_set_lock(&ss->lock[h]);
    int r = tupset_add(&ss->s[h], t);
    omp_unset_lock(&ss->lock[h]);
    return r;
}

typedef struct {
    const hgraph *g;
    int k;
    shardset *visited;
    int64_t *M;
    int failed;
} mt_ctx;

static void mt_emit_unvisited(void *p, const uint32_t *V)
{
    mt_ctx *c = (mt_ctx *)p;
    tup t = make_tup(V, c->k);
    const tupset *s = &c->visited->s[shard_of(&t)];
    if (tupset_has(s, &t)) return;
    int cls = pattern_class(fill_in(c->g, V, c->k), c->k);
    if (cls < 0) { c->failed = 1; return; }
    c->M[cls]++;
}

/* oracle_count_exact on up to n_threads threads (0: all the host's).
 * Returns the number of threads used, or -1 on bad arguments or allocation
 * failure. */
int oracle_count_exact_threads(int k, uint32_t n_nodes,
                               const uint32_t *e2, int64_t n2, const uint32_t *e3, int64_t n3,
                               const uint32_t *e4, int64_t n4, int n_threads, int64_t *counts)
{
    if (k != 3 && k != 4) return -1;
    build_tables();
    if (n_threads <= 0) n_threads = omp_get_num_procs();
    hgraph g;
    if (hgraph_build(&g, k, n_nodes, e2, n2, e3, n3, e4, n4) != 0) { hgraph_free(&g); return -1; }
    shardset *vis = (shardset *)calloc(1, sizeof(shardset));
    int failed = !vis;
    for (int h = 0; h < N_SHARDS && !failed; h++) {
        if (tupset_init(&vis->s[h], 64) != 0) failed = 1;
        omp_init_lock(&vis->lock[h]);
    }
    int64_t M[256];
    memset(M, 0, sizeof(M));
    int used = 1;
    if (!failed) {
        #pragma omp parallel num_threads(n_threads)
        {
            int64_t Mt[256];
            memset(Mt, 0, sizeof(Mt));
            int bad = 0;
            #pragma omp single
            used = omp_get_num_threads();
            /* step 1: the k-node hyperedges; their node sets are visited */
            const int64_t n_top = g.ne[k];
            #pragma omp for schedule(dynamic, 256)
            for (int64_t i = 0; i < n_top; i++) {
                const uint32_t *V = g.e[k] + (size_t)k * i;
                int cls = pattern_class(fill_in(&g, V, k), k);
                if (cls < 0) { bad = 1; continue; }
                Mt[cls]++;
                tup t = make_tup(V, k);
                if (shard_add(vis, &t) < 0) bad = 1;
            }
            /* (implicit barrier) step 2 at order 4: 3-node hyperedges with
             * every adjacent hyperedge of size 2 or 3 adding one node */
            if (k == 4) {
                #pragma omp for schedule(dynamic, 64)
                for (int64_t i = 0; i < g.ne[3]; i++) {
                    const uint32_t *e = g.e[3] + 3 * i;
                    for (int m = 0; m < 3; m++) {
                        uint32_t u = e[m];
                        for (int64_t x = g.inc_off[u]; x < g.inc_off[u + 1]; x++) {
                            int fs = g.inc_size[x];
                            if (fs > 3) continue;
                            const uint32_t *f = g.e[fs] + (size_t)g.inc_idx[x] * fs;
                            uint32_t U[7];
                            int nu = 0;
                            for (int a = 0; a < 3; a++) U[nu++] = e[a];
                            for (int a = 0; a < fs; a++) {
                                int in = 0;
                                for (int b = 0; b < 3; b++) if (e[b] == f[a]) in = 1;
                                if (!in) U[nu++] = f[a];
                            }
                            if (nu != 4) continue;
                            sort_nodes(U, 4);
                            tup t = make_tup(U, 4);
                            int r = shard_add(vis, &t);
                            if (r < 0) { bad = 1; continue; }
                            if (r == 0) continue;
                            int cls = pattern_class(fill_in(&g, U, 4), 4);
                            if (cls < 0) { bad = 1; continue; }
                            Mt[cls]++;
                        }
                    }
                }
            }
            /* last step: ESU on the pairwise graph, roots spread over threads */
            mt_ctx c = { &g, k, vis, Mt, 0 };
            esu_ctx ec = { g.g2_off, g.g2_adj, k, mt_emit_unvisited, &c, 0 };
            #pragma omp for schedule(dynamic, 1)
            for (int64_t v = 0; v < (int64_t)g.n_nodes; v++) esu_root(&ec, (uint32_t)v);
            if (c.failed || ec.failed) bad = 1;
            #pragma omp critical
            {
                for (int i = 0; i < 256; i++) M[i] += Mt[i];
                if (bad) failed = 1;
            }
        }
    }
    if (vis) {
        for (int h = 0; h < N_SHARDS; h++) { tupset_free(&vis->s[h]); omp_destroy_lock(&vis->lock[h]); }
        free(vis);
    }
    hgraph_free(&g);
    if (failed) return -1;
    memcpy(counts, M, sizeof(int64_t) * (size_t)n_class[k]);
    return used;
}

/* ------------------------------------------------------------------ */
/* Algorithm 1: the baseline of Section 4.1.                           */
/* ------------------------------------------------------------------ */
typedef struct {
    const hgraph *g;
    int k;
    int64_t *M;
    int64_t candidates, discarded;
} base_ctx;

/* a connected k-node set of the projection: count it when the
 * sub-hypergraph it induces is connected, else discard it */
static void base_emit(void *p, const uint32_t *V)
{
    base_ctx *c = (base_ctx *)p;
    c->candidates++;
    int cls = pattern_class(fill_in(c->g, V, c->k), c->k);
    if (cls < 0) { c->discarded++; return; }
    c->M[cls]++;
}

/* Count every order-k motif (k = 3 or 4) the way the baseline does: build the
 * projection G of the hypergraph (every hyperedge of size >= 2, whatever its
 * size, replaced by a clique), enumerate the connected k-node sets of G with
 * ESU, and keep those whose induced sub-hypergraph is connected.  members /
 * offsets hold every unique hyperedge of size >= 2 (n_all of them); e2..e4 the
 * unique hyperedges of sizes 2..k, for fill-in.  stats[0] receives the number
 * of candidates ESU produced, stats[1] the number discarded.  Returns 0 on
 * success, -1 on bad arguments or allocation failure. */
int oracle_count_baseline(int k, uint32_t n_nodes, const uint32_t *members, const int64_t *offsets, int64_t n_all,
                          const uint32_t *e2, int64_t n2, const uint32_t *e3, int64_t n3,
                          const uint32_t *e4, int64_t n4, int64_t *counts, int64_t *stats)
{
    if (k != 3 && k != 4) return -1;
    build_tables();
    hgraph g;
    if (hgraph_build(&g, k, n_nodes, e2, n2, e3, n3, e4, n4) != 0) { hgraph_free(&g); return -1; }
    /* the projection: every ordered pair of distinct members of every
     * hyperedge, then each row sorted and its repeats dropped */
    int64_t n_pairs = 0;
    for (int64_t i = 0; i < n_all; i++) {
        int64_t s = offsets[i + 1] - offsets[i];
        n_pairs += s * (s - 1);
    }
    int64_t *off = (int64_t *)calloc((size_t)n_nodes + 1, sizeof(int64_t));
    int64_t *fill = (int64_t *)malloc(((size_t)n_nodes + 1) * sizeof(int64_t));
    uint32_t *adj = (uint32_t *)malloc((size_t)(n_pairs + 1) * sizeof(uint32_t));
    int failed = !off || !fill || !adj;
    if (!failed) {
        for (int64_t i = 0; i < n_all; i++)
            for (int64_t x = offsets[i]; x < offsets[i + 1]; x++)
                off[members[x] + 1] += offsets[i + 1] - offsets[i] - 1;
        for (uint32_t v = 0; v < n_nodes; v++) off[v + 1] += off[v];
        memcpy(fill, off, ((size_t)n_nodes + 1) * sizeof(int64_t));
        for (int64_t i = 0; i < n_all; i++)
            for (int64_t x = offsets[i]; x < offsets[i + 1]; x++)
                for (int64_t y = offsets[i]; y < offsets[i + 1]; y++)
                    if (x != y) adj[fill[members[x]]++] = members[y];
        /* compact: row v keeps its distinct neighbours, ascending */
        int64_t w = 0, start = 0;
        for (uint32_t v = 0; v < n_nodes; v++) {
            int64_t end = off[v + 1];
            qsort(adj + start, (size_t)(end - start), sizeof(uint32_t), cmp_u32);
            int64_t row = w;
            for (int64_t x = start; x < end; x++)
                if (x == start || adj[x] != adj[x - 1]) adj[w++] = adj[x];
            off[v] = row;
            start = end;
        }
        off[n_nodes] = w;
    }
    int64_t M[256];
    memset(M, 0, sizeof(M));
    base_ctx c = { &g, k, M, 0, 0 };
    if (!failed) {
        int esu_failed = 0;
        esu(off, adj, n_nodes, k, base_emit, &c, &esu_failed);
        failed = esu_failed;
    }
    free(off); free(fill); free(adj);
    hgraph_free(&g);
    if (failed) return -1;
    memcpy(counts, M, sizeof(int64_t) * (size_t)n_class[k]);
    stats[0] = c.candidates;
    stats[1] = c.discarded;
    return 0;
}

/* ------------------------------------------------------------------ */
/* Algorithm 4: sampled counts on an explicit sample list.             */
/* ------------------------------------------------------------------ */

/* nodes within `hops` of e through hyperedges of size <= smax (e excluded);
 * returns the count written to out (capacity n_nodes) */
static int64_t ball(const hgraph *g, const uint32_t *e, int j, int hops, int smax,
                    uint32_t *out, unsigned char *mark, uint32_t *frontier_buf)
{
    int64_t n_out = 0, f_begin = 0, f_end = 0;
    for (int a = 0; a < j; a++) { mark[e[a]] = 1; frontier_buf[f_end++] = e[a]; }
    for (int h = 0; h < hops; h++) {
        int64_t next_end = f_end;
        for (int64_t q = f_begin; q < f_end; q++) {
            uint32_t u = frontier_buf[q];
            for (int64_t x = g->inc_off[u]; x < g->inc_off[u + 1]; x++) {
                int fs = g->inc_size[x];
                if (fs > smax) continue;
                const uint32_t *f = g->e[fs] + (size_t)g->inc_idx[x] * fs;
                for (int a = 0; a < fs; a++) {
                    if (mark[f[a]]) continue;
                    mark[f[a]] = 1;
                    frontier_buf[next_end++] = f[a];
                    out[n_out++] = f[a];
                }
            }
        }
        f_begin = f_end;
        f_end = next_end;
    }
    for (int64_t q = 0; q < f_end; q++) mark[frontier_buf[q]] = 0;
    return n_out;
}

/* For every sampled hyperedge e (with multiplicity): every k-node set V
 * containing e whose induced sub-hypergraph is connected and holds no
 * hyperedge larger than e adds one to its class (raw counts, before the
 * correction factor).  samples[j] holds indices into the size-j list. */
int oracle_sampled_raw(int k, uint32_t n_nodes,
                       const uint32_t *e2, int64_t n2, const uint32_t *e3, int64_t n3,
                       const uint32_t *e4, int64_t n4,
                       const int64_t *s2, int64_t ns2, const int64_t *s3, int64_t ns3,
                       const int64_t *s4, int64_t ns4, int64_t *raw)
{
    if (k != 3 && k != 4) return -1;
    build_tables();
    hgraph g;
    if (hgraph_build(&g, k, n_nodes, e2, n2, e3, n3, e4, n4) != 0) { hgraph_free(&g); return -1; }
    const int64_t *S[5] = { 0, 0, s2, s3, s4 };
    int64_t NS[5] = { 0, 0, ns2, ns3, k == 4 ? ns4 : 0 };
    int64_t M[256];
    memset(M, 0, sizeof(M));
    uint32_t *cand = (uint32_t *)malloc(((size_t)n_nodes + 4) * sizeof(uint32_t));
    uint32_t *buf = (uint32_t *)malloc(((size_t)n_nodes + 4) * sizeof(uint32_t));
    unsigned char *mark = (unsigned char *)calloc((size_t)n_nodes + 1, 1);
    int failed = (!cand || !buf || !mark);
    for (int j = 2; j <= k && !failed; j++) {
        for (int64_t s = 0; s < NS[j] && !failed; s++) {
            int64_t idx = S[j][s];
            if (idx < 0 || idx >= g.ne[j]) { failed = 1; break; }
            const uint32_t *e = g.e[j] + (size_t)idx * j;
            int need = k - j;
            int64_t nb = ball(&g, e, j, need, j, cand, mark, buf);
            uint32_t V[4];
            if (need == 0) {
                memcpy(V, e, sizeof(uint32_t) * (size_t)j);
                uint32_t p = fill_in(&g, V, k);
                int cls = pattern_class(p, k);
                if (cls >= 0 && pattern_maxcard(p, k) == j) M[cls]++;
            } else if (need == 1) {
                for (int64_t a = 0; a < nb; a++) {
                    for (int t = 0; t < j; t++) V[t] = e[t];
                    V[j] = cand[a];
                    sort_nodes(V, k);
                    uint32_t p = fill_in(&g, V, k);
                    int cls = pattern_class(p, k);
                    if (cls >= 0 && pattern_maxcard(p, k) == j) M[cls]++;
                }
            } else {                                   /* need == 2: k = 4, j = 2 */
                for (int64_t a = 0; a < nb; a++)
                    for (int64_t b = a + 1; b < nb; b++) {
                        V[0] = e[0]; V[1] = e[1]; V[2] = cand[a]; V[3] = cand[b];
                        sort_nodes(V, 4);
                        uint32_t p = fill_in(&g, V, 4);
                        int cls = pattern_class(p, 4);
                        if (cls >= 0 && pattern_maxcard(p, 4) == 2) M[cls]++;
                    }
            }
        }
    }
    free(cand); free(buf); free(mark);
    hgraph_free(&g);
    if (failed) return -1;
    memcpy(raw, M, sizeof(int64_t) * (size_t)n_class[k]);
    return 0;
}

/* The oracle's own class list (canonical pattern per class id); returns the
 * number of classes. */
int oracle_class_canon(int k, uint32_t *canon_out)
{
    if (k != 3 && k != 4) return -1;
    build_tables();
    memcpy(canon_out, class_canon[k], sizeof(uint32_t) * (size_t)n_class[k]);
    return n_class[k];
}

/* Class id of one pattern (-1 when not connected). */
int oracle_pattern_class(int k, uint32_t pattern)
{
    if (k != 3 && k != 4) return -2;
    build_tables();
    return pattern_class(pattern, k);
}
