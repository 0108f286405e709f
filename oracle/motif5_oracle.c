/*
 * motif5_oracle.c -- reference implementation of order-5 higher-order motif
 * counting (the paper's Section 6.4 applies the sampling algorithm of
 * Section 5 at order 5).
 *
 * TEST INFRASTRUCTURE ONLY.  Plain, slow C written from the definitions;
 * only the test-suite and the benchmark's CPU-baseline leg load it.  It
 * shares no code with the HIP library (nor with the order-3/4 oracle).
 *
 * A node set V of 5 nodes is labelled by ascending node id (local positions
 * 0..4).  Its pattern has one bit per subset of {0..4} with at least two
 * members, in ascending subset-mask order (26 bits): bit i is set when the
 * i-th subset is a hyperedge of H (fill-in, Section 4.3).  Its class is the
 * smallest pattern value over the 120 relabellings (the isomorphism class of
 * Section 3), so classes are reported by that canonical value.
 *
 * Inputs are the unique hyperedges of each size j = 2..5 as ascending
 * j-tuples (the set semantics of Section 3 applied by the caller).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define K 5
#define NSUB 26
#define NPERM 120

static int sub_mask[NSUB];
static int bit_of_mask[32];
static uint8_t perms[NPERM][K];
static int ready = 0;

static int popc(unsigned x) { int c = 0; while (x) { c += x & 1; x >>= 1; } return c; }

static void init(void)
{
    if (ready) return;
    int n = 0;
    for (int m = 0; m < 32; m++) {
        bit_of_mask[m] = -1;
        if (popc((unsigned)m) >= 2) { bit_of_mask[m] = n; sub_mask[n++] = m; }
    }
    /* every permutation of {0..4}, by counting in base 5 and keeping those
       with distinct digits */
    int np = 0;
    for (int x = 0; x < 3125; x++) {
        int d[K], t = x, seen = 0, ok = 1;
        for (int i = 0; i < K; i++) { d[i] = t % 5; t /= 5; if (seen & (1 << d[i])) ok = 0; seen |= 1 << d[i]; }
        if (!ok) continue;
        for (int i = 0; i < K; i++) perms[np][i] = (uint8_t)d[i];
        np++;
    }
    ready = 1;
}

static uint32_t relabel(uint32_t p, const uint8_t *perm)
{
    uint32_t out = 0;
    for (int b = 0; b < NSUB; b++) {
        if (!((p >> b) & 1)) continue;
        int img = 0;
        for (int i = 0; i < K; i++)
            if ((sub_mask[b] >> i) & 1) img |= 1 << perm[i];
        out |= 1u << bit_of_mask[img];
    }
    return out;
}

uint32_t oracle5_canonical(uint32_t p)
{
    init();
    uint32_t best = 0xFFFFFFFFu;
    for (int g = 0; g < NPERM; g++) {
        uint32_t q = relabel(p, perms[g]);
        if (q < best) best = q;
    }
    return best;
}

int oracle5_connected(uint32_t p)
{
    init();
    int parent[K];
    unsigned covered = 0;
    for (int i = 0; i < K; i++) parent[i] = i;
    for (int b = 0; b < NSUB; b++) {
        if (!((p >> b) & 1)) continue;
        int m = sub_mask[b], first = -1;
        covered |= (unsigned)m;
        for (int i = 0; i < K; i++) {
            if (!((m >> i) & 1)) continue;
            if (first < 0) { first = i; continue; }
            int a = first, c = i;
            while (parent[a] != a) a = parent[a];
            while (parent[c] != c) c = parent[c];
            if (a != c) parent[a] = c;
        }
    }
    if (covered != (1u << K) - 1) return 0;
    int root = 0;
    while (parent[root] != root) root = parent[root];
    for (int i = 1; i < K; i++) {
        int r = i;
        while (parent[r] != r) r = parent[r];
        if (r != root) return 0;
    }
    return 1;
}

/* largest hyperedge size in the pattern, and how many hyperedges have it */
int oracle5_maxcard(uint32_t p, int *countmax)
{
    init();
    int mc = 0, cm = 0;
    for (int b = 0; b < NSUB; b++) {
        if (!((p >> b) & 1)) continue;
        int s = popc((unsigned)sub_mask[b]);
        if (s > mc) { mc = s; cm = 1; } else if (s == mc) cm++;
    }
    if (countmax) *countmax = cm;
    return mc;
}

/* ---------------------------------------------------------------- sets */
typedef struct { uint32_t v[K]; } tup5;
typedef struct { tup5 *key; unsigned char *full; size_t cap; } tset;

static uint64_t mix(uint64_t x)
{
    x ^= x >> 31; x *= 0x7fb5d329728ea185ULL; x ^= x >> 27; x *= 0x81dadef4bc2dd44dULL; x ^= x >> 33;
    return x;
}

static uint64_t thash(const tup5 *t)
{
    uint64_t h = 0x9e3779b97f4a7c15ULL;
    for (int i = 0; i < K; i++) h = mix(h + t->v[i]);
    return h;
}

static tup5 mk(const uint32_t *nodes, int n)       /* nodes ascending */
{
    tup5 t;
    for (int i = 0; i < K; i++) t.v[i] = i < n ? nodes[i] : 0xFFFFFFFFu;
    return t;
}

static int tset_init(tset *s, size_t n)
{
    size_t cap = 16;
    while (cap < 2 * n + 16) cap <<= 1;
    s->key = (tup5 *)malloc(cap * sizeof(tup5));
    s->full = (unsigned char *)calloc(cap, 1);
    s->cap = cap;
    return (s->key && s->full) ? 0 : -1;
}

static void tset_free(tset *s) { free(s->key); free(s->full); }

static void tset_add(tset *s, const tup5 *t)
{
    size_t m = s->cap - 1, i = (size_t)thash(t) & m;
    while (s->full[i]) {
        if (!memcmp(&s->key[i], t, sizeof(tup5))) return;
        i = (i + 1) & m;
    }
    s->full[i] = 1;
    s->key[i] = *t;
}

static int tset_has(const tset *s, const tup5 *t)
{
    size_t m = s->cap - 1, i = (size_t)thash(t) & m;
    while (s->full[i]) {
        if (!memcmp(&s->key[i], t, sizeof(tup5))) return 1;
        i = (i + 1) & m;
    }
    return 0;
}

/* ---------------------------------------------------------------- graph */
typedef struct {
    uint32_t n_nodes;
    const uint32_t *e[6];
    int64_t ne[6];
    tset edges;
    int64_t *inc_off;      /* node -> incident hyperedges of size 2..4 */
    int32_t *inc_size;
    int64_t *inc_idx;
} hg5;

static void hg5_free(hg5 *g) { tset_free(&g->edges); free(g->inc_off); free(g->inc_size); free(g->inc_idx); }

static int hg5_build(hg5 *g, uint32_t n_nodes, const uint32_t *const e[6], const int64_t ne[6])
{
    memset(g, 0, sizeof(*g));
    g->n_nodes = n_nodes;
    int64_t tot = 0, inc = 0;
    for (int j = 2; j <= 5; j++) { g->e[j] = e[j]; g->ne[j] = ne[j]; tot += ne[j]; if (j <= 4) inc += ne[j] * j; }
    if (tset_init(&g->edges, (size_t)tot) != 0) return -1;
    for (int j = 2; j <= 5; j++)
        for (int64_t i = 0; i < ne[j]; i++) { tup5 t = mk(e[j] + (size_t)i * j, j); tset_add(&g->edges, &t); }
    g->inc_off = (int64_t *)calloc((size_t)n_nodes + 1, sizeof(int64_t));
    g->inc_size = (int32_t *)malloc((size_t)(inc + 1) * sizeof(int32_t));
    g->inc_idx = (int64_t *)malloc((size_t)(inc + 1) * sizeof(int64_t));
    int64_t *fill = (int64_t *)malloc(((size_t)n_nodes + 1) * sizeof(int64_t));
    if (!g->inc_off || !g->inc_size || !g->inc_idx || !fill) { free(fill); return -1; }
    for (int j = 2; j <= 4; j++)
        for (int64_t i = 0; i < ne[j] * j; i++) g->inc_off[e[j][i] + 1]++;
    for (uint32_t v = 0; v < n_nodes; v++) g->inc_off[v + 1] += g->inc_off[v];
    memcpy(fill, g->inc_off, ((size_t)n_nodes + 1) * sizeof(int64_t));
    for (int j = 2; j <= 4; j++)
        for (int64_t i = 0; i < ne[j]; i++)
            for (int m = 0; m < j; m++) {
                uint32_t v = e[j][i * j + m];
                g->inc_size[fill[v]] = j;
                g->inc_idx[fill[v]] = i;
                fill[v]++;
            }
    free(fill);
    return 0;
}

/* pattern of the 5-node set V (ascending) */
static uint32_t fill5(const hg5 *g, const uint32_t *V)
{
    uint32_t p = 0;
    for (int b = 0; b < NSUB; b++) {
        uint32_t nodes[K];
        int n = 0;
        for (int i = 0; i < K; i++)
            if ((sub_mask[b] >> i) & 1) nodes[n++] = V[i];
        tup5 t = mk(nodes, n);
        if (tset_has(&g->edges, &t)) p |= 1u << b;
    }
    return p;
}

static void sort_small(uint32_t *V, int n)
{
    for (int i = 1; i < n; i++) {
        uint32_t x = V[i];
        int j = i - 1;
        while (j >= 0 && V[j] > x) { V[j + 1] = V[j]; j--; }
        V[j + 1] = x;
    }
}

/* ---------------------------------------------------------------- class tally */
typedef struct { uint32_t *canon; int64_t *count; int64_t n, cap; int failed; } tally;

static void tally_add(tally *t, uint32_t c)
{
    for (int64_t i = 0; i < t->n; i++)
        if (t->canon[i] == c) { t->count[i]++; return; }
    if (t->n == t->cap) {
        int64_t cap = t->cap ? 2 * t->cap : 64;
        uint32_t *a = (uint32_t *)realloc(t->canon, (size_t)cap * sizeof(uint32_t));
        int64_t *b = (int64_t *)realloc(t->count, (size_t)cap * sizeof(int64_t));
        if (!a || !b) { t->failed = 1; if (a) t->canon = a; if (b) t->count = b; return; }
        t->canon = a; t->count = b; t->cap = cap;
    }
    t->canon[t->n] = c;
    t->count[t->n] = 1;
    t->n++;
}

/* sort by canonical value and copy out; returns the number of classes, or -1
   when they do not fit in cap */
static int64_t tally_out(tally *t, uint32_t *canon_out, int64_t *count_out, int64_t cap)
{
    for (int64_t i = 1; i < t->n; i++) {
        uint32_t c = t->canon[i];
        int64_t x = t->count[i], j = i - 1;
        while (j >= 0 && t->canon[j] > c) { t->canon[j + 1] = t->canon[j]; t->count[j + 1] = t->count[j]; j--; }
        t->canon[j + 1] = c;
        t->count[j + 1] = x;
    }
    int64_t n = t->n;
    if (n > cap || t->failed) n = -1;
    else for (int64_t i = 0; i < n; i++) { canon_out[i] = t->canon[i]; count_out[i] = t->count[i]; }
    free(t->canon);
    free(t->count);
    return n;
}

/* ---------------------------------------------------------------- brute force */
/* Every 5-node subset whose induced sub-hypergraph is connected, by class. */
int64_t oracle5_exact_brute(uint32_t n_nodes, const uint32_t *e2, int64_t n2, const uint32_t *e3, int64_t n3,
                            const uint32_t *e4, int64_t n4, const uint32_t *e5, int64_t n5,
                            uint32_t *canon_out, int64_t *count_out, int64_t cap)
{
    init();
    const uint32_t *e[6] = { 0, 0, e2, e3, e4, e5 };
    const int64_t ne[6] = { 0, 0, n2, n3, n4, n5 };
    hg5 g;
    if (hg5_build(&g, n_nodes, e, ne) != 0) { hg5_free(&g); return -1; }
    tally t = { 0, 0, 0, 0, 0 };
    uint32_t V[K];
    for (V[0] = 0; V[0] < n_nodes; V[0]++)
        for (V[1] = V[0] + 1; V[1] < n_nodes; V[1]++)
            for (V[2] = V[1] + 1; V[2] < n_nodes; V[2]++)
                for (V[3] = V[2] + 1; V[3] < n_nodes; V[3]++)
                    for (V[4] = V[3] + 1; V[4] < n_nodes; V[4]++) {
                        uint32_t p = fill5(&g, V);
                        if (oracle5_connected(p)) tally_add(&t, oracle5_canonical(p));
                    }
    hg5_free(&g);
    return tally_out(&t, canon_out, count_out, cap);
}

/* ---------------------------------------------------------------- sampled */
/* nodes within `hops` of e through hyperedges of size <= smax (e excluded) */
static int64_t ball5(const hg5 *g, const uint32_t *e, int j, int hops, int smax, uint32_t *out,
                     unsigned char *mark, uint32_t *frontier)
{
    int64_t n_out = 0, f0 = 0, f1 = 0;
    for (int a = 0; a < j; a++) { mark[e[a]] = 1; frontier[f1++] = e[a]; }
    for (int h = 0; h < hops; h++) {
        int64_t next = f1;
        for (int64_t q = f0; q < f1; q++) {
            uint32_t u = frontier[q];
            for (int64_t x = g->inc_off[u]; x < g->inc_off[u + 1]; x++) {
                int fs = g->inc_size[x];
                if (fs > smax) continue;
                const uint32_t *f = g->e[fs] + (size_t)g->inc_idx[x] * fs;
                for (int a = 0; a < fs; a++) {
                    if (mark[f[a]]) continue;
                    mark[f[a]] = 1;
                    frontier[next++] = f[a];
                    out[n_out++] = f[a];
                }
            }
        }
        f0 = f1;
        f1 = next;
    }
    for (int64_t q = 0; q < f1; q++) mark[frontier[q]] = 0;
    return n_out;
}

/* Algorithm 4 at order 5: for every sampled hyperedge e of size j (with
 * multiplicity), every 5-node set V containing e whose induced
 * sub-hypergraph is connected and holds no hyperedge larger than e adds one
 * to its class.  samples[j] index the size-j list.  Raw counts by class
 * (canonical value, ascending) into canon_out / raw_out; returns the number
 * of classes, or -1. */
int64_t oracle5_sampled_raw(uint32_t n_nodes, const uint32_t *e2, int64_t n2, const uint32_t *e3, int64_t n3,
                            const uint32_t *e4, int64_t n4, const uint32_t *e5, int64_t n5,
                            const int64_t *s2, int64_t ns2, const int64_t *s3, int64_t ns3,
                            const int64_t *s4, int64_t ns4, const int64_t *s5, int64_t ns5,
                            uint32_t *canon_out, int64_t *raw_out, int64_t cap)
{
    init();
    const uint32_t *e[6] = { 0, 0, e2, e3, e4, e5 };
    const int64_t ne[6] = { 0, 0, n2, n3, n4, n5 };
    const int64_t *S[6] = { 0, 0, s2, s3, s4, s5 };
    const int64_t NS[6] = { 0, 0, ns2, ns3, ns4, ns5 };
    hg5 g;
    if (hg5_build(&g, n_nodes, e, ne) != 0) { hg5_free(&g); return -1; }
    uint32_t *ball = (uint32_t *)malloc(((size_t)n_nodes + 8) * sizeof(uint32_t));
    uint32_t *buf = (uint32_t *)malloc(((size_t)n_nodes + 8) * sizeof(uint32_t));
    unsigned char *mark = (unsigned char *)calloc((size_t)n_nodes + 1, 1);
    tally t = { 0, 0, 0, 0, 0 };
    int failed = !ball || !buf || !mark;
    for (int j = 2; j <= 5 && !failed; j++)
        for (int64_t s = 0; s < NS[j] && !failed; s++) {
            int64_t idx = S[j][s];
            if (idx < 0 || idx >= ne[j]) { failed = 1; break; }
            const uint32_t *eh = e[j] + (size_t)idx * j;
            int need = K - j;
            int64_t nb = ball5(&g, eh, j, need, j, ball, mark, buf);
            int64_t pick[3] = { 0, 0, 0 };
            /* every subset of `need` ball nodes, as increasing positions */
            for (int level = 0; level < need; level++) pick[level] = level;
            if (need > nb) continue;
            for (;;) {
                uint32_t V[K];
                for (int a = 0; a < j; a++) V[a] = eh[a];
                for (int a = 0; a < need; a++) V[j + a] = ball[pick[a]];
                sort_small(V, K);
                uint32_t p = fill5(&g, V);
                int cm;
                if (oracle5_connected(p) && oracle5_maxcard(p, &cm) == j) tally_add(&t, oracle5_canonical(p));
                /* next combination */
                int l = need - 1;
                while (l >= 0 && pick[l] == nb - need + l) l--;
                if (l < 0) break;
                pick[l]++;
                for (int m = l + 1; m < need; m++) pick[m] = pick[m - 1] + 1;
            }
        }
    free(ball); free(buf); free(mark);
    hg5_free(&g);
    if (failed) { free(t.canon); free(t.count); return -1; }
    return tally_out(&t, canon_out, raw_out, cap);
}
