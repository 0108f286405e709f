/*
 * homotif.h -- C ABI of the homotif library: exact and hyperedge-sampled
 * counting of higher-order motifs of order 3 and 4 on AMD MI355X (gfx950).
 *
 * Paper: Lotito, Musciotto, Battiston, Montresor, "Exact and sampling methods
 * for mining higher-order motifs in large hypergraphs" (arXiv 2209.10241).
 *
 * Problem (Section 3, "Mining higher-order motifs"): given a hypergraph
 * H = (V, E) and an order k, count, for every isomorphism class of connected
 * k-node sub-hypergraphs, how many node sets V' (|V'| = k) induce a
 * sub-hypergraph H[V'] = (V', {e in E : e subset of V'}) of that class.
 *
 * Conventions shared by every entry point
 *   - Node ids are uint32 in [0, n_nodes).  A hypergraph is given in CSR form:
 *     hyperedge i is members[offsets[i] .. offsets[i+1]), offsets[0] = 0.
 *   - Hyperedges form a set (Section 3): repeated hyperedges collapse, the
 *     first occurrence is kept.  Singletons are dropped (the fill-in step of
 *     Section 4.3 ignores them).  Hyperedges with more than k nodes cannot lie
 *     inside a k-node set and do not affect counts.
 *   - Stratum order: the unique hyperedges of size j, in order of first
 *     occurrence in the input, are indexed 0 .. |E_j|-1 (Algorithm 4 samples
 *     these strata).
 *   - Class numbering: the k nodes of a set take local positions 0..k-1 in
 *     ascending id order; pattern bit i marks the i-th subset of size >= 2 of
 *     {0..k-1} in ascending mask order (k=4: masks 3,5,6,7,9,10,11,12,13,14,15;
 *     k=3: 3,5,6,7) as a hyperedge; the canonical pattern of a class is the
 *     smallest pattern value over all k! relabellings; class ids rank the
 *     canonical patterns of connected classes ascending.  There are 6 classes
 *     for k=3 and 171 for k=4 (hm_num_classes, hm_class_info).
 *   - Ownership: the caller owns every buffer it passes.  Output pointers of
 *     the count_* calls are DEVICE pointers; the work is enqueued on `stream`
 *     (a hipStream_t, NULL for the default stream) and the outputs are valid
 *     once that stream has synchronised.  The library never keeps caller
 *     pointers after a call returns.  A graph handle owns its device memory
 *     until hm_graph_destroy.  Calls that use one graph handle must be
 *     serialised (one stream at a time): the handle holds reusable scratch.
 *     Calls on different handles may run at once from several host threads,
 *     each on its own stream; what the library shares between them (the
 *     device memory cache, the pinned report words, tuning and occupancy
 *     caches) is guarded by locks.  Exceptions are stated per entry point
 *     (count_exact_noalloc, the profiling calls).
 *   - Errors: every entry point returns HM_OK (0) or a negative HM_E* code and
 *     never aborts; on error outputs are left unspecified and hm_last_error()
 *     returns a message (thread-local).
 */
#ifndef HOMOTIF_H
#define HOMOTIF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HM_OK 0
#define HM_EINVAL (-1)        /* bad argument or malformed input */
#define HM_EUNSUPPORTED (-2)  /* valid request the library does not implement */
#define HM_ENOMEM (-3)        /* device allocation failed */
#define HM_EDEVICE (-4)       /* HIP runtime error */
#define HM_EINTERNAL (-5)     /* internal consistency check failed */

#define HM_MEM_HOST 0
#define HM_MEM_DEVICE 1

typedef struct hm_graph hm_graph;

/* Message describing the last error on this thread ("" if none). */
const char* hm_last_error(void);

/* Library version string. */
const char* hm_version(void);

/* ---------------------------------------------------------------- classes */

/* Number of isomorphism classes of connected k-node patterns: 6 for k=3,
 * 171 for k=4 (Section 4.3 builds them by relabelling every pattern);
 * HM_EUNSUPPORTED for other k. */
int hm_num_classes(int k);

/* Canonical pattern, maxcard (size of the largest hyperedge) and countmax
 * (number of hyperedges of that size) of class `cls` of order k; the last two
 * are the quantities of the correction factor of Algorithm 4.  Any output
 * pointer may be NULL.  Host pointers. */
int hm_class_info(int k, int cls, uint32_t* canon_pattern, int* maxcard, int* countmax);

/* Class id of a labelled pattern (encoding above) into *cls (host pointer),
 * -1 when the pattern is not connected; HM_EINVAL for a pattern out of
 * range. */
int hm_pattern_class(int k, uint32_t pattern, int* cls);

/* ---------------------------------------------------------------- graphs */

/* Build the device-resident hypergraph (Definition of a hypergraph,
 * Section 3): validate, sort members, collapse repeated hyperedges, split by
 * size, hash every hyperedge of size 2..4 (Section 4.3, Fig. 3b) and build the
 * adjacency used by the enumeration.
 *   members   node ids; hyperedge i is members[offsets[i] .. offsets[i+1])
 *   offsets   n_edges+1 values, offsets[0] = 0, non-decreasing
 *   n_members number of entries of members (offsets[n_edges] <= n_members;
 *             at most 2^32-1)
 *   mem_kind  HM_MEM_HOST or HM_MEM_DEVICE: where members and offsets live
 *   stream    hipStream_t for the build.  The call returns once the input
 *             has been validated and the sizes are known (hm_graph_stats is
 *             then exact); the rest of the build stays enqueued on the
 *             stream, so later calls on the same stream see the finished
 *             graph, and work on another stream must first wait for this
 *             one.  The caller's members/offsets buffers may be reused as
 *             soon as it returns.
 *   out       receives the handle
 * Errors: HM_EINVAL for an empty hyperedge, a node id >= n_nodes, a node
 * repeated inside a hyperedge, offsets that do not start at 0, decrease or
 * exceed n_members, or n_nodes = 0; HM_EUNSUPPORTED for n_members >= 2^32. */
int hm_graph_create(const uint32_t* members, const uint64_t* offsets, uint64_t n_edges, uint64_t n_members,
                    uint32_t n_nodes, int mem_kind, void* stream, hm_graph** out);

/* Release a graph handle (NULL is accepted).  Does not wait for the device:
 * when all work on the graph was enqueued on one stream its memory is reused
 * only by work enqueued after this call; otherwise (several streams, or a
 * null-model pipeline or learned proposal attached) the call first waits for
 * the device to be idle. */
int hm_graph_destroy(hm_graph* H);

/* Host array of 10 values: n_nodes, unique hyperedges of size 2, 3, 4, unique
 * hyperedges of size >= 5, input hyperedges, dropped singletons, collapsed
 * repeats, unique hyperedges of size >= 2, their total number of members. */
int hm_graph_stats(const hm_graph* H, uint64_t* out10);

/* Copy the unique hyperedges of size j (2..4), stratum order, as ascending
 * j-tuples into the host buffer `out` (|E_j| * j values). */
int hm_graph_export(const hm_graph* H, int j, uint32_t* out);

/* ---------------------------------------------------------------- exact */

/* Exact counts of every order-k motif (k = 3: Algorithm 2; k = 4:
 * Algorithm 3).  counts: device int64 array of hm_num_classes(k) values,
 * overwritten.  Asynchronous on `stream`. */
int count_exact(const hm_graph* H, int k, int64_t* counts, void* stream);

/* Exact counts of every order-k motif (k = 3 or 4, as count_exact) of each
 * of n_graphs hypergraphs: hypergraph g is members[g], offsets[g],
 * n_edges[g], n_members[g], n_nodes[g] with the meaning hm_graph_create
 * gives them (members and offsets in the memory mem_kind names; the five
 * arrays of n_graphs entries are host memory), and its counts go to
 * counts[g * hm_num_classes(k) ...] (device, overwritten).  The hypergraphs
 * are shared among `workers` host threads (1..16: the calling thread and up
 * to workers - 1 that it starts), each building, counting and releasing its
 * graphs on a stream of its own (the library keeps these
 * streams per device for the process), so that one graph's build, which
 * waits for its validation on the host, runs beside another's count.  The
 * workers start after the work already enqueued on `stream`, and `stream`
 * waits for all of theirs: the counts are valid once it has synchronised.
 * The call returns once every graph has been validated.
 * Errors: HM_EINVAL for n_graphs < 0, workers outside 1..16, a NULL array,
 * or a hypergraph that hm_graph_create refuses (any of its errors; the
 * message names the lowest such graph index among those attempted, and the
 * workers take no new graph after a failure, leaving the counts of graphs
 * not reached unspecified); HM_EUNSUPPORTED for k other than 3 or 4. */
int count_exact_many(int n_graphs, const uint32_t* const* members, const uint64_t* const* offsets,
                     const uint64_t* n_edges, const uint64_t* n_members, const uint32_t* n_nodes, int mem_kind,
                     int k, int64_t* counts, int workers, void* stream);

/* count_exact for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, same counts, and no hipMalloc, hipFree or other device
 * allocation in the call: its per-class counters (16 copies of 3 x 256
 * int64) and the class tables live in a fixed device array of the library
 * (about 130 KB, one per device, held until the process ends), whose device
 * address is looked up on the first call on each device.
 * Limit: graphs with adjacency bit rows only (at most
 * HM_OPT_BITSET_MAX_NODES nodes, 8192 by default): counting without them
 * needs temporaries sized by the graph.
 * Every call on one device shares that array, which keeps the last call's
 * contents; each call clears what it needs first.  Calls that overlap on one
 * device (on different streams, or from several threads) race and give
 * wrong counts: the caller serialises them.
 * Errors: HM_EINVAL for a NULL argument or when the current device is not
 * the graph's; HM_EUNSUPPORTED for k other than 3 or 4 or a graph without
 * bit rows; HM_EDEVICE when the array's address cannot be obtained. */
int count_exact_noalloc(const hm_graph* H, int k, int64_t* counts, void* stream);

/* Exact counts of every order-k motif (k = 3 or 4) by the baseline of
 * Section 4.1 (Algorithm 1): the clique projection G of the hypergraph (two
 * nodes joined when a hyperedge of any size >= 2 holds both), every connected
 * k-node set of G enumerated once by ESU, and each kept when the
 * sub-hypergraph it induces is connected.  The counts equal count_exact's;
 * the path exists to measure what the hyperedge-based generators save.
 * counts: device int64 array of hm_num_classes(k) values, overwritten.
 * stats: device uint64 array of 2 values, overwritten: the candidates ESU
 * produced, and those discarded (induced sub-hypergraph not connected).
 * The first call allocates the projection's bit rows (n_nodes * ceil(n_nodes
 * / 32) words, kept with the graph); every call rebuilds them.  Asynchronous
 * on `stream`; calls on one graph are serialised by the caller, as for
 * count_exact.
 * Errors: HM_EINVAL for a NULL argument; HM_EUNSUPPORTED for k other than 3
 * or 4, or for a graph without adjacency bit rows (more nodes than
 * HM_OPT_BITSET_MAX_NODES); HM_ENOMEM when the bit rows cannot be
 * allocated. */
int count_baseline(const hm_graph* H, int k, int64_t* counts, uint64_t* stats, void* stream);

/* ---------------------------------------------------------------- sampled */

/* Sample allocation over strata (Section 5: S_j draws from the hyperedges of
 * size j, with replacement).
 *   HM_ALLOC_PROPORTIONAL  S_j = ceil(fraction * |E_j|) for j = 2..k
 *   HM_ALLOC_PAPER         k = 4: S = ceil(fraction * (|E_2|+|E_3|+|E_4|)),
 *                          S_2 = floor(S/6), S_3 = floor(S/2), S_4 = the rest
 *                          (the ratio S_3 = 3 S_2, S_4 = 2 S_2 of the
 *                          appendix's parameter search); k = 3: proportional.
 * A stratum with no hyperedge gets no sample.  Under HM_ALLOC_PAPER a stratum
 * with at least one hyperedge gets at least one sample (so S_2 = 1 when
 * S < 6), which keeps every class's estimate unbiased. */
#define HM_ALLOC_PROPORTIONAL 0
#define HM_ALLOC_PAPER 1

/* Sample sizes S_2, S_3, S_4 (host array of 3) for the given fraction in
 * (0, 1] and allocation; S_4 = 0 when k = 3. */
int hm_sample_sizes(const hm_graph* H, int k, double fraction, int allocation, uint64_t* s_out);

/* The same rule from the stratum sizes alone: n_by_size is a host array of
 * 3 values |E_2|, |E_3|, |E_4| (the last is ignored when k = 3).  Host
 * only: needs no device and no graph.
 * Errors: HM_EINVAL for a NULL argument, a fraction outside (0, 1] or an
 * unknown allocation; HM_EUNSUPPORTED for k other than 3 or 4. */
int hm_sample_sizes_for(int k, const uint64_t* n_by_size, double fraction, int allocation, uint64_t* s_out);

/* count_sampled with the number of draws of each stratum given (s2, s3, s4
 * draws from the hyperedges of size 2, 3, 4; s4 is ignored when k = 3; a
 * stratum with no hyperedge gets none).  Draws and estimator as
 * count_sampled.  Errors: HM_EINVAL for a NULL argument or a size >= 2^31;
 * HM_EUNSUPPORTED for k other than 3 or 4. */
int count_sampled_sizes(const hm_graph* H, int k, uint64_t s2, uint64_t s3, uint64_t s4, uint64_t seed, float* est,
                        int64_t* raw, void* stream);

/* ---------------------------------------------------------------- order 5 */

/* Section 6.4 samples motifs of order 5, where exact counting does not
 * reach.  Algorithm 4 at order 5: S_j = ceil(fraction * |E_j|) draws from
 * the unique hyperedges of each size j = 2..5 (with replacement; draw i of
 * stratum j is hi64(w * |E_j|), w the first word of Philox4x64-10 at counter
 * (i, 0, 0, 0) under key (seed, (1 << 32) | j)); each drawn e of size j
 * counts every 5-node set V containing e whose induced sub-hypergraph is
 * connected and holds no hyperedge larger than |e|.
 * A class is reported by its canonical pattern: local positions 0..4 follow
 * ascending node id, pattern bit b is the b-th subset of {0..4} with at
 * least two members in ascending subset-mask order (26 bits), and the
 * canonical pattern is the smallest value over the 120 relabellings.  Its
 * maxcard j is its largest hyperedge size and countmax the number of its
 * hyperedges of that size; est = raw * |E_j| / (S_j * countmax), formed in
 * fp64 and rounded once to fp32 (0 when S_j = 0).
 * Outputs (device, `capacity` entries): canon (uint32), raw (int64), est
 * (float), the classes found in ascending canonical order; *n_classes (host)
 * receives their number.  Synchronous.  The first call on a graph builds its
 * list and hash set of 5-node hyperedges (kept with the graph).
 * Limits: each sampled hyperedge may have at most 4096 nodes within
 * 5 - |e| hops and fewer than 2^32 candidate sets (HM_EUNSUPPORTED past
 * that: the enumeration is meant for the sparse or small hypergraphs the
 * paper samples at order 5).
 * Errors: HM_EINVAL for a NULL argument, a fraction outside (0, 1], or more
 * classes than capacity (n_classes still tells how many). */
int count_sampled5(const hm_graph* H, double fraction, uint64_t seed, uint64_t capacity, uint32_t* canon, int64_t* raw,
                   float* est, uint64_t* n_classes, void* stream);

/* count_sampled5 on explicit draws (device uint32 index arrays per stratum,
 * with s2..s5 entries; NULL allowed for 0), as count_sampled_indices.
 * Errors as count_sampled5, and HM_EINVAL for an index outside its stratum. */
int count_sampled5_indices(const hm_graph* H, const uint32_t* idx2, uint64_t s2, const uint32_t* idx3, uint64_t s3,
                           const uint32_t* idx4, uint64_t s4, const uint32_t* idx5, uint64_t s5, uint64_t capacity,
                           uint32_t* canon, int64_t* raw, float* est, uint64_t* n_classes, void* stream);

/* |E_2|, |E_3|, |E_4|, |E_5| (host array of 4): the unique hyperedges of each
 * size; builds the order-5 structures on first use.  Synchronous. */
int hm_order5_sizes(const hm_graph* H, uint64_t* n_by_size4, void* stream);

/* Write the drawn stratum indices (device uint32 arrays of S_2, S_3, S_4
 * values; pointers for empty strata may be NULL).  Draw i of stratum j is
 * hi64(w * |E_j|) with w the first word of Philox4x64-10 (Salmon et al.,
 * SC'11) at counter (i, 0, 0, 0) under key (seed, (1 << 32) | j).
 * Asynchronous on `stream`. */
int hm_sample_draw(const hm_graph* H, int k, double fraction, uint64_t seed, int allocation, uint32_t* idx2,
                   uint32_t* idx3, uint32_t* idx4, void* stream);

/* Sampled counts (Algorithm 4): draw the samples as hm_sample_draw does;
 * around every sampled hyperedge e enumerate the connected k-node sets that
 * contain e and hold no hyperedge larger than e, adding one to their class;
 * scale class m by |E_maxcard| / (S_maxcard * countmax) (the correction factor
 * of Algorithm 4; unbiased by Section 5's argument), in fp64 rounded once to
 * fp32.
 *   est  device float array of hm_num_classes(k) values (required)
 *   raw  device int64 array of the unscaled counts, or NULL
 * fraction in (0, 1]; HM_EINVAL otherwise.  Asynchronous on `stream`. */
int count_sampled(const hm_graph* H, int k, double fraction, uint64_t seed, int allocation, float* est,
                  int64_t* raw, void* stream);

/* The same on an explicit sample: device uint32 arrays of stratum indices
 * (repetitions allowed), s_j entries each; a NULL array needs s_j = 0; idx4
 * is ignored for k = 3.  HM_EINVAL when an index lies outside its stratum
 * (checked before counting; this call synchronises the stream once). */
int count_sampled_indices(const hm_graph* H, int k, const uint32_t* idx2, uint64_t s2, const uint32_t* idx3,
                          uint64_t s3, const uint32_t* idx4, uint64_t s4, float* est, int64_t* raw, void* stream);

/* ---------------------------------------------------------------- nulls */

/* Motif over/under-expression against randomised hypergraphs (Section 1:
 * count, count again on randomisations, score; Section 6.3 uses a
 * configuration model).  The null model is stub matching that keeps every
 * node degree and every hyperedge size: the stubs are the members (ascending)
 * of the unique hyperedges of size >= 2 in stratum order; copy c uses the
 * Philox4x64-10 key (seed, (2 << 32) | c); round 0 orders the stubs by
 * (word0 of counter (t, 0, 0, 0), t) and cuts them into the size sequence;
 * while a hyperedge repeats a node (rounds r = 1..64), the offending
 * hyperedges B (ascending) each take a partner hi64(word0 of counter
 * (q, r, 1, 0) * E), and the members of B u partners are reordered by
 * (word0 of counter (t, r, 0, 0), t) and dealt back in ascending hyperedge
 * order.  Each copy is counted exactly (repeated hyperedges collapse) and
 * z_m = (real_m - mean_m) / sd_m (sd over the copies with n_rand - 1; fp64,
 * rounded to fp32; +-inf when sd = 0 and real differs from the mean, 0 when
 * it does not).
 *   real   device int64[C] exact counts of H, or NULL
 *   nulls  device int64[n_rand * C], copy-major (required)
 *   z      device float[C], or NULL
 * n_rand in [2, 65535]; HM_EINVAL when a copy cannot be repaired.
 * All copies are generated, ingested and counted together: batched kernels
 * over (copy, hyperedge) index spaces and one persistent counting kernel that
 * takes (phase, copy, chunk) tiles from a device queue.  The first call for a
 * (graph, k, n_rand) allocates the buffers, picks the tile sizes by timing
 * (cached per device and shape for the process) and captures the pipeline in
 * a HIP graph; every call replays that graph (the seed is read from device
 * memory).  Synchronises `stream` before returning. */
int count_nulls(const hm_graph* H, int k, int n_rand, uint64_t seed, int64_t* real, int64_t* nulls, float* z,
                void* stream);

/* Null models of count_nulls_model:
 *   HM_NULL_STUBS   stub matching with local repair (count_nulls' model)
 *   HM_NULL_CONFIG  the configuration model of Section 6.3 (Chodrow, J.
 *                   Complex Networks 2020), sampled by Markov chain Monte
 *                   Carlo: copy c starts from H's unique hyperedges of size
 *                   >= 2 (first-occurrence order) and runs `sweeps` rounds;
 *                   round r orders the hyperedges by (word 0 of Philox4x64-10
 *                   at counter (i, r, 0, 0), i) under key (seed, (5 << 32) |
 *                   c), pairs them two by two, and reshuffles each pair e, f:
 *                   shared nodes stay in both, the others (e - f then f - e,
 *                   ascending) are dealt out by a partial Fisher-Yates shuffle
 *                   (draw q: q + hi64(w (|D| - q)), w = word q mod 4 at counter
 *                   (t, r, 1 + q div 4, 0) for pair t) keeping both sizes.
 * Both keep every node degree and hyperedge size and repeat no node inside a
 * hyperedge; a copy may hold one node set twice, which counting collapses. */
#define HM_NULL_STUBS 0
#define HM_NULL_CONFIG 1

/* count_nulls with a choice of null model; sweeps (1..4096) is the number of
 * reshuffle rounds of HM_NULL_CONFIG and is ignored for HM_NULL_STUBS.  The
 * same batched, graph-captured pipeline as count_nulls (a call with another
 * model, order or copy count re-plans it).  Errors as count_nulls, and
 * HM_EINVAL for an unknown model or sweeps out of range. */
int count_nulls_model(const hm_graph* H, int k, int n_rand, int model, int sweeps, uint64_t seed, int64_t* real,
                      int64_t* nulls, float* z, void* stream);

/* Null copy `copy` of count_nulls_model's model, as hm_null_export. */
int hm_null_export_model(const hm_graph* H, int model, int sweeps, uint64_t seed, uint32_t copy, uint32_t* members,
                         uint64_t* offsets);

/* Motif profile (Section 6.3: observed frequencies against a null model;
 * the relative abundance of the cited higher-order motif work):
 *   delta_m = (x_m - mu_m) / (x_m + mu_m + eps),  mu_m the mean of the n_rand
 *   null rows, and the significance profile sp = delta / ||delta||_2 (zeros
 *   when delta is zero).
 * real: device double [n_classes] (exact counts or estimates); nulls: device
 * double [n_rand][n_classes]; delta, sp: device double [n_classes] outputs,
 * either may be NULL.  fp64 throughout.  Asynchronous on `stream`.
 * Errors: HM_EINVAL for NULL inputs (or both outputs NULL), n_rand < 1,
 * n_classes outside [1, 65536] or eps < 0. */
int hm_motif_profile(const double* real, const double* nulls, int n_rand, int n_classes, double eps, double* delta,
                     double* sp, void* stream);

/* The stratum-budget search of the appendix (Fig. 6): with S draws in total
 * split S_2 : S_3 : S_4 = 1 : ratio3[i] : ratio4[j] (S_2 = llround(S / (1 +
 * ratio3 + ratio4)), S_3 = min(S - S_2, llround(ratio3 S_2)), S_4 the rest;
 * k = 3: S_3 = S - S_2 and ratio4 is unused), every cell runs `reps` sampled
 * estimates (count_sampled_sizes with seeds seed, seed + 1, ...), forms each
 * estimate's profile against the null rows (hm_motif_profile with eps) and
 * its Pearson correlation with exact_profile (hm_profile_quality); rho
 * (host double [n3 * n4], row i, column j) receives the mean correlation over
 * the repetitions.  nulls: device double [n_rand][C]; exact_profile: device
 * double [C].  Synchronous.
 * Errors: HM_EINVAL for a NULL argument, S = 0 or >= 2^31, an empty grid or
 * more than 4096 cells, reps outside [1, 1024], n_rand < 1, eps < 0 or a
 * negative ratio; HM_EUNSUPPORTED for k other than 3 or 4. */
int hm_stratum_search(const hm_graph* H, int k, uint64_t S, const double* ratio3, int n3, const double* ratio4, int n4,
                      int reps, uint64_t seed, const double* nulls, int n_rand, const double* exact_profile, double eps,
                      double* rho, void* stream);

/* Accuracy of an estimated profile against the exact one (Section 6.3,
 * Table 3): out3 (device double [3]) receives Pearson's correlation rho, the
 * largest absolute error MaxAE and the mean absolute error MAE over the
 * n_classes values (est, exact: device double).  rho is 0 when either profile
 * is constant.  Asynchronous on `stream`.
 * Errors: HM_EINVAL for a NULL argument or n_classes outside [1, 65536]. */
int hm_profile_quality(const double* est, const double* exact, int n_classes, double* out3, void* stream);

/* Items per tile chosen for the last count_nulls on H (host array of 3:
 * 3-node hyperedges, pairs, hyperedges of size k); HM_EINVAL before any.  A
 * tile is taken by one wavefront, or, at order 4 when a copy's adjacency bit
 * rows and row starts fit in 48 KB of LDS, by one workgroup whose four
 * wavefronts share its items. */
int hm_null_tile_sizes(const hm_graph* H, uint32_t* out3);

/* Null copy `copy` of count_nulls' model (host outputs): members in the
 * copy's stored order (offsets[n_unique] values) and the offsets of the size
 * sequence (n_unique + 1 values, n_unique = unique hyperedges of size >= 2).
 * Synchronous. */
int hm_null_export(const hm_graph* H, uint64_t seed, uint32_t copy, uint32_t* members, uint64_t* offsets);

/* ---------------------------------------------------------------- learned proposal */

/* Algorithm 4 draws uniformly inside each stratum; any proposal p_e > 0 keeps
 * the estimate unbiased when each draw of stratum j weighs 1 / (S_j p_e)
 * (Hansen-Hurwitz; with p_e = 1/|E_j| this is Algorithm 4's correction).  The
 * learned proposal scores hyperedges with an MLP (16 features -> 64 -> 64 ->
 * 1, ReLU; bf16 weights and activations on MFMA, fp32 accumulation) trained on
 * exact per-hyperedge contributions y_e = sum_m raw_e[m] / countmax_m
 * (Algorithm 4's count for the single sample e), computed by the library on a
 * (sub)hypergraph.  Parameters (5313 floats): W1[64][16], b1[64],
 * W2[64][64], b2[64], w3[64], b3. */
typedef struct hm_model hm_model;

typedef struct {
  int epochs;      /* passes over the training rows */
  int batch;       /* rows per Adam step (>= 16) */
  float lr;        /* Adam learning rate */
  float gamma;     /* proposal q_e = (1 + predicted y_e)^gamma */
  float epsilon;   /* mixture weight of the uniform proposal, in (0, 1] */
  uint64_t seed;   /* initial weights and row order */
} hm_train_opts;

/* Standardised features of every hyperedge of size 2..k (device float
 * [n_rows][16], rows: the strata of size 2, 3, 4 in stratum order). */
int hm_features(const hm_graph* H, int k, float* x, void* stream);

/* Exact per-hyperedge contributions y_e (device double [n_rows], same rows);
 * the y_e of stratum j sum to the exact total of the classes with maxcard j.
 * Synchronous. */
int hm_contrib(const hm_graph* H, int k, double* y, void* stream);

/* MLP forward over n rows of 16 features (device pointers). */
int hm_mlp_forward(const float* params, const float* x, uint64_t n, float* out, void* stream);

/* Gradient of the mean squared error (device grad[5314]: 5313 parameter
 * gradients, then the loss) for n rows with targets t.  Synchronous. */
int hm_mlp_grad(const float* params, const float* x, const float* t, uint64_t n, float* grad, void* stream);

/* Train a proposal on H (usually a subsampled hypergraph): contributions,
 * features, per-stratum standardised targets log(1 + y_e), Adam on the GPU.
 * Synchronous. */
int hm_model_train(const hm_graph* H, int k, const hm_train_opts* opts, hm_model** out);
int hm_model_destroy(hm_model* M);
/* Host copy of the 5313 parameters. */
int hm_model_params(const hm_model* M, float* params_out);
/* Mean training loss per epoch (host array); returns the number of epochs. */
int hm_model_loss(const hm_model* M, int max_epochs, float* loss_out);

/* Proposal probabilities of every hyperedge of size 2..k of H under model M
 * (device double [n_rows]).  Synchronous. */
int hm_proposal_probs(const hm_graph* H, const hm_model* M, int k, double* p, void* stream);

/* Sampled counts with the learned proposal: S_j = ceil(fraction |E_j|)
 * draws per stratum with probabilities hm_proposal_probs; draw i of stratum j
 * is the first hyperedge whose cumulative probability exceeds u * total,
 * u = (word0 >> 11) 2^-53 of Philox4x64-10 at counter (i, 0, 0, 0) under key
 * (seed, (3 << 32) | j); est_m = sum over draws of raw[m] / (S_j p_e
 * countmax_m), fp64 rounded to fp32.  raw (optional): unweighted raw counts.
 * Synchronous. */
int count_sampled_learned(const hm_graph* H, const hm_model* M, int k, double fraction, uint64_t seed, float* est,
                          int64_t* raw, void* stream);

/* The Hansen-Hurwitz estimate on explicit draws: per stratum, device uint32
 * indices and device double probabilities p of each draw.  Synchronous. */
int count_sampled_weighted_indices(const hm_graph* H, int k, const uint32_t* idx2, const double* p2, uint64_t s2,
                                   const uint32_t* idx3, const double* p3, uint64_t s3, const uint32_t* idx4,
                                   const double* p4, uint64_t s4, float* est, int64_t* raw, void* stream);

/* ---------------------------------------------------------------- options */

/* Process-wide tuning options (read when a graph is created).
 *   HM_OPT_BITSET_MAX_NODES  graphs with at most this many nodes (default and
 *                            maximum 8192) also keep adjacency bit rows, which
 *                            the counting kernels use for pair tests and
 *                            neighbour intersections; 0 forces the hash-set
 *                            probes everywhere.
 *   HM_OPT_SAMPLE_CHUNK_SCALE the sampled counts of graphs without bit rows
 *                            hand the long walks of heavy samples to a work
 *                            queue in chunks (2 nodes of T, 4 correction
 *                            items, 128 exception positions, 256 hyperedges;
 *                            pair samples with a bound above 4096 visited
 *                            positions); every chunk size and that bound
 *                            are divided by this value
 *                            (default 1, range 1..1024), so larger values
 *                            route more of the work through the queue.  The
 *                            results do not depend on it.
 *   HM_OPT_ONE_PASS_MAX_EDGES graphs that keep bit rows and have at most this
 *                            many input hyperedges (default and maximum
 *                            2^20) are built in one pass: buffers are sized
 *                            by upper bounds and hm_graph_create waits for
 *                            the device once, at the end of the build; larger
 *                            graphs wait once the sizes are known and are
 *                            sized exactly.  0 builds every graph the second
 *                            way.  The graph does not depend on it.
 *   HM_OPT_HUB_MIN_DEGREE     graphs without bit rows keep, from their first
 *                            counting call on, a dense adjacency bit row for
 *                            each node with at least this many pairwise
 *                            neighbours (default 256), highest degrees first,
 *                            within 32 MiB; pair tests against such a node
 *                            read a bit instead of probing the hash set.  0
 *                            keeps none.  Taken when a graph's rows are
 *                            built; results do not depend on it.
 *   HM_OPT_DEDUP_TAG_BITS    the build finds repeated hyperedges in one
 *                            launch: each enters a hash table whose entries
 *                            carry this many bits of its hash as a tag
 *                            (default and maximum 32), and an entry it meets
 *                            with an equal tag is taken as its copy; the
 *                            next launch compares the members of every such
 *                            meeting, and if two different hyperedges met,
 *                            the build starts again with the exact search
 *                            (members compared at insertion, one launch
 *                            more).  Fewer bits make such meetings frequent
 *                            (0: every probe meets), to exercise that path;
 *                            -1 always uses the exact search.  The graph
 *                            does not depend on it.
 * HM_EINVAL for an unknown option or a value out of range. */
#define HM_OPT_BITSET_MAX_NODES 1
#define HM_OPT_SAMPLE_CHUNK_SCALE 2
#define HM_OPT_ONE_PASS_MAX_EDGES 3
#define HM_OPT_HUB_MIN_DEGREE 4
#define HM_OPT_DEDUP_TAG_BITS 5
int hm_set_option(int option, int64_t value);
int hm_get_option(int option, int64_t* value);

/* ---------------------------------------------------------------- timing */

/* Per-kernel timing for observability.  While enabled (on != 0), the counting
 * calls bracket each kernel launch with HIP events on the caller's stream.
 * Process-wide; not meant for concurrent use from several threads. */
int hm_profile_enable(int on);

/* Wait for recorded events and clear the accumulated totals. */
int hm_profile_reset(void);

/* Wait for recorded events and report up to max_entries kernels: names
 * (64 bytes each, NUL-terminated), launch counts and summed milliseconds
 * (host arrays, any may be NULL).  Returns the number of entries written. */
int hm_profile_read(int max_entries, char* names, uint64_t* launches, double* total_ms);

#ifdef __cplusplus
}
#endif

#endif /* HOMOTIF_H */
