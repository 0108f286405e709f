// Internal declarations of the homotif HIP library (gfx950).
//
// Device-resident hypergraph layout, hash sets of hyperedges (Section 4.3,
// Fig. 3b: every hyperedge is hashed so that its existence is checked in
// constant time), error plumbing and small wavefront helpers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/homotif.h"

namespace hm {

constexpr int kWave = 64;
// Device histograms that many workgroups add to are kept in kHistCopies
// copies: workgroup b adds to copy b mod kHistCopies, so that no counter takes
// the atomics of more than a kHistCopies-th of the workgroups; the kernel
// that reads them sums the copies.
constexpr uint32_t kHistCopies = 16;
constexpr uint32_t kExactHistStride = 1024;   // per copy: main, sub, G2 regions, 256 unused
constexpr uint32_t kSampleHistStride = 256;
constexpr uint32_t kEmpty32 = 0xFFFFFFFFu;
constexpr unsigned long long kEmpty64 = ~0ull;
// adjacency bit rows are kept when the node count is at most this (the
// largest value HM_OPT_BITSET_MAX_NODES accepts)
constexpr uint32_t kBitsetMaxNodes = 8192;
uint32_t bitset_max_nodes();
uint32_t sample_chunk_scale();
// graphs with bit rows and at most this many input hyperedges are built in
// one pass, with buffers sized by upper bounds (largest value and default of
// HM_OPT_ONE_PASS_MAX_EDGES)
constexpr uint64_t kOnePassMaxEdges = 1ull << 20;
uint64_t one_pass_max_edges();
// graphs without bit rows keep a dense adjacency bit row for each node with
// at least hub_min_degree() pairwise neighbours (HM_OPT_HUB_MIN_DEGREE; 0:
// none), the highest degrees first, in at most kHubRowBytes
constexpr uint32_t kHubMinDegree = 256;
constexpr uint64_t kHubRowBytes = 32ull << 20;
uint32_t hub_min_degree();
// bits of a hyperedge's hash kept as its tag in the build's one-launch
// duplicate search (HM_OPT_DEDUP_TAG_BITS; -1: the exact search only)
int dedup_tag_bits();

// ----------------------------------------------------------------- errors
void set_error(const char* fmt, ...);
// Called from the catch clause that every entry point of the C ABI wraps its
// body in, so that no exception crosses the ABI: a failed host allocation
// (std::bad_alloc, what the library's host code can throw) becomes HM_ENOMEM,
// anything else HM_EINTERNAL, with the message set.
int api_failure();
const char* last_error();
struct Status {
  int code = HM_OK;
};

#define HM_HIP(call)                                                              \
  do {                                                                            \
    hipError_t _e = (call);                                                       \
    if (_e != hipSuccess) {                                                       \
      ::hm::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(_e),      \
                      __FILE__, __LINE__);                                        \
      return HM_EDEVICE;                                                          \
    }                                                                             \
  } while (0)

#define HM_TRY(expr)          \
  do {                        \
    int _rc = (expr);         \
    if (_rc != HM_OK) return _rc; \
  } while (0)

// ----------------------------------------------------------------- hashing
__host__ __device__ inline unsigned long long mix64(unsigned long long x) {
  x ^= x >> 31;
  x *= 0x7fb5d329728ea185ull;
  x ^= x >> 27;
  x *= 0x81dadef4bc2dd44dull;
  x ^= x >> 33;
  return x;
}

// Keys: a 2-node hyperedge {a<b} is (a<<32)|b; 3- and 4-node hyperedges are
// 128-bit (hi = a<<32|b, lo = c<<32|d), with d = 0xFFFFFFFF for 3 nodes.
__host__ __device__ inline unsigned long long key2(uint32_t a, uint32_t b) {
  return ((unsigned long long)a << 32) | b;
}
struct Key128 {
  unsigned long long hi, lo;
};
__host__ __device__ inline Key128 key3(uint32_t a, uint32_t b, uint32_t c) {
  return Key128{((unsigned long long)a << 32) | b, ((unsigned long long)c << 32) | 0xFFFFFFFFull};
}
__host__ __device__ inline Key128 key4(uint32_t a, uint32_t b, uint32_t c, uint32_t d) {
  return Key128{((unsigned long long)a << 32) | b, ((unsigned long long)c << 32) | d};
}
__host__ __device__ inline unsigned long long hash128(Key128 k) {
  return mix64(k.hi ^ mix64(k.lo + 0x9e3779b97f4a7c15ull));
}

// Open-addressing (linear probing) set of 64-bit keys; capacity is a power
// of two with load at most 1/2; empty slots hold kEmpty64.
struct Set64 {
  unsigned long long* slot = nullptr;
  unsigned long long mask = 0;
};
// Same with 128-bit keys stored as (hi, lo) pairs.
struct Set128 {
  unsigned long long* slot = nullptr;  // 2 words per slot
  unsigned long long mask = 0;
};

__device__ inline bool set64_has(const Set64& s, unsigned long long key) {
  unsigned long long pos = mix64(key) & s.mask;
  while (true) {
    unsigned long long v = s.slot[pos];
    if (v == key) return true;
    if (v == kEmpty64) return false;
    pos = (pos + 1) & s.mask;
  }
}

__device__ inline bool set128_has(const Set128& s, Key128 key) {
  unsigned long long pos = hash128(key) & s.mask;
  while (true) {
    const ulonglong2 v = *reinterpret_cast<const ulonglong2*>(s.slot + 2 * pos);
    if (v.x == key.hi && v.y == key.lo) return true;
    if (v.x == kEmpty64) return false;
    pos = (pos + 1) & s.mask;
  }
}

inline unsigned long long pow2_capacity(unsigned long long n) {
  unsigned long long cap = 64;
  while (cap < 2 * n + 2) cap <<= 1;
  return cap;
}

// ----------------------------------------------------------------- class tables
// Built once per process on the host from the definitions (see classes.cpp),
// copied to device memory per device.
struct ClassTables {
  int n_classes[5];             // [3] = 6, [4] = 171
  uint8_t lut3[16];             // pattern -> class, 0xFF = not connected
  uint8_t lut4[2048];
  uint32_t canon[5][256];       // canonical pattern per class
  uint8_t maxcard[5][256];
  uint8_t countmax[5][256];
};
const ClassTables& class_tables();
// device copy of lut4 (2048 bytes) followed by lut3 (16 bytes), per device
int device_luts(int device, const uint8_t** lut4, const uint8_t** lut3);

// ----------------------------------------------------------------- primitives
int scan_exclusive_u32(const uint32_t* in, uint32_t* out, uint64_t n, uint32_t* total_dev,
                       hipStream_t stream);
int scan_exclusive_u64(const unsigned long long* in, unsigned long long* out, uint64_t n,
                       hipStream_t stream);
// Stable LSD radix sort of (key, value) pairs on bits [0, bits) of the key.
// Buffers are ping-ponged; the sorted result ends in keys/vals (the first pair).
int radix_sort_pairs(unsigned long long* keys, uint32_t* vals, unsigned long long* keys_tmp,
                     uint32_t* vals_tmp, uint64_t n, int bits, hipStream_t stream);
int fill_u32(uint32_t* p, uint32_t value, uint64_t n, hipStream_t stream);
int copy_u32(const uint32_t* src, uint32_t* dst, uint64_t n, hipStream_t stream);
int copy_u64(const unsigned long long* src, unsigned long long* dst, uint64_t n, hipStream_t stream);
// Workspace variants: no allocation, no host synchronisation (usable under
// stream capture).  The workspace sizes are in uint32 words.
uint64_t scan_ws_words(uint64_t n);
int scan_u32_ws(const uint32_t* in, uint32_t* out, uint64_t n, uint32_t* total_dev, uint32_t* ws,
                hipStream_t stream);
uint64_t radix_ws_words(uint64_t n);
int radix_sort_ws(unsigned long long* keys, uint32_t* vals, unsigned long long* keys_tmp, uint32_t* vals_tmp,
                  uint64_t n, int bits, uint32_t* ws, hipStream_t stream);
int fill_u64(unsigned long long* p, unsigned long long value, uint64_t n, hipStream_t stream);
// *out = max(*out, v[0..n)) (out zeroed by the caller)
int max_u32(const uint32_t* v, uint64_t n, uint32_t* out, hipStream_t stream);

// ----------------------------------------------------------------- profiling
// While hm_profile_enable(1) is in effect, a scope records HIP events around
// the launches it encloses on `st`, under `name`.
bool profiling();
// Kernel launches enqueued between capture_begin and capture_end go into a
// HIP graph; profiling scopes stay inactive meanwhile.
void capture_begin();
void capture_end();
class ProfileScope {
 public:
  ProfileScope(const char* name, hipStream_t st);
  ~ProfileScope();
  ProfileScope(const ProfileScope&) = delete;
  ProfileScope& operator=(const ProfileScope&) = delete;

 private:
  const char* name_;
  hipStream_t st_;
  hipEvent_t start_{}, stop_{};
  bool active_ = false;
};

// ----------------------------------------------------------------- device allocations
int dalloc(void** p, size_t bytes);
// release a block whose users are synchronised
void dfree(void* p);
// release blocks that work already enqueued on st may still use (one event
// recorded on st for the batch)
void dfree_on(void* p, hipStream_t st);
void dfree_on(void* const* ps, size_t n, hipStream_t st);
// A block for a table whose idle state is every byte 0xFF: a cached block
// left that way by its last user when one is free (*filled true), else any
// block (*filled false: the caller fills it).  mark_filled(p) before the
// release of p promises that the work enqueued before the release leaves it
// all 0xFF again; a block released without it goes back to the ordinary
// cache.
int dalloc_filled(void** p, size_t bytes, bool* filled);
void mark_filled(void* p);

// Order-k counts of the pairs-only shapes and of case (b) without bit rows
// into H->hist (case (a) is counted by the caller).
int count_sparse(const hm_graph* H, int k, hipStream_t st);
int ensure_pair_links(hm_graph* H, hipStream_t st);
int ensure_hub_rows(hm_graph* H, hipStream_t st);
int ensure_node_stats(hm_graph* H, hipStream_t st);
int ensure_edge_stats(hm_graph* H, hipStream_t st);

struct NullPlan;
void destroy_null_plan(NullPlan* p);
struct ProposalCache;
void destroy_proposal_cache(ProposalCache* c);

}  // namespace hm

// ----------------------------------------------------------------- the graph handle
struct hm_graph {
  int device = 0;
  uint32_t n_nodes = 0;
  uint64_t n_input = 0;
  uint64_t n_by_size[6] = {0, 0, 0, 0, 0, 0};  // unique hyperedges of size 2,3,4; [5] = size >= 5
  uint64_t n_singletons = 0;
  uint64_t n_duplicates = 0;
  uint64_t n_unique = 0;           // unique hyperedges of size >= 2
  uint64_t n_unique_members = 0;   // total members of those

  // one device block holding the arrays the build sizes (from e2 to the
  // histograms below), when they were carved from it; else each is its own
  void* arena = nullptr;
  // unique hyperedges per size, ascending tuples, first-occurrence order
  uint32_t* e2 = nullptr;
  uint32_t* e3 = nullptr;
  uint32_t* e4 = nullptr;
  // every unique hyperedge of size >= 2 (ascending members), first-occurrence order
  uint32_t* all_members = nullptr;
  unsigned long long* all_off = nullptr;   // n_unique + 1

  hm::Set64 hs2;
  hm::Set128 hs3, hs4;

  // pairwise graph: ascending neighbour rows
  uint32_t* g2_off = nullptr;   // n_nodes + 1
  uint32_t* g2_adj = nullptr;   // 2 * n2
  uint32_t* g2_eid = nullptr;   // 2 * n2: position in e2 of the pair of each adjacency entry
  // node -> incident 3-node hyperedges (indices into e3)
  uint32_t* i3_off = nullptr;
  uint32_t* i3_idx = nullptr;
  // node -> incident 4-node hyperedges (indices into e4)
  uint32_t* i4_off = nullptr;
  uint32_t* i4_idx = nullptr;
  // with bit rows: beside each incidence entry, the hyperedge's other members
  // (others3 / others4 of hm_device.h)
  uint32_t* i3_oth = nullptr;
  unsigned long long* i4_oth = nullptr;
  // adjacency bit rows of the pairwise graph (n_nodes x words), when kept
  uint32_t* bits = nullptr;
  uint32_t words = 0;

  // histogram scratch, reused by the counting calls (serialised per graph):
  // kHistCopies copies of main, sub and G2 regions of 256 counters (and 256
  // unused); zero between calls (hist_dirty: a call failed part-way and left
  // it unknown)
  unsigned long long* hist = nullptr;      // kHistCopies x kExactHistStride counters
  mutable bool hist_dirty = false;
  // the streams work on the graph was enqueued on (hm_graph_destroy releases
  // the memory in stream order when there is only one)
  mutable std::vector<hipStream_t> streams;
  // pairs inside 3-node hyperedges, sorted ((x << 32) | y), with the position
  // of their hyperedge in e3; built on first use without bit rows
  unsigned long long* pl_keys = nullptr;
  uint32_t* pl_edge = nullptr;
  // hash index over the distinct pair keys: slot = (key, start << 32 | count)
  // of the key's run in pl_keys; pl_mask + 1 slots
  unsigned long long* pl_slot = nullptr;
  unsigned long long pl_mask = 0;
  // per slot of the index: the common pairwise neighbours of its pair
  uint32_t* pl_codeg = nullptr;
  // per pair entry: the third node of its hyperedge, and that node's pairwise
  // adjacency to the pair's two nodes (bits 0 and 1)
  uint32_t* pl_third = nullptr;
  uint8_t* pl_adj = nullptr;
  uint32_t* pl_pre = nullptr;
  // 3-node subset -> 4-node hyperedges (see quad_find; q_bits = 0: not built)
  unsigned long long* q_slot = nullptr;
  unsigned long long q_mask = 0;
  uint32_t* q_fourth = nullptr;
  int q_bits = 0;   // 4 x (entries + 1) prefix counts by adjacency class
  // the 3-node hyperedges by decreasing estimated cost of their exact
  // neighbourhood count (built on first use without bit rows)
  uint32_t* b4_order = nullptr;
  // dense adjacency bit rows of the highest-degree nodes (built on first use
  // without bit rows): hub_rank[v] is v's row or -1; rows of hub_words words
  int32_t* hub_rank = nullptr;
  uint32_t* hub_bits = nullptr;
  uint32_t hub_words = 0;
  bool hub_built = false;
  // bit rows of the clique projection (n_nodes x words), allocated by the
  // first projection-baseline count and rewritten by every one
  mutable uint32_t* proj_bits = nullptr;
  // per node, built on first use without bit rows: triangles at the node, sum
  // of its neighbours' degrees, its 3-node hyperedges by pairwise pattern (8)
  unsigned long long* ns_tri = nullptr;
  unsigned long long* ns_nbr = nullptr;
  uint32_t* ns_h3 = nullptr;
  // per pair of e2 (u < w), built on first use without bit rows, 6 x n2:
  // triangles, 4-cliques and 4-cycles through it; over its common neighbours
  // x: sum of t_{ux}, sum of t_{wx}, sum of deg x
  unsigned long long* es = nullptr;
  // the unique 5-node hyperedges (ascending tuples, first-occurrence order)
  // and a hash set of their positions (slot = position + 1, 0 empty; hs5_mask
  // + 1 slots), built on first use at order 5
  uint32_t* e5 = nullptr;
  uint32_t* hs5 = nullptr;
  unsigned long long hs5_mask = 0;
  uint64_t n5 = 0;
  bool order5_built = false;
  // raw counters of the sampled counting calls (kHistCopies copies of 256),
  // then the tail and head of their work queue (the two words after one
  // unused); zero between calls
  unsigned long long* sample_hist = nullptr;
  // buffers and captured HIP graph of the batched null-model pipeline
  hm::NullPlan* null_plan = nullptr;
  // learned-proposal probabilities of the last model used with this graph
  hm::ProposalCache* proposal = nullptr;
};

namespace hm {
// Record that work on H is enqueued on st (every entry point that enqueues
// work on a graph calls this).
inline void note_use(const hm_graph* H, hipStream_t st) {
  for (hipStream_t s : H->streams)
    if (s == st) return;
  H->streams.push_back(st);
}
}  // namespace hm
