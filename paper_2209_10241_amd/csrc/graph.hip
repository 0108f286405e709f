// Building the device-resident hypergraph (ingest).
//
// A hypergraph's hyperedges form a set (Definition of a hypergraph,
// Section 3): repeated hyperedges collapse onto their first occurrence;
// singletons are ignored (the fill-in of Section 4.3 skips them).  Every
// hyperedge of size 2..4 is hashed so that fill-in checks existence in
// constant time (Section 4.3, Fig. 3b).  The pairwise graph (hyperedges of
// size 2) is kept as ascending CSR rows, plus adjacency bit rows when the
// node count is small, and every node lists its incident 3- and 4-node
// hyperedges: the neighbourhoods Algorithms 3 and 4 explore.
#include <algorithm>
#include <mutex>
#include <vector>

#include "hm_device.h"

namespace hm {
namespace {

enum : uint32_t {
  kErrEmpty = 1u,
  kErrBadId = 2u,
  kErrRepeat = 4u,
  kErrOffsets = 8u,
  // not an error of the input: two different hyperedges met in one entry of
  // the one-launch duplicate search, which the build then repeats exactly
  kErrCollide = 16u,
};

struct DevFlags {
  uint32_t err;
  uint32_t err_edge;
  unsigned long long singletons;
  unsigned long long duplicates;
};

constexpr int kRegSort = 16;
constexpr uint32_t kNetSort = 8;   // hyperedges up to this size: loaded at once, sorted by a network

// Batcher's odd-even merge sorting network for 8 values (19 comparators).
__device__ inline void sort8(uint32_t* r) {
  constexpr int kNet[19][2] = {{0, 2}, {1, 3}, {4, 6}, {5, 7}, {0, 4}, {1, 5}, {2, 6}, {3, 7}, {0, 1}, {2, 3},
                               {4, 5}, {6, 7}, {2, 4}, {3, 5}, {1, 4}, {3, 6}, {1, 2}, {3, 4}, {5, 6}};
#pragma unroll
  for (int q = 0; q < 19; ++q) {
    const uint32_t x = r[kNet[q][0]], y = r[kNet[q][1]];
    r[kNet[q][0]] = min(x, y);
    r[kNet[q][1]] = max(x, y);
  }
}

__device__ inline unsigned long long tuple_hash_start(uint32_t s) { return mix64(0x51ed270b27a3ffb1ull ^ s); }
__device__ inline unsigned long long tuple_hash_step(unsigned long long h, uint32_t x, uint32_t i) {
  return mix64(h ^ (x + 0x9e3779b97f4a7c15ull * (i + 1)));
}
__device__ inline unsigned long long tuple_hash(const uint32_t* m, uint32_t s) {
  unsigned long long h = tuple_hash_start(s);
  for (uint32_t i = 0; i < s; ++i) h = tuple_hash_step(h, m[i], i);
  return h;
}

// Up to sixteen fills in one launch.
struct FillRegions {
  void* ptr[16];
  unsigned long long count[16];
  unsigned long long value[16];
  uint32_t wide[16];   // 1: 64-bit elements, 0: 32-bit
  uint32_t n;
};

__device__ void multi_fill(const FillRegions& r) {
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint32_t k = 0; k < r.n; ++k) {
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < r.count[k]; i += stride) {
      if (r.wide[k]) static_cast<unsigned long long*>(r.ptr[k])[i] = r.value[k];
      else static_cast<uint32_t*>(r.ptr[k])[i] = uint32_t(r.value[k]);
    }
  }
}

__global__ void k_multi_fill(FillRegions r) { multi_fill(r); }

// The duplicate search of one launch: a table of (tag << 32) | index
// entries, all-ones when empty.  A hyperedge probes from its hash; an entry
// with its tag (the hash's high half under tag_mask) is taken to be its copy,
// and the entry keeps the smaller index (first occurrence).  The members are
// compared one launch later (k_first_tiles), where a meeting of two different
// hyperedges is reported (kErrCollide).
struct FastDedup {
  unsigned long long* slots;   // null: the exact search (k_dedup_insert) runs instead
  unsigned long long mask;
  unsigned long long tag_mask;
  unsigned long long* slot_of;
};

// One thread per input hyperedge: copy its members, sort them, check ids and
// repeats, record its size and hash, and (dd.slots set) enter it in the
// duplicate search.  Offsets start at 0, never decrease and stay within the
// n_members entries of members.
//
// Each hyperedge's error code (kErr* bits, 0 when valid) goes to ecode; the
// workgroups also carry out `fills` (the tables the later kernels start from;
// not the duplicate search's, which is filled before the launch).
__global__ void k_prepare(const uint32_t* __restrict__ members, const uint64_t* __restrict__ offsets,
                          uint64_t n_edges, uint64_t n_members, uint32_t n_nodes, uint32_t* __restrict__ sm,
                          uint32_t* __restrict__ size, unsigned long long* __restrict__ hash,
                          uint8_t* __restrict__ ecode, FillRegions fills, FastDedup dd) {
  // (the hyperedges first: their chain of dependent loads starts at once, and
  // the fills' stores follow it)
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n_edges;
       i += uint64_t(gridDim.x) * blockDim.x) {
    const uint64_t b = offsets[i], e = offsets[i + 1];
    uint32_t err = 0;
    if (e < b || e > n_members || (i == 0 && b != 0)) {
      err |= kErrOffsets;
      size[i] = 0;
      hash[i] = 0;
    } else {
      const uint64_t s64 = e - b;
      const uint32_t s = s64 > 0xFFFFFFFFull ? 0xFFFFFFFFu : uint32_t(s64);
      if (s == 0) err |= kErrEmpty;
      uint32_t* out = sm + b;
      unsigned long long h = 0;
      if (s <= kNetSort) {
        // every member load in flight at once; the padding (above any node
        // id) sorts last
        uint32_t r[kNetSort];
#pragma unroll
        for (uint32_t j = 0; j < kNetSort; ++j) r[j] = j < s ? members[b + j] : 0xFFFFFFFFu;
#pragma unroll
        for (uint32_t j = 0; j < kNetSort; ++j)
          if (j < s && r[j] >= n_nodes) err |= kErrBadId;
        sort8(r);
#pragma unroll
        for (uint32_t j = 0; j < kNetSort; ++j)
          if (j < s) out[j] = r[j];
#pragma unroll
        for (uint32_t j = 1; j < kNetSort; ++j)
          if (j < s && r[j] == r[j - 1]) err |= kErrRepeat;
        h = tuple_hash_start(s);
#pragma unroll
        for (uint32_t j = 0; j < kNetSort; ++j)
          if (j < s) h = tuple_hash_step(h, r[j], j);
      } else if (s <= kRegSort) {
        uint32_t r[kRegSort];
        for (uint32_t j = 0; j < s; ++j) {
          uint32_t v = members[b + j];
          if (v >= n_nodes) err |= kErrBadId;
          uint32_t k = j;
          while (k > 0 && r[k - 1] > v) {
            r[k] = r[k - 1];
            --k;
          }
          r[k] = v;
        }
        for (uint32_t j = 0; j < s; ++j) out[j] = r[j];
      } else {
        for (uint32_t j = 0; j < s; ++j) {
          uint32_t v = members[b + j];
          if (v >= n_nodes) err |= kErrBadId;
          uint32_t k = j;
          while (k > 0 && out[k - 1] > v) {
            out[k] = out[k - 1];
            --k;
          }
          out[k] = v;
        }
      }
      if (s > kNetSort) {
        for (uint32_t j = 1; j < s; ++j)
          if (out[j] == out[j - 1]) err |= kErrRepeat;
        h = tuple_hash(out, s);
      }
      size[i] = s;
      hash[i] = h;
      if (dd.slots && s >= 2) {
        const unsigned long long tag = (h >> 32) & dd.tag_mask;
        const unsigned long long mine = (tag << 32) | i;
        unsigned long long pos = h & dd.mask;
        while (true) {
          const unsigned long long cur = atomicCAS(&dd.slots[pos], kEmpty64, mine);
          if (cur == kEmpty64) break;
          if ((cur >> 32) == tag) {
            atomicMin(&dd.slots[pos], mine);
            break;
          }
          pos = (pos + 1) & dd.mask;
        }
        dd.slot_of[i] = pos;
      }
    }
    ecode[i] = uint8_t(err);
  }
  multi_fill(fills);
}

__device__ inline bool same_tuple(const uint32_t* sm, const uint64_t* off, const uint32_t* size,
                                  const unsigned long long* hash, uint64_t a, uint64_t b) {
  if (size[a] != size[b] || hash[a] != hash[b]) return false;
  const uint32_t* x = sm + off[a];
  const uint32_t* y = sm + off[b];
  for (uint32_t j = 0; j < size[a]; ++j)
    if (x[j] != y[j]) return false;
  return true;
}

// Insert every hyperedge of size >= 2 into a table whose slots hold
// (tag << 32) | index, the tag being the high half of the hyperedge's hash;
// equal tuples meet in one slot, which keeps the smallest index (first
// occurrence).  slot_of[i] records the slot of hyperedge i.
__global__ void k_dedup_insert(const uint32_t* __restrict__ sm, const uint64_t* __restrict__ off,
                               const uint32_t* __restrict__ size, const unsigned long long* __restrict__ hash,
                               uint64_t n_edges, unsigned long long* slots, unsigned long long mask,
                               unsigned long long* __restrict__ slot_of) {
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n_edges;
       i += uint64_t(gridDim.x) * blockDim.x) {
    const uint32_t si = size[i];
    const unsigned long long h = hash[i];   // (loaded with the size)
    if (si < 2) continue;
    const unsigned long long tag = h >> 32;
    const unsigned long long mine = (tag << 32) | i;
    unsigned long long pos = h & mask;
    while (true) {
      const unsigned long long cur = atomicCAS(&slots[pos], kEmpty64, mine);
      if (cur == kEmpty64) break;
      if ((cur >> 32) == tag && same_tuple(sm, off, size, hash, uint32_t(cur), i)) {
        atomicMin(&slots[pos], mine);
        break;
      }
      pos = (pos + 1) & mask;
    }
    slot_of[i] = pos;
  }
}

// Ingest works in tiles of 256 input hyperedges: k_first_tiles marks first
// occurrences and counts, per tile, the unique hyperedges (all, of size 2, 3,
// 4) and their members; k_tile_scan turns the tile counts into tile offsets;
// k_gather_tiles recomputes each hyperedge's position inside its tile and
// writes it out.
constexpr uint32_t kTile = 256;
constexpr int kTileN = 5;   // unique, unique of size 2, 3, 4, members of the unique
// per tile: the kTileN counters above, then singletons, repeats (collapsed
// duplicates), the OR of the error codes and the first erroneous index
constexpr int kTileS = kTileN + 4;
enum : int { kTSingles = kTileN, kTDups = kTileN + 1, kTErr = kTileN + 2, kTErrMin = kTileN + 3 };
// up to this many tiles, a one-pass build lets every workgroup of the gather
// sum the counts of the tiles before it instead of running k_tile_scan
constexpr uint64_t kSelfOffsetTiles = 1024;

// Per-thread contribution of hyperedge i to the five tile counters.
__device__ inline void tile_terms(uint32_t first, uint32_t s, uint32_t t[kTileN]) {
  t[0] = first;
  t[1] = first && s == 2;
  t[2] = first && s == 3;
  t[3] = first && s == 4;
  t[4] = first ? s : 0;
}

// Node degrees of the pairwise graph and of the 3- and 4-node incidence
// lists are counted in R copies per node (R a power of two, node-major), so
// that no counter takes more than about 1/R of its node's incidences: a
// hyperedge counts in, and later fills through, the copy this hash of its
// sorted members picks.
__device__ inline uint32_t degree_copy(const uint32_t* m, uint32_t s, uint32_t R) {
  uint32_t h = 0x9E3779B9u * s;
  for (uint32_t j = 0; j < s; ++j) h = (h ^ m[j]) * 0x85EBCA6Bu;
  return (h >> 16) & (R - 1);
}

struct Degrees {
  uint32_t *deg2, *deg3, *deg4;
  uint32_t R;
};

// Each first occurrence of size 2, 3 or 4 also counts its members' degrees
// (deg).  (verify: the table came from the one-launch search, so a hyperedge
// that met an earlier one compares their members, and a meeting of two
// different hyperedges sets kErrCollide)
__global__ void __launch_bounds__(kTile) k_first_tiles(const uint32_t* __restrict__ size, uint64_t n_edges,
                                                        const unsigned long long* __restrict__ slots,
                                                        const unsigned long long* __restrict__ slot_of,
                                                        const uint8_t* __restrict__ ecode,
                                                        uint8_t* __restrict__ first_out,
                                                        uint32_t* __restrict__ tile_cnt, bool verify,
                                                        const uint32_t* __restrict__ sm,
                                                        const uint64_t* __restrict__ off,
                                                        const unsigned long long* __restrict__ hash,
                                                        Degrees deg) {
  __shared__ uint32_t part[kTileS][kTile / kWave];
  const uint64_t i = uint64_t(blockIdx.x) * kTile + threadIdx.x;
  uint32_t first = 0, s = 0, singles = 0, dups = 0, err = 0, err_at = 0xFFFFFFFFu;
  if (i < n_edges) {
    // (slot_of[i] and the member offset are loaded with the others; they are
    // meaningful when s >= 2)
    s = size[i];
    err = ecode[i];
    const unsigned long long so = slot_of[i];
    const uint64_t at = off[i];
    if (err) err_at = uint32_t(i);
    if (s >= 2) {
      // the entry's holder and the members go out together
      const uint32_t holder = uint32_t(slots[so]);
      uint32_t mm[4];
#pragma unroll
      for (uint32_t j = 0; j < 4; ++j) mm[j] = j < s && s <= 4 ? sm[at + j] : 0u;
      first = holder == uint32_t(i);
      dups = !first;
      const bool collide = verify && !first && !same_tuple(sm, off, size, hash, holder, i);
      // (only a hyperedge that passed validation: its ids are below n)
      if (first && s <= 4 && !err) {
        uint32_t* d = s == 2 ? deg.deg2 : s == 3 ? deg.deg3 : deg.deg4;
        const uint32_t cp = degree_copy(mm, s, deg.R);
#pragma unroll
        for (uint32_t j = 0; j < 4; ++j)
          if (j < s) atomicAdd(&d[uint64_t(mm[j]) * deg.R + cp], 1u);
      }
      if (collide) err |= kErrCollide;
    } else if (s == 1) {
      singles = 1;
    }
    first_out[i] = uint8_t(first);
  }
  uint32_t t[kTileN];
  tile_terms(first, s, t);
  const int wv = threadIdx.x / kWave;
  const uint32_t lane = threadIdx.x & (kWave - 1);
  for (int k = 0; k < kTileN; ++k) {
    uint32_t w;
    (void)wave_exclusive_scan(t[k], &w);
    if (lane == 0) part[k][wv] = w;
  }
  singles = wave_sum_u32(singles);
  dups = wave_sum_u32(dups);
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) {
    err |= __shfl_xor(err, o, kWave);
    err_at = min(err_at, uint32_t(__shfl_xor(err_at, o, kWave)));
  }
  if (lane == 0) {
    part[kTSingles][wv] = singles;
    part[kTDups][wv] = dups;
    part[kTErr][wv] = err;
    part[kTErrMin][wv] = err_at;
  }
  __syncthreads();
  if (threadIdx.x < kTileS) {
    uint32_t x = threadIdx.x == kTErrMin ? 0xFFFFFFFFu : 0u;
    for (int q = 0; q < int(kTile / kWave); ++q) {
      const uint32_t y = part[threadIdx.x][q];
      x = threadIdx.x == kTErr ? (x | y) : (threadIdx.x == kTErrMin ? min(x, y) : x + y);
    }
    tile_cnt[uint64_t(blockIdx.x) * kTileS + threadIdx.x] = x;
  }
}

// The validation summary of the tiles a workgroup's threads take (thread:
// t_first, t_first + t_step, ... below t_end), reduced over the workgroup:
// singletons, repeats, error bits, first erroneous index.  Every thread must
// call it and receives the result.
__device__ DevFlags tile_flags(const uint32_t* __restrict__ tile_cnt, uint64_t t_first, uint64_t t_end,
                               uint64_t t_step) {
  __shared__ unsigned long long s_single, s_dup;
  __shared__ uint32_t s_err, s_min;
  if (threadIdx.x == 0) {
    s_single = 0;
    s_dup = 0;
    s_err = 0;
    s_min = 0xFFFFFFFFu;
  }
  __syncthreads();
  unsigned long long sg = 0, dp = 0;
  uint32_t er = 0, mn = 0xFFFFFFFFu;
  for (uint64_t t = t_first; t < t_end; t += t_step) {
    const uint32_t* c = tile_cnt + t * kTileS;
    sg += c[kTSingles];
    dp += c[kTDups];
    er |= c[kTErr];
    mn = min(mn, c[kTErrMin]);
  }
  if (sg) atomicAdd(&s_single, sg);
  if (dp) atomicAdd(&s_dup, dp);
  if (er) atomicOr(&s_err, er);
  if (mn != 0xFFFFFFFFu) atomicMin(&s_min, mn);
  __syncthreads();
  DevFlags f;
  f.err = s_err;
  f.err_edge = s_min;
  f.singletons = s_single;
  f.duplicates = s_dup;
  return f;
}

// What the build reads back once: validation flags and the five totals.
struct Report {
  DevFlags flags;
  unsigned long long totals[kTileN];
  uint32_t ready;   // set to 1 (after the fields above) by the kernel that writes them
  uint32_t pad;
};

// Publish a report written by this workgroup: every thread of the workgroup
// calls this (wrote: it wrote part of the report), and thread 0 sets `ready`
// once those writes are visible to the host.
__device__ inline void publish_report(Report* out, bool wrote) {
  if (wrote) __threadfence_system();
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(&out->ready, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Exclusive scan of the tiles' position counters in place; the five totals
// and the validation summary go to the report (pinned host memory), the
// totals and the error bits also to dev_totals (kTileN + 1 words) for the
// kernels that follow.  One workgroup of 1024: thread t takes a run of
// consecutive tiles, the runs' sums are scanned across the workgroup, and each
// thread then writes the offsets of its run.  Every count is below 2^32 (so
// are the incidences).
__global__ void __launch_bounds__(1024) k_tile_scan(uint32_t* __restrict__ tile_cnt, uint64_t n_tiles, Report* out,
                                                    unsigned long long* __restrict__ dev_totals) {
  __shared__ uint32_t wsum[kTileN][1024 / kWave];
  const uint32_t lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  const uint64_t per = (n_tiles + 1023) / 1024;
  const uint64_t t0 = min(n_tiles, uint64_t(threadIdx.x) * per), t1 = min(n_tiles, t0 + per);
  const DevFlags f = tile_flags(tile_cnt, t0, t1, 1);
  uint32_t pre[kTileN];
#pragma unroll
  for (int k = 0; k < kTileN; ++k) pre[k] = 0;
  for (uint64_t t = t0; t < t1; ++t) {
#pragma unroll
    for (int k = 0; k < kTileN; ++k) pre[k] += tile_cnt[t * kTileS + k];
  }
#pragma unroll
  for (int k = 0; k < kTileN; ++k) {
    uint32_t tot;
    pre[k] = wave_exclusive_scan(pre[k], &tot);
    if (lane == 0) wsum[k][wv] = tot;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kTileN; ++k)
    for (uint32_t q = 0; q < wv; ++q) pre[k] += wsum[k][q];
  for (uint64_t t = t0; t < t1; ++t) {
#pragma unroll
    for (int k = 0; k < kTileN; ++k) {
      const uint32_t x = tile_cnt[t * kTileS + k];
      tile_cnt[t * kTileS + k] = pre[k];
      pre[k] += x;
    }
  }
  if (threadIdx.x == 1023) {
#pragma unroll
    for (int k = 0; k < kTileN; ++k) {
      out->totals[k] = pre[k];
      dev_totals[k] = pre[k];
    }
  }
  if (threadIdx.x == 0) {
    out->flags = f;
    dev_totals[kTileN] = f.err;
  }
  publish_report(out, threadIdx.x == 0 || threadIdx.x == 1023);
}

// Write the unique hyperedges out, in first-occurrence order, with everything
// that only needs them once: the strata e2/e3/e4, the list of all unique
// hyperedges with its member offsets, the hash-set entries, the adjacency bit
// rows (when kept) and the node degrees of the pairwise graph and of the
// incidence lists.
struct GatherOut {
  uint32_t *e2, *e3, *e4, *all_members;
  unsigned long long* all_off;
  Set64 hs2;
  Set128 hs3, hs4;
  uint32_t* bits;
  uint32_t W;
  // scan: three workgroups after the tiles' scan the degree arrays (counted
  // by k_first_tiles) into the row offsets o2, o3, o4 (n + 1 each) and the
  // fill cursors c3, c4 (n * R each)
  bool scan;
  Degrees deg;
  uint32_t n;
  uint32_t *o2, *o3, *o4, *c3, *c4;
  // self_offsets: tile_cnt holds the raw tile counters (no k_tile_scan ran);
  // each workgroup sums those of the tiles before it, and workgroup 0 also
  // writes the report and dev_totals.  Otherwise dev_totals holds what
  // k_tile_scan wrote.  Nothing is written when the input is invalid.
  bool self_offsets;
  Report* report;
  unsigned long long* dev_totals;
  // the one-launch duplicate search's table, returned to all-ones: each
  // first occurrence clears its entry (null: nothing to clear)
  unsigned long long* dedup_clear;
  const unsigned long long* slot_of;
};

// Exclusive scan of one degree array d (n nodes x R copies) by the calling
// workgroup: row offsets o[v] = (scan at v * R) for v = 0..n and, when c is
// not null, the fill cursor of every (node, copy).  Thread t takes a run of
// at most RUN consecutive counters (n * R <= RUN * blockDim.x), loaded at
// once; wsum is LDS of blockDim.x / kWave words.
template <uint32_t RUN>
__device__ void scan_degree_array(const uint32_t* __restrict__ d, uint32_t* __restrict__ o,
                                  uint32_t* __restrict__ c, uint32_t n, uint32_t R, uint32_t* wsum) {
  const uint32_t lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  const uint32_t m = n * R;
  const uint32_t per = (m + blockDim.x - 1) / blockDim.x;
  const uint32_t t0 = min(m, threadIdx.x * per), t1 = min(m, t0 + per);
  uint32_t x[RUN];
  uint32_t sum = 0;
#pragma unroll
  for (uint32_t j = 0; j < RUN; ++j) x[j] = t0 + j < t1 ? d[t0 + j] : 0u;
#pragma unroll
  for (uint32_t j = 0; j < RUN; ++j) sum += x[j];
  uint32_t tot;
  uint32_t pre = wave_exclusive_scan(sum, &tot);
  if (lane == 0) wsum[wv] = tot;
  __syncthreads();
  for (uint32_t q = 0; q < wv; ++q) pre += wsum[q];
#pragma unroll
  for (uint32_t j = 0; j < RUN; ++j) {
    const uint32_t t = t0 + j;
    if (t < t1) {
      if (c) c[t] = pre;
      if ((t & (R - 1)) == 0) o[t / R] = pre;
      pre += x[j];
    }
  }
  // (the last thread's sum includes every run: the total)
  if (threadIdx.x == blockDim.x - 1) o[n] = pre;
}
// counters per thread of the gather's scan workgroups
constexpr uint32_t kGatherScanRun = 32;
constexpr uint64_t kGatherScanMax = uint64_t(kGatherScanRun) * kTile;   // n * R at most

__global__ void __launch_bounds__(kTile) k_gather_tiles(const uint32_t* __restrict__ sm,
                                                         const uint64_t* __restrict__ off,
                                                         const uint32_t* __restrict__ size, uint64_t n_edges,
                                                         const uint8_t* __restrict__ first_in,
                                                         const uint32_t* __restrict__ tile_off,
                                                         GatherOut g) {
  __shared__ uint32_t part[kTileN][kTile / kWave];
  __shared__ uint32_t red[2 * kTileN][kTile / kWave];
  __shared__ uint32_t base[kTileN];
  __shared__ unsigned long long total[kTileN];
  const int wv = threadIdx.x / kWave;
  const uint32_t lane = threadIdx.x & (kWave - 1);
  __shared__ uint32_t bad;
  const uint64_t n_tiles = (n_edges + kTile - 1) / kTile;
  if (blockIdx.x >= n_tiles) {
    // a degree scan (g.scan): array blockIdx.x - n_tiles
    const uint32_t a = uint32_t(blockIdx.x - n_tiles);
    scan_degree_array<kGatherScanRun>(a == 0 ? g.deg.deg2 : a == 1 ? g.deg.deg3 : g.deg.deg4,
                                      a == 0 ? g.o2 : a == 1 ? g.o3 : g.o4, a == 0 ? nullptr : a == 1 ? g.c3 : g.c4,
                                      g.n, g.deg.R, part[0]);
    return;
  }
  // The hyperedge's flags and, for a first occurrence, its first four
  // members go out before the tile counters are summed, so that their round
  // trips overlap (the rest of a larger hyperedge is read later, one by one).
  const uint64_t i = uint64_t(blockIdx.x) * kTile + threadIdx.x;
  uint32_t first = 0, s = 0;
  uint64_t at = 0;   // the hyperedge's members in sm
  unsigned long long so = 0;
  if (i < n_edges) {
    first = first_in[i];
    s = size[i];
    at = off[i];
    if (g.dedup_clear) so = g.slot_of[i];   // (meaningful when first)
  }
  uint32_t mm[4];
#pragma unroll
  for (uint32_t j = 0; j < 4; ++j) mm[j] = first && j < s ? sm[at + j] : 0u;
  if (g.self_offsets) {
    // every counter of the tiles a thread takes in one round of loads: the
    // five position counters, and the validation summary (singletons,
    // repeats, error bits, first erroneous index)
    __shared__ uint32_t fred[4][kTile / kWave];
    uint32_t before[kTileN], all[kTileN];
#pragma unroll
    for (int k = 0; k < kTileN; ++k) before[k] = all[k] = 0;
    uint32_t sg = 0, dp = 0, er = 0, mn = 0xFFFFFFFFu;
    for (uint64_t t = threadIdx.x; t < n_tiles; t += kTile) {
      uint32_t x[kTileS];
#pragma unroll
      for (int k = 0; k < kTileS; ++k) x[k] = tile_off[t * kTileS + k];
#pragma unroll
      for (int k = 0; k < kTileN; ++k) {
        all[k] += x[k];
        if (t < blockIdx.x) before[k] += x[k];
      }
      sg += x[kTSingles];
      dp += x[kTDups];
      er |= x[kTErr];
      mn = min(mn, x[kTErrMin]);
    }
#pragma unroll
    for (int k = 0; k < kTileN; ++k) {
      const uint32_t b = wave_sum_u32(before[k]), a = wave_sum_u32(all[k]);
      if (lane == 0) {
        red[k][wv] = b;
        red[kTileN + k][wv] = a;
      }
    }
    sg = wave_sum_u32(sg);
    dp = wave_sum_u32(dp);
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
      er |= __shfl_xor(er, o, kWave);
      mn = min(mn, uint32_t(__shfl_xor(mn, o, kWave)));
    }
    if (lane == 0) {
      fred[0][wv] = sg;
      fred[1][wv] = dp;
      fred[2][wv] = er;
      fred[3][wv] = mn;
    }
    __syncthreads();
    DevFlags f;
    f.singletons = 0;
    f.duplicates = 0;
    f.err = 0;
    f.err_edge = 0xFFFFFFFFu;
    for (int q = 0; q < kTile / kWave; ++q) {
      f.singletons += fred[0][q];
      f.duplicates += fred[1][q];
      f.err |= fred[2][q];
      f.err_edge = min(f.err_edge, fred[3][q]);
    }
    if (threadIdx.x < 2 * kTileN) {
      uint32_t x = 0;
      for (int q = 0; q < kTile / kWave; ++q) x += red[threadIdx.x][q];
      if (threadIdx.x < kTileN) {
        base[threadIdx.x] = x;
      } else {
        total[threadIdx.x - kTileN] = x;
        if (blockIdx.x == 0) {
          g.report->totals[threadIdx.x - kTileN] = x;
          g.dev_totals[threadIdx.x - kTileN] = x;
        }
      }
    }
    if (threadIdx.x == 0) {
      bad = f.err;
      if (blockIdx.x == 0) {
        g.report->flags = f;
        g.dev_totals[kTileN] = f.err;
      }
    }
    if (blockIdx.x == 0)
      publish_report(g.report, threadIdx.x == 0 || (threadIdx.x >= kTileN && threadIdx.x < 2 * kTileN));
    __syncthreads();
  } else {
    if (threadIdx.x < kTileN) {
      base[threadIdx.x] = tile_off[uint64_t(blockIdx.x) * kTileS + threadIdx.x];
      total[threadIdx.x] = g.dev_totals[threadIdx.x];
    }
    if (threadIdx.x == 0) bad = uint32_t(g.dev_totals[kTileN]);
    __syncthreads();
  }
  if (bad) return;
  uint32_t t[kTileN];
  tile_terms(first, s, t);
  uint32_t pre[kTileN];
  for (int k = 0; k < kTileN; ++k) {
    uint32_t tot;
    pre[k] = wave_exclusive_scan(t[k], &tot);
    if (lane == 0) part[k][wv] = tot;
  }
  __syncthreads();
  if (!first) return;
  if (g.dedup_clear) g.dedup_clear[so] = kEmpty64;
  unsigned long long pos[kTileN];
  for (int k = 0; k < kTileN; ++k) {
    unsigned long long p = base[k] + pre[k];
    for (int q = 0; q < wv; ++q) p += part[k][q];
    pos[k] = p;
  }
  const uint32_t* m = sm + at;
#pragma unroll
  for (uint32_t j = 0; j < 4; ++j)
    if (j < s) g.all_members[pos[4] + j] = mm[j];
  for (uint32_t j = 4; j < s; ++j) g.all_members[pos[4] + j] = m[j];
  g.all_off[pos[0]] = pos[4];
  if (pos[0] + 1 == total[0]) g.all_off[total[0]] = total[4];
  if (s == 2) {
    const uint32_t a = mm[0], b = mm[1];
    g.e2[2 * pos[1]] = a;
    g.e2[2 * pos[1] + 1] = b;
    const unsigned long long key = key2(a, b);
    unsigned long long h = mix64(key) & g.hs2.mask;
    while (atomicCAS(g.hs2.slot + h, kEmpty64, key) != kEmpty64) h = (h + 1) & g.hs2.mask;
    if (g.bits) {
      atomicOr(&g.bits[uint64_t(a) * g.W + (b >> 5)], 1u << (b & 31));
      atomicOr(&g.bits[uint64_t(b) * g.W + (a >> 5)], 1u << (a & 31));
    }
  } else if (s == 3 || s == 4) {
    uint32_t* e = s == 3 ? g.e3 + 3 * pos[2] : g.e4 + 4 * pos[3];
#pragma unroll
    for (uint32_t j = 0; j < 4; ++j)
      if (j < s) e[j] = mm[j];
    const Key128 key = s == 3 ? key3(mm[0], mm[1], mm[2]) : key4(mm[0], mm[1], mm[2], mm[3]);
    const Set128& set = s == 3 ? g.hs3 : g.hs4;
    unsigned long long h = hash128(key) & set.mask;
    while (atomicCAS(set.slot + 2 * h, kEmpty64, key.hi) != kEmpty64) h = (h + 1) & set.mask;
    set.slot[2 * h + 1] = key.lo;
  }
}

// Exclusive scans of the three degree arrays (n nodes x R copies) into row
// offsets o[v] = (scan at v * R), n + 1 entries, and, for the incidence lists,
// fill cursors c of every (node, copy).  One workgroup of 1024 per array:
// thread t takes a run of consecutive counters, the runs' sums are scanned
// across the workgroup, and each thread then writes the results of its run.
// Runs of at most kScanRun counters are loaded at once and kept in
// registers.
constexpr uint32_t kScanRun = 8;
__global__ void __launch_bounds__(1024) k_scan_degrees(const uint32_t* __restrict__ d0, uint32_t* __restrict__ o0,
                                                       const uint32_t* __restrict__ d1, uint32_t* __restrict__ o1,
                                                       uint32_t* __restrict__ c1, const uint32_t* __restrict__ d2,
                                                       uint32_t* __restrict__ o2, uint32_t* __restrict__ c2, uint32_t n,
                                                       uint32_t R) {
  __shared__ uint32_t wsum[1024 / kWave];
  const uint32_t* d = blockIdx.x == 0 ? d0 : blockIdx.x == 1 ? d1 : d2;
  uint32_t* o = blockIdx.x == 0 ? o0 : blockIdx.x == 1 ? o1 : o2;
  uint32_t* c = blockIdx.x == 0 ? nullptr : blockIdx.x == 1 ? c1 : c2;
  const uint32_t lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  const uint32_t m = n * R;
  const uint32_t per = (m + 1023) / 1024;
  const uint32_t t0 = min(m, threadIdx.x * per), t1 = min(m, t0 + per);
  const bool short_run = per <= kScanRun;
  uint32_t x[kScanRun];
  uint32_t sum = 0;
  if (short_run) {
#pragma unroll
    for (uint32_t j = 0; j < kScanRun; ++j) x[j] = t0 + j < t1 ? d[t0 + j] : 0u;
#pragma unroll
    for (uint32_t j = 0; j < kScanRun; ++j) sum += x[j];
  } else {
    for (uint32_t t = t0; t < t1; ++t) sum += d[t];
  }
  uint32_t tot;
  uint32_t pre = wave_exclusive_scan(sum, &tot);
  if (lane == 0) wsum[wv] = tot;
  __syncthreads();
  for (uint32_t q = 0; q < wv; ++q) pre += wsum[q];
  if (short_run) {
#pragma unroll
    for (uint32_t j = 0; j < kScanRun; ++j) {
      const uint32_t t = t0 + j;
      if (t < t1) {
        if (c) c[t] = pre;
        if ((t & (R - 1)) == 0) o[t / R] = pre;
        pre += x[j];
      }
    }
  } else {
    for (uint32_t t = t0; t < t1; ++t) {
      const uint32_t v = d[t];
      if (c) c[t] = pre;
      if ((t & (R - 1)) == 0) o[t / R] = pre;
      pre += v;
    }
  }
  if (threadIdx.x == 1023) o[n] = pre;
}

// Row offsets o[v] = s[v * R] for v = 0..n from scans s of n * R + 1 entries
// (the last one the total), for three arrays.
__global__ void k_offsets_of_copies(const uint32_t* __restrict__ s0, uint32_t* __restrict__ o0,
                                    const uint32_t* __restrict__ s1, uint32_t* __restrict__ o1,
                                    const uint32_t* __restrict__ s2, uint32_t* __restrict__ o2, uint32_t n,
                                    uint32_t R) {
  for (uint64_t v = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; v <= n; v += uint64_t(gridDim.x) * blockDim.x) {
    o0[v] = s0[v * R];
    o1[v] = s1[v * R];
    o2[v] = s2[v * R];
  }
}

// Sorted pairwise rows read off the adjacency bit rows: one wavefront per
// node, 64 words at a time, set bits written in ascending order (workgroup
// `block` of `n_blocks`).
__device__ void rows_from_bits(const uint32_t* __restrict__ bits, uint32_t n, uint32_t W,
                               const uint32_t* __restrict__ row_off, uint32_t* __restrict__ adj, uint32_t block,
                               uint32_t n_blocks) {
  const uint32_t lane = threadIdx.x & (kWave - 1);
  const uint64_t wave = (uint64_t(block) * blockDim.x + threadIdx.x) / kWave;
  const uint64_t n_waves = uint64_t(n_blocks) * blockDim.x / kWave;
  for (uint64_t x = wave; x < n; x += n_waves) {
    uint32_t base = row_off[x];
    const uint32_t* row = bits + x * W;
    for (uint32_t w0 = 0; w0 < W; w0 += kWave) {
      uint32_t word = w0 + lane < W ? row[w0 + lane] : 0u;
      uint32_t tot;
      uint32_t p = base + wave_exclusive_scan(__popc(word), &tot);
      while (word) {
        adj[p++] = ((w0 + lane) << 5) | uint32_t(__ffs(word) - 1);
        word &= word - 1;
      }
      base += tot;
    }
  }
}

// Incidence lists of the 3- and 4-node hyperedges (positions in any order):
// a hyperedge fills through the cursor of copy degree_copy() of each member,
// the copy its degree was counted in (workgroup `block` of `n_blocks`).
// With bit rows (oth3, oth4 not null) each entry also gets the hyperedge's
// other members.
__device__ void inc_fill(const uint32_t* __restrict__ e3, uint64_t n3, uint32_t* cur3, uint32_t* idx3,
                         const uint32_t* __restrict__ e4, uint64_t n4, uint32_t* cur4, uint32_t* idx4, uint32_t R,
                         uint32_t* __restrict__ oth3, unsigned long long* __restrict__ oth4, uint32_t block,
                         uint32_t n_blocks) {
  for (uint64_t i = uint64_t(block) * blockDim.x + threadIdx.x; i < n3 + n4; i += uint64_t(n_blocks) * blockDim.x) {
    // (the cursors of all members are taken before any entry is written, so
    // that the atomics go out together)
    if (i < n3) {
      const uint32_t m[3] = {e3[3 * i], e3[3 * i + 1], e3[3 * i + 2]};
      const uint32_t cp = degree_copy(m, 3, R);
      uint32_t at[3];
#pragma unroll
      for (int j = 0; j < 3; ++j) at[j] = atomicAdd(&cur3[uint64_t(m[j]) * R + cp], 1u);
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        idx3[at[j]] = uint32_t(i);
        if (oth3) oth3[at[j]] = others3(m, j);
      }
    } else {
      const uint64_t q = i - n3;
      const uint32_t m[4] = {e4[4 * q], e4[4 * q + 1], e4[4 * q + 2], e4[4 * q + 3]};
      const uint32_t cp = degree_copy(m, 4, R);
      uint32_t at[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) at[j] = atomicAdd(&cur4[uint64_t(m[j]) * R + cp], 1u);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        idx4[at[j]] = uint32_t(q);
        if (oth4) oth4[at[j]] = others4(m, j);
      }
    }
  }
}

// (the counts of 3- and 4-node hyperedges are totals[2] and totals[3];
// nothing is written when the input is invalid, totals[kTileN] != 0)
__global__ void k_inc_fill(const uint32_t* __restrict__ e3, uint32_t* cur3, uint32_t* idx3,
                           const uint32_t* __restrict__ e4, uint32_t* cur4, uint32_t* idx4, uint32_t R,
                           const unsigned long long* __restrict__ totals) {
  if (totals[kTileN]) return;
  inc_fill(e3, totals[2], cur3, idx3, e4, totals[3], cur4, idx4, R, nullptr, nullptr, blockIdx.x, gridDim.x);
}

// Pairwise rows from the bit rows (workgroups [0, row_blocks)) and the
// incidence lists (the rest) in one launch.
__global__ void k_rows_and_incidence(const uint32_t* __restrict__ bits, uint32_t n, uint32_t W,
                                     const uint32_t* __restrict__ row_off, uint32_t* __restrict__ adj,
                                     uint32_t row_blocks, const uint32_t* __restrict__ e3, uint32_t* cur3,
                                     uint32_t* idx3, const uint32_t* __restrict__ e4, uint32_t* cur4, uint32_t* idx4,
                                     uint32_t R, uint32_t* oth3, unsigned long long* oth4,
                                     const unsigned long long* __restrict__ totals) {
  if (totals[kTileN]) return;
  if (blockIdx.x < row_blocks)
    rows_from_bits(bits, n, W, row_off, adj, blockIdx.x, row_blocks);
  else
    inc_fill(e3, totals[2], cur3, idx3, e4, totals[3], cur4, idx4, R, oth3, oth4, blockIdx.x - row_blocks,
             gridDim.x - row_blocks);
}

__global__ void k_pair_keys(const uint32_t* __restrict__ e2, uint64_t n, int bits_per_node,
                            unsigned long long* keys, uint32_t* vals) {
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += uint64_t(gridDim.x) * blockDim.x) {
    const uint32_t a = e2[2 * i], b = e2[2 * i + 1];
    keys[2 * i] = ((unsigned long long)a << bits_per_node) | b;
    keys[2 * i + 1] = ((unsigned long long)b << bits_per_node) | a;
    vals[2 * i] = uint32_t(i);
    vals[2 * i + 1] = uint32_t(i);
  }
}

__global__ void k_pair_adj(const unsigned long long* __restrict__ keys, uint64_t n, unsigned long long low_mask,
                           uint32_t* adj) {
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += uint64_t(gridDim.x) * blockDim.x)
    adj[i] = uint32_t(keys[i] & low_mask);
}

unsigned grid_for(uint64_t n, unsigned block = 256) {
  uint64_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > 16384) g = 16384;
  return unsigned(g);
}

// Arrays carved from one device block, each 256-byte aligned: one call to the
// caching allocator instead of one per array (the build's host time before
// its first launch is mostly such calls).  Above kCarveMaxBytes in all, where
// a power-of-two block would waste much memory and the calls cost little
// beside the work, each array gets a block of its own.
constexpr size_t kCarveMaxBytes = size_t(64) << 20;
struct Carve {
  std::vector<std::pair<void**, size_t>> parts;
  template <typename T>
  void add(T** p, uint64_t count) {
    parts.emplace_back(reinterpret_cast<void**>(p), (size_t(count ? count : 1) * sizeof(T) + 255) & ~size_t(255));
  }
  // sets every added array; the blocks taken go to *blocks (one when carved)
  int take(std::vector<void*>* blocks) {
    size_t total = 0;
    for (auto& q : parts) total += q.second;
    if (total <= kCarveMaxBytes) {
      void* base = nullptr;
      HM_TRY(dalloc(&base, total));
      blocks->push_back(base);
      char* at = static_cast<char*>(base);
      for (auto& q : parts) {
        *q.first = at;
        at += q.second;
      }
    } else {
      for (auto& q : parts) {
        HM_TRY(dalloc(q.first, q.second));
        blocks->push_back(*q.first);
      }
    }
    parts.clear();
    return HM_OK;
  }
};

// RAII holder for temporary device buffers of the build, released after the
// work enqueued on the build's stream
struct Temps {
  hipStream_t st;
  std::vector<void*> ptrs;
  Carve staged;
  explicit Temps(hipStream_t s) : st(s) {}
  ~Temps() { dfree_on(ptrs.data(), ptrs.size(), st); }
  template <typename T>
  int get(T** p, uint64_t count) {
    void* q = nullptr;
    HM_TRY(dalloc(&q, size_t(count ? count : 1) * sizeof(T)));
    ptrs.push_back(q);
    *p = static_cast<T*>(q);
    return HM_OK;
  }
  // stage(): set by the next commit(), which carves every staged array from one block
  template <typename T>
  void stage(T** p, uint64_t count) {
    staged.add(p, count);
  }
  int commit() { return staged.take(&ptrs); }
};

template <typename T>
int owned(T** p, uint64_t count) {
  void* q = nullptr;
  HM_TRY(dalloc(&q, size_t(count ? count : 1) * sizeof(T)));
  *p = static_cast<T*>(q);
  return HM_OK;
}

int node_bits(uint32_t n_nodes) {
  int b = 1;
  while (b < 32 && (1ull << b) < n_nodes) ++b;
  return b;
}

// Copies of each node's degree counters (see GatherOut): a power of two up to
// 16, with at most 2^22 counters per array.
uint32_t degree_copies(uint64_t n_nodes) {
  uint32_t R = 1;
  while (R < 16 && n_nodes * R * 2 <= (1ull << 22)) R *= 2;
  return R;
}

// The report lands in pinned host memory, taken from a pool kept for the
// process.

std::mutex g_report_mu;
std::vector<Report*> g_report_pool;

struct PinnedReport {
  Report* p = nullptr;
  hipStream_t st = nullptr;
  bool pending = false;   // a kernel enqueued on st may still write to it
  int take() {
    {
      std::lock_guard<std::mutex> lock(g_report_mu);
      if (!g_report_pool.empty()) {
        p = g_report_pool.back();
        g_report_pool.pop_back();
        return HM_OK;
      }
    }
    void* q = nullptr;
    // fine-grained: the host reads it while the kernels that write it run
    if (hipHostMalloc(&q, sizeof(Report), hipHostMallocCoherent) != hipSuccess) {
      (void)hipGetLastError();
      set_error("pinned host allocation failed");
      return HM_ENOMEM;
    }
    p = static_cast<Report*>(q);
    return HM_OK;
  }
  ~PinnedReport() {
    if (!p) return;
    if (pending) (void)hipStreamSynchronize(st);
    std::lock_guard<std::mutex> lock(g_report_mu);
    g_report_pool.push_back(p);
  }
};

// Wait until a kernel on `st` sets *ready (a word of fine-grained host
// memory).  The stream is queried now and then, so that the wait ends with an
// error when it fails or drains without setting the word.
int wait_ready(const uint32_t* ready, hipStream_t st) {
  for (uint64_t spin = 0;; ++spin) {
    if (__atomic_load_n(ready, __ATOMIC_ACQUIRE)) return HM_OK;
    if ((spin & 1023) == 1023) {
      const hipError_t e = hipStreamQuery(st);
      if (e == hipSuccess) {
        if (__atomic_load_n(ready, __ATOMIC_ACQUIRE)) return HM_OK;
        set_error("the build's report was not written");
        return HM_EINTERNAL;
      }
      if (e != hipErrorNotReady) {
        (void)hipGetLastError();
        set_error("HIP error while building the graph: %s", hipGetErrorString(e));
        return HM_EDEVICE;
      }
    }
  }
}

// Fills gathered into one launch.
struct FillList {
  FillRegions r{};
  void add(void* p, unsigned long long n, unsigned long long v, uint32_t wide) {
    r.ptr[r.n] = p;
    r.count[r.n] = n;
    r.value[r.n] = v;
    r.wide[r.n] = wide;
    ++r.n;
  }
  void launch(hipStream_t st) {
    unsigned long long most = 0;
    for (uint32_t k = 0; k < r.n; ++k) most = std::max(most, r.count[k]);
    k_multi_fill<<<grid_for(most), 256, 0, st>>>(r);
  }
};

// The build.  Graphs that keep bit rows and have at most one_pass_max_edges()
// input hyperedges are built in one pass: every buffer whose size depends on
// the unique counts is sized by an upper bound (E per stratum, the hash sets
// by E), all kernels are enqueued, and the host waits once at the end.  Other
// graphs wait after the counting pass and size everything exactly.  Kernels
// after validation read the counts from the device and do nothing when the
// input is invalid.
// build() returns this when two different hyperedges met in the one-launch
// duplicate search; the caller builds again with exact_dedup.
constexpr int kRetryExactDedup = 1;

int build(hm_graph* H, const uint32_t* members_in, const uint64_t* offsets_in, uint64_t n_edges, uint64_t n_members,
          int mem_kind, hipStream_t st, bool exact_dedup) {
  Temps tmp(st);
  if (n_members > 0xFFFFFFFFull) {
    set_error("more than 2^32-1 incidences are not supported");
    return HM_EUNSUPPORTED;
  }
  const uint32_t* members = members_in;
  const uint64_t* offsets = offsets_in;
  if (mem_kind == HM_MEM_HOST) {
    uint32_t* dm = nullptr;
    uint64_t* doff = nullptr;
    HM_TRY(tmp.get(&dm, n_members));
    HM_TRY(tmp.get(&doff, n_edges + 1));
    if (n_members) HM_HIP(hipMemcpyAsync(dm, members_in, n_members * sizeof(uint32_t), hipMemcpyHostToDevice, st));
    HM_HIP(hipMemcpyAsync(doff, offsets_in, (n_edges + 1) * sizeof(uint64_t), hipMemcpyHostToDevice, st));
    members = dm;
    offsets = doff;
  }
  const uint64_t E = n_edges;
  const uint64_t N = H->n_nodes;
  const uint64_t n_tiles = (E + kTile - 1) / kTile;
  const bool keep_bits = H->n_nodes <= bitset_max_nodes();
  const bool one_pass = keep_bits && E <= one_pass_max_edges();
  const bool self_offsets = one_pass && n_tiles <= kSelfOffsetTiles;
  const uint32_t R = degree_copies(N);
  const uint64_t NR = N * R;
  // the degree scans ride on the gather's launch when its workgroups can
  // hold a run each (else a launch of their own after it)
  const bool gather_scan = E > 0 && NR <= kGatherScanMax;

  unsigned long long* dev_totals = nullptr;
  uint32_t *sm = nullptr, *size = nullptr, *tile_cnt = nullptr;
  unsigned long long *hash = nullptr, *slots = nullptr, *slot_of = nullptr;
  uint8_t *first = nullptr, *ecode = nullptr;
  // dedup table: a lower load (1/8 instead of 1/2) shortens the longest probe
  // chain, which sets the dedup kernel's time; kept at 1/2 for large inputs
  const unsigned long long cap = pow2_capacity(E <= (1ull << 20) ? 4 * E : E);
  // the duplicate search: one launch (inserted by k_prepare into a table that
  // is all-ones before it starts, and left that way by the gather), or the
  // exact search of k_dedup_insert
  const int tag_bits = dedup_tag_bits();
  const bool fast_dedup = E > 0 && !exact_dedup && tag_bits >= 0;
  bool table_filled = false;
  if (fast_dedup) {
    void* q = nullptr;
    HM_TRY(dalloc_filled(&q, cap * sizeof(unsigned long long), &table_filled));
    tmp.ptrs.push_back(q);
    slots = static_cast<unsigned long long*>(q);
    if (!table_filled) {
      FillList f0;
      f0.add(slots, cap, kEmpty64, 1);
      f0.launch(st);
    }
  } else {
    tmp.stage(&slots, cap);
  }
  // degree counters (counted by k_first_tiles, so staged and filled with the
  // first temporaries in either kind of build)
  uint32_t *deg2 = nullptr, *deg3 = nullptr, *deg4 = nullptr, *cur3 = nullptr, *cur4 = nullptr;
  tmp.stage(&deg2, NR);
  tmp.stage(&deg3, NR);
  tmp.stage(&deg4, NR);
  tmp.stage(&dev_totals, kTileN + 1);
  tmp.stage(&sm, n_members);
  tmp.stage(&size, E);
  tmp.stage(&hash, E);
  tmp.stage(&slot_of, E);
  tmp.stage(&first, E);
  tmp.stage(&ecode, E);
  tmp.stage(&tile_cnt, n_tiles * kTileS);
  // (in one pass they share a block with the temporaries allocate() stages)
  if (!one_pass) HM_TRY(tmp.commit());
  PinnedReport rep;
  HM_TRY(rep.take());
  Report* rep_dev = nullptr;
  HM_HIP(hipHostGetDevicePointer(reinterpret_cast<void**>(&rep_dev), rep.p, 0));
  if (!E) {
    *rep.p = Report{};
    rep.p->ready = 1;
  } else {
    __atomic_store_n(&rep.p->ready, 0u, __ATOMIC_RELEASE);
  }

  // buffers sized by the unique counts (bounds in one pass), and their fills
  auto allocate = [&](uint64_t n2, uint64_t n3, uint64_t n4, uint64_t n_unique, uint64_t n_unique_members,
                      FillList& fl) -> int {
    Carve own;
    own.add(&H->e2, 2 * n2);
    own.add(&H->e3, 3 * n3);
    own.add(&H->e4, 4 * n4);
    own.add(&H->all_members, n_unique_members);
    own.add(&H->all_off, n_unique + 1);
    const unsigned long long c2 = pow2_capacity(n2), c3 = pow2_capacity(n3), c4 = pow2_capacity(n4);
    own.add(&H->hs2.slot, c2);
    own.add(&H->hs3.slot, 2 * c3);
    own.add(&H->hs4.slot, 2 * c4);
    H->hs2.mask = c2 - 1;
    H->hs3.mask = c3 - 1;
    H->hs4.mask = c4 - 1;
    if (keep_bits) {
      H->words = (H->n_nodes + 31) / 32;
      own.add(&H->bits, N * H->words);
      own.add(&H->i3_oth, 3 * n3);
      own.add(&H->i4_oth, 4 * n4);
    }
    tmp.stage(&cur3, NR + 1);
    tmp.stage(&cur4, NR + 1);
    own.add(&H->g2_off, N + 1);
    own.add(&H->g2_adj, 2 * n2);
    own.add(&H->i3_off, N + 1);
    own.add(&H->i3_idx, 3 * n3);
    own.add(&H->i4_off, N + 1);
    own.add(&H->i4_idx, 4 * n4);
    own.add(&H->hist, uint64_t(kHistCopies) * kExactHistStride);
    own.add(&H->sample_hist, uint64_t(kHistCopies) * kSampleHistStride + 8);
    std::vector<void*> blocks;
    const int rc = own.take(&blocks);
    // carved: the graph frees the one block; else every array is its own
    H->arena = blocks.size() == 1 ? blocks[0] : nullptr;
    HM_TRY(rc);
    HM_TRY(tmp.commit());
    fl.add(H->hs2.slot, c2, kEmpty64, 1);
    fl.add(H->hs3.slot, 2 * c3, kEmpty64, 1);
    fl.add(H->hs4.slot, 2 * c4, kEmpty64, 1);
    fl.add(H->sample_hist, uint64_t(kHistCopies) * kSampleHistStride + 8, 0, 1);
    fl.add(H->hist, uint64_t(kHistCopies) * kExactHistStride, 0, 1);
    if (keep_bits) fl.add(H->bits, N * H->words, 0, 0);
    fl.add(H->all_off, 1, 0, 1);   // all_off[0]; the rest is written by the gather
    return HM_OK;
  };
  // the dedup table (and in one pass every output table), filled by k_prepare
  // (in one pass the table is carved by allocate(), so it is added after)
  FillList fl;
  if (one_pass) HM_TRY(allocate(E, E, E, E, n_members, fl));
  if (!fast_dedup) fl.add(slots, cap, kEmpty64, 1);
  fl.add(deg2, NR, 0, 0);
  fl.add(deg3, NR, 0, 0);
  fl.add(deg4, NR, 0, 0);
  if (!E) fl.launch(st);
  if (E) {
    // validate and sort; collapse repeated hyperedges onto first occurrences
    unsigned long long most = E;
    for (uint32_t k = 0; k < fl.r.n; ++k) most = std::max(most, fl.r.count[k]);
    FastDedup dd{};
    if (fast_dedup) {
      dd.slots = slots;
      dd.mask = cap - 1;
      dd.tag_mask = tag_bits >= 32 ? 0xFFFFFFFFull : (1ull << tag_bits) - 1;
      dd.slot_of = slot_of;
    }
    k_prepare<<<grid_for(most), 256, 0, st>>>(members, offsets, E, n_members, H->n_nodes, sm, size, hash, ecode,
                                              fl.r, dd);
    if (!fast_dedup)
      k_dedup_insert<<<grid_for(E), 256, 0, st>>>(sm, offsets, size, hash, E, slots, cap - 1, slot_of);
    k_first_tiles<<<unsigned(n_tiles), kTile, 0, st>>>(size, E, slots, slot_of, ecode, first, tile_cnt, fast_dedup,
                                                        sm, offsets, hash, Degrees{deg2, deg3, deg4, R});
    // in one pass with few tiles the gather sums the tile counts itself
    if (!self_offsets) k_tile_scan<<<1, 1024, 0, st>>>(tile_cnt, n_tiles, rep_dev, dev_totals);
    rep.st = st;
    rep.pending = true;
    HM_HIP(hipGetLastError());
  }

  // what the report says: error, or the unique counts
  auto read_report = [&]() -> int {
    HM_TRY(wait_ready(&rep.p->ready, st));
    rep.pending = false;
    const DevFlags got = rep.p->flags;
    if (got.err == kErrCollide) return kRetryExactDedup;
    if (got.err) {
      const char* what = (got.err & kErrOffsets) ? "offsets[0] is not 0, or offsets decrease or exceed n_members"
                         : (got.err & kErrEmpty) ? "an empty hyperedge"
                         : (got.err & kErrBadId) ? "a node id >= n_nodes"
                                                 : "a node repeated inside a hyperedge";
      set_error("invalid hypergraph: %s (first offending hyperedge index %u)", what, got.err_edge);
      return HM_EINVAL;
    }
    const unsigned long long* tot = rep.p->totals;
    H->n_unique = tot[0];
    H->n_by_size[2] = tot[1];
    H->n_by_size[3] = tot[2];
    H->n_by_size[4] = tot[3];
    H->n_by_size[5] = tot[0] - tot[1] - tot[2] - tot[3];
    H->n_singletons = got.singletons;
    H->n_duplicates = got.duplicates;
    H->n_unique_members = tot[4];
    return HM_OK;
  };
  // host-side bounds of the unique counts for grid sizes: exact after the
  // report, E in one pass
  uint64_t b2 = E, b34 = 2 * E;
  if (!one_pass) {
    HM_TRY(read_report());
    FillList fl2;
    HM_TRY(allocate(H->n_by_size[2], H->n_by_size[3], H->n_by_size[4], H->n_unique, H->n_unique_members, fl2));
    fl2.launch(st);
    b2 = H->n_by_size[2];
    b34 = H->n_by_size[3] + H->n_by_size[4];
  }
  if (E) {
    GatherOut g;
    g.e2 = H->e2;
    g.e3 = H->e3;
    g.e4 = H->e4;
    g.all_members = H->all_members;
    g.all_off = H->all_off;
    g.hs2 = H->hs2;
    g.hs3 = H->hs3;
    g.hs4 = H->hs4;
    g.bits = H->bits;
    g.W = H->words;
    g.scan = gather_scan;
    g.deg = Degrees{deg2, deg3, deg4, R};
    g.n = uint32_t(N);
    g.o2 = H->g2_off;
    g.o3 = H->i3_off;
    g.o4 = H->i4_off;
    g.c3 = cur3;
    g.c4 = cur4;
    g.self_offsets = self_offsets;
    g.report = rep_dev;
    g.dev_totals = dev_totals;
    g.dedup_clear = fast_dedup ? slots : nullptr;
    g.slot_of = slot_of;
    k_gather_tiles<<<unsigned(n_tiles) + (gather_scan ? 3u : 0u), kTile, 0, st>>>(sm, offsets, size, E, first,
                                                                                  tile_cnt, g);
  }
  HM_HIP(hipGetLastError());

  // row offsets: pairwise rows, incidence lists of 3- and 4-node hyperedges;
  // fill cursors per (node, copy) (with gather_scan, done by the gather's
  // last three workgroups)
  if (!gather_scan && NR <= 64 * 1024) {
    k_scan_degrees<<<3, 1024, 0, st>>>(deg2, H->g2_off, deg3, H->i3_off, cur3, deg4, H->i4_off, cur4, uint32_t(N), R);
    HM_HIP(hipGetLastError());
  } else if (!gather_scan) {
    uint32_t* cur2 = nullptr;
    HM_TRY(tmp.get(&cur2, NR + 1));
    HM_TRY(scan_exclusive_u32(deg2, cur2, NR, cur2 + NR, st));
    HM_TRY(scan_exclusive_u32(deg3, cur3, NR, cur3 + NR, st));
    HM_TRY(scan_exclusive_u32(deg4, cur4, NR, cur4 + NR, st));
    k_offsets_of_copies<<<grid_for(N + 1), 256, 0, st>>>(cur2, H->g2_off, cur3, H->i3_off, cur4, H->i4_off,
                                                         uint32_t(N), R);
    HM_HIP(hipGetLastError());
  }
  if (keep_bits && (b2 || b34)) {
    // ascending rows straight from the bit rows, and the incidence lists
    const uint32_t row_blocks = b2 ? grid_for(N * kWave) : 0;
    const uint32_t inc_blocks = b34 ? grid_for(b34) : 0;
    k_rows_and_incidence<<<row_blocks + inc_blocks, 256, 0, st>>>(H->bits, uint32_t(N), H->words, H->g2_off,
                                                                  H->g2_adj, row_blocks, H->e3, cur3, H->i3_idx,
                                                                  H->e4, cur4, H->i4_idx, R, H->i3_oth, H->i4_oth,
                                                                  dev_totals);
    HM_HIP(hipGetLastError());
  } else if (b34) {
    k_inc_fill<<<grid_for(b34), 256, 0, st>>>(H->e3, cur3, H->i3_idx, H->e4, cur4, H->i4_idx, R, dev_totals);
    HM_HIP(hipGetLastError());
  }
  if (!keep_bits && b2) {
    // ascending rows from a radix sort of directed pairs, with the position
    // in e2 of each entry's pair
    const uint64_t n2 = b2;
    const int B = node_bits(H->n_nodes);
    const uint64_t m = 2 * n2;
    unsigned long long *keys, *keys_tmp;
    uint32_t* vals_tmp;
    HM_TRY(tmp.get(&keys, m));
    HM_TRY(tmp.get(&keys_tmp, m));
    HM_TRY(tmp.get(&vals_tmp, m));
    HM_TRY(owned(&H->g2_eid, m));
    k_pair_keys<<<grid_for(n2), 256, 0, st>>>(H->e2, n2, B, keys, H->g2_eid);
    HM_HIP(hipGetLastError());
    HM_TRY(radix_sort_pairs(keys, H->g2_eid, keys_tmp, vals_tmp, m, 2 * B, st));
    k_pair_adj<<<grid_for(m), 256, 0, st>>>(keys, m, (1ull << B) - 1, H->g2_adj);
    HM_HIP(hipGetLastError());
  }
  if (one_pass) HM_TRY(read_report());
  // the gather leaves the duplicate search's table all-ones again (it ran:
  // the input is valid and no two different hyperedges met)
  if (fast_dedup) mark_filled(slots);
  // no wait: later calls on the stream are ordered after the build, and the
  // temporaries return to the cache only once it has run
  return HM_OK;
}

// Device memory of a graph.  With a stream, it returns to the cache once the
// work enqueued on that stream so far has run; without, at once (its users
// have been synchronised).
void release(hm_graph* H, hipStream_t st = nullptr, bool ordered = false) {
  // the arrays the build sizes: one carved block, or one block each
  void* built[] = {H->e2,     H->e3,     H->e4,     H->all_members, H->all_off, H->hs2.slot, H->hs3.slot,
                   H->hs4.slot, H->bits, H->i3_oth, H->i4_oth,      H->g2_off,  H->g2_adj,   H->i3_off,
                   H->i3_idx, H->i4_off, H->i4_idx, H->hist,        H->sample_hist};
  // and those built later, on first use
  void* later[] = {H->g2_eid,  H->pl_keys,  H->pl_edge,  H->pl_slot,   H->pl_codeg, H->pl_third, H->pl_adj,
                   H->pl_pre,  H->q_slot,   H->q_fourth, H->b4_order,  H->hub_rank, H->hub_bits, H->proj_bits,
                   H->ns_tri,  H->ns_nbr,   H->ns_h3,    H->es,        H->e5,       H->hs5};
  std::vector<void*> ps(std::begin(later), std::end(later));
  if (H->arena)
    ps.push_back(H->arena);
  else
    ps.insert(ps.end(), std::begin(built), std::end(built));
  if (ordered) {
    dfree_on(ps.data(), ps.size(), st);
  } else {
    for (void* p : ps) dfree(p);
  }
  if (H->null_plan) destroy_null_plan(H->null_plan);
  H->null_plan = nullptr;
  if (H->proposal) destroy_proposal_cache(H->proposal);
  H->proposal = nullptr;
}

}  // namespace
}  // namespace hm

extern "C" {

int hm_graph_create(const uint32_t* members, const uint64_t* offsets, uint64_t n_edges, uint64_t n_members,
                    uint32_t n_nodes, int mem_kind, void* stream, hm_graph** out) {
  try {
    if (!out) {
      hm::set_error("out is NULL");
      return HM_EINVAL;
    }
    *out = nullptr;
    if (!offsets || (!members && n_members > 0)) {
      hm::set_error("members/offsets must not be NULL");
      return HM_EINVAL;
    }
    if (n_nodes == 0 || n_nodes == 0xFFFFFFFFu) {
      hm::set_error("n_nodes must be in [1, 2^32-2]");
      return HM_EINVAL;
    }
    if (mem_kind != HM_MEM_HOST && mem_kind != HM_MEM_DEVICE) {
      hm::set_error("mem_kind must be HM_MEM_HOST or HM_MEM_DEVICE");
      return HM_EINVAL;
    }
    if (n_edges >= 0xFFFFFFFFull) {
      hm::set_error("at most 2^32-2 hyperedges are supported");
      return HM_EUNSUPPORTED;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    hm_graph* H = new (std::nothrow) hm_graph();
    if (!H) {
      hm::set_error("host allocation failed");
      return HM_ENOMEM;
    }
    if (hipGetDevice(&H->device) != hipSuccess) {
      delete H;
      hm::set_error("no HIP device");
      return HM_EDEVICE;
    }
    H->n_nodes = n_nodes;
    H->n_input = n_edges;
    int rc = hm::build(H, members, offsets, n_edges, n_members, mem_kind, st, false);
    if (rc == hm::kRetryExactDedup) {
      // two different hyperedges met in the one-launch duplicate search: the
      // graph is built again with the exact search
      (void)hipStreamSynchronize(st);
      hm::release(H);
      const int device = H->device;
      *H = hm_graph();
      H->device = device;
      H->n_nodes = n_nodes;
      H->n_input = n_edges;
      rc = hm::build(H, members, offsets, n_edges, n_members, mem_kind, st, true);
    }
    if (rc != HM_OK) {
      (void)hipStreamSynchronize(st);
      hm::release(H);
      delete H;
      return rc;
    }
    hm::note_use(H, st);
    *out = H;
    return HM_OK;
  } catch (...) {
    return hm::api_failure();
  }
}

int hm_graph_destroy(hm_graph* H) {
  try {
    if (!H) return HM_OK;
    // a graph used on one stream only, with no captured pipeline or proposal
    // cache, is released in that stream's order; otherwise after a device-wide
    // synchronisation
    if (H->streams.size() == 1 && !H->null_plan && !H->proposal) {
      hm::release(H, H->streams[0], true);
    } else {
      (void)hipDeviceSynchronize();
      hm::release(H);
    }
    delete H;
    return HM_OK;
  } catch (...) {
    return hm::api_failure();
  }
}

int hm_graph_stats(const hm_graph* H, uint64_t* out10) {
  try {
    uint64_t* out8 = out10;
    if (!H || !out8) {
      hm::set_error("NULL argument");
      return HM_EINVAL;
    }
    out8[0] = H->n_nodes;
    out8[1] = H->n_by_size[2];
    out8[2] = H->n_by_size[3];
    out8[3] = H->n_by_size[4];
    out8[4] = H->n_by_size[5];
    out8[5] = H->n_input;
    out8[6] = H->n_singletons;
    out8[7] = H->n_duplicates;
    out8[8] = H->n_unique;
    out8[9] = H->n_unique_members;
    return HM_OK;
  } catch (...) {
    return hm::api_failure();
  }
}

int hm_graph_export(const hm_graph* H, int j, uint32_t* out) {
  try {
    if (!H || !out || j < 2 || j > 4) {
      hm::set_error("bad arguments to hm_graph_export");
      return HM_EINVAL;
    }
    const uint32_t* src = j == 2 ? H->e2 : j == 3 ? H->e3 : H->e4;
    const uint64_t n = H->n_by_size[j] * uint64_t(j);
    HM_HIP(hipDeviceSynchronize());   // the build may still be running on its stream
    if (n) HM_HIP(hipMemcpy(out, src, n * sizeof(uint32_t), hipMemcpyDeviceToHost));
    return HM_OK;
  } catch (...) {
    return hm::api_failure();
  }
}

}  // extern "C"
