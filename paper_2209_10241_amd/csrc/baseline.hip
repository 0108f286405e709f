// The baseline of Section 4.1 (Algorithm 1) on gfx950: exact order-3 and
// order-4 counts from the clique projection of the hypergraph.
//
// The projection G joins two nodes when some hyperedge (of any size >= 2)
// holds both.  ESU (Wernicke 2006) enumerates every connected k-node set of G
// once, from its smallest node; each is a candidate, classified by fill-in
// (Section 4.3 Fig. 3b) and the pattern->class table (Section 4.3 Fig. 3a),
// and discarded when the sub-hypergraph it induces is not connected (the
// table maps such patterns to 0xFF).  The result equals Algorithms 2 and 3;
// the point of this path is what it costs, not what it finds.
//
// Layout: G is kept as bit rows (n_nodes x W words, rebuilt by every call)
// beside the graph's pairwise rows.  One wavefront takes a root r and a first
// extension w1 > r joined to it, and forms ESU's extension set of {r, w1} in
// LDS; at order 3 every member closes a
// candidate, at order 4 the lanes share the second extensions w2 (by rank) and
// each walks the third extension set of {r, w1, w2} word by word.
#include <algorithm>

#include "hm_items.h"

namespace hm {
namespace {

constexpr uint32_t kBaseThreads = 256;
constexpr uint32_t kBaseWaves = kBaseThreads / kWave;
constexpr unsigned kBaseGrid = 2048;

// Projection rows: one thread per unique hyperedge; every ordered pair of
// distinct members sets its bit.
__global__ void k_proj_rows(const uint32_t* __restrict__ members, const unsigned long long* __restrict__ off,
                            uint64_t n_edges, uint32_t W, uint32_t* __restrict__ P) {
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n_edges;
       i += uint64_t(gridDim.x) * blockDim.x) {
    const uint64_t b = off[i], e = off[i + 1];
    for (uint64_t x = b; x < e; ++x) {
      const uint32_t u = members[x];
      for (uint64_t y = b; y < e; ++y) {
        if (y == x) continue;
        const uint32_t w = members[y];
        atomicOr(&P[uint64_t(u) * W + (w >> 5)], 1u << (w & 31));
      }
    }
  }
}

// Bits of word x that stand for nodes above t.
__device__ inline uint32_t above(uint32_t t, uint32_t x) {
  const uint32_t tw = t >> 5;
  if (x != tw) return x > tw ? 0xFFFFFFFFu : 0u;
  const uint32_t s = (t & 31) + 1;
  return s == 32 ? 0u : (0xFFFFFFFFu << s);
}

__device__ inline uint32_t row_bit(const uint32_t* __restrict__ rows, uint32_t W, uint32_t a, uint32_t b) {
  return (rows[uint64_t(a) * W + (b >> 5)] >> (b & 31)) & 1u;
}

__device__ inline void sort2(uint32_t& a, uint32_t& b) {
  const uint32_t lo = min(a, b), hi = max(a, b);
  a = lo;
  b = hi;
}

// Fill-in of a candidate {a, b, c} (any order): its pairs from the pairwise
// rows, its triple from the 3-node hash set when the projection makes it a
// triangle (the members of a hyperedge are pairwise joined in G).
__device__ inline uint32_t base_pattern3(const View& v, const uint32_t* __restrict__ P, uint32_t a, uint32_t b,
                                         uint32_t c) {
  sort2(a, b);
  sort2(b, c);
  sort2(a, b);
  const uint32_t gab = row_bit(P, v.W, a, b), gac = row_bit(P, v.W, a, c), gbc = row_bit(P, v.W, b, c);
  uint32_t p = row_bit(v.bits, v.W, a, b) | (row_bit(v.bits, v.W, a, c) << 1) | (row_bit(v.bits, v.W, b, c) << 2);
  if (gab & gac & gbc) p |= uint32_t(set128_has(v.hs3, key3(a, b, c))) << 3;
  return p;
}

// Fill-in of a candidate {a, b, c, d} (any order).  Subset order: ab ac bc
// abc ad bd abd cd acd bcd abcd.
__device__ inline uint32_t base_pattern4(const View& v, const uint32_t* __restrict__ P, uint32_t a, uint32_t b,
                                         uint32_t c, uint32_t d) {
  sort2(a, b);
  sort2(c, d);
  sort2(a, c);
  sort2(b, d);
  sort2(b, c);
  const uint32_t W = v.W;
  const uint32_t gab = row_bit(P, W, a, b), gac = row_bit(P, W, a, c), gbc = row_bit(P, W, b, c);
  const uint32_t gad = row_bit(P, W, a, d), gbd = row_bit(P, W, b, d), gcd = row_bit(P, W, c, d);
  uint32_t p = row_bit(v.bits, W, a, b) | (row_bit(v.bits, W, a, c) << 1) | (row_bit(v.bits, W, b, c) << 2) |
               (row_bit(v.bits, W, a, d) << 4) | (row_bit(v.bits, W, b, d) << 5) | (row_bit(v.bits, W, c, d) << 7);
  if (gab & gac & gbc) p |= uint32_t(set128_has(v.hs3, key3(a, b, c))) << 3;
  if (gab & gad & gbd) p |= uint32_t(set128_has(v.hs3, key3(a, b, d))) << 6;
  if (gac & gad & gcd) p |= uint32_t(set128_has(v.hs3, key3(a, c, d))) << 8;
  if (gbc & gbd & gcd) p |= uint32_t(set128_has(v.hs3, key3(b, c, d))) << 9;
  if (gab & gac & gbc & gad & gbd & gcd) p |= uint32_t(set128_has(v.hs4, key4(a, b, c, d))) << 10;
  return p;
}

// ESU over G, counting per class in LDS (bin 0xFF: discarded candidates).
// Items are the ordered node pairs (r, w1), taken when w1 > r is joined to r
// (ESU's first extension of root r); the waves stride over them, so the
// heavy roots (small r) spread over the grid.  Dynamic LDS holds W words per
// wavefront (the extension set of {r, w1}).
template <int K>
__global__ void __launch_bounds__(kBaseThreads) k_base_esu(View v, const uint32_t* __restrict__ P,
                                                           const uint8_t* __restrict__ lut_g,
                                                           unsigned long long* __restrict__ hist) {
  extern __shared__ uint32_t ext_lds[];
  __shared__ uint8_t lut[2048];
  __shared__ unsigned long long h_main[256];
  load_lut(lut, lut_g, K == 4 ? 2048 : 16);
  h_main[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t N = v.N, W = v.W;
  const uint32_t wv = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  uint32_t* ext = ext_lds + wv * W;
  const uint64_t items = uint64_t(N) * N;
  const uint64_t n_waves = uint64_t(gridDim.x) * kBaseWaves;
  for (uint64_t it = uint64_t(blockIdx.x) * kBaseWaves + wv; it < items; it += n_waves) {
    const uint32_t r = uint32_t(it / N), w1 = uint32_t(it % N);
    const uint32_t* Pr = P + uint64_t(r) * W;
    if (w1 <= r || !((Pr[w1 >> 5] >> (w1 & 31)) & 1u)) continue;
    const uint32_t* P1 = P + uint64_t(w1) * W;
    // extension set of {r, w1}: r's neighbours after w1, and w1's
    // neighbours above r that are not r's
    for (uint32_t x = lane; x < W; x += kWave) ext[x] = (Pr[x] & above(w1, x)) | (P1[x] & ~Pr[x] & above(r, x));
    wave_sync();
    if (K == 3) {
      for (uint32_t x = lane; x < W; x += kWave) {
        uint32_t m = ext[x];
        while (m) {
          const uint32_t u = (x << 5) | uint32_t(__ffs(m) - 1);
          m &= m - 1;
          atomicAdd(&h_main[lut[base_pattern3(v, P, r, w1, u)]], 1ull);
        }
      }
    } else {
      // second extensions by rank: a word holds at most 32, so each lane
      // takes at most one per word
      uint32_t rank = 0;
      for (uint32_t x = 0; x < W; ++x) {
        const uint32_t m = ext[x];
        const uint32_t c = __popc(m);
        const uint32_t j = (lane - rank) & (kWave - 1);
        rank += c;
        if (j >= c) continue;
        uint32_t mm = m;
        for (uint32_t q = 0; q < j; ++q) mm &= mm - 1;
        const uint32_t w2 = (x << 5) | uint32_t(__ffs(mm) - 1);
        const uint32_t* P2 = P + uint64_t(w2) * W;
        // extension set of {r, w1, w2}: the set above after w2, and w2's
        // neighbours above r joined to neither r nor w1
        for (uint32_t y = 0; y < W; ++y) {
          uint32_t e = (ext[y] & above(w2, y)) | (P2[y] & ~Pr[y] & ~P1[y] & above(r, y));
          while (e) {
            const uint32_t w3 = (y << 5) | uint32_t(__ffs(e) - 1);
            e &= e - 1;
            atomicAdd(&h_main[lut[base_pattern4(v, P, r, w1, w2, w3)]], 1ull);
          }
        }
      }
    }
    wave_sync();   // ext is rewritten for the next item
  }
  __syncthreads();
  flush(h_main, hist_copy(hist, kExactHistStride) + kMain, 256);
}

// counts[c] for the n_classes classes, stats = (candidates, discarded); the
// main region of every copy is left zero.  One workgroup of 256.
__global__ void k_base_combine(unsigned long long* __restrict__ hist, int n_classes, int64_t* __restrict__ counts,
                               unsigned long long* __restrict__ stats) {
  __shared__ unsigned long long part[256 / kWave];
  const int c = threadIdx.x;
  // every copy is loaded before any is cleared (the loads go out together)
  unsigned long long x[kHistCopies];
#pragma unroll
  for (uint32_t q = 0; q < kHistCopies; ++q) x[q] = hist[uint64_t(q) * kExactHistStride + kMain + c];
  unsigned long long m = 0;
#pragma unroll
  for (uint32_t q = 0; q < kHistCopies; ++q) m += x[q];
#pragma unroll
  for (uint32_t q = 0; q < kHistCopies; ++q) hist[uint64_t(q) * kExactHistStride + kMain + c] = 0;
  if (c < n_classes) counts[c] = int64_t(m);
  const unsigned long long s = wave_sum(m);
  if ((c & (kWave - 1)) == 0) part[c / kWave] = s;
  __syncthreads();
  if (c == 0) {
    unsigned long long t = 0;
    for (int q = 0; q < 256 / kWave; ++q) t += part[q];
    stats[0] = t;
  }
  if (c == 0xFF) stats[1] = m;
}

}  // namespace

int count_baseline_impl(const hm_graph* H, int k, int64_t* counts, unsigned long long* stats, hipStream_t st) {
  note_use(H, st);
  if (!H->bits) {
    set_error("the projection baseline needs adjacency bit rows (at most %u nodes)", bitset_max_nodes());
    return HM_EUNSUPPORTED;
  }
  const uint8_t *lut4 = nullptr, *lut3 = nullptr;
  HM_TRY(device_luts(H->device, &lut4, &lut3));
  const uint64_t words = uint64_t(H->n_nodes) * H->words;
  if (!H->proj_bits) {
    void* p = nullptr;
    HM_TRY(dalloc(&p, words * sizeof(uint32_t)));
    H->proj_bits = static_cast<uint32_t*>(p);
  }
  if (H->hist_dirty) {
    HM_TRY(fill_u64(H->hist, 0, uint64_t(kHistCopies) * kExactHistStride, st));
    H->hist_dirty = false;
  }
  H->hist_dirty = true;   // until the combine below is enqueued
  HM_TRY(fill_u32(H->proj_bits, 0, words, st));
  if (H->n_unique) {
    const unsigned g = unsigned(std::min<uint64_t>(4096, (H->n_unique + 255) / 256));
    ProfileScope ps("k_proj_rows", st);
    k_proj_rows<<<g, 256, 0, st>>>(H->all_members, H->all_off, H->n_unique, H->words, H->proj_bits);
  }
  HM_HIP(hipGetLastError());
  const View v = view_of(H);
  const size_t lds = size_t(kBaseWaves) * H->words * sizeof(uint32_t);
  const uint64_t items = uint64_t(H->n_nodes) * H->n_nodes;
  const unsigned grid = unsigned(std::max<uint64_t>(1, std::min<uint64_t>(kBaseGrid, (items + kBaseWaves - 1) / kBaseWaves)));
  {
    ProfileScope ps("k_base_esu", st);
    if (k == 4)
      k_base_esu<4><<<grid, kBaseThreads, lds, st>>>(v, H->proj_bits, lut4, H->hist);
    else
      k_base_esu<3><<<grid, kBaseThreads, lds, st>>>(v, H->proj_bits, lut3, H->hist);
  }
  HM_HIP(hipGetLastError());
  k_base_combine<<<1, 256, 0, st>>>(H->hist, class_tables().n_classes[k], counts, stats);
  HM_HIP(hipGetLastError());
  H->hist_dirty = false;
  return HM_OK;
}

}  // namespace hm

extern "C" int count_baseline(const hm_graph* H, int k, int64_t* counts, uint64_t* stats, void* stream) {
  try {
    if (!H || !counts || !stats) {
      hm::set_error("NULL argument to count_baseline");
      return HM_EINVAL;
    }
    if (k != 3 && k != 4) {
      hm::set_error("order %d is not supported (3 or 4)", k);
      return HM_EUNSUPPORTED;
    }
    return hm::count_baseline_impl(H, k, counts, reinterpret_cast<unsigned long long*>(stats),
                                   static_cast<hipStream_t>(stream));
  } catch (...) {
    return hm::api_failure();
  }
}
