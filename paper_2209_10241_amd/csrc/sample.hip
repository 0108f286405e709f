// Hyperedge-sampled counting of order-3 and order-4 motifs (Algorithm 4,
// Section 5).
//
// Stratified sampling with replacement: S_j draws from the unique hyperedges
// of size j (j = 2..k), index i of stratum j = hi64(word0 * |E_j|) where word0
// is Philox4x64-10 of counter (i, 0, 0, 0) under key (seed, 1<<32 | j).  For
// each sampled hyperedge e, every connected k-node set V' containing e whose
// sub-hypergraph holds no hyperedge larger than e adds one to its class (raw
// counts).  The estimate of class m is raw_m * |E_mc| / (S_mc * countmax_m)
// with mc = maxcard(m), formed in fp64 and rounded once to fp32.
#include <algorithm>
#include <cmath>

#include "hm_sparse.h"

namespace hm {
namespace {

constexpr int kRaw = 0;   // raw counts in hm_graph::hist[0..255]

__global__ void k_draw(uint32_t* __restrict__ idx, uint64_t S, uint64_t n_j, unsigned long long seed, uint32_t j) {
  const unsigned long long k1 = (kDomainSample << 32) | j;
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < S; i += uint64_t(gridDim.x) * blockDim.x) {
    const Philox4 r = philox4x64_10(i, 0, 0, 0, seed, k1);
    idx[i] = uint32_t(bounded64(r.v[0], n_j));
  }
}

__global__ void k_check_indices(const uint32_t* __restrict__ idx, uint64_t S, uint64_t n_j, uint32_t* bad) {
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < S; i += uint64_t(gridDim.x) * blockDim.x)
    if (idx[i] >= n_j) atomicOr(bad, 1u);
}

// Where sample s of stratum j comes from: an explicit index list, or draw s of
// the stratum's Philox stream (the same words k_draw writes out).
struct Draws {
  const uint32_t* idx[5];
  unsigned long long S[5];
  unsigned long long n[5];
  unsigned long long seed;
  __device__ uint64_t at(int j, uint64_t s) const {
    if (idx[j]) return idx[j][s];
    const Philox4 r = philox4x64_10(s, 0, 0, 0, seed, (kDomainSample << 32) | uint64_t(j));
    return bounded64(r.v[0], n[j]);
  }
};

__device__ inline unsigned long long* row_or(unsigned long long* rows, uint64_t s, unsigned long long* h) {
  return rows ? rows + s * 256 : h;
}

// Per-sample-row mode without bit rows: a sample's (or a queued job's) counts
// gather in LDS and reach its row in device memory once, at the end, by the
// threads [t0, t0 + n) that worked on it (which then clear the LDS copy).
__device__ inline void flush_row(unsigned long long* h, unsigned long long* row, uint32_t t, uint32_t n) {
  for (uint32_t c = t; c < 256; c += n) {
    const unsigned long long x = h[c];
    if (x) {
      atomicAdd(&row[c], x);
      h[c] = 0;
    }
  }
}

// j = 4: the sampled 4-node hyperedge is the only candidate set.  One thread
// per sample.
__device__ void sample_j4(const View& v, const Draws& d, uint32_t part, uint32_t n_parts, const uint8_t* lut,
                          unsigned long long* h_lds, unsigned long long* rows) {
  for (uint64_t s = uint64_t(part) * kThreads + threadIdx.x; s < d.S[4]; s += uint64_t(n_parts) * kThreads) {
    const uint64_t i = d.at(4, s);
    if (i >= d.n[4]) continue;
    const uint32_t a = v.e4[4 * i], b = v.e4[4 * i + 1], c = v.e4[4 * i + 2], e = v.e4[4 * i + 3];
    uint32_t p = 1u << 10;
    p |= pair_bit(v.hs2, v.bits, v.W, a, b) << 0;
    p |= pair_bit(v.hs2, v.bits, v.W, a, c) << 1;
    p |= pair_bit(v.hs2, v.bits, v.W, b, c) << 2;
    p |= uint32_t(set128_has(v.hs3, key3(a, b, c))) << 3;
    p |= pair_bit(v.hs2, v.bits, v.W, a, e) << 4;
    p |= pair_bit(v.hs2, v.bits, v.W, b, e) << 5;
    p |= uint32_t(set128_has(v.hs3, key3(a, b, e))) << 6;
    p |= pair_bit(v.hs2, v.bits, v.W, c, e) << 7;
    p |= uint32_t(set128_has(v.hs3, key3(a, c, e))) << 8;
    p |= uint32_t(set128_has(v.hs3, key3(b, c, e))) << 9;
    atomicAdd(&row_or(rows, s, h_lds)[lut[p]], 1ull);
  }
}

// Work chunks of heavy samples (without bit rows), drained by every
// workgroup of a second launch so that one sample's work spreads over many.
enum : uint32_t { kJobNone = 0, kJobPairT = 1, kJobPairR = 2, kJobTriple = 3, kJobPairS = 4, kJobPairQ = 5 };
// default chunk sizes (divided by the HM_OPT_SAMPLE_CHUNK_SCALE option)
constexpr uint32_t kChunkT = 2;    // nodes of T per chunk
constexpr uint32_t kChunkR = 4;    // correction items per chunk
constexpr uint32_t kChunkX = 128;  // exception positions per chunk
constexpr uint32_t kChunkH = 256;  // hyperedges at s (3-node) or holding e (4-node) per chunk
// queue entries per sample of strata 2 and 3 (times the chunk option), at
// most kQueueMax in all; work that finds the queue full is done in place
constexpr uint64_t kQueuePerSample = 2048;
// pair samples whose walks visit at most about this many positions walk them
// in place (divided by the HM_OPT_SAMPLE_CHUNK_SCALE option)
constexpr uint64_t kInlineWork = 4096;
constexpr uint64_t kQueueMax = 1ull << 26;

struct Queue {
  uint4* job;                   // {kind, sample, first, last}
  unsigned long long cap;
  unsigned long long* tail;     // reserved entries (may pass cap: those are done in place)
  unsigned long long* head;     // claimed entries
  uint32_t* tcls;               // per pair sample: |T n A_q|, q = 1..3
  uint32_t ct, cr, cx, ch;      // chunk sizes: nodes of T, correction items, exception positions, hyperedges
  uint64_t inline_work;         // pair samples with a smaller bound on visited positions walk in place
};

// Reserve n entries; returns the first, or ~0 when they do not fit (the
// caller then does the work in place; entries it reserved below cap are
// marked empty).
__device__ inline unsigned long long queue_reserve(const Queue& q, uint32_t n) {
  const unsigned long long base = atomicAdd(q.tail, (unsigned long long)n);
  if (base + n <= q.cap) return base;
  for (unsigned long long e = base; e < q.cap && e < base + n; ++e) q.job[e] = make_uint4(kJobNone, 0, 0, 0);
  return ~0ull;
}

// j = 3 at order 4: the neighbourhood of the sampled 3-node hyperedge.  One
// wavefront per sample.  Without bit rows the exceptional nodes go to the
// work queue when they span more than one chunk.
__device__ __forceinline__ void j3_exceptions(const View& v, const PairLinks& pl, const B4Ctx& x, uint64_t first,
                                     uint64_t last, uint32_t lane, uint32_t stride, const uint8_t* lut,
                                     unsigned long long* h) {
  for (uint64_t t = first + lane; t < last; t += stride) {
    uint32_t pat;
    const uint32_t r = b4_exception<false>(v, pl, x, t, &pat, b4_short_none());
    if (!r) continue;
    if (r & 7u) {
      const uint8_t cc = lut[b4_combo_pattern(x, r & 7u)];
      atomicAdd(&h[cc], ~0ull);   // counted among its combination: minus one
    }
    if (r & 8u) atomicAdd(&h[lut[pat]], 1ull);
  }
}

template <bool BITS>
// hw: without bit rows in per-sample-row mode, 256 counters of LDS per
// wavefront (zero on entry, left zero) in which each sample's counts gather.
__device__ void sample_j3_k4(const View& v, const PairLinks& pl, const Queue& q, const Draws& d, uint32_t part,
                             uint32_t n_parts, uint32_t* sets, const uint8_t* lut, unsigned long long* h_lds,
                             unsigned long long* rows, unsigned long long (*hw)[256]) {
  const int wv = threadIdx.x / kWave;
  const uint32_t lane = threadIdx.x & (kWave - 1);
  for (uint64_t s = uint64_t(part) * kWavesPerBlock + wv; s < d.S[3]; s += uint64_t(n_parts) * kWavesPerBlock) {
    const uint64_t i = d.at(3, s);
    if (i >= d.n[3]) continue;
    const uint32_t a = v.e3[3 * i], b = v.e3[3 * i + 1], c = v.e3[3 * i + 2];
    unsigned long long* h = (!BITS && rows) ? hw[wv] : row_or(rows, s, h_lds);
    if constexpr (BITS) {
      b4_edge_bits_count<false>(a, b, c, v.i3_off, v.i3_oth, v.i4_off, v.i4_oth, v.bits, v.W,
                                sets + wv * b4_set_words(v.W), lut, h, nullptr);
    } else {
      const B4Ctx x = b4_ctx(v, pl, a, b, c);
      uint32_t n[8];
      b4_combo_counts(v, pl, x, n);
      if (lane == 0) {
#pragma unroll
        for (uint32_t cmb = 1; cmb < 8; ++cmb)
          if (n[cmb]) atomicAdd(&h[lut[b4_combo_pattern(x, cmb)]], (unsigned long long)n[cmb]);
      }
      const uint64_t jobs = (x.total + q.cx - 1) / q.cx;
      unsigned long long base = ~0ull;
      if (q.job && jobs > 1) {
        if (lane == 0) base = queue_reserve(q, uint32_t(jobs));
        base = __shfl(base, 0, kWave);
      }
      if (base == ~0ull) {
        j3_exceptions(v, pl, x, 0, x.total, lane, kWave, lut, h);
      } else {
        for (uint64_t k = lane; k < jobs; k += kWave)
          q.job[base + k] = make_uint4(kJobTriple, uint32_t(s), uint32_t(k * q.cx),
                                       uint32_t(min<uint64_t>((k + 1) * q.cx, x.total)));
      }
      if (rows) {
        wave_sync();
        flush_row(h, rows + s * 256, lane, kWave);
        wave_sync();
      }
    }
  }
}

__device__ inline uint32_t nodeL(const uint32_t* g2_adj, uint32_t ub, uint32_t du, uint32_t wb, uint32_t p) {
  return p < du ? g2_adj[ub + p] : g2_adj[wb + (p - du)];
}

// Per-node statistics for the pair sampler without bit rows.
struct NodeStats {
  const unsigned long long* tri;   // triangles at the node
  const unsigned long long* nbr;   // sum of the neighbours' degrees
  const uint32_t* h3;              // 3-node hyperedges {x, y, z} at x by (x~y, x~z, y~z), y < z
};

// j = 2 at order 4 without bit rows, for the sampled pair e = {s, o}, s the
// end of smaller degree.  The kept sets are those of the bit-row version
// (below): e u {x, y} with x, y outside X = e u T, T = {t : {s,o,t} is a
// 3-node hyperedge}, connected through pairs, and no larger hyperedge inside.
// Nodes z outside e fall in classes by adjacency to (s, o): 1 = s only, 2 = o
// only, 3 = both; A_1, A_2, A_3 partition A = N(s) u N(o) \ e.
//   First term without T: class sizes |A_3| = t_e, |A_1| = d_s - 1 - t_e,
//   |A_2| = d_o - 1 - t_e; pairs of A joined by a pair, per class pair, from
//   the triangles at s and o and the per-pair statistics of e (4-cliques and
//   4-cycles through e, triangle and degree sums over the common
//   neighbours); pairs of A not joined by complement; sets with y hanging off
//   x alone from the neighbour-degree sums.
//   Pairs touching T come off through the rows of the nodes of T (as if every
//   pair inside T were not joined, then corrected per joined pair).
//   Second term: the 3-node hyperedges at s one by one, those at o from its
//   8-bin pattern histogram (valid when neither other node meets s's side),
//   corrected one by one for the 3-node hyperedges {o, y, z} where y or z is
//   in N(s) u T or {s, y, z} is a 3-node hyperedge; the 4-node hyperedges
//   holding e one by one.
// One workgroup per sample; the walks over T and over the corrections of a
// heavy sample go to the work queue in chunks.
struct J2SparseLds {
  uint32_t tcls[4];
  uint32_t tlo[4];   // nodes of T below s, by class
  // flat walks over up to 256 items, each with up to three row segments
  uint32_t pre[kThreads + 1];
  uint32_t wave_tot[kWavesPerBlock];
  uint32_t item[kThreads];
  uint32_t seg_base[kThreads][3];
  uint32_t seg_len[kThreads][3];
  uint32_t cnt[kThreads][11];
  // the sorted lists the correction walk searches, when they fit (at most
  // kHeldList entries): T and the pairwise row of s
  uint32_t t_list[1024], s_list[1024];
};
constexpr uint32_t kHeldList = 1024;

// Whether z is in the ascending list l[0, n) (LDS).
__device__ inline bool lds_find(const uint32_t* l, uint32_t n, uint32_t z) {
  uint32_t lo = 0, hi = n;
  while (hi > lo) {
    const uint32_t m = (lo + hi) >> 1;
    const uint32_t y = l[m];
    if (y == z) return true;
    if (y < z) lo = m + 1; else hi = m;
  }
  return false;
}

// Walk, for items [first, last) 256 at a time, the concatenated segments
// seg(i) defines (up to three, each a start and a length), as one flat range
// over the workgroup: body(slot, segment, position) for every position; then
// fin(slot, item) once per item.  Every thread must call it.
template <typename Seg, typename Body, typename Fin>
__device__ void block_flat(uint32_t first, uint32_t last, J2SparseLds& L, Seg seg, Body body, Fin fin) {
  const uint32_t tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
  for (uint32_t c0 = first; c0 < last; c0 += kThreads) {
    uint32_t len = 0;
    L.seg_len[tid][0] = L.seg_len[tid][1] = L.seg_len[tid][2] = 0;
    for (int q = 0; q < 11; ++q) L.cnt[tid][q] = 0;
    if (c0 + tid < last) {
      seg(c0 + tid, L.seg_base[tid], L.seg_len[tid]);
      len = L.seg_len[tid][0] + L.seg_len[tid][1] + L.seg_len[tid][2];
    }
    L.item[tid] = c0 + tid;
    uint32_t wtot;
    uint32_t off = wave_exclusive_scan(len, &wtot);
    if (lane == 0) L.wave_tot[wv] = wtot;
    __syncthreads();
    for (uint32_t q = 0; q < wv; ++q) off += L.wave_tot[q];
    L.pre[tid] = off;
    if (tid == kThreads - 1) L.pre[kThreads] = off + len;
    __syncthreads();
    const uint32_t work = L.pre[kThreads];
    for (uint32_t t = tid; t < work; t += kThreads) {
      uint32_t lo = 0, hi = kThreads;   // pre[lo] <= t < pre[hi]
      while (hi - lo > 1) {
        const uint32_t m = (lo + hi) >> 1;
        if (L.pre[m] <= t) lo = m; else hi = m;
      }
      uint32_t k = t - L.pre[lo], sg = 0;
      while (k >= L.seg_len[lo][sg]) {
        k -= L.seg_len[lo][sg];
        ++sg;
      }
      body(lo, sg, L.seg_base[lo][sg] + k);
    }
    __syncthreads();
    if (c0 + tid < last) fin(tid, c0 + tid);
    __syncthreads();
  }
}

struct J2Ctx;
__device__ inline void j2_hold_lists(const View& v, const PairLinks& pl, const J2Ctx& c, J2SparseLds& L);

struct J2Ctx {
  uint32_t e0, s, o, ds, dO;
  int rs, ro;   // dense adjacency rows of s and o, or -1
  uint64_t tlo, thi;
  bool any_t;
  unsigned long long na[4];
};

__device__ inline J2Ctx j2_ctx(const View& v, const PairLinks& pl, const unsigned long long* es, uint64_t n2,
                               uint64_t i) {
  J2Ctx c;
  const uint32_t e0 = v.e2[2 * i], e1 = v.e2[2 * i + 1];
  const uint32_t d0 = deg2_of(v, e0), d1 = deg2_of(v, e1);
  c.e0 = e0;
  c.s = d0 <= d1 ? e0 : e1;
  c.o = d0 <= d1 ? e1 : e0;
  c.ds = d0 <= d1 ? d0 : d1;
  c.dO = d0 <= d1 ? d1 : d0;
  c.rs = hub_of(pl, c.s);
  c.ro = hub_of(pl, c.o);
  const unsigned long long key = ((unsigned long long)e0 << 32) | e1;
  uint32_t nt;
  pl_find(pl, key, &c.tlo, &nt);
  c.thi = c.tlo + nt;
  c.any_t = c.thi > c.tlo;
  const unsigned long long te = es[i];
  c.na[0] = 0;
  c.na[1] = c.ds - 1 - te;
  c.na[2] = c.dO - 1 - te;
  c.na[3] = te;
  return c;
}

__device__ inline uint32_t j2_pat(uint32_t cx, uint32_t cy, uint32_t xy) {
  return 1u | ((cx & 1u) << 1) | ((cx >> 1) << 2) | ((cy & 1u) << 4) | ((cy >> 1) << 5) | (xy << 7);
}
__device__ inline void hsub(const uint8_t* lut, unsigned long long* h, uint32_t pat, unsigned long long n) {
  const uint8_t c = lut[pat];
  if (c != 0xFF && n) atomicAdd(&h[c], 0ull - n);
}
__device__ inline void hadd(const uint8_t* lut, unsigned long long* h, uint32_t pat, unsigned long long n) {
  const uint8_t c = lut[pat];
  if (c != 0xFF && n) atomicAdd(&h[c], n);
}
__device__ inline bool j2_in_t(const View& v, const J2Ctx& c, uint32_t y) {
  return c.any_t && has3(v.hs3, c.s, c.o, y);
}
// s ~ z and o ~ z, from the dense rows of s and o when they have them
__device__ inline uint32_t j2_s_adj(const View& v, const PairLinks& pl, const J2Ctx& c, uint32_t z) {
  return c.rs >= 0 ? hub_adj(pl, c.rs, z) : uint32_t(has2(v.hs2, c.s, z));
}
__device__ inline uint32_t j2_o_adj(const View& v, const PairLinks& pl, const J2Ctx& c, uint32_t z) {
  return c.ro >= 0 ? hub_adj(pl, c.ro, z) : uint32_t(has2(v.hs2, c.o, z));
}
__device__ inline uint32_t j2_cls(const View& v, const PairLinks& pl, const J2Ctx& c, uint32_t y) {
  return j2_s_adj(v, pl, c, y) | (j2_o_adj(v, pl, c, y) << 1);
}
__device__ inline uint32_t j2_t_node(const View& v, const PairLinks& pl, const J2Ctx& c, uint64_t p) {
  return pl.third[p];
}
// j2_cls of the node of T at index entry p, from the entry's adjacency bits
// (bit 0: e0 ~ t, bit 1: e1 ~ t, with e0 < e1 the sampled pair)
__device__ inline uint32_t j2_t_cls(const PairLinks& pl, const J2Ctx& c, uint64_t p) {
  const uint32_t adj = pl.adj[p];
  return c.s == c.e0 ? adj : (((adj & 1u) << 1) | (adj >> 1));
}
// j2_agg_pat(v, c, s, t) for t in T with class cls: o ~ s holds (e is a pair)
__device__ inline uint32_t j2_agg_pat_t(const J2Ctx& c, uint32_t t, uint32_t cls) {
  const uint32_t st = cls & 1u, ot = cls >> 1;
  return c.s < t ? (1u | (1u << 2) | (ot << 5) | (st << 7)) : (1u | (ot << 2) | (1u << 5) | (st << 7));
}
// a pair {x, y} outside X whose set holds a larger hyperedge, taken off
__device__ inline void j2_remove(const View& v, const J2Ctx& c, const uint8_t* lut, unsigned long long* h, uint32_t x,
                                 uint32_t y) {
  if (x == c.s || x == c.o || y == c.s || y == c.o || j2_in_t(v, c, x) || j2_in_t(v, c, y)) return;
  hsub(lut, h,
       1u | (has2(v.hs2, c.s, x) << 1) | (has2(v.hs2, c.o, x) << 2) | (has2(v.hs2, c.s, y) << 4) |
           (has2(v.hs2, c.o, y) << 5) | (has2(v.hs2, x, y) << 7),
       1);
}
// a 3-node hyperedge {o, y, z} as the histogram at o counts it
__device__ inline uint32_t j2_agg_pat(const View& v, const J2Ctx& c, uint32_t y, uint32_t z) {
  if (z < y) {
    const uint32_t t = y;
    y = z;
    z = t;
  }
  return 1u | (has2(v.hs2, c.o, y) << 2) | (has2(v.hs2, c.o, z) << 5) | (has2(v.hs2, y, z) << 7);
}
__device__ inline bool j2_near_s(const View& v, const J2Ctx& c, uint32_t y) {
  return has2(v.hs2, c.s, y) || j2_in_t(v, c, y);
}

// Pairs touching T, for the nodes t of T at positions [first, last) of its
// index range.  The neighbours y of t outside e by class follow from
// |N(t) n N(s)| and |N(t) n N(s) n N(o)| (the shorter of the two rows walked)
// and |N(t) n N(o)| (likewise); those inside T from the shorter of N(t) and T
// (all of them, and those after t, which take each joined pair inside T once).
// T (the run of {s, o}) and the row of s, both ascending, into LDS when they
// have at most kHeldList entries.  Every thread of the workgroup calls this.
__device__ inline void j2_hold_lists(const View& v, const PairLinks& pl, const J2Ctx& c, J2SparseLds& L) {
  const uint32_t n_t = uint32_t(c.thi - c.tlo), sb = v.g2_off[c.s];
  const bool hold_t = c.any_t && n_t <= kHeldList, hold_s = c.ds <= kHeldList;
  for (uint32_t i = threadIdx.x; i < (hold_t ? n_t : 0u); i += kThreads) L.t_list[i] = pl.third[c.tlo + i];
  for (uint32_t i = threadIdx.x; i < (hold_s ? c.ds : 0u); i += kThreads) L.s_list[i] = v.g2_adj[sb + i];
  __syncthreads();
}

__device__ void j2_walk_t(const View& v, const PairLinks& pl, const J2Ctx& c, uint32_t tc1, uint32_t tc2, uint32_t tc3,
                          uint32_t first, uint32_t last, J2SparseLds& L, const uint8_t* lut, unsigned long long* h) {
  const uint32_t n_t = uint32_t(c.thi - c.tlo);
  j2_hold_lists(v, pl, c, L);
  const bool hold_t = c.any_t && n_t <= kHeldList, hold_s = c.ds <= kHeldList;
  auto s_adj = [&](uint32_t z) {
    return hold_s ? uint32_t(lds_find(L.s_list, c.ds, z)) : j2_s_adj(v, pl, c, z);
  };
  auto in_t = [&](uint32_t y) {
    return c.any_t && (hold_t ? lds_find(L.t_list, n_t, y) : has3(v.hs3, c.s, c.o, y));
  };
  block_flat(
      first, last, L,
      [&](uint32_t j, uint32_t* base, uint32_t* len) {
        const uint32_t t = j2_t_node(v, pl, c, c.tlo + j);
        const uint32_t dt = deg2_of(v, t);
        base[0] = dt <= c.ds ? v.g2_off[t] : v.g2_off[c.s];
        len[0] = dt <= c.ds ? dt : c.ds;
        base[1] = dt <= c.dO ? v.g2_off[t] : v.g2_off[c.o];
        len[1] = dt <= c.dO ? dt : c.dO;
        base[2] = dt <= n_t ? v.g2_off[t] : uint32_t(c.tlo);
        len[2] = dt <= n_t ? dt : n_t;
      },
      [&](uint32_t slot, uint32_t sg, uint32_t pos) {
        const uint32_t t = j2_t_node(v, pl, c, c.tlo + L.item[slot]);
        const uint32_t dt = deg2_of(v, t);
        if (sg == 0) {
          const uint32_t z = v.g2_adj[pos];
          const uint32_t hit = dt <= c.ds ? s_adj(z) : uint32_t(has2(v.hs2, t, z));
          if (hit) {
            atomicAdd(&L.cnt[slot][0], 1u);
            if (j2_o_adj(v, pl, c, z)) atomicAdd(&L.cnt[slot][1], 1u);
          }
        } else if (sg == 1) {
          const uint32_t z = v.g2_adj[pos];
          if (dt <= c.dO ? j2_o_adj(v, pl, c, z) : uint32_t(has2(v.hs2, t, z))) atomicAdd(&L.cnt[slot][2], 1u);
        } else {
          uint32_t y, cy;
          if (dt <= n_t) {
            y = v.g2_adj[pos];
            if (y == c.s || y == c.o || !in_t(y)) return;
            cy = s_adj(y) | (j2_o_adj(v, pl, c, y) << 1);
          } else {
            y = j2_t_node(v, pl, c, pos);
            if (y == t || !has2(v.hs2, t, y)) return;
            cy = j2_t_cls(pl, c, pos);
          }
          atomicAdd(&L.cnt[slot][3 + cy], 1u);
          if (y > t) atomicAdd(&L.cnt[slot][7 + cy], 1u);
        }
      },
      [&](uint32_t slot, uint32_t j) {
        const uint32_t t = j2_t_node(v, pl, c, c.tlo + j);
        const uint32_t ct = j2_t_cls(pl, c, c.tlo + j);
        const uint32_t ts = ct & 1u, to = ct >> 1;
        const uint32_t dt = deg2_of(v, t);
        const uint32_t a_s = L.cnt[slot][0], a_so = L.cnt[slot][1], a_o = L.cnt[slot][2];
        const uint32_t c3 = a_so, c1 = a_s - to - a_so, c2 = a_o - ts - a_so;
        const uint32_t c0 = dt - ts - to - c1 - c2 - c3;
        // neighbours outside T by class
        const unsigned long long m0 = c0 - L.cnt[slot][3], m1 = c1 - L.cnt[slot][4], m2 = c2 - L.cnt[slot][5],
                                 m3 = c3 - L.cnt[slot][6];
        if (ct) {
          hsub(lut, h, j2_pat(ct, 1, 1), m1);
          hsub(lut, h, j2_pat(ct, 2, 1), m2);
          hsub(lut, h, j2_pat(ct, 3, 1), m3);
          hsub(lut, h, j2_pat(ct, 0, 1), m0);
          // pairs {t, y}, y in A outside T, not joined
          hsub(lut, h, j2_pat(ct, 1, 0), c.na[1] - tc1 - m1);
          hsub(lut, h, j2_pat(ct, 2, 0), c.na[2] - tc2 - m2);
          hsub(lut, h, j2_pat(ct, 3, 0), c.na[3] - tc3 - m3);
        } else {
          hsub(lut, h, j2_pat(1, 0, 1), m1);
          hsub(lut, h, j2_pat(2, 0, 1), m2);
          hsub(lut, h, j2_pat(3, 0, 1), m3);
        }
        // joined pairs {t, y} inside T, y after t: they were taken off as not
        // joined (both in A) or not at all (y hanging off t or t off y)
#pragma unroll
        for (uint32_t cy = 0; cy < 4; ++cy) {
          const unsigned long long k = L.cnt[slot][7 + cy];
          if (!k) continue;
          if (ct && cy) {
            hadd(lut, h, j2_pat(ct, cy, 0), k);
            hsub(lut, h, j2_pat(ct, cy, 1), k);
          } else if (ct || cy) {
            hsub(lut, h, j2_pat(ct | cy, 0, 1), k);
          }
        }
      });
}

// Corrections for the 3-node hyperedges {o, y, z} with y in N(s) u T, for the
// items [first, last) of the list N(s) then T (a node of T that is also a
// neighbour of s taken once; each hyperedge from the smaller of y, z when both
// qualify).  What depends on y alone (y ~ s, y ~ o, y in T) is looked up once
// per y and kept in the item's counters; each hyperedge then needs s ~ z,
// o ~ z, y ~ z, z in T and whether {s, y, z} is a 3-node hyperedge.
__device__ void j2_walk_r(const View& v, const PairLinks& pl, const J2Ctx& c, uint32_t first, uint32_t last,
                          J2SparseLds& L, const uint8_t* lut, unsigned long long* h) {
  const uint32_t sb = v.g2_off[c.s];
  const uint32_t n_t = uint32_t(c.thi - c.tlo);
  j2_hold_lists(v, pl, c, L);
  const bool hold_t = c.any_t && n_t <= kHeldList, hold_s = c.ds <= kHeldList;
  auto y_of = [&](uint32_t j) { return j < c.ds ? v.g2_adj[sb + j] : j2_t_node(v, pl, c, c.tlo + (j - c.ds)); };
  block_flat(
      first, last, L,
      [&](uint32_t j, uint32_t* base, uint32_t* len) {
        const uint32_t y = y_of(j);
        // a node of T: its pairs with s and o from the index entry
        const uint32_t ycls = j < c.ds ? 0u : j2_t_cls(pl, c, c.tlo + (j - c.ds));
        if (y == c.o || (ycls & 1u)) return;
        const unsigned long long ky =
            y < c.o ? (((unsigned long long)y << 32) | c.o) : (((unsigned long long)c.o << 32) | y);
        uint64_t lo;
        pl_find(pl, ky, &lo, len);
        base[0] = uint32_t(lo);
        if (!*len) return;
        // the run of {s, y}: {s, y, z} is a 3-node hyperedge exactly when z is
        // among its third nodes (kept sorted), usually none
        const unsigned long long ks =
            y < c.s ? (((unsigned long long)y << 32) | c.s) : (((unsigned long long)c.s << 32) | y);
        uint64_t slo;
        uint32_t slen;
        pl_find(pl, ks, &slo, &slen);
        L.cnt[threadIdx.x][2] = uint32_t(slo);
        L.cnt[threadIdx.x][3] = slen;
        // y ~ s holds exactly for the first part of the list (a node of T
        // adjacent to s was taken there); y is in T in the second part
        const uint32_t sy = j < c.ds,
                       ty = j < c.ds ? uint32_t(c.any_t && (hold_t ? lds_find(L.t_list, n_t, y) : j2_in_t(v, c, y)))
                                     : 1u;
        const uint32_t oy = j < c.ds ? j2_o_adj(v, pl, c, y) : (ycls >> 1);
        L.cnt[threadIdx.x][0] = y;
        L.cnt[threadIdx.x][1] = sy | (oy << 1) | (ty << 2);
      },
      [&](uint32_t slot, uint32_t, uint32_t r) {
        const uint32_t y = L.cnt[slot][0], fy = L.cnt[slot][1];
        const uint32_t sy = fy & 1u, oy = (fy >> 1) & 1u, ty = fy >> 2;
        const uint32_t z = pl.third[r];
        if (z == c.s) return;   // an {s, o, t}
        // o ~ z and y ~ z come with the entry (its key is the pair {o, y})
        const uint32_t za = pl.adj[r];
        const uint32_t oz = c.o < y ? (za & 1u) : (za >> 1), yz = c.o < y ? (za >> 1) : (za & 1u);
        // s ~ z; {s, o, z} a 3-node hyperedge exactly when z is in T, the run
        // of {s, o} (sorted by third node)
        const uint32_t sz = hold_s ? uint32_t(lds_find(L.s_list, c.ds, z))
                                   : (c.rs >= 0 ? hub_adj(pl, c.rs, z) : uint32_t(has2(v.hs2, c.s, z)));
        const uint32_t tz = c.any_t && (hold_t ? lds_find(L.t_list, n_t, z) : run_find(pl, c.tlo, n_t, z) != ~0ull);
        if (z < y && (sz | tz)) return;   // taken from z
        // as the histogram at o counts it (the smaller node first)
        const uint32_t olo = y < z ? oy : oz, ohi = y < z ? oz : oy;
        hadd(lut, h, 1u | (olo << 2) | (ohi << 5) | (yz << 7), 1);
        const uint32_t slen = L.cnt[slot][3];
        if (slen && run_find(pl, L.cnt[slot][2], slen, z) != ~0ull) return;   // removed at s
        // the pair {y, z} outside X whose set holds {o, y, z}, taken off
        if (ty | tz) return;
        hsub(lut, h, 1u | (sy << 1) | (oy << 2) | (sz << 4) | (oz << 5) | (yz << 7), 1);
      },
      [](uint32_t, uint32_t) {});
}

// The 3-node hyperedges at s, entries [first, last) of its incidence row, one
// by one (with the hyperedges at o that match one at s on the far side).
__device__ void j2_pass_s(const View& v, const J2Ctx& c, uint32_t first, uint32_t last, uint32_t lane,
                          uint32_t stride, const uint8_t* lut, unsigned long long* h) {
  for (uint32_t p = v.i3_off[c.s] + first + lane; p < v.i3_off[c.s] + last; p += stride) {
    const uint32_t* f = v.e3 + 3ull * v.i3_idx[p];
    if (f[0] == c.o || f[1] == c.o || f[2] == c.o) continue;
    const uint32_t y = f[0] == c.s ? f[1] : f[0], z = f[2] == c.s ? f[1] : f[2];
    j2_remove(v, c, lut, h, y, z);
    if (!j2_near_s(v, c, y) && !j2_near_s(v, c, z) && has3(v.hs3, c.o, y, z)) hadd(lut, h, j2_agg_pat(v, c, y, z), 1);
  }
}

// The 4-node hyperedges holding e, entries [first, last) of the incidence row
// of whichever of s, o has fewer of them.
__device__ inline uint32_t j2_q_node(const View& v, const J2Ctx& c) {
  const uint32_t fs = v.i4_off[c.s + 1] - v.i4_off[c.s], fo = v.i4_off[c.o + 1] - v.i4_off[c.o];
  return fs <= fo ? c.s : c.o;
}
__device__ void j2_pass_q(const View& v, const J2Ctx& c, uint32_t first, uint32_t last, uint32_t lane,
                          uint32_t stride, const uint8_t* lut, unsigned long long* h) {
  const uint32_t a = j2_q_node(v, c), other = a == c.s ? c.o : c.s;
  for (uint32_t p = v.i4_off[a] + first + lane; p < v.i4_off[a] + last; p += stride) {
    const uint32_t* f = v.e4 + 4ull * v.i4_idx[p];
    const uint32_t g0 = f[0], g1 = f[1], g2 = f[2], g3 = f[3];
    if (g0 != other && g1 != other && g2 != other && g3 != other) continue;
    uint32_t x = 0xFFFFFFFFu, y = 0xFFFFFFFFu;
    for (const uint32_t m : {g0, g1, g2, g3}) {
      if (m == c.s || m == c.o) continue;
      if (x == 0xFFFFFFFFu) x = m; else y = m;
    }
    if (has3(v.hs3, c.s, x, y) || has3(v.hs3, c.o, x, y)) continue;   // removed with a 3-node hyperedge
    j2_remove(v, c, lut, h, x, y);
  }
}

__device__ void sample_j2_k4_sparse(const View& v, const PairLinks& pl, const NodeStats& ns,
                                    const unsigned long long* __restrict__ es, const Queue& q, const Draws& d,
                                    uint32_t part, uint32_t n_parts, J2SparseLds& L, const uint8_t* lut,
                                    unsigned long long* h_lds, unsigned long long* rows) {
  const uint32_t tid = threadIdx.x;
  __shared__ unsigned long long q_base;
  for (uint64_t smp = part; smp < d.S[2]; smp += n_parts) {
    const uint64_t i = d.at(2, smp);
    if (i >= d.n[2]) continue;
    unsigned long long* h = h_lds;   // in per-sample-row mode, flushed to the row below
    const J2Ctx c = j2_ctx(v, pl, es, d.n[2], i);
    const uint32_t s = c.s, o = c.o, ds = c.ds, dO = c.dO;
    const uint32_t n_t = uint32_t(c.thi - c.tlo);
    if (tid < 4) {
      L.tcls[tid] = 0;
      L.tlo[tid] = 0;
    }
    __syncthreads();
    // one pass over T: its class sizes, and how many of each class lie below
    // s (for the corrections {s, o, t} below), counted per thread and summed
    // per wavefront before they reach LDS
    {
      uint32_t k0 = 0, k1 = 0, k2 = 0, k3 = 0, b0 = 0, b1 = 0, b2 = 0, b3 = 0;
      for (uint64_t p = c.tlo + tid; p < c.thi; p += kThreads) {
        const uint32_t cls = j2_t_cls(pl, c, p), lo = j2_t_node(v, pl, c, p) < s;
        k0 += cls == 0;
        k1 += cls == 1;
        k2 += cls == 2;
        k3 += cls == 3;
        b0 += lo & (cls == 0);
        b1 += lo & (cls == 1);
        b2 += lo & (cls == 2);
        b3 += lo & (cls == 3);
      }
      k0 = wave_sum_u32(k0);
      k1 = wave_sum_u32(k1);
      k2 = wave_sum_u32(k2);
      k3 = wave_sum_u32(k3);
      b0 = wave_sum_u32(b0);
      b1 = wave_sum_u32(b1);
      b2 = wave_sum_u32(b2);
      b3 = wave_sum_u32(b3);
      if ((tid & (kWave - 1)) == 0) {
        atomicAdd(&L.tcls[0], k0);
        atomicAdd(&L.tcls[1], k1);
        atomicAdd(&L.tcls[2], k2);
        atomicAdd(&L.tcls[3], k3);
        atomicAdd(&L.tlo[0], b0);
        atomicAdd(&L.tlo[1], b1);
        atomicAdd(&L.tlo[2], b2);
        atomicAdd(&L.tlo[3], b3);
      }
    }
    __syncthreads();
    const uint32_t tc1 = L.tcls[1], tc2 = L.tcls[2], tc3 = L.tcls[3];
    // ---- first term (all of A), less every pair inside T as if not joined
    if (tid == 0) {
      const uint64_t n2 = d.n[2];
      const unsigned long long te = es[i], k4 = es[n2 + i], c4 = es[2 * n2 + i];
      const unsigned long long s_lo = es[3 * n2 + i], s_hi = es[4 * n2 + i], d3 = es[5 * n2 + i];
      const unsigned long long ss = s == c.e0 ? s_lo : s_hi, so = s == c.e0 ? s_hi : s_lo;
      // over the common neighbours x: codeg(s,x)-1, codeg(o,x)-1, |N(x) n A_3|;
      // over the other neighbours x of s: codeg(o,x)-1
      const unsigned long long cs = ss - te, co = so - te, cc = 2 * k4, c1o = c4 - co;
      const unsigned long long e33 = cc / 2, e13 = cs - cc, e23 = co - cc;
      const unsigned long long e11 = (ns.tri[s] - te) - e13 - e33;
      const unsigned long long e22 = (ns.tri[o] - te) - e23 - e33;
      const unsigned long long e12 = c1o - e13;
      const unsigned long long dsum[4] = {0, ns.nbr[s] - dO - d3, ns.nbr[o] - ds - d3, d3};
      const unsigned long long e[4][4] = {{0, 0, 0, 0}, {0, e11, e12, e13}, {0, e12, e22, e23}, {0, e13, e23, e33}};
      const unsigned long long tcl[4] = {0, tc1, tc2, tc3};
#pragma unroll
      for (uint32_t p = 1; p <= 3; ++p) {
#pragma unroll
        for (uint32_t r = p; r <= 3; ++r) {
          const unsigned long long tot = p == r ? c.na[p] * (c.na[p] - (c.na[p] > 0)) / 2 : c.na[p] * c.na[r];
          hadd(lut, h, j2_pat(p, r, 1), e[p][r]);
          hadd(lut, h, j2_pat(p, r, 0), tot - e[p][r]);
          const unsigned long long tp = tcl[p], tr = tcl[r];
          hsub(lut, h, j2_pat(p, r, 0), p == r ? tp * (tp - (tp > 0)) / 2 : tp * tr);
        }
        const unsigned long long inside = 2 * e[p][p] + e[p][1] + e[p][2] + e[p][3] - e[p][p];
        hadd(lut, h, j2_pat(p, 0, 1), dsum[p] - c.na[p] * (p == 3 ? 2 : 1) - inside);
      }
    }
    // ---- second term
    // at o, from its histogram
    if (tid < 8) {
      const uint32_t bb = tid;
      hsub(lut, h, 1u | ((bb & 1u) << 2) | (((bb >> 1) & 1u) << 5) | ((bb >> 2) << 7), ns.h3[8ull * o + bb]);
    }
    // corrections: the hyperedges {s, o, t}, by the class of t and its side of s
    if (tid < 8) {
      const uint32_t cls = tid & 3u, below_s = tid >> 2;
      const uint32_t n = below_s ? L.tlo[cls] : L.tcls[cls] - L.tlo[cls];
      hadd(lut, h, j2_agg_pat_t(c, below_s ? 0u : 0xFFFFFFFFu, cls), n);
    }
    // ---- the walks over T and over the corrections, and the hyperedges at s
    // and holding e: here when light, else queued in chunks
    const uint32_t n_r = ds + n_t;
    const uint32_t n_s = v.i3_off[s + 1] - v.i3_off[s];
    const uint32_t qn = j2_q_node(v, c), n_q = v.i4_off[qn + 1] - v.i4_off[qn];
    const uint32_t jobs_t = (n_t + q.ct - 1) / q.ct, jobs_r = (n_r + q.cr - 1) / q.cr;
    const uint32_t jobs_s = (n_s + q.ch - 1) / q.ch, jobs_q = (n_q + q.ch - 1) / q.ch;
    const uint32_t jobs = jobs_t + jobs_r + jobs_s + jobs_q;
    // the walks stay here only when a bound on the positions they visit is
    // small (the correction walk meets at most one run of 3-node hyperedges
    // at o per item); otherwise they go to the queue, whose claiming
    // balances them
    const uint64_t work_bound = uint64_t(n_r) * (v.i3_off[o + 1] - v.i3_off[o]) +
                                uint64_t(n_t) * (uint64_t(ds) + dO + n_t) + n_s + n_q;
    bool here = q.job == nullptr || work_bound <= q.inline_work;
    if (!here) {
      if (tid == 0) {
        q_base = queue_reserve(q, jobs);
        if (q_base != ~0ull) {
          q.tcls[3 * smp] = tc1;
          q.tcls[3 * smp + 1] = tc2;
          q.tcls[3 * smp + 2] = tc3;
        }
      }
      __syncthreads();
      here = q_base == ~0ull;
      if (!here) {
        for (uint32_t k = tid; k < jobs; k += kThreads) {
          uint32_t kind, first, last;
          if (k < jobs_t) {
            kind = kJobPairT;
            first = k * q.ct;
            last = min(first + q.ct, n_t);
          } else if (k < jobs_t + jobs_r) {
            kind = kJobPairR;
            first = (k - jobs_t) * q.cr;
            last = min(first + q.cr, n_r);
          } else if (k < jobs_t + jobs_r + jobs_s) {
            kind = kJobPairS;
            first = (k - jobs_t - jobs_r) * q.ch;
            last = min(first + q.ch, n_s);
          } else {
            kind = kJobPairQ;
            first = (k - jobs_t - jobs_r - jobs_s) * q.ch;
            last = min(first + q.ch, n_q);
          }
          q.job[q_base + k] = make_uint4(kind, uint32_t(smp), first, last);
        }
      }
    }
    if (here) {
      j2_pass_s(v, c, 0, n_s, tid, kThreads, lut, h);
      j2_pass_q(v, c, 0, n_q, tid, kThreads, lut, h);
      j2_walk_t(v, pl, c, tc1, tc2, tc3, 0, n_t, L, lut, h);
      j2_walk_r(v, pl, c, 0, n_r, L, lut, h);
    }
    __syncthreads();
    if (rows) {
      flush_row(h_lds, rows + smp * 256, tid, kThreads);
      __syncthreads();
    }
  }
}

// j = 2 at order 4 with adjacency bit rows.  The kept sets for the sampled
// pair e = {u, w} are e u {x, y} connected through pairs and holding no larger
// hyperedge: none of {u,w,x}, {u,w,y}, {u,x,y}, {w,x,y} is a 3-node hyperedge
// and {u,w,x,y} is not a 4-node hyperedge.  With T = {c : {u,w,c} is a 3-node
// hyperedge} and X = T u e, the count by pairwise pattern is
//   (pairs {x, y} outside X that connect e u {x, y} through pairs)
//   - (those of them that close a 3-node hyperedge with u or with w, or a
//      4-node hyperedge with e).
// First term, with popcounts over bit rows: A = (N(u) u N(w)) \ X; every such
// pair has x in A and either y in A with y > x, or y a neighbour of x outside
// N(u) u N(w) u X.  Second term: the 3-node hyperedges at u and at w and the
// 4-node hyperedges at u, each pair taken once.  One workgroup per sample.
constexpr uint32_t kMaxWordsJ2 = kBitsetMaxNodes / 32;
static_assert(kMaxWordsJ2 <= kThreads, "one thread per bit-row word");

struct J2Lds {
  uint32_t RU[kMaxWordsJ2], RW[kMaxWordsJ2], XS[kMaxWordsJ2], AS[kMaxWordsJ2];
  uint32_t xs[kBitsetMaxNodes];
  uint32_t wave_tot[kWavesPerBlock];
  uint32_t red[21];
};

__device__ inline uint32_t node_bit(const uint32_t* row, uint32_t x) { return (row[x >> 5] >> (x & 31)) & 1u; }

__device__ void sample_j2_k4_bits(const View& v, const Draws& d, uint32_t part, uint32_t n_parts, J2Lds& L,
                                  const uint8_t* lut, unsigned long long* h_lds, unsigned long long* rows) {
  const uint32_t tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
  const uint32_t W = v.W;
  const uint32_t* bits = v.bits;
  for (uint64_t s = part; s < d.S[2]; s += n_parts) {
    const uint64_t i = d.at(2, s);
    if (i >= d.n[2]) continue;
    unsigned long long* h = row_or(rows, s, h_lds);
    const uint32_t u = v.e2[2 * i], w = v.e2[2 * i + 1];
    // the rows of u and w and the bounds of the three incidence lists the
    // sample walks go out together
    if (tid < W) {
      L.RU[tid] = bits[uint64_t(u) * W + tid];
      L.RW[tid] = bits[uint64_t(w) * W + tid];
      L.XS[tid] = 0;
    }
    if (tid < 21) L.red[tid] = 0;
    const uint32_t u0 = v.i3_off[u], u1 = v.i3_off[u + 1];
    const uint32_t w0 = v.i3_off[w], w1 = v.i3_off[w + 1];
    const uint32_t f0 = v.i4_off[u], f1 = v.i4_off[u + 1];
    // Each list's first kThreads entries, one per thread, in one round (each
    // entry carries the hyperedge's other members, ascending), and from them
    // the pairs {x, y} the second term (below) removes, with the probes that
    // decide it and the pair bit of x, y, before the first barrier: an
    // entry of u's 3-node hyperedges without w (cand 0), of w's without u
    // whose set is not a 3-node hyperedge at u (cand 1), and of u's 4-node
    // hyperedges holding w whose other two members close no 3-node
    // hyperedge with u or w (cand 2).
    const bool has_u = u0 + tid < u1, has_w = w0 + tid < w1, has_f = f0 + tid < f1;
    const uint32_t ou = has_u ? v.i3_oth[u0 + tid] : 0u;
    const uint32_t ow = has_w ? v.i3_oth[w0 + tid] : 0u;
    const unsigned long long of = has_f ? v.i4_oth[f0 + tid] : 0ull;
    uint32_t cx[3], cy[3], cb[3];
    bool cand[3];
    cx[0] = ou & 0xFFFFu;
    cy[0] = ou >> 16;
    cand[0] = has_u && cx[0] != w && cy[0] != w;
    cx[1] = ow & 0xFFFFu;
    cy[1] = ow >> 16;
    cand[1] = has_w && cx[1] != u && cy[1] != u;
    {
      const uint32_t a = uint32_t(of) & 0xFFFFu, b = uint32_t(of >> 16) & 0xFFFFu, c = uint32_t(of >> 32) & 0xFFFFu;
      cand[2] = has_f && (a == w || b == w || c == w);
      cx[2] = a == w ? b : a;
      cy[2] = c == w ? b : c;
    }
    if (cand[1] && has3(v.hs3, u, cx[1], cy[1])) cand[1] = false;   // taken at u
    if (cand[2] && (has3(v.hs3, u, cx[2], cy[2]) || has3(v.hs3, w, cx[2], cy[2]))) cand[2] = false;
#pragma unroll
    for (int c = 0; c < 3; ++c) cb[c] = cand[c] ? uint32_t(bit_of(bits, W, cx[c], cy[c])) : 0u;
    __syncthreads();
    if (tid == 0) {
      atomicOr(&L.XS[u >> 5], 1u << (u & 31));
      atomicOr(&L.XS[w >> 5], 1u << (w & 31));
    }
    // the 3-node hyperedges at u holding w give T
    if (has_u && !cand[0]) {
      const uint32_t c = cx[0] ^ cy[0] ^ w;
      atomicOr(&L.XS[c >> 5], 1u << (c & 31));
    }
    for (uint32_t p = u0 + tid + kThreads; p < u1; p += kThreads) {
      const uint32_t o = v.i3_oth[p], y = o & 0xFFFFu, z = o >> 16;
      if (y == w || z == w) {
        const uint32_t c = y ^ z ^ w;
        atomicOr(&L.XS[c >> 5], 1u << (c & 31));
      }
    }
    __syncthreads();
    // A, compacted in ascending node order
    uint32_t a = 0;
    if (tid < W) {
      a = (L.RU[tid] | L.RW[tid]) & ~L.XS[tid];
      L.AS[tid] = a;
    }
    uint32_t wtot;
    uint32_t off = wave_exclusive_scan(__popc(a), &wtot);
    if (lane == 0) L.wave_tot[wv] = wtot;
    __syncthreads();
    uint32_t nA = 0;
    for (uint32_t q = 0; q < uint32_t(kWavesPerBlock); ++q) {
      if (q < wv) off += L.wave_tot[q];
      nA += L.wave_tot[q];
    }
    while (a) {
      L.xs[off++] = (tid << 5) | uint32_t(__ffs(a) - 1);
      a &= a - 1;
    }
    __syncthreads();
    // first term, by x's pattern to e (3) x y's pattern to u, w, x (7)
    uint32_t acc[3][7];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int j = 0; j < 7; ++j) acc[c][j] = 0;
    const uint32_t n_tasks = nA * W;
    // two tasks per round, their row words loaded together
    for (uint32_t t0 = tid; t0 < n_tasks; t0 += 2 * kThreads) {
      uint32_t rxs[2];
#pragma unroll
      for (uint32_t k = 0; k < 2; ++k) {
        const uint32_t t = t0 + k * kThreads;
        const uint32_t xi = t < n_tasks ? t / W : 0u;
        rxs[k] = t < n_tasks ? bits[uint64_t(L.xs[xi]) * W + (t - xi * W)] : 0u;
      }
#pragma unroll
      for (uint32_t k = 0; k < 2; ++k) {
        const uint32_t t = t0 + k * kThreads;
        if (t >= n_tasks) break;
        const uint32_t xi = t / W, wd = t - xi * W;
        const uint32_t x = L.xs[xi];
        const uint32_t xc = node_bit(L.RU, x) | (node_bit(L.RW, x) << 1);
        const uint32_t rx = rxs[k];
        const uint32_t ru = L.RU[wd], rw = L.RW[wd];
        const uint32_t yA = L.AS[wd] & mask_gt(x, wd);
        const uint32_t m10 = yA & ru & ~rw, m01 = yA & ~ru & rw, m11 = yA & ru & rw;
        uint32_t c7[7];
        c7[0] = __popc(m10 & ~rx);
        c7[1] = __popc(m10 & rx);
        c7[2] = __popc(m01 & ~rx);
        c7[3] = __popc(m01 & rx);
        c7[4] = __popc(m11 & ~rx);
        c7[5] = __popc(m11 & rx);
        c7[6] = __popc(rx & ~(ru | rw | L.XS[wd]));
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
          for (int j = 0; j < 7; ++j) acc[c][j] += xc == uint32_t(c + 1) ? c7[j] : 0u;
      }
    }
    // second term: each pair {x, y} outside X whose set holds a larger
    // hyperedge (pb: the pair bit of x, y)
    auto remove = [&](uint32_t x, uint32_t y, uint32_t pb) {
      if (node_bit(L.XS, x) | node_bit(L.XS, y)) return;
      const uint32_t pat = 1u | (node_bit(L.RU, x) << 1) | (node_bit(L.RW, x) << 2) | (node_bit(L.RU, y) << 4) |
                           (node_bit(L.RW, y) << 5) | (pb << 7);
      const uint8_t cls = lut[pat];
      if (cls != 0xFF) atomicAdd(&h[cls], ~0ull);   // minus one
    };
#pragma unroll
    for (int c = 0; c < 3; ++c)
      if (cand[c]) remove(cx[c], cy[c], cb[c]);
    // (entries past each list's first kThreads)
    for (uint32_t p = u0 + tid + kThreads; p < u1; p += kThreads) {
      const uint32_t o = v.i3_oth[p], y = o & 0xFFFFu, z = o >> 16;
      if (y == w || z == w) continue;
      remove(y, z, bit_of(bits, W, y, z));
    }
    for (uint32_t p = w0 + tid + kThreads; p < w1; p += kThreads) {
      const uint32_t o = v.i3_oth[p], x = o & 0xFFFFu, y = o >> 16;   // w's hyperedge {w, x, y}
      if (x == u || y == u) continue;
      if (has3(v.hs3, u, x, y)) continue;   // taken at u
      remove(x, y, bit_of(bits, W, x, y));
    }
    for (uint32_t p = f0 + tid + kThreads; p < f1; p += kThreads) {
      // u's hyperedge {u, a, b, c}, a < b < c
      const unsigned long long o = v.i4_oth[p];
      const uint32_t a = uint32_t(o) & 0xFFFFu, b = uint32_t(o >> 16) & 0xFFFFu, c = uint32_t(o >> 32) & 0xFFFFu;
      if (a != w && b != w && c != w) continue;
      // the two members other than u and w, ascending
      const uint32_t x = a == w ? b : a, y = c == w ? b : c;
      if (has3(v.hs3, u, x, y) || has3(v.hs3, w, x, y)) continue;   // taken at u or w
      remove(x, y, bit_of(bits, W, x, y));
    }
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int j = 0; j < 7; ++j) {
        const uint32_t sum = wave_sum_u32(acc[c][j]);
        if (lane == 0 && sum) atomicAdd(&L.red[c * 7 + j], sum);
      }
    __syncthreads();
    if (tid < 21 && L.red[tid]) {
      // y's pattern (bit 0: to u, bit 1: to w, bit 2: to x) of each column
      const uint32_t ycol = tid % 7;
      const uint32_t yp = ycol == 6 ? 4u : ((ycol >> 1) + 1) | ((ycol & 1u) << 2);
      const uint32_t xc = tid / 7 + 1;
      const uint32_t pat = 1u | ((xc & 1u) << 1) | ((xc >> 1) << 2) | ((yp & 1u) << 4) | (((yp >> 1) & 1u) << 5) |
                           ((yp >> 2) << 7);
      atomicAdd(&h[lut[pat]], (unsigned long long)L.red[tid]);
    }
    __syncthreads();
  }
}

// order 3, j = 3: the sampled 3-node hyperedge with its pairs.  One thread per
// sample.
__device__ void sample_j3_k3(const View& v, const Draws& d, uint32_t part, uint32_t n_parts, const uint8_t* lut,
                             unsigned long long* h_lds, unsigned long long* rows) {
  for (uint64_t s = uint64_t(part) * kThreads + threadIdx.x; s < d.S[3]; s += uint64_t(n_parts) * kThreads) {
    const uint64_t i = d.at(3, s);
    if (i >= d.n[3]) continue;
    const uint32_t a = v.e3[3 * i], b = v.e3[3 * i + 1], c = v.e3[3 * i + 2];
    const uint32_t p = (1u << 3) | pair_bit(v.hs2, v.bits, v.W, a, b) | (pair_bit(v.hs2, v.bits, v.W, a, c) << 1) |
                       (pair_bit(v.hs2, v.bits, v.W, b, c) << 2);
    atomicAdd(&row_or(rows, s, h_lds)[lut[p]], 1ull);
  }
}

// order 3, j = 2: the sampled pair {u, w} and one neighbour x of u or w
// (taken once) such that {u, w, x} is not a 3-node hyperedge.  One wavefront
// per sample.
__device__ void sample_j2_k3(const View& v, const Draws& d, uint32_t part, uint32_t n_parts, const uint8_t* lut,
                             unsigned long long* h_lds, unsigned long long* rows) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wv = threadIdx.x / kWave;
  for (uint64_t s = uint64_t(part) * kWavesPerBlock + wv; s < d.S[2]; s += uint64_t(n_parts) * kWavesPerBlock) {
    const uint64_t i = d.at(2, s);
    if (i >= d.n[2]) continue;
    const uint32_t u = v.e2[2 * i], w = v.e2[2 * i + 1];
    const uint32_t ub = v.g2_off[u], du = v.g2_off[u + 1] - ub;
    const uint32_t wb = v.g2_off[w], dw = v.g2_off[w + 1] - wb;
    unsigned long long* h = row_or(rows, s, h_lds);
    for (uint32_t p = lane; p < du + dw; p += kWave) {
      const uint32_t x = nodeL(v.g2_adj, ub, du, wb, p);
      if (x == u || x == w) continue;
      const uint32_t ux = pair_bit(v.hs2, v.bits, v.W, u, x);
      if (p >= du && ux) continue;            // taken from u's row
      if (has3(v.hs3, u, w, x)) continue;
      const uint32_t wx = pair_bit(v.hs2, v.bits, v.W, w, x);
      // local positions u=0, w=1, x=2
      atomicAdd(&h[lut[1u | (ux << 1) | (wx << 2)]], 1ull);
    }
  }
}

struct ScaleArgs {
  double n_by_size[5];
  double s_by_size[5];
  uint8_t maxcard[256];
  uint8_t countmax[256];
};

struct SampledArgs {
  View v;
  PairLinks pl;                  // pair -> 3-node hyperedge index (no bit rows)
  NodeStats ns;                  // per-node statistics (no bit rows)
  const unsigned long long* es;  // per-pair statistics (no bit rows)
  Queue q;                       // work queue (no bit rows; q.job == null otherwise)
  Draws d;
  const uint8_t* lut;
  uint32_t blocks[5];            // workgroups of strata 2, 3, 4 (in this order in the grid)
  unsigned long long* rows[5];   // per-sample rows (256 counters) of each stratum, or null
  unsigned long long* hist;      // raw counters (kHistCopies x 256), zero on entry; left zero after scaling
  float* est;                    // null: no scaling (row mode)
  int64_t* raw;
  int n_classes;
};

template <int K, bool BITS>
struct SampledLds {
  uint32_t unused;
};
template <>
struct SampledLds<4, true> {
  union {
    uint32_t b4[kWavesPerBlock * b4_set_words(kMaxWordsB)];
    J2Lds j2;
  };
};
template <>
struct SampledLds<4, false> {
  union {
    J2SparseLds j2;
    unsigned long long hw[kWavesPerBlock][256];   // per-sample counters of the 3-node samples (row mode)
  };
};

// After the sampler (and its queue's drain): scale the raw counts in a.hist
// (Algorithm 4's correction: est_m = raw_m * |E_mc| / (S_mc * countmax_m) in
// fp64, rounded once to fp32, 0 when the stratum was not sampled) and clear
// a.hist and the queue counters.  One workgroup of 256; the kernel boundary
// makes the atomics of every workgroup of the sampler visible to it.
__global__ void __launch_bounds__(kThreads) k_finish_sampled(SampledArgs a, ScaleArgs sc) {
  const int c = threadIdx.x;
  // every copy is loaded before any is cleared, so that the loads go out
  // together rather than each behind the previous store
  unsigned long long x[kHistCopies];
#pragma unroll
  for (uint32_t q = 0; q < kHistCopies; ++q) x[q] = a.hist[uint64_t(q) * kSampleHistStride + c];
  unsigned long long r = 0;
#pragma unroll
  for (uint32_t q = 0; q < kHistCopies; ++q) r += x[q];
#pragma unroll
  for (uint32_t q = 0; q < kHistCopies; ++q) a.hist[uint64_t(q) * kSampleHistStride + c] = 0;
  if (a.est && c < a.n_classes) {
    const int j = sc.maxcard[c];
    double e = 0.0;
    if (sc.s_by_size[j] > 0.0) e = (double(r) * sc.n_by_size[j]) / (sc.s_by_size[j] * double(sc.countmax[c]));
    a.est[c] = float(e);
    if (a.raw) a.raw[c] = int64_t(r);
  }
  if (c == 0) {
    *a.q.tail = 0;
    *a.q.head = 0;
  }
}

// Every stratum's samples in one launch.  The grid holds a.blocks[2]
// workgroups for the sampled pairs, then a.blocks[3] for the 3-node and
// a.blocks[4] for the 4-node hyperedges.  Each workgroup adds its LDS counts to
// a.hist (k_finish_sampled scales them).
template <int K, bool BITS>
__global__ void __launch_bounds__(kThreads) k_sampled(SampledArgs a) {
  constexpr int kLut = K == 4 ? 2048 : 16;
  __shared__ uint8_t lut[kLut];
  __shared__ unsigned long long h_lds[256];
  __shared__ SampledLds<K, BITS> lds;
  load_lut(lut, a.lut, kLut);
  h_lds[threadIdx.x] = 0;
  __syncthreads();
  uint32_t b = blockIdx.x;
  if (b < a.blocks[2]) {
    if constexpr (K == 4 && BITS)
      sample_j2_k4_bits(a.v, a.d, b, a.blocks[2], lds.j2, lut, h_lds, a.rows[2]);
    else if constexpr (K == 4)
      sample_j2_k4_sparse(a.v, a.pl, a.ns, a.es, a.q, a.d, b, a.blocks[2], lds.j2, lut, h_lds, a.rows[2]);
    else
      sample_j2_k3(a.v, a.d, b, a.blocks[2], lut, h_lds, a.rows[2]);
  } else if ((b -= a.blocks[2]) < a.blocks[3]) {
    if constexpr (K == 4 && BITS)
      sample_j3_k4<true>(a.v, a.pl, a.q, a.d, b, a.blocks[3], lds.b4, lut, h_lds, a.rows[3], nullptr);
    else if constexpr (K == 4) {
      if (a.rows[3]) {
        const uint32_t lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
        for (uint32_t c = lane; c < 256; c += kWave) lds.hw[wv][c] = 0;
        wave_sync();
      }
      sample_j3_k4<false>(a.v, a.pl, a.q, a.d, b, a.blocks[3], nullptr, lut, h_lds, a.rows[3], lds.hw);
    }
    else
      sample_j3_k3(a.v, a.d, b, a.blocks[3], lut, h_lds, a.rows[3]);
  } else if (K == 4) {
    b -= a.blocks[3];
    sample_j4(a.v, a.d, b, a.blocks[4], lut, h_lds, a.rows[4]);
  }
  __syncthreads();
  flush(h_lds, hist_copy(a.hist, kSampleHistStride), 256);
}

// Drain the work queue that k_sampled filled (without bit rows).
__global__ void __launch_bounds__(kThreads) k_sampled_drain(SampledArgs a) {
  __shared__ uint8_t lut[2048];
  __shared__ unsigned long long h_lds[256];
  __shared__ J2SparseLds L;
  __shared__ uint4 job;
  __shared__ uint32_t tcls[3];
  load_lut(lut, a.lut, 2048);
  h_lds[threadIdx.x] = 0;
  const unsigned long long n_jobs = min(__hip_atomic_load(a.q.tail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT), a.q.cap);
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) {
      const unsigned long long k = atomicAdd(a.q.head, 1ull);
      job = k < n_jobs ? a.q.job[k] : make_uint4(0xFFFFFFFFu, 0, 0, 0);
    }
    __syncthreads();
    const uint4 jb = job;
    if (jb.x == 0xFFFFFFFFu) break;
    // counts gather in h_lds; in per-sample-row mode each job's go to its
    // sample's row at the end of the job
    unsigned long long* h = h_lds;
    unsigned long long* row = nullptr;
    if (jb.x == kJobPairS || jb.x == kJobPairQ) {
      const J2Ctx c = j2_ctx(a.v, a.pl, a.es, a.d.n[2], a.d.at(2, jb.y));
      if (a.rows[2]) row = a.rows[2] + uint64_t(jb.y) * 256;
      if (jb.x == kJobPairS) j2_pass_s(a.v, c, jb.z, jb.w, threadIdx.x, kThreads, lut, h);
      else j2_pass_q(a.v, c, jb.z, jb.w, threadIdx.x, kThreads, lut, h);
    } else if (jb.x == kJobPairT || jb.x == kJobPairR) {
      const uint64_t i = a.d.at(2, jb.y);
      const J2Ctx c = j2_ctx(a.v, a.pl, a.es, a.d.n[2], i);
      if (a.rows[2]) row = a.rows[2] + uint64_t(jb.y) * 256;
      if (jb.x == kJobPairT) {
        if (threadIdx.x < 3) tcls[threadIdx.x] = a.q.tcls[3ull * jb.y + threadIdx.x];
        __syncthreads();
        j2_walk_t(a.v, a.pl, c, tcls[0], tcls[1], tcls[2], jb.z, jb.w, L, lut, h);
      } else {
        j2_walk_r(a.v, a.pl, c, jb.z, jb.w, L, lut, h);
      }
    } else if (jb.x == kJobTriple) {
      const uint64_t i = a.d.at(3, jb.y);
      const B4Ctx x = b4_ctx(a.v, a.pl, a.v.e3[3 * i], a.v.e3[3 * i + 1], a.v.e3[3 * i + 2]);
      if (a.rows[3]) row = a.rows[3] + uint64_t(jb.y) * 256;
      j3_exceptions(a.v, a.pl, x, jb.z, jb.w, threadIdx.x, kThreads, lut, h);
    }
    if (row) {
      __syncthreads();
      flush_row(h_lds, row, threadIdx.x, kThreads);
    }
  }
  __syncthreads();
  flush(h_lds, hist_copy(a.hist, kSampleHistStride), 256);
}

unsigned grid_for(uint64_t items, uint64_t per_block, unsigned cap = 512) {
  uint64_t g = (items + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return unsigned(g);
}

uint32_t blocks_for(uint64_t items, uint64_t per_block, uint32_t cap) {
  if (!items) return 0;
  return uint32_t(std::min<uint64_t>((items + per_block - 1) / per_block, cap));
}

// Launch the sampler over every stratum: explicit indices (idx[j] non-null)
// or draws of the stratum's stream under `seed`.  rows != null: sample s of
// stratum j adds to row rows[row0[j] + s] and nothing is scaled; otherwise
// est (and raw) receive the scaled (and raw) counts.
int launch_sampled(const hm_graph* H, int k, const uint32_t* const idx[5], const uint64_t S[5], uint64_t seed,
                   unsigned long long* rows, const uint64_t row0[5], float* est, int64_t* raw, hipStream_t st) {
  note_use(H, st);
  const uint8_t *lut4 = nullptr, *lut3 = nullptr;
  HM_TRY(device_luts(H->device, &lut4, &lut3));
  const bool bits = H->bits != nullptr;
  if (k == 4 && bits && H->words > kMaxWordsJ2) {
    set_error("bit rows of %u words exceed the sampler's %u", H->words, kMaxWordsJ2);
    return HM_EINTERNAL;
  }
  if (k == 4 && !bits) {
    HM_TRY(ensure_pair_links(const_cast<hm_graph*>(H), st));
    HM_TRY(ensure_node_stats(const_cast<hm_graph*>(H), st));
    HM_TRY(ensure_edge_stats(const_cast<hm_graph*>(H), st));
    HM_TRY(ensure_hub_rows(const_cast<hm_graph*>(H), st));
  }
  SampledArgs a;
  a.v = view_of(H);
  a.pl.keys = H->pl_keys;
  a.pl.edge = H->pl_edge;
  a.pl.n = H->pl_keys ? 3 * H->n_by_size[3] : 0;
  a.pl.slot = reinterpret_cast<const ulonglong2*>(H->pl_slot);
  a.pl.mask = H->pl_mask;
  a.pl.codeg = H->pl_codeg;
  a.pl.third = H->pl_third;
  a.pl.adj = H->pl_adj;
  a.pl.pre = H->pl_pre;
  a.pl.q_slot = reinterpret_cast<const ulonglong2*>(H->q_slot);
  a.pl.q_mask = H->q_mask;
  a.pl.q_fourth = H->q_fourth;
  a.pl.q_bits = H->q_bits;
  a.pl.hub_rank = H->hub_rank;
  a.pl.hub_bits = H->hub_bits;
  a.pl.hub_w = H->hub_words;
  a.ns.tri = H->ns_tri;
  a.ns.nbr = H->ns_nbr;
  a.ns.h3 = H->ns_h3;
  a.es = H->es;
  for (int j = 0; j < 5; ++j) {
    const bool in = j >= 2 && j <= k;
    a.d.idx[j] = in ? idx[j] : nullptr;
    a.d.S[j] = in ? S[j] : 0;
    a.d.n[j] = in ? H->n_by_size[j] : 0;
    a.rows[j] = (rows && in) ? rows + row0[j] * 256 : nullptr;
    a.blocks[j] = 0;
  }
  a.d.seed = seed;
  a.lut = k == 4 ? lut4 : lut3;
  if (k == 4) {
    a.blocks[2] = blocks_for(a.d.S[2], 1, 2048);
    a.blocks[3] = blocks_for(a.d.S[3], kWavesPerBlock, 1024);
    a.blocks[4] = blocks_for(a.d.S[4], kThreads, 256);
  } else {
    a.blocks[2] = blocks_for(a.d.S[2], kWavesPerBlock, 1024);
    a.blocks[3] = blocks_for(a.d.S[3], kThreads, 256);
  }
  uint32_t grid = a.blocks[2] + a.blocks[3] + a.blocks[4];
  if (grid == 0) {   // nothing sampled: one idle workgroup
    a.blocks[2] = 1;
    grid = 1;
  }
  a.hist = H->sample_hist;
  a.est = rows ? nullptr : est;
  a.raw = rows ? nullptr : raw;
  const ClassTables& t = class_tables();
  a.n_classes = t.n_classes[k];
  ScaleArgs sc;
  for (int j = 0; j < 5; ++j) {
    sc.n_by_size[j] = (j >= 2 && j <= 4) ? double(H->n_by_size[j]) : 0.0;
    sc.s_by_size[j] = (j >= 2 && j <= k) ? double(S[j]) : 0.0;
  }
  for (int c = 0; c < 256; ++c) {
    sc.maxcard[c] = c < t.n_classes[k] ? t.maxcard[k][c] : 0;
    sc.countmax[c] = c < t.n_classes[k] ? t.countmax[k][c] : 1;
  }
  // work queue of heavy samples (order 4 without bit rows); its buffers are
  // released in stream order: the caching allocator hands them out again only
  // once an event recorded on st after the drain and the finish has completed
  a.q.job = nullptr;
  a.q.cap = 0;
  a.q.tail = H->sample_hist + uint64_t(kHistCopies) * kSampleHistStride + 1;
  a.q.head = H->sample_hist + uint64_t(kHistCopies) * kSampleHistStride + 2;
  a.q.tcls = nullptr;
  const uint32_t scale = sample_chunk_scale();
  a.q.ct = std::max<uint32_t>(1, kChunkT / scale);
  a.q.cr = std::max<uint32_t>(1, kChunkR / scale);
  a.q.cx = std::max<uint32_t>(1, kChunkX / scale);
  a.q.ch = std::max<uint32_t>(1, kChunkH / scale);
  a.q.inline_work = kInlineWork / scale;
  struct Release {
    void* p[2] = {nullptr, nullptr};
    hipStream_t st;
    ~Release() { dfree_on(p, 2, st); }
  } rel{{nullptr, nullptr}, st};
  if (k == 4 && !bits) {
    a.q.cap = std::min<uint64_t>(kQueuePerSample * scale * (a.d.S[2] + a.d.S[3]) + 65536, kQueueMax);
    HM_TRY(dalloc(&rel.p[0], a.q.cap * sizeof(uint4)));
    HM_TRY(dalloc(&rel.p[1], (3 * a.d.S[2] + 1) * sizeof(uint32_t)));
    a.q.job = static_cast<uint4*>(rel.p[0]);
    a.q.tcls = static_cast<uint32_t*>(rel.p[1]);
  }
  ProfileScope pscope("k_sampled", st);
  if (k == 4 && bits)
    k_sampled<4, true><<<grid, kThreads, 0, st>>>(a);
  else if (k == 4)
    k_sampled<4, false><<<grid, kThreads, 0, st>>>(a);
  else
    k_sampled<3, false><<<grid, kThreads, 0, st>>>(a);
  HM_HIP(hipGetLastError());
  if (a.q.job) {
    k_sampled_drain<<<1024, kThreads, 0, st>>>(a);
    HM_HIP(hipGetLastError());
  }
  k_finish_sampled<<<1, kThreads, 0, st>>>(a, sc);
  HM_HIP(hipGetLastError());
  return HM_OK;
}

}  // namespace

// Sample sizes from the stratum sizes n[j] = |E_j| (j = 2..4).
int sample_sizes_for(const uint64_t n[5], int k, double fraction, int allocation, uint64_t* S) {
  if (k != 3 && k != 4) {
    set_error("order %d is not supported (3 or 4)", k);
    return HM_EUNSUPPORTED;
  }
  if (!(fraction > 0.0 && fraction <= 1.0)) {
    set_error("fraction must be in (0, 1]");
    return HM_EINVAL;
  }
  if (allocation != HM_ALLOC_PROPORTIONAL && allocation != HM_ALLOC_PAPER) {
    set_error("unknown allocation %d", allocation);
    return HM_EINVAL;
  }
  for (int j = 0; j < 5; ++j) S[j] = 0;
  if (allocation == HM_ALLOC_PAPER && k == 4) {
    // S = ceil(f * |E_2 u E_3 u E_4|) split S_2 : S_3 : S_4 = 1 : 3 : 2; a
    // stratum with hyperedges gets at least one draw, so that every class
    // keeps an unbiased estimate however small S is
    const double tot = double(n[2] + n[3] + n[4]);
    const uint64_t s = uint64_t(std::ceil(fraction * tot));
    S[2] = s / 6;
    S[3] = s / 2;
    S[4] = s - S[2] - S[3];
    for (int j = 2; j <= 4; ++j) S[j] = n[j] == 0 ? 0 : std::max<uint64_t>(S[j], 1);
  } else {
    for (int j = 2; j <= k; ++j) S[j] = uint64_t(std::ceil(fraction * double(n[j])));
  }
  return HM_OK;
}

int sample_sizes(const hm_graph* H, int k, double fraction, int allocation, uint64_t* S) {
  const uint64_t n[5] = {0, 0, H->n_by_size[2], H->n_by_size[3], H->n_by_size[4]};
  return sample_sizes_for(n, k, fraction, allocation, S);
}

// Enumerate around explicit samples (device index arrays): sample s of stratum
// j adds to row ps[row0[j] + s] (256 counters per row, zeroed by the caller).
int enumerate_samples(const hm_graph* H, int k, const uint32_t* const idx[5], const uint64_t S[5],
                      unsigned long long* ps, const uint64_t row0[5], hipStream_t st) {
  if (!ps) {
    set_error("enumerate_samples needs per-sample rows");
    return HM_EINTERNAL;
  }
  return launch_sampled(H, k, idx, S, 0, ps, row0, nullptr, nullptr, st);
}

// Draw S[j] samples of each stratum in the kernel and scale (Algorithm 4 with
// the stratum sizes given).
int sampled_with_sizes(const hm_graph* H, int k, const uint64_t S[5], uint64_t seed, float* est, int64_t* raw,
                       hipStream_t st) {
  const uint32_t* idx[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  const uint64_t row0[5] = {0, 0, 0, 0, 0};
  uint64_t s[5] = {0, 0, 0, 0, 0};
  for (int j = 2; j <= k; ++j) s[j] = H->n_by_size[j] ? S[j] : 0;
  return launch_sampled(H, k, idx, s, seed, nullptr, row0, est, raw, st);
}

// Enumerate around explicit samples and scale (Algorithm 4).
int sampled_from_indices(const hm_graph* H, int k, const uint32_t* const idx[5], const uint64_t S[5], float* est,
                         int64_t* raw, hipStream_t st) {
  const uint64_t row0[5] = {0, 0, 0, 0, 0};
  return launch_sampled(H, k, idx, S, 0, nullptr, row0, est, raw, st);
}

}  // namespace hm

extern "C" {

int hm_sample_sizes(const hm_graph* H, int k, double fraction, int allocation, uint64_t* s_out) {
  try {
    if (!H || !s_out) {
      hm::set_error("NULL argument");
      return HM_EINVAL;
    }
    uint64_t S[5];
    HM_TRY(hm::sample_sizes(H, k, fraction, allocation, S));
    s_out[0] = S[2];
    s_out[1] = S[3];
    s_out[2] = S[4];
    return HM_OK;
  } catch (...) {
    return hm::api_failure();
  }
}

int hm_sample_sizes_for(int k, const uint64_t* n_by_size, double fraction, int allocation, uint64_t* s_out) {
  try {
    if (!n_by_size || !s_out) {
      hm::set_error("NULL argument");
      return HM_EINVAL;
    }
    const uint64_t n[5] = {0, 0, n_by_size[0], n_by_size[1], k == 4 ? n_by_size[2] : 0};
    uint64_t S[5];
    HM_TRY(hm::sample_sizes_for(n, k, fraction, allocation, S));
    s_out[0] = S[2];
    s_out[1] = S[3];
    s_out[2] = S[4];
    return HM_OK;
  } catch (...) {
    return hm::api_failure();
  }
}

int hm_sample_draw(const hm_graph* H, int k, double fraction, uint64_t seed, int allocation, uint32_t* idx2,
                   uint32_t* idx3, uint32_t* idx4, void* stream) {
  try {
    if (!H) {
      hm::set_error("NULL graph");
      return HM_EINVAL;
    }
    uint64_t S[5];
    HM_TRY(hm::sample_sizes(H, k, fraction, allocation, S));
    uint32_t* out[5] = {nullptr, nullptr, idx2, idx3, idx4};
    hipStream_t st = static_cast<hipStream_t>(stream);
    for (int j = 2; j <= k; ++j) {
      if (!S[j]) continue;
      if (!out[j]) {
        hm::set_error("index buffer for stratum %d is NULL", j);
        return HM_EINVAL;
      }
      hm::k_draw<<<hm::grid_for(S[j], 256, 1024), 256, 0, st>>>(out[j], S[j], H->n_by_size[j], seed, uint32_t(j));
      HM_HIP(hipGetLastError());
    }
    return HM_OK;
  } catch (...) {
    return hm::api_failure();
  }
}

int count_sampled(const hm_graph* H, int k, double fraction, uint64_t seed, int allocation, float* est,
                  int64_t* raw, void* stream) {
  try {
    if (!H || !est) {
      hm::set_error("NULL argument to count_sampled");
      return HM_EINVAL;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    uint64_t S[5];
    HM_TRY(hm::sample_sizes(H, k, fraction, allocation, S));
    const uint32_t* idx[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};   // drawn in the kernel
    const uint64_t row0[5] = {0, 0, 0, 0, 0};
    return hm::launch_sampled(H, k, idx, S, seed, nullptr, row0, est, raw, st);
  } catch (...) {
    return hm::api_failure();
  }
}

int count_sampled_sizes(const hm_graph* H, int k, uint64_t s2, uint64_t s3, uint64_t s4, uint64_t seed, float* est,
                        int64_t* raw, void* stream) {
  try {
    if (!H || !est) {
      hm::set_error("NULL argument to count_sampled_sizes");
      return HM_EINVAL;
    }
    if (k != 3 && k != 4) {
      hm::set_error("order %d is not supported (3 or 4)", k);
      return HM_EUNSUPPORTED;
    }
    const uint64_t limit = 1ull << 31;
    if (s2 >= limit || s3 >= limit || s4 >= limit) {
      hm::set_error("a stratum sample size of 2^31 or more");
      return HM_EINVAL;
    }
    const uint64_t S[5] = {0, 0, s2, s3, k == 4 ? s4 : 0};
    return hm::sampled_with_sizes(H, k, S, seed, est, raw, static_cast<hipStream_t>(stream));
  } catch (...) {
    return hm::api_failure();
  }
}

int count_sampled_indices(const hm_graph* H, int k, const uint32_t* idx2, uint64_t s2, const uint32_t* idx3,
                          uint64_t s3, const uint32_t* idx4, uint64_t s4, float* est, int64_t* raw, void* stream) {
  try {
    if (!H || !est) {
      hm::set_error("NULL argument to count_sampled_indices");
      return HM_EINVAL;
    }
    if (k != 3 && k != 4) {
      hm::set_error("order %d is not supported (3 or 4)", k);
      return HM_EUNSUPPORTED;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    const uint32_t* idx[5] = {nullptr, nullptr, idx2, idx3, k == 4 ? idx4 : nullptr};
    uint64_t S[5] = {0, 0, s2, s3, k == 4 ? s4 : 0};
    // every index must lie in its stratum
    void* bad_p = nullptr;
    HM_TRY(hm::dalloc(&bad_p, sizeof(uint32_t)));
    uint32_t* bad = static_cast<uint32_t*>(bad_p);
    int rc = hm::fill_u32(bad, 0, 1, st);
    for (int j = 2; j <= k && rc == HM_OK; ++j) {
      if (!S[j]) continue;
      if (!idx[j]) {
        hm::set_error("index array for stratum %d is NULL", j);
        rc = HM_EINVAL;
        break;
      }
      hm::k_check_indices<<<hm::grid_for(S[j], 256, 1024), 256, 0, st>>>(idx[j], S[j], H->n_by_size[j], bad);
      if (hipGetLastError() != hipSuccess) rc = HM_EDEVICE;
    }
    uint32_t host_bad = 0;
    if (rc == HM_OK && (hipMemcpyAsync(&host_bad, bad, sizeof(uint32_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
                        hipStreamSynchronize(st) != hipSuccess))
      rc = HM_EDEVICE;
    hm::dfree(bad_p);
    if (rc != HM_OK) return rc;
    if (host_bad) {
      hm::set_error("a sample index lies outside its stratum");
      return HM_EINVAL;
    }
    return hm::sampled_from_indices(H, k, idx, S, est, raw, st);
  } catch (...) {
    return hm::api_failure();
  }
}

}  // extern "C"
