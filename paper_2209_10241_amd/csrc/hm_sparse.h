// Neighbourhood of one 3-node hyperedge without adjacency bit rows, counted
// rather than enumerated (Algorithm 3's exploration around a 3-node
// hyperedge; Algorithm 4's around a sampled one).
//
// For e = {a<b<c} the candidate sets are e u {v}.  A node v is *exceptional*
// when {a,b,v}, {a,c,v} or {b,c,v} is another 3-node hyperedge or {a,b,c,v}
// is a 4-node hyperedge; every other v has e as the only hyperedge of size
// >= 3 in e u {v}, so its class depends only on which of a, b, c it is
// paired with (the combination (av, bv, cv)).  The number of such v per
// combination follows from |N(a)|, |N(b)|, |N(c)|, the three pairwise and the
// triple intersection sizes (inclusion-exclusion, members of e excluded), less
// the exceptional v of that combination; exceptional v are classified one by
// one by fill-in.
//
// OWN = true (exact counting): a set is counted only when e is its
// lexicographically smallest 3-node hyperedge and it is not a 4-node
// hyperedge (those are counted on their own); the pairwise shape of counted
// sets whose pairs connect them goes to h_sub.
// OWN = false (sampling): every set whose largest hyperedge has 3 nodes
// counts.
//
// One wavefront per hyperedge; per-class counters are LDS (or per-sample rows).
#pragma once

#include "hm_items.h"

namespace hm {

// Pairs inside 3-node hyperedges, sorted: keys (x << 32) | y with x < y, and
// the position in e3 of the hyperedge each came from; a hash index (linear
// probing, slots of (key, start << 32 | count)) finds the run of one key.
struct PairLinks {
  const unsigned long long* keys;
  const uint32_t* edge;
  uint64_t n;
  const ulonglong2* slot;
  unsigned long long mask;
  const uint32_t* codeg;   // per slot: |N(x) n N(y)| in the pairwise graph
  // per entry: the third node t of its 3-node hyperedge, and t's pairwise
  // adjacency to the key's nodes (bit 0: x ~ t, bit 1: y ~ t)
  const uint32_t* third;
  const uint8_t* adj;
  // entries of a run are in ascending third node; pre[c * (n + 1) + p] is the
  // number of entries before position p whose adj is c (c = 0..3)
  const uint32_t* pre;
  // 4-node hyperedges by their 3-node subsets: for a < b < c, the run of the
  // key (a << 2q) | (b << q) | c (q = q_bits) in q_slot lists the fourth
  // nodes (q_fourth) of the 4-node hyperedges holding {a, b, c}; q_bits = 0
  // when not built (node ids too wide), and then the 4-node incidence list of
  // a member is walked instead
  const ulonglong2* q_slot;
  unsigned long long q_mask;
  const uint32_t* q_fourth;
  int q_bits;
  // dense adjacency rows of the highest-degree nodes: hub_rank[v] is v's row
  // (hub_w words at hub_bits + row * hub_w) or -1; hub_rank null: none
  const int32_t* hub_rank;
  const uint32_t* hub_bits;
  uint32_t hub_w;
};

// The dense adjacency row of x, or -1.
__device__ inline int hub_of(const PairLinks& pl, uint32_t x) { return pl.hub_rank ? pl.hub_rank[x] : -1; }
// Whether z is a pairwise neighbour of the node with dense row r.
__device__ inline uint32_t hub_adj(const PairLinks& pl, int r, uint32_t z) {
  return (pl.hub_bits[uint64_t(r) * pl.hub_w + (z >> 5)] >> (z & 31)) & 1u;
}

// Run [*lo, *lo + *len) of pl.keys holding `key` (empty when absent).
__device__ inline void pl_find(const PairLinks& pl, unsigned long long key, uint64_t* lo, uint32_t* len) {
  *lo = 0;
  *len = 0;
  if (!pl.n) return;
  unsigned long long h = mix64(key) & pl.mask;
  while (true) {
    const ulonglong2 s = pl.slot[h];
    if (s.x == key) {
      *lo = s.y >> 32;
      *len = uint32_t(s.y);
      return;
    }
    if (s.x == kEmpty64) return;
    h = (h + 1) & pl.mask;
  }
}

// The number of common pairwise neighbours of x < y, a pair inside some
// 3-node hyperedge (so present in the index).
// Run [*lo, *lo + *len) of q_fourth: the fourth nodes of the 4-node
// hyperedges holding {a < b < c} (pl.q_bits != 0).
__device__ inline void quad_find(const PairLinks& pl, uint32_t a, uint32_t b, uint32_t c, uint64_t* lo,
                                 uint32_t* len) {
  const int q = pl.q_bits;
  const unsigned long long key = ((unsigned long long)a << (2 * q)) | ((unsigned long long)b << q) | c;
  *lo = 0;
  *len = 0;
  unsigned long long h = mix64(key) & pl.q_mask;
  while (true) {
    const ulonglong2 s = pl.q_slot[h];
    if (s.x == key) {
      *lo = s.y >> 32;
      *len = uint32_t(s.y);
      return;
    }
    if (s.x == kEmpty64) return;
    h = (h + 1) & pl.q_mask;
  }
}

__device__ inline uint32_t pl_codeg(const PairLinks& pl, uint32_t x, uint32_t y) {
  const unsigned long long key = ((unsigned long long)x << 32) | y;
  unsigned long long h = mix64(key) & pl.mask;
  while (pl.slot[h].x != key) h = (h + 1) & pl.mask;
  return pl.codeg[h];
}

__device__ inline uint32_t deg2_of(const View& v, uint32_t x) { return v.g2_off[x + 1] - v.g2_off[x]; }

// |N(s) n N(x)| and, with y given, |N(s) n N(x) n N(y)|, over s's row (wave)
__device__ inline void row_probe(const View& v, uint32_t s, uint32_t x, uint32_t y, uint32_t& cx, uint32_t& cy,
                                 uint32_t& cxy) {
  const int lane = threadIdx.x & (kWave - 1);
  uint32_t nx = 0, ny = 0, nxy = 0;
  for (uint32_t p = v.g2_off[s] + lane; p < v.g2_off[s + 1]; p += kWave) {
    const uint32_t z = v.g2_adj[p];
    const uint32_t hx = has2(v.hs2, x, z), hy = has2(v.hs2, y, z);
    nx += hx;
    ny += hy;
    nxy += hx & hy;
  }
  cx = wave_sum_u32(nx);
  cy = wave_sum_u32(ny);
  cxy = wave_sum_u32(nxy);
}

__device__ inline uint32_t row_count(const View& v, uint32_t s, uint32_t x) {
  const int lane = threadIdx.x & (kWave - 1);
  uint32_t n = 0;
  for (uint32_t p = v.g2_off[s] + lane; p < v.g2_off[s + 1]; p += kWave) n += has2(v.hs2, x, v.g2_adj[p]);
  return wave_sum_u32(n);
}

// The hyperedge e = {a<b<c} with its pairwise pattern and the ranges of its
// exceptional nodes: slot 0..2 the pair index entries of {a,b}, {a,c},
// {b,c}; slot 3 the fourth nodes of the 4-node hyperedges holding e (with
// pl.q_bits), else the 4-node hyperedges of the member with the fewest.
struct B4Ctx {
  uint32_t a, b, c, base_p;
  int ra, rb, rc;   // dense adjacency rows of a, b, c, or -1
  // named scalars, not arrays: a dynamically indexed array would live in scratch
  uint64_t lo0, lo1, lo2, lo3, len0, len1, len2, len3, total;
};

__device__ __forceinline__ uint64_t readlane_u64(uint64_t x, int lane) {
  return (uint64_t(uint32_t(__builtin_amdgcn_readlane(int(uint32_t(x >> 32)), lane))) << 32) |
         uint32_t(__builtin_amdgcn_readlane(int(uint32_t(x)), lane));
}

// Every lane of the wavefront calls this.  The ten lookups e needs are spread
// over lanes 0..9, which run the same probe loop each on its own table, so
// that they take one round of memory latency rather than ten in a row; the
// results are then read from those lanes.  Lanes 0..2: the pair index runs of
// {a,b}, {a,c}, {b,c}; 3..5: the pairs' membership in the pair set; 6: the
// run of e in the 4-node index; 7..9: the dense rows of a, b, c.
__device__ __forceinline__ B4Ctx b4_ctx(const View& v, const PairLinks& pl, uint32_t a, uint32_t b, uint32_t c) {
  const int lane = threadIdx.x & (kWave - 1);
  B4Ctx x;
  x.a = a;
  x.b = b;
  x.c = c;
  const unsigned long long* base = nullptr;
  unsigned long long key = 0, mask = 0;
  uint32_t stride = 2;   // 64-bit words per slot: key, then value
  if (lane < 3 && pl.n) {
    const uint32_t u = lane == 2 ? b : a, w = lane == 0 ? b : c;
    key = ((unsigned long long)u << 32) | w;
    base = reinterpret_cast<const unsigned long long*>(pl.slot);
    mask = pl.mask;
  } else if (lane >= 3 && lane < 6) {
    const uint32_t u = lane == 5 ? b : a, w = lane == 3 ? b : c;
    key = key2(u, w);
    base = v.hs2.slot;
    mask = v.hs2.mask;
    stride = 1;
  } else if (lane == 6 && pl.q_bits) {
    const int q = pl.q_bits;
    key = ((unsigned long long)a << (2 * q)) | ((unsigned long long)b << q) | c;
    base = reinterpret_cast<const unsigned long long*>(pl.q_slot);
    mask = pl.q_mask;
  }
  unsigned long long val = 0;
  if (base) {
    unsigned long long h = mix64(key) & mask;
    while (true) {
      const unsigned long long k = base[stride * h];
      if (k == key) {
        val = stride == 2 ? base[2 * h + 1] : 1ull;
        break;
      }
      if (k == kEmpty64) break;
      h = (h + 1) & mask;
    }
  } else if (lane >= 7 && lane < 10) {
    val = uint32_t(hub_of(pl, lane == 7 ? a : (lane == 8 ? b : c)));
  }
  // the same in every lane: kept in scalar registers
  const uint64_t r0 = readlane_u64(val, 0), r1 = readlane_u64(val, 1), r2 = readlane_u64(val, 2);
  x.lo0 = r0 >> 32;
  x.len0 = uint32_t(r0);
  x.lo1 = r1 >> 32;
  x.len1 = uint32_t(r1);
  x.lo2 = r2 >> 32;
  x.len2 = uint32_t(r2);
  x.base_p = uint32_t(__builtin_amdgcn_readlane(int(val), 3)) | (uint32_t(__builtin_amdgcn_readlane(int(val), 4)) << 1) |
             (uint32_t(__builtin_amdgcn_readlane(int(val), 5)) << 2) | (1u << 3);
  x.ra = __builtin_amdgcn_readlane(int(val), 7);
  x.rb = __builtin_amdgcn_readlane(int(val), 8);
  x.rc = __builtin_amdgcn_readlane(int(val), 9);
  if (pl.q_bits) {
    const uint64_t r6 = readlane_u64(val, 6);
    x.lo3 = r6 >> 32;
    x.len3 = uint32_t(r6);
  } else {
    const uint32_t fa = v.i4_off[a + 1] - v.i4_off[a], fb = v.i4_off[b + 1] - v.i4_off[b],
                   fc = v.i4_off[c + 1] - v.i4_off[c];
    const uint32_t m4 = (fa <= fb && fa <= fc) ? a : (fb <= fc ? b : c);
    x.lo3 = uniform_u64(v.i4_off[m4]);
    x.len3 = uniform_u64(v.i4_off[m4 + 1] - v.i4_off[m4]);
  }
  x.total = x.len0 + x.len1 + x.len2 + x.len3;
  return x;
}

// Number of nodes v outside e per pairwise combination (av | bv<<1 | cv<<2),
// exceptional ones included, valid in every lane: the smallest row walked
// against the other two members, the common neighbours of those two from
// the pair index; inclusion-exclusion with the members of e removed.
__device__ __forceinline__ void b4_combo_counts(const View& v, const PairLinks& pl, const B4Ctx& x, uint32_t n[8]) {
  const int lane = threadIdx.x & (kWave - 1);
  const uint32_t a = x.a, b = x.b, c = x.c;
  const uint32_t pab = x.base_p & 1u, pac = (x.base_p >> 1) & 1u, pbc = (x.base_p >> 2) & 1u;
  const uint32_t da = deg2_of(v, a), db = deg2_of(v, b), dc = deg2_of(v, c);
  uint32_t r1, x1, y1, r2, x2;   // rows walked and the members they are probed against
  if (da <= db && da <= dc) {
    r1 = a; x1 = b; y1 = c;
    r2 = db <= dc ? b : c; x2 = db <= dc ? c : b;
  } else if (db <= dc) {
    r1 = b; x1 = a; y1 = c;
    r2 = da <= dc ? a : c; x2 = da <= dc ? c : a;
  } else {
    r1 = c; x1 = a; y1 = b;
    r2 = da <= db ? a : b; x2 = da <= db ? b : a;
  }
  uint32_t n1x = 0, n1y = 0, n1xy = 0;
  const uint32_t b1 = v.g2_off[r1], l1 = v.g2_off[r1 + 1] - b1;
  const int ra = x.ra, rb = x.rb, rc = x.rc;
  const int hx1 = x1 == a ? ra : (x1 == b ? rb : rc), hy1 = y1 == a ? ra : (y1 == b ? rb : rc);
  for (uint32_t t = lane; t < l1; t += kWave) {
    const uint32_t z = v.g2_adj[b1 + t];
    Probe64 px, py;
    if (hx1 < 0) px = probe2_start(v.hs2, x1, z);
    if (hy1 < 0) py = probe2_start(v.hs2, y1, z);
    const uint32_t hx = hx1 >= 0 ? hub_adj(pl, hx1, z) : uint32_t(probe64_end(v.hs2, px));
    const uint32_t hy = hy1 >= 0 ? hub_adj(pl, hy1, z) : uint32_t(probe64_end(v.hs2, py));
    n1x += hx;
    n1y += hy;
    n1xy += hx & hy;
  }
  n1x = wave_sum_u32(n1x);
  n1y = wave_sum_u32(n1y);
  n1xy = wave_sum_u32(n1xy);
  const uint32_t n2x = pl_codeg(pl, min(r2, x2), max(r2, x2));
  const uint32_t tri = n1xy;
  uint32_t cab, cac, cbc;
  if (r1 == a) { cab = n1x; cac = n1y; cbc = n2x; }
  else if (r1 == b) { cab = n1x; cbc = n1y; cac = n2x; }
  else { cac = n1x; cbc = n1y; cab = n2x; }
  const uint32_t sa = da - pab - pac, sb = db - pab - pbc, sc = dc - pac - pbc;
  const uint32_t iab = cab - pac * pbc, iac = cac - pab * pbc, ibc = cbc - pab * pac;
  n[0] = 0;
  n[7] = tri;
  n[3] = iab - tri;
  n[5] = iac - tri;
  n[6] = ibc - tri;
  n[1] = sa - n[3] - n[5] - n[7];
  n[2] = sb - n[3] - n[6] - n[7];
  n[4] = sc - n[5] - n[6] - n[7];
}

// Short lists of e's neighbourhood in a wavefront's LDS, so that a membership
// test is a comparison rather than a hash probe: the third nodes of the run
// of each pair of e when it has at most kB4ShortRun entries, the fourth
// nodes of the 4-node hyperedges holding e (at most kB4ShortQ of them,
// found in a 4-node incidence list of at most kWave entries), and the
// pairwise neighbours of each member of e with at most kB4ShortAdj of them.
// Lists are padded with kNoNode to a multiple of 4; a count of kB4NotHeld
// means the list is not held and membership is probed.
constexpr uint32_t kB4ShortRun = kWave;
constexpr uint32_t kB4ShortQ = 16;
constexpr uint32_t kB4ShortAdj = kWave;
constexpr uint32_t kB4NotHeld = 0xFFFFFFFFu;
constexpr uint32_t kNoNode = 0xFFFFFFFFu;
constexpr uint32_t kB4QAt = 3 * kB4ShortRun;                      // after ab, ac, bc
constexpr uint32_t kB4AdjAt = kB4QAt + kB4ShortQ;                 // after the 4-node list
constexpr uint32_t kB4ShortWords = kB4AdjAt + 3 * kB4ShortAdj;   // per wavefront

struct B4Short {
  const uint32_t* mem;   // 16-byte aligned, kB4ShortWords words
  uint32_t n_ab, n_ac, n_bc, n_q;
  uint32_t n_a, n_b, n_c;   // pairwise neighbours of a, b, c
};

// No list held: every membership test probes.
__device__ __forceinline__ B4Short b4_short_none() {
  B4Short s;
  s.mem = nullptr;
  s.n_ab = s.n_ac = s.n_bc = s.n_q = s.n_a = s.n_b = s.n_c = kB4NotHeld;
  return s;
}

__device__ __forceinline__ bool in_short(const uint32_t* l, uint32_t n, uint32_t y) {
  bool r = false;
  for (uint32_t k = 0; k < n; k += 4) {
    const uint4 q = *reinterpret_cast<const uint4*>(l + k);
    r |= (q.x == y) | (q.y == y) | (q.z == y) | (q.w == y);
  }
  return r;
}

// Every lane of the wavefront calls this; mem is the wavefront's LDS.
// `want` selects the lists to hold (the others are probed): bits 0..2 the
// runs of {a,b}, {a,c}, {b,c}; 3..5 the rows of a, b, c; 6 the 4-node list.
constexpr uint32_t kB4WantAll = 0x7F;
__device__ __forceinline__ B4Short b4_short(const View& v, const PairLinks& pl, const B4Ctx& x, uint32_t* mem,
                                            uint32_t want = kB4WantAll) {
  const uint32_t lane = threadIdx.x & (kWave - 1);
  const unsigned long long below = (1ull << lane) - 1ull;
  B4Short s;
  s.mem = mem;
  s.n_ab = (want & 1u) && x.len0 <= kB4ShortRun ? uint32_t(x.len0) : kB4NotHeld;
  s.n_ac = (want & 2u) && x.len1 <= kB4ShortRun ? uint32_t(x.len1) : kB4NotHeld;
  s.n_bc = (want & 4u) && x.len2 <= kB4ShortRun ? uint32_t(x.len2) : kB4NotHeld;
  if (lane < kB4ShortRun) {
    if (s.n_ab != kB4NotHeld) mem[lane] = lane < x.len0 ? pl.third[x.lo0 + lane] : kNoNode;
    if (s.n_ac != kB4NotHeld) mem[kB4ShortRun + lane] = lane < x.len1 ? pl.third[x.lo1 + lane] : kNoNode;
    if (s.n_bc != kB4NotHeld) mem[2 * kB4ShortRun + lane] = lane < x.len2 ? pl.third[x.lo2 + lane] : kNoNode;
  }
  const uint32_t da = (want & 8u) ? uniform_u32(deg2_of(v, x.a)) : kB4NotHeld;
  const uint32_t db = (want & 16u) ? uniform_u32(deg2_of(v, x.b)) : kB4NotHeld;
  const uint32_t dc = (want & 32u) ? uniform_u32(deg2_of(v, x.c)) : kB4NotHeld;
  s.n_a = da <= kB4ShortAdj ? da : kB4NotHeld;
  s.n_b = db <= kB4ShortAdj ? db : kB4NotHeld;
  s.n_c = dc <= kB4ShortAdj ? dc : kB4NotHeld;
  if (lane < kB4ShortAdj) {
    if (s.n_a != kB4NotHeld) mem[kB4AdjAt + lane] = lane < da ? v.g2_adj[v.g2_off[x.a] + lane] : kNoNode;
    if (s.n_b != kB4NotHeld) mem[kB4AdjAt + kB4ShortAdj + lane] = lane < db ? v.g2_adj[v.g2_off[x.b] + lane] : kNoNode;
    if (s.n_c != kB4NotHeld) mem[kB4AdjAt + 2 * kB4ShortAdj + lane] = lane < dc ? v.g2_adj[v.g2_off[x.c] + lane] : kNoNode;
  }
  s.n_q = kB4NotHeld;
  if ((want & 64u) && x.len3 <= kWave) {
    bool hold = false;
    uint32_t y = 0;
    if (lane < x.len3 && pl.q_bits) {
      hold = true;
      y = pl.q_fourth[x.lo3 + lane];
    } else if (lane < x.len3) {
      const uint32_t* f = v.e4 + 4ull * v.i4_idx[x.lo3 + lane];
      const uint32_t f0 = f[0], f1 = f[1], f2 = f[2], f3 = f[3];
      const uint32_t hit = uint32_t(f0 == x.a || f0 == x.b || f0 == x.c) + uint32_t(f1 == x.a || f1 == x.b || f1 == x.c) +
                           uint32_t(f2 == x.a || f2 == x.b || f2 == x.c) + uint32_t(f3 == x.a || f3 == x.b || f3 == x.c);
      hold = hit == 3;
      y = f0 ^ f1 ^ f2 ^ f3 ^ x.a ^ x.b ^ x.c;
    }
    const unsigned long long m = __ballot(hold);
    const uint32_t nq = uint32_t(__popcll(m));
    if (nq <= kB4ShortQ) {
      if (lane < kB4ShortQ) mem[kB4QAt + lane] = kNoNode;
      wave_sync();
      if (hold) mem[kB4QAt + uint32_t(__popcll(m & below))] = y;
      s.n_q = nq;
    }
  }
  wave_sync();
  return s;
}

// Membership probes of b4_exception_node: with SEQ each test runs to its end
// where it starts, so that only its result stays live (fewer registers, for
// kernels where most tests are list comparisons); without, the first slot
// is loaded at the start and the tests of one node resolve together.
template <bool SEQ>
struct P128 {
  Probe128 p;
};
template <>
struct P128<true> {
  bool r;
};
template <bool SEQ>
struct P64 {
  Probe64 p;
};
template <>
struct P64<true> {
  bool r;
};
template <bool SEQ>
__device__ __forceinline__ P128<SEQ> p128_start(const Set128& s, Key128 k) {
  if constexpr (SEQ) return P128<true>{set128_has(s, k)};
  else return P128<false>{probe128_start(s, k)};
}
template <bool SEQ>
__device__ __forceinline__ P128<SEQ> p3_start(const Set128& s, uint32_t a, uint32_t b, uint32_t c) {
  sort3(a, b, c);
  return p128_start<SEQ>(s, key3(a, b, c));
}
template <bool SEQ>
__device__ __forceinline__ bool p128_end(const Set128& s, const P128<SEQ>& q) {
  if constexpr (SEQ) return q.r;
  else return probe128_end(s, q.p);
}
template <bool SEQ>
__device__ __forceinline__ P64<SEQ> p2_start(const Set64& s, uint32_t u, uint32_t w) {
  if constexpr (SEQ) return P64<true>{has2(s, u, w)};
  else return P64<false>{probe2_start(s, u, w)};
}
template <bool SEQ>
__device__ __forceinline__ bool p64_end(const Set64& s, const P64<SEQ>& q) {
  if constexpr (SEQ) return q.r;
  else return probe64_end(s, q.p);
}

// The exceptional node at flat position t of the ranges of x, each node
// once (by the first hyperedge that makes it exceptional).  Returns 0 when the
// position holds none; else bit 4 set, its pairwise combination in bits 0..2,
// bit 3 set when its set counts (not a 4-node hyperedge and, with OWN, e its
// smallest 3-node hyperedge), with the set's pattern in *pat.  With sh, the
// lists it holds replace the corresponding probes.
//
// b4_exception_node takes the node itself: y with its slot (0..2: the third
// node of a 3-node hyperedge on pair {a,b}, {a,c} or {b,c} of e, pair_adj its
// pairwise adjacency to that pair's lower and higher node in bits 0 and 1;
// 3: the fourth node of a 4-node hyperedge holding e, pair_adj unused).
template <bool OWN, bool SEQ = false>
__device__ __forceinline__ uint32_t b4_exception_node(const View& v, const PairLinks& pl, const B4Ctx& x, int slot,
                                                      uint32_t y, uint32_t pair_adj, uint32_t* pat,
                                                      const B4Short& sh) {
  const uint32_t a = x.a, b = x.b, c = x.c;
  const bool hab = sh.n_ab != kB4NotHeld, hac = sh.n_ac != kB4NotHeld, hbc = sh.n_bc != kB4NotHeld,
             hq = sh.n_q != kB4NotHeld;
  const bool ha = sh.n_a != kB4NotHeld, hb = sh.n_b != kB4NotHeld, hc = sh.n_c != kB4NotHeld;
  const int ra = x.ra, rb = x.rb, rc = x.rc;
  if (slot < 3) {
    if (y == a || y == b || y == c) return 0;   // e itself
    // The slot's own 3-node hyperedge {y} u pair comes after e only when y is
    // above m, the member of e outside the pair (c, b, a for slots 0, 1, 2).
    // Otherwise e is not the smallest 3-node hyperedge of e u {y}, so with
    // OWN the set is not counted here: y only needs the earlier-slot test
    // and its pair with m, for its pairwise combination.
    const uint32_t m = slot == 0 ? c : (slot == 1 ? b : a);
    if (OWN && y < m) {
      P128<SEQ> qab, qac;
      if (slot >= 1 && !hab) qab = p3_start<SEQ>(v.hs3, a, b, y);
      if (slot == 2 && !hac) qac = p3_start<SEQ>(v.hs3, a, c, y);
      // m's neighbours, when held: c's for slot 0, b's for slot 1, a's for slot 2
      const bool hm = slot == 0 ? hc : (slot == 1 ? hb : ha);
      const int rm = slot == 0 ? rc : (slot == 1 ? rb : ra);
      P64<SEQ> pm;
      if (!hm && rm < 0) pm = p2_start<SEQ>(v.hs2, m, y);
      if (slot >= 1 && (hab ? in_short(sh.mem, sh.n_ab, y) : p128_end<SEQ>(v.hs3, qab))) return 0;
      if (slot == 2 && (hac ? in_short(sh.mem + kB4ShortRun, sh.n_ac, y) : p128_end<SEQ>(v.hs3, qac))) return 0;
      const uint32_t mv =
          hm ? uint32_t(in_short(sh.mem + kB4AdjAt + (2 - uint32_t(slot)) * kB4ShortAdj,
                                 slot == 0 ? sh.n_c : (slot == 1 ? sh.n_b : sh.n_a), y))
             : (rm >= 0 ? hub_adj(pl, rm, y) : uint32_t(p64_end<SEQ>(v.hs2, pm)));
      const uint32_t lo = pair_adj & 1u, hi = pair_adj >> 1;
      const uint32_t av = slot == 2 ? mv : lo;
      const uint32_t bv = slot == 0 ? hi : (slot == 1 ? mv : lo);
      const uint32_t cv = slot == 0 ? mv : hi;
      return 16u | av | (bv << 1) | (cv << 2);
    }
  }
  // Every membership test the set e u {y} needs, issued together: the
  // 3-node sets through y not already known from the slot, the 4-node set
  // (unless the slot is the 4-node hyperedges'), y's pairs with a, b, c.
  P128<SEQ> pab, pac, pbc, pq;
  if (slot != 0 && !hab) pab = p3_start<SEQ>(v.hs3, a, b, y);
  if (slot != 1 && !hac) pac = p3_start<SEQ>(v.hs3, a, c, y);
  if (slot != 2 && !hbc) pbc = p3_start<SEQ>(v.hs3, b, c, y);
  if (slot < 3 && !hq) {
    uint32_t s0 = a, s1 = b, s2 = c, s3 = y;
    // ascending 4-tuple for the 4-node probe
    if (s3 < s2) { const uint32_t tt = s2; s2 = s3; s3 = tt; }
    if (s2 < s1) { const uint32_t tt = s1; s1 = s2; s2 = tt; }
    if (s1 < s0) { const uint32_t tt = s0; s0 = s1; s1 = tt; }
    pq = p128_start<SEQ>(v.hs4, key4(s0, s1, s2, s3));
  }
  // y's pairs with the two members of the slot's pair come with the entry
  P64<SEQ> pa, pb, pc;
  if ((slot == 2 || slot == 3) && !ha && ra < 0) pa = p2_start<SEQ>(v.hs2, a, y);
  if ((slot == 1 || slot == 3) && !hb && rb < 0) pb = p2_start<SEQ>(v.hs2, b, y);
  if ((slot == 0 || slot == 3) && !hc && rc < 0) pc = p2_start<SEQ>(v.hs2, c, y);
  const uint32_t abv =
      slot == 0 ? 1u : uint32_t(hab ? in_short(sh.mem, sh.n_ab, y) : p128_end<SEQ>(v.hs3, pab));
  const uint32_t acv =
      slot == 1 ? 1u : uint32_t(hac ? in_short(sh.mem + kB4ShortRun, sh.n_ac, y) : p128_end<SEQ>(v.hs3, pac));
  const uint32_t bcv =
      slot == 2 ? 1u : uint32_t(hbc ? in_short(sh.mem + 2 * kB4ShortRun, sh.n_bc, y) : p128_end<SEQ>(v.hs3, pbc));
  // each exceptional node once: a 3-node hyperedge of an earlier slot takes it
  if (slot == 1 && abv) return 0;
  if (slot == 2 && (abv || acv)) return 0;
  if (slot == 3 && (abv || acv || bcv)) return 0;
  const uint32_t quad =
      slot == 3 ? 1u : uint32_t(hq ? in_short(sh.mem + kB4QAt, sh.n_q, y) : p128_end<SEQ>(v.hs4, pq));
  const uint32_t av =
      slot == 0 || slot == 1
          ? (pair_adj & 1u)
          : (ha ? uint32_t(in_short(sh.mem + kB4AdjAt, sh.n_a, y))
                : (ra >= 0 ? hub_adj(pl, ra, y) : uint32_t(p64_end<SEQ>(v.hs2, pa))));
  const uint32_t bv =
      slot == 0 ? (pair_adj >> 1)
                : (slot == 2 ? (pair_adj & 1u)
                             : (hb ? uint32_t(in_short(sh.mem + kB4AdjAt + kB4ShortAdj, sh.n_b, y))
                                   : (rb >= 0 ? hub_adj(pl, rb, y) : uint32_t(p64_end<SEQ>(v.hs2, pb)))));
  const uint32_t cv =
      slot == 1 || slot == 2
          ? (pair_adj >> 1)
          : (hc ? uint32_t(in_short(sh.mem + kB4AdjAt + 2 * kB4ShortAdj, sh.n_c, y))
                : (rc >= 0 ? hub_adj(pl, rc, y) : uint32_t(p64_end<SEQ>(v.hs2, pc))));
  const uint32_t combo = av | (bv << 1) | (cv << 2);
  bool counted = !quad;   // a 4-node hyperedge: counted on its own, or larger than a sampled 3-node one
  if (OWN && counted) {
    // e must be the smallest 3-node hyperedge of the set
    uint32_t t0 = a, t1 = b, t2 = y;
    if (abv) { sort3(t0, t1, t2); counted = counted && !tri_less(t0, t1, t2, a, b, c); }
    t0 = a; t1 = c; t2 = y;
    if (acv) { sort3(t0, t1, t2); counted = counted && !tri_less(t0, t1, t2, a, b, c); }
    t0 = b; t1 = c; t2 = y;
    if (bcv) { sort3(t0, t1, t2); counted = counted && !tri_less(t0, t1, t2, a, b, c); }
  }
  *pat = x.base_p | (av << 4) | (bv << 5) | (abv << 6) | (cv << 7) | (acv << 8) | (bcv << 9);
  return 16u | (counted ? 8u : 0u) | combo;
}

template <bool OWN, bool SEQ = false>
__device__ __forceinline__ uint32_t b4_exception(const View& v, const PairLinks& pl, const B4Ctx& x, uint64_t t,
                                                 uint32_t* pat, const B4Short& sh) {
  // slot and offset of t, with constant indices only (registers)
  if (t < x.len0) {
    const uint64_t p = x.lo0 + t;
    return b4_exception_node<OWN, SEQ>(v, pl, x, 0, pl.third[p], pl.adj[p], pat, sh);
  }
  if (t < x.len0 + x.len1) {
    const uint64_t p = x.lo1 + (t - x.len0);
    return b4_exception_node<OWN, SEQ>(v, pl, x, 1, pl.third[p], pl.adj[p], pat, sh);
  }
  if (t < x.len0 + x.len1 + x.len2) {
    const uint64_t p = x.lo2 + (t - x.len0 - x.len1);
    return b4_exception_node<OWN, SEQ>(v, pl, x, 2, pl.third[p], pl.adj[p], pat, sh);
  }
  if (pl.q_bits) return b4_exception_node<OWN, SEQ>(v, pl, x, 3, pl.q_fourth[x.lo3 + (t - x.len0 - x.len1 - x.len2)], 0u,
                                              pat, sh);
  const uint32_t* f = v.e4 + 4ull * v.i4_idx[x.lo3 + (t - x.len0 - x.len1 - x.len2)];
  const uint32_t f0 = f[0], f1 = f[1], f2 = f[2], f3 = f[3];
  const uint32_t a = x.a, b = x.b, c = x.c;
  const uint32_t hit = uint32_t(f0 == a || f0 == b || f0 == c) + uint32_t(f1 == a || f1 == b || f1 == c) +
                       uint32_t(f2 == a || f2 == b || f2 == c) + uint32_t(f3 == a || f3 == b || f3 == c);
  if (hit != 3) return 0;
  return b4_exception_node<OWN, SEQ>(v, pl, x, 3, f0 ^ f1 ^ f2 ^ f3 ^ a ^ b ^ c, 0u, pat, sh);
}

// The combination pattern of e u {v} for a non-exceptional v.
__device__ inline uint32_t b4_combo_pattern(const B4Ctx& x, uint32_t cmb) {
  return x.base_p | ((cmb & 1u) << 4) | (((cmb >> 1) & 1u) << 5) | ((cmb >> 2) << 7);
}

// Exact counting (OWN = true) and the bit-free sampler's inline path: one
// wavefront per hyperedge.
template <bool OWN, bool SEQ = false>
__device__ void b4_sparse(const View& v, const PairLinks& pl, uint32_t a, uint32_t b, uint32_t c, const uint8_t* lut,
                          unsigned long long* h_main, unsigned long long* h_sub, uint32_t* short_mem = nullptr,
                          bool runs = true) {
  const int lane = threadIdx.x & (kWave - 1);
  const B4Ctx x = b4_ctx(v, pl, a, b, c);
  uint32_t n[8];
  b4_combo_counts(v, pl, x, n);
  const B4Short sh = short_mem ? b4_short(v, pl, x, short_mem) : b4_short_none();
  // exceptional nodes, in one lane-strided range; per lane, the number of
  // them in each pairwise combination
  uint32_t dn1 = 0, dn2 = 0, dn3 = 0, dn4 = 0, dn5 = 0, dn6 = 0, dn7 = 0;
  // without `runs`, the positions of the pair runs (slots 0..2) are left to
  // the pair-run pass (b4_run_entry), which adds their terms itself
  const uint64_t t0 = runs ? 0 : x.len0 + x.len1 + x.len2;
  for (uint64_t t = t0 + lane; t < x.total; t += kWave) {
    uint32_t pat;
    const uint32_t r = b4_exception<OWN, SEQ>(v, pl, x, t, &pat, sh);
    if (!r) continue;
    const uint32_t combo = r & 7u;
    dn1 += combo == 1;
    dn2 += combo == 2;
    dn3 += combo == 3;
    dn4 += combo == 4;
    dn5 += combo == 5;
    dn6 += combo == 6;
    dn7 += combo == 7;
    if (!(r & 8u)) continue;
    atomicAdd(&h_main[lut[pat]], 1ull);
    if (OWN) {
      const uint8_t g = lut[pat & kPairBits4];
      if (g != 0xFF) atomicAdd(&h_sub[g], 1ull);
    }
  }
  dn1 = wave_sum_u32(dn1);
  dn2 = wave_sum_u32(dn2);
  dn3 = wave_sum_u32(dn3);
  dn4 = wave_sum_u32(dn4);
  dn5 = wave_sum_u32(dn5);
  dn6 = wave_sum_u32(dn6);
  dn7 = wave_sum_u32(dn7);
  if (lane == 0) {
    n[1] -= dn1;
    n[2] -= dn2;
    n[3] -= dn3;
    n[4] -= dn4;
    n[5] -= dn5;
    n[6] -= dn6;
    n[7] -= dn7;
#pragma unroll
    for (uint32_t cmb = 1; cmb < 8; ++cmb) {
      if (!n[cmb]) continue;
      const uint32_t pat = b4_combo_pattern(x, cmb);
      atomicAdd(&h_main[lut[pat]], (unsigned long long)n[cmb]);
      if (OWN) {
        const uint8_t g = lut[pat & kPairBits4];
        if (g != 0xFF) atomicAdd(&h_sub[g], (unsigned long long)n[cmb]);
      }
    }
  }
}

// Position of node z among the third nodes of the run [lo, lo + len) (sorted),
// or ~0 when absent.
__device__ inline uint64_t run_find(const PairLinks& pl, uint64_t lo, uint32_t len, uint32_t z) {
  uint64_t l = lo, h = lo + len;   // pl.third[l..h) may hold z
  while (h > l) {
    const uint64_t m = l + ((h - l) >> 1);
    const uint32_t y = pl.third[m];
    if (y == z) return m;
    if (y < z) l = m + 1; else h = m;
  }
  return ~0ull;
}

// The pair-run terms of exact counting for entry p of the pair index: the
// 3-node hyperedge e = {x, y, t} (pair {x < y} of the entry's key, t its
// third node) against every other entry z of the same run, which are the
// positions of one slot of e's exception walk (slot 0, 1, 2 when the pair is
// {a,b}, {a,c}, {b,c} of e).  Every lane of the wavefront calls this.
//
// An entry z related to t in none of four ways (z a pairwise neighbour of t;
// {x,t,z} or {y,t,z} a 3-node hyperedge; {x,y,t,z} a 4-node hyperedge) has
// an outcome fixed by z's adjacency class to the pair (bits lo, hi) and by
// whether z < t: below t it is one more node of its combination (e does not
// own the set, whose 3-node hyperedge {x,y,z} precedes e); above t it is also
// counted once, its pattern holding e's pattern, z's two pairs and the
// 3-node hyperedge of the slot's pair.  Those are counted from the run's
// prefix counts by class.  The related entries are listed from t's side (its
// pairwise row, the runs of {x,t} and {y,t}, the 4-node hyperedges holding
// e; each node from the first list that holds it) and classified one by one
// as the exception walk does; when the run is not longer than those lists,
// the run itself is walked instead.
__device__ void b4_run_entry(const View& v, const PairLinks& pl, uint64_t p, const uint8_t* lut,
                             unsigned long long* h_main, unsigned long long* h_sub, uint32_t* short_mem) {
  const int lane = threadIdx.x & (kWave - 1);
  const unsigned long long key = pl.keys[p];
  const bool alone = (p == 0 || pl.keys[p - 1] != key) && (p + 1 == pl.n || pl.keys[p + 1] != key);
  if (alone) return;   // no other entry in the run
  const uint32_t px = uint32_t(key >> 32), py = uint32_t(key), t = pl.third[p];
  const int slot = t > py ? 0 : (t > px ? 1 : 2);
  const uint32_t a = slot == 2 ? t : px, b = slot == 0 ? py : (slot == 1 ? t : px), c = slot == 0 ? t : py;
  const uint32_t t_off = uniform_u32(v.g2_off[t]), dt = uniform_u32(v.g2_off[t + 1]) - t_off;
  const B4Ctx x = b4_ctx(v, pl, a, b, c);
  // the run of the pair
  const uint64_t lo = slot == 0 ? x.lo0 : (slot == 1 ? x.lo1 : x.lo2);
  const uint32_t L = uint32_t(slot == 0 ? x.len0 : (slot == 1 ? x.len1 : x.len2));
  // the runs of {x, t} and {y, t}
  const uint64_t lo_xt = slot == 0 ? x.lo1 : x.lo0;
  const uint32_t len_xt = uint32_t(slot == 0 ? x.len1 : x.len0);
  const uint64_t lo_yt = slot == 2 ? x.lo1 : x.lo2;
  const uint32_t len_yt = uint32_t(slot == 2 ? x.len1 : x.len2);
  const uint64_t listed = uint64_t(dt) + len_xt + len_yt + x.len3;
  const bool walk_run = uint64_t(L) - 1 <= listed;
  const int rt = slot == 0 ? x.rc : (slot == 1 ? x.rb : x.ra);   // t's dense row, or -1
  // the short lists this pass tests against, in LDS (at most 64 entries; the
  // 4-node hyperedges holding e): the runs of {x, t} and {y, t}, t's row;
  // membership tests against them are comparisons.  (The pair's own run and
  // the rows of x and y are never tested: the entries carry them.)
  const uint32_t want = (slot == 0 ? (2u | 4u | 32u) : (slot == 1 ? (1u | 4u | 16u) : (1u | 2u | 8u))) | 64u;
  const B4Short sh = b4_short(v, pl, x, short_mem, want);
  const bool ht = (slot == 0 ? sh.n_c : (slot == 1 ? sh.n_b : sh.n_a)) != kB4NotHeld;
  const uint32_t* t_row = sh.mem + kB4AdjAt + (slot == 0 ? 2u : (slot == 1 ? 1u : 0u)) * kB4ShortAdj;
  // runs of {x, t} and {y, t} among e's three pair runs: slot 0 holds them at
  // ac, bc; slot 1 at ab, bc; slot 2 at ab, ac
  const uint32_t n_xt = slot == 0 ? sh.n_ac : sh.n_ab, n_yt = slot == 2 ? sh.n_ac : sh.n_bc;
  const uint32_t* xt_list = sh.mem + (slot == 0 ? kB4ShortRun : 0u);
  const uint32_t* yt_list = sh.mem + (slot == 2 ? kB4ShortRun : 2 * kB4ShortRun);
  uint32_t dn1 = 0, dn2 = 0, dn3 = 0, dn4 = 0, dn5 = 0, dn6 = 0, dn7 = 0;
  uint32_t ml0 = 0, ml1 = 0, ml2 = 0, ml3 = 0, mg0 = 0, mg1 = 0, mg2 = 0, mg3 = 0;
  const uint64_t n_items = walk_run ? L : listed;
  for (uint64_t q = lane; q < n_items; q += kWave) {
    uint32_t z, cls;
    if (walk_run) {
      if (lo + q == p) continue;
      z = pl.third[lo + q];
      cls = pl.adj[lo + q];
    } else {
      int src;
      if (q < dt) {
        z = v.g2_adj[t_off + q];
        src = 0;
      } else if (q < uint64_t(dt) + len_xt) {
        z = pl.third[lo_xt + (q - dt)];
        src = 1;
      } else if (q < uint64_t(dt) + len_xt + len_yt) {
        z = pl.third[lo_yt + (q - dt - len_xt)];
        src = 2;
      } else if (pl.q_bits) {
        z = pl.q_fourth[x.lo3 + (q - dt - len_xt - len_yt)];
        src = 3;
      } else {
        const uint32_t* f = v.e4 + 4ull * v.i4_idx[x.lo3 + (q - dt - len_xt - len_yt)];
        const uint32_t f0 = f[0], f1 = f[1], f2 = f[2], f3 = f[3];
        const uint32_t hit = uint32_t(f0 == a || f0 == b || f0 == c) + uint32_t(f1 == a || f1 == b || f1 == c) +
                             uint32_t(f2 == a || f2 == b || f2 == c) + uint32_t(f3 == a || f3 == b || f3 == c);
        if (hit != 3) continue;
        z = f0 ^ f1 ^ f2 ^ f3 ^ a ^ b ^ c;
        src = 3;
      }
      if (z == px || z == py || z == t) continue;
      // each related node once, from the first list holding it
      if (src >= 1 &&
          (ht ? in_short(t_row, slot == 0 ? sh.n_c : (slot == 1 ? sh.n_b : sh.n_a), z)
              : (rt >= 0 ? hub_adj(pl, rt, z) : uint32_t(has2(v.hs2, t, z)))))
        continue;
      if (src >= 2) {
        uint32_t s0 = px, s1 = t, s2 = z;
        sort3(s0, s1, s2);
        if (n_xt != kB4NotHeld ? in_short(xt_list, n_xt, z) : set128_has(v.hs3, key3(s0, s1, s2))) continue;
      }
      if (src >= 3) {
        uint32_t s0 = py, s1 = t, s2 = z;
        sort3(s0, s1, s2);
        if (n_yt != kB4NotHeld ? in_short(yt_list, n_yt, z) : set128_has(v.hs3, key3(s0, s1, s2))) continue;
      }
      const uint64_t j = run_find(pl, lo, L, z);
      if (j == ~0ull) continue;   // {x, y, z} is not a 3-node hyperedge
      cls = pl.adj[j];
      const bool below = z < t;
      ml0 += below && cls == 0;
      ml1 += below && cls == 1;
      ml2 += below && cls == 2;
      ml3 += below && cls == 3;
      mg0 += !below && cls == 0;
      mg1 += !below && cls == 1;
      mg2 += !below && cls == 2;
      mg3 += !below && cls == 3;
    }
    uint32_t pat;
    const uint32_t r = b4_exception_node<true, true>(v, pl, x, slot, z, cls, &pat, sh);
    if (!r) continue;
    const uint32_t combo = r & 7u;
    dn1 += combo == 1;
    dn2 += combo == 2;
    dn3 += combo == 3;
    dn4 += combo == 4;
    dn5 += combo == 5;
    dn6 += combo == 6;
    dn7 += combo == 7;
    if (!(r & 8u)) continue;
    atomicAdd(&h_main[lut[pat]], 1ull);
    const uint8_t g = lut[pat & kPairBits4];
    if (g != 0xFF) atomicAdd(&h_sub[g], 1ull);
  }
  uint32_t dn[8];
  dn[0] = 0;
  dn[1] = wave_sum_u32(dn1);
  dn[2] = wave_sum_u32(dn2);
  dn[3] = wave_sum_u32(dn3);
  dn[4] = wave_sum_u32(dn4);
  dn[5] = wave_sum_u32(dn5);
  dn[6] = wave_sum_u32(dn6);
  dn[7] = wave_sum_u32(dn7);
  // walking the lists: the related entries by class below and above t,
  // whose complement the prefix counts give
  uint32_t ml[4] = {0, 0, 0, 0}, mg[4] = {0, 0, 0, 0};
  if (!walk_run) {
    ml[0] = wave_sum_u32(ml0);
    ml[1] = wave_sum_u32(ml1);
    ml[2] = wave_sum_u32(ml2);
    ml[3] = wave_sum_u32(ml3);
    mg[0] = wave_sum_u32(mg0);
    mg[1] = wave_sum_u32(mg1);
    mg[2] = wave_sum_u32(mg2);
    mg[3] = wave_sum_u32(mg3);
  }
  if (lane != 0) return;
  // the unrelated entries, by class, below and above t (constant indices
  // only, so that the arrays stay in registers)
  uint32_t all[4] = {0, 0, 0, 0}, cmb_of[4] = {0, 0, 0, 0};
  if (!walk_run) {
    const uint64_t n1 = pl.n + 1;
#pragma unroll
    for (uint32_t cl = 0; cl < 4; ++cl) {
      const uint32_t* pre = pl.pre + cl * n1;
      const uint32_t nl = (pre[p] - pre[lo]) - ml[cl];
      const uint32_t ng = (pre[lo + L] - pre[p + 1]) - mg[cl];
      const uint32_t l = cl & 1u, h = cl >> 1;
      cmb_of[cl] = slot == 0 ? (l | (h << 1)) : (slot == 1 ? (l | (h << 2)) : ((l << 1) | (h << 2)));
      all[cl] = nl + ng;
      if (!ng) continue;
      const uint32_t pat = slot == 0 ? (x.base_p | (l << 4) | (h << 5) | (1u << 6))
                                     : (slot == 1 ? (x.base_p | (l << 4) | (h << 7) | (1u << 8))
                                                  : (x.base_p | (l << 5) | (h << 7) | (1u << 9)));
      atomicAdd(&h_main[lut[pat]], (unsigned long long)ng);
      const uint8_t g = lut[pat & kPairBits4];
      if (g != 0xFF) atomicAdd(&h_sub[g], (unsigned long long)ng);
    }
  }
  // every exceptional node of the slot is one fewer of its combination
#pragma unroll
  for (uint32_t cmb = 1; cmb < 8; ++cmb) {
#pragma unroll
    for (uint32_t cl = 0; cl < 4; ++cl) dn[cmb] += cmb_of[cl] == cmb ? all[cl] : 0u;
    if (!dn[cmb]) continue;
    const uint32_t pat = b4_combo_pattern(x, cmb);
    atomicAdd(&h_main[lut[pat]], 0ull - (unsigned long long)dn[cmb]);
    const uint8_t g = lut[pat & kPairBits4];
    if (g != 0xFF) atomicAdd(&h_sub[g], 0ull - (unsigned long long)dn[cmb]);
  }
}

}  // namespace hm
