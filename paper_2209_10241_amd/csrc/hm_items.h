// Per-item bodies of the exact counting kernels, shared by the one-graph
// kernels (exact.hip) and the persistent batched kernel of the null model
// (nulls_batch.hip).  A View holds the device structures of one hypergraph
// (or of one null copy); incidence indices are positions in e3 / e4.
//
// Order 4 (Algorithm 3, Section 4.2), with the "visited" set replaced by
// ownership rules decided from the node set alone:
//   (a) a 4-node hyperedge counts its own node set;
//   (b) a set that is not a 4-node hyperedge but holds a 3-node hyperedge is
//       counted by its smallest 3-node hyperedge (hm_b4.h);
//   (c) a set whose sub-hypergraph holds only pairs is a connected 4-node set
//       of the pairwise graph G2 that (a) and (b) did not count: the pairwise
//       graph's connected 4-node sets are counted per induced shape (each set
//       from its smallest node r), and the shapes of the G2-connected sets
//       counted by (a) and (b) are subtracted.
// Order 3 (Algorithm 2): (a) each 3-node hyperedge, (c) wedges and triangles
// of G2 minus those that are 3-node hyperedges.
#pragma once

#include "hm_b4.h"

namespace hm {

struct View {
  const uint32_t* e2;       // pairs (r < x) of this graph
  const uint32_t* e3;       // 3-node hyperedges (positions referenced by i3_idx)
  const uint32_t* e4;       // 4-node hyperedges (positions referenced by i4_idx)
  const uint32_t* g2_off;   // n_nodes + 1 absolute row starts in g2_adj
  const uint32_t* g2_adj;   // ascending neighbour rows
  const uint32_t* i3_off;
  const uint32_t* i3_idx;
  const uint32_t* i4_off;
  const uint32_t* i4_idx;
  const uint32_t* i3_oth;               // with bit rows: others3 of each i3 entry
  const unsigned long long* i4_oth;     // with bit rows: others4 of each i4 entry
  Set64 hs2;
  Set128 hs3, hs4;
  const uint32_t* bits;     // n_nodes x W words, or null
  uint32_t W;
  uint32_t N;
};

inline View view_of(const hm_graph* H) {
  View v;
  v.e2 = H->e2;
  v.e3 = H->e3;
  v.e4 = H->e4;
  v.g2_off = H->g2_off;
  v.g2_adj = H->g2_adj;
  v.i3_off = H->i3_off;
  v.i3_idx = H->i3_idx;
  v.i4_off = H->i4_off;
  v.i4_idx = H->i4_idx;
  v.i3_oth = H->i3_oth;
  v.i4_oth = H->i4_oth;
  v.hs2 = H->hs2;
  v.hs3 = H->hs3;
  v.hs4 = H->hs4;
  v.bits = H->bits;
  v.W = H->words;
  v.N = H->n_nodes;
  return v;
}

// histogram regions (256 counters each)
constexpr int kMain = 0;    // classes counted by (a) and (b)
constexpr int kSub = 256;   // G2 shape of G2-connected sets counted by (a) and (b)
constexpr int kG2 = 512;    // G2 shape counts of all connected sets of G2
constexpr int kHistWords = 768;
constexpr int kIdAcc = 768;  // the seven sums of the identity route for (c) (exact counts only)

// (a) at order 4: the pattern of a 4-node hyperedge; local positions a..d = 0..3
// (the four 3-node probes are started together and resolved afterwards, so
// that their first loads are in flight at once)
__device__ inline uint32_t a4_pattern(const View& v, uint32_t a, uint32_t b, uint32_t c, uint32_t d) {
  const Probe128 q3 = probe128_start(v.hs3, key3(a, b, c)), q6 = probe128_start(v.hs3, key3(a, b, d)),
                 q8 = probe128_start(v.hs3, key3(a, c, d)), q9 = probe128_start(v.hs3, key3(b, c, d));
  uint32_t p = 1u << 10;
  p |= pair_bit(v.hs2, v.bits, v.W, a, b) << 0;
  p |= pair_bit(v.hs2, v.bits, v.W, a, c) << 1;
  p |= pair_bit(v.hs2, v.bits, v.W, b, c) << 2;
  p |= pair_bit(v.hs2, v.bits, v.W, a, d) << 4;
  p |= pair_bit(v.hs2, v.bits, v.W, b, d) << 5;
  p |= pair_bit(v.hs2, v.bits, v.W, c, d) << 7;
  p |= uint32_t(probe128_end(v.hs3, q3)) << 3;
  p |= uint32_t(probe128_end(v.hs3, q6)) << 6;
  p |= uint32_t(probe128_end(v.hs3, q8)) << 8;
  p |= uint32_t(probe128_end(v.hs3, q9)) << 9;
  return p;
}

// (a) at order 3: the pattern of a 3-node hyperedge; local positions a,b,c = 0,1,2
__device__ inline uint32_t a3_pattern(const View& v, uint32_t a, uint32_t b, uint32_t c) {
  return (1u << 3) | pair_bit(v.hs2, v.bits, v.W, a, b) | (pair_bit(v.hs2, v.bits, v.W, a, c) << 1) |
         (pair_bit(v.hs2, v.bits, v.W, b, c) << 2);
}

// (b) at order 4 for the 3-node hyperedge at position i of v.e3
__device__ inline void b4_item(const View& v, uint64_t i, uint32_t* sets, const uint8_t* lut, unsigned long long* h_main,
                               unsigned long long* h_sub) {
  const uint32_t a = v.e3[3 * i], b = v.e3[3 * i + 1], c = v.e3[3 * i + 2];
  if (v.bits)
    b4_edge_bits_count<true>(a, b, c, v.i3_off, v.i3_oth, v.i4_off, v.i4_oth, v.bits, v.W, sets, lut, h_main, h_sub);
  else
    b4_edge_hash<true>(a, b, c, v.e3, v.g2_off, v.g2_adj, v.i3_off, v.i3_idx, v.hs2, v.hs3, v.hs4, lut, h_main, h_sub);
}

// ---------------------------------------------------------------- (c), order 4, bit rows
// One wavefront per pair {r < x}.  Shapes with A = N(r) n V':
//   |A| = 3: {r,x,y,z}, x<y<z all neighbours of r
//   |A| = 2: x<y neighbours of r, z > r not a neighbour of r, adjacent to x or y
//   |A| = 1: x the only neighbour of r; y,z > r non-neighbours of r with
//            {x,y,z} connected: y<z both adjacent to x, or y~x, z~y, z!~x.
// A row has W words.  With W <= 64 the wavefront is split into 64/W groups of
// W lanes, lane (g, w) owning word w of every y its group takes, so the words
// of r and x and the masks that depend only on r are loaded once per pair;
// wider rows loop over words.  Each word adds popcounts of the candidate z it
// holds, split by the adjacency of z to x and y.  The y of a batch are
// ordered with those not adjacent to x first, so that x~y is fixed within
// each of the two inner loops.
// Named scalars (no arrays) keep every counter in registers.  Counters are
// 32-bit: one pair adds at most 32 * 4 * 8192 < 2^20 to a lane's counter, so
// flushing every kC4FlushItems pairs keeps them below 2^31.
constexpr uint32_t kC4FlushItems = 2048;

struct C4Acc {
  // |A| = 3, by (x~y, x~z, y~z)
  uint32_t a000, a001, a010, a011, a100, a101, a110, a111;
  // |A| = 2, by x~y and z adjacent to both / x only / y only
  uint32_t b0b, b0x, b0y, b1b, b1x, b1y;
  // |A| = 1
  uint32_t paw, star, path;
  uint32_t items;   // pairs since the last flush
};

struct C4Lanes {
  uint32_t G, g, w0, wstep;
  bool on;
};

__device__ inline C4Lanes c4_lanes(uint32_t W) {
  const int lane = threadIdx.x & (kWave - 1);
  const bool grouped = W <= uint32_t(kWave);
  C4Lanes L;
  L.G = grouped ? uint32_t(kWave) / W : 1u;
  L.g = grouped ? uint32_t(lane) / W : 0u;
  L.w0 = grouped ? uint32_t(lane) % W : uint32_t(lane);
  L.wstep = grouped ? W : uint32_t(kWave);
  L.on = grouped ? (L.g < L.G) : true;
  return L;
}

__device__ inline void c4_zero(C4Acc& a) {
  a.a000 = a.a001 = a.a010 = a.a011 = a.a100 = a.a101 = a.a110 = a.a111 = 0;
  a.b0b = a.b0x = a.b0y = a.b1b = a.b1x = a.b1y = 0;
  a.paw = a.star = a.path = 0;
  a.items = 0;
}

// one word of z candidates for a y with x~y = XY
template <bool XY>
__device__ inline void c4_word(uint32_t Nr, uint32_t Nx, uint32_t Ny, uint32_t gy, uint32_t wr, C4Acc& a) {
  const uint32_t z3 = Nr & gy;
  const uint32_t z2 = wr & (Nx | Ny);
  if (XY) {
    a.a111 += __popc(z3 & Nx & Ny);
    a.a110 += __popc(z3 & Nx & ~Ny);
    a.a101 += __popc(z3 & ~Nx & Ny);
    a.a100 += __popc(z3 & ~Nx & ~Ny);
    a.b1b += __popc(z2 & Nx & Ny);
    a.b1x += __popc(z2 & Nx & ~Ny);
    a.b1y += __popc(z2 & ~Nx & Ny);
  } else {
    a.a011 += __popc(z3 & Nx & Ny);
    a.a010 += __popc(z3 & Nx & ~Ny);
    a.a001 += __popc(z3 & ~Nx & Ny);
    a.a000 += __popc(z3 & ~Nx & ~Ny);
    a.b0b += __popc(z2 & Nx & Ny);
    a.b0x += __popc(z2 & Nx & ~Ny);
    a.b0y += __popc(z2 & ~Nx & Ny);
  }
}

// Number of set bits of the bit row R (W words) at positions <= x; every
// lane of the wavefront calls this and receives the count.
__device__ inline uint32_t bits_upto(const uint32_t* R, uint32_t W, uint32_t x) {
  const uint32_t lane = threadIdx.x & (kWave - 1);
  const uint32_t xw = x >> 5;
  uint32_t c = 0;
  for (uint32_t w = lane; w < W && w <= xw; w += kWave) {
    const uint32_t m = w < xw ? ~0u : (0xFFFFFFFFu >> (31 - (x & 31)));
    c += __popc(R[w] & m);
  }
  return wave_sum_u32(c);
}

__device__ inline void c4_flush(const C4Acc& a, const uint8_t* lut, unsigned long long* h_g2);

// ys: 64 words of wavefront-private LDS.  Every lane of the wavefront calls
// this; the counters go to h_g2 (LDS) every kC4FlushItems pairs and at
// c4_flush.
__device__ inline void c4_bits_item(const View& v, uint32_t r, uint32_t x, const C4Lanes& L, uint32_t* ys, C4Acc& acc,
                                    const uint8_t* lut, unsigned long long* h_g2) {
  const int lane = threadIdx.x & (kWave - 1);
  const uint32_t W = v.W;
  const uint32_t* Rr = v.bits + uint64_t(r) * W;
  const uint32_t* Rx = v.bits + uint64_t(x) * W;
  const uint32_t re = v.g2_off[r + 1];
  const uint32_t xe = v.g2_off[x + 1];
  // first neighbour of r above x and of x above r: the row start plus the
  // number of set bits up to x (up to r) in the bit row
  const uint32_t p = v.g2_off[r] + bits_upto(Rr, W, x);
  const uint32_t q = v.g2_off[x] + bits_upto(Rx, W, r);
  const unsigned long long below = (1ull << lane) - 1ull;
  // |A| = 3 and |A| = 2: y over the neighbours of r above x, 64 at a time
  for (uint32_t base = p; base < re; base += kWave) {
    const uint32_t cnt = min(uint32_t(kWave), re - base);
    const bool in = uint32_t(lane) < cnt;
    const uint32_t y0 = in ? v.g2_adj[base + lane] : 0u;
    const bool xy0 = in && ((Rx[y0 >> 5] >> (y0 & 31)) & 1u);
    const unsigned long long m0 = __ballot(in && !xy0), m1 = __ballot(xy0);
    const uint32_t n0 = uint32_t(__popcll(m0));
    if (in) ys[xy0 ? n0 + uint32_t(__popcll(m1 & below)) : uint32_t(__popcll(m0 & below))] = y0;
    wave_sync();
    if (L.on)
      for (uint32_t w = L.w0; w < W; w += L.wstep) {
        const uint32_t Nr = Rr[w], Nx = Rx[w];
        const uint32_t wr = ~Nr & mask_gt(r, w) & mask_below(v.N, w);
        for (uint32_t j = L.g; j < n0; j += L.G) {
          const uint32_t y = ys[j];
          c4_word<false>(Nr, Nx, v.bits[uint64_t(y) * W + w], mask_gt(y, w), wr, acc);
        }
        for (uint32_t j = n0 + L.g; j < cnt; j += L.G) {
          const uint32_t y = ys[j];
          c4_word<true>(Nr, Nx, v.bits[uint64_t(y) * W + w], mask_gt(y, w), wr, acc);
        }
      }
    wave_sync();
  }
  // |A| = 1: y over the neighbours of x above r that are not neighbours of r
  for (uint32_t base = q; base < xe; base += kWave) {
    const bool in = base + lane < xe;
    const uint32_t y0 = in ? v.g2_adj[base + lane] : 0u;
    const bool keep = in && !((Rr[y0 >> 5] >> (y0 & 31)) & 1u);
    const unsigned long long mk = __ballot(keep);
    const uint32_t cnt = uint32_t(__popcll(mk));
    if (keep) ys[__popcll(mk & below)] = y0;
    wave_sync();
    if (L.on)
      for (uint32_t w = L.w0; w < W; w += L.wstep) {
        const uint32_t Nr = Rr[w], Nx = Rx[w];
        const uint32_t wr = ~Nr & mask_gt(r, w) & mask_below(v.N, w);
        const uint32_t nxw = Nx & wr;
        const uint32_t pw = wr & ~Nx;
        for (uint32_t j = L.g; j < cnt; j += L.G) {
          const uint32_t y = ys[j];
          const uint32_t Ny = v.bits[uint64_t(y) * W + w];
          const uint32_t zz = nxw & mask_gt(y, w);
          acc.paw += __popc(zz & Ny);
          acc.star += __popc(zz & ~Ny);
          acc.path += __popc(Ny & pw);
        }
      }
    wave_sync();
  }
  if (++acc.items == kC4FlushItems) {
    c4_flush(acc, lut, h_g2);
    c4_zero(acc);
  }
}

// Reduce the accumulators over the wavefront and add them to the G2-shape
// counters h_g2 (lane 0 adds); every lane of the wavefront must call this.
__device__ inline void c4_emit(uint32_t value, uint32_t pattern, const uint8_t* lut, unsigned long long* h_g2) {
  const unsigned long long sum = wave_sum((unsigned long long)value);
  if ((threadIdx.x & (kWave - 1)) == 0 && sum) atomicAdd(&h_g2[lut[pattern]], sum);
}

__device__ inline void c4_flush(const C4Acc& a, const uint8_t* lut, unsigned long long* h_g2) {
  // local positions r=0, x=1, y=2, z=3; pair bits: rx 0, ry 1, xy 2, rz 4, xz 5, yz 7
  constexpr uint32_t rx = 1u << 0, ry = 1u << 1, xy = 1u << 2, rz = 1u << 4, xz = 1u << 5, yz = 1u << 7;
  c4_emit(a.a000, rx | ry | rz, lut, h_g2);
  c4_emit(a.a001, rx | ry | rz | yz, lut, h_g2);
  c4_emit(a.a010, rx | ry | rz | xz, lut, h_g2);
  c4_emit(a.a011, rx | ry | rz | xz | yz, lut, h_g2);
  c4_emit(a.a100, rx | ry | xy | rz, lut, h_g2);
  c4_emit(a.a101, rx | ry | xy | rz | yz, lut, h_g2);
  c4_emit(a.a110, rx | ry | xy | rz | xz, lut, h_g2);
  c4_emit(a.a111, rx | ry | xy | rz | xz | yz, lut, h_g2);
  c4_emit(a.b0b, rx | ry | xz | yz, lut, h_g2);
  c4_emit(a.b0x, rx | ry | xz, lut, h_g2);
  c4_emit(a.b0y, rx | ry | yz, lut, h_g2);
  c4_emit(a.b1b, rx | ry | xy | xz | yz, lut, h_g2);
  c4_emit(a.b1x, rx | ry | xy | xz, lut, h_g2);
  c4_emit(a.b1y, rx | ry | xy | yz, lut, h_g2);
  c4_emit(a.paw, rx | xy | xz | yz, lut, h_g2);
  c4_emit(a.star, rx | xy | xz, lut, h_g2);
  c4_emit(a.path, rx | xy | yz, lut, h_g2);
}

// ---------------------------------------------------------------- (c), order 4, by graph identities
// The induced pairwise shapes of G2's connected 4-node sets follow from seven
// sums over G2 (each a count of non-induced copies of a small graph):
//   t3   = sum over edges of t_e (|N(u) n N(v)|; = 3 x triangles)
//   p4   = sum over edges of (d_u - 1)(d_v - 1)   (3-paths, plus 3 x triangles)
//   dia  = sum over edges of C(t_e, 2)           (diamonds through their diagonal)
//   paw2 = sum over edges of t_e (d_u + d_v - 4) (= 2 x sum over nodes t_v (d_v - 2))
//   k4   = 4-cliques, each from its smallest edge {u < v}: pairs w < x of
//          common neighbours above v with w ~ x
//   c4x2 = sum over node pairs u < w of C(|N(u) n N(w)|, 2) (= 2 x 4-cycles)
//   star = sum over nodes of C(d, 3)
// and k_combine turns them into induced counts by inverting the containment
// of each shape in the larger ones.  Edge items (one per edge of G2) and node
// items (one per node) run on bit rows.
struct IdAcc {
  unsigned long long t3, p4, dia, paw2, k4, c4x2, star;
};

__device__ inline void id_zero(IdAcc& a) { a.t3 = a.p4 = a.dia = a.paw2 = a.k4 = a.c4x2 = a.star = 0; }

// degree of node x from the row starts
__device__ inline uint32_t g2_degree(const View& v, uint32_t x) { return v.g2_off[x + 1] - v.g2_off[x]; }

// Edges among the listed common neighbours ys[0..cnt) of {u, x} (all above
// x): lane (g, word) of C4Lanes takes the w of its group and adds the
// popcount of C'[word] & N(w)[word] above w.
__device__ inline void id_k4_list(const View& v, const uint32_t* Ru, const uint32_t* Rx, uint32_t x, const C4Lanes& L,
                                  const uint32_t* ys, uint32_t cnt, IdAcc& acc) {
  if (!L.on) return;
  const uint32_t W = v.W;
  for (uint32_t ww = L.w0; ww < W; ww += L.wstep) {
    const uint32_t cw = Ru[ww] & Rx[ww] & mask_gt(x, ww);
    if (!cw) continue;
    uint32_t k = 0;
    for (uint32_t j = L.g; j < cnt; j += L.G) {
      const uint32_t y = ys[j];
      k += __popc(cw & v.bits[uint64_t(y) * W + ww] & mask_gt(y, ww));
    }
    acc.k4 += k;
  }
}

// One wavefront per edge {u < x}; ys: 64 words of wavefront-private LDS.
// The common neighbours above x, C', are listed in ys (each lane writing the
// set bits of its word at its offset in a wavefront scan) when they number
// at most 64, else taken one set bit per lane per round.
__device__ inline void id_edge_item(const View& v, uint32_t u, uint32_t x, const C4Lanes& L, uint32_t* ys,
                                    IdAcc& acc) {
  const uint32_t lane = threadIdx.x & (kWave - 1);
  const uint32_t W = v.W;
  const uint32_t* Ru = v.bits + uint64_t(u) * W;
  const uint32_t* Rx = v.bits + uint64_t(x) * W;
  uint32_t t_lane = 0, c_word = 0;
  for (uint32_t w = lane; w < W; w += kWave) {
    const uint32_t cn = Ru[w] & Rx[w];
    t_lane += __popc(cn);
    if (w < uint32_t(kWave)) c_word = cn & mask_gt(x, w);
  }
  const uint32_t t = wave_sum_u32(t_lane);
  if (lane == 0) {
    const unsigned long long du = g2_degree(v, u), dx = g2_degree(v, x), tt = t;
    acc.t3 += tt;
    acc.p4 += (du - 1) * (dx - 1);
    acc.dia += tt * (tt - 1) / 2;
    if (tt) acc.paw2 += tt * (du + dx - 4);   // then du, dx >= t + 1 >= 2
  }
  if (t < 2) return;   // a 4-clique on {u, x} needs two common neighbours
  if (W <= uint32_t(kWave)) {
    uint32_t total;
    uint32_t off = wave_exclusive_scan(__popc(c_word), &total);
    if (total <= uint32_t(kWave)) {
      for (uint32_t b = c_word; b; b &= b - 1) ys[off++] = (lane << 5) | uint32_t(__ffs(b) - 1);
      wave_sync();
      id_k4_list(v, Ru, Rx, x, L, ys, total, acc);
      wave_sync();
      return;
    }
  }
  for (uint32_t w0 = 0; w0 < W; w0 += kWave) {
    const uint32_t w = w0 + lane;
    uint32_t word = w < W ? (Ru[w] & Rx[w] & mask_gt(x, w)) : 0u;
    while (__ballot(word != 0)) {
      const bool has = word != 0;
      const unsigned long long m = __ballot(has);
      if (has) {
        ys[__popcll(m & ((1ull << lane) - 1ull))] = (w << 5) | uint32_t(__ffs(word) - 1);
        word &= word - 1;
      }
      wave_sync();
      id_k4_list(v, Ru, Rx, x, L, ys, uint32_t(__popcll(m)), acc);
      wave_sync();
    }
  }
}

// One wavefront per node u: C(d_u, 3), and C(|N(u) n N(w)|, 2) for every
// w > u, one w per lane.
__device__ inline void id_node_item(const View& v, uint32_t u, IdAcc& acc) {
  const uint32_t lane = threadIdx.x & (kWave - 1);
  const uint32_t W = v.W;
  if (lane == 0) {
    const unsigned long long d = g2_degree(v, u);
    acc.star += d < 3 ? 0ull : d * (d - 1) * (d - 2) / 6;
  }
  if (g2_degree(v, u) < 2) return;   // no pair of neighbours, no C(c, 2)
  const uint32_t* Ru = v.bits + uint64_t(u) * W;
  for (uint32_t w = u + 1 + lane; w < v.N; w += kWave) {
    const uint32_t* Rw = v.bits + uint64_t(w) * W;
    uint32_t c = 0;
    for (uint32_t j = 0; j < W; ++j) c += __popc(Ru[j] & Rw[j]);
    acc.c4x2 += c < 2 ? 0ull : (unsigned long long)c * (c - 1) / 2;
  }
}

// The identity route runs while the node items' codegrees (every node pair,
// W words each) stay within this many word operations.
constexpr uint64_t kIdPairWordsMax = 1ull << 28;

__host__ __device__ inline bool use_identities(uint32_t N, uint32_t W) {
  return uint64_t(N) * N * W / 2 <= kIdPairWordsMax;
}

// Classes of the six connected 4-node graphs; with `on`, their G2 counts come
// from the seven identity sums rather than from the G2 region.
struct IdShapes {
  int on;
  int path, star, cycle, paw, diamond, clique;
};

// Induced count of class c's pairwise shape from the seven sums (0 for a
// class that is not one of the six shapes): each shape's copies inside the
// larger shapes are subtracted, largest first.
__device__ inline unsigned long long id_shape_count(const unsigned long long* ids, const IdShapes& sh, int c) {
  const unsigned long long T = ids[0] / 3, k4 = ids[4];
  const unsigned long long dia = ids[2] - 6 * k4;
  const unsigned long long cyc = ids[5] / 2 - dia - 3 * k4;
  const unsigned long long paw = ids[3] / 2 - 4 * dia - 12 * k4;
  const unsigned long long star = ids[6] - paw - 2 * dia - 4 * k4;
  const unsigned long long path = (ids[1] - 3 * T) - 4 * cyc - 2 * paw - 6 * dia - 12 * k4;
  return c == sh.clique ? k4 : c == sh.diamond ? dia : c == sh.cycle ? cyc : c == sh.paw ? paw
         : c == sh.star ? star : c == sh.path ? path : 0ull;
}

// Reduce the sums over the wavefront and add them to the seven counters at
// h_acc (LDS or device memory); every lane of the wavefront must call this.
__device__ inline void id_flush(const IdAcc& a, unsigned long long* h_acc) {
  const unsigned long long s[7] = {wave_sum(a.t3), wave_sum(a.p4),   wave_sum(a.dia), wave_sum(a.paw2),
                                   wave_sum(a.k4), wave_sum(a.c4x2), wave_sum(a.star)};
  if ((threadIdx.x & (kWave - 1)) == 0)
    for (int i = 0; i < 7; ++i)
      if (s[i]) atomicAdd(&h_acc[i], s[i]);
}

// ---------------------------------------------------------------- (c), order 4, hash set
// The same shapes enumerated one set at a time with pair lookups in the hash
// set (used when no bit rows are kept).  One wavefront per pair, lanes over y.
__device__ inline void c4_hash_item(const View& v, uint32_t r, uint32_t x, const uint8_t* lut,
                                    unsigned long long* h_g2) {
  const int lane = threadIdx.x & (kWave - 1);
  const uint32_t* adj = v.g2_adj;
  const uint32_t rb = v.g2_off[r], re = v.g2_off[r + 1];
  const uint32_t xb = v.g2_off[x], xe = v.g2_off[x + 1];
  const uint32_t p = upper_bound(adj, rb, re, x);
  // |A| = 3 and |A| = 2
  for (uint32_t yi = p + lane; yi < re; yi += kWave) {
    const uint32_t y = adj[yi];
    const uint32_t xy = has2(v.hs2, x, y);
    for (uint32_t zi = yi + 1; zi < re; ++zi) {   // z > y, z ~ r
      const uint32_t z = adj[zi];
      const uint32_t pz = (1u << 0) | (1u << 1) | (xy << 2) | (1u << 4) | (uint32_t(has2(v.hs2, x, z)) << 5) |
                          (uint32_t(has2(v.hs2, y, z)) << 7);
      atomicAdd(&h_g2[lut[pz]], 1ull);
    }
    for (uint32_t zi = xb; zi < xe; ++zi) {       // z ~ x
      const uint32_t z = adj[zi];
      if (z <= r || z == y || has2(v.hs2, r, z)) continue;
      const uint32_t pz = (1u << 0) | (1u << 1) | (xy << 2) | (1u << 5) | (uint32_t(has2(v.hs2, y, z)) << 7);
      atomicAdd(&h_g2[lut[pz]], 1ull);
    }
    const uint32_t yb = v.g2_off[y], ye = v.g2_off[y + 1];
    for (uint32_t zi = yb; zi < ye; ++zi) {       // z ~ y, z !~ x
      const uint32_t z = adj[zi];
      if (z <= r || z == x || has2(v.hs2, r, z) || has2(v.hs2, x, z)) continue;
      const uint32_t pz = (1u << 0) | (1u << 1) | (xy << 2) | (1u << 7);
      atomicAdd(&h_g2[lut[pz]], 1ull);
    }
  }
  // |A| = 1
  const uint32_t q = upper_bound(adj, xb, xe, r);
  for (uint32_t yi = q + lane; yi < xe; yi += kWave) {
    const uint32_t y = adj[yi];
    if (has2(v.hs2, r, y)) continue;
    for (uint32_t zi = yi + 1; zi < xe; ++zi) {   // z > y, z ~ x
      const uint32_t z = adj[zi];
      if (has2(v.hs2, r, z)) continue;
      const uint32_t pz = (1u << 0) | (1u << 2) | (1u << 5) | (uint32_t(has2(v.hs2, y, z)) << 7);
      atomicAdd(&h_g2[lut[pz]], 1ull);
    }
    const uint32_t yb = v.g2_off[y], ye = v.g2_off[y + 1];
    for (uint32_t zi = yb; zi < ye; ++zi) {       // z ~ y, z !~ x, z !~ r, z > r
      const uint32_t z = adj[zi];
      if (z <= r || z == x || has2(v.hs2, r, z) || has2(v.hs2, x, z)) continue;
      atomicAdd(&h_g2[lut[(1u << 0) | (1u << 2) | (1u << 7)]], 1ull);
    }
  }
}

// ---------------------------------------------------------------- (c), order 3
// Connected triples of G2 from their smallest node r, for the pair {r < y}:
// z > y both neighbours of r (triangle or wedge centred at r), or z > r a
// neighbour of y only (wedge centred at y).  Local positions r=0, y=1, z=2.
struct C3Acc {
  unsigned long long tri, wedge_r, wedge_y;
};

__device__ inline void c3_bits_word(const View& v, uint32_t r, uint32_t y, uint32_t w, C3Acc& a) {
  const uint32_t Nr = v.bits[uint64_t(r) * v.W + w], Ny = v.bits[uint64_t(y) * v.W + w];
  const uint32_t z = Nr & mask_gt(y, w);
  a.tri += __popc(z & Ny);
  a.wedge_r += __popc(z & ~Ny);
  a.wedge_y += __popc(Ny & ~Nr & mask_gt(r, w) & mask_below(v.N, w));
}

__device__ inline void c3_hash_item(const View& v, uint32_t r, uint32_t y, C3Acc& a) {
  const uint32_t re = v.g2_off[r + 1];
  for (uint32_t zi = upper_bound(v.g2_adj, v.g2_off[r], re, y); zi < re; ++zi) {
    if (has2(v.hs2, y, v.g2_adj[zi])) ++a.tri; else ++a.wedge_r;
  }
  for (uint32_t zi = v.g2_off[y]; zi < v.g2_off[y + 1]; ++zi) {
    const uint32_t z = v.g2_adj[zi];
    if (z > r && !has2(v.hs2, r, z)) ++a.wedge_y;
  }
}

// every lane of the wavefront must call this
__device__ inline void c3_flush(const C3Acc& a, const uint8_t* lut, unsigned long long* h_g2) {
  const unsigned long long s_tri = wave_sum(a.tri), s_wr = wave_sum(a.wedge_r), s_wy = wave_sum(a.wedge_y);
  if ((threadIdx.x & (kWave - 1)) == 0) {
    if (s_tri) atomicAdd(&h_g2[lut[7]], s_tri);
    if (s_wr) atomicAdd(&h_g2[lut[3]], s_wr);
    if (s_wy) atomicAdd(&h_g2[lut[5]], s_wy);
  }
}

}  // namespace hm
