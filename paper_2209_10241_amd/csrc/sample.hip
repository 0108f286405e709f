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

// j = 3 at order 4: the neighbourhood of the sampled 3-node hyperedge.  One
// wavefront per sample.
template <bool BITS>
__device__ void sample_j3_k4(const View& v, const PairLinks& pl, const Draws& d, uint32_t part, uint32_t n_parts,
                             B4Scratch* scratch, const uint8_t* lut, unsigned long long* h_lds,
                             unsigned long long* rows) {
  const int wv = threadIdx.x / kWave;
  for (uint64_t s = uint64_t(part) * kWavesPerBlock + wv; s < d.S[3]; s += uint64_t(n_parts) * kWavesPerBlock) {
    const uint64_t i = d.at(3, s);
    if (i >= d.n[3]) continue;
    const uint32_t a = v.e3[3 * i], b = v.e3[3 * i + 1], c = v.e3[3 * i + 2];
    if constexpr (BITS)
      b4_edge_bits<false>(a, b, c, v.e3, v.e4, v.i3_off, v.i3_idx, v.i4_off, v.i4_idx, v.bits, v.W, scratch[wv], lut,
                          row_or(rows, s, h_lds), nullptr);
    else
      b4_sparse<false>(v, pl, a, b, c, lut, row_or(rows, s, h_lds), nullptr);
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
// only, 3 = both; A_1, A_2, A_3 partition A = N(s) u N(o) \ e.  All work is
// done from s's side:
//   first term without T: class sizes |A_3| = t_e, |A_1| = d_s - 1 - t_e,
//     |A_2| = d_o - 1 - t_e; pairs of A joined by a pair, per class pair, from
//     the triangles at s and o, and for each neighbour x of s the
//     intersections of N(x) with N(s), N(o) and both; pairs of A not joined by
//     complement; sets with y hanging off x alone from the neighbour-degree sums;
//   pairs touching T are taken off through the rows of the nodes of T;
//   second term: the 3-node hyperedges at s one by one, those at o from its
//     8-bin pattern histogram (valid when neither other node meets s's side),
//     corrected one by one for the 3-node hyperedges {o, y, z} where y or z is
//     in N(s) u T or {s, y, z} is a 3-node hyperedge; the 4-node hyperedges
//     holding e one by one.
// One workgroup per sample.
struct J2SparseLds {
  unsigned long long acc[8];   // |A_3|, sums for A_3: codeg(s,x)-1, codeg(o,x)-1, |N(x) n A_3|, deg; for A_1: codeg(o,x)-1
  unsigned long long adj_tt[16];   // joined pairs inside T by (class, class), from both ends
  uint32_t tcls[4];
  // flat walks over up to 256 items, each with up to three row segments
  uint32_t pre[kThreads + 1];
  uint32_t wave_tot[kWavesPerBlock];
  uint32_t item[kThreads];
  uint32_t seg_base[kThreads][3];
  uint32_t seg_len[kThreads][3];
  uint32_t cnt[kThreads][7];
};

// Walk, for items [0, n) 256 at a time, the concatenated segments seg(i)
// defines (up to three, each a start and a length), as one flat range over
// the workgroup: body(slot, segment, position) for every position; then
// fin(slot, item) once per item.  Every thread must call it.
template <typename Seg, typename Body, typename Fin>
__device__ void block_flat(uint32_t n, J2SparseLds& L, Seg seg, Body body, Fin fin) {
  const uint32_t tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
  for (uint32_t c0 = 0; c0 < n; c0 += kThreads) {
    uint32_t len = 0;
    L.seg_len[tid][0] = L.seg_len[tid][1] = L.seg_len[tid][2] = 0;
    for (int q = 0; q < 7; ++q) L.cnt[tid][q] = 0;
    if (c0 + tid < n) {
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
    if (c0 + tid < n) fin(tid, c0 + tid);
    __syncthreads();
  }
}

__device__ inline uint32_t j2_pat(uint32_t cx, uint32_t cy, uint32_t xy) {
  return 1u | ((cx & 1u) << 1) | ((cx >> 1) << 2) | ((cy & 1u) << 4) | ((cy >> 1) << 5) | (xy << 7);
}

__device__ void sample_j2_k4_sparse(const View& v, const PairLinks& pl, const NodeStats& ns,
                                    const unsigned long long* __restrict__ es, const Draws& d,
                                    uint32_t part, uint32_t n_parts, J2SparseLds& L, const uint8_t* lut,
                                    unsigned long long* h_lds, unsigned long long* rows) {
  const uint32_t tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
  for (uint64_t smp = part; smp < d.S[2]; smp += n_parts) {
    const uint64_t i = d.at(2, smp);
    if (i >= d.n[2]) continue;
    unsigned long long* h = row_or(rows, smp, h_lds);
    const uint32_t e0 = v.e2[2 * i], e1 = v.e2[2 * i + 1];
    const uint32_t d0 = deg2_of(v, e0), d1 = deg2_of(v, e1);
    const uint32_t s = d0 <= d1 ? e0 : e1, o = d0 <= d1 ? e1 : e0;
    const uint32_t ds = d0 <= d1 ? d0 : d1, dO = d0 <= d1 ? d1 : d0;
    const unsigned long long key = ((unsigned long long)e0 << 32) | e1;
    const uint64_t tlo = pl.n ? pl_lower(pl, key) : 0, thi = pl.n ? pl_lower(pl, key + 1) : 0;
    const bool any_t = thi > tlo;
    auto in_t = [&](uint32_t y) { return any_t && has3(v.hs3, s, o, y); };
    auto in_x = [&](uint32_t y) { return y == s || y == o || in_t(y); };
    auto cls_of = [&](uint32_t y) { return has2(v.hs2, s, y) | (has2(v.hs2, o, y) << 1); };
    auto t_node = [&](uint64_t p) {
      const uint32_t* f = v.e3 + 3ull * pl.edge[p];
      return f[0] ^ f[1] ^ f[2] ^ s ^ o;
    };
    auto sub = [&](uint32_t pat, unsigned long long n) {
      const uint8_t c = lut[pat];
      if (c != 0xFF && n) atomicAdd(&h[c], 0ull - n);
    };
    auto add = [&](uint32_t pat, unsigned long long n) {
      const uint8_t c = lut[pat];
      if (c != 0xFF && n) atomicAdd(&h[c], n);
    };
    if (tid < 8) L.acc[tid] = 0;
    if (tid < 16) L.adj_tt[tid] = 0;
    if (tid < 4) L.tcls[tid] = 0;
    __syncthreads();
    // ---- the neighbourhood sums of e, from the per-pair statistics: with C
    // the common neighbours, |C| = t_e; over x in C: codeg(s,x)-1, codeg(o,x)-1,
    // |N(x) n C| (twice the 4-cliques through e) and deg x; over the other
    // neighbours x of s: codeg(o,x)-1 = (4-cycles through e) - sum over C of (codeg(o,x)-1)
    if (tid == 0) {
      const uint64_t n2 = d.n[2];
      const unsigned long long te = es[i], k4 = es[n2 + i], c4 = es[2 * n2 + i];
      const unsigned long long s_lo = es[3 * n2 + i], s_hi = es[4 * n2 + i], dsum = es[5 * n2 + i];
      const unsigned long long ss = s == e0 ? s_lo : s_hi, so = s == e0 ? s_hi : s_lo;
      L.acc[0] = te;
      L.acc[1] = ss - te;
      L.acc[2] = so - te;
      L.acc[3] = 2 * k4;
      L.acc[4] = dsum;
      L.acc[5] = c4 - (so - te);
    }
    // class sizes of T
    for (uint64_t p = tlo + tid; p < thi; p += kThreads) atomicAdd(&L.tcls[cls_of(t_node(p))], 1u);
    __syncthreads();
    const unsigned long long n3 = L.acc[0];
    const unsigned long long na[4] = {0, ds - 1 - n3, dO - 1 - n3, n3};
    // ---- pairs touching T.  The neighbours y of t outside e, by class,
    // follow from |N(t) n N(s)|, |N(t) n N(s) n N(o)| (the shorter of the two
    // rows walked) and |N(t) n N(o)| (likewise); those inside T from the
    // shorter of N(t) and T.  Pairs with both nodes in T are taken off once,
    // by class, at the end.
    const uint32_t n_t = uint32_t(thi - tlo);
    block_flat(
        n_t, L,
        [&](uint32_t j, uint32_t* base, uint32_t* len) {
          const uint32_t t = t_node(tlo + j);
          const uint32_t dt = deg2_of(v, t);
          base[0] = dt <= ds ? v.g2_off[t] : v.g2_off[s];
          len[0] = dt <= ds ? dt : ds;
          base[1] = dt <= dO ? v.g2_off[t] : v.g2_off[o];
          len[1] = dt <= dO ? dt : dO;
          base[2] = dt <= n_t ? v.g2_off[t] : uint32_t(tlo);
          len[2] = dt <= n_t ? dt : n_t;
        },
        [&](uint32_t slot, uint32_t sg, uint32_t pos) {
          const uint32_t t = t_node(tlo + L.item[slot]);
          const uint32_t dt = deg2_of(v, t);
          if (sg == 0) {
            const uint32_t z = v.g2_adj[pos];
            const uint32_t hit = dt <= ds ? has2(v.hs2, s, z) : has2(v.hs2, t, z);
            if (hit) {
              atomicAdd(&L.cnt[slot][0], 1u);
              if (has2(v.hs2, o, z)) atomicAdd(&L.cnt[slot][1], 1u);
            }
          } else if (sg == 1) {
            const uint32_t z = v.g2_adj[pos];
            if (dt <= dO ? has2(v.hs2, o, z) : has2(v.hs2, t, z)) atomicAdd(&L.cnt[slot][2], 1u);
          } else {
            uint32_t y;
            if (dt <= n_t) {
              y = v.g2_adj[pos];
              if (y == s || y == o || !in_t(y)) return;
            } else {
              y = t_node(pos);
              if (y == t || !has2(v.hs2, t, y)) return;
            }
            atomicAdd(&L.cnt[slot][3 + cls_of(y)], 1u);
          }
        },
        [&](uint32_t slot, uint32_t j) {
          const uint32_t t = t_node(tlo + j);
          const uint32_t ts = has2(v.hs2, s, t), to = has2(v.hs2, o, t);
          const uint32_t ct = ts | (to << 1);
          const uint32_t dt = deg2_of(v, t);
          const uint32_t a_s = L.cnt[slot][0], a_so = L.cnt[slot][1], a_o = L.cnt[slot][2];
          const uint32_t q0 = L.cnt[slot][3], q1 = L.cnt[slot][4], q2 = L.cnt[slot][5], q3 = L.cnt[slot][6];
          const uint32_t c3 = a_so, c1 = a_s - to - a_so, c2 = a_o - ts - a_so;
          const uint32_t c0 = dt - ts - to - c1 - c2 - c3;
          // neighbours outside T by class
          const unsigned long long m0 = c0 - q0, m1 = c1 - q1, m2 = c2 - q2, m3 = c3 - q3;
          if (ct) {
            sub(j2_pat(ct, 1, 1), m1);
            sub(j2_pat(ct, 2, 1), m2);
            sub(j2_pat(ct, 3, 1), m3);
            sub(j2_pat(ct, 0, 1), m0);
            // pairs {t, y}, y in A outside T, not joined
            sub(j2_pat(ct, 1, 0), na[1] - L.tcls[1] - m1);
            sub(j2_pat(ct, 2, 0), na[2] - L.tcls[2] - m2);
            sub(j2_pat(ct, 3, 0), na[3] - L.tcls[3] - m3);
          } else {
            sub(j2_pat(1, 0, 1), m1);
            sub(j2_pat(2, 0, 1), m2);
            sub(j2_pat(3, 0, 1), m3);
          }
          // joined pairs inside T, each seen from both ends
          if (q0) atomicAdd(&L.adj_tt[ct * 4 + 0], (unsigned long long)q0);
          if (q1) atomicAdd(&L.adj_tt[ct * 4 + 1], (unsigned long long)q1);
          if (q2) atomicAdd(&L.adj_tt[ct * 4 + 2], (unsigned long long)q2);
          if (q3) atomicAdd(&L.adj_tt[ct * 4 + 3], (unsigned long long)q3);
        });
    // ---- second term
    auto remove = [&](uint32_t x, uint32_t y) {
      if (in_x(x) || in_x(y)) return;
      sub(1u | (has2(v.hs2, s, x) << 1) | (has2(v.hs2, o, x) << 2) | (has2(v.hs2, s, y) << 4) |
              (has2(v.hs2, o, y) << 5) | (has2(v.hs2, x, y) << 7),
          1);
    };
    // a 3-node hyperedge {o, y, z} as the histogram at o counts it
    auto agg_pat = [&](uint32_t y, uint32_t z) {
      if (z < y) {
        const uint32_t t = y;
        y = z;
        z = t;
      }
      return 1u | (has2(v.hs2, o, y) << 2) | (has2(v.hs2, o, z) << 5) | (has2(v.hs2, y, z) << 7);
    };
    auto near_s = [&](uint32_t y) { return has2(v.hs2, s, y) || in_t(y); };
    // at s, one by one (and the hyperedges at o that match one at s on the far side)
    for (uint32_t p = v.i3_off[s] + tid; p < v.i3_off[s + 1]; p += kThreads) {
      const uint32_t* f = v.e3 + 3ull * v.i3_idx[p];
      if (f[0] == o || f[1] == o || f[2] == o) continue;
      const uint32_t y = f[0] == s ? f[1] : f[0], z = f[2] == s ? f[1] : f[2];
      remove(y, z);
      if (!near_s(y) && !near_s(z) && has3(v.hs3, o, y, z)) add(agg_pat(y, z), 1);
    }
    // at o, from its histogram
    if (tid < 8) {
      const uint32_t b = tid;
      sub(1u | ((b & 1u) << 2) | (((b >> 1) & 1u) << 5) | ((b >> 2) << 7), ns.h3[8ull * o + b]);
    }
    // corrections: the hyperedges {s, o, t}
    for (uint64_t p = tlo + tid; p < thi; p += kThreads) add(agg_pat(s, t_node(p)), 1);
    // corrections: {o, y, z} with y in N(s) u T (taken from the smaller of y, z when both are)
    {
      const uint32_t sb = v.g2_off[s];
      auto y_of = [&](uint32_t j) { return j < ds ? v.g2_adj[sb + j] : t_node(tlo + (j - ds)); };
      block_flat(
          ds + n_t, L,
          [&](uint32_t j, uint32_t* base, uint32_t* len) {
            const uint32_t y = y_of(j);
            if (y == o || (j >= ds && has2(v.hs2, s, y))) return;   // o, or a node of T taken as a neighbour of s
            const unsigned long long ky =
                y < o ? (((unsigned long long)y << 32) | o) : (((unsigned long long)o << 32) | y);
            const uint64_t lo = pl_lower(pl, ky);
            base[0] = uint32_t(lo);
            len[0] = uint32_t(pl_lower(pl, ky + 1) - lo);
          },
          [&](uint32_t slot, uint32_t, uint32_t r) {
            const uint32_t y = y_of(L.item[slot]);
            const uint32_t* f = v.e3 + 3ull * pl.edge[r];
            const uint32_t z = f[0] ^ f[1] ^ f[2] ^ o ^ y;
            if (z == s) return;                 // an {s, o, t}
            if (z < y && near_s(z)) return;     // taken from z
            add(agg_pat(y, z), 1);
            if (has3(v.hs3, s, y, z)) return;   // removed at s
            remove(y, z);
          },
          [](uint32_t, uint32_t) {});
    }
    // 4-node hyperedges holding e
    {
      const uint32_t fs = v.i4_off[s + 1] - v.i4_off[s], fo = v.i4_off[o + 1] - v.i4_off[o];
      const uint32_t a = fs <= fo ? s : o, other = fs <= fo ? o : s;
      for (uint32_t p = v.i4_off[a] + tid; p < v.i4_off[a + 1]; p += kThreads) {
        const uint32_t* f = v.e4 + 4ull * v.i4_idx[p];
        const uint32_t g0 = f[0], g1 = f[1], g2 = f[2], g3 = f[3];
        if (g0 != other && g1 != other && g2 != other && g3 != other) continue;
        uint32_t x = 0xFFFFFFFFu, y = 0xFFFFFFFFu;
        for (const uint32_t m : {g0, g1, g2, g3}) {
          if (m == s || m == o) continue;
          if (x == 0xFFFFFFFFu) x = m; else y = m;
        }
        if (has3(v.hs3, s, x, y) || has3(v.hs3, o, x, y)) continue;   // removed with a 3-node hyperedge
        remove(x, y);
      }
    }
    __syncthreads();
    // ---- first term (all of A), and the pairs inside T not joined
    if (tid == 0) {
      const unsigned long long cs = L.acc[1], co = L.acc[2], cc = L.acc[3], d3 = L.acc[4], c1o = L.acc[5];
      const unsigned long long e33 = cc / 2, e13 = cs - cc, e23 = co - cc;
      const unsigned long long e11 = (ns.tri[s] - n3) - e13 - e33;
      const unsigned long long e22 = (ns.tri[o] - n3) - e23 - e33;
      const unsigned long long e12 = c1o - e13;
      const unsigned long long dsum[4] = {0, ns.nbr[s] - dO - d3, ns.nbr[o] - ds - d3, d3};
      const unsigned long long e[4][4] = {{0, 0, 0, 0}, {0, e11, e12, e13}, {0, e12, e22, e23}, {0, e13, e23, e33}};
      for (uint32_t p = 1; p <= 3; ++p) {
        for (uint32_t q = p; q <= 3; ++q) {
          const unsigned long long tot = p == q ? na[p] * (na[p] - (na[p] > 0)) / 2 : na[p] * na[q];
          add(j2_pat(p, q, 1), e[p][q]);
          add(j2_pat(p, q, 0), tot - e[p][q]);
          // pairs inside T in these classes: joined (seen twice) and not joined
          const unsigned long long tp = L.tcls[p], tq = L.tcls[q];
          const unsigned long long ttot = p == q ? tp * (tp - (tp > 0)) / 2 : tp * tq;
          const unsigned long long tadj = p == q ? L.adj_tt[p * 4 + p] / 2 : L.adj_tt[p * 4 + q];
          sub(j2_pat(p, q, 1), tadj);
          sub(j2_pat(p, q, 0), ttot - tadj);
        }
        // joined pairs inside T with one node outside A: it hangs off the other
        sub(j2_pat(p, 0, 1), L.adj_tt[p * 4 + 0]);
        const unsigned long long inside = 2 * e[p][p] + e[p][1] + e[p][2] + e[p][3] - e[p][p];
        add(j2_pat(p, 0, 1), dsum[p] - na[p] * (p == 3 ? 2 : 1) - inside);
      }
    }
    __syncthreads();
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

__device__ inline uint32_t wave_sum32(uint32_t x) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, kWave);
  return x;
}

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
    if (tid < W) {
      L.RU[tid] = bits[uint64_t(u) * W + tid];
      L.RW[tid] = bits[uint64_t(w) * W + tid];
      L.XS[tid] = 0;
    }
    if (tid < 21) L.red[tid] = 0;
    __syncthreads();
    if (tid == 0) {
      atomicOr(&L.XS[u >> 5], 1u << (u & 31));
      atomicOr(&L.XS[w >> 5], 1u << (w & 31));
    }
    const uint32_t u0 = v.i3_off[u], u1 = v.i3_off[u + 1];
    for (uint32_t p = u0 + tid; p < u1; p += kThreads) {
      const uint32_t* t = v.e3 + 3ull * v.i3_idx[p];
      if (t[0] == w || t[1] == w || t[2] == w) {
        const uint32_t c = t[0] ^ t[1] ^ t[2] ^ u ^ w;
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
    for (uint32_t t = tid; t < n_tasks; t += kThreads) {
      const uint32_t xi = t / W, wd = t - xi * W;
      const uint32_t x = L.xs[xi];
      const uint32_t xc = node_bit(L.RU, x) | (node_bit(L.RW, x) << 1);
      const uint32_t rx = bits[uint64_t(x) * W + wd];
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
    // second term: each pair {x, y} outside X whose set holds a larger hyperedge
    auto remove = [&](uint32_t x, uint32_t y) {
      if (node_bit(L.XS, x) | node_bit(L.XS, y)) return;
      const uint32_t pat = 1u | (node_bit(L.RU, x) << 1) | (node_bit(L.RW, x) << 2) | (node_bit(L.RU, y) << 4) |
                           (node_bit(L.RW, y) << 5) | (bit_of(bits, W, x, y) << 7);
      const uint8_t cls = lut[pat];
      if (cls != 0xFF) atomicAdd(&h[cls], ~0ull);   // minus one
    };
    for (uint32_t p = u0 + tid; p < u1; p += kThreads) {
      const uint32_t* t = v.e3 + 3ull * v.i3_idx[p];
      if (t[0] == w || t[1] == w || t[2] == w) continue;
      remove(t[0] == u ? t[1] : t[0], t[2] == u ? t[1] : t[2]);
    }
    const uint32_t w0 = v.i3_off[w], w1 = v.i3_off[w + 1];
    for (uint32_t p = w0 + tid; p < w1; p += kThreads) {
      const uint32_t* t = v.e3 + 3ull * v.i3_idx[p];
      if (t[0] == u || t[1] == u || t[2] == u) continue;
      const uint32_t x = t[0] == w ? t[1] : t[0], y = t[2] == w ? t[1] : t[2];
      if (has3(v.hs3, u, x, y)) continue;   // taken at u
      remove(x, y);
    }
    const uint32_t f0 = v.i4_off[u], f1 = v.i4_off[u + 1];
    for (uint32_t p = f0 + tid; p < f1; p += kThreads) {
      const uint32_t* f = v.e4 + 4ull * v.i4_idx[p];
      const uint32_t f_0 = f[0], f_1 = f[1], f_2 = f[2], f_3 = f[3];
      if (f_0 != w && f_1 != w && f_2 != w && f_3 != w) continue;
      // the two members other than u and w, ascending
      uint32_t x = 0xFFFFFFFFu, y = 0xFFFFFFFFu;
      for (const uint32_t m : {f_0, f_1, f_2, f_3}) {
        if (m == u || m == w) continue;
        if (x == 0xFFFFFFFFu) x = m; else y = m;
      }
      if (has3(v.hs3, u, x, y) || has3(v.hs3, w, x, y)) continue;   // taken at u or w
      remove(x, y);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int j = 0; j < 7; ++j) {
        const uint32_t sum = wave_sum32(acc[c][j]);
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
  Draws d;
  const uint8_t* lut;
  uint32_t blocks[5];            // workgroups of strata 2, 3, 4 (in this order in the grid)
  unsigned long long* rows[5];   // per-sample rows (256 counters) of each stratum, or null
  unsigned long long* hist;      // 256 raw counters, zero on entry; left zero after scaling
  unsigned int* ticket;          // workgroups done; zero on entry and left zero
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
    B4Scratch b4[kWavesPerBlock];
    J2Lds j2;
  };
};
template <>
struct SampledLds<4, false> {
  J2SparseLds j2;
};

// Every stratum's samples in one launch.  The grid holds a.blocks[2]
// workgroups for the sampled pairs, then a.blocks[3] for the 3-node and
// a.blocks[4] for the 4-node hyperedges.  Each workgroup adds its LDS counts to
// a.hist; the last one to finish scales them (Algorithm 4's correction:
// est_m = raw_m * |E_mc| / (S_mc * countmax_m) in fp64, rounded once to fp32,
// 0 when the stratum was not sampled) and clears a.hist and a.ticket.
template <int K, bool BITS>
__global__ void __launch_bounds__(kThreads) k_sampled(SampledArgs a, ScaleArgs sc) {
  constexpr int kLut = K == 4 ? 2048 : 16;
  __shared__ uint8_t lut[kLut];
  __shared__ unsigned long long h_lds[256];
  __shared__ SampledLds<K, BITS> lds;
  __shared__ uint32_t last;
  load_lut(lut, a.lut, kLut);
  h_lds[threadIdx.x] = 0;
  __syncthreads();
  uint32_t b = blockIdx.x;
  if (b < a.blocks[2]) {
    if constexpr (K == 4 && BITS)
      sample_j2_k4_bits(a.v, a.d, b, a.blocks[2], lds.j2, lut, h_lds, a.rows[2]);
    else if constexpr (K == 4)
      sample_j2_k4_sparse(a.v, a.pl, a.ns, a.es, a.d, b, a.blocks[2], lds.j2, lut, h_lds, a.rows[2]);
    else
      sample_j2_k3(a.v, a.d, b, a.blocks[2], lut, h_lds, a.rows[2]);
  } else if ((b -= a.blocks[2]) < a.blocks[3]) {
    if constexpr (K == 4 && BITS)
      sample_j3_k4<true>(a.v, a.pl, a.d, b, a.blocks[3], lds.b4, lut, h_lds, a.rows[3]);
    else if constexpr (K == 4)
      sample_j3_k4<false>(a.v, a.pl, a.d, b, a.blocks[3], nullptr, lut, h_lds, a.rows[3]);
    else
      sample_j3_k3(a.v, a.d, b, a.blocks[3], lut, h_lds, a.rows[3]);
  } else if (K == 4) {
    b -= a.blocks[3];
    sample_j4(a.v, a.d, b, a.blocks[4], lut, h_lds, a.rows[4]);
  }
  __syncthreads();
  flush(h_lds, a.hist, 256);
  if (!a.est) return;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) last = atomicAdd(a.ticket, 1u) == gridDim.x - 1;
  __syncthreads();
  if (!last) return;
  __threadfence();
  const int c = threadIdx.x;
  const unsigned long long r = __hip_atomic_load(a.hist + c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (c < a.n_classes) {
    const int j = sc.maxcard[c];
    double e = 0.0;
    if (sc.s_by_size[j] > 0.0) e = (double(r) * sc.n_by_size[j]) / (sc.s_by_size[j] * double(sc.countmax[c]));
    a.est[c] = float(e);
    if (a.raw) a.raw[c] = int64_t(r);
  }
  a.hist[c] = 0;
  if (c == 0) *a.ticket = 0;
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
  }
  SampledArgs a;
  a.v = view_of(H);
  a.pl.keys = H->pl_keys;
  a.pl.edge = H->pl_edge;
  a.pl.n = H->pl_keys ? 3 * H->n_by_size[3] : 0;
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
  if (grid == 0) {   // nothing sampled: one workgroup still scales (to zeros)
    a.blocks[2] = 1;
    grid = 1;
  }
  a.hist = H->sample_hist;
  a.ticket = reinterpret_cast<unsigned int*>(H->sample_hist + 256);
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
  ProfileScope pscope("k_sampled", st);
  if (k == 4 && bits)
    k_sampled<4, true><<<grid, kThreads, 0, st>>>(a, sc);
  else if (k == 4)
    k_sampled<4, false><<<grid, kThreads, 0, st>>>(a, sc);
  else
    k_sampled<3, false><<<grid, kThreads, 0, st>>>(a, sc);
  HM_HIP(hipGetLastError());
  return HM_OK;
}

}  // namespace

int sample_sizes(const hm_graph* H, int k, double fraction, int allocation, uint64_t* S) {
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
    // S = ceil(f * |E_2 u E_3 u E_4|) split S_2 : S_3 : S_4 = 1 : 3 : 2
    const double tot = double(H->n_by_size[2] + H->n_by_size[3] + H->n_by_size[4]);
    const uint64_t s = uint64_t(std::ceil(fraction * tot));
    S[2] = s / 6;
    S[3] = s / 2;
    S[4] = s - S[2] - S[3];
    for (int j = 2; j <= 4; ++j)
      if (H->n_by_size[j] == 0) S[j] = 0;
  } else {
    for (int j = 2; j <= k; ++j) S[j] = uint64_t(std::ceil(fraction * double(H->n_by_size[j])));
  }
  return HM_OK;
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

// Enumerate around explicit samples and scale (Algorithm 4).
int sampled_from_indices(const hm_graph* H, int k, const uint32_t* const idx[5], const uint64_t S[5], float* est,
                         int64_t* raw, hipStream_t st) {
  const uint64_t row0[5] = {0, 0, 0, 0, 0};
  return launch_sampled(H, k, idx, S, 0, nullptr, row0, est, raw, st);
}

}  // namespace hm

extern "C" {

int hm_sample_sizes(const hm_graph* H, int k, double fraction, int allocation, uint64_t* s_out) {
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
}

int hm_sample_draw(const hm_graph* H, int k, double fraction, uint64_t seed, int allocation, uint32_t* idx2,
                   uint32_t* idx3, uint32_t* idx4, void* stream) {
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
}

int count_sampled(const hm_graph* H, int k, double fraction, uint64_t seed, int allocation, float* est,
                  int64_t* raw, void* stream) {
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
}

int count_sampled_indices(const hm_graph* H, int k, const uint32_t* idx2, uint64_t s2, const uint32_t* idx3,
                          uint64_t s3, const uint32_t* idx4, uint64_t s4, float* est, int64_t* raw, void* stream) {
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
}

}  // extern "C"
