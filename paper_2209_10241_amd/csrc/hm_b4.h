// The neighbourhood of one 3-node hyperedge e = {a<b<c} at order 4: every
// node v that a hyperedge of size 2 or 3 joins to e gives the candidate set
// e u {v} (Algorithm 3's exploration of "the hyperedges adjacent to e" with
// |e u e_i| = 4, and Algorithm 4's exploration around a sampled 3-node
// hyperedge).  A wavefront handles one e; v is taken once.  Sets that are
// 4-node hyperedges are skipped (their largest hyperedge has 4 nodes).
//
// OWN = true (exact counting): e counts e u {v} only if no other 3-node
// hyperedge inside it precedes e in lexicographic order, so each set is
// counted by exactly one 3-node hyperedge.  The G2 shape of counted sets
// whose pairs connect them goes to h_sub.
// OWN = false (sampling): every sampled e counts every such set.
#pragma once

#include "hm_device.h"

namespace hm {

constexpr uint32_t kMaxWordsB = kBitsetMaxNodes / 32;
constexpr int kB4Batch = 4;   // incidence entries a lane loads at once
// LDS words one wavefront needs for rows of W words: T_ab, T_ac, T_bc, Q and
// a list of kWave candidate nodes
__host__ __device__ constexpr uint32_t b4_set_words(uint32_t W) { return 4 * W + kWave; }

__device__ inline void count_class(const uint8_t* lut, unsigned long long* h_main, unsigned long long* h_sub,
                                   uint32_t pattern, uint32_t pair_bits) {
  atomicAdd(&h_main[lut[pattern]], 1ull);
  if (h_sub) {
    const uint8_t g = lut[pattern & pair_bits];
    if (g != 0xFF) atomicAdd(&h_sub[g], 1ull);
  }
}

// Hash-set version.  Generator instances: every pairwise neighbour v of a, b
// or c (witness 0, 1, 2), and every 3-node hyperedge f sharing exactly two
// nodes with e, reached from the row of the smaller shared node (witness 3
// for {a,b}, 4 for {a,c}, 5 for {b,c}).  An instance counts only when no
// witness ahead of its own exists, so each v is taken once.
template <bool OWN>
__device__ void b4_edge_hash(uint32_t a, uint32_t b, uint32_t c, const uint32_t* __restrict__ e3,
                             const uint32_t* __restrict__ g2_off, const uint32_t* __restrict__ g2_adj,
                             const uint32_t* __restrict__ i3_off, const uint32_t* __restrict__ i3_idx,
                             const Set64& hs2, const Set128& hs3, const Set128& hs4, const uint8_t* lut,
                             unsigned long long* h_main, unsigned long long* h_sub) {
  const int lane = threadIdx.x & (kWave - 1);
  const uint32_t pab = has2(hs2, a, b), pac = has2(hs2, a, c), pbc = has2(hs2, b, c);
  const uint32_t base_p = pab | (pac << 1) | (pbc << 2) | (1u << 3);
  uint32_t sb[5], sl[5];
  sb[0] = g2_off[a]; sl[0] = g2_off[a + 1] - sb[0];
  sb[1] = g2_off[b]; sl[1] = g2_off[b + 1] - sb[1];
  sb[2] = g2_off[c]; sl[2] = g2_off[c + 1] - sb[2];
  sb[3] = i3_off[a]; sl[3] = i3_off[a + 1] - sb[3];
  sb[4] = i3_off[b]; sl[4] = i3_off[b + 1] - sb[4];
  const uint32_t total = sl[0] + sl[1] + sl[2] + sl[3] + sl[4];
  for (uint32_t t = lane; t < total; t += kWave) {
    uint32_t seg = 0, off = t;
    while (off >= sl[seg]) { off -= sl[seg]; ++seg; }
    uint32_t v, src;
    if (seg < 3) {
      v = g2_adj[sb[seg] + off];
      if (v == a || v == b || v == c) continue;
      src = seg;
    } else {
      const uint32_t f = i3_idx[sb[seg] + off];
      const uint32_t x = e3[3ull * f], y = e3[3ull * f + 1], z = e3[3ull * f + 2];
      const bool xa = (x == a || x == b || x == c), ya = (y == a || y == b || y == c), za = (z == a || z == b || z == c);
      if (int(xa) + int(ya) + int(za) != 2) continue;
      v = !xa ? x : (!ya ? y : z);
      const bool hasa = (x == a || y == a || z == a), hasb = (x == b || y == b || z == b);
      if (seg == 3) {
        src = hasb ? 3 : 4;          // {a,b,v} or {a,c,v}
      } else {
        if (hasa) continue;          // {a,b,v} is taken from a's row
        src = 5;                     // {b,c,v}
      }
    }
    // fill-in, cheapest witnesses first
    const uint32_t qa = has2(hs2, a, v);
    if (src > 0 && qa) continue;
    const uint32_t qb = has2(hs2, b, v);
    if (src > 1 && qb) continue;
    const uint32_t qc = has2(hs2, c, v);
    if (src > 2 && qc) continue;
    uint32_t x0 = a, x1 = b, x2 = v;
    sort3(x0, x1, x2);
    const uint32_t tab = set128_has(hs3, key3(x0, x1, x2));
    if (src > 3 && tab) continue;
    if (OWN && tab && v < c) continue;                       // {a,b,v} precedes e
    uint32_t y0 = a, y1 = c, y2 = v;
    sort3(y0, y1, y2);
    const uint32_t tac = set128_has(hs3, key3(y0, y1, y2));
    if (src > 4 && tac) continue;
    if (OWN && tac && v < b) continue;                       // {a,c,v} precedes e
    uint32_t z0 = b, z1 = c, z2 = v;
    sort3(z0, z1, z2);
    const uint32_t tbc = set128_has(hs3, key3(z0, z1, z2));
    if (OWN && tbc && v < a) continue;                       // {b,c,v} precedes e
    uint32_t w0 = a, w1 = b, w2 = c, w3 = v;
    if (w3 < w2) { w3 = w2; w2 = v; if (w2 < w1) { w2 = w1; w1 = v; if (w1 < w0) { w1 = w0; w0 = v; } } }
    if (set128_has(hs4, key4(w0, w1, w2, w3))) continue;   // a 4-node hyperedge
    // local positions a=0, b=1, c=2, v=3
    const uint32_t p = base_p | (qa << 4) | (qb << 5) | (tab << 6) | (qc << 7) | (tac << 8) | (tbc << 9);
    count_class(lut, h_main, h_sub, p, kPairBits4);
  }
}

// Bit-row version, counting instead of listing.  The wavefront builds, in
// LDS (sets: b4_set_words(W) words), bit sets of the nodes v with {a,b,v}, {a,c,v} or
// {b,c,v} a 3-node hyperedge (T_ab, T_ac, T_bc, from the incident 3-node
// hyperedges of the two members with the fewest) and with e u {v} a 4-node
// hyperedge (Q, from those of the member with the fewest).  The incidence
// entries carry the other members of their hyperedge (others3, others4), so
// each is one load.  Any other v leaves e the only hyperedge of size >= 3 in
// e u {v}, so those v are counted per pairwise combination (av, bv, cv) with
// popcounts over the rows of a, b, c.  The nodes that lie in a T set and
// outside Q are listed in LDS and classified one per lane.
template <bool OWN>
__device__ void b4_edge_bits_count(uint32_t a, uint32_t b, uint32_t c, const uint32_t* __restrict__ i3_off,
                                   const uint32_t* __restrict__ i3_oth, const uint32_t* __restrict__ i4_off,
                                   const unsigned long long* __restrict__ i4_oth, const uint32_t* __restrict__ bits,
                                   uint32_t W, uint32_t* sets, const uint8_t* lut, unsigned long long* h_main,
                                   unsigned long long* h_sub) {
  const int lane = threadIdx.x & (kWave - 1);
  uint32_t* Tab = sets;
  uint32_t* Tac = sets + W;
  uint32_t* Tbc = sets + 2 * W;
  uint32_t* Q = sets + 3 * W;
  const uint32_t* Ra = bits + uint64_t(a) * W;
  const uint32_t* Rb = bits + uint64_t(b) * W;
  const uint32_t* Rc = bits + uint64_t(c) * W;
  for (uint32_t w = lane; w < 4 * W; w += kWave) sets[w] = 0;
  // 3-node hyperedges sharing two nodes with e: each holds one of any two
  // members of e, so the lists of the two members with the fewest are read
  // (one found twice sets its bit twice)
  const uint32_t la0 = i3_off[a], la = i3_off[a + 1] - la0;
  const uint32_t lb0 = i3_off[b], lb = i3_off[b + 1] - lb0;
  const uint32_t lc0 = i3_off[c], lc = i3_off[c + 1] - lc0;
  const bool skip_a = la >= lb && la >= lc, skip_b = !skip_a && lb >= lc;
  const uint32_t o1 = skip_a ? b : a, pa = skip_a ? lb0 : la0, l1 = skip_a ? lb : la;
  const uint32_t o2 = (skip_a || skip_b) ? c : b, pb = (skip_a || skip_b) ? lc0 : lb0,
                 l2 = (skip_a || skip_b) ? lc : lb;
  // 4-node hyperedges containing e, from the shortest list of a member
  const uint32_t fa = i4_off[a + 1] - i4_off[a], fb = i4_off[b + 1] - i4_off[b], fc = i4_off[c + 1] - i4_off[c];
  const uint32_t m4 = (fa <= fb && fa <= fc) ? a : (fb <= fc ? b : c);
  const uint32_t p4 = i4_off[m4], l4 = i4_off[m4 + 1] - p4;
  wave_sync();
  // the entries of both walks are loaded kB4Batch per lane at a time before
  // any is used, so that their latencies overlap
  // (batch q: 3-node entries [q * kB4Batch * kWave, (q + 1) * kB4Batch * kWave),
  // 4-node entries [q * kWave, (q + 1) * kWave))
  const uint32_t l3 = l1 + l2;
  for (uint32_t q = 0; q * (kB4Batch * kWave) < l3 || q * kWave < l4; ++q) {
    const uint32_t t0 = q * (kB4Batch * kWave);
    uint32_t o3[kB4Batch];
#pragma unroll
    for (int u = 0; u < kB4Batch; ++u) {
      const uint32_t t = t0 + u * kWave + lane;
      o3[u] = t < l3 ? i3_oth[t < l1 ? pa + t : pb + (t - l1)] : 0u;
    }
    const uint32_t t4 = q * kWave + lane;
    const unsigned long long o4 = t4 < l4 ? i4_oth[p4 + t4] : 0ull;
#pragma unroll
    for (int u = 0; u < kB4Batch; ++u) {
      const uint32_t t = t0 + u * kWave + lane;
      if (t >= l3) continue;
      const uint32_t p = t < l1 ? o1 : o2;   // the list's node; the hyperedge is {p, y, z}
      const uint32_t y = o3[u] & 0xFFFFu, z = o3[u] >> 16;
      const bool hy = (y == a || y == b || y == c), hz = (z == a || z == b || z == c);
      if (hy == hz) continue;                // e itself, or only p shared
      const uint32_t v = hy ? z : y, w = hy ? y : z;   // shared pair {p, w}
      const bool ha = p == a || w == a, hb = p == b || w == b;
      uint32_t* T = (ha && hb) ? Tab : (ha ? Tac : Tbc);
      atomicOr(&T[v >> 5], 1u << (v & 31));
    }
    if (t4 < l4) {   // the hyperedge is {m4, x, y, z}
      const uint32_t x = uint32_t(o4) & 0xFFFFu, y = uint32_t(o4 >> 16) & 0xFFFFu, z = uint32_t(o4 >> 32) & 0xFFFFu;
      const bool ix = x == a || x == b || x == c, iy = y == a || y == b || y == c, iz = z == a || z == b || z == c;
      if (int(ix) + int(iy) + int(iz) == 2) {
        const uint32_t v = !ix ? x : (!iy ? y : z);
        atomicOr(&Q[v >> 5], 1u << (v & 31));
      }
    }
  }
  wave_sync();
  const uint32_t pab = (Ra[b >> 5] >> (b & 31)) & 1u, pac = (Ra[c >> 5] >> (c & 31)) & 1u,
                 pbc = (Rb[c >> 5] >> (c & 31)) & 1u;
  const uint32_t base_p = pab | (pac << 1) | (pbc << 2) | (1u << 3);
  uint32_t n1 = 0, n2 = 0, n3 = 0, n4 = 0, n5 = 0, n6 = 0, n7 = 0;
  uint32_t* list = sets + 4 * W;   // kWave candidate nodes
  for (uint32_t w0 = 0; w0 < W; w0 += kWave) {
    const uint32_t w = w0 + lane;
    uint32_t cw = 0;
    if (w < W) {
      const uint32_t ra = Ra[w], rb = Rb[w], rc = Rc[w];
      const uint32_t tab_w = Tab[w], tac_w = Tac[w], tbc_w = Tbc[w], q_w = Q[w];
      uint32_t self = 0;
      if ((a >> 5) == w) self |= 1u << (a & 31);
      if ((b >> 5) == w) self |= 1u << (b & 31);
      if ((c >> 5) == w) self |= 1u << (c & 31);
      // the ordinary fourth nodes, per combination
      const uint32_t m = (ra | rb | rc) & ~(tab_w | tac_w | tbc_w | q_w | self);
      n1 += __popc(m & ra & ~rb & ~rc);
      n2 += __popc(m & ~ra & rb & ~rc);
      n3 += __popc(m & ra & rb & ~rc);
      n4 += __popc(m & ~ra & ~rb & rc);
      n5 += __popc(m & ra & ~rb & rc);
      n6 += __popc(m & ~ra & rb & rc);
      n7 += __popc(m & ra & rb & rc);
      // the fourth nodes on another 3-node hyperedge (not on a 4-node one)
      cw = (tab_w | tac_w | tbc_w) & ~(q_w | self);
    }
    // which are listed in order, kWave at a time, and classified one per lane
    uint32_t tot;
    uint32_t at = wave_exclusive_scan(__popc(cw), &tot);
    for (uint32_t base = 0; base < tot; base += kWave) {
      while (cw && at < base + kWave) {
        list[at - base] = (w << 5) | uint32_t(__ffs(cw) - 1);
        cw &= cw - 1;
        ++at;
      }
      wave_sync();
      if (base + lane < tot) {
        const uint32_t v = list[lane], vw = v >> 5, vb = v & 31u;
        const uint32_t tab = (Tab[vw] >> vb) & 1u, tac = (Tac[vw] >> vb) & 1u, tbc = (Tbc[vw] >> vb) & 1u;
        // (an earlier 3-node hyperedge inside e u {v} owns it)
        if (!(OWN && ((tab && v < c) || (tac && v < b) || (tbc && v < a)))) {
          const uint32_t qa = (Ra[vw] >> vb) & 1u, qb = (Rb[vw] >> vb) & 1u, qc = (Rc[vw] >> vb) & 1u;
          // local positions a=0, b=1, c=2, v=3
          const uint32_t pt = base_p | (qa << 4) | (qb << 5) | (tab << 6) | (qc << 7) | (tac << 8) | (tbc << 9);
          count_class(lut, h_main, h_sub, pt, kPairBits4);
        }
      }
      wave_sync();
    }
  }
  // Reduce over the wavefront (lanes without words hold zeros); a
  // combination's total over the wavefront is below the node count, at most
  // 8192, so two of them share a 32-bit word.
  uint32_t pk[4] = {n1 | (n2 << 16), n3 | (n4 << 16), n5 | (n6 << 16), n7};
#pragma unroll
  for (int k = 0; k < 4; ++k) pk[k] = wave_sum_u32(pk[k]);
  uint32_t n[8];
  n[1] = pk[0] & 0xFFFFu; n[2] = pk[0] >> 16; n[3] = pk[1] & 0xFFFFu; n[4] = pk[1] >> 16;
  n[5] = pk[2] & 0xFFFFu; n[6] = pk[2] >> 16; n[7] = pk[3];
  if (lane == 0) {
#pragma unroll
    for (uint32_t cmb = 1; cmb < 8; ++cmb) {
      if (!n[cmb]) continue;
      const uint32_t pt = base_p | ((cmb & 1u) << 4) | (((cmb >> 1) & 1u) << 5) | ((cmb >> 2) << 7);
      atomicAdd(&h_main[lut[pt]], (unsigned long long)n[cmb]);
      if (h_sub) {
        const uint8_t g = lut[pt & kPairBits4];
        if (g != 0xFF) atomicAdd(&h_sub[g], (unsigned long long)n[cmb]);
      }
    }
  }
  wave_sync();   // the sets are rewritten by the wavefront's next 3-node hyperedge
}

}  // namespace hm
