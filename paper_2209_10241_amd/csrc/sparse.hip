// Exact order-3 and order-4 counts on hypergraphs without adjacency bit rows
// (Algorithms 2 and 3, Section 4.2), sized for graphs with millions of
// hyperedges and heavy-tailed degrees.
//
// The generators and ownership rules are those of the bit-row path:
//   (a) every k-node hyperedge, classified by fill-in;
//   (b) order 4: every 3-node hyperedge with each fourth node, counted per
//       pairwise combination by inclusion-exclusion (hm_sparse.h);
//   (c) sets connected through pairs only: never enumerated.  The number of
//       connected k-node sets of the pairwise graph G2 per induced shape
//       follows from non-induced subgraph counts: 3-stars sum C(d,3),
//       3-paths sum over edges (d_u-1)(d_v-1) - 3T, paws sum t_v (d_v-2),
//       diamonds sum over edges C(t_e,2), 4-cycles and 4-cliques by
//       degree-ordered enumeration, inverted through the matrix of how often
//       each shape contains another; then the sets that (a) or (b) own are
//       subtracted by shape.
// Degree order: x precedes y when (deg x, x) < (deg y, y); a node's
// neighbours that follow it number at most sqrt(2 |E2|).
#include <algorithm>
#include <map>
#include <mutex>
#include <vector>

#include "hm_sparse.h"

namespace hm {
namespace {

enum : int { kAccT3 = 0, kAccDiamond, kAccP4, kAccStar, kAccPaw, kAccC4, kAccK4, kAccWedge, kAccN };

__device__ inline bool rank_less(const View& v, uint32_t x, uint32_t y) {
  const uint32_t dx = deg2_of(v, x), dy = deg2_of(v, y);
  return dx < dy || (dx == dy && x < y);
}

// sum of x over the workgroup, added to *out by one thread
__device__ inline void block_add(unsigned long long x, unsigned long long* out) {
  __shared__ unsigned long long part[kWavesPerBlock];
  x = wave_sum(x);
  const int wv = threadIdx.x / kWave;
  if ((threadIdx.x & (kWave - 1)) == 0) part[wv] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long s = 0;
    for (int i = 0; i < kWavesPerBlock; ++i) s += part[i];
    if (s) atomicAdd(out, s);
  }
  __syncthreads();
}

// Triangles on each pair {a, b} of G2: t_e = |N(a) n N(b)| over the smaller
// row.  tv[x] collects sum of t_e over the pairs at x (= 2 t_x).
__global__ void __launch_bounds__(kThreads) k_sp_edge_tri(View v, uint64_t n2, uint32_t* __restrict__ tri_e,
                                                          unsigned long long* __restrict__ tv,
                                                          unsigned long long* __restrict__ acc) {
  const int lane = threadIdx.x & (kWave - 1);
  const uint64_t wave = uint64_t(blockIdx.x) * kWavesPerBlock + threadIdx.x / kWave;
  const uint64_t n_waves = uint64_t(gridDim.x) * kWavesPerBlock;
  unsigned long long st = 0, sd = 0, sp = 0;
  for (uint64_t e = wave; e < n2; e += n_waves) {
    const uint32_t a = v.e2[2 * e], b = v.e2[2 * e + 1];
    const uint32_t da = deg2_of(v, a), db = deg2_of(v, b);
    const uint32_t s = da <= db ? a : b, o = da <= db ? b : a;
    const uint32_t t = row_count(v, s, o);
    if (lane == 0) {
      tri_e[e] = t;
      if (t) {
        atomicAdd(&tv[a], (unsigned long long)t);
        atomicAdd(&tv[b], (unsigned long long)t);
      }
      st += t;
      sd += (unsigned long long)t * (t - 1) / 2;
      sp += (unsigned long long)(da - 1) * (db - 1);
    }
  }
  block_add(st, acc + kAccT3);
  block_add(sd, acc + kAccDiamond);
  block_add(sp, acc + kAccP4);
}

// Per node: C(d,3) (3-stars), C(d,2) (wedges), t_x (d - 2) (paws).
__global__ void __launch_bounds__(kThreads) k_sp_nodes(View v, const unsigned long long* __restrict__ tv,
                                                       unsigned long long* __restrict__ acc) {
  unsigned long long s3 = 0, s2 = 0, sp = 0;
  for (uint32_t x = blockIdx.x * kThreads + threadIdx.x; x < v.N; x += gridDim.x * kThreads) {
    const unsigned long long d = deg2_of(v, x);
    if (d >= 2) {
      s2 += d * (d - 1) / 2;
      sp += (tv[x] / 2) * (d - 2);
    }
    if (d >= 3) s3 += d * (d - 1) / 2 * (d - 2) / 3;
  }
  block_add(s3, acc + kAccStar);
  block_add(s2, acc + kAccWedge);
  block_add(sp, acc + kAccPaw);
}


// 4-cycles without atomics per wedge: every wedge (u, x, w) with x and w
// before the top node u in degree order becomes the key (u << B) | w; sorted,
// each run of equal keys holds the middle nodes of one (u, w) and adds
// C(run, 2) cycles.  Each pair {x, u} of G2 (x the earlier) walks the row of x,
// so the walked positions are laid out flat, pair after pair, and cut into
// tiles of kC4Tile positions that span at most kC4Tile + 1 pairs (every row
// walked is non-empty).  Positions that are not wedges get the key kC4None.
constexpr unsigned long long kC4None = ~0ull;
constexpr uint32_t kC4Tile = 2048;

// Walked positions of each pair (the degree of its earlier node) and their sum.
__global__ void k_c4_len(View v, uint64_t n2, uint32_t* __restrict__ len, unsigned long long* __restrict__ total) {
  unsigned long long s = 0;
  for (uint64_t e = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n2; e += uint64_t(gridDim.x) * blockDim.x) {
    const uint32_t a = v.e2[2 * e], b = v.e2[2 * e + 1];
    const uint32_t d = deg2_of(v, rank_less(v, a, b) ? a : b);
    len[e] = d;
    s += d;
  }
  block_add(s, total);
}

// The pair that holds the first position of each tile (pos = exclusive scan of len).
__global__ void k_c4_tile_starts(const uint32_t* __restrict__ pos, const uint32_t* __restrict__ len, uint64_t n2,
                                 uint32_t* __restrict__ start) {
  for (uint64_t e = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n2; e += uint64_t(gridDim.x) * blockDim.x) {
    const uint64_t lo = pos[e], hi = lo + len[e];
    for (uint64_t t = (lo + kC4Tile - 1) / kC4Tile; t * kC4Tile < hi; ++t) start[t] = uint32_t(e);
  }
}

// One workgroup per tile: the tile's pairs are staged in LDS (start offset,
// top node, row of the earlier node) and each position finds its pair there.
__global__ void __launch_bounds__(kThreads) k_c4_keys(View v, int B, const uint32_t* __restrict__ pos,
                                                      const uint32_t* __restrict__ start, uint64_t n2,
                                                      uint32_t n_pos, uint32_t n_tiles,
                                                      unsigned long long* __restrict__ keys,
                                                      uint32_t* __restrict__ vals) {
  __shared__ uint32_t s_pos[kC4Tile + 2], s_top[kC4Tile + 2], s_row[kC4Tile + 2];
  const uint32_t tid = threadIdx.x, t = blockIdx.x;
  const uint32_t p0 = t * kC4Tile;
  const uint32_t p1 = n_pos - p0 < kC4Tile ? n_pos : p0 + kC4Tile;
  const uint32_t c0 = start[t];
  const uint32_t c1 = t + 1 < n_tiles ? start[t + 1] : uint32_t(n2 - 1);
  const uint32_t cnt = c1 - c0 + 1;   // at most kC4Tile + 1
  for (uint32_t i = tid; i < cnt; i += kThreads) {
    const uint32_t e = c0 + i, a = v.e2[2 * uint64_t(e)], b = v.e2[2 * uint64_t(e) + 1];
    const bool ab = rank_less(v, a, b);
    s_pos[i] = pos[e];
    s_top[i] = ab ? b : a;
    s_row[i] = v.g2_off[ab ? a : b];
  }
  __syncthreads();
  for (uint32_t p = p0 + tid; p < p1; p += kThreads) {
    uint32_t lo = 0, hi = cnt;   // s_pos[lo] <= p < s_pos[hi]
    while (hi - lo > 1) {
      const uint32_t m = (lo + hi) >> 1;
      if (s_pos[m] <= p) lo = m; else hi = m;
    }
    const uint32_t u = s_top[lo], w = v.g2_adj[s_row[lo] + (p - s_pos[lo])];
    keys[p] = (w == u || !rank_less(v, w, u)) ? kC4None : ((unsigned long long)u << B) | (unsigned long long)w;
    vals[p] = p;
  }
}

// Per-pair 4-cycle counts from the sorted wedge keys (vals: the walked
// position of each key): a wedge (u, x, w) in a run of r >= 2 equal keys
// closes r - 1 cycles, one with each other middle node of the run, and each
// holds its pairs {u, x} (the pair whose walk the position belongs to) and
// {x, w} (x's row entry).  One thread per key: it finds its run's ends by
// galloping search (runs of hub pairs are long, most runs hold one key).
__device__ inline uint64_t run_end(const unsigned long long* keys, uint64_t n, uint64_t i, unsigned long long key) {
  uint64_t step = 1, lo = i;   // keys[lo] == key
  while (lo + step < n && keys[lo + step] == key) {
    lo += step;
    step <<= 1;
  }
  uint64_t hi = min<uint64_t>(n, lo + step);   // keys[hi] != key or hi == n
  while (hi - lo > 1) {
    const uint64_t m = lo + ((hi - lo) >> 1);
    if (keys[m] == key) lo = m; else hi = m;
  }
  return hi;
}
__device__ inline uint64_t run_begin(const unsigned long long* keys, uint64_t i, unsigned long long key) {
  uint64_t step = 1, hi = i;   // keys[hi] == key
  while (hi >= step && keys[hi - step] == key) {
    hi -= step;
    step <<= 1;
  }
  uint64_t lo = hi >= step ? hi - step : 0;   // keys[lo] != key, or lo == 0
  if (keys[lo] == key) return lo;
  while (hi - lo > 1) {
    const uint64_t m = lo + ((hi - lo) >> 1);
    if (keys[m] == key) hi = m; else lo = m;
  }
  return hi;
}

__global__ void k_c4_pair_counts(View v, const unsigned long long* __restrict__ keys, const uint32_t* __restrict__ vals,
                                 uint64_t n, const uint32_t* __restrict__ pos, const uint32_t* __restrict__ start,
                                 uint64_t n2, const uint32_t* __restrict__ eid, unsigned long long* __restrict__ c4e) {
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += uint64_t(gridDim.x) * blockDim.x) {
    const unsigned long long key = keys[i];
    if (key == kC4None) continue;
    const bool prev = i > 0 && keys[i - 1] == key, next = i + 1 < n && keys[i + 1] == key;
    if (!prev && !next) continue;   // a run of one closes no cycle
    const unsigned long long c = run_end(keys, n, i, key) - run_begin(keys, i, key) - 1;
    const uint32_t p = vals[i];
    // the pair whose walk holds position p: from the first pair of p's tile
    uint64_t a = start[p / kC4Tile], b = min<uint64_t>(n2, a + kC4Tile + 2);   // pos[a] <= p < pos[b]
    while (b - a > 1) {
      const uint64_t m = (a + b) >> 1;
      if (pos[m] <= p) a = m; else b = m;
    }
    const uint32_t x0 = v.e2[2 * a], x1 = v.e2[2 * a + 1];
    const uint32_t x = rank_less(v, x0, x1) ? x0 : x1;
    atomicAdd(&c4e[a], c);
    atomicAdd(&c4e[eid[v.g2_off[x] + (p - pos[a])]], c);
  }
}

// Sum of C(run, 2) over the runs of equal keys (kC4None excluded) of the
// sorted keys[0, n).
__global__ void k_c4_runs(const unsigned long long* __restrict__ keys, uint64_t n, unsigned long long none,
                          unsigned long long* __restrict__ acc) {
  unsigned long long s = 0;
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += uint64_t(gridDim.x) * blockDim.x) {
    const unsigned long long key = keys[i];
    if (key == none || (i > 0 && keys[i - 1] == key)) continue;
    uint64_t lo = i, hi = n;   // keys[lo] == key, keys[hi] != key (or hi = n)
    while (hi - lo > 1) {
      const uint64_t m = lo + ((hi - lo) >> 1);
      if (keys[m] == key) lo = m; else hi = m;
    }
    const unsigned long long run = hi - i;
    s += run * (run - 1) / 2;
  }
  block_add(s, acc);
}

int node_bits_of(uint32_t n) {
  int b = 1;
  while (b < 32 && (1ull << b) < n) ++b;
  return b;
}

// The sorted wedge keys of the 4-cycle count (see k_c4_keys).
struct C4Keys {
  unsigned long long* keys = nullptr;   // ascending, n_keys
  uint32_t* vals = nullptr;             // the walked position of each key
  uint32_t* pos = nullptr;              // first position of each pair of G2
  uint32_t* start = nullptr;            // first pair of each tile of positions
  uint64_t n_keys = 0;
};

// Neighbours that follow each node in degree order (outdeg zeroed by the caller).
__global__ void k_sp_outdeg(View v, uint64_t n2, uint32_t* __restrict__ outdeg) {
  for (uint64_t e = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n2; e += uint64_t(gridDim.x) * blockDim.x) {
    const uint32_t a = v.e2[2 * e], b = v.e2[2 * e + 1];
    atomicAdd(&outdeg[rank_less(v, a, b) ? a : b], 1u);
  }
}

// 4-cliques: for each pair {lo, hi} of G2 (lo before hi in degree order),
// W = common neighbours after hi; every pair of W joined by a pair of G2
// closes one 4-clique, found once at its first two nodes.  One wavefront per
// pair; W goes to a per-wavefront list of cap entries.
__device__ inline uint32_t row_pos(const View& v, uint32_t r, uint32_t x) {
  uint32_t lo = v.g2_off[r], hi = v.g2_off[r + 1];
  while (lo < hi) {
    const uint32_t m = lo + ((hi - lo) >> 1);
    if (v.g2_adj[m] < x) lo = m + 1; else hi = m;
  }
  return lo;
}

template <bool PER_EDGE>
__global__ void __launch_bounds__(kThreads) k_sp_k4(View v, uint64_t n2, uint32_t cap, uint32_t* __restrict__ wlist,
                                                    unsigned long long* __restrict__ acc,
                                                    const uint32_t* __restrict__ eid,
                                                    unsigned long long* __restrict__ k4e) {
  const uint32_t lane = threadIdx.x & (kWave - 1);
  const uint64_t wave = uint64_t(blockIdx.x) * kWavesPerBlock + threadIdx.x / kWave;
  const uint64_t n_waves = uint64_t(gridDim.x) * kWavesPerBlock;
  uint32_t* W = wlist + wave * cap * (PER_EDGE ? 2 : 1);
  uint32_t* Wp = W + cap;   // position of each W entry in lo's row (PER_EDGE)
  unsigned long long total = 0;
  for (uint64_t e = wave; e < n2; e += n_waves) {
    uint32_t lo = v.e2[2 * e], hi = v.e2[2 * e + 1];
    if (rank_less(v, hi, lo)) {
      const uint32_t t = lo;
      lo = hi;
      hi = t;
    }
    uint32_t nw = 0;
    for (uint32_t p0 = v.g2_off[lo]; p0 < v.g2_off[lo + 1]; p0 += kWave) {
      const uint32_t p = p0 + lane;
      bool keep = false;
      uint32_t w = 0;
      if (p < v.g2_off[lo + 1]) {
        w = v.g2_adj[p];
        keep = rank_less(v, hi, w) && has2(v.hs2, hi, w);
      }
      const unsigned long long m = __ballot(keep);
      if (keep) {
        const uint32_t slot = nw + uint32_t(__popcll(m & ((1ull << lane) - 1ull)));
        W[slot] = w;
        if (PER_EDGE) Wp[slot] = p;
      }
      nw += uint32_t(__popcll(m));
    }
    wave_sync();
    if (PER_EDGE) {
      // Each lane owns slots s and counts, over every other slot t, the
      // cliques {lo, hi, w_s, w_t}: the pairs {lo, w_s} and {hi, w_s} take
      // that count once, the pair {w_s, w_t} one per clique (from s < t), and
      // {lo, hi} the wavefront's total over the slots, halved.
      unsigned long long twice = 0;
      for (uint32_t s = lane; s < nw; s += kWave) {
        const uint32_t ws = W[s];
        uint32_t cs = 0;
        for (uint32_t t = 0; t < nw; ++t) {
          const uint32_t wt = W[t];
          if (t == s || !has2(v.hs2, ws, wt)) continue;
          ++cs;
          if (s < t) {
            const bool sw = deg2_of(v, ws) <= deg2_of(v, wt);
            atomicAdd(&k4e[eid[sw ? row_pos(v, ws, wt) : row_pos(v, wt, ws)]], 1ull);
          }
        }
        if (cs) {
          atomicAdd(&k4e[eid[Wp[s]]], (unsigned long long)cs);
          atomicAdd(&k4e[eid[row_pos(v, hi, ws)]], (unsigned long long)cs);
          twice += cs;
        }
      }
      twice = wave_sum(twice);
      if (lane == 0 && twice) atomicAdd(&k4e[e], twice / 2);
      total += twice / 2;
    } else {
      uint32_t c = 0;
      for (uint32_t i = 0; i + 1 < nw; ++i) {
        const uint32_t wi = W[i];
        for (uint32_t j = i + 1 + lane; j < nw; j += kWave) {
          if (has2(v.hs2, wi, W[j])) ++c;
        }
      }
      total += wave_sum_u32(c);
    }
    wave_sync();
  }
  if (lane == 0) atomicAdd(acc + kAccK4, total);
}

// Per pair e = {u < w}: over the common neighbours x, the sums of t_{ux},
// t_{wx} and deg x (the smaller row walked, the other row searched).
__global__ void __launch_bounds__(kThreads) k_es_sums(View v, uint64_t n2, const uint32_t* __restrict__ eid,
                                                      const uint32_t* __restrict__ tri_e,
                                                      unsigned long long* __restrict__ su,
                                                      unsigned long long* __restrict__ sw,
                                                      unsigned long long* __restrict__ sd) {
  const uint32_t lane = threadIdx.x & (kWave - 1);
  const uint64_t wave = uint64_t(blockIdx.x) * kWavesPerBlock + threadIdx.x / kWave;
  const uint64_t n_waves = uint64_t(gridDim.x) * kWavesPerBlock;
  for (uint64_t e = wave; e < n2; e += n_waves) {
    const uint32_t u = v.e2[2 * e], w = v.e2[2 * e + 1];
    const bool walk_u = deg2_of(v, u) <= deg2_of(v, w);
    const uint32_t r = walk_u ? u : w, o = walk_u ? w : u;
    unsigned long long a = 0, b = 0, c = 0;   // sums over the walked and the searched side
    for (uint32_t p = v.g2_off[r] + lane; p < v.g2_off[r + 1]; p += kWave) {
      const uint32_t x = v.g2_adj[p];
      if (!has2(v.hs2, o, x)) continue;
      a += tri_e[eid[p]];
      b += tri_e[eid[row_pos(v, o, x)]];
      c += deg2_of(v, x);
    }
    a = wave_sum(a);
    b = wave_sum(b);
    c = wave_sum(c);
    if (lane == 0) {
      su[e] = walk_u ? a : b;
      sw[e] = walk_u ? b : a;
      sd[e] = c;
    }
  }
}

__global__ void k_es_widen(const uint32_t* __restrict__ t32, uint64_t n, unsigned long long* __restrict__ t64) {
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += uint64_t(gridDim.x) * blockDim.x)
    t64[i] = t32[i];
}

// (b) at order 4 without bit rows: one wavefront per 3-node hyperedge, taken
// in the order `order` (decreasing estimated cost), so that the grid's
// wavefronts, each taking every n_waves-th, get like shares of a
// heavy-tailed workload.
__global__ void __launch_bounds__(kThreads) k_sp_b4(View v, PairLinks pl, uint64_t n3, const uint32_t* __restrict__ order,
                                                    const uint8_t* __restrict__ lut_g,
                                                    unsigned long long* __restrict__ hist) {
  __shared__ uint8_t lut[2048];
  __shared__ unsigned long long h_main[256], h_sub[256];
  __shared__ __align__(16) uint32_t short_lists[kWavesPerBlock][kB4ShortWords];
  load_lut(lut, lut_g, 2048);
  h_main[threadIdx.x] = 0;
  h_sub[threadIdx.x] = 0;
  __syncthreads();
  const uint64_t wave = uint64_t(blockIdx.x) * kWavesPerBlock + threadIdx.x / kWave;
  const uint64_t n_waves = uint64_t(gridDim.x) * kWavesPerBlock;
  uint32_t* short_mem = short_lists[threadIdx.x / kWave];
  for (uint64_t j = wave; j < n3; j += n_waves) {
    const uint64_t i = order[j];
    b4_sparse<true, true>(v, pl, v.e3[3 * i], v.e3[3 * i + 1], v.e3[3 * i + 2], lut, h_main, h_sub, short_mem, false);
  }
  __syncthreads();
  unsigned long long* hc = hist_copy(hist, kExactHistStride);
  flush(h_main, hc + kMain, 256);
  flush(h_sub, hc + kSub, 256);
}

// (b) at order 4 without bit rows, the pair-run terms: one wavefront per
// entry of the pair index, in index order, so that the entries of one run
// (and their shared lists) are taken by neighbouring wavefronts.
// (four wavefronts per SIMD: its items are chains of dependent lookups)
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4, 8))) k_sp_b4_runs(View v, PairLinks pl, const uint8_t* __restrict__ lut_g,
                                                         unsigned long long* __restrict__ hist) {
  __shared__ uint8_t lut[2048];
  __shared__ unsigned long long h_main[256], h_sub[256];
  __shared__ __align__(16) uint32_t short_lists[kWavesPerBlock][kB4ShortWords];
  load_lut(lut, lut_g, 2048);
  h_main[threadIdx.x] = 0;
  h_sub[threadIdx.x] = 0;
  __syncthreads();
  const uint64_t wave = uint64_t(blockIdx.x) * kWavesPerBlock + threadIdx.x / kWave;
  const uint64_t n_waves = uint64_t(gridDim.x) * kWavesPerBlock;
  uint32_t* short_mem = short_lists[threadIdx.x / kWave];
  for (uint64_t p = wave; p < pl.n; p += n_waves) b4_run_entry(v, pl, p, lut, h_main, h_sub, short_mem);
  __syncthreads();
  unsigned long long* hc = hist_copy(hist, kExactHistStride);
  flush(h_main, hc + kMain, 256);
  flush(h_sub, hc + kSub, 256);
}

// Sort keys of the 3-node hyperedges for k_sp_b4: the complement of an
// estimate of the memory transactions of each (two per entry of its shortest
// pairwise row, six per entry of the 4-node incidence list it reads when
// there is no 4-node index), with the hyperedge as value.
__global__ void k_b4_cost_keys(View v, PairLinks pl, uint64_t n3, unsigned long long* __restrict__ keys,
                               uint32_t* __restrict__ vals) {
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n3; i += uint64_t(gridDim.x) * blockDim.x) {
    const uint32_t a = v.e3[3 * i], b = v.e3[3 * i + 1], c = v.e3[3 * i + 2];
    const uint64_t dmin = min(deg2_of(v, a), min(deg2_of(v, b), deg2_of(v, c)));
    const uint32_t fa = v.i4_off[a + 1] - v.i4_off[a], fb = v.i4_off[b + 1] - v.i4_off[b],
                   fc = v.i4_off[c + 1] - v.i4_off[c];
    // (with the 4-node index, the 4-node hyperedges holding e are one lookup)
    const uint64_t cost = 2 * dmin + (pl.q_bits ? 0 : 6 * uint64_t(min(fa, min(fb, fc))));
    keys[i] = 0xFFFFFFFFull - min<uint64_t>(cost, 0xFFFFFFFFull);
    vals[i] = uint32_t(i);
  }
}

// Induced shape counts from the non-induced ones, into the G2 region.
struct ShapeClasses {
  int k3_path, k3_triangle;
  int path, star, cycle, paw, diamond, clique;
};

__global__ void k_sp_shapes(const unsigned long long* __restrict__ acc, int k, ShapeClasses cls,
                            unsigned long long* __restrict__ hist) {
  if (threadIdx.x != 0) return;
  const unsigned long long T = acc[kAccT3] / 3;
  if (k == 3) {
    hist[kG2 + cls.k3_triangle] = T;
    hist[kG2 + cls.k3_path] = acc[kAccWedge] - 3 * T;
    return;
  }
  const unsigned long long k4 = acc[kAccK4];
  const unsigned long long dia = acc[kAccDiamond] - 6 * k4;
  const unsigned long long cyc = acc[kAccC4] - dia - 3 * k4;
  const unsigned long long paw = acc[kAccPaw] - 4 * dia - 12 * k4;
  const unsigned long long star = acc[kAccStar] - paw - 2 * dia - 4 * k4;
  const unsigned long long path = (acc[kAccP4] - 3 * T) - 4 * cyc - 2 * paw - 6 * dia - 12 * k4;
  hist[kG2 + cls.clique] = k4;
  hist[kG2 + cls.diamond] = dia;
  hist[kG2 + cls.cycle] = cyc;
  hist[kG2 + cls.paw] = paw;
  hist[kG2 + cls.star] = star;
  hist[kG2 + cls.path] = path;
}

// Entries of the pair index: code 3i + s for 3-node hyperedge i = {a<b<c} and
// slot s, the pair {a,b} (third node c), {a,c} (b) or {b,c} (a).  The
// entries are sorted by third node, then stably by pair, so that each pair's
// run lists its third nodes in ascending order.
__device__ inline uint32_t pl_third_of(const uint32_t* e3, uint32_t code) {
  const uint64_t i = code / 3;
  const uint32_t s = code % 3;
  return e3[3 * i + 2 - s];
}

__global__ void k_pl_third_keys(const uint32_t* __restrict__ e3, uint64_t n, unsigned long long* __restrict__ keys,
                                uint32_t* __restrict__ codes) {
  for (uint64_t p = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; p < n; p += uint64_t(gridDim.x) * blockDim.x) {
    keys[p] = pl_third_of(e3, uint32_t(p));
    codes[p] = uint32_t(p);
  }
}

__global__ void k_pl_pair_keys(const uint32_t* __restrict__ e3, const uint32_t* __restrict__ codes, uint64_t n,
                               unsigned long long* __restrict__ keys) {
  for (uint64_t p = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; p < n; p += uint64_t(gridDim.x) * blockDim.x) {
    const uint32_t code = codes[p];
    const uint64_t i = code / 3;
    const uint32_t s = code % 3;
    const unsigned long long a = e3[3 * i], b = e3[3 * i + 1], c = e3[3 * i + 2];
    keys[p] = s == 0 ? ((a << 32) | b) : (s == 1 ? ((a << 32) | c) : ((b << 32) | c));
  }
}

// One-hot of adjacency class cl over the entries (for the prefix counts).
__global__ void k_pl_class_flags(const uint8_t* __restrict__ adj, uint64_t n, uint32_t cl, uint32_t* __restrict__ out) {
  for (uint64_t p = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; p < n; p += uint64_t(gridDim.x) * blockDim.x)
    out[p] = adj[p] == cl ? 1u : 0u;
}

// Hash index over the runs of the sorted pair keys.  First pass: every run's
// first position claims a slot for its key (start << 32); second pass: its
// last position adds the count.
__global__ void k_pl_index_starts(const unsigned long long* __restrict__ keys, uint64_t n, unsigned long long* slot,
                                  unsigned long long mask) {
  for (uint64_t p = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; p < n; p += uint64_t(gridDim.x) * blockDim.x) {
    const unsigned long long key = keys[p];
    if (p > 0 && keys[p - 1] == key) continue;
    unsigned long long h = mix64(key) & mask;
    while (atomicCAS(&slot[2 * h], kEmpty64, key) != kEmpty64) h = (h + 1) & mask;
    slot[2 * h + 1] = (unsigned long long)p << 32;
  }
}

__global__ void k_pl_index_counts(const unsigned long long* __restrict__ keys, uint64_t n, unsigned long long* slot,
                                  unsigned long long mask) {
  for (uint64_t p = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; p < n; p += uint64_t(gridDim.x) * blockDim.x) {
    const unsigned long long key = keys[p];
    if (p + 1 < n && keys[p + 1] == key) continue;
    unsigned long long h = mix64(key) & mask;
    while (slot[2 * h] != key) h = (h + 1) & mask;
    const unsigned long long start = slot[2 * h + 1] >> 32;
    slot[2 * h + 1] = (start << 32) | (p + 1 - start);
  }
}

// Per pair entry: its 3-node hyperedge (the code, in place), the third node
// and that node's pairwise adjacency to the two nodes of the key.
__global__ void k_pl_third(const uint32_t* __restrict__ e3, const unsigned long long* __restrict__ keys,
                           uint32_t* __restrict__ edge, uint64_t n, Set64 hs2, uint32_t* __restrict__ third,
                           uint8_t* __restrict__ adj) {
  for (uint64_t p = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; p < n; p += uint64_t(gridDim.x) * blockDim.x) {
    const unsigned long long key = keys[p];
    const uint32_t x = uint32_t(key >> 32), y = uint32_t(key);
    const uint32_t code = edge[p];
    const uint32_t t = pl_third_of(e3, code);
    edge[p] = code / 3;
    third[p] = t;
    adj[p] = uint8_t(uint32_t(has2(hs2, x, t)) | (uint32_t(has2(hs2, y, t)) << 1));
  }
}

// Common pairwise neighbours of every distinct pair of the index, into the
// pair's slot: each wavefront takes 64 positions of the sorted keys at a
// time and, for each run that starts among them, walks the shorter of the two
// rows and probes the other.
__global__ void k_pl_codeg(View v, const unsigned long long* __restrict__ keys, uint64_t n,
                           const unsigned long long* __restrict__ slot, unsigned long long mask,
                           uint32_t* __restrict__ codeg) {
  const uint32_t lane = threadIdx.x & (kWave - 1);
  const uint64_t wave = (uint64_t(blockIdx.x) * blockDim.x + threadIdx.x) / kWave;
  const uint64_t n_waves = uint64_t(gridDim.x) * blockDim.x / kWave;
  for (uint64_t p0 = wave * kWave; p0 < n; p0 += n_waves * kWave) {
    const uint64_t p = p0 + lane;
    const bool start = p < n && (p == 0 || keys[p - 1] != keys[p]);
    unsigned long long m = __ballot(start);
    while (m) {
      const uint32_t l = uint32_t(__ffsll(m) - 1);
      m &= m - 1;
      const unsigned long long key = keys[p0 + l];
      const uint32_t x = uint32_t(key >> 32), y = uint32_t(key);
      const uint32_t dx = deg2_of(v, x), dy = deg2_of(v, y);
      const uint32_t sn = dx <= dy ? x : y, on = dx <= dy ? y : x;
      uint32_t c = 0;
      for (uint32_t q = v.g2_off[sn] + lane; q < v.g2_off[sn + 1]; q += kWave) c += has2(v.hs2, on, v.g2_adj[q]);
      c = wave_sum_u32(c);
      if (lane == 0) {
        unsigned long long h = mix64(key) & mask;
        while (slot[2 * h] != key) h = (h + 1) & mask;
        codeg[h] = c;
      }
    }
  }
}

// Temporaries of one call, released in stream order (see dfree_on), also
// when the call returns early on an error.
struct Scratch {
  std::vector<void*> ptrs;
  hipStream_t st;
  explicit Scratch(hipStream_t s) : st(s) {}
  ~Scratch() { dfree_on(ptrs.data(), ptrs.size(), st); }
  template <typename T>
  int get(T** p, uint64_t n) {
    void* q = nullptr;
    HM_TRY(dalloc(&q, size_t(n ? n : 1) * sizeof(T)));
    ptrs.push_back(q);
    *p = static_cast<T*>(q);
    return HM_OK;
  }
};

unsigned grid_cap(uint64_t items, uint64_t per_block, unsigned cap) {
  uint64_t g = (items + per_block - 1) / per_block;
  return unsigned(std::max<uint64_t>(1, std::min<uint64_t>(g, cap)));
}


// The wedge keys of the 4-cycle count, built and sorted into scratch (one
// host read-back: the number of walked positions).
int c4_sorted_keys(const hm_graph* H, hipStream_t st, Scratch& tmp, C4Keys* out) {
  const View v = view_of(H);
  const uint64_t n2 = H->n_by_size[2];
  *out = C4Keys{};
  if (!n2) return HM_OK;
  unsigned long long* walk = nullptr;
  uint32_t* len = nullptr;
  HM_TRY(tmp.get(&walk, 1));
  HM_TRY(tmp.get(&len, n2));
  HM_TRY(tmp.get(&out->pos, n2));
  HM_TRY(fill_u64(walk, 0, 1, st));
  k_c4_len<<<grid_cap(n2, 256, 2048), 256, 0, st>>>(v, n2, len, walk);
  HM_HIP(hipGetLastError());
  unsigned long long n_keys = 0;
  HM_HIP(hipMemcpyAsync(&n_keys, walk, sizeof(n_keys), hipMemcpyDeviceToHost, st));
  HM_HIP(hipStreamSynchronize(st));
  const int B = node_bits_of(H->n_nodes);
  if (n_keys >= 0xFFFFFFFFull || 2 * B > 63 || n2 >= 0xFFFFFFFFull) {
    set_error("4-cycle wedges of %llu positions exceed the sort's range", n_keys);
    return HM_EUNSUPPORTED;
  }
  if (!n_keys) return HM_OK;
  const uint32_t n_tiles = uint32_t((n_keys + kC4Tile - 1) / kC4Tile);
  unsigned long long* keys_tmp = nullptr;
  uint32_t* vals_tmp = nullptr;
  HM_TRY(tmp.get(&out->start, n_tiles));
  HM_TRY(tmp.get(&out->keys, n_keys));
  HM_TRY(tmp.get(&keys_tmp, n_keys));
  HM_TRY(tmp.get(&out->vals, n_keys));
  HM_TRY(tmp.get(&vals_tmp, n_keys));
  HM_TRY(scan_exclusive_u32(len, out->pos, n2, nullptr, st));
  k_c4_tile_starts<<<grid_cap(n2, 256, 4096), 256, 0, st>>>(out->pos, len, n2, out->start);
  HM_HIP(hipGetLastError());
  {
    ProfileScope ps("k_c4_keys", st);
    k_c4_keys<<<n_tiles, kThreads, 0, st>>>(v, B, out->pos, out->start, n2, uint32_t(n_keys), n_tiles, out->keys,
                                           out->vals);
  }
  HM_HIP(hipGetLastError());
  // the positions that are not wedges carry all ones and sort last
  {
    ProfileScope ps("c4_sort", st);
    HM_TRY(radix_sort_pairs(out->keys, out->vals, keys_tmp, vals_tmp, n_keys, 2 * B + 1, st));
  }
  out->n_keys = n_keys;
  return HM_OK;
}

// Workgroups of kThreads threads (no dynamic LDS) of `kernel` resident on the
// current device at once.
unsigned resident_blocks(const void* kernel) {
  static std::mutex mu;
  static std::map<std::pair<const void*, int>, unsigned> cache;
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find({kernel, dev});
  if (it != cache.end()) return it->second;
  int cus = 256, per_cu = 1;
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kThreads, 0) != hipSuccess || per_cu < 1) per_cu = 1;
  const unsigned r = unsigned(std::max(cus, 1)) * unsigned(per_cu);
  cache[{kernel, dev}] = r;
  return r;
}

}  // namespace

namespace {

__global__ void k_ns_half(const unsigned long long* __restrict__ tv, uint32_t n, unsigned long long* __restrict__ tri) {
  for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < n; x += gridDim.x * blockDim.x) tri[x] = tv[x] / 2;
}

// sum of the neighbours' degrees, per node
__global__ void k_ns_nbr(View v, uint64_t n2, unsigned long long* __restrict__ nbr) {
  for (uint64_t e = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n2; e += uint64_t(gridDim.x) * blockDim.x) {
    const uint32_t a = v.e2[2 * e], b = v.e2[2 * e + 1];
    atomicAdd(&nbr[a], (unsigned long long)deg2_of(v, b));
    atomicAdd(&nbr[b], (unsigned long long)deg2_of(v, a));
  }
}

// per node o, its 3-node hyperedges {o, y, z} (y < z) by (o~y, o~z, y~z)
__global__ void k_ns_h3(View v, uint64_t n3, uint32_t* __restrict__ h3) {
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n3; i += uint64_t(gridDim.x) * blockDim.x) {
    const uint32_t a = v.e3[3 * i], b = v.e3[3 * i + 1], c = v.e3[3 * i + 2];
    const uint32_t pab = has2(v.hs2, a, b), pac = has2(v.hs2, a, c), pbc = has2(v.hs2, b, c);
    atomicAdd(&h3[8ull * a + (pab | (pac << 1) | (pbc << 2))], 1u);
    atomicAdd(&h3[8ull * b + (pab | (pbc << 1) | (pac << 2))], 1u);
    atomicAdd(&h3[8ull * c + (pac | (pbc << 1) | (pab << 2))], 1u);
  }
}

}  // namespace

// Per-node statistics of H for the pair samplers without bit rows, built on
// first use: triangles at each node, the sum of its neighbours' degrees, and
// its 3-node hyperedges by pairwise pattern.
int ensure_node_stats(hm_graph* H, hipStream_t st) {
  note_use(H, st);
  if (H->ns_tri) return HM_OK;
  const View v = view_of(H);
  const uint64_t n2 = H->n_by_size[2], n3 = H->n_by_size[3], N = H->n_nodes;
  Scratch tmp(st);
  unsigned long long *acc = nullptr, *tv = nullptr;
  uint32_t* tri_e = nullptr;
  HM_TRY(tmp.get(&acc, kAccN));
  HM_TRY(tmp.get(&tv, N));
  HM_TRY(tmp.get(&tri_e, n2));
  HM_TRY(fill_u64(acc, 0, kAccN, st));
  HM_TRY(fill_u64(tv, 0, N, st));
  void *p_tri = nullptr, *p_nbr = nullptr, *p_h3 = nullptr;
  int rc = dalloc(&p_tri, N * sizeof(unsigned long long));
  if (rc == HM_OK) rc = dalloc(&p_nbr, N * sizeof(unsigned long long));
  if (rc == HM_OK) rc = dalloc(&p_h3, 8 * N * sizeof(uint32_t));
  auto* tri = static_cast<unsigned long long*>(p_tri);
  auto* nbr = static_cast<unsigned long long*>(p_nbr);
  auto* h3 = static_cast<uint32_t*>(p_h3);
  if (rc == HM_OK) rc = fill_u64(nbr, 0, N, st);
  if (rc == HM_OK) rc = fill_u32(h3, 0, 8 * N, st);
  if (rc == HM_OK) {
    if (n2) k_sp_edge_tri<<<grid_cap(n2, kWavesPerBlock, 2048), kThreads, 0, st>>>(v, n2, tri_e, tv, acc);
    k_ns_half<<<grid_cap(N, 256, 1024), 256, 0, st>>>(tv, uint32_t(N), tri);
    if (n2) k_ns_nbr<<<grid_cap(n2, 256, 2048), 256, 0, st>>>(v, n2, nbr);
    if (n3) k_ns_h3<<<grid_cap(n3, 256, 2048), 256, 0, st>>>(v, n3, h3);
    if (hipGetLastError() != hipSuccess) rc = HM_EDEVICE;
  }
  if (rc == HM_OK && hipStreamSynchronize(st) != hipSuccess) rc = HM_EDEVICE;
  if (rc != HM_OK) {
    dfree(p_tri);
    dfree(p_nbr);
    dfree(p_h3);
    return rc;
  }
  H->ns_tri = tri;
  H->ns_nbr = nbr;
  H->ns_h3 = h3;
  return HM_OK;
}

// Per-pair statistics of H for the pair sampler without bit rows (layout in
// hm_graph::es), built on first use.
int ensure_edge_stats(hm_graph* H, hipStream_t st) {
  note_use(H, st);
  if (H->es) return HM_OK;
  const View v = view_of(H);
  const uint64_t n2 = H->n_by_size[2], N = H->n_nodes;
  void* p_es = nullptr;
  HM_TRY(dalloc(&p_es, 6 * std::max<uint64_t>(n2, 1) * sizeof(unsigned long long)));
  auto* es = static_cast<unsigned long long*>(p_es);
  int rc = fill_u64(es, 0, 6 * n2, st);
  {
    Scratch tmp(st);
    unsigned long long *acc = nullptr, *tv = nullptr;
    uint32_t *tri_e = nullptr, *outdeg = nullptr, *dmax = nullptr, *wlist = nullptr;
    if (rc == HM_OK) rc = tmp.get(&acc, kAccN);
    if (rc == HM_OK) rc = tmp.get(&tv, N);
    if (rc == HM_OK) rc = tmp.get(&tri_e, n2);
    if (rc == HM_OK) rc = tmp.get(&outdeg, N);
    if (rc == HM_OK) rc = tmp.get(&dmax, 1);
    if (rc == HM_OK) rc = fill_u64(acc, 0, kAccN, st);
    if (rc == HM_OK) rc = fill_u64(tv, 0, N, st);
    if (rc == HM_OK) rc = fill_u32(dmax, 0, 1, st);
    if (rc == HM_OK && n2) {
      k_sp_edge_tri<<<grid_cap(n2, kWavesPerBlock, 2048), kThreads, 0, st>>>(v, n2, tri_e, tv, acc);
      k_es_widen<<<grid_cap(n2, 256, 2048), 256, 0, st>>>(tri_e, n2, es);
      k_es_sums<<<grid_cap(n2, kWavesPerBlock, 2048), kThreads, 0, st>>>(v, n2, H->g2_eid, tri_e, es + 3 * n2,
                                                                         es + 4 * n2, es + 5 * n2);
      // per-pair 4-cycles from the sorted wedge keys
      C4Keys ck;
      if (rc == HM_OK) rc = c4_sorted_keys(H, st, tmp, &ck);
      if (rc == HM_OK && ck.n_keys)
        k_c4_pair_counts<<<grid_cap(ck.n_keys, 256, 4096), 256, 0, st>>>(v, ck.keys, ck.vals, ck.n_keys, ck.pos,
                                                                        ck.start, n2, H->g2_eid, es + 2 * n2);
      if (fill_u32(outdeg, 0, N, st) != HM_OK) rc = HM_EDEVICE;
      k_sp_outdeg<<<grid_cap(n2, 256, 2048), 256, 0, st>>>(v, n2, outdeg);
      if (hipGetLastError() != hipSuccess) rc = HM_EDEVICE;
      if (rc == HM_OK) rc = max_u32(outdeg, N, dmax, st);
      uint32_t cap = 0;
      if (rc == HM_OK && hipMemcpyAsync(&cap, dmax, sizeof(uint32_t), hipMemcpyDeviceToHost, st) != hipSuccess)
        rc = HM_EDEVICE;
      if (rc == HM_OK && hipStreamSynchronize(st) != hipSuccess) rc = HM_EDEVICE;
      cap = std::max<uint32_t>(cap, 1);
      const unsigned gk = grid_cap(n2, kWavesPerBlock, 1024);
      if (rc == HM_OK) rc = tmp.get(&wlist, uint64_t(gk) * kWavesPerBlock * cap * 2);
      if (rc == HM_OK) {
        k_sp_k4<true><<<gk, kThreads, 0, st>>>(v, n2, cap, wlist, acc, H->g2_eid, es + 1 * n2);
        if (hipGetLastError() != hipSuccess) rc = HM_EDEVICE;
      }
    }
    if (rc == HM_OK && hipStreamSynchronize(st) != hipSuccess) rc = HM_EDEVICE;
  }
  if (rc != HM_OK) {
    dfree(p_es);
    return rc;
  }
  H->es = es;
  return HM_OK;
}

// Every 3-node subset of every 4-node hyperedge, packed as in quad_find, with
// the hyperedge's fourth node.
__global__ void k_quad_keys(const uint32_t* __restrict__ e4, uint64_t n4, int q, unsigned long long* __restrict__ keys,
                            uint32_t* __restrict__ fourth) {
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n4; i += uint64_t(gridDim.x) * blockDim.x) {
    const unsigned long long m[4] = {e4[4 * i], e4[4 * i + 1], e4[4 * i + 2], e4[4 * i + 3]};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const unsigned long long x = m[s == 0 ? 1 : 0], y = m[s <= 1 ? 2 : 1], z = m[s <= 2 ? 3 : 2];
      keys[4 * i + s] = (x << (2 * q)) | (y << q) | z;
      fourth[4 * i + s] = uint32_t(m[s]);
    }
  }
}

// The 3-node subset -> 4-node hyperedge index (H->q_*), when the packed key
// fits 63 bits; otherwise none (q_bits = 0) and the incidence lists serve.
int build_quad_index(hm_graph* H, hipStream_t st) {
  const uint64_t n4 = H->n_by_size[4];
  int bits = 1;
  while (bits < 32 && (1ull << bits) < H->n_nodes) ++bits;
  if (n4 == 0 || 3 * bits > 63) return HM_OK;
  const uint64_t n = 4 * n4;
  void *k = nullptr, *f = nullptr, *kt = nullptr, *ft = nullptr, *slots = nullptr;
  int rc = dalloc(&k, n * sizeof(unsigned long long));
  if (rc == HM_OK) rc = dalloc(&f, n * sizeof(uint32_t));
  if (rc == HM_OK) rc = dalloc(&kt, n * sizeof(unsigned long long));
  if (rc == HM_OK) rc = dalloc(&ft, n * sizeof(uint32_t));
  if (rc == HM_OK) {
    k_quad_keys<<<grid_cap(n4, 256, 4096), 256, 0, st>>>(H->e4, n4, bits, static_cast<unsigned long long*>(k),
                                                         static_cast<uint32_t*>(f));
    if (hipGetLastError() != hipSuccess) rc = HM_EDEVICE;
  }
  if (rc == HM_OK)
    rc = radix_sort_pairs(static_cast<unsigned long long*>(k), static_cast<uint32_t*>(f),
                          static_cast<unsigned long long*>(kt), static_cast<uint32_t*>(ft), n, 3 * bits, st);
  const unsigned long long cap = pow2_capacity(n);
  if (rc == HM_OK) rc = dalloc(&slots, 2 * cap * sizeof(unsigned long long));
  if (rc == HM_OK) rc = fill_u64(static_cast<unsigned long long*>(slots), kEmpty64, 2 * cap, st);
  if (rc == HM_OK) {
    const unsigned g = grid_cap(n, 256, 4096);
    k_pl_index_starts<<<g, 256, 0, st>>>(static_cast<const unsigned long long*>(k), n,
                                         static_cast<unsigned long long*>(slots), cap - 1);
    k_pl_index_counts<<<g, 256, 0, st>>>(static_cast<const unsigned long long*>(k), n,
                                         static_cast<unsigned long long*>(slots), cap - 1);
    if (hipGetLastError() != hipSuccess) rc = HM_EDEVICE;
  }
  if (rc == HM_OK && hipStreamSynchronize(st) != hipSuccess) rc = HM_EDEVICE;
  dfree(k);
  dfree(kt);
  dfree(ft);
  if (rc != HM_OK) {
    dfree(f);
    dfree(slots);
    return rc;
  }
  H->q_slot = static_cast<unsigned long long*>(slots);
  H->q_mask = cap - 1;
  H->q_fourth = static_cast<uint32_t*>(f);
  H->q_bits = bits;
  return HM_OK;
}

// The pair -> 3-node hyperedge index of H, built on first use (with the
// 4-node index beside it).
int ensure_pair_links(hm_graph* H, hipStream_t st) {
  note_use(H, st);
  if (H->pl_keys || H->n_by_size[3] == 0) return HM_OK;
  const uint64_t n = 3 * H->n_by_size[3];
  void *k = nullptr, *e = nullptr, *kt = nullptr, *et = nullptr;
  HM_TRY(dalloc(&k, n * sizeof(unsigned long long)));
  int rc = dalloc(&e, n * sizeof(uint32_t));
  if (rc == HM_OK) rc = dalloc(&kt, n * sizeof(unsigned long long));
  if (rc == HM_OK) rc = dalloc(&et, n * sizeof(uint32_t));
  int bits = 1;
  while (bits < 32 && (1ull << bits) < H->n_nodes) ++bits;
  if (rc == HM_OK) {
    k_pl_third_keys<<<grid_cap(n, 256, 4096), 256, 0, st>>>(H->e3, n, static_cast<unsigned long long*>(k),
                                                            static_cast<uint32_t*>(e));
    if (hipGetLastError() != hipSuccess) rc = HM_EDEVICE;
  }
  if (rc == HM_OK)
    rc = radix_sort_pairs(static_cast<unsigned long long*>(k), static_cast<uint32_t*>(e),
                          static_cast<unsigned long long*>(kt), static_cast<uint32_t*>(et), n, bits, st);
  if (rc == HM_OK) {
    k_pl_pair_keys<<<grid_cap(n, 256, 4096), 256, 0, st>>>(H->e3, static_cast<const uint32_t*>(e), n,
                                                           static_cast<unsigned long long*>(k));
    if (hipGetLastError() != hipSuccess) rc = HM_EDEVICE;
  }
  if (rc == HM_OK)
    rc = radix_sort_pairs(static_cast<unsigned long long*>(k), static_cast<uint32_t*>(e),
                          static_cast<unsigned long long*>(kt), static_cast<uint32_t*>(et), n, 32 + bits, st);
  // the index: at most n distinct keys, load at most 1/2
  const unsigned long long cap = pow2_capacity(n);
  void *slots = nullptr, *codeg = nullptr, *third = nullptr, *adj = nullptr, *pre = nullptr;
  if (rc == HM_OK) rc = dalloc(&slots, 2 * cap * sizeof(unsigned long long));
  if (rc == HM_OK) rc = dalloc(&codeg, cap * sizeof(uint32_t));
  if (rc == HM_OK) rc = dalloc(&third, n * sizeof(uint32_t));
  if (rc == HM_OK) rc = dalloc(&adj, n * sizeof(uint8_t));
  if (rc == HM_OK) rc = dalloc(&pre, 4 * (n + 1) * sizeof(uint32_t));
  if (rc == HM_OK) rc = fill_u64(static_cast<unsigned long long*>(slots), kEmpty64, 2 * cap, st);
  if (rc == HM_OK) {
    const unsigned g = grid_cap(n, 256, 4096);
    k_pl_index_starts<<<g, 256, 0, st>>>(static_cast<const unsigned long long*>(k), n,
                                         static_cast<unsigned long long*>(slots), cap - 1);
    k_pl_index_counts<<<g, 256, 0, st>>>(static_cast<const unsigned long long*>(k), n,
                                         static_cast<unsigned long long*>(slots), cap - 1);
    k_pl_third<<<g, 256, 0, st>>>(H->e3, static_cast<const unsigned long long*>(k), static_cast<uint32_t*>(e), n,
                                  H->hs2, static_cast<uint32_t*>(third), static_cast<uint8_t*>(adj));
    k_pl_codeg<<<grid_cap((n + kWave - 1) / kWave, kWavesPerBlock, 4096), kThreads, 0, st>>>(
        view_of(H), static_cast<const unsigned long long*>(k), n, static_cast<const unsigned long long*>(slots),
        cap - 1, static_cast<uint32_t*>(codeg));
    if (hipGetLastError() != hipSuccess) rc = HM_EDEVICE;
  }
  // prefix counts of the entries by adjacency class (the flags reuse et)
  for (uint32_t cl = 0; cl < 4 && rc == HM_OK; ++cl) {
    uint32_t* out = static_cast<uint32_t*>(pre) + cl * (n + 1);
    k_pl_class_flags<<<grid_cap(n, 256, 4096), 256, 0, st>>>(static_cast<const uint8_t*>(adj), n, cl,
                                                             static_cast<uint32_t*>(et));
    if (hipGetLastError() != hipSuccess) rc = HM_EDEVICE;
    if (rc == HM_OK) rc = scan_exclusive_u32(static_cast<const uint32_t*>(et), out, n, out + n, st);
  }
  if (rc == HM_OK && hipStreamSynchronize(st) != hipSuccess) rc = HM_EDEVICE;
  dfree(kt);
  dfree(et);
  if (rc != HM_OK) {
    dfree(k);
    dfree(e);
    dfree(slots);
    dfree(codeg);
    dfree(third);
    dfree(adj);
    dfree(pre);
    return rc;
  }
  H->pl_keys = static_cast<unsigned long long*>(k);
  H->pl_edge = static_cast<uint32_t*>(e);
  H->pl_slot = static_cast<unsigned long long*>(slots);
  H->pl_mask = cap - 1;
  H->pl_codeg = static_cast<uint32_t*>(codeg);
  H->pl_third = static_cast<uint32_t*>(third);
  H->pl_adj = static_cast<uint8_t*>(adj);
  H->pl_pre = static_cast<uint32_t*>(pre);
  return build_quad_index(H, st);
}

PairLinks pair_links_of(const hm_graph* H) {
  PairLinks pl;
  pl.keys = H->pl_keys;
  pl.edge = H->pl_edge;
  pl.n = H->pl_keys ? 3 * H->n_by_size[3] : 0;
  pl.slot = reinterpret_cast<const ulonglong2*>(H->pl_slot);
  pl.mask = H->pl_mask;
  pl.codeg = H->pl_codeg;
  pl.third = H->pl_third;
  pl.adj = H->pl_adj;
  pl.pre = H->pl_pre;
  pl.q_slot = reinterpret_cast<const ulonglong2*>(H->q_slot);
  pl.q_mask = H->q_mask;
  pl.q_fourth = H->q_fourth;
  pl.q_bits = H->q_bits;
  pl.hub_rank = H->hub_rank;
  pl.hub_bits = H->hub_bits;
  pl.hub_w = H->hub_words;
  return pl;
}

// One workgroup per dense row: the bits of the node's pairwise neighbours.
__global__ void k_hub_rows(const uint32_t* __restrict__ g2_off, const uint32_t* __restrict__ g2_adj,
                           const uint32_t* __restrict__ hubs, uint32_t n_hub, uint32_t words,
                           uint32_t* __restrict__ bits) {
  for (uint32_t r = blockIdx.x; r < n_hub; r += gridDim.x) {
    const uint32_t x = hubs[r];
    uint32_t* row = bits + uint64_t(r) * words;
    for (uint32_t p = g2_off[x] + threadIdx.x; p < g2_off[x + 1]; p += blockDim.x) {
      const uint32_t z = g2_adj[p];
      atomicOr(&row[z >> 5], 1u << (z & 31));
    }
  }
}

// H->hub_rank and H->hub_bits: the nodes with at least hub_min_degree()
// pairwise neighbours, highest degree first (ties by id), as many as fit in
// kHubRowBytes.  Built once per graph.
int ensure_hub_rows(hm_graph* H, hipStream_t st) {
  note_use(H, st);
  if (H->hub_built) return HM_OK;
  const uint32_t n = H->n_nodes, min_deg = hub_min_degree();
  const uint32_t words = (n + 31) / 32;
  if (n == 0 || min_deg == 0 || !H->g2_off) {
    H->hub_built = true;
    return HM_OK;
  }
  std::vector<uint32_t> off(size_t(n) + 1);
  HM_HIP(hipMemcpyAsync(off.data(), H->g2_off, off.size() * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
  HM_HIP(hipStreamSynchronize(st));
  std::vector<uint32_t> hubs;
  for (uint32_t x = 0; x < n; ++x)
    if (off[x + 1] - off[x] >= min_deg) hubs.push_back(x);
  std::sort(hubs.begin(), hubs.end(), [&](uint32_t p, uint32_t q) {
    const uint32_t dp = off[p + 1] - off[p], dq = off[q + 1] - off[q];
    return dp != dq ? dp > dq : p < q;
  });
  const uint64_t max_rows = kHubRowBytes / (uint64_t(words) * sizeof(uint32_t));
  if (hubs.size() > max_rows) hubs.resize(size_t(max_rows));
  if (hubs.empty()) {
    H->hub_built = true;
    return HM_OK;
  }
  std::vector<int32_t> rank(n, -1);
  for (size_t r = 0; r < hubs.size(); ++r) rank[hubs[r]] = int32_t(r);
  const uint32_t n_hub = uint32_t(hubs.size());
  void *rank_d = nullptr, *hubs_d = nullptr, *bits_d = nullptr;
  int rc = dalloc(&rank_d, size_t(n) * sizeof(int32_t));
  if (rc == HM_OK) rc = dalloc(&hubs_d, size_t(n_hub) * sizeof(uint32_t));
  if (rc == HM_OK) rc = dalloc(&bits_d, size_t(n_hub) * words * sizeof(uint32_t));
  if (rc == HM_OK && (hipMemcpyAsync(rank_d, rank.data(), rank.size() * sizeof(int32_t), hipMemcpyHostToDevice, st) !=
                          hipSuccess ||
                      hipMemcpyAsync(hubs_d, hubs.data(), hubs.size() * sizeof(uint32_t), hipMemcpyHostToDevice, st) !=
                          hipSuccess))
    rc = HM_EDEVICE;
  if (rc == HM_OK) rc = fill_u32(static_cast<uint32_t*>(bits_d), 0, uint64_t(n_hub) * words, st);
  if (rc == HM_OK) {
    k_hub_rows<<<std::min<uint32_t>(n_hub, 4096), 256, 0, st>>>(H->g2_off, H->g2_adj, static_cast<const uint32_t*>(hubs_d),
                                                               n_hub, words, static_cast<uint32_t*>(bits_d));
    if (hipGetLastError() != hipSuccess) rc = HM_EDEVICE;
  }
  // the host vectors stay alive until the copies have run
  if (hipStreamSynchronize(st) != hipSuccess && rc == HM_OK) rc = HM_EDEVICE;
  dfree(hubs_d);
  if (rc != HM_OK) {
    dfree(rank_d);
    dfree(bits_d);
    return rc;
  }
  H->hub_rank = static_cast<int32_t*>(rank_d);
  H->hub_bits = static_cast<uint32_t*>(bits_d);
  H->hub_words = words;
  H->hub_built = true;
  return HM_OK;
}

// H->b4_order, after the pair index: the 3-node hyperedges sorted by
// decreasing cost estimate.
int ensure_b4_order(hm_graph* H, hipStream_t st) {
  note_use(H, st);
  const uint64_t n3 = H->n_by_size[3];
  if (H->b4_order || n3 == 0) return HM_OK;
  void *k = nullptr, *o = nullptr, *kt = nullptr, *ot = nullptr;
  int rc = dalloc(&k, n3 * sizeof(unsigned long long));
  if (rc == HM_OK) rc = dalloc(&o, n3 * sizeof(uint32_t));
  if (rc == HM_OK) rc = dalloc(&kt, n3 * sizeof(unsigned long long));
  if (rc == HM_OK) rc = dalloc(&ot, n3 * sizeof(uint32_t));
  if (rc == HM_OK) {
    k_b4_cost_keys<<<grid_cap(n3, 256, 4096), 256, 0, st>>>(view_of(H), pair_links_of(H), n3,
                                                            static_cast<unsigned long long*>(k), static_cast<uint32_t*>(o));
    if (hipGetLastError() != hipSuccess) rc = HM_EDEVICE;
  }
  if (rc == HM_OK)
    rc = radix_sort_pairs(static_cast<unsigned long long*>(k), static_cast<uint32_t*>(o),
                          static_cast<unsigned long long*>(kt), static_cast<uint32_t*>(ot), n3, 32, st);
  if (rc == HM_OK && hipStreamSynchronize(st) != hipSuccess) rc = HM_EDEVICE;
  dfree(k);
  dfree(kt);
  dfree(ot);
  if (rc != HM_OK) {
    dfree(o);
    return rc;
  }
  H->b4_order = static_cast<uint32_t*>(o);
  return HM_OK;
}

// Fills the main, sub and G2 regions of H->hist (zeroed by the caller) except
// case (a), which the caller counts.
int count_sparse(const hm_graph* H, int k, hipStream_t st) {
  note_use(H, st);
  const uint8_t *lut4 = nullptr, *lut3 = nullptr;
  HM_TRY(device_luts(H->device, &lut4, &lut3));
  const View v = view_of(H);
  const uint64_t n2 = H->n_by_size[2], n3 = H->n_by_size[3];
  Scratch tmp(st);
  unsigned long long *acc = nullptr, *tv = nullptr;
  uint32_t* tri_e = nullptr;
  HM_TRY(tmp.get(&acc, kAccN));
  HM_TRY(tmp.get(&tv, H->n_nodes));
  HM_TRY(tmp.get(&tri_e, n2));
  HM_TRY(fill_u64(acc, 0, kAccN, st));
  HM_TRY(fill_u64(tv, 0, H->n_nodes, st));
  if (n2) {
    ProfileScope ps("k_sp_edge_tri", st);
    k_sp_edge_tri<<<grid_cap(n2, kWavesPerBlock, 2048), kThreads, 0, st>>>(v, n2, tri_e, tv, acc);
  }
  {
    ProfileScope ps("k_sp_nodes", st);
    k_sp_nodes<<<grid_cap(H->n_nodes, kThreads, 1024), kThreads, 0, st>>>(v, tv, acc);
  }
  HM_HIP(hipGetLastError());
  const ClassTables& t = class_tables();
  ShapeClasses cls;
  // representative pair patterns (local nodes 0..3; bits: 01=0, 02=1, 12=2, 03=4, 13=5, 23=7)
  cls.k3_path = t.lut3[0x3];       // 01, 02
  cls.k3_triangle = t.lut3[0x7];   // 01, 02, 12
  cls.path = t.lut4[(1u << 0) | (1u << 2) | (1u << 7)];
  cls.star = t.lut4[(1u << 0) | (1u << 1) | (1u << 4)];
  cls.cycle = t.lut4[(1u << 0) | (1u << 2) | (1u << 7) | (1u << 4)];
  cls.paw = t.lut4[(1u << 0) | (1u << 1) | (1u << 2) | (1u << 4)];
  cls.diamond = t.lut4[(1u << 0) | (1u << 1) | (1u << 2) | (1u << 4) | (1u << 5)];
  cls.clique = t.lut4[kPairBits4];
  if (k == 4 && n2) {
    // 4-cycles: wedge keys, sorted, counted by runs
    C4Keys ck;
    HM_TRY(c4_sorted_keys(H, st, tmp, &ck));
    if (ck.n_keys) {
      ProfileScope ps("k_c4_runs", st);
      k_c4_runs<<<grid_cap(ck.n_keys, 256, 4096), 256, 0, st>>>(ck.keys, ck.n_keys, kC4None, acc + kAccC4);
    }
    HM_HIP(hipGetLastError());
    // 4-cliques
    uint32_t *outdeg = nullptr, *dmax = nullptr;
    HM_TRY(tmp.get(&outdeg, H->n_nodes));
    HM_TRY(tmp.get(&dmax, 1));
    HM_TRY(fill_u32(dmax, 0, 1, st));
    HM_TRY(fill_u32(outdeg, 0, H->n_nodes, st));
    k_sp_outdeg<<<grid_cap(n2, 256, 2048), 256, 0, st>>>(v, n2, outdeg);
    HM_TRY(max_u32(outdeg, H->n_nodes, dmax, st));
    uint32_t cap = 0;
    HM_HIP(hipMemcpyAsync(&cap, dmax, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    HM_HIP(hipStreamSynchronize(st));
    const unsigned gk = grid_cap(n2, kWavesPerBlock, 1024);
    uint32_t* wlist = nullptr;
    HM_TRY(tmp.get(&wlist, uint64_t(gk) * kWavesPerBlock * std::max<uint32_t>(cap, 1)));
    {
      ProfileScope ps("k_sp_k4", st);
      k_sp_k4<false><<<gk, kThreads, 0, st>>>(v, n2, std::max<uint32_t>(cap, 1), wlist, acc, nullptr, nullptr);
    }
    HM_HIP(hipGetLastError());
  }
  if (k == 4 && n3) {
    HM_TRY(ensure_pair_links(const_cast<hm_graph*>(H), st));
    HM_TRY(ensure_b4_order(const_cast<hm_graph*>(H), st));
    HM_TRY(ensure_hub_rows(const_cast<hm_graph*>(H), st));
    // no more workgroups than are resident at once: each wavefront's share is
    // fixed, and a workgroup that starts late would finish late
    const unsigned grid = grid_cap(n3, kWavesPerBlock, resident_blocks(reinterpret_cast<const void*>(k_sp_b4)));
    {
      ProfileScope ps("k_sp_b4", st);
      k_sp_b4<<<grid, kThreads, 0, st>>>(v, pair_links_of(H), n3, H->b4_order, lut4, H->hist);
    }
    HM_HIP(hipGetLastError());
    const uint64_t n_entries = 3 * n3;
    const unsigned grid_r =
        grid_cap(n_entries, kWavesPerBlock, resident_blocks(reinterpret_cast<const void*>(k_sp_b4_runs)));
    {
      ProfileScope ps("k_sp_b4_runs", st);
      k_sp_b4_runs<<<grid_r, kThreads, 0, st>>>(v, pair_links_of(H), lut4, H->hist);
    }
    HM_HIP(hipGetLastError());
  }
  k_sp_shapes<<<1, 64, 0, st>>>(acc, k, cls, H->hist);
  HM_HIP(hipGetLastError());
  // the scratch is released when the work is done
  HM_HIP(hipStreamSynchronize(st));
  return HM_OK;
}

}  // namespace hm
